// batch.hip -- many independent simulations of uneven sizes advanced together.
//
// Each case is a full problem statement (lattice, EOS, T/Tc, force model, tau, precision, grid).
// A step of a case has two phases:
//   phase 1: pull-gather every node -> rho, signed psi, g = rho u^3 into the case's fields;
//   phase 2: two-ring Korteweg force from the fields, correction, product-form equilibria
//            and LBGK (the same device functions as the single-case kernels), written to
//            the other lattice.
// Stepped design (default): one launch per phase (and lattice) and step covers every case,
// each case split into blocks of nodes, so the cases of a sweep share all CUs; the phases
// are ordered by the stream. The block split (threads per block, nodes per thread) is tuned
// per case list and kept in a cache file keyed by the GPU target. Persistent design
// (LBM2P_BATCH_STEPPED=0): one workgroup owns a case and runs its whole step loop with
// workgroup barriers only; its workgroup size is tuned the same way. Either way a chunk of
// steps is captured once in a HIP graph that lbm_batch_step replays.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm2p.h"
#include "kernels.hpp"
#include "lattice.hpp"
#include "runtime_common.hpp"
#include "step_common.hpp"

using namespace lbm;

namespace {

struct CaseDesc {
    int D;          // 2 or 3
    int fp64;       // storage/compute precision
    Geom g;
    void *A, *B;    // population lattices (A = current)
    void *frho, *fpsi, *fg;   // fields in compute precision: rho, s*psi, g[D]
    const uint8_t *mask;      // nullable
    double *totals;           // 5 slots: mass, j, domain-error count (FP64)
    Params<double> pd;
    Params<float> pf;
};

// --------------------------------------------------------------- device part
// The per-node step functions see a case through a view: node indices, solid flags, the
// pull gather, the field arrays, 1- and 2-ring neighbour indices and the store. GlobalView
// addresses the case's device arrays; TileView a tile of a D2Q9 case held in LDS. Both
// designs run the same arithmetic in the same order, so they give the same bits.
template <int D, class S, class C> struct GlobalView {
    const Geom &g;
    const uint8_t *mask;
    const S *A;
    S *B;
    C *frho, *fpsi, *fg;
    struct Node {
        int x, y, z;
        Nbr<D> nb;
    };
    __device__ __forceinline__ Node node(int n) const {
        const int x = n % g.nx, t = n / g.nx, y = t % g.ny, z = t / g.ny;
        return Node{x, y, z, Nbr<D>(g, x, y, z)};
    }
    __device__ __forceinline__ bool solid(int n) const { return mask && mask[n]; }
    __device__ __forceinline__ int global_index(int n) const { return n; }
    __device__ __forceinline__ void gather_at(const Node &nd, int n, C (&h)[Lat<D>::Q]) const {
        if (mask) gather<D, S, C, true>(A, g.qs, mask, nd.nb, n, h);
        else gather<D, S, C, false>(A, g.qs, mask, nd.nb, n, h);
    }
    __device__ __forceinline__ int at1(const Node &nd, int cx, int cy, int cz) const { return nd.nb.at(cx, cy, cz); }
    __device__ __forceinline__ int at2(const Node &nd, int cx, int cy, int cz) const {
        const int x2 = wrapi(nd.x + 2 * cx, g.nx), y2 = wrapi(nd.y + 2 * cy, g.ny);
        const int z2 = D == 3 ? wrapi(nd.z + 2 * cz, g.nz) : 0;
        return x2 + g.nx * (y2 + g.ny * z2);
    }
    __device__ __forceinline__ C &rho(int n) const { return frho[n]; }
    __device__ __forceinline__ C &psi(int n) const { return fpsi[n]; }
    __device__ __forceinline__ C &gfield(int a, int n) const { return fg[a * g.N + n]; }
    __device__ __forceinline__ void store(int i, int n, C v) const { st_at(B + i * g.qs, (unsigned)n, S(v)); }
};

// phase 1 at node n (view coordinates nd): rho, signed psi and g = rho u^3 of the current
// state into the fields
template <int D, class S, class C, class V>
__device__ __forceinline__ void phase1_at(const V &v, const Params<C> &p, int n, const typename V::Node &nd) {
    constexpr int Q = Lat<D>::Q;
    C rho, ga[3] = {C(0), C(0), C(0)};
    if (v.solid(n)) {
        rho = wall_density(p, v.global_index(n));
    } else {
        C h[Q];
        v.gather_at(nd, n, h);
        C sum, j[3];
        moments_of<D, C>(h, sum, j);
        rho = p.rho_ref + sum;
        const C rinv = rcp(rho);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const C ua = j[a] * rinv;
            ga[a] = rho * ua * ua * ua;
        }
    }
    v.rho(n) = rho;
    v.psi(n) = signed_psi(p.eos, rho);
#pragma unroll
    for (int a = 0; a < D; ++a) v.gfield(a, n) = ga[a];
}

// phase 2 at fluid node n (view coordinates nd): force from the fields, correction,
// equilibria, LBGK, store
template <int D, class S, class C, class V>
__device__ __forceinline__ void phase2_at(const V &v, const Params<C> &p, int n, const typename V::Node &nd) {
    constexpr int Q = Lat<D>::Q;
    if (v.solid(n)) return;
    const C rho = v.rho(n), spc = v.psi(n);
    C Fp[3] = {C(0), C(0), C(0)}, Fc[3] = {C(0), C(0), C(0)};
    static_for<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
        constexpr int cls = cx * cx + cy * cy + cz * cz - 1;   // weight class of c_i
        const int n1 = v.at1(nd, cx, cy, cz), n2 = v.at2(nd, cx, cy, cz);
        const C p1 = fabs(v.psi(n1)), p2 = fabs(v.psi(n2));
        const C r1 = v.rho(n1), r2 = v.rho(n2);
        const C tp = p.gw[cls][0] * p1 + p.gw[cls][1] * p2;   // 3w (G1 psi1 + G2 psi2)
        const C tc = p.gw[cls][2] * r1 + p.gw[cls][3] * r2;   // 3w (G3 rho1 + G4 rho2)
        static_for<0, D>([&](auto A_) {
            constexpr int a = decltype(A_)::value;
            constexpr int ca = Lat<D>::c(i, a);
            if constexpr (ca == 1) { Fp[a] += tp; Fc[a] += tc; }
            if constexpr (ca == -1) { Fp[a] -= tp; Fc[a] -= tc; }
        });
    });
    C Sf[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) Sf[a] = rho * p.accel[a] - (C(2) * spc * Fp[a] + rho * Fc[a]);
    C h[Q];
    v.gather_at(nd, n, h);
    C drho, j[3];
    moments_of<D, C>(h, drho, j);
    const C rinv = rcp(rho);
    C u[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = j[a] * rinv;
    const C omega = omega_of(p, rho);
    const C cf = (C(1) - C(0.5) * omega) * C(0.5);
    C Phi[3] = {C(0), C(0), C(0)};
    Phi[0] = cf * (v.gfield(0, v.at1(nd, 1, 0, 0)) - v.gfield(0, v.at1(nd, -1, 0, 0)));
    Phi[1] = cf * (v.gfield(1, v.at1(nd, 0, 1, 0)) - v.gfield(1, v.at1(nd, 0, -1, 0)));
    if constexpr (D == 3) Phi[2] = cf * (v.gfield(2, v.at1(nd, 0, 0, 1)) - v.gfield(2, v.at1(nd, 0, 0, -1)));
    collide<D, C>(h, rho, drho, u, Sf, Phi, omega);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        v.store(i, n, h[i]);
    });
}

template <int D, class S, class C>
__device__ __forceinline__ GlobalView<D, S, C> global_view(const CaseDesc &cd, const S *A, S *B) {
    return GlobalView<D, S, C>{cd.g, cd.mask, A, B, (C *)cd.frho, (C *)cd.fpsi, (C *)cd.fg};
}

template <int D, class S, class C>
__device__ __forceinline__ void phase1_node(const CaseDesc &cd, const Params<C> &p, const S *A, int n) {
    const auto v = global_view<D, S, C>(cd, A, nullptr);
    phase1_at<D, S, C>(v, p, n, v.node(n));
}

template <int D, class S, class C>
__device__ __forceinline__ void phase2_node(const CaseDesc &cd, const Params<C> &p, const S *A, S *B, int n) {
    const auto v = global_view<D, S, C>(cd, A, B);
    if (!v.solid(n)) phase2_at<D, S, C>(v, p, n, v.node(n));
}

// ---------------------------------------------------------------- several steps per launch
// A D2Q9 case whose full y extent fits in LDS is advanced S steps per launch in tiles of TX
// columns: a workgroup loads its tile plus H = 3 S halo columns on each side (all rows,
// y periodic inside the tile), steps them in LDS and writes back its own TX columns. A node
// at step t + 1 depends on nodes at most three columns away at step t (one for the pull, two
// for the ring stencils of the nodes it pulls from), so after s steps columns [3 s, W - 3 s)
// of the tile (W = TX + 2 H) are exact and after S steps the tile's own columns are. Halo
// columns are recomputed by the neighbouring tiles: the price of dropping 2 S - 1 launches.
struct TileWork {
    int c, x0, tx;   // case, first column, columns of the tile
};

template <class S, class C> struct TileView {
    const S *A;      // LDS populations of the current state, [9][M]
    S *B;            // LDS populations of the next state
    C *frho, *fpsi, *fg;
    const uint8_t *mask;   // LDS solid flags or nullptr
    const int *col;        // LDS: global column of each tile column (wrapped)
    int W, M, nx;          // tile width with halo, nodes, case width
    // a node's column and the LDS offsets of rows y - 2 .. y + 2 (periodic in y)
    struct Node {
        int j;
        int row[5];
    };
    __device__ __forceinline__ bool solid(int n) const { return mask && mask[n]; }
    __device__ __forceinline__ int global_index(int n) const { return col[n % W] + nx * (n / W); }
    __device__ __forceinline__ int at1(const Node &nd, int cx, int cy, int) const { return nd.row[2 + cy] + nd.j + cx; }
    __device__ __forceinline__ int at2(const Node &nd, int cx, int cy, int) const {
        return nd.row[2 + 2 * cy] + nd.j + 2 * cx;
    }
    // the same pull as the global gather: f_i(r) = A_i(r - c_i), or A_opp(i)(r) from a solid source
    __device__ __forceinline__ void gather_at(const Node &nd, int n, C (&h)[9]) const {
        static_for<0, 9>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i == 0) {
                h[0] = C(A[n]);
            } else {
                const int src = at1(nd, -Lat<2>::c(i, 0), -Lat<2>::c(i, 1), 0);
                h[i] = solid(src) ? C(A[opp<2>(i) * M + n]) : C(A[i * M + src]);
            }
        });
    }
    __device__ __forceinline__ C &rho(int n) const { return frho[n]; }
    __device__ __forceinline__ C &psi(int n) const { return fpsi[n]; }
    __device__ __forceinline__ C &gfield(int a, int n) const { return fg[a * M + n]; }
    __device__ __forceinline__ void store(int i, int n, C v) const { B[i * M + n] = S(v); }
};

// LDS bytes of a tile of W x ny nodes: two population sets, rho, s psi, g_x, g_y, the column
// map and solid flags
__host__ __device__ constexpr long long tile_lds_bytes(int W, int ny, int sbytes) {
    return (long long)W * ny * (22LL * sbytes + 1) + 4LL * W + 16;
}

// Tile threads: 4 row lanes of CL column lanes (CL = 64 or 128), so that a node's tile
// coordinates need no division; row offsets are wrapped by adding or subtracting ny.
__device__ __forceinline__ int wrap_row(int y, int ny) {
    while (y < 0) y += ny;
    while (y >= ny) y -= ny;
    return y;
}

// nsteps steps of one tile of a case (storage S, compute C) in LDS
template <class S, class C, int CL>
__device__ __forceinline__ void tile_run(const CaseDesc *cd, const TileWork &w, int nsteps, bool even, char *lds) {
    constexpr int NT = 4 * CL;
    // the case's parameters in registers, read once
    const Params<C> p = *(const Params<C> *)(sizeof(C) == 8 ? (const void *)&cd->pd : (const void *)&cd->pf);
    const uint8_t *gmask = cd->mask;
    const S *gA = (const S *)(even ? cd->A : cd->B);
    S *gB = (S *)(even ? cd->B : cd->A);
    const int ny = cd->g.ny, nx = cd->g.nx;
    const long long qs = cd->g.qs;
    const int H = 3 * nsteps, W = w.tx + 2 * H, M = W * ny;
    S *pop0 = (S *)lds;
    S *pop1 = pop0 + 9 * M;
    C *frho = (C *)(pop1 + 9 * M);
    C *fpsi = frho + M;
    C *fg = fpsi + M;
    int *col = (int *)(fg + 2 * M);
    uint8_t *msk = gmask ? (uint8_t *)(col + W) : nullptr;
    const int tc = threadIdx.x & (CL - 1), tr = threadIdx.x / CL;   // column lane, row lane
    for (int j = threadIdx.x; j < W; j += NT) col[j] = wrapi(w.x0 - H + j, nx);
    __syncthreads();
    // the tile with its halo from the current lattice, straight into LDS: rows (population,
    // y) by the four row lanes, each wave copying 64 consecutive 4-byte words of a row per
    // load (an FP64 value is two words), every load in flight before the single wait
    const int rows = 9 * ny;
    {
        constexpr int WPV = (int)(sizeof(S) / 4);   // 4-byte words per value
        const int words = W * WPV;                  // words of one tile row
        const int lane0 = tc & ~63;                 // the wave's first column lane
        for (int r = tr; r < rows; r += 4) {
            const int i = r / ny, y = r - i * ny;
            const char *grow = (const char *)(gA + i * qs + (long long)nx * y);
            char *lrow = (char *)(pop0 + (long long)r * W);
            for (int k0 = lane0; k0 < words; k0 += CL) {
                const int k = k0 + (tc & 63);
                if (k < words) {
                    const int j = k / WPV, part = k - j * WPV;
                    __builtin_amdgcn_global_load_lds((const void *)(grow + (long long)col[j] * (long long)sizeof(S) + 4 * part),
                                                     (__attribute__((address_space(3))) void *)(lrow + 4 * k0), 4, 0, 0);
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the copies have landed
    }
    if (msk)
        for (int y = tr; y < ny; y += 4)
            for (int j = tc; j < W; j += CL) msk[y * W + j] = gmask[col[j] + nx * y];
    __syncthreads();
    S *cur = pop0, *nxt = pop1;
    for (int st = 1; st <= nsteps; ++st) {
        const TileView<S, C> v{cur, nxt, frho, fpsi, fg, msk, col, W, M, nx};
        auto node = [&](int j, int y) __attribute__((always_inline)) {
            typename TileView<S, C>::Node nd;
            nd.j = j;
#pragma unroll
            for (int d = 0; d < 5; ++d) nd.row[d] = wrap_row(y + d - 2, ny) * W;
            return nd;
        };
        // fields on columns [3 st - 2, W - 3 st + 2): the ring stencils of the exact columns
        const int a1 = 3 * st - 2, b1 = W - a1;
        for (int y = tr; y < ny; y += 4)
            for (int j = a1 + tc; j < b1; j += CL) phase1_at<2, S, C>(v, p, y * W + j, node(j, y));
        __syncthreads();
        const int a2 = 3 * st, b2 = W - a2;
        for (int y = tr; y < ny; y += 4)
            for (int j = a2 + tc; j < b2; j += CL) phase2_at<2, S, C>(v, p, y * W + j, node(j, y));
        __syncthreads();
        S *t = cur; cur = nxt; nxt = t;
    }
    // the tile's own columns [H, H + tx) into the next lattice
    for (int r = tr; r < rows; r += 4) {
        const int i = r / ny, y = r - i * ny;
        for (int j = tc; j < w.tx; j += CL) gB[i * qs + (w.x0 + j) + nx * y] = cur[r * W + H + j];
    }
}

// one launch: nsteps steps of the tiles listed in work; launch index li selects the current
// lattice of each case with its parity
template <int CL>
__global__ __launch_bounds__(4 * CL) void k_batch_tile(const CaseDesc *__restrict__ cases, const TileWork *__restrict__ work,
                                                       int nsteps, int li, const int *__restrict__ parity) {
    extern __shared__ __align__(16) char lds[];
    const TileWork w = work[blockIdx.x];
    const CaseDesc *cd = cases + w.c;
    const bool even = ((li + parity[w.c]) & 1) == 0;
    if (cd->fp64) tile_run<double, double, CL>(cd, w, nsteps, even, lds);
    else tile_run<float, float, CL>(cd, w, nsteps, even, lds);
}

// the whole step loop of one case in one workgroup (persistent design)
template <int D, class S, class C>
__device__ void case_steps(const CaseDesc &cd, const Params<C> &p, int nsteps, int parity) {
    S *L0 = (S *)cd.A, *L1 = (S *)cd.B;
    for (int st = 0; st < nsteps; ++st) {
        const bool even = ((st + parity) & 1) == 0;
        const S *A = even ? L0 : L1;
        S *B = even ? L1 : L0;
        for (int n = threadIdx.x; n < cd.g.N; n += blockDim.x) phase1_node<D, S, C>(cd, p, A, n);
        __syncthreads();
        for (int n = threadIdx.x; n < cd.g.N; n += blockDim.x) phase2_node<D, S, C>(cd, p, A, B, n);
        __syncthreads();
    }
}

// Stepped design: one launch per phase (and lattice) and step over every case at once,
// each case split into blocks of work items in proportion to its size, so that the
// cases of a sweep share all CUs instead of one workgroup each. A block has TPB threads
// (the launch's block size) and each thread NPT nodes of its case: thread t of block k
// takes nodes k TPB + t + m nk TPB, m < NPT (nk blocks per case). The split changes which
// thread computes a node, never the node's arithmetic, so every split gives the same bits.
struct Work {
    int c, k, nk;   // case, block of the case, blocks of the case
};
constexpr int kStepMaxBlock = 256;   // largest threads per block of the stepped kernels

template <int D, int PHASE, int NPT>
__global__ __launch_bounds__(kStepMaxBlock) void k_batch_phase(const CaseDesc *__restrict__ cases,
                                                               const Work *__restrict__ work, int st,
                                                               const int *__restrict__ parity) {
    const Work w = work[blockIdx.x];
    const CaseDesc cd = cases[w.c];
    const bool even = ((st + parity[w.c]) & 1) == 0;
    const int tpb = (int)blockDim.x;
    const int stride = w.nk * tpb;
    const int n0 = w.k * tpb + (int)threadIdx.x;
    if (cd.fp64) {
        const double *A = (const double *)(even ? cd.A : cd.B);
        double *B = (double *)(even ? cd.B : cd.A);
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const int n = n0 + m * stride;
            if (n >= cd.g.N) break;
            if constexpr (PHASE == 1) phase1_node<D, double, double>(cd, cd.pd, A, n);
            else phase2_node<D, double, double>(cd, cd.pd, A, B, n);
        }
    } else {
        const float *A = (const float *)(even ? cd.A : cd.B);
        float *B = (float *)(even ? cd.B : cd.A);
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const int n = n0 + m * stride;
            if (n >= cd.g.N) break;
            if constexpr (PHASE == 1) phase1_node<D, float, float>(cd, cd.pf, A, n);
            else phase2_node<D, float, float>(cd, cd.pf, A, B, n);
        }
    }
}

// block splits the stepped design's tuner tries: (threads per block, nodes per thread)
struct Split {
    int tpb, npt;
};
constexpr Split kSplits[] = {{256, 1}, {128, 1}, {64, 1}, {256, 2}, {128, 2}, {64, 2}, {128, 4}, {64, 4}};

// one kernel per lattice: the register budget of a D2Q9 sweep is not set by the D3Q27 body
// (D3Q27 cases run with at most 256 threads, which leaves room for the 27-population body)
template <int D>
__global__ __launch_bounds__(D == 2 ? 1024 : 256) void k_batch(const CaseDesc *__restrict__ cases, const int *__restrict__ order,
                                                 int ncases, int nsteps, const int *__restrict__ parity) {
    const int c = order[blockIdx.x];
    if (c >= ncases) return;
    const CaseDesc cd = cases[c];
    const int par = parity[c];
    if (cd.fp64) case_steps<D, double, double>(cd, cd.pd, nsteps, par);
    else case_steps<D, float, float>(cd, cd.pf, nsteps, par);
}

// flips the per-case lattice parity after a launch of an odd number of steps
__global__ void k_flip_parity(int *parity, const int *tiled, int ncases, int nsteps, int nlaunch) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncases) parity[c] = (parity[c] + (tiled[c] ? nlaunch : nsteps)) & 1;
}

// End-of-call divergence check: the non-finite stored populations of every case's current
// lattice (fluid nodes), kCheckBlocks workgroups per case (workgroup b: case b / kCheckBlocks);
// bad[b] receives workgroup b's count, so the host sums a fixed set of integers.
constexpr int kCheckBlocks = 16;
__global__ __launch_bounds__(256) void k_batch_nonfinite(const CaseDesc *__restrict__ cases, const int *__restrict__ parity,
                                                         int *__restrict__ bad) {
    __shared__ int s_bad[4];
    const int c = blockIdx.x / kCheckBlocks, k0 = blockIdx.x % kCheckBlocks;
    const CaseDesc &cd = cases[c];
    const char *L = (const char *)((parity[c] & 1) ? cd.B : cd.A);
    const long long N = cd.g.N, qs = cd.g.qs, total = (cd.D == 3 ? 27LL : 9LL) * N;
    int n_bad = 0;
    for (long long k = (long long)k0 * 256 + threadIdx.x; k < total; k += (long long)kCheckBlocks * 256) {
        const long long i = k / N, n = k - i * N;
        if (cd.mask && cd.mask[n]) continue;
        const double v = cd.fp64 ? ((const double *)L)[i * qs + n] : (double)((const float *)L)[i * qs + n];
        n_bad += isfinite(v) ? 0 : 1;
    }
    for (int o = 32; o > 0; o >>= 1) n_bad += __shfl_xor(n_bad, o, 64);
    if ((threadIdx.x & 63) == 0) s_bad[threadIdx.x >> 6] = n_bad;
    __syncthreads();
    if (threadIdx.x == 0) bad[blockIdx.x] = s_bad[0] + s_bad[1] + s_bad[2] + s_bad[3];
}

thread_local std::string g_batch_err;
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;   // case-list signature -> workgroup size

}  // namespace

// --------------------------------------------------------------- host part
struct lbm_batch {
    std::vector<lbm_params> params;
    std::vector<CaseDesc> host;       // A/B pointers as allocated (parity tracked on the device)
    std::vector<KernelSet> ks;
    std::vector<int> nblk;
    CaseDesc *d_cases = nullptr;
    int *d_order = nullptr, *d_parity = nullptr;
    int n2 = 0, n3 = 0;              // cases per lattice; d_order lists the D2Q9 cases first
    std::vector<void *> allocs;
    double *partials = nullptr, *d_tot = nullptr, *io = nullptr, *rscratch = nullptr;
    size_t io_elems = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int block = 256, chunk = 200;
    bool stepped = true;             // stepped kernels over all cases; false: one workgroup per case
    bool tuned = false;              // the block split (stepped) or workgroup size (persistent) is set
    Split split{256, 1};             // stepped design: threads per block, nodes per thread
    std::vector<int> order;          // cases, D2Q9 first, largest first
    Work *d_work2 = nullptr, *d_work3 = nullptr;
    int nw2 = 0, nw3 = 0;            // work items per lattice for the stepped kernels
    // several steps per launch (D2Q9 cases whose tile fits in LDS): tile lists per precision
    TileWork *d_tile = nullptr;      // tiles of both precisions (one launch)
    int nt = 0;
    size_t tcap = 0;
    int tile_steps = 0, tile_tx = 0;  // steps per launch (0: no case tiled), tile row width
    int tile_lanes = 64;             // column lanes of a tile workgroup (4 row lanes each)
    size_t tlds = 0;                 // dynamic LDS of the tile launches (the largest tile)
    int *d_tiled = nullptr;          // per case: 1 when the case runs in tiles
    int *d_bad = nullptr;            // divergence check: non-finite counts per case and workgroup
    size_t cap2 = 0, cap3 = 0;       // capacity of the work lists (the finest split)
    std::string gfx;                 // the device's target name (tuning cache key)
    std::vector<int> initialized;
    std::string err;
};

namespace {

int bfail(lbm_batch *b, int code, const std::string &m) {
    if (b) b->err = m; else g_batch_err = m;
    return code;
}

#define BHIP(b, call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return bfail((b), LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void free_batch(lbm_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *q : b->allocs) (void)hipFree(q);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

template <int PHASE>
void launch_phase(lbm_batch *b, int st) {
    const dim3 tb(b->split.tpb);
    auto go = [&](auto kern2, auto kern3) {
        if (b->nw2) hipLaunchKernelGGL(kern2, dim3(b->nw2), tb, 0, b->stream, b->d_cases, b->d_work2, st, b->d_parity);
        if (b->nw3) hipLaunchKernelGGL(kern3, dim3(b->nw3), tb, 0, b->stream, b->d_cases, b->d_work3, st, b->d_parity);
    };
    switch (b->split.npt) {
    case 1: go(k_batch_phase<2, PHASE, 1>, k_batch_phase<3, PHASE, 1>); break;
    case 2: go(k_batch_phase<2, PHASE, 2>, k_batch_phase<3, PHASE, 2>); break;
    default: go(k_batch_phase<2, PHASE, 4>, k_batch_phase<3, PHASE, 4>); break;
    }
}

int launch(lbm_batch *b, int nsteps, int block) {
    const int nc = (int)b->host.size();
    const dim3 fg((nc + 255) / 256);
    if (b->stepped) {
        for (int st = 0; st < nsteps; ++st) {
            launch_phase<1>(b, st);   // every case's phase 1 before any phase 2 (stream order)
            launch_phase<2>(b, st);
        }
        int nl = 0;
        if (b->tile_steps > 0 && b->nt)
            for (int k = 0; k < nsteps; k += b->tile_steps, ++nl) {
                const int st = std::min(b->tile_steps, nsteps - k);
                if (b->tile_lanes == 128)
                    hipLaunchKernelGGL(k_batch_tile<128>, dim3(b->nt), dim3(512), b->tlds, b->stream, b->d_cases, b->d_tile,
                                       st, nl, b->d_parity);
                else
                    hipLaunchKernelGGL(k_batch_tile<64>, dim3(b->nt), dim3(256), b->tlds, b->stream, b->d_cases, b->d_tile,
                                       st, nl, b->d_parity);
            }
        if ((nsteps & 1) || (nl & 1))
            hipLaunchKernelGGL(k_flip_parity, fg, dim3(256), 0, b->stream, b->d_parity, b->d_tiled, nc, nsteps, nl);
        return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
    }
    if (b->n2)
        hipLaunchKernelGGL(k_batch<2>, dim3(b->n2), dim3(block), 0, b->stream, b->d_cases, b->d_order, nc, nsteps,
                           b->d_parity);
    if (b->n3)
        hipLaunchKernelGGL(k_batch<3>, dim3(b->n3), dim3(block < 256 ? block : 256), 0, b->stream, b->d_cases, b->d_order + b->n2, nc,
                           nsteps, b->d_parity);
    if (nsteps & 1)
        hipLaunchKernelGGL(k_flip_parity, fg, dim3(256), 0, b->stream, b->d_parity, b->d_tiled, nc, nsteps, nsteps);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

// current lattice of case c (host view of the device parity)
void *current_A(lbm_batch *b, int c, int parity) { return parity ? b->host[c].B : b->host[c].A; }

std::string signature(const lbm_batch *b) {
    std::string s;
    for (const auto &cd : b->host)
        s += std::to_string(cd.D) + ":" + std::to_string(cd.fp64) + ":" + std::to_string(cd.g.N) + ";";
    return s;
}

// LDS budget of one tile workgroup: two workgroups per CU in gfx950's 160 KB
constexpr long long kTileLdsMax = 81920;

// Columns per tile of case c for the tiling (steps per launch, tile row width W: the tile's own
// columns plus a halo of 3 columns per step on each side). Row widths that are multiples of a
// wave's 64 column lanes keep every lane busy in the per-node loops. The own width is W - 6
// steps (the case's width if smaller), W narrowed by 32 columns at a time until the tile fits
// the LDS budget (at least 8 own columns), then evened out over the case's tiles; 0 when no
// width fits or the case is not D2Q9 (it then takes the stepped kernels).
int tile_width(const lbm_batch *b, int c, int steps, int W) {
    const CaseDesc &cd = b->host[c];
    if (cd.D != 2 || steps <= 0) return 0;
    for (int w = W; w - 6 * steps >= 8; w -= 32) {
        const int t = std::min(w - 6 * steps, cd.g.nx);
        if (tile_lds_bytes(t + 6 * steps, cd.g.ny, cd.fp64 ? 8 : 4) <= kTileLdsMax) {
            const int k = (cd.g.nx + t - 1) / t;   // tiles of the case
            return (cd.g.nx + k - 1) / k;
        }
    }
    return 0;
}

// Work lists for the split sp and the tiling (steps per launch, tile row width, column lanes of
// a tile workgroup; steps 0: no tiles): tiled cases in tiles of tile_width columns, the others
// in blocks of tpb npt nodes for the stepped kernels, largest case first; uploaded into the
// lists allocated at create
int build_work(lbm_batch *b, Split sp, int steps = 0, int tx = 128, int lanes = 64) {
    std::vector<Work> w2, w3;
    std::vector<TileWork> tl;
    std::vector<int> tiled(b->host.size(), 0);
    size_t lds = 0;
    const int per = sp.tpb * sp.npt;
    for (int c : b->order) {
        const CaseDesc &cd = b->host[c];
        if (const int tw = tile_width(b, c, steps, tx)) {
            tiled[c] = 1;
            for (int x0 = 0; x0 < cd.g.nx; x0 += tw) {
                const int t = std::min(tw, cd.g.nx - x0);
                tl.push_back(TileWork{c, x0, t});
                lds = std::max(lds, (size_t)tile_lds_bytes(t + 6 * steps, cd.g.ny, cd.fp64 ? 8 : 4));
            }
            continue;
        }
        const int nk = std::max(1, (int)((cd.g.N + per - 1) / per));
        for (int k = 0; k < nk; ++k) (cd.D == 2 ? w2 : w3).push_back(Work{c, k, nk});
    }
    if (w2.size() > b->cap2 || w3.size() > b->cap3 || tl.size() > b->tcap) return LBM_E_INVAL;
    if ((!w2.empty() && hipMemcpy(b->d_work2, w2.data(), w2.size() * sizeof(Work), hipMemcpyHostToDevice) != hipSuccess) ||
        (!w3.empty() && hipMemcpy(b->d_work3, w3.data(), w3.size() * sizeof(Work), hipMemcpyHostToDevice) != hipSuccess) ||
        (!tl.empty() && hipMemcpy(b->d_tile, tl.data(), tl.size() * sizeof(TileWork), hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(b->d_tiled, tiled.data(), tiled.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return LBM_E_HIP;
    b->nw2 = (int)w2.size();
    b->nw3 = (int)w3.size();
    b->nt = (int)tl.size();
    b->tlds = lds;
    b->tile_steps = tl.empty() ? 0 : steps;
    b->tile_tx = tx;
    b->tile_lanes = lanes == 128 ? 128 : 64;
    b->split = sp;
    return LBM_OK;
}

// 64-bit FNV-1a of the case-list signature: the key of a tuning-cache entry
std::string sig_hash(const std::string &s) {
    unsigned long long h = 1469598103934665603ull;
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    char buf[17];
    snprintf(buf, sizeof buf, "%016llx", h);
    return buf;
}

// The tuning cache (LBM2P_TUNE_CACHE names a text file): one line per tuned case list,
//   <gfx target> <signature hash> <design: s | p> <v0> <v1> <v2> <v3> <v4>
// stepped: threads per block, nodes per thread, steps per tile launch (0: no tiles), tile
// columns, tile column lanes; persistent: the workgroup size and four zeros.
// cache key: the case list and the meaning of the tuned values (tile row widths)
std::string cache_signature(const lbm_batch *b) { return "tile-rows;" + signature(b); }

bool cache_lookup(const lbm_batch *b, char design, int (&v)[5]) {
    const char *path = getenv("LBM2P_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    const std::string key = sig_hash(cache_signature(b));
    char gfx[128], h[64], d[8];
    int x[5];
    bool found = false;
    while (fscanf(f, "%127s %63s %7s %d %d %d %d %d", gfx, h, d, &x[0], &x[1], &x[2], &x[3], &x[4]) == 8)
        if (b->gfx == gfx && key == h && d[0] == design) {
            for (int k = 0; k < 5; ++k) v[k] = x[k];
            found = true;   // the last entry for a key wins
        }
    fclose(f);
    return found;
}

void cache_store(const lbm_batch *b, char design, const int (&v)[5]) {
    const char *path = getenv("LBM2P_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %s %c %d %d %d %d %d\n", b->gfx.c_str(), sig_hash(cache_signature(b)).c_str(), design, v[0], v[1], v[2], v[3],
            v[4]);
    fclose(f);
}

}  // namespace

extern "C" {

int lbm_batch_create(const lbm_params *cases, int ncases, lbm_batch **out) {
    if (!out) return bfail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!cases || ncases < 1) return bfail(nullptr, LBM_E_INVAL, "need at least one case");
    for (int c = 0; c < ncases; ++c) {
        std::string why;
        if (!validate_params(&cases[c], &why)) return bfail(nullptr, LBM_E_INVAL, "case " + std::to_string(c) + ": " + why);
        if (cases[c].link_q)
            return bfail(nullptr, LBM_E_INVAL, "case " + std::to_string(c) + ": link_q (interpolated bounce-back) is not supported by the batch");
        // the batch kernels index a case's fields in 32-bit ints: field a of node n at a N + n
        // (a < D) and the block loop's n + stride < 2 N + 256
        const int D = cases[c].lattice == LBM_D3Q27 ? 3 : 2;
        if ((double)(D + 1) * cases[c].nx * cases[c].ny * cases[c].nz + 1024.0 >= 2147483648.0)
            return bfail(nullptr, LBM_E_INVAL, "case " + std::to_string(c) + ": too large for the batch ((D + 1) N must stay below 2^31)");
    }
    lbm_batch *b = new (std::nothrow) lbm_batch;
    if (!b) return bfail(nullptr, LBM_E_NOMEM, "host allocation failed");
    if (hipStreamCreate(&b->stream) != hipSuccess) { free_batch(b); return bfail(nullptr, LBM_E_HIP, "stream creation failed"); }
    b->params.assign(cases, cases + ncases);
    b->host.resize(ncases);
    b->ks.resize(ncases);
    b->nblk.resize(ncases);
    b->initialized.assign(ncases, 0);
    auto dalloc = [&](size_t bytes) -> void * {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
        b->allocs.push_back(q);
        return q;
    };
    int max_nblk = 0;
    for (int c = 0; c < ncases; ++c) {
        const lbm_params &p = cases[c];
        CaseDesc &cd = b->host[c];
        cd.D = p.lattice == LBM_D3Q27 ? 3 : 2;
        cd.fp64 = p.precision == LBM_FP64;
        cd.g = make_geom(p.nx, p.ny, cd.D == 3 ? p.nz : 1);
        fill_params(&p, &cd.pd);
        fill_params(&p, &cd.pf);
        const size_t s = cd.fp64 ? 8 : 4, N = (size_t)cd.g.N, Q = cd.D == 3 ? 27 : 9;
        cd.A = dalloc(Q * cd.g.qs * s);
        cd.B = dalloc(Q * cd.g.qs * s);
        cd.frho = dalloc(N * s);
        cd.fpsi = dalloc(N * s);
        cd.fg = dalloc((size_t)cd.D * N * s);
        cd.totals = (double *)dalloc(8 * sizeof(double));
        cd.mask = nullptr;
        if (!cd.A || !cd.B || !cd.frho || !cd.fpsi || !cd.fg || !cd.totals) { free_batch(b); return bfail(nullptr, LBM_E_NOMEM, "device allocation failed"); }
        if (p.mask) {
            uint8_t *m = (uint8_t *)dalloc(N);
            if (!m || hipMemcpy(m, p.mask, N, hipMemcpyHostToDevice) != hipSuccess) { free_batch(b); return bfail(nullptr, LBM_E_HIP, "mask upload failed"); }
            cd.mask = m;
        }
        if (p.rho_wall_field) {   // per-node wall densities of this case
            void *w = cd.fp64 ? (void *)upload_wall_field<double>(p.rho_wall_field, cd.g)
                              : (void *)upload_wall_field<float>(p.rho_wall_field, cd.g);
            if (!w) { free_batch(b); return bfail(nullptr, LBM_E_NOMEM, "wall density upload failed"); }
            b->allocs.push_back(w);
            if (cd.fp64) cd.pd.rho_wf = (const double *)w;
            else cd.pf.rho_wf = (const float *)w;
        }
        b->params[c].mask = nullptr;
        b->params[c].rho_wall_field = nullptr;
        b->ks[c] = kernel_set(cd.D, cd.fp64, cd.mask != nullptr);
        b->nblk[c] = moment_block_count(cd.D, cd.g);
        max_nblk = std::max(max_nblk, b->nblk[c]);
        b->io_elems = std::max(b->io_elems, (size_t)(1 + cd.D) * N);
    }
    b->d_cases = (CaseDesc *)dalloc(ncases * sizeof(CaseDesc));
    b->d_order = (int *)dalloc(ncases * sizeof(int));
    b->d_parity = (int *)dalloc(ncases * sizeof(int));
    b->partials = (double *)dalloc((size_t)max_nblk * kPartialSlots * sizeof(double));
    b->d_tot = (double *)dalloc(8 * sizeof(double));
    b->io = (double *)dalloc(b->io_elems * sizeof(double));
    b->rscratch = (double *)dalloc((size_t)reduce_scratch_rows(max_nblk) * kPartialSlots * sizeof(double));
    if (!b->d_cases || !b->d_order || !b->d_parity || !b->partials || !b->d_tot || !b->io || !b->rscratch) { free_batch(b); return bfail(nullptr, LBM_E_NOMEM, "device allocation failed"); }
    // largest cases first: they bound the launch, so they are dispatched first
    std::vector<int> order(ncases);
    for (int c = 0; c < ncases; ++c) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        if (b->host[x].D != b->host[y].D) return b->host[x].D < b->host[y].D;   // D2Q9 cases first
        const double cx = double(b->host[x].g.N) * (b->host[x].fp64 ? 2 : 1);
        const double cy = double(b->host[y].g.N) * (b->host[y].fp64 ? 2 : 1);
        return cx > cy;
    });
    for (int c = 0; c < ncases; ++c) (b->host[c].D == 2 ? b->n2 : b->n3) += 1;
    // work lists of the stepped kernels, sized for the finest split (64 threads, one node each)
    b->order = order;
    for (int c : order) {
        const size_t nk = (size_t)std::max(1, (b->host[c].g.N + 63) / 64);
        (b->host[c].D == 2 ? b->cap2 : b->cap3) += nk;
    }
    for (int c : order)   // the tile list sized for the narrowest tiles (8 columns)
        if (b->host[c].D == 2) b->tcap += (size_t)(b->host[c].g.nx + 7) / 8;
    if ((b->tcap && !(b->d_tile = (TileWork *)dalloc(b->tcap * sizeof(TileWork)))) ||
        !(b->d_tiled = (int *)dalloc(ncases * sizeof(int))) ||
        !(b->d_bad = (int *)dalloc((size_t)ncases * kCheckBlocks * sizeof(int)))) {
        free_batch(b);
        return bfail(nullptr, LBM_E_NOMEM, "device allocation failed");
    }
    if (b->cap2 && !(b->d_work2 = (Work *)dalloc(b->cap2 * sizeof(Work)))) { free_batch(b); return bfail(nullptr, LBM_E_NOMEM, "device allocation failed"); }
    if (b->cap3 && !(b->d_work3 = (Work *)dalloc(b->cap3 * sizeof(Work)))) { free_batch(b); return bfail(nullptr, LBM_E_NOMEM, "device allocation failed"); }
    if (build_work(b, Split{256, 1})) { free_batch(b); return bfail(nullptr, LBM_E_HIP, "work list upload failed"); }
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            b->gfx = prop.gcnArchName;
            const size_t colon = b->gfx.find(':');
            if (colon != std::string::npos) b->gfx.resize(colon);
        }
        if (b->gfx.empty()) b->gfx = "unknown";
    }
    // LBM2P_BATCH_STEPPED=0: the persistent design (one workgroup per case)
    {
        const char *sv = getenv("LBM2P_BATCH_STEPPED");
        b->stepped = !(sv && atoi(sv) == 0);
    }
    std::vector<int> zero(ncases, 0);
    if (hipMemcpy(b->d_cases, b->host.data(), ncases * sizeof(CaseDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_order, order.data(), ncases * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_parity, zero.data(), ncases * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        free_batch(b);
        return bfail(nullptr, LBM_E_HIP, "descriptor upload failed");
    }
    // LBM2P_BATCH_CHUNK: steps per captured graph launch (default 200)
    const char *cs = getenv("LBM2P_BATCH_CHUNK");
    b->chunk = (cs && atoi(cs) > 0) ? atoi(cs) : 200;
    *out = b;
    return LBM_OK;
}

int lbm_batch_init_fields(lbm_batch *b, int icase, const double *rho, const double *u) {
    if (!b || !rho || icase < 0 || icase >= (int)b->host.size()) return bfail(b, LBM_E_INVAL, "bad argument");
    CaseDesc &cd = b->host[icase];
    const size_t N = (size_t)cd.g.N;
    for (size_t n = 0; n < N; ++n)
        if (!(rho[n] > 0.0) || !isfinite(rho[n])) return bfail(b, LBM_E_DOMAIN, "initial density must be finite and > 0");
    int parity = 0;
    BHIP(b, hipMemcpy(&parity, b->d_parity + icase, sizeof(int), hipMemcpyDeviceToHost));
    void *A = current_A(b, icase, parity);
    const void *prm = cd.fp64 ? (const void *)&cd.pd : (const void *)&cd.pf;
    BHIP(b, hipMemcpyAsync(b->io, rho, N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    if (u) BHIP(b, hipMemcpyAsync(b->io + N, u, cd.D * N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    const long long count = (long long)(cd.D == 3 ? 27 : 9) * cd.g.qs;
    b->ks[icase].fill_zero(b->stream, cd.A, count);
    b->ks[icase].fill_zero(b->stream, cd.B, count);
    b->ks[icase].init(b->stream, A, cd.g, cd.mask, prm, cd.frho, b->io, u ? b->io + N : nullptr);
    BHIP(b, hipGetLastError());
    BHIP(b, hipStreamSynchronize(b->stream));
    b->initialized[icase] = 1;
    return LBM_OK;
}

// Saves every case's current lattice (host copies) and its parity, to be restored after
// timed trial steps.
struct Saved {
    std::vector<std::vector<char>> pops;
    std::vector<int> par;
};

static int save_states(lbm_batch *b, Saved *sv) {
    sv->pops.resize(b->host.size());
    sv->par.resize(b->host.size());
    BHIP(b, hipMemcpy(sv->par.data(), b->d_parity, sv->par.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (size_t c = 0; c < b->host.size(); ++c) {
        const CaseDesc &cd = b->host[c];
        const size_t bytes = (size_t)(cd.D == 3 ? 27 : 9) * cd.g.qs * (cd.fp64 ? 8 : 4);
        sv->pops[c].resize(bytes);
        BHIP(b, hipMemcpy(sv->pops[c].data(), current_A(b, (int)c, sv->par[c]), bytes, hipMemcpyDeviceToHost));
    }
    return LBM_OK;
}

static int restore_states(lbm_batch *b, const Saved &sv) {
    BHIP(b, hipMemcpy(b->d_parity, sv.par.data(), sv.par.size() * sizeof(int), hipMemcpyHostToDevice));
    for (size_t c = 0; c < b->host.size(); ++c)
        BHIP(b, hipMemcpy(current_A(b, (int)c, sv.par[c]), sv.pops[c].data(), sv.pops[c].size(), hipMemcpyHostToDevice));
    return LBM_OK;
}

// wall time of `steps` directly launched steps of the current configuration
static int trial(lbm_batch *b, int steps, int block, double *sec) {
    BHIP(b, hipStreamSynchronize(b->stream));
    auto t0 = std::chrono::steady_clock::now();
    if (launch(b, steps, block)) return bfail(b, LBM_E_HIP, "trial launch failed");
    BHIP(b, hipStreamSynchronize(b->stream));
    *sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return LBM_OK;
}

// Picks the stepped design's block split, or the persistent design's workgroup size, once
// per batch: an environment override first (LBM2P_BATCH_SPLIT="threads,nodes" or
// LBM2P_BATCH_BLOCK), then the tuning cache, else timed trials of a few steps on the live
// state, which is restored afterwards (results never depend on the choice); a tuned choice
// is appended to the cache.
static int autotune(lbm_batch *b) {
    if (b->tuned) return LBM_OK;
    b->tuned = true;
    const int trial_steps = 20;
    if (b->stepped) {
        auto valid_split = [](int tpb, int npt) {
            for (const Split &sp : kSplits)
                if (sp.tpb == tpb && sp.npt == npt) return true;
            return false;
        };
        auto valid_tiles = [](int steps, int width, int lanes) {
            return steps >= 0 && steps <= 16 && width >= 32 && width <= 512 && width % 32 == 0 &&
                   (lanes == 64 || lanes == 128);
        };
        auto apply = [&](int tpb, int npt, int steps, int tx, int lanes) {
            return build_work(b, Split{tpb, npt}, steps, tx, lanes) ? bfail(b, LBM_E_HIP, "work list upload failed")
                                                                    : LBM_OK;
        };
        // environment overrides: LBM2P_BATCH_SPLIT="threads,nodes" and LBM2P_BATCH_TILE=
        // "steps,row width[,lanes]" (steps 0: no tiles); either one fixes the choice, the other
        // part taking its default
        int v[5] = {256, 1, 0, 128, 64};
        const char *es = getenv("LBM2P_BATCH_SPLIT"), *et = getenv("LBM2P_BATCH_TILE");
        bool fixed = false;
        if (es && sscanf(es, "%d,%d", &v[0], &v[1]) == 2 && valid_split(v[0], v[1])) fixed = true;
        else { v[0] = 256; v[1] = 1; }
        v[4] = 64;
        if (et && sscanf(et, "%d,%d,%d", &v[2], &v[3], &v[4]) >= 2 && valid_tiles(v[2], v[3], v[4])) fixed = true;
        else { v[2] = 0; v[3] = 128; v[4] = 64; }
        if (fixed) return apply(v[0], v[1], v[2], v[3], v[4]);
        if (cache_lookup(b, 's', v) && valid_split(v[0], v[1]) && valid_tiles(v[2], v[3], v[4]))
            return apply(v[0], v[1], v[2], v[3], v[4]);
        Saved sv;
        int rc = save_states(b, &sv);
        if (rc) return rc;
        auto time_config = [&](Split sp, int steps, int tx, int lanes, double *t) {
            if (build_work(b, sp, steps, tx, lanes)) return bfail(b, LBM_E_HIP, "work list upload failed");
            int r;
            if ((r = trial(b, 2, b->block, t)) || (r = trial(b, trial_steps, b->block, t))) return r;
            return LBM_OK;
        };
        // first the tiling (steps per launch, tile row width, lanes) with the default split, then
        // the split of the cases left to the stepped kernels
        const int tilings[][3] = {{0, 128, 64}, {3, 64, 64},  {4, 64, 64},   {3, 128, 64},  {4, 128, 64},
                                  {5, 128, 64}, {4, 192, 64}, {6, 192, 64},  {4, 128, 128}, {8, 256, 64},
                                  {8, 256, 128}};
        int bs = 0, btx = 128, bl = 64;
        double best_t = 1e30;
        for (const auto &tl : tilings) {
            double t = 0.0;
            if ((rc = time_config(kSplits[0], tl[0], tl[1], tl[2], &t))) return rc;
            if (t < best_t) { best_t = t; bs = tl[0]; btx = tl[1]; bl = tl[2]; }
        }
        Split best = kSplits[0];
        if ((rc = build_work(b, best, bs, btx, bl))) return bfail(b, LBM_E_HIP, "work list upload failed");
        if (b->nw2 || b->nw3)
            for (const Split &sp : kSplits) {
                double t = 0.0;
                if ((rc = time_config(sp, bs, btx, bl, &t))) return rc;
                if (t < best_t) { best_t = t; best = sp; }
            }
        if ((rc = restore_states(b, sv))) return rc;
        if ((rc = apply(best.tpb, best.npt, bs, btx, bl))) return rc;
        const int chosen[5] = {best.tpb, best.npt, bs, btx, bl};
        std::lock_guard<std::mutex> lk(g_tune_mu);
        cache_store(b, 's', chosen);
        return LBM_OK;
    }
    // LBM2P_BATCH_BLOCK: a fixed workgroup size, a multiple of 64 up to 1024 (others are ignored)
    const char *env = getenv("LBM2P_BATCH_BLOCK");
    const int fixed = env ? atoi(env) : 0;
    if (fixed >= 64 && fixed <= 1024 && fixed % 64 == 0) { b->block = fixed; return LBM_OK; }
    const std::string sig = signature(b);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(sig);
        if (it != g_tune_cache.end()) { b->block = it->second; return LBM_OK; }
    }
    int pv[5] = {0, 0, 0, 0, 0};
    if (cache_lookup(b, 'p', pv) && pv[0] >= 64 && pv[0] <= 1024 && pv[0] % 64 == 0) {
        b->block = pv[0];
        return LBM_OK;
    }
    Saved sv;
    int rc = save_states(b, &sv);
    if (rc) return rc;
    int best = 256;
    double best_t = 1e30;
    for (int blk : {256, 512, 1024}) {
        double t = 0.0;
        if ((rc = trial(b, trial_steps, blk, &t))) return rc;
        if (t < best_t) { best_t = t; best = blk; }
    }
    if ((rc = restore_states(b, sv))) return rc;
    b->block = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[sig] = best;
    const int chosen[5] = {best, 0, 0, 0, 0};
    cache_store(b, 'p', chosen);
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t n) {
    if (!b || n < 0) return bfail(b, LBM_E_INVAL, "bad argument");
    for (size_t c = 0; c < b->host.size(); ++c)
        if (!b->initialized[c]) return bfail(b, LBM_E_STATE, "case " + std::to_string(c) + " not initialised");
    if (n == 0) return LBM_OK;
    if (!b->exec) {
        int rc = autotune(b);
        if (rc) return rc;
        BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        if (launch(b, b->chunk, b->block)) {
            hipGraph_t g;
            (void)hipStreamEndCapture(b->stream, &g);
            return bfail(b, LBM_E_HIP, "capture failed");
        }
        BHIP(b, hipStreamEndCapture(b->stream, &b->graph));
        BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    int64_t left = n;
    while (left >= b->chunk) {
        BHIP(b, hipGraphLaunch(b->exec, b->stream));
        left -= b->chunk;
    }
    if (left > 0 && launch(b, (int)left, b->block)) return bfail(b, LBM_E_HIP, "launch failed");
    // divergence check of every case in one pass: non-finite stored populations
    const int nc = (int)b->host.size();
    hipLaunchKernelGGL(k_batch_nonfinite, dim3((unsigned)(kCheckBlocks * nc)), dim3(256), 0, b->stream, b->d_cases,
                       b->d_parity, b->d_bad);
    BHIP(b, hipGetLastError());
    std::vector<int> bad((size_t)nc * kCheckBlocks);
    BHIP(b, hipMemcpyAsync(bad.data(), b->d_bad, bad.size() * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    for (int c = 0; c < nc; ++c) {
        long long nb = 0;
        for (int k = 0; k < kCheckBlocks; ++k) nb += bad[(size_t)c * kCheckBlocks + k];
        if (nb) return bfail(b, LBM_E_DIVERGED, "case " + std::to_string(c) + " diverged (" + std::to_string(nb) +
                                                    " non-finite populations)");
    }
    return LBM_OK;
}

int lbm_batch_moments(lbm_batch *b, int icase, double *rho, double *U, double totals[4]) {
    if (!b || icase < 0 || icase >= (int)b->host.size()) return bfail(b, LBM_E_INVAL, "bad argument");
    CaseDesc &cd = b->host[icase];
    int parity = 0;
    BHIP(b, hipMemcpy(&parity, b->d_parity + icase, sizeof(int), hipMemcpyDeviceToHost));
    void *A = current_A(b, icase, parity);
    const void *prm = cd.fp64 ? (const void *)&cd.pd : (const void *)&cd.pf;
    const size_t N = (size_t)cd.g.N;
    // the two-pass moment kernel refreshes rho and g in the case's fields and writes partials
    b->ks[icase].moments(b->stream, A, cd.g, cd.mask, prm, cd.frho, cd.fg, b->partials);
    launch_reduce(b->stream, b->partials, b->nblk[icase], b->rscratch, b->d_tot);
    double t[5];
    BHIP(b, hipMemcpyAsync(t, b->d_tot, 5 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (rho || U) {
        b->ks[icase].output(b->stream, A, cd.g, cd.mask, prm, cd.frho, cd.fg, b->io, b->io + N);
        if (rho) BHIP(b, hipMemcpyAsync(rho, b->io, N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        if (U) BHIP(b, hipMemcpyAsync(U, b->io + N, cd.D * N * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    BHIP(b, hipGetLastError());
    BHIP(b, hipStreamSynchronize(b->stream));
    if (totals) for (int k = 0; k < 4; ++k) totals[k] = t[k];
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_batch(b);
}

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

int lbm_batch_layout(const lbm_batch *b, int out[6]) {
    if (!b || !out) return LBM_E_INVAL;
    out[0] = b->stepped ? 1 : 0;
    out[1] = b->stepped ? b->split.tpb : b->block;
    out[2] = b->stepped ? b->split.npt : 0;
    out[3] = b->stepped ? b->tile_steps : 0;
    out[4] = b->stepped && b->tile_steps ? b->tile_tx : 0;
    out[5] = b->stepped && b->tile_steps ? b->nt : 0;
    return LBM_OK;
}

}  // extern "C"
