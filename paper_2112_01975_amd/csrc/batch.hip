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
// phase 1 at node n: rho, signed psi and g = rho u^3 of the state in A into the case's fields
template <int D, class S, class C>
__device__ __forceinline__ void phase1_node(const CaseDesc &cd, const Params<C> &p, const S *A, int n) {
    constexpr int Q = Lat<D>::Q;
    const Geom &g = cd.g;
    const uint8_t *mask = cd.mask;
    C *frho = (C *)cd.frho, *fpsi = (C *)cd.fpsi, *fg = (C *)cd.fg;
    const int x = n % g.nx, t = n / g.nx, y = t % g.ny, z = t / g.ny;
    C rho, ga[3] = {C(0), C(0), C(0)};
    if (mask && mask[n]) {
        rho = wall_density(p, n);
    } else {
        C h[Q];
        if (mask)
            gather<D, S, C, true>(A, g.qs, mask, Nbr<D>(g, x, y, z), n, h);
        else
            gather<D, S, C, false>(A, g.qs, mask, Nbr<D>(g, x, y, z), n, h);
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
    frho[n] = rho;
    fpsi[n] = signed_psi(p.eos, rho);
#pragma unroll
    for (int a = 0; a < D; ++a) fg[a * g.N + n] = ga[a];
}

// phase 2 at fluid node n: force from the fields, correction, equilibria, LBGK; A -> B
template <int D, class S, class C>
__device__ __forceinline__ void phase2_node(const CaseDesc &cd, const Params<C> &p, const S *A, S *B, int n) {
    constexpr int Q = Lat<D>::Q;
    const Geom &g = cd.g;
    const uint8_t *mask = cd.mask;
    const C *frho = (const C *)cd.frho, *fpsi = (const C *)cd.fpsi, *fg = (const C *)cd.fg;
    if (mask && mask[n]) return;
    const int x = n % g.nx, t = n / g.nx, y = t % g.ny, z = t / g.ny;
    const Nbr<D> nb(g, x, y, z);
    const C rho = frho[n], spc = fpsi[n];
    C Fp[3] = {C(0), C(0), C(0)}, Fc[3] = {C(0), C(0), C(0)};
    static_for<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
        constexpr int cls = cx * cx + cy * cy + cz * cz - 1;   // weight class of c_i
        const int n1 = nb.at(cx, cy, cz);
        const int x2 = wrapi(x + 2 * cx, g.nx), y2 = wrapi(y + 2 * cy, g.ny);
        const int z2 = D == 3 ? wrapi(z + 2 * cz, g.nz) : 0;
        const int n2 = x2 + g.nx * (y2 + g.ny * z2);
        const C p1 = fabs(fpsi[n1]), p2 = fabs(fpsi[n2]);
        const C r1 = frho[n1], r2 = frho[n2];
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
    if (mask)
        gather<D, S, C, true>(A, g.qs, mask, nb, n, h);
    else
        gather<D, S, C, false>(A, g.qs, mask, nb, n, h);
    C drho, j[3];
    moments_of<D, C>(h, drho, j);
    const C rinv = rcp(rho);
    C u[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] = j[a] * rinv;
    const C omega = omega_of(p, rho);
    const C cf = (C(1) - C(0.5) * omega) * C(0.5);
    C Phi[3] = {C(0), C(0), C(0)};
    Phi[0] = cf * (fg[nb.at(1, 0, 0)] - fg[nb.at(-1, 0, 0)]);
    Phi[1] = cf * (fg[g.N + nb.at(0, 1, 0)] - fg[g.N + nb.at(0, -1, 0)]);
    if constexpr (D == 3) Phi[2] = cf * (fg[2 * g.N + nb.at(0, 0, 1)] - fg[2 * g.N + nb.at(0, 0, -1)]);
    collide<D, C>(h, rho, drho, u, Sf, Phi, omega);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        st_at(B + i * g.qs, (unsigned)n, S(h[i]));
    });
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
__global__ void k_flip_parity(int *parity, int ncases, int nsteps) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncases) parity[c] = (parity[c] + nsteps) & 1;
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
    if (b->stepped) {
        for (int st = 0; st < nsteps; ++st) {
            launch_phase<1>(b, st);   // every case's phase 1 before any phase 2 (stream order)
            launch_phase<2>(b, st);
        }
        if (nsteps & 1)
            hipLaunchKernelGGL(k_flip_parity, dim3((nc + 255) / 256), dim3(256), 0, b->stream, b->d_parity, nc, nsteps);
        return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
    }
    if (b->n2)
        hipLaunchKernelGGL(k_batch<2>, dim3(b->n2), dim3(block), 0, b->stream, b->d_cases, b->d_order, nc, nsteps,
                           b->d_parity);
    if (b->n3)
        hipLaunchKernelGGL(k_batch<3>, dim3(b->n3), dim3(block < 256 ? block : 256), 0, b->stream, b->d_cases, b->d_order + b->n2, nc,
                           nsteps, b->d_parity);
    if (nsteps & 1) hipLaunchKernelGGL(k_flip_parity, dim3((nc + 255) / 256), dim3(256), 0, b->stream, b->d_parity, nc, nsteps);
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

// Work lists of the stepped kernels for the split sp: each case in blocks of tpb npt nodes,
// largest case first; uploaded into the lists allocated for the finest split
int build_work(lbm_batch *b, Split sp) {
    std::vector<Work> w2, w3;
    const int per = sp.tpb * sp.npt;
    for (int c : b->order) {
        const int nk = std::max(1, (int)((b->host[c].g.N + per - 1) / per));
        for (int k = 0; k < nk; ++k) (b->host[c].D == 2 ? w2 : w3).push_back(Work{c, k, nk});
    }
    if (w2.size() > b->cap2 || w3.size() > b->cap3) return LBM_E_INVAL;
    if ((!w2.empty() && hipMemcpy(b->d_work2, w2.data(), w2.size() * sizeof(Work), hipMemcpyHostToDevice) != hipSuccess) ||
        (!w3.empty() && hipMemcpy(b->d_work3, w3.data(), w3.size() * sizeof(Work), hipMemcpyHostToDevice) != hipSuccess))
        return LBM_E_HIP;
    b->nw2 = (int)w2.size();
    b->nw3 = (int)w3.size();
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
//   <gfx target> <signature hash> <design: s | p> <a> <b>
// stepped: a = threads per block, b = nodes per thread; persistent: a = workgroup size.
bool cache_lookup(const lbm_batch *b, char design, int *a, int *bb) {
    const char *path = getenv("LBM2P_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    const std::string key = sig_hash(signature(b));
    char gfx[128], h[64], d[8];
    int x = 0, y = 0;
    bool found = false;
    while (fscanf(f, "%127s %63s %7s %d %d", gfx, h, d, &x, &y) == 5)
        if (b->gfx == gfx && key == h && d[0] == design) {
            *a = x;
            *bb = y;
            found = true;   // the last entry for a key wins
        }
    fclose(f);
    return found;
}

void cache_store(const lbm_batch *b, char design, int a, int bb) {
    const char *path = getenv("LBM2P_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %s %c %d %d\n", b->gfx.c_str(), sig_hash(signature(b)).c_str(), design, a, bb);
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
        int a = 0, nb = 0;
        const char *env = getenv("LBM2P_BATCH_SPLIT");
        if (env && sscanf(env, "%d,%d", &a, &nb) == 2) {
            for (const Split &sp : kSplits)
                if (sp.tpb == a && sp.npt == nb) return build_work(b, sp) ? bfail(b, LBM_E_HIP, "work list upload failed") : LBM_OK;
        }
        if (cache_lookup(b, 's', &a, &nb))
            for (const Split &sp : kSplits)
                if (sp.tpb == a && sp.npt == nb) return build_work(b, sp) ? bfail(b, LBM_E_HIP, "work list upload failed") : LBM_OK;
        Saved sv;
        int rc = save_states(b, &sv);
        if (rc) return rc;
        Split best = kSplits[0];
        double best_t = 1e30;
        for (const Split &sp : kSplits) {
            if (build_work(b, sp)) return bfail(b, LBM_E_HIP, "work list upload failed");
            double t = 0.0;
            if ((rc = trial(b, 2, b->block, &t)) || (rc = trial(b, trial_steps, b->block, &t))) return rc;
            if (t < best_t) { best_t = t; best = sp; }
        }
        if ((rc = restore_states(b, sv))) return rc;
        if (build_work(b, best)) return bfail(b, LBM_E_HIP, "work list upload failed");
        std::lock_guard<std::mutex> lk(g_tune_mu);
        cache_store(b, 's', best.tpb, best.npt);
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
    int a = 0, nb = 0;
    if (cache_lookup(b, 'p', &a, &nb) && a >= 64 && a <= 1024 && a % 64 == 0) {
        b->block = a;
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
    cache_store(b, 'p', best, 0);
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
    BHIP(b, hipStreamSynchronize(b->stream));
    // FP64 watchdog over every case
    for (size_t c = 0; c < b->host.size(); ++c) {
        double t[4];
        int rc = lbm_batch_moments(b, (int)c, nullptr, nullptr, t);
        if (rc) return rc;
        if (!isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2]) || !isfinite(t[3]))
            return bfail(b, LBM_E_DIVERGED, "case " + std::to_string(c) + " diverged");
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

}  // extern "C"
