// fused_kernels.hip -- single-pass D3Q27 stream-collide step with a z-march (gfx950).
//
// One workgroup owns a TX x TY column tile of (x, y) and marches over a chunk of
// TZ planes in z. Each plane p is pulled once: the 27 populations of every tile
// node, plus rho / g of a two-node halo ((TX + 4) x (TY + 4) nodes), give rho, the
// signed pseudo-potential (eq force_form) and g = rho u^3; rho and s*psi go into a
// six-plane LDS ring, g into registers (z difference) and a double-buffered LDS
// plane (x, y differences). Plane z is collided once planes z-2..z+2 are resident:
// the two-ring Korteweg force (eq Kforce_final) comes from the ring, the diagonal
// correction (eq correction) from g, and the populations from a register queue,
// so every population crosses HBM once in each direction (2 Q s bytes per lattice update plus the chunk's z halo).
//
// In FP32 on grids without solid nodes the FP64 mass and momentum totals of the input
// state ride along: each thread adds the moments of the tile nodes it collides as they are staged, and
// each work item leaves one row of partial sums (wave shuffles, then LDS) for the watchdog's
// reduction tree.
//
// Software pipeline, one barrier per plane: while plane z is collided, the
// population registers of plane z are refilled with the pulls of plane z+3 as soon
// as each collided value is stored, and the halo pulls of plane z+3 are in flight
// during the stencil. The three queue planes are renamed by unrolling the march by
// three instead of being moved.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "fused.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "step_common.hpp"

namespace lbm {

namespace {

constexpr int NXCD = 8;   // MI355X: 8 XCDs, workgroups dispatched round-robin

// Cache policy of the population stores: non-temporal. The lattice written in a step is not
// read again in that step, and streaming its lines through L2 leaves the room to the lines
// that neighbouring tiles share (x edges, y halo) between their reads.
constexpr int STORE_NT = 2;

// Populations the FP64 unmasked step keeps in LDS for three planes instead of pulling them
// again when the plane is collided: the first NQ in library order with c_x and c_z nonzero
// (row-misaligned pulls from the neighbouring planes: (1,0,+-1), (1,1,+-1)). NQ is what the LDS left
// beside the rho / psi ring and the g planes holds (3 NQ x 512 doubles = 48 KB).
constexpr int NQ = 4;
constexpr int queued(int q) {
    for (int i = 1; i < 27; ++i)
        if (Lat<3>::c(i, 0) != 0 && Lat<3>::c(i, 2) != 0 && q-- == 0) return i;
    return -1;
}
constexpr bool is_queued(int i) {
    for (int q = 0; q < NQ; ++q)
        if (queued(q) == i) return true;
    return false;
}

// library index of the velocity (cx, cy, cz)
constexpr int index3(int cx, int cy, int cz) {
    for (int i = 0; i < 27; ++i)
        if (Lat<3>::c(i, 0) == cx && Lat<3>::c(i, 1) == cy && Lat<3>::c(i, 2) == cz) return i;
    return -1;
}

// Addresses of one node's pull stencil as byte offsets into a population lattice:
// v[a][b] = offset of the node at (x + a - 1, y + b - 1) in its plane (per lane, fixed
// for the whole march), zs[l] = offset of plane z + l - 1 (uniform). Population i
// of node (x, y, z) is pulled from (x, y, z) - c_i at v[1 - cx][1 - cy] + zs[1 - cz] +
// i * qs * sizeof(S); the uniform part goes into the scalar offset of the load.
struct Stencil {
    unsigned v[3][3];
};

// One population lattice through one buffer resource (lattices below 4 GiB). Same
// interface as Lattice2; a bounce-back pull is one load at a per-lane offset.
template <class S> struct Lattice1 {
    __amdgpu_buffer_rsrc_t r;
    unsigned qsb;
    __device__ __forceinline__ Lattice1(const S *base, long long qs, bool null)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(base), (short)0,
                                              null ? 0 : (int)(unsigned)(27 * qs * (long long)sizeof(S)), 0x00020000)),
          qsb((unsigned)(qs * (long long)sizeof(S))) {}
    template <int i> __device__ __forceinline__ S load(unsigned voff, unsigned soff) const {
        return raw_load(voff, soff + (unsigned)i * qsb);
    }
    // population i from (voff, soff), or population opp(i) of the node itself at (vself,
    // sself) where solid is set
    template <int i> __device__ __forceinline__ S load_or_bounce(bool solid, unsigned voff, unsigned soff, unsigned vself,
                                                               unsigned sself) const {
        const unsigned off = solid ? vself + sself + (unsigned)opp<3>(i) * qsb : voff + soff + (unsigned)i * qsb;
        return raw_load(off, 0u);
    }
    template <int i> __device__ __forceinline__ void store(unsigned voff, unsigned soff, S v) const {
        if constexpr (sizeof(S) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff + (unsigned)i * qsb, STORE_NT);
        } else {
            using u2 = unsigned __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff + (unsigned)i * qsb, STORE_NT);
        }
    }
    __device__ __forceinline__ S raw_load(unsigned voff, unsigned soff) const {
        if constexpr (sizeof(S) == 4) return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
        else return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
};

// One population lattice through two buffer resources, populations [0, SPLIT) and
// [SPLIT, 27): each part stays below the 4 GiB reach of a resource (an FP64 lattice of
// 33.5 M nodes is 7.2 GB). The population index is a compile-time constant at every
// access, so the choice of resource costs nothing. voff: per-lane byte offset of the
// node in its plane; soff: uniform byte offset of the plane. A zero-extent view (null)
// returns 0 for every load without touching memory.
template <class S> struct Lattice2 {
    static constexpr int SPLIT = 14;
    __amdgpu_buffer_rsrc_t r0, r1;
    unsigned qsb;   // qs * sizeof(S): bytes between two populations
    __device__ __forceinline__ Lattice2(const S *base, long long qs, bool null)
        : r0(__builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(base), (short)0,
                                               null ? 0 : (int)(unsigned)(SPLIT * qs * (long long)sizeof(S)), 0x00020000)),
          r1(__builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(base) + SPLIT * qs, (short)0,
                                               null ? 0 : (int)(unsigned)((27 - SPLIT) * qs * (long long)sizeof(S)),
                                               0x00020000)),
          qsb((unsigned)(qs * (long long)sizeof(S))) {}
    template <int i> __device__ __forceinline__ S load(unsigned voff, unsigned soff) const {
        if constexpr (i < SPLIT) return raw_load(r0, voff, soff + (unsigned)i * qsb);
        else return raw_load(r1, voff, soff + (unsigned)(i - SPLIT) * qsb);
    }
    // i and opp(i) sit in different resources: both are loaded and one is kept
    template <int i> __device__ __forceinline__ S load_or_bounce(bool solid, unsigned voff, unsigned soff, unsigned vself,
                                                               unsigned sself) const {
        const S f = load<i>(voff, soff);
        const S b = load<opp<3>(i)>(vself, sself);
        return solid ? b : f;
    }
    template <int i> __device__ __forceinline__ void store(unsigned voff, unsigned soff, S v) const {
        if constexpr (i < SPLIT) raw_store(r0, voff, soff + (unsigned)i * qsb, v);
        else raw_store(r1, voff, soff + (unsigned)(i - SPLIT) * qsb, v);
    }
    static __device__ __forceinline__ S raw_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        if constexpr (sizeof(S) == 4) return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
        else return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void raw_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, S v) {
        if constexpr (sizeof(S) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, STORE_NT);
        } else {
            using u2 = unsigned __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, STORE_NT);
        }
    }
};

// One population lattice through K = ceil(27 / P) buffer resources of P populations each,
// for lattices past the 8 GiB of two resources: population i is in resource i / P at
// byte offset (i mod P) qs sizeof(S) + soff + voff, which stays below 4 GiB while P
// population arrays do. The resource index is a compile-time constant at every access;
// a bounce-back whose two populations sit in different resources loads both and keeps
// one. A zero-extent view (null) returns 0 for every load without touching memory.
template <class S, int P> struct LatticeK {
    static constexpr int K = (27 + P - 1) / P;
    __amdgpu_buffer_rsrc_t r[K];
    unsigned qsb;
    __device__ __forceinline__ LatticeK(const S *base, long long qs, bool null) : qsb((unsigned)(qs * (long long)sizeof(S))) {
        static_for<0, K>([&](auto Kk) {
            constexpr int k = decltype(Kk)::value;
            constexpr int n = (k + 1) * P <= 27 ? P : 27 - k * P;
            r[k] = __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(base) + (long long)k * P * qs, (short)0,
                                                     null ? 0 : (int)(unsigned)(n * qs * (long long)sizeof(S)),
                                                     0x00020000);
        });
    }
    template <int i> __device__ __forceinline__ S load(unsigned voff, unsigned soff) const {
        return Lattice2<S>::raw_load(r[i / P], voff, soff + (unsigned)(i % P) * qsb);
    }
    template <int i> __device__ __forceinline__ S load_or_bounce(bool solid, unsigned voff, unsigned soff, unsigned vself,
                                                               unsigned sself) const {
        constexpr int o = opp<3>(i);
        if constexpr (i / P == o / P) {
            const unsigned off = solid ? vself + sself + (unsigned)(o % P) * qsb : voff + soff + (unsigned)(i % P) * qsb;
            return Lattice2<S>::raw_load(r[i / P], off, 0u);
        } else {
            const S f = load<i>(voff, soff);
            const S b = load<o>(vself, sself);
            return solid ? b : f;
        }
    }
    template <int i> __device__ __forceinline__ void store(unsigned voff, unsigned soff, S v) const {
        Lattice2<S>::raw_store(r[i / P], voff, soff + (unsigned)(i % P) * qsb, v);
    }
};

// Solid-neighbour bits of a node (built once per geometry by k_links): bit i is set
// when the source node r - c_i of population i is solid, bit LINK_SELF when r is.
constexpr int LINK_SELF = 27;

template <int i, class S, class C, bool MASK, class LT>
__device__ __forceinline__ C pull(const LT &A, uint32_t lm, const Stencil &st, const unsigned (&zs)[3]) {
    constexpr int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
    const unsigned vo = st.v[1 - cx][1 - cy];
    if constexpr (MASK && i != 0) {
        // halfway bounce-back: from a solid source node take the opposite population
        // that this node produced itself (only planes that touch a solid come here)
        return C(A.template load_or_bounce<i>((lm >> i) & 1u, vo, zs[1 - cz], st.v[1][1], zs[1]));
    } else {
        return C(A.template load<i>(vo, zs[1 - cz]));
    }
}

// Interpolated bounce-back over the pulled populations h of the node at stencil st in
// plane zs[1] (links lm): a pull across a wall link returned A_opp(i) of the node itself
// (halfway); with the link's wall fraction q (lq, [Q][qs], stored under opp(i)) it
// becomes the linear interpolation of Bouzidi et al. used for curved walls (Sec. 4.5,
// 5.3): q < 1/2 mixes in A_opp(i) of the node n + c_i behind (unless that node is
// solid), q >= 1/2 mixes in A_i of the node itself. Lanes without wall links skip it.
// k-th link (k = 0.., rest excluded) with z component cz, in library order
constexpr int zlink(int cz, int k) {
    for (int i = 1; i < 27; ++i)
        if (Lat<3>::c(i, 2) == cz && k-- == 0) return i;
    return -1;
}

// Links go in three groups by c_z (a floor or ceiling node only crosses one of them)
// without branches inside a group: the fractions and the partner values of a group (the
// partner's address chosen per lane by the precomputed bit qlo_i = (q < 1/2)) are loaded
// together and then selected, so a wall node waits for one load latency per group it
// needs instead of two per link; a group no lane of the wave needs is skipped.
template <class S, class C, int CZ, class LT>
__device__ __forceinline__ void interp_group(const LT &A, const C *__restrict__ lq, long long qs, unsigned n,
                                             uint32_t lm, uint32_t qlo, const Stencil &st, const unsigned (&zs)[3],
                                             C (&h)[27]) {
    constexpr int K = CZ == 0 ? 8 : 9;
    constexpr uint32_t gmask = [] {
        uint32_t m = 0;
        for (int k = 0; k < K; ++k) m |= 1u << zlink(CZ, k);
        return m;
    }();
    if (!(lm & gmask)) return;
    C qv[K], xv[K];
    static_for<0, K>([&](auto I) {
        constexpr int k = decltype(I)::value, i = zlink(CZ, k), o = opp<3>(i);
        constexpr int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
        qv[k] = lq[(long long)o * qs + n];
        // population o of n + c_i, or (q >= 1/2) population opp(o) = i of n itself
        xv[k] = C(A.template load_or_bounce<o>(!((qlo >> i) & 1u), st.v[1 + cx][1 + cy], zs[1 + cz], st.v[1][1],
                                               zs[1]));
    });
    static_for<0, K>([&](auto I) {
        constexpr int k = decltype(I)::value, i = zlink(CZ, k), o = opp<3>(i);
        const C q = qv[k], back = h[i], x = xv[k];
        const C h2q = C(2) * q;
        const C lo = ((lm >> o) & 1u) ? back : h2q * back + (C(1) - h2q) * x;
        const C hi = back / h2q + (C(1) - C(1) / h2q) * x;
        if ((lm >> i) & 1u) h[i] = ((qlo >> i) & 1u) ? lo : hi;
    });
}

template <class S, class C, class LT>
__device__ __forceinline__ void interp_walls(const LT &A, const C *__restrict__ lq, long long qs, uint32_t lm,
                                             uint32_t qlo, const Stencil &st, const unsigned (&zs)[3], C (&h)[27]) {
    if (!(lm & ((1u << 27) - 2u))) return;
    const unsigned n = (st.v[1][1] + zs[1]) / (unsigned)sizeof(S);
    interp_group<S, C, 1>(A, lq, qs, n, lm, qlo, st, zs, h);
    interp_group<S, C, 0>(A, lq, qs, n, lm, qlo, st, zs, h);
    interp_group<S, C, -1>(A, lq, qs, n, lm, qlo, st, zs, h);
}

template <class S, class C, bool MASK, class LT>
__device__ __forceinline__ void pull_all(const LT &A, uint32_t lm, const Stencil &st, const unsigned (&zs)[3],
                                         C (&h)[27]) {
    static_for<0, 27>([&](auto I) {
        constexpr int i = decltype(I)::value;
        h[i] = pull<i, S, C, MASK>(A, lm, st, zs);
    });
}

template <class S, class C, bool MASK, int FTX, int TY, bool REPULL, int LAT, bool INTERP>
__global__ __launch_bounds__(FTX * TY) void k_fused3(const S *__restrict__ A, S *__restrict__ B, Geom g,
                                                      FusedMask fm, Params<C> p, FusedGrid fg) {
    constexpr int NT = FTX * TY;
    constexpr int HX = FTX + 4, HY = TY + 4, HP = HX * HY;
    constexpr int NHALO = HP - FTX * TY;
    constexpr int RING = 6;
    constexpr unsigned SB = sizeof(S);
    __shared__ C s_rho[RING * HP];
    __shared__ C s_psi[RING * HP];
    __shared__ C s_gxy[2][2][HP];
    // FP64 unmasked: NQ populations of the own node kept for three planes in LDS instead of
    // re-pulled at collide time. Slot k % 3 holds plane z0 + k, written when that plane is
    // pulled for staging and read when it is collided; each thread reads and writes only
    // its own entries, so no barrier orders them.
    constexpr bool LQ = REPULL && !MASK;
    __shared__ C s_q[LQ ? 3 * NQ * NT : 1];

    // XCD-aware work item: consecutive items on one XCD are spatial neighbours
    const int b = blockIdx.x;
    const int local = (b % NXCD) * fg.per_xcd + b / NXCD;
    if (local >= fg.count) return;
    const int item = fg.item0 + local;
    const int tix = item % fg.ntx;
    const int rest = item / fg.ntx;
    const int tiy = rest % fg.nty;
    const int zc = rest / fg.nty;
    const int x0 = tix * FTX, y0 = tiy * TY, z0 = fg.zb + zc * fg.tz;
    const int tzi = min(fg.tz, fg.ze - z0);   // planes this item collides (the range's last chunk is ragged)

    // lattice view: one buffer resource (LAT 0), two past 4 GiB (1), and past 8 GiB groups
    // of four (FP32) or two (FP64) populations per resource (2)
    using LT = std::conditional_t<LAT == 2, LatticeK<S, sizeof(S) == 4 ? 4 : 2>,
                                  std::conditional_t<LAT == 1, Lattice2<S>, Lattice1<S>>>;
    const LT Ab(A, g.qs, false), Bb(B, g.qs, false);
    // a zero-extent view of A: loads through it return 0 without touching memory
    const LT Anull(A, g.qs, true);
    const int t = threadIdx.x;
    const int tx = t & (FTX - 1), ty = t / FTX;
    const int e_int = (ty + 2) * HX + tx + 2;
    const bool own = (x0 + tx < g.nx) && (y0 + ty < g.ny);
    const int nxy = g.px * g.ny;   // plane stride (rows pitched)
    auto stencil_of = [&](int x, int y, Stencil &st) __attribute__((always_inline)) {
        const int gx = wrapi(x, g.nx), gy = wrapi(y, g.ny);
        const int xs[3] = {wrapi(gx - 1, g.nx), gx, wrapi(gx + 1, g.nx)};
        const int ry[3] = {g.px * wrapi(gy - 1, g.ny), g.px * gy, g.px * wrapi(gy + 1, g.ny)};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) st.v[a][c] = (unsigned)(xs[a] + ry[c]) * SB;
    };
    // this thread's tile node and the (at most one) halo node it stages: rows 0, 1,
    // TY+2, TY+3, then columns 0, 1, HX-2, HX-1 of the staged plane
    Stencil si, sh;
    stencil_of(x0 + tx, y0 + ty, si);
    static_assert(NHALO <= NT, "one halo node per thread at most");
    const bool has_halo = t < NHALO;
    int e_halo = 0;
    {
        int lx = 0, ly = 0;
        if (t < 4 * HX) {
            const int r = t / HX;
            lx = t % HX;
            ly = r < 2 ? r : TY + r;
        } else if (has_halo) {
            const int q = t - 4 * HX, c4 = q % 4;
            ly = 2 + q / 4;
            lx = c4 < 2 ? c4 : FTX + c4;
        }
        e_halo = ly * HX + lx;
        stencil_of(x0 - 2 + lx, y0 - 2 + ly, sh);
    }

    // register windows: gz of planes z-1..z+2, dgx/dgy of planes z..z+2
    C gz_m1 = C(0), gz_0 = C(0), gz_p1 = C(0), gz_p2 = C(0);
    C dgx_0 = C(0), dgx_p1 = C(0), dgx_p2 = C(0);
    C dgy_0 = C(0), dgy_p1 = C(0), dgy_p2 = C(0);
    // populations this thread pulled for planes z, z+1, z+2 and their (sum h, j). REPULL
    // (FP64: three queued planes do not fit in registers) keeps only the moments and pulls
    // plane z again when it is collided.
    C q0[27], q1[REPULL ? 1 : 27], q2[REPULL ? 1 : 27];
    C m0[4], m1[4], m2[4];
    // FP64 totals of the tile nodes this thread collides: mass, momentum, and the count of
    // densities outside the EOS domain. Only the unmasked FP32 kernels keep them: in the
    // others the nine registers cost spills (the FP64 step 4% of its time), and their checks
    // run the moment pass.
    constexpr bool TOT = !MASK && sizeof(C) == 4;
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    int bad = 0;

    // byte offsets of planes pz-1, pz, pz+1 (any integer pz)
    auto planes = [&](int pz, unsigned (&zs)[3]) __attribute__((always_inline)) {
        zs[0] = (unsigned)(nxy * wrapi(pz - 1, g.nz)) * SB;
        zs[1] = (unsigned)(nxy * wrapi(pz, g.nz)) * SB;
        zs[2] = (unsigned)(nxy * wrapi(pz + 1, g.nz)) * SB;
    };
    // solid-neighbour bits of the node of stencil st in plane zs[1]
    auto links_at = [&](const Stencil &st, const unsigned (&zs)[3]) __attribute__((always_inline)) {
        return fm.links[(st.v[1][1] + zs[1]) / SB];
    };
    // interpolated walls (INTERP) on a node's pulled populations; only bodies whose pulls
    // may bounce back (MM) call it
    auto fix = [&](const LT &src, uint32_t lm, uint32_t qlo, const Stencil &st, const unsigned (&zs)[3], C (&h)[27])
        __attribute__((always_inline)) {
        if constexpr (INTERP) interp_walls<S, C>(src, p.link_q, g.qs, lm, qlo, st, zs, h);
    };
    // the q < 1/2 bits of the node of stencil st in plane zs[1] (INTERP only)
    auto qlo_at = [&](const Stencil &st, const unsigned (&zs)[3]) __attribute__((always_inline)) {
        return INTERP ? fm.qlo[(st.v[1][1] + zs[1]) / SB] : 0u;
    };
    // per-plane solid flags (uniform): bit 0 plane pz has a solid node, bit 1 planes pz-1..pz+1 do,
    // i.e. some pull of plane pz may bounce back
    auto plane_flags = [&](int pz) __attribute__((always_inline)) {
        return MASK ? fm.pflags[wrapi(pz, g.nz)] : 0u;
    };
    // rho, s*psi and g_x, g_y of one staged node into ring slot `slot` / g buffer `buf`;
    // returns g_z. h holds the node's pulled populations, m receives (sum h, j); node is
    // its lattice index (for the wall density of a solid node).
    auto stage = [&](int e, bool solid, unsigned node, const C (&h)[27], C (&m)[4], int slot, int buf, bool count)
        __attribute__((always_inline)) {
        C rho, ga[3] = {C(0), C(0), C(0)};
        if (MASK && solid) {
            rho = wall_density(p, (int)node);
        } else {
            C sum, j[3];
            moments_of<3, C>(h, sum, j);
            m[0] = sum; m[1] = j[0]; m[2] = j[1]; m[3] = j[2];
            rho = p.rho_ref + sum;
            if (TOT && count) {   // a tile node of a plane this item collides
                tot[0] += double(rho);
                tot[1] += double(j[0]);
                tot[2] += double(j[1]);
                tot[3] += double(j[2]);
                bad += p.eos.in_domain(rho) ? 0 : 1;
            }
            const C rinv = rcp(rho);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const C ua = j[a] * rinv;
                ga[a] = rho * ua * ua * ua;
            }
        }
        s_rho[slot + e] = rho;
        s_psi[slot + e] = signed_psi(p.eos, rho);
        s_gxy[buf][0][e] = ga[0];
        s_gxy[buf][1][e] = ga[1];
        return ga[2];
    };
    // after the barrier that publishes a plane: shift the windows, x / y differences of g
    auto shift_windows = [&](C gz_new, int buf) __attribute__((always_inline)) {
        gz_m1 = gz_0; gz_0 = gz_p1; gz_p1 = gz_p2; gz_p2 = gz_new;
        dgx_0 = dgx_p1; dgx_p1 = dgx_p2;
        dgy_0 = dgy_p1; dgy_p1 = dgy_p2;
        dgx_p2 = s_gxy[buf][0][e_int + 1] - s_gxy[buf][0][e_int - 1];
        dgy_p2 = s_gxy[buf][1][e_int + HX] - s_gxy[buf][1][e_int - HX];
    };
    // whole plane z0 + j (prologue, j = -2..2): pull into h, stage, publish
    auto prologue_body = [&](int j, C (&h)[27], C (&m)[4], auto MP) __attribute__((always_inline)) {
        constexpr bool MM = decltype(MP)::value;   // pulls of this plane may bounce back
        unsigned zs[3];
        planes(z0 + j, zs);
        const int slot = ((j + 2) % RING) * HP, buf = (j + 2) & 1;
        const uint32_t lm = MM ? links_at(si, zs) : 0u;
        const bool solid = (lm >> LINK_SELF) & 1u;
        if (!solid) {
            pull_all<S, C, MM>(Ab, lm, si, zs, h);
            if constexpr (MM) fix(Ab, lm, qlo_at(si, zs), si, zs, h);
        }
        if constexpr (LQ)
            if (j >= 0)
                static_for<0, NQ>([&](auto Q) {
                    constexpr int q = decltype(Q)::value;
                    s_q[(j * NQ + q) * NT + t] = h[queued(q)];
                });
        const C gzn = stage(e_int, solid, (si.v[1][1] + zs[1]) / SB, h, m, slot, buf, own && j >= 0 && j < tzi);
        if (has_halo) {
            C hh[27], mh[4];
            const uint32_t lh = MM ? links_at(sh, zs) : 0u;
            const bool hs = (lh >> LINK_SELF) & 1u;
            if (!hs) {
                pull_all<S, C, MM>(Ab, lh, sh, zs, hh);
                if constexpr (MM) fix(Ab, lh, qlo_at(sh, zs), sh, zs, hh);
            }
            stage(e_halo, hs, (sh.v[1][1] + zs[1]) / SB, hh, mh, slot, buf, false);
        }
        __syncthreads();
        shift_windows(gzn, buf);
    };
    auto prologue_plane = [&](int j, C (&h)[27], C (&m)[4]) __attribute__((always_inline)) {
        if (plane_flags(z0 + j) & 2u) prologue_body(j, h, m, std::integral_constant<bool, MASK>{});
        else prologue_body(j, h, m, std::false_type{});
    };

    // one plane of the march (k = 0 .. tz-1, z = z0 + k): collide plane z from (qa, ma),
    // refill qa with the pulls of plane z+3 as the collided values leave, stage plane z+3
    auto march_body = [&](int k, C (&qa)[27], C (&ma)[4], auto MP) __attribute__((always_inline)) {
        constexpr bool MM = decltype(MP)::value;   // pulls of plane z+3 may bounce back
        const int z = z0 + k;
        unsigned zs3[3];
        planes(z + 3, zs3);
        const int slot = ((k + 5) % RING) * HP, buf = (k + 5) & 1;
        const bool need3 = k + 1 < tzi;   // plane z+3 feeds the stencil of z+1
        const bool halo = has_halo && need3;
        C hh[27];
        const uint32_t lh = MM && halo ? links_at(sh, zs3) : 0u;
        const uint32_t bh = MM && halo ? qlo_at(sh, zs3) : 0u;
        // halo pulls of plane z+3 in flight during the stencil (FP32; REPULL pulls them below)
        if (!REPULL && halo && !((lh >> LINK_SELF) & 1u)) pull_all<S, C, MM>(Ab, lh, sh, zs3, hh);
        const uint32_t l3 = MM ? links_at(si, zs3) : 0u;
        const uint32_t b3 = MM && need3 ? qlo_at(si, zs3) : 0u;

        const unsigned zoff = (unsigned)(nxy * (z < g.nz ? z : 0)) * SB;
        const bool act = own && z < g.nz &&
                         !(MASK && (plane_flags(z) & 1u) && ((fm.links[(si.v[1][1] + zoff) / SB] >> LINK_SELF) & 1u));
        if constexpr (REPULL) {
            // plane z again: the loads are in flight during the stencil (the halo node of
            // plane z+3 is then pulled when it is staged, so that both sets of loads are
            // never held at once: FP64 registers do not hold them)
            unsigned zsz[3];
            planes(z, zsz);
            if (act) {
                if (MASK && (plane_flags(z) & 2u)) {
                    const uint32_t lz = links_at(si, zsz);
                    pull_all<S, C, MASK>(Ab, lz, si, zsz, qa);
                    fix(Ab, lz, qlo_at(si, zsz), si, zsz, qa);
                } else if constexpr (LQ) {
                    static_for<0, 27>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        if constexpr (!is_queued(i)) qa[i] = pull<i, S, C, false>(Ab, 0u, si, zsz);
                    });
                    static_for<0, NQ>([&](auto Q) {
                        constexpr int q = decltype(Q)::value;
                        qa[queued(q)] = s_q[((k % 3) * NQ + q) * NT + t];
                    });
                } else {
                    pull_all<S, C, false>(Ab, 0u, si, zsz, qa);
                }
            }
        }
        C Sf[3] = {C(0), C(0), C(0)};
        C rho = C(1);
        if (act) {
            const int base[5] = {(k % RING) * HP, ((k + 1) % RING) * HP, ((k + 2) % RING) * HP,
                                 ((k + 3) % RING) * HP, ((k + 4) % RING) * HP};   // planes z-2..z+2
            rho = s_rho[base[2] + e_int];
            const C spc = s_psi[base[2] + e_int];
            C Fp[3] = {C(0), C(0), C(0)}, Fc[3] = {C(0), C(0), C(0)};
            static_for<1, 27>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
                constexpr int o1 = cy * HX + cx;
                constexpr int cls = cx * cx + cy * cy + cz * cz - 1;   // weight class of c_i
                const int r1 = base[2 + cz] + e_int + o1, r2 = base[2 + 2 * cz] + e_int + 2 * o1;
                // 3w (G1 psi1 + G2 psi2) and 3w (G3 rho1 + G4 rho2)
                const C tp = p.gw[cls][0] * fabs(s_psi[r1]) + p.gw[cls][1] * fabs(s_psi[r2]);
                const C tc = p.gw[cls][2] * s_rho[r1] + p.gw[cls][3] * s_rho[r2];
                static_for<0, 3>([&](auto A_) {
                    constexpr int a = decltype(A_)::value;
                    constexpr int ca = Lat<3>::c(i, a);
                    if constexpr (ca == 1) { Fp[a] += tp; Fc[a] += tc; }
                    if constexpr (ca == -1) { Fp[a] -= tp; Fc[a] -= tc; }
                });
            });
#pragma unroll
            for (int a = 0; a < 3; ++a) Sf[a] = rho * p.accel[a] - (C(2) * spc * Fp[a] + rho * Fc[a]);
        }
        if (halo) {
            C mh[4];
            if (REPULL && !((lh >> LINK_SELF) & 1u)) pull_all<S, C, MM>(Ab, lh, sh, zs3, hh);
            if constexpr (MM)
                if (!((lh >> LINK_SELF) & 1u)) fix(Ab, lh, bh, sh, zs3, hh);
            stage(e_halo, (lh >> LINK_SELF) & 1u, (sh.v[1][1] + zs3[1]) / SB, hh, mh, slot, buf, false);
        }

        // refill with plane z+3, which feeds the stencil of z+1; past the chunk the
        // loads go to Anull
        // (grouped resources: Ab itself, which reads wrapped planes never used, so that a
        // second set of resources does not take scalar registers)
        const LT src = (LAT == 2 || need3) ? Ab : Anull;
        if (act) {
            constexpr C W0 = C(1.0 / 6.0), W1 = C(2.0 / 3.0);
            const C drho = ma[0];
            const C rinv = rcp(rho);
            const C omega = omega_of(p, rho);
            const C cf = (C(1) - C(0.5) * omega) * C(0.5);
            const C Phi[3] = {cf * dgx_0, cf * dgy_0, cf * (gz_p1 - gz_m1)};
            // per-axis triplets of the deviation-form equilibria (see collide())
            C dv[3][3], Av[3][3], Dv[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const C ua = ma[1 + a] * rinv, u2 = ua * ua;
                dv[a][0] = C(0.5) * (u2 - ua);
                dv[a][1] = -u2;
                dv[a][2] = C(0.5) * (u2 + ua);
                const C s = Sf[a] * rinv;
                const C de = s * (C(2) * ua + s) + Phi[a] * rinv;
                Dv[a][0] = C(0.5) * (de - s);
                Dv[a][1] = -de;
                Dv[a][2] = C(0.5) * (de + s);
                Av[a][0] = W0 + dv[a][0]; Av[a][1] = W1 + dv[a][1]; Av[a][2] = W0 + dv[a][2];
            }
            const C om1 = C(1) - omega, omd = omega * drho;
            C rem = drho;
            // (c_x, c_y) pairs outermost so that only one pair's x-y factors are live
            static_for<0, 9>([&](auto P_) {
                constexpr int kx = decltype(P_)::value / 3, ky = decltype(P_)::value % 3;
                constexpr C Wx = kx == 1 ? W1 : W0;
                constexpr C WW = (kx == 1 ? W1 : W0) * (ky == 1 ? W1 : W0);
                const C E = dv[0][kx] * Av[1][ky] + Wx * dv[1][ky];
                const C F = Dv[0][kx] * (Av[1][ky] + Dv[1][ky]) + Av[0][kx] * Dv[1][ky];
                const C AA = Av[0][kx] * Av[1][ky];
                static_for<0, 3>([&](auto Z_) {
                    constexpr int kz = decltype(Z_)::value;
                    constexpr int i = index3(kx - 1, ky - 1, kz - 1);
                    if constexpr (i != 0) {
                        constexpr C wi = C(weight<3>(i));
                        const C eqd = Av[2][kz] * E + WW * dv[2][kz];
                        const C fsd = (Av[2][kz] + Dv[2][kz]) * F + AA * Dv[2][kz];
                        const C hn = om1 * qa[i] + omd * wi + rho * (omega * eqd + fsd);
                        rem -= hn;
                        Bb.template store<i>(si.v[1][1], zoff, S(hn));
                        qa[i] = pull<i, S, C, MM>(src, l3, si, zs3);
                        // keep the refill load here: left to itself the scheduler sinks all
                        // loads below the last store, and nothing overlaps their latency
                        __builtin_amdgcn_sched_barrier(0);
                    }
                });
            });
            // rest population as the remainder: the per-node mass error stays an unbiased rounding
            Bb.template store<0>(si.v[1][1], zoff, S(rem));
            qa[0] = pull<0, S, C, MM>(src, l3, si, zs3);
        } else {
            pull_all<S, C, MM>(src, l3, si, zs3, qa);
        }
        C gzn = C(0);
        if constexpr (MM)
            if (need3 && !((l3 >> LINK_SELF) & 1u)) fix(Ab, l3, b3, si, zs3, qa);
        if (need3)
            gzn = stage(e_int, (l3 >> LINK_SELF) & 1u, (si.v[1][1] + zs3[1]) / SB, qa, ma, slot, buf,
                        own && k + 3 < tzi);
        if constexpr (LQ)
            if (need3)
                static_for<0, NQ>([&](auto Q) {
                    constexpr int q = decltype(Q)::value;
                    s_q[((k % 3) * NQ + q) * NT + t] = qa[queued(q)];
                });
        __syncthreads();
        shift_windows(gzn, buf);
    };
    // FP32: planes whose pulls cannot bounce back take the unmasked body (a uniform branch).
    // FP64 keeps one body: the two bodies in one loop cost it hundreds of spilled registers,
    // more than the per-link selects cost on the few solid-free planes of a masked run.
    auto march = [&](int k, C (&qa)[27], C (&ma)[4]) __attribute__((always_inline)) {
        if constexpr (REPULL) {
            march_body(k, qa, ma, std::integral_constant<bool, MASK>{});
        } else {
            if (plane_flags(z0 + k + 3) & 2u) march_body(k, qa, ma, std::integral_constant<bool, MASK>{});
            else march_body(k, qa, ma, std::false_type{});
        }
    };

    prologue_plane(-2, q0, m0);
    prologue_plane(-1, q0, m0);
    prologue_plane(0, q0, m0);
    if constexpr (REPULL) {
        prologue_plane(1, q0, m1);
        prologue_plane(2, q0, m2);
    } else {
        prologue_plane(1, q1, m1);
        prologue_plane(2, q2, m2);
    }
    if constexpr (REPULL) {
#pragma unroll 1
        for (int k = 0; k < tzi; k += 3) {
            march(k, q0, m0);
            if (k + 1 < tzi) march(k + 1, q0, m1);
            if (k + 2 < tzi) march(k + 2, q0, m2);
        }
    } else {
#pragma unroll 1
        for (int k = 0; k < tzi; k += 3) {
            march(k, q0, m0);
            if (k + 1 < tzi) march(k + 1, q1, m1);
            if (k + 2 < tzi) march(k + 2, q2, m2);
        }
    }
    // one row of FP64 partial sums per work item, in a fixed order: wave64 shuffles, then the
    // waves' sums from LDS
    if (TOT && fg.partials) {
        __shared__ double s_red[NT / 64][kPartialSlots];
        double v[kPartialSlots] = {tot[0], tot[1], tot[2], tot[3], double(bad)};
#pragma unroll
        for (int q = 0; q < kPartialSlots; ++q)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
        if ((t & 63) == 0)
#pragma unroll
            for (int q = 0; q < kPartialSlots; ++q) s_red[t >> 6][q] = v[q];
        __syncthreads();
        if (t < kPartialSlots) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) sum += s_red[w][t];
            fg.partials[(long long)(fg.slot0 + item) * kPartialSlots + t] = sum;
        }
    }
}

template <class S, class C, bool MASK, int TX, int TY, bool REPULL, int LAT, bool INTERP = false>
void launch_fused(hipStream_t s, const void *A, void *B, const Geom &g, const FusedMask &fm, const void *prm,
                  const FusedGrid &fg) {
    hipLaunchKernelGGL((k_fused3<S, C, MASK, TX, TY, REPULL, LAT, INTERP>), dim3(fg.blocks), dim3(TX * TY), 0, s,
                       (const S *)A, (S *)B, g, fm, *(const Params<C> *)prm, fg);
}

__global__ void k_links(const uint8_t *__restrict__ mask, uint32_t *__restrict__ links, Geom g) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = n % g.px, y = (n / g.px) % g.ny, z = n / (g.px * g.ny);
    if (x >= g.nx) {   // row padding
        links[n] = 0u;
        return;
    }
    uint32_t b = mask[n] ? (1u << LINK_SELF) : 0u;
    static_for<1, 27>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int s = wrapi(x - Lat<3>::c(i, 0), g.nx) +
                      g.px * (wrapi(y - Lat<3>::c(i, 1), g.ny) + g.ny * wrapi(z - Lat<3>::c(i, 2), g.nz));
        if (mask[s]) b |= 1u << i;
    });
    links[n] = b;
}

// bit i set when population i of fluid node n crosses a wall link whose fraction (stored
// under opp(i)) is below 1/2, compared in the compute precision C of the step
template <class C>
__global__ void k_qlo(const uint32_t *__restrict__ links, const C *__restrict__ lq, uint32_t *__restrict__ qlo, Geom g) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const uint32_t lm = links[n];
    uint32_t b = 0u;
    if (!((lm >> LINK_SELF) & 1u))
        static_for<1, 27>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if (((lm >> i) & 1u) && lq[(long long)opp<3>(i) * g.qs + n] < C(0.5)) b |= 1u << i;
        });
    qlo[n] = b;
}

}  // namespace

void fused_links(hipStream_t s, const uint8_t *mask, uint32_t *links, const Geom &g) {
    hipLaunchKernelGGL(k_links, dim3((g.N + 255) / 256), dim3(256), 0, s, mask, links, g);
}

void fused_qlo(hipStream_t s, const uint32_t *links, const void *lq, bool fp64, uint32_t *qlo, const Geom &g) {
    if (fp64)
        hipLaunchKernelGGL(k_qlo<double>, dim3((g.N + 255) / 256), dim3(256), 0, s, links, (const double *)lq, qlo, g);
    else
        hipLaunchKernelGGL(k_qlo<float>, dim3((g.N + 255) / 256), dim3(256), 0, s, links, (const float *)lq, qlo, g);
}

FusedGrid fused_grid(const Geom &g, int tx, int ty, int tz, int zb, int ze) {
    FusedGrid f;
    f.tx = tx;
    f.ty = ty;
    f.tz = tz;
    f.zb = zb;
    f.ze = ze;
    f.ntx = (g.nx + tx - 1) / tx;
    f.nty = (g.ny + ty - 1) / ty;
    f.nzc = (ze - zb + tz - 1) / tz;
    f.items = f.ntx * f.nty * f.nzc;
    f.item0 = 0;
    f.count = f.items;
    f.per_xcd = (f.items + NXCD - 1) / NXCD;
    f.blocks = f.per_xcd * NXCD;
    f.partials = nullptr;
    f.slot0 = 0;
    return f;
}

std::vector<FusedGrid> fused_windows(const FusedGrid &fg, int window) {
    std::vector<FusedGrid> out;
    if (window < NXCD) window = NXCD;
    for (int i0 = 0; i0 < fg.items; i0 += window) {
        FusedGrid w = fg;
        w.item0 = i0;
        w.count = std::min(window, fg.items - i0);
        w.per_xcd = (w.count + NXCD - 1) / NXCD;
        w.blocks = w.per_xcd * NXCD;
        out.push_back(w);
    }
    return out;
}

namespace {
template <int TX, int TY> FusedLaunch pick(bool masked) {
    return masked ? launch_fused<float, float, true, TX, TY, false, 0>
                  : launch_fused<float, float, false, TX, TY, false, 0>;
}
}  // namespace

FusedLaunch fused_launcher(bool fp64, bool masked, int tx, int ty, int lat, bool interp) {
    if (lat == 2) {   // grouped resources: 64 x 8 only
        if (tx != 64 || ty != 8) return nullptr;
        if (fp64)
            return interp   ? (masked ? launch_fused<double, double, true, 64, 8, true, 2, true> : nullptr)
                   : masked ? launch_fused<double, double, true, 64, 8, true, 2>
                            : launch_fused<double, double, false, 64, 8, true, 2>;
        return interp   ? (masked ? launch_fused<float, float, true, 64, 8, false, 2, true> : nullptr)
               : masked ? launch_fused<float, float, true, 64, 8, false, 2>
                        : launch_fused<float, float, false, 64, 8, false, 2>;
    }
    const bool split = lat == 1;
    if (interp) {   // interpolated walls: masked 64 x 8 variants only
        if (!masked || tx != 64 || ty != 8) return nullptr;
        if (fp64)
            return split ? launch_fused<double, double, true, 64, 8, true, 1, true>
                         : launch_fused<double, double, true, 64, 8, true, 0, true>;
        return split ? nullptr : launch_fused<float, float, true, 64, 8, false, 0, true>;
    }
    if (fp64) {
        if (tx != 64 || ty != 8) return nullptr;
        if (split)
            return masked ? launch_fused<double, double, true, 64, 8, true, 1>
                          : launch_fused<double, double, false, 64, 8, true, 1>;
        return masked ? launch_fused<double, double, true, 64, 8, true, 0>
                      : launch_fused<double, double, false, 64, 8, true, 0>;
    }
    if (split) return nullptr;
    if (tx == 64 && ty == 8) return pick<64, 8>(masked);
    if (tx == 32 && ty == 8) return pick<32, 8>(masked);
    if (tx == 32 && ty == 16) return pick<32, 16>(masked);
    return nullptr;
}

}  // namespace lbm
