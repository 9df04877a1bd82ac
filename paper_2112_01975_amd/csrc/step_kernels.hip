// step_kernels.hip -- the D2Q9 stream-collide step in one pass, and the two-pass step
// (D3Q27 grids the fused z-march does not take), of the two-phase LBGK model (Sec. 2.3)
// for gfx950.
//
// Storage: structure of arrays A[i*qs + n], n = x + nx*(y + ny*z). The array holds
// post-collision populations at the node that produced them; every pass pulls
// f_i(r) = A_i(r - c_i), or A_opp(i)(r) when r - c_i is solid (halfway bounce-back),
// or with per-link wall fractions an interpolation of A_opp(i) at r and r + c_i or of
// A_opp(i) and A_i at r (interpolated bounce-back).
//
// Pass 1 (moments): rho = rho_ref + sum h_i, j = sum c_i h_i, g_a = rho u_a^3; FP64
//   per-workgroup partial sums of mass and momentum for the watchdog.
// Pass 2 (collide): stages rho and the signed pseudo-potential of a 64x4xZB tile
//   plus a two-node halo in LDS (the D2Q9 single pass: a 64x8 tile whose staged nodes
//   take rho and g from their own pulls), evaluates the two-ring Korteweg force
//   (eq Kforce_final, or the stencil coefficients of another force model), the diagonal correction Phi (eq correction), the product-form
//   equilibrium and extended equilibrium (eqs LBMeq, LBMstar) in cancellation-free
//   deviation form, and the LBGK update (eq LBGK).
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"
#include "lattice.hpp"
#include "step_common.hpp"

namespace lbm {

namespace {

constexpr int TX = 64;   // tile width in x: one wave64 row, coalesced 256 B (FP32) loads
constexpr int TY = 4;    // tile height in y: 4 waves per workgroup
constexpr int HALO = 2;  // two neighbour rings
constexpr int kSingleTY = 8;   // D2Q9 single pass: tile height (one wave per row)
constexpr int kXcds = 8;       // MI355X: workgroups are dealt to 8 XCDs in turn
constexpr int kXcdChunk = 128; // single pass: consecutive tiles per XCD chunk

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block of 256 threads: sums 5 values in a fixed order, thread 0 writes them
__device__ __forceinline__ void block_sum5(double (&v)[kPartialSlots], double *__restrict__ dst) {
    __shared__ double red[4][kPartialSlots];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kPartialSlots; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kPartialSlots; ++k) red[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x < kPartialSlots) {
        const int k = threadIdx.x;
        dst[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
}

// ------------------------------------------------------------------ pass 1
template <int D, class S, class C, bool MASK>
__global__ __launch_bounds__(256) void k_moments(const S *__restrict__ A, Geom g, const uint8_t *__restrict__ mask,
                                                 Params<C> p, C *__restrict__ rho_out, C *__restrict__ gf,
                                                 double *__restrict__ partials) {
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int x = blockIdx.x * TX + tx, y = blockIdx.y * TY + ty, z = blockIdx.z;
    double v[kPartialSlots] = {0, 0, 0, 0, 0};
    if (x < g.nx && y < g.ny) {
        const int n = x + g.px * (y + g.ny * z);
        C rho, ga[3] = {C(0), C(0), C(0)};
        if (MASK && mask[n]) {
            rho = wall_density(p, n);
        } else {
            Nbr<D> nb(g, x, y, z);
            C h[Lat<D>::Q];
            gather<D, S, C, MASK>(A, g.qs, mask, nb, n, h, p.link_q);
            C sum, j[3];
            moments_of<D, C>(h, sum, j);
            rho = p.rho_ref + sum;
            const C rinv = rcp(rho);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const C ua = j[a] * rinv;
                ga[a] = rho * ua * ua * ua;
            }
            v[0] = double(rho);
            v[1] = double(j[0]);
            v[2] = double(j[1]);
            v[3] = D == 3 ? double(j[2]) : 0.0;
            v[4] = p.eos.in_domain(rho) ? 0.0 : 1.0;
        }
        rho_out[n] = rho;
#pragma unroll
        for (int a = 0; a < D; ++a) gf[(long long)a * g.N + n] = ga[a];
    }
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_sum5(v, partials + (long long)blk * kPartialSlots);
}

// ------------------------------------------------------------------ pass 2
// TYT: tile height in y, one wave per row (the D2Q9 single pass takes 8 rows and 512 threads,
// which stages a halo of 59% of the tile instead of 113%)
template <int D, int TYT = TY> struct Tile {
    static constexpr int ZB = D == 3 ? 2 : 1;                  // z-planes per workgroup
    static constexpr int LX = TX + 2 * HALO, LY = TYT + 2 * HALO;
    static constexpr int LZ = D == 3 ? ZB + 2 * HALO : 1;
    static constexpr int LS = LX * LY * LZ;
};

enum { MODE_STEP = 0, MODE_OUT = 1, MODE_INIT = 2, MODE_PT = 3, MODE_SINGLE = 4 };

// MODE_STEP: one collide-stream step A -> B.
// MODE_OUT:  rho and U = u + S/(2 rho) of the state in A, FP64, into out_rho / out_U.
// MODE_INIT: equilibrium of the density in rho_f and the flow velocity U0 (= out_U, may be
//            NULL): bare u = U0 - S/(2 rho), written into B in pull layout.
// MODE_PT:   discrete pressure tensor of the state in A (Appendix E) into out_U, FP64
//            [D(D+1)/2][N]: xx, yy, [zz,] xy[, xz, yz]; zero at solid nodes. The lattice
//            momentum flux of the pulled (pre-collision) populations minus the one- and
//            two-ring pseudo-potential and capillary tensors, which enter with the sign of
//            the momentum source S = -F.
// MODE_SINGLE: one collide-stream step A -> B in a single pass (D2Q9): the staged tile and
//            halo nodes pull their own populations and take rho and g = rho u^3 from them, as
//            the moment pass computes them, instead of reading the moment pass's fields.
template <int D, class S, class C, bool MASK, int MODE>
__global__ __launch_bounds__(MODE == MODE_SINGLE ? TX * kSingleTY : TX * TY) void k_collide(
    const S *__restrict__ A, S *__restrict__ B, Geom g, const uint8_t *__restrict__ mask, Params<C> p,
    const C *__restrict__ rho_f, const C *__restrict__ gf, double *__restrict__ out_rho, double *__restrict__ out_U) {
    constexpr bool OUT = MODE == MODE_OUT;
    constexpr bool SINGLE = MODE == MODE_SINGLE;
    static_assert(!SINGLE || D == 2, "single-pass mode: D2Q9");
    constexpr int TYK = SINGLE ? kSingleTY : TY, NTH = TX * TYK;
    using T = Tile<D, TYK>;
    __shared__ C s_rho[T::LS];
    __shared__ C s_psi[T::LS];
    __shared__ C s_g[SINGLE ? 2 : 1][SINGLE ? T::LS : 1];   // single pass: g_x, g_y of the staged nodes
    // single pass: a 1-D grid. The hardware deals workgroups to the 8 XCDs in turn; the tiles,
    // in row-major order, go to them in chunks of up to kXcdChunk consecutive tiles, so that
    // neighbouring tiles mostly share an XCD and read each other's halo rows from its L2
    int bx = blockIdx.x, by = blockIdx.y;
    if constexpr (SINGLE) {
        const int ntx = (g.nx + TX - 1) / TX, nt = ntx * ((g.ny + TYK - 1) / TYK);
        const int per = (nt + kXcds - 1) / kXcds, ch = per < kXcdChunk ? per : kXcdChunk, b = blockIdx.x;
        const int i = b / kXcds;
        const int tile = ((i / ch) * kXcds + b % kXcds) * ch + i % ch;
        if (tile >= nt) return;   // the padding of the last XCD's share (whole workgroup)
        bx = tile % ntx;
        by = tile / ntx;
    }
    const int x0 = bx * TX, y0 = by * TYK, z0 = D == 3 ? blockIdx.z * T::ZB : 0;
    // single pass: the populations this thread pulled for its own node, kept for its update
    C h_own[Lat<D>::Q];
    if constexpr (SINGLE) {
        // Staging: every thread its own tile node (wrapped past the grid's edge: those feed the
        // stencils of the last columns and rows), and at most one of the NH halo nodes: rows 0,
        // 1, LY-2, LY-1 of the staged tile, then columns 0, 1, LX-2, LX-1 of the rows between.
        // Both nodes' pulls are issued before either is reduced, with the moment pass's
        // arithmetic, to rho, s psi and g.
        const int t = threadIdx.x, tx = t & (TX - 1), ty = t / TX;
        constexpr int NH = T::LS - NTH;
        static_assert(NH <= NTH, "one halo node per thread at most");
        const bool has_halo = t < NH;
        int lx = 0, ly = 0;
        if (t < 4 * T::LX) {
            const int r = t / T::LX;
            lx = t % T::LX;
            ly = r < 2 ? r : TYK + r;
        } else if (has_halo) {
            const int q = t - 4 * T::LX, c4 = q % 4;
            ly = 2 + q / 4;
            lx = c4 < 2 ? c4 : TX + c4;
        }
        const int e_own = (ty + HALO) * T::LX + tx + HALO, e_halo = ly * T::LX + lx;
        const int ox = wrapi(x0 + tx, g.nx), oy = wrapi(y0 + ty, g.ny);
        const int hx = wrapi(x0 - HALO + lx, g.nx), hy = wrapi(y0 - HALO + ly, g.ny);
        const int on = ox + g.px * oy, hn = hx + g.px * hy;
        const bool osolid = MASK && mask[on], hsolid = MASK && has_halo && mask[hn];
        C hh[Lat<D>::Q];
        if (!osolid) {
            Nbr<D> nb(g, ox, oy, 0);
            gather<D, S, C, MASK>(A, g.qs, mask, nb, on, h_own, p.link_q);
        }
        if (has_halo && !hsolid) {
            Nbr<D> nb(g, hx, hy, 0);
            gather<D, S, C, MASK>(A, g.qs, mask, nb, hn, hh, p.link_q);
        }
        auto finish = [&](int e, int gn, bool solid, const C (&h)[Lat<D>::Q]) __attribute__((always_inline)) {
            C r, ga[2] = {C(0), C(0)};
            if (solid) {
                r = wall_density(p, gn);
            } else {
                C sum, j[3];
                moments_of<D, C>(h, sum, j);
                r = p.rho_ref + sum;
                const C rinv = rcp(r);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const C ua = j[a] * rinv;
                    ga[a] = r * ua * ua * ua;
                }
            }
            s_rho[e] = r;
            s_psi[e] = signed_psi(p.eos, r);
            s_g[0][e] = ga[0];
            s_g[1][e] = ga[1];
        };
        finish(e_own, on, osolid, h_own);
        if (has_halo) finish(e_halo, hn, hsolid, hh);
    } else {
        for (int e = threadIdx.x; e < T::LS; e += NTH) {
            const int lx = e % T::LX, t = e / T::LX, ly = t % T::LY, lz = t / T::LY;
            const int gx = wrapi(x0 - HALO + lx, g.nx), gy = wrapi(y0 - HALO + ly, g.ny);
            const int gz = D == 3 ? wrapi(z0 - HALO + lz, g.nz) : 0;
            const C r = rho_f[gx + g.px * (gy + g.ny * gz)];
            s_rho[e] = r;
            s_psi[e] = signed_psi(p.eos, r);
        }
    }
    __syncthreads();
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= g.nx || y >= g.ny) return;
#pragma unroll 1
    for (int zz = 0; zz < T::ZB; ++zz) {
        const int z = z0 + zz;
        if (z >= g.nz) break;
        const int n = x + g.px * (y + g.ny * z);
        if (MASK && mask[n]) {
            if constexpr (OUT) {
                out_rho[n] = double(wall_density(p, n));
                for (int a = 0; a < D; ++a) out_U[(long long)a * g.N + n] = 0.0;
            }
            if constexpr (MODE == MODE_PT)
                for (int k = 0; k < D * (D + 1) / 2; ++k) out_U[(long long)k * g.N + n] = 0.0;
            continue;
        }
        const int lc0 = ((D == 3 ? zz + HALO : 0) * T::LY + ty + HALO) * T::LX + tx + HALO;
        if constexpr (MODE == MODE_PT) {
            Nbr<D> nb(g, x, y, z);
            C h[Lat<D>::Q];
            gather<D, S, C, MASK>(A, g.qs, mask, nb, n, h, p.link_q);
            constexpr int NC = D * (D + 1) / 2;
            constexpr int ca[6] = {0, 1, D == 3 ? 2 : 0, 0, 0, 1}, cb[6] = {0, 1, D == 3 ? 2 : 1, 1, 2, 2};
            C flux[NC], ringA[NC], ringB[NC], across[NC], cap1[NC], cap2[NC], capx[NC];
            for (int k = 0; k < NC; ++k) flux[k] = ringA[k] = ringB[k] = across[k] = cap1[k] = cap2[k] = capx[k] = C(0);
            static_for<0, Lat<D>::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
                constexpr int off = (cz * T::LY + cy) * T::LX + cx;
                constexpr C w3 = C(3.0 * weight<D>(i));
                const C p1 = fabs(s_psi[lc0 + off]), p2 = fabs(s_psi[lc0 + 2 * off]), m1 = fabs(s_psi[lc0 - off]);
                const C r1 = s_rho[lc0 + off], r2 = s_rho[lc0 + 2 * off], rm = s_rho[lc0 - off];
                static_for<0, NC>([&](auto K) {
                    constexpr int k = decltype(K)::value;
                    constexpr int cc = Lat<D>::c(i, ca[k]) * Lat<D>::c(i, cb[k]);
                    if constexpr (cc != 0) {
                        flux[k] += C(cc) * h[i];
                        constexpr C wc = w3 * C(cc);
                        ringA[k] += wc * p1;
                        ringB[k] += wc * p2;
                        across[k] += wc * m1 * p1;
                        cap1[k] += wc * r1;
                        cap2[k] += wc * r2;
                        capx[k] += wc * rm * r1;
                    }
                });
            });
            const C rho = s_rho[lc0], sp = s_psi[lc0];
            const C psi = fabs(sp), sg = sp > C(0) ? C(1) : C(-1);
            for (int k = 0; k < NC; ++k) {
                // Appendix E's parts for the stencil pairs (G1, G2), (G3, G4): each part is
                // linear in its coefficient (printed for 4/3, -1/6, 2 kappa, -kappa)
                const C PA = -sg * p.G[0] * psi * ringA[k];
                const C PB = -sg * p.G[1] * (psi * ringB[k] + across[k]);
                const C PC = C(-0.5) * p.G[2] * rho * cap1[k];
                const C PD = C(-0.5) * p.G[3] * (rho * cap2[k] + capx[k]);
                // FP32 deviation storage: the reference part w_i rho_ref adds rho_ref/3 on the diagonal
                const C kin = flux[k] + (k < D ? p.rho_ref * C(1.0 / 3.0) : C(0));
                out_U[(long long)k * g.N + n] = double(kin) - (double(PA) + double(PB) + double(PC) + double(PD));
            }
            continue;
        }
        const int lc = ((D == 3 ? zz + HALO : 0) * T::LY + ty + HALO) * T::LX + tx + HALO;
        const C rho = s_rho[lc], spc = s_psi[lc];
        C Fp[3] = {C(0), C(0), C(0)}, Fc[3] = {C(0), C(0), C(0)};
        static_for<1, Lat<D>::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
            constexpr int off = (cz * T::LY + cy) * T::LX + cx;
            constexpr int cls = cx * cx + cy * cy + cz * cz - 1;   // weight class of c_i
            const C p1 = fabs(s_psi[lc + off]), p2 = fabs(s_psi[lc + 2 * off]);
            const C r1 = s_rho[lc + off], r2 = s_rho[lc + 2 * off];
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
        for (int a = 0; a < D; ++a) Sf[a] = rho * p.accel[a] - (C(2) * spc * Fp[a] + rho * Fc[a]);   // S = -F + rho g

        Nbr<D> nb(g, x, y, z);
        C h[Lat<D>::Q];
        if constexpr (MODE == MODE_INIT) {
            C u[3] = {C(0), C(0), C(0)};
#pragma unroll
            for (int a = 0; a < D; ++a)
                u[a] = (out_U ? C(out_U[(long long)a * g.N + n]) : C(0)) - Sf[a] * (C(0.5) * rcp(rho));
#pragma unroll
            for (int i = 0; i < Lat<D>::Q; ++i) h[i] = C(0);
            // omega = 1 with no source and no correction returns the equilibrium deviation
            const C zero3[3] = {C(0), C(0), C(0)};
            collide<D, C>(h, rho, rho - p.rho_ref, u, zero3, zero3, C(1));
            static_for<0, Lat<D>::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
                if constexpr (i == 0) {
                    B[n] = S(h[0]);
                } else {
                    // pulled at n from n - c_i, or from opp(i) at n when n - c_i is solid
                    const int src = nb.at(-cx, -cy, -cz);
                    if (MASK && mask[src])
                        B[(long long)opp<D>(i) * g.qs + n] = S(h[i]);
                    else
                        B[(long long)i * g.qs + src] = S(h[i]);
                }
            });
            continue;
        } else {
        if constexpr (SINGLE) {
#pragma unroll
            for (int i = 0; i < Lat<D>::Q; ++i) h[i] = h_own[i];
        } else {
            gather<D, S, C, MASK>(A, g.qs, mask, nb, n, h, p.link_q);
        }
        C drho, j[3];
        moments_of<D, C>(h, drho, j);
        C u[3] = {C(0), C(0), C(0)};
        const C rinv = rcp(rho);
#pragma unroll
        for (int a = 0; a < D; ++a) u[a] = j[a] * rinv;
        const C omega = omega_of(p, rho);
        C Phi[3] = {C(0), C(0), C(0)};
        if constexpr (SINGLE) {
            const C cf = (C(1) - C(0.5) * omega) * C(0.5);
            Phi[0] = cf * (s_g[0][lc + 1] - s_g[0][lc - 1]);
            Phi[1] = cf * (s_g[1][lc + T::LX] - s_g[1][lc - T::LX]);
        } else {
            const C cf = (C(1) - C(0.5) * omega) * C(0.5);
            Phi[0] = cf * (gf[nb.at(1, 0, 0)] - gf[nb.at(-1, 0, 0)]);
            Phi[1] = cf * (gf[(long long)g.N + nb.at(0, 1, 0)] - gf[(long long)g.N + nb.at(0, -1, 0)]);
            if constexpr (D == 3)
                Phi[2] = cf * (gf[2LL * g.N + nb.at(0, 0, 1)] - gf[2LL * g.N + nb.at(0, 0, -1)]);
        }
        if constexpr (OUT) {
            out_rho[n] = double(rho);
#pragma unroll
            for (int a = 0; a < D; ++a) out_U[(long long)a * g.N + n] = double(u[a] + Sf[a] * (C(0.5) * rinv));
        } else {
            collide<D, C>(h, rho, drho, u, Sf, Phi, omega);
            static_for<0, Lat<D>::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                st_nt_at(B + i * g.qs, (unsigned)n, S(h[i]));
            });
        }
        }
    }
}

// ------------------------------------------------------------------ init
// density field of the initial state in compute precision; solid nodes carry rho_w
template <class C, bool MASK>
__global__ __launch_bounds__(256) void k_prep_rho(C *__restrict__ rho_f, const double *__restrict__ rho0,
                                                  const uint8_t *__restrict__ mask, Params<C> p, int N) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    rho_f[n] = (MASK && mask[n]) ? wall_density(p, n) : C(rho0[n]);
}

// Interpolated bounce-back at init. The init kernel folds the equilibrium population i
// of a fluid node n whose source n - c_i is solid into slot opp(i) at n, which only that
// wall link reads. The interpolated pull mixes this slot X with a second entry:
//   q <  1/2: 2q X + (1 - 2q) Y, Y = slot opp(i) at n + c_i (fluid: already f_eq_opp(i)(n);
//             solid: the pull uses X alone)
//   q >= 1/2: a X + (1 - a) Z,  a = 1/(2q), Z = slot i at n (n + c_i fluid: already the
//             equilibrium pulled there; solid: the slot X' of the opposite wall link)
// so X is re-solved for the pull to return the folded value P; the opposite-pair case is a
// 2x2 system with determinant a + a' - 1 (bounded away from 0 by host validation). Only
// the node's own wall slots change, and every entry read is either one of them, read
// before any write, or a regular entry, so nodes are independent.
template <int D, class S, class C>
__global__ __launch_bounds__(256) void k_wall_init(S *__restrict__ A, Geom g, const uint8_t *__restrict__ mask,
                                                   const C *__restrict__ lq) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= g.N) return;
    const int x = n % g.px, t = n / g.px, y = t % g.ny, z = t / g.ny;
    if (x >= g.nx || mask[n]) return;   // row padding, or solid
    Nbr<D> nb(g, x, y, z);
    constexpr int Q = Lat<D>::Q;
    C P[Q], X[Q];
    bool wall[Q];
    static_for<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
        wall[i] = mask[nb.at(-cx, -cy, -cz)] != 0;
        P[i] = wall[i] ? C(A[(long long)opp<D>(i) * g.qs + n]) : C(0);
    });
    static_for<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value, o = opp<D>(i);
        constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
        X[i] = P[i];
        if (!wall[i]) return;
        const C q = lq[(long long)o * g.qs + n];
        const int b = nb.at(cx, cy, cz);
        const bool bsolid = mask[b] != 0;   // n + c_i solid <=> (n, opp(i)) is a wall link too
        if (q < C(0.5)) {
            if (!bsolid) X[i] = (P[i] - (C(1) - C(2) * q) * C(A[(long long)o * g.qs + b])) / (C(2) * q);
            return;
        }
        const C a = C(1) / (C(2) * q);
        if (!bsolid) {
            X[i] = (P[i] - (C(1) - a) * C(A[(long long)i * g.qs + n])) / a;
            return;
        }
        const C q2 = lq[(long long)i * g.qs + n];
        if (q2 < C(0.5)) {                   // the opposite link keeps its folded value
            X[i] = (P[i] - (C(1) - a) * P[o]) / a;
            return;
        }
        const C a2 = C(1) / (C(2) * q2);
        X[i] = (a2 * P[i] - (C(1) - a) * P[o]) / (a + a2 - C(1));
    });
    static_for<1, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (wall[i]) A[(long long)opp<D>(i) * g.qs + n] = S(X[i]);
    });
}

template <class S> __global__ __launch_bounds__(256) void k_fill_zero(S *__restrict__ A, long long count) {
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < count; k += (long long)gridDim.x * 256)
        A[k] = S(0);
}

// One level of the deterministic FP64 tree over partial rows of kPartialSlots values: block b
// sums rows [b R, (b + 1) R) (R = 2048) into out[b]. Each thread adds its eight rows
// t, t + 256, ... in order, then the block halves in LDS; the order depends only on n.
constexpr int kReduceRows = 2048;
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ in, int n, double *__restrict__ out) {
    __shared__ double red[256][kPartialSlots];
    double acc[kPartialSlots] = {0, 0, 0, 0, 0};
    const long long r0 = (long long)blockIdx.x * kReduceRows;
    for (int k = 0; k < kReduceRows / 256; ++k) {
        const long long r = r0 + threadIdx.x + 256LL * k;
        if (r < n)
#pragma unroll
            for (int q = 0; q < kPartialSlots; ++q) acc[q] += in[r * kPartialSlots + q];
    }
#pragma unroll
    for (int q = 0; q < kPartialSlots; ++q) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < kPartialSlots; ++q) red[threadIdx.x][q] += red[threadIdx.x + h][q];
        __syncthreads();
    }
    if (threadIdx.x < kPartialSlots) out[(long long)blockIdx.x * kPartialSlots + threadIdx.x] = red[0][threadIdx.x];
}

// ------------------------------------------------------------------ launchers
dim3 moment_grid(int D, const Geom &g) {
    return dim3((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, D == 3 ? g.nz : 1);
}

// workgroups of the single pass: its tiles, padded to a whole number per XCD
inline unsigned single_blocks(const Geom &g) {
    const long long nt = (long long)((g.nx + TX - 1) / TX) * ((g.ny + kSingleTY - 1) / kSingleTY);
    const long long per = (nt + kXcds - 1) / kXcds, ch = per < kXcdChunk ? per : kXcdChunk;
    return (unsigned)((per + ch - 1) / ch * ch * kXcds);
}

template <int D, class S, class C, bool MASK> struct Launch {
    static dim3 collide_grid(const Geom &g) {
        return dim3((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, D == 3 ? (g.nz + Tile<D>::ZB - 1) / Tile<D>::ZB : 1);
    }
    static void fill_zero(hipStream_t s, void *A, long long count) {
        long long blocks = (count + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_fill_zero<S>, dim3((unsigned)blocks), dim3(256), 0, s, (S *)A, count);
    }
    static void init(hipStream_t s, void *A, const Geom &g, const uint8_t *mask, const void *prm, void *rho,
                     const double *rho0, const double *U0) {
        const Params<C> &p = *(const Params<C> *)prm;
        hipLaunchKernelGGL((k_prep_rho<C, MASK>), dim3((g.N + 255) / 256), dim3(256), 0, s, (C *)rho, rho0, mask,
                           p, g.N);
        hipLaunchKernelGGL((k_collide<D, S, C, MASK, MODE_INIT>), collide_grid(g), dim3(256), 0, s,
                           (const S *)nullptr, (S *)A, g, mask, p, (const C *)rho, (const C *)nullptr,
                           (double *)nullptr, (double *)U0);
        if constexpr (MASK)
            if (p.link_q)
                hipLaunchKernelGGL((k_wall_init<D, S, C>), dim3((g.N + 255) / 256), dim3(256), 0, s, (S *)A, g, mask,
                                   p.link_q);
    }
    static void moments(hipStream_t s, const void *A, const Geom &g, const uint8_t *mask, const void *prm, void *rho,
                        void *gfl, double *partials) {
        hipLaunchKernelGGL((k_moments<D, S, C, MASK>), moment_grid(D, g), dim3(256), 0, s, (const S *)A, g, mask,
                           *(const Params<C> *)prm, (C *)rho, (C *)gfl, partials);
    }
    static void collide(hipStream_t s, const void *A, void *B, const Geom &g, const uint8_t *mask, const void *prm,
                        const void *rho, const void *gfl) {
        hipLaunchKernelGGL((k_collide<D, S, C, MASK, MODE_STEP>), collide_grid(g), dim3(256), 0, s, (const S *)A, (S *)B, g,
                           mask, *(const Params<C> *)prm, (const C *)rho, (const C *)gfl, nullptr, nullptr);
    }
    static void single(hipStream_t s, const void *A, void *B, const Geom &g, const uint8_t *mask, const void *prm) {
        if constexpr (D == 2)
            hipLaunchKernelGGL((k_collide<D, S, C, MASK, MODE_SINGLE>), dim3(single_blocks(g)),
                               dim3(TX * kSingleTY), 0, s,
                               (const S *)A, (S *)B, g, mask, *(const Params<C> *)prm, (const C *)nullptr,
                               (const C *)nullptr, nullptr, nullptr);
    }
    static void pressure(hipStream_t s, const void *A, const Geom &g, const uint8_t *mask, const void *prm,
                         const void *rho, double *out) {
        hipLaunchKernelGGL((k_collide<D, S, C, MASK, MODE_PT>), collide_grid(g), dim3(256), 0, s, (const S *)A,
                           (S *)nullptr, g, mask, *(const Params<C> *)prm, (const C *)rho, (const C *)nullptr, nullptr,
                           out);
    }
    static void output(hipStream_t s, const void *A, const Geom &g, const uint8_t *mask, const void *prm,
                       const void *rho, const void *gfl, double *orho, double *oU) {
        hipLaunchKernelGGL((k_collide<D, S, C, MASK, MODE_OUT>), collide_grid(g), dim3(256), 0, s, (const S *)A,
                           (S *)nullptr, g, mask, *(const Params<C> *)prm, (const C *)rho, (const C *)gfl, orho, oU);
    }
    static KernelSet set() {
        KernelSet k;
        k.fill_zero = fill_zero;
        k.init = init;
        k.moments = moments;
        k.collide = collide;
        k.single = D == 2 ? single : nullptr;
        k.output = output;
        k.pressure = pressure;
        k.moment_blocks = 0;
        return k;
    }
};

}  // namespace

int moment_block_count(int D, const Geom &g) {
    dim3 gr = moment_grid(D, g);
    return (int)(gr.x * gr.y * gr.z);
}

KernelSet kernel_set(int D, bool fp64, bool masked) {
    if (D == 2) {
        if (fp64) return masked ? Launch<2, double, double, true>::set() : Launch<2, double, double, false>::set();
        return masked ? Launch<2, float, float, true>::set() : Launch<2, float, float, false>::set();
    }
    if (fp64) return masked ? Launch<3, double, double, true>::set() : Launch<3, double, double, false>::set();
    return masked ? Launch<3, float, float, true>::set() : Launch<3, float, float, false>::set();
}

long long reduce_scratch_rows(int n) {
    long long rows = 0;
    for (long long m = n; m > 1;) {
        m = (m + kReduceRows - 1) / kReduceRows;
        rows += m;
    }
    return rows + 1;
}

void launch_reduce(hipStream_t s, const double *partials, int n, double *scratch, double *totals) {
    // levels of k_reduce until one row is left; the intermediate rows go to consecutive
    // regions of scratch, the last level writes totals
    const double *src = partials;
    double *dst = scratch;
    long long m = n;
    do {
        const long long nb = (m + kReduceRows - 1) / kReduceRows;
        double *out = nb == 1 ? totals : dst;
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, src, (int)m, out);
        src = out;
        dst += nb * kPartialSlots;
        m = nb;
    } while (m > 1);
}

}  // namespace lbm
