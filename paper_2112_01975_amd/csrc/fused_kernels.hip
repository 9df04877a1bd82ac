// fused_kernels.hip -- single-pass D3Q27 stream-collide step with a z-march (gfx950).
//
// One workgroup owns a TX x TY column tile of (x, y) and marches over a chunk of
// TZ planes in z. For every plane p it pulls the 27 populations of each node of
// the tile plus a two-node halo ((TX + 4) x (TY + 4) nodes), forms rho, the signed
// pseudo-potential (eq force_form) and g = rho u^3, and keeps rho / s*psi in a
// six-plane LDS ring. Two planes later, when planes z-2..z+2 are resident, the
// tile's plane z is collided: the two-ring Korteweg force (eq Kforce_final) is
// read from the ring, the diagonal correction (eq correction) from g held in
// registers (x, y differences) and a four-plane register window (z difference),
// and the populations are pulled again (the re-read hits L2 / MALL: the same
// lines were fetched two planes earlier) and written in pull layout to B.
// Only the populations move through HBM: ~2 Q s bytes per lattice update, with
// halo and chunk-boundary re-reads served from cache when neighbouring tiles are
// co-resident (tiles are mapped so that each XCD works on a compact block).
#include <hip/hip_runtime.h>
#include <math.h>

#include "fused.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "step_common.hpp"

namespace lbm {

namespace {

constexpr int NXCD = 8;   // MI355X: 8 XCDs, workgroups dispatched round-robin

template <class S, class C, bool MASK, int FTX, int TY, bool QUEUE>
__global__ __launch_bounds__(FTX * TY) void k_fused3(const S *__restrict__ A, S *__restrict__ B, Geom g,
                                                      const uint8_t *__restrict__ mask, Params<C> p, FusedGrid fg) {
    constexpr int NT = FTX * TY;
    constexpr int HX = FTX + 4, HY = TY + 4, HP = HX * HY;
    constexpr int NHALO = HP - FTX * TY;
    constexpr int RING = 6;
    __shared__ C s_rho[RING * HP];
    __shared__ C s_psi[RING * HP];
    __shared__ C s_gxy[2][2][HP];

    // XCD-aware work item: consecutive items on one XCD are spatial neighbours
    const int b = blockIdx.x;
    const int item = (b % NXCD) * fg.per_xcd + b / NXCD;
    if (item >= fg.items) return;
    const int tix = item % fg.ntx;
    const int rest = item / fg.ntx;
    const int tiy = rest % fg.nty;
    const int zc = rest / fg.nty;
    const int x0 = tix * FTX, y0 = tiy * TY, z0 = zc * fg.tz;

    const PopBuf<S> Ab(A, g.qs, fg.pop_bytes), Bb(B, g.qs, fg.pop_bytes);
    const int t = threadIdx.x;
    const int tx = t & (FTX - 1), ty = t / FTX;
    const int e_int = (ty + 2) * HX + tx + 2;
    const bool own = (x0 + tx < g.nx) && (y0 + ty < g.ny);
    const int nxy = g.nx * g.ny;
    // loop-invariant neighbour coordinates of this thread's interior node
    int ixs[3], iry[3];
    {
        const int gx = wrapi(x0 + tx, g.nx), gy = wrapi(y0 + ty, g.ny);
        ixs[0] = wrapi(gx - 1, g.nx); ixs[1] = gx; ixs[2] = wrapi(gx + 1, g.nx);
        iry[0] = g.nx * wrapi(gy - 1, g.ny); iry[1] = g.nx * gy; iry[2] = g.nx * wrapi(gy + 1, g.ny);
    }
    // ... and of the (at most one) halo node it fills: rows 0, 1, TY+2, TY+3, then
    // columns 0, 1, HX-2, HX-1 of the staged plane
    static_assert(NHALO <= NT, "one halo node per thread at most");
    const bool has_halo = t < NHALO;
    int e_halo = 0, hxs[3] = {0, 0, 0}, hry[3] = {0, 0, 0};
    if (has_halo) {
        int lx, ly;
        if (t < 4 * HX) {
            const int r = t / HX;
            lx = t % HX;
            ly = r < 2 ? r : TY + r;
        } else {
            const int q = t - 4 * HX, c4 = q % 4;
            ly = 2 + q / 4;
            lx = c4 < 2 ? c4 : FTX + c4;
        }
        e_halo = ly * HX + lx;
        const int hx = wrapi(x0 - 2 + lx, g.nx), hy = wrapi(y0 - 2 + ly, g.ny);
        hxs[0] = wrapi(hx - 1, g.nx); hxs[1] = hx; hxs[2] = wrapi(hx + 1, g.nx);
        hry[0] = g.nx * wrapi(hy - 1, g.ny); hry[1] = g.nx * hy; hry[2] = g.nx * wrapi(hy + 1, g.ny);
    }

    // register windows: gz of planes z-1..z+2, dgx/dgy of planes z..z+2
    C gz_m1 = C(0), gz_0 = C(0), gz_p1 = C(0), gz_p2 = C(0);
    C dgx_0 = C(0), dgx_p1 = C(0), dgx_p2 = C(0);
    C dgy_0 = C(0), dgy_p1 = C(0), dgy_p2 = C(0);
    // QUEUE: the populations this thread pulled for planes z, z+1, z+2 stay in registers
    // until plane z is collided (no second pull); otherwise they are pulled again.
    C q0[27], q1[27], q2[27];
    C m0[4], m1[4], m2[4];   // QUEUE: (sum h, j) of the queued planes

#pragma unroll 1
    for (int k = -4; k < fg.tz; ++k) {
        // ---------------- gather plane pz = z0 + k + 2 into ring slot (k + 4) % 6
        const int pz = wrapi(z0 + k + 2, g.nz);
        const int pl[3] = {nxy * wrapi(pz - 1, g.nz), nxy * pz, nxy * wrapi(pz + 1, g.nz)};
        const int slot = ((k + 4) % RING) * HP;
        const int buf = (k + 4) & 1;
        {
            C rho, ga[3] = {C(0), C(0), C(0)};
            const int n = ixs[1] + iry[1] + pl[1];
            if (MASK && mask[n]) {
                rho = p.rho_w;
            } else {
                C (&h)[27] = q2;
                gather_buf<3, S, C, MASK>(Ab, mask, Nbr<3>(ixs, iry, pl), n, h);
                C sum, j[3];
                moments_of<3, C>(h, sum, j);
                m2[0] = sum; m2[1] = j[0]; m2[2] = j[1]; m2[3] = j[2];
                rho = p.rho_ref + sum;
                const C rinv = rcp(rho);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const C ua = j[a] * rinv;
                    ga[a] = rho * ua * ua * ua;
                }
            }
            s_rho[slot + e_int] = rho;
            s_psi[slot + e_int] = signed_psi(p.eos, rho);
            s_gxy[buf][0][e_int] = ga[0];
            s_gxy[buf][1][e_int] = ga[1];
            gz_p2 = ga[2];
        }
        if (has_halo) {
            C rho, ga[2] = {C(0), C(0)};
            const int n = hxs[1] + hry[1] + pl[1];
            if (MASK && mask[n]) {
                rho = p.rho_w;
            } else {
                C h[27];
                gather_buf<3, S, C, MASK>(Ab, mask, Nbr<3>(hxs, hry, pl), n, h);
                C sum, j[3];
                moments_of<3, C>(h, sum, j);
                rho = p.rho_ref + sum;
                const C rinv = rcp(rho);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const C ua = j[a] * rinv;
                    ga[a] = rho * ua * ua * ua;
                }
            }
            s_rho[slot + e_halo] = rho;
            s_psi[slot + e_halo] = signed_psi(p.eos, rho);
            s_gxy[buf][0][e_halo] = ga[0];
            s_gxy[buf][1][e_halo] = ga[1];
        }
        __syncthreads();
        dgx_p2 = s_gxy[buf][0][e_int + 1] - s_gxy[buf][0][e_int - 1];
        dgy_p2 = s_gxy[buf][1][e_int + HX] - s_gxy[buf][1][e_int - HX];

        // ---------------- collide plane z = z0 + k
        const int z = z0 + k;
        if (k >= 0 && own && z < g.nz) {
            const int zpl[3] = {nxy * wrapi(z - 1, g.nz), nxy * z, nxy * wrapi(z + 1, g.nz)};
            const int n = ixs[1] + iry[1] + zpl[1];
            if (!(MASK && mask[n])) {
                const int sb = (k + 2) % RING;   // ring slot of plane z
                const int base[5] = {((sb + 4) % RING) * HP, ((sb + 5) % RING) * HP, sb * HP,
                                     ((sb + 1) % RING) * HP, ((sb + 2) % RING) * HP};   // planes z-2..z+2
                const C rho = s_rho[base[2] + e_int], spc = s_psi[base[2] + e_int];
                C Fp[3] = {C(0), C(0), C(0)}, Fc[3] = {C(0), C(0), C(0)};
                static_for<1, 27>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr int cx = Lat<3>::c(i, 0), cy = Lat<3>::c(i, 1), cz = Lat<3>::c(i, 2);
                    constexpr int o1 = cy * HX + cx;
                    constexpr C w3 = C(3.0 * weight<3>(i));
                    const int q1 = base[2 + cz] + e_int + o1, q2 = base[2 + 2 * cz] + e_int + 2 * o1;
                    const C p1 = fabs(s_psi[q1]), p2 = fabs(s_psi[q2]);
                    const C r1 = s_rho[q1], r2 = s_rho[q2];
                    const C tp = w3 * (C(4.0 / 3.0) * p1 - C(1.0 / 6.0) * p2);
                    const C tc = w3 * (C(2) * r1 - r2);
                    static_for<0, 3>([&](auto A_) {
                        constexpr int a = decltype(A_)::value;
                        constexpr int ca = Lat<3>::c(i, a);
                        if constexpr (ca == 1) { Fp[a] += tp; Fc[a] += tc; }
                        if constexpr (ca == -1) { Fp[a] -= tp; Fc[a] -= tc; }
                    });
                });
                C Sf[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) Sf[a] = -(C(2) * spc * Fp[a] + p.kappa * rho * Fc[a]);
                C h[27];
                C drho, j[3];
                if constexpr (QUEUE) {
#pragma unroll
                    for (int i = 0; i < 27; ++i) h[i] = q0[i];
                    drho = m0[0]; j[0] = m0[1]; j[1] = m0[2]; j[2] = m0[3];
                } else {
                    gather_buf<3, S, C, MASK>(Ab, mask, Nbr<3>(ixs, iry, zpl), n, h);
                    moments_of<3, C>(h, drho, j);
                }
                const C rinv = rcp(rho);
                C u[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) u[a] = j[a] * rinv;
                const C omega = omega_of(p, rho);
                const C cf = (C(1) - C(0.5) * omega) * C(0.5);
                const C Phi[3] = {cf * dgx_0, cf * dgy_0, cf * (gz_p1 - gz_m1)};
                collide<3, C>(h, rho, drho, u, Sf, Phi, omega);
                static_for<0, 27>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    Bb.store(i, (unsigned)n, S(h[i]));
                });
            }
        }
        // ---------------- shift the register windows by one plane
        gz_m1 = gz_0; gz_0 = gz_p1; gz_p1 = gz_p2;
        dgx_0 = dgx_p1; dgx_p1 = dgx_p2;
        dgy_0 = dgy_p1; dgy_p1 = dgy_p2;
        if constexpr (QUEUE) {
#pragma unroll
            for (int i = 0; i < 27; ++i) { q0[i] = q1[i]; q1[i] = q2[i]; }
#pragma unroll
            for (int i = 0; i < 4; ++i) { m0[i] = m1[i]; m1[i] = m2[i]; }
        }
    }
}

template <class S, class C, bool MASK, int TX, int TY, bool QUEUE>
void launch_fused(hipStream_t s, const void *A, void *B, const Geom &g, const uint8_t *mask, const void *prm,
                  const FusedGrid &fg) {
    hipLaunchKernelGGL((k_fused3<S, C, MASK, TX, TY, QUEUE>), dim3(fg.blocks), dim3(TX * TY), 0, s, (const S *)A, (S *)B, g,
                       mask, *(const Params<C> *)prm, fg);
}

}  // namespace

FusedGrid fused_grid(const Geom &g, int tx, int ty, int tz) {
    FusedGrid f;
    f.tx = tx;
    f.ty = ty;
    f.tz = tz;
    f.ntx = (g.nx + tx - 1) / tx;
    f.nty = (g.ny + ty - 1) / ty;
    f.nzc = (g.nz + tz - 1) / tz;
    f.items = f.ntx * f.nty * f.nzc;
    f.per_xcd = (f.items + NXCD - 1) / NXCD;
    f.blocks = f.per_xcd * NXCD;
    return f;
}

namespace {
template <int TX, int TY, bool QUEUE> FusedLaunch pick(bool masked) {
    return masked ? launch_fused<float, float, true, TX, TY, QUEUE> : launch_fused<float, float, false, TX, TY, QUEUE>;
}
}  // namespace

FusedLaunch fused_launcher(bool fp64, bool masked, int tx, int ty, bool queue) {
    if (fp64) return nullptr;
    if (queue) {
        if (tx == 64 && ty == 8) return pick<64, 8, true>(masked);
        if (tx == 32 && ty == 8) return pick<32, 8, true>(masked);
        if (tx == 32 && ty == 16) return pick<32, 16, true>(masked);
        return nullptr;
    }
    if (tx == 64 && ty == 8) return pick<64, 8, false>(masked);
    if (tx == 32 && ty == 8) return pick<32, 8, false>(masked);
    if (tx == 32 && ty == 16) return pick<32, 16, false>(masked);
    return nullptr;
}

}  // namespace lbm
