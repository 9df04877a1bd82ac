// step_common.hpp -- device code shared by the two-pass and the fused step kernels:
// pull gather with halfway or interpolated bounce-back, moments, and the deviation-form
// collision.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {

__device__ __forceinline__ int wrapi(int v, int n) {
    if ((unsigned)v < (unsigned)n) return v;
    v %= n;
    return v < 0 ? v + n : v;
}

// virtual density of solid node n (Sec. 4.5): per node when a wall field is given
template <class C> __device__ __forceinline__ C wall_density(const Params<C> &p, int n) {
    return p.rho_wf ? p.rho_wf[n] : p.rho_w;
}

template <class C> __device__ __forceinline__ C omega_of(const Params<C> &p, C rho) {
    if (!p.var_visc) return p.omega_l;
    C s = (rho - p.rho_v) / (p.rho_l - p.rho_v);
    s = s < C(0) ? C(0) : (s > C(1) ? C(1) : s);
    C nu = p.nu_v + (p.nu_l - p.nu_v) * s;
    return rcp(C(3) * nu + C(0.5));
}

// wrapped neighbour coordinates of (x, y, z): xs[k] = x + k - 1, ro[j][l] = row offset of (y + j - 1, z + l - 1)
template <int D> struct Nbr {
    int xs[3];
    int ro[3][3];
    __device__ __forceinline__ Nbr(const Geom &g, int x, int y, int z) {
        xs[0] = wrapi(x - 1, g.nx); xs[1] = x; xs[2] = wrapi(x + 1, g.nx);
        int ys[3] = {wrapi(y - 1, g.ny), y, wrapi(y + 1, g.ny)};
        if constexpr (D == 3) {
            int zs[3] = {wrapi(z - 1, g.nz), z, wrapi(z + 1, g.nz)};
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int l = 0; l < 3; ++l) ro[j][l] = g.px * (ys[j] + g.ny * zs[l]);
        } else {
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int l = 0; l < 3; ++l) ro[j][l] = g.px * ys[j];
        }
    }
    // from per-axis wrapped coordinates already multiplied out: xs = x-1, x, x+1;
    // ry = nx * (y-1, y, y+1); pz = nx * ny * (z-1, z, z+1)
    __device__ __forceinline__ Nbr(const int (&xs_)[3], const int (&ry)[3], const int (&pz)[3]) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xs[k] = xs_[k];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int l = 0; l < 3; ++l) ro[j][l] = ry[j] + pz[l];
    }
    // node index of r + k*c for k = +-1
    __device__ __forceinline__ int at(int dx, int dy, int dz) const { return xs[1 + dx] + ro[1 + dy][1 + dz]; }
};

// Element idx of the array that starts at `base`, addressed as a uniform 64-bit base plus
// a 32-bit byte offset: the compiler then issues global loads/stores with an SGPR base
// and one VGPR offset (saddr form) instead of a 64-bit address per lane. Every
// population array is smaller than 4 GiB (checked when a context is created).
template <class T> __device__ __forceinline__ T ld_at(const T *__restrict__ base, unsigned idx) {
    return *(const T *)((const char *)base + idx * (unsigned)sizeof(T));
}
template <class T> __device__ __forceinline__ void st_at(T *__restrict__ base, unsigned idx, T v) {
    *(T *)((char *)base + idx * (unsigned)sizeof(T)) = v;
}
// The same store with the non-temporal cache policy, for a lattice that the step writing it
// does not read again (its lines then do not displace the ones being read from L2).
template <class T> __device__ __forceinline__ void st_nt_at(T *__restrict__ base, unsigned idx, T v) {
    __builtin_nontemporal_store(v, (T *)((char *)base + idx * (unsigned)sizeof(T)));
}

// Population i arriving at fluid node n whose source n - c_i is solid. Halfway bounce-back
// returns the opposite post-collision population of n itself. With wall fractions lq
// ([Q][qs]; the link n -> n - c_i is stored under opp(i)) the linearly interpolated
// bounce-back of Bouzidi et al. that the paper uses for curved walls (Sec. 4.5, 5.3):
//   q <  1/2: 2q A_opp(n) + (1 - 2q) A_opp(n + c_i)   (A_opp(n) when n + c_i is solid)
//   q >= 1/2: A_opp(n) / (2q) + (1 - 1/(2q)) A_i(n)
// Both weight pairs sum to one and w_i = w_opp(i), so FP32 deviations interpolate as is.
template <int D, int i, class S, class C>
__device__ __forceinline__ C wall_pull(const S *__restrict__ A, long long qs, const uint8_t *__restrict__ mask,
                                       const C *__restrict__ lq, const Nbr<D> &nb, int n) {
    constexpr int o = opp<D>(i);
    const C back = C(ld_at(A + o * qs, (unsigned)n));
    if (!lq) return back;
    const C q = ld_at(lq + o * qs, (unsigned)n);
    if (q < C(0.5)) {
        constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
        const unsigned b = (unsigned)nb.at(cx, cy, cz);
        const C behind = ld_at(mask, b) ? back : C(ld_at(A + o * qs, b));
        return C(2) * q * back + (C(1) - C(2) * q) * behind;
    }
    const C h2q = C(2) * q;
    return back / h2q + (C(1) - C(1) / h2q) * C(ld_at(A + i * qs, (unsigned)n));
}

// pull gather of the Q populations arriving at node n (= r) at this time step; lq: wall
// fractions for interpolated bounce-back, or nullptr (halfway)
template <int D, class S, class C, bool MASK>
__device__ __forceinline__ void gather(const S *__restrict__ A, long long qs, const uint8_t *__restrict__ mask,
                                       const Nbr<D> &nb, int n, C (&h)[Lat<D>::Q],
                                       const C *__restrict__ lq = nullptr) {
    static_for<0, Lat<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = Lat<D>::c(i, 0), cy = Lat<D>::c(i, 1), cz = Lat<D>::c(i, 2);
        if constexpr (i == 0) {
            h[0] = C(ld_at(A, (unsigned)n));
        } else {
            const unsigned s = (unsigned)nb.at(-cx, -cy, -cz);
            if constexpr (MASK) {
                h[i] = ld_at(mask, s) ? wall_pull<D, i, S, C>(A, qs, mask, lq, nb, n) : C(ld_at(A + i * qs, s));
            } else {
                h[i] = C(ld_at(A + i * qs, s));
            }
        }
    });
}


// sum h and j = sum c h in a fixed order (pass 1 and pass 2 must agree bit for bit)
template <int D, class C>
__device__ __forceinline__ void moments_of(const C (&h)[Lat<D>::Q], C &sum, C (&j)[3]) {
    sum = C(0);
    j[0] = j[1] = j[2] = C(0);
    static_for<0, Lat<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        sum += h[i];
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ca = Lat<D>::c(i, a);
            if constexpr (ca == 1) j[a] += h[i];
            if constexpr (ca == -1) j[a] -= h[i];
        });
    });
}

// Product-form equilibrium and extended equilibrium in deviation form, then LBGK.
// drho = sum of the pre-collision deviations (the node's mass minus rho_ref).
// Per axis the triplet Psi_c(xi, zeta) = W_c + d_c with W = (1/6, 2/3, 1/6) for
// c = (-1, 0, 1); products are differenced by telescoping so no O(1) terms cancel:
//   f_eq - w rho_ref = drho w + rho [prod(W + d) - prod W]
//   f*   - f_eq      = rho [prod(W + d + D) - prod(W + d)]
// with the x-y parts of both telescoped sums formed once per (c_x, c_y) pair.
// The update f + omega (f_eq - f) + (f* - f_eq) is evaluated as
//   (1 - omega) h + (omega drho) w + rho (omega eqd + fsd).
template <int D, class C>
__device__ __forceinline__ void collide(C (&h)[Lat<D>::Q], C rho, C drho, const C (&u)[3], const C (&S)[3],
                                        const C (&Phi)[3], C omega) {
    constexpr C W0 = C(1.0 / 6.0), W1 = C(2.0 / 3.0);
    C dv[3][3], Av[3][3], Dv[3][3], Bv[3][3];
    const C rinv = rcp(rho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const C ua = u[a], u2 = ua * ua;
        dv[a][0] = C(0.5) * (u2 - ua);
        dv[a][1] = -u2;
        dv[a][2] = C(0.5) * (u2 + ua);
        const C s = S[a] * rinv;                           // xi* - u
        const C de = s * (C(2) * ua + s) + Phi[a] * rinv;  // zeta* - zeta_eq
        Dv[a][0] = C(0.5) * (de - s);
        Dv[a][1] = -de;
        Dv[a][2] = C(0.5) * (de + s);
        Av[a][0] = W0 + dv[a][0]; Av[a][1] = W1 + dv[a][1]; Av[a][2] = W0 + dv[a][2];
#pragma unroll
        for (int k = 0; k < 3; ++k) Bv[a][k] = Av[a][k] + Dv[a][k];
    }
    // x-y factors: E = d_x A_y + W_x d_y, F = D_x B_y + A_x D_y, AA = A_x A_y
    C E[3][3], F[3][3], AA[3][3];
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const C Wx = kx == 1 ? W1 : W0;
            E[kx][ky] = dv[0][kx] * Av[1][ky] + Wx * dv[1][ky];
            F[kx][ky] = Dv[0][kx] * Bv[1][ky] + Av[0][kx] * Dv[1][ky];
            AA[kx][ky] = Av[0][kx] * Av[1][ky];
        }
    const C om1 = C(1) - omega, omd = omega * drho;
    static_for<1, Lat<D>::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int kx = Lat<D>::c(i, 0) + 1, ky = Lat<D>::c(i, 1) + 1, kz = Lat<D>::c(i, 2) + 1;
        constexpr C WW = (kx == 1 ? W1 : W0) * (ky == 1 ? W1 : W0);
        constexpr C wi = C(weight<D>(i));
        C eqd, fsd;
        if constexpr (D == 2) {
            eqd = E[kx][ky];
            fsd = F[kx][ky];
        } else {
            eqd = Av[2][kz] * E[kx][ky] + WW * dv[2][kz];
            fsd = Bv[2][kz] * F[kx][ky] + AA[kx][ky] * Dv[2][kz];
        }
        h[i] = om1 * h[i] + omd * wi + rho * (omega * eqd + fsd);
    });
    // The update conserves mass exactly (sum heq = drho, sum of the source term = 0), but
    // the rounded weights of the storage precision do not sum to one; taking the rest
    // population as the remainder keeps the per-node mass error an unbiased rounding.
    C rest = drho;
    static_for<1, Lat<D>::Q>([&](auto I) { rest -= h[decltype(I)::value]; });
    h[0] = rest;
}

}  // namespace lbm
