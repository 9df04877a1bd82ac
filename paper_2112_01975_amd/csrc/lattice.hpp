// lattice.hpp -- compile-time lattice tables and equation-of-state device code.
//
// Velocity sets (eq d3q27vel): D3Q27 = {-1,0,1}^3, D2Q9 = {-1,0,1}^2. This
// library orders them as: index 0 = rest, then H "positive" links, then their
// opposites in the same order, so opp(i) = i +- H. Weights come from the
// product form at xi = 0, zeta = 1/3 (eq wi): per axis 2/3 for c = 0 and 1/6
// for c = +-1.
#pragma once
#include <hip/hip_runtime.h>
#include <utility>

namespace lbm {

template <int D> struct Lat;

template <> struct Lat<2> {
    static constexpr int Q = 9;
    static constexpr int H = 4;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[9][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}, {1, -1},
                                 {-1, 0}, {0, -1}, {-1, -1}, {-1, 1}};
        return a < 2 ? t[i][a] : 0;
    }
};

template <> struct Lat<3> {
    static constexpr int Q = 27;
    static constexpr int H = 13;
    __host__ __device__ static constexpr int c(int i, int a) {
        constexpr int t[27][3] = {
            {0, 0, 0},
            {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1},
            {0, 1, 1}, {0, 1, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1},
            {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, 0}, {-1, 1, 0}, {-1, 0, -1}, {-1, 0, 1},
            {0, -1, -1}, {0, -1, 1}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}};
        return t[i][a];
    }
};

template <int D> __host__ __device__ constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= Lat<D>::H ? i + Lat<D>::H : i - Lat<D>::H);
}

__host__ __device__ constexpr double axis_w(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

template <int D> __host__ __device__ constexpr double weight(int i) {
    return axis_w(Lat<D>::c(i, 0)) * axis_w(Lat<D>::c(i, 1)) * (D == 3 ? axis_w(Lat<D>::c(i, 2)) : 1.0);
}

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, class F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(static_cast<F &&>(f));
    }
}

// ---------------------------------------------------------------- EOS (Sec. 3.1)
enum { EOS_VDW = 0, EOS_PR = 1, EOS_RKS = 2, EOS_CS = 3, EOS_IDEAL = 4, EOS_SC1 = 5, EOS_SC2 = 6 };

// Reciprocal and square root in compute precision: FP32 uses the hardware
// v_rcp_f32 / v_sqrt_f32 (1 ulp); FP64 keeps the correctly rounded operations.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_c(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_c(double x) { return sqrt(x); }
__device__ __forceinline__ float exp_c(float x) { return expf(x); }
__device__ __forceinline__ double exp_c(double x) { return exp(x); }

template <class C> struct Eos {
    int kind;
    C RT;   // R * T with T = T_reduced * Tc
    C aa;   // a * alpha(T) (alpha = 1 for vdW and CS); the coupling G for Shan-Chen
    C b;

    // P(rho) with a single reciprocal of the combined denominator
    __device__ __forceinline__ C pressure(C r) const {
        const C one = C(1);
        const C m = one - b * r;
        switch (kind) {
        case EOS_VDW: return r * RT * rcp(m) - aa * r * r;
        case EOS_PR: {
            const C q = one + C(2) * b * r - b * b * r * r;
            return (r * RT * q - aa * r * r * m) * rcp(m * q);
        }
        case EOS_RKS: {
            const C q = one + b * r;
            return (r * RT * q - aa * r * r * m) * rcp(m * q);
        }
        case EOS_CS: {
            const C e = C(0.25) * b * r;
            const C me = one - e;
            return r * RT * (one + e + e * e - e * e * e) * rcp(me * me * me) - aa * r * r;
        }
        case EOS_SC1: {   // P = rho/3 + (G/6) psi^2, psi = 1 - exp(-rho)
            const C s = one - exp_c(-r);
            return r * C(1.0 / 3.0) + aa * C(1.0 / 6.0) * s * s;
        }
        case EOS_SC2: {   // psi = exp(-1/rho): psi^2 = exp(-2/rho)
            return r * C(1.0 / 3.0) + aa * C(1.0 / 6.0) * exp_c(C(-2) * rcp(r));
        }
        default: return r * C(1.0 / 3.0);
        }
    }
    // largest admissible density (repulsive pole); infinity for the ideal gas
    __device__ __forceinline__ bool in_domain(C r) const {
        if (!(r > C(0))) return false;
        if (kind == EOS_VDW || kind == EOS_PR || kind == EOS_RKS) return b * r < C(1);
        if (kind == EOS_CS) return C(0.25) * b * r < C(1);
        return true;
    }
};

// signed pseudo-potential s*psi with psi = sqrt|P - P0|, P0 = rho/3, s = +1 iff P > P0
// (eq force_form); neighbours use |s psi|, the centre its sign.
template <class C> __device__ __forceinline__ C signed_psi(const Eos<C> &e, C r) {
    C d = e.pressure(r) - r * C(1.0 / 3.0);
    C s = sqrt_c(fabs(d));
    return d > C(0) ? s : -s;
}

}  // namespace lbm
