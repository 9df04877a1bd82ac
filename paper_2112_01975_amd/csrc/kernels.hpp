// kernels.hpp -- host-side view of the step kernels (launch wrappers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

// Grid geometry. Device arrays are pitched in x: node (x, y, z) is stored at
// n = x + px (y + ny z) with px >= nx (rows padded to whole cache lines; the padding
// nodes x >= nx are never read into real nodes nor written). N = px ny nz < 2^31 stored
// nodes; qs = element stride between the Q population arrays.
struct Geom {
    int nx, ny, nz;
    int px;
    int N;
    long long qs;
};

// per-simulation constants of the step in compute precision C
template <class C> struct Params {
    C rho_ref;      // deviation-storage reference density (0 for plain FP64 storage)
    C rho_w;        // virtual wall density
    C G[4];         // stencil coefficients: G1, G2 (pseudo-potential rings), G3, G4 (capillary
                    // rings, kappa~ included)
    C gw[3][4];     // 3 w G_k for the weight class |c|^2 - 1 of a direction: the factors of
                    // the ring terms, so that a direction costs a multiply and an add
    C omega_l;      // 1/tau_liquid
    C nu_l, nu_v;   // kinematic viscosities of the bulk phases (variable-viscosity mode)
    C rho_l, rho_v; // bulk densities of the viscosity interpolation
    int var_visc;
    Eos<C> eos;
    C accel[3];       // body-force acceleration g: the source gains rho g
    const C *rho_wf;  // device [N] wall density of each solid node, or nullptr (rho_w)
    const C *link_q;  // device [Q][qs] wall fraction of the link n -> n + c_j, or nullptr (halfway)
};

// number of reduction slots written per workgroup by the moment pass
constexpr int kPartialSlots = 5;   // sum rho, sum j_x, j_y, j_z, domain-error count

// one table of launchers per (lattice, precision, mask) combination
struct KernelSet {
    // zero the population array (fill kernel, safe under graph capture)
    void (*fill_zero)(hipStream_t, void *A, long long count);
    // f = f_eq(rho0, u) with u = U0 - S/(2 rho0), written in pull layout with bounce-back
    // links folded in; rho is the compute-precision density scratch field
    // populations folded for halfway bounce-back; with link_q the wall slots are then
    // re-solved so that the interpolated pull returns the same equilibria
    void (*init)(hipStream_t, void *A, const Geom &, const uint8_t *mask, const void *params, void *rho,
                 const double *rho0, const double *U0);
    // rho and g = rho u^3 of the current state, per-workgroup FP64 partials
    void (*moments)(hipStream_t, const void *A, const Geom &, const uint8_t *mask, const void *params,
                    void *rho, void *g, double *partials);
    // one collide-stream step A -> B (reads rho, g written by moments)
    void (*collide)(hipStream_t, const void *A, void *B, const Geom &, const uint8_t *mask, const void *params,
                    const void *rho, const void *g);
    // one collide-stream step A -> B in a single pass, rho and g from the tile's own pulls
    // (D2Q9; nullptr for D3Q27)
    void (*single)(hipStream_t, const void *A, void *B, const Geom &, const uint8_t *mask, const void *params);
    // rho and U = u + S/(2 rho) of the current state in FP64 (reads rho, g)
    void (*output)(hipStream_t, const void *A, const Geom &, const uint8_t *mask, const void *params,
                   const void *rho, const void *g, double *out_rho, double *out_U);
    // discrete pressure tensor of the state in A (reads rho written by moments), FP64
    // [D(D+1)/2][N] into out
    void (*pressure)(hipStream_t, const void *A, const Geom &, const uint8_t *mask, const void *params,
                     const void *rho, double *out);
    int moment_blocks;  // filled by kernel_blocks()
};

KernelSet kernel_set(int D, bool fp64, bool masked);
int moment_block_count(int D, const Geom &g);

// deterministic FP64 tree over n partial rows of kPartialSlots values -> totals[0..4]: levels
// of 2048 rows per workgroup; scratch holds reduce_scratch_rows(n) rows of intermediate sums
void launch_reduce(hipStream_t s, const double *partials, int n, double *scratch, double *totals);
long long reduce_scratch_rows(int n);

}  // namespace lbm
