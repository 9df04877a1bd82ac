// runtime_common.hpp -- parameter checks and derived constants shared by the
// single-simulation and batched runtimes.
#pragma once
#include <math.h>

#include <string>
#include <vector>

#include "../../include/lbm2p.h"
#include "kernels.hpp"
#include "thermo_host.hpp"

namespace lbm {

// Element stride between population arrays: N rounded up to a 256 B multiple plus
// a 768 B (FP32) skew so that the Q arrays do not start on the same HBM channel.
inline Geom make_geom(int nx, int ny, int nz, int px = 0) {
    Geom g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.px = px > nx ? px : nx;
    g.N = g.px * ny * nz;
    g.qs = (((long long)g.N + 63) / 64) * 64 + 192;
    return g;
}

// Wall fractions of every link from a fluid node into a solid one must lie in (0, 1]; a
// node cut on both links of one axis pair with q, q' >= 1/2 needs 1/(2q) + 1/(2q') - 1 >=
// 0.01, the determinant of the 2x2 system that places its initial populations.
inline bool check_link_q(const lbm_params *p, std::string *why) {
    const int D = p->lattice == LBM_D3Q27 ? 3 : 2, Q = D == 3 ? 27 : 9;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t N = (size_t)nx * ny * nz;
    int c[27][3];
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) c[i][a] = D == 3 ? Lat<3>::c(i, a) : Lat<2>::c(i, a);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = (size_t)x + nx * ((size_t)y + (size_t)ny * z);
                if (p->mask[n]) continue;
                double qs[27];
                for (int i = 1; i < Q; ++i) {
                    const size_t d = (size_t)((x + c[i][0] + nx) % nx) +
                                     nx * ((size_t)((y + c[i][1] + ny) % ny) + (size_t)ny * ((z + c[i][2] + nz) % nz));
                    qs[i] = -1.0;
                    if (!p->mask[d]) continue;
                    const double q = p->link_q[(size_t)i * N + n];
                    if (!(q > 0.0 && q <= 1.0)) {
                        *why = "link_q must lie in (0, 1] on every link from a fluid into a solid node";
                        return false;
                    }
                    qs[i] = q;
                }
                for (int i = 1; i < Q; ++i) {
                    const int j = D == 3 ? opp<3>(i) : opp<2>(i);
                    if (qs[i] >= 0.5 && qs[j] >= 0.5 && 0.5 / qs[i] + 0.5 / qs[j] - 1.0 < 0.01) {
                        *why = "link_q: a node cut on two opposite links with q, q' >= 1/2 needs 1/(2q) + 1/(2q') >= 1.01";
                        return false;
                    }
                }
            }
    return true;
}

inline bool validate_params(const lbm_params *p, std::string *why) {
    if (!p) { *why = "params is NULL"; return false; }
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q27) { *why = "lattice must be LBM_D2Q9 or LBM_D3Q27"; return false; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { *why = "grid sizes must be >= 1"; return false; }
    if (p->lattice == LBM_D2Q9 && p->nz != 1) { *why = "D2Q9 requires nz == 1"; return false; }
    if ((double)p->nx * p->ny * p->nz >= 2147483647.0) { *why = "grid larger than 2^31 nodes"; return false; }
    if (p->eos < LBM_EOS_VDW || p->eos > LBM_EOS_SC2) { *why = "unknown equation of state"; return false; }
    const bool shan_chen = p->eos == LBM_EOS_SC1 || p->eos == LBM_EOS_SC2;
    if (p->eos != LBM_EOS_IDEAL && !shan_chen) {
        if (!(p->a > 0) || !(p->b > 0) || !(p->R > 0)) { *why = "EOS parameters a, b, R must be > 0"; return false; }
    }
    if (p->eos != LBM_EOS_IDEAL && !(p->T_reduced > 0 && isfinite(p->T_reduced))) {
        *why = "T_reduced must be > 0";
        return false;
    }
    if (!(p->kappa >= 0) || !isfinite(p->kappa)) { *why = "kappa must be finite and >= 0"; return false; }
    if (p->force_model < LBM_FORCE_KORTEWEG || p->force_model > LBM_FORCE_GENERAL) {
        *why = "unknown force model";
        return false;
    }
    for (int k = 0; k < 4; ++k)
        if (!isfinite(p->force_g[k])) { *why = "force_g must be finite"; return false; }
    if (!(p->tau_liquid > 0.5) || !isfinite(p->tau_liquid)) { *why = "tau_liquid must be > 1/2"; return false; }
    if (p->tau_vapour > 0) {
        if (!(p->tau_vapour > 0.5)) { *why = "tau_vapour must be > 1/2 (or <= 0 for constant tau)"; return false; }
        if (!(p->rho_liquid > p->rho_vapour) || !(p->rho_vapour >= 0)) {
            *why = "variable viscosity needs rho_liquid > rho_vapour >= 0";
            return false;
        }
    }
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32_DEV) { *why = "unknown precision"; return false; }
    if (!isfinite(p->rho_ref) || !isfinite(p->rho_wall)) { *why = "rho_ref and rho_wall must be finite"; return false; }
    if (p->mask && !(p->rho_wall > 0)) { *why = "a mask needs rho_wall > 0"; return false; }
    for (int a = 0; a < 3; ++a)
        if (!isfinite(p->accel[a])) { *why = "accel must be finite"; return false; }
    if (p->lattice == LBM_D2Q9 && p->accel[2] != 0.0) { *why = "D2Q9 has no z acceleration"; return false; }
    if (p->rho_wall_field && p->mask) {
        const size_t N = (size_t)p->nx * p->ny * p->nz;
        for (size_t n = 0; n < N; ++n)
            if (p->mask[n] && !(p->rho_wall_field[n] > 0)) { *why = "rho_wall_field must be > 0 at solid nodes"; return false; }
    }
    if (p->link_q) {
        if (!p->mask) { *why = "link_q needs a mask"; return false; }
        if (!check_link_q(p, why)) return false;
    }
    return true;
}

// Stencil coefficients (G1, G2, G3, G4) of the force model (Sec. 2.3.4): eq Kforce_final's
// (4/3, -1/6) from eqs PPcond1/2 and capillary pair (2, -1) kappa~; eq SCforce's single ring
// (1, 0) without capillary pair; eq DRforce's G2 = (1 - G1)/2 (eq PPcond1 only); or as given.
inline void force_coefficients(const lbm_params *p, double G[4]) {
    switch (p->force_model) {
    case LBM_FORCE_SHAN_CHEN: G[0] = 1.0; G[1] = 0.0; G[2] = 0.0; G[3] = 0.0; break;
    case LBM_FORCE_DUAL_RANGE:
        G[0] = p->force_g[0]; G[1] = 0.5 * (1.0 - p->force_g[0]); G[2] = 0.0; G[3] = 0.0;
        break;
    case LBM_FORCE_GENERAL: for (int k = 0; k < 4; ++k) G[k] = p->force_g[k]; break;
    default: G[0] = 4.0 / 3.0; G[1] = -1.0 / 6.0; G[2] = 2.0 * p->kappa; G[3] = -p->kappa; break;
    }
}

template <class C> inline void fill_params(const lbm_params *p, Params<C> *q) {
    HostEos e(p->eos, p->a, p->b, p->R, p->acentric, p->T_reduced);
    q->rho_ref = C(p->rho_ref);
    q->rho_w = C(p->rho_wall);
    double G[4];
    force_coefficients(p, G);
    // 3 w of a direction by |c|^2: D3Q27 faces 2/9, edges 1/18, corners 1/72; D2Q9 axes 1/3,
    // diagonals 1/12 (the product-form weights times 1/cs^2)
    const bool d3 = p->lattice == LBM_D3Q27;
    const double w3[3] = {d3 ? 2.0 / 9.0 : 1.0 / 3.0, d3 ? 1.0 / 18.0 : 1.0 / 12.0, d3 ? 1.0 / 72.0 : 0.0};
    for (int k = 0; k < 4; ++k) {
        q->G[k] = C(G[k]);
        for (int m = 0; m < 3; ++m) q->gw[m][k] = C(w3[m] * G[k]);
    }
    q->omega_l = C(1.0 / p->tau_liquid);
    q->var_visc = p->tau_vapour > 0 ? 1 : 0;
    q->nu_l = C((p->tau_liquid - 0.5) / 3.0);
    q->nu_v = C(p->tau_vapour > 0 ? (p->tau_vapour - 0.5) / 3.0 : 0.0);
    q->rho_l = C(p->rho_liquid);
    q->rho_v = C(p->rho_vapour);
    q->eos.kind = p->eos;
    q->eos.RT = C(p->R * e.T);
    q->eos.aa = C(e.aa);
    q->eos.b = C(p->b);
    for (int a = 0; a < 3; ++a) q->accel[a] = C(p->accel[a]);
    q->rho_wf = nullptr;   // set by the caller once the wall field is on the device
    q->link_q = nullptr;   // likewise the link fractions
}

// Pitched copy of a host array in the user layout (x fastest, rows of nx): element (x, y, z)
// at x + g.px (y + g.ny z); padding entries are zero.
template <class C, class H> inline std::vector<C> pitched(const H *host, const Geom &g) {
    std::vector<C> out((size_t)g.N, C(0));
    const size_t rows = (size_t)g.ny * g.nz;
    for (size_t r = 0; r < rows; ++r)
        for (int x = 0; x < g.nx; ++x) out[r * g.px + x] = C(host[r * g.nx + x]);
    return out;
}

// device copy of a per-node wall density field in compute precision C (solid entries
// used; fluid entries copied as given), pitched; nullptr on failure
template <class C> inline C *upload_wall_field(const double *host, const Geom &g) {
    const std::vector<C> tmp = pitched<C>(host, g);
    const size_t N = tmp.size();
    C *d = nullptr;
    if (hipMalloc((void **)&d, N * sizeof(C)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, tmp.data(), N * sizeof(C), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    return d;
}

// device copy of the wall fractions, [Q][nx ny nz] host doubles -> [Q][qs] pitched in
// compute precision (the population layout, so a kernel addresses them like a population
// array); nullptr on failure
template <class C> inline C *upload_link_q(const double *host, int Q, const Geom &g) {
    const long long qs = g.qs;
    const size_t Nu = (size_t)g.nx * g.ny * g.nz, rows = (size_t)g.ny * g.nz;
    C *d = nullptr;
    if (hipMalloc((void **)&d, (size_t)Q * (size_t)qs * sizeof(C)) != hipSuccess) return nullptr;
    std::vector<C> row((size_t)qs, C(0));   // one population at a time: host memory stays one row
    for (int i = 0; i < Q; ++i) {
        for (size_t r = 0; r < rows; ++r)
            for (int x = 0; x < g.nx; ++x) row[r * g.px + x] = C(host[(size_t)i * Nu + r * g.nx + x]);
        if (hipMemcpy(d + (size_t)i * (size_t)qs, row.data(), row.size() * sizeof(C), hipMemcpyHostToDevice) !=
            hipSuccess) {
            (void)hipFree(d);
            return nullptr;
        }
    }
    return d;
}

}  // namespace lbm
