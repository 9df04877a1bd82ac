// Host-side checks of the library's parameter validation, derived constants and
// thermodynamics (Sec. 3.1), built with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host pass only. No device code runs: every function called here is host code.
// Exits 0 when every expectation holds; a sanitizer report aborts the process.
#include <math.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "runtime_common.hpp"
#include "thermo_host.hpp"

using namespace lbm;

static int failures = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "expectation failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static lbm_params base(int lattice, int nx, int ny, int nz) {
    lbm_params p{};
    p.lattice = lattice;
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.eos = LBM_EOS_VDW;
    p.a = 9.0 / 49.0; p.b = 2.0 / 21.0; p.R = 1.0; p.T_reduced = 0.9;
    p.kappa = 0.02;
    p.tau_liquid = 0.8;
    p.rho_liquid = 6.0; p.rho_vapour = 0.5;
    p.precision = LBM_FP64;
    return p;
}

static bool valid(const lbm_params &p) {
    std::string why;
    const bool ok = validate_params(&p, &why);
    EXPECT(ok || !why.empty());
    return ok;
}

int main() {
    // validation: a valid problem, then one broken field at a time
    const lbm_params ok2 = base(LBM_D2Q9, 12, 9, 1), ok3 = base(LBM_D3Q27, 5, 6, 7);
    EXPECT(valid(ok2) && valid(ok3));
    {
        std::string why;
        EXPECT(!validate_params(nullptr, &why));
    }
    {
        lbm_params p = ok2; p.lattice = 7; EXPECT(!valid(p));
        p = ok2; p.nz = 2; EXPECT(!valid(p));
        p = ok2; p.nx = 0; EXPECT(!valid(p));
        p = ok3; p.nx = 2048; p.ny = 1024; p.nz = 1024; EXPECT(!valid(p));
        p = ok2; p.eos = 99; EXPECT(!valid(p));
        p = ok2; p.a = -1.0; EXPECT(!valid(p));
        p = ok2; p.T_reduced = NAN; EXPECT(!valid(p));
        p = ok2; p.kappa = -0.1; EXPECT(!valid(p));
        p = ok2; p.kappa = INFINITY; EXPECT(!valid(p));
        p = ok2; p.force_model = 9; EXPECT(!valid(p));
        p = ok2; p.force_model = LBM_FORCE_GENERAL; p.force_g[2] = NAN; EXPECT(!valid(p));
        p = ok2; p.tau_liquid = 0.5; EXPECT(!valid(p));
        p = ok2; p.tau_vapour = 0.4; EXPECT(!valid(p));
        p = ok2; p.tau_vapour = 0.9; p.rho_liquid = 0.1; EXPECT(!valid(p));
        p = ok2; p.precision = 5; EXPECT(!valid(p));
        p = ok2; p.rho_ref = NAN; EXPECT(!valid(p));
        p = ok2; p.accel[2] = 1e-6; EXPECT(!valid(p));
        p = ok3; p.accel[2] = 1e-6; EXPECT(valid(p));
        p = ok2; p.eos = LBM_EOS_SC1; p.a = 0.0; p.b = 0.0; EXPECT(valid(p));
        p = ok2; p.eos = LBM_EOS_IDEAL; p.a = 0.0; p.T_reduced = 0.0; EXPECT(valid(p));
    }
    // masks, wall fields and link fractions (every node and link visited)
    {
        const int nx = 7, ny = 6, nz = 5, N = nx * ny * nz, Q = 27;
        std::vector<uint8_t> mask(N, 0);
        for (int n = 0; n < N; ++n) mask[n] = (n % 11 == 0) ? 1 : 0;
        std::vector<double> wall(N, 0.0), lq((size_t)Q * N, 0.5);
        for (int n = 0; n < N; ++n) wall[n] = mask[n] ? 1.5 : 0.0;
        lbm_params p = ok3;
        p.nx = nx; p.ny = ny; p.nz = nz;
        p.mask = mask.data();
        EXPECT(!valid(p));                 // a mask needs rho_wall > 0
        p.rho_wall = 1.0;
        EXPECT(valid(p));
        p.rho_wall_field = wall.data();
        EXPECT(valid(p));
        wall[0] = 0.0;
        EXPECT(!valid(p));                 // solid node without a wall density
        wall[0] = 1.5;
        p.link_q = lq.data();
        EXPECT(valid(p));
        for (size_t k = 0; k < lq.size(); ++k) lq[k] = 0.05 + 0.9 * (double)((k * 7919) % 1000) / 1000.0;
        (void)valid(p);                    // the two-link determinant rule decides; no out-of-range access
        for (size_t k = 0; k < lq.size(); ++k) lq[k] = 1.5;
        EXPECT(!valid(p));
        lbm_params q = ok3; q.link_q = lq.data(); EXPECT(!valid(q));   // link_q needs a mask
        // pitched copies of the device layout
        const Geom g = make_geom(nx, ny, nz, 32);
        EXPECT(g.px == 32 && g.N == 32 * ny * nz && g.qs >= g.N);
        const std::vector<uint8_t> mp = pitched<uint8_t>(mask.data(), g);
        const std::vector<float> wp = pitched<float>(wall.data(), g);
        EXPECT(mp.size() == (size_t)g.N && wp.size() == (size_t)g.N);
        EXPECT(mp[g.px * 1] == mask[nx * 1] && wp[g.px * ny] == (float)wall[nx * ny]);
    }
    // derived constants for every force model, both precisions
    for (int fm = LBM_FORCE_KORTEWEG; fm <= LBM_FORCE_GENERAL; ++fm) {
        lbm_params p = ok3;
        p.force_model = fm;
        p.force_g[0] = 1.2; p.force_g[1] = -0.1; p.force_g[2] = 0.03; p.force_g[3] = -0.02;
        double G[4];
        force_coefficients(&p, G);
        EXPECT(fm == LBM_FORCE_GENERAL || fabs(G[0] + 2.0 * G[1] - 1.0) < 1e-15);
        Params<double> pd{};
        Params<float> pf{};
        fill_params(&p, &pd);
        fill_params(&p, &pf);
        for (int k = 0; k < 4; ++k) EXPECT(pd.G[k] == G[k] && isfinite(pf.gw[0][k]));
    }
    // thermodynamics of every EOS: a loop below Tc, none above
    const int eos[] = {LBM_EOS_VDW, LBM_EOS_PR, LBM_EOS_RKS, LBM_EOS_CS, LBM_EOS_SC1, LBM_EOS_SC2};
    for (int k = 0; k < 6; ++k) {
        const bool sc = eos[k] == LBM_EOS_SC1 || eos[k] == LBM_EOS_SC2;
        for (double tr : {0.6, 0.8, 0.95}) {
            HostEos e(eos[k], sc ? 0.0 : 0.02, sc ? 0.0 : 2.0 / 21.0, 1.0, eos[k] == LBM_EOS_PR ? 0.344 : 0.0, tr);
            double rv, rl, ps, sigma, kappa;
            EXPECT(coexistence(e, &rv, &rl, &ps) == 0 && rv > 0 && rl > rv && isfinite(ps));
            EXPECT(surface_tension(e, 0.02, &sigma) == 0 && sigma > 0);
            EXPECT(kappa_for_width(e, 5.0, &kappa) == 0 && kappa > 0);
            EXPECT(isfinite(e.P(0.5 * (rv + rl))) && isfinite(e.dP(rv)));
        }
        HostEos hot(eos[k], sc ? 0.0 : 0.02, sc ? 0.0 : 2.0 / 21.0, 1.0, 0.0, 1.2);
        double rv, rl, ps;
        EXPECT(coexistence(hot, &rv, &rl, &ps) != 0);
    }
    EXPECT(fabs(critical_temperature(LBM_EOS_VDW, 9.0 / 49.0, 2.0 / 21.0, 1.0) -
                8.0 * (9.0 / 49.0) / (27.0 * (2.0 / 21.0))) < 1e-14);
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("host driver ok\n");
    return 0;
}
