/* The FP64 oracle (test infrastructure) built with AddressSanitizer and
 * UndefinedBehaviorSanitizer: every public entry point on small grids of both lattices,
 * every EOS and force model, masks with per-node wall densities, interpolated walls, two
 * viscosities, a body force and the test-only variants. The oracle's source is compiled
 * into this driver as it is. Exits 0 when every result is finite; a sanitizer report
 * aborts the process. */
#include "../../oracle/lbm_oracle.c"

#include <stdio.h>

static int failures = 0;

static void expect_finite(const double *v, long n, const char *what)
{
    for (long k = 0; k < n; ++k)
        if (!isfinite(v[k])) {
            fprintf(stderr, "%s[%ld] not finite\n", what, k);
            ++failures;
            return;
        }
}

/* density in [rv, rl] from a fixed integer hash of the node */
static double density(long n, double rv, double rl)
{
    unsigned long h = (unsigned long)n * 2654435761ul;
    return rv + (rl - rv) * (double)((h >> 8) % 1000) / 999.0;
}

static void run(int D, int nx, int ny, int nz, int eos, int force_model, int masked, int interp, int variant,
                double tau_vapour)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.lattice = D;
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.eos = eos;
    const int sc = eos == 5 || eos == 6;
    p.a = sc ? 0.0 : 0.02;
    p.b = sc ? 0.0 : 2.0 / 21.0;
    p.R = 1.0;
    p.acentric = eos == 1 ? 0.344 : 0.0;
    p.T_reduced = 0.8;
    p.kappa = 0.02;
    p.tau_liquid = 0.8;
    p.tau_vapour = tau_vapour;
    p.rho_vapour = sc ? 0.3 : 0.5;
    p.rho_liquid = sc ? 1.5 : 5.0;
    p.rho_wall = 1.0;
    p.variant = variant;
    p.accel[0] = 1e-5;
    p.force_model = force_model;
    p.force_g[0] = 1.2; p.force_g[1] = -0.1; p.force_g[2] = 0.03; p.force_g[3] = -0.02;
    const long N = (long)nx * ny * nz;
    int c[27 * 3], opp[27];
    double w[27];
    const int Q = orc_lattice(D, c, w, opp);
    unsigned char *mask = NULL;
    double *wall = NULL, *lq = NULL;
    if (masked) {
        mask = calloc((size_t)N, 1);
        wall = malloc((size_t)N * sizeof(double));
        for (long n = 0; n < N; ++n) {
            mask[n] = (n % 9 == 4);
            wall[n] = mask[n] ? 0.8 + 0.1 * (double)(n % 3) : 0.0;
        }
        p.rho_wall_field = wall;
        if (interp) {
            lq = malloc((size_t)Q * N * sizeof(double));
            for (long k = 0; k < (long)Q * N; ++k) lq[k] = 0.25 + 0.5 * (double)(k % 7) / 6.0;
            p.link_q = lq;
        }
    }
    void *h = orc_create(&p, mask);
    if (!h) {
        fprintf(stderr, "orc_create failed (D%d eos %d force %d)\n", D, eos, force_model);
        ++failures;
        goto done;
    }
    double *rho = malloc((size_t)N * sizeof(double)), *U = calloc((size_t)3 * N, sizeof(double));
    double *S = malloc((size_t)3 * N * sizeof(double)), *F = malloc((size_t)3 * N * sizeof(double));
    double *P = malloc((size_t)6 * N * sizeof(double)), *f = malloc((size_t)Q * N * sizeof(double));
    double tot[4];
    for (long n = 0; n < N; ++n) {
        rho[n] = density(n, p.rho_vapour, p.rho_liquid);
        U[n] = 1e-3 * (double)(n % 5);
    }
    orc_init(h, rho, U);
    orc_step(h, 3);
    orc_moments(h, rho, U, tot);
    expect_finite(rho, N, "rho");
    expect_finite(U, (long)D * N, "U");
    expect_finite(tot, 4, "totals");
    orc_source(h, S);
    expect_finite(S, 3 * N, "S");
    orc_korteweg_force(h, rho, F);
    expect_finite(F, 3 * N, "F");
    orc_pressure_tensor(h, P);
    expect_finite(P, (long)(D * (D + 1) / 2) * N, "P");
    orc_get_f(h, f);
    orc_set_f(h, f);
    orc_step(h, 1);
    {
        double fn[27], out[27], Sn[3] = {1e-4, -2e-4, 3e-4}, Phi[3] = {1e-6, 0.0, -1e-6};
        for (int i = 0; i < Q; ++i) fn[i] = w[i] * 2.0;
        orc_collide(h, fn, Sn, Phi, 1.25, out);
        expect_finite(out, Q, "collide");
    }
    if (!isfinite(orc_pressure(h, 1.0)) || !(orc_temperature(h) > 0)) ++failures;
    orc_destroy(h);
    free(rho); free(U); free(S); free(F); free(P); free(f);
done:
    free(mask); free(wall); free(lq);
}

int main(void)
{
    for (int eos = 0; eos <= 6; ++eos) {
        run(2, 9, 7, 1, eos, 0, 0, 0, 0, 0.0);
        run(3, 5, 4, 6, eos, 0, eos % 2, 0, 0, 0.0);
    }
    for (int fm = 0; fm <= 3; ++fm) {
        run(2, 8, 6, 1, 0, fm, 1, 0, 0, 0.9);
        run(3, 4, 5, 5, 1, fm, 1, 1, 0, 0.0);
    }
    run(2, 10, 7, 1, 0, 0, 1, 1, 0, 0.0);
    for (int v = 1; v <= 8; v <<= 1) run(2, 6, 5, 1, 0, 0, 0, 0, v, 0.0);
    run(2, 1, 1, 1, 0, 0, 0, 0, 0, 0.0);   /* degenerate one-node grids */
    run(3, 1, 2, 3, 4, 0, 0, 0, 0, 0.0);
    {
        double out[27], xi[3] = {0.01, -0.02, 0.03}, zeta[3] = {0.34, 0.35, 0.36};
        orc_product_form(3, 1.1, xi, zeta, out);
        expect_finite(out, 27, "product form");
    }
    if (failures) {
        fprintf(stderr, "%d failure(s)\n", failures);
        return 1;
    }
    printf("oracle driver ok (%d threads)\n", orc_max_threads());
    return 0;
}
