/*
 * lbm_oracle.c -- plain, slow FP64 reference of the two-phase lattice BGK step of
 * Hosseini, Dorschner & Karlin, "Towards a consistent lattice Boltzmann model for
 * two-phase fluid" (Sec. 2.3).
 *
 * TEST INFRASTRUCTURE ONLY. The only callers are tests/, __graft_entry__.smoke()
 * and bench.py's CPU-baseline leg. It shares no code, header or table with the HIP
 * library; its lattice tables are generated here from the product form.
 *
 * One step t -> t+1 reads every neighbour at time t (a Jacobi update) and follows
 * the paper's construction in order:
 *   1. moments rho = sum_i f_i, rho u = sum_i c_i f_i (Sec. 2.3.3); a solid node
 *      carries the virtual wall density rho_w and u = 0 (Sec. 4.5);
 *   2. equation of state P(rho) (Sec. 3.1), reference pressure P0 = rho/3 (end of
 *      Sec. 2.3), pseudo-potential psi = sqrt|P - P0| and its sign (eq force_form);
 *   3. discrete Korteweg force (eq Kforce_final): pseudo-potential pair
 *      G1 = 4/3, G2 = -1/6 (eqs PPcond1, PPcond2) and capillary pair (2, -1) kappa;
 *      the same two-ring stencils with other coefficients give the single-ring
 *      Shan-Chen force (G2 = 0, no capillary term, eq SCforce) and the dual-range
 *      force (only eq PPcond1 imposed, eq DRforce), the special cases the paper
 *      discusses after eq Kforce_final;
 *   4. momentum source S = -F (reading: the kinetic model eq gen_kinetic_model_ext
 *      enters the force with a minus sign; the literal sign is kept as a test-only
 *      variant);
 *   5. diagonal correction Phi_aa = (1 - omega/2) d_a(rho u_a^3) (eq correction with
 *      P0 = rho/3), d_a by the central difference of the two axis neighbours;
 *   6. equilibrium f_eq = rho prod Psi(u_a, 1/3 + u_a^2) (eq LBMeq) and extended
 *      equilibrium f* = rho prod Psi(xi*_a, zeta*_a) (eq LBMstar) with
 *      xi* = u + S/rho and zeta* = 1/3 + xi*^2 + Phi/rho (reading of eq zetastar
 *      that makes f* the equilibrium at the incremented velocity when Phi = 0);
 *   7. LBGK update f + omega (f_eq - f) + (f* - f_eq) (eq LBGK) and streaming to
 *      r + c_i; a link whose target is solid is reflected back into the opposite
 *      population of its own node (halfway bounce-back), or, with per-link wall
 *      distances, by the linearly interpolated bounce-back of Bouzidi et al. that the
 *      paper uses for curved walls (Sec. 4.5, Sec. 5.3).
 * Output velocity U = u + S/(2 rho) (Sec. 2.3.5, Appendix D). The discrete pressure tensor
 * of a state (Appendix E) is orc_pressure_tensor.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int lattice;            /* 2 = D2Q9, 3 = D3Q27 */
    int nx, ny, nz;
    int eos;                /* 0 vdW, 1 PR, 2 RKS, 3 CS, 4 ideal (P = rho/3), 5 SC-I, 6 SC-II */
    double a, b, R, acentric, T_reduced;
    double kappa;
    double tau_liquid, tau_vapour, rho_liquid, rho_vapour;
    double rho_wall;
    int variant;            /* test-only switches: 1 literal zeta*, 2 literal force sign, 4 no Phi,
                               8 initial velocity taken as the bare u */
    double accel[3];        /* body-force acceleration g: the source gains rho g (Sec. 4.2) */
    const double *rho_wall_field; /* NULL or [N]: wall density of each solid node (copied) */
    const double *link_q;   /* NULL or [Q][N] in this oracle's population order: for a fluid
                               node n whose link n -> n + c_i ends in a solid node, the wall's
                               fractional distance q in (0, 1] along that link (interpolated
                               bounce-back, Sec. 4.5); NULL = halfway, q = 1/2 (copied) */
    int force_model;        /* stencil coefficients (G1, G2) of eq PP_discrete and (G3, G4) of
                               eq capillary_discrete: 0 eq Kforce_final (4/3, -1/6, 2 kappa,
                               -kappa); 1 single-ring Shan-Chen force eq SCforce (1, 0, 0, 0);
                               2 dual-range force eq DRforce (force_g[0], (1 - force_g[0])/2,
                               0, 0); 3 all four from force_g */
    double force_g[4];
} orc_params;

typedef struct {
    orc_params p;
    int D, Q;
    long N;
    int c[27][3];
    double w[27];
    int opp[27];
    double T, aalpha;
    double G[4];            /* stencil coefficients G1..G4 of eqs PP_discrete, capillary_discrete */
    unsigned char *mask;    /* NULL = fully periodic */
    double *rho_wf;         /* NULL or [N]: per-node wall density */
    double *lq, *fpost;     /* interpolated bounce-back: [Q][N] link distances, post-collision */
    double *f, *fn;         /* [Q][N], pre-collision populations at time t */
    double *rho, *u, *psi, *sgn, *g, *S; /* u, g, S: [3][N] */
} orc_ctx;

/* ---- lattice from the product form (eqs d3q27vel, prod, wi) ---- */
static double psi_c(int c, double xi, double zeta)
{
    if (c == 0) return 1.0 - zeta;
    if (c == 1) return 0.5 * (xi + zeta);
    return 0.5 * (-xi + zeta);
}

int orc_lattice(int D, int *c, double *w, int *opp)
{
    int Q = (D == 3) ? 27 : 9;
    int i = 0;
    for (int cz = (D == 3 ? -1 : 0); cz <= (D == 3 ? 1 : 0); ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                int v[3] = {cx, cy, cz};
                double wi = 1.0;
                for (int a = 0; a < D; ++a) wi *= psi_c(v[a], 0.0, 1.0 / 3.0);
                if (c) { c[3 * i] = cx; c[3 * i + 1] = cy; c[3 * i + 2] = cz; }
                if (w) w[i] = wi;
                ++i;
            }
    if (opp)
        for (int k = 0; k < Q; ++k) opp[k] = Q - 1 - k;  /* enumeration is point-symmetric */
    return Q;
}

/* rho * prod_a Psi_{c_ia}(xi_a, zeta_a) for every i (eq prod) */
void orc_product_form(int D, double rho, const double *xi, const double *zeta, double *out)
{
    int c[27 * 3];
    int Q = orc_lattice(D, c, NULL, NULL);
    for (int i = 0; i < Q; ++i) {
        double v = rho;
        for (int a = 0; a < D; ++a) v *= psi_c(c[3 * i + a], xi[a], zeta[a]);
        out[i] = v;
    }
}

/* ---- equation of state (Sec. 3.1) ---- */
static double crit_temperature(const orc_params *p)
{
    switch (p->eos) {
    case 0: return 8.0 * p->a / (27.0 * p->b * p->R);
    case 1: return 0.0778 * p->a / (0.45724 * p->b * p->R);
    case 2: return 0.08664 * p->a / (0.42748 * p->b * p->R);
    case 3: return 0.18727 * p->a / (0.4963 * p->b * p->R);
    default: return 1.0 / 3.0;
    }
}

static double alpha_T(const orc_params *p)
{
    double w = p->acentric, m;
    if (p->eos == 1) m = 0.37464 + 1.54226 * w - 0.26992 * w * w;
    else if (p->eos == 2) m = 0.480 + 1.574 * w - 0.176 * w * w;
    else return 1.0;
    double s = 1.0 + m * (1.0 - sqrt(p->T_reduced));
    return s * s;
}

/* Shan-Chen equations of state (sound-speed appendix, eqs SCeos, SC1, SC2), read as
 * P = rho/3 + (G/6) psi^2 (the form whose critical points the paper prints), with
 * G = G_c / T_reduced: G_c = -4 for psi = 1 - exp(-rho), -e^2 for psi = exp(-1/rho). */
static double sc_coupling(const orc_params *p)
{
    return (p->eos == 5 ? -4.0 : -exp(2.0)) / p->T_reduced;
}

static double eos_pressure(const orc_ctx *x, double rho)
{
    const orc_params *p = &x->p;
    double RT = p->R * x->T, b = p->b;
    switch (p->eos) {
    case 5: {
        double psi = 1.0 - exp(-rho);
        return rho / 3.0 + sc_coupling(p) / 6.0 * psi * psi;
    }
    case 6: {
        double psi = exp(-1.0 / rho);
        return rho / 3.0 + sc_coupling(p) / 6.0 * psi * psi;
    }
    case 0: return rho * RT / (1.0 - b * rho) - p->a * rho * rho;
    case 1: return rho * RT / (1.0 - b * rho) - x->aalpha * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    case 2: return rho * RT / (1.0 - b * rho) - x->aalpha * rho * rho / (1.0 + b * rho);
    case 3: {
        double e = 0.25 * b * rho;
        return rho * RT * (1.0 + e + e * e - e * e * e) / ((1.0 - e) * (1.0 - e) * (1.0 - e)) - p->a * rho * rho;
    }
    default: return rho / 3.0;
    }
}

double orc_pressure(const void *h, double rho) { return eos_pressure((const orc_ctx *)h, rho); }
double orc_temperature(const void *h) { return ((const orc_ctx *)h)->T; }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- grid helpers ---- */
static long wrap(long v, long n) { long r = v % n; return r < 0 ? r + n : r; }

static long nbr(const orc_ctx *x, long n, int k, const int *c)
{
    long nx = x->p.nx, ny = x->p.ny, nz = x->p.nz;
    long ix = n % nx, iy = (n / nx) % ny, iz = n / (nx * ny);
    ix = wrap(ix + k * c[0], nx);
    iy = wrap(iy + k * c[1], ny);
    iz = wrap(iz + k * c[2], nz);
    return ix + nx * (iy + ny * iz);
}

static int solid(const orc_ctx *x, long n) { return x->mask && x->mask[n]; }

/* relaxation parameter: constant 1/tau, or nu linear in rho between the bulk phases */
static double omega_at(const orc_ctx *x, double rho)
{
    const orc_params *p = &x->p;
    if (p->tau_vapour <= 0.0) return 1.0 / p->tau_liquid;
    double nl = (p->tau_liquid - 0.5) / 3.0, nv = (p->tau_vapour - 0.5) / 3.0;
    double s = (rho - p->rho_vapour) / (p->rho_liquid - p->rho_vapour);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double nu = nv + (nl - nv) * s;
    return 1.0 / (3.0 * nu + 0.5);
}

/* Coefficients of the two-ring stencils (Sec. 2.3.4). The pseudo-potential pair (G1, G2) of
 * eq PP_discrete and the capillary pair (G3, G4) of eq capillary_discrete, the latter
 * including kappa~:
 *   Korteweg (eq Kforce_final): G1 + 2 G2 = 1 (eq PPcond1) and G1 + 8 G2 = 0 (eq PPcond2)
 *     give (4/3, -1/6); the capillary pair is (2, -1) kappa~;
 *   Shan-Chen (eq SCforce): G2 = 0 and G3 = G4 = 0, so G1 = 1 by eq PPcond1;
 *   dual range (eq DRforce): eq PPcond1 alone, G2 = (1 - G1)/2, no capillary pair;
 *   general: the four values as given.
 * Returns nonzero for an unknown model. */
static int stencil_coefficients(const orc_params *p, double G[4])
{
    switch (p->force_model) {
    case 0: G[0] = 4.0 / 3.0; G[1] = -1.0 / 6.0; G[2] = 2.0 * p->kappa; G[3] = -p->kappa; return 0;
    case 1: G[0] = 1.0; G[1] = 0.0; G[2] = 0.0; G[3] = 0.0; return 0;
    case 2: G[0] = p->force_g[0]; G[1] = 0.5 * (1.0 - p->force_g[0]); G[2] = 0.0; G[3] = 0.0; return 0;
    case 3: for (int k = 0; k < 4; ++k) G[k] = p->force_g[k]; return 0;
    default: return 1;
    }
}

/* ---- lifecycle ---- */
void orc_destroy(void *h)
{
    orc_ctx *x = (orc_ctx *)h;
    if (!x) return;
    free(x->mask); free(x->f); free(x->fn); free(x->rho); free(x->u);
    free(x->psi); free(x->sgn); free(x->g); free(x->S); free(x->rho_wf); free(x->lq); free(x->fpost);
    free(x);
}

void *orc_create(const orc_params *p, const unsigned char *mask)
{
    if (!p || (p->lattice != 2 && p->lattice != 3) || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    if (p->lattice == 2 && p->nz != 1) return NULL;
    orc_ctx *x = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    if (!x) return NULL;
    x->p = *p;
    x->D = p->lattice;
    int cf[27 * 3];
    x->Q = orc_lattice(x->D, cf, x->w, x->opp);
    for (int i = 0; i < x->Q; ++i)
        for (int a = 0; a < 3; ++a) x->c[i][a] = cf[3 * i + a];
    x->N = (long)p->nx * p->ny * p->nz;
    x->T = p->T_reduced * crit_temperature(p);
    x->aalpha = p->a * alpha_T(p);
    if (stencil_coefficients(p, x->G)) { orc_destroy(x); return NULL; }
    long N = x->N;
    x->f = (double *)calloc((size_t)x->Q * N, sizeof(double));
    x->fn = (double *)calloc((size_t)x->Q * N, sizeof(double));
    x->rho = (double *)calloc(N, sizeof(double));
    x->u = (double *)calloc(3 * N, sizeof(double));
    x->psi = (double *)calloc(N, sizeof(double));
    x->sgn = (double *)calloc(N, sizeof(double));
    x->g = (double *)calloc(3 * N, sizeof(double));
    x->S = (double *)calloc(3 * N, sizeof(double));
    if (!x->f || !x->fn || !x->rho || !x->u || !x->psi || !x->sgn || !x->g || !x->S) { orc_destroy(x); return NULL; }
    if (mask) {
        x->mask = (unsigned char *)malloc(N);
        if (!x->mask) { orc_destroy(x); return NULL; }
        memcpy(x->mask, mask, N);
    }
    x->p.rho_wall_field = NULL;
    x->p.link_q = NULL;
    if (p->link_q) {
        x->lq = (double *)malloc((size_t)x->Q * N * sizeof(double));
        x->fpost = (double *)malloc((size_t)x->Q * N * sizeof(double));
        if (!x->lq || !x->fpost) { orc_destroy(x); return NULL; }
        memcpy(x->lq, p->link_q, (size_t)x->Q * N * sizeof(double));
    }
    if (p->rho_wall_field) {
        x->rho_wf = (double *)malloc(N * sizeof(double));
        if (!x->rho_wf) { orc_destroy(x); return NULL; }
        memcpy(x->rho_wf, p->rho_wall_field, N * sizeof(double));
    }
    return x;
}

/* Initial state from the density and the velocity U of the flow. U is the velocity the
 * hydrodynamic limit transports (Sec. 2.3.5, Appendix D: U = u + F dt/(2 rho)), so the
 * bare velocity of the equilibrium is u = U - S/(2 rho), with S the source of the given
 * density field; f = f_eq(rho0, u) at fluid nodes (U0 may be NULL = at rest). */
static void source_of_density(orc_ctx *x, const double *rho);

int orc_init(void *h, const double *rho0, const double *U0)
{
    orc_ctx *x = (orc_ctx *)h;
    long N = x->N;
    int D = x->D, Q = x->Q;
    source_of_density(x, rho0);
    for (long n = 0; n < N; ++n) {
        double feq[27], xi[3] = {0, 0, 0}, zeta[3];
        if (solid(x, n)) { for (int i = 0; i < Q; ++i) x->f[i * N + n] = 0.0; continue; }
        for (int a = 0; a < D; ++a) {
            double Ua = U0 ? U0[a * N + n] : 0.0;
            xi[a] = (x->p.variant & 8) ? Ua : Ua - x->S[a * N + n] / (2.0 * rho0[n]);
            zeta[a] = 1.0 / 3.0 + xi[a] * xi[a];
        }
        orc_product_form(D, rho0[n], xi, zeta, feq);
        for (int i = 0; i < Q; ++i) x->f[i * N + n] = feq[i];
    }
    return 0;
}

/* virtual density of solid node n (Sec. 4.5): per node if given, else rho_wall */
static double wall_rho(const orc_ctx *x, long n) { return x->rho_wf ? x->rho_wf[n] : x->p.rho_wall; }

/* step 2 for every node: psi = sqrt|P - P0| and the sign of P - P0 (eq force_form) of the
 * density field x->rho */
static void pseudo_potential(orc_ctx *x)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < x->N; ++n) {
        double r = x->rho[n], P = eos_pressure(x, r), P0 = r / 3.0;
        x->psi[n] = sqrt(fabs(P - P0));
        x->sgn[n] = (P > P0) ? 1.0 : -1.0;
    }
}

/* step 3 at node n: the discrete force of eq Kforce_final (with the stencil pairs of
 * eqs PP_discrete and capillary_discrete) from x->psi, x->sgn and x->rho,
 *   F = s 2 psi(r) sum_i 3 w_i c_i [G1 psi(r + c_i) + G2 psi(r + 2 c_i)]
 *     + rho(r) sum_i 3 w_i c_i [G3 rho(r + c_i) + G4 rho(r + 2 c_i)],   3 w_i = w_i / cs^2 */
static void force_at(const orc_ctx *x, long n, double F[3])
{
    const double *G = x->G;
    double Fp[3] = {0, 0, 0}, Fc[3] = {0, 0, 0};
    for (int i = 0; i < x->Q; ++i) {
        long n1 = nbr(x, n, 1, x->c[i]), n2 = nbr(x, n, 2, x->c[i]);
        double wp = 3.0 * x->w[i] * (G[0] * x->psi[n1] + G[1] * x->psi[n2]);
        double wc = 3.0 * x->w[i] * (G[2] * x->rho[n1] + G[3] * x->rho[n2]);
        for (int a = 0; a < 3; ++a) { Fp[a] += x->c[i][a] * wp; Fc[a] += x->c[i][a] * wc; }
    }
    for (int a = 0; a < 3; ++a) F[a] = x->sgn[n] * 2.0 * x->psi[n] * Fp[a] + x->rho[n] * Fc[a];
}

/* step 4 for every node: momentum source S = -F + rho g (reading of the force sign), zero at
 * solid nodes and beyond the lattice dimension */
static void source(orc_ctx *x)
{
    long N = x->N;
    const orc_params *p = &x->p;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double F[3];
        force_at(x, n, F);
        for (int a = 0; a < 3; ++a) {
            double s = ((p->variant & 2) ? F[a] : -F[a]) + x->rho[n] * p->accel[a];
            x->S[a * N + n] = (solid(x, n) || a >= x->D) ? 0.0 : s;
        }
    }
}

/* steps 1-4: moments, EOS, pseudo-potential, g = rho u^3, source S = -F_K + rho g */
static void fields(orc_ctx *x)
{
    long N = x->N;
    int D = x->D, Q = x->Q;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double r, j[3] = {0, 0, 0};
        if (solid(x, n)) {
            r = wall_rho(x, n);
        } else {
            r = 0.0;
            for (int i = 0; i < Q; ++i) {
                double fi = x->f[i * N + n];
                r += fi;
                for (int a = 0; a < 3; ++a) j[a] += x->c[i][a] * fi;
            }
        }
        x->rho[n] = r;
        for (int a = 0; a < 3; ++a) {
            double ua = solid(x, n) ? 0.0 : j[a] / r;
            x->u[a * N + n] = (a < D) ? ua : 0.0;
            x->g[a * N + n] = (a < D) ? r * ua * ua * ua : 0.0;
        }
    }
    pseudo_potential(x);
    source(x);
}

/* steps 2-4 for a given density field (solid nodes read as rho_w): x->S = -F_K */
static void source_of_density(orc_ctx *x, const double *rho)
{
    for (long n = 0; n < x->N; ++n) x->rho[n] = solid(x, n) ? wall_rho(x, n) : rho[n];
    pseudo_potential(x);
    source(x);
}

/* steps 5-7 at one node: f -> f_post; S and Phi given; returns rho via *rho_out */
static void collide_node(const orc_ctx *x, const double *f, const double *S, const double *Phi,
                         double omega, double *out)
{
    int D = x->D, Q = x->Q;
    double r = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        for (int a = 0; a < 3; ++a) j[a] += x->c[i][a] * f[i];
    }
    double u[3], xi[3], zeq[3], zst[3], feq[27], fst[27];
    for (int a = 0; a < 3; ++a) {
        u[a] = j[a] / r;
        xi[a] = u[a] + S[a] / r;
        zeq[a] = 1.0 / 3.0 + u[a] * u[a];
        if (x->p.variant & 1)
            zst[a] = 1.0 / 3.0 + u[a] * u[a] + Phi[a] / r;
        else
            zst[a] = 1.0 / 3.0 + xi[a] * xi[a] + Phi[a] / r;
    }
    orc_product_form(D, r, u, zeq, feq);
    orc_product_form(D, r, xi, zst, fst);
    for (int i = 0; i < Q; ++i) out[i] = f[i] + omega * (feq[i] - f[i]) + (fst[i] - feq[i]);
}

void orc_collide(const void *h, const double *f, const double *S, const double *Phi, double omega, double *out)
{
    collide_node((const orc_ctx *)h, f, S, Phi, omega, out);
}

/* post-collision populations of fluid node n (steps 5-6) into fp */
static void collide_at(orc_ctx *x, long n, double *fp)
{
    long N = x->N;
    int D = x->D, Q = x->Q;
    double f[27], S[3], Phi[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) f[i] = x->f[i * N + n];
    double omega = omega_at(x, x->rho[n]);
    for (int a = 0; a < 3; ++a) S[a] = x->S[a * N + n];
    if (!(x->p.variant & 4))
        for (int a = 0; a < D; ++a) {
            int e[3] = {0, 0, 0};
            e[a] = 1;
            long np = nbr(x, n, 1, e), nm = nbr(x, n, -1, e);
            Phi[a] = (1.0 - 0.5 * omega) * 0.5 * (x->g[a * N + np] - x->g[a * N + nm]);
        }
    collide_node(x, f, S, Phi, omega, fp);
}

/* One step with interpolated bounce-back (Bouzidi et al., the scheme the paper cites for
 * walls, Sec. 4.5): every fluid node is collided first; then each post-collision
 * population streams to n + c_i, or, when that node is solid and the wall cuts the link
 * at fraction q, returns to n as the opposite population, linearly interpolated:
 *   q <  1/2: 2q fp_i(n) + (1 - 2q) fp_i(n - c_i)   (fp_i(n) if n - c_i is solid)
 *   q >= 1/2: fp_i(n)/(2q) + (1 - 1/(2q)) fp_opp(i)(n)
 * q = 1/2 is halfway bounce-back. */
static void step_interpolated(orc_ctx *x)
{
    long N = x->N;
    int Q = x->Q;
    fields(x);
    memset(x->fn, 0, sizeof(double) * (size_t)Q * N);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid(x, n)) continue;
        double fp[27];
        collide_at(x, n, fp);
        for (int i = 0; i < Q; ++i) x->fpost[i * N + n] = fp[i];
    }
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid(x, n)) continue;
        for (int i = 0; i < Q; ++i) {
            long d = nbr(x, n, 1, x->c[i]);
            double v = x->fpost[i * N + n];
            if (!solid(x, d)) {
                x->fn[i * N + d] = v;
                continue;
            }
            double q = x->lq[i * N + n], r;
            if (q < 0.5) {
                long b = nbr(x, n, -1, x->c[i]);
                r = solid(x, b) ? v : 2.0 * q * v + (1.0 - 2.0 * q) * x->fpost[i * N + b];
            } else {
                r = v / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * x->fpost[x->opp[i] * N + n];
            }
            x->fn[x->opp[i] * N + n] = r;
        }
    }
    double *tmp = x->f; x->f = x->fn; x->fn = tmp;
}

void orc_step(void *h, long steps)
{
    orc_ctx *x = (orc_ctx *)h;
    long N = x->N;
    int Q = x->Q;
    if (x->lq) {
        for (long t = 0; t < steps; ++t) step_interpolated(x);
        return;
    }
    for (long t = 0; t < steps; ++t) {
        fields(x);
        memset(x->fn, 0, sizeof(double) * (size_t)Q * N);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            if (solid(x, n)) continue;
            double fp[27];
            collide_at(x, n, fp);
            for (int i = 0; i < Q; ++i) {
                long d = nbr(x, n, 1, x->c[i]);
                if (solid(x, d))
                    x->fn[x->opp[i] * N + n] = fp[i];
                else
                    x->fn[i * N + d] = fp[i];
            }
        }
        double *tmp = x->f; x->f = x->fn; x->fn = tmp;
    }
}

/* rho (N), U = u + S/(2 rho) ([D][N]), totals = {sum rho, sum rho u_x, _y, _z} over fluid nodes */
void orc_moments(void *h, double *rho, double *U, double *totals)
{
    orc_ctx *x = (orc_ctx *)h;
    long N = x->N;
    int D = x->D;
    fields(x);
    double M = 0.0, J[3] = {0, 0, 0};
    for (long n = 0; n < N; ++n) {
        double r = x->rho[n];
        if (rho) rho[n] = r;
        for (int a = 0; a < D; ++a)
            if (U) U[a * N + n] = solid(x, n) ? 0.0 : x->u[a * N + n] + x->S[a * N + n] / (2.0 * r);
        if (!solid(x, n)) {
            M += r;
            for (int a = 0; a < D; ++a) J[a] += r * x->u[a * N + n];
        }
    }
    if (totals) { totals[0] = M; totals[1] = J[0]; totals[2] = J[1]; totals[3] = J[2]; }
}

/* momentum source S = -F_K of the current state, [3][N] */
void orc_source(void *h, double *S)
{
    orc_ctx *x = (orc_ctx *)h;
    fields(x);
    memcpy(S, x->S, sizeof(double) * 3 * (size_t)x->N);
}

/* F_K of eq Kforce_final for a given density field (all nodes read as given, solid or not);
 * overwrites the context's density and pseudo-potential fields, which the next step
 * recomputes from the populations */
void orc_korteweg_force(void *h, const double *rho, double *F)
{
    orc_ctx *x = (orc_ctx *)h;
    long N = x->N;
    memcpy(x->rho, rho, sizeof(double) * (size_t)N);
    pseudo_potential(x);
    for (long n = 0; n < N; ++n) {
        double Fn[3];
        force_at(x, n, Fn);
        for (int a = 0; a < 3; ++a) F[a * N + n] = Fn[a];
    }
}

/* Discrete pressure tensor of the current state (Appendix E), [D(D+1)/2][N] in the order
 * xx, yy, [zz,] xy[, xz, yz]; zero at solid nodes. Appendix E writes the discrete force as
 * the sum of four parts (one- and two-ring pseudo-potential and capillary terms) and gives
 * each part's tensor, with the force the negative divergence of the tensor. With the
 * reading S = -F of the momentum source, the momentum flux that the tensors complete is
 * P = Pi - (P^A + P^B + P^C + P^D), where Pi_ab = sum_i c_ia c_ib f_i is the second moment of
 * the node's pre-collision populations (the lattice momentum flux; rho/3 only without a
 * force). Per node, with 3 w_i = w_i / cs^2 and s the sign of P - P0, for the stencil pairs
 * (G1, G2) and (G3, G4) of the force (printed for (4/3, -1/6) and (2, -1) kappa, where the
 * factors are 8/6, -1/6, kappa and -kappa/2; each part is linear in its coefficient):
 *   P^A = -s G1 psi(r) sum 3w c c psi(r + c)
 *   P^B = -s G2 [psi(r) sum 3w c c psi(r + 2c) + sum 3w c c psi(r - c) psi(r + c)]
 *   P^C = -(G3/2) rho(r) sum 3w c c rho(r + c)
 *   P^D = -(G4/2) [rho(r) sum 3w c c rho(r + 2c) + sum 3w c c rho(r - c) rho(r + c)]
 * Solid nodes enter psi and rho with the wall density, as in the force. */
void orc_pressure_tensor(void *h, double *out)
{
    orc_ctx *x = (orc_ctx *)h;
    long N = x->N;
    int D = x->D, Q = x->Q;
    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    const int ncomp = D == 3 ? 6 : 3;
    int comp[6][2];
    for (int k = 0; k < ncomp; ++k) {
        int kk = D == 3 ? k : (k < 2 ? k : 3);   /* D2Q9: xx, yy, xy */
        comp[k][0] = pa[kk];
        comp[k][1] = pb[kk];
    }
    fields(x);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        for (int k = 0; k < ncomp; ++k) {
            if (solid(x, n)) { out[k * N + n] = 0.0; continue; }
            const int a = comp[k][0], b = comp[k][1];
            double pi = 0.0, sA = 0.0, sB1 = 0.0, sB2 = 0.0, sC = 0.0, sD1 = 0.0, sD2 = 0.0;
            for (int i = 0; i < Q; ++i) {
                const double cc = 3.0 * x->w[i] * x->c[i][a] * x->c[i][b];
                pi += x->c[i][a] * x->c[i][b] * x->f[i * N + n];
                if (cc == 0.0) continue;
                long p1 = nbr(x, n, 1, x->c[i]), p2 = nbr(x, n, 2, x->c[i]), m1 = nbr(x, n, -1, x->c[i]);
                sA += cc * x->psi[p1];
                sB1 += cc * x->psi[p2];
                sB2 += cc * x->psi[m1] * x->psi[p1];
                sC += cc * x->rho[p1];
                sD1 += cc * x->rho[p2];
                sD2 += cc * x->rho[m1] * x->rho[p1];
            }
            const double s = x->sgn[n], psi = x->psi[n], r = x->rho[n];
            const double *G = x->G;
            const double PA = -s * G[0] * psi * sA;
            const double PB = -s * G[1] * (psi * sB1 + sB2);
            const double PC = -0.5 * G[2] * r * sC;
            const double PD = -0.5 * G[3] * (r * sD1 + sD2);
            out[k * N + n] = pi - (PA + PB + PC + PD);
        }
    }
}

void orc_get_f(const void *h, double *out)
{
    const orc_ctx *x = (const orc_ctx *)h;
    memcpy(out, x->f, sizeof(double) * (size_t)x->Q * x->N);
}

void orc_set_f(void *h, const double *in)
{
    orc_ctx *x = (orc_ctx *)h;
    memcpy(x->f, in, sizeof(double) * (size_t)x->Q * x->N);
}
