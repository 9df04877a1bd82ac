/*
 * lbm2p.h -- C ABI of the MI355X (gfx950) two-phase lattice Boltzmann library.
 *
 * The library advances the lattice BGK model of Hosseini, Dorschner & Karlin,
 * "Towards a consistent lattice Boltzmann model for two-phase fluid", Sec. 2.3:
 * populations on the D2Q9 or D3Q27 lattice (eq d3q27vel; D2Q9 drops z), a
 * non-ideal equation of state entering through the pseudo-potential and the
 * capillary Korteweg force on two neighbour rings (eq Kforce_final), the
 * product-form equilibrium and extended equilibrium (eqs LBMeq, LBMstar) with
 * the diagonal correction (eq correction), and the LBGK update (eq LBGK).
 *
 * Conventions for every entry point:
 *   - return LBM_OK (0) on success or a negative LBM_E_* code; the message is
 *     available from lbm_last_error();
 *   - host arrays are owned by the caller and only read or written during the
 *     call; all host fields are FP64 whatever the storage precision;
 *   - node index n = x + nx*(y + ny*z), x fastest; vector fields are SoA [D][N];
 *   - a context owns all of its device memory and one HIP stream; it is bound
 *     to the device that was current at lbm_create and must be used from one
 *     host thread at a time; different contexts are independent;
 *   - errors raised by the watchdog (LBM_E_DIVERGED, LBM_E_DOMAIN) are sticky
 *     until the next successful lbm_init_fields / lbm_set_populations.
 */
#ifndef LBM2P_H
#define LBM2P_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_E_INVAL (-1)    /* bad argument or parameter */
#define LBM_E_NOMEM (-2)    /* device or host allocation failed */
#define LBM_E_HIP (-3)      /* a HIP runtime call failed */
#define LBM_E_DOMAIN (-4)   /* rho <= 0, b*rho >= 1 (outside the EOS domain) or no van der Waals loop */
#define LBM_E_DIVERGED (-5) /* non-finite values at a watchdog check */
#define LBM_E_STATE (-6)    /* call out of order (e.g. step before init) */

enum { LBM_D2Q9 = 0, LBM_D3Q27 = 1 };
/* Equations of state of Sec. 3.1: van der Waals (eq vdWEoS), Peng-Robinson
 * (eq PREoS), Redlich-Kwong-Soave (eq RKSEoS), Carnahan-Starling (eq CSEos);
 * LBM_EOS_IDEAL is P = rho/3 = P0, i.e. no non-ideal force (plain LBGK).
 * LBM_EOS_SC1 / LBM_EOS_SC2 are the Shan-Chen equations of state of the sound-speed
 * appendix (eqs SCeos, SC1, SC2), P = rho/3 + (G/6) psi^2 with psi = 1 - exp(-rho) or
 * exp(-1/rho), in the form whose critical points the paper prints (G_c = -4 at
 * rho_c = ln 2; G_c = -e^2 at rho_c = 1). Their coupling is G = G_c / T_reduced, a
 * pseudo-temperature with liquid-vapour coexistence for T_reduced < 1; a, b, R and
 * the acentric factor are not used. */
enum { LBM_EOS_VDW = 0, LBM_EOS_PR = 1, LBM_EOS_RKS = 2, LBM_EOS_CS = 3, LBM_EOS_IDEAL = 4,
       LBM_EOS_SC1 = 5, LBM_EOS_SC2 = 6 };
/* Stencil coefficients of the non-ideal force (Sec. 2.3.4): the pseudo-potential ring
 * pair (G1, G2) of eq PP_discrete and the capillary pair (G3, G4) of eq capillary_discrete,
 *   dt F = s 2 psi(r) sum_i (w_i/cs^2) c_i [G1 psi(r + c_i) + G2 psi(r + 2 c_i)]
 *        + rho(r) sum_i (w_i/cs^2) c_i [G3 rho(r + c_i) + G4 rho(r + 2 c_i)]
 * with s the sign of P - P0 (eq force_form), and the momentum source S = -F + rho g.
 * LBM_FORCE_KORTEWEG: eq Kforce_final, (4/3, -1/6, 2 kappa, -kappa) (the default);
 * LBM_FORCE_SHAN_CHEN: the single-ring force of eq SCforce, (1, 0, 0, 0): kappa unused;
 * LBM_FORCE_DUAL_RANGE: the dual-range force of eq DRforce, G1 = force_g[0],
 *   G2 = (1 - G1)/2 (eq PPcond1 only), no capillary pair: kappa unused;
 * LBM_FORCE_GENERAL: G1..G4 = force_g[0..3] as given (G3, G4 carry any kappa). */
enum { LBM_FORCE_KORTEWEG = 0, LBM_FORCE_SHAN_CHEN = 1, LBM_FORCE_DUAL_RANGE = 2, LBM_FORCE_GENERAL = 3 };
/* LBM_FP64: populations stored and updated in FP64.
 * LBM_FP32_DEV: populations stored as FP32 deviations h_i = f_i - w_i rho_ref and
 * updated in FP32; mass and momentum reductions stay FP64. */
enum { LBM_FP64 = 0, LBM_FP32_DEV = 1 };

/* Problem statement (Sec. 2.3 and Sec. 3.1). Units: lattice units, dr = dt = 1. */
typedef struct {
    int lattice;            /* LBM_D2Q9 or LBM_D3Q27 */
    int nx, ny, nz;         /* grid; periodic on every axis; nz must be 1 for D2Q9 */
    int eos;                /* LBM_EOS_* */
    double a, b, R;         /* EOS attraction, co-volume, gas constant (cubic EOS only) */
    double acentric;        /* acentric factor omega' of PR / RKS */
    double T_reduced;       /* T/Tc; Tc from the printed a(Tc,Pc), b(Tc,Pc) relations
                               (Shan-Chen: G_c / G) */
    double kappa;           /* capillary coefficient kappa~ of eq capillary_discrete */
    double tau_liquid;      /* relaxation time, omega = 1/tau; viscosity (tau - 1/2)/3 */
    double tau_vapour;      /* > 0: kinematic viscosity linear in rho between the two
                               bulk densities below (clamped); <= 0: constant tau_liquid */
    double rho_liquid, rho_vapour; /* bulk densities for the viscosity interpolation */
    double rho_wall;        /* virtual density of solid nodes (wetting, Sec. 4.5) */
    const uint8_t *mask;    /* nullable host array [N], 1 = solid; copied at create */
    int precision;          /* LBM_FP64 or LBM_FP32_DEV */
    double rho_ref;         /* reference density of the FP32 deviation storage */
    int check_every;        /* watchdog period in steps inside lbm_step: > 0 every
                               check_every steps and at the end, 0 at the end only,
                               < 0 never. A check reduces FP64 mass and momentum totals
                               and the count of densities outside the EOS domain. After
                               a single-pass (D3Q27) FP32 step on a grid without mask it
                               reduces the totals that step accumulated while pulling its
                               input state, i.e. the state one step before the check, with
                               no extra pass over the lattice; otherwise it runs a moment
                               pass on the current state. lbm_moments always reports the
                               current state */
    double accel[3];        /* body-force acceleration g (layered Poiseuille flow, Sec. 4.2):
                               the momentum source gains rho g, so U and the equilibria
                               carry it as they carry the Korteweg force; finite; z = 0
                               for D2Q9 */
    const double *rho_wall_field; /* nullable host array [N]: virtual density of each solid
                               node (> 0 where mask is set), replacing rho_wall, so that
                               walls of different wettability or walls touching different
                               phases can coexist; copied at create */
    const double *link_q;   /* nullable host array [Q][N] in lbm_velocities order: for a
                               fluid node n whose neighbour n + c_j is solid, entry (j, n)
                               is the fraction q in (0, 1] of the link from n to n + c_j
                               at which the wall lies; other entries are ignored. Walls
                               then use the linearly interpolated bounce-back of Bouzidi
                               et al. that the paper applies to curved walls (Sec. 4.5,
                               Sec. 5.3) instead of halfway bounce-back (q = 1/2 gives the
                               same step). Needs a mask; a node cut on two opposite links
                               with q, q' >= 1/2 needs 1/(2q) + 1/(2q') >= 1.01 (the
                               initial state is otherwise not representable). D3Q27
                               contexts take the single-pass interpolating kernel on
                               planes within three planes of a solid node (the two-pass
                               step when the single-pass step is not available for the
                               grid); D2Q9 takes it in its single-pass step (and in the
                               two-pass step under LBM2P_TWO_PASS=1); lbm_batch_create
                               rejects it. Copied at create */
    int force_model;        /* LBM_FORCE_* (0: eq Kforce_final) */
    double force_g[4];      /* coefficients for LBM_FORCE_DUAL_RANGE ([0] = G1) and
                               LBM_FORCE_GENERAL (G1..G4); finite */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

/* Allocates a context for one simulation (Sec. 2.3). Validates p (lattice, sizes,
 * tau > 1/2, kappa >= 0, EOS parameters, 0 < T_reduced for non-ideal EOS),
 * derives T = T_reduced * Tc (Sec. 3.1), allocates two population lattices in
 * device memory and uploads the mask. *out receives the context; on failure *out
 * is NULL and the message is available from lbm_last_error(NULL). */
int lbm_create(const lbm_params *p, lbm_ctx **out);

/* Sets f_i = f_i^eq(rho, u) (eq LBMeq) at every fluid node. rho: host [N] (> 0);
 * u: host [D][N] flow velocity U or NULL for rest. U is the velocity the moments
 * report (U = u + S/(2 rho), Sec. 2.3.5, Appendix D), so the equilibrium is taken at
 * the bare velocity u = U - S/(2 rho) with S the source of the given density field;
 * lbm_moments of the initial state returns (rho, U). Clears sticky errors. Synchronous. */
int lbm_init_fields(lbm_ctx *c, const double *rho, const double *u);

/* Advances n time steps of eq LBGK (stream-collide with the Korteweg force and
 * halfway, or with link_q interpolated, bounce-back at solid nodes). Runs the FP64 watchdog as selected by
 * check_every; returns LBM_E_DIVERGED / LBM_E_DOMAIN when it trips. When no
 * check runs, the call only enqueues work on the context stream. A D2Q9 step is one
 * kernel; a D3Q27 step is the fused z-march, or on grids too small for it the moment
 * pass and then the collide (LBM2P_TWO_PASS=1 takes the latter for both lattices;
 * in D2Q9 the two agree to rounding). Contexts off the fused D3Q27 step
 * capture 32 steps into a HIP graph on the first call with at least 32 steps between
 * two checks. Such runs then replay that graph on the context stream, with results
 * identical bit for bit; the capture uses the context's own stream. Steps are
 * launched one by one when the context stream is itself being captured, or when the
 * environment sets LBM2P_GRAPH=0. */
int lbm_step(lbm_ctx *c, int64_t n);

/* Density and velocity of the current state. rho: host [N] (nullable); U: host
 * [D][N] (nullable), the velocity U = u + S/(2 rho) shifted by half the force
 * increment (Sec. 2.3.5, Appendix D); solid nodes report rho_wall and U = 0.
 * totals: host [4] (nullable) = {sum rho, sum rho u_x, sum rho u_y, sum rho u_z}
 * over fluid nodes with the unshifted u, reduced in FP64 in a fixed order.
 * Synchronous. */
int lbm_moments(lbm_ctx *c, double *rho, double *U, double totals[4]);

/* For callers that cannot allocate device memory or wait on the device: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The values of lbm_moments,
 * bit for bit, written into caller-owned DEVICE buffers and only enqueued on the context
 * stream: no allocation, no synchronisation, no host copy. rho: device [N] (nullable);
 * U: device [D][N] (nullable); both in the user layout (rows of nx, x fastest). totals:
 * device [5] (nullable) = the four FP64 totals of lbm_moments, then the number of fluid
 * nodes whose density is outside the EOS domain. The moment pass's partial rows and the
 * reduction tree's rows use one static 8 MiB array per device, held until the process ends:
 * a grid whose moment pass has more than 209,610 workgroups (ceil(nx/64) ceil(ny/4) nz; a
 * 256^3 grid has 65,536) is rejected with LBM_E_INVAL before anything is enqueued. Every
 * call on a device shares that array and leaves its contents there (nothing in it needs to
 * start at zero), so calls that overlap on one GPU (other streams, threads or contexts, not
 * ordered with this call) race and give wrong results; calls ordered on one stream do not.
 * LBM_E_STATE before lbm_init_fields; a failed launch is LBM_E_HIP (possibly reported by a
 * later call, as for any asynchronous work). A captured call records the population lattice
 * that is current at capture; the context alternates its two lattices every step, so a replay
 * reports the current state after an even number of steps since the capture (or capture the
 * call together with an even number of steps taken with check_every < 0). */
int lbm_moments_noalloc(lbm_ctx *c, double *rho, double *U, double *totals);

/* Discrete pressure tensor of the current state (Appendix E). P: host [D(D+1)/2][N]
 * (caller-owned), components xx, yy, xy for D2Q9 and xx, yy, zz, xy, xz, yz for D3Q27; zero
 * at solid nodes. Appendix E splits the discrete Korteweg force into one- and two-ring
 * pseudo-potential and capillary parts and gives each part's tensor (the force being its
 * negative divergence). With the momentum source S = -F these tensors enter with a minus
 * sign, and the kinetic part is the lattice momentum flux sum_i c_i c_i f_i of the
 * pre-collision populations:
 *   P = sum_i c_i c_i f_i - (P^A + P^B + P^C + P^D).
 * At rest it is uniform in the normal direction across flat interfaces and reduces to the
 * EOS pressure in uniform regions; the integral of P_nn - P_tt across an interface is the
 * surface tension (Kirkwood-Buff, Sec. 3.2). Synchronous; the first call allocates
 * D(D+1)/2 N doubles of device memory kept until lbm_destroy. */
int lbm_pressure_tensor(lbm_ctx *c, double *P);

/* Releases all device memory and the stream. NULL-safe. */
void lbm_destroy(lbm_ctx *c);

/* Last error message of c, or of the calling thread's last lbm_create /
 * lbm_batch_create when c is NULL. Never NULL; valid until the next call. */
const char *lbm_last_error(const lbm_ctx *c);

/* Result of the latest watchdog check (lbm_init_fields, lbm_set_populations, and the checks
 * of lbm_step selected by check_every): out[0..3] = FP64 totals {sum rho, sum rho u_x,
 * sum rho u_y, sum rho u_z} over fluid nodes (unshifted u), out[4] = the number of fluid
 * nodes whose density is outside the EOS domain; *state_step (nullable) = the number of
 * steps since the last initialisation of the state they describe (one less than the steps
 * taken when the check reduced the totals the single-pass step accumulates). Host copy of
 * values already read; LBM_E_STATE before the first check. */
int lbm_last_check(const lbm_ctx *c, double out[5], int64_t *state_step);

/* Makes the context enqueue its work on hip_stream (a hipStream_t, not owned);
 * NULL restores the context's own stream. */
int lbm_set_stream(lbm_ctx *c, void *hip_stream);

/* Checkpoint: copies the population lattice to / from a host buffer of
 * lbm_population_bytes(c) bytes in storage precision (FP64 f_i or FP32 h_i), as
 * Q rows of N values in the order of lbm_velocities; a set of what get returned
 * resumes bit-exactly. Synchronous. */
int64_t lbm_population_bytes(const lbm_ctx *c);
int lbm_get_populations(lbm_ctx *c, void *host);
int lbm_set_populations(lbm_ctx *c, const void *host);

/* Velocity set of the library's population order (eq d3q27vel; D2Q9 drops z): writes
 * Q triplets (c_x, c_y, c_z) into c (caller-owned, 3*Q ints) and returns Q (9 or 27),
 * or LBM_E_INVAL. Together with lbm_get_populations this documents the checkpoint
 * layout: population i of node n is the post-collision value that node n produced,
 * so the pre-collision f_i(r) is entry i at r - c_i (entry opp(i) at r when r - c_i is
 * solid; with link_q, the interpolation of entries opp(i) at r and r + c_i, or opp(i)
 * and i at r, that the link's q selects); FP32 storage holds f_i - w_i rho_ref. */
int lbm_velocities(int lattice, int *c);

/* Runs n steps with HIP events around every kernel launch on the context
 * stream and returns the summed device time per kernel kind in ms:
 * ms[0] = moment pass, ms[1] = collide-stream pass (or the fused step kernel),
 * ms[2] = everything in the step loop. launches[0..1] = number of launches.
 * A measurement mode for the bench; the state advances exactly as lbm_step. */
int lbm_step_timed(lbm_ctx *c, int64_t n, double ms[3], int64_t launches[2]);

/* Attainable HBM bandwidth (measurement aid, not part of the method): copies `bytes`
 * (a multiple of 16) from src to dst, both device buffers of at least that size owned by
 * the caller, with a hand-written streaming kernel (16-byte accesses, non-temporal loads
 * and stores) in a few launch shapes, reps timed launches each, on hip_stream (a
 * hipStream_t, NULL = the default stream). out[0] = the fastest shape's bandwidth in GB/s
 * counting bytes read plus written, out[1] = its ms per copy, out[2] = its shape code
 * (loads in flight per lane x 100000 + workgroups). Synchronous; LBM_E_INVAL for bad
 * arguments, LBM_E_HIP if a launch or event fails. */
int lbm_copy_probe(void *dst, const void *src, int64_t bytes, int reps, void *hip_stream, double out[3]);

/* Thermodynamics of the problem statement, host only (Sec. 3.1). out[0] = rho_v,
 * out[1] = rho_l, out[2] = P_sat from the Maxwell equal-area rule
 * (eq Maxwell_equal_area), out[3] = T = T_reduced * Tc (Shan-Chen: the coupling G).
 * Returns LBM_E_DOMAIN when the EOS has no van der Waals loop at that temperature. */
int lbm_coexistence(const lbm_params *p, double out[4]);

/* Surface tension of the flat equilibrium interface of the second-gradient fluid
 * (Sec. 2.1, Sec. 3.2) with the capillary coefficient p->kappa at the problem's
 * temperature: sigma = integral kappa rho'^2 dx over the interface, evaluated as the
 * integral over [rho_v, rho_l] of sqrt(2 kappa (Omega(rho) - Omega_sat)). Host only.
 * Returns LBM_E_DOMAIN when the EOS has no van der Waals loop at that temperature. */
int lbm_surface_tension(const lbm_params *p, double *sigma);

/* Equation of state of the problem statement (Sec. 3.1; Shan-Chen as documented at
 * LBM_EOS_SC1): P[k] = P(rho[k]) for k < n, host arrays (caller-owned). For pressure
 * probes such as the Young-Laplace contact-angle measurement (Sec. 4.5). Host only. */
int lbm_eos_pressure(const lbm_params *p, const double *rho, int64_t n, double *P);

/* Capillary coefficient for which the flat equilibrium interface of the
 * second-gradient fluid (Sec. 2.1) has width W = (rho_l - rho_v)/max|grad rho|
 * (eq interface_W). Host only. */
int lbm_kappa_for_width(const lbm_params *p, double width, double *kappa);

/* Batched sweep: ncases independent simulations (each a full lbm_params,
 * D2Q9 or D3Q27, FP64 or FP32_DEV, uneven sizes, any force model) advanced together,
 * with chunks of steps captured in a HIP graph that lbm_batch_step replays:
 *   - D2Q9 cases whose tile (all rows, a strip of columns plus a halo of 3 columns per
 *     step on each side) fits in LDS advance several steps per launch in tiles;
 *   - the other cases take one launch per phase and step covering all of them, each case
 *     split into blocks in proportion to its size.
 * The layout (steps per tile launch, tile row width, block split) is chosen at the first
 * lbm_batch_step by timed trials on the live state, which is then restored; results do not
 * depend on it (bit for bit). LBM2P_TUNE_CACHE names a text file that keeps the choice per
 * GPU target and case list. Interpolated walls (link_q) and cases with (D+1) N >= 2^31 are
 * rejected with LBM_E_INVAL. At its end lbm_batch_step checks every case for divergence in
 * one pass over all cases (non-finite stored populations at fluid nodes): LBM_E_DIVERGED names
 * the first such case. */
int lbm_batch_create(const lbm_params *cases, int ncases, lbm_batch **out);
int lbm_batch_init_fields(lbm_batch *b, int icase, const double *rho, const double *u);
int lbm_batch_step(lbm_batch *b, int64_t n);
int lbm_batch_moments(lbm_batch *b, int icase, double *rho, double *U, double totals[4]);
void lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);
/* The layout in use (after the first lbm_batch_step): out[0] = 1 for the stepped design (0:
 * one workgroup per case), out[1] = threads per block (persistent: the workgroup size),
 * out[2] = nodes per thread, out[3] = steps per tile launch (0: no case in tiles),
 * out[4] = tile row width (own columns plus 3 halo columns per step on each side, before a
 * case's tiles are narrowed to fit LDS and evened out), out[5] = tiles. */
int lbm_batch_layout(const lbm_batch *b, int out[6]);

#ifdef __cplusplus
}
#endif
#endif /* LBM2P_H */
