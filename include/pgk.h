/*
 * pgk.h -- C ABI of the MI355X library for the reduced polyatomic ES-BGK
 * lattice-Boltzmann step (Kolluru, Atif & Ansumali, "Reduced kinetic model of
 * polyatomic gases", arXiv:2201.05280).
 *
 * One step advances, on a body-centred-cubic grid with the 41-velocity RD3Q41
 * set (Sec. 5, Table of velocities and weights):
 *   - the auxiliary populations g_i = f_i - (dt/2) Omega_i of the translational
 *     distribution (Sec. 5, trapezoid rule), whose collision relaxes f towards
 *     an ES-BGK target at rate 1/tau and a BGK target at rate 1/tau1 (Sec. 4,
 *     kinetic equation of the reduced model), followed by pull streaming;
 *   - the rotational temperature theta_R, split into half relaxation,
 *     MacCormack advection, FTCS diffusion and a second half relaxation
 *     (Sec. 5, the four steps of the theta_Rot solver).
 *
 * Conventions
 *   status    every call returns PGK_OK (0) or a negative PGK_E* code; the
 *             context keeps a message for pgk_last_error().  Nothing throws.
 *   sites     a grid of nx*ny*nz cells holds ns = 2*nx*ny*nz sites: corner
 *             sites (sub 0) at integer positions and body-centre sites (sub 1)
 *             offset by (1/2,1/2,1/2).  Every per-site array is ordered
 *             [sub][z][y][x] (x fastest); vector fields are [3][ns] and the
 *             pressure tensor [6][ns] (xx, yy, zz, xy, xz, yz).
 *   memory    the caller owns every buffer.  pgk_buffer_sizes() tells how many
 *             bytes each of the PGK_NBUF device buffers needs; the caller
 *             allocates them (e.g. as torch tensors) and hands them over with
 *             pgk_bind().  The library allocates no device memory and never
 *             frees caller memory.  Field arrays passed to pgk_init_fields()
 *             and pgk_read_moments() are device pointers to doubles.
 *   streams   all work is enqueued on the HIP stream given to pgk_create()
 *             (0 = the null stream); calls return before the work finishes,
 *             except pgk_conserved() and the error checks it implies.
 *   threads   one context per host thread at a time.
 */
#ifndef PGK_H
#define PGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PGK_OK           0
#define PGK_EINVAL      -1   /* bad argument (null pointer, size, enum value) */
#define PGK_ENOMEM      -2   /* a bound buffer is too small */
#define PGK_EDEVICE     -3   /* a HIP call failed */
#define PGK_EINFEASIBLE -4   /* requested transport coefficients cannot be reached */
#define PGK_ENOTBOUND   -6   /* buffers not bound yet */
#define PGK_ETOOBIG     -7   /* the request exceeds a fixed capacity of the library */

/* population storage (Sec. 5 populations; the FP32 form stores deviations) */
#define PGK_FP64     0       /* g_i in double precision */
#define PGK_FP32DEV  1       /* h_i = g_i - w_i in single precision; moments,
                                per-site solve and reductions in double */

/* second half of the theta_R relaxation and the diffusion form */
#define PGK_CN   0           /* explicit complement of the first half (Crank-Nicolson
                                overall) and flux-form diffusion: the exchange with the
                                translational energy conserves E_T + E_R exactly */
#define PGK_LIT  1           /* backward Euler and D_R lap(theta_R), as printed */

/* discrete equilibrium (Sec. 5 leaves it open) */
#define PGK_F3   0           /* third-order Hermite projection of the anisotropic Gaussian */
#define PGK_E2   1           /* discrete quasi-equilibrium F_i = w_i exp(l . phi(c_i)) with
                                phi = (1, c, cc): the H minimiser on the 41 velocities under
                                the target's density, momentum and pressure tensor (Sec. 2,
                                Sec. 3), found per site by damped Newton in double precision.
                                It stays positive at Mach numbers where F3 turns negative, but
                                a target beyond what a positive distribution on the lattice can
                                carry has no solution: that site's populations become NaN.
                                Diffuse walls re-emit F3 in either case; Dirichlet faces take
                                E2 (pgk_set_bc returns PGK_EINFEASIBLE if the face state
                                has none) */
#define PGK_F4   2           /* F3 plus the contracted fourth-order Hermite terms
                                w_i sum_ab K_ab h_ab(c_i), h_ab(c) = c_a c_b (c^2 - 7 theta0)
                                - delta_ab theta0 (c^2 - 5 theta0): moments of orders 0 to 3
                                as F3, and the contracted fourth moment sum F c^2 c_a c_b
                                of the Gaussian N(u, lam) for every state (the lattice's
                                weights satisfy the contracted moment conditions this needs,
                                Sec. 5), so heat conducts at kappa/(rho c_p) at any
                                temperature, not only near theta0.  Not linear in lam: the
                                gain term mixes F4(lam_ES) and F4(theta I) at their rates.
                                Walls re-emit F3, Dirichlet faces take F4.  Single grid only
                                (not in the batched sweep) */

/* boundary kinds of the faces: the two x faces and the two y faces (z is
 * periodic).  A position beyond an x face and a y face at once (a corner of a
 * box bounded on both axes) belongs to the x face. */
#define PGK_PERIODIC   0
#define PGK_WALL       1     /* diffuse (Maxwell) wall at u_w, theta_w */
#define PGK_DIRICHLET  2     /* equilibrium ghost state rho, u, theta */

/* device buffers the caller allocates */
#define PGK_BUF_POP0   0     /* 41*ns populations (ping) */
#define PGK_BUF_POP1   1     /* 41*ns populations (pong) */
#define PGK_BUF_THETAR 2     /* ns doubles: theta_R */
#define PGK_BUF_AUX    3     /* per-site fields handed from the collision to the theta_R
                                transport, reduction partials, wall densities; with
                                PGK_E2 also each site's last Newton multipliers
                                (2 x 10 doubles, the next step's starting point) */
#define PGK_NBUF       4

typedef struct pgk_ctx pgk_ctx;

typedef struct {
    int nx, ny, nz;          /* cells per axis, each >= 1 */
    int precision;           /* PGK_FP64 | PGK_FP32DEV */
    int variant;             /* PGK_CN | PGK_LIT */
    int equilibrium;         /* PGK_F3 | PGK_E2 | PGK_F4 */
    int bc_x[2];             /* kind of the low and high x faces */
    int bc_y[2];             /* kind of the low and high y faces (bounded: ny >= 2) */
} pgk_grid;

/* The model parameters of Sec. 4: relaxation times tau (ES-BGK part) and tau1
 * (BGK part and rotational relaxation), ES parameter b, k_r = kappa_R/kappa_T,
 * rotational degrees of freedom delta (> 0: the rotational energy equation
 * divides by it; a monatomic gas is approached with a small delta, as in the
 * paper's table of fluids), lattice reference temperature theta0 (0 selects
 * the printed value 0.2948964908710633). */
typedef struct {
    double tau, tau1, b, kr, delta, theta0;
} pgk_params;

/* Targets for the parameter map of Sec. 4 (hydrodynamics): kinematic shear
 * viscosity nu = eta/rho at theta0, Prandtl number, bulk-to-shear viscosity
 * ratio, rotational dof.  b and kr may be NaN (free) or fixed. */
typedef struct {
    double nu, Pr, mub_over_mu, delta, b, kr, theta0;
} pgk_targets;

/* derived constants of one step (filled by pgk_resolve / pgk_set_params) */
typedef struct {
    double tau, tau1, b, kr, delta, theta0;
    double tau_star;         /* 1/tau* = 1/tau + 1/tau1 */
    double beta;             /* dt/(2 tau* + dt) */
    double X, Y;             /* 3/(2 tau1 (3+delta)), delta/(2 tau1 (3+delta)) */
    double s_sigma;          /* sigma(g) = sigma(f) s_sigma */
    double B;                /* 1 + tau/tau1 */
    double nu, mub_over_mu, Pr, gamma;  /* transport coefficients these imply */
    double D_R;              /* rotational diffusivity 2 kappa_R/(rho delta) at theta0 */
} pgk_resolved;

/* Parameter map (Sec. 4, shear and bulk viscosity, Prandtl number).  Rule when
 * b is NaN: start from k_r = delta/5 (or the fixed kr), solve b from Pr, clamp b
 * to the ES range [-1/2, 1] (Sec. 2), then tau1/tau from the viscosity ratio,
 * k_r from Pr and tau from nu.  An explicit b may also lie above 1, up to
 * B = 1 + tau/tau1 (positive shear viscosity), as the Landau-number runs of
 * Sec. 6 at Pr 5 and 10 need; b = 1 exactly leaves tau1/tau undetermined.
 * Returns PGK_EINFEASIBLE when no positive tau1/tau meets mub_over_mu (for
 * b < 1: mub_over_mu at or below the floor 2 delta / (3 (3+delta)); for b > 1:
 * above it), when b is 1, below -1/2 or at or above B, or k_r would be
 * negative; PGK_EINVAL for delta <= 0 or non-positive targets.  Host only. */
int pgk_resolve(const pgk_targets *t, pgk_resolved *out);

/* The RD3Q41 velocity set (Sec. 5, table of velocities and weights) in the
 * library's population order: 0 the rest velocity, 1 + p the representative
 * c_p of opposite pair p (p = 0..19), 21 + p its negative.  c receives 41 x 3
 * velocities in lattice units (half-integers included), w the 41 weights at
 * reference temperature theta0 (0 = the printed value).  Host memory, host
 * only. */
int pgk_lattice(double theta0, double *c, double *w);

/* Populations F[41] (library order) of the discrete equilibrium `equilibrium`
 * (PGK_F3, PGK_E2 or PGK_F4) with density rho, velocity u[3] and covariance lam[6]
 * (xx yy zz xy xz yz), reference temperature theta0 (0 = printed).  The same
 * host code fills the Dirichlet face ghosts.  Returns PGK_EINFEASIBLE when E2
 * has no solution, PGK_EINVAL for rho <= 0 or an unknown kind.  Host memory,
 * host only. */
int pgk_equilibrium(int equilibrium, double theta0, double rho, const double *u, const double *lam, double *F);

/* Bytes needed for each device buffer of this grid. */
int pgk_buffer_sizes(const pgk_grid *g, size_t sizes[PGK_NBUF]);

/* Create a context for grid g on HIP stream `stream` (a hipStream_t, may be 0). */
int pgk_create(const pgk_grid *g, void *stream, pgk_ctx **out);

/* Bind caller-allocated device buffers (see PGK_BUF_*); bytes[] are their sizes. */
int pgk_bind(pgk_ctx *ctx, void *const bufs[PGK_NBUF], const size_t bytes[PGK_NBUF]);

/* Set the resolved parameters; `out` (may be NULL) receives the derived constants.
 * Returns PGK_EINVAL for tau, tau1 <= 0, delta <= 0, kr < 0, b < -1/2 or
 * b >= 1 + tau/tau1 (zero or negative shear viscosity).  b in (1, 1 + tau/tau1)
 * lies beyond the ES range of Sec. 2, where the covariance T I + b sigma/rho can
 * lose positive definiteness far from equilibrium: accepted for PGK_F3 and
 * PGK_F4 (polynomial targets, as the Landau-number runs of Sec. 6 use it) and
 * refused with PGK_EINVAL on a PGK_E2 grid. */
int pgk_set_params(pgk_ctx *ctx, const pgk_params *p, pgk_resolved *out);

/* Boundary data of face `side` (0 low, 1 high) of axis `axis` (0 x, 1 y):
 * wall velocity and temperature for PGK_WALL (rho ignored; the velocity
 * component normal to the wall must be 0), ghost state for PGK_DIRICHLET.
 * A diffuse wall re-emits, into every ghost column beyond it, the mass the
 * last collision sent into that column (zero net mass flux per column), at
 * the equilibrium of its velocity and temperature (Sec. 6 uses diffuse walls
 * on one axis for the Couette flows and on both for the heated cavity).
 * Every bounded face needs its state before pgk_init_fields (PGK_EINVAL
 * otherwise); with PGK_E2, a Dirichlet state without an E2 equilibrium gives
 * PGK_EINFEASIBLE.  Between steps, a new state acts as in a push scheme: the
 * pull of the next step still reads what the face in force during the last
 * collision sends (the library fills those ghosts first), the step after
 * reads the new state.  Dirichlet ghosts are filled once per state, wall
 * ghosts every step.  PGK_EINVAL for a periodic face. */
int pgk_set_bc(pgk_ctx *ctx, int axis, int side, double rho, const double u[3], double theta);
/* pgk_set_bc(ctx, 0, side, ...) */
int pgk_set_bc_x(pgk_ctx *ctx, int side, double rho, const double u[3], double theta);

/* Initial state from device fields rho[ns], u[3][ns], theta_T[ns], theta_R[ns]:
 * g_i = F_i(rho, u, theta_T I) and the rotational temperature theta_R. */
int pgk_init_fields(pgk_ctx *ctx, const double *rho, const double *u,
                    const double *theta_T, const double *theta_R);

/* Advance n time steps (asynchronous on the context stream; one step is
 * Sec. 5: collide and stream g, then the four steps of the theta_Rot solver).
 * With graph steps K > 0 (pgk_set_graph_steps) and timing off, K steps are
 * recorded once as a HIP graph per starting buffer (on a private stream) and
 * replayed n/K times, the rest launched directly; the launches and results
 * are those of stepping one by one, bit for bit.  The recorded chunks are
 * dropped by pgk_bind, pgk_set_params, pgk_set_bc and a new K.
 * Errors: PGK_EINVAL before pgk_init_fields, PGK_EDEVICE on a failed launch,
 * capture or graph instantiation (message in pgk_last_error). */
int pgk_step(pgk_ctx *ctx, int64_t n);

/* Steps per replayed graph for pgk_step: 0 launches every kernel directly,
 * an even K in [2, 4096] replays K-step graphs (default 32); PGK_EINVAL
 * otherwise. */
int pgk_set_graph_steps(pgk_ctx *ctx, int k);

/* Moments of the translational distribution f at the current time level
 * (after the g -> f map of Sec. 5) into device arrays; any pointer may be
 * NULL.  theta_T is theta_T(f), theta_R the stored rotational temperature,
 * P the pressure tensor of f. */
int pgk_read_moments(pgk_ctx *ctx, double *rho, double *u, double *theta_T,
                     double *theta_R, double *P);

/* Totals over the grid at the current time level: mass, momentum (3) and
 * total energy sum(1/2 sum_i g_i c_i^2 + delta rho theta_R / 2).  Synchronises
 * the context stream; `out` is host memory. */
int pgk_conserved(pgk_ctx *ctx, double out[5]);

/* The theta_R transport (Sec. 5, steps 2-4) by its plain reference kernels on
 * every grid (on != 0): one MacCormack launch and n_sub diffusion launches
 * that read and write global memory only, instead of the LDS kernels chosen by
 * grid shape (the fused periodic kernel, the one-work-group kernel of small
 * grids, the line kernel with its halo).  The one-work-group kernel runs the
 * reference kernels' per-site code, so its results are the same bits; the
 * fused periodic and line kernels evaluate the same formulas in the same
 * order, with fused multiply-adds that the compiler may round differently, and
 * agree to round-off.  The switch checks the LDS kernels (a
 * missing barrier or a halo indexing slip shows as a difference) and costs
 * speed only.  Takes effect at the next pgk_step; recorded step graphs are
 * dropped.  Off by default. */
int pgk_set_transport_reference(pgk_ctx *ctx, int on);

/* Per-kernel timing with HIP events on the context stream.  While enabled,
 * pgk_step records an event before its first launch and after every launch.
 * pgk_kernel_times() waits for the stream, returns the summed milliseconds and
 * the launch counts of [0] the fused pull-collide kernel, [1] the MacCormack
 * advection (on a periodic grid with one diffusion sub-step: the single fused
 * transport kernel, advection + diffusion + second half), [2] the diffusion
 * and second half relaxation (on a bounded or sub-cycled line, ny = nz = 1,
 * with at most 63 sub-steps: the whole transport in one launch of work-groups
 * of WG threads, each producing WG - 2 (n_sub + 1) cells, WG = 64 up to 15
 * sub-steps and 256 beyond; on another bounded
 * or sub-cycled grid of at most 4096 sites:
 * the whole transport in one work-group), [3] the ghost fill of the bounded faces, and clears the
 * record.  Event handles are created on demand and
 * kept until pgk_destroy. */
#define PGK_NKERNEL 4
int pgk_set_timing(pgk_ctx *ctx, int enable);
int pgk_kernel_times(pgk_ctx *ctx, double ms[PGK_NKERNEL], int64_t launches[PGK_NKERNEL]);

/* ------------------------------------------------------------------------
 * Batched sweep: many independent 1D cases (one cell in y and z, x faces
 * bounded) in double precision.  Each case is a Couette layer between two
 * diffuse walls or a stationary normal shock between two Dirichlet faces
 * (Sec. 6 uses Couette flows; shocks are outside the paper's tests).  One
 * persistent launch advances every running case by K steps, one work-group
 * per case; the launch is captured once in a HIP graph and replayed.  After
 * each chunk a case is checked:
 *   residual = max over phi in {rho, u_axis, theta_T, theta_R} of
 *              ||phi^n - phi^(n-1)||_2 / ||phi^n||_2   (one-step change)
 * and is frozen when it falls to `tol` (CONVERGED), when a density or a
 * temperature turns non-positive or non-finite (DIVERGED), or at max_steps.
 * Work-group size and K come from a built-in autotuner unless set: at the
 * start of a run and again whenever the number of running cases has halved,
 * one chunk of each candidate (work-groups of 256 or 512 threads, E2 batches
 * 256 only; K = 32, 64, 128 or 256 steps) is timed on the live state (or the choice for
 * that mix is read from the JSON cache, $PGK_TUNE_CACHE or
 * ~/.cache/pgk_tune.json, keyed by the running case count and the longest
 * running case).
 * ------------------------------------------------------------------------ */
#define PGK_CASE_RUNNING   0
#define PGK_CASE_CONVERGED 1
#define PGK_CASE_DIVERGED  2
#define PGK_CASE_MAXSTEPS  3
#define PGK_CASE_STALLED   4   /* residual stopped falling (see pgk_batch_stall) */

typedef struct {
    int L;                   /* cells along x, 4 <= L <= 8192 */
    int bc;                  /* PGK_WALL or PGK_DIRICHLET, both faces */
    int vel_axis;            /* velocity component used by the residual (0, 1, 2) */
    int variant;             /* PGK_CN | PGK_LIT */
    pgk_params p;            /* resolved model parameters of this case */
    double rho[2];           /* Dirichlet densities (ignored for walls) */
    double u[2][3];          /* face velocities (walls: tangential only) */
    double theta[2];         /* face temperatures */
    int equilibrium;         /* PGK_F3 | PGK_E2 (a batch holding E2 cases runs with
                                work-groups of 256; PGK_EINFEASIBLE if a Dirichlet face
                                state has no E2 equilibrium) */
} pgk_case;

typedef struct pgk_batch pgk_batch;

/* Bytes of the single device buffer a batch of n cases needs. */
int pgk_batch_bytes(const pgk_case *cases, int n, size_t *bytes);

/* Create a batch on `stream` over the caller's device buffer `buf` (256-byte
 * aligned, at least pgk_batch_bytes).  Case c owns sites [off_c, off_c + 2 L_c)
 * of every per-site field; pgk_batch_offsets() returns off_0..off_n.  A case
 * must keep b within the ES range [-1/2, 1] of Sec. 2 (a batch may hold E2
 * cases, whose target needs a definite covariance), besides 4 <= L <= 8192
 * and positive tau, tau1, delta and face temperatures: PGK_EINVAL otherwise. */
int pgk_batch_create(const pgk_case *cases, int n, void *stream, void *buf, size_t bytes, pgk_batch **out);
int pgk_batch_offsets(const pgk_batch *b, int64_t *off);

/* Initial state of every case from device fields over all sites (same meaning
 * and [3][ns_total] layout as pgk_init_fields); resets steps and status. */
int pgk_batch_init(pgk_batch *b, const double *rho, const double *u, const double *theta_T,
                   const double *theta_R);

/* Fix the work-group size (256 or 512) and chunk length K (>= 2); 0, 0 = autotune. */
int pgk_batch_config(pgk_batch *b, int wg, int K);

/* Run until every case has stopped or max_steps per case.  Host arrays of n
 * entries receive the steps taken, the last residual and the status.  A case
 * that an earlier call stopped at its lower max_steps (PGK_CASE_MAXSTEPS)
 * runs on when a later call raises the cap, so a caller can advance a batch
 * in stages; the stall bookkeeping carries over between calls until
 * pgk_batch_init. */
int pgk_batch_run(pgk_batch *b, int64_t max_steps, double tol, int64_t *steps, double *resid, int *status);

/* Stall detection for pgk_batch_run: a running case whose residual has not
 * fallen below half of its best value for `window` steps (counted in whole
 * chunks) stops with PGK_CASE_STALLED (a structure that creeps instead of
 * settling, such as a thin shock between two Dirichlet faces, holds its
 * residual at a floor).  window = 0 (the default) turns it off. */
int pgk_batch_stall(pgk_batch *b, int64_t window);

/* Work-group size and K last chosen, and nanoseconds per site update over
 * the last run. */
int pgk_batch_tuned(const pgk_batch *b, int *wg, int *K, double *ns_per_site_update);

/* f-moments of every case into device arrays over all sites (NULL = skip). */
int pgk_batch_read_moments(pgk_batch *b, double *rho, double *u, double *theta_T, double *theta_R);

const char *pgk_batch_last_error(const pgk_batch *b);
void pgk_batch_destroy(pgk_batch *b);

/* ------------------------------------------------------------------------
 * Coordinate MLP of the learned warm start: 6 inputs (normalised x/L, Ma, Pr,
 * mu_b/mu, log10 Kn, delta) -> 4 hidden layers of 128 with SiLU -> 4 outputs
 * (normalised rho, u, theta_T, theta_R).  Weights and activations enter the
 * products as bfloat16 (round to nearest even), products accumulate in FP32;
 * FP32 master weights and Adam.  Parameters are one flat FP32 vector:
 * W1[128][6], b1[128], W2[128][128], b2, W3, b3, W4, b4, W5[4][128], b5[4].
 * Loss: mean squared error over points and outputs.  X is [n][6], Y [n][4],
 * row-major FP32 device arrays.  One device buffer (pgk_mlp_bytes) holds the
 * parameters, the Adam state and the working set of a minibatch of up to nmax
 * points; a minibatch's gradient is summed in a fixed order (the same bits on
 * every run).
 * ------------------------------------------------------------------------ */
#define PGK_MLP_NPARAM 50948
typedef struct pgk_mlp pgk_mlp;
int pgk_mlp_bytes(int nmax, size_t *bytes);
int pgk_mlp_create(void *stream, void *buf, size_t bytes, int nmax, pgk_mlp **out);
/* theta: device vector of PGK_MLP_NPARAM floats; resets the Adam state */
int pgk_mlp_set_params(pgk_mlp *m, const float *theta);
int pgk_mlp_get_params(pgk_mlp *m, float *theta);
/* inference of n points (any n, processed nmax at a time) */
int pgk_mlp_forward(pgk_mlp *m, const float *X, float *Y, int n);
/* mean loss (host, synchronises) and its gradient (device, may be NULL) on n <= nmax points */
int pgk_mlp_loss_grad(pgk_mlp *m, const float *X, const float *Y, int n, float *grad, float *loss);
/* one Adam update with the gradient of the last pgk_mlp_loss_grad */
int pgk_mlp_adam_step(pgk_mlp *m, float lr, float beta1, float beta2, float eps);
/* epochs of minibatch Adam (beta 0.9, 0.999, eps 1e-8) over n points in
 * contiguous minibatches visited in a seeded random order; loss_per_epoch
 * (host, may be NULL) receives each epoch's loss, the squared errors met
 * during the epoch summed over all n points and divided by 4 n (every point
 * counts once, whatever the size of the last minibatch).  An epoch is one
 * replayed HIP graph (recorded on a private stream, launched on the handle's
 * stream); the host writes the epoch's minibatch records (24 bytes each) into
 * the working set, so n / batch, rounded up, may be at most
 * 4 * 128 * nmax / 24 (nmax rounded up to 64): PGK_EINVAL beyond it, as when
 * the Adam step count would pass 2^31 - 1; PGK_EDEVICE if capture fails.
 * Synchronises the handle's stream. */
int pgk_mlp_train(pgk_mlp *m, const float *X, const float *Y, int64_t n, int batch, int epochs, float lr,
                  uint64_t seed, float *loss_per_epoch);
/* The whole trainable state: FP32 master weights, their bfloat16 copies (the
 * values the products use), the Adam moments m and v (device arrays of
 * PGK_MLP_NPARAM values, any may be NULL) and the Adam step count t (host).
 * pgk_mlp_set_state restores master, m, v and t (the bf16 copies are rounded
 * from master, the gradient accumulator is cleared), so that training resumes
 * bit for bit.  Asynchronous on the MLP stream. */
int pgk_mlp_get_state(pgk_mlp *m, float *master, uint16_t *wbf, float *adam_m, float *adam_v, int64_t *t);
int pgk_mlp_set_state(pgk_mlp *m, const float *master, const float *adam_m, const float *adam_v, int64_t t);
/* The same state in a file at `path`: an 8-byte tag "PGKMLP1", the parameter
 * count and t as int64, then master, m and v as FP32 (host byte order).
 * pgk_mlp_load refuses a file of another tag or parameter count (PGK_EINVAL,
 * message in pgk_mlp_last_error).  Both synchronise the MLP stream. */
int pgk_mlp_save(pgk_mlp *m, const char *path);
int pgk_mlp_load(pgk_mlp *m, const char *path);
const char *pgk_mlp_last_error(const pgk_mlp *m);

/* Inference for callers that cannot allocate device memory at all (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the forward pass of pgk_mlp_forward, the same kernels and the same bits,
 * from the FP32 parameters theta (device, PGK_MLP_NPARAM values, layout of
 * pgk_mlp_set_params) without a pgk_mlp object.  X [n][6] and Y [n][4] are
 * device arrays the caller owns.  The bf16 weights and activations live in a
 * fixed device array inside the library, one per GPU (4.3 MB, kept until
 * the process ends); its address is looked up once per GPU at the first call
 * with that GPU current.  The call allocates nothing and never calls hipMalloc.
 * Limits: n <= PGK_MLP_STATIC_NMAX points per call (PGK_ETOOBIG above it,
 * before any GPU work); `stream` must belong to the current device.  Every
 * call on a GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams or host threads) race and must be serialised by the
 * caller; calls in one stream are ordered.  PGK_EINVAL for a null pointer or
 * n < 0, PGK_EDEVICE if the array's address cannot be obtained or a launch
 * fails.  Asynchronous on `stream`. */
#define PGK_MLP_STATIC_NMAX 4096
int pgk_mlp_forward_static(const float *theta, const float *X, float *Y, int n, void *stream);
void pgk_mlp_destroy(pgk_mlp *m);

/* Steps taken since the last pgk_init_fields. */
int64_t pgk_steps_done(const pgk_ctx *ctx);

/* Checkpoints.  Between steps the state of a grid is the content of its four
 * bound buffers plus this clock: the steps taken, which population buffer
 * holds the state, and whether the face ghosts hold what the next pull reads
 * (and a face state changed since).  A caller that copies the buffers out
 * (after synchronising the stream) with pgk_get_clock, and later back into a
 * grid of the same shape, precision, equilibrium, parameters and faces
 * followed by pgk_set_clock, continues bit for bit.  pgk_get_clock needs an
 * initialised grid; pgk_set_clock needs bound buffers, parameters and face
 * states, and marks the grid initialised (PGK_EINVAL for a bad clock). */
typedef struct {
    int64_t steps;
    int cur;                 /* 0: PGK_BUF_POP0 holds the state, 1: PGK_BUF_POP1 */
    int ghosts_ok;
    int face_changed;
} pgk_clock;
int pgk_get_clock(const pgk_ctx *ctx, pgk_clock *out);
int pgk_set_clock(pgk_ctx *ctx, const pgk_clock *in);

/* Message of the last failed call on this context (never NULL). */
const char *pgk_last_error(const pgk_ctx *ctx);

void pgk_destroy(pgk_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PGK_H */
