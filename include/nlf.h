/*
 * nlf.h -- C ABI of the MI355X (gfx950) library for nonlocal potentials of the nonlinear
 * Schroedinger equation evaluated through the nonuniform FFT, and the ground-state and
 * dynamics solvers built on it.
 *
 * Method (Bao, Jiang, Tang, Zhang, "Computing the ground state and dynamics of the NLSE
 * with nonlocal interactions via the nonuniform FFT"):
 *   u = U * rho = (2 pi)^-d int Uhat(k) rhohat(k) e^{i k.x} dk            (Sec. 2, Eq. 'nonlocal53')
 * truncated to the ball |k| <= P and written in spherical/polar coordinates, where the
 * Jacobian |k|^(d-1) cancels the Coulomb symbol (Sec. 2.1, Eq. 'ifft').  The quadrature sum
 * is evaluated with a type-2 NUFFT (grid -> Fourier nodes), a pointwise symbol-times-weight
 * multiply, and a type-1 NUFFT (nodes -> grid).  The 2D Laplace kernel has a stronger
 * singularity and is handled by subtracting a Gaussian with the density's first two moments
 * (Sec. 2.2, Alg. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Grid: box [-L_0,L_0) x ... , n_i points per axis, x_j = -L_i + j h_i, h_i = 2 L_i / n_i,
 *    row-major (C order): the LAST axis is contiguous.  n_i must be a power of two in [8, 1024].
 *  * Precision: a plan is FP64 (NLF_F64) or FP32 (NLF_F32).  Every bulk array handed to the
 *    library (densities, potentials, node values, wave functions) has the plan's precision;
 *    complex arrays are interleaved (re, im).  Quadrature weights, the symbol, the Laplace
 *    subtraction and all reductions are FP64 in both precisions.
 *  * Memory: every pointer argument named *_dev is device memory owned by the caller, valid for
 *    the duration of the call's stream work; the library never frees caller memory.  Plans own
 *    their workspaces (allocated in nlf_plan_create, freed in nlf_plan_destroy).
 *  * Streams: all device work of a plan is enqueued on the HIP stream given at plan creation
 *    (NULL = the default stream), the one-time work too (table uploads, buffer clears), so a
 *    non-blocking stream is safe.  Calls return when the work is enqueued unless stated
 *    otherwise; the solvers synchronise the stream to read convergence flags.
 *  * Concurrency: a plan is not re-entrant; use one plan per stream.  Different plans may be
 *    driven from different host threads at the same time.
 *  * Errors: every call returns an int status; 0 is success, negative values are errors.
 *    nlf_last_error() returns a message for the calling thread's last error.  No C++
 *    exception crosses this boundary.
 *  * Batching: a plan with opts.batch = B processes B independent fields per call; arrays are
 *    laid out batch-major ([B][...]).
 */
#ifndef NLF_H
#define NLF_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------- */
#define NLF_OK            0
#define NLF_EINVAL       -1   /* NULL pointer, bad size, inconsistent argument            */
#define NLF_EUNSUPPORTED -2   /* dimension not 2/3, n_i not a power of two in [8,1024], ... */
#define NLF_ENOMEM       -3   /* device or host allocation failed                          */
#define NLF_EHIP         -4   /* HIP runtime error (message kept for nlf_last_error)       */
#define NLF_ENOCONV      -5   /* iteration cap reached; statistics are still filled        */
#define NLF_ENONFINITE   -6   /* a NaN/Inf was detected in a reduction                      */

/* ---- enums ---------------------------------------------------------------------------- */
#define NLF_F64 0
#define NLF_F32 1

/* Interaction kernels (Sec. 1, Eqs. 'Kernal' and 'Kernal21d'; Sec. 2, Eq. 'Kernal124d').     */
#define NLF_COULOMB3D 1   /* U = 1/(4 pi |x|),     Uhat = 1/|k|^2, d = 3                    */
#define NLF_COULOMB2D 2   /* U = 1/(2 pi |x|),     Uhat = 1/|k|,   d = 2                    */
#define NLF_LAPLACE2D 3   /* U = -ln|x| / (2 pi),  Uhat = 1/|k|^2, d = 2 (Gaussian subtraction) */
/* Confined Coulomb kernel U_Con^eps of a strongly confined 3D Schroedinger-Poisson system,
 * d = 2 (Sec. 2.3, Eqs. 'ifft2d' and '2Dw1'): the polar quadrature of the 2D Coulomb kernel with
 * symbol x Jacobian W1(|k|) = (2/pi) int_0^inf e^{-eps^2 |k|^2 s^2 / 2} / (1 + s^2) ds, which
 * equals erfcx(eps |k| / sqrt 2) = e^{a^2} erfc(a) at a = eps |k| / sqrt 2 (W1(0) = 1).  The
 * plan tabulates W1 per node on the host in FP64; opts.eps > 0 is required.               */
#define NLF_CONFINED2D 4

/* ---- plan ----------------------------------------------------------------------------- */
typedef struct {
    int    dim;      /* 2 or 3                                                               */
    int    n[3];     /* grid points per axis (n[2] ignored in 2D)                             */
    double L[3];     /* half-widths: axis i spans [-L_i, L_i)                                 */
} nlf_box;

/* Plan options.  Any field left 0 takes its default.                                        */
typedef struct {
    int    prec;     /* NLF_F64 (default) or NLF_F32                                          */
    int    n_r;      /* radial Gauss-Legendre nodes on [0,P]        (default n[0])             */
    int    n_theta;  /* Gauss-Legendre nodes in cos(theta), 3D only (default n[0])             */
    int    n_phi;    /* trapezoid nodes in the azimuth, even        (default 2 n[0])           */
    double P;        /* Fourier cutoff radius                       (default pi / max_i h_i)   */
    double sigma;    /* Laplace subtraction width                   (default 6 sqrt(2) / P)    */
    int    msp;      /* Gaussian half-width in oversampled cells    (default 12 FP64, 7 FP32)  */
    int    batch;    /* independent fields per call                 (default 1)                */
    double eps;      /* confinement ratio of NLF_CONFINED2D, > 0     (no default; other kernels
                        ignore it)                                                             */
    int    split;    /* NLF_COULOMB3D only: nonzero evaluates the split form of Sec. 2.1,
                        Eq. '3.9', see below                                                    */
    double split_a;  /* width a of the partition p(k) = e^{-|k|^2/a}  (default (5.5/min L_i)^2) */
    int    deterministic;   /* nonzero: bitwise-reproducible results, see below                  */
    int    check_finite;    /* nonzero: nlf_potential and nlf_type2 wait for their work and return
                               NLF_ENONFINITE if the density held a NaN or Inf, see below         */
} nlf_opts;

/* Non-finite densities.  The pass that loads the density into the oversampled grid (the first
 * step of nlf_potential and nlf_type2, and of the potentials inside the solvers) sets a device flag
 * of the plan when a value is NaN or +-Inf; the potential of such a density is not defined and the
 * outputs then hold NaN.  On a plan created with opts.check_finite != 0, nlf_potential and
 * nlf_type2 synchronise the plan's stream at their end, return NLF_ENONFINITE if the flag was set
 * by this call, and clear it.  With the default 0 they return as soon as their work is enqueued
 * and do not look at the flag.  The gradient-flow solver reports NLF_ENONFINITE from its own
 * FP64 reductions whatever the option.
 *
 * Workspace cap.  If the environment variable NLF_MAX_WORKSPACE_BYTES holds a positive integer,
 * every device allocation a plan makes for itself (at nlf_plan_create, and the solver workspace
 * at the first solver call) fails with NLF_ENOMEM once the plan's total would exceed it; it is
 * read at each allocation.                                                                      */

/* Deterministic plans (opts.deterministic != 0; project addition, not in the paper).  By default
 * the spreading adds a tile's sum with one floating-point atomic per cell and work item, so two
 * calls agree only up to the order of those additions (and the 3D tile-gathered interpolation
 * adds each tile's part of a node's sum atomically).  On a deterministic plan a tile's only work
 * item stores its sums, the items of a tile of several store partial sums in slots of their own,
 * and a second kernel adds those in a fixed order; the 3D interpolation is the plane-streamed
 * kernel (one thread per node).  Every call, and every solver run on the plan, then gives the
 * same bits, at some cost (512^2: 6% FP64, 14% FP32 per evaluation; 256^3 split: 3.5%).
 * nlf_plan_set_spread returns NLF_EINVAL on such a plan and nlf_plan_autotune times its fixed
 * decomposition without changing it.  Plans that have neither candidate lists nor neighbour bins
 * (only the LDS-atomic scatter) return NLF_EUNSUPPORTED.                                       */

/* Split evaluation (Sec. 2.1, Eq. '3.9', Fig. 'fig3.1'; opts.split != 0, 3D Coulomb only):
 *   u = I1 + I2,  I1 = (2 pi)^-3 int_D e^{ik.x} (1 - p(k)) / |k|^2 rhohat dk  over the cube
 *   D = prod [-pi/h_i, pi/h_i) of the grid's frequencies, by the trapezoid rule on the lattice of
 *   the zero-padded FFT (a cyclic convolution: forward FFT of the padded density, a multiply by
 *   the smooth w = (1 - p)/|k|^2 (w(0) = 1/a), inverse FFT); and
 *   I2 = (2 pi)^-3 int_{|k| <= P2} e^{ik.x} p(k) rhohat d|k| dmu dphi  by the NUFFT path of this
 *   library on the small ball P2 = sqrt(34.5 a) (p(P2) ~ 1e-15), whose node count does not grow
 *   with the grid.  The default a puts I1's kernel erfc(sqrt(a) r/2)/(4 pi r) at erfc(5.5) at the
 *   nearest periodic image.  n_r, n_theta, n_phi set the ball's rule (default
 *   ceil(3 P2 D/8) + 8, the same, twice that; D = 2 |L| the box diameter); P and sigma must be 0.
 *   Needs pi / max h_i >= P2 (NLF_EUNSUPPORTED otherwise, e.g. 16^3 on [-8,8]^3).  On a split
 *   plan nlf_type2, nlf_type1, nlf_plan_nodes and the spreading controls act on the ball's
 *   nodes; stage times add the ball's stages to I1's (its forward FFT under FFT_FWD, the
 *   multiply and inverse FFT under FFT_INV).                                                  */

typedef struct nlf_plan nlf_plan;

/* Facts about a built plan, for callers that size their buffers.                            */
typedef struct {
    int    dim, kernel, prec, batch, msp;
    int    n[3];
    double L[3], h[3];
    double P, sigma;
    long long n_grid;      /* prod n_i                                                       */
    long long n_nodes;     /* M = n_r n_theta n_phi (3D) or n_r n_phi (2D), the full node set  */
    long long n_half;      /* M / 2 nodes actually evaluated (the other half by symmetry)      */
    long long workspace_bytes;
    /* spreading work decomposition in use (see nlf_plan_set_spread / nlf_plan_autotune) */
    int spread_mode;       /* NLF_SPREAD_GATHER, NLF_SPREAD_SCATTER or NLF_SPREAD_BINS        */
    int spread_block;      /* candidates per block of the gather kernel (64 or 128)         */
    int spread_item;       /* candidates per work item of the gather kernel (256 .. 2048)   */
    int gather_available;  /* 1 if the plan built its gather-tile candidate lists           */
    int bins_available;    /* 1 if the neighbour-bin gather applies (grids large enough)    */
    double eps;            /* confinement ratio (NLF_CONFINED2D), else 0                     */
    int split;             /* 1 for a split plan; then n_nodes/n_half/spread_* are the ball's */
    double split_a, split_P2;   /* partition width a and ball radius P2 (split plans)     */
    int deterministic;     /* 1 for a deterministic plan                                     */
} nlf_plan_info;

/* Create a plan for the potential of `kernel` on `box` (Sec. 2.1 nodes and weights, Eq.
 * 'ifft').  Builds the node tables on the host in FP64, sorts the nodes into bins of the
 * oversampled grid, uploads them and allocates the workspace.  `stream` is a hipStream_t.
 * Returns NLF_EUNSUPPORTED for a dimension/kernel mismatch or a non-power-of-two grid.     */
int nlf_plan_create(const nlf_box* box, int kernel, const nlf_opts* opts, void* stream,
                    nlf_plan** out);
int nlf_plan_destroy(nlf_plan* plan);
int nlf_plan_get_info(const nlf_plan* plan, nlf_plan_info* info);

/* ---- spreading work decomposition (project addition, not in the paper) -----------------------
 * NLF_SPREAD_GATHER: every gather tile of the oversampled grid (8 x 16 cells in 2D, 8 x 4 x 4 in
 *   3D) sums its candidate nodes as matrix products, in work items of `item` candidates taken
 *   `block` at a time, one atomic per cell and item.
 * NLF_SPREAD_SCATTER: each node adds its stencil into an LDS window of its bin (LDS atomics),
 *   then the window into the grid.
 * NLF_SPREAD_BINS: as GATHER, but a tile reads its candidates as the node ranges of a fixed box
 *   of neighbouring node bins (bins have the tile's shape) instead of a stored per-tile list:
 *   about 1.4x (3D) to 1.6x (2D) more candidates, no list memory; the default where the lists
 *   would be too large (e.g. 256^3).  Items of 512, 1024 or 2048 candidates.
 * nlf_plan_set_spread selects one (block 64 or 128; item 256, 512, 1024 or 2048; GATHER needs
 * the plan's candidate lists, info.gather_available; SCATTER is not available to FP32 plans with
 * candidate lists, which spread into an FP64 grid); returns NLF_EINVAL otherwise.
 * nlf_plan_autotune times every decomposition the plan supports on its own buffers (node values
 * set to 1, `reps` timed calls each, default 5 if reps <= 0), keeps the fastest and returns
 * its time per call in *best_ms (may be NULL).  Results are the same up to the summation order
 * of floating-point atomics.  Synchronises the plan's stream.                               */
enum { NLF_SPREAD_GATHER = 0, NLF_SPREAD_SCATTER = 1, NLF_SPREAD_BINS = 2 };
int nlf_plan_set_spread(nlf_plan* plan, int mode, int block, int item);
int nlf_plan_autotune(nlf_plan* plan, int reps, double* best_ms);

/* Quadrature nodes of the plan in canonical order (radial index slowest, then polar in 3D,
 * then azimuth fastest): k_host receives M*dim doubles (k_m components in grid-axis order),
 * w_host receives M doubles, the weight of d|k| dphi (2D) or d|k| dmu dphi (3D) without the
 * Jacobian (Sec. 2.1, Eq. 'ifft').  Host memory owned by the caller; either may be NULL.    */
int nlf_plan_nodes(const nlf_plan* plan, double* k_host, double* w_host);

/* u = U * rho on the grid (Sec. 2.1 Eq. 'ifft'; for NLF_LAPLACE2D Sec. 2.2 Alg. 1).
 * rho_dev: [batch][n] real; u_dev: [batch][n] real; plan precision; may not alias.        */
int nlf_potential(nlf_plan* plan, const void* rho_dev, void* u_dev);

/* Type-2 stage alone: rhohat_m = (prod h_i) sum_j rho_j e^{-i k_m . x_j} at all M nodes in
 * canonical order (the trapezoid transform of the grid data, Alg. 1 first step).
 * rho_dev: [batch][n] real; rhohat_dev: [batch][M] complex; plan precision.              */
int nlf_type2(nlf_plan* plan, const void* rho_dev, void* rhohat_dev);

/* Type-1 stage alone: u_j = Re sum_m c_m e^{+i k_m . x_j} over all M nodes in canonical
 * order (the final sum of Eq. 'ifft' once the symbol and weights are applied).
 * c_dev: [batch][M] complex; u_dev: [batch][n] real; plan precision.                     */
int nlf_type1(nlf_plan* plan, const void* c_dev, void* u_dev);

/* ---- stage timing (tracing) ----------------------------------------------------------------
 * When profiling is on, every potential evaluation of the plan records HIP events around each
 * stage on the plan's stream (this adds an event record between kernels; leave it off for
 * production use).  nlf_plan_stage_times synchronises the stream, returns the accumulated
 * milliseconds and the number of timed launches of each stage since the last reset, and resets
 * the accumulators if `reset` is non-zero.  ms and counts are host arrays of NLF_NSTAGES entries
 * (either may be NULL).                                                                         */
#define NLF_STAGE_MOMENTS   0   /* the FP64 moments of rho (Laplace kernel) are summed inside the
                                 * forward FFT passes; this stage reports 0                      */
#define NLF_STAGE_FFT_FWD   1   /* precorrect + pad + forward FFT of the oversampled grid          */
#define NLF_STAGE_INTERP    2   /* Gaussian interpolation to the nodes + symbol x weight           */
#define NLF_STAGE_ZERO      3   /* clearing the spreading grid                                     */
#define NLF_STAGE_SPREAD    4   /* Gaussian spreading from the nodes                               */
#define NLF_STAGE_FFT_INV   5   /* inverse FFT + truncate + postcorrect (+ u1)                     */
#define NLF_NSTAGES         6
int nlf_plan_set_profiling(nlf_plan* plan, int on);
int nlf_plan_stage_times(nlf_plan* plan, double* ms, long long* counts, int reset);

/* ---- solvers -------------------------------------------------------------------------- */
/* Physical parameters of one field: V = (1/2) sum_i gamma_i^2 x_i^2 unless V_dev != NULL, in
 * which case V_dev ([n] real FP64, device) is used.  beta is the interaction constant of Eq.
 * 'sps-eq'.  The solvers take a host array of `batch` entries, one per field; the V_dev of the
 * first entry, if set, applies to every field.                                               */
typedef struct {
    double      beta;
    double      gamma[3];
    const void* V_dev;
} nlf_phys;

/* Gradient-flow options (Sec. 3.1/3.2).  tau: time step (default 1e-2); eps0: stopping
 * tolerance on max|phi^{n+1}-phi^n|/tau (default 1e-10); max_iter (default 100000);
 * check_every: outer steps between host convergence checks (default 10);
 * cg_tol: final relative residual of the inner linear solve (default 1e-13 FP64, 1e-6 FP32; the
 * tolerance of each solve follows the outer residual down to it); cg_max_iter (default 200);
 * mixed: with an FP32 plan, run the flow in FP32 until the residual reaches eps_switch (default
 * 1e-5) or stops decreasing, then finish in FP64 on an FP64 twin of the plan (created on first
 * use, owned by the plan) down to eps0.  Energies are then those of the FP64 state; psi_dev is
 * returned rounded to the plan's precision.
 * graph: nonzero captures each outer step's kernels once (the potential and the set-up of the
 * linear solve, one inner iteration, the normalisation) as HIP graphs and replays them from the
 * second step on; 0 (default) launches every kernel individually.  Both give the same flow; on
 * the batched 2D workloads measured, the solve is bound by device time and direct launches were
 * the faster.  Stage profiling forces direct launches.                                       */
typedef struct {
    double tau, eps0;
    int    max_iter, check_every;
    double cg_tol;
    int    cg_max_iter;
    int    mixed;
    double eps_switch;
    int    graph;
    int    persistent;   /* nlf_ground_state_batch: nonzero runs an eligible batch in one persistent
                            launch (see there); 0 (default): one host thread per plan              */
} nlf_gf_opts;

typedef struct {
    int    iters;           /* outer gradient-flow steps this field took (all precisions)   */
    int    iters_fp32;      /* of which in FP32 (mixed schedule)                            */
    int    cg_iters;        /* inner linear-solver iterations, summed                       */
    double E, mu, Ekin, Epot, Eint;
    double residual;        /* last max|phi^{n+1}-phi^n|/tau                                 */
    double virial;          /* 2E_kin - 2E_pot + (E_int | beta/(4 pi)), Sec. 3.2             */
    double mass;            /* h^d sum |phi|^2                                               */
    int    persistent;      /* 1 if the field was solved inside the single persistent launch of
                               nlf_ground_state_batch (see there), 0 otherwise                  */
} nlf_gs_stats;

/* Ground state by the backward-Euler normalized gradient flow, Fourier pseudospectral in
 * space, potential by this plan (Sec. 3.1, Eqs. 'gf-eq2'-'gffg33').  The linear part is
 * implicit: (1/tau - Delta/2 + V + beta varphi^n) phi1 = phi^n / tau, solved by conjugate
 * gradients preconditioned with the inverse of (1/tau + alpha + |mu|^2/2) in Fourier space.
 * phys: host array of `batch` entries.  Converged fields are retired (their kernels exit early)
 * while the others continue.
 * psi0_dev: [batch][n] real initial guess or NULL (harmonic-oscillator Gaussian);
 * psi_dev: [batch][n] real output; stats: host array of `batch` entries.
 * Returns NLF_ENOCONV if any field hit max_iter (stats still filled).                       */
int nlf_ground_state(nlf_plan* plan, const nlf_phys* phys, const nlf_gf_opts* gf,
                     const void* psi0_dev, void* psi_dev, nlf_gs_stats* stats);

/* Several ground-state solves at once, e.g. one plan per grid size of a batch of instances of
 * uneven size: plan i (with its own batch B_i) takes phys[i] (B_i entries), psi0_dev[i] (or NULL),
 * psi_dev[i] and stats[i] (B_i entries), exactly as nlf_ground_state.
 * One persistent launch (project addition): with gf->persistent set, when every plan is 2D with at
 * most 256 points per axis, all plans share one precision and the default stencil widths, spread by
 * gather lists and are neither deterministic nor profiled, and gf->graph is 0 (at most 16 plans),
 * the whole batch runs in ONE cooperative kernel launch on the first plan's stream.  The kernels of one outer step
 * of each plan are recorded once and replayed on the device for every plan together, with grid
 * barriers between them; the inner and outer loops, the retirement of each field at eps0 and,
 * with gf->mixed, the switch of every plan from its FP32 stage to its FP64 twin run on the device.
 * The launch is ordered after the earlier work of every plan's stream and before its later work.
 * stats[].persistent is 1 for fields solved this way.  The launch's grid barriers (about a hundred
 * per outer step) each cost a write-back of every XCD's L2, so on the batches measured this path is
 * slower than the default.  Otherwise the solves run concurrently, one host thread per plan (give
 * the plans distinct streams so that their kernels overlap).  Returns the
 * first error, else NLF_ENOCONV if any field did not reach eps0, else NLF_OK.                  */
int nlf_ground_state_batch(int count, nlf_plan* const plans[], const nlf_phys* const phys[],
                           const nlf_gf_opts* gf, const void* const psi0_dev[], void* const psi_dev[],
                           nlf_gs_stats* const stats[]);

/* Time-splitting pseudospectral dynamics (Sec. 4.1, Eqs. 'sps-eq65'-'sps-eq68').
 * order 2: Strang K(dt/2) P(dt) K(dt/2); order 4: Yoshida composition of three Strang steps.
 * phys: host array of `batch` entries.  Adjacent kinetic half steps are merged.
 * psi_dev: [batch][n] complex, in/out.  diag_host: if non-NULL, receives (mass, energy) per
 * field every diag_every steps and at step 0: 2 * batch * (nsteps/diag_every + 1) doubles.   */
typedef struct {
    double dt;
    int    nsteps, order, diag_every;
} nlf_ts_opts;

int nlf_evolve(nlf_plan* plan, const nlf_phys* phys, const nlf_ts_opts* ts, void* psi_dev,
               double* diag_host);

/* ---- learned warm start (project addition, not in the paper) ----------------------------------
 * A small FP32 MLP, x (n_in) -> tanh(W1 x + b1) (H) -> tanh(W2 . + b2) (H) -> W3 . + b3 (n_out),
 * whose inputs are standardised by (x - mean) / stdv.  For the warm start the inputs are
 * (ln beta, gamma_0, .., gamma_{d-1}) of a field and the outputs its ground state on a coarse
 * grid of coarse_n^d points of the same box.  All device arrays are FP32 and row-major; the
 * parameter vector is W1 [n_in][H], b1 [H], W2 [H][H], b2 [H], W3 [H][n_out], b3 [n_out].
 * The model owns its device buffers; calls run on its stream.                                 */
typedef struct nlf_model nlf_model;
int nlf_ws_create(int n_in, int n_hidden, int n_out, unsigned long long seed, void* stream,
                  nlf_model** out);      /* Glorot-uniform weights from seed, zero biases       */
int nlf_ws_destroy(nlf_model* model);
int nlf_ws_num_params(const nlf_model* model, long long* count);
/* copy the parameters out to / in from host memory (either pointer may be NULL)                */
int nlf_ws_params(nlf_model* model, float* host_out, const float* host_in);
int nlf_ws_set_standardisation(nlf_model* model, const float* mean_host, const float* stdv_host);
/* y_dev [batch][n_out] = network(x_dev [batch][n_in])                                           */
int nlf_ws_forward(nlf_model* model, int batch, const float* x_dev, float* y_dev);
/* mean-squared-error loss of one batch against t_dev [batch][n_out] and its gradient with respect
 * to the parameters (grad_dev: n_params floats, or NULL); loss_host may be NULL               */
int nlf_ws_loss_grad(nlf_model* model, int batch, const float* x_dev, const float* t_dev, float* grad_dev,
                     double* loss_host);
/* Adam (b1 0.9, b2 0.999, eps 1e-8) over `epochs` passes of minibatches of the n samples;
 * loss_host (epochs entries, or NULL) receives the mean minibatch loss of each epoch           */
int nlf_ws_train(nlf_model* model, int n, const float* x_dev, const float* t_dev, int epochs, int minibatch,
                 double lr, double* loss_host);
/* Initial guesses for the plan's fields from their parameters (phys: batch entries, beta > 0):
 * network output on the coarse grid (coarse_n even, <= 1024), resampled to the plan grid by
 * band-limited (periodic Dirichlet-kernel) interpolation along each axis in FP64, absolute value;
 * psi0_dev [batch][n] in the plan precision (nlf_ground_state normalises it).                  */
int nlf_ws_predict(nlf_model* model, nlf_plan* plan, const nlf_phys* phys, int coarse_n, void* psi0_dev);

/* Warm-started ground states: the network's guess (nlf_ws_predict) and the harmonic-oscillator
 * Gaussian each take one gradient-flow step; per field the start with the smaller residual
 * max|phi^1 - phi^0|/tau is kept (the Gaussian is the fallback), then nlf_ground_state runs from
 * it.  used_host (batch ints, or NULL) receives 1 where the network's guess was kept.  The two
 * judging steps are included in stats[].iters.                                                */
int nlf_ws_ground_state(nlf_model* model, int coarse_n, nlf_plan* plan, const nlf_phys* phys,
                        const nlf_gf_opts* gf, void* psi_dev, nlf_gs_stats* stats, int* used_host);

/* ---- no-allocation entry point (project addition, not in the paper) -------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, serving loops that
 * forbid allocation.  Computes exactly what nlf_potential computes, with the same kernels, but the
 * call's scratch (the two oversampled grids, the node values, the 3D node accumulators, the moments
 * and their partial sums) lives in a fixed device array of the library of NLF_NOALLOC_MAX_BYTES
 * bytes, of which every GPU the library runs on holds its own copy until the process ends.  The
 * call allocates nothing (no hipMalloc, no hipFree, no allocating library routine).
 * A plan whose scratch would exceed the array returns NLF_EINVAL; split and deterministic plans
 * return NLF_EUNSUPPORTED.  All calls on one GPU share that GPU's array and it keeps the last
 * call's contents (each call writes every scratch value before reading it): calls that overlap in
 * time on one GPU, from other streams or threads, race, and the caller must serialise them.
 * Arguments, stream and errors as nlf_potential.                                                 */
#define NLF_NOALLOC_MAX_BYTES (64ull << 20)
int nlf_potential_noalloc(nlf_plan* plan, const void* rho_dev, void* u_dev);

/* Message for the calling thread's last error ("" if none).                                 */
const char* nlf_last_error(void);
/* Static description of a status code.                                                      */
const char* nlf_strerror(int status);
/* Library version string.                                                                    */
const char* nlf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NLF_H */
