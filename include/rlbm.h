/*
 * rlbm.h -- C ABI of the MI355X (gfx950) relativistic lattice Boltzmann
 * solver for massless particles in (2+1) dimensions.
 *
 * The method is that of Bazzanini, Gabbana, Simeoni, Succi and Tripiccione,
 * "A Lattice Boltzmann Method for Relativistic Rarefied Flows in (2+1)
 * Dimensions" (arXiv:2011.06856):
 *   - discrete velocities from the product quadrature of Sec. 2.3, Eq.
 *     off-lattice-quad: Np radial Gauss-Laguerre shells times K equispaced
 *     angles, shell i rotated by i/Np of the angular spacing; every velocity
 *     has unit speed and none lies on the lattice;
 *   - one time step (Eq. discrete-rbe) = bilinear upwind streaming (Eq.
 *     streaming, Eq. interpolation), moments (Eq. discrete_sum_moments),
 *     Landau-frame solve (eps U^a = T^{ab} U_b, eps = 2P = 2nT), the truncated
 *     Maxwell-Juttner equilibrium of order N (Eq. mj-feq-expansion-truncated)
 *     and Anderson-Witting relaxation (Eq. collision, with the relaxing sign of
 *     Eq. discrete-rbe), fused into one kernel.
 *
 * Units: lattice units, dx = dy = 1, c = 1, weighting temperature T0 = 1.
 * Grids are [ny][nx] row-major.  Velocity index v = i*K + j (shell i, angle j).
 * Populations live on the device as f[v][y][x] (structure of arrays).
 *
 * Every call returns an int status: RLBM_OK (0) or a negative error code; no
 * exception crosses the ABI.  rlbm_last_error() gives a message for the last
 * failing call on a context.  One host thread may use a context at a time;
 * distinct contexts are independent.
 */
#ifndef RLBM_H
#define RLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlbm_ctx_s* rlbm_ctx;

enum {
    RLBM_OK = 0,
    RLBM_EINVAL = -1,   /* invalid argument; nothing was changed */
    RLBM_ENOMEM = -2,   /* device allocation failed or workspace too small */
    RLBM_EDEVICE = -3,  /* a HIP call failed (no device, launch failure) */
    RLBM_ENONPHYS = -4, /* some site had no physical Landau frame (sticky) */
    RLBM_ESTATE = -5    /* call out of order (e.g. step before init_fields) */
};

/* Population storage.
 *   F64, F32   the populations f, in FP64 or FP32.
 *   BF16DEV    the departure g = f - F of the populations from the truncated
 *              equilibrium F of each site's last collision (Eq.
 *              mj-feq-expansion-truncated), stored in bfloat16, with F kept as
 *              per-shell harmonic coefficients in FP32 (Np x (2 Nm + 1) per
 *              site, Nm = 3, 5 or 7 the order class of N): 2 bytes per
 *              site-velocity instead of 4.  Arithmetic in FP32, Landau frame in
 *              FP64.  Rounding g to bfloat16 each step is the only departure
 *              from the FP32 method.
 *   F32DEV     the same representation with g in FP32;
 *   F64DEV     with g and the coefficients in FP64 (equal to the FP64 method up
 *              to rounding).
 * The deviation storages run on the push kernel (RLBM_KERNEL_PUSH) with
 * periodic or clamped axes and Maxwell-Juttner statistics, one problem per
 * context (not in a batch, not with the learned-form calls). */
enum { RLBM_F64 = 0, RLBM_F32 = 1, RLBM_BF16DEV = 2, RLBM_F32DEV = 3, RLBM_F64DEV = 4 };
/* Boundary condition per axis: what an upwind point outside the grid holds
 * (the paper's box domain states none and names boundary conditions as the
 * next step, Sec. 4):
 *   PERIODIC  the point on the opposite side;
 *   CLAMP     the edge cell's population (zero gradient: free outflow);
 *   WALL      the target cell's population of the reversed velocity
 *             (theta + pi, same shell): halfway bounce-back, conserving mass
 *             and energy per cell; needs an even number of angles;
 *   FIXED     the population the edge cell had at rlbm_init_fields (a
 *             reservoir at the initial state: inflow and outflow).
 * WALL and FIXED run on the tile kernel (RLBM_KERNEL_TILE). */
enum { RLBM_BC_PERIODIC = 0, RLBM_BC_CLAMP = 1, RLBM_BC_WALL = 2, RLBM_BC_FIXED = 3 };   /* per axis */
enum { RLBM_KERNEL_AUTO = 0, RLBM_KERNEL_TILE = 1, RLBM_KERNEL_PUSH = 2 };   /* step kernel */
enum { RLBM_STAT_MJ = 0, RLBM_STAT_FERMI = 1, RLBM_STAT_BOSE = 2 };           /* equilibrium statistics */

/*
 * Build the quadrature of Sec. 2.3 (Eq. off-lattice-quad) on the host and
 * create a context.  No device call is made.
 *   n_radial  Np >= 1 shells at the roots of L_Np, weights
 *             p_i / ((Np+1)^2 L_{Np+1}(p_i)^2);
 *   n_angle   K angles per shell, K >= 2N+1 (exactness of the angular rule);
 *   order     N >= 1, order of the equilibrium expansion, N <= 7, and
 *             Np >= ceil((N+3)/2) so that N^mu and T^{mu nu} of f_eq are exact;
 *   rotate    1: theta_ij = (j + i/Np) 2 pi / K; 0: theta_ij = 2 pi j / K.
 * On success *out owns host memory released by rlbm_destroy.
 * Errors: RLBM_EINVAL for out == NULL or any bound above.
 */
int rlbm_init_quadrature(rlbm_ctx* out, int n_radial, int n_angle, int order, int rotate);

/* Number of discrete velocities Np*K of the context. */
int rlbm_nvel(rlbm_ctx ctx);

/*
 * Copy the quadrature out: p[v] = p^0 (shell energy), theta[v], w[v] (weights
 * summing to 2 pi).  Each pointer is a caller-owned host array of rlbm_nvel()
 * doubles, or NULL to skip it.
 */
int rlbm_get_quadrature(rlbm_ctx ctx, double* p, double* theta, double* w);

/* Device workspace in bytes needed by rlbm_init_fields for an nx x ny grid at
 * the given precision: two population buffers of nvel + 1 planes, the field
 * outputs (4 doubles per site), the partial charges, and the two partial-sum
 * buffers of the push kernel (3 row slots x 8 moments per site plus a halo
 * per tile edge), present whichever step kernel is used, and for deviation
 * storage two buffers of equilibrium coefficients (Np x (2 Nm + 1) per site,
 * FP32, or FP64 for RLBM_F64DEV). */
int rlbm_workspace_bytes(rlbm_ctx ctx, int nx, int ny, int precision, size_t* bytes);

/*
 * Set the initial populations to the truncated equilibrium of the given
 * fields (a fluid whose sites are each in local equilibrium; Sec. 3) and fix
 * the run parameters.
 *   n, T, ux, uy  host arrays [ny][nx], caller-owned, read only during the
 *                 call: density, temperature and the spatial components U^i of
 *                 the four-velocity; ux/uy may be NULL (zero).  Rejected with
 *                 RLBM_EINVAL unless finite, n > 0, T > 0.
 *   tau           proper relaxation time > 0 (Eq. boltz_eq); +inf = free
 *                 streaming.  Kn = tau / L (Sec. 3.1).
 *   dt            time step in (0, 1] (the bilinear weights dt |v_x|, dt |v_y|
 *                 must stay in [0, 1]).
 *   bc_x, bc_y    RLBM_BC_PERIODIC, RLBM_BC_CLAMP, RLBM_BC_WALL (n_angle
 *                 even) or RLBM_BC_FIXED, per axis (see the enum above).
 *   precision     population storage: RLBM_F64, RLBM_F32, or a deviation
 *                 storage (RLBM_BF16DEV, RLBM_F32DEV, RLBM_F64DEV), which
 *                 starts from g = 0 (f is exactly the truncated equilibrium
 *                 of the fields) and needs periodic or clamped axes and
 *                 Maxwell-Juttner statistics (RLBM_EINVAL otherwise).
 *   d_workspace   device memory of at least rlbm_workspace_bytes() bytes,
 *                 256-byte aligned, owned by the caller (e.g. a torch tensor)
 *                 and alive until rlbm_destroy; NULL lets the library
 *                 allocate and own it.
 *   hip_stream    hipStream_t for all work of this context; NULL = default.
 * Builds the device tables of both step kernels (library-owned, freed by the
 * next rlbm_init_fields or rlbm_destroy) and the initial populations;
 * synchronises the stream.  May be called again to restart a context (same
 * or different grid).  Any failure after the argument checks leaves the
 * context without fields: rlbm_step and rlbm_moments then return
 * RLBM_ESTATE until a call succeeds.
 */
int rlbm_init_fields(rlbm_ctx ctx, int nx, int ny,
                     const double* n, const double* T, const double* ux, const double* uy,
                     double tau, double dt, int bc_x, int bc_y, int precision,
                     void* d_workspace, void* hip_stream);

/*
 * Advance nsteps >= 0 time steps (Eq. discrete-rbe), one fused
 * stream-and-collide launch per step, asynchronously on the context's
 * stream.  Allocates nothing and makes no synchronising call, so the
 * launches can be captured into a HIP graph: the two population buffers
 * alternate, so a graph of an even number of steps replays correctly any
 * number of times (the push kernel's partial sums must be valid first: one
 * eager step after rlbm_init_fields, rlbm_set_populations or
 * rlbm_set_kernel).  Non-physical sites (no timelike Landau eigenvector,
 * n <= 0 or eps <= 0) are streamed without collision and raise a sticky
 * device flag reported by the next rlbm_moments.
 */
int rlbm_step(rlbm_ctx ctx, int nsteps);

/*
 * Like rlbm_step, bracketing the launches with HIP events on the context's
 * stream; synchronises and returns the elapsed milliseconds in *ms.
 */
int rlbm_step_timed(rlbm_ctx ctx, int nsteps, double* ms);

/*
 * Macroscopic fields of the current populations (moments, Eq.
 * discrete_sum_moments, then the Landau frame, all in FP64): n, eps = T^{ab}
 * U_a U_b, ux = U^x, uy = U^y, each a caller-owned host array [ny][nx] or
 * NULL; charges = {sum N^0, sum T^00, sum T^0x, sum T^0y} over the grid
 * (4 doubles) or NULL.  Synchronises the stream.  Returns RLBM_ENONPHYS if any
 * step or this call met a non-physical site (the outputs are still written;
 * such sites hold NaN); the flag is then cleared.
 */
int rlbm_moments(rlbm_ctx ctx, double* n, double* eps, double* ux, double* uy, double* charges);

/*
 * For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid allocation): the fields and charges of
 * rlbm_moments, computed by the same kernel, into caller-owned DEVICE memory,
 * asynchronously on the context's stream.
 *   d_fields   device [4][ny][nx] doubles: n, eps, U^x, U^y (NaN at
 *              non-physical sites), or NULL to skip;
 *   d_charges  device [4] doubles: sum N^0, T^00, T^0x, T^0y, or NULL.
 * Allocates nothing and makes no synchronising call: the per-block partial
 * charges go to a fixed device scratch array of the library (2 MiB on each
 * device it runs on, held until the process ends), which limits the grid to
 * 16,777,216 sites (RLBM_EINVAL beyond).  Every call on one device shares
 * that array, so calls that overlap in time on one device (other streams,
 * other host threads) race: order them.  A non-physical site raises the
 * context's sticky flag, reported by the next rlbm_moments.  RLBM_ESTATE
 * before rlbm_init_fields.
 */
int rlbm_moments_device(rlbm_ctx ctx, double* d_fields, double* d_charges);

/* Checkpoint: copy the current populations (storage precision, layout
 * f[v][y][x]) to / from a caller-owned host buffer of exactly
 * rlbm_populations_bytes() bytes; other sizes give RLBM_EINVAL.  Plain
 * storage: nvel * nx * ny elements (8 bytes for F64, 4 for F32).  Deviation
 * storage: the deviations g[v][y][x] (2, 4 or 8 bytes for BF16DEV, F32DEV,
 * F64DEV), then the equilibrium coefficients C[i][t][y][x] (FP32, FP32,
 * FP64) of shell i and harmonic t = {1, cos th, sin th, ..., cos Nm th,
 * sin Nm th} (2 Nm + 1 per shell), with f_v = g_v + w_v sum_t C[shell(v)][t]
 * harmonic_t(th_v).  A run resumed from a checkpoint continues bit for bit.
 * Synchronous. */
int rlbm_populations_bytes(rlbm_ctx ctx, size_t* bytes);
int rlbm_get_populations(rlbm_ctx ctx, void* host, size_t bytes);
int rlbm_set_populations(rlbm_ctx ctx, const void* host, size_t bytes);

/*
 * Kernel shape: waves per work-group (1..16) of the fused kernel, 0 = the
 * built-in choice.  Results do not depend on it beyond rounding order.  Used
 * by the autotuner and by tile-shape tests.  RLBM_EINVAL if unsupported.
 */
int rlbm_set_waves(rlbm_ctx ctx, int waves);

/*
 * Step kernel (Sec. 2.2, Eqs. streaming, interpolation, discrete_sum_moments,
 * collision: the same step, two schedules):
 *   RLBM_KERNEL_TILE  a work-group gathers, holds and reduces all streamed
 *                     values of 64 sites before their collision;
 *   RLBM_KERNEL_PUSH  each wave runs through all velocities of 64 sites once;
 *                     its moments come from partial sums pushed by the
 *                     previous step (3 row slots x 8 moments per site plus a
 *                     halo per tile edge, in two buffers of the workspace;
 *                     recomputed by the next rlbm_step after any external
 *                     change of the populations);
 *   RLBM_KERNEL_AUTO  (default) PUSH from 320 velocities on, else TILE
 *                     (measured crossover between 256 and 384); TILE on a
 *                     grid with a WALL or FIXED axis.
 * The results agree to rounding.  rlbm_get_kernel returns the kernel that
 * rlbm_step uses.  RLBM_EINVAL for an unknown kind, and for PUSH on a grid
 * with a WALL or FIXED axis.
 */
int rlbm_set_kernel(rlbm_ctx ctx, int kind);
int rlbm_get_kernel(rlbm_ctx ctx, int* kind);
int rlbm_get_waves(rlbm_ctx ctx, int* waves);

/* ------------------------------------------------------------------------ */
/* Batched form: many independent problems of uneven grid size, quadrature   */
/* and Knudsen number advance together.                                       */
/* ------------------------------------------------------------------------ */

typedef struct rlbm_batch_s* rlbm_batch;

/* One problem of a batch: the arguments of rlbm_init_quadrature and
 * rlbm_init_fields (host field arrays [ny][nx], read during
 * rlbm_batch_create only). */
typedef struct {
    int n_radial, n_angle, order, rotate;
    int nx, ny;
    const double *n, *T, *ux, *uy;
    double tau, dt;
    int bc_x, bc_y;
} rlbm_problem;

/*
 * Create a batch of count problems at one population precision (RLBM_F32 or
 * RLBM_F64), each initialised to local equilibrium as by rlbm_init_fields,
 * with library-owned device memory; all work goes to hip_stream, which must
 * not be the null stream (graphs cannot capture it); NULL makes the batch
 * create and own a stream.  Boundaries: RLBM_BC_PERIODIC or RLBM_BC_CLAMP per
 * axis.  All problems must share the equilibrium order class (order <= 3,
 * 4..5 or 6..7), since one kernel instance serves the launch.  RLBM_EINVAL as
 * for the single-problem calls.
 */
int rlbm_batch_create(rlbm_batch* out, const rlbm_problem* probs, int count, int precision, void* hip_stream);
int rlbm_batch_count(rlbm_batch b);

/* The context of problem i (0-based), for rlbm_moments, rlbm_get_populations
 * and rlbm_set_populations; owned by the batch, valid until
 * rlbm_batch_destroy; must not be stepped on its own. */
int rlbm_batch_problem(rlbm_batch b, int i, rlbm_ctx* ctx);

/*
 * Advance every problem nsteps steps.  A step of the problems that the tile
 * kernel serves is one persistent launch whose work-groups take (problem,
 * tile) items from per-XCD work queues until all are drained (the launch
 * leaves its queue counters at zero for the next one); the problems that the
 * push kernel serves (RLBM_KERNEL_AUTO's choice, as for one problem) follow
 * in one flat launch.  Pairs of steps are replayed from a captured HIP graph.
 * Asynchronous; allocates nothing after the first call for a shape.
 * rlbm_batch_step_eager issues the same launches without the graph.
 */
int rlbm_batch_step(rlbm_batch b, int nsteps);
int rlbm_batch_step_eager(rlbm_batch b, int nsteps);
int rlbm_batch_step_timed(rlbm_batch b, int nsteps, double* ms);

/* Work-group shape (waves per group, 1..16; 0 = built-in choice). */
int rlbm_batch_set_waves(rlbm_batch b, int waves);
int rlbm_batch_get_waves(rlbm_batch b, int* waves);

/*
 * Launch mode of a batch step:
 *   RLBM_BATCH_PERSISTENT  resident work-groups take (problem, tile) items
 *                          from 8 XCD-local atomic work queues (default);
 *   RLBM_BATCH_FLAT        one work-group per item, dispatched by the hardware.
 * Both run the same tile computation, so results are identical bit for bit.
 */
enum { RLBM_BATCH_PERSISTENT = 0, RLBM_BATCH_FLAT = 1 };
int rlbm_batch_set_mode(rlbm_batch b, int mode);
int rlbm_batch_get_mode(rlbm_batch b, int* mode);

/*
 * Work-group order of the push-kernel problems: work-groups run through
 * groups of `bands` bands of 4 grid rows column by column (1..64; 0 = built-in
 * choice, 2).  Only the order in which the hardware meets the work-groups
 * changes (how long an upwind row stays in the L2), so results are identical
 * bit for bit for every value.  Takes effect at the next step (descriptors
 * and graph are rebuilt then, outside the timed region of
 * rlbm_batch_step_timed).
 */
int rlbm_batch_set_push_bands(rlbm_batch b, int bands);
int rlbm_batch_get_push_bands(rlbm_batch b, int* bands);

/*
 * Autotuner: time `steps` graph-replayed steps for each candidate shape
 * (waves per work-group) in both launch modes and keep the fastest pair;
 * then, when the batch holds push-kernel problems, time the band groupings
 * 1, 2, 4 and 8 with that pair and keep the fastest.  Reports the shape and
 * the best time (rlbm_batch_get_mode and rlbm_batch_get_push_bands give the
 * rest); the populations are saved before and restored after, so the state
 * is unchanged.  Allocates a temporary copy of the populations.
 */
int rlbm_batch_autotune(rlbm_batch b, const int* candidates, int ncand, int steps, int* best_waves, double* best_ms);

/* Launch shape for the current work-group shape: resident work-groups of the
 * persistent launch and (problem, tile) work items per step. */
int rlbm_batch_info(rlbm_batch b, int* grid, int* items);

const char* rlbm_batch_last_error(rlbm_batch b);
int rlbm_batch_destroy(rlbm_batch b);

/* ------------------------------------------------------------------------ */
/* Learned form: an MLP correction of the traceless stress of a coarse-angle  */
/* run, trained on fine-angle runs.                                           */
/* ------------------------------------------------------------------------ */

typedef struct rlbm_mlp_s* rlbm_mlp;

/*
 * A fully connected network in_dim -> hidden (n_hidden layers, GELU) ->
 * out_dim, for batches of up to max_batch rows, its work on hip_stream.
 * Parameters: one flat FP32 vector [W1 (hidden x in_dim, row-major), b1, W2,
 * b2, ..., Wout (out_dim x hidden), bout], zero at creation.  The forward
 * pass uses the weights rounded to bfloat16 (round to nearest even) with FP32
 * accumulation; gradients are taken with respect to those rounded weights and
 * applied by Adam to the FP32 master copy.
 */
int rlbm_mlp_create(rlbm_mlp* out, int in_dim, int hidden, int n_hidden, int out_dim, int max_batch,
                    void* hip_stream);
long rlbm_mlp_nparams(rlbm_mlp m);
int rlbm_mlp_set_params(rlbm_mlp m, const float* host);   /* also resets Adam */
int rlbm_mlp_get_params(rlbm_mlp m, float* host);
int rlbm_mlp_get_grad(rlbm_mlp m, float* host);          /* last rlbm_mlp_grad result */

/* Feature and output scales of the correction: network input k of a site is
 * (field - in_mu[k]) / in_sig[k] for the 7 fields (n, eps, U^x, U^y, pi^xx,
 * pi^xy, pi^yy); output j is de-normalised as out_mu[j] + out_sig[j] * y_j
 * (out_mu, out_sig: out_dim values each, out_dim <= 8). */
int rlbm_mlp_set_norm(rlbm_mlp m, const float* in_mu, const float* in_sig, const float* out_mu, const float* out_sig);

/* Device pointers: dX [B][in_dim], dY [B][out_dim], dT [B][out_dim]. */
int rlbm_mlp_forward(rlbm_mlp m, const float* dX, int B, float* dY);
/* Loss 0.5/B sum (y - t)^2 and its gradient (kept inside; rlbm_mlp_get_grad). */
int rlbm_mlp_grad(rlbm_mlp m, const float* dX, const float* dT, int B, double* loss);
int rlbm_mlp_adam_step(rlbm_mlp m, float lr, float beta1, float beta2, float eps);

/* Per-site fields of a context's current populations (FP64 moments and
 * Landau frame), device [S][8] = n, eps, U^x, U^y, pi^xx, pi^xy, pi^yy, 0, where
 * pi^ij = T^ij - (eps + P) U^i U^j - P delta^ij, P = eps/2 (Eq. ll-decomp). */
int rlbm_site_stats(rlbm_ctx c, float* dstats);
/* Network inputs of every site: the 7 fields of its 3x3 neighbourhood
 * (periodic), normalised, device [S][64]; column 63 holds the network's
 * per-run input (rlbm_mlp_set_extra, 0 by default). */
int rlbm_mlp_features(rlbm_ctx c, rlbm_mlp m, float* dX);
/* The per-run input of the features' column 63 (e.g. log10 Kn), used by
 * rlbm_mlp_features and rlbm_mlp_correct until changed. */
int rlbm_mlp_set_extra(rlbm_mlp m, float extra);
/*
 * In-loop correction: inputs, forward pass, and the predicted change
 * (dT^xx, dT^xy, dT^yy), times scale, put into the populations through the
 * m = 2 basis function p^2 {cos, sin}(2 theta):
 *   f_v += w_v p_v^2 [(dT^xx - dT^yy) cos 2th_v + 2 dT^xy sin 2th_v] / (24 pi),
 * which changes T^xx - T^yy and T^xy and leaves N^mu, T^00 and T^0i unchanged.
 * relax = 0: the output is the change itself (dT = scale * output).
 * relax = 1: the output is a target shear stress and the site relaxes
 *            toward it, dT = scale * (output - pi) with pi the site's
 *            current Landau-frame shear stress.
 * Requires S <= max_batch and a shared stream.
 */
int rlbm_mlp_correct(rlbm_ctx c, rlbm_mlp m, float scale, int relax);
/*
 * Readout correction of the macroscopic fields of a coarse-angle run (a
 * network with out_dim = 4; the correction is to the fields of Eq. rel_err,
 * not to the populations):
 *   inputs   the features of rlbm_mlp_features with column 63 = extra (the
 *            network is trained with a per-run scalar there, log10 Kn; it
 *            also becomes the network's rlbm_mlp_set_extra value);
 *   outputs  y (de-normalised with rlbm_mlp_set_norm's out_mu, out_sig);
 *   fields   n (1 + y0), eps (1 + y1), U^x + y2, U^y + y3 of the current
 *            populations, to host arrays [ny][nx] (caller-owned, any NULL).
 * The populations are not changed.  Synchronous; RLBM_ENONPHYS as
 * rlbm_moments; RLBM_EINVAL if out_dim != 4 or S > max_batch.
 */
int rlbm_mlp_readout(rlbm_ctx c, rlbm_mlp m, float extra, double* n, double* eps, double* ux, double* uy);
/* The same change of the traceless stress from a device array [S][3] =
 * (dT^xx, dT^xy, dT^yy), times scale (e.g. to give a local-equilibrium state
 * a prescribed shear stress). */
int rlbm_add_stress(rlbm_ctx c, const float* dstress, float scale);
/* Resample src's populations onto dst's angle set: both contexts on the same
 * grid and radial shells (same n_radial and rotation), any K each, FP32 or
 * FP64.  Per shell the angular harmonics |m| <= M = (min(K_src, K_dst)-1)/2
 * of src are evaluated at dst's angles, so every moment of angular order <= M
 * (N^mu, T^munu) is kept.  Used to restrict a fine-angle state to a coarse
 * one (training data of the learned correction) and to lift it back.
 * Synchronous.  RLBM_EINVAL on mismatched grids or shells. */
int rlbm_resample(rlbm_ctx src, rlbm_ctx dst);
const char* rlbm_mlp_last_error(rlbm_mlp m);
int rlbm_mlp_destroy(rlbm_mlp m);

/*
 * Host-side evaluations with the context's own tables; no device call is
 * made, so they run without a GPU.
 *   rlbm_host_feq     the discrete truncated equilibrium f_eq_v of fields
 *                     (n, T, U^x, U^y) (Eq. mj-feq-expansion-truncated) into a
 *                     caller-owned array of rlbm_nvel() doubles;
 *   rlbm_host_landau  the Landau frame (eps U^a = T^{ab} U_b, eps = 2nT) of
 *                     mom9 = (N^0, N^x, N^y, T^00, T^0x, T^0y, T^xx, T^xy,
 *                     T^yy): out6 = (n, eps, U^x, U^y, T, U^0); returns
 *                     RLBM_ENONPHYS for a state without a physical frame.
 */
int rlbm_host_feq(rlbm_ctx ctx, double n, double T, double ux, double uy, double* feq);
int rlbm_host_landau(const double* mom9, double* out6);

/*
 * The Landau frame evaluated by the device code of the kernels for count
 * moment sets: mom = host [count][9] as for rlbm_host_landau, out = host
 * [count][7] = (n, eps, U^x, U^y, T, U^0, ok).  Synchronous on the default
 * stream; allocates and frees its own device scratch.  RLBM_EDEVICE on a HIP
 * failure.  A check of the device arithmetic, not part of the time step.
 */
int rlbm_device_landau(int count, const double* mom, double* out);

/* Message for the last failing call on ctx (static storage of the context). */
const char* rlbm_last_error(rlbm_ctx ctx);

/*
 * Equilibrium statistics of the context (Sec. 2.1, Eq. feq_dist:
 * f_eq proportional to 1 / (z^-1 exp(U.p / T) + epsilon), z = exp(mu / T)):
 *   RLBM_STAT_MJ     Maxwell-Juttner (epsilon = 0; the default);
 *   RLBM_STAT_FERMI  Fermi-Dirac (epsilon = 1);
 *   RLBM_STAT_BOSE   Bose-Einstein (epsilon = -1).
 * The normalisation is 1/(2 pi) for all three, so that n = T^2 G_1(z) with
 * G_k(z) = z, -Li_{k+1}(-z), Li_{k+1}(z); the truncated expansion uses the
 * same basis and quadrature, its rank-k coefficients scaled by
 * G_k(z) / G_1(z).  Each step takes (n, eps, U) from the Landau frame, then
 * z from eps^2 / n^3 = 4 G_2^2 / G_1^3 and T = sqrt(n / G_1); a frame without
 * such an equilibrium (Fermi-Dirac below the degenerate limit eps^2 / n^3 =
 * 8/9, Bose-Einstein above condensation) is non-physical.  Takes effect at
 * the next rlbm_init_fields (which, for Bose-Einstein, rejects sites with
 * n / T^2 >= zeta(2)) and applies to rlbm_host_feq at once.  Fermi-Dirac and
 * Bose-Einstein run on the tile kernel.  RLBM_EINVAL for another value.
 */
int rlbm_set_statistics(rlbm_ctx ctx, int statistics);

/* Release the context, its tables and any library-owned workspace. */
int rlbm_destroy(rlbm_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* RLBM_H */
