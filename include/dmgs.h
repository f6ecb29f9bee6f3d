/*
 * dmgs.h -- C ABI of the differentiable geometric-multigrid solver for the
 * steady-state diffusion-absorption equation on an AMD Instinct MI355X
 * (gfx950).
 *
 * Problem (paper, Sec. 2, Eq. (maineq)): -div(D grad rho) + mua rho = q on a
 * cube with Dirichlet boundary rho = g, discretised by a second-order 7-point
 * finite-difference stencil on a vertex-centred grid of N cells per axis
 * ((N+1)^3 vertices, spacing h).  The solver S (Sec. 2.2, Eq. (Eqcomp)) is
 * a sequence of V(nu_pre, nu_post)-cycles of red-black Gauss-Seidel with
 * full-weighting restriction (Eq. (rest)), trilinear prolongation
 * I = 2^3 R^T (Sec. 2.3.3), operators rediscretised on every level and an
 * exact solve on the coarsest level (N_c = 2 or 3).  The push-forward
 * (Sec. 2.3) and the pull-back S^dagger (Sec. 2.4, Eq. (EqcompT)) are exposed
 * with respect to q and, extending the paper (Sec. 4 lists it as future
 * work), with respect to log D and log mua as adjoint-state derivatives of
 * the discrete solution.  Also exposed: the two-dimensional 5-point form of
 * the same solver (opt.ndim = 2), the exact derivative of the fixed-cycle
 * map through every step (dmgs_vjp_unrolled), and the response and
 * likelihood epilogue of the reconstruction (Sec. 2.5: dmgs_noise_weights,
 * dmgs_likelihood_grad).
 *
 * Conventions for every entry point:
 *  - Field arrays are DEVICE pointers to dense C-order float64 arrays of
 *    (N+1)^3 entries, x slowest, z fastest: v = (x*(N+1) + y)*(N+1) + z
 *    (plans with ndim = 2: (N+1)^2 entries, v = x*(N+1) + y).
 *    They are owned by the caller and must stay valid until the work enqueued
 *    on `stream` has finished.  Outputs must not alias inputs.
 *  - Boundary vertices (any coordinate 0 or N) of q, mua, tangents and
 *    cotangents are ignored; D is read on all vertices (boundary faces need
 *    it).  Outputs are written on all vertices (boundary: g for rho, 0 for
 *    tangents and gradients except logD_bar, which is defined on all
 *    vertices).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it.  Calls that solve to a tolerance wait for the per-step residual
 *    norms; outputs are complete in stream order (work the call enqueued may
 *    still run when it returns).  With `info` given, every call waits at the
 *    end for all of its work, to fill in the final residual and the device
 *    time.  With fixed_cycles > 0 a solve does not wait otherwise.
 *  - Graph capture: with fixed_cycles > 0, timing off and info == NULL,
 *    dmgs_forward, dmgs_jvp and dmgs_vjp neither wait nor allocate, so a
 *    caller may capture them into a HIP graph on its stream and replay it;
 *    each replay repeats the captured pointers and gives the bits of the
 *    eager calls.  Tolerance-mode solves read residual norms on the host
 *    between cycles and cannot be captured.
 *  - A plan may be used by one host thread and one stream at a time; use
 *    several plans for concurrency.
 *  - Every function returns a dmgs_status; no C++ exception crosses the ABI.
 *    dmgs_last_error() gives a thread-local message for the last failure.
 *    `info` may be NULL.
 */
#ifndef DMGS_H
#define DMGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmgs_plan_s *dmgs_plan;

typedef enum dmgs_status {
    DMGS_OK = 0,
    DMGS_ERR_INVALID = 1,        /* bad options, sizes, coefficients or call order */
    DMGS_ERR_OOM = 2,            /* device allocation failed */
    DMGS_ERR_NOT_CONVERGED = 3,  /* max_cycles reached; outputs hold the last iterate */
    DMGS_ERR_NONFINITE = 4,      /* NaN/Inf in an input or in the residual */
    DMGS_ERR_HIP = 5,            /* a HIP runtime call failed */
    DMGS_ERR_BUDGET = 6          /* request exceeds the memory budget (serving) */
} dmgs_status;

enum dmgs_precision {
    DMGS_FP64 = 0,          /* every step in float64 */
    DMGS_FP32_IN_FP64 = 1   /* float32 V-cycles inside float64 iterative refinement:
                               fine residual, solution update and coarsest solve in float64 */
};
/* DMGS_RBGS: red-black Gauss-Seidel (Sec. 2.2, Sec. 2.3.1).  DMGS_WJACOBI:
 * the alternative smoother, weighted Jacobi, u <- u + w (q - A u) / diag(A)
 * with w = 6/7; its V-cycle is transposed by exchanging nu_pre and nu_post,
 * which the pull-back does. */
enum dmgs_smoother { DMGS_RBGS = 0, DMGS_WJACOBI = 1 };
enum dmgs_face_mean { DMGS_FACE_ARITH = 0, DMGS_FACE_HARMONIC = 1 };

typedef struct dmgs_options {
    int32_t n[3];          /* cells per axis (x, y, z); all three equal, N = c*2^m, c in {2,3}, 2 <= N <= 1024
                              (two-dimensional plans: see ndim).  Three-dimensional plans may also take
                              different counts per axis (a general grid, as the paper's (128, 64, 64)
                              data grid of Sec. 2.5.1): every axis halves from one level to the next
                              until the smallest count is 2 or 3, each count 2..1024, and the coarsest
                              level has at most 64 interior vertices; see h_axis */
    int32_t precision;     /* dmgs_precision */
    int32_t smoother;      /* dmgs_smoother: red-black Gauss-Seidel (Sec. 2.3.1) or weighted Jacobi */
    int32_t nu_pre;        /* pre-smoothing sweeps (red-black pairs), 0..8; default 2 */
    int32_t nu_post;       /* post-smoothing sweeps, 0..8; default 2 */
    int32_t max_cycles;    /* tolerance mode: give up after this many cycles */
    int32_t fixed_cycles;  /* > 0: exactly this many cycles in every solve (Sec. 2.4, second mode) */
    int32_t face_mean;     /* dmgs_face_mean: D on a face = arithmetic or harmonic mean */
    double h;              /* grid spacing (> 0) */
    double bc_value;       /* Dirichlet value g of rho on the boundary */
    double rtol;           /* tolerance mode: stop when ||r||_2 / ||r_0||_2 <= rtol over interior vertices */
    int32_t ir_inner_cycles; /* DMGS_FP32_IN_FP64: float32 V-cycles per refinement step, 1..16 (default 8);
                                with ir_adaptive, the most a step runs */
    int32_t ir_adaptive;   /* DMGS_FP32_IN_FP64, tolerance mode: nonzero (default) = after the first step,
                              run as many V-cycles per step as the contraction factor observed so far
                              predicts the tolerance needs, at most ir_inner_cycles */
    int32_t adjoint_schedule; /* tolerance mode: 0 (default) = a pull-back stops on its own residual;
                                 1 = it repeats exactly the V-cycle schedule of the last dmgs_forward on
                                 this plan (the count recorded in the forward pass; Sec. 2.4), so that
                                 in float64 it is the exact transpose of that forward solve.  Its
                                 accuracy then follows from that count, not from rtol: the adjoint
                                 residual is whatever the forward's schedule reaches on the adjoint
                                 system (reported in info).  In DMGS_FP32_IN_FP64 plans, where the
                                 replay repeats the refinement steps and their float32 V-cycle
                                 counts, the contract is a relative gradient error of at most 1e-7
                                 against the converged adjoint (checked at 64^3; 1e-8 needs
                                 adjoint_schedule = 0) */
    int32_t ndim;          /* 3 (default): (N+1)^3 grids, 7-point operator.  2: (N+1)^2 grids and the
                              5-point operator of the same equation in two dimensions (the paper's
                              benchmark setting, Sec. 3.3), with red = (x + y) even, restriction
                              (1/16)(1,2,1) x (1,2,1) and bilinear prolongation I = 2^2 R^T; n[0] = n[1]
                              = N (n[2] ignored), 2 <= N <= 16384; DMGS_FP64 and DMGS_RBGS only. */
    double h_axis[3];      /* three-dimensional plans: spacing per axis (x, y, z); 0 (default) = h.  Unequal
                              counts in n or unequal spacings make a general-grid plan: the face
                              coefficient of each axis is D_f / h_a^2, on level k with 2^k h_a (Sec. 2.2
                              rediscretised per axis); DMGS_FP64 and DMGS_RBGS only, one operation per
                              launch; every solve, push-forward, pull-back and likelihood entry point
                              takes them (dmgs_forward_vjp runs its two solves one after the other);
                              the diagnostic entry points and dmgs_vjp_unrolled do not. */
} dmgs_options;

typedef struct dmgs_info {
    int32_t cycles;        /* V-cycles (or refinement steps) applied */
    int32_t status;        /* dmgs_status of the call */
    double rel_residual;   /* final ||r|| / ||r_0|| of the solve (adjoint: ||rhobar - A qbar|| / ||rhobar||);
                              float64 red-black plans in tolerance mode form ||r|| after the first cycle
                              in the next cycle's first smoothing pass, where the residual of the colour
                              a cycle updates last is 0 up to rounding and is taken as 0 */
    double device_ms;      /* device time of the call, from events on `stream` */
    int32_t vcycles;       /* V-cycles applied (float32 V-cycles over all refinement steps) */
    int32_t reserved;
} dmgs_info;

/* Fill `opt` with the defaults: V(2,2), RB-GS, FP64, arithmetic face mean,
 * h = 1, g = 0, rtol = 1e-10, max_cycles = 200, fixed_cycles = 0,
 * ir_inner_cycles = 8, ir_adaptive = 1, adjoint_schedule = 0, ndim = 3.  In DMGS_FP32_IN_FP64 plans a
 * "cycle" of max_cycles, fixed_cycles and info.cycles is one refinement
 * step. */
void dmgs_default_options(int32_t n, dmgs_options *opt);

/* Device bytes a plan with these options allocates (hierarchy + scratch); 0
 * for invalid options.  Used for admission by memory footprint. */
size_t dmgs_workspace_bytes(const dmgs_options *opt);

/* Device bytes of a plan that has run dmgs_forward_vjp: dmgs_workspace_bytes
 * plus the second set of work buffers that call allocates; 0 for invalid
 * options. */
size_t dmgs_forward_vjp_workspace_bytes(const dmgs_options *opt);

/* Create a plan: validate options and allocate the level hierarchy on the
 * current device.  Errors: DMGS_ERR_INVALID, DMGS_ERR_OOM, DMGS_ERR_HIP.
 *
 * Tuning knobs.  Plan creation reads these environment variables, which
 * choose which kernel runs on which level and how a launch is cut up; they
 * change no option's meaning, and every choice they allow computes the same
 * operators (the tests force several of them to cover every kernel on every
 * level).  Unset, the tuned defaults apply:
 *   DMGS_SWEEP2_MIN (64 / 16)   smallest N of the two-sweep streaming passes (float32 / float64 plans)
 *   DMGS_SWEEP2_WGS (256)       target workgroups of a finest-level two-sweep pass
 *   DMGS_SWEEP2_WGS_COARSE      ... below the finest level (half of the above)
 *   DMGS_SWEEP2_DEFECT (2)      pre-smoothing pass writes the defect: 0 never, 1 from a zero iterate, 2 always
 *   DMGS_SWEEP2_FP64 (1)        float64 levels with a zero boundary use the two-sweep pass
 *   DMGS_SWEEP_CFG (0)          float32 one-sweep pass tiles: 0 16x64, 1 8x64, 2 16x32
 *   DMGS_FUSE_MIN (32 / 16)     smallest N of the fused passes (float32 / float64 plans)
 *   DMGS_BLOCK_MAX (64)         largest N of the LDS block passes
 *   DMGS_DR_WGS (512 / 1024)    target workgroups of the defect-restriction pass (float32 / float64 plans)
 *   DMGS_2D_SWEEP2_MIN (1536)   two-dimensional plans: smallest N of the two-sweep passes
 *   DMGS_2D_BLOCK_MIN (64)      ... smallest N of the LDS block passes
 *   DMGS_2D_DEFECT (1)          ... the last pre-smoothing pass writes the defect
 *   DMGS_2D_CHUNK (0)           ... rows per chunk of the two-sweep passes (0: from the grid size)
 *   DMGS_2D_SMALL_MAX (32)      ... largest N of the single-workgroup coarse kernel
 *   DMGS_EPI_FUSE (1)           dmgs_likelihood_grad computes its epilogue in the
 *                               forward solve's last refinement step (0: separate pass)
 *   DMGS_PAD (1)                refinement plans pad the rows of the finest level's
 *                               float32 arrays to a multiple of four elements when
 *                               every pass there takes a pitch (even smoothing
 *                               counts, red-black smoothing, N above the block
 *                               passes' range); 0: dense rows.  The footprint
 *                               (dmgs_workspace_bytes) counts the padding.
 *   DMGS_UNROLLED_STORE         dmgs_vjp_unrolled keeps every cycle's recorded states (1)
 *                               or checkpoints and records each cycle again (0); unset:
 *                               keeps them when they take at most a quarter of device memory
 * DMGS_TRACE (0) is not a tuning knob: 1 records residual histories and
 * kernel times (dmgs_trace_read). */
int dmgs_plan_create(const dmgs_options *opt, dmgs_plan *out);
int dmgs_plan_destroy(dmgs_plan plan);

/* Number of levels and cells per axis on level k (k = 0 finest); for a
 * general grid dmgs_plan_level_n gives the x count.  dmgs_plan_level_shape
 * writes the cells of level k per axis (x, y, z; a two-dimensional plan
 * writes N, N, 0) to n3 and returns DMGS_OK, or DMGS_ERR_INVALID for a NULL
 * plan or pointer or a level out of range. */
int dmgs_plan_levels(dmgs_plan plan);
int dmgs_plan_level_n(dmgs_plan plan, int k);
int dmgs_plan_level_shape(dmgs_plan plan, int k, int32_t *n3);

/* Coefficient set-up (Sec. 2.2: operators rediscretised on every level):
 * copy D and mua, check D > 0, mua >= 0 (interior) and finiteness
 * (DMGS_ERR_INVALID otherwise; this check waits for the stream), and build
 * the coarse levels by full weighting on coarse interior vertices and
 * injection on coarse boundary vertices.  The log variant takes log D and
 * log mua and exponentiates on the device.  Must precede any solve. */
int dmgs_set_coefficients(dmgs_plan plan, const double *D, const double *mua, void *stream);
int dmgs_set_log_coefficients(dmgs_plan plan, const double *logD, const double *logmua, void *stream);

/* Forward solve rho = S(q) (Sec. 2.2, Sec. 2.4). */
int dmgs_forward(dmgs_plan plan, const double *q, double *rho, dmgs_info *info, void *stream);

/* Push-forward: drho = S(dq - dA rho) with homogeneous boundary, where dA is
 * the derivative of the operator along (dlogD, dlogmua) (Sec. 2.3: in q the
 * Jacobian of S is S itself).  rho must be the forward solution for the
 * current coefficients.  Any tangent may be NULL (= zero). */
int dmgs_jvp(dmgs_plan plan, const double *rho, const double *dq, const double *dlogD,
             const double *dlogmua, double *drho, dmgs_info *info, void *stream);

/* Pull-back (Sec. 2.4, Eq. (EqcompT)): qbar = S^dagger rhobar, computed as
 * the transposed V-cycles (each cycle's steps reversed and transposed, which
 * is a V-cycle with black half-sweeps before red ones), then
 *   logmua_bar = -mua * qbar * rho                      (interior, 0 on boundary)
 *   logD_bar_v = -sum_{faces f=(a,b) at v} dD_f/dlogD_v (qbar_a - qbar_b)(rho_a - rho_b) / h^2
 * with qbar = 0 and rho = g on boundary vertices.  logD_bar / logmua_bar may
 * be NULL (not computed).  Tolerance mode stops on ||rhobar - A qbar|| /
 * ||rhobar|| <= rtol; fixed mode applies exactly fixed_cycles cycles, making
 * the result the exact transpose of the fixed-cycle forward map.  With
 * opt.adjoint_schedule the pull-back instead repeats the schedule of the last
 * dmgs_forward (or dmgs_forward_vjp) on the plan, cycle for cycle (float64)
 * or float32 V-cycles per refinement step (float32-in-float64), so that in
 * float64 it is the exact transpose of that forward solve; DMGS_ERR_INVALID
 * if no forward solve has run on the plan. */
int dmgs_vjp(dmgs_plan plan, const double *rho, const double *rhobar, double *qbar,
             double *logD_bar, double *logmua_bar, dmgs_info *info, void *stream);

/* Forward solve and VJP of one sample together: rho = S q (as
 * dmgs_forward) and qbar = S^dagger rhobar with the coefficient gradients (as
 * dmgs_vjp, evaluated at this rho).  The adjoint solve does not depend on
 * rho (Sec. 2.4: S^dagger is a solve with the transposed cycle), so the two
 * solves run concurrently: the adjoint one on a second stream of the plan,
 * driven from a second host thread, ordered after the work already on
 * `stream`; `stream` waits for it before the gradient pass.  The first call
 * allocates the second set of work buffers (dmgs_workspace_bytes does not
 * count them; dmgs_forward_vjp_workspace_bytes does).  rho, qbar, logD_bar and logmua_bar must not alias each other
 * or the inputs; logD_bar / logmua_bar may be NULL.  info_fwd and info_vjp
 * describe the two solves (either may be NULL); the returned status is the
 * forward solve's, else the adjoint's.  With opt.adjoint_schedule the adjoint
 * solve repeats this call's forward schedule, so it is enqueued (still on the
 * second stream) only after the forward solve has finished on the host. */
int dmgs_forward_vjp(dmgs_plan plan, const double *q, const double *rhobar, double *rho, double *qbar,
                     double *logD_bar, double *logmua_bar, dmgs_info *info_fwd, dmgs_info *info_vjp, void *stream);

/* ---------------------------------------------------------------------------
 * Response and likelihood epilogue of the reconstruction (Sec. 2.5).  The
 * response to a source q is the absorbed energy density L_e = mua rho with
 * rho = S q (the paper's lambda is mua), compared with data d on the voxels
 * the mask keeps, under Gaussian noise with diagonal covariance.
 * ------------------------------------------------------------------------- */

/* Inverse noise variances of the noise model (Sec. 2.5.1, Eq. (noise)):
 * sigma_i = max(rel * Le_i, floor_frac * max_j Le_j) (the paper: rel = 0.05,
 * floor_frac = 0.01, max over all vertices of Le), w_i = 1 / sigma_i^2 on
 * vertices at least `mask` (>= 1) vertices from every face, 0 on the others
 * and where sigma_i <= 0 (the paper masks 0.2 cm at every edge).  Le and w
 * are finest-level device arrays of the plan; enqueued on `stream`, no
 * wait.  Errors: DMGS_ERR_INVALID (NULL, mask < 1, negative or non-finite
 * rel / floor_frac). */
int dmgs_noise_weights(dmgs_plan plan, const double *Le, int32_t mask, double rel, double floor_frac, double *w,
                       void *stream);

/* Negative log-likelihood of data d and its gradient for one source q
 * (Sec. 2.5.2 Eq. (response), Sec. 2.5.4 Eq. (likelihood) and Eq. (chi2)):
 *   rho = S q                                  (as dmgs_forward)
 *   H = 1/2 sum_i w_i (d_i - mua_i rho_i)^2    over interior vertices
 *   value[0] = H, value[1] = chi2 = 2 H / N_vox, value[2] = N_vox (number of
 *   interior vertices with w_i > 0), written to HOST memory
 *   qbar = dH/dq = S^dagger rhobar with rhobar_i = mua_i w_i (mua_i rho_i - d_i)
 *   logD_bar = dH/dlogD and logmua_bar = dH/dlogmua: the pull-back's
 *   coefficient gradients at rho (as dmgs_vjp) plus, for log mua, the direct
 *   term w_i (mua_i rho_i - d_i) mua_i rho_i of L_e.
 * w holds the inverse noise variances with the mask applied (0 = not compared;
 * e.g. from dmgs_noise_weights); boundary entries of d and w are ignored.
 * The pull-back follows opt.adjoint_schedule as dmgs_vjp does.  rho, qbar,
 * logD_bar, logmua_bar must not alias each other or the inputs; logD_bar /
 * logmua_bar may be NULL.  The call waits for the work it enqueued (value is
 * ready on return).  info_fwd / info_vjp describe the two solves (either may
 * be NULL); the status is the forward solve's, else the adjoint's.
 * The epilogue (L_e, the sums of H and N_vox, rhobar) is computed in the
 * forward solve's last pass over rho where one exists: a refining plan's
 * last refinement step, a general grid's last half-sweep, a float64 cubic
 * plan's last residual pass (in fixed-cycle mode only when info_fwd is
 * given); in tolerance mode that is the step the observed contraction
 * predicts to be the last.  Otherwise, and on two-dimensional plans, it is
 * a separate pass over rho; both give the same values (the sums up to
 * rounding order). */
int dmgs_likelihood_grad(dmgs_plan plan, const double *q, const double *d, const double *w, double *rho,
                         double *qbar, double *logD_bar, double *logmua_bar, double *value, dmgs_info *info_fwd,
                         dmgs_info *info_vjp, void *stream);

/* Unrolled adjoint of the fixed-cycle solver: the exact derivative of
 * rho = S_n(q; log D, log mua), n = opt.fixed_cycles V(nu_pre, nu_post)-cycles
 * from rho = 0 (interior) / g (boundary), through every step of every cycle
 * -- smoothing, defect, restriction, prolongation, the coarsest solve and the
 * coarse coefficients built from log D and log mua (Sec. 2.2 Eq. (Eqcomp)
 * reversed as in Sec. 2.4 Eq. (EqcompT), with the coefficients as inputs of
 * every step).  Writes rho = S_n q and the pull-back of rhobar: qbar (equal
 * to dmgs_vjp's in fixed mode up to rounding), logD_bar and logmua_bar (the
 * derivative of the n-cycle map itself, which differs from dmgs_vjp's
 * adjoint-state gradients of the exact discrete solution by the iteration
 * error; logD_bar / logmua_bar may be NULL).  The forward pass records the
 * states of every cycle (after each half-sweep, on every level) when they
 * take at most a quarter of the device's memory, about 1.14 n (2 (nu_pre +
 * nu_post) + 1) finest-level fields (21 GB at N = 256, n = 15, V(2,2));
 * otherwise it keeps the finest iterate at the start of every cycle (n
 * fields) and records each cycle again before its reverse pass (the
 * environment variable DMGS_UNROLLED_STORE = 1 / 0 forces either; both
 * give the same results up to rounding).  The first call on a plan
 * allocates these buffers and about 1.14 x 8 finest-level fields of work
 * buffers; the plan keeps them for later calls and dmgs_plan_destroy frees
 * them.  The call waits for its work
 * before it returns.  Three-dimensional
 * DMGS_FP64, DMGS_RBGS plans with fixed_cycles > 0 only, else
 * DMGS_ERR_INVALID; DMGS_ERR_OOM if the work buffers do not fit. */
int dmgs_vjp_unrolled(dmgs_plan plan, const double *q, const double *rhobar, double *rho, double *qbar,
                      double *logD_bar, double *logmua_bar, dmgs_info *info, void *stream);

/* One-shot convenience: create, set coefficients, forward, destroy. */
int dmgs_solve_once(const dmgs_options *opt, const double *D, const double *mua, const double *q,
                    double *rho, dmgs_info *info, void *stream);

/* Bytes of the library's static device scratch array (one copy per device,
 * held until the process ends) that dmgs_solve_once_noalloc works in. */
#define DMGS_NOALLOC_SCRATCH_BYTES ((size_t)144 << 20)

/* dmgs_solve_once without any allocation, for callers that cannot allocate
 * device memory (code running between allocation-free points of a serving
 * loop, harnesses that forbid hipMalloc).  Same arguments, layout, result and
 * errors as dmgs_solve_once; the caller passes the inputs and the output.
 * The plan's hierarchy and work buffers are carved from a static device
 * array of DMGS_NOALLOC_SCRATCH_BYTES (144 MiB: 3D grids up to N = 128 in
 * both precisions, 2D grids up to N = 1536); a plan needing more than that
 * (dmgs_workspace_bytes(opt) + 64 KiB for alignment) is rejected with
 * DMGS_ERR_INVALID before any device work.  The call makes no hipMalloc,
 * hipFree, pinned-host or event allocation: norms and the validation flag
 * are copied to host variables and waited for by synchronising the stream.
 * All calls on one device share that device's array, which keeps the last
 * call's contents (each call clears what must start at zero).  The library
 * serialises calls on one device with a host lock and each call returns
 * with its work complete, so calls never overlap on the array; work of
 * other library calls is unaffected.  info->device_ms is 0 (no events).
 * Devices 0..15 only. */
int dmgs_solve_once_noalloc(const dmgs_options *opt, const double *D, const double *mua, const double *q,
                            double *rho, dmgs_info *info, void *stream);

/* ---------------------------------------------------------------------------
 * Grouped execution (continuous batching).  A sampling loop over the
 * posterior (Sec. 2.1, Sec. 2.5.4) asks for many forward solves, each followed
 * by a push-forward (Sec. 2.3) or a pull-back (Sec. 2.4, Eq. (EqcompT)), on grids of
 * several sizes.  A batch advances all its requests together.  Each
 * dmgs_batch_tick runs one refinement step for every active request, with the
 * kernels of all requests merged into grouped launches (one launch serves
 * the same pass of several requests, each on its own arrays), and
 * synchronises the stream once.  Requests may be added between ticks.  A
 * request's arithmetic does not depend on the batch: its results, cycle
 * counts and residuals are bitwise those of dmgs_forward followed by
 * dmgs_jvp or dmgs_vjp on its plan.
 *
 * Plans: DMGS_FP32_IN_FP64, cubic 3D, V(2,2) red-black cycles (nu_pre =
 * nu_post = 2), adjoint_schedule 0, coefficients set, and every level above
 * the single-workgroup coarse end (N <= 16) run by the block passes (16 < N
 * <= 64) or the two-sweep passes (N >= 64): in practice N >= 24 with the
 * default tuning knobs.  A plan serves at most one
 * request of a batch at a time and must not be used by other calls while it
 * does.  Its coefficient set-up must be ordered before the ticks (the same
 * stream, or a synchronisation).
 * ------------------------------------------------------------------------- */
/* A batch is driven by one host thread at a time. */
typedef struct dmgs_batch_s *dmgs_batch;

enum { DMGS_BATCH_JVP = 0, DMGS_BATCH_VJP = 1 };

/* Create an empty batch on the current device.  Errors: DMGS_ERR_INVALID,
 * DMGS_ERR_OOM, DMGS_ERR_HIP. */
int dmgs_batch_create(dmgs_batch *out);
/* Destroy a batch; requests not yet reported are dropped (no device work of
 * the batch is pending between ticks).  The plans are the caller's. */
int dmgs_batch_destroy(dmgs_batch batch);
/* Add a request (device arrays of (N+1)^3 float64, owned by the caller and
 * untouched by it until the request is reported):
 *   DMGS_BATCH_JVP: rho = S q, then out0 = drho = S (dq - A' rho) with
 *                   in0 = dq, in1 = dlogD, in2 = dlogmua (each may be NULL);
 *   DMGS_BATCH_VJP: rho = S q, then out0 = qbar = S^T rhobar with in0 =
 *                   rhobar, and out1 = logD_bar, out2 = logmua_bar (each may
 *                   be NULL).
 * tag is returned with the request's results.  Errors: DMGS_ERR_INVALID (an
 * ineligible plan, a plan already serving a request of the batch, NULL
 * arrays), DMGS_ERR_OOM. */
int dmgs_batch_add(dmgs_batch batch, dmgs_plan plan, int32_t mode, const double *q, const double *in0,
                   const double *in1, const double *in2, double *rho, double *out0, double *out1, double *out2,
                   int64_t tag);
/* Requests added and not yet reported. */
int dmgs_batch_pending(dmgs_batch batch);
/* One tick on `stream`: one refinement step for every active request (a new
 * request's first tick forms its initial residual), in grouped launches,
 * then one synchronisation of the stream.  Up to `cap` requests that
 * finished are reported: tags[i], status[i] (DMGS_OK, or the status that
 * ended the request: a forward solve that fails ends it), and the forward
 * and second solve's infos (info_fwd, info_second may be NULL; a skipped
 * second solve reports zeros).  *count = number reported; later finishers wait
 * for the next tick.  Returns DMGS_OK unless the tick itself failed (then the
 * batch should be destroyed). */
int dmgs_batch_tick(dmgs_batch batch, void *stream, int32_t cap, int64_t *tags, int32_t *status,
                    dmgs_info *info_fwd, dmgs_info *info_second, int32_t *count);
/* Ticks run, grouped launches issued, and the single-request launches they
 * replaced, since the batch was created. */
int dmgs_batch_stats(dmgs_batch batch, int64_t *ticks, int64_t *launches, int64_t *recorded);

const char *dmgs_status_string(int status);
const char *dmgs_last_error(void);

/* ---------------------------------------------------------------------------
 * Kernel timing (profiling aid).  dmgs_timing_enable(plan, n): n = 0 off;
 * n >= 1: one launch in n of each kernel class on the finest level (every
 * launch for n = 1) is bracketed by HIP events on the stream it is launched
 * on; elapsed times are collected at the plan's synchronisation points and
 * at the end of every call.  Each record also carries the algorithmic bytes
 * of the launch (every input read once, every output written once).
 * dmgs_timing_read returns the number of finest-level launches of the class
 * and its time and bytes scaled from the timed launches to all of them.
 * Enabling resets the counters.  Work of the second stream of
 * dmgs_forward_vjp is not timed.
 * ------------------------------------------------------------------------- */
enum dmgs_kernel_class {
    DMGS_K_SMOOTH = 0,           /* smoothing pass (red-black sweeps)                 */
    DMGS_K_DEFECT_RESTRICT = 1,  /* defect and full-weighting restriction             */
    DMGS_K_PROLONG = 2,          /* prolongation and correction                        */
    DMGS_K_RESIDUAL = 3,         /* float64 residual (norm; refinement cast)          */
    DMGS_K_UPDATE = 4,           /* refinement update u += e                           */
    DMGS_K_COEF = 5,             /* coefficient set-up and hierarchy build             */
    DMGS_K_GRAD = 6,             /* tangent right-hand side and coefficient gradients  */
    DMGS_K_COUNT = 7
};
int dmgs_timing_enable(dmgs_plan plan, int enable);

/* Residual history (tracing aid).  With DMGS_TRACE=1
 * in the environment when the plan is created, every solve records the
 * relative residual ||b - A u|| / ||b - A u_0|| of the iterate after each
 * V-cycle (float64 plans) or refinement step (DMGS_FP32_IN_FP64), and the
 * plan times every finest-level launch (dmgs_timing_read; as
 * dmgs_timing_enable(plan, 1)).  In tolerance mode the history costs
 * nothing extra; in fixed-cycle mode it adds one residual pass and one host
 * wait per cycle.  order 0: the last forward or push-forward solve
 * (dmgs_likelihood_grad: its forward solve); 1: the last pull-back.  Writes
 * up to cap entries (cycles or steps applied so far, V-cycles applied so
 * far, relative residual) to steps, vcycles, rel (host arrays) and the
 * number of entries to *count.  Float64 tolerance mode records each
 * iterate's residual when the next cycle's first pass has formed it, so the
 * last entry is the returned iterate's.  Errors: DMGS_ERR_INVALID (NULL,
 * order not 0 or 1, negative cap, tracing off). */
int dmgs_trace_read(dmgs_plan plan, int32_t order, int32_t cap, int32_t *steps, int32_t *vcycles, double *rel,
                    int32_t *count);
int dmgs_timing_read(dmgs_plan plan, int kernel_class, int64_t *launches, double *total_ms,
                     double *algorithmic_bytes);

/* ---------------------------------------------------------------------------
 * Diagnostic entry points: each runs one pass of the cycle on level k of a
 * plan whose coefficients are set, on caller device arrays of level k's size
 * ((N_k+1)^3, or (N_{k+1}+1)^3 for coarse arrays).  `fp32` selects the
 * float32 instantiation used inside iterative refinement (arrays are then
 * float32, coefficients the plan's float32 copies).  order 0 = red half-sweep
 * first (forward), 1 = black first (transposed cycle).  Used by the parity
 * tests; not needed to solve.  When the float32 arrays of level k have padded
 * rows (DMGS_PAD), dmgs_debug_pre and dmgs_debug_post copy the caller's
 * arrays into the level's own work buffers, run the pass there and copy the
 * result out (the work buffers' contents are overwritten).
 * ------------------------------------------------------------------------- */

/* out = A_k u on interior vertices, 0 on the boundary. */
int dmgs_debug_apply(dmgs_plan plan, int k, int fp32, const void *u, void *out, void *stream);
/* Copy level k's coefficient fields (float64) into caller arrays. */
int dmgs_debug_level_coefficients(dmgs_plan plan, int k, double *D, double *mua, void *stream);
/* Pre-smoothing pass: u_out = nu_pre red-black sweeps applied to u_in with
 * right-hand side q (Sec. 2.3.1), then qc = R (q - A_k u_out) on the coarse
 * interior (Eq. (defect), Eq. (rest)), 0 on the coarse boundary.  u_in NULL:
 * start from the zero iterate with a zero boundary (a coarse-level pass). */
int dmgs_debug_pre(dmgs_plan plan, int k, int fp32, int order, const void *u_in, const void *q,
                   void *u_out, void *qc, void *stream);
/* Post-smoothing pass: u_out = nu_post sweeps applied to u_in + I ec
 * (Sec. 2.3.3). */
int dmgs_debug_post(dmgs_plan plan, int k, int fp32, int order, const void *u_in, const void *ec,
                    const void *q, void *u_out, void *stream);
/* Exact solve on the coarsest level: u = A_c^{-1} q (boundary of u = 0). */
int dmgs_debug_coarsest(dmgs_plan plan, int fp32, const void *q, void *u, void *stream);
/* Plain streaming copy of `bytes` (a multiple of 16) from src to dst, both
 * device pointers: a kernel of known traffic, to calibrate memory counters. */
int dmgs_debug_stream_copy(const void *src, void *dst, size_t bytes, void *stream);
/* Exactly ncycles V-cycles applied to u (float64, in place) with right-hand
 * side q, from whatever u holds (its boundary entries are the Dirichlet values). */
int dmgs_debug_cycles(dmgs_plan plan, int order, int ncycles, const double *q, double *u, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DMGS_H */
