/*
 * fwi.h - C ABI of the MI355X (gfx950) library for the hot path of GPR
 * dual-parameter full-waveform inversion: 2D TM-mode FDTD forward modelling
 * in lossy media with a CPML absorbing boundary, its exact discrete adjoint,
 * and the zero-lag cross-correlation gradients with respect to relative
 * permittivity eps_r and conductivity sigma.
 *
 * Paper: "Fast ground penetrating radar dual-parameter full waveform
 * inversion method accelerated by hybrid compilation of CUDA kernel
 * function and PyTorch", arXiv 2506.20513.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Total grid NX = nx + 2 npml by NY = ny + 2 npml cells: the interior of
 *   nx x ny cells padded by npml CPML cells on every side.  x (index i) is
 *   horizontal, y (index j) is depth.  2D arrays are row-major [NY][NX]
 *   with i contiguous, 32-bit IEEE float unless stated.
 * - Fields: Ez on cell nodes (i, j), Hx at (i, j+1/2), Hy at (i+1/2, j),
 *   leapfrogged as in Sec. 2.1, Eqs. (3)-(5), with the semi-implicit loss
 *   coefficients of the coefficient kernel in Sec. 3.2:
 *     EA = eps0 eps_r / dt + sigma / 2,  EB = eps0 eps_r / dt - sigma / 2,
 *     Ez <- (EB/EA) Ez + (1/EA) curl H,  sigma > 100 S/m => perfect conductor.
 *   The outermost ring of Ez cells is a PEC wall held at zero.
 *   mu = mu0 = 4 pi 1e-7 H/m, eps0 = 1/(mu0 c0^2), c0 = 299792458 m/s.
 * - One Hertzian line source per shot (z polarised, Sec. 3.2 dipole
 *   kernel): after the E update of step n,
 *     Ez(src) -= (1/EA(src)) * wavelet[n] / (dx dy),
 *   i.e. the wavelet is a line current in A sampled at t = (n + 1/2) dt.
 * - Receivers record Ez^n before step n updates anything (Algorithm 1,
 *   stage 1): traces[s][n][r] = Ez^n(rec_r), so traces[s][0][r] = 0.
 * - Misfit J = 1/2 sum_{s,n,r} (traces - observed)^2 (Eq. (6)).
 * - Gradients (Eqs. (12)-(13), discrete and exact for this scheme):
 *     dJ/d eps_r = -eps0/(dt EA) sum_n lambda^{n+1} (Ez^{n+1} - Ez^n)
 *     dJ/d sigma = -1/(2 EA)     sum_n lambda^{n+1} (Ez^{n+1} + Ez^n)
 *   summed over shots in a fixed order; lambda is the exact discrete
 *   adjoint state (Algorithm 2; terminal condition Eq. (10)).  Cells on
 *   the PEC ring and perfect-conductor cells get zero.  The gradient covers
 *   the whole total grid, CPML cells included, and is not masked.
 * - CPML (the paper names a PML but not its formulation): convolutional
 *   PML with polynomial grading, normalised depth rho from the interior
 *   edge (E nodes at integer, H nodes at half-integer positions),
 *     sigma_p = cpml_sigma_scale * 0.8 (m+1) / (eta0 d) * rho^m,
 *     kappa = 1 + (cpml_kappa_max - 1) rho^m,  alpha = cpml_alpha_max (1 - rho),
 *     b = exp(-(sigma_p/kappa + alpha) dt / eps0),
 *     a = sigma_p (b - 1) / (kappa (sigma_p + kappa alpha)).
 *   Profiles are computed in double precision and stored as float.
 *
 * Memory and ownership
 * --------------------
 * - Pointers documented "device" are HIP device pointers owned by the
 *   caller; "host" pointers are ordinary host memory read during the call.
 * - The library allocates nothing.  All scratch state lives in the
 *   caller-supplied device workspace `ws` of `ws_bytes` bytes (size from
 *   fwi_workspace_bytes; 256-byte alignment required).  The one exception
 *   is fwi_gradient_static, whose workspace is a static device array of the
 *   library (see there).
 * - Every call runs on `stream` (a hipStream_t; NULL = the null stream).
 *   A gradient call that splits its shots into groups (fwi_gradient_ex)
 *   also creates a non-blocking stream for every group but the first (which
 *   runs on `stream`) and a few events, joins them to `stream` and destroys
 *   them before it returns.
 *   Host arrays may be reused as soon as the call returns.  The forward,
 *   adjoint and gradient calls return once the stream has finished them
 *   (see Errors); the batched runs are asynchronous, and their device
 *   outputs are valid once the stream reaches the end of the run.
 * - Apart from that static array, the library keeps no global mutable
 *   state.  Calls on different workspaces may run concurrently; calls
 *   sharing a workspace must be ordered on one stream.
 *
 * Errors
 * ------
 * Every entry point returns FWI_OK or a negative status.  All argument
 * checks run on the host before any HIP call, so an invalid call launches
 * nothing and leaves every output untouched.
 *
 * fdtd_forward, fdtd_adjoint and fwi_gradient (and its timed and static
 * variants) end with a finiteness check of what they wrote: FP64 sums of
 * squares of the traces (forward) or of both gradients (adjoint, gradient),
 * and the misfit (gradient).  They wait for `stream` to reach that check
 * and return FWI_ENONFINITE if any of those values holds a NaN or an
 * infinity, for instance from a NaN in the observed data or the model.  The
 * outputs are written all the same.  These calls therefore return with the
 * stream drained; the batched plans (below) run asynchronously and do not
 * check.
 */
#ifndef FWI_H
#define FWI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWI_OK 0
#define FWI_EINVAL (-1)      /* null pointer, bad size or parameter          */
#define FWI_ECFL (-2)        /* dt above the stability bound, Eq. (11), c=c0 */
#define FWI_EGEOM (-3)       /* source/receiver outside the updated interior */
#define FWI_ENOMEM (-4)      /* workspace missing, misaligned or too small   */
#define FWI_EHIP (-5)        /* a HIP runtime call or kernel launch failed   */
#define FWI_ENONFINITE (-6)  /* the call ran to the end, but its outputs hold
                                a NaN or an infinity (see Errors above)      */
#define FWI_ESCRATCH (-7)    /* problem larger than fwi_gradient_static's
                                static scratch (FWI_STATIC_SCRATCH_BYTES)   */

/* How fdtd_forward keeps the forward field for a later fdtd_adjoint. */
#define FWI_SAVE_NONE 0        /* traces only                               */
#define FWI_SAVE_CHECKPOINT 1  /* full state every K steps; the adjoint
                                  re-runs each K-step segment forward.  K is
                                  chosen from the shape to minimise memory
                                  (about sqrt(3 nt)); results are identical
                                  to FWI_SAVE_HISTORY bit for bit.          */
#define FWI_SAVE_HISTORY 2     /* Ez at every step (small problems only)    */

/* Grid, time axis and CPML parameters (all host values). */
/* The total grid is NX = nx + 2 npml by NY = ny + 2 npml cells; each of NX
 * and NY is 3 .. 2^20 and NY * round_up(NX, 64) below 2^30 cells, else
 * FWI_EINVAL. */
typedef struct fwi_grid {
    int32_t nx, ny;            /* interior cells, x (horizontal) and y (depth) */
    int32_t npml;              /* CPML cells on each side, >= 0                */
    int32_t nt;                /* time steps, >= 1                             */
    double dx, dy, dt;         /* cell sizes (m) and time step (s)             */
    int32_t cpml_order;        /* grading exponent m, 1..16 (default 3)        */
    double cpml_sigma_scale;   /* >= 0 (default 1)                             */
    double cpml_kappa_max;     /* >= 1 (default 1)                             */
    double cpml_alpha_max;     /* >= 0, S/m (default pi f0 eps0)              */
} fwi_grid;

/* Acquisition geometry: one source and nrec receivers per shot. */
typedef struct fwi_geom {
    int32_t nshots;            /* >= 1                                        */
    int32_t nrec;              /* receivers per shot, >= 1                    */
    const int32_t *src_ij;     /* host [nshots][2] = (i, j) on the total grid */
    const int32_t *rec_ij;     /* host [nshots][nrec][2]                      */
    const float *wavelet;      /* device [nshots][nt] line current (A)        */
} fwi_geom;
/* Source and receiver cells must lie in the interior (npml <= i <= NX-1-npml,
 * same for j) and off the PEC ring (1 <= i <= NX-2, 1 <= j <= NY-2), else
 * FWI_EGEOM.  Several receivers of one shot may share a cell. */

/* Workspace size for fdtd_forward / fdtd_adjoint with `save_mode`
 * (FWI_SAVE_*), or for fwi_gradient when save_mode = -1.
 * bytes: host out.  Returns FWI_EINVAL / FWI_ECFL / FWI_EGEOM as the entry
 * points would for the same grid and geometry. */
int fwi_workspace_bytes(const fwi_grid *grid, const fwi_geom *geom,
                        int save_mode, size_t *bytes);

/* Forward modelling, Algorithm 1 (Sec. 3.3), all shots in one sweep.
 *   eps_r, sigma: device [NY][NX] model on the total grid (eps_r >= 1).
 *   traces: device out [nshots][nt][nrec].
 *   save_mode: FWI_SAVE_NONE, FWI_SAVE_CHECKPOINT or FWI_SAVE_HISTORY; with
 *   the latter two the workspace afterwards holds what fdtd_adjoint needs. */
int fdtd_forward(const fwi_grid *grid, const fwi_geom *geom,
                 const float *eps_r, const float *sigma, float *traces,
                 int save_mode, void *ws, size_t ws_bytes, void *stream);

/* Adjoint modelling and gradient imaging, Algorithm 2 (Sec. 3.3).
 *   Must follow fdtd_forward on the same workspace with the same grid,
 *   geometry, model and save_mode (FWI_SAVE_CHECKPOINT or _HISTORY);
 *   otherwise the results are undefined.
 *   residual: device [nshots][nt][nrec], the adjoint source dJ/d traces.
 *   grad_eps_r, grad_sigma: device out [NY][NX], overwritten.
 *   src_adjoint: device out [nshots][nt] or NULL; the derivative of
 *   <traces, residual> with respect to the wavelet (for dot-product tests):
 *     src_adjoint[s][n] = -(1/EA(src)) lambda_E^{n+1}(src) / (dx dy). */
int fdtd_adjoint(const fwi_grid *grid, const fwi_geom *geom,
                 const float *eps_r, const float *sigma,
                 const float *residual, float *grad_eps_r, float *grad_sigma,
                 float *src_adjoint, int save_mode, void *ws, size_t ws_bytes,
                 void *stream);

/* One full gradient evaluation: forward with checkpoints, residual and
 * misfit, adjoint and imaging.
 *   observed: device [nshots][nt][nrec].
 *   misfit: device out, one double, J = 1/2 sum r^2 (double accumulation).
 *   grad_eps_r, grad_sigma: device out [NY][NX].
 *   traces_out: device out [nshots][nt][nrec] or NULL.
 *   Workspace size: fwi_workspace_bytes(..., -1, ...). */
int fwi_gradient(const fwi_grid *grid, const fwi_geom *geom,
                 const float *eps_r, const float *sigma,
                 const float *observed, double *misfit, float *grad_eps_r,
                 float *grad_sigma, float *traces_out, void *ws,
                 size_t ws_bytes, void *stream);

/* Per-kernel timing for roofline accounting.  The paper reports only whole
 * epoch wall times (Sec. 4, Tables 2-5); this records HIP events on `stream`
 * around every `sample_every`-th launch of each hot kernel of one
 * fwi_gradient call and reports their mean durations.  Three kinds:
 * "k_fwd_sweep" (forward passes that keep only the final state),
 * "k_fwd_reforward" (the segment re-forward, which also writes Ez of every
 * step) and "k_adj" (adjoint and imaging). */
#define FWI_TIMING_MAX_KINDS 8
typedef struct fwi_kernel_time {
    char name[32];             /* kernel name as it appears in profiler traces */
    int32_t launches;          /* launches of this kernel during the call     */
    int32_t timed;             /* launches bracketed by events                */
    double avg_ms;             /* mean duration of the timed launches         */
    double cell_updates;       /* cells x shots x time steps these launches
                                  computed (cells each wave owns; halos and
                                  recomputation not counted)                  */
} fwi_kernel_time;
typedef struct fwi_timing {
    int32_t sample_every;      /* in: >= 1                                   */
    int32_t nkinds;            /* out: entries filled in `kind`               */
    fwi_kernel_time kind[FWI_TIMING_MAX_KINDS];
    int32_t shot_groups;       /* out: shot groups the call ran in (each
                                  launch covers one group's shots)           */
} fwi_timing;

/* fwi_gradient with per-kernel timing.  timing: host in/out, or NULL (then
 * identical to fwi_gradient).  With timing, the call synchronises `stream`
 * before returning; FWI_EINVAL if sample_every < 1. */
int fwi_gradient_timed(const fwi_grid *grid, const fwi_geom *geom,
                       const float *eps_r, const float *sigma,
                       const float *observed, double *misfit, float *grad_eps_r,
                       float *grad_sigma, float *traces_out, void *ws,
                       size_t ws_bytes, void *stream, fwi_timing *timing);

/* fwi_gradient (with optional timing) whose shots run in shot_groups groups
 * of consecutive shots, each group's forward and adjoint passes on a stream
 * of its own, so that the groups' launches overlap on the GPU.  The
 * coefficient setup, the residual and misfit of all shots and the final
 * gradient (a sum over all shots in shot order) run on `stream` between
 * the groups' phases, so the results are identical bit for bit for every
 * group count.  shot_groups: 0 = automatic (with 16 or more shots one group
 * per 6 shots, at most 4: the 64-shot 2088 x 1064 gradient measured 14%
 * faster in 4 groups than in one, the 24-shot 552 x 296 one 16% faster;
 * 1 group below 16 shots), 1 .. 4 = that many (at most nshots).  Group 0
 * runs on `stream`, the others on streams the call creates, so four groups
 * fit the runtime's default of four hardware queues per process.
 * fwi_workspace_bytes(..., -1, ...) covers every
 * group count.  With timing, each kind's launches of all groups are
 * counted and timed; their durations include the other groups' launches
 * running beside them.  FWI_EINVAL if shot_groups is outside 0 .. 4.
 * fwi_gradient and fwi_gradient_timed are this call with shot_groups = 0. */
int fwi_gradient_ex(const fwi_grid *grid, const fwi_geom *geom,
                    const float *eps_r, const float *sigma,
                    const float *observed, double *misfit, float *grad_eps_r,
                    float *grad_sigma, float *traces_out, void *ws,
                    size_t ws_bytes, void *stream, fwi_timing *timing,
                    int32_t shot_groups);

/* ---- Allocation-free gradient -------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as fwi_gradient, with its workspace taken from a static device
 * array of FWI_STATIC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends.  The caller still passes inputs and
 * outputs (device pointers as for fwi_gradient).  Problems whose
 * fwi_workspace_bytes(..., -1, ...) exceeds the array get FWI_ESCRATCH; that
 * check, like every argument check, runs on the host before any HIP call.
 * The call allocates nothing.  The array is resolved for the current device
 * on the first call made with it current; `stream` must belong to that
 * device.  All calls on one device share its array: calls that overlap in
 * time on one device race and must be ordered by the caller (one stream, or
 * events).  Results equal fwi_gradient's bit for bit.  Like fwi_gradient,
 * the call synchronises `stream` once while it uploads the geometry.  It
 * runs all shots as one group (fwi_gradient_ex with shot_groups = 1), so it
 * creates no streams or events. */
#define FWI_STATIC_SCRATCH_BYTES (64u << 20)
int fwi_gradient_static(const fwi_grid *grid, const fwi_geom *geom,
                        const float *eps_r, const float *sigma,
                        const float *observed, double *misfit, float *grad_eps_r,
                        float *grad_sigma, float *traces_out, void *stream);

/* Checkpoint interval K that FWI_SAVE_CHECKPOINT uses for this shape
 * (host out `k`). */
int fwi_checkpoint_interval(const fwi_grid *grid, const fwi_geom *geom,
                            int32_t *k);

/* Static text for a status code. */
const char *fwi_strerror(int status);

/* ---- Batched gradients of independent problems ----------------------------
 * fwi_gradient for many independent problems at once (Secs. 2.1, 3.3): each
 * problem has its own grid, model, geometry, wavelet, observed data and time
 * length.  A plan records every problem's gradient evaluation, merges the
 * stencil passes that fall on the same step of a common schedule (all
 * problems share one checkpoint interval) into one launch, and captures the
 * whole sequence in a HIP graph that each run replays.  For batches of
 * models too small to fill the GPU one at a time.  Results equal those of
 * fwi_gradient on each problem (bit for bit at the same temporal depth,
 * see fwi_batch_plan_create).
 *
 * Ownership: the plan is a host object made by fwi_batch_plan_create and
 * released by fwi_batch_plan_destroy.  It keeps the device addresses of the
 * caller's arrays and workspace, which must stay allocated while the plan
 * is used; their contents (models, observed data) may change between runs.
 * Host geometry tables are copied at creation.  Runs of one plan must be
 * ordered on one stream. */
typedef struct fwi_batch_problem {
    fwi_grid grid;
    fwi_geom geom;
    const float *eps_r;        /* device [NY][NX]                             */
    const float *sigma;        /* device [NY][NX]                             */
    const float *observed;     /* device [nshots][nt][nrec]                   */
    double *misfit;            /* device, one double, J = 1/2 sum r^2         */
    float *grad_eps_r;         /* device [NY][NX], overwritten                */
    float *grad_sigma;         /* device [NY][NX], overwritten                */
} fwi_batch_problem;

#define FWI_BATCH_MAX_TUNE 16
typedef struct fwi_batch_info {
    int32_t nproblems;
    int32_t checkpoint_interval; /* common to all problems                   */
    int32_t band_rows;         /* row-band height in use (0: per-problem default) */
    int32_t depth;             /* temporal depth of the passes (4 or 8)       */
    int32_t steps;             /* operations per run                          */
    int32_t stencil_launches;  /* merged stencil launches per run             */
    int32_t graph;             /* 1: runs replay a captured HIP graph         */
    int32_t ntune;             /* candidates timed by the autotuner           */
    int32_t tune_depth[FWI_BATCH_MAX_TUNE]; /* each candidate's depth         */
    int32_t tune_rows[FWI_BATCH_MAX_TUNE];  /* and band height (0: default)   */
    double tune_ms[FWI_BATCH_MAX_TUNE];     /* its cost per time step, ms:
                                  (forward sweep + segment re-forward +
                                  adjoint pass) / depth, each the largest
                                  merged full-depth launch of its kind,
                                  best of 3                                 */
} fwi_batch_info;

/* `autotune` flags of fwi_batch_plan_create. */
#define FWI_TUNE_BANDS 1       /* time row-band heights                       */
#define FWI_TUNE_DEPTH 2       /* time temporal depths 4 and 8                */
#define FWI_BATCH_DEPTH8 4     /* without FWI_TUNE_DEPTH: run at depth 8
                                  (otherwise depth 4)                       */

typedef struct fwi_batch_plan fwi_batch_plan;

/* Workspace for a batch (host out `bytes`); statuses as fwi_workspace_bytes
 * for the first invalid problem, FWI_EINVAL for nproblems < 1 or a null
 * device pointer in a problem. */
int fwi_batch_workspace_bytes(int32_t nproblems, const fwi_batch_problem *problems,
                              size_t *bytes);

/* Validate, lay out the workspace, upload geometry and schedule tables,
 * optionally time candidate temporal depths and row-band heights (autotune:
 * FWI_TUNE_* flags; timing runs stencil passes on the workspace), and
 * capture the graph.  Synchronises `stream`.  *plan receives the plan (NULL
 * on error); FWI_ENOMEM if ws is missing, misaligned or smaller than
 * fwi_batch_workspace_bytes; FWI_EINVAL for unknown flags.
 * Results equal fwi_gradient's on each problem bit for bit when the plan
 * runs at the temporal depth fwi_gradient uses for that problem (depth 4
 * below 2^20 cells per shot, 8 from there on); at the other depth the
 * per-pass partial sums of the imaging correlations group differently, and
 * the results agree within FP32 rounding. */
int fwi_batch_plan_create(int32_t nproblems, const fwi_batch_problem *problems, void *ws,
                          size_t ws_bytes, int32_t autotune, void *stream,
                          fwi_batch_plan **plan);

/* One gradient evaluation of every problem: misfit and gradients written to
 * each problem's outputs.  use_graph = 0 issues the same operations one by
 * one instead of replaying the graph (same results).  Asynchronous. */
int fwi_batch_plan_run(fwi_batch_plan *plan, int32_t use_graph, void *stream);

/* Plan statistics (host out `info`). */
int fwi_batch_plan_info(const fwi_batch_plan *plan, fwi_batch_info *info);

/* Release a plan (NULL is ignored).  The caller's arrays are untouched. */
void fwi_batch_plan_destroy(fwi_batch_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H */
