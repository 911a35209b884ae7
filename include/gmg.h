/*
 * gmg.h -- C ABI of libgmg.so, a geometric-multigrid (GMG) solver for the
 * variable-coefficient pressure Poisson problem  div(L grad p) = sigma  on a
 * Cartesian grid, written for AMD Instinct MI355X (gfx950).
 *
 * The method is the one of "Scaling WaterLily.jl with MPI and an improved
 * geometric multigrid solver" (Font, Lauber, Huang, Weymouth):
 *   - GMG = smoothing plus coarse-grid correction (Sec. 3);
 *   - red-black Gauss-Seidel smoothing with a relaxation factor that is
 *     lowered on residual growth and raised on decay after every V-cycle
 *     (Sec. 3.1);
 *   - anisotropic coarsening: every direction is halved independently until
 *     it reaches the coarsening limit; isotropic coarsening stops when the
 *     smallest direction does (Sec. 3.2).
 *
 * Discretisation (unit cell size, finite-volume flux form):
 *   (A x)(I) = sum_d L_d(I+e_d) (x(I+e_d) - x(I)) + L_d(I) (x(I-e_d) - x(I)),
 *   D(I) = -sum of the six face coefficients; cells with D = 0 are inactive
 *   (decoupled): their residual is 0 and the solver never changes them.
 *
 * Memory layout of every array argument (all DEVICE pointers unless stated):
 *   cell fields x, sigma, r: C order [nz][ny][nx], x fastest, no ghost cells;
 *   face coefficients L: [3][nz][ny][nx]; L[d][I] is the LOW d-face of cell I
 *   (between I - e_d and I).  The high face of the last cell wraps to index 0
 *   in a periodic direction and is a wall (coefficient 0) otherwise; the low
 *   face at index 0 of a wall direction is treated as 0 whatever it holds.
 *
 * Precision: `dtype` is the element type of the caller's x, sigma, r and L;
 * `cycle_dtype` is the V-cycle arithmetic; `l_storage` is how the handle
 * stores the face coefficients of the hierarchy (BF16 = round to nearest
 * even, loaded and computed in FP32).  Norms accumulate in FP64.
 *
 * Streams: all work is enqueued on the HIP stream given to gmg_setup (NULL =
 * the legacy default stream).  Calls that return host scalars or fill an
 * info struct synchronise that stream before returning; the others are
 * asynchronous.  A handle is not thread-safe; distinct handles are
 * independent.
 *
 * Errors: every call returns a gmg_status; no C++ exception crosses the ABI.
 * Argument errors are detected before any side effect.  gmg_last_error()
 * returns a thread-local message about the last failure.
 */
#ifndef GMG_H
#define GMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gmg_status {
  GMG_OK = 0,
  GMG_EINVAL = 1,   /* null pointer, bad parameter, dtype mismatch, or a
                       non-finite input (NaN/Inf face, sigma or initial
                       guess, detected on the device; see each call) */
  GMG_ESHAPE = 2,   /* n_d < 1, or an odd size (or 1) in a periodic direction */
  GMG_ENOMEM = 3,   /* device or pinned-host allocation failed */
  GMG_EHIP = 4,     /* a HIP runtime error (message in gmg_last_error) */
  GMG_ENOCONV = 5   /* max_cycles / max_outer reached before the tolerance */
} gmg_status;

typedef enum gmg_dtype { GMG_F32 = 0, GMG_F64 = 1, GMG_BF16 = 2 } gmg_dtype;

typedef enum gmg_smoother { GMG_SMOOTH_RBGS = 0, GMG_SMOOTH_PCG = 1 } gmg_smoother;

/* Solver parameters.  gmg_default_params fills the defaults noted here. */
typedef struct gmg_params {
  int32_t n[3];          /* cells (nx, ny, nz)                                 */
  int32_t periodic[3];   /* 1 periodic, 0 wall (Neumann), per direction x,y,z  */
  int32_t dtype;         /* caller arrays: GMG_F32 or GMG_F64 (default F32)    */
  int32_t cycle_dtype;   /* V-cycle arithmetic: GMG_F32 or GMG_F64; F64 needs
                            dtype F64 (default: same as dtype)                 */
  int32_t l_storage;     /* hierarchy faces: GMG_F32, GMG_F64 (F64 cycles
                            only) or GMG_BF16 (F32 cycles only); default: the
                            cycle dtype                                         */
  int32_t anisotropic;   /* 1: coarsen each direction independently (Sec. 3.2,
                            default); 0: isotropic, stop when any direction
                            cannot be halved                                   */
  int32_t min_coarse;    /* a direction is halved only if the result has at
                            least this many cells (default 4), n is even, and
                            (periodic) the half is even                        */
  int32_t max_levels;    /* cap on the number of levels, 0 = none (default)   */
  int32_t nu_pre;        /* red-black sweeps before restriction (default 2)   */
  int32_t nu_post;       /* sweeps after the correction (default 2)           */
  int32_t nu_coarse;     /* sweeps on the coarsest level when coarse_rtol is 0,
                            the group size of the coarse_rtol rule otherwise;
                            no direct solve (4)                                */
  int32_t rollback;      /* 1: a V-cycle that grows the residual is discarded
                            (default 1)                                        */
  int32_t graphs;        /* 1: replay the solve's V-cycle (and refinement step)
                            as a captured HIP graph (default); 0: launch each
                            kernel directly.  Results are identical.           */
  int32_t tail_cells;    /* levels >= 1 with at most this many cells (and all
                            coarser ones) are cycled by one workgroup in one
                            launch (same arithmetic as the grid-wide kernels);
                            0 = off, at most 32768 (default 4096)             */
  int32_t smoother;      /* GMG_SMOOTH_RBGS (default): adaptive under-relaxed
                            red-black Gauss-Seidel (Sec. 3.1).  GMG_SMOOTH_PCG:
                            each smoothing step is a Jacobi-preconditioned CG
                            run of nu_pre / nu_post / nu_coarse iterations,
                            restarted from the current iterate (the GMG-PCG
                            comparison of Sec. 3 and Table 1); omega is then
                            unused, every cycle is accepted (no rollback) and
                            no single-workgroup tail is used                  */
  int32_t deferred_norm; /* 0 (default): a separate norm kernel after every
                            cycle of gmg_solve.  1: the norm of a cycle's
                            result is taken by the next cycle's first sweep
                            and the decision made there (a conditional sweep
                            redoes it when omega changes otherwise): one
                            level-0 pass less per cycle and one extra buffer.
                            Same decisions and iterates either way.  Needs
                            dtype == cycle_dtype, the red-black smoother,
                            nu_pre >= 1 and two levels; otherwise 0 is used.  */
  int32_t pair_sweeps;   /* 1 (default): where a level uses it, two
                            consecutive red-black sweeps of one smoothing step
                            run as one two-sweep pass (temporal blocking: the
                            faces and sigma are read once for both sweeps),
                            bitwise the same result.  On at level 0 by
                            default; gmg_autotune and gmg_set_pair_sweeps
                            choose per level.  Needs FP32 cycles, the
                            red-black smoother, an even nx and at most 2^28
                            cells on the level (32-bit buffer offsets); the
                            deferred norm's sweeps stay single.  0: separate
                            sweeps.                                           */
  double omega0;         /* relaxation factor at the start of a solve (1.0)   */
  double omega_min;      /* lower bound (0.1)                                 */
  double omega_max;      /* upper bound (1.0)                                 */
  double theta_dec;      /* factor applied on residual growth (0.5)           */
  double theta_inc;      /* factor applied on residual decay (1.2)            */
  double coarse_rtol;    /* smoothing of the coarsest level of a hierarchy of
                            two or more levels (red-black smoother): its
                            right-hand side loses its mean over the active
                            cells (the level is singular; the mean holds only
                            rounding), then sweeps in groups of nu_coarse,
                            the residual norm (active cells, FP64 sum)
                            checked after each group, until it is at most
                            coarse_rtol times its value on entry or
                            coarse_max sweeps are done.  Sec. 3.2: the
                            coarsest grid is where the smoother removes the
                            lowest wavenumbers.  Needs a coarsest level of at
                            most 2^20 cells (else gmg_setup returns
                            GMG_ESHAPE).  0: exactly nu_coarse sweeps.  A
                            single-level grid always takes nu_coarse sweeps
                            per cycle.  Must be in [0, 1) (default 0.1)      */
  int32_t coarse_max;    /* sweep cap of that rule, 1 .. 4096 (default 64)    */
  double ir_target;      /* refinement (gmg_solve_ir, gmg_batch_solve_ir): the
                            inner tolerance of an outer step that starts from
                            residual r is max(inner_rtol, ir_target * rtol *
                            ||sigma|| / ||r||), so the step's inner solve
                            stops once the outer tolerance is within reach
                            instead of always reducing its own residual by
                            inner_rtol.  0: inner_rtol alone.  In [0, 1]
                            (default 0.5)                                      */
  int32_t uniform_bricks; /* 1 (default): gmg_setup and gmg_update_faces mark,
                            on every level of at least 2^21 cells, the
                            128 x 2 x 2-cell bricks in which every face of
                            direction d reads one value u_d bit for bit (the
                            faces just beyond the brick's high sides
                            included, the zero faces of a low wall
                            excepted); the residual kernels (norm, fused
                            residual + restriction) take such blocks' faces
                            from u instead of loading them, and so does the
                            two-sweep pass for tiles whose region lies in
                            such bricks.  2: the same on every level.  0:
                            off.  Bitwise the same results in every case;
                            less memory traffic where the faces are uniform
                            (away from immersed bodies).                      */
} gmg_params;

#define GMG_MAX_HISTORY 512

/* Filled by gmg_solve.  history[k] is ||r||/||sigma|| after cycle k (of the
 * cycle's own result, accepted or not), omegas[k] the factor cycle k used,
 * accepted[k] 1 if it was kept. */
typedef struct gmg_solve_info {
  int32_t status;        /* GMG_OK, GMG_ENOCONV or GMG_EINVAL (non-finite)     */
  int32_t cycles;        /* V-cycles run                                       */
  int32_t accepted_cycles;
  int32_t launches;      /* host launch rounds (diagnostic)                    */
  double rnorm0;         /* ||sigma - A x0|| over the active cells            */
  double rnorm;          /* ||sigma - A x|| of the returned x                  */
  double snorm;          /* ||sigma|| over the active cells                    */
  double omega;          /* factor after the last cycle                        */
  double history[GMG_MAX_HISTORY];
  double omegas[GMG_MAX_HISTORY];
  int32_t accepted[GMG_MAX_HISTORY];
} gmg_solve_info;

typedef struct gmg_handle gmg_handle;

/* Fill *p with the defaults above for an n[0] x n[1] x n[2] wall-bounded FP32
 * problem.  Returns GMG_EINVAL if p is NULL. */
gmg_status gmg_default_params(gmg_params* p);

/* Plan the level hierarchy (Sec. 3.2 coarsening rule), copy L (device, dtype
 * p->dtype, [3][nz][ny][nx]) into handle-owned storage (wall low faces
 * zeroed, rounded to l_storage) and restrict it level by level:
 *   L_d^{l+1}[J] = (1/c_d) * sum of the fine d-faces tiling the low d-face of
 *   coarse cell J.
 * The caller keeps ownership of L and may free it once this call returns.
 * `stream` is a hipStream_t (may be NULL).  On success *out owns all device
 * workspace (levels, work buffers, reduction partials, solver state) until
 * gmg_destroy.  Errors: GMG_EINVAL (NULL p/L/out, bad dtype combination or
 * parameter, or a face coefficient that is NaN or Inf, found on the device
 * while copying; the low faces at index 0 of wall directions are not
 * checked since they are treated as 0), GMG_ESHAPE, GMG_ENOMEM, GMG_EHIP.
 * Synchronises the stream. */
gmg_status gmg_setup(const gmg_params* p, const void* L, void* stream,
                     gmg_handle** out);

/* New face coefficients for an existing hierarchy: the per-time-step update
 * of a moving or deforming body, whose faces change every step while the
 * grid does not (the paper's solver restricts L afresh on every level each
 * time step, Sec. 3.2).  L: device, [3][nz][ny][nx] in params.dtype, as for
 * gmg_setup; copied and restricted into the handle's storage on every level
 * (same results as a new gmg_setup with this L), the caller may free it
 * afterwards.  Allocates nothing; recorded graphs stay valid.  Synchronises
 * the stream.  A non-finite face gives GMG_EINVAL and leaves the hierarchy
 * unusable until a valid update. */
gmg_status gmg_update_faces(gmg_handle* h, const void* L);

/* Free everything the handle owns.  NULL is accepted. */
gmg_status gmg_destroy(gmg_handle* h);

/* Number of levels, and the shape (cells) and coarsening factor (to the next
 * level, 0 0 0 on the coarsest) of level `level`.  Host pointers. */
gmg_status gmg_num_levels(const gmg_handle* h, int32_t* nlevels);
gmg_status gmg_level_shape(const gmg_handle* h, int32_t level, int32_t n[3],
                           int32_t c[3]);

/* Copy the stored face coefficients of `level` ([3][nz][ny][nx] of that
 * level, element type l_storage; BF16 as raw uint16) into the caller's
 * device buffer `L_out`.  Asynchronous. */
gmg_status gmg_level_faces(gmg_handle* h, int32_t level, void* L_out);

/* Uniform-brick map of level `level` (see gmg_params.uniform_bricks): the
 * number of bricks whose faces are uniform, of those the number whose cells
 * are all active (D != 0; may be NULL), and the number of bricks (all 0 when
 * the map is off).  Synchronises the handle's stream. */
gmg_status gmg_level_uniform(gmg_handle* h, int32_t level, int64_t* uniform,
                             int64_t* uniform_active, int64_t* total);

/* Residual of the level-0 problem in dtype arithmetic (Sec. 3: the quantity
 * the V-cycle drives to zero):  r = sigma - A x on active cells, 0 elsewhere.
 * x, sigma: device, dtype.  r: device output or NULL (not written).
 * rnorm, snorm: host outputs or NULL: ||r||_2 and ||sigma||_2 over the active
 * cells, FP64 accumulation.  If rnorm or snorm is given the call synchronises.
 * The operator is the stored level-0 one, except that a handle with
 * dtype F64 and cycle_dtype F32 uses an exact FP64 copy of L. */
gmg_status gmg_residual(gmg_handle* h, const void* x, const void* sigma,
                        void* r, double* rnorm, double* snorm);

/* gmg_residual without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the same
 * kernels and the same results, with the reduction partials in a
 * fixed-size array that the library keeps in each device's memory until the
 * process ends, and the norms written to device memory.  It allocates
 * nothing and never synchronises: all work is enqueued on the handle's
 * stream, so the call can be captured into a HIP graph.
 * x, sigma, r: as in gmg_residual (r: device output or NULL).
 * rnorm, snorm: DEVICE pointers to one double each, or NULL: receive
 * ||r||_2 and ||sigma||_2 over the active cells (FP64 accumulation), as
 * gmg_residual returns them on the host.
 * Limit: level 0 may need at most 2^18 reduction blocks (128 x 2 columns by
 * 16 z-planes each; every grid up to 1024^3 cells fits); larger grids get
 * GMG_EINVAL before any work is enqueued.  The array is shared by every call
 * on that device: calls whose work overlaps on the device (different
 * streams, or different threads without ordering) race and may return wrong
 * norms.  Uses the array of the device current at the call, which must be
 * the device of the handle. */
gmg_status gmg_residual_noalloc(gmg_handle* h, const void* x, const void* sigma, void* r,
                                double* rnorm, double* snorm);

/* `sweeps` red-black Gauss-Seidel sweeps (Sec. 3.1) in place on level
 * `level`, at the handle's current omega: each sweep updates every active
 * cell of colour (i+j+k) mod 2 == 0 at once, x(I) += omega r(I) / D(I) from
 * the residual before that half-sweep, then every active cell of colour 1.
 * Consecutive sweeps run as two-sweep passes where the level uses them
 * (pair_sweeps), with the same result.  x, sigma: device arrays of that
 * level's shape in cycle_dtype.  Async. */
gmg_status gmg_smooth(gmg_handle* h, int32_t level, void* x,
                      const void* sigma, int32_t sweeps);

/* Fused residual and restriction from `level` to level+1 (coarse-grid
 * correction, Sec. 3):  sigma_c[J] = sum over the c-block of J of
 * (sigma - A x), and x_c = 0 (the coarse initial guess).  Arrays in
 * cycle_dtype, shapes of `level` (x, sigma) and level+1 (sigma_c, x_c);
 * x_c may be NULL.  Async.  GMG_EINVAL on the coarsest level. */
gmg_status gmg_restrict_residual(gmg_handle* h, int32_t level, const void* x,
                                 const void* sigma, void* sigma_c, void* x_c);

/* Piecewise-constant prolongation and correction from level+1 to `level`:
 * x[a] += x_c[a / c] for active cells a.  Async. */
gmg_status gmg_prolong_correct(gmg_handle* h, int32_t level,
                               const void* x_c, void* x);

/* Current relaxation factor (used by gmg_smooth and gmg_vcycle; set to
 * omega0 at the start of each gmg_solve).  get synchronises. */
gmg_status gmg_get_omega(gmg_handle* h, double* omega);
gmg_status gmg_set_omega(gmg_handle* h, double omega);

/* Number of red-black sweeps the coarsest level received in the handle's
 * most recent V-cycle that reached it through the single-workgroup tail
 * (nu_coarse, or the count chosen by the coarse_rtol rule, Sec. 3.2);
 * 0 before any.  Synchronises the handle's stream. */
gmg_status gmg_coarse_sweeps(gmg_handle* h, int32_t* sweeps);

/* One V(nu_pre, nu_post) cycle (Sec. 3) in place on x (device, dtype ==
 * cycle_dtype) at the current omega, with no adaptation:
 *   nu_pre sweeps; restrict the residual; recurse (x_c = 0); prolong and
 *   correct; nu_post sweeps; nu_coarse sweeps on the coarsest level.
 * If rnorm_after is non-NULL it receives ||sigma - A x|| (synchronises). */
gmg_status gmg_vcycle(gmg_handle* h, void* x, const void* sigma,
                      double* rnorm_after);

/* Adaptive GMG solve (Sec. 3.1): V-cycles from x (in: initial guess, out:
 * solution; dtype == cycle_dtype) until ||r|| <= rtol ||sigma|| (norms over
 * active cells) or max_cycles.  After each cycle the new residual norm is
 * compared with the last accepted one: growth multiplies omega by theta_dec
 * (>= omega_min) and, with rollback, discards the cycle; decay (or a tie)
 * keeps it and multiplies omega by theta_inc (<= omega_max).  Decisions are
 * taken on the device; the host only polls a flag between launch rounds.
 * If ||sigma|| = 0, x is returned unchanged with status GMG_OK.
 * Returns GMG_OK or GMG_ENOCONV (x then holds the last accepted iterate);
 * GMG_EINVAL if ||sigma|| or ||sigma - A x0|| is not finite (NaN or Inf in
 * sigma or x0: no cycle runs and x is unchanged), or if a cycle's residual
 * norm is not finite (an overflow: the solve stops there and x holds the
 * last accepted iterate).  info (host, may be NULL) is filled in every case.
 * Synchronises. */
gmg_status gmg_solve(gmg_handle* h, void* x, const void* sigma, double rtol,
                     int32_t max_cycles, gmg_solve_info* info);

/* Filled by gmg_pcg.  history[k] is ||r||/||sigma|| of the recursive residual
 * after iteration k (the first GMG_MAX_HISTORY iterations). */
typedef struct gmg_pcg_info {
  int32_t status;        /* GMG_OK, GMG_ENOCONV or GMG_EINVAL (non-finite)     */
  int32_t iterations;
  double snorm;          /* ||sigma|| over active cells                        */
  double rnorm0;         /* ||sigma - A x0||                                   */
  double rnorm;          /* final recursive ||r||                              */
  double history[GMG_MAX_HISTORY];
} gmg_pcg_info;

/* The general-purpose solver the paper compares GMG with (Sec. 3, Table 1):
 * Jacobi-preconditioned conjugate gradient on level 0 of the handle, i.e.
 * conjugate gradient on (-A) x = -sigma over the active cells with the
 * preconditioner diag(-A).  x (dtype, in/out) is the initial guess and the
 * result; sigma (dtype) as for gmg_solve.  Iterates until the recursive
 * residual satisfies ||r||/||sigma|| <= rtol (rtol > 0) or max_iter
 * iterations; the vectors are in the cycle precision (dtype == cycle_dtype
 * required), the inner products FP64 on the device.  One iteration is a
 * captured graph of four kernels replayed in rounds; the host reads back a
 * small header between rounds.  Allocates the level-0 work vectors (six
 * arrays) on first use.  info (host) may be NULL.  Returns GMG_ENOCONV if the
 * tolerance was not reached (x holds the last iterate), GMG_EINVAL if a
 * residual norm is not finite (NaN or Inf in sigma or x0). */
gmg_status gmg_pcg(gmg_handle* h, void* x, const void* sigma, double rtol, int32_t max_iter,
                   gmg_pcg_info* info);

/* Filled by gmg_solve_ir.  history[m] is ||sigma - A x||/||sigma|| (FP64,
 * exact faces) before outer step m, and after the last one. */
typedef struct gmg_ir_info {
  int32_t status;        /* GMG_OK, GMG_ENOCONV or GMG_EINVAL (non-finite)     */
  int32_t outer;         /* refinement steps applied                           */
  int32_t inner_total;   /* inner V-cycles over all steps                      */
  int32_t pad;
  double snorm;          /* ||sigma|| over the active cells (FP64)             */
  double rnorm;          /* final ||sigma - A x|| (FP64)                       */
  double history[GMG_MAX_HISTORY];
  int32_t inner_cycles[GMG_MAX_HISTORY];
} gmg_ir_info;

/* Mixed-precision iterative refinement: the residual and the update are FP64
 * on the exact level-0 faces, the corrections come from FP32 V-cycles on the
 * stored (FP32 or BF16) hierarchy.  Needs a handle with dtype F64 and
 * cycle_dtype F32.  Outer step m:
 *   r = sigma - A x (FP64); stop if ||r|| <= rtol ||sigma|| or m == max_outer;
 *   beta = ||r|| / sqrt(#active cells); b = fp32(r / beta);
 *   e = adaptive FP32 GMG solve of A e = b from e = 0 (omega reset to omega0,
 *       same rule as gmg_solve) until ||b - A e|| <= t ||b|| or max_inner
 *       cycles, t = max(inner_rtol, ir_target rtol ||sigma|| / ||r||)
 *       (t = inner_rtol with ir_target 0);
 *   x += beta * e (FP64).
 * x (in: initial guess, out: solution) and sigma are device FP64 arrays of the
 * level-0 shape.  All decisions are taken on the device; the host polls one
 * flag per outer step.  Returns GMG_OK or GMG_ENOCONV; GMG_EINVAL if ||sigma||
 * or an outer residual norm is not finite (NaN or Inf in sigma or x0; the
 * refinement stops before applying any further step).  info may be NULL.
 * Synchronises the stream. */
gmg_status gmg_solve_ir(gmg_handle* h, double* x, const double* sigma, double rtol,
                        int32_t max_outer, int32_t max_inner, double inner_rtol,
                        gmg_ir_info* info);

typedef struct gmg_batch gmg_batch;

/* Set up a batch of nprob independent problems of (possibly) different sizes
 * for gmg_batch_solve_ir.  params: host array of nprob parameter sets, each
 * with dtype F64 and cycle_dtype F32, the red-black smoother, all sharing
 * l_storage, the sweep counts (with nu_coarse == nu_pre + nu_post) and the
 * relaxation rule.  L: host array
 * of nprob device pointers to FP64 faces ([3][nz][ny][nx] of each problem).
 * Each problem gets its own hierarchy as in gmg_setup; device descriptor
 * tables let one launch cover the same step of every problem.  The caller
 * may free the L arrays after the call.  Synchronises the stream. */
gmg_status gmg_batch_setup(const gmg_params* params, const void* const* L, int32_t nprob,
                           void* stream, gmg_batch** out);

/* Iterative refinement (as gmg_solve_ir) of every problem of the batch.  With
 * graphs on, the set-up and ONE refinement step of every problem (max_inner
 * cycles, the FP64 update, the new residual and its check) are recorded as two
 * HIP graphs (kept and replayed while x, sigma and the tolerances stay the
 * same).  The host launches the set-up graph, then replays the step graph
 * until a device flag, read back into pinned memory after each replay (one
 * stream synchronisation per replay), reports every problem finished, at
 * most max_outer times: one graph launch per refinement step, not one launch
 * for the whole solve.  Problems that converge become no-ops inside the
 * graph.  x, sigma: host arrays of nprob device FP64 pointers.  infos: host
 * array of nprob results, or NULL.  Returns GMG_ENOCONV if any problem missed
 * rtol, GMG_EINVAL if a norm of some problem was not finite (that problem
 * stops; the others finish).  Synchronises the stream. */
gmg_status gmg_batch_solve_ir(gmg_batch* b, double* const* x, const double* const* sigma,
                              double rtol, int32_t max_outer, int32_t max_inner,
                              double inner_rtol, gmg_ir_info* infos);

/* Tune the z-chunk of the batched fused sweep (tile rows fixed at 8) once per
 * distinct level shape of the batch (timed with HIP events on the problems'
 * own inner buffers), apply it to every problem and rebuild the descriptor
 * tables; the recorded graph is dropped.  The tiles of the batched two-sweep
 * passes are not tuned: they follow a fixed rule (64 x 16 at depth 0, 64 x 8
 * below, z-chunks sized to fill about two rounds of the CUs).  Results do
 * not depend on the choice.  Synchronises. */
gmg_status gmg_batch_autotune(gmg_batch* b, int32_t reps);

/* Free the batch and all its problems.  NULL is accepted. */
gmg_status gmg_batch_destroy(gmg_batch* b);

/* Sweep choice per level, as measured by gmg_autotune: the fused sweep with
 * ty = 4 or 8 rows per tile and kchunk z-planes per workgroup, or ty = 1:
 * the sweep as two plain half-sweep launches (red, then black), faster where
 * a level's plane march is latency-bound; with the mean sweep time of the
 * chosen and the default choice. */
typedef struct gmg_tune_report {
  int32_t nlevels;
  int32_t ty[32], kchunk[32];
  int32_t ty_default[32], kchunk_default[32];
  double us[32], us_default[32];
  int32_t pair_kchunk[32];  /* z-chunk of the two-sweep pass kept, 0 = none  */
  double us_pair[32];       /* mean time of one two-sweep pass without and with
                               the folded correction (0: not tried)          */
  int32_t pair_ty[32];      /* tile rows of that pass (8 or 16)               */
} gmg_tune_report;

/* Time `reps` sweeps of every level for each candidate (fused with ty in
 * {8, 4} and kchunk in {2, 4, ..., 64} up to nz, FP64 cycles: ty 4; and the
 * split half-sweeps, ty 1), and where pair_sweeps allows, `reps` two-sweep
 * passes with ty in {16, 8} and kchunk in {default, 4, 8, ..., 256} (a pass
 * is kept if it beats two of the chosen sweeps), with
 * HIP events on the handle's stream, and keep the fastest per level.  x and
 * sigma are level-0 device arrays (dtype == cycle_dtype) used as the sweep's
 * input (x is overwritten with smoothed values; coarse levels use internal
 * buffers).  Recorded graphs are dropped.  report (host) may be NULL.  The
 * results do not depend on the tile choice.  Synchronises. */
gmg_status gmg_autotune(gmg_handle* h, void* x, const void* sigma, int32_t reps,
                        gmg_tune_report* report);

/* Apply a known sweep choice to one level (e.g. from a cache of earlier
 * gmg_autotune runs).  GMG_EINVAL for ty not in {1, 4, 8} (1 or 4 with FP64
 * cycles) or kchunk outside [1, nz].  With ty = 1 on level 0, gmg_solve does
 * not use the deferred norm. */
gmg_status gmg_set_tiles(gmg_handle* h, int32_t level, int32_t ty, int32_t kchunk);

/* Run the smoothing steps of one level with two-sweep passes on tiles of
 * 64 x ty cells (ty 8 or 16) with kchunk z-planes per workgroup (kchunk = 0:
 * separate sweeps, ty ignored).  GMG_EINVAL if the handle's parameters do not
 * allow passes (pair_sweeps 0, FP64 cycles, the PCG smoother, an odd nx or
 * more than 2^28 cells on the level),
 * ty is not 8 or 16, or kchunk is outside [0, nz].  Results do not depend on
 * the choice.  Recorded graphs are dropped. */
gmg_status gmg_set_pair_sweeps(gmg_handle* h, int32_t level, int32_t ty, int32_t kchunk);

/* Thread-local description of the last error ("" if none). */
const char* gmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GMG_H */
