/* sphgpu -- the SPH neighbour loops of the SWIFT method (Borrow et al.,
 * arXiv:1807.01341) on one AMD MI355X (gfx950).
 *
 * The calls follow the paper's statement of one time-step: build the adaptive
 * cells (Sec. III-A), sort cell contents for neighbour finding (Fig. 5, the
 * "sort" task), mark the particles and cells active in the current time-bin
 * (Sec. II-A Eq. 2, Sec. III-D), run the density loop with the ghost's
 * smoothing-length correction and then the force loop over the active cell
 * pairs (Sec. III-A, Fig. 5), and kick/drift with individual time-steps
 * (Sec. II-A, Eq. 1).
 *
 * Conventions that hold for every call:
 *  - All particle arrays are DEVICE pointers owned by the caller, structure of
 *    arrays, contiguous, length n.  They must stay valid until the work the
 *    call enqueued has finished.
 *  - Every call enqueues work on the stream given to sph_create and returns
 *    without waiting, except where a host output is requested (stated below).
 *  - Everything the library derives (cells, sorts, active lists, cell-pair
 *    lists, scratch) belongs to the context.  Its device memory comes from
 *    the allocator callbacks given to sph_create (the Python binding passes
 *    PyTorch's caching allocator), or from hipMalloc / hipFree when none are
 *    given; it is freed by sph_destroy.
 *  - No exception crosses this boundary.  Calls return sph_status; on an
 *    error the context keeps a message readable with sph_last_error.  A
 *    device fault surfaces as SPH_EDEVICE at the next call that synchronises.
 *  - Call order per step: build_cells -> sort_cells -> mark_active ->
 *    density_pass -> force_pass -> kick_drift; a call out of this order
 *    returns SPH_ESTATE.  kick_drift moves particles, so the next step starts
 *    with build_cells again.
 */
#ifndef SPHGPU_H
#define SPHGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;

typedef enum {
  SPH_OK = 0,
  SPH_EINVAL = -1,   /* bad argument (null pointer, n <= 0, bin out of range, box too small) */
  SPH_ENOMEM = -2,   /* device allocation failed */
  SPH_EDEVICE = -3,  /* HIP runtime or kernel error */
  SPH_ENOCONV = -4,  /* smoothing-length solve not converged for some particles;
                        outputs are written with the last iterate */
  SPH_EREBUILD = -5, /* a smoothing length outgrew what the cells allow; rebuild */
  SPH_ESTATE = -6    /* call out of order */
} sph_status;

/* Method parameters.  sph_default_params fills the values used throughout. */
typedef struct {
  double box;          /* periodic cube side L (1.0) */
  double gamma;        /* adiabatic index (5/3) */
  double cfl;          /* Courant factor C of Eq. 1 (0.2) */
  float eta;           /* h = eta (m/rho)^(1/3) (1.2348, about 48 neighbours) */
  float alpha;         /* Monaghan viscosity strength (0.8) */
  float balsara_eps;   /* Balsara switch softening, times c/h (1e-4) */
  float h_tol;         /* relative Newton step that ends the h solve (1e-6) */
  int n_bins;          /* time-bins 0..n_bins-1 of Eq. 2 (14) */
  int split_count;     /* a cell with at least this many particles is split (400, Sec. III-A) */
  int morton_depth;    /* bits per axis of the Morton keys, D <= 21 (16) */
  int top_cap;         /* top-level grid has at most 2^top_cap cells per side (7) */
  int h_max_iter;      /* Newton passes of the h solve (30); a one-wave-per-particle density
                          pass p also takes up to h_max_iter - p steps of its own */
  int compensated;     /* 1: compensated FP32 sums in the loops (1) */
  int cand_cap;        /* loop tiling: candidate slots per wave (512) */
  int list_cap;        /* loop tiling: neighbour-list slots per lane (96) */
  int waves_per_chunk; /* loop tiling: waves sharing one chunk's cell pairs, 1/2/4/8,
                          0 = chosen from the number of active chunks (0) */
  int chunk_split;     /* loop work items: 0 = one per chunk; 1 / 2 = a chunk's cell-pair
                          list split into parts of about 1024 / 4096 staged partner
                          particles (at most 16), when no tuned entry applies (0) */
  int sweep_below;     /* density Newton passes with fewer particles to do, and force passes
                          with fewer active particles, than this run waves per particle
                          (a sweep of each partner leaf in reach) instead of the chunk
                          loop (0: never; batched passes use chunks) (2^18: the sweep
                          wins on sparse deep time-bins, the chunk loop on dense ones);
                          after the first pass of a group the count is read on the device */
  int sweep_waves;     /* waves per particle in those passes: 1, 2 or 4; 0 = one (0) */
  float rebuild_frac;  /* sph_build_cells keeps the cells of its last full build while no
                          leaf's particles moved more than this fraction of the leaf's
                          width since that build (0 = rebuild every call) (0.125) */
  float pair_slack;    /* the density cell-pair lists of sph_mark_active reach this factor
                          times each active leaf's max H, so that smoothing lengths can grow
                          that much in the h solve before the lists are widened, in [1, 2]
                          (1.1) */
  int lazy_drift;      /* 1: drift only the particles a step needs (Sec. II-A, Sec. III-D):
                          sph_kick_drift kicks the active particles and advances the time
                          line; a leaf's particles are drifted to the current time when its
                          step needs them (active leaves, partners of the cell pairs), so
                          the caller's x, v, A, h of other particles lag until
                          sph_drift_all.  Only the library may change the particle state
                          between steps; batched passes refuse such contexts.  0: every
                          particle drifts in sph_kick_drift (0) */
} sph_params;

/* The particle state.  Arrays marked (opt) may be NULL.  build_cells reorders
 * every non-NULL array of this struct in place into cell order. */
typedef struct {
  double *x, *y, *z;        /* positions; wrapped into [0, L) by build_cells */
  double *vx, *vy, *vz;     /* velocity at the current time, read by the loops */
  double *vfx, *vfy, *vfz;  /* kicked velocity, advanced by kicks only (kick_drift) */
  float *m;                 /* mass */
  float *u;                 /* specific internal energy: input when density_pass is
                               called with entropy_from_u=1, else output */
  float *A;                 /* entropic function at the current time (P = A rho^gamma) */
  float *Af;                /* kicked entropic function (kick_drift) */
  float *h;                 /* smoothing length: initial guess in, solution out */
  int8_t *time_bin;         /* Eq. 2 time-bin */
  /* density-loop outputs (for active particles; kept for inactive ones) */
  float *rho, *drho_dh, *f_gradh, *divv, *curlx, *curly, *curlz, *P, *c, *balsara;
  /* force-loop outputs (for active particles) */
  float *ax, *ay, *az, *dA_dt, *du_dt, *vsig;
  int32_t *nngb_density;    /* (opt) neighbours j != i with r < H_i at the final h */
  int32_t *nngb_force;      /* (opt) neighbours j != i with r < max(H_i, H_j) */
} sph_particles;

/* Fills p with the defaults listed in sph_params. */
void sph_default_params(sph_params *p);

/* Device memory of a context.  alloc returns `bytes` of device memory (256-byte
 * aligned) usable by work queued on `hip_stream` from now on, or NULL when it
 * has none; free returns a block alloc gave.  Both are stream-ordered: a
 * freed block may be handed out again for work queued later on the same
 * stream, so the library frees a buffer it outgrows without waiting for the
 * work still queued on it (PyTorch's caching allocator has exactly these
 * semantics).  `user` is passed through unchanged. */
typedef void *(*sph_alloc_fn)(size_t bytes, void *hip_stream, void *user);
typedef void (*sph_free_fn)(void *ptr, void *hip_stream, void *user);

/* Creates a context that enqueues on `hip_stream` (a hipStream_t, NULL for the
 * default stream) of the current device.  Every device buffer the context
 * ever holds is taken from alloc and returned through free (both non-NULL),
 * so no call of the context allocates or frees device memory itself or
 * waits to grow a buffer.  With alloc and free both NULL the context uses
 * hipMalloc and hipFree, and growing a buffer waits for the stream first.
 * The page-locked host slots of the small device-to-host reads (64 int32) are
 * allocated here with hipHostMalloc.  Returns SPH_EINVAL for invalid
 * parameters (morton_depth outside 2..21, split_count < 2, ...) or only one
 * of alloc / free; SPH_ENOMEM when an allocation fails. */
sph_status sph_create(const sph_params *p, void *hip_stream, sph_alloc_fn alloc, sph_free_fn free, void *user,
                      sph_ctx **out);
void sph_destroy(sph_ctx *ctx);

/* Adaptive cells (Sec. III-A: a fixed top-level grid refined while a cell has
 * at least split_count particles).  Wraps positions into [0, L), computes
 * Morton keys on D-bit integer coordinates, sorts particles stably by
 * (key, index), reorders every particle array into that order, builds the
 * octree leaves and their max H = 1.825742*h, and the FP32 offsets of every
 * particle from its leaf centre.  perm_out (opt, device, n) receives the
 * original index of each sorted position.  Synchronises once (the top-level
 * size depends on the largest H).  SPH_EINVAL if max H > L/4.
 * Rebuild criterion (the paper's Fig. 7, Sec. IV, sets apart the steps that
 * rebuild the cells but does not state when a rebuild happens; this rule is
 * the library's reading): when the context's last full build had the same n
 * and rebuild_frac > 0, the call first tries to keep those cells.  It wraps
 * the positions and recomputes the offsets from the same leaves (minimum
 * image), H, each leaf's max H and each leaf's largest displacement since the
 * full build; the particle order is unchanged (perm_out = identity).  The
 * cell-pair searches then widen every leaf-pair distance test by both
 * leaves' displacement bounds, so no pair is missed.  If some leaf's
 * displacement exceeds rebuild_frac times its width (or max H > L/4), the
 * full build runs.  The criterion compares positions index by index, so
 * arrays changed or reordered by the caller are caught as large
 * displacements.  Synchronises once either way. */
sph_status sph_build_cells(sph_ctx *ctx, sph_particles *p, int64_t n, int64_t *perm_out);

/* Per-cell particle sorts for neighbour pruning (Fig. 5 "sort" task): for
 * each leaf and each of the 13 directions of the half neighbour stencil, the
 * in-leaf order by projection of the FP32 offset (ties by in-leaf index).
 * The offsets are those of the last full build: cell updates keep the
 * orders, and the loops widen the point where a sweep stops by twice the
 * leaf's drift margin (a particle's projection moves at most that far from
 * its sorted place).  Keeping the orders between full builds is the
 * library's own rule; the paper does not state when sorts are redone.
 * After a full build this call sorts every leaf of more than
 * 128 particles in one launch (the loops read smaller leaves whole), after
 * one synchronisation that checks the largest leaf (SPH_EINVAL above 4096
 * particles).  It also orders every leaf's particles by H, largest first,
 * for the force loop: with the symmetric cutoff r < max(H_i, H_j), a partner
 * leaf beyond H_i is read only as far as some H_j can reach it.  After a
 * cell update it orders again by the current H the leaves whose H grew more
 * than 2 % past the H they were ordered by (no synchronisation).
 * sph_copy_axis_order sorts every leaf first and copies the 13 axis orders. */
sph_status sph_sort_cells(sph_ctx *ctx);

/* Active set for the current time-bin (Eq. 2, Sec. III-D): particle i is
 * active iff time_bin[i] <= max_active_bin; a leaf is active if it holds an
 * active particle; every active leaf A is paired with each leaf B (A
 * included) whose periodic box distance is below max H over A's active
 * particles.  Synchronises twice (the active-set totals, the cell-pair
 * count); writes the number of active particles to n_active_host if it is
 * non-NULL.  SPH_EINVAL if max_active_bin is outside [0, n_bins-1]. */
sph_status sph_mark_active(sph_ctx *ctx, const sph_particles *p, int max_active_bin, int64_t *n_active_host);

/* Density loop over the active cell pairs with the ghost's smoothing-length
 * correction (Sec. III-A, Fig. 5): for every active i, Newton iterations on
 * h^3 sum_j W(r_ij, h) = eta^3 (cubic spline, H = 1.825742 h), each pass
 * re-running the loop for particles not yet converged; then rho, drho/dh,
 * div v, curl v, the grad-h factor, pressure, sound speed, Balsara switch and
 * the entropic function.  entropy_from_u=1 takes u as the thermal input
 * (A = (gamma-1) u rho^(1-gamma), written to A and to the kicked copy Af, the
 * state a first kick starts from); 0 takes A (and writes u).  A pass that
 * runs one wave per particle also takes Newton steps on the neighbours it
 * keeps within 1.1 H while the new H stays inside, leaving the last step to
 * the ghost (the same iterates, fewer passes).  Synchronises once per group
 * of Newton passes (passes 1-4, then two at a time, or two at a time from the
 * start when the first pass runs one wave per particle; a pass reads on the
 * device which particles the previous one left unconverged).
 * SPH_ENOCONV / SPH_EREBUILD as described above. */
sph_status sph_density_pass(sph_ctx *ctx, sph_particles *p, int entropy_from_u);

/* Force loop over the active cell pairs (Fig. 5): for active i and j != i
 * with r_ij < max(H_i, H_j): pressure acceleration with grad-h terms,
 * Monaghan viscosity with signal speed c_i + c_j - 3 min(0, v_ij.r_ij/r_ij)
 * (Eq. 1) and the Balsara switch, dA/dt, du/dt and the max signal speed. */
sph_status sph_force_pass(sph_ctx *ctx, sph_particles *p);

/* Kick-drift-kick with individual time-steps (Sec. II-A): at integer time ti
 * (units of t_min), for active particles the closing half-kick (skipped if
 * first_step), the new time-step from Eq. 1 (C h / vsig) and bin from Eq. 2
 * (limited to bins whose period divides ti), and the opening half-kick; then
 * every particle drifts by drift_int * t_min (x += vf dt, v += a dt,
 * A += dA/dt dt) and is wrapped into the box.  FP64 for x, v. */
sph_status sph_kick_drift(sph_ctx *ctx, sph_particles *p, int64_t ti, double t_min, int64_t drift_int,
                          int first_step);

/* One whole step of the method (Sec. II-A, Sec. III-D) in one call:
 * sph_build_cells(p, n, perm_out), sph_sort_cells, sph_mark_active(
 * max_active_bin, n_active_host), sph_density_pass(entropy_from_u),
 * sph_force_pass and sph_kick_drift(ti, t_min, drift_int, first_step), with
 * the same arguments, results and errors as those calls (the first failing
 * one ends the step and its status is returned), and no return to the caller
 * between them, so the device does not wait on the caller at the step's
 * synchronisation points.  perm_out and n_active_host may be NULL. */
sph_status sph_step(sph_ctx *ctx, sph_particles *p, int64_t n, int64_t *perm_out, int max_active_bin,
                    int64_t *n_active_host, int entropy_from_u, int64_t ti, double t_min, int64_t drift_int,
                    int first_step);

/* ---- Batches of independent periodic boxes in ONE context (the batching
 * workload: many boxes whose uneven active cell-pair lists run as one launch
 * per loop pass).
 *
 * sph_batch_create turns a context that has not been used yet (no build)
 * into a batch of n_boxes boxes: box b owns particles [box_offsets_host[b],
 * box_offsets_host[b+1]) of every particle array and has side box_L_host[b]
 * (host arrays of n_boxes + 1 and n_boxes entries, copied; offsets start at 0
 * and increase strictly).  Each box gets its own cells, sorts, active set and
 * cell-pair lists (a child context with the batch's parameters, stream and
 * allocator).  On a batch context:
 *  - sph_build_cells(n = last offset) builds every box's cells, reordering
 *    each box's slice of the arrays within the slice; perm_out[i] is the
 *    original (global) index of position i;
 *  - sph_sort_cells, sph_kick_drift and sph_step apply to every box;
 *  - sph_mark_active uses one max_active_bin for every box,
 *    sph_batch_mark_active one per box (host array of n_boxes);
 *  - sph_density_pass and sph_force_pass run each loop pass as ONE launch over
 *    the active chunks of all boxes (work items in decreasing order of
 *    staged partner particles, tiled by the batch autotuner's table), with the
 *    per-box results of each box's own passes under the same tiling;
 *    sph_batch_density_force is the two in one call;
 *  - sph_autotune tunes the batched loops; sph_info sums over the boxes;
 *    sph_adjoint and the sph_copy_* calls return SPH_EINVAL (use
 *    sph_batch_box for a box's structures).
 * Errors name the failing box.  Batches need lazy_drift = 0 (SPH_EINVAL). */
sph_status sph_batch_create(sph_ctx *ctx, int n_boxes, const int64_t *box_offsets_host, const double *box_L_host);
sph_status sph_batch_mark_active(sph_ctx *ctx, const sph_particles *p, const int *max_active_bin_host,
                                 int64_t *n_active_host);
sph_status sph_batch_density_force(sph_ctx *ctx, sph_particles *p, int entropy_from_u);
/* The context of box b of a batch (owned by the batch; NULL if b is out of
 * range or ctx is not a batch), for sph_info and the sph_copy_* calls. */
sph_ctx *sph_batch_box(sph_ctx *ctx, int b);

/* ---- Batched passes over several contexts (independent periodic boxes, or any
 * set of particle systems), each built, sorted and marked by its own calls
 * and all created on the SAME stream, run each loop pass of the density /
 * force pass as ONE launch over the concatenation of their active chunks
 * (work items (box, chunk) in decreasing order of staged partner particles,
 * pulled from one atomic counter by a grid sized to the machine, or one
 * workgroup per item, as the batch tuning table says).  ctxs[0] leads: it
 * holds the work list, the batch tuning table and, on an error, the message
 * (prefixed with the failing box).  ps is an array of n_boxes particle sets,
 * ps[b] belonging to ctxs[b].  A box's results are those of its own
 * sph_density_pass / sph_force_pass run with the same loop tiling (bitwise;
 * the tiling is the batch's).  Each call synchronises (once per Newton pass
 * for the density, once for the force pass's cell-pair sizes).  SPH_EINVAL
 * for a null or repeated context or one on another stream, SPH_ESTATE if a
 * box is not marked (density) or has no density pass (force); the single-box
 * errors otherwise. */
sph_status sph_batch_density_pass(sph_ctx **ctxs, sph_particles *ps, int n_boxes, int entropy_from_u);
sph_status sph_batch_force_pass(sph_ctx **ctxs, sph_particles *ps, int n_boxes);
/* Autotuner of the batched loops: after a batched force pass, times every
 * valid tiling (waves per chunk, candidate/list capacity) with persistent and
 * one-workgroup-per-item launches over the whole batch, keeps the fastest per
 * loop in ctxs[0]'s batch table (keyed by the log2 class of the total chunk
 * count) and appends "batch_candidate" / "batch_best" lines to `path` (NULL:
 * table only).  sph_load_tuning reads "batch_best" lines too.  Synchronises. */
sph_status sph_batch_autotune(sph_ctx **ctxs, sph_particles *ps, int n_boxes, const char *path);

/* Reverse mode of the density and force loops (differentiable-simulation
 * use of the Sec. III-A loops): after a force pass in which every particle
 * was active and whose density pass took the pressure from u
 * (entropy_from_u = 1), for the loss L = sum_i w_i . a_i with weights
 * (wx, wy, wz) (device, float, length n, cell order as the particle arrays)
 * writes dL/dx into gx, gy, gz (device, double, length n) and dL/du into gu
 * (device, float, length n).  The smoothing lengths are the converged roots
 * of h^3 n(h) = eta^3, differentiated implicitly; neighbours are recomputed
 * from fresh cell-pair lists; FP32 pair arithmetic with compensated sums.
 * Does not change the particle arrays or the step state.  SPH_EINVAL if a
 * particle is inactive or an array is missing, SPH_ESTATE before a force
 * pass or after a density pass that took A as the thermal input.
 * Synchronises twice (cell-pair list sizes). */
sph_status sph_adjoint(sph_ctx *ctx, sph_particles *p, const float *wx, const float *wy, const float *wz,
                       double *gx, double *gy, double *gz, float *gu);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): one whole step of
 * sph_step -- build_cells, sort_cells, mark_active, density_pass, force_pass,
 * kick_drift with the same arguments and results as sph_step on a newly
 * created context with parameters *p on hip_stream -- run on a context that
 * lives only for this call, every device buffer of which is carved from a
 * fixed 256 MiB array of the library (each GPU it runs on holds its own copy
 * until the process ends), and whose small device-to-host reads go through
 * host memory of that context.  The call allocates no device or page-locked
 * memory and returns after the work has finished (it synchronises the
 * stream).  n is at most 2^18 = 262144 (SPH_EINVAL beyond); a step that needs
 * more than the array returns SPH_ENOMEM.  The array keeps the previous
 * call's contents; calls that overlap on one GPU (from several host threads
 * or streams) race on it and must not be made.  perm_out and n_active_host
 * may be NULL; scratch_used_host (opt) receives the bytes of the array the
 * step used; err (opt, err_cap bytes) receives the error message, empty on
 * success. */
sph_status sph_step_noalloc(const sph_params *p, void *hip_stream, sph_particles *parts, int64_t n,
                            int64_t *perm_out, int max_active_bin, int64_t *n_active_host, int entropy_from_u,
                            int64_t ti, double t_min, int64_t drift_int, int first_step,
                            int64_t *scratch_used_host, char *err, size_t err_cap);

/* Moves the time line on by drift_int units of t_min with no kick: the
 * times passed over are ones at which no particle is active (Sec. II-A), so
 * the step there would only drift.  With lazy_drift only the line moves
 * (the particles follow when a step needs them); without it every particle
 * drifts as in sph_kick_drift (x by the kicked velocity, v, A and h
 * predicted).  Allowed after a build and the step's sph_kick_drift (before
 * the next build_cells); SPH_ESTATE otherwise, SPH_EINVAL for t_min <= 0,
 * drift_int < 0 or a missing array.  No synchronisation. */
sph_status sph_drift(sph_ctx *ctx, sph_particles *p, double t_min, int64_t drift_int);

/* The first time after ti, in units of t_min, at which some particle is
 * active (Sec. II-A: a particle in time-bin b is active at the multiples of
 * 2^b, so this is the next multiple of 2^b_min, b_min the smallest bin of
 * p->time_bin over the context's particles; for a batch context, the
 * earliest over the boxes).  A caller that advances the time line from step
 * to step takes no step at the times in between, where nothing is active,
 * and moves the time line there (drift_int = *ti_next - ti, in the step's
 * kick_drift or with sph_drift).  Reads
 * p->time_bin (device, int8, length n of the last build_cells, cell order);
 * changes nothing.  SPH_EINVAL for a null argument or ti < 0, SPH_ESTATE
 * before the first build_cells or if a bin is outside [0, n_bins).
 * Synchronises the stream once. */
sph_status sph_next_active_time(sph_ctx *ctx, const sph_particles *p, int64_t ti, int64_t *ti_next);

/* With lazy_drift: drifts every particle still behind the time line to it
 * (x, v, A, h and the derived offsets), e.g. before the caller reads the
 * state of all particles.  Without lazy_drift, or before the first build,
 * nothing to do.  No synchronisation. */
sph_status sph_drift_all(sph_ctx *ctx, sph_particles *p);

/* Waits for the context's stream and reports a pending device error. */
sph_status sph_sync(sph_ctx *ctx);
const char *sph_last_error(const sph_ctx *ctx);

/* Autotuner for the loop tiling (waves per chunk, candidate/list capacity,
 * work order, grid or persistent launch): after a force pass, times every
 * valid configuration of both loops on the current active chunks with HIP
 * events (best of two launches after a warm-up), keeps the fastest per loop
 * for this number of chunks (log2 class), and appends the measurements and
 * the winners to the text file `path` (NULL: keep in the context only).
 * Later passes of the context with a chunk count of the same class use the
 * winner.  Synchronises. */
sph_status sph_autotune(sph_ctx *ctx, sph_particles *p, const char *path);
/* Loads the "best" lines of a file written by sph_autotune. */
sph_status sph_load_tuning(sph_ctx *ctx, const char *path);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * each launch (or group of launches) of the library.  sph_profile(ctx, 1)
 * clears the table and starts recording, 0 stops.  sph_profile_read
 * synchronises, folds the recorded events into the table and writes it as
 * text lines "name launches total_ms" into buf (NUL-terminated, truncated to
 * cap); it returns the full length. */
sph_status sph_profile(sph_ctx *ctx, int enable);
int64_t sph_profile_read(sph_ctx *ctx, char *buf, int64_t cap);

/* ---- Introspection, for checking the derived structures (all copies are
 * enqueued on the context's stream into caller DEVICE buffers of the sizes
 * given by sph_info). ---- */
typedef struct {
  int64_t n;                 /* particles */
  int64_t n_leaves;
  int32_t top_level;         /* top-level grid has 2^top_level cells per side */
  int64_t n_active;          /* after mark_active */
  int64_t n_active_leaves;
  int64_t n_density_pairs;   /* current density cell-pair list */
  int64_t n_force_pairs;     /* force cell-pair list of the last force pass */
  int32_t density_iterations;/* Newton passes of the last density pass */
  int64_t n_unconverged;     /* particles left unconverged by the last density pass */
  int64_t interactions_density; /* cumulative over the context's life: in-support
                                   pairs j != i of each finished density solve */
  int64_t interactions_force;   /* cumulative: pairs j != i of every force loop */
  int32_t unconverged_after_pass[32]; /* last density pass: particles still unconverged
                                         after each Newton pass (first 32 passes) */
  int32_t pair_rebuilds;     /* last density pass: cell-pair lists widened mid-solve */
  int64_t full_builds;       /* cumulative: sph_build_cells calls that rebuilt the cells */
  int64_t cell_updates;      /* cumulative: calls that kept them (offsets, H_max, drift margins) */
  float dx_max;              /* largest displacement since the last full build */
  int64_t device_bytes;      /* device memory the context holds now (all of it from its
                                allocator) */
} sph_info_t;
sph_status sph_info(sph_ctx *ctx, sph_info_t *out); /* synchronises */

/* Leaf table in Morton order: level, integer coordinates at that level,
 * first sorted index, particle count, max H, and (opt) the drift margin of
 * each leaf (0 right after a full build). */
sph_status sph_copy_leaves(sph_ctx *ctx, int32_t *level, int32_t *ix, int32_t *iy, int32_t *iz, int32_t *begin,
                           int32_t *count, float *hmax, float *drift);
/* Sorted Morton keys and FP32 leaf-centre offsets (length n). */
sph_status sph_copy_particles(sph_ctx *ctx, uint64_t *keys, float *ox, float *oy, float *oz);
/* 13 x n in-leaf order (axis-major), by the offsets of the last full build. */
sph_status sph_copy_axis_order(sph_ctx *ctx, uint16_t *order);
/* Active flags (n), active leaves and their max active H (n_active_leaves). */
sph_status sph_copy_active(sph_ctx *ctx, uint8_t *active, int32_t *active_leaves, float *hmax_act);
/* Cell-pair list (which = 0 density, 1 force): leaf A, leaf B, FP32 shift. */
sph_status sph_copy_pairs(sph_ctx *ctx, int which, int32_t *a, int32_t *b, float *sx, float *sy, float *sz);

#ifdef __cplusplus
}
#endif
#endif
