// Internal declarations of the sphgpu library: the context, device buffers,
// shared device helpers and the host launchers of every kernel file.
#pragma once

#include <limits.h>

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sphgpu.h"

// Kernel support over smoothing length (H = GK32 * h), rounded to float.
#define GK32 1.825742f
// 3-D normalisation of the M4 cubic spline on q = r/H: 8/pi.
#define KNORM32 2.5464790894703255f

#define WAVE 64

// Where a context's device memory comes from: the caller's allocator
// callbacks (stream-ordered, e.g. PyTorch's caching allocator), or hipMalloc
// and hipFree when the caller gives none.
struct DevAlloc {
  sph_alloc_fn alloc = nullptr;
  sph_free_fn free = nullptr;
  void *user = nullptr;
  hipStream_t stream = nullptr;
  mutable int64_t live_bytes = 0;         // held by the context's buffers now
};

// Device allocation owned by the context: grown by sph_ensure, freed with the
// context, both through the allocator it was taken from.
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  const DevAlloc *from = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  void release() {
    if (p) {
      if (from && from->free)
        from->free(p, (void *)from->stream, from->user);
      else
        (void)hipFree(p);
      if (from) from->live_bytes -= (int64_t)cap;
    }
    p = nullptr;
    cap = 0;
  }
  ~DevBuf() { release(); }
};

// Page-locked host memory for the small device-to-host reads of a step: a
// copy into it is queued like a kernel, so several reads share one stream
// synchronisation (a copy into pageable memory waits for the stream itself).
struct HostPin {
  int32_t *p = nullptr;
  HostPin() = default;
  HostPin(const HostPin &) = delete;
  HostPin &operator=(const HostPin &) = delete;
  ~HostPin() {
    if (p) (void)hipHostFree(p);
  }
};

// Pair-list entry: partner leaf index (as int bits) and the FP32 shift of the
// partner's offsets into the owner leaf's frame.
struct PairEntry {
  int32_t b;
  float sx, sy, sz;
};

// The 13 directions (dx, dy, dz) in {-1,0,1}^3 of the half neighbour stencil
// (first non-zero component positive, lexicographic order), normalised in
// double and rounded to float: the axes of the per-leaf sorts.
struct AxisTab {
  float e[13][3];
};

// Row of axis_order that lists each leaf's particles by H at the full build,
// largest first (ties by in-leaf index), and the ranks of that order at which
// leaf_hq samples H: every particle at rank >= hq_rank(q) has H at the build
// <= sample q.
constexpr int HORD_ROW = 13;
constexpr int HQ_N = 16;
__host__ __device__ __forceinline__ int hq_rank(int q) {
  return q < 6 ? 4 * (q + 1) : (q < 9 ? 32 + 8 * (q - 6) : (q < 12 ? 64 + 16 * (q - 9) : (q < 13 ? 128 : 64 * (q - 10))));
}

inline AxisTab host_axes() {
  AxisTab a;
  int k = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        const int first = dx != 0 ? dx : (dy != 0 ? dy : dz);
        if (first <= 0) continue;
        const double nrm = sqrt((double)(dx * dx + dy * dy + dz * dz));
        a.e[k][0] = (float)(dx / nrm);
        a.e[k][1] = (float)(dy / nrm);
        a.e[k][2] = (float)(dz / nrm);
        ++k;
      }
  return a;
}

// Sweep axis of a cell pair with shift (sx, sy, sz): the stencil direction
// closest to the offset, coded as axis | 0x80 when the partner lies on the
// negative side.  Made once per pair when the lists are filled.
__device__ __forceinline__ uint8_t sweep_axis_code(const AxisTab &ax, float sx, float sy, float sz) {
  int axis = 0;
  bool neg = false;
  float best = -1.f;
#pragma unroll
  for (int a = 0; a < 13; ++a) {
    const float d = fmaf(sz, ax.e[a][2], fmaf(sy, ax.e[a][1], sx * ax.e[a][0]));
    if (fabsf(d) > best) {
      best = fabsf(d);
      axis = a;
      neg = !(d >= 0.f);
    }
  }
  return (uint8_t)(axis | (neg ? 0x80 : 0));
}

struct Chunk {
  int32_t act_leaf;  // index into the active-leaf list
  int32_t begin;     // first active index (into active_idx)
  int32_t count;     // <= 64 active particles
  int32_t leaf;      // leaf index
};

struct sph_ctx {
  sph_params prm;
  hipStream_t stream = nullptr;
  DevAlloc mem;                           // declared before every DevBuf: outlives them
  // a batch context (sph_batch_create): one child context per box, each over
  // the slice [box_off[b], box_off[b+1]) of the particle arrays
  std::vector<sph_ctx *> kids;
  std::vector<int64_t> box_off;
  int device = 0;
  int n_cu = 256;
  std::string err;
  int state = 0;  // 0 none, 1 built, 2 sorted, 3 marked, 4 density done, 5 force done
  int64_t n = 0;
  int top_level = 0;
  int64_t n_leaves = 0;
  int64_t n_active = 0, n_active_leaves = 0, n_chunks = 0;
  int64_t n_dpairs = 0, n_fpairs = 0;
  int64_t fpairs_counted = -1;  // force pair total counted at the end of the density solve (-1: none)
  int max_active_bin = 0;
  int density_iterations = 0;
  int64_t n_unconverged = 0;
  int32_t unconv_hist[32] = {0};
  int32_t pair_rebuilds = 0;
  // cells kept between builds: positions of the last full build, per-leaf and
  // largest displacement since then (the cell-pair search margin)
  DevBuf x_build, leaf_dx, leaf_half;
  // lazy drift (params.lazy_drift): the internal time line in units of t_min
  // (advanced by each kick's drift interval), the time each leaf's particles
  // were drifted to, a bound on their full-step speed, their displacement
  // bound from the full build at that time, and the leaves a claim collects
  int64_t ti_now = 0;
  double t_min_line = 0.0;
  DevBuf leaf_ti, leaf_vmax, leaf_dx_base, drift_claim, drift_list;
  int32_t drift_stamp = 0;
  float dx_max = 0.f;
  int64_t built_n = 0;
  int64_t n_full_builds = 0, n_updates = 0;

  // build
  DevBuf keys_a, keys_b, vals_a, vals_b, radix_counts, scan_tmp, gather_tmp;
  DevBuf scalars;                         // small device counters
  HostPin pin;                            // page-locked host slots of the reads (PinSlot)
  int32_t *pin_dev = nullptr;             // the slots as kernels address them
  int32_t *pin_h = nullptr;               // the slots as the host reads them
  int pin_mapped = 1;                     // 1: pin_h and pin_dev are one mapped page-locked
                                          // block; 0: pin_dev is device memory, copied to
                                          // pin_local by pin_fetch
  int32_t pin_local[64] = {0};
  DevBuf pin_devbuf;                      // device side of the slots when not mapped
  DevBuf flags, scan_out, nodes_a, nodes_b, leaf_lvl_at;
  DevBuf leaf_level, leaf_ix, leaf_iy, leaf_iz, leaf_begin, leaf_count, leaf_hmax, leaf_of;
  DevBuf top_first, top_last;
  DevBuf block_box;                       // per run of LEAF_BLOCK leaves: int4 lo, int4 hi (half-units)
  int blocks_valid = 0;                   // block_box made for the current full build
  DevBuf pos4;                            // float4 (ox, oy, oz, H) per particle
  DevBuf pos4_build;                      // pos4 of the last full build (the axis sorts' keys)
  DevBuf gbox_lo, gbox_hi;                // boxes of 8-particle groups of each leaf at the full build
  // sort
  DevBuf axis_order;                      // uint16 14 x n: the 13 axes, then the H order (HORD_ROW)
  // force-loop pruning by H: each particle's H at the full build, per leaf a
  // bound on H now / H at the build over its particles, and H at the build at
  // the ranks hq_rank(0..15) of the leaf's H order (0 past its count)
  DevBuf h_build, leaf_hgrow, leaf_hq;
  DevBuf refresh_args;                    // batched leaf max-H refresh: device copy of the per-box arguments
  std::vector<char> refresh_host;         // and its host staging
  DevBuf gather_src;                      // batched force pass: where each box's pair total is
  std::vector<char> gather_host;          // and its host staging
  int max_leaf = 0;                       // largest leaf of the build
  int leaves_checked = 0;                 // max_leaf read and the leaves sorted for the current build
  // mark
  DevBuf active, leaf_nact, leaf_act_off, leaf_actleaf, act_leaves, act_hmax, act_leaf_chunk_off;
  DevBuf active_idx, chunk_of, chunks, chunk_todo;
  DevBuf dpair_off, dpairs, fpair_off, fpairs, pair_cnt;
  DevBuf dpair_axis, fpair_axis;          // per pair: sweep axis code (sweep_axis_code)
  // loops
  DevBuf jvm;                             // float4 (vx, vy, vz, m)
  DevBuf jth;                             // float4 (rho, f P / rho^2, c, B)
  DevBuf sums, hlo, hhi, conv, todo_list, pass_stats;
  int todo_collect = 0;                   // the ghosts of this density pass append to todo_list
  DevBuf counters64;                      // cumulative interaction counts (2 x uint64)
  DevBuf act_cost;                        // staged partner particles per active leaf
  DevBuf act_reach;                       // per active leaf: the radius its density pair list is complete for
  DevBuf work, work_tmp, box_args, box_work;
  int work_valid = 0;                     // the work items match the current chunks and costs
  // loop work items (codes chunk * 16 + part): chunk order and cost order,
  // first item of every chunk, arrival counters and partial results of split chunks
  DevBuf items_nat, chunk_item0, chunk_ctr, partials;
  int64_t n_items = 0;
  int items_target = -1;                  // staged particles per part the items were built for
  int density_from_u = 0;                 // the last density pass took P from u
  int widen_pending = 0;                  // a smoothing length reached the density pair reach
  // adjoint
  DevBuf adj_w, adj1, adj2, adj_out;

  // tuned loop configurations per pass (0 density, 1 force) and chunk-count class
  struct TuneEntry {
    int valid = 0, nw = 1, tile = 2, ordered = 0, persistent = 0, split = 0;
    float ms = 0.f;
  };
  TuneEntry tune[2][32];
  TuneEntry btune[2][32];                 // batched passes led by this context (total chunks)

  // batched passes led by this context: per-box descriptors and the work list
  DevBuf batch_args, batch_ghost, batch_items, batch_work, batch_tmp, batch_status;
  std::vector<char> batch_host;           // host staging of the descriptors

  // optional per-kernel timing with HIP events on ctx->stream
  int prof = 0;
  struct Pending {
    const char *name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  struct Acc {
    std::string name;
    long count;
    double ms;
  };
  std::vector<Acc> acc;
};

// The particle arrays of box b: every non-NULL pointer advanced to the box's
// first particle.
inline sph_particles slice_particles(const sph_particles &p, int64_t off) {
  sph_particles q = p;
  double **d[] = {&q.x, &q.y, &q.z, &q.vx, &q.vy, &q.vz, &q.vfx, &q.vfy, &q.vfz};
  for (double **a : d)
    if (*a) *a += off;
  float **f[] = {&q.m, &q.u, &q.A, &q.Af, &q.h, &q.rho, &q.drho_dh, &q.f_gradh, &q.divv, &q.curlx, &q.curly,
                 &q.curlz, &q.P, &q.c, &q.balsara, &q.ax, &q.ay, &q.az, &q.dA_dt, &q.du_dt, &q.vsig};
  for (float **a : f)
    if (*a) *a += off;
  if (q.time_bin) q.time_bin += off;
  if (q.nngb_density) q.nngb_density += off;
  if (q.nngb_force) q.nngb_force += off;
  return q;
}

inline std::vector<sph_particles> box_slices(const sph_ctx *ctx, const sph_particles *p) {
  std::vector<sph_particles> v;
  for (size_t b = 0; b < ctx->kids.size(); ++b) v.push_back(slice_particles(*p, ctx->box_off[b]));
  return v;
}

// Records events around the enclosed launches when profiling is on.
struct ProfScope {
  sph_ctx *ctx;
  sph_ctx::Pending ev;
  bool on;
  ProfScope(sph_ctx *c, const char *name);
  ~ProfScope();
};
#define SPH_CAT2(a, b) a##b
#define SPH_CAT(a, b) SPH_CAT2(a, b)
#define PROF(ctx, name) ProfScope SPH_CAT(_prof_scope_, __LINE__)((ctx), (name))

// ---------------------------------------------------------------- host helpers
sph_status sph_fail(sph_ctx *ctx, sph_status code, const char *fmt, ...);
// Initialises a context made with new: parameters, stream, allocator, the
// small counters (zeroed) and the read slots -- page-locked and mapped
// (hipHostMalloc) when `mapped`, else taken from the allocator and read back
// by pin_fetch.
sph_status ctx_init(sph_ctx *ctx, const sph_params *p, void *hip_stream, sph_alloc_fn alloc, sph_free_fn free_fn,
                    void *user, bool mapped);
sph_status sph_hip_check(sph_ctx *ctx, hipError_t e, const char *what);
sph_status sph_ensure(sph_ctx *ctx, DevBuf &b, size_t bytes);

#define SPH_TRY(expr)                    \
  do {                                   \
    sph_status _s = (expr);              \
    if (_s != SPH_OK) return _s;         \
  } while (0)
#define HIP_TRY(ctx, expr) SPH_TRY(sph_hip_check((ctx), (expr), #expr))

// Scratch counters in ctx->scalars (int32 slots).
enum ScalarSlot {
  SC_TOTAL0 = 0,      // scan totals
  SC_TOTAL1 = 1,
  SC_TOTAL2 = 2,
  SC_NODES_A = 4,
  SC_NODES_B = 5,
  SC_HMAX_BITS = 6,
  SC_UNCONV = 8,
  SC_REBUILD = 9,
  SC_PAIRTOT = 10,
  SC_MAXLEAF = 11,
  SC_WORKCTR = 12,
  SC_UPD_HMAX = 13,   // cell update: max H bits, max displacement bits, rebuild flag
  SC_UPD_DX = 14,
  SC_UPD_FLAG = 15,
  SC_UPD_FLAG_ACC = 16,  // the rebuild flag as the update kernel raises it (moved to SC_UPD_FLAG and
                         // cleared by the reduction, so that it starts at zero for the next update)
  SC_MINBIN = 17,     // next_active_time: smallest time-bin held
  SC_COUNT = 32
};

// Slots of ctx->pin (int32).  Each read is queued, followed by one stream
// synchronisation, then taken from its slot; slots in flight together differ.
enum PinSlot {
  PIN_SCALARS = 0,    // read_scalars (at most 16 values)
  PIN_MARK = 16,      // mark: active particles, active leaves, chunks (scan totals)
  PIN_NPAIRS = 20,    // cell-pair total of build_pairs
  PIN_FCOUNT = 21,    // force cell-pair total counted during the density solve
  PIN_ITEMS = 22,     // loop work items
  PIN_UPD = 24,       // cell update: max H bits, max displacement bits, rebuild flag (written by the reduction)
  PIN_STATS = 32,     // density solve: per-pass counters of one group of passes
  PIN_COUNT = 64
};
static_assert(PIN_COUNT == sizeof(((sph_ctx *)nullptr)->pin_local) / sizeof(int32_t), "pin_local holds every slot");

// ---------------------------------------------------------------- primitives (primitives.hip)
// Exclusive prefix sum of n int32 values; the total lands in *total_dev.
sph_status scan_exclusive_i32(sph_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev);
// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
// The sorted result is left in ctx->keys_a / ctx->vals_a.
sph_status radix_sort_pairs(sph_ctx *ctx, int64_t n, int bits);
sph_status read_scalars(sph_ctx *ctx, int first, int count, int32_t *host);
// After a stream synchronisation: the host view of the pin slots [first,
// first + count) that kernels wrote (a copy from the device side when the
// slots are not mapped page-locked memory).
sph_status pin_fetch(sph_ctx *ctx, int first, int count);

// ---------------------------------------------------------------- stages
sph_status build_cells_impl(sph_ctx *ctx, sph_particles *p, int64_t n, int64_t *perm_out);
sph_status update_cells(sph_ctx *ctx, sph_particles *p, int64_t *perm_out, int *rebuild);
// Lazy drift: the cell-keep test from the per-leaf bounds (no particle
// access), the drift of listed leaves (or all: list == nullptr) to the
// current time, the drift of the partner leaves of cell-pair list `which`,
// and the per-leaf state of a new full build.
sph_status lazy_keep_cells(sph_ctx *ctx, int *rebuild);
sph_status drift_leaves(sph_ctx *ctx, const sph_particles *p, const int32_t *list, const int32_t *list_n,
                        int64_t cap);
sph_status drift_partners(sph_ctx *ctx, const sph_particles *p, int which);
sph_status lazy_init_leaves(sph_ctx *ctx, const sph_particles *p);
#define LAZY_HGROW 1.2215f  // bound on H's growth in one drift (the h prediction is clipped at e^0.2)
sph_status sort_cells_impl(sph_ctx *ctx);
sph_status mark_active_impl(sph_ctx *ctx, const sph_particles *p, int m, int64_t *n_active_host);
sph_status build_pairs(sph_ctx *ctx, int which, float slack);
sph_status build_pairs_count(sph_ctx *ctx, int which, float slack, int32_t *host_total);
sph_status build_pairs_fill(sph_ctx *ctx, int which, float slack, int32_t np);
sph_status refresh_leaf_hmax(sph_ctx *ctx);
// The same for the boxes cs[boxes[0..nbox)] (one stream), in one launch.
sph_status refresh_leaf_hmax_boxes(sph_ctx *lead, sph_ctx **cs, const int *boxes, int nbox);
#define LEAF_BLOCK 32
sph_status sort_all_leaves(sph_ctx *ctx);
sph_status pack_neighbour_data(sph_ctx *ctx, const sph_particles *p);
struct PackArgs;
// The pack arguments when every array is given (else *ok = false: the pack
// kernels fill what is missing with zeros); sizes jvm and jth.
sph_status pack_args(sph_ctx *ctx, const sph_particles *p, PackArgs *a, bool *ok);
sph_status density_pass_impl(sph_ctx *ctx, sph_particles *p, int entropy_from_u);
sph_status force_pass_impl(sph_ctx *ctx, sph_particles *p);
sph_status batch_density_impl(sph_ctx **cs, sph_particles *ps, int nb, int entropy_from_u);
sph_status batch_force_impl(sph_ctx **cs, sph_particles *ps, int nb);
sph_status batch_autotune_impl(sph_ctx **cs, sph_particles *ps, int nb, const char *path);
sph_status adjoint_impl(sph_ctx *ctx, sph_particles *p, const float *wx, const float *wy, const float *wz,
                        double *gx, double *gy, double *gz, float *gu);
sph_status kick_drift_impl(sph_ctx *ctx, sph_particles *p, int64_t ti, double t_min, int64_t drift_int,
                           int first_step);
sph_status drift_impl(sph_ctx *ctx, sph_particles *p, double t_min, int64_t drift_int);
// First time after ti at which some particle of bin[0..n) is active.
sph_status next_active_impl(sph_ctx *ctx, const int8_t *bin, int64_t n, int64_t ti, int64_t *ti_next);

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
// Number of set bits of `mask` below this lane.
// The loops' packed neighbour data of particle s: (v, m) and the density
// state (rho, f P / rho^2, c, B).
struct PackArgs {
  const double *vx, *vy, *vz;
  const float *m, *rho, *f, *P, *c, *B;
  float4 *jvm, *jth;
};

__device__ __forceinline__ void pack_one(const PackArgs &a, int64_t s) {
  a.jvm[s] = make_float4((float)a.vx[s], (float)a.vy[s], (float)a.vz[s], a.m[s]);
  const float r = a.rho[s];
  a.jth[s] = make_float4(r, a.f[s] * a.P[s] / (r * r), a.c[s], a.B[s]);
}

__device__ __forceinline__ int rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-wide scans and reductions on the DPP lane network (VALU only, no
// LDS round trips): Hillis-Steele shifts by 1, 2, 4, 8 lanes inside each row
// of 16, then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31 into
// rows 2 and 3.  Lanes without a source take the identity `id`.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_from(int id, int v) {
  return __builtin_amdgcn_update_dpp(id, v, CTRL, ROWS, 0xf, false);
}
template <class F>
__device__ __forceinline__ int wave_scan_bits(int v, int id, F op) {
  v = op(v, dpp_from<0x111, 0xf>(id, v));  // row_shr:1
  v = op(v, dpp_from<0x112, 0xf>(id, v));  // row_shr:2
  v = op(v, dpp_from<0x114, 0xf>(id, v));  // row_shr:4
  v = op(v, dpp_from<0x118, 0xf>(id, v));  // row_shr:8
  v = op(v, dpp_from<0x142, 0xa>(id, v));  // row_bcast:15 into rows 1, 3
  v = op(v, dpp_from<0x143, 0xc>(id, v));  // row_bcast:31 into rows 2, 3
  return v;
}
// Inclusive prefix sum over the lanes.
__device__ __forceinline__ int wave_incl_scan_dpp(int v) {
  return wave_scan_bits(v, 0, [](int a, int b) { return a + b; });
}
__device__ __forceinline__ int wave_last(int v) { return __builtin_amdgcn_readlane(v, 63); }
// Reductions to every lane; the DPP forms need all 64 lanes active.
__device__ __forceinline__ float wave_max_f_dpp(float v) {
  const int s = wave_scan_bits(__float_as_int(v), __float_as_int(-INFINITY),
                               [](int a, int b) { return __float_as_int(fmaxf(__int_as_float(a), __int_as_float(b))); });
  return __int_as_float(wave_last(s));
}
__device__ __forceinline__ float wave_min_f_dpp(float v) {
  const int s = wave_scan_bits(__float_as_int(v), __float_as_int(INFINITY),
                               [](int a, int b) { return __float_as_int(fminf(__int_as_float(a), __int_as_float(b))); });
  return __int_as_float(wave_last(s));
}
__device__ __forceinline__ int wave_sum_i_dpp(int v) { return wave_last(wave_incl_scan_dpp(v)); }
__device__ __forceinline__ int wave_max_i_dpp(int v) {
  return wave_last(wave_scan_bits(v, INT_MIN, [](int a, int b) { return max(a, b); }));
}

__device__ __forceinline__ float wave_max_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_min_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// max of non-negative floats through their int bit patterns
__device__ __forceinline__ void atomic_max_pos_f(float *addr, float v) {
  atomicMax(reinterpret_cast<int *>(addr), __float_as_int(v));
}

// Morton helpers (21 bits per axis)
__host__ __device__ __forceinline__ uint64_t spread3_21(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
__host__ __device__ __forceinline__ uint32_t compact3_21(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return (uint32_t)v;
}

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Chunk-count class of a pass for the tuning table: floor(log2(n_chunks)).
inline int tune_class(int64_t n_chunks) {
  int c = 0;
  while (c < 31 && ((int64_t)1 << (c + 1)) <= n_chunks) ++c;
  return c;
}
