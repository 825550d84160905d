// Single-box passes: the density loop with the ghost's h solve, and the
// force loop, over the active chunks of one context.
#include <stdio.h>

#include <algorithm>

#include "loops_common.h"

namespace {

__global__ __launch_bounds__(256) void fill_work_kernel(const int32_t *__restrict__ order, int64_t n,
                                                        int2 *__restrict__ work) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    work[q] = make_int2(0, order ? order[q] : (int)(q << 4));
}

__global__ __launch_bounds__(256) void pack_jvm_kernel(const double *__restrict__ vx, const double *__restrict__ vy,
                                                       const double *__restrict__ vz, const float *__restrict__ m,
                                                       int64_t n, float4 *__restrict__ out) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256)
    out[s] = make_float4((float)vx[s], (float)vy[s], (float)vz[s], m[s]);
}

__global__ __launch_bounds__(256) void pack_kernel(PackArgs a, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) pack_one(a, s);
}

__global__ __launch_bounds__(256) void pack_jth_kernel(const float *__restrict__ rho, const float *__restrict__ f,
                                                       const float *__restrict__ P, const float *__restrict__ c,
                                                       const float *__restrict__ B, int64_t n,
                                                       float4 *__restrict__ out) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) {
    const float r = rho[s];
    out[s] = make_float4(r, f[s] * P[s] / (r * r), c[s], B[s]);
  }
}

__global__ __launch_bounds__(256) void density_init_kernel(int64_t n_chunks, int32_t *__restrict__ todo,
                                                           int64_t n_act, float *__restrict__ lo,
                                                           float *__restrict__ hi, uint8_t *__restrict__ conv,
                                                           int32_t *__restrict__ stats, int n_stats) {
  const int64_t m = n_chunks > n_act ? n_chunks : n_act;
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < n_stats; q += 256) stats[q] = 0;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < m; s += (int64_t)gridDim.x * 256) {
    if (s < n_chunks) todo[s] = 1;
    if (s < n_act) {
      lo[s] = 0.f;
      hi[s] = INFINITY;
      conv[s] = 0;
    }
  }
}

// Particles that waited for wider cell-pair lists become ordinary
// unconverged ones again, their chunks to do.
__global__ __launch_bounds__(256) void release_waiting_kernel(uint8_t *__restrict__ conv,
                                                              const int32_t *__restrict__ chunk_of, int64_t n_act,
                                                              int32_t *__restrict__ chunk_todo,
                                                              int32_t *__restrict__ todo, int32_t *__restrict__ todo_n) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n_act; k += (int64_t)gridDim.x * 256) {
    const bool rel = conv[k] == 2;
    if (rel) {
      conv[k] = 0;
      chunk_todo[chunk_of[k]] = 1;
    }
    if (todo) {
      const uint64_t m = __ballot(rel);
      int base = 0;
      if ((threadIdx.x & 63) == 0 && m) base = atomicAdd(todo_n, __popcll(m));
      base = __shfl(base, 0, 64);
      if (rel) todo[base + rank_below(m)] = (int32_t)k;
    }
  }
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) p[s] = v;
}

unsigned grid256(int64_t n) {
  int64_t g = ceil_div(n, 256);
  if (g > 8192) g = 8192;
  return (unsigned)(g < 1 ? 1 : g);
}

// Work items: every chunk's cell-pair list in parts of about `target` staged
// partner particles (at most 16 parts and at most one per cell pair; one part
// when target is 0), as codes chunk * 16 + part, in chunk order and in
// decreasing order of part cost (log2 buckets: histogram, offsets, scatter).
__global__ __launch_bounds__(256) void split_count_kernel(const Chunk *__restrict__ chunks, int64_t n_chunks,
                                                          const int32_t *__restrict__ act_cost,
                                                          const int32_t *__restrict__ pair_off, int target,
                                                          int32_t *__restrict__ parts) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n_chunks; q += (int64_t)gridDim.x * 256) {
    const int al = chunks[q].act_leaf;
    int P = 1;
    if (target > 0) {
      const int cost = max(1, act_cost[al]);
      const int np = pair_off[al + 1] - pair_off[al];
      P = min(16, min(np, (cost + target - 1) / target));
      P = max(P, 1);
    }
    parts[q] = P;
  }
}

__global__ __launch_bounds__(256) void split_fill_kernel(const Chunk *__restrict__ chunks, int64_t n_chunks,
                                                         const int32_t *__restrict__ act_cost,
                                                         const int32_t *__restrict__ item0,
                                                         int32_t *__restrict__ items, int32_t *__restrict__ bucket_of,
                                                         int32_t *__restrict__ hist) {
  __shared__ int h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n_chunks; q += (int64_t)gridDim.x * 256) {
    const int i0 = item0 ? item0[q] : (int)q, P = item0 ? item0[q + 1] - i0 : 1;
    const int cost = max(1, act_cost[chunks[q].act_leaf] / P);
    const int b = __clz(cost);  // larger cost, smaller bucket
    for (int p = 0; p < P; ++p) {
      items[i0 + p] = (int)(q << 4) | p;
      bucket_of[i0 + p] = b;
    }
    atomicAdd(&h[b], P);
  }
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void cost_bucket_scan_kernel(int32_t *hist) {
  if (threadIdx.x == 0) {
    int s = 0;
    for (int b = 0; b < 32; ++b) {
      const int v = hist[b];
      hist[b] = s;
      s += v;
    }
  }
}

// Slot of a lane's item in its bucket (valid lanes): the lanes of a wave
// with the same bucket take consecutive slots through one atomic per
// distinct bucket (per-lane atomics on the few bucket cursors serialise).
// Every lane of the wave calls it.
__device__ __forceinline__ int bucket_slot(int32_t *__restrict__ cursor, int bucket, bool valid) {
  const int lane = threadIdx.x & 63;
  int slot = -1;
  for (uint64_t todo = __ballot(valid); todo;) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int b = __shfl(bucket, leader, 64);
    const uint64_t m = __ballot(valid && bucket == b);
    int base = 0;
    if (lane == leader) base = atomicAdd(&cursor[b], __popcll(m));
    base = __shfl(base, leader, 64);
    if (valid && bucket == b) slot = base + rank_below(m);
    todo &= ~m;
  }
  return slot;
}

__global__ __launch_bounds__(256) void item_scatter_kernel(const int32_t *__restrict__ items,
                                                           const int32_t *__restrict__ bucket_of, int64_t n,
                                                           int32_t *__restrict__ cursor, int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int64_t q0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); q0 < n; q0 += (int64_t)gridDim.x * 256) {
    const int64_t q = q0 + lane;
    const bool valid = q < n;
    const int s = bucket_slot(cursor, valid ? bucket_of[q] : 0, valid);
    if (valid) out[s] = items[q];
  }
}

// Workgroups of a persistent launch: every CU filled to the occupancy its
// LDS allows (bytes per wave of the force variant, the larger of the two).
int persistent_grid_for(int n_cu, const LoopConfig &c) {
  static const int wave_bytes[5] = {6656, 13312, 23040, 36864, 65536};
  int per_cu = 163840 / (c.nw * wave_bytes[c.tile]);
  if (per_cu < 1) per_cu = 1;
  if (per_cu * c.nw > 32) per_cu = 32 / c.nw;
  return n_cu * per_cu;
}

unsigned grid_for_items(int64_t n) {
  int64_t g = ceil_div(n, 256);
  if (g > 4096) g = 4096;
  return (unsigned)(g < 1 ? 1 : g);
}

// The configuration for a pass: a tuned entry for this number of chunks if
// one exists, else a rule that keeps enough waves in flight.
LoopConfig choose_config(sph_ctx *ctx, int mode) {
  const int cls = tune_class(ctx->n_chunks);
  // the pass's own chunk-count class, else the nearest tuned class within a
  // factor of four in chunks (a time-stepping run tunes on one pass; its
  // partly active dense steps fall in the classes next to it)
  int tc = -1;
  for (int d = 0; d <= 2 && tc < 0; ++d) {
    if (cls + d < 32 && ctx->tune[mode][cls + d].valid) tc = cls + d;
    else if (cls - d >= 0 && ctx->tune[mode][cls - d].valid) tc = cls - d;
  }
  LoopConfig c;
  if (tc >= 0) {
    const auto &t = ctx->tune[mode][tc];
    c.nw = t.nw;
    c.tile = t.tile;
    c.ordered = t.ordered;
    c.persistent = t.persistent;
    c.split = t.split;
    return c;
  }
  c.split = ctx->prm.chunk_split;
  if (ctx->prm.waves_per_chunk > 0) {
    c.nw = ctx->prm.waves_per_chunk;
    const int cap = ctx->prm.cand_cap, lcap = ctx->prm.list_cap;
    if (c.nw == 1) c.tile = cap <= 128 && lcap <= 32 ? 0 : cap <= 256 && lcap <= 64 ? 1 : cap <= 512 && lcap <= 96 ? 2 : cap <= 1024 && lcap <= 128 ? 3 : 4;
    if (c.nw == 2) c.tile = cap <= 128 && lcap <= 32 ? 0 : cap <= 256 && lcap <= 64 ? 1 : 2;
    if (c.nw == 4) c.tile = cap <= 128 && lcap <= 32 ? 0 : 1;
    if (c.nw == 8) c.tile = 0;  // the one tile class whose eight waves fit the LDS
    return c;
  }
  // The loop is bound by instruction issue, and the smallest tile keeps the
  // most waves resident; with few chunks, more waves share one chunk.
  const int64_t nc = ctx->n_chunks;
  c.tile = 0;
  if (nc < 2048) {
    c.nw = 8, c.ordered = 1;
  } else if (nc < 8192) {
    c.nw = 4, c.ordered = 1;
  } else if (nc < 32768) {
    c.nw = 2;
  } else {
    c.nw = 1;
  }
  return c;
}

}  // namespace

// Work items for a split target, in two phases so that several contexts can
// share one synchronisation: the count phase enqueues the parts per chunk,
// their scan and the copy of the total into *host_total; the fill phase
// writes the items in chunk order and in cost order and clears the arrival
// counters.  The costs come from the density cell-pair lists.
sph_status items_count(sph_ctx *ctx, int target, int32_t *host_total) {
  const int64_t nc = ctx->n_chunks;
  SPH_TRY(sph_ensure(ctx, ctx->chunk_item0, 4 * (size_t)(nc + 1)));
  SPH_TRY(sph_ensure(ctx, ctx->work_tmp, 4 * (size_t)(nc + 1) + 256));
  *host_total = 0;
  if (nc == 0) return SPH_OK;
  if (target == 0) {  // one item per chunk: nothing to count
    *host_total = (int32_t)nc;
    return SPH_OK;
  }
  int32_t *parts = (int32_t *)ctx->work_tmp.p + 64;
  PROF(ctx, "cost_order");
  split_count_kernel<<<grid_for_items(nc), 256, 0, ctx->stream>>>(
      (const Chunk *)ctx->chunks.p, nc, (const int32_t *)ctx->act_cost.p, (const int32_t *)ctx->dpair_off.p, target,
      parts);
  HIP_TRY(ctx, hipGetLastError());
  int32_t *i0 = (int32_t *)ctx->chunk_item0.p;
  SPH_TRY(scan_exclusive_i32(ctx, parts, i0, nc, i0 + nc));
  HIP_TRY(ctx, hipMemcpyAsync(host_total, i0 + nc, 4, hipMemcpyDeviceToHost, ctx->stream));
  return SPH_OK;
}

sph_status items_fill(sph_ctx *ctx, int target, int32_t total) {
  const int64_t nc = ctx->n_chunks;
  ctx->n_items = total;
  ctx->items_target = target;
  ctx->work_valid = 1;
  if (nc == 0) return SPH_OK;
  SPH_TRY(sph_ensure(ctx, ctx->items_nat, 4 * (size_t)total));
  SPH_TRY(sph_ensure(ctx, ctx->work, 4 * (size_t)total));
  SPH_TRY(sph_ensure(ctx, ctx->work_tmp, 4 * (size_t)(total > nc + 1 ? total : nc + 1) + 256));
  SPH_TRY(sph_ensure(ctx, ctx->chunk_ctr, 4 * (size_t)nc));
  if (target > 0) SPH_TRY(sph_ensure(ctx, ctx->partials, sizeof(float) * 11 * 64 * (size_t)total));
  int32_t *hist = (int32_t *)ctx->work_tmp.p;
  int32_t *bucket_of = hist + 64;
  HIP_TRY(ctx, hipMemsetAsync(hist, 0, 32 * sizeof(int32_t), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(ctx->chunk_ctr.p, 0, 4 * (size_t)nc, ctx->stream));
  PROF(ctx, "cost_order");
  split_fill_kernel<<<grid_for_items(nc), 256, 0, ctx->stream>>>(
      (const Chunk *)ctx->chunks.p, nc, (const int32_t *)ctx->act_cost.p,
      target > 0 ? (const int32_t *)ctx->chunk_item0.p : nullptr, (int32_t *)ctx->items_nat.p, bucket_of, hist);
  cost_bucket_scan_kernel<<<1, 64, 0, ctx->stream>>>(hist);
  item_scatter_kernel<<<grid_for_items(total), 256, 0, ctx->stream>>>(
      (const int32_t *)ctx->items_nat.p, bucket_of, total, hist, (int32_t *)ctx->work.p);
  return sph_hip_check(ctx, hipGetLastError(), "work items");
}

sph_status ensure_items(sph_ctx *ctx, int target) {
  if (ctx->work_valid && ctx->items_target == target) return SPH_OK;
  int32_t *total = ctx->pin_h + PIN_ITEMS;
  SPH_TRY(items_count(ctx, target, total));
  if (ctx->n_chunks > 0 && target > 0) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return items_fill(ctx, target, *total);
}

// The loop arguments' work list for a configuration (items built if needed).
sph_status apply_config(sph_ctx *ctx, const LoopConfig &cfg, LoopArgs &a) {
  const int target = split_target(cfg.split);
  a.work = nullptr;
  a.chunk_item0 = nullptr;
  a.chunk_ctr = nullptr;
  a.partials = nullptr;
  if (!cfg.ordered && target == 0) return SPH_OK;
  SPH_TRY(ensure_items(ctx, target));
  a.work = cfg.ordered ? (const int32_t *)ctx->work.p : (const int32_t *)ctx->items_nat.p;
  a.n_items = ctx->n_items;
  if (target > 0) {
    a.chunk_item0 = (const int32_t *)ctx->chunk_item0.p;
    a.chunk_ctr = (int32_t *)ctx->chunk_ctr.p;
    a.partials = (float *)ctx->partials.p;
  }
  return SPH_OK;
}

namespace {

template <int MODE, bool COMP>
sph_status launch_loop(sph_ctx *ctx, const LoopArgs &a0) {
  const LoopConfig cfg = choose_config(ctx, MODE);
  LoopArgs a = a0;
  SPH_TRY(apply_config(ctx, cfg, a));
  PROF(ctx, MODE == 0 ? "density_loop" : "force_loop");
  if (cfg.persistent) {
    // one box through the persistent kernel: a device copy of the arguments
    // and a (0, item) work list
    const int64_t ni = a.work ? a.n_items : ctx->n_chunks;
    SPH_TRY(sph_ensure(ctx, ctx->box_args, sizeof(LoopArgs)));
    SPH_TRY(sph_ensure(ctx, ctx->box_work, sizeof(int2) * (size_t)(ni > 0 ? ni : 1)));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->box_args.p, &a, sizeof(LoopArgs), hipMemcpyHostToDevice, ctx->stream));
    fill_work_kernel<<<grid_for_items(ni), 256, 0, ctx->stream>>>(a.work, ni, (int2 *)ctx->box_work.p);
    HIP_TRY(ctx, hipGetLastError());
    return sph_hip_check(ctx,
                         launch_loop_any<MODE, COMP>(ctx->stream, a, cfg, (const LoopArgs *)ctx->box_args.p,
                                                     (const int2 *)ctx->box_work.p, (int)ni,
                                                     (int *)ctx->scalars.p + SC_WORKCTR, persistent_grid_for(ctx->n_cu, cfg)),
                         MODE == 0 ? "density loop" : "force loop");
  }
  return sph_hip_check(ctx, launch_loop_any<MODE, COMP>(ctx->stream, a, cfg, nullptr, nullptr, 0, nullptr, 0),
                       MODE == 0 ? "density loop" : "force loop");
}

}  // namespace

LoopArgs base_args(sph_ctx *ctx) {
  LoopArgs a;
  memset(&a, 0, sizeof a);
  a.chunks = (const Chunk *)ctx->chunks.p;
  a.chunk_todo = (int32_t *)ctx->chunk_todo.p;
  a.n_chunks = ctx->n_chunks;
  a.active_idx = (const int32_t *)ctx->active_idx.p;
  a.pos4 = (const float4 *)ctx->pos4.p;
  a.jvm = (const float4 *)ctx->jvm.p;
  a.jth = (const float4 *)ctx->jth.p;
  a.leaf_begin = (const int32_t *)ctx->leaf_begin.p;
  a.leaf_count = (const int32_t *)ctx->leaf_count.p;
  a.leaf_hmax = (const float *)ctx->leaf_hmax.p;
  a.leaf_half = (const float *)ctx->leaf_half.p;
  a.gbox_lo = (const float4 *)ctx->gbox_lo.p;
  a.gbox_hi = (const float4 *)ctx->gbox_hi.p;
  a.leaf_dx = (const float *)ctx->leaf_dx.p;
  a.axis_order = (const uint16_t *)ctx->axis_order.p;
  a.leaf_hgrow = (const float *)ctx->leaf_hgrow.p;
  a.leaf_hq = (const float4 *)ctx->leaf_hq.p;
  a.n = ctx->n;
  a.ax = host_axes();
  a.n_active = ctx->n_active;
  a.half_alpha = 0.5f * ctx->prm.alpha;
  a.gm1 = (float)(ctx->prm.gamma - 1.0);
  return a;
}

// Per-particle neighbour data in cell order, packed once per build: velocity
// and mass, and the density-loop state (rho, f P/rho^2, c, B) that inactive
// neighbours keep from their last active step.  The ghost refreshes the
// latter for every active particle it finishes.
sph_status pack_args(sph_ctx *ctx, const sph_particles *p, PackArgs *a, bool *ok) {
  const int64_t n = ctx->n;
  SPH_TRY(sph_ensure(ctx, ctx->jvm, 16 * (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->jth, 16 * (size_t)n));
  *ok = p->vx && p->vy && p->vz && p->m && p->rho && p->f_gradh && p->P && p->c && p->balsara;
  a->vx = p->vx;
  a->vy = p->vy;
  a->vz = p->vz;
  a->m = p->m;
  a->rho = p->rho;
  a->f = p->f_gradh;
  a->P = p->P;
  a->c = p->c;
  a->B = p->balsara;
  a->jvm = (float4 *)ctx->jvm.p;
  a->jth = (float4 *)ctx->jth.p;
  return SPH_OK;
}

sph_status pack_neighbour_data(sph_ctx *ctx, const sph_particles *p) {
  const int64_t n = ctx->n;
  PackArgs pa;
  bool all;
  SPH_TRY(pack_args(ctx, p, &pa, &all));
  if (all) {
    {
      PROF(ctx, "pack");
      pack_kernel<<<grid256(n), 256, 0, ctx->stream>>>(pa, n);
    }
    return sph_hip_check(ctx, hipGetLastError(), "pack_kernel");
  }
  if (p->vx && p->vy && p->vz && p->m) {
    {
      PROF(ctx, "pack");
      pack_jvm_kernel<<<grid256(n), 256, 0, ctx->stream>>>(p->vx, p->vy, p->vz, p->m, n, (float4 *)ctx->jvm.p);
    }
    HIP_TRY(ctx, hipGetLastError());
  } else {
    HIP_TRY(ctx, hipMemsetAsync(ctx->jvm.p, 0, 16 * (size_t)n, ctx->stream));
  }
  if (p->rho && p->f_gradh && p->P && p->c && p->balsara) {
    {
      PROF(ctx, "pack");
      pack_jth_kernel<<<grid256(n), 256, 0, ctx->stream>>>(p->rho, p->f_gradh, p->P, p->c, p->balsara, n,
                                                          (float4 *)ctx->jth.p);
    }
    HIP_TRY(ctx, hipGetLastError());
  } else {
    HIP_TRY(ctx, hipMemsetAsync(ctx->jth.p, 0, 16 * (size_t)n, ctx->stream));
  }
  return SPH_OK;
}

struct GhostArgs {
  int64_t n_active;
  const int32_t *active_idx, *chunk_of;
  const Chunk *chunks;
  int32_t *chunk_todo;
  const float *sums;
  const int32_t *act_cnt;
  const float *act_reach;  // per active leaf: the radius its density cell-pair list is complete for
  float *hlo, *hhi;
  uint8_t *conv;
  float4 *pos4;
  float4 *jth;
  float *h;
  int last;
  int from_u;
  float eta3, kc, tol, gamma, eps, box_quarter;
  // outputs
  float *rho, *drho_dh, *f, *divv, *curlx, *curly, *curlz, *P, *c, *B, *A, *u;
  float *Af;  // (opt) the kicked copy of A, set with A when u is the thermal input
  int32_t *nngb;
  int32_t *n_unconv, *rebuild;
  unsigned long long *ctr;  // cumulative density interactions of finished solves
  int32_t *todo, *todo_n;   // (opt) appends the particles the next pass evaluates
};

// One Newton step of the h solve from the sums at h: sum_j w(q_ij) (S_w) and
// sum_j (3 w + q w') (S_d), with the bracket [lo, hi] of the root.  Newton in
// ln h on G = ln(h^3 n / eta^3), with h^3 n = (8/pi)/GK^3 sum w and
// dG/dln h = (3 sum w - sum (3w + q w')) / sum w: the same root as
// h^3 n = eta^3, reached in one step where the density is locally uniform.
// The ghost and the sweep's own steps share it, so that both take bitwise
// the same step from the same sums.
struct HStep {
  float hn, lo, hi;
  bool done;  // |hn - h| < tol h: h is the solution
};
__device__ __forceinline__ HStep h_newton_step(float S_w, float S_d, float h, float lo, float hi, float kc,
                                               float eta3, float tol) {
  const float hn3 = kc * S_w;
  const float G = __logf(hn3 / eta3);
  const float Gp = (3.f * S_w - S_d) / S_w;
  if (G < 0.f) lo = fmaxf(lo, h);
  if (G > 0.f) hi = fminf(hi, h);
  float hn = h * __expf(fminf(fmaxf(-G / Gp, -0.6931472f), 0.6931472f));
  // a step that lands on (or beyond) an end of the bracket falls back to
  // bisection: a clamped step of exactly x2 / x0.5 between two earlier
  // iterates would otherwise cycle
  const bool small = Gp > 0.f && fabsf(hn - h) < tol * h;
  if (!small && (!(hn > lo && hn < hi) || !(Gp > 0.f))) hn = (hi < INFINITY) ? 0.5f * (lo + hi) : 2.f * h;
  if (G == 0.f) hn = h;
  HStep r;
  r.hn = hn;
  r.lo = lo;
  r.hi = hi;
  r.done = fabsf(hn - h) < tol * h;
  return r;
}

// Newton step on F(h) = h^3 sum_j W(r_ij, h) - eta^3 for each active particle
// not yet converged; converged (or last-pass) particles get their ghost
// quantities written.
__device__ __forceinline__ void ghost_body(const GhostArgs &g) {
  int finished = 0;
  int unconv = 0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < g.n_active; k += (int64_t)gridDim.x * 256) {
    // finished and waiting particles read nothing more (after the first
    // pass most are finished); for the others every load that does not
    // depend on another is issued first (a chain of dependent loads)
    const uint8_t cv = g.conv[k];
    // whether the next pass evaluates particle k
    const bool again = [&]() -> bool {
    if (cv == 1) return false;
    if (cv == 2) {  // waiting for wider cell-pair lists: not converged
      ++unconv;
      return false;
    }
    const int i = g.active_idx[k];
    const int co = g.chunk_of[k];
    const float lo0 = g.hlo[k], hi0 = g.hhi[k];
    const int64_t na = g.n_active;
    const float S_w = g.sums[k], S_mw = g.sums[na + k], S_d = g.sums[2 * na + k], S_md = g.sums[3 * na + k];
    const float S_dv = g.sums[4 * na + k], S_cx = g.sums[5 * na + k], S_cy = g.sums[6 * na + k],
                S_cz = g.sums[7 * na + k];
    const int cnt_k = g.act_cnt[k];
    const float h = g.h[i];
    const Chunk ch = g.chunks[co];
    const HStep st = h_newton_step(S_w, S_d, h, lo0, hi0, g.kc, g.eta3, g.tol);
    const float hn = st.hn, lo = st.lo, hi = st.hi;
    const bool done = st.done;
    if (done || g.last) {
      const float H = GK32 * h;
      const float iH = 1.f / H;
      const float C3 = KNORM32 * iH * iH * iH;
      const float rho = C3 * S_mw;
      const float drho = -C3 / h * S_md;
      const float fg = 1.f / (1.f + h / (3.f * rho) * drho);
      float P, A, u;
      const float rg = __powf(rho, g.gamma);
      if (g.from_u) {
        u = g.u[i];
        P = (g.gamma - 1.f) * rho * u;
        A = P / rg;
        g.A[i] = A;
        if (g.Af) g.Af[i] = A;
      } else {
        A = g.A[i];
        P = A * rg;
        u = P / ((g.gamma - 1.f) * rho);
        if (g.u) g.u[i] = u;
      }
      const float cs = sqrtf(g.gamma * P / rho);
      const float C4 = C3 * iH;
      const float dv = -C4 * S_dv / rho;
      const float cx = C4 * S_cx / rho;
      const float cy = C4 * S_cy / rho;
      const float cz = C4 * S_cz / rho;
      const float adv = fabsf(dv);
      const float acu = sqrtf(fmaf(cz, cz, fmaf(cy, cy, cx * cx)));
      const float Bs = adv > 0.f ? adv / (adv + acu + g.eps * cs / h) : 0.f;
      g.rho[i] = rho;
      g.drho_dh[i] = drho;
      g.f[i] = fg;
      g.divv[i] = dv;
      g.curlx[i] = cx;
      g.curly[i] = cy;
      g.curlz[i] = cz;
      g.P[i] = P;
      g.c[i] = cs;
      g.B[i] = Bs;
      if (g.nngb) g.nngb[i] = cnt_k;
      g.jth[i] = make_float4(rho, fg * P / (rho * rho), cs, Bs);
      finished += cnt_k;
      g.conv[k] = 1;
      if (!done) ++unconv;
      return false;
    }
    const float Hn = GK32 * hn;
    bool wait = false;
    if (Hn > g.act_reach[ch.act_leaf]) {
      // beyond the reach of the cell-pair lists: the particle waits (no
      // evaluation) until they are widened, so that every evaluation sees
      // all its neighbours
      atomicOr(g.rebuild, 1);
      g.conv[k] = 2;
      wait = true;
    }
    if (Hn > g.box_quarter) atomicOr(g.rebuild, 2);
    g.hlo[k] = lo;
    g.hhi[k] = hi;
    g.h[i] = hn;
    g.pos4[i].w = Hn;
    g.chunk_todo[co] = 1;
    ++unconv;
    return !wait;
    }();
    if (g.todo) {
      // one append per wave (lane 0 holds the wave's lowest k, so it is in
      // the loop whenever any lane is)
      const uint64_t m = __ballot(again);
      int base = 0;
      if ((threadIdx.x & 63) == 0 && m) base = atomicAdd(g.todo_n, __popcll(m));
      base = __shfl(base, 0, 64);
      if (again) g.todo[base + rank_below(m)] = (int32_t)k;
    }
  }
  // one pair of counter updates per block (every block reaches this point)
  finished = wave_sum_i(finished);
  unconv = wave_sum_i(unconv);
  __shared__ int bf[4], bu[4];
  if ((threadIdx.x & 63) == 0) {
    bf[threadIdx.x >> 6] = finished;
    bu[threadIdx.x >> 6] = unconv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int f = bf[0] + bf[1] + bf[2] + bf[3], u = bu[0] + bu[1] + bu[2] + bu[3];
    if (f) atomicAdd(g.ctr, (unsigned long long)f);
    if (u) atomicAdd(g.n_unconv, u);
  }
}

__global__ __launch_bounds__(256) void ghost_kernel(GhostArgs g) { ghost_body(g); }

// Several boxes in one launch: box blockIdx.y.
__global__ __launch_bounds__(256) void ghost_multi_kernel(const GhostArgs *__restrict__ boxes) {
  const GhostArgs g = boxes[blockIdx.y];
  ghost_body(g);
}

// Density loop, one wave per particle: for Newton passes with few particles
// left (and deep time-bins, whose chunks hold few active particles).  The
// partner leaves of at most 128 particles (and the particle's own leaf) are
// read as one flat candidate range, 64 candidates per step across leaves, so
// that their loads are issued together; larger partner leaves are swept in
// the order of their sort along the stencil axis nearest to the pair offset
// (the paper's sorted sweep), from the side facing the particle to past its
// reach.  Same predicate, per-pair terms and outputs as the chunk loop (sums
// per active index, count); the lanes' sums are reduced in a fixed butterfly.
struct SweepPair {
  int off, bb;
  float sx, sy, sz;
  int hord;  // nonzero: the range is the head of the leaf's H order, not the leaf itself
};

// Logical block of a sweep launch whose grid is a multiple of 8: the blocks
// the dispatcher sends to one XCD (blockIdx % 8) take one contiguous range of
// the nblk blocks of work, so particles that share partner leaves read them
// from the same L2.  Returns -1 for a block beyond the work.
__device__ __forceinline__ int64_t xcd_block(int64_t nblk) {
  const int64_t per = (nblk + 7) >> 3;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  return lb < nblk ? lb : -1;
}

static unsigned xcd_grid(int64_t nblk) { return (unsigned)(8 * std::max<int64_t>(1, (nblk + 7) / 8)); }

// The partners of up to 64 cell pairs (one per lane) that a wave reads as one
// flat candidate range: those with `small` set, compacted into `my` in lane
// order with their first flat index.  ns entries; steps = ceil(log2(ns)).
struct FlatRange {
  int total, ns, steps;
};

__device__ __forceinline__ FlatRange compact_small(SweepPair *my, bool small, int bc, int bb, const PairEntry &e,
                                                   int lane, bool hord = false) {
  const int n_small = small ? bc : 0;
  int incl = n_small;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  FlatRange r;
  r.total = __shfl(incl, 63, 64);
  const uint64_t m = __ballot(small);
  r.ns = __popcll(m);
  r.steps = 0;
  while ((1 << r.steps) < r.ns) ++r.steps;
  wave_sync();  // earlier readers of `my` are done
  if (small) {
    SweepPair q;
    q.off = incl - n_small;
    q.bb = bb;
    q.sx = e.sx;
    q.sy = e.sy;
    q.sz = e.sz;
    q.hord = hord ? 1 : 0;
    my[rank_below(m)] = q;
  }
  wave_sync();
  return r;
}

// The compacted partner whose flat range holds index f (offsets increase
// strictly: every leaf holds a particle).
__device__ __forceinline__ SweepPair locate(const SweepPair *my, const FlatRange &r, int f) {
  int lo = 0;
  for (int s = r.steps - 1; s >= 0; --s) {
    const int mid = lo + (1 << s);
    if (mid < r.ns && my[mid].off <= f) lo = mid;
  }
  return my[lo];
}

// A value every lane of the wave holds alike, moved to a scalar register.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ float4 wave_uniform(float4 v) {
  return make_float4(wave_uniform(v.x), wave_uniform(v.y), wave_uniform(v.z), wave_uniform(v.w));
}

// A partner leaf of the flat range, for the group-by-group test.
struct GroupPart {
  int goff, bb, bc, b;
  float sx, sy, sz, m;  // shift into the particle's frame; drift margin
};

// Whether the 8-particle group `slot` of a partner leaf (box of the full
// build, widened by the leaf's drift margin m, shifted into the particle's
// frame) can hold a particle within R of the particle at offset pi; the
// relative guard covers the FP32 rounding of the predicate as in
// leaf_in_reach.
__device__ __forceinline__ bool group_in_reach(const LoopArgs &g, int64_t slot, const GroupPart &q, const float4 &pi,
                                               float R) {
  const float4 lo = g.gbox_lo[slot], hi = g.gbox_hi[slot];
  const float gx = fmaxf(fmaxf((lo.x + q.sx - q.m) - pi.x, pi.x - (hi.x + q.sx + q.m)), 0.f);
  const float gy = fmaxf(fmaxf((lo.y + q.sy - q.m) - pi.y, pi.y - (hi.y + q.sy + q.m)), 0.f);
  const float gz = fmaxf(fmaxf((lo.z + q.sz - q.m) - pi.z, pi.z - (hi.z + q.sz + q.m)), 0.f);
  const float Rg = 1.0001f * R + 1e-6f * (fabsf(pi.x) + fabsf(pi.y) + fabsf(pi.z) + fabsf(q.sx) + fabsf(q.sy) +
                                         fabsf(q.sz) + fmaxf(fabsf(lo.x), fabsf(hi.x)) + fmaxf(fabsf(lo.y), fabsf(hi.y)) +
                                         fmaxf(fabsf(lo.z), fabsf(hi.z)) + q.m);
  return fmaf(gz, gz, fmaf(gy, gy, gx * gx)) < Rg * Rg;
}

// Whether partner leaf e.b can hold a particle within R of the particle at
// offset pi: the distance from pi to the leaf's box (in the particle's leaf
// frame, widened by the leaf's drift margin) against R, with a relative
// guard for rounding.  The leaf's own cell-pair reach covers the union of
// its particles; this prunes per particle.
__device__ __forceinline__ bool leaf_in_reach(const LoopArgs &g, const PairEntry &e, const float4 &pi, float R) {
  const float hw = g.leaf_half[e.b] + g.leaf_dx[e.b];
  const float gx = fmaxf(fabsf(pi.x - e.sx) - hw, 0.f);
  const float gy = fmaxf(fabsf(pi.y - e.sy) - hw, 0.f);
  const float gz = fmaxf(fabsf(pi.z - e.sz) - hw, 0.f);
  const float Rg = 1.0001f * R + 1e-6f * (fabsf(pi.x) + fabsf(pi.y) + fabsf(pi.z) + hw);
  return fmaf(gz, gz, fmaf(gy, gy, gx * gx)) < Rg * Rg;
}

// Waves per particle of a sweep pass.  One wave per particle measured fastest
// on the deep-bin steps (the partial sums of several waves cost more in the
// merge than the extra waves gain in latency), so several are only taken on
// request.
int sweep_waves(const sph_ctx *ctx, int64_t n_todo) {
  (void)n_todo;
  return ctx->prm.sweep_waves > 0 ? ctx->prm.sweep_waves : 1;
}

// Compensated sums of the sweep kernels: a lane sums its own terms (a few
// per particle: a particle's neighbours are spread over the 64 lanes) in
// plain FP32, and the 64 lane partials are added in a butterfly whose every
// level is a TwoSum, the rounding errors carried in c; the waves sharing a
// particle are then added with Neumaier's update.  TwoSum's error term is
// exact, so both lanes of a butterfly level compute the same pair and every
// lane ends with the same total s + c.
__device__ __forceinline__ void neu_add(float &s, float &c, float b) {
  const float t = s + b;
  c += fabsf(s) >= fabsf(b) ? (s - t) + b : (b - t) + s;
  s = t;
}
__device__ __forceinline__ void two_sum_butterfly(float &s, float &c) {
  for (int o = 32; o > 0; o >>= 1) {
    const float s2 = __shfl_xor(s, o, 64), c2 = __shfl_xor(c, o, 64);
    const float t = s + s2;
    const float bp = t - s;
    const float e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = (c + c2) + e;
  }
}

__device__ __forceinline__ void density_term(const float4 &pi, const float4 &vi, float invHi, float dx, float dy,
                                             float dz, float r2, const float4 &vj, float (&acc)[8]) {
  const float rinv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
  const float r = r2 * rinv;
  const float vx = vi.x - vj.x, vy = vi.y - vj.y, vz = vi.z - vj.z;
  const float vr = fmaf(vz, dz, fmaf(vy, dy, vx * dx));
  const float mj = vj.w;
  float wq, wp;
  const float q = r * invHi;
  kernel_w_dw(q, wq, wp);
  const float d3 = fmaf(q, wp, 3.f * wq);
  acc[0] += wq;
  acc[1] = fmaf(mj, wq, acc[1]);
  acc[2] += d3;
  acc[3] = fmaf(mj, d3, acc[3]);
  const float fac = mj * wp * rinv;
  acc[4] = fmaf(fac, vr, acc[4]);
  acc[5] = fmaf(fac, fmaf(vy, dz, -vz * dy), acc[5]);
  acc[6] = fmaf(fac, fmaf(vz, dx, -vx * dz), acc[6]);
  acc[7] = fmaf(fac, fmaf(vx, dy, -vy * dx), acc[7]);
  (void)pi;
}

// The sweep's own steps of the h solve (one wave per particle).  The walk
// keeps every candidate within a cache radius Rc >= H (at most cache_f H, and
// within the radius the particle's cell-pair list is complete for) in LDS;
// the kernel then evaluates the sums at h from that cache, takes the Newton
// step while the new H stays within Rc, and evaluates again.  The step that
// ends the solve, or would leave the cache, is left to the ghost: the kernel
// writes the sums at the last h it evaluated and the solver state (h, its
// bracket) that step starts from, and the ghost takes it bitwise as the
// kernel would (the same function from the same sums).  A pass p takes at
// most h_max_iter - p steps of its own.
struct SweepSolve {
  int steps;  // Newton steps the kernel may take itself (0: none)
  float cache_f, kc, eta3, tol, box_quarter;
  const float *act_reach;  // per active leaf: radius the density cell-pair list is complete for
  float *h, *hlo, *hhi;
  float4 *pos4;  // H (w) follows h
  int32_t *chunk_todo;
};

// Entries of a wave's neighbour queue: with the cache at most SWEEP_QCAP - 64
// (more neighbours within Rc than that and the particle goes on without it).
#define SWEEP_QCAP 256

// NWP waves share one particle: wave s of it takes the flat candidates
// s*64 + NWP*64*t and every NWP-th large partner; the waves' sums are added
// in wave order.  The neighbours a wave finds are queued in LDS and their
// pair terms evaluated 64 at a time, one per lane, so that the terms run on
// full waves although few of the candidates tested together are neighbours
// (with one wave per particle and the solver's steps on, all of them are
// evaluated from the cache after the walk).
//
// Work: the particles todo[0 .. n_todo) (all active ones with todo null),
// or, with SCAN, the active particles k whose scan_conv[k] is 0, a wave
// taking 64 consecutive k (n_todo = ceil(n_active / 64)) and the particles
// among them one after the other.  With gate, the launch does nothing unless
// *gate < gate_min.
template <int NWP, bool COMP, bool SCAN = false>
__global__ __launch_bounds__(256) void density_sweep_kernel(LoopArgs g, const int32_t *__restrict__ todo,
                                                            const int32_t *__restrict__ n_todo_dev, int64_t n_todo,
                                                            const int32_t *__restrict__ chunk_of,
                                                            int32_t *__restrict__ next_n, SweepSolve sv,
                                                            const uint8_t *__restrict__ scan_conv,
                                                            const int32_t *__restrict__ gate, int32_t gate_min) {
  if (gate && *gate >= gate_min) return;
  __shared__ SweepPair sp[4][64];
  __shared__ GroupPart gpart[4][64];  // per wave: the small partners of the current 64 pairs
  __shared__ float4 hq[4][SWEEP_QCAP];  // per wave: queued neighbours (dx, dy, dz, j)
  __shared__ float red[4][9];
  const int wave = threadIdx.x >> 6;
  const int sub = wave % NWP;
  if (n_todo_dev) n_todo = *n_todo_dev;
  // the next pass's list starts empty (its ghost appends after this launch)
  if (next_n && blockIdx.x == 0 && threadIdx.x == 0) *next_n = 0;
  const int lane = threadIdx.x & 63;
  // grid-stride over the logical blocks of the particles to do (known on the
  // device only, so the grid is sized to the machine): the blocks the
  // dispatcher sends to one XCD (blockIdx % 8, the grid being a multiple of
  // 8) take one contiguous range, so particles sharing partner leaves read
  // them from the same L2
  const int64_t nblk = ceil_div(n_todo, 4 / NWP);
  const int64_t per = (nblk + 7) >> 3;
  for (int64_t bi = blockIdx.x; bi < 8 * per; bi += gridDim.x) {
  const int64_t lb = (bi & 7) * per + (bi >> 3);
  const int64_t w = lb < nblk ? lb * (4 / NWP) + wave / NWP : n_todo;
  if (w < n_todo) {
  // one particle, or with scan_conv those of the wave's 64 still to do
  uint64_t pend = 1ull;
  if (SCAN) {
    const int64_t kk = w * 64 + lane;
    pend = __ballot(kk < g.n_active && scan_conv[kk] == 0);
  }
  while (pend) {
  const int bit = __ffsll((unsigned long long)pend) - 1;
  pend = SCAN ? pend & (pend - 1) : 0ull;
  SweepPair *my = sp[wave];
  // the particle's values are the same on every lane: scalar registers
  const int k = wave_uniform(SCAN ? (int)(w * 64) + bit : (todo ? todo[w] : (int)w));
  const int i = wave_uniform(g.active_idx[k]);
  const float4 pi = wave_uniform(g.pos4[i]);
  const float Hi = pi.w, H2i = wave_uniform(Hi * Hi), invHi = wave_uniform(1.f / Hi);
  const float4 vi = wave_uniform(g.jvm[i]);
  const int co = wave_uniform(chunk_of[k]);
  const Chunk ch = g.chunks[co];
  const int pbeg = wave_uniform(g.pair_off[ch.act_leaf]), pend = wave_uniform(g.pair_off[ch.act_leaf + 1]);
  // the solver's own steps: cache radius and the state the steps start from
  const bool cache_on = NWP == 1 && sv.steps > 0;
  bool caching = cache_on;
  // radius of the walk: the cache radius Rc while caching, else H
  float Rw = wave_uniform(cache_on ? fmaxf(Hi, fminf(sv.cache_f * Hi, sv.act_reach[ch.act_leaf])) : Hi);
  float Rw2 = wave_uniform(Rw * Rw);
  float acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.f;
  int cnt = 0;
  float4 *Q = hq[wave];
  int qn = 0;  // queue length (wave-uniform)
  // pair terms of queue entries base + lane (lane < m) within H
  auto drain = [&](int base, int m) {
    if (lane < m) {
      const float4 e = Q[base + lane];
      const int j = __float_as_int(e.w);
      const float r2 = fmaf(e.z, e.z, fmaf(e.y, e.y, e.x * e.x));
      if (r2 < H2i) {
        density_term(pi, vi, invHi, e.x, e.y, e.z, r2, g.jvm[j], acc);
        cnt += (j != i);
      }
    }
  };
  // queue the lanes' hits; without the cache a full wave of them is
  // evaluated at once
  auto push = [&](bool hit, float dx, float dy, float dz, int j) {
    const uint64_t m = __ballot(hit);
    if (m == 0ull) return;
    if (hit) Q[qn + rank_below(m)] = make_float4(dx, dy, dz, __int_as_float(j));
    qn += __popcll(m);
    if (caching) {
      if (qn > SWEEP_QCAP - 64) {
        // more candidates within Rc than the cache holds: those within H
        // are evaluated and the walk goes on at H, without the cache
        wave_sync();
        for (int b = 0; b < qn; b += 64) drain(b, min(64, qn - b));
        wave_sync();
        qn = 0;
        caching = false;
        Rw = Hi;
        Rw2 = H2i;
      }
    } else if (qn >= 64) {
      wave_sync();
      drain(0, 64);
      const int rest = qn - 64;
      float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
      if (lane < rest) t = Q[64 + lane];
      wave_sync();
      if (lane < rest) Q[lane] = t;
      wave_sync();
      qn = rest;
    }
  };
  for (int p0 = pbeg; p0 < pend; p0 += 64) {
    const int p = p0 + lane;
    PairEntry e;
    e.b = 0;
    e.sx = e.sy = e.sz = 0.f;
    int bb = 0, bc = 0;
    bool near = false;
    if (p < pend) {
      e = g.pairs[p];
      bb = g.leaf_begin[e.b];
      bc = g.leaf_count[e.b];
      near = leaf_in_reach(g, e, pi, Rw);
    }
    const bool big = near && e.b != ch.leaf && bc > 128;
    int axl = 0;
    float sgl = 1.f;
    if (big) {
      const uint8_t code = g.pair_axis[p];
      axl = code & 0x7f;
      sgl = (code & 0x80) ? -1.f : 1.f;
    }
    // The small partners within reach, tested group by group: 64 groups of 8
    // particles per round (one per lane) against the particle's sphere, the
    // groups within reach then read as one flat candidate range.
    const bool sm = near && !big;
    const int ng = sm ? (bc + 7) >> 3 : 0;
    int ginc = ng;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(ginc, o, 64);
      if (lane >= o) ginc += v;
    }
    const int tg = __shfl(ginc, 63, 64);
    const uint64_t smask = __ballot(sm);
    const int nsm = __popcll(smask);
    int gsteps = 0;
    while ((1 << gsteps) < nsm) ++gsteps;
    GroupPart *gp = gpart[wave];
    wave_sync();  // the previous batch's readers of gp are done
    if (sm) {
      GroupPart q;
      q.goff = ginc - ng;
      q.bb = bb;
      q.bc = bc;
      q.b = e.b;
      q.sx = e.sx;
      q.sy = e.sy;
      q.sz = e.sz;
      q.m = g.leaf_dx[e.b];
      gp[rank_below(smask)] = q;
    }
    wave_sync();
    for (int gb = 0; gb < tg; gb += 64) {
      const int fg = gb + lane;
      const bool gv = fg < tg;
      int k = 0;
      for (int st = gsteps - 1; st >= 0; --st) {
        const int mid = k + (1 << st);
        if (mid < nsm && gp[mid].goff <= fg) k = mid;
      }
      const GroupPart q = gp[k];
      const int gi = fg - q.goff;
      bool keep = false;
      if (gv) keep = group_in_reach(g, (int64_t)(q.bb >> 3) + q.b + gi, q, pi, Rw);
      PairEntry ge;
      ge.b = q.b;
      ge.sx = q.sx;
      ge.sy = q.sy;
      ge.sz = q.sz;
      const FlatRange fr = compact_small(my, keep, keep ? min(8, q.bc - 8 * gi) : 0, q.bb + 8 * gi, ge, lane);
      for (int t = sub * 64; t < fr.total; t += 2 * NWP * 64) {
        // two candidates per lane, their loads in flight together
        const int f0 = t + lane, f1 = t + NWP * 64 + lane;
        const bool v0 = f0 < fr.total, v1 = f1 < fr.total;
        const SweepPair q0 = locate(my, fr, v0 ? f0 : 0), q1 = locate(my, fr, v1 ? f1 : 0);
        const int j0 = q0.bb + (v0 ? f0 - q0.off : 0), j1 = q1.bb + (v1 ? f1 - q1.off : 0);
        const float4 pj0 = g.pos4[j0], pj1 = g.pos4[j1];
        const float dx0 = pi.x - (pj0.x + q0.sx), dy0 = pi.y - (pj0.y + q0.sy), dz0 = pi.z - (pj0.z + q0.sz);
        const float dx1 = pi.x - (pj1.x + q1.sx), dy1 = pi.y - (pj1.y + q1.sy), dz1 = pi.z - (pj1.z + q1.sz);
        push(v0 && fmaf(dz0, dz0, fmaf(dy0, dy0, dx0 * dx0)) < Rw2, dx0, dy0, dz0, j0);
        push(v1 && fmaf(dz1, dz1, fmaf(dy1, dy1, dx1 * dx1)) < Rw2, dx1, dy1, dz1, j1);
      }
    }
    // large partners, one after the other: sorted sweep
    uint64_t bigm = __ballot(big);
    int nb = 0;
    while (bigm) {
      const int src = __ffsll((unsigned long long)bigm) - 1;
      bigm &= bigm - 1;
      if ((nb++ % NWP) != sub) continue;
      const int bbq = __shfl(bb, src, 64), bcq = __shfl(bc, src, 64), Bq = __shfl(e.b, src, 64);
      const float sx = __shfl(e.sx, src, 64), sy = __shfl(e.sy, src, 64), sz = __shfl(e.sz, src, 64);
      // the partner's sweep axis, found by its own lane in the pair phase
      const int axis = __builtin_amdgcn_readfirstlane(__shfl(axl, src, 64));
      const float sgn = __shfl(sgl, src, 64);
      const float ex = g.ax.e[axis][0], ey = g.ax.e[axis][1], ez = g.ax.e[axis][2];
      const float pp = fmaf(pi.z, ez, fmaf(pi.y, ey, pi.x * ex));
      const float sproj = fmaf(sz, ez, fmaf(sy, ey, sx * ex));
      // orders are by the offsets of the full build (see the chunk loop)
      const float margin = 1.0001f * Rw + 2.0001f * g.leaf_dx[Bq] + 1e-6f * (2.f * fabsf(pp) + fabsf(sproj));
      const float lo_b = pp - margin - sproj, hi_b = pp + margin - sproj;
      const uint16_t *ord = g.axis_order + (int64_t)axis * g.n + bbq;
      // two tiles per step, their loads in flight together; the sweep stops
      // at the first tile wholly past the reach
      for (int t = 0; t < bcq; t += 128) {
        const int k0 = t + lane, k1 = t + 64 + lane;
        const bool v0 = k0 < bcq, v1 = k1 < bcq;
        const int j0 = bbq + (v0 ? (int)ord[sgn > 0.f ? k0 : bcq - 1 - k0] : 0);
        const int j1 = bbq + (v1 ? (int)ord[sgn > 0.f ? k1 : bcq - 1 - k1] : 0);
        const float4 pj0 = g.pos4[j0], pj1 = g.pos4[j1];
        const float key0 = fmaf(pj0.z, ez, fmaf(pj0.y, ey, pj0.x * ex));
        if (__ballot(v0 && !(sgn > 0.f ? key0 > hi_b : key0 < lo_b)) == 0ull) break;
        const float dx0 = pi.x - (pj0.x + sx), dy0 = pi.y - (pj0.y + sy), dz0 = pi.z - (pj0.z + sz);
        push(v0 && fmaf(dz0, dz0, fmaf(dy0, dy0, dx0 * dx0)) < Rw2, dx0, dy0, dz0, j0);
        const float key1 = fmaf(pj1.z, ez, fmaf(pj1.y, ey, pj1.x * ex));
        if (__ballot(v1 && !(sgn > 0.f ? key1 > hi_b : key1 < lo_b)) == 0ull) break;
        const float dx1 = pi.x - (pj1.x + sx), dy1 = pi.y - (pj1.y + sy), dz1 = pi.z - (pj1.z + sz);
        push(v1 && fmaf(dz1, dz1, fmaf(dy1, dy1, dx1 * dx1)) < Rw2, dx1, dy1, dz1, j1);
      }
    }
  }
  wave_sync();
  bool moved = false;
  float h_s = 0.f, lo_s = 0.f, hi_s = 0.f;
  if (caching) {
    const float Rc = Rw;
    h_s = sv.h[i];
    lo_s = sv.hlo[k];
    hi_s = sv.hhi[k];
    // the cache, entries lane + 64 u in registers (qn <= SWEEP_QCAP - 64)
    constexpr int NU = (SWEEP_QCAP - 64) / 64;
    float4 ce[NU], cv[NU];
    uint32_t notself = 0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int idx = lane + 64 * u;
      ce[u] = make_float4(0.f, 0.f, 0.f, INFINITY);
      cv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < qn) {
        const float4 e = Q[idx];
        const int j = __float_as_int(e.w);
        ce[u] = make_float4(e.x, e.y, e.z, fmaf(e.z, e.z, fmaf(e.y, e.y, e.x * e.x)));
        cv[u] = g.jvm[j];
        notself |= (j != i) ? (1u << u) : 0u;
      }
    }
    float H = Hi, H2 = H2i, iH = invHi;
    for (int left = sv.steps;; --left) {
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.f;
      cnt = 0;
#pragma unroll
      for (int u = 0; u < NU; ++u)
        if (ce[u].w < H2) {
          density_term(pi, vi, iH, ce[u].x, ce[u].y, ce[u].z, ce[u].w, cv[u], acc);
          cnt += (notself >> u) & 1u;
        }
      if (left == 0) break;
      // the two sums the step reads, totalled as below
      float Sw = acc[0], Sd = acc[2];
      if (COMP) {
        float c0 = 0.f, c2 = 0.f;
        two_sum_butterfly(Sw, c0);
        two_sum_butterfly(Sd, c2);
        Sw += c0;
        Sd += c2;
      } else {
        for (int o = 32; o > 0; o >>= 1) {
          Sw += __shfl_xor(Sw, o, 64);
          Sd += __shfl_xor(Sd, o, 64);
        }
      }
      const HStep st = h_newton_step(Sw, Sd, h_s, lo_s, hi_s, sv.kc, sv.eta3, sv.tol);
      if (st.done) break;
      const float Hn = GK32 * st.hn;
      if (!(Hn <= Rc) || Hn > sv.box_quarter) break;  // the ghost takes this step
      h_s = st.hn;
      lo_s = st.lo;
      hi_s = st.hi;
      moved = true;
      H = Hn;
      H2 = H * H;
      iH = 1.f / H;
    }
  } else {
    for (int b = 0; b < qn; b += 64) drain(b, min(64, qn - b));
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (COMP) {
      float c = 0.f;
      two_sum_butterfly(acc[q], c);
      acc[q] += c;
    } else {
      float v = acc[q];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      acc[q] = v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (NWP == 1) {
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) g.sums[(int64_t)q * g.n_active + k] = acc[q];
      g.act_cnt[k] = cnt;
      if (moved) {
        // the state the ghost's step starts from
        sv.h[i] = h_s;
        sv.pos4[i].w = GK32 * h_s;
        sv.hlo[k] = lo_s;
        sv.hhi[k] = hi_s;
        sv.chunk_todo[co] = 1;
      }
    }
  } else {
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) red[wave][q] = acc[q];
      red[wave][8] = __int_as_float(cnt);
    }
  }
  wave_sync();  // the next particle of the wave reuses its LDS
  }
  }
  if (NWP > 1) {
    __syncthreads();
    if (sub == 0 && lane == 0 && w < n_todo) {
      const int k = todo ? todo[w] : (int)w;
      float s[8], c[8];
      int cs = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) s[q] = c[q] = 0.f;
      for (int u = 0; u < NWP; ++u) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (COMP)
            neu_add(s[q], c[q], red[wave + u][q]);
          else
            s[q] += red[wave + u][q];
        }
        cs += __float_as_int(red[wave + u][8]);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s[q] += c[q];
#pragma unroll
      for (int q = 0; q < 8; ++q) g.sums[(int64_t)q * g.n_active + k] = s[q];
      g.act_cnt[k] = cs;
    }
    __syncthreads();  // red is reused by the next logical block
  }
  }
}

// Force loop, one wave per active particle (as the density sweep): partner
// leaves of at most 128 particles and the own leaf as one flat candidate
// range, larger ones swept in their axis order up to max(H_i, that leaf's max
// H).  Same predicate (j != i, r < max(H_i, H_j)), pair terms and outputs as
// the chunk loop; neighbours queued in LDS and evaluated a full wave at a
// time (as in the density sweep); lane sums reduced in a fixed butterfly,
// v_sig by max.
struct ForceAcc {
  float ax, ay, az, visc, adiab, vmax;
};

__device__ __forceinline__ void force_term(const float4 &vi, const float4 &thi, float invHi, float half_alpha,
                                           float dx, float dy, float dz, float r2, float Hj, const float4 &vj,
                                           const float4 &th, ForceAcc &f) {
  const float rinv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
  const float r = r2 * rinv;
  const float invHj = __builtin_amdgcn_rcpf(Hj);
  const float vx = vi.x - vj.x, vy = vi.y - vj.y, vz = vi.z - vj.z;
  const float vr = fmaf(vz, dz, fmaf(vy, dy, vx * dx));
  const float mj = vj.w;
  const float wpi = kernel_dw_only(r * invHi);
  const float wpj = kernel_dw_only(r * invHj);
  const float ih2 = invHj * invHj;
  const float Fi = (KNORM32 * invHi * invHi * invHi * invHi) * wpi * rinv;
  const float Fj = KNORM32 * (ih2 * ih2) * wpj * rinv;
  const float mu = fminf(vr * rinv, 0.f);
  const float vsig = thi.z + th.z - 3.f * mu;
  f.vmax = fmaxf(f.vmax, vsig);
  const float Pi = -half_alpha * vsig * mu * (thi.w + th.w) * __builtin_amdgcn_rcpf(thi.x + th.x);
  const float gbar = 0.5f * (Fi + Fj);
  const float coef = mj * fmaf(thi.y, Fi, fmaf(th.y, Fj, Pi * gbar));
  f.ax = fmaf(-coef, dx, f.ax);
  f.ay = fmaf(-coef, dy, f.ay);
  f.az = fmaf(-coef, dz, f.az);
  f.visc = fmaf(mj * Pi * vr, gbar, f.visc);
  f.adiab = fmaf(mj * vr, Fi, f.adiab);
}

template <int NWP, bool COMP>
__global__ __launch_bounds__(256) void force_sweep_kernel(LoopArgs g, const int32_t *__restrict__ chunk_of) {
  __shared__ SweepPair sp[4][64];
  __shared__ float4 hq[4][128];  // per wave: queued neighbours (dx, dy, dz, j) and their H
  __shared__ float hqH[4][128];
  __shared__ int blk_cnt[4];
  __shared__ float red[4][7];
  const int wave = threadIdx.x >> 6;
  const int sub = wave % NWP;
  const int lane = threadIdx.x & 63;
  const int64_t lb = xcd_block(ceil_div(g.n_active, 4 / NWP));
  const int64_t k = lb < 0 ? g.n_active : lb * (4 / NWP) + wave / NWP;
  int cnt = 0;
  if (k < g.n_active) {
    SweepPair *my = sp[wave];
    // the particle's values are the same on every lane: scalar registers
    const int i = wave_uniform(g.active_idx[k]);
    const float4 pi = wave_uniform(g.pos4[i]);
    const float Hi = pi.w, H2i = wave_uniform(Hi * Hi), invHi = wave_uniform(1.f / Hi);
    const float4 vi = wave_uniform(g.jvm[i]);
    const float4 thi = wave_uniform(g.jth[i]);
    const Chunk ch = g.chunks[wave_uniform(chunk_of[k])];
    const int pbeg = wave_uniform(g.pair_off[ch.act_leaf]), pend = wave_uniform(g.pair_off[ch.act_leaf + 1]);
    ForceAcc f = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float4 *Q = hq[wave];
    float *QH = hqH[wave];
    int qn = 0;  // queue length (wave-uniform)
    auto drain = [&](int m) {
      if (lane < m) {
        const float4 e = Q[lane];
        const int j = __float_as_int(e.w);
        const float r2 = fmaf(e.z, e.z, fmaf(e.y, e.y, e.x * e.x));
        force_term(vi, thi, invHi, g.half_alpha, e.x, e.y, e.z, r2, QH[lane], g.jvm[j], g.jth[j], f);
        ++cnt;
      }
    };
    // tests candidate j at pj (valid lanes) and queues it if it is a neighbour
    auto visit = [&](bool valid, int j, const float4 &pj, float sx, float sy, float sz) {
      const float dx = pi.x - (pj.x + sx), dy = pi.y - (pj.y + sy), dz = pi.z - (pj.z + sz);
      const float Hj = pj.w;
      const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      const bool hit = valid && (r2 < H2i || r2 < Hj * Hj) && j != i;
      const uint64_t m = __ballot(hit);
      if (m == 0ull) return;
      if (hit) {
        const int s = qn + rank_below(m);
        Q[s] = make_float4(dx, dy, dz, __int_as_float(j));
        QH[s] = Hj;
      }
      qn += __popcll(m);
      if (qn >= 64) {
        wave_sync();
        drain(64);
        const int rest = qn - 64;
        float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
        float th = 0.f;
        if (lane < rest) {
          t = Q[64 + lane];
          th = QH[64 + lane];
        }
        wave_sync();
        if (lane < rest) {
          Q[lane] = t;
          QH[lane] = th;
        }
        wave_sync();
        qn = rest;
      }
    };
    for (int p0 = pbeg; p0 < pend; p0 += 64) {
      const int p = p0 + lane;
      PairEntry e;
      e.b = 0;
      e.sx = e.sy = e.sz = 0.f;
      int bb = 0, bc = 0, nflat = 0;
      bool near = false, head = false;
      if (p < pend) {
        e = g.pairs[p];
        bb = g.leaf_begin[e.b];
        bc = g.leaf_count[e.b];
        nflat = bc;
        // distance from pi to the leaf's box (widened by its drift margin),
        // with the relative rounding guard of leaf_in_reach
        const float hw = g.leaf_half[e.b] + g.leaf_dx[e.b];
        const float gx = fmaxf(fabsf(pi.x - e.sx) - hw, 0.f);
        const float gy = fmaxf(fabsf(pi.y - e.sy) - hw, 0.f);
        const float gz = fmaxf(fabsf(pi.z - e.sz) - hw, 0.f);
        const float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
        const float c = 1e-6f * (fabsf(pi.x) + fabsf(pi.y) + fabsf(pi.z) + hw);
        const float Rm = 1.0001f * fmaxf(Hi, g.leaf_hmax[e.b]) + c, Ri = 1.0001f * Hi + c;
        near = g2 < Rm * Rm;
        if (near && !(g2 < Ri * Ri)) {
          // beyond H_i from the whole leaf: only particles whose own H
          // exceeds T (the gap less the guard) can be neighbours, and every
          // one past rank hq_rank(q) of the leaf's H order has H at most
          // sample q times the leaf's growth bound
          const float T = (sqrtf(g2) - c) * (0.99999f / 1.0001f);
          const float gr = g.leaf_hgrow[e.b] * 1.00001f;
          const float4 *hq = g.leaf_hq + 4 * (int64_t)e.b;
          int above = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float4 s = hq[u];
            above += (s.x * gr > T) + (s.y * gr > T) + (s.z * gr > T) + (s.w * gr > T);
          }
          const int need = above < HQ_N ? min(hq_rank(above), bc) : bc;
          if (need < bc) {
            head = true;
            nflat = need;
          }
        }
      }
      const bool big = near && !head && e.b != ch.leaf && bc > 128;
      int axl = 0;
      float sgl = 1.f;
      if (big) {
        const uint8_t code = g.pair_axis[p];
        axl = code & 0x7f;
        sgl = (code & 0x80) ? -1.f : 1.f;
      }
      // the own leaf, small partners and the heads of H orders as one flat range
      const FlatRange fr = compact_small(my, near && !big, nflat, bb, e, lane, head);
      const uint16_t *hrow = g.axis_order + (int64_t)HORD_ROW * g.n;
      for (int t = sub * 64; t < fr.total; t += 2 * NWP * 64) {
        // two candidates per lane, their loads in flight together
        const int f0 = t + lane, f1 = t + NWP * 64 + lane;
        const bool v0 = f0 < fr.total, v1 = f1 < fr.total;
        const SweepPair q0 = locate(my, fr, v0 ? f0 : 0), q1 = locate(my, fr, v1 ? f1 : 0);
        const int l0 = v0 ? f0 - q0.off : 0, l1 = v1 ? f1 - q1.off : 0;
        const int j0 = q0.bb + (q0.hord ? (int)hrow[q0.bb + l0] : l0);
        const int j1 = q1.bb + (q1.hord ? (int)hrow[q1.bb + l1] : l1);
        const float4 pj0 = g.pos4[j0], pj1 = g.pos4[j1];
        visit(v0, j0, pj0, q0.sx, q0.sy, q0.sz);
        visit(v1, j1, pj1, q1.sx, q1.sy, q1.sz);
      }
      uint64_t bigm = __ballot(big);
      int nb = 0;
      while (bigm) {
        const int src = __ffsll((unsigned long long)bigm) - 1;
        bigm &= bigm - 1;
        if ((nb++ % NWP) != sub) continue;
        const int bbq = __shfl(bb, src, 64), bcq = __shfl(bc, src, 64), Bq = __shfl(e.b, src, 64);
        const float sx = __shfl(e.sx, src, 64), sy = __shfl(e.sy, src, 64), sz = __shfl(e.sz, src, 64);
        const int axis = __builtin_amdgcn_readfirstlane(__shfl(axl, src, 64));
        const float sgn = __shfl(sgl, src, 64);
        const float ex = g.ax.e[axis][0], ey = g.ax.e[axis][1], ez = g.ax.e[axis][2];
        const float Rb = fmaxf(Hi, g.leaf_hmax[Bq]);
        const float pp = fmaf(pi.z, ez, fmaf(pi.y, ey, pi.x * ex));
        const float sproj = fmaf(sz, ez, fmaf(sy, ey, sx * ex));
        const float margin = 1.0001f * Rb + 2.0001f * g.leaf_dx[Bq] + 1e-6f * (2.f * fabsf(pp) + fabsf(sproj));
        const float lo_b = pp - margin - sproj, hi_b = pp + margin - sproj;
        const uint16_t *ord = g.axis_order + (int64_t)axis * g.n + bbq;
        // two tiles per step (as in the density sweep)
        for (int t = 0; t < bcq; t += 128) {
          const int k0 = t + lane, k1 = t + 64 + lane;
          const bool v0 = k0 < bcq, v1 = k1 < bcq;
          const int j0 = bbq + (v0 ? (int)ord[sgn > 0.f ? k0 : bcq - 1 - k0] : 0);
          const int j1 = bbq + (v1 ? (int)ord[sgn > 0.f ? k1 : bcq - 1 - k1] : 0);
          const float4 pj0 = g.pos4[j0], pj1 = g.pos4[j1];
          const float key0 = fmaf(pj0.z, ez, fmaf(pj0.y, ey, pj0.x * ex));
          if (__ballot(v0 && !(sgn > 0.f ? key0 > hi_b : key0 < lo_b)) == 0ull) break;
          visit(v0, j0, pj0, sx, sy, sz);
          const float key1 = fmaf(pj1.z, ez, fmaf(pj1.y, ey, pj1.x * ex));
          if (__ballot(v1 && !(sgn > 0.f ? key1 > hi_b : key1 < lo_b)) == 0ull) break;
          visit(v1, j1, pj1, sx, sy, sz);
        }
      }
    }
    wave_sync();
    drain(qn);
    float v[5] = {f.ax, f.ay, f.az, f.visc, f.adiab};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      if (COMP) {
        float c = 0.f;
        two_sum_butterfly(v[q], c);
        v[q] += c;
      } else {
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
      }
    }
    float vm = f.vmax;
    for (int o = 32; o > 0; o >>= 1) vm = fmaxf(vm, __shfl_xor(vm, o, 64));
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (NWP > 1 && lane == 0) {
#pragma unroll
      for (int q = 0; q < 5; ++q) red[wave][q] = v[q];
      red[wave][5] = vm;
      red[wave][6] = __int_as_float(cnt);
    }
    if (NWP == 1 && lane == 0) {
      g.ax_out[i] = v[0];
      g.ay_out[i] = v[1];
      g.az_out[i] = v[2];
      const float rho = thi.x;
      g.dA_out[i] = 0.5f * g.gm1 * __powf(rho, -g.gm1) * v[3];
      g.du_out[i] = fmaf(thi.y, v[4], 0.5f * v[3]);
      g.vsig_out[i] = vm;
      if (g.nngb_out) g.nngb_out[i] = cnt;
    }
  }
  if (NWP > 1) {
    __syncthreads();
    if (sub == 0 && lane == 0 && k < g.n_active) {
      const int i = g.active_idx[k];
      const float4 thi = g.jth[i];
      float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, c[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
      float vm = 0.f;
      int cs = 0;
      for (int u = 0; u < NWP; ++u) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          if (COMP)
            neu_add(v[q], c[q], red[wave + u][q]);
          else
            v[q] += red[wave + u][q];
        }
        vm = fmaxf(vm, red[wave + u][5]);
        cs += __float_as_int(red[wave + u][6]);
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] += c[q];
      g.ax_out[i] = v[0];
      g.ay_out[i] = v[1];
      g.az_out[i] = v[2];
      const float rho = thi.x;
      g.dA_out[i] = 0.5f * g.gm1 * __powf(rho, -g.gm1) * v[3];
      g.du_out[i] = fmaf(thi.y, v[4], 0.5f * v[3]);
      g.vsig_out[i] = vm;
      if (g.nngb_out) g.nngb_out[i] = cs;
    }
  }
  // interactions of the block, one counter update
  if (lane == 0) blk_cnt[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int s = blk_cnt[0] + blk_cnt[1] + blk_cnt[2] + blk_cnt[3];
    if (s) atomicAdd(g.ctr, (unsigned long long)s);
  }
}

// ---------------------------------------------------------------- density pass phases

// Checks the arrays, resets the pass counters and, with active particles,
// sizes the solver state and marks every chunk to do.  Returns SPH_OK with
// *any = 0 when nothing is active (the pass is then complete).
sph_status density_begin(sph_ctx *ctx, const sph_particles *p, int entropy_from_u, int *any) {
  *any = 0;
  if (!p->vx || !p->vy || !p->vz || !p->m || !p->h)
    return sph_fail(ctx, SPH_EINVAL, "density_pass: v, m and h are required");
  if (!p->rho || !p->drho_dh || !p->f_gradh || !p->divv || !p->curlx || !p->curly || !p->curlz || !p->P || !p->c ||
      !p->balsara || !p->A)
    return sph_fail(ctx, SPH_EINVAL, "density_pass: an output array is missing");
  if (entropy_from_u && !p->u) return sph_fail(ctx, SPH_EINVAL, "density_pass: u is required with entropy_from_u");
  const int64_t na = ctx->n_active;
  ctx->density_from_u = entropy_from_u ? 1 : 0;
  ctx->widen_pending = 0;
  ctx->todo_collect = 0;
  ctx->fpairs_counted = -1;
  ctx->density_iterations = 0;
  ctx->n_unconverged = 0;
  ctx->pair_rebuilds = 0;
  for (int q = 0; q < 32; ++q) ctx->unconv_hist[q] = 0;
  if (na == 0) {
    ctx->state = 4;
    return SPH_OK;
  }
  SPH_TRY(sph_ensure(ctx, ctx->sums, sizeof(float) * 9 * (size_t)na));
  SPH_TRY(sph_ensure(ctx, ctx->hlo, 4 * (size_t)na));
  SPH_TRY(sph_ensure(ctx, ctx->hhi, 4 * (size_t)na));
  SPH_TRY(sph_ensure(ctx, ctx->conv, (size_t)na));
  // the per-pass counters (unconverged, rebuild flags) start at zero
  const int n_stats = 2 * (ctx->prm.h_max_iter + 1);
  SPH_TRY(sph_ensure(ctx, ctx->pass_stats, sizeof(int32_t) * (size_t)n_stats));
  {
    PROF(ctx, "ghost");
    density_init_kernel<<<grid256(na > ctx->n_chunks ? na : ctx->n_chunks), 256, 0, ctx->stream>>>(
        ctx->n_chunks, (int32_t *)ctx->chunk_todo.p, na, (float *)ctx->hlo.p, (float *)ctx->hhi.p,
        (uint8_t *)ctx->conv.p, (int32_t *)ctx->pass_stats.p, n_stats);
  }
  HIP_TRY(ctx, hipGetLastError());
  *any = 1;
  return SPH_OK;
}

LoopArgs density_loop_args(sph_ctx *ctx) {
  LoopArgs a = base_args(ctx);
  a.pair_off = (const int32_t *)ctx->dpair_off.p;
  a.pairs = (const PairEntry *)ctx->dpairs.p;
  a.pair_axis = (const uint8_t *)ctx->dpair_axis.p;
  a.sums = (float *)ctx->sums.p;
  a.act_cnt = (int32_t *)ctx->sums.p + 8 * ctx->n_active;
  return a;
}

// Ghost arguments of Newton pass `it`; the pass counters go to status[0]
// (unconverged) and status[1] (rebuild flags).
GhostArgs density_ghost_args(sph_ctx *ctx, sph_particles *p, int it, int entropy_from_u, int32_t *status) {
  const int64_t na = ctx->n_active;
  GhostArgs gh;
  gh.n_active = na;
  gh.active_idx = (const int32_t *)ctx->active_idx.p;
  gh.chunk_of = (const int32_t *)ctx->chunk_of.p;
  gh.chunks = (const Chunk *)ctx->chunks.p;
  gh.chunk_todo = (int32_t *)ctx->chunk_todo.p;
  gh.sums = (const float *)ctx->sums.p;
  gh.act_cnt = (const int32_t *)ctx->sums.p + 8 * na;
  gh.act_reach = (const float *)ctx->act_reach.p;
  gh.hlo = (float *)ctx->hlo.p;
  gh.hhi = (float *)ctx->hhi.p;
  gh.conv = (uint8_t *)ctx->conv.p;
  gh.pos4 = (float4 *)ctx->pos4.p;
  gh.jth = (float4 *)ctx->jth.p;
  gh.h = p->h;
  gh.last = it == ctx->prm.h_max_iter;
  gh.from_u = entropy_from_u;
  gh.eta3 = ctx->prm.eta * ctx->prm.eta * ctx->prm.eta;
  gh.kc = (float)((8.0 / M_PI) / ((double)GK32 * GK32 * GK32));
  gh.tol = ctx->prm.h_tol;
  gh.gamma = (float)ctx->prm.gamma;
  gh.eps = ctx->prm.balsara_eps;
  gh.box_quarter = (float)(0.25 * ctx->prm.box);
  gh.rho = p->rho;
  gh.drho_dh = p->drho_dh;
  gh.f = p->f_gradh;
  gh.divv = p->divv;
  gh.curlx = p->curlx;
  gh.curly = p->curly;
  gh.curlz = p->curlz;
  gh.P = p->P;
  gh.c = p->c;
  gh.B = p->balsara;
  gh.A = p->A;
  gh.Af = p->Af;
  gh.u = p->u;
  gh.nngb = p->nngb_density;
  gh.n_unconv = status;
  gh.rebuild = status + 1;
  gh.ctr = (unsigned long long *)ctx->counters64.p;
  gh.todo = nullptr;
  gh.todo_n = nullptr;
  return gh;
}

// The sweep's own solver steps in Newton pass `pass`: as the ghost's, at
// most h_max_iter - pass of them, within 1.1 H.
SweepSolve sweep_solve_args(sph_ctx *ctx, sph_particles *p, int pass) {
  SweepSolve sv;
  sv.steps = std::max(0, ctx->prm.h_max_iter - pass);
  sv.cache_f = 1.1f;
  sv.kc = (float)((8.0 / M_PI) / ((double)GK32 * GK32 * GK32));
  sv.eta3 = ctx->prm.eta * ctx->prm.eta * ctx->prm.eta;
  sv.tol = ctx->prm.h_tol;
  sv.box_quarter = (float)(0.25 * ctx->prm.box);
  sv.act_reach = (const float *)ctx->act_reach.p;
  sv.h = p->h;
  sv.hlo = (float *)ctx->hlo.p;
  sv.hhi = (float *)ctx->hhi.p;
  sv.pos4 = (float4 *)ctx->pos4.p;
  sv.chunk_todo = (int32_t *)ctx->chunk_todo.p;
  return sv;
}

// Book-keeping after Newton pass `it` with the ghost's counters st: returns
// SPH_OK with *done = 1 when the solve is over; widens the pair lists when a
// smoothing length outgrew them.
// Passes are grouped like the single-box path's batches (passes 1-4, then
// 5-6, 7-8, ...): widening happens only at the end of a group.
// The force cell-pair total and a group's per-pass counters into page-locked
// host slots.
__global__ void group_read_kernel(const int32_t *__restrict__ ftotal, const int32_t *__restrict__ stats, int nst,
                                  int32_t *host_fc, int32_t *host_st) {
  if (threadIdx.x == 0) host_fc[0] = *ftotal;
  for (int q = threadIdx.x; q < nst; q += blockDim.x) host_st[q] = stats[q];
}

// The int32 at src[q] into host slot q (page-locked), q < n.
__global__ void gather_totals_kernel(const int32_t *const *__restrict__ src, int n, int32_t *host) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) host[q] = *src[q];
}

static inline bool group_end(int it) { return it == 4 || (it > 4 && (it % 2) == 0); }

sph_status density_after_pass(sph_ctx *ctx, const sph_particles *p, int it, const int32_t st[2], bool group_last,
                              int *done) {
  *done = 0;
  ctx->density_iterations = it;
  if (it <= 32) ctx->unconv_hist[it - 1] = st[0];
  if (st[1] & 2) return sph_fail(ctx, SPH_EREBUILD, "density_pass: a smoothing length exceeds a quarter of the box");
  if (it == ctx->prm.h_max_iter) {
    ctx->n_unconverged = st[0];
    *done = 1;
    return SPH_OK;
  }
  if (st[0] == 0) {
    *done = 1;
    return SPH_OK;
  }
  if (st[1] & 1) ctx->widen_pending = 1;
  if (ctx->widen_pending && group_last) {
    // a smoothing length outgrew its cell's pair reach: widen the pair lists,
    // then the waiting particles go on
    ctx->widen_pending = 0;
    ctx->pair_rebuilds++;
    SPH_TRY(refresh_leaf_hmax(ctx));
    SPH_TRY(build_pairs(ctx, 0, 1.5f));
    SPH_TRY(drift_partners(ctx, p, 0));
    // (single-box passes: the released particles join the next pass's list)
    int32_t *todo = ctx->todo_collect ? (int32_t *)ctx->todo_list.p : nullptr;
    int32_t *todo_n = todo ? todo + ctx->n_active + ((it + 1) & 1) : nullptr;
    release_waiting_kernel<<<grid256(ctx->n_active), 256, 0, ctx->stream>>>(
        (uint8_t *)ctx->conv.p, (const int32_t *)ctx->chunk_of.p, ctx->n_active, (int32_t *)ctx->chunk_todo.p, todo,
        todo_n);
    HIP_TRY(ctx, hipGetLastError());
  }
  return SPH_OK;
}

// Leaf max H follows the new smoothing lengths, so that any later cell-pair
// list (the force list, or a later active set without a rebuild) sees them.
sph_status density_end(sph_ctx *ctx, bool refreshed) {
  if (!refreshed) SPH_TRY(refresh_leaf_hmax(ctx));
  ctx->state = 4;
  if (ctx->n_unconverged > 0)
    return sph_fail(ctx, SPH_ENOCONV, "density_pass: %lld particles not converged after %d iterations",
                    (long long)ctx->n_unconverged, ctx->prm.h_max_iter);
  return SPH_OK;
}

// Newton passes are enqueued in groups without waiting for the host (four,
// then pairs; pairs from the start when the first pass is a sweep, whose own
// steps leave few particles to a second): each pass's loop runs over what the
// previous ghost left to do, read on the device, and a pass past convergence
// does nothing.  One synchronisation per group reads its passes' counters.
sph_status density_pass_impl(sph_ctx *ctx, sph_particles *p, int entropy_from_u) {
  int any;
  SPH_TRY(density_begin(ctx, p, entropy_from_u, &any));
  if (!any) return SPH_OK;
  const int64_t na = ctx->n_active;
  const int maxit = ctx->prm.h_max_iter;
  SPH_TRY(sph_ensure(ctx, ctx->pass_stats, sizeof(int32_t) * 2 * (size_t)(maxit + 1)));
  // the particles each pass evaluates: appended by the ghost (and by the
  // release of waiting particles) before it; two counters, pass p reading
  // counter p % 2
  SPH_TRY(sph_ensure(ctx, ctx->todo_list, 4 * (size_t)(na + 2)));
  ctx->todo_collect = 1;
  int32_t *stats = (int32_t *)ctx->pass_stats.p;
  int32_t *list = (int32_t *)ctx->todo_list.p, *list_n = list + na;
  int64_t n_todo = na;  // upper bound of the particles left to do
  int it = 0, done = 0;
  while (!done) {
    const int first = it + 1, last = std::min(it == 0 && n_todo >= ctx->prm.sweep_below ? 4 : it + 2, maxit);
    const bool sweep_group = n_todo < ctx->prm.sweep_below;
    for (int pass = first; pass <= last; ++pass) {
      LoopArgs a = density_loop_args(ctx);
      int32_t *next_n = list_n + ((pass + 1) & 1);
      if (sweep_group) {
        // few particles to do: one wave per particle.  The number to do only
        // falls from here on, so no later pass of this solve runs the chunk
        // loop (whose chunk flags the sweep leaves as they are).
        PROF(ctx, "density_sweep");
        const int nwp = sweep_waves(ctx, n_todo);
        const unsigned grid = xcd_grid(std::min<int64_t>(ceil_div(n_todo * nwp, 4), (int64_t)ctx->n_cu * 16));
        const int32_t *tl = pass > 1 ? list : nullptr, *tn = pass > 1 ? list_n + (pass & 1) : nullptr;
        const int32_t *co = (const int32_t *)ctx->chunk_of.p;
        const bool comp = ctx->prm.compensated != 0;
        const SweepSolve sv = sweep_solve_args(ctx, p, pass);
#define SPH_DSWEEP(NWP_, C_)                                                                          \
  density_sweep_kernel<NWP_, C_><<<grid, 256, 0, ctx->stream>>>(a, tl, tn, n_todo, co, next_n, sv, nullptr, \
                                                                nullptr, 0)
        if (nwp == 4)
          { if (comp) SPH_DSWEEP(4, true); else SPH_DSWEEP(4, false); }
        else if (nwp == 2)
          { if (comp) SPH_DSWEEP(2, true); else SPH_DSWEEP(2, false); }
        else
          { if (comp) SPH_DSWEEP(1, true); else SPH_DSWEEP(1, false); }
#undef SPH_DSWEEP
        HIP_TRY(ctx, hipGetLastError());
      } else {
        HIP_TRY(ctx, hipMemsetAsync(next_n, 0, sizeof(int32_t), ctx->stream));
        // after the group's first pass the number left to do is known on the
        // device only (the previous ghost's count): the chunk loop works
        // while it is at least sweep_below, else a sweep takes the pass: over
        // the list the previous ghost appended to (passes after the second of
        // the group), or over the particles whose conv flag is 0 (the second:
        // the first pass's ghost appends nothing, nearly every particle being
        // left to do)
        const bool gated = pass > first && sweep_waves(ctx, na) == 1;
        const int32_t *gate = stats + 2 * (pass - 1);
        const int32_t gate_min = (int32_t)std::min<int64_t>(ctx->prm.sweep_below, INT32_MAX);
        LoopArgs ac = a;
        if (gated) {
          ac.gate = gate;
          ac.gate_min = gate_min;
        }
        if (ctx->prm.compensated)
          SPH_TRY((launch_loop<0, true>(ctx, ac)));
        else
          SPH_TRY((launch_loop<0, false>(ctx, ac)));
        if (gated && pass > first + 1) {
          PROF(ctx, "density_sweep");
          const unsigned grid = xcd_grid(std::min<int64_t>(ceil_div(na, 4), (int64_t)ctx->n_cu * 16));
          const int32_t *co = (const int32_t *)ctx->chunk_of.p;
          const int32_t *tn = list_n + (pass & 1);
          const SweepSolve sv = sweep_solve_args(ctx, p, pass);
          if (ctx->prm.compensated)
            density_sweep_kernel<1, true><<<grid, 256, 0, ctx->stream>>>(a, list, tn, na, co, nullptr, sv, nullptr,
                                                                          gate, gate_min);
          else
            density_sweep_kernel<1, false><<<grid, 256, 0, ctx->stream>>>(a, list, tn, na, co, nullptr, sv, nullptr,
                                                                           gate, gate_min);
          HIP_TRY(ctx, hipGetLastError());
        } else if (gated) {
          PROF(ctx, "density_sweep");
          const int64_t ngroups = ceil_div(na, 64);
          const unsigned grid = xcd_grid(std::min<int64_t>(ceil_div(ngroups, 4), (int64_t)ctx->n_cu * 16));
          const int32_t *co = (const int32_t *)ctx->chunk_of.p;
          const uint8_t *conv = (const uint8_t *)ctx->conv.p;
          const SweepSolve sv = sweep_solve_args(ctx, p, pass);
          if (ctx->prm.compensated)
            density_sweep_kernel<1, true, true><<<grid, 256, 0, ctx->stream>>>(a, nullptr, nullptr, ngroups, co,
                                                                               nullptr, sv, conv, gate, gate_min);
          else
            density_sweep_kernel<1, false, true><<<grid, 256, 0, ctx->stream>>>(a, nullptr, nullptr, ngroups, co,
                                                                                nullptr, sv, conv, gate, gate_min);
          HIP_TRY(ctx, hipGetLastError());
        }
      }
      GhostArgs gh = density_ghost_args(ctx, p, pass, entropy_from_u, stats + 2 * pass);
      // the list of the next pass: read by a sweep, the next group's first
      // pass, or a later pass of a chunk-loop group that the device hands to
      // the sweep.  Only the ghost of a chunk-loop group's first pass appends
      // nothing: nearly every particle is left after it, and the chunk loop
      // reads its chunk flags
      if (sweep_group || pass > first || pass == last) {
        gh.todo = list;
        gh.todo_n = next_n;
      }
      {
        PROF(ctx, "ghost");
        ghost_kernel<<<grid256(na), 256, 0, ctx->stream>>>(gh);
      }
      HIP_TRY(ctx, hipGetLastError());
    }
    // in case this group ends the solve: the leaf max H from the new
    // smoothing lengths and the force cell-pair count, read in the same
    // synchronisation (wasted work when another group follows)
    SPH_TRY(refresh_leaf_hmax(ctx));
    // both read through page-locked slots that one small kernel writes, one
    // synchronisation
    int32_t *fcount = ctx->pin_h + PIN_FCOUNT;
    SPH_TRY(build_pairs_count(ctx, 1, 1.0f, nullptr));
    const size_t nst = 2 * (size_t)(last - first + 1);
    if (nst > PIN_COUNT - PIN_STATS) return sph_fail(ctx, SPH_EINVAL, "density pass: group of passes too long");
    group_read_kernel<<<1, 64, 0, ctx->stream>>>((const int32_t *)ctx->fpair_off.p + ctx->n_active_leaves,
                                                 stats + 2 * first, (int)nst, ctx->pin_dev + PIN_FCOUNT,
                                                 ctx->pin_dev + PIN_STATS);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    SPH_TRY(pin_fetch(ctx, PIN_FCOUNT, 1));
    SPH_TRY(pin_fetch(ctx, PIN_STATS, (int)nst));
    // density_after_pass may issue reads of its own: the counters leave the slots first
    int32_t st[PIN_COUNT - PIN_STATS];
    memcpy(st, ctx->pin_h + PIN_STATS, sizeof(int32_t) * nst);
    const int32_t fc = *fcount;
    for (int pass = first; pass <= last && !done; ++pass) {
      SPH_TRY(density_after_pass(ctx, p, pass, &st[2 * (pass - first)], pass == last, &done));
      n_todo = st[2 * (pass - first)];
    }
    if (done) ctx->fpairs_counted = fc;
    it = last;
  }
  return density_end(ctx, true);
}

// Force loop arguments with the outputs of p.
LoopArgs force_loop_args(sph_ctx *ctx, sph_particles *p) {
  LoopArgs a = base_args(ctx);
  a.pair_off = (const int32_t *)ctx->fpair_off.p;
  a.pairs = (const PairEntry *)ctx->fpairs.p;
  a.pair_axis = (const uint8_t *)ctx->fpair_axis.p;
  a.ax_out = p->ax;
  a.ay_out = p->ay;
  a.az_out = p->az;
  a.dA_out = p->dA_dt;
  a.du_out = p->du_dt;
  a.vsig_out = p->vsig;
  a.nngb_out = p->nngb_force;
  a.ctr = (unsigned long long *)ctx->counters64.p + 1;
  return a;
}

sph_status force_pass_impl(sph_ctx *ctx, sph_particles *p) {
  if (!p->ax || !p->ay || !p->az || !p->dA_dt || !p->du_dt || !p->vsig)
    return sph_fail(ctx, SPH_EINVAL, "force_pass: an output array is missing");
  const int64_t n = ctx->n;
  if (ctx->n_active == 0) {
    ctx->n_fpairs = 0;
    ctx->state = 5;
    return SPH_OK;
  }
  (void)n;
  if (ctx->fpairs_counted >= 0) {
    // counted at the end of the density solve (same smoothing lengths)
    SPH_TRY(build_pairs_fill(ctx, 1, 1.0f, (int32_t)ctx->fpairs_counted));
    ctx->fpairs_counted = -1;
  } else {
    SPH_TRY(build_pairs(ctx, 1, 1.0f));
  }
  SPH_TRY(drift_partners(ctx, p, 1));
  LoopArgs a = force_loop_args(ctx, p);
  if (ctx->n_active < ctx->prm.sweep_below) {
    {
      PROF(ctx, "force_sweep");
      const int nwp = sweep_waves(ctx, ctx->n_active);
      const unsigned grid = xcd_grid(ceil_div(ctx->n_active * nwp, 4));
      const bool comp = ctx->prm.compensated != 0;
      const int32_t *co = (const int32_t *)ctx->chunk_of.p;
#define SPH_FSWEEP(NWP_, C_) force_sweep_kernel<NWP_, C_><<<grid, 256, 0, ctx->stream>>>(a, co)
      if (nwp == 4)
        { if (comp) SPH_FSWEEP(4, true); else SPH_FSWEEP(4, false); }
      else if (nwp == 2)
        { if (comp) SPH_FSWEEP(2, true); else SPH_FSWEEP(2, false); }
      else
        { if (comp) SPH_FSWEEP(1, true); else SPH_FSWEEP(1, false); }
#undef SPH_FSWEEP
    }
    HIP_TRY(ctx, hipGetLastError());
  } else {
    fill_i32_kernel<<<grid256(ctx->n_chunks), 256, 0, ctx->stream>>>((int32_t *)ctx->chunk_todo.p, ctx->n_chunks,
                                                                      1);
    HIP_TRY(ctx, hipGetLastError());
    if (ctx->prm.compensated)
      SPH_TRY((launch_loop<1, true>(ctx, a)));
    else
      SPH_TRY((launch_loop<1, false>(ctx, a)));
  }
  ctx->state = 5;
  return SPH_OK;
}

// ---------------------------------------------------------------- autotuner

namespace {

struct TimedLaunch {
  LoopConfig cfg;
  float ms;
};

template <int MODE>
sph_status time_config(sph_ctx *ctx, const LoopArgs &a0, const LoopConfig &cfg, int reps, float *ms_out) {
  LoopArgs a = a0;
  SPH_TRY(apply_config(ctx, cfg, a));
  const int64_t ni = a.work ? a.n_items : ctx->n_chunks;
  SPH_TRY(sph_ensure(ctx, ctx->box_args, sizeof(LoopArgs)));
  SPH_TRY(sph_ensure(ctx, ctx->box_work, sizeof(int2) * (size_t)(ni > 0 ? ni : 1)));
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  float best = INFINITY;
  for (int r = 0; r <= reps; ++r) {
    fill_i32_kernel<<<grid256(ctx->n_chunks), 256, 0, ctx->stream>>>((int32_t *)ctx->chunk_todo.p, ctx->n_chunks, 1);
    HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
    hipError_t err;
    if (cfg.persistent) {
      HIP_TRY(ctx, hipMemcpyAsync(ctx->box_args.p, &a, sizeof(LoopArgs), hipMemcpyHostToDevice, ctx->stream));
      fill_work_kernel<<<grid_for_items(ni), 256, 0, ctx->stream>>>(a.work, ni, (int2 *)ctx->box_work.p);
      err = launch_loop_any<MODE, true>(ctx->stream, a, cfg, (const LoopArgs *)ctx->box_args.p,
                                        (const int2 *)ctx->box_work.p, (int)ni, (int *)ctx->scalars.p + SC_WORKCTR,
                                        persistent_grid_for(ctx->n_cu, cfg));
    } else {
      err = launch_loop_any<MODE, true>(ctx->stream, a, cfg, nullptr, nullptr, 0, nullptr, 0);
    }
    HIP_TRY(ctx, err);
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
    if ((r > 0 || reps == 0) && ms < best) best = ms;  // the first launch warms caches
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = best;
  return SPH_OK;
}

struct Timed {
  LoopConfig c;
  float ms;
};

}  // namespace

extern "C" sph_status sph_autotune(sph_ctx *ctx, sph_particles *p, const char *path) {
  if (ctx && !ctx->kids.empty()) {
    // a batch context tunes its batched loops
    if (!p) return sph_fail(ctx, SPH_EINVAL, "autotune: null particles");
    std::vector<sph_particles> sl = box_slices(ctx, p);
    const sph_status st = batch_autotune_impl(ctx->kids.data(), sl.data(), (int)sl.size(), path);
    return st == SPH_OK ? st : sph_fail(ctx, st, "%s", ctx->kids[0]->err.c_str());
  }
  if (!ctx || !p) return SPH_EINVAL;
  if (ctx->state < 5) return sph_fail(ctx, SPH_ESTATE, "autotune: run a force pass first");
  if (ctx->n_chunks == 0) return SPH_OK;
  const int cls = tune_class(ctx->n_chunks);
  const int prof = ctx->prof;
  ctx->prof = 0;
  FILE *f = path ? fopen(path, "a") : nullptr;
  sph_status st = SPH_OK;
  for (int mode = 0; mode < 2 && st == SPH_OK; ++mode) {
    LoopArgs a;
    if (mode == 0) {
      a = density_loop_args(ctx);
    } else {
      a = force_loop_args(ctx, p);
      // counts of tuning launches are not interactions of a step
      SPH_TRY(sph_ensure(ctx, ctx->box_args, sizeof(LoopArgs) + 64));
      a.ctr = (unsigned long long *)((char *)ctx->box_args.p + sizeof(LoopArgs) + 32);
    }
    sph_ctx::TuneEntry best;
    best.ms = INFINITY;
    std::vector<Timed> scan;
    const int nws[4] = {1, 2, 4, 8};
    for (int wi = 0; wi < 4 && st == SPH_OK; ++wi)
      for (int tile = 0; tile <= 4 && st == SPH_OK; ++tile)
        for (int split = 0; split <= 2 && st == SPH_OK; ++split)
          for (int ordered = 0; ordered <= 1 && st == SPH_OK; ++ordered)
            for (int pers = 0; pers <= 1 && st == SPH_OK; ++pers) {
              LoopConfig c;
              c.nw = nws[wi];
              c.tile = tile;
              c.ordered = ordered;
              c.persistent = pers;
              c.split = split;
              if (!loop_config_valid(c)) continue;
              float ms = 0.f;
              st = mode == 0 ? time_config<0>(ctx, a, c, 2, &ms) : time_config<1>(ctx, a, c, 2, &ms);
              if (st != SPH_OK) break;
              if (f)
                fprintf(f, "candidate %d %d %d %d %d %d %d %.6f %lld\n", mode, cls, c.nw, c.tile, c.ordered,
                        c.persistent, c.split, ms, (long long)ctx->n_chunks);
              scan.push_back({c, ms});
            }
    if (st != SPH_OK) break;
    // the three fastest of the scan timed again, in turns, five times each:
    // the one of smallest median wins, the scan's order deciding between
    // medians within 3 % (single launches of similar tilings swing by more
    // than the differences between them)
    std::sort(scan.begin(), scan.end(), [](const Timed &x, const Timed &y) { return x.ms < y.ms; });
    const int nf = std::min<int>(3, (int)scan.size());
    std::vector<std::vector<float>> runs(nf);
    for (int r = 0; r < 5 && st == SPH_OK; ++r)
      for (int q = 0; q < nf && st == SPH_OK; ++q) {
        float ms = 0.f;
        st = mode == 0 ? time_config<0>(ctx, a, scan[q].c, 0, &ms) : time_config<1>(ctx, a, scan[q].c, 0, &ms);
        runs[q].push_back(ms);
      }
    if (st != SPH_OK) break;
    int win = -1;
    float win_med = INFINITY;
    for (int q = 0; q < nf; ++q) {
      std::vector<float> v = runs[q];
      std::sort(v.begin(), v.end());
      const float med = v[v.size() / 2];
      if (win < 0 || med < 0.97f * win_med) {
        win = q;
        win_med = med;
      }
    }
    if (win >= 0) {
      best.valid = 1;
      best.nw = scan[win].c.nw;
      best.tile = scan[win].c.tile;
      best.ordered = scan[win].c.ordered;
      best.persistent = scan[win].c.persistent;
      best.split = scan[win].c.split;
      best.ms = win_med;
    }
    ctx->tune[mode][cls] = best;
    if (f)
      fprintf(f, "best %d %d %d %d %d %d %d %.6f %lld\n", mode, cls, best.nw, best.tile, best.ordered,
              best.persistent, best.split, best.ms, (long long)ctx->n_chunks);
  }
  if (f) fclose(f);
  ctx->prof = prof;
  if (st != SPH_OK) return st;
  // leave every chunk marked done, as after a completed pass
  HIP_TRY(ctx, hipMemsetAsync(ctx->chunk_todo.p, 0, 4 * (size_t)ctx->n_chunks, ctx->stream));
  return sph_sync(ctx);
}

extern "C" sph_status sph_load_tuning(sph_ctx *ctx, const char *path) {
  if (!ctx || !path) return SPH_EINVAL;
  FILE *f = fopen(path, "r");
  if (!f) return sph_fail(ctx, SPH_EINVAL, "load_tuning: cannot open %s", path);
  char tag[32];
  int mode, cls, nw, tile, ord, pers, split;
  float ms;
  long long nc;
  int loaded = 0;
  while (fscanf(f, "%31s %d %d %d %d %d %d %d %f %lld", tag, &mode, &cls, &nw, &tile, &ord, &pers, &split, &ms,
                &nc) == 10) {
    const bool single = strcmp(tag, "best") == 0, batch = strcmp(tag, "batch_best") == 0;
    if ((!single && !batch) || mode < 0 || mode > 1 || cls < 0 || cls > 31) continue;
    LoopConfig c;
    c.nw = nw;
    c.tile = tile;
    c.split = split;
    if (!loop_config_valid(c)) continue;
    auto &t = single ? ctx->tune[mode][cls] : ctx->btune[mode][cls];
    t.valid = 1;
    t.nw = nw;
    t.tile = tile;
    t.ordered = ord != 0;
    t.persistent = pers != 0;
    t.split = split;
    t.ms = ms;
    ++loaded;
  }
  fclose(f);
  return loaded > 0 ? SPH_OK : sph_fail(ctx, SPH_EINVAL, "load_tuning: no entries in %s", path);
}

// ---------------------------------------------------------------- batched passes
//
// Several contexts (independent periodic boxes, each built, sorted and marked
// by its own calls, all on one stream) run each loop pass as ONE launch over
// the concatenated work items (box, chunk), ordered by decreasing cost (staged
// partner particles of the chunk's leaf), pulled from one atomic counter by a
// machine-sized grid (persistent) or one workgroup per item.  The per-chunk
// work is the single-box chunk body, so a box's results equal those of its
// own pass run with the same loop tiling.

namespace {

struct BatchItems {
  const int32_t *items;     // the box's work items in chunk order (codes chunk * 16 + part)
  const int32_t *item0;     // first item of each chunk (null: one part per chunk)
  const Chunk *chunks;
  const int32_t *act_cost;
  int32_t *todo;
  int64_t n_items, n_chunks;
  int64_t off;  // first work item of this box
  int32_t box;  // index into the launch's box descriptors
};

__global__ __launch_bounds__(256) void batch_bucket_kernel(const BatchItems *__restrict__ boxes,
                                                           int32_t *__restrict__ bucket_of,
                                                           int32_t *__restrict__ hist, int set_todo) {
  __shared__ int h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const BatchItems b = boxes[blockIdx.y];
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < b.n_items; q += (int64_t)gridDim.x * 256) {
    const int cid = b.items[q] >> 4;
    const int P = b.item0 ? b.item0[cid + 1] - b.item0[cid] : 1;
    const int cost = max(1, b.act_cost[b.chunks[cid].act_leaf] / P);
    const int k = __clz(cost);
    bucket_of[b.off + q] = k;
    atomicAdd(&h[k], 1);
  }
  if (set_todo)
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < b.n_chunks; q += (int64_t)gridDim.x * 256)
      b.todo[q] = 1;
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void batch_scatter_kernel(const BatchItems *__restrict__ boxes,
                                                            const int32_t *__restrict__ bucket_of,
                                                            int32_t *__restrict__ cursor, int2 *__restrict__ work) {
  const BatchItems b = boxes[blockIdx.y];
  const int lane = threadIdx.x & 63;
  for (int64_t q0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); q0 < b.n_items;
       q0 += (int64_t)gridDim.x * 256) {
    const int64_t q = q0 + lane;
    const bool valid = q < b.n_items;
    const int s = bucket_slot(cursor, valid ? bucket_of[b.off + q] : 0, valid);
    if (valid) work[s] = make_int2(b.box, b.items[q]);
  }
}

__global__ __launch_bounds__(256) void batch_todo_kernel(const BatchItems *__restrict__ boxes) {
  const BatchItems b = boxes[blockIdx.y];
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < b.n_chunks; q += (int64_t)gridDim.x * 256)
    b.todo[q] = 1;
}

unsigned grid_x_for(int64_t n) {
  int64_t g = ceil_div(n, 256);
  if (g > 1024) g = 1024;
  return (unsigned)(g < 1 ? 1 : g);
}

// Host staging: [LoopArgs x nb | GhostArgs x nb | BatchItems x nb], rewritten
// only after the stream has drained past the previous upload.
struct Staging {
  LoopArgs *args;
  GhostArgs *ghost;
  BatchItems *items;
};

Staging staging(sph_ctx *lead, int nb) {
  const size_t need = (sizeof(LoopArgs) + sizeof(GhostArgs) + sizeof(BatchItems)) * (size_t)nb;
  if (lead->batch_host.size() < need) lead->batch_host.resize(need);
  char *base = lead->batch_host.data();
  Staging s;
  s.args = reinterpret_cast<LoopArgs *>(base);
  s.ghost = reinterpret_cast<GhostArgs *>(base + sizeof(LoopArgs) * nb);
  s.items = reinterpret_cast<BatchItems *>(base + (sizeof(LoopArgs) + sizeof(GhostArgs)) * nb);
  return s;
}

LoopConfig batch_config(sph_ctx *lead, int mode, int64_t total) {
  const auto &t = lead->btune[mode][tune_class(total)];
  LoopConfig c;
  c.ordered = 1;
  if (t.valid) {
    c.nw = t.nw;
    c.tile = t.tile;
    c.persistent = t.persistent;
    c.split = t.split;
    return c;
  }
  c.persistent = 1;
  c.split = lead->prm.chunk_split;
  if (lead->prm.waves_per_chunk > 0) {
    const LoopConfig s = choose_config(lead, mode);  // the parameter rule
    c.nw = s.nw;
    c.tile = s.tile;
    c.split = s.split;
    return c;
  }
  if (total < 2048) {
    c.nw = 8, c.tile = 0;
  } else if (total < 8192) {
    c.nw = 4, c.tile = 1;
  } else if (total < 32768) {
    c.nw = 2, c.tile = 2;
  } else {
    c.nw = 1, c.tile = 2;
  }
  return c;
}

sph_status batch_fail(sph_ctx *lead, int b, sph_ctx *box, sph_status st) {
  if (box != lead) return sph_fail(lead, st, "box %d: %s", b, box->err.c_str());
  return st;
}

#define BATCH_TRY(b, expr)                                   \
  do {                                                       \
    sph_status _s = (expr);                                  \
    if (_s != SPH_OK) return batch_fail(lead, (b), cs[(b)], _s); \
  } while (0)

// Builds every live box's work items for the batch's split target (one
// synchronisation for all boxes), uploads the item descriptors and writes the
// cost-ordered (box, item) list; returns the number of items.
sph_status batch_work_list(sph_ctx *lead, sph_ctx **cs, const std::vector<int> &live, Staging &s, int set_todo,
                           int target, int64_t *total_out) {
  const int nl = (int)live.size();
  // each box's item total into its page-locked slot, one synchronisation
  bool any = false;
  for (int q = 0; q < nl; ++q) {
    sph_ctx *c = cs[live[q]];
    if (c->work_valid && c->items_target == target) continue;
    SPH_TRY(items_count(c, target, c->pin_h + PIN_ITEMS));
    any = true;
  }
  if (any && target > 0) HIP_TRY(lead, hipStreamSynchronize(lead->stream));
  for (int q = 0; q < nl; ++q) {
    sph_ctx *c = cs[live[q]];
    if (c->work_valid && c->items_target == target) continue;
    SPH_TRY(items_fill(c, target, c->pin_h[PIN_ITEMS]));
  }
  int64_t total = 0, maxc = 0;
  for (int q = 0; q < nl; ++q) {
    sph_ctx *c = cs[live[q]];
    s.items[q].items = (const int32_t *)c->items_nat.p;
    s.items[q].item0 = target > 0 ? (const int32_t *)c->chunk_item0.p : nullptr;
    s.items[q].chunks = (const Chunk *)c->chunks.p;
    s.items[q].act_cost = (const int32_t *)c->act_cost.p;
    s.items[q].todo = (int32_t *)c->chunk_todo.p;
    s.items[q].n_items = c->n_items;
    s.items[q].n_chunks = c->n_chunks;
    s.items[q].off = total;
    s.items[q].box = q;
    total += c->n_items;
    maxc = std::max<int64_t>(maxc, std::max<int64_t>(c->n_items, c->n_chunks));
  }
  *total_out = total;
  SPH_TRY(sph_ensure(lead, lead->batch_items, sizeof(BatchItems) * (size_t)nl));
  SPH_TRY(sph_ensure(lead, lead->batch_work, sizeof(int2) * (size_t)(total > 0 ? total : 1)));
  SPH_TRY(sph_ensure(lead, lead->batch_tmp, 4 * (size_t)(total + 64)));
  HIP_TRY(lead, hipMemcpyAsync(lead->batch_items.p, s.items, sizeof(BatchItems) * nl, hipMemcpyHostToDevice,
                               lead->stream));
  int32_t *hist = (int32_t *)lead->batch_tmp.p;
  int32_t *bucket_of = hist + 64;
  HIP_TRY(lead, hipMemsetAsync(hist, 0, 32 * sizeof(int32_t), lead->stream));
  PROF(lead, "cost_order");
  const dim3 grid(grid_x_for(maxc), nl);
  batch_bucket_kernel<<<grid, 256, 0, lead->stream>>>((const BatchItems *)lead->batch_items.p, bucket_of, hist,
                                                      set_todo);
  cost_bucket_scan_kernel<<<1, 64, 0, lead->stream>>>(hist);
  batch_scatter_kernel<<<grid, 256, 0, lead->stream>>>((const BatchItems *)lead->batch_items.p, bucket_of, hist,
                                                       (int2 *)lead->batch_work.p);
  return sph_hip_check(lead, hipGetLastError(), "batch work list");
}

// Per-box loop arguments of a batched launch: the box's split-chunk state.
void batch_split_args(sph_ctx *c, int target, LoopArgs &a) {
  a.work = nullptr;
  a.chunk_item0 = target > 0 ? (const int32_t *)c->chunk_item0.p : nullptr;
  a.chunk_ctr = target > 0 ? (int32_t *)c->chunk_ctr.p : nullptr;
  a.partials = target > 0 ? (float *)c->partials.p : nullptr;
}

template <int MODE, bool COMP>
sph_status batch_launch(sph_ctx *lead, const LoopConfig &cfg, int64_t total, const char *what) {
  PROF(lead, what);
  LoopArgs unused;
  memset(&unused, 0, sizeof unused);
  return sph_hip_check(lead,
                       launch_loop_any<MODE, COMP>(lead->stream, unused, cfg, (const LoopArgs *)lead->batch_args.p,
                                                   (const int2 *)lead->batch_work.p, (int)total,
                                                   (int *)lead->scalars.p + SC_WORKCTR,
                                                   persistent_grid_for(lead->n_cu, cfg)),
                       what);
}

sph_status batch_check(sph_ctx **cs, int nb, int at_least, const char *call) {
  if (!cs || nb < 1 || !cs[0]) return SPH_EINVAL;
  sph_ctx *lead = cs[0];
  for (int b = 0; b < nb; ++b) {
    if (!cs[b]) return sph_fail(lead, SPH_EINVAL, "%s: context %d is null", call, b);
    if (cs[b]->stream != lead->stream)
      return sph_fail(lead, SPH_EINVAL, "%s: context %d is on another stream", call, b);
    if (cs[b]->state < at_least)
      return sph_fail(lead, SPH_ESTATE, "%s: box %d is not ready (state %d, need %d)", call, b, cs[b]->state,
                      at_least);
    for (int q = 0; q < b; ++q)
      if (cs[q] == cs[b]) return sph_fail(lead, SPH_EINVAL, "%s: context %d appears twice", call, b);
    if (cs[b]->prm.lazy_drift) return sph_fail(lead, SPH_EINVAL, "%s: box %d drifts lazily", call, b);
  }
  return SPH_OK;
}

}  // namespace

sph_status batch_density_impl(sph_ctx **cs, sph_particles *ps, int nb, int entropy_from_u) {
  SPH_TRY(batch_check(cs, nb, 3, "batch_density_pass"));
  sph_ctx *lead = cs[0];
  HIP_TRY(lead, hipStreamSynchronize(lead->stream));
  std::vector<int> live;
  for (int b = 0; b < nb; ++b) {
    int any;
    BATCH_TRY(b, density_begin(cs[b], &ps[b], entropy_from_u, &any));
    if (any) live.push_back(b);
  }
  if (live.empty()) return SPH_OK;
  const int nl = (int)live.size();
  Staging s = staging(lead, nl);
  int64_t nchunks = 0;
  for (int b : live) nchunks += cs[b]->n_chunks;
  const LoopConfig cfg = batch_config(lead, 0, nchunks);
  const int target = split_target(cfg.split);
  int64_t total;
  SPH_TRY(batch_work_list(lead, cs, live, s, 0, target, &total));
  SPH_TRY(sph_ensure(lead, lead->batch_args, sizeof(LoopArgs) * (size_t)nl));
  SPH_TRY(sph_ensure(lead, lead->batch_ghost, sizeof(GhostArgs) * (size_t)nl));
  SPH_TRY(sph_ensure(lead, lead->batch_status, 8 * (size_t)nl));
  std::vector<int> iterating(live);  // boxes (indices into cs) still solving
  std::vector<int32_t> st(2 * (size_t)nl);
  const int maxit = lead->prm.h_max_iter;
  for (int b : live)
    if (cs[b]->prm.h_max_iter != maxit)
      return sph_fail(lead, SPH_EINVAL, "batch_density_pass: box %d has another h_max_iter", b);
  for (int it = 1; it <= maxit && !iterating.empty(); ++it) {
    // loop over every live box's chunks (finished boxes have no chunk to do)
    for (int q = 0; q < nl; ++q) {
      s.args[q] = density_loop_args(cs[live[q]]);
      batch_split_args(cs[live[q]], target, s.args[q]);
    }
    HIP_TRY(lead, hipMemcpyAsync(lead->batch_args.p, s.args, sizeof(LoopArgs) * nl, hipMemcpyHostToDevice,
                                 lead->stream));
    if (lead->prm.compensated)
      SPH_TRY((batch_launch<0, true>(lead, cfg, total, "density_loop")));
    else
      SPH_TRY((batch_launch<0, false>(lead, cfg, total, "density_loop")));
    // one ghost launch over the boxes still solving
    int32_t *status = (int32_t *)lead->batch_status.p;
    HIP_TRY(lead, hipMemsetAsync(status, 0, 8 * (size_t)nl, lead->stream));
    int64_t max_na = 0;
    const int ni = (int)iterating.size();
    for (int q = 0; q < ni; ++q) {
      sph_ctx *c = cs[iterating[q]];
      s.ghost[q] = density_ghost_args(c, &ps[iterating[q]], it, entropy_from_u, status + 2 * q);
      if (c->n_active > max_na) max_na = c->n_active;
    }
    HIP_TRY(lead, hipMemcpyAsync(lead->batch_ghost.p, s.ghost, sizeof(GhostArgs) * ni, hipMemcpyHostToDevice,
                                 lead->stream));
    {
      PROF(lead, "ghost");
      ghost_multi_kernel<<<dim3(grid_x_for(max_na), ni), 256, 0, lead->stream>>>(
          (const GhostArgs *)lead->batch_ghost.p);
    }
    HIP_TRY(lead, hipGetLastError());
    HIP_TRY(lead, hipMemcpyAsync(st.data(), status, 8 * (size_t)ni, hipMemcpyDeviceToHost, lead->stream));
    HIP_TRY(lead, hipStreamSynchronize(lead->stream));
    std::vector<int> next;
    for (int q = 0; q < ni; ++q) {
      const int b = iterating[q];
      int done;
      BATCH_TRY(b, density_after_pass(cs[b], &ps[b], it, &st[2 * q], group_end(it), &done));
      if (!done) next.push_back(b);
    }
    iterating.swap(next);
  }
  // leaf max H per box (and its running global max, on the device), one launch
  SPH_TRY(refresh_leaf_hmax_boxes(lead, cs, live.data(), nl));
  sph_status first = SPH_OK;
  for (int q = 0; q < nl; ++q) {
    sph_ctx *c = cs[live[q]];
    const sph_status e = density_end(c, true);
    if (e != SPH_OK && first == SPH_OK) first = batch_fail(lead, live[q], c, e);
  }
  return first;
}

sph_status batch_force_impl(sph_ctx **cs, sph_particles *ps, int nb) {
  SPH_TRY(batch_check(cs, nb, 4, "batch_force_pass"));
  sph_ctx *lead = cs[0];
  for (int b = 0; b < nb; ++b)
    if (!ps[b].ax || !ps[b].ay || !ps[b].az || !ps[b].dA_dt || !ps[b].du_dt || !ps[b].vsig)
      return sph_fail(lead, SPH_EINVAL, "batch_force_pass: box %d: an output array is missing", b);
  HIP_TRY(lead, hipStreamSynchronize(lead->stream));
  std::vector<int> live;
  for (int b = 0; b < nb; ++b) {
    if (cs[b]->n_active == 0) {
      cs[b]->n_fpairs = 0;
      cs[b]->state = 5;
    } else {
      live.push_back(b);
    }
  }
  if (live.empty()) return SPH_OK;
  const int nl = (int)live.size();
  // force cell pairs of every box with one synchronisation
  // (the totals gathered into the lead's page-locked slots by one kernel per
  // PIN_COUNT boxes)
  for (int q = 0; q < nl; ++q) BATCH_TRY(live[q], build_pairs_count(cs[live[q]], 1, 1.0f, nullptr));
  std::vector<int32_t> np(nl);
  SPH_TRY(sph_ensure(lead, lead->gather_src, sizeof(const int32_t *) * PIN_COUNT));
  lead->gather_host.resize(sizeof(const int32_t *) * PIN_COUNT);
  const int32_t **src = reinterpret_cast<const int32_t **>(lead->gather_host.data());
  for (int g0 = 0; g0 < nl; g0 += PIN_COUNT) {
    const int ng = std::min(nl - g0, (int)PIN_COUNT);
    for (int q = 0; q < ng; ++q) {
      sph_ctx *c = cs[live[g0 + q]];
      src[q] = (const int32_t *)c->fpair_off.p + c->n_active_leaves;
    }
    HIP_TRY(lead, hipMemcpyAsync(lead->gather_src.p, src, sizeof(const int32_t *) * (size_t)ng,
                                 hipMemcpyHostToDevice, lead->stream));
    gather_totals_kernel<<<1, 64, 0, lead->stream>>>((const int32_t *const *)lead->gather_src.p, ng, lead->pin_dev);
    HIP_TRY(lead, hipGetLastError());
    HIP_TRY(lead, hipStreamSynchronize(lead->stream));
    SPH_TRY(pin_fetch(lead, 0, ng));
    for (int q = 0; q < ng; ++q) np[g0 + q] = lead->pin_h[q];
  }
  for (int q = 0; q < nl; ++q) BATCH_TRY(live[q], build_pairs_fill(cs[live[q]], 1, 1.0f, np[q]));
  Staging s = staging(lead, nl);
  int64_t nchunks = 0;
  for (int b : live) nchunks += cs[b]->n_chunks;
  const LoopConfig cfg = batch_config(lead, 1, nchunks);
  const int target = split_target(cfg.split);
  int64_t total;
  SPH_TRY(batch_work_list(lead, cs, live, s, 1, target, &total));
  SPH_TRY(sph_ensure(lead, lead->batch_args, sizeof(LoopArgs) * (size_t)nl));
  for (int q = 0; q < nl; ++q) {
    s.args[q] = force_loop_args(cs[live[q]], &ps[live[q]]);
    batch_split_args(cs[live[q]], target, s.args[q]);
  }
  HIP_TRY(lead, hipMemcpyAsync(lead->batch_args.p, s.args, sizeof(LoopArgs) * nl, hipMemcpyHostToDevice,
                               lead->stream));
  if (lead->prm.compensated)
    SPH_TRY((batch_launch<1, true>(lead, cfg, total, "force_loop")));
  else
    SPH_TRY((batch_launch<1, false>(lead, cfg, total, "force_loop")));
  for (int b : live) cs[b]->state = 5;
  return SPH_OK;
}

sph_status batch_autotune_impl(sph_ctx **cs, sph_particles *ps, int nb, const char *path) {
  SPH_TRY(batch_check(cs, nb, 5, "batch_autotune"));
  sph_ctx *lead = cs[0];
  HIP_TRY(lead, hipStreamSynchronize(lead->stream));
  std::vector<int> live;
  for (int b = 0; b < nb; ++b)
    if (cs[b]->n_active > 0) live.push_back(b);
  if (live.empty()) return SPH_OK;
  const int nl = (int)live.size();
  Staging s = staging(lead, nl);
  int64_t nchunks = 0;
  for (int b : live) nchunks += cs[b]->n_chunks;
  SPH_TRY(sph_ensure(lead, lead->batch_args, sizeof(LoopArgs) * (size_t)nl));
  SPH_TRY(sph_ensure(lead, lead->batch_status, 8 * (size_t)nl + 64));
  // counts of tuning launches are not interactions of a step
  unsigned long long *scratch_ctr = (unsigned long long *)((char *)lead->batch_status.p + 8 * (size_t)nl);
  const int cls = tune_class(nchunks);
  const int prof = lead->prof;
  lead->prof = 0;
  FILE *f = path ? fopen(path, "a") : nullptr;
  hipEvent_t e0, e1;
  HIP_TRY(lead, hipEventCreate(&e0));
  HIP_TRY(lead, hipEventCreate(&e1));
  sph_status st = SPH_OK;
  // the work list and per-box arguments of a split class; returns the item count
  auto prepare = [&](int mode, int split, int64_t *total) -> sph_status {
    const int target = split_target(split);
    SPH_TRY(batch_work_list(lead, cs, live, s, 1, target, total));
    HIP_TRY(lead, hipStreamSynchronize(lead->stream));
    for (int q = 0; q < nl; ++q) {
      s.args[q] = mode == 0 ? density_loop_args(cs[live[q]]) : force_loop_args(cs[live[q]], &ps[live[q]]);
      batch_split_args(cs[live[q]], target, s.args[q]);
      if (mode == 1) s.args[q].ctr = scratch_ctr;
    }
    HIP_TRY(lead, hipMemcpyAsync(lead->batch_args.p, s.args, sizeof(LoopArgs) * nl, hipMemcpyHostToDevice,
                                 lead->stream));
    return SPH_OK;
  };
  // one timed launch of a configuration
  auto time_once = [&](int mode, const LoopConfig &c, int64_t total, float *ms) -> sph_status {
    batch_todo_kernel<<<dim3(grid_x_for(nchunks), nl), 256, 0, lead->stream>>>(
        (const BatchItems *)lead->batch_items.p);
    HIP_TRY(lead, hipEventRecord(e0, lead->stream));
    SPH_TRY((mode == 0 ? batch_launch<0, true>(lead, c, total, "tune")
                       : batch_launch<1, true>(lead, c, total, "tune")));
    HIP_TRY(lead, hipEventRecord(e1, lead->stream));
    HIP_TRY(lead, hipEventSynchronize(e1));
    HIP_TRY(lead, hipEventElapsedTime(ms, e0, e1));
    return SPH_OK;
  };
  for (int mode = 0; mode < 2 && st == SPH_OK; ++mode) {
    sph_ctx::TuneEntry best;
    best.ms = INFINITY;
    std::vector<Timed> scan;
    for (int split = 0; split <= 2 && st == SPH_OK; ++split) {
      int64_t total = 0;
      st = prepare(mode, split, &total);
      if (st != SPH_OK) break;
      const int nws[4] = {1, 2, 4, 8};
      for (int wi = 0; wi < 4 && st == SPH_OK; ++wi)
        for (int tile = 0; tile <= 4 && st == SPH_OK; ++tile)
          for (int pers = 0; pers <= 1 && st == SPH_OK; ++pers) {
            LoopConfig c;
            c.nw = nws[wi];
            c.tile = tile;
            c.ordered = 1;
            c.persistent = pers;
            c.split = split;
            if (!loop_config_valid(c)) continue;
            float bestc = INFINITY;
            for (int r = 0; r <= 2 && st == SPH_OK; ++r) {
              float ms = 0.f;
              st = time_once(mode, c, total, &ms);
              if (r > 0 && ms < bestc) bestc = ms;  // the first launch warms caches
            }
            if (st != SPH_OK) break;
            if (f)
              fprintf(f, "batch_candidate %d %d %d %d %d %d %d %.6f %lld\n", mode, cls, c.nw, c.tile, c.ordered,
                      c.persistent, c.split, bestc, (long long)nchunks);
            scan.push_back({c, bestc});
          }
    }
    if (st != SPH_OK) break;
    // the three fastest timed again, five launches each (after one warm-up):
    // smallest median wins, the scan's order deciding between medians within 3 %
    std::sort(scan.begin(), scan.end(), [](const Timed &x, const Timed &y) { return x.ms < y.ms; });
    const int nf = std::min<int>(3, (int)scan.size());
    int win = -1;
    float win_med = INFINITY;
    for (int q = 0; q < nf && st == SPH_OK; ++q) {
      int64_t total = 0;
      st = prepare(mode, scan[q].c.split, &total);
      std::vector<float> v;
      for (int r = 0; r <= 5 && st == SPH_OK; ++r) {
        float ms = 0.f;
        st = time_once(mode, scan[q].c, total, &ms);
        if (r > 0) v.push_back(ms);
      }
      if (st != SPH_OK) break;
      std::sort(v.begin(), v.end());
      const float med = v[v.size() / 2];
      if (win < 0 || med < 0.97f * win_med) {
        win = q;
        win_med = med;
      }
    }
    if (st == SPH_OK && win >= 0) {
      best.valid = 1;
      best.nw = scan[win].c.nw;
      best.tile = scan[win].c.tile;
      best.ordered = 1;
      best.persistent = scan[win].c.persistent;
      best.split = scan[win].c.split;
      best.ms = win_med;
      lead->btune[mode][cls] = best;
      if (f)
        fprintf(f, "batch_best %d %d %d %d %d %d %d %.6f %lld\n", mode, cls, best.nw, best.tile, best.ordered,
                best.persistent, best.split, best.ms, (long long)nchunks);
    }
  }
  if (f) fclose(f);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  lead->prof = prof;
  if (st != SPH_OK) return st;
  // leave every chunk marked done, as after a completed pass
  for (int b : live)
    HIP_TRY(lead, hipMemsetAsync(cs[b]->chunk_todo.p, 0, 4 * (size_t)cs[b]->n_chunks, lead->stream));
  HIP_TRY(lead, hipStreamSynchronize(lead->stream));
  return SPH_OK;
}
