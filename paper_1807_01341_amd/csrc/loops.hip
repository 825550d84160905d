// Single-box passes: the density loop with the ghost's h solve, and the
// force loop, over the active chunks of one context.
#include <stdio.h>

#include "loops_common.h"

namespace {

__global__ __launch_bounds__(256) void fill_work_kernel(const int32_t *__restrict__ order, int64_t n,
                                                        int2 *__restrict__ work) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    work[q] = make_int2(0, order ? order[q] : (int)q);
}

__global__ __launch_bounds__(256) void pack_jvm_kernel(const double *__restrict__ vx, const double *__restrict__ vy,
                                                       const double *__restrict__ vz, const float *__restrict__ m,
                                                       int64_t n, float4 *__restrict__ out) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256)
    out[s] = make_float4((float)vx[s], (float)vy[s], (float)vz[s], m[s]);
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
                                                           float *__restrict__ hi, uint8_t *__restrict__ conv) {
  const int64_t m = n_chunks > n_act ? n_chunks : n_act;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < m; s += (int64_t)gridDim.x * 256) {
    if (s < n_chunks) todo[s] = 1;
    if (s < n_act) {
      lo[s] = 0.f;
      hi[s] = INFINITY;
      conv[s] = 0;
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

// Chunks in decreasing order of staged partner particles (longest first),
// by log2 buckets: histogram, bucket offsets, scatter.
__global__ __launch_bounds__(256) void cost_bucket_kernel(const Chunk *__restrict__ chunks, int64_t n_chunks,
                                                          const int32_t *__restrict__ act_cost,
                                                          int32_t *__restrict__ bucket_of,
                                                          int32_t *__restrict__ hist) {
  __shared__ int h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n_chunks; q += (int64_t)gridDim.x * 256) {
    const int cost = max(1, act_cost[chunks[q].act_leaf]);
    const int b = __clz(cost);  // larger cost, smaller bucket
    bucket_of[q] = b;
    atomicAdd(&h[b], 1);
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

__global__ __launch_bounds__(256) void cost_scatter_kernel(const int32_t *__restrict__ bucket_of, int64_t n_chunks,
                                                           int32_t *__restrict__ cursor, int32_t *__restrict__ work) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n_chunks; q += (int64_t)gridDim.x * 256)
    work[atomicAdd(&cursor[bucket_of[q]], 1)] = (int32_t)q;
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
  const auto &t = ctx->tune[mode][cls];
  LoopConfig c;
  if (t.valid) {
    c.nw = t.nw;
    c.tile = t.tile;
    c.ordered = t.ordered;
    c.persistent = t.persistent;
    return c;
  }
  if (ctx->prm.waves_per_chunk > 0) {
    c.nw = ctx->prm.waves_per_chunk;
    c.tile = c.nw >= 4 ? 1 : 2;
    const int cap = ctx->prm.cand_cap, lcap = ctx->prm.list_cap;
    if (c.nw == 1) c.tile = cap <= 128 && lcap <= 32 ? 0 : cap <= 256 && lcap <= 64 ? 1 : cap <= 512 && lcap <= 96 ? 2 : cap <= 1024 && lcap <= 128 ? 3 : 4;
    if (c.nw == 2) c.tile = cap <= 128 && lcap <= 32 ? 0 : cap <= 256 && lcap <= 64 ? 1 : 2;
    if (c.nw >= 4) c.tile = cap <= 128 && lcap <= 32 ? 0 : 1;
    return c;
  }
  const int64_t nc = ctx->n_chunks;
  if (nc < 2048) {
    c.nw = 8, c.tile = 0, c.ordered = 1;
  } else if (nc < 8192) {
    c.nw = 4, c.tile = 1, c.ordered = 1;
  } else if (nc < 32768) {
    c.nw = 2, c.tile = 2;
  } else {
    c.nw = 1, c.tile = 2;
  }
  return c;
}

sph_status order_chunks_by_cost(sph_ctx *ctx) {
  const int64_t nc = ctx->n_chunks;
  SPH_TRY(sph_ensure(ctx, ctx->work, 4 * (size_t)(nc > 0 ? nc : 1)));
  SPH_TRY(sph_ensure(ctx, ctx->work_tmp, 4 * (size_t)(nc > 0 ? nc : 1) + 256));
  int32_t *bucket_of = (int32_t *)ctx->work_tmp.p + 64;
  int32_t *hist = (int32_t *)ctx->work_tmp.p;
  HIP_TRY(ctx, hipMemsetAsync(hist, 0, 32 * sizeof(int32_t), ctx->stream));
  PROF(ctx, "cost_order");
  cost_bucket_kernel<<<grid_for_items(nc), 256, 0, ctx->stream>>>((const Chunk *)ctx->chunks.p, nc,
                                                                 (const int32_t *)ctx->act_cost.p, bucket_of, hist);
  cost_bucket_scan_kernel<<<1, 64, 0, ctx->stream>>>(hist);
  cost_scatter_kernel<<<grid_for_items(nc), 256, 0, ctx->stream>>>(bucket_of, nc, hist, (int32_t *)ctx->work.p);
  return sph_hip_check(ctx, hipGetLastError(), "cost order");
}

template <int MODE, bool COMP>
sph_status launch_loop(sph_ctx *ctx, const LoopArgs &a0) {
  const LoopConfig cfg = choose_config(ctx, MODE);
  LoopArgs a = a0;
  if (cfg.ordered) {
    if (!ctx->work_valid) {
      SPH_TRY(order_chunks_by_cost(ctx));
      ctx->work_valid = 1;
    }
    a.work = (const int32_t *)ctx->work.p;
    a.n_items = ctx->n_chunks;
  }
  PROF(ctx, MODE == 0 ? "density_loop" : "force_loop");
  if (cfg.persistent) {
    // one box through the persistent kernel: a device copy of the arguments
    // and a (0, chunk) work list
    SPH_TRY(sph_ensure(ctx, ctx->box_args, sizeof(LoopArgs)));
    SPH_TRY(sph_ensure(ctx, ctx->box_work, sizeof(int2) * (size_t)(ctx->n_chunks > 0 ? ctx->n_chunks : 1)));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->box_args.p, &a, sizeof(LoopArgs), hipMemcpyHostToDevice, ctx->stream));
    fill_work_kernel<<<grid_for_items(ctx->n_chunks), 256, 0, ctx->stream>>>(
        cfg.ordered ? (const int32_t *)ctx->work.p : nullptr, ctx->n_chunks, (int2 *)ctx->box_work.p);
    HIP_TRY(ctx, hipGetLastError());
    return sph_hip_check(ctx,
                         launch_loop_any<MODE, COMP>(ctx->stream, a, cfg, (const LoopArgs *)ctx->box_args.p,
                                                     (const int2 *)ctx->box_work.p, (int)ctx->n_chunks,
                                                     (int *)ctx->scalars.p + SC_WORKCTR, persistent_grid_for(ctx->n_cu, cfg)),
                         MODE == 0 ? "density loop" : "force loop");
  }
  return sph_hip_check(ctx, launch_loop_any<MODE, COMP>(ctx->stream, a, cfg, nullptr, nullptr, 0, nullptr, 0),
                       MODE == 0 ? "density loop" : "force loop");
}

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
  a.axis_order = (const uint16_t *)ctx->axis_order.p;
  a.n = ctx->n;
  a.ax = host_axes();
  a.n_active = ctx->n_active;
  a.half_alpha = 0.5f * ctx->prm.alpha;
  a.gm1 = (float)(ctx->prm.gamma - 1.0);
  return a;
}

}  // namespace

// Per-particle neighbour data in cell order, packed once per build: velocity
// and mass, and the density-loop state (rho, f P/rho^2, c, B) that inactive
// neighbours keep from their last active step.  The ghost refreshes the
// latter for every active particle it finishes.
sph_status pack_neighbour_data(sph_ctx *ctx, const sph_particles *p) {
  const int64_t n = ctx->n;
  SPH_TRY(sph_ensure(ctx, ctx->jvm, 16 * (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->jth, 16 * (size_t)n));
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

sph_status density_pass_impl(sph_ctx *ctx, sph_particles *p, int entropy_from_u) {
  if (!p->vx || !p->vy || !p->vz || !p->m || !p->h)
    return sph_fail(ctx, SPH_EINVAL, "density_pass: v, m and h are required");
  if (!p->rho || !p->drho_dh || !p->f_gradh || !p->divv || !p->curlx || !p->curly || !p->curlz || !p->P || !p->c ||
      !p->balsara || !p->A)
    return sph_fail(ctx, SPH_EINVAL, "density_pass: an output array is missing");
  if (entropy_from_u && !p->u) return sph_fail(ctx, SPH_EINVAL, "density_pass: u is required with entropy_from_u");
  const int64_t n = ctx->n, na = ctx->n_active;
  ctx->density_iterations = 0;
  ctx->n_unconverged = 0;
  ctx->pair_rebuilds = 0;
  for (int q = 0; q < 32; ++q) ctx->unconv_hist[q] = 0;
  (void)n;
  if (na == 0) {
    ctx->state = 4;
    return SPH_OK;
  }
  SPH_TRY(sph_ensure(ctx, ctx->sums, sizeof(float) * 9 * (size_t)na));
  SPH_TRY(sph_ensure(ctx, ctx->hlo, 4 * (size_t)na));
  SPH_TRY(sph_ensure(ctx, ctx->hhi, 4 * (size_t)na));
  SPH_TRY(sph_ensure(ctx, ctx->conv, (size_t)na));
  {
    PROF(ctx, "ghost");
    density_init_kernel<<<grid256(na > ctx->n_chunks ? na : ctx->n_chunks), 256, 0, ctx->stream>>>(
        ctx->n_chunks, (int32_t *)ctx->chunk_todo.p, na, (float *)ctx->hlo.p, (float *)ctx->hhi.p,
        (uint8_t *)ctx->conv.p);
  }
  HIP_TRY(ctx, hipGetLastError());

  int32_t *sc = (int32_t *)ctx->scalars.p;
  const float G = (float)ctx->prm.gamma;
  const double kc = (8.0 / M_PI) / ((double)GK32 * GK32 * GK32);
  const int maxit = ctx->prm.h_max_iter;
  for (int it = 1; it <= maxit; ++it) {
    LoopArgs a = base_args(ctx);
    a.pair_off = (const int32_t *)ctx->dpair_off.p;
    a.pairs = (const PairEntry *)ctx->dpairs.p;
    a.sums = (float *)ctx->sums.p;
    a.act_cnt = (int32_t *)ctx->sums.p + 8 * na;
    if (ctx->prm.compensated)
      SPH_TRY((launch_loop<0, true>(ctx, a)));
    else
      SPH_TRY((launch_loop<0, false>(ctx, a)));
    HIP_TRY(ctx, hipMemsetAsync(sc + SC_UNCONV, 0, 8, ctx->stream));
    GhostArgs gh;
    gh.n_active = na;
    gh.active_idx = (const int32_t *)ctx->active_idx.p;
    gh.chunk_of = (const int32_t *)ctx->chunk_of.p;
    gh.chunks = (const Chunk *)ctx->chunks.p;
    gh.chunk_todo = (int32_t *)ctx->chunk_todo.p;
    gh.sums = (const float *)ctx->sums.p;
    gh.act_cnt = (const int32_t *)ctx->sums.p + 8 * na;
    gh.act_hmax = (const float *)ctx->act_hmax.p;
    gh.hlo = (float *)ctx->hlo.p;
    gh.hhi = (float *)ctx->hhi.p;
    gh.conv = (uint8_t *)ctx->conv.p;
    gh.pos4 = (float4 *)ctx->pos4.p;
    gh.jth = (float4 *)ctx->jth.p;
    gh.h = p->h;
    gh.last = it == maxit;
    gh.from_u = entropy_from_u;
    gh.eta3 = ctx->prm.eta * ctx->prm.eta * ctx->prm.eta;
    gh.kc = (float)kc;
    gh.tol = ctx->prm.h_tol;
    gh.gamma = G;
    gh.eps = ctx->prm.balsara_eps;
    gh.box_quarter = (float)(0.25 * ctx->prm.box);
    gh.reach = ctx->dpair_slack;
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
    gh.u = p->u;
    gh.nngb = p->nngb_density;
    gh.n_unconv = sc + SC_UNCONV;
    gh.rebuild = sc + SC_REBUILD;
    gh.ctr = (unsigned long long *)ctx->counters64.p;
    {
      PROF(ctx, "ghost");
      ghost_kernel<<<grid256(na), 256, 0, ctx->stream>>>(gh);
    }
    HIP_TRY(ctx, hipGetLastError());
    int32_t st[2];
    SPH_TRY(read_scalars(ctx, SC_UNCONV, 2, st));
    ctx->density_iterations = it;
    if (it <= 32) ctx->unconv_hist[it - 1] = st[0];
    if (st[1] & 2) return sph_fail(ctx, SPH_EREBUILD, "density_pass: a smoothing length exceeds a quarter of the box");
    if (gh.last) {
      ctx->n_unconverged = st[0];
      break;
    }
    if (st[0] == 0) break;
    if (st[1] & 1) {
      // a smoothing length outgrew its cell's pair reach: widen the pair lists
      ctx->pair_rebuilds++;
      SPH_TRY(refresh_leaf_hmax(ctx, false));
      SPH_TRY(build_pairs(ctx, 0, 1.5f));
    }
  }
  // leaf max H follows the new smoothing lengths, so that any later cell-pair
  // list (the force list, or a later active set without a rebuild) sees them
  SPH_TRY(refresh_leaf_hmax(ctx, true));
  ctx->state = 4;
  if (ctx->n_unconverged > 0)
    return sph_fail(ctx, SPH_ENOCONV, "density_pass: %lld particles not converged after %d iterations",
                    (long long)ctx->n_unconverged, maxit);
  return SPH_OK;
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
  SPH_TRY(build_pairs(ctx, 1, 1.0f));
  fill_i32_kernel<<<grid256(ctx->n_chunks), 256, 0, ctx->stream>>>((int32_t *)ctx->chunk_todo.p, ctx->n_chunks, 1);
  HIP_TRY(ctx, hipGetLastError());
  LoopArgs a = base_args(ctx);
  a.pair_off = (const int32_t *)ctx->fpair_off.p;
  a.pairs = (const PairEntry *)ctx->fpairs.p;
  a.ax_out = p->ax;
  a.ay_out = p->ay;
  a.az_out = p->az;
  a.dA_out = p->dA_dt;
  a.du_out = p->du_dt;
  a.vsig_out = p->vsig;
  a.nngb_out = p->nngb_force;
  a.ctr = (unsigned long long *)ctx->counters64.p + 1;
  if (ctx->prm.compensated)
    SPH_TRY((launch_loop<1, true>(ctx, a)));
  else
    SPH_TRY((launch_loop<1, false>(ctx, a)));
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
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  float best = INFINITY;
  for (int r = 0; r <= reps; ++r) {
    fill_i32_kernel<<<grid256(ctx->n_chunks), 256, 0, ctx->stream>>>((int32_t *)ctx->chunk_todo.p, ctx->n_chunks, 1);
    LoopArgs a = a0;
    if (cfg.ordered) {
      a.work = (const int32_t *)ctx->work.p;
      a.n_items = ctx->n_chunks;
    }
    HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
    hipError_t err;
    if (cfg.persistent) {
      HIP_TRY(ctx, hipMemcpyAsync(ctx->box_args.p, &a, sizeof(LoopArgs), hipMemcpyHostToDevice, ctx->stream));
      fill_work_kernel<<<grid_for_items(ctx->n_chunks), 256, 0, ctx->stream>>>(
          cfg.ordered ? (const int32_t *)ctx->work.p : nullptr, ctx->n_chunks, (int2 *)ctx->box_work.p);
      err = launch_loop_any<MODE, true>(ctx->stream, a, cfg, (const LoopArgs *)ctx->box_args.p,
                                        (const int2 *)ctx->box_work.p, (int)ctx->n_chunks,
                                        (int *)ctx->scalars.p + SC_WORKCTR, persistent_grid_for(ctx->n_cu, cfg));
    } else {
      err = launch_loop_any<MODE, true>(ctx->stream, a, cfg, nullptr, nullptr, 0, nullptr, 0);
    }
    HIP_TRY(ctx, err);
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
    if (r > 0 && ms < best) best = ms;  // the first launch warms caches
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = best;
  return SPH_OK;
}

}  // namespace

extern "C" sph_status sph_autotune(sph_ctx *ctx, sph_particles *p, const char *path) {
  if (!ctx || !p) return SPH_EINVAL;
  if (ctx->state < 5) return sph_fail(ctx, SPH_ESTATE, "autotune: run a force pass first");
  if (ctx->n_chunks == 0) return SPH_OK;
  const int cls = tune_class(ctx->n_chunks);
  SPH_TRY(order_chunks_by_cost(ctx));
  ctx->work_valid = 1;
  SPH_TRY(sph_ensure(ctx, ctx->box_args, sizeof(LoopArgs)));
  SPH_TRY(sph_ensure(ctx, ctx->box_work, sizeof(int2) * (size_t)ctx->n_chunks));
  const int prof = ctx->prof;
  ctx->prof = 0;
  FILE *f = path ? fopen(path, "a") : nullptr;
  for (int mode = 0; mode < 2; ++mode) {
    LoopArgs a = base_args(ctx);
    if (mode == 0) {
      a.pair_off = (const int32_t *)ctx->dpair_off.p;
      a.pairs = (const PairEntry *)ctx->dpairs.p;
      a.sums = (float *)ctx->sums.p;
      a.act_cnt = (int32_t *)ctx->sums.p + 8 * ctx->n_active;
    } else {
      a.pair_off = (const int32_t *)ctx->fpair_off.p;
      a.pairs = (const PairEntry *)ctx->fpairs.p;
      a.ax_out = p->ax;
      a.ay_out = p->ay;
      a.az_out = p->az;
      a.dA_out = p->dA_dt;
      a.du_out = p->du_dt;
      a.vsig_out = p->vsig;
      a.nngb_out = p->nngb_force;
      // counts of tuning launches are not interactions of a step
      a.ctr = (unsigned long long *)ctx->work_tmp.p;
    }
    sph_ctx::TuneEntry best;
    best.ms = INFINITY;
    const int nws[4] = {1, 2, 4, 8};
    for (int wi = 0; wi < 4; ++wi)
      for (int tile = 0; tile <= 4; ++tile)
        for (int ordered = 0; ordered <= 1; ++ordered)
          for (int pers = 0; pers <= 1; ++pers) {
            LoopConfig c;
            c.nw = nws[wi];
            c.tile = tile;
            c.ordered = ordered;
            c.persistent = pers;
            if (!loop_config_valid(c)) continue;
            float ms = 0.f;
            if (mode == 0)
              SPH_TRY(time_config<0>(ctx, a, c, 2, &ms));
            else
              SPH_TRY(time_config<1>(ctx, a, c, 2, &ms));
            if (f)
              fprintf(f, "candidate %d %d %d %d %d %d %.6f %lld\n", mode, cls, c.nw, c.tile, c.ordered, c.persistent,
                      ms, (long long)ctx->n_chunks);
            if (ms < best.ms) {
              best.valid = 1;
              best.nw = c.nw;
              best.tile = c.tile;
              best.ordered = c.ordered;
              best.persistent = c.persistent;
              best.ms = ms;
            }
          }
    ctx->tune[mode][cls] = best;
    if (f)
      fprintf(f, "best %d %d %d %d %d %d %.6f %lld\n", mode, cls, best.nw, best.tile, best.ordered, best.persistent,
              best.ms, (long long)ctx->n_chunks);
  }
  if (f) fclose(f);
  ctx->prof = prof;
  // leave every chunk marked done, as after a completed pass
  HIP_TRY(ctx, hipMemsetAsync(ctx->chunk_todo.p, 0, 4 * (size_t)ctx->n_chunks, ctx->stream));
  return sph_sync(ctx);
}

extern "C" sph_status sph_load_tuning(sph_ctx *ctx, const char *path) {
  if (!ctx || !path) return SPH_EINVAL;
  FILE *f = fopen(path, "r");
  if (!f) return sph_fail(ctx, SPH_EINVAL, "load_tuning: cannot open %s", path);
  char tag[32];
  int mode, cls, nw, tile, ord, pers;
  float ms;
  long long nc;
  int loaded = 0;
  while (fscanf(f, "%31s %d %d %d %d %d %d %f %lld", tag, &mode, &cls, &nw, &tile, &ord, &pers, &ms, &nc) == 9) {
    if (strcmp(tag, "best") != 0 || mode < 0 || mode > 1 || cls < 0 || cls > 31) continue;
    LoopConfig c;
    c.nw = nw;
    c.tile = tile;
    if (!loop_config_valid(c)) continue;
    auto &t = ctx->tune[mode][cls];
    t.valid = 1;
    t.nw = nw;
    t.tile = tile;
    t.ordered = ord != 0;
    t.persistent = pers != 0;
    t.ms = ms;
    ++loaded;
  }
  fclose(f);
  return loaded > 0 ? SPH_OK : sph_fail(ctx, SPH_EINVAL, "load_tuning: no entries in %s", path);
}
