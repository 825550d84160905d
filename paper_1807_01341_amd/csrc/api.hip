// Public C-ABI entry points: argument and call-order checks around the stages.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "sph_internal.h"

static hipEvent_t take_event(sph_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(sph_ctx *c, const char *name) : ctx(c), on(c && c->prof) {
  if (!on) return;
  ev.name = name;
  ev.a = take_event(ctx);
  ev.b = take_event(ctx);
  if (!ev.a || !ev.b) {
    on = false;
    return;
  }
  (void)hipEventRecord(ev.a, ctx->stream);
}

ProfScope::~ProfScope() {
  if (!on) return;
  (void)hipEventRecord(ev.b, ctx->stream);
  ctx->pending.push_back(ev);
}

static void resolve_profile(sph_ctx *ctx) {
  if (ctx->pending.empty()) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &p : ctx->pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    bool found = false;
    for (auto &a : ctx->acc)
      if (a.name == p.name) {
        a.count += 1;
        a.ms += ms;
        found = true;
        break;
      }
    if (!found) ctx->acc.push_back({p.name, 1, (double)ms});
    ctx->event_pool.push_back(p.a);
    ctx->event_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

// ---------------------------------------------------------------- context set-up

static bool params_valid(const sph_params *p) {
  return p->box > 0 && p->morton_depth >= 2 && p->morton_depth <= 21 && p->split_count >= 2 && p->top_cap >= 2 &&
         p->top_cap <= 8 && p->n_bins >= 1 && p->n_bins <= 63 && p->h_max_iter >= 1 && p->eta > 0 &&
         p->gamma > 1.0 && p->cand_cap >= 64 && p->list_cap >= 64 && p->chunk_split >= 0 && p->chunk_split <= 2 &&
         p->rebuild_frac >= 0.f && p->rebuild_frac <= 1.f && p->pair_slack >= 1.f && p->pair_slack <= 2.f &&
         (p->lazy_drift == 0 || p->lazy_drift == 1) && p->sweep_below >= 0 &&
         (p->sweep_waves == 0 || p->sweep_waves == 1 || p->sweep_waves == 2 || p->sweep_waves == 4) &&
         (p->waves_per_chunk == 0 || p->waves_per_chunk == 1 || p->waves_per_chunk == 2 || p->waves_per_chunk == 4 ||
          p->waves_per_chunk == 8);
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) p[s] = 0;
}

sph_status ctx_init(sph_ctx *ctx, const sph_params *p, void *hip_stream, sph_alloc_fn alloc, sph_free_fn free_fn,
                    void *user, bool mapped) {
  if ((alloc == nullptr) != (free_fn == nullptr) || !params_valid(p)) return SPH_EINVAL;
  ctx->prm = *p;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->mem.alloc = alloc;
  ctx->mem.free = free_fn;
  ctx->mem.user = user;
  ctx->mem.stream = ctx->stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) return SPH_EDEVICE;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && ncu > 0)
    ctx->n_cu = ncu;
  SPH_TRY(sph_ensure(ctx, ctx->scalars, sizeof(int32_t) * SC_COUNT));
  SPH_TRY(sph_ensure(ctx, ctx->counters64, 2 * sizeof(uint64_t)));
  if (mapped) {
    // page-locked, mapped and coherent: copies land in it without a staging
    // wait, and small kernels write their results into it directly
    if (hipHostMalloc((void **)&ctx->pin.p, sizeof(int32_t) * PIN_COUNT,
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      ctx->pin.p = nullptr;
      return SPH_ENOMEM;
    }
    if (hipHostGetDevicePointer((void **)&ctx->pin_dev, ctx->pin.p, 0) != hipSuccess || !ctx->pin_dev)
      return SPH_EDEVICE;
    ctx->pin_h = ctx->pin.p;
    ctx->pin_mapped = 1;
  } else {
    SPH_TRY(sph_ensure(ctx, ctx->pin_devbuf, sizeof(int32_t) * PIN_COUNT));
    ctx->pin_dev = (int32_t *)ctx->pin_devbuf.p;
    ctx->pin_h = ctx->pin_local;
    ctx->pin_mapped = 0;
  }
  // the counters start at zero (a kernel, not a memset node: the set-up may
  // run inside a caller's stream capture)
  zero_i32_kernel<<<1, 256, 0, ctx->stream>>>((int32_t *)ctx->scalars.p, SC_COUNT);
  zero_i32_kernel<<<1, 256, 0, ctx->stream>>>((int32_t *)ctx->counters64.p, 4);
  if (!mapped) zero_i32_kernel<<<1, 256, 0, ctx->stream>>>(ctx->pin_dev, PIN_COUNT);
  if (hipGetLastError() != hipSuccess) return SPH_EDEVICE;
  return SPH_OK;
}

// ---------------------------------------------------------------- batch contexts


// A failing box's status, with its message copied to the batch context.
static sph_status box_fail(sph_ctx *ctx, size_t b, sph_status s) {
  if (s == SPH_OK) return s;
  return sph_fail(ctx, s, "box %zu: %s", b, ctx->kids[b]->err.c_str());
}

__global__ void add_offset_kernel(int64_t *p, int64_t n, int64_t off) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) p[s] += off;
}

static bool is_batch(const sph_ctx *ctx) { return ctx && !ctx->kids.empty(); }

extern "C" {

sph_status sph_profile(sph_ctx *ctx, int enable) {
  if (!ctx) return SPH_EINVAL;
  for (sph_ctx *k : ctx->kids) SPH_TRY(sph_profile(k, enable));
  resolve_profile(ctx);
  ctx->acc.clear();
  ctx->prof = enable;
  return SPH_OK;
}

int64_t sph_profile_read(sph_ctx *ctx, char *buf, int64_t cap) {
  if (!ctx) return -1;
  resolve_profile(ctx);
  // a batch context reports its boxes' launches (batched ones are recorded by the first box)
  std::vector<sph_ctx::Acc> acc = ctx->acc;
  for (sph_ctx *k : ctx->kids) {
    resolve_profile(k);
    for (auto &a : k->acc) {
      bool found = false;
      for (auto &b : acc)
        if (b.name == a.name) {
          b.count += a.count;
          b.ms += a.ms;
          found = true;
        }
      if (!found) acc.push_back(a);
    }
  }
  std::string s;
  char line[256];
  for (auto &a : acc) {
    snprintf(line, sizeof line, "%s %ld %.6f\n", a.name.c_str(), a.count, a.ms);
    s += line;
  }
  if (buf && cap > 0) {
    const int64_t m = (int64_t)s.size() < cap - 1 ? (int64_t)s.size() : cap - 1;
    memcpy(buf, s.data(), (size_t)m);
    buf[m] = 0;
  }
  return (int64_t)s.size();
}

void sph_default_params(sph_params *p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->box = 1.0;
  p->gamma = 5.0 / 3.0;
  p->cfl = 0.2;
  p->eta = 1.2348f;
  p->alpha = 0.8f;
  p->balsara_eps = 1e-4f;
  p->h_tol = 1e-6f;
  p->n_bins = 14;
  p->split_count = 400;
  p->morton_depth = 16;
  p->top_cap = 7;
  p->h_max_iter = 30;
  p->compensated = 1;
  p->cand_cap = 512;
  p->list_cap = 96;
  p->rebuild_frac = 0.125f;
  p->pair_slack = 1.1f;
  p->lazy_drift = 0;
  p->sweep_below = 1 << 18;
}

sph_status sph_create(const sph_params *p, void *hip_stream, sph_alloc_fn alloc, sph_free_fn free_fn, void *user,
                      sph_ctx **out) {
  if (!p || !out) return SPH_EINVAL;
  *out = nullptr;
  sph_ctx *ctx = new (std::nothrow) sph_ctx();
  if (!ctx) return SPH_ENOMEM;
  const sph_status st = ctx_init(ctx, p, hip_stream, alloc, free_fn, user, true);
  if (st != SPH_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return SPH_OK;
}

void sph_destroy(sph_ctx *ctx) {
  if (!ctx) return;
  for (sph_ctx *k : ctx->kids) sph_destroy(k);
  ctx->kids.clear();
  (void)hipStreamSynchronize(ctx->stream);
  resolve_profile(ctx);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  // every DevBuf member frees its allocation
  delete ctx;
}

static sph_status need_state(sph_ctx *ctx, int at_least, const char *call) {
  if (!ctx) return SPH_EINVAL;
  if (is_batch(ctx)) return sph_fail(ctx, SPH_EINVAL, "%s: not for batch contexts (see sph_batch_box)", call);
  if (ctx->state < at_least) return sph_fail(ctx, SPH_ESTATE, "%s called out of order (state %d)", call, ctx->state);
  return SPH_OK;
}

sph_status sph_batch_create(sph_ctx *ctx, int n_boxes, const int64_t *box_offsets_host, const double *box_L_host) {
  if (!ctx) return SPH_EINVAL;
  if (is_batch(ctx)) return sph_fail(ctx, SPH_ESTATE, "batch_create: already a batch context");
  if (ctx->n_full_builds != 0 || ctx->state != 0)
    return sph_fail(ctx, SPH_ESTATE, "batch_create: the context has been used");
  if (n_boxes < 1 || !box_offsets_host || !box_L_host)
    return sph_fail(ctx, SPH_EINVAL, "batch_create: need n_boxes >= 1, offsets and box sides");
  if (ctx->prm.lazy_drift) return sph_fail(ctx, SPH_EINVAL, "batch_create: batched passes need lazy_drift = 0");
  if (box_offsets_host[0] != 0) return sph_fail(ctx, SPH_EINVAL, "batch_create: box_offsets[0] must be 0");
  for (int b = 0; b < n_boxes; ++b) {
    if (box_offsets_host[b + 1] <= box_offsets_host[b])
      return sph_fail(ctx, SPH_EINVAL, "batch_create: box %d is empty or the offsets decrease", b);
    if (!(box_L_host[b] > 0.0)) return sph_fail(ctx, SPH_EINVAL, "batch_create: box %d has side <= 0", b);
  }
  std::vector<sph_ctx *> kids;
  for (int b = 0; b < n_boxes; ++b) {
    sph_params q = ctx->prm;
    q.box = box_L_host[b];
    sph_ctx *k = nullptr;
    const sph_status st = sph_create(&q, (void *)ctx->stream, ctx->mem.alloc, ctx->mem.free, ctx->mem.user, &k);
    if (st != SPH_OK) {
      for (sph_ctx *c : kids) sph_destroy(c);
      return sph_fail(ctx, st, "batch_create: box %d: context not created", b);
    }
    kids.push_back(k);
  }
  ctx->kids = kids;
  ctx->box_off.assign(box_offsets_host, box_offsets_host + n_boxes + 1);
  return SPH_OK;
}

sph_ctx *sph_batch_box(sph_ctx *ctx, int b) {
  if (!is_batch(ctx) || b < 0 || b >= (int)ctx->kids.size()) return nullptr;
  return ctx->kids[b];
}

sph_status sph_build_cells(sph_ctx *ctx, sph_particles *p, int64_t n, int64_t *perm_out) {
  if (!ctx) return SPH_EINVAL;
  if (is_batch(ctx)) {
    if (!p) return sph_fail(ctx, SPH_EINVAL, "build_cells: null particles");
    if (n != ctx->box_off.back())
      return sph_fail(ctx, SPH_EINVAL, "build_cells: n = %lld, the boxes hold %lld", (long long)n,
                      (long long)ctx->box_off.back());
    const std::vector<sph_particles> sl = box_slices(ctx, p);
    for (size_t b = 0; b < ctx->kids.size(); ++b) {
      const int64_t off = ctx->box_off[b], nb = ctx->box_off[b + 1] - off;
      sph_particles q = sl[b];
      SPH_TRY(box_fail(ctx, b, build_cells_impl(ctx->kids[b], &q, nb, perm_out ? perm_out + off : nullptr)));
      if (perm_out && off > 0) {
        add_offset_kernel<<<(unsigned)std::min<int64_t>(ceil_div(nb, 256), 4096), 256, 0, ctx->stream>>>(
            perm_out + off, nb, off);
        HIP_TRY(ctx, hipGetLastError());
      }
    }
    return SPH_OK;
  }
  return build_cells_impl(ctx, p, n, perm_out);
}

sph_status sph_sort_cells(sph_ctx *ctx) {
  if (is_batch(ctx)) {
    for (size_t b = 0; b < ctx->kids.size(); ++b) SPH_TRY(box_fail(ctx, b, sph_sort_cells(ctx->kids[b])));
    return SPH_OK;
  }
  SPH_TRY(need_state(ctx, 1, "sort_cells"));
  return sort_cells_impl(ctx);
}

sph_status sph_batch_mark_active(sph_ctx *ctx, const sph_particles *p, const int *max_active_bin_host,
                                 int64_t *n_active_host) {
  if (!is_batch(ctx)) return ctx ? sph_fail(ctx, SPH_EINVAL, "batch_mark_active: not a batch context") : SPH_EINVAL;
  if (!p || !max_active_bin_host) return sph_fail(ctx, SPH_EINVAL, "batch_mark_active: null argument");
  const std::vector<sph_particles> sl = box_slices(ctx, p);
  int64_t tot = 0;
  for (size_t b = 0; b < ctx->kids.size(); ++b) {
    int64_t na = 0;
    SPH_TRY(box_fail(ctx, b, sph_mark_active(ctx->kids[b], &sl[b], max_active_bin_host[b], &na)));
    tot += na;
  }
  if (n_active_host) *n_active_host = tot;
  return SPH_OK;
}

sph_status sph_mark_active(sph_ctx *ctx, const sph_particles *p, int max_active_bin, int64_t *n_active_host) {
  if (is_batch(ctx)) {
    std::vector<int> m(ctx->kids.size(), max_active_bin);
    return sph_batch_mark_active(ctx, p, m.data(), n_active_host);
  }
  SPH_TRY(need_state(ctx, 2, "mark_active"));
  return mark_active_impl(ctx, p, max_active_bin, n_active_host);
}

sph_status sph_density_pass(sph_ctx *ctx, sph_particles *p, int entropy_from_u) {
  if (is_batch(ctx)) {
    if (!p) return sph_fail(ctx, SPH_EINVAL, "density_pass: null particles");
    std::vector<sph_particles> sl = box_slices(ctx, p);
    const sph_status st = batch_density_impl(ctx->kids.data(), sl.data(), (int)sl.size(), entropy_from_u);
    return st == SPH_OK ? st : sph_fail(ctx, st, "%s", ctx->kids[0]->err.c_str());
  }
  SPH_TRY(need_state(ctx, 3, "density_pass"));
  if (!p) return sph_fail(ctx, SPH_EINVAL, "density_pass: null particles");
  return density_pass_impl(ctx, p, entropy_from_u);
}

sph_status sph_force_pass(sph_ctx *ctx, sph_particles *p) {
  if (is_batch(ctx)) {
    if (!p) return sph_fail(ctx, SPH_EINVAL, "force_pass: null particles");
    std::vector<sph_particles> sl = box_slices(ctx, p);
    const sph_status st = batch_force_impl(ctx->kids.data(), sl.data(), (int)sl.size());
    return st == SPH_OK ? st : sph_fail(ctx, st, "%s", ctx->kids[0]->err.c_str());
  }
  SPH_TRY(need_state(ctx, 4, "force_pass"));
  if (!p) return sph_fail(ctx, SPH_EINVAL, "force_pass: null particles");
  return force_pass_impl(ctx, p);
}

sph_status sph_batch_density_force(sph_ctx *ctx, sph_particles *p, int entropy_from_u) {
  if (!is_batch(ctx)) return ctx ? sph_fail(ctx, SPH_EINVAL, "batch_density_force: not a batch context") : SPH_EINVAL;
  SPH_TRY(sph_density_pass(ctx, p, entropy_from_u));
  return sph_force_pass(ctx, p);
}

sph_status sph_batch_density_pass(sph_ctx **ctxs, sph_particles *ps, int n_boxes, int entropy_from_u) {
  if (!ps) return ctxs && n_boxes > 0 && ctxs[0] ? sph_fail(ctxs[0], SPH_EINVAL, "batch: null particles") : SPH_EINVAL;
  return batch_density_impl(ctxs, ps, n_boxes, entropy_from_u);
}

sph_status sph_batch_force_pass(sph_ctx **ctxs, sph_particles *ps, int n_boxes) {
  if (!ps) return ctxs && n_boxes > 0 && ctxs[0] ? sph_fail(ctxs[0], SPH_EINVAL, "batch: null particles") : SPH_EINVAL;
  return batch_force_impl(ctxs, ps, n_boxes);
}

sph_status sph_batch_autotune(sph_ctx **ctxs, sph_particles *ps, int n_boxes, const char *path) {
  if (!ps) return ctxs && n_boxes > 0 && ctxs[0] ? sph_fail(ctxs[0], SPH_EINVAL, "batch: null particles") : SPH_EINVAL;
  return batch_autotune_impl(ctxs, ps, n_boxes, path);
}

sph_status sph_adjoint(sph_ctx *ctx, sph_particles *p, const float *wx, const float *wy, const float *wz, double *gx,
                       double *gy, double *gz, float *gu) {
  if (is_batch(ctx)) return sph_fail(ctx, SPH_EINVAL, "adjoint: not for batch contexts");
  SPH_TRY(need_state(ctx, 5, "adjoint"));
  if (!p) return sph_fail(ctx, SPH_EINVAL, "adjoint: null particles");
  return adjoint_impl(ctx, p, wx, wy, wz, gx, gy, gz, gu);
}

sph_status sph_kick_drift(sph_ctx *ctx, sph_particles *p, int64_t ti, double t_min, int64_t drift_int,
                          int first_step) {
  if (is_batch(ctx)) {
    if (!p) return sph_fail(ctx, SPH_EINVAL, "kick_drift: null particles");
    std::vector<sph_particles> sl = box_slices(ctx, p);
    for (size_t b = 0; b < ctx->kids.size(); ++b)
      SPH_TRY(box_fail(ctx, b, sph_kick_drift(ctx->kids[b], &sl[b], ti, t_min, drift_int, first_step)));
    return SPH_OK;
  }
  SPH_TRY(need_state(ctx, 5, "kick_drift"));
  if (!p) return sph_fail(ctx, SPH_EINVAL, "kick_drift: null particles");
  return kick_drift_impl(ctx, p, ti, t_min, drift_int, first_step);
}

sph_status sph_step(sph_ctx *ctx, sph_particles *p, int64_t n, int64_t *perm_out, int max_active_bin,
                    int64_t *n_active_host, int entropy_from_u, int64_t ti, double t_min, int64_t drift_int,
                    int first_step) {
  SPH_TRY(sph_build_cells(ctx, p, n, perm_out));
  SPH_TRY(sph_sort_cells(ctx));
  SPH_TRY(sph_mark_active(ctx, p, max_active_bin, n_active_host));
  SPH_TRY(sph_density_pass(ctx, p, entropy_from_u));
  SPH_TRY(sph_force_pass(ctx, p));
  return sph_kick_drift(ctx, p, ti, t_min, drift_int, first_step);
}

sph_status sph_drift(sph_ctx *ctx, sph_particles *p, double t_min, int64_t drift_int) {
  if (!ctx) return SPH_EINVAL;
  if (!p) return sph_fail(ctx, SPH_EINVAL, "drift: null particles");
  if (is_batch(ctx)) {
    std::vector<sph_particles> sl = box_slices(ctx, p);
    for (size_t b = 0; b < ctx->kids.size(); ++b)
      SPH_TRY(box_fail(ctx, b, sph_drift(ctx->kids[b], &sl[b], t_min, drift_int)));
    return SPH_OK;
  }
  if (ctx->n_full_builds == 0 || ctx->state != 0)
    return sph_fail(ctx, SPH_ESTATE, "drift: only after a build and the step's kick_drift (state %d)", ctx->state);
  return drift_impl(ctx, p, t_min, drift_int);
}

sph_status sph_next_active_time(sph_ctx *ctx, const sph_particles *p, int64_t ti, int64_t *ti_next) {
  if (!ctx) return SPH_EINVAL;
  if (!p || !p->time_bin || !ti_next || ti < 0)
    return sph_fail(ctx, SPH_EINVAL, "next_active_time: null argument or ti < 0");
  if (is_batch(ctx)) {
    std::vector<sph_particles> sl = box_slices(ctx, p);
    int64_t best = INT64_MAX;
    for (size_t b = 0; b < ctx->kids.size(); ++b) {
      int64_t t = 0;
      SPH_TRY(box_fail(ctx, b, next_active_impl(ctx->kids[b], sl[b].time_bin, ctx->kids[b]->n, ti, &t)));
      best = std::min(best, t);
    }
    *ti_next = best;
    return SPH_OK;
  }
  return next_active_impl(ctx, p->time_bin, ctx->n, ti, ti_next);
}

sph_status sph_drift_all(sph_ctx *ctx, sph_particles *p) {
  if (!ctx) return SPH_EINVAL;
  if (is_batch(ctx)) return SPH_OK;  // batch contexts drift every particle in kick_drift
  if (!p) return sph_fail(ctx, SPH_EINVAL, "drift_all: null particles");
  if (!ctx->prm.lazy_drift || ctx->n_leaves == 0 || ctx->built_n != ctx->n) return SPH_OK;
  return drift_leaves(ctx, p, nullptr, nullptr, 0);
}

sph_status sph_sync(sph_ctx *ctx) {
  if (!ctx) return SPH_EINVAL;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}

const char *sph_last_error(const sph_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

sph_status sph_info(sph_ctx *ctx, sph_info_t *out) {
  if (!ctx || !out) return SPH_EINVAL;
  if (is_batch(ctx)) {
    // sums over the boxes (density_iterations, top_level: the largest; dx_max: the largest)
    memset(out, 0, sizeof *out);
    for (size_t b = 0; b < ctx->kids.size(); ++b) {
      sph_info_t k;
      SPH_TRY(box_fail(ctx, b, sph_info(ctx->kids[b], &k)));
      out->n += k.n;
      out->n_leaves += k.n_leaves;
      out->top_level = std::max(out->top_level, k.top_level);
      out->n_active += k.n_active;
      out->n_active_leaves += k.n_active_leaves;
      out->n_density_pairs += k.n_density_pairs;
      out->n_force_pairs += k.n_force_pairs;
      out->density_iterations = std::max(out->density_iterations, k.density_iterations);
      out->n_unconverged += k.n_unconverged;
      out->interactions_density += k.interactions_density;
      out->interactions_force += k.interactions_force;
      for (int q = 0; q < 32; ++q) out->unconverged_after_pass[q] += k.unconverged_after_pass[q];
      out->pair_rebuilds += k.pair_rebuilds;
      out->full_builds += k.full_builds;
      out->cell_updates += k.cell_updates;
      out->dx_max = std::max(out->dx_max, k.dx_max);
      out->device_bytes += k.device_bytes;
    }
    out->device_bytes += ctx->mem.live_bytes;
    return SPH_OK;
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  out->n = ctx->n;
  out->n_leaves = ctx->n_leaves;
  out->top_level = ctx->top_level;
  out->n_active = ctx->n_active;
  out->n_active_leaves = ctx->n_active_leaves;
  out->n_density_pairs = ctx->n_dpairs;
  out->n_force_pairs = ctx->n_fpairs;
  out->density_iterations = ctx->density_iterations;
  out->n_unconverged = ctx->n_unconverged;
  uint64_t c[2] = {0, 0};
  HIP_TRY(ctx, hipMemcpy(c, ctx->counters64.p, sizeof c, hipMemcpyDeviceToHost));
  out->interactions_density = (int64_t)c[0];
  out->interactions_force = (int64_t)c[1];
  for (int q = 0; q < 32; ++q) out->unconverged_after_pass[q] = ctx->unconv_hist[q];
  out->pair_rebuilds = ctx->pair_rebuilds;
  out->full_builds = ctx->n_full_builds;
  out->cell_updates = ctx->n_updates;
  out->dx_max = ctx->dx_max;
  out->device_bytes = ctx->mem.live_bytes;
  return SPH_OK;
}

static sph_status copy_dev(sph_ctx *ctx, void *dst, const DevBuf &src, size_t bytes) {
  if (!dst || bytes == 0) return SPH_OK;
  if (!src.p || src.cap < bytes) return sph_fail(ctx, SPH_ESTATE, "copy: structure not built");
  HIP_TRY(ctx, hipMemcpyAsync(dst, src.p, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  return SPH_OK;
}

sph_status sph_copy_leaves(sph_ctx *ctx, int32_t *level, int32_t *ix, int32_t *iy, int32_t *iz, int32_t *begin,
                           int32_t *count, float *hmax, float *drift) {
  SPH_TRY(need_state(ctx, 1, "copy_leaves"));
  const size_t nl = (size_t)ctx->n_leaves;
  SPH_TRY(copy_dev(ctx, level, ctx->leaf_level, 4 * nl));
  SPH_TRY(copy_dev(ctx, ix, ctx->leaf_ix, 4 * nl));
  SPH_TRY(copy_dev(ctx, iy, ctx->leaf_iy, 4 * nl));
  SPH_TRY(copy_dev(ctx, iz, ctx->leaf_iz, 4 * nl));
  SPH_TRY(copy_dev(ctx, begin, ctx->leaf_begin, 4 * nl));
  SPH_TRY(copy_dev(ctx, count, ctx->leaf_count, 4 * nl));
  SPH_TRY(copy_dev(ctx, hmax, ctx->leaf_hmax, 4 * nl));
  if (drift) SPH_TRY(copy_dev(ctx, drift, ctx->leaf_dx, 4 * nl));
  return SPH_OK;
}

__global__ void split_pos4_kernel(const float4 *__restrict__ pos4, int64_t n, float *ox, float *oy, float *oz) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) {
    const float4 q = pos4[s];
    if (ox) ox[s] = q.x;
    if (oy) oy[s] = q.y;
    if (oz) oz[s] = q.z;
  }
}

sph_status sph_copy_particles(sph_ctx *ctx, uint64_t *keys, float *ox, float *oy, float *oz) {
  SPH_TRY(need_state(ctx, 1, "copy_particles"));
  SPH_TRY(copy_dev(ctx, keys, ctx->keys_a, 8 * (size_t)ctx->n));
  if (ox || oy || oz) {
    int64_t g = ceil_div(ctx->n, 256);
    if (g > 8192) g = 8192;
    split_pos4_kernel<<<(unsigned)g, 256, 0, ctx->stream>>>((const float4 *)ctx->pos4.p, ctx->n, ox, oy, oz);
    HIP_TRY(ctx, hipGetLastError());
  }
  return SPH_OK;
}

sph_status sph_copy_axis_order(sph_ctx *ctx, uint16_t *order) {
  SPH_TRY(need_state(ctx, 2, "copy_axis_order"));
  SPH_TRY(sort_all_leaves(ctx));
  return copy_dev(ctx, order, ctx->axis_order, 2 * 13 * (size_t)ctx->n);
}

sph_status sph_copy_active(sph_ctx *ctx, uint8_t *active, int32_t *active_leaves, float *hmax_act) {
  SPH_TRY(need_state(ctx, 3, "copy_active"));
  SPH_TRY(copy_dev(ctx, active, ctx->active, (size_t)ctx->n));
  SPH_TRY(copy_dev(ctx, active_leaves, ctx->act_leaves, 4 * (size_t)ctx->n_active_leaves));
  SPH_TRY(copy_dev(ctx, hmax_act, ctx->act_hmax, 4 * (size_t)ctx->n_active_leaves));
  return SPH_OK;
}

__global__ void split_pairs_kernel(const PairEntry *__restrict__ pe, const int32_t *__restrict__ off,
                                   const int32_t *__restrict__ act_leaves, int64_t nal, int32_t *a, int32_t *b,
                                   float *sx, float *sy, float *sz) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nal; q += (int64_t)gridDim.x * 256) {
    const int A = act_leaves[q];
    for (int p = off[q]; p < off[q + 1]; ++p) {
      const PairEntry e = pe[p];
      if (a) a[p] = A;
      if (b) b[p] = e.b;
      if (sx) sx[p] = e.sx;
      if (sy) sy[p] = e.sy;
      if (sz) sz[p] = e.sz;
    }
  }
}

sph_status sph_copy_pairs(sph_ctx *ctx, int which, int32_t *a, int32_t *b, float *sx, float *sy, float *sz) {
  SPH_TRY(need_state(ctx, which == 0 ? 3 : 5, "copy_pairs"));
  const int64_t nal = ctx->n_active_leaves;
  if (nal == 0) return SPH_OK;
  const DevBuf &off = which == 0 ? ctx->dpair_off : ctx->fpair_off;
  const DevBuf &lst = which == 0 ? ctx->dpairs : ctx->fpairs;
  int64_t g = ceil_div(nal, 256);
  if (g > 8192) g = 8192;
  split_pairs_kernel<<<(unsigned)g, 256, 0, ctx->stream>>>((const PairEntry *)lst.p, (const int32_t *)off.p,
                                                         (const int32_t *)ctx->act_leaves.p, nal, a, b, sx, sy, sz);
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}

}  // extern "C"
