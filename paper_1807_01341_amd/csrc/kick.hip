// Kick-drift-kick with individual power-of-two time-steps (Sec. II-A, Eq. 1,
// Eq. 2).  FP64 for positions and velocities.
#include <limits.h>
#include <math.h>

#include <algorithm>

#include "sph_internal.h"

struct KickArgs {
  int64_t n;
  double *x, *y, *z, *vx, *vy, *vz, *vfx, *vfy, *vfz;
  float *A, *Af, *h;
  const float *ax, *ay, *az, *dA, *vsig, *divv;
  int8_t *bin;
  const uint8_t *active;
  int64_t ti, drift_int;
  double t_min, L, cfl;
  int n_bins, first, ctz_ti;
  int kick;  // 0: drift only (no particle is active)
};

__device__ __forceinline__ double wrap_box_k(double x, double L) {
  const double q = floor(x / L);
  double xw = x - q * L;
  if (xw < 0.0) xw += L;
  if (xw >= L) xw -= L;
  return xw;
}

__global__ __launch_bounds__(256) void kick_drift_kernel(KickArgs g) {
  const double dt = (double)g.drift_int * g.t_min;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < g.n; s += (int64_t)gridDim.x * 256) {
    const double a0 = g.ax[s], a1 = g.ay[s], a2 = g.az[s], da = g.dA[s];
    double vf0 = g.vfx[s], vf1 = g.vfy[s], vf2 = g.vfz[s];
    double v0 = g.vx[s], v1 = g.vy[s], v2 = g.vz[s];
    double Af = g.Af[s], A = g.A[s];
    if (g.kick && g.active[s]) {
      if (!g.first) {
        // closing half-kick of the step that ends now
        const double h0 = 0.5 * ldexp(g.t_min, (int)g.bin[s]);
        vf0 = vf0 + a0 * h0;
        vf1 = vf1 + a1 * h0;
        vf2 = vf2 + a2 * h0;
        Af = Af + da * h0;
      }
      v0 = vf0;
      v1 = vf1;
      v2 = vf2;
      A = Af;
      // Eq. 1 then Eq. 2: largest n with 2^n t_min <= dt, within the bins
      // whose period divides the current time
      const double vs = g.vsig[s];
      const double dtn = vs > 0.0 ? g.cfl * (double)g.h[s] / vs : INFINITY;
      int nb = 0;
      for (int b = 1; b < g.n_bins; ++b)
        if (dtn >= ldexp(g.t_min, b)) nb = b;
      if (g.ti != 0 && nb > g.ctz_ti) nb = g.ctz_ti;
      g.bin[s] = (int8_t)nb;
      const double h1 = 0.5 * ldexp(g.t_min, nb);
      vf0 = vf0 + a0 * h1;
      vf1 = vf1 + a1 * h1;
      vf2 = vf2 + a2 * h1;
      Af = Af + da * h1;
      g.vfx[s] = vf0;
      g.vfy[s] = vf1;
      g.vfz[s] = vf2;
      g.Af[s] = (float)Af;
    }
    g.x[s] = wrap_box_k(g.x[s] + vf0 * dt, g.L);
    g.y[s] = wrap_box_k(g.y[s] + vf1 * dt, g.L);
    g.z[s] = wrap_box_k(g.z[s] + vf2 * dt, g.L);
    g.vx[s] = v0 + a0 * dt;
    g.vy[s] = v1 + a1 * dt;
    g.vz[s] = v2 + a2 * dt;
    g.A[s] = (float)(A + da * dt);
    // smoothing length carried along the flow: continuity with h ~ rho^(-1/3)
    // gives dh/dt = +(h/3) div v; at most a factor e^0.2 per drift.  An
    // inactive particle's h is the H_j its neighbours' force loops read.
    if (g.divv) {
      double x = (double)g.divv[s] * dt / 3.0;
      x = fmin(fmax(x, -0.2), 0.2);
      g.h[s] = (float)((double)g.h[s] * exp(x));
    }
  }
}

// Lazy drift: the kicks of the active particles only (the same formulas as
// above: closing half-kick, Eq. 1 / Eq. 2 bin, opening half-kick, v = vf,
// A = Af); their drift, like every other particle's, waits until a step
// needs them.  Each kicked particle raises its leaf's speed bound.
__global__ __launch_bounds__(256) void kick_active_kernel(KickArgs g, const int32_t *__restrict__ active_idx,
                                                          int64_t n_act, const int32_t *__restrict__ leaf_of,
                                                          float *__restrict__ leaf_vmax) {
  const int lane = threadIdx.x & 63;
  // whole waves per iteration (lanes past the end idle), so that the lanes
  // of a leaf can combine their speed bounds
  for (int64_t k0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); k0 < n_act; k0 += (int64_t)gridDim.x * 256) {
    const int64_t k = k0 + lane;
    int key = -1, bits = 0;
    if (k < n_act) {
      const int s = active_idx[k];
      const double a0 = g.ax[s], a1 = g.ay[s], a2 = g.az[s], da = g.dA[s];
      double vf0 = g.vfx[s], vf1 = g.vfy[s], vf2 = g.vfz[s];
      double Af = g.Af[s];
      if (!g.first) {
        const double h0 = 0.5 * ldexp(g.t_min, (int)g.bin[s]);
        vf0 = vf0 + a0 * h0;
        vf1 = vf1 + a1 * h0;
        vf2 = vf2 + a2 * h0;
        Af = Af + da * h0;
      }
      g.vx[s] = vf0;
      g.vy[s] = vf1;
      g.vz[s] = vf2;
      g.A[s] = (float)Af;
      const double vs = g.vsig[s];
      const double dtn = vs > 0.0 ? g.cfl * (double)g.h[s] / vs : INFINITY;
      int nb = 0;
      for (int b = 1; b < g.n_bins; ++b)
        if (dtn >= ldexp(g.t_min, b)) nb = b;
      if (g.ti != 0 && nb > g.ctz_ti) nb = g.ctz_ti;
      g.bin[s] = (int8_t)nb;
      const double h1 = 0.5 * ldexp(g.t_min, nb);
      vf0 = vf0 + a0 * h1;
      vf1 = vf1 + a1 * h1;
      vf2 = vf2 + a2 * h1;
      Af = Af + da * h1;
      g.vfx[s] = vf0;
      g.vfy[s] = vf1;
      g.vfz[s] = vf2;
      g.Af[s] = (float)Af;
      const double v = sqrt(vf0 * vf0 + vf1 * vf1 + vf2 * vf2);
      if (v > 0.0) {
        key = leaf_of[s];
        bits = __float_as_int((float)v) + 1;  // (positive floats order as their bits)
      }
    }
    // one atomic per leaf of the wave (active particles are in cell order:
    // a wave spans few leaves), with the largest bound of its lanes
    bool pend = bits > 0;
    for (uint64_t m = __ballot(pend); m != 0ull; m = __ballot(pend)) {
      const int src = __ffsll((unsigned long long)m) - 1;
      const int L = __shfl(key, src, 64);
      const bool mine = pend && key == L;
      const int top = wave_max_i(mine ? bits : 0);
      if (lane == src) atomicMax((int *)&leaf_vmax[L], top);
      pend = pend && !mine;
    }
  }
}

static bool kick_arrays_present(const sph_particles *p) {
  return p->x && p->y && p->z && p->vx && p->vy && p->vz && p->vfx && p->vfy && p->vfz && p->A && p->Af && p->ax &&
         p->ay && p->az && p->dA_dt && p->h && p->vsig && p->time_bin;
}

static KickArgs kick_args(sph_ctx *ctx, sph_particles *p, int64_t ti, double t_min, int64_t drift_int,
                          int first_step) {
  KickArgs g;
  g.n = ctx->n;
  g.x = p->x; g.y = p->y; g.z = p->z;
  g.vx = p->vx; g.vy = p->vy; g.vz = p->vz;
  g.vfx = p->vfx; g.vfy = p->vfy; g.vfz = p->vfz;
  g.A = p->A; g.Af = p->Af;
  g.ax = p->ax; g.ay = p->ay; g.az = p->az; g.dA = p->dA_dt; g.h = p->h; g.vsig = p->vsig;
  g.divv = p->divv;
  g.bin = p->time_bin;
  g.active = (const uint8_t *)ctx->active.p;
  g.ti = ti;
  g.drift_int = drift_int;
  g.t_min = t_min;
  g.L = ctx->prm.box;
  g.cfl = ctx->prm.cfl;
  g.n_bins = ctx->prm.n_bins;
  g.first = first_step;
  g.ctz_ti = ti != 0 ? __builtin_ctzll((unsigned long long)ti) : 0;
  g.kick = 1;
  return g;
}

sph_status kick_drift_impl(sph_ctx *ctx, sph_particles *p, int64_t ti, double t_min, int64_t drift_int,
                           int first_step) {
  if (!kick_arrays_present(p)) return sph_fail(ctx, SPH_EINVAL, "kick_drift: a state array is missing");
  if (!(t_min > 0.0) || drift_int < 0 || ti < 0) return sph_fail(ctx, SPH_EINVAL, "kick_drift: bad time arguments");
  KickArgs g = kick_args(ctx, p, ti, t_min, drift_int, first_step);
  if (ctx->prm.lazy_drift) {
    // the time line advances; drifts happen when steps need them
    if (ctx->t_min_line != 0.0 && t_min != ctx->t_min_line)
      return sph_fail(ctx, SPH_EINVAL, "kick_drift: lazy drift needs one t_min for the whole time line");
    const int64_t na = ctx->n_active;
    if (na > 0) {
      PROF(ctx, "kick_drift");
      kick_active_kernel<<<(unsigned)std::min<int64_t>(ceil_div(na, 256), 8192), 256, 0, ctx->stream>>>(
          g, (const int32_t *)ctx->active_idx.p, na, (const int32_t *)ctx->leaf_of.p, (float *)ctx->leaf_vmax.p);
    }
    HIP_TRY(ctx, hipGetLastError());
    ctx->t_min_line = t_min;
    ctx->ti_now += drift_int;
    ctx->state = 0;
    return SPH_OK;
  }
  int64_t grid = ceil_div(g.n, 256);
  if (grid > 8192) grid = 8192;
  {
    PROF(ctx, "kick_drift");
    kick_drift_kernel<<<(unsigned)grid, 256, 0, ctx->stream>>>(g);
  }
  HIP_TRY(ctx, hipGetLastError());
  ctx->state = 0;
  return SPH_OK;
}

// Drift with no kick: the time line moves on by drift_int units of t_min
// over times at which no particle is active.  With lazy drift only the line
// moves (drifts happen when steps need them); else every particle drifts.
sph_status drift_impl(sph_ctx *ctx, sph_particles *p, double t_min, int64_t drift_int) {
  if (!kick_arrays_present(p)) return sph_fail(ctx, SPH_EINVAL, "drift: a state array is missing");
  if (!(t_min > 0.0) || drift_int < 0) return sph_fail(ctx, SPH_EINVAL, "drift: bad time arguments");
  if (ctx->prm.lazy_drift) {
    if (ctx->t_min_line != 0.0 && t_min != ctx->t_min_line)
      return sph_fail(ctx, SPH_EINVAL, "drift: lazy drift needs one t_min for the whole time line");
    ctx->t_min_line = t_min;
    ctx->ti_now += drift_int;
    return SPH_OK;
  }
  if (drift_int == 0) return SPH_OK;
  KickArgs g = kick_args(ctx, p, 0, t_min, drift_int, 0);
  g.kick = 0;
  g.active = nullptr;
  int64_t grid = ceil_div(g.n, 256);
  if (grid > 8192) grid = 8192;
  {
    PROF(ctx, "drift");
    kick_drift_kernel<<<(unsigned)grid, 256, 0, ctx->stream>>>(g);
  }
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}

// ---------------------------------------------------------------- next active time
//
// A particle in bin b is active at the multiples of 2^b (Sec. II-A), so the
// first time after ti at which anything is active is the next multiple of
// 2^b_min, b_min the smallest bin any particle holds; the times in between
// have no active particle and take no step.

__global__ __launch_bounds__(64) void set_i32_kernel(int32_t *__restrict__ p, int32_t v) {
  if (threadIdx.x == 0) p[0] = v;
}

__global__ __launch_bounds__(256) void min_bin_kernel(const int8_t *__restrict__ bin, int64_t n,
                                                      int32_t *__restrict__ out) {
  int m = INT_MAX;
  // 16 bins per load where the array is 16-byte aligned, single bins for the rest
  const int64_t head = (int64_t)((16 - ((uintptr_t)bin & 15)) & 15);
  const int64_t h = head < n ? head : n;
  const int64_t nv = (n - h) >> 4;
  const int4 *v = reinterpret_cast<const int4 *>(bin + h);
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
  for (int64_t s = tid; s < nv; s += stride) {
    const int4 w = v[s];
    const int32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b) m = min(m, (int)(int8_t)(ws[q] >> (8 * b)));
  }
  for (int64_t s = tid; s < h; s += stride) m = min(m, (int)bin[s]);
  for (int64_t s = h + (nv << 4) + tid; s < n; s += stride) m = min(m, (int)bin[s]);
  for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
  // one atomic per block (a single address: contended atomics serialise)
  __shared__ int wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMin(out, min(min(wm[0], wm[1]), min(wm[2], wm[3])));
}

sph_status next_active_impl(sph_ctx *ctx, const int8_t *bin, int64_t n, int64_t ti, int64_t *ti_next) {
  if (n <= 0) return sph_fail(ctx, SPH_ESTATE, "next_active_time: no particles (build_cells first)");
  int32_t *slot = (int32_t *)ctx->scalars.p + SC_MINBIN;
  set_i32_kernel<<<1, 64, 0, ctx->stream>>>(slot, INT_MAX);
  const int64_t grid = std::min<int64_t>(ceil_div(n, 256 * 16 * 4), 512) + 1;
  min_bin_kernel<<<(unsigned)grid, 256, 0, ctx->stream>>>(bin, n, slot);
  HIP_TRY(ctx, hipGetLastError());
  int32_t b = 0;
  SPH_TRY(read_scalars(ctx, SC_MINBIN, 1, &b));
  if (b < 0 || b >= ctx->prm.n_bins)
    return sph_fail(ctx, SPH_ESTATE, "next_active_time: a time-bin outside [0, %d)", ctx->prm.n_bins);
  const int64_t period = (int64_t)1 << b;
  *ti_next = (ti / period + 1) * period;
  return SPH_OK;
}
