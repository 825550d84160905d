// Kick-drift-kick with individual power-of-two time-steps (Sec. II-A, Eq. 1,
// Eq. 2).  FP64 for positions and velocities.
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
    if (g.active[s]) {
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
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n_act; k += (int64_t)gridDim.x * 256) {
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
    if (v > 0.0) atomicMax((int *)&leaf_vmax[leaf_of[s]], __float_as_int((float)v) + 1);
  }
}

sph_status kick_drift_impl(sph_ctx *ctx, sph_particles *p, int64_t ti, double t_min, int64_t drift_int,
                           int first_step) {
  if (!p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->vfx || !p->vfy || !p->vfz || !p->A || !p->Af ||
      !p->ax || !p->ay || !p->az || !p->dA_dt || !p->h || !p->vsig || !p->time_bin)
    return sph_fail(ctx, SPH_EINVAL, "kick_drift: a state array is missing");
  if (!(t_min > 0.0) || drift_int < 0 || ti < 0) return sph_fail(ctx, SPH_EINVAL, "kick_drift: bad time arguments");
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
