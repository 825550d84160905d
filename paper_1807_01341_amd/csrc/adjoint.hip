// Reverse mode of one all-active density + force evaluation: given weights
// w_i = dL/da_i, the gradient of L = sum_i w_i . a_i with respect to the
// positions and internal energies.  Three loop passes over neighbours
// recomputed from the cell pairs (force adjoint; h derivatives of the density
// sums; position terms of the density sums and of the smoothing-length
// constraint) and two per-particle kernels (the ghost's reverse, and the
// constraint multiplier).  The forward is the density loop, ghost and force
// loop of Sec. III-A / Fig. 5 at converged smoothing lengths; dh/dx follows
// from the constraint h^3 n(h, x) = eta^3 by implicit differentiation, and
// the kinks min(0, .) and |.| take derivative 0 at 0.
#include "loops_common.h"

namespace {

constexpr int ADJ_CAP = 256, ADJ_LCAP = 64, ADJ_NW = 4;

unsigned grid_n(int64_t n) {
  int64_t g = ceil_div(n, 256);
  if (g > 8192) g = 8192;
  return (unsigned)(g < 1 ? 1 : g);
}

__global__ __launch_bounds__(256) void todo_all_kernel(int32_t *todo, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) todo[s] = 1;
}

__global__ __launch_bounds__(256) void pack_w_kernel(const float *__restrict__ wx, const float *__restrict__ wy,
                                                     const float *__restrict__ wz, int64_t n,
                                                     float4 *__restrict__ out) {
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256)
    out[s] = make_float4(wx[s], wy[s], wz[s], 0.f);
}

// Reverse of the ghost for one particle.  Inputs: the force adjoint's
// per-particle cotangents (rows: x3, f P/rho^2, h, c, B, rho).  Outputs
// (rho_bar, drho_dh_bar, D_bar, h_bar) with D the raw divergence sum
// (div v = -D/rho), C_bar (curl v = C/rho) and u_bar.
struct GhostAdjArgs {
  int64_t n;
  const float *fa;  // 8 x n
  const float *rho, *drho_dh, *f, *u, *c, *B, *divv, *curlx, *curly, *curlz, *h;
  float gamma, eps;
  float4 *adj1, *adj2;
  float *ubar;
};

__global__ __launch_bounds__(256) void ghost_adjoint_kernel(GhostAdjArgs g) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * 256) {
    const float Pfb = g.fa[3 * g.n + i], hb0 = g.fa[4 * g.n + i], cb0 = g.fa[5 * g.n + i];
    const float Bb = g.fa[6 * g.n + i], rb0 = g.fa[7 * g.n + i];
    const float rho = g.rho[i], drho = g.drho_dh[i], f = g.f[i], u = g.u[i], c = g.c[i], h = g.h[i];
    const float gm1 = g.gamma - 1.f;
    // f P / rho^2 = f (gamma-1) u / rho
    const float Pf = f * gm1 * u / rho;
    float rb = rb0 - Pfb * Pf / rho;
    const float fb = Pfb * gm1 * u / rho;
    float ub = Pfb * f * gm1 / rho;
    // f = 1 / (1 + z), z = h drho_dh / (3 rho)
    const float z = h * drho / (3.f * rho);
    const float zb = -f * f * fb;
    float hb = hb0 + zb * drho / (3.f * rho);
    const float drhob = zb * h / (3.f * rho);
    rb -= zb * z / rho;
    // Balsara B = a / (a + b + s): a = |div v|, b = |curl v|, s = eps c / h
    const float dv = g.divv[i];
    const float cx = g.curlx[i], cy = g.curly[i], cz = g.curlz[i];
    const float a = fabsf(dv);
    const float b = sqrtf(fmaf(cz, cz, fmaf(cy, cy, cx * cx)));
    const float s = g.eps * c / h;
    float Db = 0.f, Cbx = 0.f, Cby = 0.f, Cbz = 0.f, cb = cb0;
    if (a > 0.f) {
      const float den = a + b + s;
      const float id2 = 1.f / (den * den);
      const float ab = Bb * (b + s) * id2;
      const float bb = -Bb * a * id2;  // also the cotangent of s
      // a = |D| / rho with D = -rho div v
      Db = dv > 0.f ? -ab / rho : ab / rho;
      rb -= (ab * a + bb * b) / rho;
      if (b > 0.f) {
        const float kc = bb / (b * rho);
        Cbx = kc * cx;
        Cby = kc * cy;
        Cbz = kc * cz;
      }
      cb += bb * g.eps / h;
      hb -= bb * s / h;
    }
    // c = sqrt(gamma (gamma-1) u)
    ub += cb * c / (2.f * u);
    g.adj1[i] = make_float4(rb, drhob, Db, hb);
    g.adj2[i] = make_float4(Cbx, Cby, Cbz, 0.f);
    g.ubar[i] = ub;
  }
}

// Multiplier of the smoothing-length constraint Phi(h) = h^3 n(h) - eta^3:
// lambda = (total h cotangent) / (dPhi/dh), with the h derivatives of rho,
// drho/dh, D and C from the density adjoint sums (rows: sum w,
// sum (3w + q w'), sum m (12 w + 8 q w' + q^2 w''), and the sums of
// m (4 w' + q w'') / r times v.r and v x r).
__global__ __launch_bounds__(256) void lambda_kernel(int64_t n, const float *__restrict__ ds,
                                                     const float *__restrict__ h_, const float *__restrict__ drho_dh,
                                                     float4 *__restrict__ adj1, const float4 *__restrict__ adj2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float h = h_[i];
    const float H = GK32 * h;
    const float iH = 1.f / H;
    const float C3 = KNORM32 * iH * iH * iH;
    const float C4 = C3 * iH;
    const float Sw = ds[i], Sd = ds[n + i], Sm2 = ds[2 * n + i];
    const float Tv = ds[3 * n + i], Tx = ds[4 * n + i], Ty = ds[5 * n + i], Tz = ds[6 * n + i];
    const float ih = 1.f / h;
    // dPhi/dh = 3 h^2 n + h^3 n' = (C3 h^2) (3 sum w - sum (3w + q w'))
    const float dphi = C3 * h * h * (3.f * Sw - Sd);
    const float d2rho = C3 * ih * ih * Sm2;
    const float Dh = -C4 * ih * Tv;
    const float k = -C4 * ih;
    const float4 a1 = adj1[i];
    const float4 a2 = adj2[i];
    const float hbt = a1.w + a1.x * drho_dh[i] + a1.y * d2rho + a1.z * Dh + k * (a2.x * Tx + a2.y * Ty + a2.z * Tz);
    adj1[i].w = hbt / dphi;
  }
}

__global__ __launch_bounds__(256) void adjoint_out_kernel(int64_t n, const float *__restrict__ fa,
                                                          const float *__restrict__ da, double *__restrict__ gx,
                                                          double *__restrict__ gy, double *__restrict__ gz) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    gx[i] = (double)fa[i] + (double)da[i];
    gy[i] = (double)fa[n + i] + (double)da[n + i];
    gz[i] = (double)fa[2 * n + i] + (double)da[2 * n + i];
  }
}

template <int MODE>
sph_status adjoint_loop(sph_ctx *ctx, LoopArgs a, const char *what) {
  todo_all_kernel<<<grid_n(ctx->n_chunks), 256, 0, ctx->stream>>>((int32_t *)ctx->chunk_todo.p, ctx->n_chunks);
  HIP_TRY(ctx, hipGetLastError());
  LoopConfig cfg;
  cfg.nw = ADJ_NW;
  cfg.tile = 1;
  PROF(ctx, what);
  return sph_hip_check(ctx,
                       launch_loop_t<MODE, true, ADJ_CAP, ADJ_LCAP, ADJ_NW>(ctx->stream, a, cfg, nullptr, nullptr, 0,
                                                                            nullptr, 0),
                       what);
}

}  // namespace

sph_status adjoint_impl(sph_ctx *ctx, sph_particles *p, const float *wx, const float *wy, const float *wz,
                        double *gx, double *gy, double *gz, float *gu) {
  if (!wx || !wy || !wz || !gx || !gy || !gz || !gu)
    return sph_fail(ctx, SPH_EINVAL, "adjoint: a weight or gradient array is missing");
  if (!p->u || !p->h || !p->rho || !p->drho_dh || !p->f_gradh || !p->c || !p->balsara || !p->divv || !p->curlx ||
      !p->curly || !p->curlz)
    return sph_fail(ctx, SPH_EINVAL, "adjoint: the density-pass arrays and u are required");
  const int64_t n = ctx->n;
  if (ctx->n_active != n)
    return sph_fail(ctx, SPH_EINVAL, "adjoint: every particle must be active (%lld of %lld are)",
                    (long long)ctx->n_active, (long long)n);
  if (!ctx->density_from_u)
    return sph_fail(ctx, SPH_ESTATE, "adjoint: the density pass must take the pressure from u");
  SPH_TRY(sph_ensure(ctx, ctx->adj_w, 16 * (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->adj1, 16 * (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->adj2, 16 * (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->adj_out, sizeof(float) * 18 * (size_t)n));
  float *fa = (float *)ctx->adj_out.p;   // force adjoint, 8 rows
  float *ds = fa + 8 * n;                 // density h sums, 7 rows
  float *da = fa + 15 * n;                // density position terms, 3 rows
  {
    PROF(ctx, "adjoint_ghost");
    pack_w_kernel<<<grid_n(n), 256, 0, ctx->stream>>>(wx, wy, wz, n, (float4 *)ctx->adj_w.p);
  }
  HIP_TRY(ctx, hipGetLastError());

  // neighbour cell pairs at the converged smoothing lengths
  SPH_TRY(build_pairs(ctx, 0, 1.0f));
  SPH_TRY(build_pairs(ctx, 1, 1.0f));

  // 1. reverse of the force loop
  LoopArgs a = base_args(ctx);
  a.pair_off = (const int32_t *)ctx->fpair_off.p;
  a.pairs = (const PairEntry *)ctx->fpairs.p;
  a.pair_axis = (const uint8_t *)ctx->fpair_axis.p;
  a.jw = (const float4 *)ctx->adj_w.p;
  a.outp = fa;
  SPH_TRY(adjoint_loop<2>(ctx, a, "adjoint_force"));

  // 2. reverse of the ghost
  GhostAdjArgs g;
  g.n = n;
  g.fa = fa;
  g.rho = p->rho;
  g.drho_dh = p->drho_dh;
  g.f = p->f_gradh;
  g.u = p->u;
  g.c = p->c;
  g.B = p->balsara;
  g.divv = p->divv;
  g.curlx = p->curlx;
  g.curly = p->curly;
  g.curlz = p->curlz;
  g.h = p->h;
  g.gamma = (float)ctx->prm.gamma;
  g.eps = ctx->prm.balsara_eps;
  g.adj1 = (float4 *)ctx->adj1.p;
  g.adj2 = (float4 *)ctx->adj2.p;
  g.ubar = gu;
  {
    PROF(ctx, "adjoint_ghost");
    ghost_adjoint_kernel<<<grid_n(n), 256, 0, ctx->stream>>>(g);
  }
  HIP_TRY(ctx, hipGetLastError());

  // 3. h derivatives of the density sums, then the constraint multiplier
  a = base_args(ctx);
  a.pair_off = (const int32_t *)ctx->dpair_off.p;
  a.pairs = (const PairEntry *)ctx->dpairs.p;
  a.pair_axis = (const uint8_t *)ctx->dpair_axis.p;
  a.outp = ds;
  SPH_TRY(adjoint_loop<3>(ctx, a, "adjoint_density_h"));
  {
    PROF(ctx, "adjoint_ghost");
    lambda_kernel<<<grid_n(n), 256, 0, ctx->stream>>>(n, ds, p->h, p->drho_dh, (float4 *)ctx->adj1.p,
                                                      (const float4 *)ctx->adj2.p);
  }
  HIP_TRY(ctx, hipGetLastError());

  // 4. position terms of the density sums and of the constraint
  a = base_args(ctx);
  a.pair_off = (const int32_t *)ctx->fpair_off.p;
  a.pairs = (const PairEntry *)ctx->fpairs.p;
  a.pair_axis = (const uint8_t *)ctx->fpair_axis.p;
  a.jadj1 = (const float4 *)ctx->adj1.p;
  a.jadj2 = (const float4 *)ctx->adj2.p;
  a.outp = da;
  SPH_TRY(adjoint_loop<4>(ctx, a, "adjoint_density_x"));
  {
    PROF(ctx, "adjoint_ghost");
    adjoint_out_kernel<<<grid_n(n), 256, 0, ctx->stream>>>(n, fa, da, gx, gy, gz);
  }
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}
