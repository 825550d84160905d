// The neighbour loops over active cell pairs (Sec. III-A, Fig. 5): the density
// loop with the ghost's smoothing-length correction, and the force loop.
//
// Work item: one wave per chunk of up to 64 active particles of one leaf
// (gather formulation: each active particle's sums are produced by the single
// wave that owns it, in a fixed order, so there are no atomics and results are
// reproducible).  For every partner leaf of the chunk's cell-pair list:
//   1. staging: the partner's particles are read 64 at a time (coalesced SoA
//      loads, in the per-cell axis-sort order when the pair is not a self pair
//      so that the sweep stops once the projections leave the chunk's reach),
//      moved into the chunk leaf's frame with the FP32 pair shift, and kept if
//      they are within reach of the chunk's bounding box (wave ballot + rank
//      into an LDS candidate array);
//   2. filter: every lane tests its own particle against each candidate with
//      the FP32 predicate and appends hits to its own LDS neighbour list;
//   3. interact: every lane walks its own list (lanes have near-equal neighbour
//      counts because h adapts) and accumulates its sums in registers.
// No MFMA: pair interactions are not a dense contraction.
#include <math.h>
#include <string.h>

#include "sph_internal.h"

namespace {

struct AxisTab {
  float e[13][3];
};

AxisTab host_axes() {
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

struct LoopArgs {
  const Chunk *chunks;
  int32_t *chunk_todo;
  int64_t n_chunks;
  int64_t per_xcd;
  const int32_t *active_idx;
  const float4 *pos4;  // (ox, oy, oz, H)
  const float4 *jvm;   // (vx, vy, vz, m)
  const float4 *jth;   // (rho, f P / rho^2, c, B)  force only
  const int32_t *leaf_begin, *leaf_count;
  const float *leaf_hmax;
  const int32_t *pair_off;
  const PairEntry *pairs;
  const uint16_t *axis_order;
  int64_t n;
  AxisTab ax;
  // density outputs: per active index
  float *sums;
  int32_t *act_cnt;
  int64_t n_active;
  // force outputs: per particle
  float *ax_out, *ay_out, *az_out, *dA_out, *du_out, *vsig_out;
  int32_t *nngb_out;
  float half_alpha, gm1;
  unsigned long long *ctr;  // cumulative force interactions
};

__device__ __forceinline__ void kernel_w_dw(float q, float &w, float &wp) {
  // w = 1 - 6q^2 + 6q^3, w' = -12q + 18q^2 on [0, 1/2); 2(1-q)^3, -6(1-q)^2 on [1/2, 1)
  const float wi = fmaf(q * q, fmaf(6.f, q, -6.f), 1.f);
  const float wpi = q * fmaf(18.f, q, -12.f);
  const float t = 1.f - q;
  const float t2 = t * t;
  const float wo = 2.f * t2 * t;
  const float wpo = -6.f * t2;
  const bool in = q < 0.5f;
  w = in ? wi : wo;
  wp = in ? wpi : wpo;
}

__device__ __forceinline__ float kernel_dw_only(float q) {
  const float wpi = q * fmaf(18.f, q, -12.f);
  const float t = 1.f - q;
  const float wpo = -6.f * t * t;
  return q < 0.5f ? wpi : (q < 1.f ? wpo : 0.f);
}

struct Neu {  // compensated running sum
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float b) {
    const float t = s + b;
    if (fabsf(s) >= fabsf(b))
      c += (s - t) + b;
    else
      c += (b - t) + s;
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
};

struct Kahan {  // per-term compensated accumulator
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float b) {
    const float y = b - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
};

__device__ __forceinline__ int chunk_id(int64_t per_xcd, int64_t n_chunks) {
  // consecutive chunks (neighbours in Morton order) on the same XCD, so that
  // their shared partner cells are re-read from that XCD's L2
  const int64_t b = blockIdx.x;
  const int64_t cid = (b & 7) * per_xcd + (b >> 3);
  return cid < n_chunks ? (int)cid : -1;
}

// Orders this wave's LDS accesses across its lanes (each wave owns its own
// LDS region, so no workgroup barrier is needed between its phases).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// MODE 0: density loop; MODE 1: force loop.  NW waves share one chunk: wave w
// takes the partner cells w, w+NW, ... of the chunk's pair list, and the
// per-lane partial sums are combined across waves in wave order at the end.
template <int MODE, int CAP, int LCAP, bool COMP, int NW>
__global__ __launch_bounds__(64 * NW) void loop_kernel(LoopArgs g) {
  __shared__ float4 cand_all[NW][CAP];
  __shared__ float candH_all[NW][MODE == 1 ? CAP : 1];
  __shared__ uint16_t lists_all[NW][LCAP * 64];

  const int cid = chunk_id(g.per_xcd, g.n_chunks);
  if (cid < 0) return;
  if (!g.chunk_todo[cid]) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float4 *cand = cand_all[wave];
  float *candH = candH_all[wave];
  uint16_t *lists = lists_all[wave];
  const Chunk ch = g.chunks[cid];
  const bool live = lane < ch.count;
  const int k = ch.begin + lane;
  const int i = live ? g.active_idx[k] : -1;
  const float4 pi = live ? g.pos4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float Hi = pi.w;
  const float H2i = live ? Hi * Hi : -1.f;
  const float invHi = live ? 1.f / Hi : 0.f;
  const float4 vi = live ? g.jvm[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  float4 thi = make_float4(0.f, 0.f, 0.f, 0.f);
  if (MODE == 1 && live) thi = g.jth[i];

  // chunk bounding box and reach
  const float bminx = wave_min_f(live ? pi.x : INFINITY), bmaxx = wave_max_f(live ? pi.x : -INFINITY);
  const float bminy = wave_min_f(live ? pi.y : INFINITY), bmaxy = wave_max_f(live ? pi.y : -INFINITY);
  const float bminz = wave_min_f(live ? pi.z : INFINITY), bmaxz = wave_max_f(live ? pi.z : -INFINITY);
  const float Rc = wave_max_f(live ? Hi : 0.f);
  const float R2c = Rc * Rc;

  // accumulators: density (w, m w, 3w+qw', m(3w+qw'), div, curl x3); force (a x3, visc, adiab)
  float acc[9];
  Neu tot[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.f;
  Kahan ka[3];
  float vmax = 0.f;
  int cnt = 0;
  int len = 0;
  int ncand = 0;

  auto interact = [&]() {
    const int maxlen = wave_max_i(len);
    for (int t = 0; t < maxlen; ++t) {
      if (t < len) {
        const int c = lists[t * 64 + lane];
        const float4 cj = cand[c];
        const int j = __float_as_int(cj.w);
        const float dx = pi.x - cj.x, dy = pi.y - cj.y, dz = pi.z - cj.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float4 vj = g.jvm[j];
        const float rinv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
        const float r = r2 * rinv;
        const float vx = vi.x - vj.x, vy = vi.y - vj.y, vz = vi.z - vj.z;
        const float vr = fmaf(vz, dz, fmaf(vy, dy, vx * dx));
        const float mj = vj.w;
        if (MODE == 0) {
          float w, wp;
          const float q = r * invHi;
          kernel_w_dw(q, w, wp);
          const float d3 = fmaf(q, wp, 3.f * w);
          acc[0] += w;
          acc[1] = fmaf(mj, w, acc[1]);
          acc[2] += d3;
          acc[3] = fmaf(mj, d3, acc[3]);
          const float fac = mj * wp * rinv;
          acc[4] = fmaf(fac, vr, acc[4]);
          acc[5] = fmaf(fac, fmaf(vy, dz, -vz * dy), acc[5]);
          acc[6] = fmaf(fac, fmaf(vz, dx, -vx * dz), acc[6]);
          acc[7] = fmaf(fac, fmaf(vx, dy, -vy * dx), acc[7]);
          cnt += (j != i);
        } else {
          const float Hj = candH[c];
          const float invHj = __builtin_amdgcn_rcpf(Hj);
          const float4 th = g.jth[j];
          const float wpi = kernel_dw_only(r * invHi);
          const float wpj = kernel_dw_only(r * invHj);
          const float ih2 = invHj * invHj;
          const float Fi = (KNORM32 * invHi * invHi * invHi * invHi) * wpi * rinv;
          const float Fj = KNORM32 * (ih2 * ih2) * wpj * rinv;
          const float mu = fminf(vr * rinv, 0.f);
          const float vsig = thi.z + th.z - 3.f * mu;
          vmax = fmaxf(vmax, vsig);
          const float Pi = -g.half_alpha * vsig * mu * (thi.w + th.w) * __builtin_amdgcn_rcpf(thi.x + th.x);
          const float gbar = 0.5f * (Fi + Fj);
          const float coef = mj * fmaf(thi.y, Fi, fmaf(th.y, Fj, Pi * gbar));
          if (COMP) {
            ka[0].add(-coef * dx);
            ka[1].add(-coef * dy);
            ka[2].add(-coef * dz);
          } else {
            acc[0] = fmaf(-coef, dx, acc[0]);
            acc[1] = fmaf(-coef, dy, acc[1]);
            acc[2] = fmaf(-coef, dz, acc[2]);
          }
          acc[3] = fmaf(mj * Pi * vr, gbar, acc[3]);
          acc[4] = fmaf(mj * vr, Fi, acc[4]);
          ++cnt;
        }
      }
    }
    // fold the batch into the compensated totals
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      if (COMP)
        tot[q].add(acc[q]);
      else
        tot[q].s += acc[q];
      acc[q] = 0.f;
    }
    len = 0;
  };

  auto flush = [&]() {
    wave_sync();
    for (int b0 = 0; b0 < ncand; b0 += 64) {
      if (wave_max_i(len) > LCAP - 64) interact();
      const int bend = min(ncand, b0 + 64);
      for (int c = b0; c < bend; ++c) {
        const float4 cj = cand[c];
        const float dx = pi.x - cj.x, dy = pi.y - cj.y, dz = pi.z - cj.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        bool hit;
        if (MODE == 0) {
          hit = r2 < H2i;
        } else {
          const float Hj = candH[c];
          hit = live && (r2 < H2i || r2 < Hj * Hj) && __float_as_int(cj.w) != i;
        }
        if (hit) {
          lists[len * 64 + lane] = (uint16_t)c;
          ++len;
        }
      }
    }
    interact();
    ncand = 0;
    wave_sync();
  };

  const int pbeg = g.pair_off[ch.act_leaf], pend = g.pair_off[ch.act_leaf + 1];
  for (int pp = pbeg + wave; pp < pend; pp += NW) {
    const PairEntry e = g.pairs[pp];
    const int B = e.b;
    const int bb = g.leaf_begin[B], bc = g.leaf_count[B];
    const bool selfp = (B == ch.leaf);
    const float Rb = MODE == 0 ? Rc : fmaxf(Rc, g.leaf_hmax[B]);
    // sweep axis: the stencil direction closest to the pair offset
    int axis = 0;
    float best = -1.f, sgn = 1.f;
    if (!selfp) {
#pragma unroll
      for (int a = 0; a < 13; ++a) {
        const float d = fmaf(e.sz, g.ax.e[a][2], fmaf(e.sy, g.ax.e[a][1], e.sx * g.ax.e[a][0]));
        if (fabsf(d) > best) {
          best = fabsf(d);
          axis = a;
          sgn = d >= 0.f ? 1.f : -1.f;
        }
      }
    }
    const float ex = g.ax.e[axis][0], ey = g.ax.e[axis][1], ez = g.ax.e[axis][2];
    // reach of the chunk box along the axis, in the partner leaf's frame
    const float pmin = fminf(ex * bminx, ex * bmaxx) + fminf(ey * bminy, ey * bmaxy) + fminf(ez * bminz, ez * bmaxz);
    const float pmax = fmaxf(ex * bminx, ex * bmaxx) + fmaxf(ey * bminy, ey * bmaxy) + fmaxf(ez * bminz, ez * bmaxz);
    const float sproj = fmaf(e.sz, ez, fmaf(e.sy, ey, e.sx * ex));
    const float margin = 1.0001f * Rb + 1e-6f * (fabsf(pmin) + fabsf(pmax) + fabsf(sproj));
    const float lo_b = pmin - margin - sproj, hi_b = pmax + margin - sproj;
    const uint16_t *ord = g.axis_order + (int64_t)axis * g.n + bb;
    for (int t = 0; t < bc; t += 64) {
      const int kk = t + lane;
      const bool valid = kk < bc;
      int j = bb;
      if (valid) j = selfp ? bb + kk : bb + (int)ord[sgn > 0.f ? kk : bc - 1 - kk];
      const float4 pj = valid ? g.pos4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      if (!selfp) {
        const float key = fmaf(pj.z, ez, fmaf(pj.y, ey, pj.x * ex));
        const bool beyond = sgn > 0.f ? key > hi_b : key < lo_b;
        if (__ballot(valid && !beyond) == 0ull) break;
      }
      const float xj = pj.x + e.sx, yj = pj.y + e.sy, zj = pj.z + e.sz;
      const float gx = fmaxf(fmaxf(bminx - xj, xj - bmaxx), 0.f);
      const float gy = fmaxf(fmaxf(bminy - yj, yj - bmaxy), 0.f);
      const float gz = fmaxf(fmaxf(bminz - zj, zj - bmaxz), 0.f);
      const float d2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
      bool keep;
      if (MODE == 0)
        keep = valid && d2 < R2c;
      else
        keep = valid && (d2 < R2c || d2 < pj.w * pj.w);
      const uint64_t mask = __ballot(keep);
      if (keep) {
        const int slot = ncand + rank_below(mask);
        cand[slot] = make_float4(xj, yj, zj, __int_as_float(j));
        if (MODE == 1) candH[slot] = pj.w;
      }
      ncand += __popcll(mask);
      if (ncand > CAP - 64) flush();
    }
  }
  flush();

  // per-lane results of this wave
  float res[9];
  if (MODE == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) res[q] = tot[q].value();
    res[8] = 0.f;
  } else {
    if (COMP) {
      res[0] = ka[0].s - ka[0].c + tot[0].value();
      res[1] = ka[1].s - ka[1].c + tot[1].value();
      res[2] = ka[2].s - ka[2].c + tot[2].value();
    } else {
      res[0] = tot[0].value();
      res[1] = tot[1].value();
      res[2] = tot[2].value();
    }
    res[3] = tot[3].value();
    res[4] = tot[4].value();
    res[5] = vmax;
    res[6] = res[7] = res[8] = 0.f;
  }
  if (NW > 1) {
    // combine the waves' partial sums in wave order through LDS
    constexpr int NQ = 10;
    static_assert(CAP * 4 >= NQ * 64, "reduction buffer");
    __syncthreads();
    float *red = reinterpret_cast<float *>(cand_all[wave]);
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q * 64 + lane] = res[q];
    red[9 * 64 + lane] = __int_as_float(cnt);
    __syncthreads();
    if (wave != 0) return;
    Neu sum[9];
    int csum = 0;
    float vm = 0.f;
    for (int w = 0; w < NW; ++w) {
      const float *rw = reinterpret_cast<const float *>(cand_all[w]);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        if (MODE == 1 && q == 5)
          vm = fmaxf(vm, rw[q * 64 + lane]);
        else if (COMP)
          sum[q].add(rw[q * 64 + lane]);
        else
          sum[q].s += rw[q * 64 + lane];
      }
      csum += __float_as_int(rw[9 * 64 + lane]);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) res[q] = sum[q].value();
    res[5] = MODE == 1 ? vm : res[5];
    cnt = csum;
  }
  if (lane == 0) g.chunk_todo[cid] = 0;

  if (live) {
    if (MODE == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) g.sums[(int64_t)q * g.n_active + k] = res[q];
      g.act_cnt[k] = cnt;
    } else {
      g.ax_out[i] = res[0];
      g.ay_out[i] = res[1];
      g.az_out[i] = res[2];
      const float visc = res[3];
      const float adiab = res[4];
      const float rho = thi.x;
      g.dA_out[i] = 0.5f * g.gm1 * __powf(rho, -g.gm1) * visc;
      g.du_out[i] = fmaf(thi.y, adiab, 0.5f * visc);
      g.vsig_out[i] = res[5];
      if (g.nngb_out) g.nngb_out[i] = cnt;
    }
  }
  if (MODE == 1) {
    const int tot_cnt = wave_sum_i(live ? cnt : 0);
    if (lane == 0) atomicAdd(g.ctr, (unsigned long long)tot_cnt);
  }
}

struct GhostArgs {
  int64_t n_active;
  const int32_t *active_idx, *chunk_of;
  const Chunk *chunks;
  int32_t *chunk_todo;
  const float *sums;
  const int32_t *act_cnt;
  const float *act_hmax;
  float *hlo, *hhi;
  uint8_t *conv;
  float4 *pos4;
  float4 *jth;
  float *h;
  int last;
  int from_u;
  float eta3, kc, tol, gamma, eps, box_quarter, reach;
  // outputs
  float *rho, *drho_dh, *f, *divv, *curlx, *curly, *curlz, *P, *c, *B, *A, *u;
  int32_t *nngb;
  int32_t *n_unconv, *rebuild;
  unsigned long long *ctr;  // cumulative density interactions of finished solves
};

// Newton step on F(h) = h^3 sum_j W(r_ij, h) - eta^3 for each active particle
// not yet converged; converged (or last-pass) particles get their ghost
// quantities written.
__global__ __launch_bounds__(256) void ghost_kernel(GhostArgs g) {
  int finished = 0;
  int unconv = 0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < g.n_active; k += (int64_t)gridDim.x * 256) {
    if (g.conv[k]) continue;
    const int i = g.active_idx[k];
    const float S_w = g.sums[k], S_mw = g.sums[g.n_active + k], S_d = g.sums[2 * g.n_active + k],
                S_md = g.sums[3 * g.n_active + k];
    const float h = g.h[i];
    // Newton in ln h on G = ln(h^3 n / eta^3), with h^3 n = (8/pi)/GK^3 sum w
    // and dG/dln h = (3 sum w - sum (3w + q w')) / sum w: the same root as
    // h^3 n = eta^3, reached in one step where the density is locally uniform.
    const float hn3 = g.kc * S_w;
    const float G = __logf(hn3 / g.eta3);
    const float Gp = (3.f * S_w - S_d) / S_w;
    float lo = g.hlo[k], hi = g.hhi[k];
    if (G < 0.f) lo = fmaxf(lo, h);
    if (G > 0.f) hi = fminf(hi, h);
    float hn = h * __expf(fminf(fmaxf(-G / Gp, -0.6931472f), 0.6931472f));
    if (!(hn >= lo && hn <= hi) || !(Gp > 0.f)) hn = (hi < INFINITY) ? 0.5f * (lo + hi) : 2.f * h;
    if (G == 0.f) hn = h;
    const bool done = fabsf(hn - h) < g.tol * h;
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
      } else {
        A = g.A[i];
        P = A * rg;
        u = P / ((g.gamma - 1.f) * rho);
        if (g.u) g.u[i] = u;
      }
      const float cs = sqrtf(g.gamma * P / rho);
      const float C4 = C3 * iH;
      const float dv = -C4 * g.sums[4 * g.n_active + k] / rho;
      const float cx = C4 * g.sums[5 * g.n_active + k] / rho;
      const float cy = C4 * g.sums[6 * g.n_active + k] / rho;
      const float cz = C4 * g.sums[7 * g.n_active + k] / rho;
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
      if (g.nngb) g.nngb[i] = g.act_cnt[k];
      g.jth[i] = make_float4(rho, fg * P / (rho * rho), cs, Bs);
      finished += g.act_cnt[k];
      g.conv[k] = 1;
      if (!done) ++unconv;
    } else {
      g.hlo[k] = lo;
      g.hhi[k] = hi;
      g.h[i] = hn;
      const float Hn = GK32 * hn;
      g.pos4[i].w = Hn;
      g.chunk_todo[g.chunk_of[k]] = 1;
      ++unconv;
      const Chunk ch = g.chunks[g.chunk_of[k]];
      if (Hn > g.act_hmax[ch.act_leaf] * g.reach) atomicOr(g.rebuild, 1);
      if (Hn > g.box_quarter) atomicOr(g.rebuild, 2);
    }
  }
  finished = wave_sum_i(finished);
  unconv = wave_sum_i(unconv);
  if ((threadIdx.x & 63) == 0) {
    if (finished) atomicAdd(g.ctr, (unsigned long long)finished);
    if (unconv) atomicAdd(g.n_unconv, unconv);
  }
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

template <int MODE, bool COMP>
sph_status launch_loop(sph_ctx *ctx, const LoopArgs &a) {
  const int64_t per = ceil_div(a.n_chunks, 8);
  const unsigned grid = (unsigned)(8 * (per > 0 ? per : 1));
  LoopArgs g = a;
  g.per_xcd = per;
  const int cap = ctx->prm.cand_cap, lcap = ctx->prm.list_cap;
  // waves per chunk: enough waves in flight when few chunks are active
  int nw = ctx->prm.waves_per_chunk;
  if (nw <= 0) {
    nw = 1;
    while (nw < 8 && a.n_chunks * nw < 16384) nw <<= 1;
  }
  PROF(ctx, MODE == 0 ? "density_loop" : "force_loop");
  if (nw >= 8)
    loop_kernel<MODE, 256, 64, COMP, 8><<<grid, 512, 0, ctx->stream>>>(g);
  else if (nw >= 4)
    loop_kernel<MODE, 256, 64, COMP, 4><<<grid, 256, 0, ctx->stream>>>(g);
  else if (nw >= 2)
    loop_kernel<MODE, 512, 96, COMP, 2><<<grid, 128, 0, ctx->stream>>>(g);
  else if (cap <= 256 && lcap <= 64)
    loop_kernel<MODE, 256, 64, COMP, 1><<<grid, 64, 0, ctx->stream>>>(g);
  else if (cap <= 512 && lcap <= 96)
    loop_kernel<MODE, 512, 96, COMP, 1><<<grid, 64, 0, ctx->stream>>>(g);
  else if (cap <= 1024 && lcap <= 128)
    loop_kernel<MODE, 1024, 128, COMP, 1><<<grid, 64, 0, ctx->stream>>>(g);
  else
    loop_kernel<MODE, 2048, 192, COMP, 1><<<grid, 64, 0, ctx->stream>>>(g);
  return sph_hip_check(ctx, hipGetLastError(), MODE == 0 ? "density loop" : "force loop");
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
      SPH_TRY(refresh_leaf_hmax(ctx));
      SPH_TRY(build_pairs(ctx, 0, 1.5f));
    }
  }
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
  SPH_TRY(refresh_leaf_hmax(ctx));
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
