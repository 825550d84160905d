// Shared pieces of the neighbour loops (Sec. III-A, Fig. 5): the per-chunk
// body of the density and force loops, its grid and persistent launches, and
// the ghost's Newton step.  Included by the single-box passes, the batched
// multi-box passes and the autotuner.
//
// Work item: one chunk of up to 64 active particles of one leaf (gather
// formulation: each active particle's sums are produced by the single
// workgroup that owns it, in a fixed order, so there are no atomics and the
// results are reproducible).  For every partner leaf of the chunk's cell-pair
// list:
//   1. staging: the partner's particles are read 64 at a time (coalesced
//      loads, in the per-cell axis-sort order when the pair is not a self
//      pair so that the sweep stops once the projections leave the chunk's
//      reach), moved into the chunk leaf's frame with the FP32 pair shift, and
//      kept if they are within reach of the chunk's bounding box (wave ballot
//      + rank into an LDS candidate array);
//   2. filter: every lane tests its own particle against each candidate with
//      the FP32 predicate and appends hits to its own LDS neighbour list;
//   3. interact: every lane walks its own list (lanes have near-equal
//      neighbour counts because h adapts) and accumulates in registers.
// No MFMA: pair interactions are not a dense contraction.
#pragma once

#include <math.h>
#include <string.h>

#include "sph_internal.h"



struct LoopArgs {
  const Chunk *chunks;
  int32_t *chunk_todo;
  int64_t n_chunks;
  int64_t per_xcd;
  const int32_t *work;  // optional work-item list: codes chunk * 16 + part
  int64_t n_items;      // grid items: chunks, or entries of `work`
  int xcd;              // grid kernel: consecutive items to the same XCD
  // split chunks: a chunk's pair list in parts [chunk_item0[c], chunk_item0[c+1]);
  // null when no chunk is split
  const int32_t *chunk_item0;
  int32_t *chunk_ctr;   // arrivals per chunk (counts up; the last of a round combines)
  float *partials;      // per item: 11 x 64 per-lane partial results
  const int32_t *active_idx;
  const float4 *pos4;  // (ox, oy, oz, H)
  const float4 *jvm;   // (vx, vy, vz, m)
  const float4 *jth;   // (rho, f P / rho^2, c, B)  force only
  const int32_t *leaf_begin, *leaf_count;
  const float *leaf_hmax;
  const float *leaf_half;  // half width of each leaf (sweep pruning)
  const float4 *gbox_lo, *gbox_hi;  // 8-particle group boxes (group g of leaf l at (begin >> 3) + l + g)
  const float *leaf_dx;    // drift margin of each leaf
  const int32_t *pair_off;
  const PairEntry *pairs;
  const uint8_t *pair_axis;  // per pair: sweep axis code
  const uint16_t *axis_order;  // 13 axis orders, then the H order (HORD_ROW)
  const float *leaf_hgrow;     // per leaf: bound on H now / H at the full build
  const float4 *leaf_hq;       // per leaf: H at the build at ranks hq_rank(0..15) of its H order
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
  // adjoint passes
  const float4 *jw;     // loss weights (wx, wy, wz, 0) per particle
  const float4 *jadj1;  // (rho_bar, drho_dh_bar, D_bar, lambda) per particle
  const float4 *jadj2;  // (C_bar x, y, z, 0) per particle
  float *outp;          // per-particle outputs, [q * n + i]
  // (opt) the pass does its work only while the device count *gate is at
  // least gate_min (every work item returns at once otherwise)
  const int32_t *gate;
  int32_t gate_min;
};

// Modes of the chunk body: 0 density loop, 1 force loop, 2 force adjoint,
// 3 density adjoint (h derivatives and the implicit-h solve), 4 density
// adjoint (position terms).  Symmetric modes run over r < max(H_i, H_j)
// without the self pair; the others over r < H_i with the self pair.
template <int MODE>
struct ModeTraits {
  static constexpr bool sym = MODE == 1 || MODE == 2 || MODE == 4;
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

// w' and w'' of the cubic spline (zero beyond q = 1).
__device__ __forceinline__ void kernel_d1_d2(float q, float &wp, float &wpp) {
  const float t = 1.f - q;
  const bool in = q < 0.5f, sup = q < 1.f;
  wp = in ? q * fmaf(18.f, q, -12.f) : (sup ? -6.f * t * t : 0.f);
  wpp = in ? fmaf(36.f, q, -12.f) : (sup ? 12.f * t : 0.f);
}

// w' alone, zero (signed) from q = 1 on; one select, no branch.
__device__ __forceinline__ float kernel_dw_only(float q) {
  const float wpi = q * fmaf(18.f, q, -12.f);
  const float t = fmaxf(1.f - q, 0.f);
  const float wpo = -6.f * (t * t);
  return q < 0.5f ? wpi : wpo;
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

// Orders this wave's LDS accesses across its lanes (each wave owns its own
// LDS region, so no workgroup barrier is needed between its phases).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Bytes of LDS one wave of the loop kernel uses: per staged candidate its
// shifted offset and index, its velocity and mass, for the force loops its
// density-loop state, and H (the force loop keeps H^2 and 1/H); then the
// per-lane neighbour lists.
template <int MODE, int CAP, int LCAP>
struct WaveLds {
  static constexpr bool th = MODE == 1 || MODE == 2;
  static constexpr int cand = CAP * 16;
  static constexpr int candV = CAP * 16;
  static constexpr int candT = th ? CAP * 16 : 0;
  static constexpr int candH = MODE == 1 ? CAP * 8 : (ModeTraits<MODE>::sym ? CAP * 4 : 0);
  static constexpr int lists = LCAP * 64 * 2;
  static constexpr int bytes = cand + candV + candT + candH + lists;
  static_assert(bytes >= 10 * 64 * 4, "room for the cross-wave reduction");
  static_assert(CAP % 4 == 0, "16-byte alignment of the arrays after candH");
};

// One chunk of up to 64 active particles of one leaf.  MODE 0: density loop;
// MODE 1: force loop.  NW waves share the chunk: wave w takes the partner
// cells w, w+NW, ... of the chunk's pair list, and the per-lane partial sums
// are combined across waves in wave order at the end.  `lds` holds NW wave
// regions of WaveLds::bytes each.
template <int MODE, int CAP, int LCAP, bool COMP, int NW>
__device__ __forceinline__ void chunk_body(const LoopArgs &g, int code, bool coded, char *lds) {
  using W = WaveLds<MODE, CAP, LCAP>;
  constexpr int FB = LCAP / 2 < 64 ? LCAP / 2 : 64;  // candidates filtered between list checks
  // work item: a chunk, or one part of a chunk's cell-pair list
  const int cid = coded ? code >> 4 : code;
  const int part = coded ? code & 15 : 0;
  const int nparts = g.chunk_item0 ? g.chunk_item0[cid + 1] - g.chunk_item0[cid] : 1;
  if (g.gate && *g.gate < g.gate_min) return;
  if (!g.chunk_todo[cid]) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  char *mine = lds + wave * W::bytes;
  float4 *cand = reinterpret_cast<float4 *>(mine);
  float4 *candV = reinterpret_cast<float4 *>(mine + W::cand);
  float4 *candT = reinterpret_cast<float4 *>(mine + W::cand + W::candV);
  float *candH = reinterpret_cast<float *>(mine + W::cand + W::candV + W::candT);
  float2 *candH2 = reinterpret_cast<float2 *>(candH);  // force loop: (H^2, 1/H)
  uint16_t *lists = reinterpret_cast<uint16_t *>(mine + W::cand + W::candV + W::candT + W::candH);
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
  if ((MODE == 1 || MODE == 2) && live) thi = g.jth[i];
  float4 wi = make_float4(0.f, 0.f, 0.f, 0.f), adj1i = wi, adj2i = wi;
  if (MODE == 2 && live) wi = g.jw[i];
  if (MODE == 4 && live) {
    adj1i = g.jadj1[i];
    adj2i = g.jadj2[i];
  }
  const float hi_ = Hi * (1.f / GK32);

  // chunk bounding box and reach
  const float bminx = wave_min_f_dpp(live ? pi.x : INFINITY), bmaxx = wave_max_f_dpp(live ? pi.x : -INFINITY);
  const float bminy = wave_min_f_dpp(live ? pi.y : INFINITY), bmaxy = wave_max_f_dpp(live ? pi.y : -INFINITY);
  const float bminz = wave_min_f_dpp(live ? pi.z : INFINITY), bmaxz = wave_max_f_dpp(live ? pi.z : -INFINITY);
  const float Rc = wave_max_f_dpp(live ? Hi : 0.f);
  const float R2c = Rc * Rc;

  // accumulators: density (w, m w, 3w+qw', m(3w+qw'), div, curl x3); force (a x3, visc, adiab)
  float acc[9];
  Neu tot[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.f;
  float vmax = 0.f;
  int cnt = 0;
  int len = 0;
  int ncand = 0;

  auto interact = [&]() {
    const int maxlen = wave_max_i_dpp(len);
    // the next list entry is read one step ahead
    int cnext = len > 0 ? lists[lane] : 0;
    for (int t = 0; t < maxlen; ++t) {
      const int c = cnext;
      if (t + 1 < len) cnext = lists[(t + 1) * 64 + lane];
      if (t < len) {
        const float4 cj = cand[c];
        const int j = __float_as_int(cj.w);
        const float dx = pi.x - cj.x, dy = pi.y - cj.y, dz = pi.z - cj.z;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float4 vj = candV[c];
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
        } else if (MODE == 2) {
          // force adjoint: both orders (i,j) and (j,i) of the pair
          const float Hj = candH[c];
          const float invHj = __builtin_amdgcn_rcpf(Hj);
          const float4 th = candT[c];
          const float4 wj = g.jw[j];
          const float qi = r * invHi, qj = r * invHj;
          float wpi, wppi, wpj, wppj;
          kernel_d1_d2(qi, wpi, wppi);
          kernel_d1_d2(qj, wpj, wppj);
          const float C4i = KNORM32 * (invHi * invHi) * (invHi * invHi);
          const float C4j = KNORM32 * (invHj * invHj) * (invHj * invHj);
          const float Fi = C4i * wpi * rinv, Fj = C4j * wpj * rinv;
          const float Fri = C4i * rinv * fmaf(wppi, invHi, -wpi * rinv);
          const float Frj = C4j * rinv * fmaf(wppj, invHj, -wpj * rinv);
          const float Fhi = -C4i * fmaf(qi, wppi, 4.f * wpi) * rinv * (GK32 * invHi);
          const float mi = vi.w;
          const bool appr = vr < 0.f;
          const float mu = appr ? vr * rinv : 0.f;
          const float vsig = thi.z + th.z - 3.f * mu;
          const float rs = __builtin_amdgcn_rcpf(thi.x + th.x);
          const float Bs = thi.w + th.w;
          const float Pi = -g.half_alpha * vsig * mu * Bs * rs;
          const float Pc = -g.half_alpha * mu * Bs * rs;
          const float PB = -g.half_alpha * vsig * mu * rs;
          const float Pr = -Pi * rs;
          const float Pm = appr ? -g.half_alpha * Bs * rs * (vsig - 3.f * mu) : 0.f;
          const float Fb = 0.5f * (Fi + Fj);
          const float S = fmaf(thi.y, Fi, fmaf(th.y, Fj, Pi * Fb));
          const float wdi = fmaf(wi.z, dz, fmaf(wi.y, dy, wi.x * dx));
          const float wdj = fmaf(wj.z, dz, fmaf(wj.y, dy, wj.x * dx));
          const float sb = fmaf(mi, wdj, -mj * wdi);
          const float dS = fmaf(thi.y + 0.5f * Pi, Fri, (th.y + 0.5f * Pi) * Frj);
          const float cv = sb * Fb * Pm * rinv;
          const float cd = sb * dS * rinv - cv * mu * rinv;
          acc[0] = fmaf(S, fmaf(mi, wj.x, -mj * wi.x), fmaf(cd, dx, fmaf(cv, vx, acc[0])));
          acc[1] = fmaf(S, fmaf(mi, wj.y, -mj * wi.y), fmaf(cd, dy, fmaf(cv, vy, acc[1])));
          acc[2] = fmaf(S, fmaf(mi, wj.z, -mj * wi.z), fmaf(cd, dz, fmaf(cv, vz, acc[2])));
          acc[3] = fmaf(sb, Fi, acc[3]);
          acc[4] = fmaf(sb * (thi.y + 0.5f * Pi), Fhi, acc[4]);
          acc[5] = fmaf(sb * Fb, Pc, acc[5]);
          acc[6] = fmaf(sb * Fb, PB, acc[6]);
          acc[7] = fmaf(sb * Fb, Pr, acc[7]);
          ++cnt;
        } else if (MODE == 3) {
          // h derivatives of the density sums (self pair included)
          const float q = r * invHi;
          float w, wp, wpp;
          kernel_w_dw(q, w, wp);
          float wp2;
          kernel_d1_d2(q, wp2, wpp);
          acc[0] += w;
          acc[1] += fmaf(q, wp, 3.f * w);
          acc[2] = fmaf(mj, fmaf(q * q, wpp, fmaf(8.f * q, wp, 12.f * w)), acc[2]);
          const float t = mj * fmaf(q, wpp, 4.f * wp) * rinv;
          acc[3] = fmaf(t, vr, acc[3]);
          acc[4] = fmaf(t, fmaf(vy, dz, -vz * dy), acc[4]);
          acc[5] = fmaf(t, fmaf(vz, dx, -vx * dz), acc[5]);
          acc[6] = fmaf(t, fmaf(vx, dy, -vy * dx), acc[6]);
          cnt += (j != i);
        } else if (MODE == 4) {
          // position terms of the density sums and of the h constraint, both orders
          const float Hj = candH[c];
          const float invHj = __builtin_amdgcn_rcpf(Hj);
          const float4 a1 = g.jadj1[j];
          const float4 a2 = g.jadj2[j];
          const float qi = r * invHi, qj = r * invHj;
          float wpi, wppi, wpj, wppj;
          kernel_d1_d2(qi, wpi, wppi);
          kernel_d1_d2(qj, wpj, wppj);
          const float C4i = KNORM32 * (invHi * invHi) * (invHi * invHi);
          const float C4j = KNORM32 * (invHj * invHj) * (invHj * invHj);
          const float Fi = C4i * wpi * rinv, Fj = C4j * wpj * rinv;
          const float Fri = C4i * rinv * fmaf(wppi, invHi, -wpi * rinv);
          const float Frj = C4j * rinv * fmaf(wppj, invHj, -wpj * rinv);
          const float Fhi = -C4i * fmaf(qi, wppi, 4.f * wpi) * rinv * (GK32 * invHi);
          const float Fhj = -C4j * fmaf(qj, wppj, 4.f * wpj) * rinv * (GK32 * invHj);
          const float mi = vi.w;
          const float hj_ = Hj * (1.f / GK32);
          const float hi3 = hi_ * hi_ * hi_, hj3 = hj_ * hj_ * hj_;
          // C_bar x v and C_bar . (v x d) for both owners
          const float cxv = fmaf(vy, dz, -vz * dy), cyv = fmaf(vz, dx, -vx * dz), czv = fmaf(vx, dy, -vy * dx);
          const float ti = fmaf(adj2i.z, czv, fmaf(adj2i.y, cyv, adj2i.x * cxv));
          const float tj = fmaf(a2.z, czv, fmaf(a2.y, cyv, a2.x * cxv));
          const float ai = fmaf(adj1i.x * mj, Fi, fmaf(adj1i.y * mj, Fhi, -adj1i.w * hi3 * Fi));
          const float aj = fmaf(a1.x * mi, Fj, fmaf(a1.y * mi, Fhj, -a1.w * hj3 * Fj));
          // G_ij - G_ji = (ai + aj) d + (Di mj Fi + Dj mi Fj) v + (Di mj vr Fri + mj ti Fri
          //               + Dj mi vr Frj + mi tj Frj) d / r + mj Fi (Ci x v) + mi Fj (Cj x v)
          const float sv = fmaf(adj1i.z * mj, Fi, a1.z * mi * Fj);
          const float se = (ai + aj) + rinv * fmaf(mj * fmaf(adj1i.z, vr, ti), Fri, mi * fmaf(a1.z, vr, tj) * Frj);
          const float ci = mj * Fi, cj = mi * Fj;
          const float gxv = fmaf(ci, fmaf(adj2i.y, vz, -adj2i.z * vy), cj * fmaf(a2.y, vz, -a2.z * vy));
          const float gyv = fmaf(ci, fmaf(adj2i.z, vx, -adj2i.x * vz), cj * fmaf(a2.z, vx, -a2.x * vz));
          const float gzv = fmaf(ci, fmaf(adj2i.x, vy, -adj2i.y * vx), cj * fmaf(a2.x, vy, -a2.y * vx));
          acc[0] = fmaf(se, dx, fmaf(sv, vx, gxv + acc[0]));
          acc[1] = fmaf(se, dy, fmaf(sv, vy, gyv + acc[1]));
          acc[2] = fmaf(se, dz, fmaf(sv, vz, gzv + acc[2]));
          ++cnt;
        } else {
          const float invHj = candH2[c].y;
          const float4 th = candT[c];
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
          acc[0] = fmaf(-coef, dx, acc[0]);
          acc[1] = fmaf(-coef, dy, acc[1]);
          acc[2] = fmaf(-coef, dz, acc[2]);
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

  // Filter of the staged candidates into per-lane neighbour lists, FB
  // candidates at a time.  Two schedules give the same lists in the same
  // order: with many live lanes every lane walks the candidates (the
  // candidate broadcast from LDS); with few live lanes (sparse chunks of a
  // deep time-bin) lane t holds candidate b0 + t and the wave walks the live
  // particles instead (their data broadcast by readlane), so the work
  // follows the live particles, not the 64 lanes.
  const int nlive = ch.count;
  const float H2b = H2i, pxb = pi.x, pyb = pi.y, pzb = pi.z;
  auto flush = [&]() {
    wave_sync();
    if (nlive < FB) {
      for (int b0 = 0; b0 < ncand; b0 += FB) {
        if (__ballot(len > LCAP - FB)) interact();
        const int c = b0 + lane;
        const bool cv = lane < FB && c < ncand;
        const float4 cj = cv ? cand[c] : make_float4(0.f, 0.f, 0.f, 0.f);
        float H2j = 0.f;
        if (MODE == 1 && cv) H2j = candH2[c].x;
        if (MODE != 1 && ModeTraits<MODE>::sym && cv) H2j = candH[c] * candH[c];
        const int jj = __float_as_int(cj.w);
        for (int ii = 0; ii < nlive; ++ii) {
          const float xi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pxb), ii));
          const float yi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pyb), ii));
          const float zi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pzb), ii));
          const float H2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(H2b), ii));
          const float dx = xi - cj.x, dy = yi - cj.y, dz = zi - cj.z;
          const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          bool hit;
          if (!ModeTraits<MODE>::sym)
            hit = cv && r2 < H2;
          else
            hit = cv && (r2 < H2 || r2 < H2j) && jj != __builtin_amdgcn_readlane(i, ii);
          const uint64_t hm = __ballot(hit);
          if (hm) {
            const int base = __builtin_amdgcn_readlane(len, ii);
            if (hit) lists[(base + rank_below(hm)) * 64 + ii] = (uint16_t)c;
            if (lane == ii) len += __popcll(hm);
          }
        }
      }
      interact();
      ncand = 0;
      wave_sync();
      return;
    }
    const int nc = __builtin_amdgcn_readfirstlane(ncand);
    for (int b0 = 0; b0 < nc; b0 += FB) {
      if (__ballot(len > LCAP - FB)) interact();
      const int bend = min(nc, b0 + FB);
      for (int c0 = b0; c0 < bend; c0 += 4) {
        // four candidates per round: their LDS reads are issued together
        float4 cq[4];
        float h2q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int cc = min(c0 + u, bend - 1);
          cq[u] = cand[cc];
          h2q[u] = 0.f;
          if (MODE == 1) h2q[u] = candH2[cc].x;
          if (MODE != 1 && ModeTraits<MODE>::sym) h2q[u] = candH[cc];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u;
          if (c < bend) {
            const float4 cj = cq[u];
            const float dx = pi.x - cj.x, dy = pi.y - cj.y, dz = pi.z - cj.z;
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            bool hit;
            if (!ModeTraits<MODE>::sym) {
              hit = r2 < H2i;
            } else if (MODE == 1) {
              hit = live && r2 < fmaxf(H2i, h2q[u]) && __float_as_int(cj.w) != i;
            } else {
              hit = live && (r2 < H2i || r2 < h2q[u] * h2q[u]) && __float_as_int(cj.w) != i;
            }
            // branch-free append: the slot past the end is written and kept
            // only on a hit (len <= LCAP - 1 here: at most LCAP - FB at the
            // start of the block, at most FB - 1 appends since)
            lists[len * 64 + lane] = (uint16_t)c;
            len += hit ? 1 : 0;
          }
        }
      }
    }
    interact();
    ncand = 0;
    wave_sync();
  };

  const int pbeg0 = g.pair_off[ch.act_leaf], npair = g.pair_off[ch.act_leaf + 1] - pbeg0;
  const int pbeg = pbeg0 + (int)((int64_t)npair * part / nparts);
  const int pend = pbeg0 + (int)((int64_t)npair * (part + 1) / nparts);
  for (int pp = pbeg + wave; pp < pend; pp += NW) {
    const PairEntry e = g.pairs[pp];
    const int B = e.b;
    const int bb = g.leaf_begin[B], bc = g.leaf_count[B];
    const bool selfp = (B == ch.leaf);
    const float Rb = !ModeTraits<MODE>::sym ? Rc : fmaxf(Rc, g.leaf_hmax[B]);
    // sweep axis: the stencil direction closest to the pair offset (coded
    // when the pair list was filled)
    int axis = 0;
    float sgn = 1.f;
    if (!selfp) {
      const int code = __builtin_amdgcn_readfirstlane((int)g.pair_axis[pp]);
      axis = code & 0x7f;
      sgn = (code & 0x80) ? -1.f : 1.f;
    }
    const float ex = g.ax.e[axis][0], ey = g.ax.e[axis][1], ez = g.ax.e[axis][2];
    // reach of the chunk box along the axis, in the partner leaf's frame
    const float pmin = fminf(ex * bminx, ex * bmaxx) + fminf(ey * bminy, ey * bmaxy) + fminf(ez * bminz, ez * bmaxz);
    const float pmax = fmaxf(ex * bminx, ex * bmaxx) + fmaxf(ey * bminy, ey * bmaxy) + fmaxf(ez * bminz, ez * bmaxz);
    const float sproj = fmaf(e.sz, ez, fmaf(e.sy, ey, e.sx * ex));
    // the order is by the offsets of the full build: a projection is at most
    // the leaf's drift margin from its sorted place, so the stop waits for
    // keys twice that margin past the reach
    const float margin = 1.0001f * Rb + 2.0001f * g.leaf_dx[B] + 1e-6f * (fabsf(pmin) + fabsf(pmax) + fabsf(sproj));
    const float lo_b = pmin - margin - sproj, hi_b = pmax + margin - sproj;
    const uint16_t *ord = g.axis_order + (int64_t)axis * g.n + bb;
    for (int t = 0; t < bc; t += 64) {
      const int kk = t + lane;
      const bool valid = kk < bc;
      int j = bb;
      // a partner of at most two tiles is read in cell order (its axis order is not made)
      if (valid) j = (selfp || bc <= 128) ? bb + kk : bb + (int)ord[sgn > 0.f ? kk : bc - 1 - kk];
      const float4 pj = valid ? g.pos4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      // the candidate's neighbour data, loaded with its position (a kept
      // candidate's pair terms then read LDS only)
      const float4 vjs = valid ? g.jvm[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      float4 ths = make_float4(0.f, 0.f, 0.f, 0.f);
      if (W::th && valid) ths = g.jth[j];
      if (!selfp && bc > 128) {
        // sorted partner: stop at the first tile wholly past the reach
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
      if (!ModeTraits<MODE>::sym)
        keep = valid && d2 < R2c;
      else
        keep = valid && (d2 < R2c || d2 < pj.w * pj.w);
      const uint64_t mask = __ballot(keep);
      if (keep) {
        const int slot = ncand + rank_below(mask);
        cand[slot] = make_float4(xj, yj, zj, __int_as_float(j));
        candV[slot] = vjs;
        if (W::th) candT[slot] = ths;
        if (MODE == 1)
          candH2[slot] = make_float2(pj.w * pj.w, __builtin_amdgcn_rcpf(pj.w));
        else if (ModeTraits<MODE>::sym)
          candH[slot] = pj.w;
      }
      ncand += __popcll(mask);
      if (ncand > CAP - 64) flush();
    }
  }
  flush();

  // per-lane results of this wave
  float res[9];
  if (MODE != 1) {
#pragma unroll
    for (int q = 0; q < 9; ++q) res[q] = tot[q].value();
  } else {
    res[0] = tot[0].value();
    res[1] = tot[1].value();
    res[2] = tot[2].value();
    res[3] = tot[3].value();
    res[4] = tot[4].value();
    res[5] = vmax;
    res[6] = res[7] = res[8] = 0.f;
  }
  if (NW > 1) {
    // combine the waves' partial sums in wave order through LDS
    __syncthreads();
    float *red = reinterpret_cast<float *>(mine);
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q * 64 + lane] = res[q];
    red[9 * 64 + lane] = __int_as_float(cnt);
    __syncthreads();
    if (wave != 0) return;
    Neu sum[9];
    int csum = 0;
    float vm = 0.f;
    for (int w = 0; w < NW; ++w) {
      const float *rw = reinterpret_cast<const float *>(lds + w * W::bytes);
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
  if (nparts > 1) {
    // publish this part's per-lane results; the last part of the chunk to
    // arrive combines all parts in part order (deterministic) and finishes
    const int64_t item0 = g.chunk_item0[cid];
    float *mine_p = g.partials + (item0 + part) * (11 * 64);
#pragma unroll
    for (int q = 0; q < 9; ++q) mine_p[q * 64 + lane] = res[q];
    mine_p[9 * 64 + lane] = __int_as_float(cnt);
    __threadfence();
    int old = 0;
    if (lane == 0) old = atomicAdd(&g.chunk_ctr[cid], 1);
    old = __shfl(old, 0, 64);
    if ((old + 1) % nparts != 0) return;
    __threadfence();
    Neu sum[9];
    int csum = 0;
    float vm = 0.f;
    for (int pp = 0; pp < nparts; ++pp) {
      const float *rp = g.partials + (item0 + pp) * (11 * 64);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const float v = rp[q * 64 + lane];
        if (MODE == 1 && q == 5)
          vm = fmaxf(vm, v);
        else if (COMP)
          sum[q].add(v);
        else
          sum[q].s += v;
      }
      csum += __float_as_int(rp[9 * 64 + lane]);
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
    } else if (MODE >= 2) {
      constexpr int NOUT = MODE == 2 ? 8 : (MODE == 3 ? 7 : 3);
#pragma unroll
      for (int q = 0; q < NOUT; ++q) g.outp[(int64_t)q * g.n + i] = res[q];
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
    const int tot_cnt = wave_sum_i_dpp(live ? cnt : 0);
    if (lane == 0) atomicAdd(g.ctr, (unsigned long long)tot_cnt);
  }
}


// One workgroup per work item: items are chunk ids (or indices into a
// cost-ordered work list).  Without a work list, consecutive chunks (Morton
// neighbours) go to the same XCD so that their shared partner cells are
// re-read from that XCD's L2.
template <int MODE, int CAP, int LCAP, bool COMP, int NW>
__global__ __launch_bounds__(64 * NW) void loop_grid_kernel(LoopArgs g) {
  __shared__ __align__(16) char lds[NW * WaveLds<MODE, CAP, LCAP>::bytes];
  int item;
  if (!g.xcd) {
    item = blockIdx.x;
  } else {
    const int64_t b = blockIdx.x;
    const int64_t c = (b & 7) * g.per_xcd + (b >> 3);
    item = (int)c;
  }
  if (item >= g.n_items) return;
  if (g.work)
    chunk_body<MODE, CAP, LCAP, COMP, NW>(g, g.work[item], true, lds);
  else
    chunk_body<MODE, CAP, LCAP, COMP, NW>(g, item, false, lds);
}

// Persistent variant: a grid sized to the machine pulls work items (box,
// chunk) from one atomic counter until the list is exhausted; every
// workgroup exits once the counter passes the end.
template <int MODE, int CAP, int LCAP, bool COMP, int NW>
__global__ __launch_bounds__(64 * NW) void loop_persistent_kernel(const LoopArgs *__restrict__ boxes,
                                                                  const int2 *__restrict__ work, int n_items,
                                                                  int *__restrict__ counter) {
  __shared__ __align__(16) char lds[NW * WaveLds<MODE, CAP, LCAP>::bytes];
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
    __syncthreads();
    const int item = item_s;
    __syncthreads();
    if (item >= n_items) break;
    const int2 w = work[item];
    chunk_body<MODE, CAP, LCAP, COMP, NW>(boxes[w.x], w.y, true, lds);
    __syncthreads();
  }
}

// Multi-box grid variant: one workgroup per (box, chunk) work item.
template <int MODE, int CAP, int LCAP, bool COMP, int NW>
__global__ __launch_bounds__(64 * NW) void loop_multi_kernel(const LoopArgs *__restrict__ boxes,
                                                             const int2 *__restrict__ work, int n_items) {
  __shared__ __align__(16) char lds[NW * WaveLds<MODE, CAP, LCAP>::bytes];
  const int item = blockIdx.x;
  if (item >= n_items) return;
  const int2 w = work[item];
  chunk_body<MODE, CAP, LCAP, COMP, NW>(boxes[w.x], w.y, true, lds);
}

// Loop tiling: waves per chunk, tile class (candidate slots / list slots per
// lane), work order and launch style.  Tile classes: 0 = 128/32, 1 = 256/64,
// 2 = 512/96, 3 = 1024/128, 4 = 2048/192 (the classes that fit the 160 KB of
// LDS per CU with the waves of one chunk).
struct LoopConfig {
  int nw = 1;
  int tile = 2;
  int ordered = 0;     // 1: chunks in decreasing cost order, 0: Morton order
  int persistent = 0;  // 1: persistent grid with an atomic work counter
  int split = 0;       // chunk splitting class: 0 none, 1 / 2 parts of ~1024 / ~4096 staged particles
};

// Staged partner particles per work item of a split class (0: no splitting).
inline int split_target(int split) { return split == 1 ? 1024 : split == 2 ? 4096 : 0; }

inline bool loop_config_valid(const LoopConfig &c) {
  if (c.split < 0 || c.split > 2) return false;
  switch (c.nw) {
    case 1: return c.tile >= 0 && c.tile <= 4;
    case 2: return c.tile >= 0 && c.tile <= 2;
    case 4: return c.tile >= 0 && c.tile <= 1;
    case 8: return c.tile == 0;
    default: return false;
  }
}

// Launches one pass of the loop over the given work.  Single box: `a` with
// a.work (ordered) or without (Morton order, XCD-grouped).  Multi box or
// persistent: dev_boxes/dev_work/n_items (counter zeroed here).
template <int MODE, bool COMP, int CAP, int LCAP, int NW>
hipError_t launch_loop_t(hipStream_t st, const LoopArgs &a, const LoopConfig &cfg, const LoopArgs *dev_boxes,
                         const int2 *dev_work, int n_items, int *counter, int grid_persistent) {
  if (dev_boxes) {
    if (cfg.persistent) {
      hipError_t e = hipMemsetAsync(counter, 0, sizeof(int), st);
      if (e != hipSuccess) return e;
      loop_persistent_kernel<MODE, CAP, LCAP, COMP, NW><<<grid_persistent, 64 * NW, 0, st>>>(dev_boxes, dev_work,
                                                                                            n_items, counter);
    } else {
      loop_multi_kernel<MODE, CAP, LCAP, COMP, NW><<<n_items > 0 ? n_items : 1, 64 * NW, 0, st>>>(dev_boxes,
                                                                                                dev_work, n_items);
    }
  } else {
    LoopArgs g = a;
    int64_t grid;
    if (!g.work) g.n_items = g.n_chunks;
    g.xcd = !cfg.ordered;
    if (!g.xcd) {
      grid = g.n_items;
    } else {
      g.per_xcd = ceil_div(g.n_items, 8);
      grid = 8 * (g.per_xcd > 0 ? g.per_xcd : 1);
    }
    loop_grid_kernel<MODE, CAP, LCAP, COMP, NW><<<(unsigned)(grid > 0 ? grid : 1), 64 * NW, 0, st>>>(g);
  }
  return hipGetLastError();
}

template <int MODE, bool COMP>
hipError_t launch_loop_any(hipStream_t st, const LoopArgs &a, const LoopConfig &c, const LoopArgs *dev_boxes,
                           const int2 *dev_work, int n_items, int *counter, int grid_persistent) {
#define SPH_LAUNCH(CAP_, LCAP_, NW_) \
  return launch_loop_t<MODE, COMP, CAP_, LCAP_, NW_>(st, a, c, dev_boxes, dev_work, n_items, counter, grid_persistent)
  switch (c.nw * 10 + c.tile) {
    case 10: SPH_LAUNCH(128, 32, 1);
    case 11: SPH_LAUNCH(256, 64, 1);
    case 12: SPH_LAUNCH(512, 96, 1);
    case 13: SPH_LAUNCH(1024, 128, 1);
    case 14: SPH_LAUNCH(2048, 192, 1);
    case 20: SPH_LAUNCH(128, 32, 2);
    case 21: SPH_LAUNCH(256, 64, 2);
    case 22: SPH_LAUNCH(512, 96, 2);
    case 40: SPH_LAUNCH(128, 32, 4);
    case 41: SPH_LAUNCH(256, 64, 4);
    case 80: SPH_LAUNCH(128, 32, 8);
    default: return hipErrorInvalidValue;
  }
#undef SPH_LAUNCH
}

// Loop arguments common to every pass of one context (defined with the passes).
LoopArgs base_args(sph_ctx *ctx);
