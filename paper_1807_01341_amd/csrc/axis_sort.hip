// Per-cell particle sorts for neighbour pruning (the "sort" task of Fig. 5):
// for every leaf and each of the 13 directions of the half neighbour stencil,
// the in-leaf order of the projections d = e . o of the FP32 offsets at the
// last full build (ascending, ties by in-leaf index).  A 14th order
// (HORD_ROW) lists the particles by H, largest first, keyed by h_build (H at
// the full build, or at a later re-key of the leaf): the force loop reads
// only its head where a partner leaf lies beyond H_i, since with the
// symmetric cutoff r < max(H_i, H_j) only particles of large H_j reach there.
// Bitonic sorts of (key, index), in LDS or in registers.
#include <math.h>

#include <algorithm>

#include "sph_internal.h"

#define AS_THREADS 256

// Workgroup LDS bitonic sort for leaves of 513..4096 particles (only at the
// maximum depth, where coincident particles cannot be split further).
template <int P>
__device__ void sort_leaf_lds(const float4 *__restrict__ pos4, const float *__restrict__ hb, int b, int cnt, int64_t n,
                              const AxisTab &ax,
                              uint16_t *__restrict__ order, float *ox, float *oy, float *oz, float *key,
                              uint16_t *idx) {
  int size = 2;
  while (size < cnt) size <<= 1;
  for (int k = threadIdx.x; k < cnt; k += AS_THREADS) {
    const float4 q = pos4[b + k];
    ox[k] = q.x;
    oy[k] = q.y;
    oz[k] = q.z;
  }
  __syncthreads();
  for (int a = 0; a <= HORD_ROW; ++a) {
    const bool hrow = a == HORD_ROW;
    const float ex = hrow ? 0.f : ax.e[a][0], ey = hrow ? 0.f : ax.e[a][1], ez = hrow ? 0.f : ax.e[a][2];
    for (int k = threadIdx.x; k < size; k += AS_THREADS) {
      if (k < cnt) {
        key[k] = hrow ? -hb[b + k] + 0.0f : fmaf(oz[k], ez, fmaf(oy[k], ey, ox[k] * ex));
        idx[k] = (uint16_t)k;
      } else {
        key[k] = INFINITY;
        idx[k] = 0xffff;
      }
    }
    __syncthreads();
    for (int kk = 2; kk <= size; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < (size >> 1); t += AS_THREADS) {
          const int i0 = 2 * t - (t & (j - 1));
          const int i1 = i0 + j;
          const bool up = (i0 & kk) == 0;
          const float k0 = key[i0], k1 = key[i1];
          const uint16_t d0 = idx[i0], d1 = idx[i1];
          const bool gt = (k0 > k1) || (k0 == k1 && d0 > d1);
          if (gt == up) {
            key[i0] = k1;
            key[i1] = k0;
            idx[i0] = d1;
            idx[i1] = d0;
          }
        }
        __syncthreads();
      }
    }
    for (int k = threadIdx.x; k < cnt; k += AS_THREADS) order[(int64_t)a * n + b + k] = idx[k];
    __syncthreads();
  }
}

template <int P>
__global__ __launch_bounds__(AS_THREADS) void axis_sort_kernel(const float4 *__restrict__ pos4,
                                                               const float *__restrict__ hb,
                                                               const int32_t *__restrict__ leaf_begin,
                                                               const int32_t *__restrict__ leaf_count, int64_t nl,
                                                               int64_t n, AxisTab ax, int min_count,
                                                               uint16_t *__restrict__ order) {
  __shared__ float ox[P], oy[P], oz[P];
  __shared__ float key[P];
  __shared__ uint16_t idx[P];
  for (int64_t l = blockIdx.x; l < nl; l += gridDim.x) {
    const int cnt = leaf_count[l];
    if (cnt < min_count || cnt > P) continue;
    sort_leaf_lds<P>(pos4, hb, leaf_begin[l], cnt, n, ax, order, ox, oy, oz, key, idx);
  }
}

// (key, index) as one orderable 64-bit word: ascending float order (-0 taken
// as +0, so that equal keys tie) then ascending in-leaf index.
__device__ __forceinline__ uint64_t sort_word(float key, int idx) {
  uint32_t u = __float_as_uint(key + 0.0f);
  u ^= (u >> 31) ? 0xffffffffu : 0x80000000u;
  return ((uint64_t)u << 32) | (uint32_t)idx;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor((unsigned)(v & 0xffffffffu), m, 64);
  const uint32_t hi = __shfl_xor((unsigned)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of 64*E words held E per lane (element e = lane*E + r),
// entirely in registers: partners within a lane are swapped in place, across
// lanes exchanged with shuffles.
template <int E>
__device__ __forceinline__ void wave_bitonic(uint64_t (&w)[E], int lane) {
  constexpr int P = 64 * E;
#pragma unroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if ((r & j) == 0) {
            const int i = lane * E + r;
            const bool up = (i & k) == 0;
            const uint64_t a = w[r], b = w[r | j];
            const bool sw = (a > b) == up;
            w[r] = sw ? b : a;
            w[r | j] = sw ? a : b;
          }
        }
      } else {
        const int lm = j / E;
        const bool lower = (lane & lm) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int i = lane * E + r;
          const bool up = (i & k) == 0;
          const uint64_t o = shfl_xor_u64(w[r], lm);
          const bool keep_min = (lower == up);
          const uint64_t mn = w[r] < o ? w[r] : o;
          const uint64_t mx = w[r] < o ? o : w[r];
          w[r] = keep_min ? mn : mx;
        }
      }
    }
  }
}

template <int E>
__device__ __forceinline__ void sort_leaf_axes(const float4 *__restrict__ pos4, const float *__restrict__ hb, int b,
                                               int cnt, int64_t n,
                                               const AxisTab &ax, uint16_t *__restrict__ order, int lane,
                                               int a_first, int a_end) {
  float ox[E], oy[E], oz[E], ow[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    if (e < cnt) {
      const float4 q = pos4[b + e];
      ox[r] = q.x;
      oy[r] = q.y;
      oz[r] = q.z;
      ow[r] = hb[b + e];
    } else {
      ox[r] = oy[r] = oz[r] = ow[r] = 0.f;
    }
  }
  for (int a = a_first; a < a_end; ++a) {
    // the H order: -H ascending
    const bool hrow = a == HORD_ROW;
    const float ex = hrow ? 0.f : ax.e[a][0], ey = hrow ? 0.f : ax.e[a][1], ez = hrow ? 0.f : ax.e[a][2];
    uint64_t w[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = lane * E + r;
      const float key = hrow ? -ow[r] : fmaf(oz[r], ez, fmaf(oy[r], ey, ox[r] * ex));
      w[r] = e < cnt ? sort_word(key, e) : ~0ull;
    }
    wave_bitonic<E>(w, lane);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = lane * E + r;
      if (e < cnt) order[(int64_t)a * n + b + e] = (uint16_t)(w[r] & 0xffffu);
    }
  }
}

// One wave per (leaf of at most 512 particles, order), grid-stride over
// every (leaf, order): the axis orders of leaves of min_count particles or
// more, the H order of every leaf.
__global__ __launch_bounds__(256) void axis_sort_wave_kernel(const float4 *__restrict__ pos4,
                                                             const float *__restrict__ hb,
                                                             const int32_t *__restrict__ leaf_begin,
                                                             const int32_t *__restrict__ leaf_count, int64_t nl,
                                                             int64_t n, AxisTab ax, int min_count,
                                                             uint16_t *__restrict__ order) {
  const int lane = threadIdx.x & 63;
  // work item = (leaf, order): the 14 sorts of a leaf run on 14 waves
  constexpr int NR = HORD_ROW + 1;
  const int64_t items = NR * nl;
  for (int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < items; it += (int64_t)gridDim.x * 4) {
    const int64_t l = it / NR;
    const int a = (int)(it - NR * l);
    const int cnt = leaf_count[l], b = leaf_begin[l];
    if (a != HORD_ROW && cnt < min_count) continue;
    if (cnt <= 64)
      sort_leaf_axes<1>(pos4, hb, b, cnt, n, ax, order, lane, a, a + 1);
    else if (cnt <= 128)
      sort_leaf_axes<2>(pos4, hb, b, cnt, n, ax, order, lane, a, a + 1);
    else if (cnt <= 256)
      sort_leaf_axes<4>(pos4, hb, b, cnt, n, ax, order, lane, a, a + 1);
    else if (cnt <= 512)
      sort_leaf_axes<8>(pos4, hb, b, cnt, n, ax, order, lane, a, a + 1);
  }
}

// The key (h_build) at rank hq_rank(q) of each leaf's H order, one thread
// per (leaf, q); 0 where the rank is past the leaf's count.
__global__ __launch_bounds__(256) void leaf_hq_kernel(const float *__restrict__ hb,
                                                      const int32_t *__restrict__ leaf_begin,
                                                      const int32_t *__restrict__ leaf_count, int64_t nl, int64_t n,
                                                      const uint16_t *__restrict__ order, float *__restrict__ hq) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= HQ_N * nl) return;
  const int64_t l = t / HQ_N;
  const int q = (int)(t - HQ_N * l);
  const int r = hq_rank(q), b = leaf_begin[l];
  hq[t] = r < leaf_count[l] ? hb[b + order[(int64_t)HORD_ROW * n + b + r]] : 0.f;
}

// The float whose sort_word key is the high half of w.
__device__ __forceinline__ float sort_word_key(uint64_t w) {
  const uint32_t u = (uint32_t)(w >> 32);
  return __uint_as_float((u >> 31) ? (u ^ 0x80000000u) : ~u);
}

// A leaf whose H grew past `limit` times the keys of its H order since they
// were taken: the keys become the current H (pos4.w), the order and its
// samples are renewed, and the growth bound is 1.  Leaves of more than 512
// particles keep their order (their bound stays valid).
template <int E>
__device__ __forceinline__ void rekey_leaf(const float4 *__restrict__ pos4, int64_t l, int b, int cnt, int64_t n,
                                           float *__restrict__ hb, uint16_t *__restrict__ order,
                                           float *__restrict__ hq, float *__restrict__ hgrow, int lane) {
  uint64_t w[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    if (e < cnt) {
      const float H = pos4[b + e].w;
      hb[b + e] = H;
      w[r] = sort_word(-H, e);
    } else {
      w[r] = ~0ull;
    }
  }
  wave_bitonic<E>(w, lane);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    if (e < cnt) order[(int64_t)HORD_ROW * n + b + e] = (uint16_t)(w[r] & 0xffffu);
  }
#pragma unroll
  for (int q = 0; q < HQ_N; ++q) {
    const int pos = hq_rank(q);
    if (pos < cnt) {
      if (lane == pos / E) hq[HQ_N * l + q] = -sort_word_key(w[pos % E]);
    } else if (lane == 0) {
      hq[HQ_N * l + q] = 0.f;
    }
  }
  if (lane == 0) hgrow[l] = 1.f;
}

__global__ __launch_bounds__(256) void hrow_rekey_kernel(const float4 *__restrict__ pos4,
                                                         const int32_t *__restrict__ leaf_begin,
                                                         const int32_t *__restrict__ leaf_count, int64_t nl,
                                                         int64_t n, float limit, float *__restrict__ hb,
                                                         uint16_t *__restrict__ order, float *__restrict__ hq,
                                                         float *__restrict__ hgrow) {
  const int lane = threadIdx.x & 63;
  // each wave checks 64 leaves at once, one per lane, then keys those flagged
  for (int64_t l0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64; l0 < nl; l0 += (int64_t)gridDim.x * 256) {
    const bool flag = l0 + lane < nl && hgrow[l0 + lane] > limit;
    for (uint64_t m = __ballot(flag); m; m &= m - 1) {
    const int64_t l = l0 + __ffsll((unsigned long long)m) - 1;
    const int cnt = leaf_count[l], b = leaf_begin[l];
    if (cnt <= 64)
      rekey_leaf<1>(pos4, l, b, cnt, n, hb, order, hq, hgrow, lane);
    else if (cnt <= 128)
      rekey_leaf<2>(pos4, l, b, cnt, n, hb, order, hq, hgrow, lane);
    else if (cnt <= 256)
      rekey_leaf<4>(pos4, l, b, cnt, n, hb, order, hq, hgrow, lane);
    else if (cnt <= 512)
      rekey_leaf<8>(pos4, l, b, cnt, n, hb, order, hq, hgrow, lane);
    }
  }
}

// Sorts the 13 axes of every leaf of at least min_count particles, by the
// offsets of the full build, and the H order of every leaf with its samples.
// Grids sized to the machine, not to the leaves.
static sph_status sort_leaves(sph_ctx *ctx, int min_count) {
  const int64_t n = ctx->n, nl = ctx->n_leaves;
  if (nl <= 0) return SPH_OK;
  const AxisTab ax = host_axes();
  {
    PROF(ctx, "axis_sort");
    const int64_t blocks = std::min<int64_t>(ceil_div((HORD_ROW + 1) * nl, 4), (int64_t)ctx->n_cu * 8);
    axis_sort_wave_kernel<<<(unsigned)blocks, 256, 0, ctx->stream>>>(
        (const float4 *)ctx->pos4_build.p, (const float *)ctx->h_build.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p,
        nl, n, ax, min_count, (uint16_t *)ctx->axis_order.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  if (ctx->max_leaf > 512) {
    PROF(ctx, "axis_sort");
    const int64_t blocks = std::min<int64_t>(nl, (int64_t)ctx->n_cu * 2);
    axis_sort_kernel<4096><<<(unsigned)blocks, AS_THREADS, 0, ctx->stream>>>(
        (const float4 *)ctx->pos4_build.p, (const float *)ctx->h_build.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p,
        nl, n, ax, std::max(513, min_count), (uint16_t *)ctx->axis_order.p);
    HIP_TRY(ctx, hipGetLastError());
  }
  {
    PROF(ctx, "axis_sort");
    leaf_hq_kernel<<<(unsigned)ceil_div(HQ_N * nl, 256), 256, 0, ctx->stream>>>(
        (const float *)ctx->h_build.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p,
        nl, n, (const uint16_t *)ctx->axis_order.p, (float *)ctx->leaf_hq.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}

// After a full build: the axis orders of every leaf of more than two
// 64-particle tiles (the loops read smaller leaves whole, unsorted) and the H
// order of every leaf, at once.  The keys are the offsets and H of the full
// build, so cell updates keep the orders.  Where
// the paper runs sort tasks only for the active cells of a step, one launch
// over all leaves here costs less than the per-step launches that finding
// the newly reached leaves would take.
sph_status sort_cells_impl(sph_ctx *ctx) {
  const int64_t n = ctx->n;
  SPH_TRY(sph_ensure(ctx, ctx->axis_order, sizeof(uint16_t) * (HORD_ROW + 1) * (size_t)n));
  if (!ctx->leaves_checked) {
    int32_t maxc;
    SPH_TRY(read_scalars(ctx, SC_MAXLEAF, 1, &maxc));
    if (maxc > 4096)
      return sph_fail(ctx, SPH_EINVAL, "sort_cells: a leaf holds %d particles (max 4096 for the axis sorts)", maxc);
    ctx->max_leaf = maxc;
    SPH_TRY(sort_leaves(ctx, 129));
    ctx->leaves_checked = 1;
  } else if (ctx->n_leaves > 0) {
    // kept cells: leaves whose H outgrew the keys of their H order by more
    // than 2% are keyed again from the current H
    const int64_t nl = ctx->n_leaves;
    PROF(ctx, "axis_sort");
    hrow_rekey_kernel<<<(unsigned)std::min<int64_t>(ceil_div(nl, 256), (int64_t)ctx->n_cu * 8), 256, 0, ctx->stream>>>(
        (const float4 *)ctx->pos4.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p, nl, n,
        1.02f, (float *)ctx->h_build.p, (uint16_t *)ctx->axis_order.p, (float *)ctx->leaf_hq.p,
        (float *)ctx->leaf_hgrow.p);
    HIP_TRY(ctx, hipGetLastError());
  }
  ctx->state = 2;
  return SPH_OK;
}

// Every leaf, also those the loops read unsorted (for the introspection copy).
sph_status sort_all_leaves(sph_ctx *ctx) { return sort_leaves(ctx, 1); }
