// Per-cell particle sorts for neighbour pruning (the "sort" task of Fig. 5):
// for every leaf and each of the 13 directions of the half neighbour stencil,
// the in-leaf order of the projections d = e . o of the FP32 offsets at the
// last full build (ascending, ties by in-leaf index).  One workgroup per leaf, all 13 axes,
// bitonic sorts of (key, index) in LDS.
#include <math.h>

#include <algorithm>

#include "sph_internal.h"

#define AS_THREADS 256

// Workgroup LDS bitonic sort for leaves of 513..4096 particles (only at the
// maximum depth, where coincident particles cannot be split further).
template <int P>
__device__ void sort_leaf_lds(const float4 *__restrict__ pos4, int b, int cnt, int64_t n, const AxisTab &ax,
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
  for (int a = 0; a < 13; ++a) {
    const float ex = ax.e[a][0], ey = ax.e[a][1], ez = ax.e[a][2];
    for (int k = threadIdx.x; k < size; k += AS_THREADS) {
      if (k < cnt) {
        key[k] = fmaf(oz[k], ez, fmaf(oy[k], ey, ox[k] * ex));
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
    sort_leaf_lds<P>(pos4, leaf_begin[l], cnt, n, ax, order, ox, oy, oz, key, idx);
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
__device__ __forceinline__ void sort_leaf_axes(const float4 *__restrict__ pos4, int b, int cnt, int64_t n,
                                               const AxisTab &ax, uint16_t *__restrict__ order, int lane,
                                               int a_first, int a_end) {
  float ox[E], oy[E], oz[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    if (e < cnt) {
      const float4 q = pos4[b + e];
      ox[r] = q.x;
      oy[r] = q.y;
      oz[r] = q.z;
    } else {
      ox[r] = oy[r] = oz[r] = 0.f;
    }
  }
  for (int a = a_first; a < a_end; ++a) {
    const float ex = ax.e[a][0], ey = ax.e[a][1], ez = ax.e[a][2];
    uint64_t w[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = lane * E + r;
      w[r] = e < cnt ? sort_word(fmaf(oz[r], ez, fmaf(oy[r], ey, ox[r] * ex)), e) : ~0ull;
    }
    wave_bitonic<E>(w, lane);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = lane * E + r;
      if (e < cnt) order[(int64_t)a * n + b + e] = (uint16_t)(w[r] & 0xffffu);
    }
  }
}

// One wave per (leaf of min_count..512 particles, axis), grid-stride over
// every (leaf, axis).
__global__ __launch_bounds__(256) void axis_sort_wave_kernel(const float4 *__restrict__ pos4,
                                                             const int32_t *__restrict__ leaf_begin,
                                                             const int32_t *__restrict__ leaf_count, int64_t nl,
                                                             int64_t n, AxisTab ax, int min_count,
                                                             uint16_t *__restrict__ order) {
  const int lane = threadIdx.x & 63;
  // work item = (leaf, axis): the 13 sorts of a leaf run on 13 waves
  const int64_t items = 13 * nl;
  for (int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < items; it += (int64_t)gridDim.x * 4) {
    const int64_t l = it / 13;
    const int a = (int)(it - 13 * l);
    const int cnt = leaf_count[l], b = leaf_begin[l];
    if (cnt < min_count) continue;
    if (cnt <= 64)
      sort_leaf_axes<1>(pos4, b, cnt, n, ax, order, lane, a, a + 1);
    else if (cnt <= 128)
      sort_leaf_axes<2>(pos4, b, cnt, n, ax, order, lane, a, a + 1);
    else if (cnt <= 256)
      sort_leaf_axes<4>(pos4, b, cnt, n, ax, order, lane, a, a + 1);
    else if (cnt <= 512)
      sort_leaf_axes<8>(pos4, b, cnt, n, ax, order, lane, a, a + 1);
  }
}

// Sorts the 13 axes of every leaf of at least min_count particles, by the
// offsets of the full build.  Grids sized to the machine, not to the leaves.
static sph_status sort_leaves(sph_ctx *ctx, int min_count) {
  const int64_t n = ctx->n, nl = ctx->n_leaves;
  if (nl <= 0 || ctx->max_leaf < min_count) return SPH_OK;
  const AxisTab ax = host_axes();
  {
    PROF(ctx, "axis_sort");
    const int64_t blocks = std::min<int64_t>(ceil_div(13 * nl, 4), (int64_t)ctx->n_cu * 8);
    axis_sort_wave_kernel<<<(unsigned)blocks, 256, 0, ctx->stream>>>(
        (const float4 *)ctx->pos4_build.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p,
        nl, n, ax, min_count, (uint16_t *)ctx->axis_order.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  if (ctx->max_leaf > 512) {
    PROF(ctx, "axis_sort");
    const int64_t blocks = std::min<int64_t>(nl, (int64_t)ctx->n_cu * 2);
    axis_sort_kernel<4096><<<(unsigned)blocks, AS_THREADS, 0, ctx->stream>>>(
        (const float4 *)ctx->pos4_build.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p,
        nl, n, ax, std::max(513, min_count), (uint16_t *)ctx->axis_order.p);
    HIP_TRY(ctx, hipGetLastError());
  }
  return SPH_OK;
}

// After a full build: every leaf of more than two 64-particle tiles is
// sorted at once (the loops read smaller leaves whole, unsorted).  The keys
// are the offsets of the full build, so cell updates keep the orders.  Where
// the paper runs sort tasks only for the active cells of a step, one launch
// over all leaves here costs less than the per-step launches that finding
// the newly reached leaves would take.
sph_status sort_cells_impl(sph_ctx *ctx) {
  const int64_t n = ctx->n;
  SPH_TRY(sph_ensure(ctx, ctx->axis_order, sizeof(uint16_t) * 13 * (size_t)n));
  if (!ctx->leaves_checked) {
    int32_t maxc;
    SPH_TRY(read_scalars(ctx, SC_MAXLEAF, 1, &maxc));
    if (maxc > 4096)
      return sph_fail(ctx, SPH_EINVAL, "sort_cells: a leaf holds %d particles (max 4096 for the axis sorts)", maxc);
    ctx->max_leaf = maxc;
    SPH_TRY(sort_leaves(ctx, 129));
    ctx->leaves_checked = 1;
  }
  ctx->state = 2;
  return SPH_OK;
}

// Every leaf, also those the loops read unsorted (for the introspection copy).
sph_status sort_all_leaves(sph_ctx *ctx) { return sort_leaves(ctx, 1); }
