// Device-wide primitives: exclusive prefix sum (int32) and a stable LSD radix
// sort of (uint64 key, int32 value) pairs with 8-bit digits.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "sph_internal.h"

// ---------------------------------------------------------------- host helpers

sph_status sph_fail(sph_ctx *ctx, sph_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return code;
}

sph_status sph_hip_check(sph_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return SPH_OK;
  if (e == hipErrorOutOfMemory) return sph_fail(ctx, SPH_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return sph_fail(ctx, SPH_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

sph_status sph_ensure(sph_ctx *ctx, DevBuf &b, size_t bytes) {
  if (bytes <= b.cap && b.p) return SPH_OK;
  const DevAlloc &mem = ctx->mem;
  if (b.p) {
    if (b.from && b.from->free) {
      // stream-ordered: the allocator reuses the block only for work queued
      // after what is already on the stream
      b.release();
    } else {
      // the old buffer may still be read by queued work
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      b.release();
    }
  }
  size_t cap = bytes < 256 ? 256 : bytes + bytes / 8;
  cap = (cap + 255) & ~(size_t)255;
  if (mem.alloc) {
    b.p = mem.alloc(cap, (void *)mem.stream, mem.user);
    if (!b.p) return sph_fail(ctx, SPH_ENOMEM, "allocator callback returned no memory for %zu bytes", cap);
  } else {
    hipError_t e = hipMalloc(&b.p, cap);
    if (e != hipSuccess) {
      b.p = nullptr;
      return sph_fail(ctx, SPH_ENOMEM, "hipMalloc(%zu bytes) failed: %s", cap, hipGetErrorString(e));
    }
  }
  b.from = &ctx->mem;
  b.cap = cap;
  ctx->mem.live_bytes += (int64_t)cap;
  return SPH_OK;
}

sph_status pin_fetch(sph_ctx *ctx, int first, int count) {
  if (ctx->pin_mapped || count <= 0) return SPH_OK;
  if (first < 0 || first + count > PIN_COUNT) return sph_fail(ctx, SPH_EINVAL, "pin_fetch: slots out of range");
  HIP_TRY(ctx, hipMemcpyAsync(ctx->pin_h + first, ctx->pin_dev + first, sizeof(int32_t) * count,
                              hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return SPH_OK;
}

sph_status read_scalars(sph_ctx *ctx, int first, int count, int32_t *host) {
  if (count < 1 || count > PIN_MARK - PIN_SCALARS || first < 0 || first + count > SC_COUNT)
    return sph_fail(ctx, SPH_EINVAL, "read_scalars: slots [%d, %d) out of range", first, first + count);
  int32_t *pin = ctx->pin_h + PIN_SCALARS;
  HIP_TRY(ctx, hipMemcpyAsync(pin, (int32_t *)ctx->scalars.p + first, sizeof(int32_t) * count,
                              hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  memcpy(host, pin, sizeof(int32_t) * count);
  return SPH_OK;
}

// ---------------------------------------------------------------- scan

#define SCAN_THREADS 256
#define SCAN_ROUNDS 16
#define SCAN_TILE (SCAN_THREADS * SCAN_ROUNDS)

__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// WRITE=false: per-block totals.  WRITE=true: exclusive scan of the tile plus
// the block offset (or 0), and the grand total from the last block.  Each
// thread owns SCAN_ROUNDS consecutive elements: a serial sum in registers,
// one block-wide scan of the thread sums, then a serial write-out (no
// barrier per round).  In-place use (in == out) is safe: a thread reads its
// elements before it writes them.
template <bool WRITE>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(const int32_t *in, int32_t *out, int64_t n,
                                                            int32_t *__restrict__ block_sums,
                                                            const int32_t *__restrict__ block_offsets,
                                                            int32_t *__restrict__ total) {
  __shared__ int wsum[SCAN_THREADS / 64];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_ROUNDS;
  int v[SCAN_ROUNDS];
  int s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_ROUNDS; ++r) {
    v[r] = base + r < n ? in[base + r] : 0;
    s += v[r];
  }
  const int inc = wave_inclusive_scan(s);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int wpre = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_THREADS / 64; ++w) {
    const int t = wsum[w];
    if (w < wid) wpre += t;
    btot += t;
  }
  const int carry = (WRITE && block_offsets) ? block_offsets[blockIdx.x] : 0;
  if (WRITE) {
    int run = carry + wpre + inc - s;
#pragma unroll
    for (int r = 0; r < SCAN_ROUNDS; ++r) {
      if (base + r < n) out[base + r] = run;
      run += v[r];
    }
    if (total && blockIdx.x == gridDim.x - 1 && tid == 0) *total = carry + btot;
  } else if (tid == 0) {
    block_sums[blockIdx.x] = btot;
  }
}

static sph_status scan_rec(sph_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *total,
                           int32_t *tmp) {
  const int64_t nb = ceil_div(n, SCAN_TILE);
  if (nb <= 1) {
    {
      PROF(ctx, "scan");
      scan_kernel<true><<<1, SCAN_THREADS, 0, ctx->stream>>>(in, out, n, nullptr, nullptr, total);
    }
    return sph_hip_check(ctx, hipGetLastError(), "scan_kernel");
  }
  int32_t *bsum = tmp, *boff = tmp + nb;
  {
    PROF(ctx, "scan");
    scan_kernel<false><<<(unsigned)nb, SCAN_THREADS, 0, ctx->stream>>>(in, nullptr, n, bsum, nullptr, nullptr);
  }
  HIP_TRY(ctx, hipGetLastError());
  SPH_TRY(scan_rec(ctx, bsum, boff, nb, nullptr, tmp + 2 * nb));
  {
    PROF(ctx, "scan");
    scan_kernel<true><<<(unsigned)nb, SCAN_THREADS, 0, ctx->stream>>>(in, out, n, nullptr, boff, total);
  }
  return sph_hip_check(ctx, hipGetLastError(), "scan_kernel");
}

sph_status scan_exclusive_i32(sph_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev) {
  if (n <= 0) {
    if (total_dev) HIP_TRY(ctx, hipMemsetAsync(total_dev, 0, sizeof(int32_t), ctx->stream));
    return SPH_OK;
  }
  // temp: 2 * (n/T + n/T^2 + ...) ints
  int64_t need = 0, m = n;
  while (m > SCAN_TILE) {
    m = ceil_div(m, SCAN_TILE);
    need += 2 * m;
  }
  SPH_TRY(sph_ensure(ctx, ctx->scan_tmp, sizeof(int32_t) * (size_t)(need + 16)));
  return scan_rec(ctx, in, out, n, total_dev, (int32_t *)ctx->scan_tmp.p);
}

// ---------------------------------------------------------------- radix sort
//
// LSD radix sort with 8-bit digits.  Each pass counts the digits of every
// tile of the current arrangement (the per-tile counts of pass p depend on
// where pass p-1 put the keys), scans the counts into offsets, then ranks
// each tile stably, stages it in LDS in digit order and writes contiguous
// runs.

#define RS_THREADS 256
#define RS_ROUNDS 16
#define RS_TILE (RS_THREADS * RS_ROUNDS)

__global__ __launch_bounds__(RS_THREADS) void radix_hist_kernel(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                                int32_t *__restrict__ counts, int nblocks) {
  __shared__ int h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * RS_THREADS + tid;
    if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  counts[(int64_t)tid * nblocks + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(RS_THREADS) void radix_scatter_kernel(const uint64_t *__restrict__ kin,
                                                                   const int32_t *__restrict__ vin,
                                                                   uint64_t *__restrict__ kout,
                                                                   int32_t *__restrict__ vout, int64_t n, int shift,
                                                                   const int32_t *__restrict__ offsets, int nblocks) {
  __shared__ uint64_t sk[RS_TILE];
  __shared__ int32_t sv[RS_TILE];
  __shared__ int tcount[256];  // digit counts of this tile
  __shared__ int lbase[256];   // exclusive scan of tcount: start of each digit run in LDS
  __shared__ int run[256];
  __shared__ int wcnt[RS_THREADS / 64][256];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  tcount[tid] = 0;
  run[tid] = 0;
  __syncthreads();
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * RS_THREADS + tid;
    if (i < n) atomicAdd(&tcount[(int)((kin[i] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  // exclusive scan of the 256 tile counts by the first wave
  if (wid == 0) {
    int v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = tcount[lane * 4 + q];
      s += v[q];
    }
    int inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    int e = inc - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lbase[lane * 4 + q] = e;
      e += v[q];
    }
  }
  __syncthreads();
  // stable ranking, round by round, into the LDS tile in digit order
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)r * RS_THREADS + tid;
    const bool valid = i < n;
    const uint64_t key = valid ? kin[i] : 0ull;
    const int d = (int)((key >> shift) & 255ull);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = rank_below(peers);
    if (valid && rank == 0) wcnt[wid][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = lbase[d] + run[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      sk[pos] = key;
      sv[pos] = vin[i];
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) add += wcnt[w][tid];
    run[tid] += add;
    __syncthreads();
  }
  // contiguous runs out: element t of digit d goes to its global offset
  const int tile_n = (int)((n - base) < RS_TILE ? (n - base) : RS_TILE);
  for (int t = tid; t < tile_n; t += RS_THREADS) {
    const uint64_t key = sk[t];
    const int d = (int)((key >> shift) & 255ull);
    const int64_t g = (int64_t)offsets[(int64_t)d * nblocks + blockIdx.x] + (t - lbase[d]);
    kout[g] = key;
    vout[g] = sv[t];
  }
}

sph_status radix_sort_pairs(sph_ctx *ctx, int64_t n, int bits) {
  if (n <= 1) return SPH_OK;
  const int nblocks = (int)ceil_div(n, RS_TILE);
  const int passes = (bits + 7) / 8;
  const int64_t per = 256 * (int64_t)nblocks;
  SPH_TRY(sph_ensure(ctx, ctx->radix_counts, sizeof(int32_t) * (size_t)per * 2));
  int32_t *counts = (int32_t *)ctx->radix_counts.p;
  int32_t *offs = counts + per;
  uint64_t *ka = (uint64_t *)ctx->keys_a.p, *kb = (uint64_t *)ctx->keys_b.p;
  int32_t *va = (int32_t *)ctx->vals_a.p, *vb = (int32_t *)ctx->vals_b.p;
  for (int p = 0; p < passes; ++p) {
    {
      PROF(ctx, "radix_hist");
      radix_hist_kernel<<<nblocks, RS_THREADS, 0, ctx->stream>>>(ka, n, 8 * p, counts, nblocks);
    }
    HIP_TRY(ctx, hipGetLastError());
    SPH_TRY(scan_exclusive_i32(ctx, counts, offs, per, nullptr));
    {
      PROF(ctx, "radix_scatter");
      radix_scatter_kernel<<<nblocks, RS_THREADS, 0, ctx->stream>>>(ka, va, kb, vb, n, 8 * p, offs, nblocks);
    }
    HIP_TRY(ctx, hipGetLastError());
    uint64_t *tk = ka; ka = kb; kb = tk;
    int32_t *tv = va; va = vb; vb = tv;
  }
  if (passes & 1) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->keys_a.p, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->vals_a.p, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return SPH_OK;
}
