// Adaptive cell build (Sec. III-A): a fixed top-level grid refined by octree
// splits while a cell holds at least split_count particles.  Particles are
// ordered by Morton key of their D-bit integer coordinates (ties by original
// index), so every cell of the octree is a contiguous range of that order.
#include <math.h>
#include <string.h>

#include "sph_internal.h"

#define BT 256

// x - L floor(x/L), folded into [0, L).  Compiled without contraction, so the
// product and the difference round separately.
__device__ __forceinline__ double wrap_box(double x, double L) {
  if (x >= 0.0 && x < L) return x;  // inside already (floor(x / L) = 0)
  const double q = floor(x / L);
  double xw = x - q * L;
  if (xw < 0.0) xw += L;
  if (xw >= L) xw -= L;
  return xw;
}

__device__ __forceinline__ uint64_t coord_of(double xw, double scale, int64_t kmax) {
  int64_t k = (int64_t)(xw * scale);
  if (k > kmax) k = kmax;
  if (k < 0) k = 0;
  return (uint64_t)k;
}

// Wraps positions in place, writes Morton keys and the identity permutation,
// and the largest H = GK32 * h (as int bits of a positive float).
__global__ __launch_bounds__(BT) void morton_kernel(double *__restrict__ x, double *__restrict__ y,
                                                    double *__restrict__ z, const float *__restrict__ h, int64_t n,
                                                    double L, double scale, int64_t kmax, uint64_t *__restrict__ keys,
                                                    int32_t *__restrict__ vals, float *__restrict__ hmax_part) {
  float hm = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
    const double xw = wrap_box(x[i], L), yw = wrap_box(y[i], L), zw = wrap_box(z[i], L);
    x[i] = xw;
    y[i] = yw;
    z[i] = zw;
    keys[i] = (spread3_21(coord_of(xw, scale, kmax)) << 2) | (spread3_21(coord_of(yw, scale, kmax)) << 1) |
              spread3_21(coord_of(zw, scale, kmax));
    vals[i] = (int32_t)i;
    hm = fmaxf(hm, GK32 * h[i]);
  }
  // block maximum to a per-block slot (no contended atomics)
  __shared__ float wmax[BT / 64];
  hm = wave_max_f(hm);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = hm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = wmax[0];
    for (int w = 1; w < BT / 64; ++w) b = fmaxf(b, wmax[w]);
    hmax_part[blockIdx.x] = b;
  }
}

__global__ __launch_bounds__(1024) void max_reduce_kernel(const float *__restrict__ part, int n, int *__restrict__ out_bits) {
  float m = 0.f;
  int k = threadIdx.x;
  for (; k + 3 * 1024 < n; k += 4 * 1024)
    m = fmaxf(fmaxf(m, part[k]), fmaxf(part[k + 1024], fmaxf(part[k + 2048], part[k + 3072])));
  for (; k < n; k += 1024) m = fmaxf(m, part[k]);
  __shared__ float wmax[16];
  m = wave_max_f(m);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = wmax[0];
    for (int w = 1; w < 16; ++w) b = fmaxf(b, wmax[w]);
    *out_bits = __float_as_int(b);
  }
}

// All particle arrays are reordered by two launches: gather into one staging
// buffer, then copy back into the caller's arrays.
struct PermArray {
  void *ptr;
  int64_t size;  // bytes per element: 8, 4 or 1
};
struct PermSet {
  PermArray a[40];
  int count;
};

__global__ __launch_bounds__(BT) void multi_gather_kernel(PermSet set, const int32_t *__restrict__ perm, int64_t n,
                                                          char *__restrict__ tmp) {
  for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < n; s += (int64_t)gridDim.x * BT) {
    const int64_t p = perm[s];
    int64_t off = 0;
    for (int k = 0; k < set.count; ++k) {
      const int64_t sz = set.a[k].size;
      if (sz == 8)
        reinterpret_cast<uint64_t *>(tmp + off)[s] = reinterpret_cast<const uint64_t *>(set.a[k].ptr)[p];
      else if (sz == 4)
        reinterpret_cast<uint32_t *>(tmp + off)[s] = reinterpret_cast<const uint32_t *>(set.a[k].ptr)[p];
      else
        reinterpret_cast<uint8_t *>(tmp + off)[s] = reinterpret_cast<const uint8_t *>(set.a[k].ptr)[p];
      off += sz * n;
    }
  }
}

__global__ __launch_bounds__(BT) void multi_copyback_kernel(PermSet set, int64_t n, const char *__restrict__ tmp) {
  for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < n; s += (int64_t)gridDim.x * BT) {
    int64_t off = 0;
    for (int k = 0; k < set.count; ++k) {
      const int64_t sz = set.a[k].size;
      if (sz == 8)
        reinterpret_cast<uint64_t *>(set.a[k].ptr)[s] = reinterpret_cast<const uint64_t *>(tmp + off)[s];
      else if (sz == 4)
        reinterpret_cast<uint32_t *>(set.a[k].ptr)[s] = reinterpret_cast<const uint32_t *>(tmp + off)[s];
      else
        reinterpret_cast<uint8_t *>(set.a[k].ptr)[s] = reinterpret_cast<const uint8_t *>(tmp + off)[s];
      off += sz * n;
    }
  }
}

__global__ __launch_bounds__(BT) void perm_out_kernel(const int32_t *__restrict__ perm, int64_t *__restrict__ out,
                                                      int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < n; s += (int64_t)gridDim.x * BT) out[s] = perm[s];
}

// flags[s] = 1 where the top-level prefix changes.
__global__ __launch_bounds__(BT) void prefix_start_kernel(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                          int32_t *__restrict__ flags) {
  for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < n; s += (int64_t)gridDim.x * BT)
    flags[s] = (s == 0) || ((keys[s] >> shift) != (keys[s - 1] >> shift));
}

__global__ __launch_bounds__(BT) void top_nodes_kernel(const int32_t *__restrict__ flags,
                                                       const int32_t *__restrict__ idx, int64_t n,
                                                       int2 *__restrict__ nodes) {
  for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < n; s += (int64_t)gridDim.x * BT)
    if (flags[s]) nodes[idx[s]].x = (int)s;
}

__global__ __launch_bounds__(BT) void node_ends_kernel(int2 *__restrict__ nodes, const int32_t *__restrict__ count,
                                                       int64_t n) {
  const int m = *count;
  for (int k = blockIdx.x * BT + threadIdx.x; k < m; k += gridDim.x * BT)
    nodes[k].y = (k + 1 < m) ? nodes[k + 1].x : (int)n;
}

// One octree level: each node either becomes a leaf (marked at its first
// particle) or is split into its non-empty children (appended to `out`).
__global__ __launch_bounds__(BT) void split_level_kernel(const uint64_t *__restrict__ keys,
                                                         const int2 *__restrict__ in, const int32_t *__restrict__ n_in,
                                                         int2 *__restrict__ out, int32_t *__restrict__ n_out,
                                                         int level, int D, int split, int32_t *__restrict__ leaf_flag,
                                                         int8_t *__restrict__ leaf_lvl) {
  const int m = *n_in;
  for (int k = blockIdx.x * BT + threadIdx.x; k < m; k += gridDim.x * BT) {
    const int2 nd = in[k];
    const int cnt = nd.y - nd.x;
    if (cnt < split || level >= D) {
      leaf_flag[nd.x] = 1;
      leaf_lvl[nd.x] = (int8_t)level;
      continue;
    }
    const int shift = 3 * (D - level - 1);
    int lo = nd.x;
    for (int c = 0; c < 8; ++c) {
      // first position in [lo, end) whose child digit exceeds c
      int a = lo, b = nd.y;
      while (a < b) {
        const int mid = (a + b) >> 1;
        if ((int)((keys[mid] >> shift) & 7ull) <= c)
          a = mid + 1;
        else
          b = mid;
      }
      if (a > lo) {
        const int slot = atomicAdd(n_out, 1);
        out[slot] = make_int2(lo, a);
      }
      lo = a;
    }
  }
}

__global__ __launch_bounds__(BT) void leaf_table_kernel(const int32_t *__restrict__ leaf_flag,
                                                        const int32_t *__restrict__ leaf_idx,
                                                        const int8_t *__restrict__ leaf_lvl,
                                                        const uint64_t *__restrict__ keys, int64_t n, int D,
                                                        int32_t *__restrict__ level, int32_t *__restrict__ ix,
                                                        int32_t *__restrict__ iy, int32_t *__restrict__ iz,
                                                        int32_t *__restrict__ begin, int32_t *__restrict__ leaf_of) {
  for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < n; s += (int64_t)gridDim.x * BT) {
    const int f = leaf_flag[s];
    const int l = leaf_idx[s] + f - 1;
    leaf_of[s] = l;
    if (f) {
      const int lv = leaf_lvl[s];
      const uint64_t pre = keys[s] >> (3 * (D - lv));
      level[l] = lv;
      ix[l] = (int32_t)compact3_21(pre >> 2);
      iy[l] = (int32_t)compact3_21(pre >> 1);
      iz[l] = (int32_t)compact3_21(pre);
      begin[l] = (int32_t)s;
    }
  }
}

__global__ __launch_bounds__(BT) void leaf_count_kernel(const int32_t *__restrict__ begin, int32_t *__restrict__ count,
                                                        int64_t nl, int64_t n, int32_t *__restrict__ max_count) {
  int mc = 0;
  for (int64_t l = (int64_t)blockIdx.x * BT + threadIdx.x; l < nl; l += (int64_t)gridDim.x * BT) {
    const int c = (int32_t)(((l + 1 < nl) ? begin[l + 1] : n) - begin[l]);
    count[l] = c;
    mc = max(mc, c);
  }
  mc = wave_max_i(mc);
  if ((threadIdx.x & 63) == 0) atomicMax(max_count, mc);
}

// FP32 offsets from the leaf centre, H, and the leaf's max H: one wave per
// leaf.  H is also each particle's key of its leaf's H order (hb), so the
// leaf's H growth bound starts at 1.
// Bounding boxes of the groups of 8 consecutive particles of every leaf, from
// the offsets of the full build (the sweeps prune partner leaves group by
// group, each box widened by its leaf's drift bound).  Group g of leaf l sits
// at slot (begin_l >> 3) + l + g: disjoint ranges, (n >> 3) + nl slots in all.
__global__ __launch_bounds__(BT) void group_box_kernel(const float4 *__restrict__ pos4,
                                                       const int32_t *__restrict__ begin,
                                                       const int32_t *__restrict__ count, int64_t nl,
                                                       float4 *__restrict__ glo, float4 *__restrict__ ghi) {
  const int64_t l = (int64_t)blockIdx.x * (BT / 64) + (threadIdx.x >> 6);
  if (l >= nl) return;
  const int lane = threadIdx.x & 63;
  const int b = begin[l], c = count[l];
  const int ng = (c + 7) >> 3;
  const int64_t slot0 = (int64_t)(b >> 3) + l;
  for (int g = lane; g < ng; g += 64) {
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
    float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
    const int k1 = min(c, 8 * g + 8);
    for (int k = 8 * g; k < k1; ++k) {
      const float4 q = pos4[b + k];
      lo.x = fminf(lo.x, q.x), lo.y = fminf(lo.y, q.y), lo.z = fminf(lo.z, q.z);
      hi.x = fmaxf(hi.x, q.x), hi.y = fmaxf(hi.y, q.y), hi.z = fmaxf(hi.z, q.z);
    }
    glo[slot0 + g] = lo;
    ghi[slot0 + g] = hi;
  }
}

__global__ __launch_bounds__(BT) void offsets_kernel(const double *__restrict__ x, const double *__restrict__ y,
                                                     const double *__restrict__ z, const float *__restrict__ h,
                                                     const int32_t *__restrict__ begin, const int32_t *__restrict__ count,
                                                     const int32_t *__restrict__ level, const int32_t *__restrict__ ix,
                                                     const int32_t *__restrict__ iy, const int32_t *__restrict__ iz,
                                                     int64_t nl, int D, double unit, float4 *__restrict__ pos4,
                                                     float *__restrict__ leaf_hmax, float *__restrict__ hb,
                                                     float *__restrict__ hgrow) {
  const int64_t l = (int64_t)blockIdx.x * (BT / 64) + (threadIdx.x >> 6);
  if (l >= nl) return;
  const int lane = threadIdx.x & 63;
  const int sh = D - level[l];
  const double cx = (double)((2 * (int64_t)ix[l] + 1) << sh) * unit;
  const double cy = (double)((2 * (int64_t)iy[l] + 1) << sh) * unit;
  const double cz = (double)((2 * (int64_t)iz[l] + 1) << sh) * unit;
  const int b = begin[l], c = count[l];
  float hm = 0.f;
  for (int k = lane; k < c; k += 64) {
    const int s = b + k;
    const float H = GK32 * h[s];
    pos4[s] = make_float4((float)(x[s] - cx), (float)(y[s] - cy), (float)(z[s] - cz), H);
    hb[s] = H;
    hm = fmaxf(hm, H);
  }
  hm = wave_max_f(hm);
  if (lane == 0) {
    leaf_hmax[l] = hm;
    hgrow[l] = 1.f;
  }
}

// Cell update without a rebuild (the leaves of the last build kept): wraps
// The FP32 offset of a wrapped position from its kept leaf's centre
// (cx, cy, cz), by the minimum image, stored with H in p4; returns the largest
// component of the displacement from the full build's position (minimum
// image).
__device__ __forceinline__ double kept_offset(double cx, double cy, double cz, double L, double xw, double yw,
                                              double zw, double xb, double yb, double zb, float H, float4 &p4) {
  const double half = 0.5 * L;
  double ox = xw - cx, oy = yw - cy, oz = zw - cz;
  ox = ox > half ? ox - L : (ox < -half ? ox + L : ox);
  oy = oy > half ? oy - L : (oy < -half ? oy + L : oy);
  oz = oz > half ? oz - L : (oz < -half ? oz + L : oz);
  double dx = xw - xb, dy = yw - yb, dz = zw - zb;
  dx = dx > half ? dx - L : (dx < -half ? dx + L : dx);
  dy = dy > half ? dy - L : (dy < -half ? dy + L : dy);
  dz = dz > half ? dz - L : (dz < -half ? dz + L : dz);
  p4 = make_float4((float)ox, (float)oy, (float)oz, H);
  return fmax(fabs(dx), fmax(fabs(dy), fabs(dz)));
}

// |displacement| <= sqrt(3) * (largest component), rounded up to float.
__device__ __forceinline__ float disp_bound(double d2m) {
  return d2m > 0.0 ? __int_as_float(__float_as_int((float)(d2m * 1.7320508075688772)) + 1) : 0.f;
}

// the positions, the FP32 offsets from the leaf centre (minimum image), H,
// the leaf's max H, the bound on H / (its H-order key) and a bound on its
// particles' displacement since the last build (sqrt(3) times the largest component, rounded up to float),
// and flags a rebuild when a leaf's particles moved more than frac of its
// width.  One wave per leaf; block maxima of H and of the displacement.
__global__ __launch_bounds__(BT) void update_kernel(double *__restrict__ x, double *__restrict__ y,
                                                    double *__restrict__ z, const float *__restrict__ h,
                                                    const double *__restrict__ xb, const double *__restrict__ yb,
                                                    const double *__restrict__ zb, const int32_t *__restrict__ begin,
                                                    const int32_t *__restrict__ count,
                                                    const int32_t *__restrict__ level, const int32_t *__restrict__ ix,
                                                    const int32_t *__restrict__ iy, const int32_t *__restrict__ iz,
                                                    int64_t nl, int D, double L, double unit, float frac,
                                                    float4 *__restrict__ pos4, float *__restrict__ leaf_hmax,
                                                    float *__restrict__ leaf_dx, float2 *__restrict__ block_max,
                                                    int32_t *__restrict__ sc_flag, const float *__restrict__ hb,
                                                    float *__restrict__ hgrow, PackArgs pk) {
  const int64_t l = (int64_t)blockIdx.x * (BT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  float hm = 0.f, dm = 0.f;
  if (l < nl) {
    const int sh = D - level[l];
    const double cx = (double)((2 * (int64_t)ix[l] + 1) << sh) * unit;
    const double cy = (double)((2 * (int64_t)iy[l] + 1) << sh) * unit;
    const double cz = (double)((2 * (int64_t)iz[l] + 1) << sh) * unit;
    const int b = begin[l], cnt = count[l];
    double d2m = 0.0;  // largest displacement component
    float gr = 0.f;    // largest H / its H-order key
    for (int k = lane; k < cnt; k += 64) {
      const int s = b + k;
      const double x0 = x[s], y0 = y[s], z0 = z[s];
      const double xw = wrap_box(x0, L), yw = wrap_box(y0, L), zw = wrap_box(z0, L);
      // written back only where the wrap moved a particle
      if (xw != x0) x[s] = xw;
      if (yw != y0) y[s] = yw;
      if (zw != z0) z[s] = zw;
      const float H = GK32 * h[s];
      d2m = fmax(d2m, kept_offset(cx, cy, cz, L, xw, yw, zw, xb[s], yb[s], zb[s], H, pos4[s]));
      hm = fmaxf(hm, H);
      gr = fmaxf(gr, H / hb[s]);
      if (pk.jvm) pack_one(pk, s);  // the loops' neighbour data, in the same pass
    }
    for (int o = 32; o > 0; o >>= 1) d2m = fmax(d2m, __shfl_xor(d2m, o, 64));
    hm = wave_max_f(hm);
    gr = wave_max_f(gr);
    dm = disp_bound(d2m);
    if (lane == 0) {
      leaf_hmax[l] = hm;
      hgrow[l] = gr;
      leaf_dx[l] = dm;
      if ((double)dm > (double)frac * ldexp(L, -level[l])) atomicOr(sc_flag, 1);
    }
  }
  __shared__ float wh[BT / 64], wd[BT / 64];
  if (lane == 0) {
    wh[threadIdx.x >> 6] = hm;
    wd[threadIdx.x >> 6] = dm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = wh[0], d = wd[0];
    for (int w = 1; w < BT / 64; ++w) {
      a = fmaxf(a, wh[w]);
      d = fmaxf(d, wd[w]);
    }
    block_max[blockIdx.x] = make_float2(a, d);  // reduced by a second kernel (no contended atomics)
  }
}

// One block of RT threads: every thread takes a strided quarter of the
// partials four at a time, so that its loads are in flight together.  Writes
// the max H and max displacement bits to out[0], out[1] and to hmax_bits (the
// running max H of the kept cells: the host reads out[] only to decide on a
// rebuild, which recomputes it), and moves the raised rebuild flag *flag to
// out[2], clearing it.  The three values also go to host_out (page-locked
// host memory) for the host to read after one synchronisation.
#define RT 1024
__global__ __launch_bounds__(RT) void max2_reduce_kernel(const float2 *__restrict__ part, int n,
                                                         int32_t *__restrict__ out_bits, int32_t *__restrict__ flag,
                                                         int32_t *__restrict__ hmax_bits, int32_t *host_out) {
  float a = 0.f, d = 0.f;
  int k = threadIdx.x;
  for (; k + 3 * RT < n; k += 4 * RT) {
    const float2 p0 = part[k], p1 = part[k + RT], p2 = part[k + 2 * RT], p3 = part[k + 3 * RT];
    a = fmaxf(fmaxf(a, p0.x), fmaxf(p1.x, fmaxf(p2.x, p3.x)));
    d = fmaxf(fmaxf(d, p0.y), fmaxf(p1.y, fmaxf(p2.y, p3.y)));
  }
  for (; k < n; k += RT) {
    a = fmaxf(a, part[k].x);
    d = fmaxf(d, part[k].y);
  }
  __shared__ float wa[RT / 64], wd[RT / 64];
  a = wave_max_f(a);
  d = wave_max_f(d);
  if ((threadIdx.x & 63) == 0) {
    wa[threadIdx.x >> 6] = a;
    wd[threadIdx.x >> 6] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < RT / 64; ++w) {
      a = fmaxf(a, wa[w]);
      d = fmaxf(d, wd[w]);
    }
    const int32_t fl = *flag;
    out_bits[0] = __float_as_int(a);
    out_bits[1] = __float_as_int(d);
    out_bits[2] = fl;
    *flag = 0;
    *hmax_bits = __float_as_int(a);
    host_out[0] = __float_as_int(a);
    host_out[1] = __float_as_int(d);
    host_out[2] = fl;
  }
}

// Half width of each leaf (float of the exact dyadic value).
__global__ __launch_bounds__(BT) void leaf_half_kernel(const int32_t *__restrict__ level, int64_t nl, double L,
                                                       float *__restrict__ half) {
  for (int64_t l = (int64_t)blockIdx.x * BT + threadIdx.x; l < nl; l += (int64_t)gridDim.x * BT)
    half[l] = (float)ldexp(L, -level[l] - 1);
}

__global__ __launch_bounds__(BT) void fill_i64_kernel(int64_t *__restrict__ out, int64_t n, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) out[i] = v;
}

__global__ __launch_bounds__(BT) void iota_kernel(int64_t *__restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) out[i] = i;
}

// Leaf range of every top-level cell (leaves of one top cell are contiguous).
__global__ __launch_bounds__(BT) void top_map_kernel(const int32_t *__restrict__ level, const int32_t *__restrict__ ix,
                                                     const int32_t *__restrict__ iy, const int32_t *__restrict__ iz,
                                                     int64_t nl, int k0, int32_t *__restrict__ first,
                                                     int32_t *__restrict__ last) {
  const int ntop = 1 << k0;
  for (int64_t l = (int64_t)blockIdx.x * BT + threadIdx.x; l < nl; l += (int64_t)gridDim.x * BT) {
    auto tc = [&](int64_t q) {
      const int s = level[q] - k0;
      return ((int64_t)(ix[q] >> s) * ntop + (iy[q] >> s)) * ntop + (iz[q] >> s);
    };
    const int64_t t = tc(l);
    if (l == 0 || tc(l - 1) != t) first[t] = (int32_t)l;
    if (l == nl - 1 || tc(l + 1) != t) last[t] = (int32_t)(l + 1);
  }
}

static unsigned grid_for(int64_t n) {
  int64_t g = ceil_div(n, BT);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

static void add_perm(PermSet &set, void *p, int64_t size) {
  if (!p) return;
  set.a[set.count].ptr = p;
  set.a[set.count].size = size;
  ++set.count;
}

sph_status build_cells_impl(sph_ctx *ctx, sph_particles *p, int64_t n, int64_t *perm_out) {
  if (!p || n <= 0 || n > INT32_MAX / 2) return sph_fail(ctx, SPH_EINVAL, "build_cells: bad particle count %lld", (long long)n);
  if (!p->x || !p->y || !p->z || !p->h) return sph_fail(ctx, SPH_EINVAL, "build_cells: x, y, z and h are required");
  const int D = ctx->prm.morton_depth;
  const double L = ctx->prm.box;
  const bool have_cells = ctx->built_n == n && ctx->n_leaves > 0;
  if (ctx->prm.rebuild_frac > 0.f && have_cells) {
    // keep the cells of the last build while every leaf's particles stay
    // within rebuild_frac of its width of where that build saw them
    int rebuild = 0;
    if (ctx->prm.lazy_drift) {
      SPH_TRY(lazy_keep_cells(ctx, &rebuild));
      if (!rebuild) {
        if (perm_out) {
          iota_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(perm_out, n);
          HIP_TRY(ctx, hipGetLastError());
        }
        return SPH_OK;
      }
    } else {
      SPH_TRY(update_cells(ctx, p, perm_out, &rebuild));
      if (!rebuild) return SPH_OK;
    }
  }
  // a full build sees every particle at the current time
  if (ctx->prm.lazy_drift && have_cells) SPH_TRY(drift_leaves(ctx, p, nullptr, nullptr, 0));
  ctx->n = n;
  ctx->state = 0;
  SPH_TRY(sph_ensure(ctx, ctx->keys_a, 8 * n));
  SPH_TRY(sph_ensure(ctx, ctx->keys_b, 8 * n));
  SPH_TRY(sph_ensure(ctx, ctx->vals_a, 4 * n));
  SPH_TRY(sph_ensure(ctx, ctx->vals_b, 4 * n));
  int32_t *sc = (int32_t *)ctx->scalars.p;
  HIP_TRY(ctx, hipMemsetAsync(sc, 0, sizeof(int32_t) * SC_COUNT, ctx->stream));

  const double scale = ldexp(1.0, D) / L;
  const int64_t kmax = ((int64_t)1 << D) - 1;
  const unsigned mgrid = grid_for(n);
  SPH_TRY(sph_ensure(ctx, ctx->scan_out, 4 * n));
  {
    PROF(ctx, "morton_keys");
    morton_kernel<<<mgrid, BT, 0, ctx->stream>>>(p->x, p->y, p->z, p->h, n, L, scale, kmax,
                                                (uint64_t *)ctx->keys_a.p, (int32_t *)ctx->vals_a.p,
                                                (float *)ctx->scan_out.p);
    max_reduce_kernel<<<1, 1024, 0, ctx->stream>>>((const float *)ctx->scan_out.p, (int)mgrid, sc + SC_HMAX_BITS);
  }
  HIP_TRY(ctx, hipGetLastError());
  SPH_TRY(radix_sort_pairs(ctx, n, 3 * D));

  // reorder every particle array into key order
  {
    PermSet set;
    set.count = 0;
    double *d8[] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->vfx, p->vfy, p->vfz};
    for (double *a : d8) add_perm(set, a, 8);
    float *f4[] = {p->m, p->u, p->A, p->Af, p->h, p->rho, p->drho_dh, p->f_gradh, p->divv, p->curlx, p->curly,
                   p->curlz, p->P, p->c, p->balsara, p->ax, p->ay, p->az, p->dA_dt, p->du_dt, p->vsig};
    for (float *a : f4) add_perm(set, a, 4);
    add_perm(set, p->nngb_density, 4);
    add_perm(set, p->nngb_force, 4);
    add_perm(set, p->time_bin, 1);
    int64_t bytes = 0;
    for (int k = 0; k < set.count; ++k) bytes += set.a[k].size * n;
    SPH_TRY(sph_ensure(ctx, ctx->gather_tmp, (size_t)bytes));
    PROF(ctx, "permute");
    multi_gather_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(set, (const int32_t *)ctx->vals_a.p, n,
                                                           (char *)ctx->gather_tmp.p);
    multi_copyback_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(set, n, (const char *)ctx->gather_tmp.p);
    HIP_TRY(ctx, hipGetLastError());
  }
  if (perm_out) {
    perm_out_kernel<<<grid_for(n), BT, 0, ctx->stream>>>((const int32_t *)ctx->vals_a.p, perm_out, n);
    HIP_TRY(ctx, hipGetLastError());
  }

  // top level from the largest smoothing length
  int32_t hb;
  SPH_TRY(read_scalars(ctx, SC_HMAX_BITS, 1, &hb));
  float hmax;
  memcpy(&hmax, &hb, 4);
  if (L * 0.25 < (double)hmax)
    return sph_fail(ctx, SPH_EINVAL, "build_cells: max H = %g exceeds a quarter of the box %g", hmax, L);
  int k0 = 2;
  while (k0 < ctx->prm.top_cap && k0 < D && ldexp(L, -(k0 + 1)) >= (double)hmax) ++k0;
  ctx->top_level = k0;

  const uint64_t *keys = (const uint64_t *)ctx->keys_a.p;
  SPH_TRY(sph_ensure(ctx, ctx->flags, 4 * n));
  SPH_TRY(sph_ensure(ctx, ctx->scan_out, 4 * n));
  SPH_TRY(sph_ensure(ctx, ctx->nodes_a, 8 * n));
  SPH_TRY(sph_ensure(ctx, ctx->nodes_b, 8 * n));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_lvl_at, n));
  int32_t *flags = (int32_t *)ctx->flags.p, *sidx = (int32_t *)ctx->scan_out.p;
  {
    PROF(ctx, "leaf_build");
    prefix_start_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(keys, n, 3 * (D - k0), flags);
  }
  HIP_TRY(ctx, hipGetLastError());
  SPH_TRY(scan_exclusive_i32(ctx, flags, sidx, n, sc + SC_NODES_A));
  int2 *na = (int2 *)ctx->nodes_a.p, *nb = (int2 *)ctx->nodes_b.p;
  {
    PROF(ctx, "leaf_build");
    top_nodes_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(flags, sidx, n, na);
  }
  {
    PROF(ctx, "leaf_build");
    node_ends_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(na, sc + SC_NODES_A, n);
  }
  HIP_TRY(ctx, hipGetLastError());

  // refine level by level; leaves are flagged at their first particle
  HIP_TRY(ctx, hipMemsetAsync(flags, 0, 4 * n, ctx->stream));
  int cin = SC_NODES_A, cout = SC_NODES_B;
  for (int lv = k0; lv <= D; ++lv) {
    HIP_TRY(ctx, hipMemsetAsync(sc + cout, 0, 4, ctx->stream));
    {
      PROF(ctx, "leaf_build");
      split_level_kernel<<<grid_for(n / 16 + 1), BT, 0, ctx->stream>>>(keys, na, sc + cin, nb, sc + cout, lv, D,
                                                             ctx->prm.split_count, flags,
                                                             (int8_t *)ctx->leaf_lvl_at.p);
    }
    HIP_TRY(ctx, hipGetLastError());
    int2 *t = na; na = nb; nb = t;
    int tc = cin; cin = cout; cout = tc;
  }
  SPH_TRY(scan_exclusive_i32(ctx, flags, sidx, n, sc + SC_TOTAL0));
  int32_t nl;
  SPH_TRY(read_scalars(ctx, SC_TOTAL0, 1, &nl));
  ctx->n_leaves = nl;
  SPH_TRY(sph_ensure(ctx, ctx->leaf_level, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_ix, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_iy, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_iz, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_begin, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_count, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_hmax, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_of, 4 * n));
  SPH_TRY(sph_ensure(ctx, ctx->pos4, 16 * n));
  SPH_TRY(sph_ensure(ctx, ctx->h_build, 4 * n));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_hgrow, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_hq, sizeof(float) * HQ_N * (size_t)nl));
  int32_t *lvl = (int32_t *)ctx->leaf_level.p, *lix = (int32_t *)ctx->leaf_ix.p, *liy = (int32_t *)ctx->leaf_iy.p,
          *liz = (int32_t *)ctx->leaf_iz.p, *lb = (int32_t *)ctx->leaf_begin.p, *lc = (int32_t *)ctx->leaf_count.p,
          *lof = (int32_t *)ctx->leaf_of.p;
  {
    PROF(ctx, "leaf_build");
    leaf_table_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(flags, sidx, (const int8_t *)ctx->leaf_lvl_at.p, keys, n, D,
                                                          lvl, lix, liy, liz, lb, lof);
  }
  {
    PROF(ctx, "leaf_build");
    leaf_count_kernel<<<grid_for(nl), BT, 0, ctx->stream>>>(lb, lc, nl, n, sc + SC_MAXLEAF);
  }
  HIP_TRY(ctx, hipGetLastError());
  {
    PROF(ctx, "offsets");
    offsets_kernel<<<(unsigned)ceil_div(nl, BT / 64), BT, 0, ctx->stream>>>(
        p->x, p->y, p->z, p->h, lb, lc, lvl, lix, liy, liz, nl, D, ldexp(L, -(D + 1)), (float4 *)ctx->pos4.p,
        (float *)ctx->leaf_hmax.p, (float *)ctx->h_build.p, (float *)ctx->leaf_hgrow.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  const int64_t ntop3 = (int64_t)1 << (3 * k0);
  SPH_TRY(sph_ensure(ctx, ctx->top_first, 4 * (size_t)ntop3));
  SPH_TRY(sph_ensure(ctx, ctx->top_last, 4 * (size_t)ntop3));
  HIP_TRY(ctx, hipMemsetAsync(ctx->top_first.p, 0, 4 * (size_t)ntop3, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(ctx->top_last.p, 0, 4 * (size_t)ntop3, ctx->stream));
  {
    PROF(ctx, "leaf_build");
    top_map_kernel<<<grid_for(nl), BT, 0, ctx->stream>>>(lvl, lix, liy, liz, nl, k0, (int32_t *)ctx->top_first.p,
                                                        (int32_t *)ctx->top_last.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  // positions the cells were built from (for the update criterion); no drift margin yet
  SPH_TRY(sph_ensure(ctx, ctx->x_build, 24 * (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_dx, 4 * (size_t)(nl > 0 ? nl : 1)));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_half, 4 * (size_t)(nl > 0 ? nl : 1)));
  leaf_half_kernel<<<grid_for(nl), BT, 0, ctx->stream>>>(lvl, nl, L, (float *)ctx->leaf_half.p);
  HIP_TRY(ctx, hipGetLastError());
  {
    double *xb = (double *)ctx->x_build.p;
    HIP_TRY(ctx, hipMemcpyAsync(xb, p->x, 8 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(xb + n, p->y, 8 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(xb + 2 * n, p->z, 8 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(ctx->leaf_dx.p, 0, 4 * (size_t)nl, ctx->stream));
  }
  // the axis sorts order these offsets until the next full build
  SPH_TRY(sph_ensure(ctx, ctx->pos4_build, 16 * (size_t)n));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->pos4_build.p, ctx->pos4.p, 16 * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
  {
    const size_t ngs = (size_t)(n >> 3) + (size_t)nl + 1;
    SPH_TRY(sph_ensure(ctx, ctx->gbox_lo, 16 * ngs));
    SPH_TRY(sph_ensure(ctx, ctx->gbox_hi, 16 * ngs));
    PROF(ctx, "leaf_build");
    group_box_kernel<<<(unsigned)ceil_div(nl, BT / 64), BT, 0, ctx->stream>>>(
        (const float4 *)ctx->pos4.p, lb, lc, nl, (float4 *)ctx->gbox_lo.p, (float4 *)ctx->gbox_hi.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  ctx->dx_max = 0.f;
  ctx->built_n = n;
  ctx->n_full_builds++;
  ctx->leaves_checked = 0;
  ctx->blocks_valid = 0;
  SPH_TRY(pack_neighbour_data(ctx, p));
  if (ctx->prm.lazy_drift) SPH_TRY(lazy_init_leaves(ctx, p));
  ctx->state = 1;
  return SPH_OK;
}

// ---------------------------------------------------------------- lazy drift
//
// With lazy_drift, sph_kick_drift only kicks the active particles and
// advances ctx->ti_now by the drift interval; a leaf's particles are drifted
// when a step needs them (the active leaves at sph_mark_active, the partner
// leaves of every new cell-pair list), with the drift-all formulas applied
// over the whole interval since the leaf's last drift: x += vf dt (wrapped),
// v += a dt, A += dA/dt dt, h *= exp(clip(div v dt / 3, +-0.2)).  Between
// drifts a leaf's displacement bound from the full build grows by its speed
// bound times the elapsed time; that bound is the leaf's drift margin for
// the pair search and the sweep stops of the step.

struct DriftArgs {
  double *x, *y, *z, *vx, *vy, *vz;
  const double *vfx, *vfy, *vfz;
  const float *ax, *ay, *az, *dA, *divv, *m;
  float *A, *h;
  float4 *jvm;
  double t_min;
  int64_t ti_now;
};

// Per leaf (one thread): this step's drift margin (the displacement bound at
// the current time), the rebuild flag, and block maxima of the margin and of
// a bound on the leaf's max H (a leaf behind the time line may grow by the
// clipped h prediction).
__global__ __launch_bounds__(BT) void lazy_bound_kernel(const int64_t *__restrict__ leaf_ti,
                                                        const float *__restrict__ vmax,
                                                        const float *__restrict__ dx_base,
                                                        const float *__restrict__ leaf_hmax,
                                                        const int32_t *__restrict__ level, int64_t nl, double L,
                                                        float frac, int64_t ti_now, double t_min,
                                                        float *__restrict__ leaf_dx, float2 *__restrict__ block_max,
                                                        int32_t *__restrict__ sc_flag) {
  const int64_t l = (int64_t)blockIdx.x * BT + threadIdx.x;
  float dm = 0.f, hb = 0.f;
  if (l < nl) {
    const int64_t t0 = leaf_ti[l];
    dm = dx_base[l];
    hb = leaf_hmax[l];
    if (t0 != ti_now) {
      const double bnd = (double)dm + (double)vmax[l] * ((double)(ti_now - t0) * t_min);
      dm = __int_as_float(__float_as_int((float)bnd) + 1);  // rounded up
      hb = hb * LAZY_HGROW;
    }
    leaf_dx[l] = dm;
    if ((double)dm > (double)frac * ldexp(L, -level[l])) atomicOr(sc_flag, 1);
  }
  dm = wave_max_f(dm);
  hb = wave_max_f(hb);
  __shared__ float wh[BT / 64], wd[BT / 64];
  if ((threadIdx.x & 63) == 0) {
    wh[threadIdx.x >> 6] = hb;
    wd[threadIdx.x >> 6] = dm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = wh[0], d = wd[0];
    for (int w = 1; w < BT / 64; ++w) {
      a = fmaxf(a, wh[w]);
      d = fmaxf(d, wd[w]);
    }
    block_max[blockIdx.x] = make_float2(a, d);
  }
}

// One wave per listed leaf (list_n on the device, or n_items when list_n is
// null; every leaf when list is null), grid-stride: a leaf behind the time
// line is drifted to it and its offsets, H, packed velocity, max H, H growth
// bound and exact displacement bound are renewed.
__global__ __launch_bounds__(BT) void drift_leaves_kernel(DriftArgs d, const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ list_n, int64_t n_items,
                                                          const double *__restrict__ xb,
                                                          const double *__restrict__ yb,
                                                          const double *__restrict__ zb,
                                                          const int32_t *__restrict__ begin,
                                                          const int32_t *__restrict__ count,
                                                          const int32_t *__restrict__ level,
                                                          const int32_t *__restrict__ ix,
                                                          const int32_t *__restrict__ iy,
                                                          const int32_t *__restrict__ iz, int D, double L,
                                                          double unit, int64_t *__restrict__ leaf_ti,
                                                          float4 *__restrict__ pos4, float *__restrict__ leaf_hmax,
                                                          float *__restrict__ dx_base, const float *__restrict__ hb,
                                                          float *__restrict__ hgrow) {
  const int lane = threadIdx.x & 63;
  const int64_t items = list_n ? (int64_t)*list_n : n_items;
  for (int64_t it = (int64_t)blockIdx.x * (BT / 64) + (threadIdx.x >> 6); it < items;
       it += (int64_t)gridDim.x * (BT / 64)) {
    const int64_t l = list ? list[it] : it;
    const int64_t t0 = leaf_ti[l];
    if (t0 == d.ti_now) continue;
    const double dt = (double)(d.ti_now - t0) * d.t_min;
    const int sh = D - level[l];
    const double cx = (double)((2 * (int64_t)ix[l] + 1) << sh) * unit;
    const double cy = (double)((2 * (int64_t)iy[l] + 1) << sh) * unit;
    const double cz = (double)((2 * (int64_t)iz[l] + 1) << sh) * unit;
    const int b = begin[l], cnt = count[l];
    double d2m = 0.0;
    float hm = 0.f, gr = 0.f;
    for (int k = lane; k < cnt; k += 64) {
      const int s = b + k;
      const double xw = wrap_box(d.x[s] + d.vfx[s] * dt, L);
      const double yw = wrap_box(d.y[s] + d.vfy[s] * dt, L);
      const double zw = wrap_box(d.z[s] + d.vfz[s] * dt, L);
      d.x[s] = xw;
      d.y[s] = yw;
      d.z[s] = zw;
      const double vx = d.vx[s] + (double)d.ax[s] * dt, vy = d.vy[s] + (double)d.ay[s] * dt,
                   vz = d.vz[s] + (double)d.az[s] * dt;
      d.vx[s] = vx;
      d.vy[s] = vy;
      d.vz[s] = vz;
      d.A[s] = (float)((double)d.A[s] + (double)d.dA[s] * dt);
      double e = (double)d.divv[s] * dt / 3.0;
      e = fmin(fmax(e, -0.2), 0.2);
      const float h = (float)((double)d.h[s] * exp(e));
      d.h[s] = h;
      const float H = GK32 * h;
      d2m = fmax(d2m, kept_offset(cx, cy, cz, L, xw, yw, zw, xb[s], yb[s], zb[s], H, pos4[s]));
      hm = fmaxf(hm, H);
      gr = fmaxf(gr, H / hb[s]);
      d.jvm[s] = make_float4((float)vx, (float)vy, (float)vz, d.m[s]);
    }
    for (int o = 32; o > 0; o >>= 1) d2m = fmax(d2m, __shfl_xor(d2m, o, 64));
    hm = wave_max_f(hm);
    gr = wave_max_f(gr);
    if (lane == 0) {
      leaf_hmax[l] = hm;
      hgrow[l] = gr;
      dx_base[l] = disp_bound(d2m);
      leaf_ti[l] = d.ti_now;
    }
  }
}

// Per leaf: the largest |vf| of its particles, rounded up to float.
__global__ __launch_bounds__(BT) void leaf_vmax_kernel(const double *__restrict__ vfx, const double *__restrict__ vfy,
                                                       const double *__restrict__ vfz,
                                                       const int32_t *__restrict__ begin,
                                                       const int32_t *__restrict__ count, int64_t nl,
                                                       float *__restrict__ vmax) {
  const int64_t l = (int64_t)blockIdx.x * (BT / 64) + (threadIdx.x >> 6);
  if (l >= nl) return;
  const int lane = threadIdx.x & 63;
  const int b = begin[l], cnt = count[l];
  double v2 = 0.0;
  for (int k = lane; k < cnt; k += 64) {
    const int s = b + k;
    v2 = fmax(v2, vfx[s] * vfx[s] + vfy[s] * vfy[s] + vfz[s] * vfz[s]);
  }
  for (int o = 32; o > 0; o >>= 1) v2 = fmax(v2, __shfl_xor(v2, o, 64));
  if (lane == 0) vmax[l] = v2 > 0.0 ? __int_as_float(__float_as_int((float)sqrt(v2)) + 1) : 0.f;
}

// Partner leaves of a cell-pair list that are behind the time line, each
// listed once per stamp.
__global__ __launch_bounds__(BT) void claim_drift_kernel(const PairEntry *__restrict__ pairs, int64_t np,
                                                         const int64_t *__restrict__ leaf_ti, int64_t ti_now,
                                                         int32_t *__restrict__ claim, int32_t stamp,
                                                         int32_t *__restrict__ list, int32_t *__restrict__ list_n) {
  for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < np; q += (int64_t)gridDim.x * BT) {
    const int B = pairs[q].b;
    if (leaf_ti[B] == ti_now) continue;
    if (atomicExch(&claim[B], stamp) != stamp) list[atomicAdd(list_n, 1)] = B;
  }
}

static DriftArgs drift_args(sph_ctx *ctx, const sph_particles *p) {
  DriftArgs d;
  d.x = p->x;
  d.y = p->y;
  d.z = p->z;
  d.vx = p->vx;
  d.vy = p->vy;
  d.vz = p->vz;
  d.vfx = p->vfx;
  d.vfy = p->vfy;
  d.vfz = p->vfz;
  d.ax = p->ax;
  d.ay = p->ay;
  d.az = p->az;
  d.dA = p->dA_dt;
  d.divv = p->divv;
  d.m = p->m;
  d.A = p->A;
  d.h = p->h;
  d.jvm = (float4 *)ctx->jvm.p;
  d.t_min = ctx->t_min_line;
  d.ti_now = ctx->ti_now;
  return d;
}

sph_status drift_leaves(sph_ctx *ctx, const sph_particles *p, const int32_t *list, const int32_t *list_n,
                        int64_t cap) {
  if (!ctx->prm.lazy_drift || ctx->n_leaves == 0) return SPH_OK;
  if (!p->vx || !p->vy || !p->vz || !p->vfx || !p->vfy || !p->vfz || !p->ax || !p->ay || !p->az || !p->dA_dt ||
      !p->divv || !p->m || !p->A || !p->h)
    return sph_fail(ctx, SPH_EINVAL, "lazy drift: a state array is missing");
  const int64_t nl = ctx->n_leaves;
  const int64_t items = list ? std::min<int64_t>(cap, nl) : nl;
  if (items <= 0) return SPH_OK;
  const double *xb = (const double *)ctx->x_build.p;
  const int64_t n = ctx->n;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(items, BT / 64), (int64_t)ctx->n_cu * 16);
  {
    PROF(ctx, "drift");
    drift_leaves_kernel<<<grid, BT, 0, ctx->stream>>>(
        drift_args(ctx, p), list, list_n, items, xb, xb + n, xb + 2 * n, (const int32_t *)ctx->leaf_begin.p,
        (const int32_t *)ctx->leaf_count.p, (const int32_t *)ctx->leaf_level.p, (const int32_t *)ctx->leaf_ix.p,
        (const int32_t *)ctx->leaf_iy.p, (const int32_t *)ctx->leaf_iz.p, ctx->prm.morton_depth, ctx->prm.box,
        ldexp(ctx->prm.box, -(ctx->prm.morton_depth + 1)), (int64_t *)ctx->leaf_ti.p, (float4 *)ctx->pos4.p,
        (float *)ctx->leaf_hmax.p, (float *)ctx->leaf_dx_base.p, (const float *)ctx->h_build.p,
        (float *)ctx->leaf_hgrow.p);
  }
  return sph_hip_check(ctx, hipGetLastError(), "drift_leaves_kernel");
}

sph_status drift_partners(sph_ctx *ctx, const sph_particles *p, int which) {
  if (!ctx->prm.lazy_drift) return SPH_OK;
  const int64_t np = which == 0 ? ctx->n_dpairs : ctx->n_fpairs;
  if (np <= 0) return SPH_OK;
  const int64_t nl = ctx->n_leaves;
  int32_t *list = (int32_t *)ctx->drift_list.p, *list_n = list + nl;
  HIP_TRY(ctx, hipMemsetAsync(list_n, 0, sizeof(int32_t), ctx->stream));
  ++ctx->drift_stamp;
  {
    PROF(ctx, "drift");
    claim_drift_kernel<<<(unsigned)std::min<int64_t>(ceil_div(np, BT), 4096), BT, 0, ctx->stream>>>(
        (const PairEntry *)(which == 0 ? ctx->dpairs.p : ctx->fpairs.p), np, (const int64_t *)ctx->leaf_ti.p,
        ctx->ti_now, (int32_t *)ctx->drift_claim.p, ctx->drift_stamp, list, list_n);
  }
  HIP_TRY(ctx, hipGetLastError());
  return drift_leaves(ctx, p, list, list_n, std::min<int64_t>(np, nl));
}

// After a full build: every leaf at the current time, no displacement, speed
// bounds from the full-step velocities.
sph_status lazy_init_leaves(sph_ctx *ctx, const sph_particles *p) {
  const int64_t nl = ctx->n_leaves;
  const size_t nl1 = (size_t)(nl > 0 ? nl : 1);
  SPH_TRY(sph_ensure(ctx, ctx->leaf_ti, sizeof(int64_t) * nl1));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_vmax, sizeof(float) * nl1));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_dx_base, sizeof(float) * nl1));
  SPH_TRY(sph_ensure(ctx, ctx->drift_claim, sizeof(int32_t) * nl1));
  SPH_TRY(sph_ensure(ctx, ctx->drift_list, sizeof(int32_t) * (nl1 + 1)));
  if (nl == 0) return SPH_OK;
  if (!p->vfx || !p->vfy || !p->vfz) return sph_fail(ctx, SPH_EINVAL, "lazy drift: vf is required");
  fill_i64_kernel<<<(unsigned)ceil_div(nl, BT), BT, 0, ctx->stream>>>((int64_t *)ctx->leaf_ti.p, nl, ctx->ti_now);
  HIP_TRY(ctx, hipMemsetAsync(ctx->leaf_dx_base.p, 0, sizeof(float) * (size_t)nl, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(ctx->drift_claim.p, 0, sizeof(int32_t) * (size_t)nl, ctx->stream));
  ctx->drift_stamp = 0;
  leaf_vmax_kernel<<<(unsigned)ceil_div(nl, BT / 64), BT, 0, ctx->stream>>>(
      p->vfx, p->vfy, p->vfz, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p, nl,
      (float *)ctx->leaf_vmax.p);
  return sph_hip_check(ctx, hipGetLastError(), "leaf_vmax_kernel");
}

// The lazy update path of sph_build_cells: the keep test from the per-leaf
// bounds only (one synchronisation); *rebuild = 1 when the full build must
// run (the caller drifts every leaf first).
sph_status lazy_keep_cells(sph_ctx *ctx, int *rebuild) {
  const int64_t nl = ctx->n_leaves;
  const double L = ctx->prm.box;
  int32_t *sc = (int32_t *)ctx->scalars.p;
  const int64_t blocks = ceil_div(nl, BT);
  SPH_TRY(sph_ensure(ctx, ctx->scan_out, sizeof(float2) * (size_t)blocks));
  {
    PROF(ctx, "cell_update");
    lazy_bound_kernel<<<(unsigned)blocks, BT, 0, ctx->stream>>>(
        (const int64_t *)ctx->leaf_ti.p, (const float *)ctx->leaf_vmax.p, (const float *)ctx->leaf_dx_base.p,
        (const float *)ctx->leaf_hmax.p, (const int32_t *)ctx->leaf_level.p, nl, L, ctx->prm.rebuild_frac,
        ctx->ti_now, ctx->t_min_line, (float *)ctx->leaf_dx.p, (float2 *)ctx->scan_out.p, sc + SC_UPD_FLAG_ACC);
    max2_reduce_kernel<<<1, RT, 0, ctx->stream>>>((const float2 *)ctx->scan_out.p, (int)blocks, sc + SC_UPD_HMAX,
                                                  sc + SC_UPD_FLAG_ACC, sc + SC_HMAX_BITS, ctx->pin_dev + PIN_UPD);
  }
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  SPH_TRY(pin_fetch(ctx, PIN_UPD, 3));
  int32_t st[3];
  memcpy(st, ctx->pin_h + PIN_UPD, sizeof st);
  float hmax, dxm;
  memcpy(&hmax, &st[0], 4);
  memcpy(&dxm, &st[1], 4);
  if (st[2] || L * 0.25 < (double)hmax) {
    *rebuild = 1;
    return SPH_OK;
  }
  *rebuild = 0;
  // (the reduction also set the running global max H to the kept cells' max H)
  ctx->dx_max = dxm;
  ctx->n_updates++;
  ctx->state = 1;
  return SPH_OK;
}

// The update path of sph_build_cells (see there): one launch over the leaves
// and one synchronisation; *rebuild = 1 when the full build must run.
sph_status update_cells(sph_ctx *ctx, sph_particles *p, int64_t *perm_out, int *rebuild) {
  const int64_t n = ctx->n, nl = ctx->n_leaves;
  const int D = ctx->prm.morton_depth;
  const double L = ctx->prm.box;
  int32_t *sc = (int32_t *)ctx->scalars.p;
  const double *xb = (const double *)ctx->x_build.p;
  const int64_t blocks = ceil_div(nl, BT / 64);
  SPH_TRY(sph_ensure(ctx, ctx->scan_out, sizeof(float2) * (size_t)blocks));
  // with every array given, the neighbour data are packed in the update pass
  // (the kernel writes them whether or not the cells are kept: a full build
  // packs again after its reorder)
  PackArgs pk;
  bool pack_all;
  SPH_TRY(pack_args(ctx, p, &pk, &pack_all));
  if (!pack_all) pk.jvm = nullptr;
  {
    PROF(ctx, "cell_update");
    update_kernel<<<(unsigned)blocks, BT, 0, ctx->stream>>>(
        p->x, p->y, p->z, p->h, xb, xb + n, xb + 2 * n, (const int32_t *)ctx->leaf_begin.p,
        (const int32_t *)ctx->leaf_count.p, (const int32_t *)ctx->leaf_level.p, (const int32_t *)ctx->leaf_ix.p,
        (const int32_t *)ctx->leaf_iy.p, (const int32_t *)ctx->leaf_iz.p, nl, D, L, ldexp(L, -(D + 1)),
        ctx->prm.rebuild_frac, (float4 *)ctx->pos4.p, (float *)ctx->leaf_hmax.p, (float *)ctx->leaf_dx.p,
        (float2 *)ctx->scan_out.p, sc + SC_UPD_FLAG_ACC, (const float *)ctx->h_build.p, (float *)ctx->leaf_hgrow.p, pk);
    max2_reduce_kernel<<<1, RT, 0, ctx->stream>>>((const float2 *)ctx->scan_out.p, (int)blocks, sc + SC_UPD_HMAX,
                                                  sc + SC_UPD_FLAG_ACC, sc + SC_HMAX_BITS, ctx->pin_dev + PIN_UPD);
  }
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  SPH_TRY(pin_fetch(ctx, PIN_UPD, 3));
  int32_t st[3];
  memcpy(st, ctx->pin_h + PIN_UPD, sizeof st);
  float hmax, dxm;
  memcpy(&hmax, &st[0], 4);
  memcpy(&dxm, &st[1], 4);
  if (st[2] || L * 0.25 < (double)hmax) {
    *rebuild = 1;
    return SPH_OK;
  }
  *rebuild = 0;
  // (the reduction also set the running global max H to the kept cells' max H)
  ctx->dx_max = dxm;
  ctx->n_updates++;
  if (perm_out) {
    iota_kernel<<<grid_for(n), BT, 0, ctx->stream>>>(perm_out, n);
    HIP_TRY(ctx, hipGetLastError());
  }
  if (!pack_all) SPH_TRY(pack_neighbour_data(ctx, p));
  ctx->state = 1;
  return SPH_OK;
}
