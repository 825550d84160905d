// Active set for the current time-bin (Eq. 2, Sec. III-D) and the cell-pair
// lists of the active cells (Sec. III-A: every pair of cells with at least one
// member on the active list, paired where the geometry allows an interaction).
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "sph_internal.h"

#define MT 256
#define CHUNK 64

// One wave per MARK_LEAVES consecutive leaves: active flags, the number of
// active particles, their max H, and the number of 64-particle chunks.  The
// leaves' first 64 particles are read together (most leaves hold fewer), so
// their loads are in flight at once; longer leaves continue one by one.
#define MARK_LEAVES 4
__global__ __launch_bounds__(MT) void mark_count_kernel(const int8_t *__restrict__ bin, int m,
                                                        const float4 *__restrict__ pos4,
                                                        const int32_t *__restrict__ leaf_begin,
                                                        const int32_t *__restrict__ leaf_count, int64_t nl,
                                                        uint8_t *__restrict__ active, int32_t *__restrict__ nact,
                                                        int32_t *__restrict__ isact, int32_t *__restrict__ nchunk,
                                                        float *__restrict__ hmax_act_leaf) {
  const int64_t l0 = ((int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6)) * MARK_LEAVES;
  if (l0 >= nl) return;
  const int lane = threadIdx.x & 63;
  int b[MARK_LEAVES], c[MARK_LEAVES], na[MARK_LEAVES];
  float hm[MARK_LEAVES];
  int8_t bn[MARK_LEAVES];
#pragma unroll
  for (int u = 0; u < MARK_LEAVES; ++u) {
    const int64_t l = l0 + u;
    b[u] = l < nl ? leaf_begin[l] : 0;
    c[u] = l < nl ? leaf_count[l] : 0;
    na[u] = 0;
    hm[u] = 0.f;
  }
#pragma unroll
  for (int u = 0; u < MARK_LEAVES; ++u) bn[u] = lane < c[u] ? bin[b[u] + lane] : (int8_t)127;
#pragma unroll
  for (int u = 0; u < MARK_LEAVES; ++u) {
    const bool a = lane < c[u] && bn[u] <= m;
    if (lane < c[u]) active[b[u] + lane] = a;
    if (a) hm[u] = pos4[b[u] + lane].w;
    na[u] = __popcll(__ballot(a));
  }
#pragma unroll
  for (int u = 0; u < MARK_LEAVES; ++u) {
    for (int t = 64; t < c[u]; t += 64) {
      const int k = t + lane;
      const bool a = k < c[u] && bin[b[u] + k] <= m;
      if (k < c[u]) active[b[u] + k] = a;
      if (a) hm[u] = fmaxf(hm[u], pos4[b[u] + k].w);
      na[u] += __popcll(__ballot(a));
    }
    const float h = wave_max_f(hm[u]);
    const int64_t l = l0 + u;
    if (lane == 0 && l < nl) {
      nact[l] = na[u];
      isact[l] = na[u] > 0;
      nchunk[l] = (na[u] + CHUNK - 1) / CHUNK;
      hmax_act_leaf[l] = h;
    }
  }
}

// One wave per active leaf: the ordered list of its active particles, the
// chunk of each, the active-leaf table and the chunk table.
__global__ __launch_bounds__(MT) void mark_fill_kernel(const uint8_t *__restrict__ active,
                                                       const int32_t *__restrict__ leaf_begin,
                                                       const int32_t *__restrict__ leaf_count, int64_t nl,
                                                       const int32_t *__restrict__ nact,
                                                       const int32_t *__restrict__ act_off,
                                                       const int32_t *__restrict__ actleaf_idx,
                                                       const int32_t *__restrict__ chunk_off,
                                                       const float *__restrict__ hmax_act_leaf,
                                                       int32_t *__restrict__ active_idx, int32_t *__restrict__ chunk_of,
                                                       int32_t *__restrict__ act_leaves, float *__restrict__ act_hmax,
                                                       int32_t *__restrict__ leaf_actleaf, Chunk *__restrict__ chunks) {
  const int64_t l = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6);
  if (l >= nl) return;
  const int lane = threadIdx.x & 63;
  const int na = nact[l];
  if (na == 0) {
    if (lane == 0) leaf_actleaf[l] = -1;
    return;
  }
  const int b = leaf_begin[l], c = leaf_count[l];
  const int ao = act_off[l];
  const int al = actleaf_idx[l] - act_off[nl];
  const int co = chunk_off[l] - actleaf_idx[nl];
  int run = 0;
  for (int t = 0; t < c; t += 64) {
    const int k = t + lane;
    const bool a = k < c && active[b + k];
    const uint64_t mask = __ballot(a);
    if (a) {
      const int r = run + rank_below(mask);
      active_idx[ao + r] = b + k;
      chunk_of[ao + r] = co + r / CHUNK;
    }
    run += __popcll(mask);
  }
  if (lane == 0) {
    act_leaves[al] = (int32_t)l;
    act_hmax[al] = hmax_act_leaf[l];
    leaf_actleaf[l] = al;
  }
  for (int q = lane; q * CHUNK < na; q += 64) {
    Chunk ch;
    ch.act_leaf = al;
    ch.begin = ao + q * CHUNK;
    ch.count = min(CHUNK, na - q * CHUNK);
    ch.leaf = (int32_t)l;
    chunks[co + q] = ch;
  }
}

struct PairGeom {
  int D, k0;
  int64_t nu;    // half-units per box side, 2^(D+1)
  double unit;   // L / 2^(D+1)
  double wtop;   // top-level cell side
};

__device__ __forceinline__ void leaf_centre_units(int D, int lvl, int ix, int iy, int iz, int64_t *c) {
  const int sh = D - lvl;
  c[0] = (2 * (int64_t)ix + 1) << sh;
  c[1] = (2 * (int64_t)iy + 1) << sh;
  c[2] = (2 * (int64_t)iz + 1) << sh;
}

// Bounding boxes (in half-units) of each run of LEAF_BLOCK consecutive leaves
// in Morton order, for pruning the pair search before its leaf tests.
__global__ __launch_bounds__(MT) void leaf_block_box_kernel(int D, const int32_t *__restrict__ level,
                                                           const int32_t *__restrict__ ix,
                                                           const int32_t *__restrict__ iy,
                                                           const int32_t *__restrict__ iz, int64_t nl,
                                                           int4 *__restrict__ box) {
  const int64_t q = (int64_t)blockIdx.x * MT + threadIdx.x;
  const int64_t b0 = q * LEAF_BLOCK;
  if (b0 >= nl) return;
  const int64_t b1 = b0 + LEAF_BLOCK < nl ? b0 + LEAF_BLOCK : nl;
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  for (int64_t l = b0; l < b1; ++l) {
    const int sh = D - level[l];
    const int c[3] = {(2 * ix[l] + 1) << sh, (2 * iy[l] + 1) << sh, (2 * iz[l] + 1) << sh};
    const int hw = 1 << sh;
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], c[d] - hw);
      hi[d] = max(hi[d], c[d] + hw);
    }
  }
  box[2 * q] = make_int4(lo[0], lo[1], lo[2], 0);
  box[2 * q + 1] = make_int4(hi[0], hi[1], hi[2], 0);
}

// One wave per active leaf A: walk the top-level cells within reach, test
// every leaf B there by periodic box distance (exact integer gaps, compared in
// double) and count (FILL=false) or write (FILL=true) the pairs in a fixed
// order.  mode 0: R = max active H of A; mode 1: R = max(that, max H of B).
// Runs of LEAF_BLOCK leaves are tested first by their bounding box with the
// largest reach any of their leaves can have (global max H, largest drift
// margin), so the leaves of a run out of reach are never read: the box gap is
// at most any member's gap and that reach at least any member's, so no pair
// is lost and the set and its order are those of the leaf tests alone.
template <bool FILL>
__global__ __launch_bounds__(MT) void pairs_kernel(int mode, float slack, PairGeom g, int64_t n_act_leaves,
                                                   const int32_t *__restrict__ act_leaves,
                                                   const float *__restrict__ act_hmax,
                                                   const int32_t *__restrict__ level, const int32_t *__restrict__ ix,
                                                   const int32_t *__restrict__ iy, const int32_t *__restrict__ iz,
                                                   const float *__restrict__ leaf_hmax,
                                                   const int32_t *__restrict__ top_first,
                                                   const int32_t *__restrict__ top_last,
                                                   const int32_t *__restrict__ hmax_bits,
                                                   const float *__restrict__ leaf_dx, float dx_max,
                                                   const int4 *__restrict__ block_box,
                                                   int32_t *__restrict__ counts, const int32_t *__restrict__ offs,
                                                   PairEntry *__restrict__ out, uint8_t *__restrict__ out_axis,
                                                   AxisTab ax, const int32_t *__restrict__ leaf_count,
                                                   int32_t *__restrict__ act_cost, float *__restrict__ reach_out,
                                                   const int64_t *__restrict__ leaf_ti, int64_t ti_now) {
  const int64_t a = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6);
  if (a >= n_act_leaves) return;
  const int lane = threadIdx.x & 63;
  const int A = act_leaves[a];
  const float RA = act_hmax[a] * slack;
  const int lvA = level[A];
  int64_t ca[3];
  leaf_centre_units(g.D, lvA, ix[A], iy[A], iz[A], ca);
  const int64_t hwa = (int64_t)1 << (g.D - lvA);
  // particles may have drifted out of their leaves since the cells were
  // built: leaf_dx widens every test by both leaves' displacement bounds
  const float dxA = leaf_dx[A];
  // the running max H over all particles (device scalar, raised by every
  // refresh of the leaf max H)
  const float hmax_global = __int_as_float(*hmax_bits);
  const float Rreach = (mode == 0 ? RA : fmaxf(RA, hmax_global)) + dxA + dx_max;
  const int ntop = 1 << g.k0;
  const double rr = ceil((double)Rreach / g.wtop);
  const int ring = (rr >= 0.0 && rr < (double)ntop) ? (int)rr : ntop;  // non-finite reach: every top cell
  const int sA = lvA - g.k0;
  const int t[3] = {ix[A] >> sA, iy[A] >> sA, iz[A] >> sA};
  int lo[3], cnt3[3];
  for (int d = 0; d < 3; ++d) {
    if (2 * ring + 1 >= ntop) {
      lo[d] = 0;
      cnt3[d] = ntop;
    } else {
      lo[d] = t[d] - ring;
      cnt3[d] = 2 * ring + 1;
    }
  }
  int written = 0;
  int staged = 0;
  const int base = FILL ? offs[a] : 0;
  // the top cells of the search box, 64 at a time; their runs of leaves as
  // one flat range (cells in order, runs in order), 64 runs per step; the
  // leaves of the runs in reach as a second flat range, 64 leaves per step
  __shared__ int cell_off[MT / 64][64], cell_first[MT / 64][64], cell_end[MT / 64][64];
  __shared__ int run_off[MT / 64][64], run_first[MT / 64][64];
  const int wv = threadIdx.x >> 6;
  int *coff = cell_off[wv], *cfirst = cell_first[wv], *cend = cell_end[wv];
  int *roff = run_off[wv], *rfirst = run_first[wv];
  const int ncell = cnt3[0] * cnt3[1] * cnt3[2];
  for (int c0 = 0; c0 < ncell; c0 += 64) {
    const int cc = c0 + lane;
    int f = 0, nleaf = 0;
    if (cc < ncell) {
      const int u = cc / (cnt3[1] * cnt3[2]), v = (cc / cnt3[2]) % cnt3[1], w = cc % cnt3[2];
      const int tx = ((lo[0] + u) % ntop + ntop) % ntop;
      const int ty = ((lo[1] + v) % ntop + ntop) % ntop;
      const int tz = ((lo[2] + w) % ntop + ntop) % ntop;
      const int64_t tc = ((int64_t)tx * ntop + ty) * ntop + tz;
      f = top_first[tc];
      nleaf = top_last[tc] - f;
    }
    const int nrun = nleaf > 0 ? (f + nleaf - 1) / LEAF_BLOCK - f / LEAF_BLOCK + 1 : 0;
    int incl = nrun;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    const int total_r = __shfl(incl, 63, 64);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    coff[lane] = incl - nrun;
    cfirst[lane] = f;
    cend[lane] = f + nleaf;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int r0 = 0; r0 < total_r; r0 += 64) {
      const int ri = r0 + lane;
      int lf = 0, nl_run = 0;
      if (ri < total_r) {
        // last cell whose runs start at or before ri (cells without runs
        // share the offset of the next one)
        int lo_ = 0, hi_ = 63;
        while (lo_ < hi_) {
          const int mid = (lo_ + hi_ + 1) >> 1;
          if (coff[mid] <= ri) lo_ = mid; else hi_ = mid - 1;
        }
        const int run = cfirst[lo_] / LEAF_BLOCK + (ri - coff[lo_]);
        lf = max(cfirst[lo_], run * LEAF_BLOCK);
        const int ll = min(cend[lo_], run * LEAF_BLOCK + LEAF_BLOCK);
        // the run's box against A's, nearest periodic image per axis
        const int4 blo = block_box[2 * run], bhi = block_box[2 * run + 1];
        const int64_t rl[3] = {blo.x, blo.y, blo.z}, rh[3] = {bhi.x, bhi.y, bhi.z};
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          int64_t best = INT64_MAX;
          for (int k = -1; k <= 1; ++k) {
            const int64_t s = (int64_t)k * g.nu;
            int64_t gap = rl[d] + s - (ca[d] + hwa);
            const int64_t g2 = (ca[d] - hwa) - (rh[d] + s);
            if (g2 > gap) gap = g2;
            if (gap < 0) gap = 0;
            if (gap < best) best = gap;
          }
          const double gd = (double)best * g.unit;
          d2 = d2 + gd * gd;
        }
        const double Rd = (double)Rreach;
        if (d2 < Rd * Rd) nl_run = ll - lf;
      }
      int incl2 = nl_run;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl2, o, 64);
        if (lane >= o) incl2 += t;
      }
      const int total = __shfl(incl2, 63, 64);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      roff[lane] = incl2 - nl_run;
      rfirst[lane] = lf;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    for (int t0 = 0; t0 < total; t0 += 64) {
      const int fi = t0 + lane;
      bool ok = false;
      int64_t dl[3] = {0, 0, 0};
      int B = 0;
      if (fi < total) {
        // last run whose leaves start at or before fi (runs out of reach
        // share the offset of the next one)
        int lo_ = 0, hi_ = 63;
        while (lo_ < hi_) {
          const int mid = (lo_ + hi_ + 1) >> 1;
          if (roff[mid] <= fi) lo_ = mid; else hi_ = mid - 1;
        }
        B = rfirst[lo_] + (fi - roff[lo_]);
        int64_t cb[3];
        const int lvB = level[B];
        leaf_centre_units(g.D, lvB, ix[B], iy[B], iz[B], cb);
        const int64_t hwb = (int64_t)1 << (g.D - lvB);
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          int64_t dd = cb[d] - ca[d];
          if (dd > g.nu / 2) dd -= g.nu;
          if (dd < -g.nu / 2) dd += g.nu;
          dl[d] = dd;
          int64_t gap = (dd < 0 ? -dd : dd) - hwa - hwb;
          if (gap < 0) gap = 0;
          const double gd = (double)gap * g.unit;
          d2 = d2 + gd * gd;
        }
        float R = RA;
        if (mode == 1) {
          // (lazy drift: a leaf behind the time line may grow by its drift)
          float hB = leaf_hmax[B];
          if (leaf_ti && leaf_ti[B] != ti_now) hB *= LAZY_HGROW;
          R = fmaxf(R, hB);
        }
        R = (R + dxA) + leaf_dx[B];
        const double Rd = (double)R;
        ok = d2 < Rd * Rd;
      }
      const uint64_t mask = __ballot(ok);
      if (FILL && ok) {
        PairEntry pe;
        pe.b = B;
        pe.sx = (float)((double)dl[0] * g.unit);
        pe.sy = (float)((double)dl[1] * g.unit);
        pe.sz = (float)((double)dl[2] * g.unit);
        out[base + written + rank_below(mask)] = pe;
        out_axis[base + written + rank_below(mask)] = sweep_axis_code(ax, pe.sx, pe.sy, pe.sz);
        if (act_cost) staged += leaf_count[B];
      }
      written += __popcll(mask);
    }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if (!FILL && lane == 0) counts[a] = written;
  if (FILL && act_cost) {
    staged = wave_sum_i(staged);
    if (lane == 0) act_cost[a] = staged;
  }
  // the radius the list is complete for (the h solve's steps stay within it)
  if (FILL && reach_out && lane == 0) reach_out[a] = RA;
}

// Max H over each active leaf's particles (all of them), the max over its
// active ones, the H growth bound of its H order, and the running global max,
// after the density loop changed active smoothing lengths.  One wave per
// active leaf; `boxes` holds one set of arguments per box (blockIdx.y).
struct RefreshArgs {
  const float4 *pos4;
  const uint8_t *active;
  const int32_t *leaf_begin, *leaf_count, *act_leaves;
  int64_t n_act_leaves;
  float *leaf_hmax, *act_hmax;
  int *hmax_bits;
  const float *hb;
  float *hgrow;
};

__device__ __forceinline__ void refresh_body(const RefreshArgs &r) {
  const int lane = threadIdx.x & 63;
  for (int64_t a = (int64_t)blockIdx.x * (MT / 64) + (threadIdx.x >> 6); a < r.n_act_leaves;
       a += (int64_t)gridDim.x * (MT / 64)) {
    const int A = r.act_leaves[a];
    const int b = r.leaf_begin[A], c = r.leaf_count[A];
    float hm = 0.f, ha = 0.f, gr = 0.f;
    for (int k = lane; k < c; k += 64) {
      const float H = r.pos4[b + k].w;
      hm = fmaxf(hm, H);
      gr = fmaxf(gr, H / r.hb[b + k]);
      if (r.active[b + k]) ha = fmaxf(ha, H);
    }
    hm = wave_max_f(hm);
    ha = wave_max_f(ha);
    gr = wave_max_f(gr);
    if (lane == 0) {
      r.leaf_hmax[A] = hm;
      r.hgrow[A] = gr;
      r.act_hmax[a] = ha;
      // the running max rarely rises: most waves skip the contended atomic
      if (hm > __int_as_float(__atomic_load_n(r.hmax_bits, __ATOMIC_RELAXED)))
        atomicMax(r.hmax_bits, __float_as_int(hm));
    }
  }
}

__global__ __launch_bounds__(MT) void leaf_hmax_refresh_kernel(RefreshArgs r) { refresh_body(r); }

__global__ __launch_bounds__(MT) void leaf_hmax_refresh_multi_kernel(const RefreshArgs *__restrict__ boxes) {
  refresh_body(boxes[blockIdx.y]);
}

static RefreshArgs refresh_args(sph_ctx *ctx) {
  RefreshArgs r;
  r.pos4 = (const float4 *)ctx->pos4.p;
  r.active = (const uint8_t *)ctx->active.p;
  r.leaf_begin = (const int32_t *)ctx->leaf_begin.p;
  r.leaf_count = (const int32_t *)ctx->leaf_count.p;
  r.act_leaves = (const int32_t *)ctx->act_leaves.p;
  r.n_act_leaves = ctx->n_active_leaves;
  r.leaf_hmax = (float *)ctx->leaf_hmax.p;
  r.act_hmax = (float *)ctx->act_hmax.p;
  r.hmax_bits = (int32_t *)ctx->scalars.p + SC_HMAX_BITS;
  r.hb = (const float *)ctx->h_build.p;
  r.hgrow = (float *)ctx->leaf_hgrow.p;
  return r;
}

// One int32 into a page-locked host slot.
__global__ void copy_total_kernel(const int32_t *__restrict__ src, int32_t *host) {
  if (threadIdx.x == 0) host[0] = *src;
}

// The three totals of the active-set scan (active particles, active leaves,
// chunks: the scan output at nl, 2 nl and 3 nl) into page-locked host slots.
__global__ void mark_totals_kernel(const int32_t *__restrict__ aoff, int64_t nl, int32_t *host) {
  if (threadIdx.x < 3) host[threadIdx.x] = aoff[(threadIdx.x + 1) * nl];
}

static unsigned waves_grid(int64_t n_items) { return (unsigned)(ceil_div(n_items, MT / 64) > 0 ? ceil_div(n_items, MT / 64) : 1); }

static PairGeom pair_geom(const sph_ctx *ctx) {
  PairGeom g;
  g.D = ctx->prm.morton_depth;
  g.k0 = ctx->top_level;
  g.nu = (int64_t)1 << (g.D + 1);
  g.unit = ldexp(ctx->prm.box, -(g.D + 1));
  g.wtop = ldexp(ctx->prm.box, -g.k0);
  return g;
}

// which = 0: density lists, 1: force lists.  slack > 1 widens the reach of
// every active leaf (used when smoothing lengths grow during the h solve).
// Two phases so that several contexts can share one synchronisation: the
// count phase enqueues the per-leaf counts, their scan and the copy of the
// total into *host_total (valid once the stream has been synchronised); the
// fill phase writes the lists.
sph_status build_pairs_count(sph_ctx *ctx, int which, float slack, int32_t *host_total) {
  const int64_t na = ctx->n_active_leaves;
  if (which == 1) ctx->fpairs_counted = -1;  // a count read back later is no longer the current one
  DevBuf &off = which == 0 ? ctx->dpair_off : ctx->fpair_off;
  SPH_TRY(sph_ensure(ctx, ctx->pair_cnt, 4 * (size_t)(na + 1)));
  SPH_TRY(sph_ensure(ctx, ctx->act_cost, 4 * (size_t)(na + 1)));
  SPH_TRY(sph_ensure(ctx, ctx->act_reach, 4 * (size_t)(na + 1)));
  SPH_TRY(sph_ensure(ctx, off, 4 * (size_t)(na + 1)));
  if (host_total) *host_total = 0;
  if (na == 0) {
    HIP_TRY(ctx, hipMemsetAsync(off.p, 0, 4, ctx->stream));
    return SPH_OK;
  }
  const PairGeom g = pair_geom(ctx);
  const int64_t *lazy_ti = ctx->prm.lazy_drift ? (const int64_t *)ctx->leaf_ti.p : nullptr;
  if (!ctx->blocks_valid) {
    // run boxes of the current full build (cell updates keep the leaves)
    const int64_t nl = ctx->n_leaves, nrun = ceil_div(nl, LEAF_BLOCK);
    SPH_TRY(sph_ensure(ctx, ctx->block_box, 2 * sizeof(int4) * (size_t)(nrun > 0 ? nrun : 1)));
    if (nrun > 0) {
      PROF(ctx, "cell_pairs");
      leaf_block_box_kernel<<<(unsigned)ceil_div(nrun, MT), MT, 0, ctx->stream>>>(
          g.D, (const int32_t *)ctx->leaf_level.p, (const int32_t *)ctx->leaf_ix.p, (const int32_t *)ctx->leaf_iy.p,
          (const int32_t *)ctx->leaf_iz.p, nl, (int4 *)ctx->block_box.p);
      HIP_TRY(ctx, hipGetLastError());
    }
    ctx->blocks_valid = 1;
  }
  {
    PROF(ctx, "cell_pairs");
    pairs_kernel<false><<<waves_grid(na), MT, 0, ctx->stream>>>(
        which, slack, g, na, (const int32_t *)ctx->act_leaves.p, (const float *)ctx->act_hmax.p,
        (const int32_t *)ctx->leaf_level.p, (const int32_t *)ctx->leaf_ix.p, (const int32_t *)ctx->leaf_iy.p,
        (const int32_t *)ctx->leaf_iz.p, (const float *)ctx->leaf_hmax.p, (const int32_t *)ctx->top_first.p,
        (const int32_t *)ctx->top_last.p, (const int32_t *)ctx->scalars.p + SC_HMAX_BITS,
        (const float *)ctx->leaf_dx.p, ctx->dx_max, (const int4 *)ctx->block_box.p, (int32_t *)ctx->pair_cnt.p,
        nullptr, nullptr, nullptr, AxisTab(), nullptr, nullptr, nullptr, lazy_ti, ctx->ti_now);
  }
  HIP_TRY(ctx, hipGetLastError());
  int32_t *o = (int32_t *)off.p;
  SPH_TRY(scan_exclusive_i32(ctx, (const int32_t *)ctx->pair_cnt.p, o, na, o + na));
  // (a null host_total: the caller reads the total at offsets[n_active_leaves])
  if (host_total) HIP_TRY(ctx, hipMemcpyAsync(host_total, o + na, 4, hipMemcpyDeviceToHost, ctx->stream));
  return SPH_OK;
}

sph_status build_pairs_fill(sph_ctx *ctx, int which, float slack, int32_t np) {
  const int64_t na = ctx->n_active_leaves;
  DevBuf &off = which == 0 ? ctx->dpair_off : ctx->fpair_off;
  DevBuf &lst = which == 0 ? ctx->dpairs : ctx->fpairs;
  DevBuf &axl = which == 0 ? ctx->dpair_axis : ctx->fpair_axis;
  if (which == 0) ctx->n_dpairs = np; else ctx->n_fpairs = np;
  if (na == 0) return SPH_OK;
  SPH_TRY(sph_ensure(ctx, lst, sizeof(PairEntry) * (size_t)(np > 0 ? np : 1)));
  SPH_TRY(sph_ensure(ctx, axl, (size_t)(np > 0 ? np : 1)));
  const PairGeom g = pair_geom(ctx);
  const int64_t *lazy_ti = ctx->prm.lazy_drift ? (const int64_t *)ctx->leaf_ti.p : nullptr;
  {
    PROF(ctx, "cell_pairs");
    pairs_kernel<true><<<waves_grid(na), MT, 0, ctx->stream>>>(
        which, slack, g, na, (const int32_t *)ctx->act_leaves.p, (const float *)ctx->act_hmax.p,
        (const int32_t *)ctx->leaf_level.p, (const int32_t *)ctx->leaf_ix.p, (const int32_t *)ctx->leaf_iy.p,
        (const int32_t *)ctx->leaf_iz.p, (const float *)ctx->leaf_hmax.p, (const int32_t *)ctx->top_first.p,
        (const int32_t *)ctx->top_last.p, (const int32_t *)ctx->scalars.p + SC_HMAX_BITS,
        (const float *)ctx->leaf_dx.p, ctx->dx_max, (const int4 *)ctx->block_box.p, nullptr,
        (int32_t *)off.p, (PairEntry *)lst.p, (uint8_t *)axl.p, host_axes(), (const int32_t *)ctx->leaf_count.p,
        which == 0 ? (int32_t *)ctx->act_cost.p : nullptr, which == 0 ? (float *)ctx->act_reach.p : nullptr,
        lazy_ti, ctx->ti_now);
  }
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}

sph_status build_pairs(sph_ctx *ctx, int which, float slack) {
  const int64_t na = ctx->n_active_leaves;
  SPH_TRY(build_pairs_count(ctx, which, slack, nullptr));
  if (na == 0) return build_pairs_fill(ctx, which, slack, 0);
  // the total (offsets[na]) written into its page-locked slot by one thread
  const DevBuf &off = which == 0 ? ctx->dpair_off : ctx->fpair_off;
  copy_total_kernel<<<1, 64, 0, ctx->stream>>>((const int32_t *)off.p + na, ctx->pin_dev + PIN_NPAIRS);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  SPH_TRY(pin_fetch(ctx, PIN_NPAIRS, 1));
  return build_pairs_fill(ctx, which, slack, ctx->pin_h[PIN_NPAIRS]);
}

// Refreshes the max H of every active leaf (all particles, and active ones)
// from the current smoothing lengths, and raises the running global max H on
// the device (the force pair search reads it there).  No synchronisation.
sph_status refresh_leaf_hmax(sph_ctx *ctx) {
  const int64_t na = ctx->n_active_leaves;
  if (na == 0) return SPH_OK;
  {
    PROF(ctx, "cell_pairs");
    leaf_hmax_refresh_kernel<<<waves_grid(na), MT, 0, ctx->stream>>>(refresh_args(ctx));
  }
  HIP_TRY(ctx, hipGetLastError());
  return SPH_OK;
}

// The refresh of several boxes (one stream) in one launch.  The host copy of
// the arguments lives in the lead context and is rewritten only by the next
// batched pass, which starts by draining the stream.
sph_status refresh_leaf_hmax_boxes(sph_ctx *lead, sph_ctx **cs, const int *boxes, int nbox) {
  lead->refresh_host.resize(sizeof(RefreshArgs) * (size_t)nbox);
  RefreshArgs *rs = reinterpret_cast<RefreshArgs *>(lead->refresh_host.data());
  int nr = 0;
  int64_t maxa = 0;
  for (int q = 0; q < nbox; ++q) {
    sph_ctx *c = cs[boxes[q]];
    if (c->n_active_leaves == 0) continue;
    rs[nr++] = refresh_args(c);
    maxa = std::max<int64_t>(maxa, c->n_active_leaves);
  }
  if (nr == 0) return SPH_OK;
  SPH_TRY(sph_ensure(lead, lead->refresh_args, sizeof(RefreshArgs) * (size_t)nr));
  {
    PROF(lead, "cell_pairs");
    HIP_TRY(lead, hipMemcpyAsync(lead->refresh_args.p, rs, sizeof(RefreshArgs) * (size_t)nr, hipMemcpyHostToDevice,
                                 lead->stream));
    leaf_hmax_refresh_multi_kernel<<<dim3(std::min<unsigned>(waves_grid(maxa), 1024u), (unsigned)nr), MT, 0,
                                     lead->stream>>>((const RefreshArgs *)lead->refresh_args.p);
  }
  return sph_hip_check(lead, hipGetLastError(), "leaf max H refresh");
}

sph_status mark_active_impl(sph_ctx *ctx, const sph_particles *p, int m, int64_t *n_active_host) {
  if (!p || !p->time_bin) return sph_fail(ctx, SPH_EINVAL, "mark_active: time_bin is required");
  if (m < 0 || m >= ctx->prm.n_bins) return sph_fail(ctx, SPH_EINVAL, "mark_active: bin %d outside [0, %d)", m, ctx->prm.n_bins);
  const int64_t n = ctx->n, nl = ctx->n_leaves;
  ctx->max_active_bin = m;
  SPH_TRY(sph_ensure(ctx, ctx->active, (size_t)n));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_nact, 4 * (size_t)(3 * nl + 3)));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_act_off, 4 * (size_t)(3 * nl + 3)));
  SPH_TRY(sph_ensure(ctx, ctx->leaf_actleaf, 4 * (size_t)nl));
  SPH_TRY(sph_ensure(ctx, ctx->act_leaf_chunk_off, 4 * (size_t)nl));
  int32_t *nact = (int32_t *)ctx->leaf_nact.p, *isact = nact + nl, *nchunk = nact + 2 * nl;
  int32_t *aoff = (int32_t *)ctx->leaf_act_off.p, *aidx = aoff + nl, *coff = aoff + 2 * nl;
  float *hmax_act_leaf = (float *)ctx->act_leaf_chunk_off.p;
  int32_t *sc = (int32_t *)ctx->scalars.p;
  {
    PROF(ctx, "mark");
    mark_count_kernel<<<waves_grid(ceil_div(nl, MARK_LEAVES)), MT, 0, ctx->stream>>>(p->time_bin, m, (const float4 *)ctx->pos4.p,
                                                              (const int32_t *)ctx->leaf_begin.p,
                                                              (const int32_t *)ctx->leaf_count.p, nl,
                                                              (uint8_t *)ctx->active.p, nact, isact, nchunk,
                                                              hmax_act_leaf);
  }
  HIP_TRY(ctx, hipGetLastError());
  // one scan over [nact | isact | nchunk]: the second and third segments come
  // out shifted by the totals before them, read back by the fill kernel
  SPH_TRY(scan_exclusive_i32(ctx, nact, aoff, 3 * nl, aoff + 3 * nl));
  // the three totals written into page-locked slots by one small kernel, one
  // synchronisation
  const int32_t *tot3 = ctx->pin_h + PIN_MARK;
  mark_totals_kernel<<<1, 64, 0, ctx->stream>>>(aoff, nl, ctx->pin_dev + PIN_MARK);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  SPH_TRY(pin_fetch(ctx, PIN_MARK, 3));
  int32_t tot[3] = {tot3[0], tot3[1] - tot3[0], tot3[2] - tot3[1]};
  ctx->n_active = tot[0];
  ctx->n_active_leaves = tot[1];
  ctx->n_chunks = tot[2];
  const int64_t nact_tot = tot[0] > 0 ? tot[0] : 1, nal = tot[1] > 0 ? tot[1] : 1, nch = tot[2] > 0 ? tot[2] : 1;
  SPH_TRY(sph_ensure(ctx, ctx->active_idx, 4 * (size_t)nact_tot));
  SPH_TRY(sph_ensure(ctx, ctx->chunk_of, 4 * (size_t)nact_tot));
  SPH_TRY(sph_ensure(ctx, ctx->act_leaves, 4 * (size_t)nal));
  SPH_TRY(sph_ensure(ctx, ctx->act_hmax, 4 * (size_t)nal));
  SPH_TRY(sph_ensure(ctx, ctx->chunks, sizeof(Chunk) * (size_t)nch));
  SPH_TRY(sph_ensure(ctx, ctx->chunk_todo, 4 * (size_t)nch));
  {
    PROF(ctx, "mark");
    mark_fill_kernel<<<waves_grid(nl), MT, 0, ctx->stream>>>(
        (const uint8_t *)ctx->active.p, (const int32_t *)ctx->leaf_begin.p, (const int32_t *)ctx->leaf_count.p, nl,
        nact, aoff, aidx, coff, hmax_act_leaf, (int32_t *)ctx->active_idx.p, (int32_t *)ctx->chunk_of.p,
        (int32_t *)ctx->act_leaves.p, (float *)ctx->act_hmax.p, (int32_t *)ctx->leaf_actleaf.p,
        (Chunk *)ctx->chunks.p);
  }
  HIP_TRY(ctx, hipGetLastError());
  // new chunks: the loop work items are rebuilt at the next launch (they keep
  // the costs of these lists through the pass, also if the lists are widened)
  ctx->work_valid = 0;
  if (ctx->prm.lazy_drift && ctx->n_active_leaves > 0) {
    // the active leaves reach the current time before their max H is taken
    SPH_TRY(drift_leaves(ctx, p, (const int32_t *)ctx->act_leaves.p, nullptr, ctx->n_active_leaves));
    SPH_TRY(refresh_leaf_hmax(ctx));
  }
  SPH_TRY(build_pairs(ctx, 0, ctx->prm.pair_slack));
  SPH_TRY(drift_partners(ctx, p, 0));
  if (n_active_host) *n_active_host = ctx->n_active;
  ctx->state = 3;
  return SPH_OK;
}
