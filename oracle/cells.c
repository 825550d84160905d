/* Bit-exact CPU definitions of the cell build, per-cell axis sorts, active
 * masks, cell-pair lists and FP32 neighbour counts -- TEST INFRASTRUCTURE ONLY
 * (the product library never links or calls this file).
 *
 * Written as plain, slow, obviously-correct loops: a comparison sort, a
 * recursive octree split, all-pairs cell tests and all-pairs particle tests.
 * Compiled with -ffp-contract=off so that every float operation rounds where
 * it is written; fmaf() is the correctly rounded C99 fused multiply-add.
 *
 * Definitions (the paper fixes the ideas, these fix the bits):
 *  - Adaptive cells (Sec. III-A): a fixed top-level grid of 2^k0 cells per
 *    side, refined by octree splits while a cell holds at least `split`
 *    particles (the paper uses 400), down to depth D.  The top level k0 is the
 *    largest with L 2^-k0 >= max H (and >= 2, i.e. at least 4 cells per side),
 *    capped at top_cap.  H = fl32(1.825742f * h).
 *  - Morton keys on D-bit integer coordinates k = min(trunc(xw * 2^D / L), 2^D-1)
 *    of the wrapped position xw; bit b of kx/ky/kz goes to key bit 3b+2/3b+1/3b.
 *    Particles are ordered by (key, original index).
 *  - Positions inside a leaf are FP32 offsets from the leaf centre:
 *    o = (float)(xw - c), c = (2 i + 1) 2^(D-level) * L / 2^(D+1).
 *  - Cell pairs (Sec. III-A, "all pairs of cells with at least one member on
 *    the list", interacting on the scale where the geometry allows it): an
 *    active leaf A is paired with every leaf B (A itself included) whose
 *    periodic box distance is below R, with R = max H over A's active
 *    particles (density loop) or max(that, max H over B) (force loop).  The
 *    pair shift is s = (float)(nearest-image centre difference).
 *  - FP32 neighbour predicate: dx = o_i - (o_j + s_AB) per axis in float,
 *    r2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx)); density: r2 < H_i*H_i; force:
 *    r2 < H_i*H_i or r2 < H_j*H_j.
 *  - Axis sorts (Fig. 5 "sort" task): for the 13 directions e of the half
 *    neighbour stencil (lexicographic (dx,dy,dz) with first non-zero > 0,
 *    normalised in double then rounded to float), key
 *    d = fmaf(o_z, e_z, fmaf(o_y, e_y, o_x * e_x)), ascending, ties by
 *    in-leaf index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GK32 1.825742f

static const int AXES[13][3] = {
    {0, 0, 1},  {0, 1, -1}, {0, 1, 0},  {0, 1, 1},  {1, -1, -1}, {1, -1, 0}, {1, -1, 1},
    {1, 0, -1}, {1, 0, 0},  {1, 0, 1},  {1, 1, -1}, {1, 1, 0},   {1, 1, 1}};

static uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}
static int64_t compact3(uint64_t v) {
  int64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= (int64_t)((v >> (3 * b)) & 1ull) << b;
  return r;
}

double emu_wrap(double x, double L) {
  double q = floor(x / L);
  double xw = x - q * L;
  if (xw < 0.0) xw += L;
  if (xw >= L) xw -= L;
  return xw;
}

/* ---------------- cell build ---------------- */

static const uint64_t *g_keys;
static int cmp_key_idx(const void *a, const void *b) {
  int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
  if (g_keys[ia] < g_keys[ib]) return -1;
  if (g_keys[ia] > g_keys[ib]) return 1;
  return (ia < ib) ? -1 : (ia > ib);
}

typedef struct {
  const uint64_t *key;
  int D, split;
  int32_t *lv;
  int64_t *lbegin;
  int32_t *lcount;
  int64_t n_leaves;
} build_state;

static void split_node(build_state *s, int level, int64_t begin, int64_t end) {
  int64_t cnt = end - begin;
  if (cnt <= 0) return;
  if (cnt < s->split || level >= s->D) {
    s->lv[s->n_leaves] = level;
    s->lbegin[s->n_leaves] = begin;
    s->lcount[s->n_leaves] = (int32_t)cnt;
    s->n_leaves++;
    return;
  }
  int shift = 3 * (s->D - level - 1);
  int64_t p = begin;
  for (int c = 0; c < 8; ++c) {
    int64_t q = p;
    while (q < end && (int)((s->key[q] >> shift) & 7ull) == c) ++q;
    split_node(s, level + 1, p, q);
    p = q;
  }
}

/* Returns 0 on success, -1 if max H exceeds L/4. */
int emu_build_cells(int64_t n, const double *x, const double *y, const double *z, const float *h,
                    double L, int split, int D, int top_cap,
                    /* outputs, sorted order */
                    int64_t *perm, uint64_t *key_sorted, double *xw_s, double *yw_s, double *zw_s,
                    float *ox, float *oy, float *oz, float *H_s, int64_t *leaf_of,
                    /* leaf table (capacity n) */
                    int32_t *leaf_level, int64_t *leaf_ix, int64_t *leaf_iy, int64_t *leaf_iz,
                    int64_t *leaf_begin, int32_t *leaf_count, float *leaf_hmax,
                    int32_t *top_level_out, int64_t *n_leaves_out) {
  float Hmax = 0.0f;
  for (int64_t i = 0; i < n; ++i) {
    float H = GK32 * h[i];
    if (H > Hmax) Hmax = H;
  }
  if (L * 0.25 < (double)Hmax) return -1;
  int k0 = 2;
  while (k0 < top_cap && k0 < D && ldexp(L, -(k0 + 1)) >= (double)Hmax) ++k0;
  *top_level_out = k0;

  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  double scale = ldexp(1.0, D) / L;
  int64_t kmax = ((int64_t)1 << D) - 1;
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {emu_wrap(x[i], L), emu_wrap(y[i], L), emu_wrap(z[i], L)};
    int64_t k[3];
    for (int a = 0; a < 3; ++a) {
      xw[3 * i + a] = p[a];
      int64_t kk = (int64_t)(p[a] * scale);
      if (kk > kmax) kk = kmax;
      if (kk < 0) kk = 0;
      k[a] = kk;
    }
    key[i] = (spread3((uint64_t)k[0]) << 2) | (spread3((uint64_t)k[1]) << 1) | spread3((uint64_t)k[2]);
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  g_keys = key;
  qsort(perm, (size_t)n, sizeof(int64_t), cmp_key_idx);
  for (int64_t s = 0; s < n; ++s) {
    int64_t i = perm[s];
    key_sorted[s] = key[i];
    xw_s[s] = xw[3 * i];
    yw_s[s] = xw[3 * i + 1];
    zw_s[s] = xw[3 * i + 2];
    H_s[s] = GK32 * h[i];
  }
  build_state st = {key_sorted, D, split, leaf_level, leaf_begin, leaf_count, 0};
  int top_shift = 3 * (D - k0);
  int64_t p = 0;
  while (p < n) {
    int64_t q = p;
    while (q < n && (key_sorted[q] >> top_shift) == (key_sorted[p] >> top_shift)) ++q;
    split_node(&st, k0, p, q);
    p = q;
  }
  *n_leaves_out = st.n_leaves;
  double unit = ldexp(L, -(D + 1));
  for (int64_t l = 0; l < st.n_leaves; ++l) {
    int lvl = leaf_level[l];
    uint64_t pre = key_sorted[leaf_begin[l]] >> (3 * (D - lvl));
    leaf_ix[l] = compact3(pre >> 2);
    leaf_iy[l] = compact3(pre >> 1);
    leaf_iz[l] = compact3(pre);
    double c[3];
    int64_t ii[3] = {leaf_ix[l], leaf_iy[l], leaf_iz[l]};
    for (int a = 0; a < 3; ++a) c[a] = (double)((2 * ii[a] + 1) << (D - lvl)) * unit;
    float hm = 0.0f;
    for (int64_t s = leaf_begin[l]; s < leaf_begin[l] + leaf_count[l]; ++s) {
      ox[s] = (float)(xw_s[s] - c[0]);
      oy[s] = (float)(yw_s[s] - c[1]);
      oz[s] = (float)(zw_s[s] - c[2]);
      if (H_s[s] > hm) hm = H_s[s];
      leaf_of[s] = l;
    }
    leaf_hmax[l] = hm;
  }
  free(key);
  free(xw);
  return 0;
}

/* ---------------- axis sorts ---------------- */

static const float *g_sortkey;
static int cmp_axis(const void *a, const void *b) {
  uint16_t ia = *(const uint16_t *)a, ib = *(const uint16_t *)b;
  float ka = g_sortkey[ia], kb = g_sortkey[ib];
  if (ka < kb) return -1;
  if (kb < ka) return 1;
  return (ia < ib) ? -1 : (ia > ib);
}

void emu_axis_vectors(float *e /* 13*3 */) {
  for (int a = 0; a < 13; ++a) {
    double nrm = sqrt((double)(AXES[a][0] * AXES[a][0] + AXES[a][1] * AXES[a][1] + AXES[a][2] * AXES[a][2]));
    for (int d = 0; d < 3; ++d) e[3 * a + d] = (float)((double)AXES[a][d] / nrm);
  }
}

/* order[a*n + begin + k] = in-leaf index of the k-th smallest key along axis a;
 * keys[a*n + s] = key of particle s along axis a. */
int emu_axis_sort(int64_t n, int64_t n_leaves, const int64_t *leaf_begin, const int32_t *leaf_count,
                  const float *ox, const float *oy, const float *oz, uint16_t *order, float *keys) {
  float e[39];
  emu_axis_vectors(e);
  for (int a = 0; a < 13; ++a) {
    for (int64_t s = 0; s < n; ++s)
      keys[a * n + s] = fmaf(oz[s], e[3 * a + 2], fmaf(oy[s], e[3 * a + 1], ox[s] * e[3 * a]));
  }
  for (int64_t l = 0; l < n_leaves; ++l) {
    if (leaf_count[l] > 65535) return -1;
    for (int a = 0; a < 13; ++a) {
      uint16_t *o = order + a * n + leaf_begin[l];
      for (int k = 0; k < leaf_count[l]; ++k) o[k] = (uint16_t)k;
      g_sortkey = keys + a * n + leaf_begin[l];
      qsort(o, (size_t)leaf_count[l], sizeof(uint16_t), cmp_axis);
    }
  }
  return 0;
}

/* ---------------- active set and cell pairs ---------------- */

static void nearest_image(int64_t nu, const int64_t *ca, const int64_t *cb, int64_t *dl) {
  for (int a = 0; a < 3; ++a) {
    int64_t d = cb[a] - ca[a];
    if (d > nu / 2) d -= nu;
    if (d < -nu / 2) d += nu;
    dl[a] = d;
  }
}

static void leaf_centre_units(int D, int lvl, int64_t ix, int64_t iy, int64_t iz, int64_t *c) {
  c[0] = (2 * ix + 1) << (D - lvl);
  c[1] = (2 * iy + 1) << (D - lvl);
  c[2] = (2 * iz + 1) << (D - lvl);
}

/* active[s] = bin[s] <= m (sorted order); returns the number of active leaves
 * written to active_leaves (ascending) with hmax_act[k] for each. */
int64_t emu_mark_active(int64_t n, const int8_t *bin, int m, int64_t n_leaves, const int64_t *leaf_begin,
                        const int32_t *leaf_count, const float *H_s, uint8_t *active,
                        int64_t *active_leaves, float *hmax_act) {
  int64_t na = 0;
  for (int64_t s = 0; s < n; ++s) active[s] = (uint8_t)(bin[s] <= m);
  for (int64_t l = 0; l < n_leaves; ++l) {
    float hm = 0.0f;
    int any = 0;
    for (int64_t s = leaf_begin[l]; s < leaf_begin[l] + leaf_count[l]; ++s)
      if (active[s]) {
        any = 1;
        if (H_s[s] > hm) hm = H_s[s];
      }
    if (any) {
      active_leaves[na] = l;
      hmax_act[na] = hm;
      ++na;
    }
  }
  return na;
}

/* All-pairs cell test.  mode 0: density (R = hmax_act[A]); mode 1: force
 * (R = max(hmax_act[A], leaf_hmax[B])); with leaf_dx (non-NULL) the test
 * radius is R + leaf_dx[A] + leaf_dx[B] in float, in that order.  Writes up to cap pairs
 * (A, B, sx, sy, sz) in (A, B) order; returns the number of pairs (which may
 * exceed cap, in which case only cap were written). */
int64_t emu_pairs(int mode, double L, int D, int64_t n_active_leaves, const int64_t *active_leaves,
                  const float *hmax_act, int64_t n_leaves, const int32_t *leaf_level, const int64_t *leaf_ix,
                  const int64_t *leaf_iy, const int64_t *leaf_iz, const float *leaf_hmax, const float *leaf_dx,
                  int64_t cap, int64_t *pa, int64_t *pb, float *sx, float *sy, float *sz) {
  int64_t nu = (int64_t)1 << (D + 1);
  double unit = ldexp(L, -(D + 1));
  int64_t np = 0;
  for (int64_t k = 0; k < n_active_leaves; ++k) {
    int64_t A = active_leaves[k];
    int64_t ca[3];
    leaf_centre_units(D, leaf_level[A], leaf_ix[A], leaf_iy[A], leaf_iz[A], ca);
    int64_t hwa = (int64_t)1 << (D - leaf_level[A]);
    for (int64_t B = 0; B < n_leaves; ++B) {
      int64_t cb[3], dl[3];
      leaf_centre_units(D, leaf_level[B], leaf_ix[B], leaf_iy[B], leaf_iz[B], cb);
      nearest_image(nu, ca, cb, dl);
      int64_t hwb = (int64_t)1 << (D - leaf_level[B]);
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        int64_t g = llabs(dl[a]) - hwa - hwb;
        if (g < 0) g = 0;
        double gd = (double)g * unit;
        d2 = d2 + gd * gd;
      }
      float R = hmax_act[k];
      if (mode == 1 && leaf_hmax[B] > R) R = leaf_hmax[B];
      /* drift margins of both leaves (cells kept from an earlier build) */
      if (leaf_dx) R = (R + leaf_dx[A]) + leaf_dx[B];
      double Rd = (double)R;
      if (d2 < Rd * Rd) {
        if (np < cap) {
          pa[np] = A;
          pb[np] = B;
          sx[np] = (float)((double)dl[0] * unit);
          sy[np] = (float)((double)dl[1] * unit);
          sz[np] = (float)((double)dl[2] * unit);
        }
        ++np;
      }
    }
  }
  return np;
}

/* ---------------- FP32 neighbour counts (all pairs) ---------------- */

/* For each sampled particle i (sorted index): the number of j != i over all
 * particles satisfying the FP32 predicate.  mode 0 density, 1 force. */
void emu_counts(int mode, double L, int D, int64_t n, const float *ox, const float *oy, const float *oz,
                const float *H_s, const int64_t *leaf_of, const int32_t *leaf_level, const int64_t *leaf_ix,
                const int64_t *leaf_iy, const int64_t *leaf_iz, int64_t n_samples, const int64_t *samples,
                int64_t *counts) {
  int64_t nu = (int64_t)1 << (D + 1);
  double unit = ldexp(L, -(D + 1));
  for (int64_t t = 0; t < n_samples; ++t) {
    int64_t i = samples[t];
    int64_t A = leaf_of[i];
    int64_t ca[3];
    leaf_centre_units(D, leaf_level[A], leaf_ix[A], leaf_iy[A], leaf_iz[A], ca);
    float Hi = H_s[i];
    float Hi2 = Hi * Hi;
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      int64_t B = leaf_of[j];
      int64_t cb[3], dl[3];
      leaf_centre_units(D, leaf_level[B], leaf_ix[B], leaf_iy[B], leaf_iz[B], cb);
      nearest_image(nu, ca, cb, dl);
      float s0 = (float)((double)dl[0] * unit);
      float s1 = (float)((double)dl[1] * unit);
      float s2 = (float)((double)dl[2] * unit);
      float jx = ox[j] + s0, jy = oy[j] + s1, jz = oz[j] + s2;
      float dx = ox[i] - jx, dy = oy[i] - jy, dz = oz[i] - jz;
      float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      int in = r2 < Hi2;
      if (mode == 1 && !in) {
        float Hj = H_s[j];
        in = r2 < Hj * Hj;
      }
      c += in;
    }
    counts[t] = c;
  }
}

/* ---------------- cells kept from an earlier build ---------------- */

/* Offsets of the (wrapped) positions from the centres of the given leaves by
 * the minimum image, H = fl32(1.825742 h), each leaf's max H and a bound on
 * the displacement of its particles from the positions xb of the build:
 * sqrt(3) times the largest displacement component (in double), rounded to
 * float, then the next float up.  Returns 1 when some leaf's bound exceeds
 * frac times its width. */
int emu_update(int64_t n, double *x, double *y, double *z, const float *h, const double *xb, const double *yb,
               const double *zb, double L, int D, int64_t n_leaves, const int64_t *leaf_begin,
               const int32_t *leaf_count, const int32_t *leaf_level, const int64_t *leaf_ix, const int64_t *leaf_iy,
               const int64_t *leaf_iz, float frac, float *ox, float *oy, float *oz, float *H, float *leaf_hmax,
               float *leaf_dx) {
  double unit = ldexp(L, -(D + 1));
  double half = 0.5 * L;
  int flag = 0;
  (void)n;
  for (int64_t l = 0; l < n_leaves; ++l) {
    int64_t c[3];
    leaf_centre_units(D, leaf_level[l], leaf_ix[l], leaf_iy[l], leaf_iz[l], c);
    double cx = (double)c[0] * unit, cy = (double)c[1] * unit, cz = (double)c[2] * unit;
    float hm = 0.0f;
    double d2m = 0.0;
    for (int64_t s = leaf_begin[l]; s < leaf_begin[l] + leaf_count[l]; ++s) {
      double p[3] = {emu_wrap(x[s], L), emu_wrap(y[s], L), emu_wrap(z[s], L)};
      x[s] = p[0];
      y[s] = p[1];
      z[s] = p[2];
      double o[3] = {p[0] - cx, p[1] - cy, p[2] - cz};
      double d[3] = {p[0] - xb[s], p[1] - yb[s], p[2] - zb[s]};
      for (int a = 0; a < 3; ++a) {
        if (o[a] > half) o[a] -= L; else if (o[a] < -half) o[a] += L;
        if (d[a] > half) d[a] -= L; else if (d[a] < -half) d[a] += L;
      }
      for (int a = 0; a < 3; ++a)
        if (fabs(d[a]) > d2m) d2m = fabs(d[a]);
      ox[s] = (float)o[0];
      oy[s] = (float)o[1];
      oz[s] = (float)o[2];
      H[s] = 1.825742f * h[s];
      if (H[s] > hm) hm = H[s];
    }
    leaf_hmax[l] = hm;
    leaf_dx[l] = d2m > 0.0 ? nextafterf((float)(d2m * 1.7320508075688772), INFINITY) : 0.0f;
    if ((double)leaf_dx[l] > (double)frac * ldexp(L, -leaf_level[l])) flag = 1;
  }
  return flag;
}

/* ---------------- neighbour counts through a grid ----------------
 *
 * The counts of emu_counts, with each sample's candidates j taken from a
 * uniform grid over the wrapped FP64 positions (x, y, z; sorted order): only
 * particles within R_i = 1.001 max(H_i, Hcut) + 1e-6 L of the sample
 * (minimum image, FP64) are tested with the FP32 predicate, Hcut = 0 for the
 * density loop and the largest H for the force loop.  The FP32 offsets and
 * shifts differ from the exact separation by well under 1e-6 L, so every
 * pair the predicate accepts lies within R_i and the counts are those of
 * emu_counts (a test compares the two on the same inputs). */
int emu_counts_grid(int mode, double L, int D, int64_t n, const double *x, const double *y, const double *z,
                    const float *ox, const float *oy, const float *oz, const float *H_s, const int64_t *leaf_of,
                    const int32_t *leaf_level, const int64_t *leaf_ix, const int64_t *leaf_iy,
                    const int64_t *leaf_iz, int64_t n_samples, const int64_t *samples, int64_t *counts) {
  int64_t nu = (int64_t)1 << (D + 1);
  double unit = ldexp(L, -(D + 1));
  float Hcut = 0.0f;
  if (mode == 1)
    for (int64_t j = 0; j < n; ++j)
      if (H_s[j] > Hcut) Hcut = H_s[j];
  double rmax = 0.0;
  for (int64_t t = 0; t < n_samples; ++t) {
    double Hi = (double)H_s[samples[t]];
    double R = 1.001 * (Hi > (double)Hcut ? Hi : (double)Hcut) + 1e-6 * L;
    if (R > rmax) rmax = R;
  }
  int64_t ng = rmax > 0.0 ? (int64_t)floor(L / rmax) : 1;
  if (ng < 1) ng = 1;
  if (ng > 256) ng = 256;
  double cell = L / (double)ng;
  int64_t ncell = ng * ng * ng;
  int64_t *head = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t *item = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *cof = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!head || !item || !cof) {
    free(head);
    free(item);
    free(cof);
    return -1;
  }
  for (int64_t j = 0; j < n; ++j) {
    int64_t c[3];
    const double p[3] = {x[j], y[j], z[j]};
    for (int a = 0; a < 3; ++a) {
      int64_t k = (int64_t)floor(p[a] / cell);
      if (k < 0) k = 0;
      if (k >= ng) k = ng - 1;
      c[a] = k;
    }
    cof[j] = (c[0] * ng + c[1]) * ng + c[2];
    head[cof[j] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
  {
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    if (!fill) {
      free(head);
      free(item);
      free(cof);
      return -1;
    }
    memcpy(fill, head, (size_t)ncell * sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) item[fill[cof[j]]++] = j;
    free(fill);
  }
  const double half = 0.5 * L;
  for (int64_t t = 0; t < n_samples; ++t) {
    int64_t i = samples[t];
    int64_t A = leaf_of[i];
    int64_t ca[3];
    leaf_centre_units(D, leaf_level[A], leaf_ix[A], leaf_iy[A], leaf_iz[A], ca);
    float Hi = H_s[i];
    float Hi2 = Hi * Hi;
    double Hd = (double)Hi > (double)Hcut ? (double)Hi : (double)Hcut;
    double R = 1.001 * Hd + 1e-6 * L;
    const double pi[3] = {x[i], y[i], z[i]};
    int64_t lo[3], span[3];
    for (int a = 0; a < 3; ++a) {
      int64_t k = (int64_t)floor(pi[a] / cell);
      if (k < 0) k = 0;
      if (k >= ng) k = ng - 1;
      int64_t r = (int64_t)ceil(R / cell);
      if (2 * r + 1 >= ng) {
        lo[a] = 0;
        span[a] = ng;
      } else {
        lo[a] = k - r;
        span[a] = 2 * r + 1;
      }
    }
    int64_t cnt = 0;
    for (int64_t u = 0; u < span[0]; ++u)
      for (int64_t v = 0; v < span[1]; ++v)
        for (int64_t w = 0; w < span[2]; ++w) {
          int64_t gx = ((lo[0] + u) % ng + ng) % ng, gy = ((lo[1] + v) % ng + ng) % ng,
                  gz = ((lo[2] + w) % ng + ng) % ng;
          int64_t c = (gx * ng + gy) * ng + gz;
          for (int64_t q = head[c]; q < head[c + 1]; ++q) {
            int64_t j = item[q];
            if (j == i) continue;
            double d2 = 0.0;
            const double pj[3] = {x[j], y[j], z[j]};
            for (int a = 0; a < 3; ++a) {
              double d = pj[a] - pi[a];
              if (d > half) d -= L;
              if (d < -half) d += L;
              d2 += d * d;
            }
            if (d2 >= R * R) continue;
            int64_t B = leaf_of[j];
            int64_t cb[3], dl[3];
            leaf_centre_units(D, leaf_level[B], leaf_ix[B], leaf_iy[B], leaf_iz[B], cb);
            nearest_image(nu, ca, cb, dl);
            float s0 = (float)((double)dl[0] * unit);
            float s1 = (float)((double)dl[1] * unit);
            float s2 = (float)((double)dl[2] * unit);
            float jx = ox[j] + s0, jy = oy[j] + s1, jz = oz[j] + s2;
            float dx = ox[i] - jx, dy = oy[i] - jy, dz = oz[i] - jz;
            float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            int in = r2 < Hi2;
            if (mode == 1 && !in) {
              float Hj = H_s[j];
              in = r2 < Hj * Hj;
            }
            cnt += in;
          }
        }
    counts[t] = cnt;
  }
  free(head);
  free(item);
  free(cof);
  return 0;
}
