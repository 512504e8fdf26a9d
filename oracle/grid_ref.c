/*
 * FP64 C oracle for convolutional gridding -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no code, header or table with the GPU path.
 *
 * It computes the plain definition of gridding (Merry 2016, Section 2.2):
 * every visibility, pre-weighted (Section 4), is multiplied by the separable
 * oversampled kernel taps (Section 4: G_ij = G^u_i G^v_j, the same for all
 * polarisations) and added to the S x S cells of its footprint.  The index
 * conversion is the same reading as oracle/gridding.py:
 *   fx = rint(u * (inv_cell_u * O)) + (W/2) O   (round half to even)
 *   ix = fx >> log2 O,  sx = fx & (O - 1),  x0 = ix - S/2 + 1
 *   plane = rint((w - w_min) * inv_dw)  (single-plane kernels ignore w)
 *   drop if non-finite, plane out of range, or footprint off the grid.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math: the
 * index conversion must be a single correctly rounded multiply).
 *
 * Threads own disjoint stripes of output rows, so the full-grid result does
 * not depend on the thread count.  Sampled-row mode splits the visibilities
 * into a fixed number of blocks and reduces them in block order, which is
 * also independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
  int32_t x0, y0, sx, sy, plane, valid;
} coords_t;

static int ilog2(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }

static void pixel_coords_one(const double* uvw, double inv_cell_u, double inv_cell_v, int O,
                             int S, int H, int W, int n_planes, double w_min, double inv_dw,
                             coords_t* c) {
  const double big = 1099511627776.0; /* 2^40 */
  double u = uvw[0], v = uvw[1], w = uvw[2];
  c->valid = 0; c->x0 = c->y0 = c->sx = c->sy = c->plane = 0;
  if (!isfinite(u) || !isfinite(v) || !isfinite(w)) return;
  double xh = u * (inv_cell_u * (double)O);
  double yh = v * (inv_cell_v * (double)O);
  if (!(fabs(xh) < big) || !(fabs(yh) < big)) return;
  int lg = ilog2(O);
  int64_t fx = (int64_t)rint(xh) + (int64_t)(W / 2) * O;
  int64_t fy = (int64_t)rint(yh) + (int64_t)(H / 2) * O;
  int64_t ix = fx >> lg, iy = fy >> lg;   /* arithmetic shift = floor */
  int64_t x0 = ix - S / 2 + 1, y0 = iy - S / 2 + 1;
  int64_t plane = 0;
  if (n_planes > 1) {
    double ph = (w - w_min) * inv_dw;
    if (!(fabs(ph) < big)) return;
    plane = (int64_t)rint(ph);
  }
  if (plane < 0 || plane >= n_planes) return;
  if (x0 < 0 || x0 + S > W || y0 < 0 || y0 + S > H) return;
  c->x0 = (int32_t)x0; c->y0 = (int32_t)y0;
  c->sx = (int32_t)(fx & (O - 1)); c->sy = (int32_t)(fy & (O - 1));
  c->plane = (int32_t)plane; c->valid = 1;
}

void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Per-visibility coordinates; out arrays may be NULL.  Returns the drop count. */
int64_t oracle_pixel_coords(int64_t n, const double* uvw, double inv_cell_u, double inv_cell_v,
                            int O, int S, int H, int W, int n_planes, double w_min,
                            double inv_dw, int32_t* x0, int32_t* y0, int32_t* sx, int32_t* sy,
                            int32_t* plane, uint8_t* valid) {
  int64_t dropped = 0;
#pragma omp parallel for schedule(static) reduction(+ : dropped)
  for (int64_t i = 0; i < n; ++i) {
    coords_t c;
    pixel_coords_one(uvw + 3 * i, inv_cell_u, inv_cell_v, O, S, H, W, n_planes, w_min, inv_dw, &c);
    if (x0) x0[i] = c.x0;
    if (y0) y0[i] = c.y0;
    if (sx) sx[i] = c.sx;
    if (sy) sy[i] = c.sy;
    if (plane) plane[i] = c.plane;
    if (valid) valid[i] = (uint8_t)c.valid;
    dropped += !c.valid;
  }
  return dropped;
}

/*
 * Grid visibilities with a separable kernel.
 *   vis      float  [n][P][2]   (complex64)
 *   weights  float  [n][P]      or NULL (= 1)
 *   taps     double [planes][O][S][2]  (complex; the same table on both axes)
 *   rows     int32  [n_rows]    absolute grid rows to compute, or NULL for all H rows
 *   out      double [P][n_rows or H][W][2], accumulated into (+=)
 * Returns the number of dropped visibilities.
 */
int64_t oracle_grid_sep(int64_t n, int P, const float* vis, const float* weights,
                        const double* uvw, const double* taps, int n_planes, int O, int S,
                        double inv_cell_u, double inv_cell_v, double w_min, double inv_dw,
                        int H, int W, const int32_t* rows, int n_rows, double* out) {
  coords_t* cs = (coords_t*)malloc(sizeof(coords_t) * (size_t)(n > 0 ? n : 1));
  if (!cs) return -1;
  int64_t dropped = 0;
#pragma omp parallel for schedule(static) reduction(+ : dropped)
  for (int64_t i = 0; i < n; ++i) {
    pixel_coords_one(uvw + 3 * i, inv_cell_u, inv_cell_v, O, S, H, W, n_planes, w_min, inv_dw, cs + i);
    /* a visibility with a non-finite value or weight is dropped too */
    for (int p = 0; p < P && cs[i].valid; ++p) {
      if (!isfinite(vis[(i * P + p) * 2]) || !isfinite(vis[(i * P + p) * 2 + 1])) cs[i].valid = 0;
      if (weights && !isfinite(weights[i * P + p])) cs[i].valid = 0;
    }
    dropped += !cs[i].valid;
  }
  if (rows == NULL) {
    /* full grid: each thread owns a stripe of rows and scans every visibility */
    int nt = omp_get_max_threads();
#pragma omp parallel num_threads(nt)
    {
      int t = omp_get_thread_num(), T = omp_get_num_threads();
      int r0 = (int)((int64_t)H * t / T), r1 = (int)((int64_t)H * (t + 1) / T);
      for (int64_t i = 0; i < n; ++i) {
        const coords_t* c = cs + i;
        if (!c->valid || c->y0 >= r1 || c->y0 + S <= r0) continue;
        int ky0 = r0 > c->y0 ? r0 - c->y0 : 0;
        int ky1 = r1 < c->y0 + S ? r1 - c->y0 : S;
        const double* tu = taps + (((size_t)c->plane * O + c->sx) * S) * 2;
        const double* tv = taps + (((size_t)c->plane * O + c->sy) * S) * 2;
        for (int p = 0; p < P; ++p) {
          double wt = weights ? (double)weights[i * P + p] : 1.0;
          double vr = (double)vis[(i * P + p) * 2] * wt, vi = (double)vis[(i * P + p) * 2 + 1] * wt;
          for (int ky = ky0; ky < ky1; ++ky) {
            /* g = Tv[ky] * Tu[kx];  contribution = g * V */
            double tvr = tv[2 * ky], tvi = tv[2 * ky + 1];
            double* orow = out + (((size_t)p * H + (c->y0 + ky)) * W + c->x0) * 2;
            for (int kx = 0; kx < S; ++kx) {
              double tur = tu[2 * kx], tui = tu[2 * kx + 1];
              double gr = tvr * tur - tvi * tui, gi = tvr * tui + tvi * tur;
              orow[2 * kx] += gr * vr - gi * vi;
              orow[2 * kx + 1] += gr * vi + gi * vr;
            }
          }
        }
      }
    }
  } else {
    /* sampled rows: fixed visibility blocks with private partial rows, reduced in order */
    int32_t* lut = (int32_t*)malloc(sizeof(int32_t) * (size_t)H);
    if (!lut) { free(cs); return -1; }
    for (int r = 0; r < H; ++r) lut[r] = -1;
    for (int j = 0; j < n_rows; ++j) if (rows[j] >= 0 && rows[j] < H) lut[rows[j]] = j;
    const int NB = 64;
    size_t plane_sz = (size_t)P * n_rows * W * 2;
    double* part = (double*)calloc((size_t)NB * plane_sz, sizeof(double));
    if (!part) { free(lut); free(cs); return -1; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < NB; ++b) {
      double* acc = part + (size_t)b * plane_sz;
      int64_t i0 = n * b / NB, i1 = n * (b + 1) / NB;
      for (int64_t i = i0; i < i1; ++i) {
        const coords_t* c = cs + i;
        if (!c->valid) continue;
        const double* tu = taps + (((size_t)c->plane * O + c->sx) * S) * 2;
        const double* tv = taps + (((size_t)c->plane * O + c->sy) * S) * 2;
        for (int ky = 0; ky < S; ++ky) {
          int j = lut[c->y0 + ky];
          if (j < 0) continue;
          double tvr = tv[2 * ky], tvi = tv[2 * ky + 1];
          for (int p = 0; p < P; ++p) {
            double wt = weights ? (double)weights[i * P + p] : 1.0;
            double vr = (double)vis[(i * P + p) * 2] * wt, vi = (double)vis[(i * P + p) * 2 + 1] * wt;
            double* orow = acc + (((size_t)p * n_rows + j) * W + c->x0) * 2;
            for (int kx = 0; kx < S; ++kx) {
              double tur = tu[2 * kx], tui = tu[2 * kx + 1];
              double gr = tvr * tur - tvi * tui, gi = tvr * tui + tvi * tur;
              orow[2 * kx] += gr * vr - gi * vi;
              orow[2 * kx + 1] += gr * vi + gi * vr;
            }
          }
        }
      }
    }
    for (int b = 0; b < NB; ++b) {
      const double* src = part + (size_t)b * plane_sz;
#pragma omp parallel for schedule(static)
      for (size_t q = 0; q < plane_sz; ++q) out[q] += src[q];
    }
    free(part);
    free(lut);
  }
  free(cs);
  return dropped;
}
