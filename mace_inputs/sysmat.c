/*
 * Seeded synthetic inputs for 2-D parallel-beam CT: the precomputed sparse
 * system matrix A (compressed sparse columns) and a forward projector used
 * only to synthesise measurements.
 *
 * This file describes the scanner, not the reconstruction method: it holds no
 * step of the MAP / MACE / ICD arithmetic.  Both the FP64 oracle and the GPU
 * library receive the matrix it produces as an input.
 *
 * Geometry (the paper precomputes and stores A once per fixed scanner
 * geometry, Sec. I and Sec. II-A; A_k is the forward projector of view k in
 * the MAP cost, eq. (global_obj)):
 *   - image of nx x ny square pixels of side `pix` (mm), centred at the origin;
 *     pixel (i, j) (row i from the top, column j) has centre
 *       x = (j - (nx-1)/2) * pix,   y = ((ny-1)/2 - i) * pix
 *     and raster index s = i * nx + j;
 *   - view k in [0, n_views): angle theta_k = k * pi / n_views (endpoint
 *     excluded);
 *   - channel d in [0, n_ch): the line  x cos(theta) + y sin(theta) = t_d,
 *     t_d = (d - (n_ch-1)/2) * chan (mm);
 *   - A[(k, d), s] = exact length (mm) of the intersection of that line with
 *     pixel s; row index r = k * n_ch + d.  Entries <= 1e-12 mm are dropped.
 *
 * The length of a line at signed offset u from a square's centre is the
 * projection of the square's indicator: a trapezoid in u with base
 * (|c|+|s|) * pix, flat top ||c|-|s|| * pix and height pix / max(|c|,|s|)
 * (the area under it is the pixel area pix^2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t nx, ny, n_views, n_ch;
  double pix, chan;
} mi_geom;

/* Length of the line at offset u (mm) from the centre of a pixel, view with
 * direction cosines (ca, sa). */
static double chord(double u, double ca, double sa, double pix) {
  double a = fabs(ca), b = fabs(sa);
  double hi = a > b ? a : b, lo = a > b ? b : a;
  double half_base = 0.5 * (a + b) * pix;
  double half_top = 0.5 * (hi - lo) * pix;
  double height = pix / hi;
  u = fabs(u);
  if (u >= half_base) return 0.0;
  if (u <= half_top) return height;
  return height * (half_base - u) / (half_base - half_top);
}

/* Channel range whose lines can cut the pixel with centre offset tc. */
static void channel_range(const mi_geom* g, double tc, double ca, double sa,
                          int32_t* d_lo, int32_t* d_hi) {
  double hb = 0.5 * (fabs(ca) + fabs(sa)) * g->pix;
  double c0 = 0.5 * (g->n_ch - 1);
  int32_t lo = (int32_t)ceil((tc - hb) / g->chan + c0) - 1;
  int32_t hi = (int32_t)floor((tc + hb) / g->chan + c0) + 1;
  if (lo < 0) lo = 0;
  if (hi > g->n_ch - 1) hi = g->n_ch - 1;
  *d_lo = lo;
  *d_hi = hi;
}

/* Walk the entries of column s in ascending row order; calls emit() for each
 * kept entry. Returns the entry count. */
typedef void (*emit_fn)(void* ctx, int32_t row, double len);

static int64_t walk_column(const mi_geom* g, const double* cosv,
                           const double* sinv, int64_t s, emit_fn emit,
                           void* ctx) {
  int64_t i = s / g->nx, j = s % g->nx;
  double x = ((double)j - 0.5 * (g->nx - 1)) * g->pix;
  double y = (0.5 * (g->ny - 1) - (double)i) * g->pix;
  double c0 = 0.5 * (g->n_ch - 1);
  int64_t cnt = 0;
  for (int32_t k = 0; k < g->n_views; ++k) {
    double ca = cosv[k], sa = sinv[k];
    double tc = x * ca + y * sa;
    int32_t lo, hi;
    channel_range(g, tc, ca, sa, &lo, &hi);
    for (int32_t d = lo; d <= hi; ++d) {
      double td = ((double)d - c0) * g->chan;
      double len = chord(td - tc, ca, sa, g->pix);
      if (len > 1e-12) {
        if (emit) emit(ctx, k * g->n_ch + d, len);
        ++cnt;
      }
    }
  }
  return cnt;
}

static void angles(const mi_geom* g, double* cosv, double* sinv) {
  for (int32_t k = 0; k < g->n_views; ++k) {
    double th = (double)k * M_PI / (double)g->n_views;
    cosv[k] = cos(th);
    sinv[k] = sin(th);
  }
}

/* Pass 1: col_ptr[0..n] (int64). Returns nnz, or -1 on bad arguments. */
int64_t mi_sysmat_colptr(const mi_geom* g, int64_t* col_ptr) {
  if (!g || g->nx <= 0 || g->ny <= 0 || g->n_views <= 0 || g->n_ch <= 0 ||
      !(g->pix > 0) || !(g->chan > 0))
    return -1;
  int64_t n = (int64_t)g->nx * g->ny;
  double* cosv = (double*)malloc(sizeof(double) * g->n_views);
  double* sinv = (double*)malloc(sizeof(double) * g->n_views);
  angles(g, cosv, sinv);
  col_ptr[0] = 0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t s = 0; s < n; ++s)
    col_ptr[s + 1] = walk_column(g, cosv, sinv, s, NULL, NULL);
  for (int64_t s = 0; s < n; ++s) col_ptr[s + 1] += col_ptr[s];
  free(cosv);
  free(sinv);
  return col_ptr[n];
}

typedef struct {
  int32_t* row;
  float* val;
  int64_t pos;
} fill_ctx;

static void fill_emit(void* vctx, int32_t row, double len) {
  fill_ctx* c = (fill_ctx*)vctx;
  c->row[c->pos] = row;
  c->val[c->pos] = (float)len;
  c->pos++;
}

/* Pass 2: rows (ascending within each column) and float32 lengths. */
int mi_sysmat_fill(const mi_geom* g, const int64_t* col_ptr, int32_t* row,
                   float* val) {
  int64_t n = (int64_t)g->nx * g->ny;
  double* cosv = (double*)malloc(sizeof(double) * g->n_views);
  double* sinv = (double*)malloc(sizeof(double) * g->n_views);
  angles(g, cosv, sinv);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t s = 0; s < n; ++s) {
    fill_ctx c = {row, val, col_ptr[s]};
    walk_column(g, cosv, sinv, s, fill_emit, &c);
  }
  free(cosv);
  free(sinv);
  return 0;
}

/* Forward projection out[r] = sum_s A[r,s] * x[s] (float64 accumulation of
 * the float32-rounded entries, so the synthetic data are consistent with the
 * stored A).  Parallel over views: each view owns its rows. */
int mi_forward_project(const mi_geom* g, const double* x, double* out) {
  int64_t n = (int64_t)g->nx * g->ny;
  int64_t m = (int64_t)g->n_views * g->n_ch;
  memset(out, 0, sizeof(double) * m);
  double c0 = 0.5 * (g->n_ch - 1);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t k = 0; k < g->n_views; ++k) {
    double th = (double)k * M_PI / (double)g->n_views;
    double ca = cos(th), sa = sin(th);
    double* o = out + (int64_t)k * g->n_ch;
    for (int64_t s = 0; s < n; ++s) {
      double xs = x[s];
      if (xs == 0.0) continue;
      int64_t i = s / g->nx, j = s % g->nx;
      double px = ((double)j - 0.5 * (g->nx - 1)) * g->pix;
      double py = (0.5 * (g->ny - 1) - (double)i) * g->pix;
      double tc = px * ca + py * sa;
      int32_t lo, hi;
      channel_range(g, tc, ca, sa, &lo, &hi);
      for (int32_t d = lo; d <= hi; ++d) {
        double len = chord(((double)d - c0) * g->chan - tc, ca, sa, g->pix);
        if (len > 1e-12) o[d] += (double)(float)len * xs;
      }
    }
  }
  return 0;
}

/* Exact chord length of row (k, d) through the whole image rectangle; used
 * only to check the matrix (its row sums must equal this). */
double mi_image_chord(const mi_geom* g, int32_t k, int32_t d) {
  double th = (double)k * M_PI / (double)g->n_views;
  double ca = cos(th), sa = sin(th);
  double t = ((double)d - 0.5 * (g->n_ch - 1)) * g->chan;
  /* Clip the line x cos + y sin = t, parametrised by p along (-sa, ca), to
   * the rectangle |x| <= W/2, |y| <= H/2 (Liang-Barsky). */
  double W = g->nx * g->pix, H = g->ny * g->pix;
  double x0 = t * ca, y0 = t * sa, dx = -sa, dy = ca;
  double p_lo = -INFINITY, p_hi = INFINITY;
  double lim[2][3] = {{x0, dx, 0.5 * W}, {y0, dy, 0.5 * H}};
  for (int a = 0; a < 2; ++a) {
    double o = lim[a][0], dv = lim[a][1], h = lim[a][2];
    if (fabs(dv) < 1e-300) {
      if (fabs(o) > h) return 0.0;
      continue;
    }
    double p1 = (-h - o) / dv, p2 = (h - o) / dv;
    if (p1 > p2) {
      double tmp = p1;
      p1 = p2;
      p2 = tmp;
    }
    if (p1 > p_lo) p_lo = p1;
    if (p2 < p_hi) p_hi = p2;
  }
  return p_hi > p_lo ? p_hi - p_lo : 0.0;
}
