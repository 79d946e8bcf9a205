/* Sanitizer driver for the FP64 oracle: a small problem through every entry
 * point (costs, gradient, ICD pass in both coordinate rules, Algorithm 1,
 * exact prox, centralised ICD, the CG MAP) under AddressSanitizer and
 * UndefinedBehaviorSanitizer; checks that the results are finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t nx, ny, n_views, n_ch;
  double pix, chan;
} mi_geom;
int64_t mi_sysmat_colptr(const mi_geom* g, int64_t* col_ptr);
int mi_sysmat_fill(const mi_geom* g, const int64_t* col_ptr, int32_t* row, float* val);

typedef struct {
  int32_t nx, ny, n_views, n_ch;
  const int64_t* col_ptr;
  const int32_t* row;
  const float* val;
  const float* y;
  const float* lam;
  int32_t n_agents;
  const int32_t* view_agent;
  int32_t prior_kind;
  double sigma_x, p, q, T, b_edge, b_diag;
  int32_t nz;
  double b_axial;
} orc_in;
typedef struct orc_state orc_state;
orc_state* orc_create(const orc_in* in);
void orc_destroy(orc_state* S);
void orc_error_sinogram(const orc_state* S, int agent, const double* x, double* e);
double orc_cost(const orc_state* S, int agent, const double* x, const double* v, double sigma);
void orc_gradient(const orc_state* S, int agent, const double* x, double* g);
int orc_icd_pass(const orc_state* S, int agent, double sigma, const double* v, double* z,
                 double* e, const int64_t* order, int mode, double relax, double* phi_trace);
int orc_mace_solve(const orc_state* S, double rho, double sigma, int sweeps, int max_iters,
                   double tol, double* w_io, const int64_t* order, int mode, double relax,
                   double* x_out, double* X_out, double* resid);
int orc_prox(const orc_state* S, int agent, double sigma, const double* v, double* z,
             int max_passes, double rtol, int mode);
int orc_centralized_icd(const orc_state* S, double* x, int max_passes, double rtol, int mode);
int orc_map_cg(const orc_state* S, double* x, int max_iters, double rtol, double* relres);

static int all_finite(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

int main(void) {
  mi_geom g = {16, 14, 24, 28, 1.0, 0.7};
  const int64_t n = (int64_t)g.nx * g.ny, m = (int64_t)g.n_views * g.n_ch;
  int64_t* cp = malloc(sizeof(int64_t) * (n + 1));
  const int64_t nnz = mi_sysmat_colptr(&g, cp);
  int32_t* row = malloc(sizeof(int32_t) * nnz);
  float* val = malloc(sizeof(float) * nnz);
  mi_sysmat_fill(&g, cp, row, val);
  const int nzmax = 3;  /* the last case is a 3-slice volume */
  float* y = malloc(sizeof(float) * m * nzmax);
  float* lam = malloc(sizeof(float) * m * nzmax);
  for (int64_t r = 0; r < m * nzmax; ++r) {
    y[r] = 0.02f * (float)((r * 37) % 11);
    lam[r] = 1000.0f + (float)(r % 7);
  }
  int32_t va[24];
  for (int k = 0; k < g.n_views; ++k) va[k] = k % 3;
  int bad = 0;
  for (int c = 0; c < 4; ++c) {
    /* prior kinds 0, 1, 2 on one slice, then a quadratic 3-slice volume */
    const int kind = c < 3 ? c : 0, nz = c < 3 ? 1 : nzmax;
    orc_in in = {g.nx, g.ny, g.n_views, g.n_ch, cp, row, val, y, lam, 3, va, kind,
                 0.01, 2.0, 1.2, 1.0, 0.1464466, 0.1035534, nz, 0.3};
    orc_state* S = orc_create(&in);
    const int64_t nv = n * nz;
    double* x = calloc(nv, sizeof(double));
    double* v = calloc(nv, sizeof(double));
    double* e = calloc(m * nz, sizeof(double));
    double* X = calloc(3 * nv, sizeof(double));
    double* gr = calloc(nv, sizeof(double));
    double res[20];
    for (int64_t s = 0; s < nv; ++s) v[s] = 0.01 * (double)(s % 5);
    orc_error_sinogram(S, 1, x, e);
    for (int mode = 0; mode < 2; ++mode) orc_icd_pass(S, 1, 0.01, v, x, e, NULL, mode, 1.0, NULL);
    const double cst = orc_cost(S, 1, x, v, 0.01);
    orc_gradient(S, -1, x, gr);
    const int k = orc_mace_solve(S, 0.8, 1e-3, 1, 20, 0.0, NULL, NULL, 0, 0.5, x, X, res);
    orc_prox(S, 0, 1e-3, v, x, 50, 1e-12, 1);
    orc_centralized_icd(S, x, 20, 1e-12, 0);
    double rel = 0.0;
    if (kind == 0) orc_map_cg(S, x, 200, 1e-12, &rel);
    bad |= !isfinite(cst) || !all_finite(gr, nv) || !all_finite(x, nv) || !all_finite(X, 3 * nv) ||
           k != 20;
    printf("prior %d, %d slice(s): cost %g, %d iterations, residual %g, CG residual %g\n", kind, nz,
           cst, k, res[k - 1], rel);
    free(x); free(v); free(e); free(X); free(gr);
    orc_destroy(S);
  }
  free(cp); free(row); free(val); free(y); free(lam);
  printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
