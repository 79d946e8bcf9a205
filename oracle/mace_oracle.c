/*
 * FP64 CPU oracle for partial-update MACE CT reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is what the GPU library is checked
 * against; the library never links, loads or calls it, and it shares no code
 * with the library.  Only the tests, the smoke check and the benchmark's CPU
 * baseline use it.
 *
 * Every quantity is computed in double precision, in the plain order the paper
 * states, without blocking, fusion or reordering.  The inputs are the system
 * matrix A in compressed sparse columns (float32 values, promoted to double),
 * the measurements y and the diagonal inverse-variance weights Lambda (float32,
 * promoted), and a partition of the views into N agents.
 *
 * Problem (Sec. II-A, eq. (global_obj) and eq. (local_obj)):
 *   f(x)   = sum_k 1/2 ||y_k - A_k x||^2_{Lambda_k} + h(x)          (beta = 1)
 *   f_i(x) = sum_{k in J_i} 1/2 ||y_k - A_k x||^2_{Lambda_k} + h(x)/N
 *   h(x)   = sum over unordered 8-neighbour pairs {s,r} of b_sr rho(x_s - x_r)
 * with b = b_edge for the 4 edge neighbours and b_diag for the 4 diagonal ones
 * and a free image boundary.  Potentials:
 *   quadratic:  rho(d) = d^2 / (2 sigma_x^2)
 *   q-GGMRF:    rho(d) = |d|^p / (p sigma_x^p) * 1/(1+s),
 *               s = (|d| / (T sigma_x))^(p-q),       1 <= q <= p <= 2
 *
 * Proximal map of agent i (eq. (prox_F)):
 *   F_i(v) = argmin_z f_i(z) + ||z - v||^2 / (2 sigma^2)
 * Partial update (Algorithm 2, ICD): visit every pixel s once, replacing z_s
 * by the minimiser along coordinate s of f_i(z) + ||z - v||^2/(2 sigma^2).
 * The error sinogram e = y - A z of the agent's rows is kept current, so the
 * data part of the coordinate function is  theta1*a + theta2*a^2/2 with
 *   theta1 = -sum_r A_rs Lambda_r e_r,   theta2 = sum_r A_rs^2 Lambda_r
 * over agent i's rows.  Two coordinate rules:
 *   mode 0 (surrogate): the prior potential is replaced by its symmetric
 *     quadratic majoriser at the current difference, curvature
 *     c(d) = rho'(d)/d; the step is then closed form.  For the quadratic
 *     prior this is the exact minimiser.
 *   mode 1 (exact): the 1-D stationarity equation is solved by bisection.
 * Both rules leave a point unchanged exactly when the gradient of the
 * coordinate function vanishes there, so they share fixed points (the
 * argument of Lemma B.1).
 *
 * MACE driver (Algorithm 1, eq. (Mann)):
 *   w^0 given (zero by default), X^0 = G(w^0)
 *   repeat: v = (2G - I) w;  X <- F~(v; X);  w <- rho (2X - v) + (1 - rho) w
 *   solution x = mean_i w_i.
 * Stopping statistic r_k = ||X^{k+1} - G w^k|| / ||w^k|| (stacked 2-norms,
 * with ||X^{k+1}|| in the denominator while w^k = 0); it vanishes exactly at a
 * fixed point, where X = G w (proof of Theorem 1).  The loop also stops when
 * r_k is not finite (a diverging run), after recording it.
 *
 * Volumes (nz > 1): a stack of nz slices of nx x ny pixels, each slice
 * measured by the same 2-D matrix A (parallel beam: every ray lies in one
 * slice), slice z's rows r + z * n_rows.  The prior adds axial cliques
 * between voxel (z, s) and (z + 1, s) with weight b_axial:
 *   h(x) = sum_z h_2D(x_z) + sum_{z, s} b_axial rho(x_{z,s} - x_{z+1,s}).
 * Voxel ids are v = z * nx * ny + s; every array over the image is over the
 * voxels, every array over the sinogram over the nz stacked sinograms.
 * nz = 1 is the 2-D problem above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t nx, ny, n_views, n_ch;
  const int64_t* col_ptr;
  const int32_t* row;
  const float* val;
  const float* y;
  const float* lam;
  int32_t n_agents;
  const int32_t* view_agent; /* [n_views] */
  int32_t prior_kind;        /* 0 quadratic, 1 q-GGMRF, 2 none (beta = 0, Sec. III) */
  double sigma_x, p, q, T, b_edge, b_diag;
  int32_t nz;                /* slices of a volume (1: a 2-D image) */
  double b_axial;            /* weight of the axial cliques (volumes) */
} orc_in;

typedef struct {
  int32_t nx, ny, n_views, n_ch, N, nz;
  int64_t n, n_rows;       /* voxels and sinogram rows of the whole stack */
  int64_t n2, nr2;         /* pixels and rows of one slice */
  /* per-agent CSC restricted to the agent's rows (global row ids) */
  int64_t** cp;
  int32_t** rw;
  double** av;
  double* y;
  double* lam;
  int32_t* row_agent;
  int32_t kind;
  double sx, p, q, T, be, bd, ba;
} orc_state;

/* ---------------- prior potential ---------------- */

static double pot(const orc_state* S, double d) {
  if (S->kind == 2) return 0.0;
  if (S->kind == 0) return d * d / (2.0 * S->sx * S->sx);
  double u = fabs(d);
  double s = pow(u / (S->T * S->sx), S->p - S->q);
  return pow(u, S->p) / (S->p * pow(S->sx, S->p)) / (1.0 + s);
}

static double pot_d1(const orc_state* S, double d) {
  if (S->kind == 2) return 0.0;
  if (S->kind == 0) return d / (S->sx * S->sx);
  double u = fabs(d);
  if (u == 0.0) return 0.0;
  double s = pow(u / (S->T * S->sx), S->p - S->q);
  double m = pow(u, S->p - 1.0) / pow(S->sx, S->p) * (1.0 + (S->q / S->p) * s) /
             ((1.0 + s) * (1.0 + s));
  return d > 0 ? m : -m;
}

/* c(d) = rho'(d)/d, the curvature of the symmetric quadratic majoriser. */
static double pot_curv(const orc_state* S, double d) {
  if (S->kind == 2) return 0.0;
  if (S->kind == 0) return 1.0 / (S->sx * S->sx);
  double u = fabs(d);
  double s = pow(u / (S->T * S->sx), S->p - S->q);
  return pow(u, S->p - 2.0) / pow(S->sx, S->p) * (1.0 + (S->q / S->p) * s) /
         ((1.0 + s) * (1.0 + s));
}

/* Neighbourhood of voxel v: the 8 in-plane neighbours in its slice and, in
 * a volume with b_axial > 0, the voxels above and below it; fills nb[] (at
 * most 10) and wt[], returns the count. */
static int neighbours(const orc_state* S, int64_t v, int64_t* nb, double* wt) {
  const int64_t z = v / S->n2, s = v % S->n2;
  int64_t i = s / S->nx, j = s % S->nx;
  int c = 0;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj) {
      if (!di && !dj) continue;
      int64_t ii = i + di, jj = j + dj;
      if (ii < 0 || ii >= S->ny || jj < 0 || jj >= S->nx) continue;
      nb[c] = z * S->n2 + ii * S->nx + jj;
      wt[c] = (di && dj) ? S->bd : S->be;
      ++c;
    }
  if (S->ba > 0) {
    if (z > 0) {
      nb[c] = v - S->n2;
      wt[c++] = S->ba;
    }
    if (z + 1 < S->nz) {
      nb[c] = v + S->n2;
      wt[c++] = S->ba;
    }
  }
  return c;
}

/* ---------------- setup ---------------- */

orc_state* orc_create(const orc_in* in) {
  if (!in || in->nx <= 0 || in->ny <= 0 || in->n_views <= 0 || in->n_ch <= 0 ||
      in->n_agents <= 0)
    return NULL;
  orc_state* S = (orc_state*)calloc(1, sizeof(orc_state));
  S->nx = in->nx;
  S->ny = in->ny;
  S->n_views = in->n_views;
  S->n_ch = in->n_ch;
  S->N = in->n_agents;
  S->nz = in->nz > 0 ? in->nz : 1;
  S->n2 = (int64_t)in->nx * in->ny;
  S->nr2 = (int64_t)in->n_views * in->n_ch;
  S->n = S->n2 * S->nz;
  S->n_rows = S->nr2 * S->nz;
  S->ba = S->nz > 1 ? in->b_axial : 0.0;
  S->kind = in->prior_kind;
  S->sx = in->sigma_x;
  S->p = in->p;
  S->q = in->q;
  S->T = in->T;
  S->be = in->b_edge;
  S->bd = in->b_diag;
  S->y = (double*)malloc(sizeof(double) * S->n_rows);
  S->lam = (double*)malloc(sizeof(double) * S->n_rows);
  S->row_agent = (int32_t*)malloc(sizeof(int32_t) * S->n_rows);
  for (int64_t r = 0; r < S->n_rows; ++r) {
    S->y[r] = in->y ? (double)in->y[r] : 0.0;
    S->lam[r] = in->lam ? (double)in->lam[r] : 0.0;
    S->row_agent[r] = in->view_agent[(r % S->nr2) / S->n_ch];
  }
  int N = S->N;
  S->cp = (int64_t**)calloc(N, sizeof(int64_t*));
  S->rw = (int32_t**)calloc(N, sizeof(int32_t*));
  S->av = (double**)calloc(N, sizeof(double*));
  /* the per-agent CSC of the 2-D matrix (slice 0's rows) */
  for (int a = 0; a < N; ++a) S->cp[a] = (int64_t*)calloc(S->n2 + 1, sizeof(int64_t));
  /* count entries per (agent, column) */
  for (int64_t s = 0; s < S->n2; ++s)
    for (int64_t t = in->col_ptr[s]; t < in->col_ptr[s + 1]; ++t)
      S->cp[S->row_agent[in->row[t]]][s + 1]++;
  for (int a = 0; a < N; ++a) {
    for (int64_t s = 0; s < S->n2; ++s) S->cp[a][s + 1] += S->cp[a][s];
    S->rw[a] = (int32_t*)malloc(sizeof(int32_t) * (S->cp[a][S->n2] + 1));
    S->av[a] = (double*)malloc(sizeof(double) * (S->cp[a][S->n2] + 1));
  }
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * N);
  for (int64_t s = 0; s < S->n2; ++s) {
    for (int a = 0; a < N; ++a) pos[a] = S->cp[a][s];
    for (int64_t t = in->col_ptr[s]; t < in->col_ptr[s + 1]; ++t) {
      int a = S->row_agent[in->row[t]];
      S->rw[a][pos[a]] = in->row[t];
      S->av[a][pos[a]] = (double)in->val[t];
      pos[a]++;
    }
  }
  free(pos);
  return S;
}

void orc_destroy(orc_state* S) {
  if (!S) return;
  for (int a = 0; a < S->N; ++a) {
    free(S->cp[a]);
    free(S->rw[a]);
    free(S->av[a]);
  }
  free(S->cp);
  free(S->rw);
  free(S->av);
  free(S->y);
  free(S->lam);
  free(S->row_agent);
  free(S);
}

/* Replace the measurements (same geometry and partition). */
void orc_set_data(orc_state* S, const float* y, const float* lam) {
  for (int64_t r = 0; r < S->n_rows; ++r) {
    S->y[r] = (double)y[r];
    S->lam[r] = (double)lam[r];
  }
}

/* ---------------- objective pieces ---------------- */

/* e_r = y_r - (A x)_r on the rows of `agent` (on all rows when agent < 0),
 * every slice of a volume. */
void orc_error_sinogram(const orc_state* S, int agent, const double* x, double* e) {
  for (int a = 0; a < S->N; ++a) {
    if (agent >= 0 && a != agent) continue;
    for (int64_t r = 0; r < S->n_rows; ++r)
      if (S->row_agent[r] == a) e[r] = S->y[r];
    for (int64_t z = 0; z < S->nz; ++z)
      for (int64_t s = 0; s < S->n2; ++s)
        for (int64_t t = S->cp[a][s]; t < S->cp[a][s + 1]; ++t)
          e[z * S->nr2 + S->rw[a][t]] -= S->av[a][t] * x[z * S->n2 + s];
  }
}

/* h(x): each unordered neighbour pair once. */
double orc_prior(const orc_state* S, const double* x) {
  double h = 0.0;
  int64_t nb[10];
  double wt[10];
  for (int64_t s = 0; s < S->n; ++s) {
    int c = neighbours(S, s, nb, wt);
    for (int k = 0; k < c; ++k)
      if (nb[k] > s) h += wt[k] * pot(S, x[s] - x[nb[k]]);
  }
  return h;
}

/* Data term of agent a (all agents when a < 0). */
double orc_data(const orc_state* S, int agent, const double* x) {
  double* e = (double*)malloc(sizeof(double) * S->n_rows);
  double d = 0.0;
  for (int a = 0; a < S->N; ++a) {
    if (agent >= 0 && a != agent) continue;
    orc_error_sinogram(S, a, x, e);
    for (int64_t r = 0; r < S->n_rows; ++r)
      if (S->row_agent[r] == a) d += 0.5 * S->lam[r] * e[r] * e[r];
  }
  free(e);
  return d;
}

/* f(x) when agent < 0; otherwise f_i(x) + ||x-v||^2/(2 sigma^2) (the prox
 * term is left out when v is NULL or sigma <= 0). */
double orc_cost(const orc_state* S, int agent, const double* x, const double* v,
                double sigma) {
  double c = orc_data(S, agent, x);
  double h = orc_prior(S, x);
  c += agent < 0 ? h : h / S->N;
  if (agent >= 0 && v && sigma > 0) {
    double q = 0.0;
    for (int64_t s = 0; s < S->n; ++s) q += (x[s] - v[s]) * (x[s] - v[s]);
    c += q / (2.0 * sigma * sigma);
  }
  return c;
}

/* Gradient of f (agent < 0) or of f_i (agent >= 0). */
void orc_gradient(const orc_state* S, int agent, const double* x, double* g) {
  double* e = (double*)malloc(sizeof(double) * S->n_rows);
  memset(g, 0, sizeof(double) * S->n);
  for (int a = 0; a < S->N; ++a) {
    if (agent >= 0 && a != agent) continue;
    orc_error_sinogram(S, a, x, e);
    for (int64_t v = 0; v < S->n; ++v) {
      const int64_t z = v / S->n2, s = v % S->n2;
      for (int64_t t = S->cp[a][s]; t < S->cp[a][s + 1]; ++t) {
        const int64_t r = z * S->nr2 + S->rw[a][t];
        g[v] -= S->av[a][t] * S->lam[r] * e[r];
      }
    }
  }
  double scale = agent < 0 ? 1.0 : 1.0 / S->N;
  int64_t nb[10];
  double wt[10];
  for (int64_t s = 0; s < S->n; ++s) {
    int c = neighbours(S, s, nb, wt);
    for (int k = 0; k < c; ++k) g[s] += scale * wt[k] * pot_d1(S, x[s] - x[nb[k]]);
  }
  free(e);
}

/* ---------------- Algorithm 2: one ICD partial update ---------------- */

/*
 * One pass of ICD for agent `agent` (agent < 0: the whole data set, i.e. the
 * centralised single-node ICD with the full prior).  Minimises, coordinate by
 * coordinate in `order` (raster when NULL),
 *   sum_{r in rows} 1/2 Lambda_r (y_r - (Az)_r)^2 + pscale*h(z)
 *     + ||z - v||^2/(2 sigma^2)          (prox term absent if sigma <= 0)
 * where pscale = 1/N for an agent and 1 for the centralised case.
 * relax scales every coordinate step (z_s += relax * alpha_s); relax = 1 is
 * the exact coordinate minimisation of Algorithm 2, relax in (0, 1) an
 * under-relaxed pass with the same fixed points (alpha_s = 0 exactly when the
 * coordinate derivative vanishes, whatever relax is).
 * z and e (= y - Az on the pass's rows, full-length array) are updated in
 * place.  If phi_trace is given, the cost after every update is stored there
 * (slow: full recomputation, small problems only).
 */
int orc_icd_pass(const orc_state* S, int agent, double sigma, const double* v,
                 double* z, double* e, const int64_t* order, int mode, double relax,
                 double* phi_trace) {
  int a0 = agent < 0 ? 0 : agent, a1 = agent < 0 ? S->N : agent + 1;
  double pscale = agent < 0 ? 1.0 : 1.0 / S->N;
  double is2 = sigma > 0 ? 1.0 / (sigma * sigma) : 0.0;
  int64_t nb[10];
  double wt[10];
  for (int64_t it = 0; it < S->n; ++it) {
    /* voxel s of the stack: column sc of A, rows of slice sz */
    const int64_t s = order ? order[it] : it;
    const int64_t sz = s / S->n2, sc = s % S->n2, roff = sz * S->nr2;
    double th1 = 0.0, th2 = 0.0;
    for (int a = a0; a < a1; ++a)
      for (int64_t t = S->cp[a][sc]; t < S->cp[a][sc + 1]; ++t) {
        const int64_t r = roff + S->rw[a][t];
        double A = S->av[a][t];
        th1 -= A * S->lam[r] * e[r];
        th2 += A * A * S->lam[r];
      }
    int c = neighbours(S, s, nb, wt);
    double zs = z[s];
    double dv = (sigma > 0 && v) ? zs - v[s] : 0.0;
    double alpha;
    if (mode == 0 || S->kind != 1) {
      double gp = 0.0, hp = 0.0;
      for (int k = 0; k < c; ++k) {
        double d = zs - z[nb[k]];
        double cw = pot_curv(S, d);
        gp += wt[k] * cw * d;
        hp += wt[k] * cw;
      }
      double num = th1 + pscale * gp + is2 * dv;
      double den = th2 + pscale * hp + is2;
      alpha = den > 0 ? -num / den : 0.0;
    } else {
      /* g(a) = th1 + th2 a + pscale sum b rho'(d_k + a) + is2 (dv + a),
       * strictly increasing; bracket the root and bisect. */
      double g0 = th1 + is2 * dv;
      for (int k = 0; k < c; ++k) g0 += pscale * wt[k] * pot_d1(S, zs - z[nb[k]]);
      if (g0 == 0.0) {
        alpha = 0.0;
      } else {
        double dir = g0 < 0 ? 1.0 : -1.0;
        double den0 = th2 + is2;
        for (int k = 0; k < c; ++k) den0 += pscale * wt[k] * pot_curv(S, zs - z[nb[k]]);
        double step = fabs(g0) / (den0 > 0 ? den0 : 1.0);
        if (!(step > 0)) step = 1e-300;
        double lo = 0.0, hi = dir * step;
        for (int guard = 0; guard < 2000; ++guard) {
          double gh = th1 + th2 * hi + is2 * (dv + hi);
          for (int k = 0; k < c; ++k) gh += pscale * wt[k] * pot_d1(S, zs - z[nb[k]] + hi);
          if ((dir > 0 && gh >= 0) || (dir < 0 && gh <= 0)) break;
          lo = hi;
          hi *= 2.0;
        }
        for (int guard = 0; guard < 400; ++guard) {
          double mid = 0.5 * (lo + hi);
          if (mid == lo || mid == hi) break;
          double gm = th1 + th2 * mid + is2 * (dv + mid);
          for (int k = 0; k < c; ++k) gm += pscale * wt[k] * pot_d1(S, zs - z[nb[k]] + mid);
          if ((dir > 0 && gm < 0) || (dir < 0 && gm > 0))
            lo = mid;
          else
            hi = mid;
        }
        alpha = 0.5 * (lo + hi);
      }
    }
    alpha *= relax;
    z[s] = zs + alpha;
    for (int a = a0; a < a1; ++a)
      for (int64_t t = S->cp[a][sc]; t < S->cp[a][sc + 1]; ++t)
        e[roff + S->rw[a][t]] -= S->av[a][t] * alpha;
    if (phi_trace) phi_trace[it] = orc_cost(S, agent, z, v, sigma);
  }
  return 0;
}

/* ---------------- Algorithm 1: partial-update MACE ---------------- */

/*
 * w_io: [N*n] initial w on entry (NULL = zeros), final w on exit if given.
 * X_out: [N*n] final agent states (optional).  resid: [max_iters] trace of
 * r_k (optional).  Returns the number of Mann iterations done.
 */
int orc_mace_solve(const orc_state* S, double rho, double sigma, int sweeps,
                   int max_iters, double tol, double* w_io, const int64_t* order,
                   int mode, double relax, double* x_out, double* X_out, double* resid) {
  int N = S->N;
  int64_t n = S->n;
  double* w = (double*)malloc(sizeof(double) * N * n);
  double* X = (double*)malloc(sizeof(double) * N * n);
  double* v = (double*)malloc(sizeof(double) * N * n);
  double* wbar = (double*)malloc(sizeof(double) * n);
  double* e = (double*)malloc(sizeof(double) * S->n_rows);
  if (w_io)
    memcpy(w, w_io, sizeof(double) * N * n);
  else
    memset(w, 0, sizeof(double) * N * n);
  /* X^0 = G(w^0) */
  for (int64_t s = 0; s < n; ++s) {
    double m = 0.0;
    for (int a = 0; a < N; ++a) m += w[a * n + s];
    wbar[s] = m / N;
  }
  for (int a = 0; a < N; ++a) memcpy(X + a * n, wbar, sizeof(double) * n);
  for (int a = 0; a < N; ++a) orc_error_sinogram(S, a, X + a * n, e);
  int k = 0;
  for (; k < max_iters; ++k) {
    /* w-bar and v = (2G - I) w */
    for (int64_t s = 0; s < n; ++s) {
      double m = 0.0;
      for (int a = 0; a < N; ++a) m += w[a * n + s];
      wbar[s] = m / N;
    }
    for (int a = 0; a < N; ++a)
      for (int64_t s = 0; s < n; ++s) v[a * n + s] = 2.0 * wbar[s] - w[a * n + s];
    /* X <- F~(v; X), agents independent */
#pragma omp parallel for schedule(static, 1)
    for (int a = 0; a < N; ++a)
      for (int sw = 0; sw < sweeps; ++sw)
        orc_icd_pass(S, a, sigma, v + a * n, X + a * n, e, order, mode, relax, NULL);
    /* stopping statistic, summed in agent order */
    double num = 0.0, den = 0.0, dx = 0.0;
    for (int a = 0; a < N; ++a)
      for (int64_t s = 0; s < n; ++s) {
        double d = X[a * n + s] - wbar[s];
        num += d * d;
        den += w[a * n + s] * w[a * n + s];
        dx += X[a * n + s] * X[a * n + s];
      }
    double r = sqrt(num) / sqrt(den > 0 ? den : dx);
    if (resid) resid[k] = r;
    /* reflection and Mann update */
    for (int a = 0; a < N; ++a)
      for (int64_t s = 0; s < n; ++s)
        w[a * n + s] = rho * (2.0 * X[a * n + s] - v[a * n + s]) + (1.0 - rho) * w[a * n + s];
    if (r < tol || !isfinite(r)) {
      ++k;
      break;
    }
  }
  for (int64_t s = 0; s < n; ++s) {
    double m = 0.0;
    for (int a = 0; a < N; ++a) m += w[a * n + s];
    x_out[s] = m / N;
  }
  if (w_io) memcpy(w_io, w, sizeof(double) * N * n);
  if (X_out) memcpy(X_out, X, sizeof(double) * N * n);
  free(w);
  free(X);
  free(v);
  free(wbar);
  free(e);
  return k;
}

/* Exact proximal map F_i(v) (eq. (prox_F)) by repeated exact ICD passes from
 * z (in/out) until the largest change is <= rtol * max|z|. Returns passes. */
int orc_prox(const orc_state* S, int agent, double sigma, const double* v,
             double* z, int max_passes, double rtol, int mode) {
  double* e = (double*)malloc(sizeof(double) * S->n_rows);
  double* zo = (double*)malloc(sizeof(double) * S->n);
  orc_error_sinogram(S, agent, z, e);
  int it = 0;
  for (; it < max_passes; ++it) {
    memcpy(zo, z, sizeof(double) * S->n);
    orc_icd_pass(S, agent, sigma, v, z, e, NULL, mode, 1.0, NULL);
    double dm = 0.0, zm = 0.0;
    for (int64_t s = 0; s < S->n; ++s) {
      double d = fabs(z[s] - zo[s]);
      if (d > dm) dm = d;
      if (fabs(z[s]) > zm) zm = fabs(z[s]);
    }
    if (dm <= rtol * zm) {
      ++it;
      break;
    }
  }
  free(e);
  free(zo);
  return it;
}

/* Centralised single-node ICD on f (all views, full prior, no prox term), the
 * paper's baseline; passes until the largest change <= rtol * max|x|. */
int orc_centralized_icd(const orc_state* S, double* x, int max_passes, double rtol,
                        int mode) {
  double* e = (double*)malloc(sizeof(double) * S->n_rows);
  double* xo = (double*)malloc(sizeof(double) * S->n);
  for (int a = 0; a < S->N; ++a) orc_error_sinogram(S, a, x, e);
  int it = 0;
  for (; it < max_passes; ++it) {
    memcpy(xo, x, sizeof(double) * S->n);
    orc_icd_pass(S, -1, 0.0, NULL, x, e, NULL, mode, 1.0, NULL);
    double dm = 0.0, zm = 0.0;
    for (int64_t s = 0; s < S->n; ++s) {
      double d = fabs(x[s] - xo[s]);
      if (d > dm) dm = d;
      if (fabs(x[s]) > zm) zm = fabs(x[s]);
    }
    if (dm <= rtol * zm) {
      ++it;
      break;
    }
  }
  free(e);
  free(xo);
  return it;
}

/* ---------------- MAP of the quadratic prior by conjugate gradients ------ */

/* out = H v with H = A^T Lambda A + L_b / sigma_x^2, the Hessian of f for the
 * quadratic prior (eq. (global_obj) with rho(d) = d^2 / (2 sigma_x^2)); L_b is
 * the weighted graph Laplacian of the 8-neighbour cliques: (L_b v)_s =
 * sum_r b_sr (v_s - v_r).  tmp: scratch of n_rows doubles. */
static void quad_hessian_apply(const orc_state* S, const double* v, double* out, double* tmp) {
  /* tmp = A v, agent by agent (the agents' rows are disjoint), slice by slice */
#pragma omp parallel for schedule(static, 1)
  for (int a = 0; a < S->N; ++a) {
    for (int64_t r = 0; r < S->n_rows; ++r)
      if (S->row_agent[r] == a) tmp[r] = 0.0;
    for (int64_t z = 0; z < S->nz; ++z)
      for (int64_t s = 0; s < S->n2; ++s)
        for (int64_t t = S->cp[a][s]; t < S->cp[a][s + 1]; ++t)
          tmp[z * S->nr2 + S->rw[a][t]] += S->av[a][t] * v[z * S->n2 + s];
  }
  const double c = 1.0 / (S->sx * S->sx);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < S->n; ++s) {
    const int64_t sz = s / S->n2, sc = s % S->n2;
    double acc = 0.0;
    for (int a = 0; a < S->N; ++a)
      for (int64_t t = S->cp[a][sc]; t < S->cp[a][sc + 1]; ++t) {
        const int64_t r = sz * S->nr2 + S->rw[a][t];
        acc += S->av[a][t] * S->lam[r] * tmp[r];
      }
    int64_t nb[10];
    double wt[10];
    int k = neighbours(S, s, nb, wt);
    for (int q = 0; q < k; ++q) acc += c * wt[q] * (v[s] - v[nb[q]]);
    out[s] = acc;
  }
}

/*
 * MAP estimate for the quadratic prior: solves the normal equations
 *   (A^T Lambda A + L_b / sigma_x^2) x = A^T Lambda y
 * by conjugate gradients with the diagonal of the matrix as preconditioner
 * (Jacobi-preconditioned CG, textbook form), from x (in/out), until
 * ||b - H x|| <= rtol ||b||.  Requires the quadratic prior (kind 0).  Returns
 * the iterations done (-1 if the prior is not quadratic); *relres receives
 * the final ||b - H x|| / ||b||.
 */
int orc_map_cg(const orc_state* S, double* x, int max_iters, double rtol, double* relres) {
  if (S->kind != 0) return -1;
  const int64_t n = S->n;
  double* b = (double*)calloc(n, sizeof(double));
  double* r = (double*)malloc(sizeof(double) * n);
  double* z = (double*)malloc(sizeof(double) * n);
  double* p = (double*)malloc(sizeof(double) * n);
  double* q = (double*)malloc(sizeof(double) * n);
  double* dinv = (double*)malloc(sizeof(double) * n);
  double* tmp = (double*)malloc(sizeof(double) * S->n_rows);
  const double c = 1.0 / (S->sx * S->sx);
  for (int64_t s = 0; s < n; ++s) {
    const int64_t sz = s / S->n2, sc = s % S->n2;
    double bs = 0.0, ds = 0.0;
    for (int a = 0; a < S->N; ++a)
      for (int64_t t = S->cp[a][sc]; t < S->cp[a][sc + 1]; ++t) {
        const int64_t rr = sz * S->nr2 + S->rw[a][t];
        bs += S->av[a][t] * S->lam[rr] * S->y[rr];
        ds += S->av[a][t] * S->av[a][t] * S->lam[rr];
      }
    int64_t nb[10];
    double wt[10];
    int k = neighbours(S, s, nb, wt);
    for (int j = 0; j < k; ++j) ds += c * wt[j];
    b[s] = bs;
    dinv[s] = ds > 0 ? 1.0 / ds : 1.0;
  }
  double bn = 0.0;
  for (int64_t s = 0; s < n; ++s) bn += b[s] * b[s];
  bn = sqrt(bn);
  quad_hessian_apply(S, x, q, tmp);
  double rz = 0.0, rn = 0.0;
  for (int64_t s = 0; s < n; ++s) {
    r[s] = b[s] - q[s];
    z[s] = dinv[s] * r[s];
    p[s] = z[s];
    rz += r[s] * z[s];
    rn += r[s] * r[s];
  }
  int it = 0;
  while (it < max_iters && sqrt(rn) > rtol * bn) {
    quad_hessian_apply(S, p, q, tmp);
    double pq = 0.0;
    for (int64_t s = 0; s < n; ++s) pq += p[s] * q[s];
    if (!(pq > 0)) break;
    const double alpha = rz / pq;
    double rz1 = 0.0;
    rn = 0.0;
    for (int64_t s = 0; s < n; ++s) {
      x[s] += alpha * p[s];
      r[s] -= alpha * q[s];
      z[s] = dinv[s] * r[s];
      rz1 += r[s] * z[s];
      rn += r[s] * r[s];
    }
    const double beta = rz1 / rz;
    rz = rz1;
    for (int64_t s = 0; s < n; ++s) p[s] = z[s] + beta * p[s];
    ++it;
  }
  /* the true residual of the returned x */
  quad_hessian_apply(S, x, q, tmp);
  double tn = 0.0;
  for (int64_t s = 0; s < n; ++s) tn += (b[s] - q[s]) * (b[s] - q[s]);
  if (relres) *relres = bn > 0 ? sqrt(tn) / bn : sqrt(tn);
  free(b);
  free(r);
  free(z);
  free(p);
  free(q);
  free(dinv);
  free(tmp);
  return it;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
