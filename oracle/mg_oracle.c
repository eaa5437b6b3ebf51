/*
 * mg_oracle.c -- plain FP64 CPU oracle for the MG-GLAM scalar-field hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's
 * cpu_baseline leg may load this library.  It shares no code, header, table
 * or constant generator with the HIP library and never calls it.
 *
 * Everything is FP64, natural layout v[(k*N + j)*N + i] with i (x) fastest,
 * periodic boundaries, cell size h in units of the finest cell.  It follows
 * "Fast full N-body simulations of generic modified gravity: conformal
 * coupling models" (Ruan et al., arXiv:2110.00328):
 *
 *   code units ......................... Sec. 3.1.1 (eq:code_units, c-tilde)
 *   f(R) equation + per-cell polynomial  Sec. 3.2.5 (eq:fR_eom_codeunit2,
 *                                        eq:fR_eom_codeunit, eq:fR_*_solns)
 *   symmetron equation + cubic ......... Sec. 3.2.4 (eq:sym_eom_code_unit,
 *                                        eq:sym_cubic_eqn, eq:sym_cubic_solns)
 *   coupled quintessence ............... Sec. 3.2.3 (eq:csf_eom_code), solved by
 *                                        Newton-Gauss-Seidel (eq:relaxation_iteration)
 *   residual, FAS coarse equation,
 *   restriction, prolongation, V-cycle . Sec. 3.2.1 (eq:residual_d,
 *                                        eq:general_pde_numerical_coarse,
 *                                        eq:solution_correction)
 *   CIC and 3-point force .............. Sec. 3.1 (GLAM description)
 *   fifth forces ....................... eq:F5_fR_codeunit, eq:F_5_codeunit,
 *                                        eq:csf_particle_geodesic_code2
 *
 * Readings of the paper where it is silent or garbled:
 *  - the Laplacian in the f(R) polynomial acts on w = u^{n+1} = -f_R, so the
 *    neighbour sum in p is a sum of w (eq:fR_eom_codeunit2 vs eq:Lijk);
 *  - the printed Cardano form cancels catastrophically; every cubic here is
 *    solved with the Viete trigonometric / hyperbolic forms, which select the
 *    same branch (single real root, else the largest real root), then one
 *    Newton polish.  The quartic (n=2) root is the unique positive root found
 *    by monotone Newton from an upper bound;
 *  - the first half-sweep updates cells with (i+j+k) even (0-based);
 *  - the coarsest level is the first of N, N/2, ... whose half is odd or
 *    below 4 (4^3 for N = 2^l, 6^3 for N = 96); it is relaxed until its RMS
 *    residual has dropped by 1e-10 (at most 1000 sweeps), or, for coupled
 *    quintessence, solved by dense Newton;
 *  - relative residual = RMS(d) / RMS(d at the background field).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_FR 0
#define ORA_SYM 1
#define ORA_CQ 2

#define ORA_C_OVER_H0 2997.92458 /* Mpc/h */
#define ORA_MAXLEV 24

typedef struct {
  int model;      /* ORA_FR / ORA_SYM / ORA_CQ */
  int n;          /* grid cells per side of the finest level */
  double box;     /* box size in Mpc/h */
  double a;       /* scale factor */
  double omega_m; /* Omega_m; Omega_Lambda = 1 - Omega_m */
  int fr_n;       /* Hu-Sawicki n in {0,1,2} */
  double fr0;     /* |f_R0| */
  double a_star;  /* symmetron a_* */
  double xi;      /* symmetron xi = H0/m_* */
  double beta_star;
  double alpha;   /* CQ alpha */
  double beta;    /* CQ beta */
  double phibar;  /* CQ background field at a */
  double lambda;  /* CQ lambda (eq:csf_param_lambda) */
  int cq_keep_exp; /* 1: keep exp(beta phi/c^2) in front of (1+delta) */
} ora_params;

/* ------------------------------------------------------------------ */
/* Constants in code units                                             */
/* ------------------------------------------------------------------ */
typedef struct {
  double ct2;     /* c-tilde squared */
  double om_a;    /* Omega_m / a */
  double K;       /* R-bar(a) a^2 / 3 = Omega_m/a + 4 Omega_L a^2 */
  double wbar;    /* |f_R(a)| */
  double wpow;    /* wbar^{1/(n+1)} */
  int n;          /* f(R) n */
  double s_ratio; /* a_*^3 / a^3 */
  double s_amp;   /* a^2 / (2 xi^2) */
  double ubar;    /* sqrt(1 - a_*^3/a^3) */
  double cq_src;  /* 3 beta Omega_m a^-1 exp(beta phibar) */
  double cq_pot;  /* alpha lambda^2 a^2 */
  double cq_pb;   /* phibar^{-(1+alpha)} */
} ora_consts;

static ora_consts consts_of(const ora_params *P) {
  ora_consts c;
  memset(&c, 0, sizeof c);
  double ct = (double)P->n * ORA_C_OVER_H0 / P->box;
  double oml = 1.0 - P->omega_m;
  double a = P->a;
  c.ct2 = ct * ct;
  c.om_a = P->omega_m / a;
  /* R-bar / H0^2 = 3 (Omega_m a^-3 + 4 Omega_L), eq:R_bar */
  c.K = (3.0 * (P->omega_m / (a * a * a) + 4.0 * oml)) * a * a / 3.0;
  c.n = P->fr_n;
  /* f_R(a) = -|f_R0| (R0/R(a))^{n+1}, eq:fR_HS with R = R-bar(a) */
  double r0 = P->omega_m + 4.0 * oml;
  double ra = P->omega_m / (a * a * a) + 4.0 * oml;
  c.wbar = P->fr0 * pow(r0 / ra, (double)(P->fr_n + 1));
  c.wpow = pow(c.wbar, 1.0 / (double)(P->fr_n + 1));
  c.s_ratio = pow(P->a_star / a, 3.0);
  c.s_amp = a * a / (2.0 * P->xi * P->xi);
  c.ubar = c.s_ratio < 1.0 ? sqrt(1.0 - c.s_ratio) : 0.0;
  c.cq_src = 3.0 * P->beta * P->omega_m / a * exp(P->beta * P->phibar);
  c.cq_pot = P->alpha * P->lambda * P->lambda * a * a;
  c.cq_pb = pow(P->phibar, -(1.0 + P->alpha));
  return c;
}

double ora_ctilde(int n, double box) { return (double)n * ORA_C_OVER_H0 / box; }

/* Background value of the solved variable (w=-f_R for f(R), u, phi~). */
double ora_background(const ora_params *P) {
  ora_consts c = consts_of(P);
  if (P->model == ORA_FR) return c.wbar;
  if (P->model == ORA_SYM) return c.ubar;
  return 0.0;
}

/* ------------------------------------------------------------------ */
/* Per-cell roots                                                      */
/* ------------------------------------------------------------------ */

/* Root of t^3 + p t + q = 0 on the paper's branch: the single real root
 * when there is one, otherwise the largest of the three (eq:sym_cubic_solns,
 * eq:fR_cubic_solns).  For q < 0 that is the unique positive root.
 * Evaluated with Viete's trigonometric / hyperbolic forms, then one Newton
 * step. */
double ora_cubic_root(double p, double q) {
  double t;
  if (p == 0.0) {
    t = cbrt(-q);
  } else if (p > 0.0) {
    double s = sqrt(p / 3.0);
    double x = (1.5 * q / p) / s; /* (3q/2p) sqrt(3/p) */
    t = -2.0 * s * sinh(asinh(x) / 3.0);
  } else {
    double s = sqrt(-p / 3.0);
    double x = (1.5 * q / p) / s; /* (3q/2p) sqrt(-3/p) */
    if (x >= 1.0)
      t = 2.0 * s * cosh(acosh(x) / 3.0);
    else if (x <= -1.0)
      t = -2.0 * s * cosh(acosh(-x) / 3.0);
    else
      t = 2.0 * s * cos(acos(x) / 3.0);
  }
  double f = (t * t + p) * t + q;
  double fp = 3.0 * t * t + p;
  if (fp != 0.0 && isfinite(fp)) {
    double tn = t - f / fp;
    if (isfinite(tn)) t = tn;
  }
  return t;
}

/* Unique positive root of u^{n+2} + p u + q = 0 with q < 0 (eq:fR_eom_codeunit). */
double ora_fr_root(int n, double p, double q) {
  if (n == 1) return ora_cubic_root(p, q);
  if (n == 0) {
    /* eq:fR_quadratic_solns; rationalised when p > 0 to avoid cancellation */
    double sq = sqrt(p * p - 4.0 * q);
    return p > 0.0 ? -2.0 * q / (p + sq) : 0.5 * (-p + sq);
  }
  /* n = 2: f(u) = u^4 + p u + q is convex for u > 0 with f(0) = q < 0, so
   * Newton from any point right of the root decreases monotonically to it. */
  double u = pow(-2.0 * q, 0.25);
  if (p < 0.0) {
    double b = cbrt(-2.0 * p);
    if (b > u) u = b;
  }
  for (int it = 0; it < 200; ++it) {
    double u3 = u * u * u;
    double f = u3 * u + p * u + q;
    double fp = 4.0 * u3 + p;
    if (!(fp > 0.0)) break;
    double un = u - f / fp;
    if (!(un < u)) break; /* monotone sequence has stopped */
    u = un;
  }
  return u;
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */
static inline size_t IDX(int n, int i, int j, int k) {
  return ((size_t)k * (size_t)n + (size_t)j) * (size_t)n + (size_t)i;
}
static inline int WRAP(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

static inline double nb_sum(const double *v, int n, int i, int j, int k) {
  return v[IDX(n, WRAP(i + 1, n), j, k)] + v[IDX(n, WRAP(i - 1, n), j, k)] +
         v[IDX(n, i, WRAP(j + 1, n), k)] + v[IDX(n, i, WRAP(j - 1, n), k)] +
         v[IDX(n, i, j, WRAP(k + 1, n))] + v[IDX(n, i, j, WRAP(k - 1, n))];
}

/* ------------------------------------------------------------------ */
/* The discrete operator L^h(v) of each model (without the source)     */
/* ------------------------------------------------------------------ */
static double cell_op(const ora_params *P, const ora_consts *c, double h,
                      double vc, double sum, double dc) {
  double lap = (sum - 6.0 * vc) / (h * h);
  if (P->model == ORA_FR) {
    /* -c^2 lap w + (Om/a) delta + K - K wbar^{1/(n+1)} w^{-1/(n+1)}  (eq:fR_eom_codeunit2) */
    return -c->ct2 * lap + c->om_a * dc + c->K -
           c->K * c->wpow * pow(vc, -1.0 / (double)(c->n + 1));
  }
  if (P->model == ORA_SYM) {
    /* c^2 lap u - a^2/(2 xi^2) [ (rho a*^3/a^3 - 1) u + u^3 ]  (eq:sym_eom_code_unit) */
    return c->ct2 * lap -
           c->s_amp * (((1.0 + dc) * c->s_ratio - 1.0) * vc + vc * vc * vc);
  }
  /* lap phi - 3 beta Om/a e^{beta phibar}[e^{beta phi/c^2}(1+delta) - 1]
   *         + alpha lambda^2 a^2 [(phibar + phi/c^2)^{-(1+alpha)} - phibar^{-(1+alpha)}]
   * (eq:csf_eom_code).
   * Both bracketed differences are evaluated in an algebraically identical
   * form that keeps their phi-dependence when phi/c^2 ~ 1e-14:
   *   e^x (1+delta) - 1 = expm1(x)(1+delta) + delta,
   *   (pb + y)^{-(1+al)} - pb^{-(1+al)} = pb^{-(1+al)} expm1(-(1+al) log1p(y/pb)). */
  double x = P->cq_keep_exp ? P->beta * vc / c->ct2 : 0.0;
  double src = expm1(x) * (1.0 + dc) + dc;
  double pot = c->cq_pb * expm1(-(1.0 + P->alpha) * log1p(vc / (c->ct2 * P->phibar)));
  return lap - c->cq_src * src + c->cq_pot * pot;
}

/* d/dv_c of cell_op (used by Newton-Gauss-Seidel, eq:relaxation_iteration). */
static double cell_op_diag(const ora_params *P, const ora_consts *c, double h,
                           double vc, double dc) {
  if (P->model == ORA_FR) {
    double m = 1.0 / (double)(c->n + 1);
    return 6.0 * c->ct2 / (h * h) + c->K * c->wpow * m * pow(vc, -m - 1.0);
  }
  if (P->model == ORA_SYM) {
    return -6.0 * c->ct2 / (h * h) -
           c->s_amp * (((1.0 + dc) * c->s_ratio - 1.0) + 3.0 * vc * vc);
  }
  double e = P->cq_keep_exp ? exp(P->beta * vc / c->ct2) : 0.0;
  return -6.0 / (h * h) - c->cq_src * P->beta / c->ct2 * e * (1.0 + dc) -
         c->cq_pot * (1.0 + P->alpha) / c->ct2 *
             pow(P->phibar + vc / c->ct2, -(2.0 + P->alpha));
}

/* ------------------------------------------------------------------ */
/* Public single-level operations                                      */
/* ------------------------------------------------------------------ */

/* d = L^h(v) - S (eq:residual_d); S may be NULL (finest level, S = 0).
 * Returns sum of d^2. */
double ora_residual(const ora_params *P, int n, double h, const double *delta,
                    const double *S, const double *v, double *d) {
  ora_consts c = consts_of(P);
  double *part = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t id = IDX(n, i, j, k);
        double r = cell_op(P, &c, h, v[id], nb_sum(v, n, i, j, k), delta[id]) -
                   (S ? S[id] : 0.0);
        if (d) d[id] = r;
        acc += r * r;
      }
    part[k] = acc;
  }
  double tot = 0.0;
  for (int k = 0; k < n; ++k) tot += part[k];
  free(part);
  return tot;
}

/* Exact (nonlinear Gauss-Seidel) or Newton update of one cell so that
 * L^h(v)_c = S_c, given its six neighbours. */
static double cell_update(const ora_params *P, const ora_consts *c, double h,
                          double vc, double sum, double dc, double sc) {
  if (P->model == ORA_FR) {
    double g = h * h / (6.0 * c->ct2);
    double p = g * (c->om_a * dc + c->K - sc) - sum / 6.0;
    double q = -g * c->K * c->wpow;
    double u = ora_fr_root(c->n, p, q);
    return pow(u, (double)(c->n + 1));
  }
  if (P->model == ORA_SYM) {
    double kap = 2.0 * c->ct2 / (c->s_amp * 2.0 * h * h); /* 2 c^2 xi^2/(a^2 h^2) */
    double p = (1.0 + dc) * c->s_ratio - 1.0 + 6.0 * kap;
    double q = -kap * sum + sc / c->s_amp;
    return ora_cubic_root(p, q);
  }
  double f = cell_op(P, c, h, vc, sum, dc) - sc;
  double df = cell_op_diag(P, c, h, vc, dc);
  return vc - f / df;
}

/* One half-sweep over cells with (i+j+k) % 2 == colour. */
void ora_relax_colour(const ora_params *P, int n, double h, const double *delta,
                      const double *S, double *v, int colour) {
  ora_consts c = consts_of(P);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = (j + k + colour) & 1; i < n; i += 2) {
        size_t id = IDX(n, i, j, k);
        v[id] = cell_update(P, &c, h, v[id], nb_sum(v, n, i, j, k), delta[id],
                            S ? S[id] : 0.0);
      }
}

/* One Gauss-Seidel sweep: (i+j+k) even cells first, then odd. */
void ora_relax(const ora_params *P, int n, double h, const double *delta,
               const double *S, double *v) {
  ora_relax_colour(P, n, h, delta, S, v, 0);
  ora_relax_colour(P, n, h, delta, S, v, 1);
}

/* Restriction: arithmetic mean of the 8 children (Sec. 3.2.1). */
void ora_restrict(int nf, const double *f, double *c) {
  int nc = nf / 2;
#pragma omp parallel for schedule(static)
  for (int K = 0; K < nc; ++K)
    for (int J = 0; J < nc; ++J)
      for (int I = 0; I < nc; ++I) {
        double s = 0.0;
        for (int dk = 0; dk < 2; ++dk)
          for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di)
              s += f[IDX(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
        c[IDX(nc, I, J, K)] = s / 8.0;
      }
}

/* fine += P(coarse): 27/64 parent, 9/64 face, 3/64 edge, 1/64 corner
 * neighbour of the parent (eq:solution_correction and the list after it). */
void ora_prolong_add(int nc, const double *c, double *f) {
  int nf = 2 * nc;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nf; ++k)
    for (int j = 0; j < nf; ++j)
      for (int i = 0; i < nf; ++i) {
        int I = i / 2, J = j / 2, Kc = k / 2;
        int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        double acc = 0.0;
        for (int ak = 0; ak < 2; ++ak)
          for (int aj = 0; aj < 2; ++aj)
            for (int ai = 0; ai < 2; ++ai) {
              double w = (ai ? 1.0 : 3.0) * (aj ? 1.0 : 3.0) * (ak ? 1.0 : 3.0) / 64.0;
              acc += w * c[IDX(nc, WRAP(I + ai * si, nc), WRAP(J + aj * sj, nc),
                               WRAP(Kc + ak * sk, nc))];
            }
        f[IDX(nf, i, j, k)] += acc;
      }
}

/* ------------------------------------------------------------------ */
/* Dense solve (coarsest level of coupled quintessence)                */
/* ------------------------------------------------------------------ */
/* Gaussian elimination with partial pivoting; A is m x m row-major,
 * overwritten; b overwritten with the solution.  Returns 0 on success. */
int ora_dense_solve(int m, double *A, double *b) {
  for (int col = 0; col < m; ++col) {
    int piv = col;
    double best = fabs(A[(size_t)col * m + col]);
    for (int r = col + 1; r < m; ++r) {
      double v = fabs(A[(size_t)r * m + col]);
      if (v > best) { best = v; piv = r; }
    }
    if (best == 0.0) return -1;
    if (piv != col) {
      for (int cc = 0; cc < m; ++cc) {
        double t = A[(size_t)col * m + cc];
        A[(size_t)col * m + cc] = A[(size_t)piv * m + cc];
        A[(size_t)piv * m + cc] = t;
      }
      double t = b[col]; b[col] = b[piv]; b[piv] = t;
    }
    for (int r = col + 1; r < m; ++r) {
      double f = A[(size_t)r * m + col] / A[(size_t)col * m + col];
      if (f == 0.0) continue;
      for (int cc = col; cc < m; ++cc) A[(size_t)r * m + cc] -= f * A[(size_t)col * m + cc];
      b[r] -= f * b[col];
    }
  }
  for (int r = m - 1; r >= 0; --r) {
    double s = b[r];
    for (int cc = r + 1; cc < m; ++cc) s -= A[(size_t)r * m + cc] * b[cc];
    b[r] = s / A[(size_t)r * m + r];
  }
  return 0;
}

/* Newton on the whole level: J dv = -(L(v) - S), J = lap/h^2-stencil + diag. */
static void dense_newton(const ora_params *P, int n, double h, const double *delta,
                         const double *S, double *v) {
  ora_consts c = consts_of(P);
  int m = n * n * n;
  double *A = (double *)malloc((size_t)m * m * sizeof(double));
  double *r = (double *)malloc((size_t)m * sizeof(double));
  double lapc = (P->model == ORA_FR ? -c.ct2 : (P->model == ORA_SYM ? c.ct2 : 1.0)) / (h * h);
  double r0 = -1.0;
  for (int it = 0; it < 60; ++it) {
    double rr = ora_residual(P, n, h, delta, S, v, r);
    if (r0 < 0.0) r0 = rr;
    if (rr == 0.0 || rr <= 1e-28 * r0) break;
    memset(A, 0, (size_t)m * m * sizeof(double));
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          size_t row = IDX(n, i, j, k);
          double *Ar = A + row * (size_t)m;
          Ar[IDX(n, WRAP(i + 1, n), j, k)] += lapc;
          Ar[IDX(n, WRAP(i - 1, n), j, k)] += lapc;
          Ar[IDX(n, i, WRAP(j + 1, n), k)] += lapc;
          Ar[IDX(n, i, WRAP(j - 1, n), k)] += lapc;
          Ar[IDX(n, i, j, WRAP(k + 1, n))] += lapc;
          Ar[IDX(n, i, j, WRAP(k - 1, n))] += lapc;
          Ar[row] += cell_op_diag(P, &c, h, v[row], delta[row]);
          r[row] = -r[row];
        }
    if (ora_dense_solve(m, A, r) != 0) break;
    for (int q = 0; q < m; ++q) v[q] += r[q];
  }
  free(A);
  free(r);
}

/* ------------------------------------------------------------------ */
/* FAS multigrid                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
  int nlev;
  int n[ORA_MAXLEV];
  double h[ORA_MAXLEV];
  double *delta[ORA_MAXLEV];
  double *v[ORA_MAXLEV];
  double *S[ORA_MAXLEV];  /* NULL on level 0 */
  double *Rv[ORA_MAXLEV]; /* restricted fine field, level l >= 1 */
  double *d[ORA_MAXLEV];  /* residual scratch */
} ora_hier;

/* Number of levels: halve while the half is even and at least 4. */
int ora_num_levels(int n) {
  int L = 1;
  while ((n / 2) >= 4 && ((n / 2) % 2) == 0 && (n % 2) == 0) {
    n /= 2;
    ++L;
  }
  return L;
}

static void hier_free(ora_hier *H) {
  for (int l = 0; l < H->nlev; ++l) {
    if (l > 0) { free(H->delta[l]); free(H->v[l]); free(H->S[l]); free(H->Rv[l]); }
    free(H->d[l]);
  }
}

static void coarsest_solve(const ora_params *P, ora_hier *H, int l) {
  int n = H->n[l];
  if (P->model == ORA_CQ) {
    dense_newton(P, n, H->h[l], H->delta[l], H->S[l], H->v[l]);
    return;
  }
  double r0 = ora_residual(P, n, H->h[l], H->delta[l], H->S[l], H->v[l], NULL);
  for (int it = 0; it < 1000; ++it) {
    ora_relax(P, n, H->h[l], H->delta[l], H->S[l], H->v[l]);
    double r = ora_residual(P, n, H->h[l], H->delta[l], H->S[l], H->v[l], NULL);
    if (r <= 1e-20 * r0 || r == 0.0) break; /* RMS dropped by 1e-10 */
  }
}

/* cycle: 0 = V, 1 = F, 2 = W (Sec. 3.2.1, fig:multigrid_cycles). */
static void mg_cycle(const ora_params *P, ora_hier *H, int l, int nu1, int nu2, int cycle) {
  if (l == H->nlev - 1) {
    coarsest_solve(P, H, l);
    return;
  }
  int n = H->n[l], nc = H->n[l + 1];
  size_t mc = (size_t)nc * nc * nc;
  for (int s = 0; s < nu1; ++s) ora_relax(P, n, H->h[l], H->delta[l], H->S[l], H->v[l]);
  /* d^h, R u^h, R d^h, S^H = L^H(R u^h) - R d^h (eq:general_pde_numerical_coarse) */
  ora_residual(P, n, H->h[l], H->delta[l], H->S[l], H->v[l], H->d[l]);
  ora_restrict(n, H->v[l], H->Rv[l + 1]);
  ora_restrict(n, H->d[l], H->S[l + 1]); /* S^H temporarily holds R d^h */
  ora_residual(P, nc, H->h[l + 1], H->delta[l + 1], NULL, H->Rv[l + 1], H->d[l + 1]);
  for (size_t q = 0; q < mc; ++q) H->S[l + 1][q] = H->d[l + 1][q] - H->S[l + 1][q];
  memcpy(H->v[l + 1], H->Rv[l + 1], mc * sizeof(double)); /* initial guess R u^h */
  int visits = (cycle == 2) ? 2 : 1;
  for (int vi = 0; vi < visits; ++vi) mg_cycle(P, H, l + 1, nu1, nu2, cycle);
  if (cycle == 1) mg_cycle(P, H, l + 1, nu1, nu2, 0); /* F: then a V from the same level */
  /* u^h += P(u^H - R u^h) (eq:solution_correction) */
  for (size_t q = 0; q < mc; ++q) H->d[l + 1][q] = H->v[l + 1][q] - H->Rv[l + 1][q];
  ora_prolong_add(nc, H->d[l + 1], H->v[l]);
  for (int s = 0; s < nu2; ++s) ora_relax(P, n, H->h[l], H->delta[l], H->S[l], H->v[l]);
}

/* Residual at the background field per unit density contrast: the
 * coefficient of delta in each equation. */
static double bg_coef(const ora_params *P) {
  ora_consts c = consts_of(P);
  if (P->model == ORA_FR) return c.om_a;
  if (P->model == ORA_SYM) return c.s_amp * c.s_ratio * c.ubar;
  return fabs(c.cq_src);
}

/* RMS of the residual at the background field: the delta term of each
 * equation (Sec. 3.2.1 global residual, evaluated at the background). */
double ora_background_resid_rms(const ora_params *P, const double *delta) {
  size_t m = (size_t)P->n * P->n * P->n;
  const double coef = bg_coef(P);
  double s = 0.0;
  for (size_t q = 0; q < m; ++q) s += (coef * delta[q]) * (coef * delta[q]);
  return sqrt(s / (double)m);
}

/* Solve L(v) = 0 on the finest level.  v holds the initial guess on entry
 * and the solution on exit (f(R): w = -f_R; symmetron: u; CQ: phi~).
 * Returns the number of cycles; *rel receives the final relative residual,
 * hist (if not NULL) the relative residual after each cycle (<= max_cycles). */
int ora_solve(const ora_params *P, const double *delta, double *v, double tol,
              int max_cycles, int nu1, int nu2, int cycle, double *rel, double *hist) {
  ora_hier H;
  memset(&H, 0, sizeof H);
  H.nlev = ora_num_levels(P->n);
  int n = P->n;
  double h = 1.0;
  for (int l = 0; l < H.nlev; ++l) {
    size_t m = (size_t)n * n * n;
    H.n[l] = n;
    H.h[l] = h;
    H.d[l] = (double *)malloc(m * sizeof(double));
    if (l == 0) {
      H.delta[0] = (double *)delta;
      H.v[0] = v;
      H.S[0] = NULL;
    } else {
      H.delta[l] = (double *)malloc(m * sizeof(double));
      H.v[l] = (double *)malloc(m * sizeof(double));
      H.S[l] = (double *)malloc(m * sizeof(double));
      H.Rv[l] = (double *)malloc(m * sizeof(double));
      ora_restrict(2 * n, H.delta[l - 1], H.delta[l]); /* rho^H = R rho^h */
    }
    n /= 2;
    h *= 2.0;
  }
  size_t m0 = (size_t)P->n * P->n * P->n;
  /* relative residual = RMS(d) / RMS(d at the background); for delta = 0 the
   * background solves the equation and the ratio is undefined: normalise by
   * the residual of a unit contrast instead */
  double eps_bg = ora_background_resid_rms(P, delta);
  if (eps_bg == 0.0) eps_bg = bg_coef(P);
  double r = sqrt(ora_residual(P, P->n, 1.0, delta, NULL, v, NULL) / (double)m0) / eps_bg;
  int cyc = 0;
  while (r > tol && cyc < max_cycles) {
    mg_cycle(P, &H, 0, nu1, nu2, cycle);
    r = sqrt(ora_residual(P, P->n, 1.0, delta, NULL, v, NULL) / (double)m0) / eps_bg;
    if (hist) hist[cyc] = r;
    ++cyc;
    if (!isfinite(r)) break;
  }
  if (rel) *rel = r;
  hier_free(&H);
  return cyc;
}

/* ------------------------------------------------------------------ */
/* Force: g5 = -grad Phi5 by central differences (Sec. 3.1)            */
/* ------------------------------------------------------------------ */
/* Potential whose negative gradient is the fifth force, without the
 * H0/a-dot time factor:
 *   f(R)      Phi5 = -c^2 f_R / 2 = c^2 w / 2        (eq:F5_fR_codeunit)
 *   symmetron Phi5 = 3 xi^2 Om beta*^2 c^2 a*^-3 u^2  (eq:F_5_codeunit)
 *   CQ        Phi5 = beta phi~                       (eq:csf_particle_geodesic_code2) */
static double phi5(const ora_params *P, const ora_consts *c, double v) {
  if (P->model == ORA_FR) return 0.5 * c->ct2 * v;
  if (P->model == ORA_SYM)
    return 3.0 * P->xi * P->xi * P->omega_m * P->beta_star * P->beta_star * c->ct2 /
           (P->a_star * P->a_star * P->a_star) * v * v;
  return P->beta * v;
}

void ora_force(const ora_params *P, const double *v, double *force) {
  ora_consts c = consts_of(P);
  int n = P->n;
  size_t m = (size_t)n * n * n;
  double *ph = (double *)malloc(m * sizeof(double));
  for (size_t q = 0; q < m; ++q) ph[q] = phi5(P, &c, v[q]);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t id = IDX(n, i, j, k);
        force[id] = -(ph[IDX(n, WRAP(i + 1, n), j, k)] - ph[IDX(n, WRAP(i - 1, n), j, k)]) / 2.0;
        force[m + id] = -(ph[IDX(n, i, WRAP(j + 1, n), k)] - ph[IDX(n, i, WRAP(j - 1, n), k)]) / 2.0;
        force[2 * m + id] = -(ph[IDX(n, i, j, WRAP(k + 1, n))] - ph[IDX(n, i, j, WRAP(k - 1, n))]) / 2.0;
      }
  free(ph);
}

/* ------------------------------------------------------------------ */
/* CIC density assignment (Sec. 3.1)                                   */
/* ------------------------------------------------------------------ */
/* Cell c covers [c, c+1) in code units, centre c + 1/2.  A particle at x
 * gives (1-t) to floor(x-1/2) and t to floor(x-1/2)+1 on each axis, with
 * t = x - 1/2 - floor(x - 1/2), periodic.  delta = rho/mean - 1. */
void ora_cic(int n, int64_t np, const double *pos, double *delta) {
  size_t m = (size_t)n * n * n;
  memset(delta, 0, m * sizeof(double));
  for (int64_t p = 0; p < np; ++p) {
    int i0[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
      double s = pos[3 * p + a] - 0.5;
      double f = floor(s);
      t[a] = s - f;
      i0[a] = WRAP(((int)f % n + n) % n, n);
    }
    for (int dk = 0; dk < 2; ++dk)
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
          double w = (di ? t[0] : 1.0 - t[0]) * (dj ? t[1] : 1.0 - t[1]) *
                     (dk ? t[2] : 1.0 - t[2]);
          delta[IDX(n, WRAP(i0[0] + di, n), WRAP(i0[1] + dj, n), WRAP(i0[2] + dk, n))] += w;
        }
  }
  double mean = (double)np / (double)m;
  for (size_t q = 0; q < m; ++q) delta[q] = delta[q] / mean - 1.0;
}

/* CIC interpolation of a mesh field to particles, the counterpart of the
 * assignment above (same cells and weights, Sec. 3.1): grid holds ncomp
 * components of n^3 values, out[p*ncomp + c] = sum_8 w grid[c][cell]. */
void ora_interp(int n, int64_t np, const double *pos, const double *grid, int ncomp,
                double *out) {
  size_t m = (size_t)n * n * n;
  for (int64_t p = 0; p < np; ++p) {
    int i0[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
      double s = pos[3 * p + a] - 0.5;
      double f = floor(s);
      t[a] = s - f;
      i0[a] = WRAP(((int)f % n + n) % n, n);
    }
    for (int c = 0; c < ncomp; ++c) out[p * ncomp + c] = 0.0;
    for (int dk = 0; dk < 2; ++dk)
      for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
          double w = (di ? t[0] : 1.0 - t[0]) * (dj ? t[1] : 1.0 - t[1]) *
                     (dk ? t[2] : 1.0 - t[2]);
          size_t cell = IDX(n, WRAP(i0[0] + di, n), WRAP(i0[1] + dj, n), WRAP(i0[2] + dk, n));
          for (int c = 0; c < ncomp; ++c) out[p * ncomp + c] += w * grid[c * m + cell];
        }
  }
}

/* Symmetron friction term, dp~/da = -(d ln A/d phi) (d phi-bar/da) p~ (the
 * last term of eq:csf_particle_geodesic_qsa in code units, with the field's
 * time derivative taken from the background under the quasi-static
 * approximation).  With A of eq:sym_coupling_function (A ~ 1),
 * phi_* of eq:varphi_ast and phi-bar of eq:varphi_min_symm this is
 *   F_x = -9 Omega_m beta_star^2 xi^2 a^-4 (u(x_p) / u-bar) p_p,
 * u-bar = sqrt(1 - (a_star / a)^3).  eq:F_x_codeunit prints u-bar in the
 * numerator; the two differ by the factor u-bar^2 (the derivation above is
 * taken).  u is CIC-interpolated from the solved field; mom and out are
 * [np][3]. */
void ora_sym_friction(const ora_params *P, const double *u, const double *pos,
                      const double *mom, int64_t np, double *out) {
  double ratio = pow(P->a_star / P->a, 3.0);
  double coef = -9.0 * P->omega_m * P->beta_star * P->beta_star * P->xi * P->xi /
                (sqrt(1.0 - ratio) * pow(P->a, 4.0));
  for (int64_t p = 0; p < np; ++p) {
    double up;
    ora_interp(P->n, 1, pos + 3 * p, u, 1, &up);
    for (int a = 0; a < 3; ++a) out[3 * p + a] = coef * up * mom[3 * p + a];
  }
}

/* -grad phi by central differences, out [3][n^3] (x, y, z) */
void ora_gradient(int n, const double *phi, double *out) {
  size_t m = (size_t)n * n * n;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t c = IDX(n, i, j, k);
        out[c] = -0.5 * (phi[IDX(n, WRAP(i + 1, n), j, k)] - phi[IDX(n, WRAP(i - 1, n), j, k)]);
        out[m + c] = -0.5 * (phi[IDX(n, i, WRAP(j + 1, n), k)] - phi[IDX(n, i, WRAP(j - 1, n), k)]);
        out[2 * m + c] =
            -0.5 * (phi[IDX(n, i, j, WRAP(k + 1, n))] - phi[IDX(n, i, j, WRAP(k - 1, n))]);
      }
}

/* ------------------------------------------------------------------ */
/* Adjoint                                                             */
/* ------------------------------------------------------------------ */
/* The linearised operator of each model is  s * A  with
 *   A v = kap (6 v - sum_nb v)/h^2 + dg_c v,   kap > 0, dg_c >= 0,
 * s = +1 for f(R) (unknown w) and s = -1 for the symmetron and CQ.
 * dfd_c = dF_c/d delta_c.  Returns kap and s. */
static void lin_coeffs(const ora_params *P, const ora_consts *c, const double *v,
                       const double *delta, size_t m, double *dg, double *dfd,
                       double *kap, double *sgn) {
  if (P->model == ORA_FR) {
    *kap = c->ct2;
    *sgn = 1.0;
  } else if (P->model == ORA_SYM) {
    *kap = c->ct2;
    *sgn = -1.0;
  } else {
    *kap = 1.0;
    *sgn = -1.0;
  }
  for (size_t q = 0; q < m; ++q) {
    double dd = cell_op_diag(P, c, 1.0, v[q], delta[q]); /* includes 6 kap s/h^2 */
    dg[q] = *sgn * dd - 6.0 * (*kap);
    if (P->model == ORA_FR) dfd[q] = c->om_a;
    else if (P->model == ORA_SYM) dfd[q] = -c->s_amp * c->s_ratio * v[q];
    else dfd[q] = -c->cq_src * (P->cq_keep_exp ? exp(P->beta * v[q] / c->ct2) : 1.0);
  }
}

static void apply_A(int n, double h, double kap, const double *dg, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t id = IDX(n, i, j, k);
        y[id] = kap * (6.0 * x[id] - nb_sum(x, n, i, j, k)) / (h * h) + dg[id] * x[id];
      }
}

static double dot_det(size_t m, const double *a, const double *b) {
  /* fixed-order blocked sum, independent of the thread count */
  size_t nb = (m + 4095) / 4096;
  double *part = (double *)malloc(nb * sizeof(double));
#pragma omp parallel for schedule(static)
  for (size_t bI = 0; bI < nb; ++bI) {
    double s = 0.0;
    size_t e = (bI + 1) * 4096 < m ? (bI + 1) * 4096 : m;
    for (size_t q = bI * 4096; q < e; ++q) s += a[q] * b[q];
    part[bI] = s;
  }
  double s = 0.0;
  for (size_t bI = 0; bI < nb; ++bI) s += part[bI];
  free(part);
  return s;
}

/* Plain conjugate gradients on A x = b (A symmetric positive definite).
 * x holds the initial guess.  Returns iterations; *rel = ||r||/||b||. */
int ora_cg(int n, double kap, const double *dg, const double *b, double *x, double tol,
           int maxit, double *rel) {
  size_t m = (size_t)n * n * n;
  double *r = (double *)malloc(m * sizeof(double));
  double *p = (double *)malloc(m * sizeof(double));
  double *Ap = (double *)malloc(m * sizeof(double));
  apply_A(n, 1.0, kap, dg, x, Ap);
  for (size_t q = 0; q < m; ++q) { r[q] = b[q] - Ap[q]; p[q] = r[q]; }
  double bb = sqrt(dot_det(m, b, b));
  if (bb == 0.0) bb = 1.0;
  double rr = dot_det(m, r, r);
  int it = 0;
  while (sqrt(rr) / bb > tol && it < maxit) {
    apply_A(n, 1.0, kap, dg, p, Ap);
    double alpha = rr / dot_det(m, p, Ap);
    for (size_t q = 0; q < m; ++q) { x[q] += alpha * p[q]; r[q] -= alpha * Ap[q]; }
    double rn = dot_det(m, r, r);
    double beta = rn / rr;
    rr = rn;
    for (size_t q = 0; q < m; ++q) p[q] = r[q] + beta * p[q];
    ++it;
  }
  if (rel) *rel = sqrt(rr) / bb;
  free(r); free(p); free(Ap);
  return it;
}

/* Linear multigrid V-cycle for A (re-discretised on each level with the
 * restricted diagonal), red-black Gauss-Seidel smoothing. */
typedef struct {
  int nlev;
  int n[ORA_MAXLEV];
  double h[ORA_MAXLEV];
  double *dg[ORA_MAXLEV], *x[ORA_MAXLEV], *b[ORA_MAXLEV], *r[ORA_MAXLEV];
} lin_hier;

static void lin_relax(int n, double h, double kap, const double *dg, const double *b, double *x) {
  for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = (j + k + colour) & 1; i < n; i += 2) {
          size_t id = IDX(n, i, j, k);
          x[id] = (b[id] + kap * nb_sum(x, n, i, j, k) / (h * h)) /
                  (6.0 * kap / (h * h) + dg[id]);
        }
  }
}

static void lin_cycle(lin_hier *H, int l, double kap, int nu1, int nu2) {
  int n = H->n[l];
  size_t m = (size_t)n * n * n;
  if (l == H->nlev - 1) {
    /* dense solve of the coarsest level */
    double *A = (double *)calloc(m * m, sizeof(double));
    double *rhs = (double *)malloc(m * sizeof(double));
    double c = kap / (H->h[l] * H->h[l]);
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          size_t row = IDX(n, i, j, k);
          double *Ar = A + row * m;
          Ar[IDX(n, WRAP(i + 1, n), j, k)] -= c;
          Ar[IDX(n, WRAP(i - 1, n), j, k)] -= c;
          Ar[IDX(n, i, WRAP(j + 1, n), k)] -= c;
          Ar[IDX(n, i, WRAP(j - 1, n), k)] -= c;
          Ar[IDX(n, i, j, WRAP(k + 1, n))] -= c;
          Ar[IDX(n, i, j, WRAP(k - 1, n))] -= c;
          Ar[row] += 6.0 * c + H->dg[l][row];
          rhs[row] = H->b[l][row];
        }
    ora_dense_solve((int)m, A, rhs);
    memcpy(H->x[l], rhs, m * sizeof(double));
    free(A);
    free(rhs);
    return;
  }
  for (int s = 0; s < nu1; ++s) lin_relax(n, H->h[l], kap, H->dg[l], H->b[l], H->x[l]);
  apply_A(n, H->h[l], kap, H->dg[l], H->x[l], H->r[l]);
  for (size_t q = 0; q < m; ++q) H->r[l][q] = H->b[l][q] - H->r[l][q];
  int nc = H->n[l + 1];
  size_t mc = (size_t)nc * nc * nc;
  ora_restrict(n, H->r[l], H->b[l + 1]);
  memset(H->x[l + 1], 0, mc * sizeof(double));
  lin_cycle(H, l + 1, kap, nu1, nu2);
  ora_prolong_add(nc, H->x[l + 1], H->x[l]);
  for (int s = 0; s < nu2; ++s) lin_relax(n, H->h[l], kap, H->dg[l], H->b[l], H->x[l]);
}

/* Solve A x = b by linear multigrid V(nu1,nu2) cycles to ||r||/||b|| <= tol. */
int ora_lin_mg(int n0, double kap, const double *dg, const double *b, double *x, double tol,
               int maxit, double *rel) {
  lin_hier H;
  memset(&H, 0, sizeof H);
  H.nlev = ora_num_levels(n0);
  int n = n0;
  double h = 1.0;
  for (int l = 0; l < H.nlev; ++l) {
    size_t m = (size_t)n * n * n;
    H.n[l] = n;
    H.h[l] = h;
    H.r[l] = (double *)malloc(m * sizeof(double));
    if (l == 0) {
      H.dg[0] = (double *)dg;
      H.x[0] = x;
      H.b[0] = (double *)b;
    } else {
      H.dg[l] = (double *)malloc(m * sizeof(double));
      H.x[l] = (double *)malloc(m * sizeof(double));
      H.b[l] = (double *)malloc(m * sizeof(double));
      ora_restrict(2 * n, H.dg[l - 1], H.dg[l]);
    }
    n /= 2;
    h *= 2.0;
  }
  size_t m0 = (size_t)n0 * n0 * n0;
  double bb = sqrt(dot_det(m0, b, b));
  if (bb == 0.0) bb = 1.0;
  double *Ax = (double *)malloc(m0 * sizeof(double));
  apply_A(n0, 1.0, kap, dg, x, Ax);
  for (size_t q = 0; q < m0; ++q) Ax[q] = b[q] - Ax[q];
  double r = sqrt(dot_det(m0, Ax, Ax)) / bb;
  int it = 0;
  while (r > tol && it < maxit) {
    lin_cycle(&H, 0, kap, 2, 2);
    apply_A(n0, 1.0, kap, dg, x, Ax);
    for (size_t q = 0; q < m0; ++q) Ax[q] = b[q] - Ax[q];
    r = sqrt(dot_det(m0, Ax, Ax)) / bb;
    ++it;
  }
  if (rel) *rel = r;
  free(Ax);
  for (int l = 0; l < H.nlev; ++l) {
    free(H.r[l]);
    if (l > 0) { free(H.dg[l]); free(H.x[l]); free(H.b[l]); }
  }
  return it;
}

/* Gradient of a loss with respect to delta through the converged field v:
 *   F(v(delta), delta) = 0  =>  dL/ddelta = -(dF/ddelta) J^{-1} dL/dv,
 * J = dF/dv symmetric (Laplacian plus a diagonal).  grad_v is dL/dv of the
 * solved variable (w for f(R)).  solver: 0 = multigrid, 1 = CG. */
int ora_adjoint(const ora_params *P, const double *delta, const double *v,
                const double *grad_v, double *grad_delta, double tol, int solver,
                double *rel) {
  ora_consts c = consts_of(P);
  size_t m = (size_t)P->n * P->n * P->n;
  double *dg = (double *)malloc(m * sizeof(double));
  double *dfd = (double *)malloc(m * sizeof(double));
  double *b = (double *)malloc(m * sizeof(double));
  double *lam = (double *)calloc(m, sizeof(double));
  double kap, sgn;
  lin_coeffs(P, &c, v, delta, m, dg, dfd, &kap, &sgn);
  /* J lam = g  <=>  A lam = s g */
  for (size_t q = 0; q < m; ++q) b[q] = sgn * grad_v[q];
  int it = solver == 1 ? ora_cg(P->n, kap, dg, b, lam, tol, 200000, rel)
                       : ora_lin_mg(P->n, kap, dg, b, lam, tol, 500, rel);
  for (size_t q = 0; q < m; ++q) grad_delta[q] = -dfd[q] * lam[q];
  free(dg); free(dfd); free(b); free(lam);
  return it;
}

/* Apply the linearised operator J = dF/dv to x (for symmetry tests). */
void ora_apply_jacobian(const ora_params *P, const double *delta, const double *v,
                        const double *x, double *y) {
  ora_consts c = consts_of(P);
  size_t m = (size_t)P->n * P->n * P->n;
  double *dg = (double *)malloc(m * sizeof(double));
  double *dfd = (double *)malloc(m * sizeof(double));
  double kap, sgn;
  lin_coeffs(P, &c, v, delta, m, dg, dfd, &kap, &sgn);
  apply_A(P->n, 1.0, kap, dg, x, y);
  for (size_t q = 0; q < m; ++q) y[q] *= sgn;
  free(dg); free(dfd);
}

/* Transpose of the force map: given dL/dg (3 x N^3) return dL/dv (N^3). */
void ora_force_adjoint(const ora_params *P, const double *v, const double *gforce,
                       double *gv) {
  ora_consts c = consts_of(P);
  int n = P->n;
  size_t m = (size_t)n * n * n;
  /* g_a(c) = -(Phi5(c+e_a) - Phi5(c-e_a))/2  =>  dL/dPhi5(c) = (G_a(c+e_a) - G_a(c-e_a))/2 summed */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t id = IDX(n, i, j, k);
        double s = (gforce[IDX(n, WRAP(i + 1, n), j, k)] - gforce[IDX(n, WRAP(i - 1, n), j, k)]) +
                   (gforce[m + IDX(n, i, WRAP(j + 1, n), k)] - gforce[m + IDX(n, i, WRAP(j - 1, n), k)]) +
                   (gforce[2 * m + IDX(n, i, j, WRAP(k + 1, n))] - gforce[2 * m + IDX(n, i, j, WRAP(k - 1, n))]);
        s *= 0.5;
        /* dPhi5/dv */
        double dphi;
        if (P->model == ORA_FR) dphi = 0.5 * c.ct2;
        else if (P->model == ORA_SYM)
          dphi = 2.0 * v[id] * 3.0 * P->xi * P->xi * P->omega_m * P->beta_star * P->beta_star *
                 c.ct2 / (P->a_star * P->a_star * P->a_star);
        else dphi = P->beta;
        gv[id] = s * dphi;
      }
}

/* Vectorised root entry points for the pin tests. */
void ora_cubic_root_vec(int64_t m, const double *p, const double *q, double *out) {
  for (int64_t i = 0; i < m; ++i) out[i] = ora_cubic_root(p[i], q[i]);
}
void ora_fr_root_vec(int n, int64_t m, const double *p, const double *q, double *out) {
  for (int64_t i = 0; i < m; ++i) out[i] = ora_fr_root(n, p[i], q[i]);
}
