/*
 * hgks_oracle.c -- TEST INFRASTRUCTURE ONLY (see hgks_oracle.h).
 *
 * A plain, slow FP64 CPU implementation of what the HIP library computes, written
 * from the paper (Mu et al., arXiv 2304.05572) step by step in its order and notation:
 *   Sec. 2.1  BGK model, Maxwellian g, moments <.>, Eq. (equ6)/(equ10) interface solution,
 *             time-integrated flux Eq. (equ12)
 *   Sec. 2.2  two-stage fourth-order (S2O4) time marching
 *   Sec. 2.3  hybrid WENO5-AO reconstruction: troubled-cell indicator Steps 1-4, linear upwind
 *             Step 5, WENO-AO(5,3) in characteristic variables, equilibrium state Eq. (equ46)-(equ47),
 *             2D dimension-by-dimension reconstruction at two Gauss points
 *   Sec. 3    collision time, CFL time step, boundary conditions of the tests
 * It deliberately uses generic machinery (reconstruction polynomials fitted from cell averages,
 * moments integrated term by term from explicitly expanded integrands, 4x4 linear solves) rather
 * than the pre-expanded coefficient formulas of the HIP kernels, so that the two share nothing
 * but the definitions. Where the paper is silent or garbled the readings are the ones listed in
 * the design notes (troubled-cell threshold in normalised units, perpendicular cell flag for the
 * tangential step, u<0 in the second half-space integral, g_l paired with H(u), ...).
 *
 * The troubled-cell discriminant is evaluated with one fixed expression tree and no floating
 * point contraction (build with -ffp-contract=off), because that decision must come out the same,
 * bit for bit, on the GPU.
 */
#include "hgks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 4    /* ghost layers: the widened flag of the first ghost cell needs 4 cells */
#define MAXC 4  /* conserved variables in 2D */

/* ======================================================================== */
/* 1. Reconstruction polynomials in the normalised coordinate xi=(x-x_i)/dx  */
/* ======================================================================== */

static double ipow(double x, int m) {
  double r = 1.0;
  for (int i = 0; i < m; ++i) r *= x;
  return r;
}

/* Average of xi^m over cell j, i.e. over [j-1/2, j+1/2]. */
static double cell_avg_monomial(int j, int m) {
  return (ipow(j + 0.5, m + 1) - ipow(j - 0.5, m + 1)) / (double)(m + 1);
}

/* Solve A x = b (n <= 6) by Gaussian elimination with partial pivoting. */
static void lin_solve(int n, const double* Ain, const double* bin, double* x) {
  double A[6][7];
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) A[r][c] = Ain[r * n + c];
    A[r][n] = bin[r];
  }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c <= n; ++c) {
        double t = A[col][c];
        A[col][c] = A[piv][c];
        A[piv][c] = t;
      }
    for (int r = col + 1; r < n; ++r) {
      double f = A[r][col] / A[col][col];
      for (int c = col; c <= n; ++c) A[r][c] -= f * A[col][c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = A[r][n];
    for (int c = r + 1; c < n; ++c) s -= A[r][c] * x[c];
    x[r] = s / A[r][r];
  }
}

static void mat_inverse(int n, const double* A, double* Ainv) {
  double e[6], col[6];
  for (int c = 0; c < n; ++c) {
    for (int r = 0; r < n; ++r) e[r] = (r == c) ? 1.0 : 0.0;
    lin_solve(n, A, e, col);
    for (int r = 0; r < n; ++r) Ainv[r * n + c] = col[r];
  }
}

/* Stencils (Sec. 2.3.1): S0={i-2,i-1,i}, S1={i-1,i,i+1}, S2={i,i+1,i+2} (quadratics p_k^{r3})
 * and S3={i-2..i+2} (quartic p_3^{r5}). Each polynomial is fixed by matching the cell averages. */
static const int g_off[4][5] = {{-2, -1, 0, 0, 0}, {-1, 0, 1, 0, 0}, {0, 1, 2, 0, 0}, {-2, -1, 0, 1, 2}};
static const int g_npts[4] = {3, 3, 3, 5};
static const int g_first[4] = {0, 1, 2, 0}; /* position in the 5-cell window of the first cell */
static double g_fit[4][25];                 /* polynomial coefficients = g_fit * cell averages */
static int g_ready = 0;

static void oracle_init(void) {
  if (g_ready) return;
  for (int k = 0; k < 4; ++k) {
    int n = g_npts[k];
    double A[25];
    for (int r = 0; r < n; ++r)
      for (int m = 0; m < n; ++m) A[r * n + m] = cell_avg_monomial(g_off[k][r], m);
    mat_inverse(n, A, g_fit[k]);
  }
  g_ready = 1;
}

/* Coefficients c[0..deg] of stencil polynomial k from the five-cell window q[0..4]. */
static void stencil_coeffs(int k, const double* q, double* c) {
  int n = g_npts[k];
  for (int m = 0; m < n; ++m) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += g_fit[k][m * n + r] * q[g_first[k] + r];
    c[m] = s;
  }
}

static void poly_eval(const double* c, int deg, double xi, double* val, double* der) {
  double v = 0.0, d = 0.0;
  for (int m = deg; m >= 0; --m) v = v * xi + c[m];
  for (int m = deg; m >= 1; --m) d = d * xi + m * c[m];
  *val = v;
  *der = d;
}

/* Smoothness indicator: sum over q of  dx^(2q-1) * integral over the cell of (d^q p/dx^q)^2, which in
 * the normalised coordinate is sum_q integral_{-1/2}^{1/2} (d^q p/dxi^q)^2 dxi. */
static double beta_of(const double* c, int deg) {
  double b = 0.0;
  for (int q = 1; q <= deg; ++q) {
    double d[5] = {0}, sq[9] = {0};
    int dd = deg - q;
    for (int m = 0; m <= dd; ++m) {
      double f = 1.0;
      for (int s = m + 1; s <= m + q; ++s) f *= s;
      d[m] = c[m + q] * f;
    }
    for (int a = 0; a <= dd; ++a)
      for (int e = 0; e <= dd; ++e) sq[a + e] += d[a] * d[e];
    for (int m = 0; m <= 2 * dd; ++m) b += sq[m] * (ipow(0.5, m + 1) - ipow(-0.5, m + 1)) / (m + 1);
  }
  return b;
}

/* WENO-AO(5,3) of the five cell averages q at xi: value and xi-derivative. The same normalised
 * weights serve the value and the derivative (the derivative is that of the same polynomial). */
static void ao_eval(const double* q, double xi, double ghi, double glo, double eps, double* val,
                    double* der) {
  double c[5], pv[4], pd[4], beta[4], gam[4], w[4], sw = 0.0;
  for (int k = 0; k < 4; ++k) {
    int deg = g_npts[k] - 1;
    stencil_coeffs(k, q, c);
    poly_eval(c, deg, xi, &pv[k], &pd[k]);
    beta[k] = beta_of(c, deg);
  }
  gam[3] = ghi;
  gam[0] = (1.0 - ghi) * (1.0 - glo) / 2.0;
  gam[2] = gam[0];
  gam[1] = (1.0 - ghi) * glo;
  double delta = (fabs(beta[3] - beta[0]) + fabs(beta[3] - beta[1]) + fabs(beta[3] - beta[2])) / 3.0;
  for (int k = 0; k < 4; ++k) {
    w[k] = gam[k] * (1.0 + delta / (beta[k] + eps));
    sw += w[k];
  }
  double v = pv[3], d = pd[3];
  for (int k = 0; k < 3; ++k) {
    v -= gam[k] * pv[k];
    d -= gam[k] * pd[k];
  }
  v *= (w[3] / sw) / gam[3];
  d *= (w[3] / sw) / gam[3];
  for (int k = 0; k < 3; ++k) {
    v += (w[k] / sw) * pv[k];
    d += (w[k] / sw) * pd[k];
  }
  *val = v;
  *der = d;
}

/* ======================================================================== */
/* 2. Troubled-cell indicator (Sec. 2.3.1, Steps 1-4)                        */
/* ======================================================================== */

/* Returns 1 if the cell is troubled for this component. q: cells i-2..i+2; h: cell size.
 * D1 = 10*a1*dx and D2 = 34*a2*dx^2 are the least-squares quadratic's coefficients in
 * normalised units; Step 1 compares |2 a2| with zeta1 = (5/17) h in normalised units. */
static int troubled_component(const double* q, double h, int zeta1_mode, double* xbar_out,
                              double* xhat_out, int* step_out) {
  double Qm2 = q[0], Qm1 = q[1], Q0 = q[2], Qp1 = q[3], Qp2 = q[4];
  double D1 = (Qp1 - Qm1) + 2.0 * (Qp2 - Qm2);
  double D2 = (4.0 * (Qm2 + Qp2) + (Qm1 + Qp1)) - 10.0 * Q0;
  double thr = (zeta1_mode == 0) ? 5.0 * h : 5.0 * h * h * h;
  *xbar_out = NAN;
  *xhat_out = NAN;
  if (fabs(D2) <= thr) { *step_out = 1; return 0; }
  double xbar = -(17.0 * D1) / (10.0 * D2); /* extreme point of the least-squares quadratic */
  *xbar_out = xbar;
  if (fabs(xbar) > 2.5) { *step_out = 2; return 0; }
  double a1h = 0.5 * (Qp1 - Qm1);           /* conservative quadratic on {i-1,i,i+1} */
  double a2h = 0.5 * ((Qm1 + Qp1) - 2.0 * Q0);
  double den = 2.0 * a2h + (a2h == 0.0 ? 1e-30 : 0.0);
  double xhat = -a1h / den;
  *xhat_out = xhat;
  *step_out = 3;
  if (fabs(xbar - xhat) <= 0.25) return 0;
  return 1;
}

/* ======================================================================== */
/* 3. Characteristic matrices                                               */
/* ======================================================================== */

/* Right eigenvectors of the Euler flux Jacobian in direction dir (1: first velocity component,
 * 2: second), columns ordered by eigenvalue u_n - c, u_n (entropy), [u_n (shear)], u_n + c. */
static void char_R(int dim, int dir, const double* W, double gamma, double* R) {
  int nc = dim + 2;
  double rho = W[0];
  double u[2] = {W[1] / rho, dim == 2 ? W[2] / rho : 0.0};
  double E = W[nc - 1];
  double q2 = u[0] * u[0] + u[1] * u[1];
  double p = (gamma - 1.0) * (E - 0.5 * rho * q2);
  double c = sqrt(gamma * p / rho);
  double H = (E + p) / rho;
  double un = u[dir - 1];
  memset(R, 0, sizeof(double) * nc * nc);
  int last = nc - 1;
  /* column 0: u_n - c */
  R[0 * nc + 0] = 1.0;
  for (int d = 0; d < dim; ++d) R[(1 + d) * nc + 0] = u[d] - (d == dir - 1 ? c : 0.0);
  R[last * nc + 0] = H - un * c;
  /* column 1: entropy wave */
  R[0 * nc + 1] = 1.0;
  for (int d = 0; d < dim; ++d) R[(1 + d) * nc + 1] = u[d];
  R[last * nc + 1] = 0.5 * q2;
  if (dim == 2) {
    /* column 2: shear wave */
    int t = (dir == 1) ? 2 : 1; /* row of the tangential momentum */
    R[t * nc + 2] = 1.0;
    R[last * nc + 2] = u[t - 1];
  }
  /* last column: u_n + c */
  R[0 * nc + last] = 1.0;
  for (int d = 0; d < dim; ++d) R[(1 + d) * nc + last] = u[d] + (d == dir - 1 ? c : 0.0);
  R[last * nc + last] = H + un * c;
}

/* ======================================================================== */
/* 4. One-sided hybrid reconstruction of a vector of conserved variables     */
/* ======================================================================== */

typedef struct {
  int dim, nc;
  double gamma, K, mu, Pr, c1, c2;
  int ns;
  double ghi, glo, eps;
  int recon, zeta1_mode, positivity;
  int tfm;  /* tangential flag: 0 the side cell's flag, 1 the indicator on the line values */
  int csm;  /* tangential characteristic state: 0 own side, 1 mean of both sides */
} params;

/* q5[r][c]: the side's five cells (offsets -2..2), xi: evaluation point. Unflagged: component-wise
 * linear quartic (Step 5). Flagged: WENO-AO on U = R^{-1} Q, then back-projection with R. */
static void recon_side(const params* pp, const double q5[5][MAXC], double xi, int flag,
                       const double* R, const double* L, double* val, double* der) {
  int nc = pp->nc;
  double q[5], c[5];
  if (!flag) {
    for (int cc = 0; cc < nc; ++cc) {
      for (int r = 0; r < 5; ++r) q[r] = q5[r][cc];
      stencil_coeffs(3, q, c);
      poly_eval(c, 4, xi, &val[cc], &der[cc]);
    }
    return;
  }
  double cv[MAXC], cd[MAXC];
  for (int k = 0; k < nc; ++k) {
    for (int r = 0; r < 5; ++r) {
      double s = 0.0;
      for (int cc = 0; cc < nc; ++cc) s += L[k * nc + cc] * q5[r][cc];
      q[r] = s;
    }
    ao_eval(q, xi, pp->ghi, pp->glo, pp->eps, &cv[k], &cd[k]);
  }
  for (int cc = 0; cc < nc; ++cc) {
    double sv = 0.0, sd = 0.0;
    for (int k = 0; k < nc; ++k) {
      sv += R[cc * nc + k] * cv[k];
      sd += R[cc * nc + k] * cd[k];
    }
    val[cc] = sv;
    der[cc] = sd;
  }
}

/* ======================================================================== */
/* 5. Kinetic part: Maxwellian moments and the gas-kinetic flux (Sec. 2.1)   */
/* ======================================================================== */

#define NMOM 12
typedef struct {
  double rho, U, V, lam;
  double Mu[NMOM]; /* <u^n> over all u */
  double Mh[NMOM]; /* <u^n> over u>0 (side +1) or u<0 (side -1) */
  double Mv[NMOM]; /* <v^n> */
  double Mx[4];    /* <(xi^2)^n> over the K internal degrees of freedom */
} maxw;

/* Moments of the normalised Maxwellian (rho = 1) of a Gaussian in u with mean U and variance
 * 1/(2 lam): integration by parts gives <u^(n+2)> = U <u^(n+1)> + (n+1)/(2 lam) <u^n>, the same
 * recurrence on a half line because the boundary term at u = 0 vanishes for n >= 0. */
static void maxw_moments(double U, double V, double lam, double K, int side, maxw* g) {
  g->Mu[0] = 1.0;
  g->Mu[1] = U;
  g->Mv[0] = 1.0;
  g->Mv[1] = V;
  for (int n = 0; n + 2 < NMOM; ++n) {
    g->Mu[n + 2] = U * g->Mu[n + 1] + (n + 1) / (2.0 * lam) * g->Mu[n];
    g->Mv[n + 2] = V * g->Mv[n + 1] + (n + 1) / (2.0 * lam) * g->Mv[n];
  }
  if (side != 0) {
    double s = (double)side;
    g->Mh[0] = 0.5 * erfc(-s * sqrt(lam) * U);
    g->Mh[1] = U * g->Mh[0] + s * exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    for (int n = 0; n + 2 < NMOM; ++n)
      g->Mh[n + 2] = U * g->Mh[n + 1] + (n + 1) / (2.0 * lam) * g->Mh[n];
  } else {
    for (int n = 0; n < NMOM; ++n) g->Mh[n] = NAN;
  }
  /* xi^2 = sum of K squared Gaussians of variance 1/(2 lam): chi-square moments */
  g->Mx[0] = 1.0;
  g->Mx[1] = K / (2.0 * lam);
  g->Mx[2] = K * (K + 2.0) / (4.0 * lam * lam);
  g->Mx[3] = K * (K + 2.0) * (K + 4.0) / (8.0 * lam * lam * lam);
}

static void maxw_from_W(const params* pp, const double* W, int side, maxw* g) {
  int nc = pp->nc;
  double rho = W[0];
  double U = W[1] / rho;
  double V = pp->dim == 2 ? W[2] / rho : 0.0;
  double p = (pp->gamma - 1.0) * (W[nc - 1] - 0.5 * rho * (U * U + V * V));
  g->rho = rho;
  g->U = U;
  g->V = V;
  g->lam = rho / (2.0 * p);
  maxw_moments(U, V, g->lam, pp->K, side, g);
}

/* Polynomials in (u, v, xi^2) as explicit term lists: coef * u^i * v^j * (xi^2)^k. */
typedef struct {
  double c;
  int i, j, k;
} term;
#define MAXT 64
typedef struct {
  int n;
  term t[MAXT];
} poly;

static void p_set(poly* p, int n, const term* t) {
  p->n = n;
  for (int s = 0; s < n; ++s) p->t[s] = t[s];
}
static void p_push(poly* p, double c, int i, int j, int k) {
  p->t[p->n].c = c;
  p->t[p->n].i = i;
  p->t[p->n].j = j;
  p->t[p->n].k = k;
  p->n++;
}

/* psi_alpha: (1, u, v, (u^2+v^2+xi^2)/2) in 2D, (1, u, (u^2+xi^2)/2) in 1D. */
static void psi_poly(const params* pp, int alpha, poly* p) {
  p->n = 0;
  if (alpha == 0) p_push(p, 1.0, 0, 0, 0);
  else if (alpha == 1) p_push(p, 1.0, 1, 0, 0);
  else if (alpha == 2 && pp->dim == 2) p_push(p, 1.0, 0, 1, 0);
  else {
    p_push(p, 0.5, 2, 0, 0);
    if (pp->dim == 2) p_push(p, 0.5, 0, 2, 0);
    p_push(p, 0.5, 0, 0, 1);
  }
}

/* The microscopic slope a = a_1 + a_2 u (+ a_3 v) + a_last (u^2 (+v^2) + xi^2)/2, i.e. a . psi. */
static void a_poly(const params* pp, const double* a, poly* p) {
  poly ps;
  p->n = 0;
  for (int al = 0; al < pp->nc; ++al) {
    psi_poly(pp, al, &ps);
    for (int s = 0; s < ps.n; ++s) p_push(p, a[al] * ps.t[s].c, ps.t[s].i, ps.t[s].j, ps.t[s].k);
  }
}

static double mom(const maxw* g, int half, int i, int j, int k) {
  return (half ? g->Mh[i] : g->Mu[i]) * g->Mv[j] * g->Mx[k];
}

/* out[alpha] = < A * B * psi_alpha > for the normalised Maxwellian g (half: over the half line). */
static void momvec(const params* pp, const poly* A, const poly* B, const maxw* g, int half,
                   double* out) {
  poly ps;
  for (int al = 0; al < pp->nc; ++al) {
    psi_poly(pp, al, &ps);
    double s = 0.0;
    for (int a = 0; a < A->n; ++a)
      for (int b = 0; b < B->n; ++b)
        for (int r = 0; r < ps.n; ++r)
          s += A->t[a].c * B->t[b].c * ps.t[r].c *
               mom(g, half, A->t[a].i + B->t[b].i + ps.t[r].i, A->t[a].j + B->t[b].j + ps.t[r].j,
                   A->t[a].k + B->t[b].k + ps.t[r].k);
    out[al] = s;
  }
}

/* scalar < A * B * C > */
static double mom3(const poly* A, const poly* B, const poly* C, const maxw* g, int half) {
  double s = 0.0;
  for (int a = 0; a < A->n; ++a)
    for (int b = 0; b < B->n; ++b)
      for (int r = 0; r < C->n; ++r)
        s += A->t[a].c * B->t[b].c * C->t[r].c *
             mom(g, half, A->t[a].i + B->t[b].i + C->t[r].i, A->t[a].j + B->t[b].j + C->t[r].j,
                 A->t[a].k + B->t[b].k + C->t[r].k);
  return s;
}

static const term T_ONE = {1.0, 0, 0, 0};
static const term T_U = {1.0, 1, 0, 0};
static const term T_V = {1.0, 0, 1, 0};
static const term T_UU = {1.0, 2, 0, 0};
static const term T_UV = {1.0, 1, 1, 0};

/* Solve <a psi> = b for the coefficients of a (the relation between a microscopic slope and the
 * macroscopic one, Sec. 2.1), with the 'mass matrix' <psi_alpha psi_beta> of g. */
static void solve_slope(const params* pp, const maxw* g, const double* b, double* a) {
  int nc = pp->nc;
  double M[16], colv[MAXC];
  poly one, ps;
  p_set(&one, 1, &T_ONE);
  for (int be = 0; be < nc; ++be) {
    psi_poly(pp, be, &ps);
    momvec(pp, &ps, &one, g, 0, colv);
    for (int al = 0; al < nc; ++al) M[al * nc + be] = colv[al];
  }
  lin_solve(nc, M, b, a);
}

/* Time integrals over [0, delta] of the coefficient functions of Eq. (equ10):
 *   C1: 1 - e^{-t/tau}                 (g0)
 *   C2: (t + tau) e^{-t/tau} - tau     (g0 (a1 u + a2 v))
 *   C3: t - tau + tau e^{-t/tau}       (g0 A)
 *   C4: e^{-t/tau}                     (g_k, and -tau g_k A^k)
 *   C5: (t + tau) e^{-t/tau}           (-g_k (a1^k u + a2^k v))
 * tau = 0 is the limit; for delta/tau < 1 the Taylor series of the same integrals is summed
 * because the closed forms cancel there. */
static void time_coeffs(double d, double tau, double* C) {
  if (tau == 0.0) {
    C[0] = d;
    C[1] = 0.0;
    C[2] = 0.5 * d * d;
    C[3] = 0.0;
    C[4] = 0.0;
    return;
  }
  double x = d / tau;
  if (x < 1.0) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, term_k = 1.0;
    for (int k = 1; k <= 40; ++k) {
      term_k *= x / k; /* x^k / k! */
      double sg = (k % 2 == 0) ? 1.0 : -1.0; /* (-1)^k */
      if (k >= 2) s1 += sg * term_k;
      if (k >= 3) {
        s2 += sg * (k - 2) * term_k;
        s3 -= sg * term_k;
      }
      s4 -= sg * term_k;
    }
    C[0] = tau * s1;
    C[1] = tau * tau * s2;
    C[2] = tau * tau * s3;
    C[3] = tau * s4;
    C[4] = tau * tau * (x + s2);
    return;
  }
  double E = exp(-x);
  C[0] = d - tau * (1.0 - E);
  C[1] = 2.0 * tau * tau - tau * d - tau * (d + 2.0 * tau) * E;
  C[2] = 0.5 * d * d - tau * d + tau * tau * (1.0 - E);
  C[3] = tau * (1.0 - E);
  C[4] = 2.0 * tau * tau - tau * (2.0 * tau + d) * E;
}

/* Gas-kinetic flux at one Gauss point: time-integrated fluxes F(W, dt) and F(W, dt/2) of
 * Eq. (equ12) with the interface distribution of Eq. (equ10). Inputs are the reconstructed
 * non-equilibrium states W^{l,r} and their normal (x) and tangential (y) derivatives. */
static void gp_flux(const params* pp, const double* Wl, const double* Wxl, const double* Wyl,
                    const double* Wr, const double* Wxr, const double* Wyr, double dt, double* Fd,
                    double* Fh, double* tau_out) {
  int nc = pp->nc, dim = pp->dim;
  maxw gs[2];
  const double* Ws[2] = {Wl, Wr};
  const double* Wxs[2] = {Wxl, Wxr};
  const double* Wys[2] = {Wyl, Wyr};
  double ax[2][MAXC], ay[2][MAXC], A[2][MAXC];
  poly one, pu, pv, puu, puv, pax, pay, pA;
  p_set(&one, 1, &T_ONE);
  p_set(&pu, 1, &T_U);
  p_set(&pv, 1, &T_V);
  p_set(&puu, 1, &T_UU);
  p_set(&puv, 1, &T_UV);

  double Wc[MAXC] = {0}, Wxc[MAXC] = {0}, Wyc[MAXC] = {0};
  double M4a[MAXC] = {0}, M4b[MAXC] = {0}, M5[MAXC] = {0};
  double tmp[MAXC], tmp2[MAXC], b[MAXC];
  for (int s = 0; s < 2; ++s) {
    int side = (s == 0) ? +1 : -1; /* g_l over u>0, g_r over u<0 */
    maxw_from_W(pp, Ws[s], side, &gs[s]);
    const maxw* g = &gs[s];
    for (int al = 0; al < nc; ++al) b[al] = Wxs[s][al] / g->rho;
    solve_slope(pp, g, b, ax[s]);
    for (int al = 0; al < nc; ++al) b[al] = (dim == 2 ? Wys[s][al] : 0.0) / g->rho;
    solve_slope(pp, g, b, ay[s]);
    /* compatibility of the initial distribution: <a1 u + a2 v + A> = 0 */
    a_poly(pp, ax[s], &pax);
    a_poly(pp, ay[s], &pay);
    momvec(pp, &pax, &pu, g, 0, tmp);
    momvec(pp, &pay, &pv, g, 0, tmp2);
    for (int al = 0; al < nc; ++al) b[al] = -(tmp[al] + tmp2[al]);
    solve_slope(pp, g, b, A[s]);
    a_poly(pp, A[s], &pA);
    /* equilibrium state and its slopes, Eq. (equ46)-(equ47) */
    momvec(pp, &one, &one, g, 1, tmp);
    for (int al = 0; al < nc; ++al) Wc[al] += g->rho * tmp[al];
    momvec(pp, &pax, &one, g, 1, tmp);
    for (int al = 0; al < nc; ++al) Wxc[al] += g->rho * tmp[al];
    momvec(pp, &pay, &one, g, 1, tmp);
    for (int al = 0; al < nc; ++al) Wyc[al] += g->rho * tmp[al];
    /* free-transport terms of Eq. (equ10) */
    momvec(pp, &one, &pu, g, 1, tmp);
    for (int al = 0; al < nc; ++al) M4a[al] += g->rho * tmp[al];
    momvec(pp, &pA, &pu, g, 1, tmp);
    for (int al = 0; al < nc; ++al) M4b[al] += g->rho * tmp[al];
    momvec(pp, &pax, &puu, g, 1, tmp);
    momvec(pp, &pay, &puv, g, 1, tmp2);
    for (int al = 0; al < nc; ++al) M5[al] += g->rho * (tmp[al] + tmp2[al]);
  }
  /* equilibrium g0 at the interface */
  maxw g0;
  maxw_from_W(pp, Wc, 0, &g0);
  /* interface vacuum: two physical sides (positive, finite pressures; a non-physical side leaves NaN
   * moments and is reported as such) whose half-space integrals leave an interface density below the
   * unit roundoff of the smaller side density and no equilibrium (temperature not positive and finite)
   * give a face without flux. Two states separating at many thermal speeds reach this where the
   * integrals underflow; every term carries a factor of those vanishing integrals, so zero is their
   * limit. An interface density above that bound without an equilibrium is left to give NaN. */
  {
    const double psl = gs[0].rho / (2.0 * gs[0].lam), psr = gs[1].rho / (2.0 * gs[1].lam);
    const double rmin = fmin(gs[0].rho, gs[1].rho);
    if (psl > 0.0 && psl < INFINITY && psr > 0.0 && psr < INFINITY && g0.rho <= 0x1p-53 * rmin &&
        !(g0.rho > 0.0 && g0.lam > 0.0 && g0.lam < INFINITY)) {
      for (int al = 0; al < nc; ++al) Fd[al] = Fh[al] = 0.0;
      if (tau_out) *tau_out = 0.0;
      return;
    }
  }
  double a0[MAXC], b0[MAXC], A0[MAXC];
  for (int al = 0; al < nc; ++al) b[al] = Wxc[al] / g0.rho;
  solve_slope(pp, &g0, b, a0);
  for (int al = 0; al < nc; ++al) b[al] = Wyc[al] / g0.rho;
  solve_slope(pp, &g0, b, b0);
  poly pa0, pb0, pA0;
  a_poly(pp, a0, &pa0);
  a_poly(pp, b0, &pb0);
  momvec(pp, &pa0, &pu, &g0, 0, tmp);
  momvec(pp, &pb0, &pv, &g0, 0, tmp2);
  for (int al = 0; al < nc; ++al) b[al] = -(tmp[al] + tmp2[al]);
  solve_slope(pp, &g0, b, A0);
  a_poly(pp, A0, &pA0);
  double M1[MAXC], M2[MAXC], M3[MAXC];
  momvec(pp, &one, &pu, &g0, 0, M1);
  momvec(pp, &pa0, &puu, &g0, 0, tmp);
  momvec(pp, &pb0, &puv, &g0, 0, tmp2);
  for (int al = 0; al < nc; ++al) {
    M1[al] *= g0.rho;
    M2[al] = g0.rho * (tmp[al] + tmp2[al]);
  }
  momvec(pp, &pA0, &pu, &g0, 0, M3);
  for (int al = 0; al < nc; ++al) M3[al] *= g0.rho;

  /* collision time (Sec. 3): pressures of the reconstructed states at this point */
  double pl = gs[0].rho / (2.0 * gs[0].lam), pr = gs[1].rho / (2.0 * gs[1].lam);
  double p0 = g0.rho / (2.0 * g0.lam);
  double jump = fabs((pl - pr) / (pl + pr));
  double tau = pp->ns ? pp->mu / p0 + pp->c2 * jump * dt : pp->c1 * dt + pp->c2 * jump * dt;
  if (tau_out) *tau_out = tau;

  /* heat-flux moments for the Prandtl-number correction (Navier-Stokes, Pr != 1) */
  int prfix = pp->ns && pp->Pr != 1.0;
  double Q1 = 0, Q2 = 0, Q3 = 0, Q4a = 0, Q4b = 0, Q5 = 0;
  if (prfix) {
    /* Q = (u-U0) ((u-U0)^2 + (v-V0)^2 + xi^2) / 2, expanded */
    double U0 = g0.U, V0 = g0.V;
    poly Q;
    Q.n = 0;
    /* (u-U0)^3 / 2 */
    p_push(&Q, 0.5, 3, 0, 0);
    p_push(&Q, -1.5 * U0, 2, 0, 0);
    p_push(&Q, 1.5 * U0 * U0, 1, 0, 0);
    p_push(&Q, -0.5 * U0 * U0 * U0, 0, 0, 0);
    if (dim == 2) { /* (u-U0)(v-V0)^2 / 2 */
      p_push(&Q, 0.5, 1, 2, 0);
      p_push(&Q, -V0, 1, 1, 0);
      p_push(&Q, 0.5 * V0 * V0, 1, 0, 0);
      p_push(&Q, -0.5 * U0, 0, 2, 0);
      p_push(&Q, U0 * V0, 0, 1, 0);
      p_push(&Q, -0.5 * U0 * V0 * V0, 0, 0, 0);
    }
    p_push(&Q, 0.5, 1, 0, 1); /* (u-U0) xi^2 / 2 */
    p_push(&Q, -0.5 * U0, 0, 0, 1);
    Q1 = g0.rho * mom3(&Q, &one, &one, &g0, 0);
    Q2 = g0.rho * (mom3(&Q, &pa0, &pu, &g0, 0) + mom3(&Q, &pb0, &pv, &g0, 0));
    Q3 = g0.rho * mom3(&Q, &pA0, &one, &g0, 0);
    for (int s = 0; s < 2; ++s) {
      const maxw* g = &gs[s];
      a_poly(pp, ax[s], &pax);
      a_poly(pp, ay[s], &pay);
      a_poly(pp, A[s], &pA);
      Q4a += g->rho * mom3(&Q, &one, &one, g, 1);
      Q4b += g->rho * mom3(&Q, &pA, &one, g, 1);
      Q5 += g->rho * (mom3(&Q, &pax, &pu, g, 1) + mom3(&Q, &pay, &pv, g, 1));
    }
  }

  double deltas[2] = {dt, 0.5 * dt};
  double* outs[2] = {Fd, Fh};
  for (int m = 0; m < 2; ++m) {
    double C[5];
    time_coeffs(deltas[m], tau, C);
    for (int al = 0; al < nc; ++al)
      outs[m][al] = C[0] * M1[al] + C[1] * M2[al] + C[2] * M3[al] + C[3] * (M4a[al] - tau * M4b[al]) -
                    C[4] * M5[al];
    if (prfix) {
      double q = C[0] * Q1 + C[1] * Q2 + C[2] * Q3 + C[3] * (Q4a - tau * Q4b) - C[4] * Q5;
      outs[m][nc - 1] += (1.0 / pp->Pr - 1.0) * q;
    }
  }
}

/* ======================================================================== */
/* 6. Grid, ghost cells, flags, directional sweeps, S2O4                     */
/* ======================================================================== */

static void make_params(const oracle_problem* p, params* pp) {
  pp->dim = p->dim;
  pp->nc = p->dim + 2;
  pp->gamma = p->gamma;
  /* internal degrees of freedom: K + 2 = 2/(gamma-1) in 2D, K + 1 = 2/(gamma-1) in 1D */
  pp->K = (p->dim == 2) ? (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0) : (3.0 - p->gamma) / (p->gamma - 1.0);
  pp->mu = p->mu;
  pp->Pr = p->Pr;
  pp->c1 = p->c1;
  pp->c2 = p->c2;
  pp->ns = (p->eqn == 1);
  pp->ghi = p->gamma_hi;
  pp->glo = p->gamma_lo;
  pp->eps = p->weno_eps;
  pp->recon = p->recon;
  pp->zeta1_mode = p->zeta1_mode;
  pp->positivity = p->positivity;
  pp->tfm = p->tangential_flag_mode;
  pp->csm = p->char_state_mode;
}

static int check_problem(const oracle_problem* p) {
  if (p->dim != 1 && p->dim != 2) return ORACLE_EINVAL;
  if (p->nx < 5 || (p->dim == 2 && p->ny < 5) || (p->dim == 1 && p->ny != 1)) return ORACLE_EINVAL;
  if (!(p->gamma > 1.0) || !(p->x1 > p->x0) || (p->dim == 2 && !(p->y1 > p->y0))) return ORACLE_EINVAL;
  if (p->eqn == 1 && !(p->Pr > 0.0 && p->mu >= 0.0)) return ORACLE_EINVAL;
  if (p->positivity != 0 && p->positivity != 1) return ORACLE_EINVAL;
  if (p->tangential_flag_mode != 0 && !(p->dim == 2 && p->tangential_flag_mode == 1)) return ORACLE_EINVAL;
  if (p->char_state_mode != 0 && !(p->dim == 2 && p->char_state_mode == 1)) return ORACLE_EINVAL;
  if (p->viscous_dt_mode != 0 && p->viscous_dt_mode != 1) return ORACLE_EINVAL;
  int nb = p->dim == 2 ? 4 : 2;
  for (int s = 0; s < nb; ++s) {
    if (p->bc[s] < 0 || p->bc[s] > 4) return ORACLE_EINVAL;
    if (p->bc[s] == 4) {
      const oracle_bc_data* d = &p->bcd[s];
      if (d->rest < 1 || d->rest > 4) return ORACLE_EINVAL;
      if (isnan(d->s0) || !isfinite(d->sn) || !isfinite(d->st)) return ORACLE_EINVAL;
      for (int k = 0; k < (d->rest == 4 ? 2 : 1); ++k) {
        const double* q = k ? d->b : d->a;
        double mv = (p->dim == 2) ? q[2] : 0.0;
        double pr = (p->gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + mv * mv) / q[0]);
        if (!(q[0] > 0.0) || !(pr > 0.0) || !isfinite(q[3]) || !isfinite(q[1]) || !isfinite(mv))
          return ORACLE_EINVAL;
      }
    }
  }
  for (int s = 0; s < nb; s += 2)
    if ((p->bc[s] == 0) != (p->bc[s + 1] == 0)) return ORACLE_EINVAL;
  return ORACLE_OK;
}

/* The state with NG ghost layers on every side that exists, filled as the boundary conditions of
 * Sec. 3 state: first the ghost columns of the interior rows (x-sides), then whole ghost rows across
 * the padded width (y-sides), so that a corner cell follows the y-side's rule applied to the x-ghost
 * column beside it. Layout G[c][jp][ip] with jp = j + NG (2D; a single row in 1D), ip = i + NG.
 *   periodic: the cell one period away; outflow: the nearest interior cell (zero gradient);
 *   reflect: the mirror cell with the normal momentum negated; no-slip adiabatic: the mirror cell with
 *   both momenta negated; prescribed: the side's state a or b at the ghost centre and stage time t,
 *   or beyond the split the ghost of the kind the side names for the rest. */
typedef struct {
  int nc, nx, ny, px, py, jo;
  double* G;
} padded;

static double* pg(const padded* g, int c, int j, int i) {
  return g->G + ((size_t)c * g->py + (size_t)(j + g->jo)) * g->px + (size_t)(i + NG);
}

/* Conserved state of a prescribed side at a ghost centre, or NULL where the rest kind applies;
 * *kind receives that kind. */
static const double* prescribed(const oracle_problem* p, int side, double tau, double nu, double t, int* kind) {
  const oracle_bc_data* d = &p->bcd[side];
  *kind = d->rest;
  if (tau < d->s0 + d->sn * nu + d->st * t) return d->a;
  if (d->rest == 4) return d->b;
  return NULL;
}

static void put_state(const padded* g, int j, int i, const double* q) {
  /* q is (rho, rho U, rho V, rho E); 1D keeps (rho, rho U, rho E) */
  if (g->nc == 4) for (int c = 0; c < 4; ++c) *pg(g, c, j, i) = q[c];
  else { *pg(g, 0, j, i) = q[0]; *pg(g, 1, j, i) = q[1]; *pg(g, 2, j, i) = q[3]; }
}

static void pad_state(const oracle_problem* p, const double* W, double t, padded* g) {
  int nc = p->dim + 2, nx = p->nx, ny = p->ny;
  double dx = (p->x1 - p->x0) / nx, dy = (p->dim == 2) ? (p->y1 - p->y0) / ny : 1.0;
  g->nc = nc; g->nx = nx; g->ny = ny;
  g->px = nx + 2 * NG;
  g->jo = (p->dim == 2) ? NG : 0;
  g->py = ny + 2 * g->jo;
  g->G = (double*)malloc(sizeof(double) * nc * g->px * g->py);
  for (int c = 0; c < nc; ++c)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) *pg(g, c, j, i) = W[((size_t)c * ny + j) * nx + i];
  /* x-sides, interior rows */
  for (int j = 0; j < ny; ++j)
    for (int k = 1; k <= NG; ++k)
      for (int side = 0; side < 2; ++side) {
        int i = side ? nx - 1 + k : -k;
        int kind = p->bc[side];
        if (kind == 4) {
          double x = p->x0 + (i + 0.5) * dx;
          double y = (p->dim == 2) ? p->y0 + (j + 0.5) * dy : 0.0;
          const double* q = prescribed(p, side, y, x, t, &kind);
          if (q) { put_state(g, j, i, q); continue; }
        }
        int src = kind == 0 ? (side ? i - nx : i + nx) : kind == 1 ? (side ? nx - 1 : 0) : (side ? 2 * nx - 1 - i : -1 - i);
        for (int c = 0; c < nc; ++c) {
          double v = *pg(g, c, j, src);
          if ((kind == 2 || kind == 3) && c == 1) v = -v;           /* normal momentum */
          if (kind == 3 && nc == 4 && c == 2) v = -v;               /* tangential momentum */
          *pg(g, c, j, i) = v;
        }
      }
  if (p->dim == 1) return;
  /* y-sides, whole padded rows (ghost columns included); every source row is an interior one */
  for (int k = 1; k <= NG; ++k)
    for (int side = 0; side < 2; ++side) {
      int j = side ? ny - 1 + k : -k;
      for (int i = -NG; i < nx + NG; ++i) {
        int kind = p->bc[2 + side];
        if (kind == 4) {
          double x = p->x0 + (i + 0.5) * dx;
          double y = p->y0 + (j + 0.5) * dy;
          const double* q = prescribed(p, 2 + side, x, y, t, &kind);
          if (q) { put_state(g, j, i, q); continue; }
        }
        int src = kind == 0 ? (side ? j - ny : j + ny) : kind == 1 ? (side ? ny - 1 : 0) : (side ? 2 * ny - 1 - j : -1 - j);
        for (int c = 0; c < nc; ++c) {
          double v = *pg(g, c, src, i);
          if ((kind == 2 || kind == 3) && c == 2) v = -v;           /* normal momentum */
          if (kind == 3 && c == 1) v = -v;                          /* tangential momentum */
          *pg(g, c, j, i) = v;
        }
      }
    }
}

/* A directional view: normal index n (fast), tangential index t, padded by NG on every side that
 * exists (no tangential padding in 1D). Components are rotated so that slot 1 is the normal
 * momentum and slot 2 the tangential one. */
typedef struct {
  int nc, dim, nn, nt, pn, pt, tp;
  double hn, ht;
  double* P;
} frame;

static double* fr_at(const frame* f, int c, int jt, int in) {
  return f->P + ((size_t)c * f->pt + (size_t)(jt + f->tp)) * f->pn + (size_t)(in + NG);
}

/* Build the padded frame for direction dir (0: x, 1: y) from the state padded at stage time t. */
static void build_frame(const oracle_problem* p, const double* W, double t, int dir, frame* f) {
  int nc = p->dim + 2, nx = p->nx, ny = p->ny;
  f->nc = nc;
  f->dim = p->dim;
  double dx = (p->x1 - p->x0) / nx, dy = (p->dim == 2) ? (p->y1 - p->y0) / ny : 1.0;
  if (dir == 0) { f->nn = nx; f->nt = ny; f->hn = dx; f->ht = dy; }
  else { f->nn = ny; f->nt = nx; f->hn = dy; f->ht = dx; }
  f->tp = (p->dim == 2) ? NG : 0;
  f->pn = f->nn + 2 * NG;
  f->pt = f->nt + 2 * f->tp;
  f->P = (double*)malloc(sizeof(double) * nc * f->pn * f->pt);
  padded g;
  pad_state(p, W, t, &g);
  for (int jt = -f->tp; jt < f->nt + f->tp; ++jt)
    for (int in = -NG; in < f->nn + NG; ++in) {
      int i = (dir == 0) ? in : jt, j = (dir == 0) ? jt : in;
      double v[MAXC];
      for (int c = 0; c < nc; ++c) v[c] = *pg(&g, c, j, i);
      if (dir == 1) { double tmp = v[1]; v[1] = v[2]; v[2] = tmp; }
      for (int c = 0; c < nc; ++c) *fr_at(f, c, jt, in) = v[c];
    }
  free(g.G);
}

/* Widened flags of every padded cell where the 7-cell stencil fits, along the normal (Fn) and
 * along the tangential direction (Ft, 2D). Cells whose flag is undefined hold 255. */
static void frame_flags(const frame* f, const params* pp, uint8_t* Fn, uint8_t* Ft) {
  int pn = f->pn, pt = f->pt, nc = f->nc;
  uint8_t* Tn = (uint8_t*)malloc((size_t)pn * pt);
  uint8_t* Tt = (uint8_t*)malloc((size_t)pn * pt);
  memset(Tn, 255, (size_t)pn * pt);
  memset(Tt, 255, (size_t)pn * pt);
  double q[5], xb, xh;
  int st;
  for (int a = 0; a < pt; ++a)
    for (int b = 2; b < pn - 2; ++b) {
      int T = 0;
      for (int c = 0; c < nc; ++c) {
        for (int r = 0; r < 5; ++r) q[r] = f->P[((size_t)c * pt + a) * pn + b - 2 + r];
        T |= troubled_component(q, f->hn, pp->zeta1_mode, &xb, &xh, &st);
      }
      Tn[(size_t)a * pn + b] = (uint8_t)T;
    }
  if (f->dim == 2)
    for (int a = 2; a < pt - 2; ++a)
      for (int b = 0; b < pn; ++b) {
        int T = 0;
        for (int c = 0; c < nc; ++c) {
          for (int r = 0; r < 5; ++r) q[r] = f->P[((size_t)c * pt + a - 2 + r) * pn + b];
          T |= troubled_component(q, f->ht, pp->zeta1_mode, &xb, &xh, &st);
        }
        Tt[(size_t)a * pn + b] = (uint8_t)T;
      }
  memset(Fn, 255, (size_t)pn * pt);
  if (Ft) memset(Ft, 255, (size_t)pn * pt);
  for (int a = 0; a < pt; ++a)
    for (int b = 3; b < pn - 3; ++b) {
      size_t o = (size_t)a * pn + b;
      uint8_t v = (uint8_t)(Tn[o - 1] | Tn[o] | Tn[o + 1]);
      if (pp->recon == 1) v = 1;
      if (pp->recon == 2) v = 0;
      Fn[o] = v;
    }
  if (Ft && f->dim == 2)
    for (int a = 3; a < pt - 3; ++a)
      for (int b = 0; b < pn; ++b) {
        size_t o = (size_t)a * pn + b;
        uint8_t v = (uint8_t)(Tt[o - pn] | Tt[o] | Tt[o + pn]);
        if (pp->recon == 1) v = 1;
        if (pp->recon == 2) v = 0;
        Ft[o] = v;
      }
  free(Tn);
  free(Tt);
}

/* Whether a reconstructed state (frame components: rho, normal and tangential momentum, energy; no
 * tangential slot in 1D) is physical: positive density, and a pressure above the rounding error of the
 * arithmetic that produced it. The state combines five stencil values q5 whose largest |energy| is emax;
 * its pressure then carries an absolute rounding error of a few units in the last place of emax, so a
 * pressure within 64 units of the unit roundoff (2^-53) times emax of zero is not taken as positive. */
static double stencil_emax(const double q5[5][MAXC], int nc) {
  double e = 0.0;
  for (int r = 0; r < 5; ++r) e = fmax(e, fabs(q5[r][nc - 1]));
  return e;
}

static int admissible(const double* w, int nc, double gamma, double emax) {
  double mt = (nc == 4) ? w[2] : 0.0;
  double pr = (gamma - 1.0) * (w[nc - 1] - 0.5 * (w[1] * w[1] + mt * mt) / w[0]);
  return w[0] > 0.0 && pr > 64.0 * 0x1p-53 * emax && isfinite(pr);
}

/* Time-integrated fluxes F(dt), F(dt/2) at every interface of the frame (normal-direction
 * interfaces k = 0..nn of rows 0..nt-1), averaged over the Gauss points of each segment.
 * Output layout: [nc][nt][nn+1], components in the frame's (rotated) order. */
static void frame_fluxes(const frame* f, const params* pp, double dt, double* Fd, double* Fh,
                         int nthreads) {
  int nc = f->nc, nn = f->nn, nt = f->nt, pn = f->pn, pt = f->pt, tp = f->tp;
  uint8_t* Fn = (uint8_t*)malloc((size_t)pn * pt);
  uint8_t* Ft = (uint8_t*)malloc((size_t)pn * pt);
  frame_flags(f, pp, Fn, f->dim == 2 ? Ft : NULL);
  /* rows -2..nt+1 carry line values in 2D; -3..nt+2 when the tangential flag is the indicator on the line
   * values (its widening needs the indicator one row beyond the interface's own rows) */
  int ext = (f->dim == 2) ? (pp->tfm ? 3 : 2) : 0;
  int nrows = (f->dim == 2) ? nt + 2 * ext : 1;
  int r0 = -ext;
  size_t lsz = (size_t)nrows * (nn + 1);
  /* line values: [kind][c][row][k], kind 0: W^l, 1: W_x^l, 2: W^r, 3: W_x^r */
  double* LV = (double*)malloc(sizeof(double) * 4 * nc * lsz);
#define LVAT(kind, c, row, k) LV[(((size_t)(kind) * nc + (c)) * nrows + ((row) - r0)) * (nn + 1) + (k)]
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
  for (int row = r0; row < r0 + nrows; ++row) {
    for (int k = 0; k <= nn; ++k) {
      double q5[5][MAXC], R[16], L[16], avg[MAXC], val[MAXC], der[MAXC];
      int fl = Fn[(size_t)(row + tp) * pn + (k - 1 + NG)];
      int fr = Fn[(size_t)(row + tp) * pn + (k + NG)];
      if (fl || fr) {
        for (int c = 0; c < nc; ++c) avg[c] = 0.5 * (*fr_at(f, c, row, k - 1) + *fr_at(f, c, row, k));
        char_R(f->dim, 1, avg, pp->gamma, R);
        mat_inverse(nc, R, L);
      }
      for (int s = 0; s < 2; ++s) {
        int cell = k - 1 + s;
        for (int r = 0; r < 5; ++r)
          for (int c = 0; c < nc; ++c) q5[r][c] = *fr_at(f, c, row, cell - 2 + r);
        recon_side(pp, q5, s == 0 ? 0.5 : -0.5, s == 0 ? fl : fr, R, L, val, der);
        if (pp->positivity && !admissible(val, nc, pp->gamma, stencil_emax(q5, nc)))
          for (int c = 0; c < nc; ++c) { /* first order: the cell's own average, no slope */
            val[c] = q5[2][c];
            der[c] = 0.0;
          }
        for (int c = 0; c < nc; ++c) {
          LVAT(2 * s, c, row, k) = val[c];
          LVAT(2 * s + 1, c, row, k) = der[c] / f->hn;
        }
      }
    }
  }
  /* Sec. 2.3.3 Step 2 reading A: the tangential reconstruction's flag is the hybrid method's indicator
   * (Steps 1-3) on the line values W^s along the interface, widened over the neighbouring rows (Step 4);
   * Tl[s][row + 1][k] for rows -1..nt */
  uint8_t* Tl = NULL;
  if (f->dim == 2 && pp->tfm) {
    Tl = (uint8_t*)malloc((size_t)2 * (nt + 2) * (nn + 1));
    for (int sd = 0; sd < 2; ++sd)
      for (int row = -1; row <= nt; ++row)
        for (int k = 0; k <= nn; ++k) {
          int T = 0;
          double q[5], xb, xh;
          int st;
          for (int c = 0; c < nc; ++c) {
            for (int r = 0; r < 5; ++r) q[r] = LVAT(2 * sd, c, row - 2 + r, k);
            T |= troubled_component(q, f->ht, pp->zeta1_mode, &xb, &xh, &st);
          }
          if (pp->recon == 1) T = 1;
          if (pp->recon == 2) T = 0;
          Tl[((size_t)sd * (nt + 2) + (row + 1)) * (nn + 1) + k] = (uint8_t)T;
        }
  }
  const double eta = 1.0 / (2.0 * sqrt(3.0)); /* two-point Gauss-Legendre on [-1/2, 1/2] */
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
  for (int j = 0; j < nt; ++j) {
    for (int k = 0; k <= nn; ++k) {
      double sumd[MAXC] = {0}, sumh[MAXC] = {0};
      double Ws[2][MAXC], Wxs[2][MAXC], Wys[2][MAXC], Fdg[MAXC], Fhg[MAXC];
      if (f->dim == 1) {
        for (int s = 0; s < 2; ++s)
          for (int c = 0; c < nc; ++c) {
            Ws[s][c] = LVAT(2 * s, c, 0, k);
            Wxs[s][c] = LVAT(2 * s + 1, c, 0, k);
            Wys[s][c] = 0.0;
          }
        gp_flux(pp, Ws[0], Wxs[0], Wys[0], Ws[1], Wxs[1], Wys[1], dt, sumd, sumh, NULL);
      } else {
        /* Tangential characteristic variables: each side is decomposed about its own line-averaged state
         * of the centre segment, the state of the cell being reconstructed (reading of "averaged
         * conservative variables" for a Gauss point inside the segment). */
        int ftf[2];
        double R[2][16], L[2][16];
        for (int s = 0; s < 2; ++s) {
          if (Tl) {
            const uint8_t* t = Tl + (size_t)s * (nt + 2) * (nn + 1);
            ftf[s] = t[(size_t)j * (nn + 1) + k] | t[(size_t)(j + 1) * (nn + 1) + k] | t[(size_t)(j + 2) * (nn + 1) + k];
          } else {
            ftf[s] = Ft[(size_t)(j + tp) * pn + (k - 1 + s + NG)];
          }
          if (ftf[s]) {
            double own[MAXC];
            for (int c = 0; c < nc; ++c)
              own[c] = pp->csm ? 0.5 * (LVAT(0, c, j, k) + LVAT(2, c, j, k)) : LVAT(2 * s, c, j, k);
            char_R(f->dim, 2, own, pp->gamma, R[s]);
            mat_inverse(nc, R[s], L[s]);
          }
        }
        for (int m = 0; m < 2; ++m) {
          double xi = (m == 0) ? -eta : eta;
          for (int s = 0; s < 2; ++s) {
            double q5[5][MAXC], val[MAXC], der[MAXC];
            for (int r = 0; r < 5; ++r)
              for (int c = 0; c < nc; ++c) q5[r][c] = LVAT(2 * s, c, j - 2 + r, k);
            recon_side(pp, q5, xi, ftf[s], R[s], L[s], val, der);
            /* first order along the interface: the centre segment's line values, no tangential slope */
            int low = pp->positivity && !admissible(val, nc, pp->gamma, stencil_emax(q5, nc));
            for (int c = 0; c < nc; ++c) {
              Ws[s][c] = low ? q5[2][c] : val[c];
              Wys[s][c] = low ? 0.0 : der[c] / f->ht;
            }
            for (int r = 0; r < 5; ++r)
              for (int c = 0; c < nc; ++c) q5[r][c] = LVAT(2 * s + 1, c, j - 2 + r, k);
            recon_side(pp, q5, xi, ftf[s], R[s], L[s], val, der);
            for (int c = 0; c < nc; ++c) Wxs[s][c] = low ? q5[2][c] : val[c];
          }
          gp_flux(pp, Ws[0], Wxs[0], Wys[0], Ws[1], Wxs[1], Wys[1], dt, Fdg, Fhg, NULL);
          for (int c = 0; c < nc; ++c) {
            sumd[c] += 0.5 * Fdg[c];
            sumh[c] += 0.5 * Fhg[c];
          }
        }
      }
      for (int c = 0; c < nc; ++c) {
        Fd[((size_t)c * nt + j) * (nn + 1) + k] = sumd[c];
        Fh[((size_t)c * nt + j) * (nn + 1) + k] = sumh[c];
      }
    }
  }
#undef LVAT
  free(LV);
  free(Tl);
  free(Fn);
  free(Ft);
}

/* Time-integrated fluxes of both directions in the grid's own component order:
 * x: [nc][ny][nx+1], y: [nc][ny+1][nx]. */
static void all_fluxes(const oracle_problem* p, const params* pp, const double* W, double t, double dt,
                       double* Fxd, double* Fxh, double* Fyd, double* Fyh, int nthreads) {
  frame f;
  build_frame(p, W, t, 0, &f);
  frame_fluxes(&f, pp, dt, Fxd, Fxh, nthreads);
  free(f.P);
  if (p->dim == 2) {
    int nx = p->nx, ny = p->ny, nc = pp->nc;
    size_t n = (size_t)nc * nx * (ny + 1);
    double* td = (double*)malloc(sizeof(double) * n);
    double* th = (double*)malloc(sizeof(double) * n);
    build_frame(p, W, t, 1, &f);
    frame_fluxes(&f, pp, dt, td, th, nthreads); /* [nc'][nx][ny+1] */
    free(f.P);
    for (int c = 0; c < nc; ++c) {
      int cs = (c == 1) ? 2 : (c == 2) ? 1 : c; /* rotate momentum back */
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
          Fyd[((size_t)c * (ny + 1) + j) * nx + i] = td[((size_t)cs * nx + i) * (ny + 1) + j];
          Fyh[((size_t)c * (ny + 1) + j) * nx + i] = th[((size_t)cs * nx + i) * (ny + 1) + j];
        }
    }
    free(td);
    free(th);
  }
}

static int admissible_cell(const oracle_problem* p, const double* W, size_t s) {
  int nc = p->dim + 2;
  size_t ncell = (size_t)p->nx * p->ny;
  double rho = W[s], mx = W[ncell + s], my = (p->dim == 2) ? W[2 * ncell + s] : 0.0;
  double E = W[(size_t)(nc - 1) * ncell + s];
  double pr = (p->gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho);
  return rho > 0.0 && pr > 0.0 && isfinite(E);
}

static int nonphysical(const oracle_problem* p, const double* W) {
  size_t ncell = (size_t)p->nx * p->ny;
  for (size_t s = 0; s < ncell; ++s)
    if (!admissible_cell(p, W, s)) return 1;
  return 0;
}

/* W_new = W - dt (dFx/dx + dFy/dy) with face fluxes Fx [nc][ny][nx+1], Fy [nc][ny+1][nx]. */
static void update_cells(const oracle_problem* p, const double* W, const double* Fx, const double* Fy, double dt,
                         double* Wn) {
  int nc = p->dim + 2, nx = p->nx, ny = p->ny;
  double dx = (p->x1 - p->x0) / nx, dy = p->dim == 2 ? (p->y1 - p->y0) / ny : 1.0;
  size_t ncell = (size_t)nx * ny;
  for (int c = 0; c < nc; ++c)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double a = (Fx[((size_t)c * ny + j) * (nx + 1) + i + 1] - Fx[((size_t)c * ny + j) * (nx + 1) + i]) / dx;
        double b = 0.0;
        if (p->dim == 2) b = (Fy[((size_t)c * (ny + 1) + j + 1) * nx + i] - Fy[((size_t)c * (ny + 1) + j) * nx + i]) / dy;
        size_t o = (size_t)c * ncell + (size_t)j * nx + i;
        Wn[o] = W[o] - dt * (a + b);
      }
}

double oracle_cfl_dt3(const oracle_problem* p, const double* W);

double oracle_cfl_dt(const oracle_problem* p, const double* W) {
  if (p->dim == 3) return oracle_cfl_dt3(p, W);
  /* dt = CFL * min over cells of min(h/(|U| + c), h^2/(4 nu)), nu = mu/rho, h = min(dx, dy) */
  int nc = p->dim + 2;
  size_t ncell = (size_t)p->nx * p->ny;
  double dx = (p->x1 - p->x0) / p->nx;
  double h = dx;
  if (p->dim == 2) {
    double dy = (p->y1 - p->y0) / p->ny;
    if (dy < h) h = dy;
  }
  double qmin = INFINITY;
  for (size_t s = 0; s < ncell; ++s) {
    double rho = W[s];
    double U = W[ncell + s] / rho;
    double V = (p->dim == 2) ? W[2 * ncell + s] / rho : 0.0;
    double pr = (p->gamma - 1.0) * (W[(size_t)(nc - 1) * ncell + s] - 0.5 * rho * (U * U + V * V));
    double c = sqrt(p->gamma * pr / rho);
    double sp = sqrt(U * U + V * V) + c;
    double q = h / sp;
    if (p->eqn == 1) {
      double qv = (h * h) / (4.0 * (p->mu / (p->viscous_dt_mode ? pr : rho)));
      q = fmin(q, qv);
    }
    qmin = fmin(qmin, q);
  }
  return p->cfl * qmin;
}

int oracle_stage_fluxes(const oracle_problem* p, const double* W, double t, double dt, double* Fx, double* Gx,
                        double* Fy, double* Gy, int nthreads) {
  oracle_init();
  int rc = check_problem(p);
  if (rc) return rc;
  params pp;
  make_params(p, &pp);
  int nc = pp.nc, nx = p->nx, ny = p->ny;
  size_t nxf = (size_t)nc * ny * (nx + 1), nyf = (size_t)nc * (ny + 1) * nx;
  double* Fxd = (double*)malloc(sizeof(double) * nxf);
  double* Fxh = (double*)malloc(sizeof(double) * nxf);
  double* Fyd = p->dim == 2 ? (double*)malloc(sizeof(double) * nyf) : NULL;
  double* Fyh = p->dim == 2 ? (double*)malloc(sizeof(double) * nyf) : NULL;
  all_fluxes(p, &pp, W, t, dt, Fxd, Fxh, Fyd, Fyh, nthreads);
  /* F = (4 F(dt/2) - F(dt))/dt, dF/dt = 4 (F(dt) - 2 F(dt/2))/dt^2 */
  for (size_t s = 0; s < nxf; ++s) {
    Fx[s] = (4.0 * Fxh[s] - Fxd[s]) / dt;
    Gx[s] = 4.0 * (Fxd[s] - 2.0 * Fxh[s]) / (dt * dt);
  }
  if (p->dim == 2)
    for (size_t s = 0; s < nyf; ++s) {
      Fy[s] = (4.0 * Fyh[s] - Fyd[s]) / dt;
      Gy[s] = 4.0 * (Fyd[s] - 2.0 * Fyh[s]) / (dt * dt);
    }
  free(Fxd);
  free(Fxh);
  free(Fyd);
  free(Fyh);
  return ORACLE_OK;
}

static int step3(const oracle_problem* p, double* W, double* t, double t_end, double* dt_taken, int nthreads);

static int step_ms(const oracle_problem* p, double* W, double* t, double t_end, double* dt_taken, int nthreads);

int oracle_step(const oracle_problem* p, double* W, double* t, double t_end, double* dt_taken,
                int nthreads) {
  oracle_init();
  if (p->stepper.stages != 0) return step_ms(p, W, t, t_end, dt_taken, nthreads < 1 ? 1 : nthreads);
  if (p->dim == 3) return step3(p, W, t, t_end, dt_taken, nthreads < 1 ? 1 : nthreads);
  int rc = check_problem(p);
  if (rc) return rc;
  if (nthreads < 1) nthreads = 1;
  params pp;
  make_params(p, &pp);
  if (dt_taken) *dt_taken = 0.0;
  if (*t >= t_end) return ORACLE_OK;
  double dt = (p->fixed_dt > 0.0) ? p->fixed_dt : oracle_cfl_dt(p, W);
  if (!(dt > 0.0) || !isfinite(dt)) return ORACLE_EDT;
  double tnew;
  if (*t + dt >= t_end) {
    dt = t_end - *t;
    tnew = t_end;
  } else {
    tnew = *t + dt;
  }
  int nc = pp.nc, nx = p->nx, ny = p->ny, dim = p->dim;
  double dx = (p->x1 - p->x0) / nx, dy = dim == 2 ? (p->y1 - p->y0) / ny : 1.0;
  size_t ncell = (size_t)nx * ny;
  size_t nxf = (size_t)nc * ny * (nx + 1), nyf = dim == 2 ? (size_t)nc * (ny + 1) * nx : 1;
  double* Fxd = (double*)malloc(sizeof(double) * nxf);
  double* Fxh = (double*)malloc(sizeof(double) * nxf);
  double* Fyd = (double*)malloc(sizeof(double) * nyf);
  double* Fyh = (double*)malloc(sizeof(double) * nyf);
  double* Fx = (double*)malloc(sizeof(double) * nxf); /* F^n + dt/6 dF^n/dt, then the final flux */
  double* Fy = (double*)malloc(sizeof(double) * nyf);
  double* Gxn = (double*)malloc(sizeof(double) * nxf);
  double* Gyn = (double*)malloc(sizeof(double) * nyf);
  double* Ws = (double*)malloc(sizeof(double) * nc * ncell);

  /* stage 1 at t_n */
  all_fluxes(p, &pp, W, *t, dt, Fxd, Fxh, Fyd, Fyh, nthreads);
  for (size_t s = 0; s < nxf; ++s) {
    Fx[s] = (4.0 * Fxh[s] - Fxd[s]) / dt;
    Gxn[s] = 4.0 * (Fxd[s] - 2.0 * Fxh[s]) / (dt * dt);
  }
  if (dim == 2)
    for (size_t s = 0; s < nyf; ++s) {
      Fy[s] = (4.0 * Fyh[s] - Fyd[s]) / dt;
      Gyn[s] = 4.0 * (Fyd[s] - 2.0 * Fyh[s]) / (dt * dt);
    }
  /* F^n kept for the time-order fallback */
  double* Fxn = (double*)malloc(sizeof(double) * nxf);
  double* Fyn = (double*)malloc(sizeof(double) * nyf);
  memcpy(Fxn, Fx, sizeof(double) * nxf);
  if (dim == 2) memcpy(Fyn, Fy, sizeof(double) * nyf);
  /* W* = W^n - [F(dt/2)_{i+1/2} - F(dt/2)_{i-1/2}]/dx - [G(dt/2)_{j+1/2} - G(dt/2)_{j-1/2}]/dy */
  for (int c = 0; c < nc; ++c)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double a = (Fxh[((size_t)c * ny + j) * (nx + 1) + i + 1] - Fxh[((size_t)c * ny + j) * (nx + 1) + i]) / dx;
        double b = 0.0;
        if (dim == 2) b = (Fyh[((size_t)c * (ny + 1) + j + 1) * nx + i] - Fyh[((size_t)c * (ny + 1) + j) * nx + i]) / dy;
        size_t o = (size_t)c * ncell + (size_t)j * nx + i;
        Ws[o] = W[o] - (a + b);
      }
  if (pp.positivity && nonphysical(p, Ws)) {
    /* first-order fallback of the first stage: every face of a cell whose intermediate state is
     * non-physical takes the gas-kinetic flux of the two cell averages (constant states, no slopes) over
     * [0, dt/2] in place of the reconstructed one, for both of its cells; then update again */
    uint8_t* bad = (uint8_t*)calloc(ncell, 1);
    for (size_t s = 0; s < ncell; ++s) bad[s] = !admissible_cell(p, Ws, s);
    const double z[MAXC] = {0};
    for (int dir = 0; dir < dim; ++dir) {
      frame f;
      build_frame(p, W, *t, dir, &f);
      for (int row = 0; row < f.nt; ++row)
        for (int k = 0; k <= f.nn; ++k) {
          /* the face's cells in grid indices: (k-1, row), (k, row) along x; (row, k-1), (row, k) along y */
          int b0 = 0, b1 = 0;
          if (k >= 1) b0 = bad[dir ? (size_t)(k - 1) * nx + row : (size_t)row * nx + (k - 1)];
          if (k < f.nn) b1 = bad[dir ? (size_t)k * nx + row : (size_t)row * nx + k];
          if (!(b0 | b1)) continue;
          double Wl[MAXC], Wr[MAXC], Fdg[MAXC], Fhg[MAXC];
          for (int c = 0; c < nc; ++c) {
            Wl[c] = *fr_at(&f, c, row, k - 1);
            Wr[c] = *fr_at(&f, c, row, k);
          }
          gp_flux(&pp, Wl, z, z, Wr, z, z, dt, Fdg, Fhg, NULL);
          for (int c = 0; c < nc; ++c) {
            int cs = (dir && c == 1) ? 2 : (dir && c == 2) ? 1 : c; /* frame slot -> grid component */
            if (dir == 0) Fxh[((size_t)cs * ny + row) * (nx + 1) + k] = Fhg[c];
            else Fyh[((size_t)cs * (ny + 1) + k) * nx + row] = Fhg[c];
          }
        }
      free(f.P);
    }
    free(bad);
    for (int c = 0; c < nc; ++c)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double a = (Fxh[((size_t)c * ny + j) * (nx + 1) + i + 1] - Fxh[((size_t)c * ny + j) * (nx + 1) + i]) / dx;
          double b = 0.0;
          if (dim == 2) b = (Fyh[((size_t)c * (ny + 1) + j + 1) * nx + i] - Fyh[((size_t)c * (ny + 1) + j) * nx + i]) / dy;
          size_t o = (size_t)c * ncell + (size_t)j * nx + i;
          Ws[o] = W[o] - (a + b);
        }
  }
  if (nonphysical(p, Ws)) rc = ORACLE_ENONPHYS;
  if (!rc) {
    /* stage 2 at t* = t_n + dt/2: only the time derivative of the flux is needed */
    all_fluxes(p, &pp, Ws, *t + 0.5 * dt, dt, Fxd, Fxh, Fyd, Fyh, nthreads);
    for (size_t s = 0; s < nxf; ++s) {
      double Gs = 4.0 * (Fxd[s] - 2.0 * Fxh[s]) / (dt * dt);
      Fx[s] = Fx[s] + dt / 6.0 * (Gxn[s] + 2.0 * Gs);
    }
    if (dim == 2)
      for (size_t s = 0; s < nyf; ++s) {
        double Gs = 4.0 * (Fyd[s] - 2.0 * Fyh[s]) / (dt * dt);
        Fy[s] = Fy[s] + dt / 6.0 * (Gyn[s] + 2.0 * Gs);
      }
    update_cells(p, W, Fx, Fy, dt, Ws);
    if (pp.positivity && nonphysical(p, Ws)) {
      /* time-order fallback: every face of a cell that this update leaves non-physical takes the
       * one-stage flux of the first stage's linear-in-time expansion, F^n + dt/2 dF^n/dt (the flux
       * integrated over the whole step, divided by dt), for both of its cells; then update again */
      uint8_t* bad = (uint8_t*)calloc(ncell, 1);
      for (size_t s = 0; s < ncell; ++s) bad[s] = !admissible_cell(p, Ws, s);
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          if (!bad[(size_t)j * nx + i]) continue;
          for (int c = 0; c < nc; ++c) {
            for (int f = 0; f < 2; ++f) {
              size_t s = ((size_t)c * ny + j) * (nx + 1) + i + f;
              Fx[s] = Fxn[s] + 0.5 * dt * Gxn[s];
            }
            if (dim == 2)
              for (int f = 0; f < 2; ++f) {
                size_t s = ((size_t)c * (ny + 1) + j + f) * nx + i;
                Fy[s] = Fyn[s] + 0.5 * dt * Gyn[s];
              }
          }
        }
      free(bad);
      update_cells(p, W, Fx, Fy, dt, Ws);
    }
    if (nonphysical(p, Ws)) rc = ORACLE_ENONPHYS;
    if (!rc) {
      memcpy(W, Ws, sizeof(double) * nc * ncell);
      *t = tnew;
      if (dt_taken) *dt_taken = dt;
    }
  }
  free(Fxd); free(Fxh); free(Fyd); free(Fyh);
  free(Fx); free(Fy); free(Gxn); free(Gyn); free(Ws); free(Fxn); free(Fyn);
  return rc;
}

int oracle_flags(const oracle_problem* p, const double* W, double t, uint8_t* fx, uint8_t* fy) {
  oracle_init();
  int rc = check_problem(p);
  if (rc) return rc;
  params pp;
  make_params(p, &pp);
  for (int dir = 0; dir < p->dim; ++dir) {
    frame f;
    build_frame(p, W, t, dir, &f);
    uint8_t* Fn = (uint8_t*)malloc((size_t)f.pn * f.pt);
    frame_flags(&f, &pp, Fn, NULL);
    uint8_t* out = (dir == 0) ? fx : fy;
    for (int jt = 0; jt < f.nt; ++jt)
      for (int in = 0; in < f.nn; ++in) {
        uint8_t v = Fn[(size_t)(jt + f.tp) * f.pn + in + NG];
        if (dir == 0) out[(size_t)jt * p->nx + in] = v;
        else out[(size_t)in * p->nx + jt] = v;
      }
    free(Fn);
    free(f.P);
  }
  return ORACLE_OK;
}

/* ======================================================================== */
/* 7. Unit-level entry points                                               */
/* ======================================================================== */

void oracle_stencil_eval(int k, const double* q, double xi, double* val, double* der) {
  oracle_init();
  double c[5];
  stencil_coeffs(k, q, c);
  poly_eval(c, g_npts[k] - 1, xi, val, der);
}

double oracle_beta(int k, const double* q) {
  oracle_init();
  double c[5];
  stencil_coeffs(k, q, c);
  return beta_of(c, g_npts[k] - 1);
}

void oracle_ao_eval(const double* q, double xi, double ghi, double glo, double eps, double* val,
                    double* der) {
  oracle_init();
  ao_eval(q, xi, ghi, glo, eps, val, der);
}

int oracle_indicator(const double* q, double h, int zeta1_mode, double* xbar, double* xhat, int* step) {
  return troubled_component(q, h, zeta1_mode, xbar, xhat, step);
}

void oracle_char_matrices(int dim, int dir, const double* W, double gamma, double* R, double* L) {
  oracle_init();
  char_R(dim, dir, W, gamma, R);
  mat_inverse(dim + 2, R, L);
}

void oracle_maxwell_moments(double rho, double U, double V, double lam, double K, int half,
                            double* Mu, double* Mv, double* Mxi) {
  maxw g;
  (void)rho;
  maxw_moments(U, V, lam, K, half, &g);
  for (int n = 0; n < 9; ++n) {
    Mu[n] = half ? g.Mh[n] : g.Mu[n];
    Mv[n] = g.Mv[n];
  }
  for (int n = 0; n < 4; ++n) Mxi[n] = g.Mx[n];
}

void oracle_slope_solve(int dim, const double* W, double gamma, const double* b, double* a) {
  oracle_problem p;
  memset(&p, 0, sizeof p);
  p.dim = dim;
  p.gamma = gamma;
  params pp;
  make_params(&p, &pp);
  maxw g;
  maxw_from_W(&pp, W, 0, &g);
  solve_slope(&pp, &g, b, a);
}

void oracle_time_coeffs(double delta, double tau, double* C) { time_coeffs(delta, tau, C); }

void oracle_gp_flux(const oracle_problem* p, const double* Wl, const double* Wxl, const double* Wyl,
                    const double* Wr, const double* Wxr, const double* Wyr, double dt, double* Fdt,
                    double* Fdt2, double* tau_out) {
  oracle_init();
  params pp;
  make_params(p, &pp);
  gp_flux(&pp, Wl, Wxl, Wyl, Wr, Wxr, Wyr, dt, Fdt, Fdt2, tau_out);
}

/* ======================================================================== */
/* 8. Three dimensions                                                       */
/* ======================================================================== */
/* The paper develops the scheme in 1D and 2D and states that the 3D extension is direct. It is taken
 * here as: the same hybrid reconstruction along the normal of each face (its cell averages give face
 * averages), then along the first and then the second tangential direction to the 2 x 2 tensor
 * Gauss-Legendre points of the face (weights 1/4), each step flagged by the side cell's troubled flag
 * in the direction of that step and, when flagged, WENO-AO in the characteristic variables of the state
 * it starts from; at each point the gas-kinetic flux of Sec. 2.1 with three velocity components
 * (u normal, v and w tangential) and K = (5 - 3 gamma)/(gamma - 1) internal degrees of freedom.
 * Euler equations, or Navier-Stokes with Pr = 1. States: W[c][k][j][i], c in (rho, rho U, rho V,
 * rho W, rho E). */

#define NC3 5

typedef struct {
  double rho, U, V, Wv, lam;
  double Mu[NMOM], Mh[NMOM], Mv[NMOM], Mw[NMOM], Mx[4];
} maxw3;

static void maxw3_from_W(double K, double gamma, const double* W, int side, maxw3* g) {
  g->rho = W[0];
  g->U = W[1] / W[0];
  g->V = W[2] / W[0];
  g->Wv = W[3] / W[0];
  double p = (gamma - 1.0) * (W[4] - 0.5 * W[0] * (g->U * g->U + g->V * g->V + g->Wv * g->Wv));
  g->lam = W[0] / (2.0 * p);
  maxw m2;
  maxw_moments(g->U, g->V, g->lam, K, side, &m2);  /* u (and half-line u) and v moments, xi^2 */
  memcpy(g->Mu, m2.Mu, sizeof g->Mu);
  memcpy(g->Mh, m2.Mh, sizeof g->Mh);
  memcpy(g->Mv, m2.Mv, sizeof g->Mv);
  memcpy(g->Mx, m2.Mx, sizeof g->Mx);
  maxw m3;
  maxw_moments(g->Wv, 0.0, g->lam, K, 0, &m3);  /* w moments: the same recurrence about W */
  memcpy(g->Mw, m3.Mu, sizeof g->Mw);
}

/* coef * u^i v^j w^l (xi^2)^k */
typedef struct {
  double c;
  int i, j, l, k;
} term3;
typedef struct {
  int n;
  term3 t[96];
} poly3;

static void p3_push(poly3* p, double c, int i, int j, int l, int k) {
  p->t[p->n].c = c;
  p->t[p->n].i = i;
  p->t[p->n].j = j;
  p->t[p->n].l = l;
  p->t[p->n].k = k;
  p->n++;
}
static void p3_mono(poly3* p, int i, int j, int l) {
  p->n = 0;
  p3_push(p, 1.0, i, j, l, 0);
}

/* psi: (1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2) */
static void psi3(int alpha, poly3* p) {
  p->n = 0;
  if (alpha < 4) {
    p3_push(p, 1.0, alpha == 1, alpha == 2, alpha == 3, 0);
    return;
  }
  p3_push(p, 0.5, 2, 0, 0, 0);
  p3_push(p, 0.5, 0, 2, 0, 0);
  p3_push(p, 0.5, 0, 0, 2, 0);
  p3_push(p, 0.5, 0, 0, 0, 1);
}

static void a3_poly(const double* a, poly3* p) {
  poly3 ps;
  p->n = 0;
  for (int al = 0; al < NC3; ++al) {
    psi3(al, &ps);
    for (int s = 0; s < ps.n; ++s) p3_push(p, a[al] * ps.t[s].c, ps.t[s].i, ps.t[s].j, ps.t[s].l, ps.t[s].k);
  }
}

static double mom3d(const maxw3* g, int half, int i, int j, int l, int k) {
  return (half ? g->Mh[i] : g->Mu[i]) * g->Mv[j] * g->Mw[l] * g->Mx[k];
}

/* out[alpha] = < A B psi_alpha > of the normalised Maxwellian g (half: over its half line) */
static void momvec3(const poly3* A, const poly3* B, const maxw3* g, int half, double* out) {
  poly3 ps;
  for (int al = 0; al < NC3; ++al) {
    psi3(al, &ps);
    double s = 0.0;
    for (int a = 0; a < A->n; ++a)
      for (int b = 0; b < B->n; ++b)
        for (int r = 0; r < ps.n; ++r) {
          const term3 *x = &A->t[a], *y = &B->t[b], *z = &ps.t[r];
          s += x->c * y->c * z->c * mom3d(g, half, x->i + y->i + z->i, x->j + y->j + z->j, x->l + y->l + z->l,
                                          x->k + y->k + z->k);
        }
    out[al] = s;
  }
}

/* <a psi> = b with the 5 x 5 moment matrix <psi_alpha psi_beta> of g */
static void solve_slope3(const maxw3* g, const double* b, double* a) {
  double M[25], col[NC3];
  poly3 one, ps;
  p3_mono(&one, 0, 0, 0);
  for (int be = 0; be < NC3; ++be) {
    psi3(be, &ps);
    momvec3(&ps, &one, g, 0, col);
    for (int al = 0; al < NC3; ++al) M[al * NC3 + be] = col[al];
  }
  lin_solve(NC3, M, b, a);
}

/* Flux of Eq. (equ10) integrated over [0, dt] (Fd) and [0, dt/2] (Fh) at one point, frame components
 * (rho, normal, first and second tangential momentum, energy); Wn, Wa, Wb: normal and tangential
 * derivatives of each side's reconstructed state. */
static void gp_flux3(const params* pp, const double* Wl, const double* Wnl, const double* Wal, const double* Wbl,
                     const double* Wr, const double* Wnr, const double* War, const double* Wbr, double dt,
                     double* Fd, double* Fh) {
  const double* Ws[2] = {Wl, Wr};
  const double* Dn[2] = {Wnl, Wnr};
  const double* Da[2] = {Wal, War};
  const double* Db[2] = {Wbl, Wbr};
  poly3 one, pu, pv, pw, puu, puv, puw;
  p3_mono(&one, 0, 0, 0);
  p3_mono(&pu, 1, 0, 0);
  p3_mono(&pv, 0, 1, 0);
  p3_mono(&pw, 0, 0, 1);
  p3_mono(&puu, 2, 0, 0);
  p3_mono(&puv, 1, 1, 0);
  p3_mono(&puw, 1, 0, 1);
  double Wc[NC3] = {0}, Wnc[NC3] = {0}, Wac[NC3] = {0}, Wbc[NC3] = {0};
  double M4a[NC3] = {0}, M4b[NC3] = {0}, M5[NC3] = {0};
  double t1[NC3], t2[NC3], t3[NC3], b[NC3];
  double pside[2], rside[2];
  for (int s = 0; s < 2; ++s) {
    maxw3 g;
    maxw3_from_W(pp->K, pp->gamma, Ws[s], s == 0 ? +1 : -1, &g); /* g_l over u > 0, g_r over u < 0 */
    pside[s] = g.rho / (2.0 * g.lam);
    rside[s] = g.rho;
    double an[NC3], aa[NC3], ab[NC3], A[NC3];
    for (int c = 0; c < NC3; ++c) b[c] = Dn[s][c] / g.rho;
    solve_slope3(&g, b, an);
    for (int c = 0; c < NC3; ++c) b[c] = Da[s][c] / g.rho;
    solve_slope3(&g, b, aa);
    for (int c = 0; c < NC3; ++c) b[c] = Db[s][c] / g.rho;
    solve_slope3(&g, b, ab);
    poly3 pan, paa, pab, pA;
    a3_poly(an, &pan);
    a3_poly(aa, &paa);
    a3_poly(ab, &pab);
    /* compatibility: <a_n u + a_a v + a_b w + A> = 0 */
    momvec3(&pan, &pu, &g, 0, t1);
    momvec3(&paa, &pv, &g, 0, t2);
    momvec3(&pab, &pw, &g, 0, t3);
    for (int c = 0; c < NC3; ++c) b[c] = -(t1[c] + t2[c] + t3[c]);
    solve_slope3(&g, b, A);
    a3_poly(A, &pA);
    /* equilibrium state and its slopes, Eq. (equ46)-(equ47) */
    momvec3(&one, &one, &g, 1, t1);
    for (int c = 0; c < NC3; ++c) Wc[c] += g.rho * t1[c];
    momvec3(&pan, &one, &g, 1, t1);
    for (int c = 0; c < NC3; ++c) Wnc[c] += g.rho * t1[c];
    momvec3(&paa, &one, &g, 1, t1);
    for (int c = 0; c < NC3; ++c) Wac[c] += g.rho * t1[c];
    momvec3(&pab, &one, &g, 1, t1);
    for (int c = 0; c < NC3; ++c) Wbc[c] += g.rho * t1[c];
    /* free transport terms of Eq. (equ10) */
    momvec3(&one, &pu, &g, 1, t1);
    for (int c = 0; c < NC3; ++c) M4a[c] += g.rho * t1[c];
    momvec3(&pA, &pu, &g, 1, t1);
    for (int c = 0; c < NC3; ++c) M4b[c] += g.rho * t1[c];
    momvec3(&pan, &puu, &g, 1, t1);
    momvec3(&paa, &puv, &g, 1, t2);
    momvec3(&pab, &puw, &g, 1, t3);
    for (int c = 0; c < NC3; ++c) M5[c] += g.rho * (t1[c] + t2[c] + t3[c]);
  }
  maxw3 g0;
  maxw3_from_W(pp->K, pp->gamma, Wc, 0, &g0);
  /* interface vacuum: no flux (the rule of two dimensions) */
  if (pside[0] > 0.0 && pside[0] < INFINITY && pside[1] > 0.0 && pside[1] < INFINITY &&
      g0.rho <= 0x1p-53 * fmin(rside[0], rside[1]) && !(g0.rho > 0.0 && g0.lam > 0.0 && g0.lam < INFINITY)) {
    for (int c = 0; c < NC3; ++c) Fd[c] = Fh[c] = 0.0;
    return;
  }
  double a0[NC3], b0[NC3], c0[NC3], A0[NC3];
  for (int c = 0; c < NC3; ++c) b[c] = Wnc[c] / g0.rho;
  solve_slope3(&g0, b, a0);
  for (int c = 0; c < NC3; ++c) b[c] = Wac[c] / g0.rho;
  solve_slope3(&g0, b, b0);
  for (int c = 0; c < NC3; ++c) b[c] = Wbc[c] / g0.rho;
  solve_slope3(&g0, b, c0);
  poly3 pa0, pb0, pc0, pA0;
  a3_poly(a0, &pa0);
  a3_poly(b0, &pb0);
  a3_poly(c0, &pc0);
  momvec3(&pa0, &pu, &g0, 0, t1);
  momvec3(&pb0, &pv, &g0, 0, t2);
  momvec3(&pc0, &pw, &g0, 0, t3);
  for (int c = 0; c < NC3; ++c) b[c] = -(t1[c] + t2[c] + t3[c]);
  solve_slope3(&g0, b, A0);
  a3_poly(A0, &pA0);
  double M1[NC3], M2[NC3], M3[NC3];
  momvec3(&one, &pu, &g0, 0, M1);
  momvec3(&pa0, &puu, &g0, 0, t1);
  momvec3(&pb0, &puv, &g0, 0, t2);
  momvec3(&pc0, &puw, &g0, 0, t3);
  momvec3(&pA0, &pu, &g0, 0, M3);
  for (int c = 0; c < NC3; ++c) {
    M1[c] *= g0.rho;
    M2[c] = g0.rho * (t1[c] + t2[c] + t3[c]);
    M3[c] *= g0.rho;
  }
  double jump = fabs((pside[0] - pside[1]) / (pside[0] + pside[1]));
  double p0 = g0.rho / (2.0 * g0.lam);
  double tau = pp->ns ? pp->mu / p0 + pp->c2 * jump * dt : pp->c1 * dt + pp->c2 * jump * dt;
  double deltas[2] = {dt, 0.5 * dt};
  double* outs[2] = {Fd, Fh};
  for (int m = 0; m < 2; ++m) {
    double C[5];
    time_coeffs(deltas[m], tau, C);
    for (int c = 0; c < NC3; ++c)
      outs[m][c] = C[0] * M1[c] + C[1] * M2[c] + C[2] * M3[c] + C[3] * (M4a[c] - tau * M4b[c]) - C[4] * M5[c];
  }
}

/* Right eigenvectors of the 3D Euler flux Jacobian in frame slot dir (1: normal, 2, 3: tangential),
 * state in frame components; columns: u_d - c, entropy, the two shear waves, u_d + c. */
static void char_R3(int dir, const double* W, double gamma, double* R) {
  double rho = W[0];
  double u[3] = {W[1] / rho, W[2] / rho, W[3] / rho};
  double q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double p = (gamma - 1.0) * (W[4] - 0.5 * rho * q2);
  double c = sqrt(gamma * p / rho);
  double H = (W[4] + p) / rho;
  int d = dir - 1;
  memset(R, 0, sizeof(double) * 25);
  R[0 * 5 + 0] = 1.0;
  for (int m = 0; m < 3; ++m) R[(1 + m) * 5 + 0] = u[m] - (m == d ? c : 0.0);
  R[4 * 5 + 0] = H - u[d] * c;
  R[0 * 5 + 1] = 1.0;
  for (int m = 0; m < 3; ++m) R[(1 + m) * 5 + 1] = u[m];
  R[4 * 5 + 1] = 0.5 * q2;
  int col = 2;
  for (int m = 0; m < 3; ++m) {
    if (m == d) continue;
    R[(1 + m) * 5 + col] = 1.0;
    R[4 * 5 + col] = u[m];
    col++;
  }
  R[0 * 5 + 4] = 1.0;
  for (int m = 0; m < 3; ++m) R[(1 + m) * 5 + 4] = u[m] + (m == d ? c : 0.0);
  R[4 * 5 + 4] = H + u[d] * c;
}

/* 5-cell reconstruction of a 5-vector at xi (value and xi-derivative): linear quartic per component,
 * or WENO-AO on R^{-1} q projected back with R. */
static void recon5(const params* pp, const double q5[5][NC3], double xi, int flag, const double* R,
                   const double* L, double* val, double* der) {
  double q[5], c[5];
  if (!flag) {
    for (int cc = 0; cc < NC3; ++cc) {
      for (int r = 0; r < 5; ++r) q[r] = q5[r][cc];
      stencil_coeffs(3, q, c);
      poly_eval(c, 4, xi, &val[cc], &der[cc]);
    }
    return;
  }
  double cv[NC3], cd[NC3];
  for (int k = 0; k < NC3; ++k) {
    for (int r = 0; r < 5; ++r) {
      double s = 0.0;
      for (int cc = 0; cc < NC3; ++cc) s += L[k * NC3 + cc] * q5[r][cc];
      q[r] = s;
    }
    ao_eval(q, xi, pp->ghi, pp->glo, pp->eps, &cv[k], &cd[k]);
  }
  for (int cc = 0; cc < NC3; ++cc) {
    double sv = 0.0, sd = 0.0;
    for (int k = 0; k < NC3; ++k) {
      sv += R[cc * NC3 + k] * cv[k];
      sd += R[cc * NC3 + k] * cd[k];
    }
    val[cc] = sv;
    der[cc] = sd;
  }
}

/* padded 3D state G[c][k+NG][j+NG][i+NG]: x-sides on interior (j, k), then y-sides across the padded
 * width in i (interior k), then z-sides across the padded i and j (corners follow the later side). */
typedef struct {
  int nx, ny, nz, px, py, pz;
  double* G;
} pad3;

static double* g3(const pad3* g, int c, int k, int j, int i) {
  return g->G + (((size_t)c * g->pz + (size_t)(k + NG)) * g->py + (size_t)(j + NG)) * g->px + (size_t)(i + NG);
}

static int mirror_src(int kind, int side, int idx, int n) {
  if (kind == 0) return side ? idx - n : idx + n;
  if (kind == 1) return side ? n - 1 : 0;
  return side ? 2 * n - 1 - idx : -1 - idx;
}

static void pad_state3(const oracle_problem* p, const double* W, pad3* g) {
  int nx = p->nx, ny = p->ny, nz = p->nz;
  g->nx = nx; g->ny = ny; g->nz = nz;
  g->px = nx + 2 * NG; g->py = ny + 2 * NG; g->pz = nz + 2 * NG;
  g->G = (double*)malloc(sizeof(double) * NC3 * g->px * g->py * g->pz);
  for (int c = 0; c < NC3; ++c)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) *g3(g, c, k, j, i) = W[(((size_t)c * nz + k) * ny + j) * nx + i];
  int kinds[3][2] = {{p->bc[0], p->bc[1]}, {p->bc[2], p->bc[3]}, {p->bcz[0], p->bcz[1]}};
  for (int d = 0; d < 3; ++d) {
    int n = d == 0 ? nx : d == 1 ? ny : nz;
    /* ranges of the other two indices: interior for later directions, padded for earlier ones */
    int lo[3] = {0, 0, 0}, hi[3] = {nx, ny, nz};
    for (int e = 0; e < d; ++e) { lo[e] = -NG; hi[e] = (e == 0 ? nx : ny) + NG; }
    for (int gk = 1; gk <= NG; ++gk)
      for (int side = 0; side < 2; ++side) {
        int idx = side ? n - 1 + gk : -gk;
        int kind = kinds[d][side];
        int src = mirror_src(kind, side, idx, n);
        for (int a = (d == 0 ? lo[1] : lo[0]); a < (d == 0 ? hi[1] : hi[0]); ++a)
          for (int b = (d == 2 ? lo[1] : lo[2]); b < (d == 2 ? hi[1] : hi[2]); ++b) {
            /* (i, j, k) of the ghost and of its source */
            int i, j, k, si, sj, sk;
            if (d == 0) { j = a; k = b; i = idx; si = src; sj = j; sk = k; }
            else if (d == 1) { i = a; k = b; j = idx; si = i; sj = src; sk = k; }
            else { i = a; j = b; k = idx; si = i; sj = j; sk = src; }
            for (int c = 0; c < NC3; ++c) {
              double v = *g3(g, c, sk, sj, si);
              if ((kind == 2 && c == 1 + d) || (kind == 3 && c >= 1 && c <= 3)) v = -v;
              *g3(g, c, k, j, i) = v;
            }
          }
      }
  }
}

/* Frame of direction d: normal index n = axis d, first tangential a = axis (d+1)%3, second b = axis
 * (d+2)%3, all padded by NG; components rotated to (rho, m_n, m_a, m_b, E). */
typedef struct {
  int nn, na, nb, pn, pa, pb;
  double hn, ha, hb;
  double* P;
} frame3;

static double* f3(const frame3* f, int c, int b, int a, int n) {
  return f->P + (((size_t)c * f->pb + (size_t)(b + NG)) * f->pa + (size_t)(a + NG)) * f->pn + (size_t)(n + NG);
}

static void build_frame3(const oracle_problem* p, const pad3* g, int d, frame3* f) {
  int N[3] = {p->nx, p->ny, p->nz};
  double h[3] = {(p->x1 - p->x0) / p->nx, (p->y1 - p->y0) / p->ny, (p->z1 - p->z0) / p->nz};
  int da = (d + 1) % 3, db = (d + 2) % 3;
  f->nn = N[d]; f->na = N[da]; f->nb = N[db];
  f->hn = h[d]; f->ha = h[da]; f->hb = h[db];
  f->pn = f->nn + 2 * NG; f->pa = f->na + 2 * NG; f->pb = f->nb + 2 * NG;
  f->P = (double*)malloc(sizeof(double) * NC3 * f->pn * f->pa * f->pb);
  for (int b = -NG; b < f->nb + NG; ++b)
    for (int a = -NG; a < f->na + NG; ++a)
      for (int n = -NG; n < f->nn + NG; ++n) {
        int ix[3];
        ix[d] = n; ix[da] = a; ix[db] = b;
        double v[NC3];
        for (int c = 0; c < NC3; ++c) v[c] = *g3(g, c, ix[2], ix[1], ix[0]);
        double m[3] = {v[1], v[2], v[3]};
        v[1] = m[d]; v[2] = m[da]; v[3] = m[db];
        for (int c = 0; c < NC3; ++c) *f3(f, c, b, a, n) = v[c];
      }
}

/* troubled flag of padded cell (n, a, b) along frame axis ax (0 normal, 1 a, 2 b), widened: OR of the
 * cell and its two neighbours along that axis, each an OR over the five components (Steps 1-4) */
static int t3_cell(const frame3* f, const params* pp, int ax, int n, int a, int b) {
  double q[5], xb, xh;
  int st, T = 0;
  double hh = ax == 0 ? f->hn : ax == 1 ? f->ha : f->hb;
  for (int c = 0; c < NC3; ++c) {
    for (int r = 0; r < 5; ++r) {
      int o = r - 2;
      q[r] = *f3(f, c, b + (ax == 2 ? o : 0), a + (ax == 1 ? o : 0), n + (ax == 0 ? o : 0));
    }
    T |= troubled_component(q, hh, pp->zeta1_mode, &xb, &xh, &st);
  }
  return T;
}

static int flag3(const frame3* f, const params* pp, int ax, int n, int a, int b) {
  if (pp->recon == 1) return 1;
  if (pp->recon == 2) return 0;
  int F = 0;
  for (int o = -1; o <= 1; ++o)
    F |= t3_cell(f, pp, ax, n + (ax == 0 ? o : 0), a + (ax == 1 ? o : 0), b + (ax == 2 ? o : 0));
  return F;
}

/* Fd, Fh: [c][b][a][n] (interfaces n = 0..nn) in frame components */
static void frame_fluxes3(const frame3* f, const params* pp, double dt, double* Fd, double* Fh, int nthreads) {
  int nn = f->nn, na = f->na, nb = f->nb;
  int la = na + 4, lb = nb + 4;  /* line values on tangential rows -2..n+1 */
  size_t lsz = (size_t)lb * la * (nn + 1);
#define LV3(kind, c, b, a, k) LV[(((size_t)(kind) * NC3 + (c)) * lsz) + (((size_t)((b) + 2) * la + (size_t)((a) + 2)) * (nn + 1)) + (k)]
  double* LV = (double*)malloc(sizeof(double) * 4 * NC3 * lsz);
  /* normal reconstruction of every line (Sec. 2.3.1 applied along the face normal) */
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(dynamic, 1)
  for (int b = -2; b < nb + 2; ++b)
    for (int a = -2; a < na + 2; ++a)
      for (int k = 0; k <= nn; ++k) {
        double q5[5][NC3], R[25], L[25], avg[NC3], val[NC3], der[NC3];
        int fl = flag3(f, pp, 0, k - 1, a, b), fr = flag3(f, pp, 0, k, a, b);
        if (fl || fr) {
          for (int c = 0; c < NC3; ++c) avg[c] = 0.5 * (*f3(f, c, b, a, k - 1) + *f3(f, c, b, a, k));
          char_R3(1, avg, pp->gamma, R);
          mat_inverse(NC3, R, L);
        }
        for (int s = 0; s < 2; ++s) {
          int cell = k - 1 + s;
          for (int r = 0; r < 5; ++r)
            for (int c = 0; c < NC3; ++c) q5[r][c] = *f3(f, c, b, a, cell - 2 + r);
          recon5(pp, q5, s == 0 ? 0.5 : -0.5, s == 0 ? fl : fr, R, L, val, der);
          for (int c = 0; c < NC3; ++c) {
            LV3(2 * s, c, b, a, k) = val[c];
            LV3(2 * s + 1, c, b, a, k) = der[c] / f->hn;
          }
        }
      }
  const double eta = 1.0 / (2.0 * sqrt(3.0));
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(dynamic, 1)
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < na; ++a)
      for (int k = 0; k <= nn; ++k) {
        double sumd[NC3] = {0}, sumh[NC3] = {0};
        for (int m1 = 0; m1 < 2; ++m1)
          for (int m2 = 0; m2 < 2; ++m2) {
            double x1 = m1 ? eta : -eta, x2 = m2 ? eta : -eta;
            double Wp[2][NC3], Wn[2][NC3], Wa[2][NC3], Wb[2][NC3];
            for (int s = 0; s < 2; ++s) {
              int cell = k - 1 + s;
              /* step 1: along a, on the five b-rows, at x1 */
              double V1[5][NC3], D1[5][NC3], N1[5][NC3];
              for (int r2 = 0; r2 < 5; ++r2) {
                int bb = b - 2 + r2;
                int fa = flag3(f, pp, 1, cell, a, bb);
                double R[25], L[25], own[NC3], q5[5][NC3], val[NC3], der[NC3];
                if (fa) {
                  for (int c = 0; c < NC3; ++c) own[c] = LV3(2 * s, c, bb, a, k);
                  char_R3(2, own, pp->gamma, R);
                  mat_inverse(NC3, R, L);
                }
                for (int r = 0; r < 5; ++r)
                  for (int c = 0; c < NC3; ++c) q5[r][c] = LV3(2 * s, c, bb, a - 2 + r, k);
                recon5(pp, q5, x1, fa, R, L, val, der);
                for (int c = 0; c < NC3; ++c) { V1[r2][c] = val[c]; D1[r2][c] = der[c] / f->ha; }
                for (int r = 0; r < 5; ++r)
                  for (int c = 0; c < NC3; ++c) q5[r][c] = LV3(2 * s + 1, c, bb, a - 2 + r, k);
                recon5(pp, q5, x1, fa, R, L, val, der);
                for (int c = 0; c < NC3; ++c) N1[r2][c] = val[c];
              }
              /* step 2: along b at x2 */
              int fb = flag3(f, pp, 2, cell, a, b);
              double R[25], L[25], val[NC3], der[NC3];
              if (fb) {
                char_R3(3, V1[2], pp->gamma, R);
                mat_inverse(NC3, R, L);
              }
              recon5(pp, (const double(*)[NC3])V1, x2, fb, R, L, val, der);
              for (int c = 0; c < NC3; ++c) { Wp[s][c] = val[c]; Wb[s][c] = der[c] / f->hb; }
              recon5(pp, (const double(*)[NC3])D1, x2, fb, R, L, val, der);
              for (int c = 0; c < NC3; ++c) Wa[s][c] = val[c];
              recon5(pp, (const double(*)[NC3])N1, x2, fb, R, L, val, der);
              for (int c = 0; c < NC3; ++c) Wn[s][c] = val[c];
            }
            double Fdg[NC3], Fhg[NC3];
            gp_flux3(pp, Wp[0], Wn[0], Wa[0], Wb[0], Wp[1], Wn[1], Wa[1], Wb[1], dt, Fdg, Fhg);
            for (int c = 0; c < NC3; ++c) {
              sumd[c] += 0.25 * Fdg[c];
              sumh[c] += 0.25 * Fhg[c];
            }
          }
        for (int c = 0; c < NC3; ++c) {
          size_t o = (((size_t)c * nb + b) * na + a) * (nn + 1) + k;
          Fd[o] = sumd[c];
          Fh[o] = sumh[c];
        }
      }
#undef LV3
  free(LV);
}

/* time-integrated fluxes of the three directions in grid components:
 * x [5][nz][ny][nx+1], y [5][nz][ny+1][nx], z [5][nz+1][ny][nx] */
static void all_fluxes3(const oracle_problem* p, const params* pp, const double* W, double dt, double* Fd[3],
                        double* Fh[3], int nthreads) {
  pad3 g;
  pad_state3(p, W, &g);
  int N[3] = {p->nx, p->ny, p->nz};
  for (int d = 0; d < 3; ++d) {
    frame3 f;
    build_frame3(p, &g, d, &f);
    int da = (d + 1) % 3, db = (d + 2) % 3;
    size_t nf = (size_t)NC3 * f.nb * f.na * (f.nn + 1);
    double* td = (double*)malloc(sizeof(double) * nf);
    double* th = (double*)malloc(sizeof(double) * nf);
    frame_fluxes3(&f, pp, dt, td, th, nthreads);
    free(f.P);
    int M[3] = {N[0], N[1], N[2]};
    M[d] += 1;
    for (int c = 0; c < NC3; ++c) {
      int cs = c;  /* frame slot of grid component c */
      if (c >= 1 && c <= 3) {
        int axis = c - 1;
        cs = axis == d ? 1 : axis == da ? 2 : 3;
      }
      for (int b = 0; b < f.nb; ++b)
        for (int a = 0; a < f.na; ++a)
          for (int n = 0; n <= f.nn; ++n) {
            int ix[3];
            ix[d] = n; ix[da] = a; ix[db] = b;
            size_t go = (((size_t)c * M[2] + ix[2]) * M[1] + ix[1]) * M[0] + ix[0];
            size_t fo = (((size_t)cs * f.nb + b) * f.na + a) * (f.nn + 1) + n;
            Fd[d][go] = td[fo];
            Fh[d][go] = th[fo];
          }
    }
    free(td);
    free(th);
  }
  free(g.G);
}

static int admissible3(const oracle_problem* p, const double* W, size_t s) {
  size_t nc = (size_t)p->nx * p->ny * p->nz;
  double rho = W[s], mx = W[nc + s], my = W[2 * nc + s], mz = W[3 * nc + s], E = W[4 * nc + s];
  double pr = (p->gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho);
  return rho > 0.0 && pr > 0.0 && isfinite(E);
}

double oracle_cfl_dt3(const oracle_problem* p, const double* W) {
  size_t nc = (size_t)p->nx * p->ny * p->nz;
  double h = fmin(fmin((p->x1 - p->x0) / p->nx, (p->y1 - p->y0) / p->ny), (p->z1 - p->z0) / p->nz);
  double qmin = INFINITY;
  for (size_t s = 0; s < nc; ++s) {
    double rho = W[s], U = W[nc + s] / rho, V = W[2 * nc + s] / rho, Z = W[3 * nc + s] / rho;
    double pr = (p->gamma - 1.0) * (W[4 * nc + s] - 0.5 * rho * (U * U + V * V + Z * Z));
    double c = sqrt(p->gamma * pr / rho);
    double q = h / (sqrt(U * U + V * V + Z * Z) + c);
    if (p->eqn == 1) q = fmin(q, (h * h) / (4.0 * (p->mu / (p->viscous_dt_mode ? pr : rho))));
    qmin = fmin(qmin, q);
  }
  return p->cfl * qmin;
}

static int check_problem3(const oracle_problem* p) {
  if (p->nx < 5 || p->ny < 5 || p->nz < 5) return ORACLE_EINVAL;
  if (!(p->gamma > 1.0) || !(p->x1 > p->x0) || !(p->y1 > p->y0) || !(p->z1 > p->z0)) return ORACLE_EINVAL;
  if (p->eqn == 1 && !(p->Pr == 1.0 && p->mu >= 0.0)) return ORACLE_EINVAL;
  if (p->positivity != 0 || p->tangential_flag_mode != 0 || p->char_state_mode != 0) return ORACLE_EINVAL;
  if (p->viscous_dt_mode != 0 && p->viscous_dt_mode != 1) return ORACLE_EINVAL;
  int k[6] = {p->bc[0], p->bc[1], p->bc[2], p->bc[3], p->bcz[0], p->bcz[1]};
  for (int s = 0; s < 6; ++s)
    if (k[s] < 0 || k[s] > 3) return ORACLE_EINVAL;
  for (int s = 0; s < 6; s += 2)
    if ((k[s] == 0) != (k[s + 1] == 0)) return ORACLE_EINVAL;
  return ORACLE_OK;
}

static void make_params3(const oracle_problem* p, params* pp) {
  make_params(p, pp);
  pp->dim = 3;
  pp->nc = NC3;
  pp->K = (5.0 - 3.0 * p->gamma) / (p->gamma - 1.0);
}

int oracle_stage_fluxes3(const oracle_problem* p, const double* W, double dt, double* F[3], double* G[3],
                         int nthreads) {
  oracle_init();
  int rc = check_problem3(p);
  if (rc) return rc;
  params pp;
  make_params3(p, &pp);
  int N[3] = {p->nx, p->ny, p->nz};
  double *Fd[3], *Fh[3];
  size_t nf[3];
  for (int d = 0; d < 3; ++d) {
    nf[d] = (size_t)NC3 * (N[0] + (d == 0)) * (N[1] + (d == 1)) * (N[2] + (d == 2));
    Fd[d] = (double*)malloc(sizeof(double) * nf[d]);
    Fh[d] = (double*)malloc(sizeof(double) * nf[d]);
  }
  all_fluxes3(p, &pp, W, dt, Fd, Fh, nthreads);
  for (int d = 0; d < 3; ++d) {
    for (size_t s = 0; s < nf[d]; ++s) {
      F[d][s] = (4.0 * Fh[d][s] - Fd[d][s]) / dt;
      G[d][s] = 4.0 * (Fd[d][s] - 2.0 * Fh[d][s]) / (dt * dt);
    }
    free(Fd[d]);
    free(Fh[d]);
  }
  return ORACLE_OK;
}

int oracle_flags3(const oracle_problem* p, const double* W, uint8_t* f[3]) {
  oracle_init();
  int rc = check_problem3(p);
  if (rc) return rc;
  params pp;
  make_params3(p, &pp);
  pad3 g;
  pad_state3(p, W, &g);
  for (int d = 0; d < 3; ++d) {
    frame3 fr;
    build_frame3(p, &g, d, &fr);
    int da = (d + 1) % 3, db = (d + 2) % 3;
    for (int b = 0; b < fr.nb; ++b)
      for (int a = 0; a < fr.na; ++a)
        for (int n = 0; n < fr.nn; ++n) {
          int ix[3];
          ix[d] = n; ix[da] = a; ix[db] = b;
          f[d][((size_t)ix[2] * p->ny + ix[1]) * p->nx + ix[0]] = (uint8_t)flag3(&fr, &pp, 0, n, a, b);
        }
    free(fr.P);
  }
  free(g.G);
  return ORACLE_OK;
}

/* one S2O4 step (Sec. 2.2) of a 3D problem */
static int step3(const oracle_problem* p, double* W, double* t, double t_end, double* dt_taken, int nthreads) {
  int rc = check_problem3(p);
  if (rc) return rc;
  params pp;
  make_params3(p, &pp);
  if (dt_taken) *dt_taken = 0.0;
  if (*t >= t_end) return ORACLE_OK;
  double dt = (p->fixed_dt > 0.0) ? p->fixed_dt : oracle_cfl_dt3(p, W);
  if (!(dt > 0.0) || !isfinite(dt)) return ORACLE_EDT;
  double tnew;
  if (*t + dt >= t_end) { dt = t_end - *t; tnew = t_end; }
  else tnew = *t + dt;
  int N[3] = {p->nx, p->ny, p->nz};
  double h[3] = {(p->x1 - p->x0) / p->nx, (p->y1 - p->y0) / p->ny, (p->z1 - p->z0) / p->nz};
  size_t ncell = (size_t)N[0] * N[1] * N[2];
  double *Fd[3], *Fh[3], *F[3], *Gn[3];
  size_t nf[3];
  for (int d = 0; d < 3; ++d) {
    nf[d] = (size_t)NC3 * (N[0] + (d == 0)) * (N[1] + (d == 1)) * (N[2] + (d == 2));
    Fd[d] = (double*)malloc(sizeof(double) * nf[d]);
    Fh[d] = (double*)malloc(sizeof(double) * nf[d]);
    F[d] = (double*)malloc(sizeof(double) * nf[d]);
    Gn[d] = (double*)malloc(sizeof(double) * nf[d]);
  }
  double* Ws = (double*)malloc(sizeof(double) * NC3 * ncell);
  /* face index of the low face of cell (i,j,k) in direction d, and the stride to its high face */
#define FACE(d, c, i, j, k) ((((size_t)(c) * (N[2] + ((d) == 2)) + (k)) * (N[1] + ((d) == 1)) + (j)) * (N[0] + ((d) == 0)) + (i))
  all_fluxes3(p, &pp, W, dt, Fd, Fh, nthreads);
  for (int d = 0; d < 3; ++d)
    for (size_t s = 0; s < nf[d]; ++s) {
      F[d][s] = (4.0 * Fh[d][s] - Fd[d][s]) / dt;
      Gn[d][s] = 4.0 * (Fd[d][s] - 2.0 * Fh[d][s]) / (dt * dt);
    }
  /* W* = W^n - sum_d [F(dt/2)_hi - F(dt/2)_lo] / h_d */
  for (int c = 0; c < NC3; ++c)
    for (int k = 0; k < N[2]; ++k)
      for (int j = 0; j < N[1]; ++j)
        for (int i = 0; i < N[0]; ++i) {
          double sdiv = 0.0;
          for (int d = 0; d < 3; ++d) {
            size_t lo = FACE(d, c, i, j, k);
            size_t hi = FACE(d, c, i + (d == 0), j + (d == 1), k + (d == 2));
            sdiv += (Fh[d][hi] - Fh[d][lo]) / h[d];
          }
          size_t o = (size_t)c * ncell + ((size_t)k * N[1] + j) * N[0] + i;
          Ws[o] = W[o] - sdiv;
        }
  for (size_t s = 0; s < ncell && !rc; ++s)
    if (!admissible3(p, Ws, s)) rc = ORACLE_ENONPHYS;
  if (!rc) {
    all_fluxes3(p, &pp, Ws, dt, Fd, Fh, nthreads);
    for (int d = 0; d < 3; ++d)
      for (size_t s = 0; s < nf[d]; ++s) {
        double Gs = 4.0 * (Fd[d][s] - 2.0 * Fh[d][s]) / (dt * dt);
        F[d][s] = F[d][s] + dt / 6.0 * (Gn[d][s] + 2.0 * Gs);
      }
    for (int c = 0; c < NC3; ++c)
      for (int k = 0; k < N[2]; ++k)
        for (int j = 0; j < N[1]; ++j)
          for (int i = 0; i < N[0]; ++i) {
            double sdiv = 0.0;
            for (int d = 0; d < 3; ++d) {
              size_t lo = FACE(d, c, i, j, k);
              size_t hi = FACE(d, c, i + (d == 0), j + (d == 1), k + (d == 2));
              sdiv += (F[d][hi] - F[d][lo]) / h[d];
            }
            size_t o = (size_t)c * ncell + ((size_t)k * N[1] + j) * N[0] + i;
            Ws[o] = W[o] - dt * sdiv;
          }
    for (size_t s = 0; s < ncell && !rc; ++s)
      if (!admissible3(p, Ws, s)) rc = ORACLE_ENONPHYS;
    if (!rc) {
      memcpy(W, Ws, sizeof(double) * NC3 * ncell);
      *t = tnew;
      if (dt_taken) *dt_taken = dt;
    }
  }
#undef FACE
  for (int d = 0; d < 3; ++d) { free(Fd[d]); free(Fh[d]); free(F[d]); free(Gn[d]); }
  free(Ws);
  return rc;
}


/* ======================================================================== */
/* 9. Two-derivative multistage steps                                        */
/* ======================================================================== */
/* Sec. 2.2 writes S2O4 through the spatial operator L and its time derivative L_t and places it in the
 * multi-stage multi-derivative family; a tableau (oracle_stepper) defines a member. Each stage takes
 * the interface fluxes F and dF/dt of its own state over a window of length dt, exactly as the first
 * stage of S2O4 does; L = -sum_d (F_{d,hi} - F_{d,lo}) / h_d and L_t likewise from dF/dt. */

static int stepper_ok(const oracle_problem* p) {
  const oracle_stepper* m = &p->stepper;
  if (m->stages < 1 || m->stages > 3) return 0;
  if (p->positivity != 0) return 0;
  for (int s = 0; s < 4; ++s)
    if (p->bc[s] == 4) return 0;
  for (int i = 0; i < 3; ++i) {
    if (!isfinite(m->b[i]) || !isfinite(m->bh[i])) return 0;
    for (int j = 0; j < 3; ++j)
      if (!isfinite(m->a[i][j]) || !isfinite(m->ah[i][j])) return 0;
  }
  return 1;
}

static size_t cells_of(const oracle_problem* p) {
  return (size_t)p->nx * (p->dim >= 2 ? p->ny : 1) * (p->dim == 3 ? p->nz : 1);
}

static int admissible_any(const oracle_problem* p, const double* W) {
  size_t n = cells_of(p);
  int nc = p->dim + 2;
  for (size_t s = 0; s < n; ++s) {
    double rho = W[s], m2 = 0.0;
    for (int d = 0; d < p->dim; ++d) m2 += W[(size_t)(1 + d) * n + s] * W[(size_t)(1 + d) * n + s];
    double E = W[(size_t)(nc - 1) * n + s];
    double pr = (p->gamma - 1.0) * (E - 0.5 * m2 / rho);
    if (!(rho > 0.0) || !(pr > 0.0) || !isfinite(E)) return 0;
  }
  return 1;
}

/* L(W) and L_t(W) of every cell, [nc][cells] */
static int ms_operators(const oracle_problem* p, const double* W, double ts, double dt, double* L, double* Lt,
                        int nthreads) {
  int dim = p->dim, nc = dim + 2;
  int N[3] = {p->nx, dim >= 2 ? p->ny : 1, dim == 3 ? p->nz : 1};
  double h[3] = {(p->x1 - p->x0) / p->nx, dim >= 2 ? (p->y1 - p->y0) / p->ny : 1.0,
                 dim == 3 ? (p->z1 - p->z0) / p->nz : 1.0};
  double *F[3] = {NULL, NULL, NULL}, *G[3] = {NULL, NULL, NULL};
  for (int d = 0; d < dim; ++d) {
    size_t nf = (size_t)nc * (N[0] + (d == 0)) * (N[1] + (d == 1)) * (N[2] + (d == 2));
    F[d] = (double*)malloc(sizeof(double) * nf);
    G[d] = (double*)malloc(sizeof(double) * nf);
  }
  int rc = (dim == 3) ? oracle_stage_fluxes3(p, W, dt, F, G, nthreads)
                      : oracle_stage_fluxes(p, W, ts, dt, F[0], G[0], F[1], G[1], nthreads);
  if (!rc) {
    size_t n = cells_of(p);
#define FACE(d, c, i, j, k) ((((size_t)(c) * (N[2] + ((d) == 2)) + (k)) * (N[1] + ((d) == 1)) + (j)) * (N[0] + ((d) == 0)) + (i))
    for (int c = 0; c < nc; ++c)
      for (int k = 0; k < N[2]; ++k)
        for (int j = 0; j < N[1]; ++j)
          for (int i = 0; i < N[0]; ++i) {
            double l = 0.0, lt = 0.0;
            for (int d = 0; d < dim; ++d) {
              size_t lo = FACE(d, c, i, j, k), hi = FACE(d, c, i + (d == 0), j + (d == 1), k + (d == 2));
              l -= (F[d][hi] - F[d][lo]) / h[d];
              lt -= (G[d][hi] - G[d][lo]) / h[d];
            }
            size_t o = (size_t)c * n + ((size_t)k * N[1] + j) * N[0] + i;
            L[o] = l;
            Lt[o] = lt;
          }
#undef FACE
  }
  for (int d = 0; d < dim; ++d) {
    free(F[d]);
    free(G[d]);
  }
  return rc;
}

static int step_ms(const oracle_problem* p, double* W, double* t, double t_end, double* dt_taken, int nthreads) {
  int rc = (p->dim == 3) ? check_problem3(p) : check_problem(p);
  if (rc) return rc;
  if (!stepper_ok(p)) return ORACLE_EINVAL;
  const oracle_stepper* m = &p->stepper;
  if (dt_taken) *dt_taken = 0.0;
  if (*t >= t_end) return ORACLE_OK;
  double dt = (p->fixed_dt > 0.0) ? p->fixed_dt : oracle_cfl_dt(p, W);
  if (!(dt > 0.0) || !isfinite(dt)) return ORACLE_EDT;
  double tnew;
  if (*t + dt >= t_end) { dt = t_end - *t; tnew = t_end; }
  else tnew = *t + dt;
  int S = m->stages;
  size_t len = (size_t)(p->dim + 2) * cells_of(p);
  double* L[3];
  double* Lt[3];
  for (int i = 0; i < S; ++i) {
    L[i] = (double*)malloc(sizeof(double) * len);
    Lt[i] = (double*)malloc(sizeof(double) * len);
  }
  double* Wi = (double*)malloc(sizeof(double) * len);
  for (int i = 0; i < S && !rc; ++i) {
    /* the stage state from the earlier stages' operators */
    double ci = 0.0;
    for (size_t o = 0; o < len; ++o) {
      double w = W[o];
      for (int j = 0; j < i; ++j) w += dt * m->a[i][j] * L[j][o] + dt * dt * m->ah[i][j] * Lt[j][o];
      Wi[o] = w;
    }
    for (int j = 0; j < i; ++j) ci += m->a[i][j];
    if (i > 0 && !admissible_any(p, Wi)) { rc = ORACLE_ENONPHYS; break; }
    rc = ms_operators(p, Wi, *t + ci * dt, dt, L[i], Lt[i], nthreads);
  }
  if (!rc) {
    for (size_t o = 0; o < len; ++o) {
      double w = W[o];
      for (int i = 0; i < S; ++i) w += dt * m->b[i] * L[i][o] + dt * dt * m->bh[i] * Lt[i][o];
      Wi[o] = w;
    }
    if (!admissible_any(p, Wi)) rc = ORACLE_ENONPHYS;
  }
  if (!rc) {
    memcpy(W, Wi, sizeof(double) * len);
    *t = tnew;
    if (dt_taken) *dt_taken = dt;
  }
  for (int i = 0; i < S; ++i) {
    free(L[i]);
    free(Lt[i]);
  }
  free(Wi);
  return rc;
}
