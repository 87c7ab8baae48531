/*
 * Driver of the CPU oracle for its sanitizer build (test infrastructure): runs every entry point of
 * hgks_oracle.h on small problems that reach each code path -- 1D, 2D and 3D steps, every boundary kind
 * (prescribed states included), Navier-Stokes with a Prandtl fix, the first-order fallbacks, the
 * reconstruction and reading modes, a three-stage tableau, the stage fluxes, the unit-level functions
 * and the error returns -- so that AddressSanitizer and UndefinedBehaviorSanitizer see them all. Prints
 * one line per case and "sanitize-driver ok" at the end; any report of a sanitizer aborts the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hgks_oracle.h"

static oracle_problem base(int dim, int nx, int ny) {
  oracle_problem p;
  memset(&p, 0, sizeof p);
  p.dim = dim;
  p.nx = nx;
  p.ny = dim == 1 ? 1 : ny;
  p.nz = 1;
  p.x1 = p.y1 = p.z1 = 1.0;
  p.gamma = 1.4;
  p.Pr = 1.0;
  p.cfl = 0.5;
  p.c1 = 0.01;
  p.c2 = 1.0;
  for (int s = 0; s < 4; ++s) p.bc[s] = 1;
  p.bcz[0] = p.bcz[1] = 1;
  p.gamma_hi = p.gamma_lo = 0.85;
  p.weno_eps = 1e-8;
  return p;
}

/* conserved state of primitive (rho, u, v, w, p) into component c of an nc-component array */
static void put(double* W, size_t n, size_t i, int nc, double r, double u, double v, double w, double pr,
                double gamma) {
  const double E = pr / (gamma - 1) + 0.5 * r * (u * u + v * v + w * w);
  W[i] = r;
  W[n + i] = r * u;
  if (nc == 3) {
    W[2 * n + i] = E;
    return;
  }
  W[2 * n + i] = r * v;
  if (nc == 4) {
    W[3 * n + i] = E;
    return;
  }
  W[3 * n + i] = r * w;
  W[4 * n + i] = E;
}

/* a four-quadrant state with a little structure inside each quadrant */
static double* quadrants(const oracle_problem* p) {
  const int nc = p->dim + 2;
  const size_t n = (size_t)p->nx * p->ny * p->nz;
  double* W = malloc(sizeof(double) * nc * n);
  for (int k = 0; k < p->nz; ++k)
    for (int j = 0; j < p->ny; ++j)
      for (int i = 0; i < p->nx; ++i) {
        const double x = (i + 0.5) / p->nx, y = (j + 0.5) / p->ny, z = (k + 0.5) / p->nz;
        const int q = (x > 0.5) + 2 * (y > 0.5 || p->dim == 1) + 4 * (z > 0.5 && p->dim == 3);
        const double r = 0.3 + 0.15 * q + 0.05 * sin(7 * x + 3 * y);
        const double pr = 0.2 + 0.1 * ((q * 5) % 7);
        const size_t c = ((size_t)k * p->ny + j) * p->nx + i;
        put(W, n, c, nc, r, 0.3 * ((q & 1) ? 1 : -1), 0.2 * ((q & 2) ? -1 : 1), 0.1 * ((q & 4) ? 1 : -1), pr,
            p->gamma);
      }
  return W;
}

static double checksum(const double* W, size_t m) {
  double s = 0;
  for (size_t i = 0; i < m; ++i) s += W[i] * (1.0 + 1e-3 * (double)(i % 97));
  return s;
}

static int run(const char* name, const oracle_problem* p, int steps, int nthreads) {
  const size_t m = (size_t)(p->dim + 2) * p->nx * p->ny * p->nz;
  double* W = quadrants(p);
  double t = 0, dt = 0;
  int rc = 0;
  for (int s = 0; s < steps && rc == 0; ++s) rc = oracle_step(p, W, &t, 1e9, &dt, nthreads);
  printf("%-28s rc %d t %.6e sum %.12e\n", name, rc, t, checksum(W, m));
  free(W);
  return rc;
}

int main(void) {
  int fail = 0;

  /* 1D: outflow and reflecting ends, every reconstruction mode, both Step-1 thresholds */
  for (int recon = 0; recon < 3; ++recon) {
    oracle_problem p = base(1, 96, 1);
    p.bc[0] = 1;
    p.bc[1] = 2;
    p.recon = recon;
    p.zeta1_mode = recon == 1;
    fail |= run("1d", &p, 4, 2) != 0;
  }

  /* 2D: each boundary kind on some side, fallbacks, readings */
  {
    const int kinds[4][4] = {{1, 1, 1, 1}, {0, 0, 0, 0}, {2, 3, 2, 3}, {3, 2, 0, 0}};
    for (int c = 0; c < 4; ++c) {
      oracle_problem p = base(2, 22, 19);
      memcpy(p.bc, kinds[c], sizeof p.bc);
      p.positivity = c & 1;
      p.tangential_flag_mode = c >= 2;
      p.char_state_mode = c == 3;
      p.recon = c == 1 ? 1 : 0;
      fail |= run("2d", &p, 3, 3) != 0;
    }
  }

  /* 2D prescribed states on the x-low and y-high sides (a moving front on the latter) */
  {
    oracle_problem p = base(2, 24, 8);
    p.x1 = 3.0;
    p.bc[0] = 4;
    p.bc[1] = 1;
    p.bc[2] = 2;
    p.bc[3] = 4;
    p.positivity = 1;
    const double a[4] = {1.5, 1.5 * 0.6, -1.5 * 0.3, 1.5 / 0.4 + 0.5 * 1.5 * (0.6 * 0.6 + 0.3 * 0.3)};
    const double b[4] = {0.8, 0, 0, 0.5 / 0.4};
    for (int s = 0; s < 4; ++s) {
      memcpy(p.bcd[s].a, a, sizeof a);
      memcpy(p.bcd[s].b, b, sizeof b);
    }
    p.bcd[0].s0 = 1e9;
    p.bcd[0].rest = 4;
    p.bcd[3].s0 = 0.17;
    p.bcd[3].sn = 0.577;
    p.bcd[3].st = 11.5;
    p.bcd[3].rest = 4;
    fail |= run("2d prescribed", &p, 3, 2) != 0;
  }

  /* Navier-Stokes, Pr = 0.73, no-slip walls, both viscous time-step readings */
  for (int mode = 0; mode < 2; ++mode) {
    oracle_problem p = base(2, 16, 12);
    p.eqn = 1;
    p.mu = 2e-3;
    p.Pr = 0.73;
    p.bc[0] = p.bc[1] = p.bc[2] = 3;
    p.bc[3] = 2;
    p.viscous_dt_mode = mode;
    fail |= run("ns", &p, 3, 2) != 0;
  }

  /* 3D, outflow and periodic z sides */
  {
    oracle_problem p = base(3, 8, 7);
    p.nz = 6;
    p.bcz[0] = 0;
    p.bcz[1] = 0;
    fail |= run("3d", &p, 2, 2) != 0;
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    double* W = quadrants(&p);
    uint8_t* f[3];
    double *F[3], *G[3];
    const size_t nf[3] = {(size_t)(p.nx + 1) * p.ny * p.nz, (size_t)p.nx * (p.ny + 1) * p.nz,
                          (size_t)p.nx * p.ny * (p.nz + 1)};
    for (int d = 0; d < 3; ++d) {
      f[d] = malloc(n);
      F[d] = malloc(sizeof(double) * 5 * nf[d]);
      G[d] = malloc(sizeof(double) * 5 * nf[d]);
    }
    const double dt = 0.5 * oracle_cfl_dt3(&p, W);
    fail |= oracle_flags3(&p, W, f) != 0;
    fail |= oracle_stage_fluxes3(&p, W, dt, F, G, 2) != 0;
    printf("%-28s dt %.6e F %.12e\n", "3d fluxes", dt, checksum(F[2], 5 * nf[2]));
    for (int d = 0; d < 3; ++d) {
      free(f[d]);
      free(F[d]);
      free(G[d]);
    }
    free(W);
  }

  /* a three-stage two-derivative tableau */
  {
    oracle_problem p = base(2, 14, 14);
    for (int s = 0; s < 4; ++s) p.bc[s] = 0;
    p.stepper.stages = 3;
    p.stepper.a[1][0] = 1.0 / 3;
    p.stepper.a[2][0] = p.stepper.a[2][1] = 1.0 / 3;
    p.stepper.ah[1][0] = p.stepper.ah[2][0] = p.stepper.ah[2][1] = 1.0 / 18;
    for (int i = 0; i < 3; ++i) {
      p.stepper.b[i] = 1.0 / 3;
      p.stepper.bh[i] = 1.0 / 18;
    }
    fail |= run("3-stage tableau", &p, 2, 2) != 0;
  }

  /* 2D stage fluxes and flags on a non-square grid */
  {
    oracle_problem p = base(2, 13, 9);
    const size_t n = (size_t)p.nx * p.ny;
    double* W = quadrants(&p);
    double* Fx = malloc(sizeof(double) * 4 * (p.nx + 1) * p.ny);
    double* Gx = malloc(sizeof(double) * 4 * (p.nx + 1) * p.ny);
    double* Fy = malloc(sizeof(double) * 4 * p.nx * (p.ny + 1));
    double* Gy = malloc(sizeof(double) * 4 * p.nx * (p.ny + 1));
    uint8_t* fx = malloc(n);
    uint8_t* fy = malloc(n);
    const double dt = oracle_cfl_dt(&p, W);
    fail |= oracle_flags(&p, W, 0.0, fx, fy) != 0;
    fail |= oracle_stage_fluxes(&p, W, 0.0, dt, Fx, Gx, Fy, Gy, 3) != 0;
    printf("%-28s dt %.6e F %.12e\n", "2d fluxes", dt, checksum(Fy, 4 * (size_t)p.nx * (p.ny + 1)));
    free(Fx);
    free(Gx);
    free(Fy);
    free(Gy);
    free(fx);
    free(fy);
    free(W);
  }

  /* unit-level entry points */
  {
    const double q[5] = {1.0, 1.2, 0.7, 3.0, 2.9};
    double v, d, s = 0;
    for (int k = 0; k < 4; ++k) {
      oracle_stencil_eval(k, q, 0.3, &v, &d);
      s += v + d + oracle_beta(k, q);
    }
    oracle_ao_eval(q, -0.5, 0.85, 0.85, 1e-8, &v, &d);
    s += v + d;
    double xbar, xhat;
    int step;
    s += oracle_indicator(q, 0.01, 0, &xbar, &xhat, &step) + step;
    if (step == 3) s += xbar + xhat;
    double R[25], L[25];
    const double W1[3] = {1.0, 0.3, 2.6}, Wc[4] = {1.0, 0.3, -0.2, 2.6};
    for (int dim = 1; dim <= 2; ++dim)
      for (int dir = 1; dir <= dim; ++dir) {
        oracle_char_matrices(dim, dir, dim == 1 ? W1 : Wc, 1.4, R, L);
        s += R[0] + L[dim + 1];
      }
    double Mu[9], Mv[9], Mxi[4];
    for (int half = -1; half <= 1; ++half) {
      oracle_maxwell_moments(1.0, 0.3, -0.2, 1.7, 3.0, half, Mu, Mv, Mxi);
      s += Mu[8] + Mv[8] + Mxi[3];
    }
    const double b[4] = {0.1, -0.2, 0.05, 0.3};
    double a[4];
    oracle_slope_solve(2, Wc, 1.4, b, a);
    double C[6];
    oracle_time_coeffs(0.01, 1e-4, C);
    oracle_problem p = base(2, 4, 4);
    const double Wl[4] = {1.0, 0.3, 0.1, 2.5}, Wr[4] = {0.5, 0.1, 0.0, 1.2}, z[4] = {0.1, 0.0, 0.0, 0.2};
    double Fdt[4], Fdt2[4], tau;
    oracle_gp_flux(&p, Wl, z, z, Wr, z, z, 0.01, Fdt, Fdt2, &tau);
    s += a[0] + C[0] + Fdt[0] + Fdt2[3] + tau;
    printf("%-28s %.12e\n", "units", s);
    fail |= !isfinite(s);
  }

  /* error returns: an invalid problem and a non-physical state */
  {
    oracle_problem p = base(2, 0, 8);
    double W1[4] = {1, 0, 0, 2.5}, t = 0, dt = 0;
    const int e1 = oracle_step(&p, W1, &t, 1.0, &dt, 1);
    p = base(2, 6, 6);
    double* W = quadrants(&p);
    W[3 * 36 + 14] = -1.0; /* rho E < 0 in one cell */
    const int e2 = oracle_step(&p, W, &t, 1.0, &dt, 2);
    free(W);
    printf("%-28s %d %d\n", "errors", e1, e2);
    fail |= e1 != ORACLE_EINVAL || e2 != ORACLE_ENONPHYS;
  }

  if (fail) {
    printf("sanitize-driver FAILED\n");
    return 1;
  }
  printf("sanitize-driver ok\n");
  return 0;
}
