// Device-side arithmetic of the hybrid WENO5-AO gas-kinetic scheme (Mu et al., arXiv 2304.05572),
// written for CDNA4 (gfx950): one thread evaluates one interface, everything in registers except the
// LDS-staged stencil tiles owned by the kernels. Templated on the bulk precision T (double for the
// FP64 path, float for the FP32-bulk path); the troubled-cell discriminant, the CFL quantity and the
// time-integration coefficients are always FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

// ---------------------------------------------------------------------------------------------
// Per-problem description and time state (device copies)
// ---------------------------------------------------------------------------------------------
// A prescribed-state side: ghost centres with tangential coordinate tau < s0 + sn * nu + st * t (nu the
// normal coordinate, t the stage time) take state a, the others state b (rest == 4) or the ghost of
// boundary kind rest.
struct BcDev {
  double a[4], b[4];         // (rho, rho U, rho V, rho E); rho V = 0 in 1D
  double s0, sn, st;
  int rest, pad;
};

struct ProbDev {
  int dim, nx, ny, ns;
  int bc[4];
  int nz, bcz[2];            // 3D: cells along z and the kinds of the z sides (nz = 1 otherwise)
  int recon, zeta1_mode;
  int positivity;            // 1: non-physical reconstructed states drop to first order
  int prescribed;            // 1 if any side is a prescribed-state side (bc == 4)
  int csm;                   // tangential characteristic state: 0 own side, 1 mean of both sides (2D)
  int vdt;                   // Navier-Stokes time step: 0 nu = mu / rho, 1 nu = mu / p
  double x0, y0;             // lower-left corner (ghost centres of prescribed sides)
  double dx, dy, h;          // cell sizes; h = min(dx, dy) for the CFL step
  double gamma, K, mu, Pr, c1, c2;  // K: internal dof of the 2D model (1D problems embed into it)
  double Kp2, iKp2, kpr;     // K + 2, 1 / (K + 2), 1 / Pr - 1 (uniform values kept out of the lanes)
  double ihx, ihy;           // 1 / dx, 1 / dy
  double dz, ihz;            // 3D: z cell size and its inverse
  double cfl, fixed_dt;
  double ghi, glo, eps;
  double* W;                 // state W^n        [nc][ny][nx]
  double* Ws;                // stage state W*, then the new state W^{n+1} until the step is committed (the
                             // commit swaps W and Ws when the step produced no non-physical state)
  double* S;                 // partial sum W^n - dt L^n - dt^2/6 L_t^n
  double* E;                 // compensated mode: rounding error of W^n, so that the carried state is W + E;
                             // nullptr in plain mode
  double* E2;                // compensated mode: rounding error of S, then of W^{n+1} (within a step)
  double* Ws2;               // three-stage tableaux: partial sum of the third stage's state
  uint8_t* flags;            // [(ny+4)][(nx+4)] (2D) / [nx+4] (1D): bit 0 x-flag, bit 1 y-flag
  void* Fx;                  // x-interfaces [4][ny][nx+1]: F (stage 1) / unused (stage 2)
  void* Gx;                  // x-interfaces: dF/dt
  void* Fy;                  // y-interfaces [4][ny+1][nx]
  void* Gy;
  void* Fz;                  // 3D: z-interfaces [5][nz+1][ny][nx]
  void* Gz;
  int* flag_count;           // [3] troubled cells per direction counted at the last flag evaluation
  BcDev bcd[4];              // read where bc[side] == 4
};

struct TimeDev {
  double dt, t, t_new, t_end;
  double dth, idt, idt2;     // dt / 2, 1 / dt, 4 / dt^2 of the current step
  int active;                // 1 while t < t_end
  int status;                // sticky: 1 when a non-physical state appeared (the problem then stops with
                             // the state of its last good step), 2 when dt came out <= 0 or not finite
  long long steps;
  int cur;                   // 0: W^n is in the problem's first state buffer, 1: in its second (each
                             // committed step swaps them)
  int pad;
  unsigned long long bad;    // first non-physical state: (stage << 32) | cell index, the lowest stage and
                             // then the lowest cell; ~0 while none
};

// Records a non-physical state of stage `stage` in cell `cell`: the sticky status and the first such cell.
__device__ inline void report_nonphysical(TimeDev& s, int stage, size_t cell) {
  atomicOr(&s.status, 1);
  atomicMin(&s.bad, ((unsigned long long)stage << 32) | (unsigned long long)cell);
}

// Derived time-step quantities of the step (set wherever dt is set).
__host__ __device__ inline void set_time_step(TimeDev& s, double dt) {
  s.dt = dt;
  s.dth = 0.5 * dt;
  s.idt = dt > 0.0 ? 1.0 / dt : 0.0;
  s.idt2 = 4.0 * s.idt * s.idt;
}

// ---------------------------------------------------------------------------------------------
// Boundary conditions. Ghost cells are synthesised where a kernel loads them: x-sides on the
// interior rows, y-sides across the full padded width (a corner follows the y-side's rule applied
// to the x-ghost beside it).
// ---------------------------------------------------------------------------------------------
// Index of the interior cell that index i reads on a side of kind bc (0..3), and the velocity sign
// flips (bit 0: normal momentum, bit 1: tangential momentum).
__host__ __device__ inline int bc_index(int i, int n, int bc, int& flip) {
  flip = 0;
  if (i >= 0 && i < n) return i;
  if (bc == 0) {  // periodic
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  if (bc == 1) return (i < 0) ? 0 : n - 1;  // zero-gradient
  flip = (bc == 2) ? 1 : 3;                  // 1: normal velocity, 3: both (no-slip)
  int m = (i < 0) ? -1 - i : 2 * n - 1 - i;  // mirror about the wall face
  return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

// State of a prescribed side at a ghost centre (tangential coordinate tau, normal coordinate nu) at
// stage time tb, or nullptr where the side's rest kind applies (returned in kind).
__device__ inline const double* bc_state(const BcDev& B, double tau, double nu, double tb, int& kind) {
#pragma clang fp contract(off)
  kind = B.rest;
  if (tau < B.s0 + B.sn * nu + B.st * tb) return B.a;
  return B.rest == 4 ? B.b : nullptr;
}

__device__ inline double cell_centre(double x0, int i, double h) {
#pragma clang fp contract(off)
  return x0 + (i + 0.5) * h;
}

// Whether cell (i, j) is a ghost of a prescribed-state side (its value then comes from load_cell only).
__device__ inline bool prescribed_ghost(const ProbDev& P, int i, int j) {
  if (P.dim == 2 && (j < 0 || j >= P.ny) && P.bc[j < 0 ? 2 : 3] == 4) return true;
  return (i < 0 || i >= P.nx) && P.bc[i < 0 ? 0 : 1] == 4;
}

// Cell (i, j) of state W with the ghost synthesis of the periodic, zero-gradient and wall sides;
// a prescribed-state side is read as zero gradient here (the flux loader overwrites those ghosts with
// load_cell in a separate pass, which keeps this, its hot loop, free of that logic).
__device__ inline void load_cell_plain(const ProbDev& P, const double* __restrict__ W, int i, int j, double q[4]) {
  int fx = 0, fy = 0, jj = 0;
  if (P.dim == 2) {
    const int ky = (j < 0) ? P.bc[2] : P.bc[3];
    jj = bc_index(j, P.ny, ky == 4 ? 1 : ky, fy);
  }
  const int kx = (i < 0) ? P.bc[0] : P.bc[1];
  const int ii = bc_index(i, P.nx, kx == 4 ? 1 : kx, fx);
  const size_t plane = (size_t)P.nx * P.ny;
  const size_t o = (size_t)jj * P.nx + ii;
  q[0] = W[o];
  q[1] = W[plane + o];
  if (P.dim == 2) {
    q[2] = W[2 * plane + o];
    q[3] = W[3 * plane + o];
  } else {
    q[2] = 0.0;
    q[3] = W[2 * plane + o];
  }
  const int negu = (fx & 1) ^ ((fy >> 1) & 1);
  const int negv = ((fx >> 1) & 1) ^ (fy & 1);
  if (negu) q[1] = -q[1];
  if (negv) q[2] = -q[2];
}

// Cell (i, j) of state W with ghost synthesis at stage time tb, every side kind included; returns
// (rho, rho U, rho V, rho E) (rho V = 0 in 1D).
__device__ inline void load_cell(const ProbDev& P, const double* __restrict__ W, int i, int j, double tb,
                                 double q[4]) {
  int fx = 0, fy = 0, jj = 0;
  const double* sy = nullptr;  // prescribed state of a y-side ghost row (whole padded width)
  const double* sx = nullptr;  // prescribed state of an x-side ghost (on the row jj maps to)
  const bool pres = P.prescribed;  // uniform: problems without prescribed sides skip all of it
  if (P.dim == 2) {
    int ky = (j < 0) ? P.bc[2] : P.bc[3];
    if (pres && (j < 0 || j >= P.ny) && ky == 4)
      sy = bc_state(P.bcd[j < 0 ? 2 : 3], cell_centre(P.x0, i, P.dx), cell_centre(P.y0, j, P.dy), tb, ky);
    jj = bc_index(j, P.ny, ky == 4 ? 1 : ky, fy);
  }
  int kx = (i < 0) ? P.bc[0] : P.bc[1];
  if (pres && (i < 0 || i >= P.nx) && kx == 4)
    sx = bc_state(P.bcd[i < 0 ? 0 : 1], P.dim == 2 ? cell_centre(P.y0, jj, P.dy) : 0.0, cell_centre(P.x0, i, P.dx),
                  tb, kx);
  const int ii = bc_index(i, P.nx, kx == 4 ? 1 : kx, fx);
  const size_t plane = (size_t)P.nx * P.ny;
  const size_t o = (size_t)jj * P.nx + ii;
  q[0] = W[o];
  q[1] = W[plane + o];
  if (P.dim == 2) {
    q[2] = W[2 * plane + o];
    q[3] = W[3 * plane + o];
  } else {
    q[2] = 0.0;
    q[3] = W[2 * plane + o];
  }
  if (sx) {  // an x-ghost's own state; the y-side's wall rule still applies to it
    fx = 0;
    q[0] = sx[0]; q[1] = sx[1]; q[2] = sx[2]; q[3] = sx[3];
  }
  const int negu = (fx & 1) ^ ((fy >> 1) & 1);  // x-walls flip U (and V if no-slip), y-walls the reverse
  const int negv = ((fx >> 1) & 1) ^ (fy & 1);
  if (negu) q[1] = -q[1];
  if (negv) q[2] = -q[2];
  if (sy) {  // a y-ghost row's own state, ahead of everything else
    q[0] = sy[0]; q[1] = sy[1]; q[2] = sy[2]; q[3] = sy[3];
  }
}

// ---------------------------------------------------------------------------------------------
// Troubled-cell indicator, Sec. 2.3.1 Steps 1-3 (FP64, fixed expression tree, no contraction).
// D1 = 10 a1 dx and D2 = 34 a2 dx^2 of the least-squares quadratic on the five cells; Step 1 smooth
// if |D2| <= 5h (normalised reading of zeta1 = 5/17 dx); Step 2 smooth if the extreme point
// xbar = -17 D1 / (10 D2) lies outside [-5/2, 5/2]; Step 3 smooth if it is within 1/4 of the
// extreme point of the conservative quadratic on the three central cells.
// ---------------------------------------------------------------------------------------------
__device__ inline int troubled5(double Qm2, double Qm1, double Q0, double Qp1, double Qp2,
                                                   double thr) {
#pragma clang fp contract(off)
  const double D1 = (Qp1 - Qm1) + 2.0 * (Qp2 - Qm2);
  const double D2 = (4.0 * (Qm2 + Qp2) + (Qm1 + Qp1)) - 10.0 * Q0;
  if (fabs(D2) <= thr) return 0;
  const double xbar = -(17.0 * D1) / (10.0 * D2);
  if (fabs(xbar) > 2.5) return 0;
  const double a1h = 0.5 * (Qp1 - Qm1);
  const double a2h = 0.5 * ((Qm1 + Qp1) - 2.0 * Q0);
  const double den = 2.0 * a2h + (a2h == 0.0 ? 1e-30 : 0.0);
  const double xhat = -a1h / den;
  return fabs(xbar - xhat) <= 0.25 ? 0 : 1;
}

// ---------------------------------------------------------------------------------------------
// Precision helpers
// ---------------------------------------------------------------------------------------------
template <typename T> __device__ constexpr T unit_roundoff() {
  return sizeof(T) == 8 ? T(1.1102230246251565e-16) : T(5.9604644775390625e-8);  // 2^-53, 2^-24
}
template <typename T> __device__ inline T dsqrt(T x);
template <> __device__ inline double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ inline float dsqrt<float>(float x) { return __builtin_sqrtf(x); }
template <typename T> __device__ inline T dexp(T x);
template <> __device__ inline double dexp<double>(double x) { return exp(x); }
template <> __device__ inline float dexp<float>(float x) { return __expf(x); }
template <typename T> __device__ inline T derfc(T x);
template <> __device__ inline double derfc<double>(double x) { return erfc(x); }
template <> __device__ inline float derfc<float>(float x) { return erfcf(x); }
// Reciprocal for the bulk arithmetic (never used by the flag or CFL decisions, which divide exactly):
// FP64 -- the hardware estimate refined by two Newton steps r <- r + r (1 - x r), within an ulp or two
// of 1/x for the normal, finite arguments that occur here; FP32 -- the hardware estimate (1 ulp).
template <typename T> __device__ inline T drcp(T x);
template <> __device__ inline double drcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <> __device__ inline float drcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------------------------
// Reconstruction (Sec. 2.3.1): WENO-AO(5,3) from sub-stencil values/derivatives and smoothness
// indicators. q[0..4] are the averages of cells -2..2 about the reconstructing cell; derivatives are
// with respect to the normalised coordinate xi = (x - x_i)/h.
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ inline void smoothness(const T q[5], T beta[4]) {
  const T d0 = q[0] - 2 * q[1] + q[2], e0 = q[0] - 4 * q[1] + 3 * q[2];
  const T d1 = q[1] - 2 * q[2] + q[3], e1 = q[1] - q[3];
  const T d2 = q[2] - 2 * q[3] + q[4], e2 = 3 * q[2] - 4 * q[3] + q[4];
  beta[0] = T(13.0 / 12.0) * d0 * d0 + T(0.25) * e0 * e0;
  beta[1] = T(13.0 / 12.0) * d1 * d1 + T(0.25) * e1 * e1;
  beta[2] = T(13.0 / 12.0) * d2 * d2 + T(0.25) * e2 * e2;
  // quartic: Legendre-like coefficients of the cell-average interpolant
  const T u1 = (T(11) * (q[0] - q[4]) + T(82) * (q[3] - q[1])) * T(1.0 / 120.0);
  const T u2 = (T(-3) * (q[0] + q[4]) + T(40) * (q[1] + q[3]) - T(74) * q[2]) * T(1.0 / 56.0);
  const T u3 = (-q[0] + 2 * q[1] - 2 * q[3] + q[4]) * T(1.0 / 12.0);
  const T u4 = (q[0] - 4 * q[1] + 6 * q[2] - 4 * q[3] + q[4]) * T(1.0 / 24.0);
  const T s1 = u1 + T(0.1) * u3, s2 = u2 + T(123.0 / 455.0) * u4;
  beta[3] = s1 * s1 + T(13.0 / 3.0) * s2 * s2 + T(781.0 / 20.0) * u3 * u3 + T(1421461.0 / 2275.0) * u4 * u4;
}

// Nonlinear AO weights -> combine sub-polynomial values pv and derivatives pd (same weights).
template <typename T>
__device__ inline void ao_combine(const T beta[4], const T pv[4], const T pd[4], T ghi, T glo, T eps, T& v,
                                  T& d) {
  const T g3 = ghi, g0 = (1 - ghi) * (1 - glo) * T(0.5), g1 = (1 - ghi) * glo;
  const T del = (fabs(beta[3] - beta[0]) + fabs(beta[3] - beta[1]) + fabs(beta[3] - beta[2])) * T(1.0 / 3.0);
  const T w0 = g0 * (1 + del * drcp(beta[0] + eps));
  const T w1 = g1 * (1 + del * drcp(beta[1] + eps));
  const T w2 = g0 * (1 + del * drcp(beta[2] + eps));
  const T w3 = g3 * (1 + del * drcp(beta[3] + eps));
  const T inv = drcp(w0 + w1 + w2 + w3);
  const T r3 = w3 * inv * drcp(g3);
  v = r3 * (pv[3] - g0 * pv[0] - g1 * pv[1] - g0 * pv[2]) + inv * (w0 * pv[0] + w1 * pv[1] + w2 * pv[2]);
  d = r3 * (pd[3] - g0 * pd[0] - g1 * pd[1] - g0 * pd[2]) + inv * (w0 * pd[0] + w1 * pd[1] + w2 * pd[2]);
}

// Sub-stencil values/derivatives at the cell faces xi = +1/2 (side = 0, left state of the interface to
// the right of the cell) and xi = -1/2 (side = 1).
template <typename T>
__device__ inline void face_polys(const T q[5], int side, T pv[4], T pd[4]) {
  if (side == 0) {
    pv[0] = T(1.0 / 3.0) * q[0] - T(7.0 / 6.0) * q[1] + T(11.0 / 6.0) * q[2];
    pv[1] = T(-1.0 / 6.0) * q[1] + T(5.0 / 6.0) * q[2] + T(1.0 / 3.0) * q[3];
    pv[2] = T(1.0 / 3.0) * q[2] + T(5.0 / 6.0) * q[3] - T(1.0 / 6.0) * q[4];
    pv[3] = (T(2) * q[0] - T(13) * q[1] + T(47) * q[2] + T(27) * q[3] - T(3) * q[4]) * T(1.0 / 60.0);
    pd[0] = q[0] - T(3) * q[1] + T(2) * q[2];
    pd[1] = q[3] - q[2];
    pd[2] = q[3] - q[2];
    pd[3] = (q[1] - T(15) * q[2] + T(15) * q[3] - q[4]) * T(1.0 / 12.0);
  } else {
    pv[0] = T(-1.0 / 6.0) * q[0] + T(5.0 / 6.0) * q[1] + T(1.0 / 3.0) * q[2];
    pv[1] = T(1.0 / 3.0) * q[1] + T(5.0 / 6.0) * q[2] - T(1.0 / 6.0) * q[3];
    pv[2] = T(11.0 / 6.0) * q[2] - T(7.0 / 6.0) * q[3] + T(1.0 / 3.0) * q[4];
    pv[3] = (T(-3) * q[0] + T(27) * q[1] + T(47) * q[2] - T(13) * q[3] + T(2) * q[4]) * T(1.0 / 60.0);
    pd[0] = q[2] - q[1];
    pd[1] = q[2] - q[1];
    pd[2] = T(-2) * q[2] + T(3) * q[3] - q[4];
    pd[3] = (q[0] - T(15) * q[1] + T(15) * q[2] - q[3]) * T(1.0 / 12.0);
  }
}

// Sub-stencil values/derivatives at the Gauss points xi = -1/(2 sqrt 3) (gp = 0) and +1/(2 sqrt 3)
// (gp = 1). Coefficients derived from the cell-average interpolants; gp = 0 is the mirror image.
#define S3 1.7320508075688772935
template <typename T>
__device__ inline void gauss_polys(const T q[5], int gp, T pv[4], T pd[4]) {
  // stencil seen in the +eta orientation
  T a0, a1, a2, a3, a4;
  if (gp == 1) { a0 = q[0]; a1 = q[1]; a2 = q[2]; a3 = q[3]; a4 = q[4]; }
  else { a0 = q[4]; a1 = q[3]; a2 = q[2]; a3 = q[1]; a4 = q[0]; }
  // p0 on (a0,a1,a2), p1 on (a1,a2,a3), p2 on (a2,a3,a4), quartic on all five, at eta = +1/(2 sqrt 3)
  pv[0] = T(S3 / 12) * a0 - T(S3 / 3) * a1 + T(1 + S3 / 4) * a2;
  pv[1] = T(-S3 / 12) * a1 + a2 + T(S3 / 12) * a3;
  pv[2] = T(1 - S3 / 4) * a2 + T(S3 / 3) * a3 - T(S3 / 12) * a4;
  pv[3] = T(-1.0 / 4320 + 7 * S3 / 432) * a0 + T(1.0 / 1080 - 25 * S3 / 216) * a1 + T(719.0 / 720) * a2 +
          T(1.0 / 1080 + 25 * S3 / 216) * a3 + T(-1.0 / 4320 - 7 * S3 / 432) * a4;
  pd[0] = T(0.5 + S3 / 6) * a0 + T(-2 - S3 / 3) * a1 + T(1.5 + S3 / 6) * a2;
  pd[1] = T(-0.5 + S3 / 6) * a1 + T(-S3 / 3) * a2 + T(0.5 + S3 / 6) * a3;
  pd[2] = T(-1.5 + S3 / 6) * a2 + T(2 - S3 / 3) * a3 + T(-0.5 + S3 / 6) * a4;
  pd[3] = T(1.0 / 12 - S3 / 54) * a0 + T(-2.0 / 3 + 13 * S3 / 54) * a1 + T(-4 * S3 / 9) * a2 +
          T(2.0 / 3 + 13 * S3 / 54) * a3 + T(-1.0 / 12 - S3 / 54) * a4;
  if (gp == 0) {  // mirrored stencil: p0 <-> p2 and derivatives change sign
    T t = pv[0]; pv[0] = pv[2]; pv[2] = t;
    t = pd[0]; pd[0] = -pd[2]; pd[2] = -t;
    pd[1] = -pd[1];
    pd[3] = -pd[3];
  }
}

// Linear fifth-order (quartic) value only at a Gauss point, and its derivative.
template <typename T>
__device__ inline void gauss_linear(const T q[5], int gp, T& v, T& d) {
  T a0, a1, a2, a3, a4;
  if (gp == 1) { a0 = q[0]; a1 = q[1]; a2 = q[2]; a3 = q[3]; a4 = q[4]; }
  else { a0 = q[4]; a1 = q[3]; a2 = q[2]; a3 = q[1]; a4 = q[0]; }
  v = T(-1.0 / 4320 + 7 * S3 / 432) * a0 + T(1.0 / 1080 - 25 * S3 / 216) * a1 + T(719.0 / 720) * a2 +
      T(1.0 / 1080 + 25 * S3 / 216) * a3 + T(-1.0 / 4320 - 7 * S3 / 432) * a4;
  d = T(1.0 / 12 - S3 / 54) * a0 + T(-2.0 / 3 + 13 * S3 / 54) * a1 + T(-4 * S3 / 9) * a2 +
      T(2.0 / 3 + 13 * S3 / 54) * a3 + T(-1.0 / 12 - S3 / 54) * a4;
  if (gp == 0) d = -d;
}
#undef S3

// ---------------------------------------------------------------------------------------------
// Characteristic variables (Sec. 2.3.1) of the 2D Euler equations along frame slot D (1: the momentum of
// slot 1, 2: that of slot 2; the other velocity slot is tangential): right eigenvectors R with columns
// u_D - c, entropy (1, u, v, q^2/2), shear (0, e_t, u_t), u_D + c, and L = R^{-1} in closed form. Neither
// matrix is stored: both projections are applied from nine scalars of the state (b1 = (gamma-1)/c^2,
// b2 = b1 q^2/2), which keeps the troubled path's register footprint small.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Char4 {
  T u[2], c, ic, H, b1, b2, hq2;
};

template <typename T>
__device__ inline void char4(const T w[4], T gamma, Char4<T>& m) {
  const T ir = drcp(w[0]);
  m.u[0] = w[1] * ir;
  m.u[1] = w[2] * ir;
  m.hq2 = T(0.5) * (m.u[0] * m.u[0] + m.u[1] * m.u[1]);
  const T p = (gamma - 1) * (w[3] - w[0] * m.hq2);
  m.c = dsqrt(gamma * p * ir);
  m.ic = drcp(m.c);
  m.H = (w[3] + p) * ir;
  m.b1 = (gamma - 1) * m.ic * m.ic;
  m.b2 = m.b1 * m.hq2;
}

// L q: (acoustic -, entropy, shear, acoustic +)
template <int D, typename T>
__device__ inline void to_char4(const Char4<T>& m, const T q[4], T out[4]) {
  constexpr int t = 3 - D;  // tangential slot
  const T um = m.u[0] * q[1] + m.u[1] * q[2];
  const T A = m.b2 * q[0] - m.b1 * um + m.b1 * q[3];
  const T X = m.ic * (m.u[D - 1] * q[0] - q[D]);
  out[0] = T(0.5) * (A + X);
  out[1] = q[0] - A;
  out[2] = q[t] - m.u[t - 1] * q[0];
  out[3] = T(0.5) * (A - X);
}

// R cv
template <int D, typename T>
__device__ inline void from_char4(const Char4<T>& m, const T cv[4], T out[4]) {
  constexpr int t = 3 - D;
  const T s = cv[0] + cv[1] + cv[3], dl = cv[3] - cv[0];
  out[0] = s;
  out[D] = m.u[D - 1] * s + m.c * dl;
  out[t] = m.u[t - 1] * s + cv[2];
  out[3] = m.H * (cv[0] + cv[3]) + m.u[D - 1] * m.c * dl + m.hq2 * cv[1] + m.u[t - 1] * cv[2];
}

// WENO-AO of one characteristic component's five values q; ev 0/1: face xi = +1/2 / -1/2, ev 2/3: Gauss
// point -eta / +eta. Value and xi-derivative.
template <typename T>
__device__ inline void ao_scalar(const T q[5], int ev, T ghi, T glo, T eps, T& v, T& d) {
  T beta[4], pv[4], pd[4];
  smoothness(q, beta);
  if (ev < 2) face_polys(q, ev, pv, pd);
  else gauss_polys(q, ev - 2, pv, pd);
  ao_combine(beta, pv, pd, ghi, glo, eps, v, d);
}

// WENO-AO of a vector (4 conserved variables) in the characteristic variables of slot D, from five rows of
// four components that may sit in registers or in LDS (component v of row r at qc[r * rs + v * cs]); each
// row is projected as it is read, so only the projections stay live.
template <int D, typename T>
__device__ inline void ao_vector(const T* qc, int rs, int cs, const Char4<T>& m, int ev, T ghi, T glo, T eps,
                                 T val[4], T der[4]) {
  T ch[5][4], cv[4], cd[4];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const T q[4] = {qc[r * rs], qc[r * rs + cs], qc[r * rs + 2 * cs], qc[r * rs + 3 * cs]};
    to_char4<D>(m, q, ch[r]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T q[5] = {ch[0][k], ch[1][k], ch[2][k], ch[3][k], ch[4][k]};
    ao_scalar(q, ev, ghi, glo, eps, cv[k], cd[k]);
  }
  from_char4<D>(m, cv, val);
  from_char4<D>(m, cd, der);
}

// ---------------------------------------------------------------------------------------------
// Kinetic part (Sec. 2.1). Moments of the normalised Maxwellian: <u^n> from the Gaussian recurrence
// (full line, or the half line u > 0 / u < 0 started from erfc and exp), <v^n>, <xi^2k>.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Maxw {
  T rho, U, V, lam;
  T Mu[7];  // <u^n>, n <= 6, over the full line or a half line
  T Mv[6];  // <v^n>, n <= 5
  T X1, X2; // <xi^2>, <xi^4>
};

template <typename T>
__device__ inline void maxw_prims(const T w[4], T gamma, Maxw<T>& g) {
  g.rho = w[0];
  const T ir = drcp(w[0]);
  g.U = w[1] * ir;
  g.V = w[2] * ir;
  const T p = (gamma - 1) * (w[3] - T(0.5) * w[0] * (g.U * g.U + g.V * g.V));
  g.lam = T(0.5) * w[0] * drcp(p);
}

// Full-line moments in u (half = 0) or half-line moments (half = +1: u > 0, -1: u < 0).
template <typename T>
__device__ inline void maxw_moments(Maxw<T>& g, T K, int half) {
  const T s = T(0.5) * drcp(g.lam);  // 1/(2 lam)
  if (half == 0) {
    g.Mu[0] = 1;
    g.Mu[1] = g.U;
  } else {
    const T sl = dsqrt(g.lam);
    const T hs = T(half);
    g.Mu[0] = T(0.5) * derfc(-hs * sl * g.U);
    g.Mu[1] = g.U * g.Mu[0] + hs * T(0.5) * dexp(-g.lam * g.U * g.U) * drcp(sl * T(1.7724538509055160273));
  }
#pragma unroll
  for (int n = 0; n < 5; ++n) g.Mu[n + 2] = g.U * g.Mu[n + 1] + T(n + 1) * s * g.Mu[n];
  g.Mv[0] = 1;
  g.Mv[1] = g.V;
#pragma unroll
  for (int n = 0; n < 4; ++n) g.Mv[n + 2] = g.V * g.Mv[n + 1] + T(n + 1) * s * g.Mv[n];
  g.X1 = K * s;
  g.X2 = K * (K + 2) * s * s;
}

// <u^n v^m a psi> for a = a0 + a1 u + a2 v + a3 (u^2 + v^2 + xi^2)/2 (n, m compile-time), using
// <u^n v^m> = Mu[n] Mv[m], <.. psi_4> and <.. psi_4^2> expanded through <xi^2>, <xi^4>.
template <int N, int M, typename T>
__device__ inline void mom_a(const Maxw<T>& g, const T a[4], T out[4]) {
#define G(n, m) (g.Mu[n] * g.Mv[m])
#define SS(n, m) (T(0.5) * (G((n) + 2, m) + G(n, (m) + 2) + G(n, m) * g.X1))
  const T S00 = SS(N, M), S10 = SS(N + 1, M), S01 = SS(N, M + 1);
  const T TT = T(0.25) * (G(N + 4, M) + G(N, M + 4) + G(N, M) * g.X2 +
                          T(2) * (G(N + 2, M + 2) + (G(N + 2, M) + G(N, M + 2)) * g.X1));
  out[0] = a[0] * G(N, M) + a[1] * G(N + 1, M) + a[2] * G(N, M + 1) + a[3] * S00;
  out[1] = a[0] * G(N + 1, M) + a[1] * G(N + 2, M) + a[2] * G(N + 1, M + 1) + a[3] * S10;
  out[2] = a[0] * G(N, M + 1) + a[1] * G(N + 1, M + 1) + a[2] * G(N, M + 2) + a[3] * S01;
  out[3] = a[0] * S00 + a[1] * S10 + a[2] * S01 + a[3] * TT;
#undef SS
#undef G
}

// <u^n v^m psi> (a = (1, 0, 0, 0)).
template <int N, int M, typename T>
__device__ inline void mom_psi(const Maxw<T>& g, T out[4]) {
  out[0] = g.Mu[N] * g.Mv[M];
  out[1] = g.Mu[N + 1] * g.Mv[M];
  out[2] = g.Mu[N] * g.Mv[M + 1];
  out[3] = T(0.5) * (g.Mu[N + 2] * g.Mv[M] + g.Mu[N] * g.Mv[M + 2] + g.Mu[N] * g.Mv[M] * g.X1);
}

// Microscopic slope a with <a psi> = b (closed-form inverse of the 4x4 moment matrix of g).
template <typename T>
__device__ inline void solve_slope(const Maxw<T>& g, T Kp2, T iKp2, const T b[4], T a[4]) {
  const T U = g.U, V = g.V, l = g.lam;
  const T q2 = U * U + V * V;
  const T ni = Kp2 * T(0.5) * drcp(l);  // (K+2)/(2 lam)
  a[3] = T(4) * l * l * iKp2 * (T(2) * b[3] - T(2) * U * b[1] - T(2) * V * b[2] + (q2 - ni) * b[0]);
  a[2] = T(2) * l * (b[2] - V * b[0]) - V * a[3];
  a[1] = T(2) * l * (b[1] - U * b[0]) - U * a[3];
  a[0] = b[0] - U * a[1] - V * a[2] - T(0.5) * a[3] * (q2 + ni);
}

// Time integrals over [0, delta] of the five coefficient functions of Eq. (equ10) (FP64):
// 1 - e, (t+tau) e - tau, t - tau + tau e, e, (t+tau) e with e = exp(-t/tau); for delta/tau < 1 the
// Taylor series of the same integrals (the closed forms cancel there). `e` is exp(-delta/tau), needed
// only when delta/tau >= 1.
__device__ inline void time_integrals(double d, double tau, double e, double C[5]) {
  if (tau == 0.0) {
    C[0] = d; C[1] = 0.0; C[2] = 0.5 * d * d; C[3] = 0.0; C[4] = 0.0;
    return;
  }
  const double x = d / tau;
  if (x < 1.0) {
    double tk = 1.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int k = 1; k <= 24; ++k) {
      tk *= x * drcp<double>(double(k));
      const double sg = (k & 1) ? -tk : tk;
      if (k >= 2) s1 += sg;
      if (k >= 3) { s2 += (k - 2) * sg; s3 -= sg; }
      s4 -= sg;
    }
    C[0] = tau * s1; C[1] = tau * tau * s2; C[2] = tau * tau * s3; C[3] = tau * s4; C[4] = tau * tau * (x + s2);
    return;
  }
  C[0] = d - tau * (1.0 - e);
  C[1] = 2.0 * tau * tau - tau * d - tau * (d + 2.0 * tau) * e;
  C[2] = 0.5 * d * d - tau * d + tau * tau * (1.0 - e);
  C[3] = tau * (1.0 - e);
  C[4] = 2.0 * tau * tau - tau * (2.0 * tau + d) * e;
}

// Both step lengths of the S2O4 flux (dt and dt/2) from one exponential: exp(-dt/tau) is the square of
// exp(-dt/(2 tau)). For dt/(2 tau) > 45 the exponential (< 3e-20) and its products with the other terms
// (at most dt/tau times larger) stay below half an ulp of every coefficient, so it is taken as 0.
__device__ inline void time_integrals_pair(double dt, double dth, double tau, double Cd[5], double Ch[5]) {
  double eh = 0.0, ed = 0.0;
  if (tau > 0.0 && dt >= tau && dth < 45.0 * tau) {
    eh = exp(-(dth / tau));
    ed = eh * eh;
  }
  time_integrals(dt, tau, ed, Cd);
  time_integrals(dth, tau, eh, Ch);
}

struct FluxParams {
  double gamma, K, mu, Pr, c1, c2, dt;
  double Kp2, iKp2, kpr, dth, idt, idt2;  // K + 2, 1/(K + 2), 1/Pr - 1, dt/2, 1/dt, 4/dt^2
  int ns;
  int want_F;  // 0: only dF/dt (second stage)
};

// Gas-kinetic flux at one Gauss point in the local frame (slot 1 = normal momentum), in two parts so
// that a caller can reconstruct one side at a time: flux_side() folds one side's reconstructed state
// W, its normal (x) and tangential (y) derivatives into the accumulators (equilibrium state and its
// slopes, Eq. (equ46)-(equ47), and the free-transport moments of Eq. (equ10)); flux_finish() builds
// g0, its slopes, the collision time and the time integrals, and adds wgt * F and wgt * dF/dt
// (Sec. 2.1-2.2).
template <typename T>
struct FluxAcc {
  T Wc[4], Wxc[4], Wyc[4];   // equilibrium state and its slopes
  T M4a[4], M4b[4], M5[4];   // rho <u psi>_h, rho <u A psi>_h, rho <u (a u + b v) psi>_h summed over sides
  T N4b[4], N5[4];           // the same with one power of u less (Prandtl correction only)
  T p_side[2];
  T rho_min;                 // smaller of the two sides' densities (interface-vacuum test)
};

// side S = 0: g_l integrated over u > 0 (the first side: its moments initialise the accumulators);
// S = 1: g_r over u < 0 (added)
template <int S, bool PRFIX, typename T>
__device__ inline void flux_side(const T W[4], const T Wx[4], const T Wy[4], T gamma, T K, T Kp2, T iKp2,
                                 FluxAcc<T>& acc) {
  constexpr int s = S;
  Maxw<T> g;
  maxw_prims(W, gamma, g);
  acc.p_side[s] = T(0.5) * g.rho * drcp(g.lam);
  acc.rho_min = (S == 0) ? g.rho : fmin(acc.rho_min, g.rho);
  const T ir = drcp(g.rho);
  T b[4], ax[4], ay[4], A[4], t1[4], t2[4];
  // full-line moments: slopes and the compatibility condition <a1 u + a2 v + A> = 0
  maxw_moments(g, K, 0);
#pragma unroll
  for (int c = 0; c < 4; ++c) b[c] = Wx[c] * ir;
  solve_slope(g, Kp2, iKp2, b, ax);
#pragma unroll
  for (int c = 0; c < 4; ++c) b[c] = Wy[c] * ir;
  solve_slope(g, Kp2, iKp2, b, ay);
  mom_a<1, 0>(g, ax, t1);
  mom_a<0, 1>(g, ay, t2);
#pragma unroll
  for (int c = 0; c < 4; ++c) b[c] = -(t1[c] + t2[c]);
  solve_slope(g, Kp2, iKp2, b, A);
  // half-line moments
  maxw_moments(g, K, s ? -1 : 1);
  const T rho = g.rho;
  auto put = [&](T (&dst)[4], const T x[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[c] = (S == 0) ? rho * x[c] : dst[c] + rho * x[c];
  };
  mom_psi<0, 0>(g, t1);
  put(acc.Wc, t1);
  mom_a<0, 0>(g, ax, t1);
  put(acc.Wxc, t1);
  mom_a<0, 0>(g, ay, t1);
  put(acc.Wyc, t1);
  mom_psi<1, 0>(g, t1);
  put(acc.M4a, t1);
  mom_a<1, 0>(g, A, t1);
  put(acc.M4b, t1);
  mom_a<2, 0>(g, ax, t1);
  mom_a<1, 1>(g, ay, t2);
#pragma unroll
  for (int c = 0; c < 4; ++c) t1[c] += t2[c];
  put(acc.M5, t1);
  if (PRFIX) {
    mom_a<0, 0>(g, A, t1);
    put(acc.N4b, t1);
    mom_a<1, 0>(g, ax, t1);
    mom_a<0, 1>(g, ay, t2);
#pragma unroll
    for (int c = 0; c < 4; ++c) t1[c] += t2[c];
    put(acc.N5, t1);
  }
}

// Coefficients that turn a moment vector of one term of Eq. (equ10) into its share of F and dF/dt.
template <typename T>
struct TermCoef {
  T f[5], d[5], f4t, d4t;
};

template <bool PRFIX, typename T>
__device__ inline void flux_finish(FluxAcc<T>& acc, const FluxParams& fp, T wgt, T F[4], T dF[4]) {
  const T gamma = T(fp.gamma), K = T(fp.K), Kp2 = T(fp.Kp2), iKp2 = T(fp.iKp2);
  // equilibrium g0 at the interface
  Maxw<T> g0;
  maxw_prims(acc.Wc, gamma, g0);
  // interface vacuum: two physical sides (positive, finite pressures; a non-physical side leaves NaN
  // moments and is reported) whose half-space integrals leave a density below the unit roundoff of the
  // smaller side density and no equilibrium (temperature not positive and finite), where two states
  // separate at many thermal speeds and the integrals underflow: the face carries no flux. An interface
  // density above that bound with no equilibrium is left to produce NaN and be reported.
  {
    const T inf = T(__builtin_inf()), pl = acc.p_side[0], pr = acc.p_side[1];
    if (pl > T(0) && pl < inf && pr > T(0) && pr < inf && g0.rho <= unit_roundoff<T>() * acc.rho_min &&
        !(g0.rho > T(0) && g0.lam > T(0) && g0.lam < inf))
      return;
  }
  // collision time (Sec. 3)
  double tau;
  {
    const double pl = double(acc.p_side[0]), pr = double(acc.p_side[1]);
    const double jump = fabs((pl - pr) / (pl + pr));
    if (fp.ns) tau = fp.mu / double(T(0.5) * g0.rho * drcp(g0.lam)) + fp.c2 * jump * fp.dt;
    else tau = fp.c1 * fp.dt + fp.c2 * jump * fp.dt;
  }
  // heat flux q = int (u-U0)((u-U0)^2+(v-V0)^2+xi^2)/2 f of one term, written through its flux moments
  // (u psi) M and conserved moments (psi) N; the energy flux of the term gains (1/Pr - 1) q
  const T U0 = g0.U, V0 = g0.V;
  const T cA = T(1.5) * U0 * U0 + T(0.5) * V0 * V0, cB = T(0.5) * U0 * (U0 * U0 + V0 * V0);
  const T kpr = T(fp.kpr);
  auto heat = [&](const T M[4], const T N[4]) -> T {
    return M[3] - U0 * M[1] - V0 * M[2] + cA * M[0] + U0 * V0 * N[2] - U0 * N[3] - cB * N[0];
  };
  if (PRFIX) {
    acc.M4a[3] += kpr * heat(acc.M4a, acc.Wc);
    acc.M4b[3] += kpr * heat(acc.M4b, acc.N4b);
    acc.M5[3] += kpr * heat(acc.M5, acc.N5);
  }

  // the time-integral combinations (FP64): F = (4 F(dt/2) - F(dt)) / dt, dF/dt = 4 (F(dt) - 2 F(dt/2)) / dt^2,
  // term by term
  TermCoef<T> tc;
  {
    double Cd[5], Ch[5];
    time_integrals_pair(fp.dt, fp.dth, tau, Cd, Ch);
    const double idt = fp.idt, idt2 = fp.idt2;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      tc.f[m] = fp.want_F ? wgt * T((4.0 * Ch[m] - Cd[m]) * idt) : T(0);
      tc.d[m] = wgt * T((Cd[m] - 2.0 * Ch[m]) * idt2);
    }
    tc.f4t = fp.want_F ? wgt * T(tau * (4.0 * Ch[3] - Cd[3]) * idt) : T(0);
    tc.d4t = wgt * T(tau * (Cd[3] - 2.0 * Ch[3]) * idt2);
  }
  const bool want_F = fp.want_F;  // the second stage needs dF/dt only (uniform per launch)
  auto fold = [&](const T M[4], T cf, T cd) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (want_F) F[c] += cf * M[c];
      dF[c] += cd * M[c];
    }
  };
  // free-transport terms of both sides: C4 (M4a - tau M4b) - C5 M5
  fold(acc.M4a, tc.f[3], tc.d[3]);
  fold(acc.M4b, -tc.f4t, -tc.d4t);
  fold(acc.M5, -tc.f[4], -tc.d[4]);
  // the equilibrium part below is scheduled on its own: interleaved with the time integrals above, the two
  // sets of live values together cost registers (and occupancy)
  __builtin_amdgcn_sched_barrier(0);

  // equilibrium terms: C1 rho0 <u psi> + C2 rho0 <u (a0 u + b0 v) psi> + C3 rho0 <u A0 psi>
  maxw_moments(g0, K, 0);
  const T ir0 = drcp(g0.rho), r0 = g0.rho;
  T b[4], a0[4], t1[4], t2[4], rhs[4];
  {
    T M[4];
    mom_psi<1, 0>(g0, M);
#pragma unroll
    for (int c = 0; c < 4; ++c) M[c] *= r0;
    if (PRFIX) {
      T N[4];
      mom_psi<0, 0>(g0, N);
#pragma unroll
      for (int c = 0; c < 4; ++c) N[c] *= r0;
      M[3] += kpr * heat(M, N);
    }
    fold(M, tc.f[0], tc.d[0]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) b[c] = acc.Wxc[c] * ir0;
  solve_slope(g0, Kp2, iKp2, b, a0);
  mom_a<1, 0>(g0, a0, rhs);
  mom_a<2, 0>(g0, a0, t2);
#pragma unroll
  for (int c = 0; c < 4; ++c) b[c] = acc.Wyc[c] * ir0;
  solve_slope(g0, Kp2, iKp2, b, a0);  // a0 now holds the y-slope b0
  mom_a<0, 1>(g0, a0, t1);
#pragma unroll
  for (int c = 0; c < 4; ++c) rhs[c] = -(rhs[c] + t1[c]);  // <A0 psi> = -<(a0 u + b0 v) psi>
  mom_a<1, 1>(g0, a0, t1);
  {
    T M[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) M[c] = r0 * (t1[c] + t2[c]);
    if (PRFIX) {
      T N[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) N[c] = -r0 * rhs[c];  // rho0 <(a0 u + b0 v) psi>
      M[3] += kpr * heat(M, N);
    }
    fold(M, tc.f[1], tc.d[1]);
  }
  solve_slope(g0, Kp2, iKp2, rhs, a0);  // a0 now holds A0
  {
    T M[4];
    mom_a<1, 0>(g0, a0, M);
#pragma unroll
    for (int c = 0; c < 4; ++c) M[c] *= r0;
    if (PRFIX) {
      T N[4];
      mom_a<0, 0>(g0, a0, N);
#pragma unroll
      for (int c = 0; c < 4; ++c) N[c] *= r0;
      M[3] += kpr * heat(M, N);
    }
    fold(M, tc.f[2], tc.d[2]);
  }
}

// Whole Gauss-point flux from both reconstructed sides at once.
template <bool PRFIX, typename T>
__device__ inline void gks_flux_gp(const T Wl[4], const T Wxl[4], const T Wyl[4], const T Wr[4], const T Wxr[4],
                                   const T Wyr[4], const FluxParams& fp, T wgt, T F[4], T dF[4]) {
  FluxAcc<T> acc;
  const T gam = T(fp.gamma), K = T(fp.K), Kp2 = T(fp.Kp2), iKp2 = T(fp.iKp2);
  flux_side<0, PRFIX>(Wl, Wxl, Wyl, gam, K, Kp2, iKp2, acc);
  flux_side<1, PRFIX>(Wr, Wxr, Wyr, gam, K, Kp2, iKp2, acc);
  flux_finish<PRFIX>(acc, fp, wgt, F, dF);
}

}  // namespace hk
