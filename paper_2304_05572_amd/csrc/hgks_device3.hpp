// Device arithmetic of the three-dimensional scheme: the same hybrid reconstruction and the
// gas-kinetic flux of Sec. 2.1 with three velocity components (u normal to the face, v and w along
// it) and K = (5 - 3 gamma)/(gamma - 1) internal degrees of freedom. Frame components of a state:
// (rho, normal momentum, first tangential momentum, second tangential momentum, rho E).
#pragma once

#include "hgks_device.hpp"

namespace hk {

template <typename T>
struct Maxw3 {
  T rho, U, V, Wv, lam;
  T Mu[7];  // <u^n>, n <= 6, over the full line or a half line
  T Mv[6];  // <v^n>, n <= 5
  T Mw[6];  // <w^n>, n <= 5
  T X1, X2; // <xi^2>, <xi^4>
};

template <typename T>
__device__ inline void maxw3_prims(const T w[5], T gamma, Maxw3<T>& g) {
  g.rho = w[0];
  const T ir = drcp(w[0]);
  g.U = w[1] * ir;
  g.V = w[2] * ir;
  g.Wv = w[3] * ir;
  const T p = (gamma - 1) * (w[4] - T(0.5) * w[0] * (g.U * g.U + g.V * g.V + g.Wv * g.Wv));
  g.lam = T(0.5) * w[0] * drcp(p);
}

// <u^n>, n <= 6, over the half line u > 0 (half = 1) or u < 0 (half = -1)
template <typename T>
__device__ inline void maxw3_half_u(const Maxw3<T>& g, int half, T Mh[7]) {
  const T s = T(0.5) * drcp(g.lam);
  const T sl = dsqrt(g.lam);
  const T hs = T(half);
  Mh[0] = T(0.5) * derfc(-hs * sl * g.U);
  Mh[1] = g.U * Mh[0] + hs * T(0.5) * dexp(-g.lam * g.U * g.U) * drcp(sl * T(1.7724538509055160273));
#pragma unroll
  for (int n = 0; n < 5; ++n) Mh[n + 2] = g.U * Mh[n + 1] + T(n + 1) * s * Mh[n];
}

template <typename T>
__device__ inline void maxw3_moments(Maxw3<T>& g, T K, int half) {
  const T s = T(0.5) * drcp(g.lam);
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
  g.Mw[0] = 1;
  g.Mw[1] = g.Wv;
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    g.Mv[n + 2] = g.V * g.Mv[n + 1] + T(n + 1) * s * g.Mv[n];
    g.Mw[n + 2] = g.Wv * g.Mw[n + 1] + T(n + 1) * s * g.Mw[n];
  }
  g.X1 = K * s;
  g.X2 = K * (K + 2) * s * s;
}

// <u^N v^M w^L a psi> with a = a0 + a1 u + a2 v + a3 w + a4 (u^2 + v^2 + w^2 + xi^2)/2, the u-moments taken
// from Mu (full or half line)
template <int N, int M, int L, typename T>
__device__ inline void mom3_au(const Maxw3<T>& g, const T* Mu, const T a[5], T out[5]) {
#define G(n, m, l) (Mu[n] * g.Mv[m] * g.Mw[l])
#define SS(n, m, l) (T(0.5) * (G((n) + 2, m, l) + G(n, (m) + 2, l) + G(n, m, (l) + 2) + G(n, m, l) * g.X1))
  const T S0 = SS(N, M, L), Su = SS(N + 1, M, L), Sv = SS(N, M + 1, L), Sw = SS(N, M, L + 1);
  const T TT = T(0.25) * (G(N + 4, M, L) + G(N, M + 4, L) + G(N, M, L + 4) + G(N, M, L) * g.X2 +
                          T(2) * (G(N + 2, M + 2, L) + G(N + 2, M, L + 2) + G(N, M + 2, L + 2)) +
                          T(2) * g.X1 * (G(N + 2, M, L) + G(N, M + 2, L) + G(N, M, L + 2)));
  out[0] = a[0] * G(N, M, L) + a[1] * G(N + 1, M, L) + a[2] * G(N, M + 1, L) + a[3] * G(N, M, L + 1) + a[4] * S0;
  out[1] = a[0] * G(N + 1, M, L) + a[1] * G(N + 2, M, L) + a[2] * G(N + 1, M + 1, L) + a[3] * G(N + 1, M, L + 1) +
           a[4] * Su;
  out[2] = a[0] * G(N, M + 1, L) + a[1] * G(N + 1, M + 1, L) + a[2] * G(N, M + 2, L) + a[3] * G(N, M + 1, L + 1) +
           a[4] * Sv;
  out[3] = a[0] * G(N, M, L + 1) + a[1] * G(N + 1, M, L + 1) + a[2] * G(N, M + 1, L + 1) + a[3] * G(N, M, L + 2) +
           a[4] * Sw;
  out[4] = a[0] * S0 + a[1] * Su + a[2] * Sv + a[3] * Sw + a[4] * TT;
#undef SS
#undef G
}

template <int N, int M, int L, typename T>
__device__ inline void mom3_a(const Maxw3<T>& g, const T a[5], T out[5]) {
  mom3_au<N, M, L>(g, g.Mu, a, out);
}

template <int N, typename T>
__device__ inline void mom3_psiu(const Maxw3<T>& g, const T* Mu, T out[5]) {
  out[0] = Mu[N];
  out[1] = Mu[N + 1];
  out[2] = Mu[N] * g.Mv[1];
  out[3] = Mu[N] * g.Mw[1];
  out[4] = T(0.5) * (Mu[N + 2] + Mu[N] * (g.Mv[2] + g.Mw[2] + g.X1));
}

template <int N, typename T>
__device__ inline void mom3_psi(const Maxw3<T>& g, T out[5]) {
  mom3_psiu<N>(g, g.Mu, out);
}

// a with <a psi> = b: closed-form inverse of the 5 x 5 moment matrix of g (N = K + 3 degrees of freedom
// besides the three velocities ... counted with them: <(u-U)^2 + (v-V)^2 + (w-W)^2 + xi^2> = N/(2 lam))
template <typename T>
__device__ inline void solve_slope3(const Maxw3<T>& g, T Kp3, T iKp3, const T b[5], T a[5]) {
  const T U = g.U, V = g.V, Wv = g.Wv, l = g.lam;
  const T q2 = U * U + V * V + Wv * Wv;
  const T ni = Kp3 * T(0.5) * drcp(l);
  a[4] = T(4) * l * l * iKp3 * (T(2) * b[4] - T(2) * U * b[1] - T(2) * V * b[2] - T(2) * Wv * b[3] + (q2 - ni) * b[0]);
  a[3] = T(2) * l * (b[3] - Wv * b[0]) - Wv * a[4];
  a[2] = T(2) * l * (b[2] - V * b[0]) - V * a[4];
  a[1] = T(2) * l * (b[1] - U * b[0]) - U * a[4];
  a[0] = b[0] - U * a[1] - V * a[2] - Wv * a[3] - T(0.5) * a[4] * (q2 + ni);
}

template <typename T>
struct FluxAcc3 {
  T Wc[5], Wnc[5], Wac[5], Wbc[5];  // equilibrium state and its normal / tangential slopes
  T M4a[5], M4b[5], M5[5];          // rho <u psi>_h, rho <u A psi>_h, rho <u (a u + b v + c w) psi>_h
  T p_side[2];
  T rho_min;                 // smaller of the two sides' densities (interface-vacuum test)
};

// one side's contribution (S = 0: g_l over u > 0, initialises; S = 1: g_r over u < 0, adds). The three
// spatial slopes are taken one at a time: each adds its term of the time slope's right-hand side (full
// moments) and its half-line moments to the accumulators before the next is solved.
template <int S, typename T>
__device__ inline void flux3_side(const T W[5], const T Wn[5], const T Wa[5], const T Wb[5], T gamma, T K, T Kp3,
                                  T iKp3, FluxAcc3<T>& acc) {
  Maxw3<T> g;
  maxw3_prims(W, gamma, g);
  acc.p_side[S] = T(0.5) * g.rho * drcp(g.lam);
  acc.rho_min = (S == 0) ? g.rho : fmin(acc.rho_min, g.rho);
  const T ir = drcp(g.rho), rho = g.rho;
  maxw3_moments(g, K, 0);
  T Mh[7];
  maxw3_half_u(g, S ? -1 : 1, Mh);
  auto put = [&](T (&dst)[5], const T x[5], bool init) {
#pragma unroll
    for (int c = 0; c < 5; ++c) dst[c] = init ? rho * x[c] : dst[c] + rho * x[c];
  };
  T b[5], a[5], t[5], bA[5];
  mom3_psiu<0>(g, Mh, t);
  put(acc.Wc, t, S == 0);
  // normal slope
#pragma unroll
  for (int c = 0; c < 5; ++c) b[c] = Wn[c] * ir;
  solve_slope3(g, Kp3, iKp3, b, a);
  mom3_au<1, 0, 0>(g, g.Mu, a, bA);
  mom3_au<0, 0, 0>(g, Mh, a, t);
  put(acc.Wnc, t, S == 0);
  mom3_au<2, 0, 0>(g, Mh, a, t);
  put(acc.M5, t, S == 0);
  // first tangential slope
#pragma unroll
  for (int c = 0; c < 5; ++c) b[c] = Wa[c] * ir;
  solve_slope3(g, Kp3, iKp3, b, a);
  mom3_au<0, 1, 0>(g, g.Mu, a, t);
#pragma unroll
  for (int c = 0; c < 5; ++c) bA[c] += t[c];
  mom3_au<0, 0, 0>(g, Mh, a, t);
  put(acc.Wac, t, S == 0);
  mom3_au<1, 1, 0>(g, Mh, a, t);
  put(acc.M5, t, false);
  // second tangential slope
#pragma unroll
  for (int c = 0; c < 5; ++c) b[c] = Wb[c] * ir;
  solve_slope3(g, Kp3, iKp3, b, a);
  mom3_au<0, 0, 1>(g, g.Mu, a, t);
#pragma unroll
  for (int c = 0; c < 5; ++c) bA[c] = -(bA[c] + t[c]);
  mom3_au<0, 0, 0>(g, Mh, a, t);
  put(acc.Wbc, t, S == 0);
  mom3_au<1, 0, 1>(g, Mh, a, t);
  put(acc.M5, t, false);
  // time slope: <A psi> = -<(a u + b v + c w) psi>
  solve_slope3(g, Kp3, iKp3, bA, a);
  mom3_psiu<1>(g, Mh, t);
  put(acc.M4a, t, S == 0);
  mom3_au<1, 0, 0>(g, Mh, a, t);
  put(acc.M4b, t, S == 0);
}

// equilibrium part, collision time and the time integrals: adds wgt * F and wgt * dF/dt
template <typename T>
__device__ inline void flux3_finish(FluxAcc3<T>& acc, const FluxParams& fp, T Kp3, T iKp3, T wgt, T F[5],
                                    T dF[5]) {
  const T gamma = T(fp.gamma), K = T(fp.K);
  Maxw3<T> g0;
  maxw3_prims(acc.Wc, gamma, g0);
  // interface vacuum (two physical sides, an interface density below the unit roundoff of the smaller side
  // density, no equilibrium): the face carries no flux
  {
    const T inf = T(__builtin_inf()), pl = acc.p_side[0], pr = acc.p_side[1];
    if (pl > T(0) && pl < inf && pr > T(0) && pr < inf && g0.rho <= unit_roundoff<T>() * acc.rho_min &&
        !(g0.rho > T(0) && g0.lam > T(0) && g0.lam < inf))
      return;
  }
  double cf[5], cd[5], tau;
  {
    const double pl = double(acc.p_side[0]), pr = double(acc.p_side[1]);
    const double jump = fabs((pl - pr) / (pl + pr));
    if (fp.ns) tau = fp.mu / double(T(0.5) * g0.rho * drcp(g0.lam)) + fp.c2 * jump * fp.dt;
    else tau = fp.c1 * fp.dt + fp.c2 * jump * fp.dt;
    double Cd[5], Ch[5];
    time_integrals_pair(fp.dt, fp.dth, tau, Cd, Ch);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      cf[m] = fp.want_F ? (4.0 * Ch[m] - Cd[m]) * fp.idt : 0.0;
      cd[m] = (Cd[m] - 2.0 * Ch[m]) * fp.idt2;
    }
  }
  const bool want_F = fp.want_F;
  auto fold = [&](const T M[5], double f, double d) {
    const T tf = wgt * T(f), td = wgt * T(d);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      if (want_F) F[c] += tf * M[c];
      dF[c] += td * M[c];
    }
  };
  fold(acc.M4a, cf[3], cd[3]);
  fold(acc.M4b, -tau * cf[3], -tau * cd[3]);
  fold(acc.M5, -cf[4], -cd[4]);
  maxw3_moments(g0, K, 0);
  const T ir0 = drcp(g0.rho), r0 = g0.rho;
  T b[5], s[5], t1[5], t2[5], rhs[5], M[5];
  mom3_psi<1>(g0, M);
#pragma unroll
  for (int c = 0; c < 5; ++c) M[c] *= r0;
  fold(M, cf[0], cd[0]);
  // slopes of g0: normal a0 -> <u a0 psi>, <u^2 a0 psi>; first tangential; second tangential
#pragma unroll
  for (int c = 0; c < 5; ++c) b[c] = acc.Wnc[c] * ir0;
  solve_slope3(g0, Kp3, iKp3, b, s);
  mom3_a<1, 0, 0>(g0, s, rhs);
  mom3_a<2, 0, 0>(g0, s, t2);
#pragma unroll
  for (int c = 0; c < 5; ++c) b[c] = acc.Wac[c] * ir0;
  solve_slope3(g0, Kp3, iKp3, b, s);
  mom3_a<0, 1, 0>(g0, s, t1);
#pragma unroll
  for (int c = 0; c < 5; ++c) rhs[c] += t1[c];
  mom3_a<1, 1, 0>(g0, s, t1);
#pragma unroll
  for (int c = 0; c < 5; ++c) t2[c] += t1[c];
#pragma unroll
  for (int c = 0; c < 5; ++c) b[c] = acc.Wbc[c] * ir0;
  solve_slope3(g0, Kp3, iKp3, b, s);
  mom3_a<0, 0, 1>(g0, s, t1);
#pragma unroll
  for (int c = 0; c < 5; ++c) rhs[c] = -(rhs[c] + t1[c]);  // <A0 psi> = -<(a0 u + b0 v + c0 w) psi>
  mom3_a<1, 0, 1>(g0, s, t1);
#pragma unroll
  for (int c = 0; c < 5; ++c) M[c] = r0 * (t2[c] + t1[c]);
  fold(M, cf[1], cd[1]);
  solve_slope3(g0, Kp3, iKp3, rhs, s);  // A0
  mom3_a<1, 0, 0>(g0, s, M);
#pragma unroll
  for (int c = 0; c < 5; ++c) M[c] *= r0;
  fold(M, cf[2], cd[2]);
}

// ---------------------------------------------------------------------------------------------
// Characteristic variables of the 3D Euler equations along frame slot D (1 normal, 2 and 3 tangential):
// right eigenvectors R with columns u_D - c, entropy, the two shear waves (the other two slots in
// ascending order, columns (0, e_k, u_k)), u_D + c; L = R^{-1} in closed form. Neither matrix is
// stored: the projections are applied from nine scalars of the state, which keeps the troubled-cell
// path's register footprint small.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Char5 {
  T u[3], c, ic, H, b1, b2, hq2;
};

template <typename T>
__device__ inline void char5(const T w[5], T gamma, Char5<T>& m) {
  const T ir = drcp(w[0]);
  m.u[0] = w[1] * ir;
  m.u[1] = w[2] * ir;
  m.u[2] = w[3] * ir;
  m.hq2 = T(0.5) * (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]);
  const T p = (gamma - 1) * (w[4] - w[0] * m.hq2);
  m.c = dsqrt(gamma * p * ir);
  m.ic = drcp(m.c);
  m.H = (w[4] + p) * ir;
  m.b1 = (gamma - 1) * m.ic * m.ic;
  m.b2 = m.b1 * m.hq2;
}

// L q: (acoustic -, entropy, shear, shear, acoustic +)
template <int D, typename T>
__device__ inline void to_char5(const Char5<T>& m, const T q[5], T out[5]) {
  constexpr int t0 = (D == 1) ? 1 : 0, t1 = (D == 3) ? 1 : 2;  // the two other velocity slots (0-based)
  const T um = m.u[0] * q[1] + m.u[1] * q[2] + m.u[2] * q[3];
  const T A = m.b2 * q[0] - m.b1 * um + m.b1 * q[4];
  const T X = m.ic * (m.u[D - 1] * q[0] - q[D]);
  out[0] = T(0.5) * (A + X);
  out[1] = q[0] - A;
  out[2] = q[1 + t0] - m.u[t0] * q[0];
  out[3] = q[1 + t1] - m.u[t1] * q[0];
  out[4] = T(0.5) * (A - X);
}

// R cv
template <int D, typename T>
__device__ inline void from_char5(const Char5<T>& m, const T cv[5], T out[5]) {
  constexpr int t0 = (D == 1) ? 1 : 0, t1 = (D == 3) ? 1 : 2;
  const T s = cv[0] + cv[1] + cv[4], dl = cv[4] - cv[0];
  out[0] = s;
  out[1 + t0] = m.u[t0] * s + cv[2];
  out[1 + t1] = m.u[t1] * s + cv[3];
  out[D] = m.u[D - 1] * s + m.c * dl;
  out[4] = m.H * (cv[0] + cv[4]) + m.u[D - 1] * m.c * dl + m.hq2 * cv[1] + m.u[t0] * cv[2] + m.u[t1] * cv[3];
}

// WENO-AO of a 5-vector in the characteristic variables of slot D; ev 0/1: face +1/2 / -1/2, ev 2/3: Gauss
// point -eta / +eta. Value and xi-derivative.
template <int D, typename T>
__device__ inline void ao_vector5(const T qc[5][5], const Char5<T>& m, int ev, T ghi, T glo, T eps, T val[5],
                                  T der[5]) {
  T ch[5][5], cv[5], cd[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) to_char5<D>(m, qc[r], ch[r]);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const T q[5] = {ch[0][k], ch[1][k], ch[2][k], ch[3][k], ch[4][k]};
    T beta[4], pv[4], pd[4];
    smoothness(q, beta);
    if (ev < 2) face_polys(q, ev, pv, pd);
    else gauss_polys(q, ev - 2, pv, pd);
    ao_combine(beta, pv, pd, ghi, glo, eps, cv[k], cd[k]);
  }
  from_char5<D>(m, cv, val);
  from_char5<D>(m, cd, der);
}

// Cell (i, j, k) of a 3D state with ghost synthesis (periodic, zero-gradient, slip wall, no-slip
// adiabatic on each of the six sides), grid components (rho, rho U, rho V, rho W, rho E).
__device__ inline void load_cell3(const ProbDev& P, const double* __restrict__ W, int i, int j, int k, double q[5]) {
  int fx, fy, fz;
  const int ii = bc_index(i, P.nx, i < 0 ? P.bc[0] : P.bc[1], fx);
  const int jj = bc_index(j, P.ny, j < 0 ? P.bc[2] : P.bc[3], fy);
  const int kk = bc_index(k, P.nz, k < 0 ? P.bcz[0] : P.bcz[1], fz);
  const size_t plane = (size_t)P.nx * P.ny * P.nz;
  const size_t o = ((size_t)kk * P.ny + jj) * P.nx + ii;
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = W[c * plane + o];
  // a wall flips its normal momentum (bit 0) or every momentum (no-slip, bit 1)
  const int f[3] = {fx, fy, fz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (f[d] & 2) { q[1] = -q[1]; q[2] = -q[2]; q[3] = -q[3]; }
    else if (f[d] & 1) q[1 + d] = -q[1 + d];
  }
}

}  // namespace hk
