// Three-dimensional kernels of the scheme (the direct extension of the 2D method that Sec. 2 names):
// widened troubled-cell flags along the three axes, the fused hybrid reconstruction + gas-kinetic flux of
// each face at its 2 x 2 Gauss points, the CFL quantity and the S2O4 stage updates (Sec. 2.2).
#include <hip/hip_runtime.h>

#include "hgks_device.hpp"
#include "hgks_device3.hpp"
#include "hgks_grid.hpp"
#include "hgks_launch.h"

namespace hk {

// =============================================================================================
// Three dimensions: flags, fused reconstruction + flux over 4 x 4 x 4 face tiles, stage updates
// =============================================================================================

// Widened troubled-cell flags of every cell of the extended range [-2, n+1]^3: bit d for direction d.
__global__ void __launch_bounds__(256) k_flags3(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts,
                                                const int* __restrict__ off, int nprob, int use_stage_state,
                                                int count) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  if (!ts[p].active) return;
  const int ex = P.nx + 4, ey = P.ny + 4, ez = P.nz + 4;
  const int e = (blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  int fl = 0, interior = 0;
  if (e < ex * ey * ez) {
    const int i = e % ex - 2, j = (e / ex) % ey - 2, k = e / (ex * ey) - 2;
    const double* W = use_stage_state ? P.Ws : P.W;
    if (P.recon == 1) {
      fl = 7;
    } else if (P.recon == 0) {
      const double h[3] = {P.dx, P.dy, P.dz};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double thr = (P.zeta1_mode == 0) ? 5.0 * h[d] : 5.0 * h[d] * h[d] * h[d];
        double q[7][5];
#pragma unroll
        for (int r = 0; r < 7; ++r)
          load_cell3(P, W, i + (d == 0 ? r - 3 : 0), j + (d == 1 ? r - 3 : 0), k + (d == 2 ? r - 3 : 0), q[r]);
        int f = 0;
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
          for (int c = 0; c < 5; ++c)
            f |= troubled5(q[s][c], q[s + 1][c], q[s + 2][c], q[s + 3][c], q[s + 4][c], thr);
        fl |= f << d;
      }
    }
    P.flags[e] = (uint8_t)fl;
    interior = (i >= 0 && i < P.nx && j >= 0 && j < P.ny && k >= 0 && k < P.nz);
  }
  if (count) {
    const unsigned long long bx = __ballot(interior && (fl & 1));
    const unsigned long long by = __ballot(interior && (fl & 2));
    const unsigned long long bz = __ballot(interior && (fl & 4));
    if ((threadIdx.x & 63) == 0) {
      if (bx) atomicAdd(&P.flag_count[0], __popcll(bx));
      if (by) atomicAdd(&P.flag_count[1], __popcll(by));
      if (bz) atomicAdd(&P.flag_count[2], __popcll(bz));
    }
  }
}

__device__ inline uint8_t flag3_at(const ProbDev& P, int i, int j, int k) {
  if (i < -2 || i > P.nx + 1 || j < -2 || j > P.ny + 1 || k < -2 || k > P.nz + 1) return 0;
  return P.flags[((size_t)(k + 2) * (P.ny + 4) + (j + 2)) * (P.nx + 4) + (i + 2)];
}

// Grid indices (i, j, k) of frame indices (along d, along d+1, along d+2): selects rather than arrays
// indexed by d, which would live in scratch memory.
__device__ inline void grid_of_frame(int d, int n, int a, int b, int& i, int& j, int& k) {
  i = d == 0 ? n : (d == 2 ? a : b);
  j = d == 1 ? n : (d == 0 ? a : b);
  k = d == 2 ? n : (d == 1 ? a : b);
}

__device__ inline int sel3(int d, int x, int y, int z) { return d == 0 ? x : (d == 1 ? y : z); }
__device__ inline double sel3(int d, double x, double y, double z) { return d == 0 ? x : (d == 1 ? y : z); }

// Linear (fifth-order) or, on a troubled side cell, WENO-AO reconstruction of five 5-vectors q[r] along one
// tangential axis at Gauss point gp (0: -eta, 1: +eta): value and xi-derivative.
template <int D, typename T>
__device__ inline void sweep5(const T q[5][5], int troubled, const Char5<T>& m, int gp, T ghi, T glo, T eps,
                              T val[5], T der[5]) {
  if (troubled) {
    ao_vector5<D>(q, m, 2 + gp, ghi, glo, eps, val, der);
  } else {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T c[5] = {q[0][v], q[1][v], q[2][v], q[3][v], q[4][v]};
      gauss_linear(c, gp, val[v], der[v]);
    }
  }
}

// One block per tile of kTN3 x kTA3 x kTB3 faces of one direction d (tangential axes da = d+1, db = d+2):
//  1. the block's cells, in frame components (rho, m_d, m_da, m_db, E), into LDS;
//  2. every line along d reconstructed at the tile's faces (both sides: values and normal slopes), for the
//     TA + 4 x TB + 4 lines the tangential sweeps need;
//  3. per side of the faces: (a) sweep 1 along da at the two Gauss coordinates, once per row of the tile
//     and its db-halo, into LDS (each result serves the five faces along db whose stencils hold the row);
//     (b) each thread takes one Gauss point (g1, g2) of a face: sweep 2 along db over five rows of (a),
//     then that side's part of the gas-kinetic flux;
//  4. the flux and its time derivative, averaged over the four Gauss points with lane exchanges.
// LDS: 72 KiB in FP64, so two blocks share a CU; the register allocator works to two waves per SIMD (in
// FP64 it spills some 50 bytes per lane, which measures faster than one wave per SIMD without spills).
template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_flux3(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts,
                                               const int* __restrict__ off, int nprob, int stage) {
  constexpr int TN = kTN3, TA = kTA3, TB = kTB3;
  static_assert(TN == 4 && TA == 4 && TB == 4, "thread mappings below assume 4 x 4 x 4 faces and 256 threads");
  constexpr int CN = TN + 5, CA = TA + 4, CB = TB + 4;  // staged cells: normal -3..TN+1, tangential -2..T+1
  constexpr int NRS = 21;  // 20 values per line and face, odd stride: conflict-free 8-byte LDS reads
  constexpr int S1 = 15;   // per sweep-1 result: value, da-derivative, value of the normal slope
  constexpr int NW = 5 * CB * CA * CN, NS1 = CB * TA * TN * 2 * S1;
  __shared__ T sNR[CB][CA][TN][NRS];
  __shared__ uint8_t sFl[CB][CA][CN];  // flags of the staged cells (0 outside the extended range)
  __shared__ T sU[NW > NS1 ? NW : NS1];  // cells (phases 1-2), then one side's sweep-1 results (phase 3)
#define SW(v, cb, ca, cn) sU[(((v) * CB + (cb)) * CA + (ca)) * CN + (cn)]
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int p = find_prob(off, nprob, b);
  const ProbDev& P = probs[p];
  const TimeDev& tsp = ts[p];
  if (!tsp.active) return;
  const int tid = threadIdx.x;
  int lt = b - off[p];
  int d = 0;
  {
    const int nt0 = ((P.nx + TN) / TN) * ((P.ny + TA - 1) / TA) * ((P.nz + TB - 1) / TB);
    const int nt1 = ((P.ny + TN) / TN) * ((P.nz + TA - 1) / TA) * ((P.nx + TB - 1) / TB);
    if (lt >= nt0) { lt -= nt0; d = 1; }
    if (d == 1 && lt >= nt1) { lt -= nt1; d = 2; }
  }
  const int da = (d + 1) % 3, db = (d + 2) % 3;
  const int nn = sel3(d, P.nx, P.ny, P.nz), na = sel3(da, P.nx, P.ny, P.nz), nb = sel3(db, P.nx, P.ny, P.nz);
  const int tn = (nn + 1 + TN - 1) / TN, ta = (na + TA - 1) / TA;
  const int n0 = (lt % tn) * TN, a0 = ((lt / tn) % ta) * TA, b0 = (lt / (tn * ta)) * TB;
  const double* __restrict__ Wsrc = (stage == 1) ? P.W : P.Ws;

  // ---- 1: cells and their flags. Consecutive threads take consecutive x (the normal for x-faces, the
  // second tangential axis for y-faces, the first for z-faces), so that the loads coalesce.
  for (int e = tid; e < CN * CA * CB; e += 256) {
    int cn, ca, cb;
    if (d == 0) { cn = e % CN; ca = (e / CN) % CA; cb = e / (CN * CA); }
    else if (d == 1) { cb = e % CB; cn = (e / CB) % CN; ca = e / (CB * CN); }
    else { ca = e % CA; cb = (e / CA) % CB; cn = e / (CA * CB); }
    int i, j, k;
    grid_of_frame(d, n0 - 3 + cn, a0 - 2 + ca, b0 - 2 + cb, i, j, k);
    double q[5];
    load_cell3(P, Wsrc, i, j, k, q);
    sFl[cb][ca][cn] = flag3_at(P, i, j, k);
    SW(0, cb, ca, cn) = T(q[0]);
    SW(1, cb, ca, cn) = T(sel3(d, q[1], q[2], q[3]));
    SW(2, cb, ca, cn) = T(sel3(da, q[1], q[2], q[3]));
    SW(3, cb, ca, cn) = T(sel3(db, q[1], q[2], q[3]));
    SW(4, cb, ca, cn) = T(q[4]);
  }
  __syncthreads();

  // ---- 2: normal reconstruction, one line and face per thread (CA * CB * TN = 256)
  const T gam = T(P.gamma), ghi = T(P.ghi), glo = T(P.glo), eps = T(P.eps);
  const T ihn = T(1.0 / sel3(d, P.dx, P.dy, P.dz)), iha = T(1.0 / sel3(da, P.dx, P.dy, P.dz)),
          ihb = T(1.0 / sel3(db, P.dx, P.dy, P.dz));
  {
    const int kl = tid % TN, al = (tid / TN) % CA, bl = tid / (TN * CA);
    T q6[6][5];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) q6[m][v] = SW(v, bl, al, kl + m);
    const int fl = (sFl[bl][al][kl + 2] >> d) & 1, fr = (sFl[bl][al][kl + 3] >> d) & 1;
    T out[20];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      out[v] = (T(2) * q6[0][v] - T(13) * q6[1][v] + T(47) * q6[2][v] + T(27) * q6[3][v] - T(3) * q6[4][v]) *
               T(1.0 / 60.0);
      const T sl = (q6[1][v] - T(15) * q6[2][v] + T(15) * q6[3][v] - q6[4][v]) * (T(1.0 / 12.0) * ihn);
      out[5 + v] = sl;
      out[15 + v] = sl;
      out[10 + v] = (T(-3) * q6[1][v] + T(27) * q6[2][v] + T(47) * q6[3][v] - T(13) * q6[4][v] + T(2) * q6[5][v]) *
                    T(1.0 / 60.0);
    }
    if (fl | fr) {
      Char5<T> m;
      T avg[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) avg[v] = T(0.5) * (q6[2][v] + q6[3][v]);
      char5(avg, gam, m);
      T val[5], der[5];
      if (fl) {
        ao_vector5<1>(reinterpret_cast<const T(*)[5]>(&q6[0][0]), m, 0, ghi, glo, eps, val, der);
#pragma unroll
        for (int v = 0; v < 5; ++v) { out[v] = val[v]; out[5 + v] = der[v] * ihn; }
      }
      if (fr) {
        ao_vector5<1>(reinterpret_cast<const T(*)[5]>(&q6[1][0]), m, 1, ghi, glo, eps, val, der);
#pragma unroll
        for (int v = 0; v < 5; ++v) { out[10 + v] = val[v]; out[15 + v] = der[v] * ihn; }
      }
    }
#pragma unroll
    for (int v = 0; v < 20; ++v) sNR[bl][al][kl][v] = out[v];
  }
  __syncthreads();

  // ---- 3: per side, sweep 1 (one result per thread: row irb, column ial, face ikl, coordinate ig1), then
  // sweep 2 + flux at Gauss point (g1, g2) of face (kl, al, bl)
  const int ig1 = tid & 1, ikl = (tid >> 1) & 3, ial = (tid >> 3) & 3, irb = tid >> 5;
  const int f = tid >> 2, g = tid & 3, g1 = g & 1, g2 = g >> 1;
  const int kl = f % TN, al = (f / TN) % TA, bl = f / (TN * TA);
  const int n = n0 + kl, a = a0 + al, bb = b0 + bl;
  const bool valid = n <= nn && a < na && bb < nb;  // the four lanes of a face agree
  const T K = T(P.K), Kp3 = T(P.K + 3.0), iKp3 = T(1.0 / (P.K + 3.0));
  // FP64: the first side's flux waits until both sides are reconstructed, so that its accumulators are not
  // live through the second side's sweeps (20 held values instead of 37: fewer spills, 15% faster);
  // FP32 has the registers and runs faster in the plain order.
  constexpr bool kDefer = sizeof(T) == 8;
  FluxAcc3<T> acc;
  T S0[4][5];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (s == 1) __syncthreads();  // side 0's sweep-2 reads are done before side 1's results overwrite them
    {
      const int fa = (sFl[irb][ial + 2][ikl + 2 + s] >> da) & 1;  // cell (n0 + ikl - 1 + s, a0 + ial, b0 - 2 + irb)
      Char5<T> m;
      if (fa) {
        T own[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) own[v] = sNR[irb][ial + 2][ikl][10 * s + v];
        char5(own, gam, m);
      }
      T q[5][5], val[5], der[5];
      T* o = &sU[tid * S1];
#pragma unroll
      for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int v = 0; v < 5; ++v) q[r][v] = sNR[irb][ial + r][ikl][10 * s + v];
      sweep5<2>(q, fa, m, ig1, ghi, glo, eps, val, der);
#pragma unroll
      for (int v = 0; v < 5; ++v) { o[v] = val[v]; o[5 + v] = der[v] * iha; }
#pragma unroll
      for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int v = 0; v < 5; ++v) q[r][v] = sNR[irb][ial + r][ikl][10 * s + 5 + v];
      sweep5<2>(q, fa, m, ig1, ghi, glo, eps, val, der);
#pragma unroll
      for (int v = 0; v < 5; ++v) o[10 + v] = val[v];
    }
    __syncthreads();
    if (valid) {
      const int fb = (sFl[bl + 2][al + 2][kl + 2 + s] >> db) & 1;  // cell (n - 1 + s, a, bb)
      const T* row = &sU[((bl * TA + al) * TN + kl) * 2 * S1 + g1 * S1];
      constexpr int RS = TA * TN * 2 * S1;  // next row along db
      T q[5][5], Wp[5], Wn[5], Wa[5], Wb[5], der[5];
#pragma unroll
      for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int v = 0; v < 5; ++v) q[r][v] = row[r * RS + v];
      Char5<T> m;
      if (fb) char5(q[2], gam, m);  // the sweep's centre value
      sweep5<3>(q, fb, m, g2, ghi, glo, eps, Wp, der);
#pragma unroll
      for (int v = 0; v < 5; ++v) Wb[v] = der[v] * ihb;
#pragma unroll
      for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int v = 0; v < 5; ++v) q[r][v] = row[r * RS + 5 + v];
      sweep5<3>(q, fb, m, g2, ghi, glo, eps, Wa, der);
#pragma unroll
      for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int v = 0; v < 5; ++v) q[r][v] = row[r * RS + 10 + v];
      sweep5<3>(q, fb, m, g2, ghi, glo, eps, Wn, der);
      if constexpr (kDefer) {
        if (s == 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) { S0[0][v] = Wp[v]; S0[1][v] = Wn[v]; S0[2][v] = Wa[v]; S0[3][v] = Wb[v]; }
        } else {
          flux3_side<0>(S0[0], S0[1], S0[2], S0[3], gam, K, Kp3, iKp3, acc);
          flux3_side<1>(Wp, Wn, Wa, Wb, gam, K, Kp3, iKp3, acc);
        }
      } else {
        if (s == 0) flux3_side<0>(Wp, Wn, Wa, Wb, gam, K, Kp3, iKp3, acc);
        else flux3_side<1>(Wp, Wn, Wa, Wb, gam, K, Kp3, iKp3, acc);
      }
    }
  }
#undef SW
  if (!valid) return;  // no barrier below

  // ---- 4: the gas-kinetic flux of the Gauss point, averaged over the face's four lanes
  FluxParams fp;
  fp.gamma = P.gamma; fp.K = P.K; fp.mu = P.mu; fp.Pr = P.Pr; fp.c1 = P.c1; fp.c2 = P.c2;
  fp.Kp2 = P.Kp2; fp.iKp2 = P.iKp2; fp.kpr = P.kpr;
  fp.dt = tsp.dt; fp.dth = tsp.dth; fp.idt = tsp.idt; fp.idt2 = tsp.idt2;
  fp.ns = P.ns; fp.want_F = (stage != 2);
  T F[5] = {0, 0, 0, 0, 0}, dF[5] = {0, 0, 0, 0, 0};
  flux3_finish(acc, fp, Kp3, iKp3, T(0.25), F, dF);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    F[v] += __shfl_xor(F[v], 1, 64);
    F[v] += __shfl_xor(F[v], 2, 64);
    dF[v] += __shfl_xor(dF[v], 1, 64);
    dF[v] += __shfl_xor(dF[v], 2, 64);
  }
  if (g != 0) return;
  // grid component of each frame slot; the second stage's dF/dt goes to the F arrays (as in 2D)
  T* Fo = reinterpret_cast<T*>(d == 0 ? P.Fx : (d == 1 ? P.Fy : P.Fz));
  T* Go = stage != 2 ? reinterpret_cast<T*>(d == 0 ? P.Gx : (d == 1 ? P.Gy : P.Gz)) : Fo;
  int i, j, k;
  grid_of_frame(d, n, a, bb, i, j, k);
  const int M0 = P.nx + (d == 0), M1 = P.ny + (d == 1), M2 = P.nz + (d == 2);
  const size_t plane = (size_t)M0 * M1 * M2;
  const size_t o = ((size_t)k * M1 + j) * M0 + i;
  const size_t oc[5] = {0, (size_t)(1 + d) * plane, (size_t)(1 + da) * plane, (size_t)(1 + db) * plane, 4 * plane};
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    if (stage != 2) Fo[oc[v] + o] = F[v];
    Go[oc[v] + o] = dF[v];
  }
}

__device__ inline double cfl_quantity3(const ProbDev& P, double rho, double mx, double my, double mz, double E) {
#pragma clang fp contract(off)
  const double U = mx / rho, V = my / rho, Z = mz / rho;
  const double pr = (P.gamma - 1.0) * (E - 0.5 * rho * (U * U + V * V + Z * Z));
  const double c = sqrt(P.gamma * pr / rho);
  double q = P.h / (sqrt(U * U + V * V + Z * Z) + c);
  if (P.ns) q = fmin(q, (P.h * P.h) / (4.0 * (P.mu / (P.vdt ? pr : rho))));
  return q;
}

__global__ void __launch_bounds__(256) k_cfl3(const ProbDev* __restrict__ probs, const int* __restrict__ off,
                                              int nprob, double* __restrict__ qpart) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  const size_t ncell = (size_t)P.nx * P.ny * P.nz;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  double q = __builtin_inf();
  if (cell < ncell) {
    const double* W = P.W;
    q = cfl_quantity3(P, W[cell], W[ncell + cell], W[2 * ncell + cell], W[3 * ncell + cell], W[4 * ncell + cell]);
  }
  q = block_min(q);
  if (threadIdx.x == 0) qpart[blockIdx.x] = q;
}

// S2O4 stage updates of a 3D problem (the same sums as k_update, over six faces)
template <typename T>
__global__ void __launch_bounds__(256) k_update3(const ProbDev* __restrict__ probs, TimeDev* __restrict__ ts,
                                                 const int* __restrict__ off, int nprob, int stage,
                                                 double* __restrict__ qpart) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  TimeDev& tsp = ts[p];
  if (!tsp.active) return;
  const size_t ncell = (size_t)P.nx * P.ny * P.nz;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  double q = __builtin_inf();
  if (cell < ncell) {
    const int i = (int)(cell % P.nx), j = (int)((cell / P.nx) % P.ny), k = (int)(cell / ((size_t)P.nx * P.ny));
    const double dt = tsp.dt;
    const double ih[3] = {1.0 / P.dx, 1.0 / P.dy, 1.0 / P.dz};
    const T* Fa[3] = {reinterpret_cast<const T*>(P.Fx), reinterpret_cast<const T*>(P.Fy),
                      reinterpret_cast<const T*>(P.Fz)};
    const T* Ga[3] = {reinterpret_cast<const T*>(stage == 1 ? P.Gx : P.Fx),
                      reinterpret_cast<const T*>(stage == 1 ? P.Gy : P.Fy),
                      reinterpret_cast<const T*>(stage == 1 ? P.Gz : P.Fz)};
    size_t plane[3], lo[3], step[3];
    plane[0] = (size_t)P.nz * P.ny * (P.nx + 1); lo[0] = ((size_t)k * P.ny + j) * (P.nx + 1) + i; step[0] = 1;
    plane[1] = (size_t)P.nz * (P.ny + 1) * P.nx; lo[1] = ((size_t)k * (P.ny + 1) + j) * P.nx + i; step[1] = P.nx;
    plane[2] = (size_t)(P.nz + 1) * P.ny * P.nx; lo[2] = ((size_t)k * P.ny + j) * P.nx + i;
    step[2] = (size_t)P.ny * P.nx;
    double wn[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double fs = 0.0, gs = 0.0;
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        const size_t o = c * plane[dd] + lo[dd];
        gs += (double(Ga[dd][o + step[dd]]) - double(Ga[dd][o])) * ih[dd];
        if (stage == 1) fs += (double(Fa[dd][o + step[dd]]) - double(Fa[dd][o])) * ih[dd];
      }
      const double w = P.W[c * ncell + cell];
      if (stage == 1) {
        const double ws = w - dt * (0.5 * fs + 0.125 * dt * gs);
        P.Ws[c * ncell + cell] = ws;
        P.S[c * ncell + cell] = w - dt * (fs + dt / 6.0 * gs);
        wn[c] = ws;
      } else {
        const double wnew = P.S[c * ncell + cell] - dt * dt / 3.0 * gs;
        P.Ws[c * ncell + cell] = wnew;  // W* is spent: the new state waits there for the commit
        wn[c] = wnew;
      }
    }
    const double rho = wn[0];
    const double pr = (P.gamma - 1.0) * (wn[4] - 0.5 * (wn[1] * wn[1] + wn[2] * wn[2] + wn[3] * wn[3]) / rho);
    if (!(rho > 0.0) || !(pr > 0.0) || !(wn[4] < __builtin_inf())) report_nonphysical(tsp, stage, cell);
    if (stage == 2) q = cfl_quantity3(P, wn[0], wn[1], wn[2], wn[3], wn[4]);
  }
  if (stage == 2) {
    q = block_min(q);
    if (threadIdx.x == 0) qpart[blockIdx.x] = q;
  }
}

// ---------------------------------------------------------------------------------------------
// Host-side launchers of the 3D kernels
// ---------------------------------------------------------------------------------------------
void launch_cfl3(const LaunchCtx& L) {
  hipLaunchKernelGGL(k_cfl3, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.off_cell, L.nprob, L.qpart);
}

void launch_flags3(const LaunchCtx& L, int stage_state, int count) {
  hipLaunchKernelGGL(k_flags3, dim3(L.ext_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_ext, L.nprob,
                     stage_state, count);
}

void launch_flux3(const LaunchCtx& L, int stage) {
  if (L.fp32)
    hipLaunchKernelGGL(k_flux3<float>, dim3(L.flux_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_flux,
                       L.nprob, stage);
  else
    hipLaunchKernelGGL(k_flux3<double>, dim3(L.flux_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_flux,
                       L.nprob, stage);
}

void launch_update3(const LaunchCtx& L, int stage) {
  if (L.fp32)
    hipLaunchKernelGGL(k_update3<float>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, stage, L.qpart);
  else
    hipLaunchKernelGGL(k_update3<double>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, stage, L.qpart);
}

}  // namespace hk
