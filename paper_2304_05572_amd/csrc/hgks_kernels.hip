// HIP kernels of the hybrid WENO5-AO gas-kinetic scheme (Mu et al., arXiv 2304.05572) for gfx950.
//
// One step of one or many problems (each with its own time step) is
//   k_dt_finalize -> [k_flags -> k_flux(stage 1) -> k_update(stage 1)]
//                 -> [k_flags -> k_flux(stage 2) -> k_update(stage 2, + CFL partials)] (-> k_repair)
//                 -> k_commit
// (a multistage tableau instead runs [k_flags -> k_flux(stage 1 or 3) -> k_update_ms] per stage).
// Work is split into tiles; a prefix-sum table maps a flat block index to (problem, tile), so a batch
// of uneven problems runs in the same launches as a single problem.
#include <hip/hip_runtime.h>

#include "hgks_device.hpp"
#include "hgks_grid.hpp"
#include "hgks_launch.h"

namespace hk {

// ---------------------------------------------------------------------------------------------
// CFL quantity of one cell: min(h / (|U| + c), h^2 / (4 mu / rho)) (Sec. 3), FP64, no contraction,
// the same expression tree as the reference evaluation so the minimum is reproducible bit for bit.
// ---------------------------------------------------------------------------------------------
__device__ inline double cfl_quantity(const ProbDev& P, double rho, double mu_, double mv,
                                                         double E) {
#pragma clang fp contract(off)
  const double U = mu_ / rho;
  const double V = (P.dim == 2) ? mv / rho : 0.0;
  const double pr = (P.gamma - 1.0) * (E - 0.5 * rho * (U * U + V * V));
  const double c = sqrt(P.gamma * pr / rho);
  const double sp = sqrt(U * U + V * V) + c;
  double q = P.h / sp;
  if (P.ns) {
    const double qv = (P.h * P.h) / (4.0 * (P.mu / (P.vdt ? pr : rho)));
    q = fmin(q, qv);
  }
  return q;
}

// The CFL minimum is reduced in two levels: every block of the cell-wise kernels (this one and the
// second-stage update) stores its minimum in qpart[block], and the next dt finalisation reduces the
// blocks of each problem. Minima are order-independent, so the time step is reproducible bit for bit.
__global__ void __launch_bounds__(256) k_cfl(const ProbDev* __restrict__ probs, const int* __restrict__ off,
                                             int nprob, double* __restrict__ qpart) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  const size_t ncell = (size_t)P.nx * P.ny;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  double q = __builtin_inf();
  if (cell < ncell) {
    const double* W = P.W;
    const double mv = (P.dim == 2) ? W[2 * ncell + cell] : 0.0;
    q = cfl_quantity(P, W[cell], W[ncell + cell], mv, W[(P.dim + 1) * ncell + cell]);
  }
  q = block_min(q);
  if (threadIdx.x == 0) qpart[blockIdx.x] = q;
}

// One block per problem: the minimum over the problem's block minima, then dt (Sec. 3) by thread 0.
__global__ void __launch_bounds__(256) k_dt_finalize(const ProbDev* __restrict__ probs, TimeDev* __restrict__ ts,
                                                     const int* __restrict__ off, const double* __restrict__ qpart,
                                                     int use_tend) {
  const int p = blockIdx.x;
  // four independent loads in flight per thread, then the tree
  double q0 = __builtin_inf(), q1 = q0, q2 = q0, q3 = q0;
  const int b1 = off[p + 1];
  const int stride = blockDim.x;
  int b = off[p] + threadIdx.x;
  for (; b + 3 * stride < b1; b += 4 * stride) {
    q0 = fmin(q0, qpart[b]);
    q1 = fmin(q1, qpart[b + stride]);
    q2 = fmin(q2, qpart[b + 2 * stride]);
    q3 = fmin(q3, qpart[b + 3 * stride]);
  }
  for (; b < b1; b += stride) q0 = fmin(q0, qpart[b]);
  double q = block_min(fmin(fmin(q0, q1), fmin(q2, q3)));
  if (threadIdx.x != 0) return;
  TimeDev& s = ts[p];
  const ProbDev& P = probs[p];
  P.flag_count[0] = 0;             // troubled cells are counted afresh by the step's first flag pass
  P.flag_count[1] = 0;
  P.flag_count[2] = 0;
  if (!s.active) {
    set_time_step(s, 0.0);
    return;
  }
  double dt = (P.fixed_dt > 0.0) ? P.fixed_dt : P.cfl * q;
  if (!(dt > 0.0) || !(dt < __builtin_inf())) {
    s.status |= 2;
    s.active = 0;
    set_time_step(s, 0.0);
    return;
  }
  if (use_tend && s.t + dt >= s.t_end) {
    dt = s.t_end - s.t;
    s.t_new = s.t_end;
  } else {
    s.t_new = s.t + dt;
  }
  set_time_step(s, dt);
}

// End of a step: a problem whose step produced a non-physical state stops with W^n (its new state, in the
// second buffer, is dropped); the others take the new state by swapping the two buffers and advance t.
__global__ void k_commit(ProbDev* __restrict__ probs, TimeDev* __restrict__ ts, int nprob, int use_tend) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  TimeDev& s = ts[p];
  if (!s.active) return;
  if (s.status & 1) {
    s.active = 0;
    return;
  }
  ProbDev& P = probs[p];
  double* w = P.W;
  P.W = P.Ws;
  P.Ws = w;
  if (P.E) {
    double* e = P.E;
    P.E = P.E2;
    P.E2 = e;
  }
  s.cur ^= 1;
  s.t = s.t_new;
  s.steps += 1;
  if (use_tend && s.t >= s.t_end) s.active = 0;
}

// After the commit a problem's current state sits in its second buffer when the step was clean: copy it
// into the first (the caller-owned state of the entry point that allocates nothing). Problems whose step
// stopped keep the first buffer as it was.
__global__ void __launch_bounds__(256) k_state_home(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts,
                                                    const int* __restrict__ off, int nprob) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  if (!ts[p].cur) return;
  const size_t ncell = (size_t)P.nx * P.ny;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  if (cell >= ncell) return;
  const int nc = P.dim + 2;
  for (int c = 0; c < nc; ++c) P.Ws[c * ncell + cell] = P.W[c * ncell + cell];
}

// ---------------------------------------------------------------------------------------------
// Troubled-cell flags (Sec. 2.3.1 Steps 1-4) of every cell of the extended range [-2, n+1]:
// T of the cell and both neighbours, OR over the four conserved components, per direction.
// ---------------------------------------------------------------------------------------------
__device__ inline int troubled_cell(const double q[5][4], double thr) {
  int t = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) t |= troubled5(q[0][c], q[1][c], q[2][c], q[3][c], q[4][c], thr);
  return t;
}

__device__ inline int widened_flag(const ProbDev& P, const double* W, int i, int j, int dir, double thr,
                                   double tb) {
  double q[7][4];
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    if (dir == 0) load_cell(P, W, i - 3 + r, j, tb, q[r]);
    else load_cell(P, W, i, j - 3 + r, tb, q[r]);
  }
  int f = 0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    double w[5][4];
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) w[r][c] = q[s + r][c];
    f |= troubled_cell(w, thr);
  }
  return f;
}

__global__ void __launch_bounds__(256) k_flags(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts,
                                               const int* __restrict__ off, int nprob, int use_stage_state,
                                               int count) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  if (!ts[p].active) return;
  const int ex = P.nx + 4, ey = (P.dim == 2) ? P.ny + 4 : 1;
  const int e = (blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  int fl = 0, interior = 0;
  if (e < ex * ey) {
    const int i = e % ex - 2, j = (P.dim == 2) ? e / ex - 2 : 0;
    const double* W = use_stage_state ? P.Ws : P.W;
    const double tb = use_stage_state ? ts[p].t + ts[p].dth : ts[p].t;  // the stage's time
    if (P.recon == 1) {
      fl = (P.dim == 2) ? 3 : 1;
    } else if (P.recon == 0) {
      const double tx = (P.zeta1_mode == 0) ? 5.0 * P.dx : 5.0 * P.dx * P.dx * P.dx;
      fl = widened_flag(P, W, i, j, 0, tx, tb);
      if (P.dim == 2) {
        const double ty = (P.zeta1_mode == 0) ? 5.0 * P.dy : 5.0 * P.dy * P.dy * P.dy;
        fl |= widened_flag(P, W, i, j, 1, ty, tb) << 1;
      }
    }
    P.flags[e] = (uint8_t)fl;
    interior = (i >= 0 && i < P.nx && j >= 0 && j < P.ny);
  }
  if (count) {
    const unsigned long long bx = __ballot(interior && (fl & 1));
    const unsigned long long by = __ballot(interior && (fl & 2));
    if ((threadIdx.x & 63) == 0) {
      if (bx) atomicAdd(&P.flag_count[0], __popcll(bx));
      if (by) atomicAdd(&P.flag_count[1], __popcll(by));
    }
  }
}

// 2D form: a block owns a kFX x kFY tile of the extended range (the tile shape is in hgks_launch.h).
// Every thread first issues the loads of its share of the tile's cells and their 3-cell halo (ghosts
// synthesised); the four conserved components then pass one at a time through a single LDS plane, and
// the indicator T of each is evaluated for the tile plus one cell on each side, along x and along y, and
// OR-ed into registers. One plane instead of four keeps the block's LDS small, so that enough blocks
// share a CU for their load latencies to overlap. Finally T is widened (Step 4) and the flags written.
__global__ void __launch_bounds__(kFThreads) k_flags2d(const ProbDev* __restrict__ probs,
                                                      const TimeDev* __restrict__ ts,
                                                      const int* __restrict__ off, int nprob,
                                                      int use_stage_state, int count) {
  constexpr int LX = kFX + 6, LY = kFY + 6;
  constexpr int RPT = kFX * kFY / kFThreads;  // output rows per thread
  constexpr int NTX = kFY * (kFX + 2), NTY = (kFY + 2) * kFX;  // T_x and T_y evaluations per component
  constexpr int EX = (NTX + kFThreads - 1) / kFThreads, EY = (NTY + kFThreads - 1) / kFThreads;
  static_assert(kFX * kFY % kFThreads == 0 && kFThreads % kFX == 0, "whole rows per thread");
  __shared__ double sQ[LY][LX];             // one component of cell (i0 - 3 + s, j0 - 3 + r) at [r][s]
  __shared__ uint8_t sTx[kFY][kFX + 2];     // T_x of cell (i0 - 1 + a, j0 + b) at [b][a]
  __shared__ uint8_t sTy[kFY + 2][kFX];     // T_y of cell (i0 + a, j0 - 1 + b) at [b][a]
  // neighbouring tiles share their halos: keep them on one XCD (and its L2)
  const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
  const int p = find_prob(off, nprob, blk);
  const ProbDev& P = probs[p];
  if (!ts[p].active) return;
  const int ex = P.nx + 4;
  const int tiles_x = (ex + kFX - 1) / kFX;
  const int lt = blk - off[p];
  const int i0 = (lt % tiles_x) * kFX - 2, j0 = (lt / tiles_x) * kFY - 2;  // first cell of the tile
  const int tid = threadIdx.x;
  const int a = tid % kFX, b0 = tid / kFX;  // rows b0, b0 + kFY / RPT, ...
  int fl[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) fl[q] = 0;
  if (P.recon == 1) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) fl[q] = 3;
  } else if (P.recon == 0) {
    const double* W = use_stage_state ? P.Ws : P.W;
    const double tb = use_stage_state ? ts[p].t + ts[p].dth : ts[p].t;  // the stage's time
    // all of a thread's loads are issued before the first LDS store (unrolled, fixed trip count)
    constexpr int NL = (LX * LY + kFThreads - 1) / kFThreads;
    double q4[NL][4];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = tid + u * kFThreads;
      if (e < LX * LY) load_cell(P, W, i0 - 3 + e % LX, j0 - 3 + e / LX, tb, q4[u]);
    }
    const double tx = (P.zeta1_mode == 0) ? 5.0 * P.dx : 5.0 * P.dx * P.dx * P.dx;
    const double ty = (P.zeta1_mode == 0) ? 5.0 * P.dy : 5.0 * P.dy * P.dy * P.dy;
    int Tx[EX], Ty[EY];
#pragma unroll
    for (int u = 0; u < EX; ++u) Tx[u] = 0;
#pragma unroll
    for (int u = 0; u < EY; ++u) Ty[u] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k) __syncthreads();  // the previous component's reads are done
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int e = tid + u * kFThreads;
        if (e < LX * LY) sQ[e / LX][e % LX] = q4[u][k];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < EX; ++u) {  // T_x: row bb, cells aa .. aa+4
        const int e = tid + u * kFThreads;
        if (e < NTX) {
          const int bb = e / (kFX + 2), aa = e % (kFX + 2);
          const double* r = &sQ[bb + 3][aa];
          if (!Tx[u]) Tx[u] = troubled5(r[0], r[1], r[2], r[3], r[4], tx);  // T is the OR over components
        }
      }
#pragma unroll
      for (int u = 0; u < EY; ++u) {  // T_y: column ay, rows by .. by+4
        const int e = tid + u * kFThreads;
        if (e < NTY) {
          const int ay = e % kFX, by = e / kFX;
          if (!Ty[u])
            Ty[u] = troubled5(sQ[by][ay + 3], sQ[by + 1][ay + 3], sQ[by + 2][ay + 3], sQ[by + 3][ay + 3],
                              sQ[by + 4][ay + 3], ty);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < EX; ++u) {
      const int e = tid + u * kFThreads;
      if (e < NTX) sTx[e / (kFX + 2)][e % (kFX + 2)] = (uint8_t)Tx[u];
    }
#pragma unroll
    for (int u = 0; u < EY; ++u) {
      const int e = tid + u * kFThreads;
      if (e < NTY) sTy[e / kFX][e % kFX] = (uint8_t)Ty[u];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int b = b0 + q * (kFY / RPT);
      fl[q] = (sTx[b][a] | sTx[b][a + 1] | sTx[b][a + 2]) | ((sTy[b][a] | sTy[b + 1][a] | sTy[b + 2][a]) << 1);
    }
  }
  int cx = 0, cy = 0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = i0 + a, j = j0 + b0 + q * (kFY / RPT);
    const bool inside = (i < P.nx + 2) && (j < P.ny + 2);
    if (inside) P.flags[(size_t)(j + 2) * ex + (i + 2)] = (uint8_t)fl[q];
    if (count) {
      const bool interior = inside && i >= 0 && i < P.nx && j >= 0 && j < P.ny;
      cx += __popcll(__ballot(interior && (fl[q] & 1)));
      cy += __popcll(__ballot(interior && (fl[q] & 2)));
    }
  }
  if (count && (tid & 63) == 0) {
    if (cx) atomicAdd(&P.flag_count[0], cx);
    if (cy) atomicAdd(&P.flag_count[1], cy);
  }
}

__global__ void k_clear_counts(const ProbDev* __restrict__ probs, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nprob) {
    probs[p].flag_count[0] = 0;
    probs[p].flag_count[1] = 0;
    probs[p].flag_count[2] = 0;
  }
}

// Whether a reconstructed state (rho, normal momentum, tangential momentum, energy) has positive
// density and a pressure above the rounding error of the arithmetic that produced it: the state is a
// combination of values whose energies reach emax, so its energy, and with it the pressure, carries an
// absolute rounding error of a few units of emax in the last place of T. A pressure within 64 such units
// of zero has no reliable sign (or digits): taken as not physical. In FP64 the margin is 7e-15 emax; in
// FP32 4e-6 emax, where the half-space moments of a state that cold would be ruled by rounding.
template <typename T>
__device__ inline bool admissible(const T* w, T gam, T emax) {
  constexpr T tol = T(64) * unit_roundoff<T>();
  const T pr = (gam - T(1)) * (w[3] - T(0.5) * (w[1] * w[1] + w[2] * w[2]) / w[0]);
  return w[0] > T(0) && pr > tol * emax && isfinite(pr);
}

// Largest |energy| of the five stencil values q[r][3] (frame slot 3 holds the energy).
template <typename T>
__device__ inline T stencil_emax(const T q0, const T q1, const T q2, const T q3, const T q4) {
  return fmax(fmax(fmax(fabs(q0), fabs(q1)), fmax(fabs(q2), fabs(q3))), fabs(q4));
}

// Stride (in values) of one interface entry of the normal-reconstruction rows in LDS, and of one row
// of TN entries: FP64 rows take 2 more values so that rows four apart fall on different banks (the
// y-interface blocks read rows tt and tt + 4 in one half-wavefront).
constexpr int kNRS = 17;
template <typename T, int TN>
constexpr int nr_row() { return TN * kNRS + (sizeof(T) == 8 ? 2 : 0); }

// Threads of a flux block: one per Gauss point in 2D (two per interface), one per interface in 1D.
constexpr int flux_threads(int tn, int tt, int dim) { return (dim == 2 ? 2 : 1) * tn * tt; }

// Tangential reconstruction (Sec. 2.3.3, Step 2) of side s of interface column k at Gauss point gp from
// the line averages of rows tt..tt+4 (value line W^s and normal-slope line W^s_x): values at the Gauss
// point, tangential slope of W^s, value of W^s_x. Linear quartic per component, or WENO-AO in the
// tangential characteristic variables about the side's own centre-segment state (csm = 0) or the mean of
// both sides' (csm = 1) when flagged.
template <typename T, int TN, int R>
__device__ inline void tangential_side(const T* sNR, int tt, int k, int s, int ft, int gp, T gam, T ghi,
                                       T glo, T eps, T iht, int pos, int csm, T Ws[4], T Wxs[4], T Wys[4]) {
  constexpr int NRW = nr_row<T, TN>();
  const int ov = 8 * s, od = 8 * s + 4;
  if (ft) {
    Char4<T> m;
    T own[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      own[v] = csm ? T(0.5) * (sNR[(tt + 2) * NRW + k * kNRS + v] + sNR[(tt + 2) * NRW + k * kNRS + 8 + v])
                   : sNR[(tt + 2) * NRW + k * kNRS + ov + v];
    char4(own, gam, m);
    T val[4], der[4];
    ao_vector<2>(sNR + tt * NRW + k * kNRS + ov, NRW, 1, m, 2 + gp, ghi, glo, eps, val, der);
#pragma unroll
    for (int v = 0; v < 4; ++v) { Ws[v] = val[v]; Wys[v] = der[v] * iht; }
    ao_vector<2>(sNR + tt * NRW + k * kNRS + od, NRW, 1, m, 2 + gp, ghi, glo, eps, val, der);
#pragma unroll
    for (int v = 0; v < 4; ++v) Wxs[v] = val[v];
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T q[5], qx[5], vv, dd, vx, dx_;
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        q[r] = sNR[(tt + r) * NRW + k * kNRS + ov + v];
        qx[r] = sNR[(tt + r) * NRW + k * kNRS + od + v];
      }
      gauss_linear(q, gp, vv, dd);
      gauss_linear(qx, gp, vx, dx_);
      Ws[v] = vv;
      Wys[v] = dd * iht;
      Wxs[v] = vx;
    }
  }
  if (pos && !admissible(Ws, gam,
                         stencil_emax(sNR[(tt + 0) * NRW + k * kNRS + ov + 3], sNR[(tt + 1) * NRW + k * kNRS + ov + 3],
                                      sNR[(tt + 2) * NRW + k * kNRS + ov + 3], sNR[(tt + 3) * NRW + k * kNRS + ov + 3],
                                      sNR[(tt + 4) * NRW + k * kNRS + ov + 3]))) {
    // first order along the interface: the centre segment's line values
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ws[v] = sNR[(tt + 2) * NRW + k * kNRS + ov + v];
      Wys[v] = T(0);
      Wxs[v] = sNR[(tt + 2) * NRW + k * kNRS + od + v];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Fused reconstruction + gas-kinetic flux. A block owns TN interfaces along the normal direction of
// TT rows (2D) and stages in LDS:
//   sW  : cell averages, normal -3..TN+1 around the interfaces, rows -2..TT+1 (ghosts synthesised)
//   sF  : flags of the cells adjacent to each interface (bit 0 normal, bit 1 tangential)
//   sNR : normal reconstruction of every row: W^l, W^l_x, W^r, W^r_x (16 values per interface, padded
//         to 17 so that the lanes of a wavefront spread over the LDS banks: neighbouring interfaces and
//         rows would otherwise sit a multiple of 128 bytes apart and hit the same banks; FP64 rows are
//         padded by 2 more values, see nr_row)
// then each thread takes one interface through the tangential reconstruction at the two Gauss
// points, the equilibrium state and the flux (Sec. 2.3.3 Steps 1-3, Sec. 2.1-2.2).
// Frame: slot 1 holds the normal momentum, slot 2 the tangential one (y-interfaces swap U and V).
// stage 1: W^n -> F, dF/dt; stage 2: W* -> dF/dt only (into the F arrays); stage 3: W* -> F, dF/dt
// (the stages of a multistage tableau after the first).
// ---------------------------------------------------------------------------------------------
template <typename T, int TN, int TT, int DIM, bool PRFIX, int TFM>
__device__ __attribute__((always_inline)) inline void flux_tile(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts,
                                 const int* __restrict__ off, int nprob, int stage, int b) {
  // rows with halo: two on each side, three when the tangential flag is the indicator on the line values
  // (its widening reaches one row further)
  constexpr int RO = (DIM == 2) ? 2 + TFM : 0;  // halo rows below
  constexpr int R = (DIM == 2) ? TT + 2 * RO : 1;
  constexpr int C = TN + 5;                   // cells along the normal: -3 .. TN+1
  constexpr int NTH = flux_threads(TN, TT, DIM);  // 2D: two threads (Gauss points) per interface
  __shared__ T sW[4][R][C];
  __shared__ uint8_t sF[R][TN + 1];
  constexpr int NRW = nr_row<T, TN>();
  __shared__ T sNR[R * NRW];
  __shared__ uint8_t sTL[TFM ? TT + 2 : 1][TN];  // line-value indicator of rows t0-1 .. t0+TT (bit s: side s)

  const int p = find_prob(off, nprob, b);
  const ProbDev& P = probs[p];
  const TimeDev& tsp = ts[p];
  if (!tsp.active) return;
  const int tid = threadIdx.x;

  // direction and tile of this block: x-interface tiles come first, then y-interface tiles
  const int nxt = (P.nx + 1 + TN - 1) / TN * ((P.ny + TT - 1) / TT);
  int lt = b - off[p];
  const int dir = (DIM == 2 && lt >= nxt) ? 1 : 0;
  if (dir) lt -= nxt;
  const int nn = dir ? P.ny : P.nx, nt = dir ? P.nx : P.ny;
  const int tilesn = (nn + 1 + TN - 1) / TN;
  const int n0 = (lt % tilesn) * TN, t0 = (lt / tilesn) * TT;

  // ---- phase 1: load cells (with ghost synthesis) and flags
  const double* __restrict__ Wsrc = (stage == 1) ? P.W : P.Ws;
  const double tb = (stage == 1) ? tsp.t : tsp.t + tsp.dth;  // the stage's time (prescribed sides)
  // all of a thread's cell loads are issued before the first LDS store (unrolled, fixed trip count)
  constexpr int NL = (R * C + NTH - 1) / NTH;
  double q[NL][4];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = tid + u * NTH;
    if (e < R * C) {
      int r, c;
      if (dir == 0) { r = e / C; c = e % C; }  // consecutive threads along x
      else { c = e / R; r = e % R; }          // consecutive threads along x (= tangential)
      const int n = n0 - 3 + c, t = (DIM == 2) ? t0 - RO + r : 0;
      const bool ok = n >= -4 && n <= nn + 3 && (DIM == 1 || (t >= -4 && t <= nt + 3));
      if (ok) {
        if (dir == 0) load_cell_plain(P, Wsrc, n, t, q[u]);
        else load_cell_plain(P, Wsrc, t, n, q[u]);
      } else {
        q[u][0] = 1.0; q[u][1] = 0.0; q[u][2] = 0.0; q[u][3] = 2.5;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = tid + u * NTH;
    if (e < R * C) {
      int r, c;
      if (dir == 0) { r = e / C; c = e % C; }
      else { c = e / R; r = e % R; }
      if (dir) { const double sw = q[u][1]; q[u][1] = q[u][2]; q[u][2] = sw; }
#pragma unroll
      for (int k = 0; k < 4; ++k) sW[k][r][c] = T(q[u][k]);
    }
  }
  if (P.prescribed) {  // ghosts of prescribed-state sides, by the thread that stored the placeholder
    for (int e = tid; e < R * C; e += NTH) {
      int r, c;
      if (dir == 0) { r = e / C; c = e % C; }
      else { c = e / R; r = e % R; }
      const int n = n0 - 3 + c, t = (DIM == 2) ? t0 - RO + r : 0;
      const int gi = dir ? t : n, gj = dir ? n : t;
      if (n < -4 || n > nn + 3 || (DIM == 2 && (t < -4 || t > nt + 3)) || !prescribed_ghost(P, gi, gj)) continue;
      double g[4];
      load_cell(P, Wsrc, gi, gj, tb, g);
      if (dir) { const double sw = g[1]; g[1] = g[2]; g[2] = sw; }
#pragma unroll
      for (int k = 0; k < 4; ++k) sW[k][r][c] = T(g[k]);
    }
  }
  const int ex = P.nx + 4;
  for (int e = tid; e < R * (TN + 1); e += NTH) {
    const int r = e / (TN + 1), c = e % (TN + 1);
    const int n = n0 - 1 + c, t = (DIM == 2) ? t0 - RO + r : 0;
    const int gi = dir ? t : n, gj = dir ? n : t;
    uint8_t f = 0;
    if (gi >= -2 && gi <= P.nx + 1 && (DIM == 1 || (gj >= -2 && gj <= P.ny + 1))) {
      const uint8_t raw = P.flags[(DIM == 2 ? (size_t)(gj + 2) * ex : 0) + (gi + 2)];
      f = dir ? (uint8_t)(((raw >> 1) & 1) | ((raw & 1) << 1)) : raw;
    }
    sF[r][c] = f;
  }
  __syncthreads();

  // ---- phase 2: normal reconstruction of every row (Sec. 2.3.1; line averages in 2D)
  const T ihn = T(dir ? P.ihy : P.ihx);
  const T gam = T(P.gamma), ghi = T(P.ghi), glo = T(P.glo), eps = T(P.eps);
  for (int e = tid; e < R * TN; e += NTH) {
    const int r = e / TN, k = e % TN;
    // the row's six cells n0+k-3 .. n0+k+2 stay in LDS: component v of cell m at cw[m + v * CS]; the
    // outputs go to sNR as they are formed, so the troubled path holds only its projections
    constexpr int CS = R * C;
    const T* cw = &sW[0][r][k];
    T* dst = sNR + r * NRW + k * kNRS;
    const int fl = sF[r][k] & 1, fr = sF[r][k + 1] & 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T* q = cw + v * CS;
      const T q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5];
      const T sl = (q1 - T(15) * q2 + T(15) * q3 - q4) * (T(1.0 / 12.0) * ihn);
      dst[v] = (T(2) * q0 - T(13) * q1 + T(47) * q2 + T(27) * q3 - T(3) * q4) * T(1.0 / 60.0);
      dst[4 + v] = sl;
      dst[8 + v] = (T(-3) * q1 + T(27) * q2 + T(47) * q3 - T(13) * q4 + T(2) * q5) * T(1.0 / 60.0);
      dst[12 + v] = sl;
    }
    if (fl | fr) {
      Char4<T> m;
      T avg[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) avg[v] = T(0.5) * (cw[2 + v * CS] + cw[3 + v * CS]);
      char4(avg, gam, m);
      T val[4], der[4];
      if (fl) {
        ao_vector<1>(cw, 1, CS, m, 0, ghi, glo, eps, val, der);
#pragma unroll
        for (int v = 0; v < 4; ++v) { dst[v] = val[v]; dst[4 + v] = der[v] * ihn; }
      }
      if (fr) {
        ao_vector<1>(cw + 1, 1, CS, m, 1, ghi, glo, eps, val, der);
#pragma unroll
        for (int v = 0; v < 4; ++v) { dst[8 + v] = val[v]; dst[12 + v] = der[v] * ihn; }
      }
    }
    if (P.positivity) {  // first order where a side's value is not a physical state
      const T* e3 = cw + 3 * CS;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const T w[4] = {dst[8 * sd], dst[8 * sd + 1], dst[8 * sd + 2], dst[8 * sd + 3]};
        if (!admissible(w, gam, stencil_emax(e3[sd], e3[sd + 1], e3[sd + 2], e3[sd + 3], e3[sd + 4]))) {
#pragma unroll
          for (int v = 0; v < 4; ++v) { dst[8 * sd + v] = cw[2 + sd + v * CS]; dst[8 * sd + 4 + v] = T(0); }
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 2b (tangential_flag_mode 1): the hybrid indicator (Steps 1-3) on the line values along the
  // interface, each side and row; phase 3 widens it over the neighbouring rows (Step 4)
  if (DIM == 2 && TFM) {
    const double hts = dir ? P.dx : P.dy;
    const double thr = (P.zeta1_mode == 0) ? 5.0 * hts : 5.0 * hts * hts * hts;
    for (int e = tid; e < (TT + 2) * TN; e += NTH) {
      const int jj = e / TN, kk = e % TN;  // row t0 - 1 + jj: line values of rows jj .. jj + 4 of sNR
      int tl = 0;
      if (P.recon == 1) {
        tl = 3;
      } else if (P.recon == 0) {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double q[5];
#pragma unroll
            for (int r = 0; r < 5; ++r) q[r] = double(sNR[(jj + r) * NRW + kk * kNRS + 8 * sd + c]);
            tl |= troubled5(q[0], q[1], q[2], q[3], q[4], thr) << sd;
          }
      }
      sTL[jj][kk] = (uint8_t)tl;
    }
    __syncthreads();
  }

  // ---- phase 3: tangential reconstruction at the Gauss points, equilibrium state and GKS flux. In 2D
  // lanes 2m and 2m+1 take the two Gauss points of interface m (they read the same LDS rows, which the
  // hardware broadcasts) and add their halves of F and dF/dt with one lane exchange; both lanes of a
  // pair are live or retired together.
  const int m = (DIM == 2) ? (tid >> 1) : tid, gp = (DIM == 2) ? (tid & 1) : 0;
  int k, tt;
  if (dir == 0) { k = m % TN; tt = m / TN; }
  else { tt = m % TT; k = m / TT; }
  const int n = n0 + k, t = t0 + tt;
  if (n > nn || (DIM == 2 && t >= nt)) return;

  FluxParams fp;
  fp.gamma = P.gamma; fp.K = P.K; fp.mu = P.mu; fp.Pr = P.Pr; fp.c1 = P.c1; fp.c2 = P.c2;
  fp.Kp2 = P.Kp2; fp.iKp2 = P.iKp2; fp.kpr = P.kpr;
  fp.dt = tsp.dt; fp.dth = tsp.dth; fp.idt = tsp.idt; fp.idt2 = tsp.idt2;
  fp.ns = P.ns; fp.want_F = (stage != 2);
  T F[4] = {0, 0, 0, 0}, dF[4] = {0, 0, 0, 0};
  if (DIM == 1) {
    T Wl[4], Wxl[4], Wr[4], Wxr[4];
    const T z[4] = {0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wl[v] = sNR[k * kNRS + v]; Wxl[v] = sNR[k * kNRS + 4 + v];
      Wr[v] = sNR[k * kNRS + 8 + v]; Wxr[v] = sNR[k * kNRS + 12 + v];
    }
    gks_flux_gp<PRFIX>(Wl, Wxl, z, Wr, Wxr, z, fp, T(1), F, dF);
  } else {
    const T iht = T(dir ? P.ihx : P.ihy);
    const T K = T(P.K), Kp2 = T(P.Kp2), iKp2 = T(P.iKp2);
    FluxAcc<T> acc;
    T Ws[4], Wxs[4], Wys[4];
    // tangential reconstruction of one side at this Gauss point, then its share of the flux
    // the side's flag along the interface: its cell's flag, or the widened line-value indicator
    const int tl = TFM ? (sTL[TFM ? tt : 0][k] | sTL[TFM ? tt + 1 : 0][k] | sTL[TFM ? tt + 2 : 0][k]) : 0;
    const int ft0 = TFM ? (tl & 1) : ((sF[tt + RO][k] >> 1) & 1);
    const int ft1 = TFM ? ((tl >> 1) & 1) : ((sF[tt + RO][k + 1] >> 1) & 1);
    tangential_side<T, TN, R>(sNR, tt + RO - 2, k, 0, ft0, gp, gam, ghi, glo, eps, iht, P.positivity, P.csm, Ws, Wxs,
                              Wys);
    __builtin_amdgcn_sched_barrier(0);
    flux_side<0, PRFIX>(Ws, Wxs, Wys, gam, K, Kp2, iKp2, acc);
    __builtin_amdgcn_sched_barrier(0);
    tangential_side<T, TN, R>(sNR, tt + RO - 2, k, 1, ft1, gp, gam, ghi, glo, eps, iht, P.positivity, P.csm, Ws, Wxs,
                              Wys);
    __builtin_amdgcn_sched_barrier(0);
    flux_side<1, PRFIX>(Ws, Wxs, Wys, gam, K, Kp2, iKp2, acc);
    __builtin_amdgcn_sched_barrier(0);
    flux_finish<PRFIX>(acc, fp, T(0.5), F, dF);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      F[v] += __shfl_xor(F[v], 1, 64);
      dF[v] += __shfl_xor(dF[v], 1, 64);
    }
  }

  // ---- write F (stages 1 and 3) and dF/dt in the grid's component order. The second stage's dF/dt goes to
  // the F arrays (F^n is spent by then), which keeps the first stage's dF/dt for the time-order fallback.
  T* Fo = reinterpret_cast<T*>(dir ? P.Fy : P.Fx);
  T* Go = reinterpret_cast<T*>(stage != 2 ? (dir ? P.Gy : P.Gx) : (dir ? P.Fy : P.Fx));
  size_t o, plane;
  if (dir == 0) { plane = (size_t)P.ny * (P.nx + 1); o = (size_t)t * (P.nx + 1) + n; }
  else { plane = (size_t)(P.ny + 1) * P.nx; o = (size_t)n * P.nx + t; }
  const int nc = (DIM == 2) ? 4 : 3;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // frame slot -> grid component: y-interfaces swap the momenta back; 1D drops the V slot
    int gc = v;
    if (dir && (v == 1 || v == 2)) gc = 3 - v;
    if (DIM == 1) {
      if (v == 2) continue;
      if (v == 3) gc = 2;
    }
    if (gc >= nc) continue;
    if (stage != 2 && gp == 0) Fo[gc * plane + o] = F[v];
    if (DIM == 1 || gp == 1) Go[gc * plane + o] = dF[v];
  }
}

// One block per tile; tiles are renumbered so that each XCD works on a contiguous range.
template <typename T, int TN, int TT, int DIM, bool PRFIX, int TFM, int WPE>
__global__ void __launch_bounds__(flux_threads(TN, TT, DIM)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_flux(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts, const int* __restrict__ off, int nprob,
       int stage) {
  flux_tile<T, TN, TT, DIM, PRFIX, TFM>(probs, ts, off, nprob, stage, xcd_swizzle(blockIdx.x, gridDim.x));
}

// Persistent form: a grid of co-resident blocks (a multiple of 8) walks the tile list of every problem
// in the batch. Blocks are dealt to the XCDs round-robin, so block b serves XCD b % 8; each XCD takes the
// same contiguous tile range as above and deals it to its blocks cyclically, which spreads the costlier
// tiles along a shock over many blocks. Every block leaves the loop after at most ceil(range / blocks)
// tiles.
template <typename T, int TN, int TT, int DIM, bool PRFIX, int TFM, int WPE>
__global__ void __launch_bounds__(flux_threads(TN, TT, DIM)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_flux_persistent(const ProbDev* __restrict__ probs, const TimeDev* __restrict__ ts, const int* __restrict__ off,
                  int nprob, int stage, int ntiles) {
  const int x = blockIdx.x & 7, li = blockIdx.x >> 3, nloc = gridDim.x >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int begin = x * q + (x < r ? x : r), end = begin + q + (x < r ? 1 : 0);
  for (int b = begin + li; b < end; b += nloc) {
    flux_tile<T, TN, TT, DIM, PRFIX, TFM>(probs, ts, off, nprob, stage, b);
    __syncthreads();  // the tile's LDS is dead before the next tile is staged
  }
}

// ---------------------------------------------------------------------------------------------
// S2O4 stage updates (Sec. 2.2), FP64 state:
//   stage 1: W* = W^n - sum_dir [F(dt/2)_{+} - F(dt/2)_{-}]/h,  F(dt/2) = dt/2 F + dt^2/8 dF/dt
//            S  = W^n - dt sum_dir [(F + dt/6 dF/dt)_{+} - (...)_{-}]/h
//   stage 2: W^{n+1} = S - dt^2/3 sum_dir [dF*/dt_{+} - dF*/dt_{-}]/h, then the CFL quantity of
//            W^{n+1} for the next step.
// ---------------------------------------------------------------------------------------------
// Compensated accumulation: (a + e) + b with a's carried rounding error e, as a rounded value `hi`
// and the new error, which is returned (error-free two-sum, then a fast renormalisation). Contraction
// stays off so that the rounding errors are recovered exactly.
__device__ inline double comp_add(double a, double b, double e, double& hi) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double err = ((a - (s - bb)) + (b - bb)) + e;
  hi = s + err;
  return err - (hi - s);
}

template <typename T>
__global__ void __launch_bounds__(256) k_update(const ProbDev* __restrict__ probs, TimeDev* __restrict__ ts,
                                                const int* __restrict__ off, int nprob, int stage,
                                                double* __restrict__ qpart) {
  // each XCD takes a contiguous range of blocks: a row's y-faces are read by the blocks of the rows on
  // either side, which then share one L2
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int p = find_prob(off, nprob, b);
  const ProbDev& P = probs[p];
  TimeDev& tsp = ts[p];
  if (!tsp.active) return;
  const size_t ncell = (size_t)P.nx * P.ny;
  const size_t cell = (size_t)(b - off[p]) * blockDim.x + threadIdx.x;
  double q = __builtin_inf();
  if (cell < ncell) {
    const int i = (int)(cell % P.nx), j = (int)(cell / P.nx);
    const int nc = P.dim + 2;
    const double dt = tsp.dt;
    const double idx = 1.0 / P.dx, idy = (P.dim == 2) ? 1.0 / P.dy : 0.0;
    const T* Fx = reinterpret_cast<const T*>(P.Fx);
    const T* Fy = reinterpret_cast<const T*>(P.Fy);
    // dF/dt: the first stage's in the G arrays, the second stage's in the F arrays
    const T* Gx = reinterpret_cast<const T*>(stage == 1 ? P.Gx : P.Fx);
    const T* Gy = reinterpret_cast<const T*>(stage == 1 ? P.Gy : P.Fy);
    const size_t px = (size_t)P.ny * (P.nx + 1), py = (size_t)(P.ny + 1) * P.nx;
    const size_t ox = (size_t)j * (P.nx + 1) + i, oy = (size_t)j * P.nx + i;
    double wn[4] = {0, 0, 0, 0};
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) {  // fixed trip count: the components' loads are all in flight together
      if (c >= nc) break;
      const double gx = (double(Gx[c * px + ox + 1]) - double(Gx[c * px + ox])) * idx;
      const double gy = (P.dim == 2) ? (double(Gy[c * py + oy + P.nx]) - double(Gy[c * py + oy])) * idy : 0.0;
      const double w = P.W[c * ncell + cell];
      if (stage == 1) {
        const double fx = (double(Fx[c * px + ox + 1]) - double(Fx[c * px + ox])) * idx;
        const double fy = (P.dim == 2) ? (double(Fy[c * py + oy + P.nx]) - double(Fy[c * py + oy])) * idy : 0.0;
        const double d1 = dt * (0.5 * fx + 0.125 * dt * gx) + dt * (0.5 * fy + 0.125 * dt * gy);
        const double d2 = dt * (fx + dt / 6.0 * gx) + dt * (fy + dt / 6.0 * gy);
        double ws, s;
        if (P.E) {
          const double e = P.E[c * ncell + cell];
          ws = w - (d1 - e);
          P.E2[c * ncell + cell] = comp_add(w, -d2, e, s);
        } else {
          ws = w - d1;
          s = w - d2;
        }
        P.Ws[c * ncell + cell] = ws;
        P.S[c * ncell + cell] = s;
        wn[c == nc - 1 ? 3 : c] = ws;
      } else {
        const double d3 = dt * dt / 3.0 * (gx + gy);
        double wnew;
        if (P.E) P.E2[c * ncell + cell] = comp_add(P.S[c * ncell + cell], -d3, P.E2[c * ncell + cell], wnew);
        else wnew = P.S[c * ncell + cell] - d3;
        P.Ws[c * ncell + cell] = wnew;  // W* is spent: the new state waits there for the commit
        wn[c == nc - 1 ? 3 : c] = wnew;
      }
    }
    const double rho = wn[0];
    const double ke = 0.5 * (wn[1] * wn[1] + wn[2] * wn[2]) / rho;
    const double pr = (P.gamma - 1.0) * (wn[3] - ke);
    bad = !(rho > 0.0) || !(pr > 0.0) || !(wn[3] < __builtin_inf());
    if (bad && P.positivity)  // left to k_repair1 / k_repair: mark the cell (flag bit 2)
      P.flags[(P.dim == 2 ? (size_t)(j + 2) * (P.nx + 4) : 0) + (i + 2)] |= 4;
    else if (bad)
      report_nonphysical(tsp, stage, cell);
    if (stage == 2) q = cfl_quantity(P, wn[0], wn[1], wn[2], wn[3]);
  }
  if (stage == 2) {
    q = block_min(q);
    if (threadIdx.x == 0) qpart[b] = q;
  }
}

// Gas-kinetic flux of two constant states (frame components, no slopes) over [0, dt/2] of the current
// step: dt/2 F + dt^2/8 dF/dt with F, dF/dt from the flux function (Sec. 2.1-2.2), in FP64.
template <bool PRFIX>
__device__ inline void constant_state_half_flux(const ProbDev& P, const TimeDev& tsp, const double Wl[4],
                                                const double Wr[4], double out[4]) {
  FluxParams fp;
  fp.gamma = P.gamma; fp.K = P.K; fp.mu = P.mu; fp.Pr = P.Pr; fp.c1 = P.c1; fp.c2 = P.c2;
  fp.Kp2 = P.Kp2; fp.iKp2 = P.iKp2; fp.kpr = P.kpr;
  fp.dt = tsp.dt; fp.dth = tsp.dth; fp.idt = tsp.idt; fp.idt2 = tsp.idt2;
  fp.ns = P.ns; fp.want_F = true;
  const double z[4] = {0, 0, 0, 0};
  FluxAcc<double> acc;
  flux_side<0, PRFIX>(Wl, z, z, P.gamma, P.K, P.Kp2, P.iKp2, acc);
  flux_side<1, PRFIX>(Wr, z, z, P.gamma, P.K, P.Kp2, P.iKp2, acc);
  double F[4] = {0, 0, 0, 0}, dF[4] = {0, 0, 0, 0};
  flux_finish<PRFIX>(acc, fp, 1.0, F, dF);
  const double dt = tsp.dt;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = dt * (0.5 * F[v] + 0.125 * dt * dF[v]);
}

// First-order fallback of the first stage (problems with positivity = 1): every face next to a cell whose
// intermediate state W* came out non-physical (flag bit 2, set by k_update in stage 1) takes the
// gas-kinetic flux of the two cell averages (constant states, no slopes) over [0, dt/2] in place of the
// reconstructed dt/2 F + dt^2/8 dF/dt; both cells of such a face see the same flux (conservative). Cells
// still non-physical set the problem's status.
template <typename T>
__global__ void __launch_bounds__(256) k_repair1(const ProbDev* __restrict__ probs, TimeDev* __restrict__ ts,
                                                 const int* __restrict__ off, int nprob) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  TimeDev& tsp = ts[p];
  if (!tsp.active || !P.positivity) return;
  const size_t ncell = (size_t)P.nx * P.ny;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  if (cell >= ncell) return;
  const int i = (int)(cell % P.nx), j = (int)(cell / P.nx);
  const int two = P.dim == 2;
  const size_t ex = (size_t)P.nx + 4;
  auto marked = [&](int a, int b) -> int {
    if (a < 0 || a >= P.nx || b < 0 || b >= P.ny) return 0;
    return (P.flags[(two ? (size_t)(b + 2) * ex : 0) + (a + 2)] >> 2) & 1;
  };
  const int m0 = marked(i, j);
  const int mf[4] = {m0 | marked(i - 1, j), m0 | marked(i + 1, j), two ? (m0 | marked(i, j - 1)) : 0,
                     two ? (m0 | marked(i, j + 1)) : 0};  // faces x-low, x-high, y-low, y-high
  if (!(mf[0] | mf[1] | mf[2] | mf[3])) return;
  const int nc = P.dim + 2;
  const double dt = tsp.dt, tb = tsp.t;
  const T* Fx = reinterpret_cast<const T*>(P.Fx);
  const T* Gx = reinterpret_cast<const T*>(P.Gx);
  const T* Fy = reinterpret_cast<const T*>(P.Fy);
  const T* Gy = reinterpret_cast<const T*>(P.Gy);
  const size_t px = (size_t)P.ny * (P.nx + 1), py = (size_t)(P.ny + 1) * P.nx;
  const size_t ox = (size_t)j * (P.nx + 1) + i, oy = (size_t)j * P.nx + i;
  const bool prfix = P.ns && P.Pr != 1.0;
  double dW[4] = {0, 0, 0, 0};  // change of W*, frame slots of the grid components
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if (!mf[f]) continue;
    const int ydir = f >= 2, high = f & 1;
    double a[4], b[4], fo[4];
    if (!ydir) {  // cells i - 1 + high and i + high
      load_cell(P, P.W, i - 1 + high, j, tb, a);
      load_cell(P, P.W, i + high, j, tb, b);
    } else {      // frame of a y-face: the tangential and normal momenta swap
      load_cell(P, P.W, i, j - 1 + high, tb, a);
      load_cell(P, P.W, i, j + high, tb, b);
      double t0 = a[1]; a[1] = a[2]; a[2] = t0;
      t0 = b[1]; b[1] = b[2]; b[2] = t0;
    }
    if (prfix) constant_state_half_flux<true>(P, tsp, a, b, fo);
    else constant_state_half_flux<false>(P, tsp, a, b, fo);
    if (ydir) { const double t0 = fo[1]; fo[1] = fo[2]; fo[2] = t0; }
    const double ih = ydir ? 1.0 / P.dy : 1.0 / P.dx;
    const double sg = high ? -1.0 : 1.0;  // W* = W - (F_high - F_low) / h
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= nc) break;
      const int slot = (c == nc - 1) ? 3 : c;  // grid component -> frame slot (1D has no slot 2)
      const size_t o = ydir ? c * py + oy + (high ? P.nx : 0) : c * px + ox + high;
      const double cur = ydir ? dt * (0.5 * double(Fy[o]) + 0.125 * dt * double(Gy[o]))
                              : dt * (0.5 * double(Fx[o]) + 0.125 * dt * double(Gx[o]));
      dW[slot] += sg * (fo[slot] - cur) * ih;
    }
  }
  double wn[4] = {0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= nc) break;
    const int slot = (c == nc - 1) ? 3 : c;
    const double w = P.Ws[c * ncell + cell] + dW[slot];
    P.Ws[c * ncell + cell] = w;
    wn[slot] = w;
  }
  const double rho = wn[0];
  const double pr = (P.gamma - 1.0) * (wn[3] - 0.5 * (wn[1] * wn[1] + wn[2] * wn[2]) / rho);
  if (!(rho > 0.0) || !(pr > 0.0) || !(wn[3] < __builtin_inf())) report_nonphysical(tsp, 1, cell);
}

// Time-order fallback after the second stage (problems with positivity = 1): every face next to a cell
// that the fourth-order update left non-physical (flag bit 2) takes the one-stage flux F^n + dt/2 dF^n/dt
// instead of the S2O4 flux F^n + dt/6 (dF^n/dt + 2 dF*/dt). The two differ by dt/3 (dF^n/dt - dF*/dt), so
// a cell next to such a face changes by -dt^2/3 times that difference's divergence over its marked faces;
// both neighbours of a face see the same flux, so the update stays conservative. Cells still
// non-physical set the problem's status. The CFL minima of the blocks are recomputed from the final state.
template <typename T>
__global__ void __launch_bounds__(256) k_repair(const ProbDev* __restrict__ probs, TimeDev* __restrict__ ts,
                                                const int* __restrict__ off, int nprob, double* __restrict__ qpart) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  TimeDev& tsp = ts[p];
  if (!tsp.active || !P.positivity) return;
  const size_t ncell = (size_t)P.nx * P.ny;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  double q = __builtin_inf();
  if (cell < ncell) {
    const int i = (int)(cell % P.nx), j = (int)(cell / P.nx);
    const int two = P.dim == 2;
    const size_t ex = (size_t)P.nx + 4;
    auto marked = [&](int a, int b) -> int {
      if (a < 0 || a >= P.nx || b < 0 || b >= P.ny) return 0;
      return (P.flags[(two ? (size_t)(b + 2) * ex : 0) + (a + 2)] >> 2) & 1;
    };
    const int m0 = marked(i, j);
    const int mxl = m0 | marked(i - 1, j), mxr = m0 | marked(i + 1, j);
    const int myl = two ? (m0 | marked(i, j - 1)) : 0, myr = two ? (m0 | marked(i, j + 1)) : 0;
    const int nc = P.dim + 2;
    double wn[4] = {0, 0, 0, 0};
    const double c3 = tsp.dt * tsp.dt / 3.0;
    const double idx = 1.0 / P.dx, idy = two ? 1.0 / P.dy : 0.0;
    const T* Gnx = reinterpret_cast<const T*>(P.Gx);
    const T* Gsx = reinterpret_cast<const T*>(P.Fx);
    const T* Gny = reinterpret_cast<const T*>(P.Gy);
    const T* Gsy = reinterpret_cast<const T*>(P.Fy);
    const size_t px = (size_t)P.ny * (P.nx + 1), py = (size_t)(P.ny + 1) * P.nx;
    const size_t ox = (size_t)j * (P.nx + 1) + i, oy = (size_t)j * P.nx + i;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= nc) break;
      double w = P.Ws[c * ncell + cell];  // the new state, before the commit
      if (mxl | mxr | myl | myr) {
        double d = 0.0;
        if (mxr) d += (double(Gnx[c * px + ox + 1]) - double(Gsx[c * px + ox + 1])) * idx;
        if (mxl) d -= (double(Gnx[c * px + ox]) - double(Gsx[c * px + ox])) * idx;
        if (myr) d += (double(Gny[c * py + oy + P.nx]) - double(Gsy[c * py + oy + P.nx])) * idy;
        if (myl) d -= (double(Gny[c * py + oy]) - double(Gsy[c * py + oy])) * idy;
        w -= c3 * d;
        P.Ws[c * ncell + cell] = w;
      }
      wn[c == nc - 1 ? 3 : c] = w;
    }
    const double rho = wn[0];
    const double pr = (P.gamma - 1.0) * (wn[3] - 0.5 * (wn[1] * wn[1] + wn[2] * wn[2]) / rho);
    if (!(rho > 0.0) || !(pr > 0.0) || !(wn[3] < __builtin_inf())) report_nonphysical(tsp, 2, cell);
    q = cfl_quantity(P, wn[0], wn[1], wn[2], wn[3]);
  }
  q = block_min(q);
  if (threadIdx.x == 0) qpart[blockIdx.x] = q;
}


// ---------------------------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------------------------
static inline unsigned nblk(int n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_cfl(const LaunchCtx& L) {
  if (L.dim == 3)
    launch_cfl3(L);
  else
    hipLaunchKernelGGL(k_cfl, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.off_cell, L.nprob, L.qpart);
}

void launch_dt_finalize(const LaunchCtx& L, int use_tend) {
  hipLaunchKernelGGL(k_dt_finalize, dim3(L.nprob), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell, L.qpart,
                     use_tend);
}

void launch_commit(const LaunchCtx& L, int use_tend) {
  hipLaunchKernelGGL(k_commit, dim3(nblk(L.nprob, 64)), dim3(64), 0, L.stream, const_cast<ProbDev*>(L.probs), L.ts,
                     L.nprob, use_tend);
}

void launch_state_home(const LaunchCtx& L) {
  hipLaunchKernelGGL(k_state_home, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell, L.nprob);
}

void launch_flags(const LaunchCtx& L, int stage_state, int count, int clear) {
  if (clear) hipLaunchKernelGGL(k_clear_counts, dim3(nblk(L.nprob, 64)), dim3(64), 0, L.stream, L.probs, L.nprob);
  if (L.dim == 3)
    launch_flags3(L, stage_state, count);
  else if (L.dim == 2)
    hipLaunchKernelGGL(k_flags2d, dim3(L.ext_blocks), dim3(kFThreads), 0, L.stream, L.probs, L.ts, L.off_ext,
                       L.nprob, stage_state, count);
  else
    hipLaunchKernelGGL(k_flags, dim3(L.ext_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_ext, L.nprob,
                       stage_state, count);
}

// Blocks of a persistent launch: what the occupancy calculator says fits on every CU at once, rounded
// down to a multiple of 8 (one share per XCD), and never more than the tiles.
static int resident_grid(const void* fn, int threads, int ntiles) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 8;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess || per < 1) per = 1;
  int g = cus * per;
  const int cap = (ntiles + 7) & ~7;
  if (g > cap) g = cap;
  g &= ~7;
  return g < 8 ? 8 : g;
}

// stage 0 asks for the persistent grid size of the variant instead of launching (written to *grid)
template <typename T, int TN, int TT, int DIM, bool PR, int TFM, int WPE>
static void flux_launch(const LaunchCtx& L, int stage, int* grid) {
  constexpr int TNd = (DIM == 1) ? TN * TT : TN, TTd = (DIM == 1) ? 1 : TT;
  constexpr int NTH = flux_threads(TNd, TTd, DIM);
  if (stage == 0) {
    *grid = resident_grid(reinterpret_cast<const void*>(k_flux_persistent<T, TNd, TTd, DIM, PR, TFM, WPE>), NTH,
                          L.flux_blocks);
    return;
  }
  if (!L.persistent)
    hipLaunchKernelGGL((k_flux<T, TNd, TTd, DIM, PR, TFM, WPE>), dim3(L.flux_blocks), dim3(NTH), 0, L.stream,
                       L.probs, L.ts, L.off_flux, L.nprob, stage);
  else
    hipLaunchKernelGGL((k_flux_persistent<T, TNd, TTd, DIM, PR, TFM, WPE>), dim3(L.persistent_grid), dim3(NTH), 0,
                       L.stream, L.probs, L.ts, L.off_flux, L.nprob, stage, L.flux_blocks);
}

template <typename T, int TN, int TT, bool PR, int WPE>
static void flux_variant_pr(const LaunchCtx& L, int stage, int* grid) {
  if (L.dim == 1) flux_launch<T, TN, TT, 1, PR, 0, WPE>(L, stage, grid);
  else if (L.tfm) flux_launch<T, TN, TT, 2, PR, 1, WPE>(L, stage, grid);
  else flux_launch<T, TN, TT, 2, PR, 0, WPE>(L, stage, grid);
}

// the Prandtl-number correction is compiled in only for launches that need it (NS with Pr != 1)
template <typename T, int TN, int TT, int WPE>
static void flux_variant(const LaunchCtx& L, int stage, int* grid) {
  if (L.prfix) flux_variant_pr<T, TN, TT, true, WPE>(L, stage, grid);
  else flux_variant_pr<T, TN, TT, false, WPE>(L, stage, grid);
}

// launch configurations: tile shape and the waves-per-SIMD target the register allocator works to
// (1: no target; 2 or 3: spill what does not fit rather than lose occupancy)
const TileShape kTiles[kNumTiles] = {{8, 8, 1}, {8, 8, 2}, {16, 8, 1}, {16, 8, 2}, {16, 8, 3}, {8, 8, 3}};

template <typename T>
static void launch_flux_t(const LaunchCtx& L, int stage, int* grid) {
  switch (L.tile) {
    case 0: flux_variant<T, 8, 8, 1>(L, stage, grid); break;
    case 1: flux_variant<T, 8, 8, 2>(L, stage, grid); break;
    case 2: flux_variant<T, 16, 8, 1>(L, stage, grid); break;
    case 3: flux_variant<T, 16, 8, 2>(L, stage, grid); break;
    case 4: flux_variant<T, 16, 8, 3>(L, stage, grid); break;
    default: flux_variant<T, 8, 8, 3>(L, stage, grid); break;
  }
}

void launch_flux(const LaunchCtx& L, int stage) {
  if (L.dim == 3) {
    launch_flux3(L, stage);
    return;
  }
  if (L.fp32) launch_flux_t<float>(L, stage, nullptr);
  else launch_flux_t<double>(L, stage, nullptr);
}

int flux_persistent_grid(const LaunchCtx& L) {
  if (L.dim == 3) return 0;
  int g = 8;
  if (L.fp32) launch_flux_t<float>(L, 0, &g);
  else launch_flux_t<double>(L, 0, &g);
  return g;
}

void launch_repair1(const LaunchCtx& L) {
  if (L.fp32)
    hipLaunchKernelGGL(k_repair1<float>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob);
  else
    hipLaunchKernelGGL(k_repair1<double>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob);
}

void launch_repair(const LaunchCtx& L) {
  if (L.fp32)
    hipLaunchKernelGGL(k_repair<float>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, L.qpart);
  else
    hipLaunchKernelGGL(k_repair<double>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, L.qpart);
}

void launch_update(const LaunchCtx& L, int stage) {
  if (L.dim == 3) {
    launch_update3(L, stage);
    return;
  }
  if (L.fp32)
    hipLaunchKernelGGL(k_update<float>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, stage, L.qpart);
  else
    hipLaunchKernelGGL(k_update<double>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, stage, L.qpart);
}

}  // namespace hk
