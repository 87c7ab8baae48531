// Two-derivative multistage time stepping (Sec. 2.2 casts S2O4 as a two-stage method in the spatial
// operator L and its time derivative L_t and names the multi-stage multi-derivative family): the stage
// update of a tableau, for problems of any dimension. L and L_t of a cell are the negative divergence of
// the interface fluxes F and dF/dt that the flux kernel wrote for the stage state.
//
// Buffers: W holds W^n; S accumulates W^n + sum_i (dt b_i L_i + dt^2 bh_i L_t,i); W* is the next stage's
// state, and the last stage writes W^{n+1} there for the commit to swap in; W2 the partial sum of the
// third stage's state.
#include <hip/hip_runtime.h>

#include "hgks_device.hpp"
#include "hgks_grid.hpp"
#include "hgks_launch.h"

namespace hk {

__device__ inline double cfl_quantity_any(const ProbDev& P, const double* w) {
#pragma clang fp contract(off)
  const int nc = P.dim + 2;
  const double rho = w[0];
  double q2 = 0.0;
  for (int d = 0; d < P.dim; ++d) q2 += (w[1 + d] / rho) * (w[1 + d] / rho);
  const double pr = (P.gamma - 1.0) * (w[nc - 1] - 0.5 * rho * q2);
  const double c = sqrt(P.gamma * pr / rho);
  double q = P.h / (sqrt(q2) + c);
  if (P.ns) q = fmin(q, (P.h * P.h) / (4.0 * (P.mu / (P.vdt ? pr : rho))));
  return q;
}

template <typename T>
__global__ void __launch_bounds__(256) k_update_ms(const ProbDev* __restrict__ probs, TimeDev* __restrict__ ts,
                                                   const int* __restrict__ off, int nprob, MsStage cs,
                                                   double* __restrict__ qpart) {
  const int p = find_prob(off, nprob, blockIdx.x);
  const ProbDev& P = probs[p];
  TimeDev& tsp = ts[p];
  if (!tsp.active) return;
  const int dim = P.dim, nc = dim + 2;
  const int nx = P.nx, ny = dim >= 2 ? P.ny : 1, nz = dim == 3 ? P.nz : 1;
  const size_t ncell = (size_t)nx * ny * nz;
  const size_t cell = (size_t)(blockIdx.x - off[p]) * blockDim.x + threadIdx.x;
  const bool last = cs.i == cs.stages - 1;
  double q = __builtin_inf();
  if (cell < ncell) {
    const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / ((size_t)nx * ny));
    const double dt = tsp.dt, dt2 = dt * dt;
    // faces of the cell: low face index and the stride to the high face, per direction
    const size_t plane[3] = {(size_t)nz * ny * (nx + 1), (size_t)nz * (ny + 1) * nx, (size_t)(nz + 1) * ny * nx};
    const size_t lo[3] = {((size_t)k * ny + j) * (nx + 1) + i, ((size_t)k * (ny + 1) + j) * nx + i,
                          ((size_t)k * ny + j) * nx + i};
    const size_t step[3] = {1, (size_t)nx, (size_t)ny * nx};
    const double ih[3] = {P.ihx, P.ihy, P.ihz};
    const T* F[3] = {reinterpret_cast<const T*>(P.Fx), reinterpret_cast<const T*>(P.Fy),
                     reinterpret_cast<const T*>(P.Fz)};
    const T* G[3] = {reinterpret_cast<const T*>(P.Gx), reinterpret_cast<const T*>(P.Gy),
                     reinterpret_cast<const T*>(P.Gz)};
    double wn[5];
    for (int c = 0; c < nc; ++c) {
      double l = 0.0, lt = 0.0;
      for (int d = 0; d < dim; ++d) {
        const size_t o = c * plane[d] + lo[d];
        l -= (double(F[d][o + step[d]]) - double(F[d][o])) * ih[d];
        lt -= (double(G[d][o + step[d]]) - double(G[d][o])) * ih[d];
      }
      const size_t s = c * ncell + cell;
      const double own = dt * cs.b * l + dt2 * cs.bh * lt;
      double wnew;
      if (cs.i == 0) {
        const double w = P.W[s];
        wnew = w + own;
        if (!last) {
          P.S[s] = wnew;
          wnew = w + (dt * cs.n1 * l + dt2 * cs.nh1 * lt);  // the next stage's state
          P.Ws[s] = wnew;
          if (cs.stages == 3) P.Ws2[s] = w + (dt * cs.n2 * l + dt2 * cs.nh2 * lt);
        } else {
          P.Ws[s] = wnew;  // the new state waits in the stage buffer for the commit
        }
      } else if (!last) {  // the second stage of three
        P.S[s] = P.S[s] + own;
        wnew = P.Ws2[s] + (dt * cs.n1 * l + dt2 * cs.nh1 * lt);
        P.Ws[s] = wnew;
      } else {
        wnew = P.S[s] + own;
        P.Ws[s] = wnew;  // the last stage's state is spent: the new state waits there for the commit
      }
      wn[c] = wnew;
    }
    // the state just completed: the next stage's, or W^{n+1}
    double m2 = 0.0;
    for (int d = 0; d < dim; ++d) m2 += wn[1 + d] * wn[1 + d];
    const double pr = (P.gamma - 1.0) * (wn[nc - 1] - 0.5 * m2 / wn[0]);
    if (!(wn[0] > 0.0) || !(pr > 0.0) || !(wn[nc - 1] < __builtin_inf())) report_nonphysical(tsp, cs.i + 1, cell);
    if (last) q = cfl_quantity_any(P, wn);
  }
  if (last) {
    q = block_min(q);
    if (threadIdx.x == 0) qpart[blockIdx.x] = q;
  }
}

void launch_update_ms(const LaunchCtx& L, const MsStage& c) {
  if (L.fp32)
    hipLaunchKernelGGL(k_update_ms<float>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts, L.off_cell,
                       L.nprob, c, L.qpart);
  else
    hipLaunchKernelGGL(k_update_ms<double>, dim3(L.cell_blocks), dim3(256), 0, L.stream, L.probs, L.ts,
                       L.off_cell, L.nprob, c, L.qpart);
}

}  // namespace hk
