// Launch interface between the host runtime (hgks_capi.cpp) and the kernels (hgks_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "hgks_device.hpp"

namespace hk {

struct TileShape {
  int tn, tt;  // interfaces along the normal, rows along the tangential direction (2D)
  int wpe;     // waves per SIMD the register allocation targets (1: unconstrained)
};
constexpr int kNumTiles = 6;
extern const TileShape kTiles[kNumTiles];

struct LaunchCtx {
  hipStream_t stream;
  const ProbDev* probs;  // device array [nprob]
  TimeDev* ts;           // device array [nprob]
  const int* off_cell;   // prefix sums of 256-cell blocks per problem
  const int* off_ext;    // prefix sums of 256-cell blocks of the extended (flag) range
  const int* off_flux;   // prefix sums of flux tiles (x then y) for the current tile shape
  int nprob, dim, fp32, tile;
  int prfix;             // 1 if any problem is Navier-Stokes with Pr != 1
  int cell_blocks, ext_blocks, flux_blocks;
};

// number of flux tiles of one problem for tile shape `tile`
inline int flux_tiles(int dim, int nx, int ny, int tile) {
  const int tn = kTiles[tile].tn, tt = kTiles[tile].tt;
  if (dim == 1) return (nx + 1 + tn * tt - 1) / (tn * tt);
  return ((nx + 1 + tn - 1) / tn) * ((ny + tt - 1) / tt) + ((ny + 1 + tn - 1) / tn) * ((nx + tt - 1) / tt);
}

void launch_cfl(const LaunchCtx& L);
void launch_dt_finalize(const LaunchCtx& L, int use_tend);
void launch_commit(const LaunchCtx& L, int use_tend);
void launch_flags(const LaunchCtx& L, int stage_state, int count);
void launch_flux(const LaunchCtx& L, int stage);
void launch_update(const LaunchCtx& L, int stage);

}  // namespace hk
