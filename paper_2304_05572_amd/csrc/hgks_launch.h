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
// launch configurations of the flux kernel: tile shape c % kNumTiles, one block per tile (c < kNumTiles)
// or a persistent grid of co-resident blocks walking the tiles (c >= kNumTiles)
constexpr int kNumConfigs = 2 * kNumTiles;

struct LaunchCtx {
  hipStream_t stream;
  const ProbDev* probs;  // device array [nprob]
  TimeDev* ts;           // device array [nprob]
  const int* off_cell;   // prefix sums of 256-cell blocks per problem
  double* qpart;         // CFL minimum of every 256-cell block (cell_blocks entries)
  const int* off_ext;    // prefix sums of flag blocks over the extended range: kFX x kFY tiles (2D) or
                         // 256-cell runs (1D)
  const int* off_flux;   // prefix sums of flux tiles (x then y) for the current tile shape
  int nprob, dim, fp32, tile;
  int persistent;        // 1: persistent flux launch of persistent_grid blocks
  int persistent_grid;
  int prfix;             // 1 if any problem is Navier-Stokes with Pr != 1
  int positivity;        // 1 if any problem asks for the first-order fallbacks
  int tfm;               // tangential flag: 0 the side cell's flag, 1 the indicator on the line values (2D)
  int cell_blocks, ext_blocks, flux_blocks;  // flux_blocks: tiles of all problems
};

// 2D flag tiles: kFX x kFY cells of the extended range [-2, n+1]^2 per block of kFThreads threads
constexpr int kFX = 32, kFY = 32, kFThreads = 256;
inline long flag_tiles2(int nx, int ny) { return (long)((nx + 4 + kFX - 1) / kFX) * ((ny + 4 + kFY - 1) / kFY); }

// number of flux tiles of one problem for tile shape `tile`
inline int flux_tiles(int dim, int nx, int ny, int tile) {
  const int tn = kTiles[tile].tn, tt = kTiles[tile].tt;
  if (dim == 1) return (nx + 1 + tn * tt - 1) / (tn * tt);
  return ((nx + 1 + tn - 1) / tn) * ((ny + tt - 1) / tt) + ((ny + 1 + tn - 1) / tn) * ((nx + tt - 1) / tt);
}

// 3D flux tiles: TN3 faces along the normal x TA3 x TB3 along the two tangential directions, one block
// of 4 threads per face (its 2 x 2 Gauss points)
constexpr int kTN3 = 4, kTA3 = 4, kTB3 = 4;
inline int flux_tiles3(int nx, int ny, int nz) {
  const int N[3] = {nx, ny, nz};
  int t = 0;
  for (int d = 0; d < 3; ++d)
    t += ((N[d] + 1 + kTN3 - 1) / kTN3) * ((N[(d + 1) % 3] + kTA3 - 1) / kTA3) * ((N[(d + 2) % 3] + kTB3 - 1) / kTB3);
  return t;
}

void launch_cfl(const LaunchCtx& L);
void launch_dt_finalize(const LaunchCtx& L, int use_tend);
void launch_commit(const LaunchCtx& L, int use_tend);
// copy a committed state from the second state buffer back into the first (1D / 2D problems)
void launch_state_home(const LaunchCtx& L);
// troubled-cell flags of the current (stage_state 0) or stage (1) state; count: tally the interior
// troubled cells; clear: zero the tallies first (the step's dt finalisation already does)
void launch_flags(const LaunchCtx& L, int stage_state, int count, int clear);
void launch_flux(const LaunchCtx& L, int stage);
int flux_persistent_grid(const LaunchCtx& L);  // blocks of the persistent flux launch for L's variant
void launch_update(const LaunchCtx& L, int stage);
void launch_repair(const LaunchCtx& L);
void launch_repair1(const LaunchCtx& L);  // first-stage fallback (problems with positivity = 1)
// One stage of a two-derivative multistage tableau (stage i of `stages`): its own weights b, bh in the
// new state, the coefficients a, ah of its operators in the next stage's state (n1, nh1) and in the one
// after (n2, nh2, three-stage tableaux after the first stage only).
struct MsStage {
  int i, stages;
  double b, bh, n1, nh1, n2, nh2;
};
void launch_update_ms(const LaunchCtx& L, const MsStage& c);
// the 3D kernels (own source file; the launchers above dispatch to these when L.dim == 3)
void launch_cfl3(const LaunchCtx& L);
void launch_flags3(const LaunchCtx& L, int stage_state, int count);
void launch_flux3(const LaunchCtx& L, int stage);
void launch_update3(const LaunchCtx& L, int stage);

}  // namespace hk
