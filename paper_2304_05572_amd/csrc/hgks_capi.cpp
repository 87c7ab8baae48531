// Host runtime and C ABI (include/hgks.h): problem table, device workspace layout, launch sequence of
// one S2O4 step (Sec. 2.2 of Mu et al., arXiv 2304.05572), HIP-graph replay, tile autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hgks.h"
#include "hgks_launch.h"

using namespace hk;

static_assert(kNumConfigs == HGKS_NUM_LAUNCH_CONFIGS, "launch configuration count of the C ABI");

#define HIPOK(x)                                  \
  do {                                            \
    hipError_t e_ = (x);                          \
    if (e_ != hipSuccess) {                       \
      last_hip_error = e_;                        \
      return HGKS_EDEVICE;                        \
    }                                             \
  } while (0)

static thread_local hipError_t last_hip_error = hipSuccess;

struct hgks {
  int nprob = 0, dim = 2, fp32 = 0, use_graph = 0, autotune = 0, compensated = 0;
  hgks_stepper ms{};        // stages 0: S2O4; 1..3: the tableau (the same for every problem)
  int tile = 0, tuned = 0;  // tile: flux launch configuration, 0 .. kNumConfigs-1
  int pgrid[kNumConfigs];   // persistent grid per configuration (0: not yet queried)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<hgks_problem> hp;
  std::vector<ProbDev> pd;
  std::vector<size_t> off_W, off_Ws, off_Ws2, off_S, off_E, off_E2, off_flags, off_Fx, off_Gx, off_Fy, off_Gy, off_Fz,
      off_Gz, off_cnt;
  size_t off_probs = 0, off_ts = 0, off_tab = 0, off_qpart = 0, ws_bytes = 0;
  char* ws = nullptr;
  bool own_ws = false, ready = false;
  std::vector<int> tab_cell, tab_ext, tab_flux[kNumTiles];
  std::vector<char> ic_set;
  hipGraphExec_t graph = nullptr;
  int graph_tile = -1, graph_tend = -1;
  std::vector<double> last_frac_x, last_frac_y, last_frac_z;
  double secs = 0.0;  // wall seconds spent in hgks_step / hgks_run (issue to completion)
  // optional per-launch HIP-event timing
  int profile = 0;
  struct Rec {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> spare;
  double prof_ms[4] = {0, 0, 0, 0};
  long prof_n[4] = {0, 0, 0, 0};
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static size_t cells_of(const hgks_problem& q) { return (size_t)q.nx * q.ny * (q.dim == 3 ? q.nz : 1); }

static hgks_status validate3(const hgks_problem& p) {
  if (p.nx < 5 || p.ny < 5 || p.nz < 5) return HGKS_EINVAL;
  if (!(p.gamma > 1.0) || !(p.x1 > p.x0) || !(p.y1 > p.y0) || !(p.z1 > p.z0)) return HGKS_EINVAL;
  if (!(p.cfl > 0.0) && !(p.fixed_dt > 0.0)) return HGKS_EINVAL;
  if (p.eqn != HGKS_EULER && p.eqn != HGKS_NS) return HGKS_EINVAL;
  if (p.eqn == HGKS_NS && !(p.Pr == 1.0 && p.mu >= 0.0)) return HGKS_EINVAL;  // no Prandtl correction in 3D
  if (p.c1 < 0.0 || p.c2 < 0.0 || p.recon < 0 || p.recon > 2 || p.tangential_flag_mode != 0) return HGKS_EINVAL;
  if (p.positivity != 0 || p.char_state_mode != 0) return HGKS_EINVAL;
  if (p.viscous_dt_mode != 0 && p.viscous_dt_mode != 1) return HGKS_EINVAL;
  if (!(p.gamma_hi > 0.0 && p.gamma_hi < 1.0) || !(p.gamma_lo > 0.0 && p.gamma_lo < 1.0) || !(p.weno_eps > 0.0))
    return HGKS_EINVAL;
  const int k[6] = {p.bc[0], p.bc[1], p.bc[2], p.bc[3], p.bcz[0], p.bcz[1]};
  for (int s = 0; s < 6; ++s)
    if (k[s] < 0 || k[s] > HGKS_BC_NOSLIP_ADIABATIC) return HGKS_EINVAL;
  for (int s = 0; s < 6; s += 2)
    if ((k[s] == HGKS_BC_PERIODIC) != (k[s + 1] == HGKS_BC_PERIODIC)) return HGKS_EINVAL;
  if ((size_t)p.nx * p.ny * p.nz > (size_t)1 << 28) return HGKS_EINVAL;
  return HGKS_OK;
}

// a multistage tableau: 1..3 stages, finite coefficients; not with prescribed-state sides (their stage
// times), the positivity fallbacks (built on S2O4's stages) or compensated accumulation
static hgks_status validate_stepper(const hgks_problem& p) {
  const hgks_stepper& m = p.stepper;
  if (m.stages == 0) return HGKS_OK;
  if (m.stages < 1 || m.stages > 3) return HGKS_EINVAL;
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(m.b[i]) || !std::isfinite(m.bh[i])) return HGKS_EINVAL;
    for (int j = 0; j < 3; ++j)
      if (!std::isfinite(m.a[i][j]) || !std::isfinite(m.ah[i][j])) return HGKS_EINVAL;
  }
  if (p.positivity != 0) return HGKS_EINVAL;
  for (int s = 0; s < 4; ++s)
    if (p.bc[s] == HGKS_BC_PRESCRIBED) return HGKS_EINVAL;
  return HGKS_OK;
}

static bool same_stepper(const hgks_stepper& a, const hgks_stepper& b) {
  if (a.stages != b.stages) return false;
  for (int i = 0; i < 3; ++i) {
    if (a.b[i] != b.b[i] || a.bh[i] != b.bh[i]) return false;
    for (int j = 0; j < i; ++j)
      if (a.a[i][j] != b.a[i][j] || a.ah[i][j] != b.ah[i][j]) return false;
  }
  return true;
}

static hgks_status validate(const hgks_problem& p) {
  if (hgks_status s = validate_stepper(p)) return s;
  if (p.dim == 3) return validate3(p);
  if (p.dim != 1 && p.dim != 2) return HGKS_EINVAL;
  if (p.nx < 5 || (p.dim == 2 && p.ny < 5) || (p.dim == 1 && p.ny != 1)) return HGKS_EINVAL;
  if (!(p.gamma > 1.0) || !(p.x1 > p.x0) || (p.dim == 2 && !(p.y1 > p.y0))) return HGKS_EINVAL;
  if (!(p.cfl > 0.0) && !(p.fixed_dt > 0.0)) return HGKS_EINVAL;
  if (p.eqn != HGKS_EULER && p.eqn != HGKS_NS) return HGKS_EINVAL;
  if (p.eqn == HGKS_NS && !(p.Pr > 0.0 && p.mu >= 0.0)) return HGKS_EINVAL;
  if (p.c1 < 0.0 || p.c2 < 0.0 || p.recon < 0 || p.recon > 2) return HGKS_EINVAL;
  if (p.tangential_flag_mode != 0 && !(p.dim == 2 && p.tangential_flag_mode == 1)) return HGKS_EINVAL;
  if (p.char_state_mode != 0 && !(p.dim == 2 && p.char_state_mode == 1)) return HGKS_EINVAL;
  if (p.viscous_dt_mode != 0 && p.viscous_dt_mode != 1) return HGKS_EINVAL;
  if (p.positivity != 0 && p.positivity != 1) return HGKS_EINVAL;
  if (!(p.gamma_hi > 0.0 && p.gamma_hi < 1.0) || !(p.gamma_lo > 0.0 && p.gamma_lo < 1.0) || !(p.weno_eps > 0.0))
    return HGKS_EINVAL;
  const int nb = p.dim == 2 ? 4 : 2;
  for (int s = 0; s < nb; ++s) {
    if (p.bc[s] < 0 || p.bc[s] > HGKS_BC_PRESCRIBED) return HGKS_EINVAL;
    if (p.bc[s] != HGKS_BC_PRESCRIBED) continue;
    const hgks_bc_data& d = p.bcd[s];
    if (d.rest < HGKS_BC_OUTFLOW || d.rest > HGKS_BC_PRESCRIBED) return HGKS_EINVAL;
    if (std::isnan(d.s0) || !std::isfinite(d.sn) || !std::isfinite(d.st)) return HGKS_EINVAL;
    for (int k = 0; k < (d.rest == HGKS_BC_PRESCRIBED ? 2 : 1); ++k) {
      const double* w = k ? d.b : d.a;
      const double mv = p.dim == 2 ? w[2] : 0.0;
      if (!std::isfinite(w[0]) || !std::isfinite(w[1]) || !std::isfinite(mv) || !std::isfinite(w[3]))
        return HGKS_EINVAL;
      if (!(w[0] > 0.0) || !((p.gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + mv * mv) / w[0]) > 0.0))
        return HGKS_EINVAL;
    }
  }
  for (int s = 0; s < nb; s += 2)
    if ((p.bc[s] == HGKS_BC_PERIODIC) != (p.bc[s + 1] == HGKS_BC_PERIODIC)) return HGKS_EINVAL;
  if ((size_t)p.nx * p.ny > (size_t)1 << 30) return HGKS_EINVAL;
  return HGKS_OK;
}

static void plan(hgks* h) {
  size_t o = 0;
  const size_t ts = h->fp32 ? sizeof(float) : sizeof(double);
  const int np = h->nprob;
  h->off_W.resize(np); h->off_Ws.resize(np); h->off_Ws2.resize(np); h->off_S.resize(np); h->off_E.resize(np);
  h->off_E2.resize(np); h->off_flags.resize(np);
  h->off_Fx.resize(np); h->off_Gx.resize(np); h->off_Fy.resize(np); h->off_Gy.resize(np); h->off_cnt.resize(np);
  h->off_Fz.resize(np); h->off_Gz.resize(np);
  for (int p = 0; p < np; ++p) {
    const hgks_problem& q = h->hp[p];
    const size_t nc = q.dim + 2, nx = q.nx, ny = q.ny, nz = (q.dim == 3) ? q.nz : 1;
    const size_t state = nc * cells_of(q) * sizeof(double);
    h->off_W[p] = o; o = align256(o + state);
    h->off_Ws[p] = o; o = align256(o + state);
    if (h->ms.stages == 3) {
      h->off_Ws2[p] = o; o = align256(o + state);
    } else {
      h->off_Ws2[p] = 0;
    }
    h->off_S[p] = o; o = align256(o + state);
    if (h->compensated) {
      h->off_E[p] = o; o = align256(o + state);
      h->off_E2[p] = o; o = align256(o + state);
    } else {
      h->off_E[p] = h->off_E2[p] = 0;
    }
    h->off_flags[p] = o; o = align256(o + (nx + 4) * (q.dim >= 2 ? ny + 4 : 1) * (q.dim == 3 ? nz + 4 : 1));
    h->off_Fx[p] = o; o = align256(o + nc * nz * ny * (nx + 1) * ts);
    h->off_Gx[p] = o; o = align256(o + nc * nz * ny * (nx + 1) * ts);
    if (q.dim >= 2) {
      h->off_Fy[p] = o; o = align256(o + nc * nz * (ny + 1) * nx * ts);
      h->off_Gy[p] = o; o = align256(o + nc * nz * (ny + 1) * nx * ts);
    } else {
      h->off_Fy[p] = h->off_Gy[p] = 0;
    }
    if (q.dim == 3) {
      h->off_Fz[p] = o; o = align256(o + nc * (nz + 1) * ny * nx * ts);
      h->off_Gz[p] = o; o = align256(o + nc * (nz + 1) * ny * nx * ts);
    } else {
      h->off_Fz[p] = h->off_Gz[p] = 0;
    }
    h->off_cnt[p] = o; o = align256(o + 3 * sizeof(int));
  }
  h->off_probs = o; o = align256(o + np * sizeof(ProbDev));
  h->off_ts = o; o = align256(o + np * sizeof(TimeDev));
  // tables: cell, ext, and one flux table per tile shape, each nprob+1 ints
  h->off_tab = o; o = align256(o + (size_t)(2 + kNumTiles) * (np + 1) * sizeof(int));
  long cell_blocks = 0;
  for (int p = 0; p < np; ++p) cell_blocks += ((long)cells_of(h->hp[p]) + 255) / 256;
  h->off_qpart = o; o = align256(o + (size_t)cell_blocks * sizeof(double));
  h->ws_bytes = o;
  // prefix sums
  h->tab_cell.assign(np + 1, 0);
  h->tab_ext.assign(np + 1, 0);
  for (int t = 0; t < kNumTiles; ++t) h->tab_flux[t].assign(np + 1, 0);
  for (int p = 0; p < np; ++p) {
    const hgks_problem& q = h->hp[p];
    const long cells = (long)cells_of(q);
    const long ext = (long)(q.nx + 4) * (q.dim >= 2 ? q.ny + 4 : 1) * (q.dim == 3 ? q.nz + 4 : 1);
    h->tab_cell[p + 1] = h->tab_cell[p] + (int)((cells + 255) / 256);
    // flag blocks: kFX x kFY tiles of the extended range in 2D, runs of 256 cells in 1D
    const long fblocks = (q.dim == 2) ? flag_tiles2(q.nx, q.ny) : (ext + 255) / 256;
    h->tab_ext[p + 1] = h->tab_ext[p] + (int)fblocks;
    for (int t = 0; t < kNumTiles; ++t)
      h->tab_flux[t][p + 1] =
          h->tab_flux[t][p] + (q.dim == 3 ? flux_tiles3(q.nx, q.ny, q.nz) : flux_tiles(q.dim, q.nx, q.ny, t));
  }
}

static int* tab_ptr(hgks* h, int which) {  // 0 cell, 1 ext, 2+t flux tile t
  return reinterpret_cast<int*>(h->ws + h->off_tab) + (size_t)which * (h->nprob + 1);
}

static LaunchCtx ctx(hgks* h) {
  LaunchCtx L;
  L.stream = h->stream;
  L.probs = reinterpret_cast<const ProbDev*>(h->ws + h->off_probs);
  L.ts = reinterpret_cast<TimeDev*>(h->ws + h->off_ts);
  L.off_cell = tab_ptr(h, 0);
  L.qpart = reinterpret_cast<double*>(h->ws + h->off_qpart);
  L.off_ext = tab_ptr(h, 1);
  const int shape = h->tile % kNumTiles;
  L.off_flux = tab_ptr(h, 2 + shape);
  L.nprob = h->nprob;
  L.dim = h->dim;
  L.fp32 = h->fp32;
  L.tile = shape;
  L.persistent = h->tile >= kNumTiles;
  L.persistent_grid = 0;
  L.prfix = 0;
  for (auto& q : h->hp) L.prfix |= (q.eqn == HGKS_NS && q.Pr != 1.0);
  L.positivity = 0;
  for (auto& q : h->hp) L.positivity |= q.positivity;
  L.tfm = h->hp[0].tangential_flag_mode;
  L.cell_blocks = h->tab_cell[h->nprob];
  L.ext_blocks = h->tab_ext[h->nprob];
  L.flux_blocks = h->tab_flux[shape][h->nprob];
  if (L.persistent) {
    if (h->pgrid[h->tile] <= 0) h->pgrid[h->tile] = flux_persistent_grid(L);
    L.persistent_grid = h->pgrid[h->tile];
  }
  return L;
}

// Device copy of a problem's parameters (buffer pointers are set by the caller).
static void fill_problem(const hgks_problem& q, ProbDev& d) {
  std::memset(&d, 0, sizeof d);
  d.dim = q.dim; d.nx = q.nx; d.ny = q.ny; d.ns = (q.eqn == HGKS_NS);
  for (int s = 0; s < 4; ++s) {
    d.bc[s] = q.bc[s];
    if (q.bc[s] != HGKS_BC_PRESCRIBED || (q.dim == 1 && s >= 2)) continue;
    d.prescribed = 1;
    BcDev& B = d.bcd[s];
    for (int c = 0; c < 4; ++c) {
      B.a[c] = q.bcd[s].a[c];
      B.b[c] = q.bcd[s].b[c];
    }
    if (q.dim == 1) B.a[2] = B.b[2] = 0.0;
    B.s0 = q.bcd[s].s0; B.sn = q.bcd[s].sn; B.st = q.bcd[s].st;
    B.rest = q.bcd[s].rest;
  }
  d.recon = q.recon; d.zeta1_mode = q.zeta1_mode; d.positivity = q.positivity;
  d.csm = q.char_state_mode; d.vdt = q.viscous_dt_mode;
  d.x0 = q.x0; d.y0 = q.dim >= 2 ? q.y0 : 0.0;
  d.nz = q.dim == 3 ? q.nz : 1;
  d.bcz[0] = q.dim == 3 ? q.bcz[0] : 0;
  d.bcz[1] = q.dim == 3 ? q.bcz[1] : 0;
  d.dz = q.dim == 3 ? (q.z1 - q.z0) / q.nz : 1.0;
  d.ihz = 1.0 / d.dz;
  d.dx = (q.x1 - q.x0) / q.nx;
  d.dy = q.dim >= 2 ? (q.y1 - q.y0) / q.ny : 1.0;
  d.h = q.dim == 2 ? std::min(d.dx, d.dy) : q.dim == 3 ? std::min(std::min(d.dx, d.dy), d.dz) : d.dx;
  d.gamma = q.gamma;
  // internal degrees of freedom of the 2D model (K + 2 = 2/(gamma-1)); a 1D problem runs as the 2D
  // model with V = 0, which has the same u-moments as the 1D model with K + 1 = 2/(gamma-1)
  d.K = (4.0 - 2.0 * q.gamma) / (q.gamma - 1.0);
  if (q.dim == 3) d.K = (5.0 - 3.0 * q.gamma) / (q.gamma - 1.0);  // K + 3 = 2/(gamma-1) with three velocities
  d.mu = q.mu; d.Pr = q.Pr; d.c1 = q.c1; d.c2 = q.c2;
  d.Kp2 = d.K + 2.0;
  d.iKp2 = 1.0 / d.Kp2;
  d.kpr = 1.0 / q.Pr - 1.0;
  d.ihx = 1.0 / d.dx;
  d.ihy = 1.0 / d.dy;
  d.cfl = q.cfl; d.fixed_dt = q.fixed_dt;
  d.ghi = q.gamma_hi; d.glo = q.gamma_lo; d.eps = q.weno_eps;
}

static hgks_status materialise(hgks* h) {
  if (h->ready) return HGKS_OK;
  if (!h->ws) {
    void* p = nullptr;
    HIPOK(hipMalloc(&p, h->ws_bytes));
    h->ws = static_cast<char*>(p);
    h->own_ws = true;
  }
  HIPOK(hipMemsetAsync(h->ws, 0, h->ws_bytes, h->stream));
  h->pd.resize(h->nprob);
  for (int p = 0; p < h->nprob; ++p) {
    const hgks_problem& q = h->hp[p];
    ProbDev& d = h->pd[p];
    fill_problem(q, d);
    d.W = reinterpret_cast<double*>(h->ws + h->off_W[p]);
    d.Ws = reinterpret_cast<double*>(h->ws + h->off_Ws[p]);
    d.S = reinterpret_cast<double*>(h->ws + h->off_S[p]);
    d.E = h->compensated ? reinterpret_cast<double*>(h->ws + h->off_E[p]) : nullptr;
    d.E2 = h->compensated ? reinterpret_cast<double*>(h->ws + h->off_E2[p]) : nullptr;
    d.Ws2 = h->ms.stages == 3 ? reinterpret_cast<double*>(h->ws + h->off_Ws2[p]) : nullptr;
    d.flags = reinterpret_cast<uint8_t*>(h->ws + h->off_flags[p]);
    d.Fx = h->ws + h->off_Fx[p];
    d.Gx = h->ws + h->off_Gx[p];
    d.Fy = q.dim >= 2 ? h->ws + h->off_Fy[p] : nullptr;
    d.Gy = q.dim >= 2 ? h->ws + h->off_Gy[p] : nullptr;
    d.Fz = q.dim == 3 ? h->ws + h->off_Fz[p] : nullptr;
    d.Gz = q.dim == 3 ? h->ws + h->off_Gz[p] : nullptr;
    d.flag_count = reinterpret_cast<int*>(h->ws + h->off_cnt[p]);
  }
  HIPOK(hipMemcpyAsync(h->ws + h->off_probs, h->pd.data(), h->nprob * sizeof(ProbDev), hipMemcpyHostToDevice,
                       h->stream));
  std::vector<TimeDev> ts(h->nprob);
  for (auto& s : ts) {
    std::memset(&s, 0, sizeof s);
    s.t_end = INFINITY;
    s.bad = ~0ull;
  }
  HIPOK(hipMemcpyAsync(h->ws + h->off_ts, ts.data(), h->nprob * sizeof(TimeDev), hipMemcpyHostToDevice, h->stream));
  std::vector<int> tabs((size_t)(2 + kNumTiles) * (h->nprob + 1));
  std::copy(h->tab_cell.begin(), h->tab_cell.end(), tabs.begin());
  std::copy(h->tab_ext.begin(), h->tab_ext.end(), tabs.begin() + (h->nprob + 1));
  for (int t = 0; t < kNumTiles; ++t)
    std::copy(h->tab_flux[t].begin(), h->tab_flux[t].end(), tabs.begin() + (size_t)(2 + t) * (h->nprob + 1));
  HIPOK(hipMemcpyAsync(h->ws + h->off_tab, tabs.data(), tabs.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPOK(hipStreamSynchronize(h->stream));
  h->ready = true;
  return HGKS_OK;
}

static hgks_status read_ts(hgks* h, std::vector<TimeDev>& ts) {
  ts.resize(h->nprob);
  HIPOK(hipMemcpyAsync(ts.data(), h->ws + h->off_ts, h->nprob * sizeof(TimeDev), hipMemcpyDeviceToHost, h->stream));
  HIPOK(hipStreamSynchronize(h->stream));
  return HGKS_OK;
}

static hgks_status write_ts(hgks* h, const std::vector<TimeDev>& ts) {
  HIPOK(hipMemcpyAsync(h->ws + h->off_ts, ts.data(), h->nprob * sizeof(TimeDev), hipMemcpyHostToDevice, h->stream));
  HIPOK(hipStreamSynchronize(h->stream));
  return HGKS_OK;
}

// Offsets of the buffers that hold the current state W^n (and, compensated, its low part E) of problem p:
// every committed step swaps the two state buffers (and the two low-part buffers).
static size_t cur_W(const hgks* h, const TimeDev& s, int p) { return s.cur ? h->off_Ws[p] : h->off_W[p]; }
static size_t cur_E(const hgks* h, const TimeDev& s, int p) { return s.cur ? h->off_E2[p] : h->off_E[p]; }

// Restores a saved device time state when a debug entry point returns, on every path (the debug calls
// temporarily change the active flags and dt of the handle's problems).
struct TimeStateRestore {
  hgks* h;
  const std::vector<TimeDev>& saved;
  bool done = false;
  hgks_status restore() {
    done = true;
    return write_ts(h, saved);
  }
  ~TimeStateRestore() {
    if (!done) (void)write_ts(h, saved);
  }
};

static hipEvent_t take_event(hgks* h) {
  if (!h->spare.empty()) {
    hipEvent_t e = h->spare.back();
    h->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch `fn` bracketed by events when profiling (kinds: 0 flux, 1 update, 2 flags, 3 scalar).
template <typename Fn>
static void timed(hgks* h, int kind, bool capturing, Fn fn) {
  if (!h->profile || capturing || (h->profile == 1 && kind != 0)) {
    fn();
    return;
  }
  hgks::Rec r{take_event(h), take_event(h), kind};
  if (r.a) (void)hipEventRecord(r.a, h->stream);
  fn();
  if (r.b) (void)hipEventRecord(r.b, h->stream);
  if (r.a && r.b) h->recs.push_back(r);
}

static void collect_profile(hgks* h) {
  for (auto& r : h->recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      h->prof_ms[r.kind] += ms;
      h->prof_n[r.kind] += 1;
    }
    h->spare.push_back(r.a);
    h->spare.push_back(r.b);
  }
  h->recs.clear();
}

// The two stages of an S2O4 step (Sec. 2.2), each launch passed to wrap(kind, launch) (kinds: 0 flux,
// 1 update, 2 flags): flags, reconstruction + flux and update per stage, the first-order fallbacks where
// a problem asks for them.
template <typename Wrap>
static void s2o4_stages(const LaunchCtx& L, Wrap wrap) {
  wrap(2, [&] { launch_flags(L, 0, 1, 0); });
  wrap(0, [&] { launch_flux(L, 1); });
  wrap(1, [&] { launch_update(L, 1); });
  if (L.positivity) wrap(1, [&] { launch_repair1(L); });
  wrap(2, [&] { launch_flags(L, 1, 0, 0); });
  wrap(0, [&] { launch_flux(L, 2); });
  wrap(1, [&] { launch_update(L, 2); });
  if (L.positivity) wrap(1, [&] { launch_repair(L); });
}

// The launches of one S2O4 step (everything stays on the device: dt, t and the CFL minimum).
static void enqueue_step(hgks* h, int use_tend, bool capturing = false) {
  const LaunchCtx L = ctx(h);
  timed(h, 3, capturing, [&] { launch_dt_finalize(L, use_tend); });
  if (h->ms.stages > 0) {  // a multistage tableau: flags, fluxes (F and dF/dt) and the update per stage
    const hgks_stepper& m = h->ms;
    for (int i = 0; i < m.stages; ++i) {
      MsStage c;
      c.i = i;
      c.stages = m.stages;
      c.b = m.b[i];
      c.bh = m.bh[i];
      c.n1 = i + 1 < m.stages ? m.a[i + 1][i] : 0.0;
      c.nh1 = i + 1 < m.stages ? m.ah[i + 1][i] : 0.0;
      c.n2 = (i == 0 && m.stages == 3) ? m.a[2][0] : 0.0;
      c.nh2 = (i == 0 && m.stages == 3) ? m.ah[2][0] : 0.0;
      timed(h, 2, capturing, [&] { launch_flags(L, i > 0, i == 0, 0); });
      timed(h, 0, capturing, [&] { launch_flux(L, i == 0 ? 1 : 3); });
      timed(h, 1, capturing, [&] { launch_update_ms(L, c); });
    }
    timed(h, 3, capturing, [&] { launch_commit(L, use_tend); });
    if (h->recs.size() > 4096) collect_profile(h);
    return;
  }
  s2o4_stages(L, [&](int kind, auto fn) { timed(h, kind, capturing, fn); });
  timed(h, 3, capturing, [&] { launch_commit(L, use_tend); });
  if (h->recs.size() > 4096) collect_profile(h);
}

static std::string tune_key(hgks* h) {
  std::string k = h->fp32 ? "fp32" : "fp64";
  k += "_d" + std::to_string(h->dim) + "_n" + std::to_string(h->nprob);
  size_t cells = 0;
  for (auto& q : h->hp) cells += (size_t)q.nx * q.ny;
  k += "_c" + std::to_string(cells) + "_x" + std::to_string(h->hp[0].nx) + "_y" + std::to_string(h->hp[0].ny);
  k += "_r" + std::to_string(h->hp[0].recon) + "_e" + std::to_string(h->hp[0].eqn);
  if (h->hp[0].tangential_flag_mode) k += "_t" + std::to_string(h->hp[0].tangential_flag_mode);
  return k;
}

static bool tune_cache_lookup(const std::string& key, int& tile) {
  const char* path = std::getenv("HGKS_AUTOTUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char kbuf[256];
  int t;
  bool found = false;
  while (std::fscanf(f, "%255s %d", kbuf, &t) == 2)
    if (key == kbuf && t >= 0 && t < kNumConfigs) { tile = t; found = true; }
  std::fclose(f);
  return found;
}

static void tune_cache_store(const std::string& key, int tile) {
  const char* path = std::getenv("HGKS_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d\n", key.c_str(), tile);
  std::fclose(f);
}

// Time the first-stage flux kernel of every launch configuration on the current state (dt already set
// by the step's finalize launch) and keep the fastest: after a burst of untimed launches that brings the
// clocks up (the autotuner usually runs first thing in a process), three interleaved rounds of three
// timed launches per configuration after one untimed launch, the best round counting, so that clock
// ramps and noise affect all candidates alike.
static hgks_status autotune(hgks* h) {
  h->tuned = 1;
  const std::string key = tune_key(h);
  int cached;
  if (tune_cache_lookup(key, cached)) {
    h->tile = cached;
    return HGKS_OK;
  }
  hipEvent_t e0, e1;
  HIPOK(hipEventCreate(&e0));
  HIPOK(hipEventCreate(&e1));
  std::vector<float> best(kNumConfigs, 1e30f);
  {
    LaunchCtx L = ctx(h);
    launch_flags(L, 0, 0, 0);
    for (int r = 0; r < 16; ++r) launch_flux(L, 1);
  }
  for (int round = 0; round < 3; ++round) {
    for (int t = 0; t < kNumConfigs; ++t) {
      h->tile = t;
      LaunchCtx L = ctx(h);
      launch_flux(L, 1);  // warm-up
      HIPOK(hipEventRecord(e0, h->stream));
      for (int r = 0; r < 3; ++r) launch_flux(L, 1);
      HIPOK(hipEventRecord(e1, h->stream));
      HIPOK(hipEventSynchronize(e1));
      float ms = 0;
      HIPOK(hipEventElapsedTime(&ms, e0, e1));
      best[t] = std::min(best[t], ms);
    }
  }
  int best_t = 0;
  for (int t = 1; t < kNumConfigs; ++t)
    if (best[t] < best[best_t]) best_t = t;
  h->tile = best_t;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tune_cache_store(key, best_t);
  return HGKS_OK;
}

static hgks_status status_from(const std::vector<TimeDev>& ts) {
  for (auto& s : ts) {
    if (s.status & 1) return HGKS_ENONPHYS;
    if (s.status & 2) return HGKS_EDT;
  }
  return HGKS_OK;
}

static hgks_status build_graph(hgks* h, int use_tend) {
  if (h->graph && h->graph_tile == h->tile && h->graph_tend == use_tend) return HGKS_OK;
  if (h->graph) {
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
  (void)ctx(h);  // queries the persistent grid size (an occupancy call) before the capture starts
  hipGraph_t g;
  HIPOK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  enqueue_step(h, use_tend, true);
  HIPOK(hipStreamEndCapture(h->stream, &g));
  hipError_t e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    last_hip_error = e;
    h->graph = nullptr;
    return HGKS_EDEVICE;
  }
  h->graph_tile = h->tile;
  h->graph_tend = use_tend;
  return HGKS_OK;
}

static hgks_status issue_steps(hgks* h, int use_tend, int64_t nsteps) {
  if (h->autotune && !h->tuned && h->dim != 3) {
    // first step: finalize once so that dt is valid, time the tile shapes on this state, then
    // recompute the CFL minimum the finalize consumed (the state is unchanged) and run the step
    launch_dt_finalize(ctx(h), use_tend);
    hgks_status s = autotune(h);
    if (s) return s;
    launch_cfl(ctx(h));
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    if (h->use_graph) {
      hgks_status s = build_graph(h, use_tend);
      if (s) return s;
      HIPOK(hipGraphLaunch(h->graph, h->stream));
    } else {
      enqueue_step(h, use_tend);
    }
  }
  HIPOK(hipGetLastError());
  return HGKS_OK;
}

// ---------------------------------------------------------------------------------------------
// One step without allocation: every buffer of the step lives in a fixed device array of
// HGKS_NOALLOC_SCRATCH_BYTES. Each device the library runs on holds its own copy of the array (from
// the code object's load until the process ends); host code reaches it only through the address
// hipGetSymbolAddress gives for the device current at the first call there.
// ---------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[HGKS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices];  // the array's device address, per device

static hgks_status scratch_address(void** out) {
  int dev = -1;
  HIPOK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HGKS_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPOK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HGKS_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HGKS_OK;
}

// Byte offsets of the step's buffers inside the scratch array for problem q (total in `bytes`).
struct NoallocPlan {
  size_t probs, ts, tab, qpart, Ws, S, flags, cnt, Fx, Gx, Fy, Gy, bytes;
  int cell_blocks, ext_blocks, flux_blocks;
};

static NoallocPlan plan_noalloc(const hgks_problem& q, int fp32) {
  NoallocPlan n;
  const size_t ts = fp32 ? sizeof(float) : sizeof(double);
  const size_t nc = q.dim + 2, nx = q.nx, ny = q.ny, cells = nx * ny;
  const size_t state = nc * cells * sizeof(double);
  n.cell_blocks = (int)((cells + 255) / 256);
  n.ext_blocks = q.dim == 2 ? (int)flag_tiles2(nx, ny) : (int)((nx + 4 + 255) / 256);
  n.flux_blocks = flux_tiles(q.dim, q.nx, q.ny, 0);
  size_t o = 0;
  n.probs = o; o = align256(o + sizeof(ProbDev));
  n.ts = o; o = align256(o + sizeof(TimeDev));
  n.tab = o; o = align256(o + 6 * sizeof(int));
  n.qpart = o; o = align256(o + (size_t)n.cell_blocks * sizeof(double));
  n.Ws = o; o = align256(o + state);
  n.S = o; o = align256(o + state);
  n.flags = o; o = align256(o + (nx + 4) * (q.dim == 2 ? ny + 4 : 1));
  n.cnt = o; o = align256(o + 3 * sizeof(int));
  n.Fx = o; o = align256(o + nc * ny * (nx + 1) * ts);
  n.Gx = o; o = align256(o + nc * ny * (nx + 1) * ts);
  n.Fy = n.Gy = 0;
  if (q.dim == 2) {
    n.Fy = o; o = align256(o + nc * (ny + 1) * nx * ts);
    n.Gy = o; o = align256(o + nc * (ny + 1) * nx * ts);
  }
  n.bytes = o;
  return n;
}

extern "C" {

hgks_status hgks_step_noalloc(const hgks_problem* prob, int32_t precision, double* W, double t, double* dt_taken,
                              void* hip_stream) {
  if (!prob || !W || !std::isfinite(t) || (precision != HGKS_FP64 && precision != HGKS_FP32_BULK))
    return HGKS_EINVAL;
  const hgks_problem& q = *prob;
  if (hgks_status s = validate(q)) return s;
  if (q.dim == 3 || q.stepper.stages != 0) return HGKS_EINVAL;
  const NoallocPlan n = plan_noalloc(q, precision == HGKS_FP32_BULK);
  if (n.bytes > (size_t)HGKS_NOALLOC_SCRATCH_BYTES) return HGKS_ENOMEM;
  void* base = nullptr;
  if (hgks_status s = scratch_address(&base)) return s;
  char* sc = static_cast<char*>(base);
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);

  ProbDev d;
  fill_problem(q, d);
  d.W = W;  // the caller's state; the step's second state buffer is in the scratch array
  d.Ws = reinterpret_cast<double*>(sc + n.Ws);
  d.S = reinterpret_cast<double*>(sc + n.S);
  d.E = d.E2 = d.Ws2 = nullptr;
  d.flags = reinterpret_cast<uint8_t*>(sc + n.flags);
  d.Fx = sc + n.Fx;
  d.Gx = sc + n.Gx;
  d.Fy = q.dim == 2 ? sc + n.Fy : nullptr;
  d.Gy = q.dim == 2 ? sc + n.Gy : nullptr;
  d.Fz = d.Gz = nullptr;
  d.flag_count = reinterpret_cast<int*>(sc + n.cnt);
  TimeDev ts;
  std::memset(&ts, 0, sizeof ts);
  ts.t = ts.t_new = t;
  ts.t_end = INFINITY;
  ts.active = 1;
  ts.bad = ~0ull;
  const int tabs[6] = {0, n.cell_blocks, 0, n.ext_blocks, 0, n.flux_blocks};
  // every table the kernels read is written here; every other buffer is written by the step before it is
  // read (flags, fluxes, S, the second state, the CFL block minima; the dt finalisation clears the counts)
  HIPOK(hipMemcpyAsync(sc + n.probs, &d, sizeof d, hipMemcpyHostToDevice, stream));
  HIPOK(hipMemcpyAsync(sc + n.ts, &ts, sizeof ts, hipMemcpyHostToDevice, stream));
  HIPOK(hipMemcpyAsync(sc + n.tab, tabs, sizeof tabs, hipMemcpyHostToDevice, stream));

  LaunchCtx L;
  L.stream = stream;
  L.probs = reinterpret_cast<const ProbDev*>(sc + n.probs);
  L.ts = reinterpret_cast<TimeDev*>(sc + n.ts);
  L.off_cell = reinterpret_cast<const int*>(sc + n.tab);
  L.off_ext = reinterpret_cast<const int*>(sc + n.tab) + 2;
  L.off_flux = reinterpret_cast<const int*>(sc + n.tab) + 4;
  L.qpart = reinterpret_cast<double*>(sc + n.qpart);
  L.nprob = 1;
  L.dim = q.dim;
  L.fp32 = precision == HGKS_FP32_BULK;
  L.tile = 0;
  L.persistent = 0;
  L.persistent_grid = 0;
  L.prfix = q.eqn == HGKS_NS && q.Pr != 1.0;
  L.positivity = q.positivity;
  L.tfm = q.tangential_flag_mode;
  L.cell_blocks = n.cell_blocks;
  L.ext_blocks = n.ext_blocks;
  L.flux_blocks = n.flux_blocks;
  launch_cfl(L);
  launch_dt_finalize(L, 0);
  s2o4_stages(L, [](int, auto fn) { fn(); });
  launch_commit(L, 0);
  launch_state_home(L);
  HIPOK(hipGetLastError());
  TimeDev out;
  HIPOK(hipMemcpyAsync(&out, sc + n.ts, sizeof out, hipMemcpyDeviceToHost, stream));
  HIPOK(hipStreamSynchronize(stream));
  if (dt_taken) *dt_taken = out.dt;
  if (out.status & 1) return HGKS_ENONPHYS;
  if (out.status & 2) return HGKS_EDT;
  return HGKS_OK;
}

hgks_status hgks_create(const hgks_problem* probs, int32_t nprob, const hgks_opts* opts, hgks_t** out) {
  if (!probs || nprob < 1 || !out) return HGKS_EINVAL;
  *out = nullptr;
  for (int p = 0; p < nprob; ++p) {
    hgks_status s = validate(probs[p]);
    if (s) return s;
    if (probs[p].dim != probs[0].dim) return HGKS_EINVAL;
    if (!same_stepper(probs[p].stepper, probs[0].stepper)) return HGKS_EINVAL;
    if (probs[p].tangential_flag_mode != probs[0].tangential_flag_mode) return HGKS_EINVAL;
  }
  hgks* h = new (std::nothrow) hgks;
  if (!h) return HGKS_ENOMEM;
  h->nprob = nprob;
  h->dim = probs[0].dim;
  h->hp.assign(probs, probs + nprob);
  h->fp32 = opts ? (opts->precision == HGKS_FP32_BULK) : 0;
  h->use_graph = opts ? opts->use_graph : 0;
  h->autotune = opts ? opts->autotune : 0;
  h->profile = opts ? opts->profile : 0;
  h->tile = (opts && opts->tile >= 0 && opts->tile < kNumConfigs) ? opts->tile : 0;
  h->compensated = opts ? (opts->compensated != 0) : 0;
  h->ms = probs[0].stepper;
  if ((h->dim == 3 || h->ms.stages > 0) && h->compensated) {
    delete h;
    return HGKS_EINVAL;
  }
  for (int c = 0; c < kNumConfigs; ++c) h->pgrid[c] = 0;
  if (opts && (opts->precision < 0 || opts->precision > 1)) {
    delete h;
    return HGKS_EINVAL;
  }
  if (opts && opts->hip_stream) {
    h->stream = static_cast<hipStream_t>(opts->hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return HGKS_EDEVICE;
    }
    h->own_stream = true;
  }
  h->ic_set.assign(nprob, 0);
  h->last_frac_x.assign(nprob, 0.0);
  h->last_frac_y.assign(nprob, 0.0);
  h->last_frac_z.assign(nprob, 0.0);
  plan(h);
  *out = h;
  return HGKS_OK;
}

size_t hgks_workspace_bytes(const hgks_t* h) { return h ? h->ws_bytes : 0; }

hgks_status hgks_bind_workspace(hgks_t* h, void* dev_ptr, size_t bytes) {
  if (!h || !dev_ptr) return HGKS_EINVAL;
  if (h->ready || h->ws) return HGKS_EINVAL;
  if (bytes < h->ws_bytes) return HGKS_ENOMEM;
  if (reinterpret_cast<uintptr_t>(dev_ptr) & 255) return HGKS_EINVAL;
  h->ws = static_cast<char*>(dev_ptr);
  h->own_ws = false;
  return HGKS_OK;
}

hgks_status hgks_set_ic(hgks_t* h, int32_t prob, const double* W, int32_t on_device, double t0) {
  if (!h || !W || prob < 0 || prob >= h->nprob || !std::isfinite(t0)) return HGKS_EINVAL;
  hgks_status s = materialise(h);
  if (s) return s;
  const hgks_problem& q = h->hp[prob];
  const size_t bytes = (size_t)(q.dim + 2) * cells_of(q) * sizeof(double);
  std::vector<TimeDev> ts;
  s = read_ts(h, ts);
  if (s) return s;
  HIPOK(hipMemcpyAsync(h->ws + cur_W(h, ts[prob], prob), W, bytes,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
  if (h->compensated) HIPOK(hipMemsetAsync(h->ws + cur_E(h, ts[prob], prob), 0, bytes, h->stream));
  ts[prob].t = t0;
  ts[prob].t_new = t0;
  ts[prob].t_end = INFINITY;
  ts[prob].active = 1;
  ts[prob].status = 0;
  ts[prob].bad = ~0ull;
  ts[prob].steps = 0;
  set_time_step(ts[prob], 0.0);
  s = write_ts(h, ts);
  if (s) return s;
  h->ic_set[prob] = 1;
  launch_cfl(ctx(h));
  HIPOK(hipGetLastError());
  HIPOK(hipStreamSynchronize(h->stream));
  return HGKS_OK;
}

static hgks_status require_ic(hgks* h) {
  for (int p = 0; p < h->nprob; ++p)
    if (!h->ic_set[p]) return HGKS_EINVAL;
  return h->ready ? HGKS_OK : HGKS_EINVAL;
}

hgks_status hgks_step(hgks_t* h, double* dt_taken) {
  if (!h) return HGKS_EINVAL;
  hgks_status s = require_ic(h);
  if (s) return s;
  std::vector<TimeDev> ts;
  s = read_ts(h, ts);
  if (s) return s;
  s = status_from(ts);
  if (s) return s;
  for (auto& x : ts) {
    x.active = 1;
    x.t_end = INFINITY;
  }
  s = write_ts(h, ts);
  if (s) return s;
  const auto t0 = std::chrono::steady_clock::now();
  s = issue_steps(h, 0, 1);
  if (s) return s;
  s = read_ts(h, ts);
  h->secs += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (s) return s;
  if (dt_taken)
    for (int p = 0; p < h->nprob; ++p) dt_taken[p] = ts[p].dt;
  return status_from(ts);
}

hgks_status hgks_run(hgks_t* h, const double* t_end, int64_t max_steps, int64_t* steps_out) {
  if (!h || !t_end || max_steps < 0) return HGKS_EINVAL;
  hgks_status s = require_ic(h);
  if (s) return s;
  std::vector<TimeDev> ts;
  s = read_ts(h, ts);
  if (s) return s;
  s = status_from(ts);
  if (s) return s;
  std::vector<long long> steps0(h->nprob);
  for (int p = 0; p < h->nprob; ++p) {
    if (std::isnan(t_end[p])) return HGKS_EINVAL;
    ts[p].t_end = t_end[p];
    ts[p].active = ts[p].t < t_end[p] ? 1 : 0;
    steps0[p] = ts[p].steps;
  }
  s = write_ts(h, ts);
  if (s) return s;
  int64_t issued = 0;
  const auto t0 = std::chrono::steady_clock::now();
  struct Clock {  // wall time of the loop, on every path out of it
    hgks* h;
    std::chrono::steady_clock::time_point t0;
    ~Clock() { h->secs += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  } timer{h, t0};
  while (issued < max_steps) {
    bool any = false;
    for (auto& x : ts) any |= (x.active != 0);
    if (!any) break;
    const int64_t chunk = std::min<int64_t>(max_steps - issued, 16);
    s = issue_steps(h, 1, chunk);
    if (s) return s;
    issued += chunk;
    s = read_ts(h, ts);
    if (s) return s;
    s = status_from(ts);
    if (s) return s;
  }
  if (steps_out)
    for (int p = 0; p < h->nprob; ++p) steps_out[p] = ts[p].steps - steps0[p];
  return HGKS_OK;
}

hgks_status hgks_get_state(const hgks_t* hc, int32_t prob, double* W, int32_t on_device, double* t) {
  hgks* h = const_cast<hgks*>(hc);
  if (!h || !W || prob < 0 || prob >= h->nprob || !h->ready) return HGKS_EINVAL;
  const hgks_problem& q = h->hp[prob];
  const size_t bytes = (size_t)(q.dim + 2) * cells_of(q) * sizeof(double);
  std::vector<TimeDev> ts;
  hgks_status s = read_ts(h, ts);
  if (s) return s;
  HIPOK(hipMemcpyAsync(W, h->ws + cur_W(h, ts[prob], prob), bytes,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  HIPOK(hipStreamSynchronize(h->stream));
  if (t) *t = ts[prob].t;
  return status_from(ts);
}

hgks_status hgks_get_state_lo(const hgks_t* hc, int32_t prob, double* E, int32_t on_device) {
  hgks* h = const_cast<hgks*>(hc);
  if (!h || !E || prob < 0 || prob >= h->nprob || !h->ready) return HGKS_EINVAL;
  const hgks_problem& q = h->hp[prob];
  const size_t bytes = (size_t)(q.dim + 2) * cells_of(q) * sizeof(double);
  std::vector<TimeDev> ts;
  hgks_status s = read_ts(h, ts);
  if (s) return s;
  if (h->compensated)
    HIPOK(hipMemcpyAsync(E, h->ws + cur_E(h, ts[prob], prob), bytes,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  else if (on_device)
    HIPOK(hipMemsetAsync(E, 0, bytes, h->stream));
  else
    std::memset(E, 0, bytes);
  HIPOK(hipStreamSynchronize(h->stream));
  return HGKS_OK;
}

static hgks_status debug_flags(hgks_t* h, int32_t prob, uint8_t* fx, uint8_t* fy, uint8_t* fz) {
  if (!h || !fx || prob < 0 || prob >= h->nprob) return HGKS_EINVAL;
  if (!h->ready || !h->ic_set[prob]) return HGKS_EINVAL;
  std::vector<TimeDev> ts, saved;
  hgks_status s = read_ts(h, ts);
  if (s) return s;
  saved = ts;
  TimeStateRestore guard{h, saved};
  for (int p = 0; p < h->nprob; ++p) ts[p].active = (p == prob);
  s = write_ts(h, ts);
  if (s) return s;
  launch_flags(ctx(h), 0, 1, 1);
  HIPOK(hipGetLastError());
  const hgks_problem& q = h->hp[prob];
  const size_t ex = q.nx + 4, ey = q.dim >= 2 ? q.ny + 4 : 1, ez = q.dim == 3 ? q.nz + 4 : 1;
  std::vector<uint8_t> buf(ex * ey * ez);
  HIPOK(hipMemcpyAsync(buf.data(), h->ws + h->off_flags[prob], buf.size(), hipMemcpyDeviceToHost, h->stream));
  int cnt[3];
  HIPOK(hipMemcpyAsync(cnt, h->ws + h->off_cnt[prob], sizeof cnt, hipMemcpyDeviceToHost, h->stream));
  s = guard.restore();  // synchronises the stream: buf and cnt are complete
  if (s) return s;
  const int jo = q.dim >= 2 ? 2 : 0, ko = q.dim == 3 ? 2 : 0, nz = q.dim == 3 ? q.nz : 1;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < q.ny; ++j)
      for (int i = 0; i < q.nx; ++i) {
        const uint8_t v = buf[((size_t)(k + ko) * ey + (j + jo)) * ex + i + 2];
        const size_t o = ((size_t)k * q.ny + j) * q.nx + i;
        fx[o] = v & 1;
        if (fy && q.dim >= 2) fy[o] = (v >> 1) & 1;
        if (fz && q.dim == 3) fz[o] = (v >> 2) & 1;
      }
  const double cells = (double)cells_of(q);
  h->last_frac_x[prob] = cnt[0] / cells;
  h->last_frac_y[prob] = cnt[1] / cells;
  h->last_frac_z[prob] = cnt[2] / cells;
  return HGKS_OK;
}

hgks_status hgks_debug_flags(hgks_t* h, int32_t prob, uint8_t* fx, uint8_t* fy) {
  if (h && prob >= 0 && prob < h->nprob && h->hp[prob].dim == 3) return HGKS_EINVAL;
  return debug_flags(h, prob, fx, fy, nullptr);
}

hgks_status hgks_debug_flags3(hgks_t* h, int32_t prob, uint8_t* fx, uint8_t* fy, uint8_t* fz) {
  if (!h || prob < 0 || prob >= h->nprob || h->hp[prob].dim != 3 || !fy || !fz) return HGKS_EINVAL;
  return debug_flags(h, prob, fx, fy, fz);
}

static hgks_status debug_stage_fluxes(hgks_t* h, int32_t prob, double dt, double* Fx, double* Gx, double* Fy,
                                      double* Gy, double* Fz, double* Gz) {
  if (!h || prob < 0 || prob >= h->nprob || !Fx || !Gx || !(dt > 0.0)) return HGKS_EINVAL;
  if (!h->ready || !h->ic_set[prob]) return HGKS_EINVAL;
  const hgks_problem& q = h->hp[prob];
  if (q.dim >= 2 && (!Fy || !Gy)) return HGKS_EINVAL;
  if (q.dim == 3 && (!Fz || !Gz)) return HGKS_EINVAL;
  std::vector<TimeDev> ts, saved;
  hgks_status s = read_ts(h, ts);
  if (s) return s;
  saved = ts;
  TimeStateRestore guard{h, saved};
  for (int p = 0; p < h->nprob; ++p) {
    ts[p].active = (p == prob);
    set_time_step(ts[p], dt);
  }
  s = write_ts(h, ts);
  if (s) return s;
  LaunchCtx L = ctx(h);
  launch_flags(L, 0, 0, 0);
  launch_flux(L, 1);
  HIPOK(hipGetLastError());
  const size_t nc = q.dim + 2, nx = q.nx, ny = q.ny, nz = q.dim == 3 ? q.nz : 1;
  const size_t nxf = nc * nz * ny * (nx + 1), nyf = q.dim >= 2 ? nc * nz * (ny + 1) * nx : 0;
  const size_t nzf = q.dim == 3 ? nc * (nz + 1) * ny * nx : 0;
  auto fetch = [&](size_t off, size_t n, double* dst) -> hgks_status {
    if (h->fp32) {
      std::vector<float> tmp(n);
      HIPOK(hipMemcpyAsync(tmp.data(), h->ws + off, n * sizeof(float), hipMemcpyDeviceToHost, h->stream));
      HIPOK(hipStreamSynchronize(h->stream));
      for (size_t k = 0; k < n; ++k) dst[k] = tmp[k];
    } else {
      HIPOK(hipMemcpyAsync(dst, h->ws + off, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIPOK(hipStreamSynchronize(h->stream));
    }
    return HGKS_OK;
  };
  if ((s = fetch(h->off_Fx[prob], nxf, Fx))) return s;
  if ((s = fetch(h->off_Gx[prob], nxf, Gx))) return s;
  if (q.dim >= 2) {
    if ((s = fetch(h->off_Fy[prob], nyf, Fy))) return s;
    if ((s = fetch(h->off_Gy[prob], nyf, Gy))) return s;
  }
  if (q.dim == 3) {
    if ((s = fetch(h->off_Fz[prob], nzf, Fz))) return s;
    if ((s = fetch(h->off_Gz[prob], nzf, Gz))) return s;
  }
  return guard.restore();
}

hgks_status hgks_debug_stage_fluxes(hgks_t* h, int32_t prob, double dt, double* Fx, double* Gx, double* Fy,
                                    double* Gy) {
  if (h && prob >= 0 && prob < h->nprob && h->hp[prob].dim == 3) return HGKS_EINVAL;
  return debug_stage_fluxes(h, prob, dt, Fx, Gx, Fy, Gy, nullptr, nullptr);
}

hgks_status hgks_debug_stage_fluxes3(hgks_t* h, int32_t prob, double dt, double* Fx, double* Gx, double* Fy,
                                     double* Gy, double* Fz, double* Gz) {
  if (!h || prob < 0 || prob >= h->nprob || h->hp[prob].dim != 3) return HGKS_EINVAL;
  return debug_stage_fluxes(h, prob, dt, Fx, Gx, Fy, Gy, Fz, Gz);
}

hgks_status hgks_get_stats(const hgks_t* hc, int32_t prob, double* out) {
  hgks* h = const_cast<hgks*>(hc);
  if (!h || !out || prob < 0 || prob >= h->nprob || !h->ready) return HGKS_EINVAL;
  std::vector<TimeDev> ts;
  hgks_status s = read_ts(h, ts);
  if (s) return s;
  int cnt[3];
  HIPOK(hipMemcpyAsync(cnt, h->ws + h->off_cnt[prob], sizeof cnt, hipMemcpyDeviceToHost, h->stream));
  HIPOK(hipStreamSynchronize(h->stream));
  const hgks_problem& q = h->hp[prob];
  const double cells = (double)cells_of(q);
  const TimeDev& st = ts[prob];
  out[0] = (double)st.steps;
  out[1] = cells;
  out[2] = st.t;
  out[3] = st.dt;
  out[4] = cnt[0] / cells;
  out[5] = cnt[1] / cells;
  out[6] = cnt[2] / cells;
  out[7] = st.bad == ~0ull ? 0.0 : (double)(st.bad >> 32);
  out[8] = st.bad == ~0ull ? -1.0 : (double)(st.bad & 0xffffffffull);
  out[9] = h->secs;
  return HGKS_OK;
}

hgks_status hgks_get_profile(hgks_t* h, double* out) {
  if (!h || !out) return HGKS_EINVAL;
  if (h->stream) HIPOK(hipStreamSynchronize(h->stream));
  collect_profile(h);
  for (int k = 0; k < 4; ++k) {
    out[2 * k] = h->prof_ms[k];
    out[2 * k + 1] = (double)h->prof_n[k];
  }
  return HGKS_OK;
}

hgks_status hgks_get_tile(const hgks_t* h, int32_t* out) {
  if (!h || !out) return HGKS_EINVAL;
  const TileShape& ts = kTiles[h->tile % kNumTiles];
  out[0] = ts.tn;
  out[1] = ts.tt;
  out[2] = ts.wpe;
  out[3] = h->tile;
  out[4] = h->tile >= kNumTiles ? h->pgrid[h->tile] : 0;
  return HGKS_OK;
}

void hgks_destroy(hgks_t* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  collect_profile(h);
  for (auto e : h->spare) (void)hipEventDestroy(e);
  if (h->own_ws && h->ws) (void)hipFree(h->ws);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

const char* hgks_status_str(hgks_status s) {
  switch (s) {
    case HGKS_OK: return "ok";
    case HGKS_EINVAL: return "invalid argument";
    case HGKS_ENOMEM: return "out of memory or workspace too small";
    case HGKS_EDEVICE: return "HIP runtime error";
    case HGKS_ENONPHYS: return "non-physical state (rho <= 0, p <= 0 or NaN)";
    case HGKS_EDT: return "time step <= 0 or not finite";
  }
  return "unknown status";
}

}  // extern "C"
