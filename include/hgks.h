/*
 * hgks.h -- C ABI of the MI355X (gfx950) hot path of the two-stage fourth-order gas-kinetic scheme
 * with hybrid WENO5-AO reconstruction (Mu, Zhuo, Zhang, Liu, Zhong, arXiv 2304.05572).
 *
 * The library advances one or many independent structured-grid problems (1D or 2D, Euler or
 * Navier-Stokes) with:
 *   - the troubled-cell indicator of Sec. 2.3.1 (Steps 1-4), evaluated in FP64 on cell averages;
 *   - linear fifth-order upwind reconstruction (Step 5) or WENO-AO(5,3) in characteristic
 *     variables for values and slopes, normal and tangential (Sec. 2.3.1, 2.3.3);
 *   - the kinetic equilibrium state of Eq. (equ46)-(equ47);
 *   - the gas-kinetic flux of Eq. (equ10) integrated over [0, dt] and [0, dt/2] (Eq. (equ12)),
 *     turned into F and dF/dt (Sec. 2.2);
 *   - the S2O4 time marching of Sec. 2.2 with the collision time and CFL step of Sec. 3.
 *
 * Conventions shared by every entry point:
 *   - State arrays are FP64, structure of arrays, x fastest:
 *       2D: W[c][j][i], c in {rho, rho*U, rho*V, rho*E}, 4*ny*nx doubles
 *       1D: W[c][i],    c in {rho, rho*U, rho*E},        3*nx doubles
 *   - Pointers flagged `on_device` are device addresses on the current HIP device (e.g. from a
 *     torch tensor); otherwise host addresses. The caller owns every buffer it passes; the library
 *     copies in and out and never keeps a caller pointer, except the workspace bound by
 *     hgks_bind_workspace, which it borrows until hgks_destroy and never frees.
 *   - Every call returns an hgks_status. Device-side failures (a non-physical state) are sticky:
 *     they are reported by the next hgks_step / hgks_run / hgks_get_state of that handle. A problem
 *     whose step produces a non-physical state stops there: its state and time stay those of its last
 *     good step (hgks_get_state returns them with HGKS_ENONPHYS), and hgks_get_stats names the stage
 *     and cell where it happened. hgks_set_ic clears the failure.
 *   - A handle is not thread-safe; calls on one handle must not overlap. It lives on the HIP device
 *     current at hgks_create; every later call must be made with that device current.
 *   - Streams: all work of a handle is issued on one stream (opts.hip_stream, or a non-blocking stream
 *     the library creates). Device buffers passed in must be ready on that stream: either the caller
 *     produced them on the same stream, or it synchronised its own stream before the call (the
 *     library's own stream does not wait for other streams). Calls that return data synchronise the
 *     stream before returning, so device buffers filled by the library are ready on return.
 */
#ifndef HGKS_H
#define HGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HGKS_OK = 0,
  HGKS_EINVAL = -1,    /* invalid argument or problem statement */
  HGKS_ENOMEM = -2,    /* device or host allocation failed, or bound workspace too small */
  HGKS_EDEVICE = -3,   /* a HIP runtime call failed */
  HGKS_ENONPHYS = -4,  /* rho <= 0, p <= 0 or NaN appeared in an intermediate or new state */
  HGKS_EDT = -5        /* the time step came out <= 0 or not finite */
} hgks_status;

typedef enum { HGKS_EULER = 0, HGKS_NS = 1 } hgks_eqn;

/* Boundary conditions (Sec. 3): periodic; zero-gradient outflow ("non-reflecting"); reflecting
 * slip wall / symmetry plane (normal momentum negated in the ghost cells); no-slip adiabatic wall
 * (both momenta negated in the ghost cells); prescribed state (hgks_bc_data), for inflow sides and
 * the double Mach reflection of Sec. 3.5 (post-shock state on part of the bottom, the exact moving
 * Mach 10 shock along the top). Ghost cells of the x-sides are synthesised on the interior rows, those
 * of the y-sides across the full padded width, so a corner cell follows the y-side's rule applied to
 * the x-ghost beside it. */
typedef enum {
  HGKS_BC_PERIODIC = 0,
  HGKS_BC_OUTFLOW = 1,
  HGKS_BC_REFLECT = 2,
  HGKS_BC_NOSLIP_ADIABATIC = 3,
  HGKS_BC_PRESCRIBED = 4
} hgks_bc;

/* Data of a HGKS_BC_PRESCRIBED side. A ghost cell of the side whose centre has tangential coordinate
 * tau (y on an x-side, 0 in 1D; x on a y-side) and normal coordinate nu takes the conserved state `a`
 * where tau < s0 + sn * nu + st * t, and beyond that split either the state `b` (rest ==
 * HGKS_BC_PRESCRIBED) or the ghost of the boundary kind `rest` (outflow, reflect or no-slip). t is the
 * time of the stage being evaluated: t_n in the first stage, t_n + dt/2 in the second (the
 * intermediate state of the two-stage step belongs to the half step). States are (rho, rho U, rho V,
 * rho E) and must be physical; 1D problems use a[0], a[1], a[3]. s0 = +infinity makes the side one
 * state. The comparison is evaluated in FP64 without contraction, so that its outcome is reproducible. */
typedef struct {
  double a[4], b[4];
  double s0, sn, st;
  int32_t rest, reserved;
} hgks_bc_data;

/* Reconstruction: the hybrid scheme, or every cell troubled (the WENO5-AO GKS the paper compares
 * against), or no cell troubled (pure linear upwind). */
typedef enum { HGKS_RECON_HYBRID = 0, HGKS_RECON_FORCE_WENOAO = 1, HGKS_RECON_FORCE_LINEAR = 2 } hgks_recon;

/* HGKS_FP64: reconstruction and flux in FP64.
 * HGKS_FP32_BULK: reconstruction and flux arithmetic in FP32; the stored state, the troubled-cell
 * flags, the CFL reduction and the time-integration coefficients of Eq. (equ10) stay FP64. */
typedef enum { HGKS_FP64 = 0, HGKS_FP32_BULK = 1 } hgks_precision;

/* Launch configurations of the fused reconstruction + flux kernel: 6 tile shapes, each launched with
 * one block per tile or as a persistent grid of co-resident blocks. */
#define HGKS_NUM_LAUNCH_CONFIGS 12

/* Time stepping (Sec. 2.2). stages == 0: the paper's two-stage fourth-order S2O4 (the default and the
 * fast path). stages 1..3: a two-derivative multistage tableau, the family Sec. 2.2 places S2O4 in:
 *   W^(i)   = W^n + sum_{j<i} (dt a[i][j] L(W^(j)) + dt^2 ah[i][j] L_t(W^(j)))
 *   W^(n+1) = W^n + sum_i   (dt b[i]    L(W^(i)) + dt^2 bh[i]    L_t(W^(i)))
 * where L and L_t are the negative divergence of the interface flux F and of dF/dt that the gas-kinetic
 * flux of the stage state gives over a window of length dt (Sec. 2.2 steps (1)-(2)). Entries a[i][j],
 * ah[i][j] with j >= i are ignored. Examples: stages 1, b = {1}, bh = {1/2} is the one-stage scheme
 * (the flux integrated over the step, second order in time); stages 2, a[1][0] = 1/2, ah[1][0] = 1/8,
 * b = {1, 0}, bh = {1/6, 1/3} is S2O4 again. Every problem of a handle takes the same stepper; stages
 * >= 1 excludes prescribed-state sides, the positivity fallbacks and compensated accumulation. */
typedef struct {
  int32_t stages;
  int32_t reserved;
  double a[3][3], ah[3][3];
  double b[3], bh[3];
} hgks_stepper;

/* One problem (Sec. 2 statement; parameters of Sec. 3). dim 1, 2 or 3. Three dimensions are the direct
 * extension the paper names: the same hybrid reconstruction along the face normal, then along the two
 * tangential directions in turn to the 2 x 2 Gauss points of each face, and the gas-kinetic flux with three
 * velocity components; states W[c][k][j][i], c in (rho, rho U, rho V, rho W, rho E). 3D problems take the
 * Euler equations or Navier-Stokes with Pr = 1, no prescribed-state sides, no positivity fallbacks and no
 * compensated accumulation. */
typedef struct {
  int32_t dim, nx, ny;          /* dim 1, 2 or 3; ny must be 1 when dim == 1; nx, ny (and nz) >= 5 */
  double x0, x1, y0, y1;        /* uniform Cartesian cells on [x0,x1] x [y0,y1] */
  int32_t eqn;                  /* hgks_eqn: Euler (f = g) or Navier-Stokes (first-order expansion) */
  double gamma, mu, Pr;         /* ratio of specific heats (> 1), dynamic viscosity, Prandtl number */
  double cfl, c1, c2;           /* CFL number; collision time tau = c1 dt + c2 |pl-pr|/(pl+pr) dt
                                   (Euler) or mu/p + c2 |pl-pr|/(pl+pr) dt (NS); c1 = c2 = 0: tau = 0 */
  double fixed_dt;              /* > 0 overrides the CFL time step */
  int32_t bc[4];                /* hgks_bc of x-low, x-high, y-low, y-high; periodic must be paired */
  int32_t recon;                /* hgks_recon */
  double gamma_hi, gamma_lo, weno_eps;  /* WENO-AO linear weights and epsilon (0.85, 0.85, 1e-8) */
  int32_t zeta1_mode;           /* Step-1 threshold: 0 -> 5*h on the normalised quadratic, 1 -> 5*h^3 */
  int32_t tangential_flag_mode; /* flag of the tangential reconstruction (Sec. 2.3.3 Step 2): 0 the side
                                   cell's flag along the interface (default); 1 (2D only) the hybrid
                                   indicator (Steps 1-4) on the line values along the interface. All problems
                                   of a handle take the same mode. */
  int32_t positivity;           /* 0: the scheme as the paper states it. 1: three first-order fallbacks.
                                   A reconstructed state with rho <= 0 or p <= 0 (or not finite) drops to
                                   first order in space: a normal interface value takes its cell's average
                                   with zero normal slope, a Gauss-point value the interface's
                                   centre-segment line values with zero tangential slope. Every face of a
                                   cell whose first-stage state W* is non-physical takes, for W*, the
                                   gas-kinetic flux of the two cell averages (no slopes) over [0, dt/2].
                                   And every face of a cell that the S2O4 update leaves non-physical takes
                                   the one-stage flux
                                   F^n + dt/2 dF^n/dt of the first stage (first order lower in time, still
                                   conservative); a cell still non-physical then is reported. The paper
                                   gives no positivity treatment; its double Mach reflection and blast wave
                                   do not run without one. */
  hgks_bc_data bcd[4];          /* per side, read where bc[side] == HGKS_BC_PRESCRIBED */
  int32_t nz;                   /* dim == 3: cells along z on [z0, z1] (>= 5) and the kinds of the z-low and */
  double z0, z1;                /* z-high sides in bcz (periodic, outflow, reflect or no-slip; bc[0..3] hold  */
  int32_t bcz[2];               /* x and y). Ignored for dim 1 and 2. */
  hgks_stepper stepper;         /* zero-initialised: S2O4 */
  int32_t char_state_mode;      /* 2D: state whose characteristic variables the tangential WENO-AO uses:
                                   0 the reconstructing side's own line value of the centre segment
                                   (default), 1 the mean of both sides' (Sec. 2.3.1's "averaged
                                   conservative variables from both sides" applied along the interface) */
  int32_t viscous_dt_mode;      /* Navier-Stokes time step (Sec. 3): 0 h^2 / (4 nu) with nu = mu / rho
                                   (default), 1 the printed nu = mu / p */
} hgks_problem;

typedef struct {
  int32_t precision;  /* hgks_precision */
  int32_t autotune;   /* 1: time the tile shapes on the first step and keep the fastest (cached on disk
                         under $HGKS_AUTOTUNE_CACHE if set) */
  int32_t use_graph;  /* 1: hgks_run replays one captured HIP graph per step */
  int32_t tile;       /* flux launch configuration when autotune == 0 (-1: library default):
                         c % 6 picks the tile shape, c >= 6 the persistent form */
  int32_t profile;    /* bracket kernel launches of hgks_step / hgks_run (without graphs) with HIP events
                         on the library's stream, read with hgks_get_profile: 1 the reconstruction + flux
                         launches only (two per step), 2 every launch; 0 none */
  int32_t compensated; /* 1: compensated stage accumulation -- a second FP64 array per problem keeps the
                          rounding error of the stored state (error-free two-sum of the S2O4 stage
                          sums of Sec. 2.2), so the state is carried to about twice FP64 precision
                          across steps; the fluxes still read the rounded state. Costs 4 more FP64
                          accesses per conserved variable and step. 0: plain FP64 sums. */
  void* hip_stream;   /* borrowed hipStream_t (NULL: the library's own stream) */
} hgks_opts;

typedef struct hgks hgks_t;

/* Validate the problems and prepare the device-side tables (Sec. 2: the conservation laws of Eq. (equ1)
 * on a structured grid of cell averages, Euler or Navier-Stokes with the gas parameters of Sec. 2.1 and the
 * test parameters of Sec. 3). nprob >= 1 independent problems are advanced together, each with its own
 * time step. Returns HGKS_EINVAL (before any HIP call) for an invalid statement: n < 5, gamma <= 1, CFL
 * and fixed dt both <= 0, Pr <= 0 with Navier-Stokes, unpaired periodic sides, a non-physical prescribed
 * state, mismatched dimensions or tableaux across the batch. *out receives the handle (owned by the caller,
 * released by hgks_destroy). Device memory is allocated at the first hgks_set_ic unless the caller binds a
 * workspace first (see hgks_workspace_bytes). */
hgks_status hgks_create(const hgks_problem* probs, int32_t nprob, const hgks_opts* opts, hgks_t** out);

/* Bytes of device memory the handle needs (states, stage buffers, flags, fluxes, scalars). */
size_t hgks_workspace_bytes(const hgks_t* h);

/* Use caller-owned device memory (>= hgks_workspace_bytes, 256-byte aligned) instead of allocating.
 * Must precede the first hgks_set_ic. */
hgks_status hgks_bind_workspace(hgks_t* h, void* dev_ptr, size_t bytes);

/* Upload the cell averages of problem `prob` ([nc][ny][nx] FP64, host or device as `on_device`
 * says; the unknowns of Eq. (equ1) averaged over each cell, Sec. 2) and set its time to t0; clears the
 * problem's failure status and recomputes the CFL minimum of the handle's problems. W stays the
 * caller's. Synchronises the stream. */
hgks_status hgks_set_ic(hgks_t* h, int32_t prob, const double* W, int32_t on_device, double t0);

/* Advance every problem by one S2O4 step (Sec. 2.2 steps (1)-(4): the flux and its time derivative of
 * the current state, the intermediate state at t + dt/2, the derivative of its flux, the new state) of
 * its own CFL time step (Sec. 3: dt = CFL h / max(|U| + c), and h^2 / (4 nu) for Navier-Stokes) or fixed
 * time step, with no end time. dt_taken: nprob entries (may be NULL). Returns HGKS_ENONPHYS /
 * HGKS_EDT when a problem's step failed (that problem keeps its last good state). Synchronises the
 * stream. */
hgks_status hgks_step(hgks_t* h, double* dt_taken);

/* Advance every problem to its t_end[p] by S2O4 steps (Sec. 2.2) of its CFL time step (Sec. 3), the
 * last step shortened to land on t_end[p], or until max_steps steps have been issued. dt and t stay on
 * the device; the host checks the problems' status every 16 steps, and a problem whose step failed stops
 * at its last good state (HGKS_ENONPHYS / HGKS_EDT). steps_out: nprob entries (may be NULL). */
hgks_status hgks_run(hgks_t* h, const double* t_end, int64_t max_steps, int64_t* steps_out);

/* Copy the state of problem `prob` out; *t receives its time (t may be NULL). */
hgks_status hgks_get_state(const hgks_t* h, int32_t prob, double* W, int32_t on_device, double* t);

/* Low-order part E of the carried state W + E of problem `prob` ([nc][ny][nx], FP64) when the handle
 * was created with opts.compensated == 1; zeros otherwise. Synchronises the stream. */
hgks_status hgks_get_state_lo(const hgks_t* h, int32_t prob, double* E, int32_t on_device);

/* Widened troubled-cell flags (Steps 1-4) of the current state of problem `prob` at its current time,
 * one byte per cell ([ny][nx]); fy is ignored in 1D. */
hgks_status hgks_debug_flags(hgks_t* h, int32_t prob, uint8_t* fx, uint8_t* fy);

/* Interface flux F and its time derivative dF/dt of the current state at its current time for time
 * step dt, as used by the first stage (Sec. 2.2). Host arrays, FP64: Fx, Gx [nc][ny][nx+1]; Fy, Gy [nc][ny+1][nx] (2D). */
/* Three-dimensional forms of the two calls above (dim == 3 only; the 2D forms reject 3D problems):
 * flags [nz][ny][nx] per direction; Fx, Gx [5][nz][ny][nx+1]; Fy, Gy [5][nz][ny+1][nx]; Fz, Gz [5][nz+1][ny][nx]. */
hgks_status hgks_debug_flags3(hgks_t* h, int32_t prob, uint8_t* fx, uint8_t* fy, uint8_t* fz);
hgks_status hgks_debug_stage_fluxes3(hgks_t* h, int32_t prob, double dt, double* Fx, double* Gx, double* Fy,
                                     double* Gy, double* Fz, double* Gz);

hgks_status hgks_debug_stage_fluxes(hgks_t* h, int32_t prob, double dt, double* Fx, double* Gx,
                                    double* Fy, double* Gy);

/* Statistics of problem `prob` (10 entries): out[0] steps taken, out[1] cells, out[2] time, out[3] last dt,
 * out[4] fraction of cells flagged in x at the last flag evaluation, out[5] the same in y, out[6] in z
 * (3D; 0 otherwise), out[7] the stage (1, 2, or the stage of a multistage tableau) of the first
 * non-physical state since hgks_set_ic (0: none), out[8] its cell index (x fastest; the lowest of that
 * stage's non-physical cells; -1: none), out[9] wall seconds the handle has spent in hgks_step and
 * hgks_run (issue to completion, all problems together). Synchronises the stream. */
hgks_status hgks_get_stats(const hgks_t* h, int32_t prob, double* out);

/* Kernel timings gathered since the handle was created (opts.profile > 0), from HIP events recorded
 * on the launching stream. out[2k] = total milliseconds and out[2k+1] = number of launches of kernel
 * group k: 0 fused reconstruction + flux, 1 stage update, 2 troubled-cell flags, 3 scalar kernels
 * (time step, commit). Synchronises the stream. */
hgks_status hgks_get_profile(hgks_t* h, double* out /* 8 entries */);

/* Launch configuration of the reconstruction + flux kernel in use (fixed by opts.tile or chosen by the
 * autotuner): out[0] interfaces per tile along the normal, out[1] rows along the tangential direction,
 * out[2] waves per SIMD the register allocation targets, out[3] the configuration index
 * (0 .. HGKS_NUM_LAUNCH_CONFIGS-1), out[4] the block count of a persistent launch (0: one block per
 * tile, or not launched yet). */
hgks_status hgks_get_tile(const hgks_t* h, int32_t* out /* 5 entries */);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): one step of hgks_step for a single 1D or 2D problem (S2O4, Euler or
 * Navier-Stokes, FP64 or FP32-bulk, the library's default launch configuration) without a handle.
 * W: device pointer to the problem's cell averages ([nc][ny][nx] FP64, as hgks_set_ic takes them) at time
 * t, advanced in place by one step of the problem's own CFL (or fixed) time step; *dt_taken (may be NULL)
 * receives that step. The step's buffers (stage states, fluxes, flags, tables) live in a fixed device
 * array of HGKS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the process
 * ends; the call allocates nothing (no hipMalloc, no host heap) and overwrites that array, so calls that
 * overlap on one GPU (other threads, other streams) race and must be serialised by the caller. Needs
 * 2 * nc * cells * 8 bytes of state plus 4 * nc * (cells + ny or nx) * sizeof(bulk type) of fluxes plus
 * about (nx + 4) (ny + 4) bytes: 2D FP64 up to about 345 000 cells (589^2), FP32-bulk about 518 000 (720^2).
 * Larger problems, 3D problems and multistage tableaux return HGKS_ENOMEM / HGKS_EINVAL before any device
 * work. A step that produces a non-physical state returns HGKS_ENONPHYS and leaves W unchanged.
 * hip_stream: borrowed hipStream_t (NULL: the null stream); W must be ready on it. Synchronises it. */
#define HGKS_NOALLOC_SCRATCH_BYTES (64u << 20)
hgks_status hgks_step_noalloc(const hgks_problem* prob, int32_t precision, double* W, double t, double* dt_taken,
                              void* hip_stream);

void hgks_destroy(hgks_t* h);
const char* hgks_status_str(hgks_status s);

#ifdef __cplusplus
}
#endif
#endif
