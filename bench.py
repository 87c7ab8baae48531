#!/usr/bin/env python3
"""Throughput of the hybrid WENO5-AO gas-kinetic scheme (S2O4 steps) on one MI355X.

Workload: 2D four-quadrant Riemann problem, Euler, 1024 x 1024 cells, quadrant states drawn from a seed
(rho in [0.1, 1.5], p in [0.03, 1.5], |u|, |v| <= 1.2, one elementary wave per edge), hybrid WENO5-AO,
CFL 0.5, c1 = 0.01, c2 = 1, outflow boundaries. One step = one full two-stage fourth-order step of every
cell (flags, fused reconstruction + gas-kinetic flux, stage update, for both stages, plus the CFL
reduction), inputs resident in device memory.

`value` is the plain FP64 path in Mcell-updates/s, timed over K steps issued eagerly with HIP events
around the flux launches only. The same line carries: the FP32-bulk path on the same workload; FP32-bulk
with compensated state; (with --variants ...,wenoao) forced WENO5-AO against the hybrid scheme; the batched
path (64 uneven problems in one set of launches; eager, one HIP graph per step, and the persistent launch
form); the viscous shock tube (Navier-Stokes, 1000 x 500, 10 steps); the three-dimensional scheme on an
eight-octant Riemann problem (FP64 and FP32-bulk); per-kernel-group times and graph-replay step times from
short side windows; the rate with host transfers included; the L1/Linf distance of the first step of each
precision to the CPU oracle over the full grid; the roofline position of the dominant kernel (fused
reconstruction + flux, VALU-bound) for FP64, FP32-bulk and the batch: the method's algorithmic operations
(tests/opcount.py counts them per Gauss point and per troubled side; the flagged fractions of the run
give the troubled sides) over the HIP-event mean launch time in the timed region, and algorithmic HBM
bytes against 8 TB/s, with the executed operations and counted HBM bytes of the committed counter summary
when it matches the sources; and the oracle's own CPU throughput on a bounded sample (one thread and all
host cores, median of 5).

Other modes: --tile-sweep times every flux launch configuration; --copy-calibration runs a plain copy for
scaling the HBM byte counters.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s, 2D Euler 1024^2: FP64 plain vs FP32 vs batched, L1 err vs oracle"
PEAK_FP64_VALU = 78.6  # TFLOP/s, MI355X vector FP64 (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X vector FP32 (published, packed; the kernels issue non-packed FP32)
PEAK_HBM = 8000.0  # GB/s
# Algorithmic operations of the method (tests/opcount.py: its formulas evaluated on a counting scalar
# type, +, -, *, / one each, a fused multiply-add two; checked against the oracle's fluxes and against
# these constants by tests/test_opcount.py):
#   per Gauss point of the linear path: the gas-kinetic flux from the two reconstructed sides (2182), the
#   tangential reconstruction of both sides (2 x 148: values, tangential slopes, normal-slope values) and
#   half of an interface row's normal reconstruction (132 / 2; a row serves its segment's two points);
#   per troubled side, what WENO-AO in characteristic variables adds: 842 per normal side-row, 1645 per
#   tangential side and Gauss point.
ALG_FLOPS_PER_GP_LINEAR = 2544.0
ALG_FLOPS_AO_NORMAL_SIDE = 842
ALG_FLOPS_AO_TANGENTIAL_SIDE = 1645


def alg_flops_per_launch(gps, flagged_cells_x, flagged_cells_y):
    """Algorithmic operations of one 2D flux launch: every Gauss point on the linear path, plus WENO-AO
    where a side is troubled. A cell flagged in x is the troubled side of the normal reconstruction of
    two x-interfaces (one row each) and of the tangential reconstruction of two y-interfaces (two Gauss
    points each); the same with x and y exchanged."""
    nf = flagged_cells_x + flagged_cells_y
    return gps * ALG_FLOPS_PER_GP_LINEAR + nf * (2 * ALG_FLOPS_AO_NORMAL_SIDE + 4 * ALG_FLOPS_AO_TANGENTIAL_SIDE)


def alg_bytes_per_launch(cells, interfaces, fp32):
    """Algorithmic HBM bytes of one flux launch, mean of the two stages: the state read once (4 x 8 B per
    cell), the flags (1 B per cell), F and dF/dt written in stage 1 (2 x 4 values per interface), dF/dt
    only in stage 2."""
    v = 4 if fp32 else 8
    return cells * (32 + 1) + interfaces * 4 * v * 1.5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in ("hgks_kernels.hip", "hgks_device.hpp", "hgks_grid.hpp"):
        with open(os.path.join(ROOT, "paper_2304_05572_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel3_hash():
    h = hashlib.sha256()
    for f in ("hgks_kernels3.hip", "hgks_device3.hpp", "hgks_device.hpp", "hgks_grid.hpp"):
        with open(os.path.join(ROOT, "paper_2304_05572_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_profile_table(name):
    """key value pairs of a committed profile summary (profiles/<name>), or {}."""
    path = os.path.join(ROOT, "profiles", name)
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        line = line.split("#")[0].strip()
        if line.startswith("@"):
            k, _, v = line[1:].partition(" ")
            out[k.strip()] = v.strip()
    return out


def rp_problem(H, n, recon=0):
    return H.Problem(dim=2, nx=n, ny=n, bc=(H.BC_OUTFLOW,) * 4, cfl=0.5, c1=0.01, c2=1.0, recon=recon)


def launch_config(tile):
    return {"tile": list(tile[:2]), "waves_per_simd_target": tile[2], "index": tile[3],
            "persistent_blocks": tile[4] if tile[4] else None}


def time_solver(H, problems, states, precision, steps, warmup, tile, compensated=False, repeats=0, out=None):
    """Seconds of exactly `steps` steps after `warmup` untimed ones, the flux kernel's mean launch time and
    the handle's stats; with `repeats`, the same window (initial data, `warmup` untimed steps, `steps` timed
    ones) is run that many more times on the same handle and launch configuration, its seconds going to
    out["repeat_seconds"] (the reported window is the first)."""
    import torch
    s = H.Solver(problems, precision=precision, tile=tile, profile=1, autotune=(tile < 0), compensated=compensated)
    for p, W in enumerate(states):
        s.set_ic(p, W)
    s.run(np.inf, warmup)
    torch.cuda.synchronize()
    prof0 = s.profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(np.inf, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof1 = s.profile()
    flux_ms = prof1["flux"][0] - prof0["flux"][0]
    flux_n = prof1["flux"][1] - prof0["flux"][1]
    stats = [s.stats(p) for p in range(len(problems))]
    tile_used = s.tile()
    prof = {k: (prof1[k][0] - prof0[k][0], prof1[k][1] - prof0[k][1]) for k in prof1}
    if repeats and out is not None:
        secs = []
        for _ in range(repeats):
            for p, W in enumerate(states):
                s.set_ic(p, W)
            s.run(np.inf, warmup)
            torch.cuda.synchronize()
            a = time.perf_counter()
            s.run(np.inf, steps)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - a)
        out["repeat_seconds"] = secs
    s.close()
    return t1 - t0, flux_ms / max(flux_n, 1), stats, tile_used, prof


def side_windows(H, problems, states, precision, tile, compensated=False, steps=10):
    """Two short windows beside the timed one, with the launch configuration it used: every kernel group
    timed with events (ms per step per group), and the same steps replayed as one HIP graph per step with
    no events (ms per step)."""
    import torch
    out = {}
    for mode in ("groups", "graph"):
        s = H.Solver(problems, precision=precision, tile=tile, compensated=compensated,
                     profile=2 if mode == "groups" else 0, use_graph=(mode == "graph"))
        for p, W in enumerate(states):
            s.set_ic(p, W)
        s.run(np.inf, 2)
        torch.cuda.synchronize()
        p0 = s.profile()
        t0 = time.perf_counter()
        s.run(np.inf, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if mode == "groups":
            p1 = s.profile()
            out["kernel_ms_per_step"] = {k: (p1[k][0] - p0[k][0]) / steps for k in p1}
        else:
            out["graph_ms_per_step"] = el / steps * 1e3
        s.close()
    return out


def host_io(H, problems, states, precision, tile, steps):
    """The same steps with the state handed over in host memory: upload (hgks_set_ic from a host array),
    the steps, download (hgks_get_state into a host array); returns ms of each part."""
    import torch
    s = H.Solver(problems, precision=precision, tile=tile)
    s.set_ic(0, states[0])
    s.run(np.inf, 1)  # first-launch costs out of the way
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, W in enumerate(states):
        s.set_ic(p, W)
    t1 = time.perf_counter()
    s.run(np.inf, steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for p in range(len(states)):
        s.get_state(p)
    t3 = time.perf_counter()
    s.close()
    return {"upload_ms": (t1 - t0) * 1e3, "steps_ms": (t2 - t1) * 1e3, "download_ms": (t3 - t2) * 1e3}


def gpu_first_step(H, W0, n, precision):
    """State after one S2O4 step from the initial data, and the step's dt."""
    s = H.Solver(rp_problem(H, n), precision=precision)
    s.set_ic(0, W0)
    dt = s.step()[0]
    W, _ = s.get_state(0)
    s.close()
    return W, dt


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_leg(W0, n, crop=256, reps=5):
    """The oracle as it stands, on host cores. cpu_baseline: one S2O4 step of a crop x crop window of the
    workload's initial data around the quadrant junction (outflow sides), median of `reps` runs on one thread
    and on every host core up to 16. Parity: one step of the full n x n grid (all threads). Returns (full
    state, dt, cpu_baseline record)."""
    import oracle
    nth = min(16, os.cpu_count() or 1)
    c0 = (n - crop) // 2
    Wc = np.ascontiguousarray(W0[:, c0:c0 + crop, c0:c0 + crop])
    Pc = oracle.Problem(dim=2, nx=crop, ny=crop, bc=(1, 1, 1, 1), c1=0.01, c2=1.0, cfl=0.5)
    med = {}
    for k in (1, nth):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.step(Pc, Wc, 0.0, nthreads=k)
            ts.append(time.perf_counter() - t0)
        med[k] = float(np.median(ts))
    rec = {"value": crop * crop / med[nth] / 1e6, "unit": "Mcell-updates/s", "cores": nth, "kind": "oracle",
           "sample": f"one S2O4 step of the central {crop}x{crop} window of the {n}x{n} initial data (outflow "
                     f"sides), FP64 C oracle (gcc -O2, OpenMP over rows), median of {reps} runs",
           "single_thread": {"value": crop * crop / med[1] / 1e6, "seconds_median": med[1], "threads": 1},
           "all_cores": {"value": crop * crop / med[nth] / 1e6, "seconds_median": med[nth], "threads": nth},
           "nproc": os.cpu_count(), "cpu_model": cpu_model()}
    Po = oracle.Problem(dim=2, nx=n, ny=n, bc=(1, 1, 1, 1), c1=0.01, c2=1.0, cfl=0.5)
    W, t, dt = oracle.step(Po, W0, 0.0, nthreads=nth)
    return W, dt, rec


def octant_problem(H, n, recon=0):
    return H.Problem(dim=3, nx=n, ny=n, nz=n, bc=(H.BC_OUTFLOW,) * 4, bcz=(H.BC_OUTFLOW,) * 2, cfl=0.5, c1=0.01,
                     c2=1.0, recon=recon)


def time_3d(H, wl, n, seed, steps, warmup):
    """The three-dimensional scheme on a seeded eight-octant Riemann problem, n^3 cells, FP64 and FP32-bulk:
    Mcell-updates/s over eagerly issued steps and the flux kernel's HIP-event mean launch time."""
    W0 = wl.octants_3d(n, n, n, seed=seed)
    out = {"workload": f"3D eight-octant Riemann problem, Euler, {n}^3 cells, seeded octant states (seed {seed}), "
                       "hybrid WENO5-AO GKS, 2 x 2 Gauss points per face, S2O4, CFL 0.5, outflow"}
    for name, prec in (("fp64", H.FP64), ("fp32_bulk", H.FP32_BULK)):
        log(f"[bench] timing 3d {name}: {n}^3, {warmup} warm-up + {steps} steps")
        el, flux_ms, stats, _, prof = time_solver(H, [octant_problem(H, n)], [W0], prec, steps, warmup, 0)
        gps = 4 * 3 * (n + 1) * n * n
        out[name] = {"value": n ** 3 * steps / el / 1e6, "ms_per_step": el / steps * 1e3,
                     "flux_ms_per_launch": flux_ms, "gauss_points_per_launch": gps,
                     "kernel": "k_flux3<%s>" % ("double" if prec == H.FP64 else "float"),
                     "flagged_x": stats[0]["flagged_x"], "flagged_y": stats[0]["flagged_y"]}
        log(f"[bench] 3d {name}: {out[name]['value']:.1f} Mcell-updates/s, flux {flux_ms:.3f} ms/launch")
    # roofline of the FP64 kernel: FP64 operations per Gauss point from the committed counter summary of the
    # 128^3 problem (valid for its sources; the troubled fraction of other sizes differs)
    t3 = read_profile_table("k_flux3_traffic_oct128_fp64.txt")
    r = out["fp64"]
    if t3.get("kernel3_hash") == kernel3_hash() and int(t3.get("n", 0)) == n and r["flux_ms_per_launch"] > 0:
        fl = float(t3["flops_per_gauss_point"])
        ach = fl * r["gauss_points_per_launch"] / (r["flux_ms_per_launch"] * 1e-3) / 1e12
        r["roofline"] = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                         "frac": ach / PEAK_FP64_VALU, "traffic": float(t3["bytes_per_launch"]),
                         "flops_per_gauss_point": fl, "traffic_unit": "bytes per launch"}
    return out


def vst_problem(H, nx, ny, Pr=0.73):
    from paper_2304_05572_amd import workloads as wl
    W0 = wl.viscous_shock_tube(nx, ny)
    P = H.Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=0.5, eqn=H.NS, mu=1.0 / 200.0, Pr=Pr,
                  cfl=0.3, c1=0.01, c2=1.0, bc=(H.BC_NOSLIP, H.BC_NOSLIP, H.BC_NOSLIP, H.BC_REFLECT))
    return P, W0


def time_vst(H, steps, warmup):
    """The viscous shock tube (Navier-Stokes, Re = 200, Pr = 0.73, 1000 x 500 cells), FP64 and FP32-bulk: steps
    from the initial data issued eagerly, the flux kernel's HIP-event mean."""
    P, W0 = vst_problem(H, 1000, 500)
    out = {"workload": "viscous shock tube, Navier-Stokes, Re 200, Pr 0.73, [0,1]x[0,0.5], 1000x500 cells, "
                       "no-slip adiabatic walls, symmetry top, CFL 0.3, hybrid WENO5-AO GKS with the Prandtl "
                       f"correction, S2O4; {steps} timed steps from the initial data"}
    for name, prec in (("fp64", H.FP64), ("fp32_bulk", H.FP32_BULK)):
        log(f"[bench] timing vst {name}: {warmup} warm-up + {steps} steps")
        el, flux_ms, stats, tile, prof = time_solver(H, [P], [W0], prec, steps, warmup, -1)
        out[name] = {"value": 1000 * 500 * steps / el / 1e6, "ms_per_step": el / steps * 1e3,
                     "flux_ms_per_launch": flux_ms, "launch_config": launch_config(tile),
                     "flagged_x": stats[0]["flagged_x"], "flagged_y": stats[0]["flagged_y"]}
        log(f"[bench] vst {name}: {out[name]['value']:.1f} Mcell-updates/s")
    return out


def tile_sweep(args):
    """Mean flux-launch time of every launch configuration on the benchmark workload, one JSON line each;
    with --variants restricting the precisions."""
    import torch
    from paper_2304_05572_amd import hgks as H
    from paper_2304_05572_amd import workloads as wl
    W0, _ = wl.riemann_2d(args.n, seed=args.seed)
    recon = {"hybrid": H.RECON_HYBRID, "wenoao": H.RECON_WENOAO, "linear": H.RECON_LINEAR}[args.recon]
    configs = range(H.NUM_LAUNCH_CONFIGS) if args.configs == "all" else [int(c) for c in args.configs.split(",")]
    for name, prec in (("fp64", H.FP64), ("fp32", H.FP32_BULK)):
        if name not in args.variants.split(","):
            continue
        for c in configs:
            s = H.Solver(rp_problem(H, args.n, recon), precision=prec, tile=c, profile=1)
            s.set_ic(0, W0)
            try:
                s.run(np.inf, 1)
                p0 = s.profile()["flux"]
                s.run(np.inf, 3)
                p1 = s.profile()["flux"]
                ms = (p1[0] - p0[0]) / max(p1[1] - p0[1], 1)
            except H.HgksError as e:  # forced linear reconstruction cannot hold the discontinuities
                ms = None
                log(f"[bench] tile sweep {name} config {c} {args.recon}: {e}")
            torch.cuda.synchronize()
            st = s.stats(0)
            print(json.dumps({"precision": name, "config": c, "recon": args.recon, "tile": s.tile(),
                              "flux_ms_per_launch": ms, "flagged_x": st["flagged_x"],
                              "flagged_y": st["flagged_y"]}), flush=True)
            s.close()


# The paper's 2D cases (Sec. 3.4, 3.5) and the reconstruction CPU times it reports for them, hybrid
# against WENO5-AO (Table of Sec. 3, seconds on its CPU; context, not a target).
PAPER_CASES = {
    "rp_config1": dict(n=(500, 500), t_end=0.2, cfl=0.5, paper_s=(706.471, 6100.513)),
    "rp_config6": dict(n=(500, 500), t_end=0.6, cfl=0.95, paper_s=(5546.881, 9628.309)),
    "double_mach": dict(n=(960, 240), t_end=0.2, cfl=0.8, paper_s=(5334.322, 13596.93)),
}


def paper_case(H, wl, name, recon):
    c = PAPER_CASES[name]
    nx, ny = c["n"]
    if name == "double_mach":
        W0, kw = wl.double_mach(nx, ny, cfl=c["cfl"])
        kw = dict(kw, recon=recon)
    else:
        W0 = wl.quadrants(nx, ny, wl.RP_CONFIG1 if name == "rp_config1" else wl.RP_CONFIG6)
        kw = dict(dim=2, nx=nx, ny=ny, bc=(H.BC_OUTFLOW,) * 4, cfl=c["cfl"], c1=0.01, c2=1.0, recon=recon)
    return H.Problem(**kw), W0


def paper_cases(args):
    """Each 2D case of the paper run to its end time on its grid, FP64, hybrid scheme and forced WENO5-AO:
    wall time of the whole run (one HIP graph per step, launch configuration autotuned beforehand), steps,
    and the troubled-cell fractions sampled every 25 steps; one JSON line per case."""
    import torch
    from paper_2304_05572_amd import hgks as H
    from paper_2304_05572_amd import workloads as wl
    for name, c in PAPER_CASES.items():
        rec = {"case": name, "grid": list(c["n"]), "t_end": c["t_end"], "cfl": c["cfl"], "dtype": "f64"}
        for label, recon in (("hybrid", H.RECON_HYBRID), ("wenoao", H.RECON_WENOAO)):
            P, W0 = paper_case(H, wl, name, recon)
            s = H.Solver(P, autotune=True)
            s.set_ic(0, W0)
            s.step()
            tile = s.tile()
            s.close()
            s = H.Solver(P, tile=tile[3], use_graph=True)
            s.set_ic(0, W0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                steps = int(s.run(c["t_end"])[0])
                status = "reached t_end"
            except H.HgksError as e:
                steps = s.stats(0)["steps"]
                status = f"stopped: {e} at t = {s.stats(0)['t']:.4f}"
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            s.close()
            fr = []
            if recon == H.RECON_HYBRID:
                s = H.Solver(P, tile=tile[3], use_graph=True)
                s.set_ic(0, W0)
                try:
                    while True:
                        n = int(s.run(c["t_end"], 25)[0])
                        st = s.stats(0)
                        fr.append((st["flagged_x"], st["flagged_y"]))
                        if n < 25 or st["t"] >= c["t_end"]:
                            break
                except H.HgksError:
                    pass
                s.close()
                rec["flagged_x_mean"] = float(np.mean([f[0] for f in fr]))
                rec["flagged_y_mean"] = float(np.mean([f[1] for f in fr]))
            rec[label] = {"status": status, "seconds": el, "steps": steps, "ms_per_step": el / max(steps, 1) * 1e3,
                          "mcell_updates_per_s": c["n"][0] * c["n"][1] * steps / el / 1e6,
                          "launch_config": launch_config(tile)}
        rec["hybrid_over_wenoao_time"] = rec["hybrid"]["seconds"] / rec["wenoao"]["seconds"]
        rec["paper_reconstruction_time_ratio"] = c["paper_s"][0] / c["paper_s"][1]
        print(json.dumps(rec), flush=True)


def copy_calibration(mib=512, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.empty(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: {reps} copies of {mib} MiB")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile", type=int, default=-1, help="tile-shape index; -1 autotunes")
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--n3", type=int, default=128, help="cells per side of the 3D variant")
    ap.add_argument("--variants", default="fp64,fp32,batched,fp32c,3d,vst",
                    help="comma list of fp64, fp32, batched, fp32c (FP32-bulk with compensated state), "
                         "3d (the three-dimensional scheme on an n3^3 octant problem), vst (the viscous shock "
                         "tube, Navier-Stokes 1000 x 500, 10 steps), "
                         "wenoao (FP64 with every cell troubled: the WENO5-AO scheme the hybrid one is "
                         "compared against; not in the default run, whose FP64 flux-kernel statistics "
                         "would mix both)")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle leg (CPU baseline and parity)")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a plain copy (counter scaling)")
    ap.add_argument("--tile-sweep", action="store_true",
                    help="only time every flux launch configuration (FP64 and FP32-bulk, 3 steps each)")
    ap.add_argument("--recon", default="hybrid", choices=("hybrid", "wenoao", "linear"),
                    help="reconstruction of the --tile-sweep runs (every cell troubled / none)")
    ap.add_argument("--configs", default="all", help="launch configurations of the --tile-sweep runs")
    ap.add_argument("--paper-cases", action="store_true",
                    help="only run the paper's 2D cases (Riemann configurations 1 and 6, double Mach reflection) "
                         "to their end times, hybrid against forced WENO5-AO")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (the sharding is a design "
              "only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    variants = set(x for x in args.variants.split(",") if x)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.tile_sweep:
        tile_sweep(args)
        return
    if args.paper_cases:
        paper_cases(args)
        return

    import torch  # device memory and streams; the compute is the HIP library
    from paper_2304_05572_amd import hgks as H
    from paper_2304_05572_amd import workloads as wl

    assert torch.cuda.is_available(), "no GPU visible"
    n = args.n
    W0, states = wl.riemann_2d(n, seed=args.seed)
    log(f"[bench] workload RP {n}^2 seed {args.seed} states {states}")
    cells = n * n

    res = {}
    for name, prec, recon, comp in (("fp64", H.FP64, H.RECON_HYBRID, False),
                                    ("fp32", H.FP32_BULK, H.RECON_HYBRID, False),
                                    ("wenoao", H.FP64, H.RECON_WENOAO, False),
                                    ("fp32c", H.FP32_BULK, H.RECON_HYBRID, True)):
        if name not in variants:
            continue
        log(f"[bench] timing {name}: {args.warmup} warm-up + {args.steps} steps")
        rep = {}
        el, flux_ms, stats, tile, prof = time_solver(H, [rp_problem(H, n, recon)], [W0], prec, args.steps,
                                                     args.warmup, args.tile, comp, repeats=4 if name == "fp64" else 0,
                                                     out=rep)
        res[name] = dict(seconds=el, flux_ms=flux_ms, stats=stats[0], tile=tile, prof=prof,
                         mcells=cells * args.steps / el / 1e6, ms_per_step=el / args.steps * 1e3)
        if rep:
            wins = [el] + rep["repeat_seconds"]
            res[name]["windows"] = {"steps_each": args.steps, "mcells": [cells * args.steps / w / 1e6 for w in wins],
                                    "median_mcells": float(np.median([cells * args.steps / w / 1e6 for w in wins]))}
        if name in ("fp64", "fp32", "fp32c"):
            res[name].update(side_windows(H, [rp_problem(H, n, recon)], [W0], prec, tile[3], comp))
        if name == "fp64":
            io = host_io(H, [rp_problem(H, n, recon)], [W0], prec, tile[3], args.steps)
            io["mcells_incl_host_io"] = cells * args.steps / ((io["upload_ms"] + io["steps_ms"] + io["download_ms"])
                                                             * 1e-3) / 1e6
            res[name]["host_io"] = io
        log(f"[bench] {name}: {res[name]['mcells']:.1f} Mcell-updates/s, {res[name]['ms_per_step']:.3f} ms/step, "
            f"flux kernel {flux_ms:.3f} ms/launch, tile {tile}, flagged x {stats[0]['flagged_x']:.4f}")

    batch = None
    if "batched" in variants:
        sizes = wl.batch_sizes(args.batch, seed=args.seed)
        probs = [rp_problem(H, m) for m in sizes]
        bstates = [wl.riemann_2d(m, seed=args.seed * 1000 + k + 1)[0] for k, m in enumerate(sizes)]
        bcells = sum(m * m for m in sizes)
        log(f"[bench] timing batched: {len(sizes)} problems, {bcells} cells")
        el, flux_ms, stats, tile, prof = time_solver(H, probs, bstates, H.FP32_BULK, args.steps, args.warmup,
                                                     args.tile)
        fcx = sum(st["flagged_x"] * m * m for st, m in zip(stats, sizes))
        fcy = sum(st["flagged_y"] * m * m for st, m in zip(stats, sizes))
        batch = dict(mcells=bcells * args.steps / el / 1e6, ms_per_step=el / args.steps * 1e3, cells=bcells,
                     problems=len(sizes), min_n=min(sizes), max_n=max(sizes), launch_config=launch_config(tile),
                     flux_ms=flux_ms, gps=sum(4 * m * (m + 1) for m in sizes),
                     interfaces=sum(2 * m * (m + 1) for m in sizes), fcx=fcx, fcy=fcy)
        # the same batch with one HIP graph per step, and in the persistent launch form of the same tile
        for label, kw in (("graph", dict(use_graph=True)), ("persistent", dict())):
            cfg = tile[3] if label == "graph" else (tile[3] % 6) + 6
            s_ = H.Solver(probs, precision=H.FP32_BULK, tile=cfg, **kw)
            for p_, W_ in enumerate(bstates):
                s_.set_ic(p_, W_)
            s_.run(np.inf, args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s_.run(np.inf, args.steps)
            torch.cuda.synchronize()
            el_ = time.perf_counter() - t0
            batch[label] = {"value": bcells * args.steps / el_ / 1e6, "ms_per_step": el_ / args.steps * 1e3,
                            "launch_config": launch_config(s_.tile())}
            s_.close()
            log(f"[bench] batched {label}: {batch[label]['value']:.1f} Mcell-updates/s")
        del bstates

    vst = time_vst(H, 10, 2) if "vst" in variants else None

    res3 = time_3d(H, wl, args.n3, args.seed, args.steps, args.warmup) if "3d" in variants else None

    parity, cpu = {}, None
    if not args.no_oracle:
        log("[bench] oracle leg: one step of the full grid on the host")
        Wo, dto, cpu = oracle_leg(W0, n)
        for name, prec in (("fp64", H.FP64), ("fp32", H.FP32_BULK)):
            if name in res:
                Wg, dtg = gpu_first_step(H, W0, n, prec)
                parity[name] = (float(np.abs(Wg - Wo).mean() / np.abs(Wo).mean()),
                                float(np.abs(Wg - Wo).max() / np.abs(Wo).max()), bool(dtg == dto))
                log(f"[bench] parity {name}: L1_rel {parity[name][0]:.3e} Linf_rel {parity[name][1]:.3e} "
                    f"dt equal {parity[name][2]}")

    if "fp64" not in res:
        print(json.dumps({"metric": METRIC, "value": None, "note": "fp64 variant not run",
                          "variants": {"three_dimensional": res3}}), flush=True)
        return
    r = res["fp64"]
    gps = 2 * ((n + 1) * n * 2)  # two Gauss points on every x- and y-interface
    nif = 2 * (n + 1) * n        # x- and y-interfaces
    traffic = read_profile_table("k_flux_traffic_rp1024.txt")
    counted = traffic.get("kernel_hash") == kernel_hash()

    def roofline(kernel, ms, gps_, cells_, nif_, fcx, fcy, fp32, key=None):
        """Roofline record of one flux launch: algorithmic operations (method formulas) and bytes over the
        HIP-event mean launch time, against the FP64 or FP32 vector peak and HBM; the executed count and the
        counted HBM bytes come from the committed counter summary when it matches the sources."""
        if not ms or ms <= 0:
            return None
        fl = alg_flops_per_launch(gps_, fcx, fcy)
        by = alg_bytes_per_launch(cells_, nif_, fp32)
        peak = PEAK_FP32_VALU if fp32 else PEAK_FP64_VALU
        ach = fl / (ms * 1e-3) / 1e12
        tr = float(traffic[key]) if (counted and key and key in traffic) else None
        ex = traffic.get("executed_flops_per_gauss_point_%s" % ("fp32" if fp32 else "fp64")) if counted else None
        return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": tr, "traffic_unit": "bytes per launch", "kernel": kernel, "ms_per_launch": ms,
                "algorithmic_flops_per_launch": fl, "algorithmic_flops_per_gauss_point": fl / gps_,
                "gauss_points_per_launch": gps_,
                "executed_flops_per_gauss_point": float(ex) if ex is not None else None,
                "hbm": {"algorithmic_bytes_per_launch": by, "achieved_GBps": by / (ms * 1e-3) / 1e9,
                        "peak_GBps": PEAK_HBM, "frac": by / (ms * 1e-3) / 1e9 / PEAK_HBM,
                        "counted_GBps": tr / (ms * 1e-3) / 1e9 if tr else None}}

    def kname(T, tile):
        return ("k_flux_persistent" if tile[4] else "k_flux") + "<%s, %d, %d, 2, false, 0, %d>" % (
            T, tile[0], tile[1], tile[2]) + " (fused reconstruction + GKS flux)"

    roof = None
    if n == 1024:
        st = r["stats"]
        roof = roofline(kname("double", r["tile"]), r["flux_ms"], gps, n * n, nif, st["flagged_x"] * n * n,
                        st["flagged_y"] * n * n, False, "bytes_per_launch_%d" % r["tile"][3])
    roof32 = None
    if "fp32" in res and n == 1024:
        f = res["fp32"]
        roof32 = roofline(kname("float", f["tile"]), f["flux_ms"], gps, n * n, nif, f["stats"]["flagged_x"] * n * n,
                          f["stats"]["flagged_y"] * n * n, True, "bytes_per_launch_fp32_%d" % f["tile"][3])
    roofb = None
    if batch:
        lc = batch["launch_config"]
        roofb = roofline(("k_flux_persistent" if lc["persistent_blocks"] else "k_flux") + "<float, %d, %d, 2, false, 0, %d>"
                         % (lc["tile"][0], lc["tile"][1], lc["waves_per_simd_target"]), batch["flux_ms"], batch["gps"],
                         batch["cells"], batch["interfaces"], batch["fcx"], batch["fcy"], True)
    out = {
        "metric": METRIC,
        "value": r["mcells"],
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D four-quadrant Riemann problem, Euler, {n}x{n} cells, seeded quadrant states "
                               f"(seed {args.seed}), hybrid WENO5-AO GKS, S2O4, CFL 0.5, c1=0.01, c2=1, outflow",
                   "nx": n, "ny": n, "seed": args.seed, "launch_config": launch_config(r["tile"]),
                   "flagged_fraction_x": r["stats"]["flagged_x"], "flagged_fraction_y": r["stats"]["flagged_y"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": {
            "fp64": {"value": r["mcells"], "ms_per_step": r["ms_per_step"], "flux_ms_per_launch": r["flux_ms"],
                     "kernel_ms_per_step": r["kernel_ms_per_step"], "graph_ms_per_step": r["graph_ms_per_step"],
                     "host_io": r["host_io"],
                     "five_windows": r.get("windows"),
                     "l1_rel_vs_oracle": parity.get("fp64", (None,) * 3)[0],
                     "linf_rel_vs_oracle": parity.get("fp64", (None,) * 3)[1],
                     "dt_bit_exact_vs_oracle": parity.get("fp64", (None,) * 3)[2]},
        },
    }
    if "fp32" in res:
        f = res["fp32"]
        out["variants"]["fp32_bulk"] = {"value": f["mcells"], "ms_per_step": f["ms_per_step"], "roofline": roof32,
                                        "flux_ms_per_launch": f["flux_ms"], "dtype": "f32 (f64 state/flags/CFL)",
                                        "l1_rel_vs_oracle": parity.get("fp32", (None,) * 3)[0],
                                        "linf_rel_vs_oracle": parity.get("fp32", (None,) * 3)[1],
                                        "speedup_vs_fp64": f["mcells"] / r["mcells"],
                                        "kernel_ms_per_step": f["kernel_ms_per_step"],
                                        "graph_ms_per_step": f["graph_ms_per_step"],
                                        "launch_config": launch_config(f["tile"])}
    if "wenoao" in res:
        f = res["wenoao"]
        out["variants"]["fp64_forced_wenoao"] = {
            "value": f["mcells"], "ms_per_step": f["ms_per_step"], "flux_ms_per_launch": f["flux_ms"],
            "note": "every cell troubled: the WENO5-AO GKS the hybrid scheme is compared against",
            "hybrid_speedup": r["mcells"] / f["mcells"], "flux_kernel_speedup": f["flux_ms"] / r["flux_ms"],
            "launch_config": launch_config(f["tile"])}
    if "fp32c" in res:
        f = res["fp32c"]
        out["variants"]["fp32_bulk_compensated"] = {
            "value": f["mcells"], "ms_per_step": f["ms_per_step"], "kernel_ms_per_step": f["kernel_ms_per_step"],
            "graph_ms_per_step": f["graph_ms_per_step"], "dtype": "f32 (f64 state + f64 compensation)",
            "launch_config": launch_config(f["tile"])}
    if res3:
        out["variants"]["three_dimensional"] = res3
    if batch:
        b = {k: v for k, v in batch.items() if k not in ("gps", "interfaces", "fcx", "fcy")}
        out["variants"]["batched"] = dict(b, value=batch["mcells"], dtype="f32 (f64 state/flags/CFL)", roofline=roofb,
                                          workload=f"{batch['problems']} independent Riemann problems, N in "
                                                   f"[{batch['min_n']}, {batch['max_n']}], one launch per kernel, "
                                                   "eager launches (graph and persistent forms beside)")
    if vst:
        out["variants"]["viscous_shock_tube"] = vst
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
