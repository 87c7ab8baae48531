#!/usr/bin/env python3
"""Throughput of the hybrid WENO5-AO gas-kinetic scheme (S2O4 steps) on one MI355X.

Workload: 2D four-quadrant Riemann problem, Euler, 1024 x 1024 cells, quadrant states drawn from a seed
(rho in [0.1, 1.5], p in [0.03, 1.5], |u|, |v| <= 1.2, one elementary wave per edge), hybrid WENO5-AO,
CFL 0.5, c1 = 0.01, c2 = 1, outflow boundaries. One step = one full two-stage fourth-order step of every
cell (flags, fused reconstruction + gas-kinetic flux, stage update, for both stages, plus the CFL
reduction), inputs resident in device memory.

`value` is the plain FP64 path in Mcell-updates/s. The same line carries the FP32-bulk path on the same
workload, the batched path (64 uneven problems in one set of launches), their L1 distance to the CPU
oracle on a sampled window after one step, the roofline position of the dominant kernel (fused flux,
VALU-bound, FP64 flops from HIP-event timing of its launches in the timed region) and the oracle's own
CPU throughput on a bounded sample.
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
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X vector FP32 (packed)
PEAK_HBM = 8000.0  # GB/s
# FP64 operations per Gauss-point flux evaluation of the fused kernel on unflagged data (FMA = 2),
# counted with the VALU instruction counters; see profiles/k_flux_counters_rp1024.txt
FLOPS_PER_GP = {"fp64": None, "fp32": None}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in ("hgks_kernels.hip", "hgks_device.hpp"):
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


def rp_problem(H, n, precision_cfl=0.5):
    return H.Problem(dim=2, nx=n, ny=n, bc=(H.BC_OUTFLOW,) * 4, cfl=precision_cfl, c1=0.01, c2=1.0)


def time_solver(H, problems, states, precision, steps, warmup, tile):
    import torch
    s = H.Solver(problems, precision=precision, tile=tile, profile=True, autotune=(tile < 0))
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
    s.close()
    return t1 - t0, flux_ms / max(flux_n, 1), stats, tile_used, prof


def window_l1(H, O, W0, n, precision, win=128, margin=10, seed=0):
    """L1 distance (relative) GPU vs oracle after one step, on a centred win x win window: the GPU advances
    the full grid; the oracle advances the window plus a margin larger than the two-stage dependency
    radius (8 cells) with the GPU's time step, so the window's interior is exact."""
    P = rp_problem(H, n)
    s = H.Solver(P, precision=precision)
    s.set_ic(0, W0)
    dt = s.step()[0]
    Wg, _ = s.get_state(0)
    s.close()
    a = n // 2 - win // 2 - margin
    b = n // 2 + win // 2 + margin
    sub = np.ascontiguousarray(W0[:, a:b, a:b])
    m = b - a
    h = 1.0 / n
    Po = O.Problem(dim=2, nx=m, ny=m, x0=0, x1=m * h, y0=0, y1=m * h, bc=(1, 1, 1, 1), c1=0.01, c2=1.0,
                   cfl=0.5, fixed_dt=dt)
    Wo, _, _ = O.step(Po, sub, 0.0, nthreads=min(16, os.cpu_count() or 1))
    A = Wg[:, a + margin:b - margin, a + margin:b - margin]
    B = Wo[:, margin:-margin, margin:-margin]
    return float(np.abs(A - B).mean() / np.abs(B).mean()), float(np.abs(A - B).max() / np.abs(B).max())


def cpu_baseline(H, O, W0, n, budget_cells=256):
    """The oracle as it stands, on host cores: two S2O4 steps of a centred 256 x 256 window of the same
    workload (outflow boundaries at the window edge), all host threads up to 16."""
    import oracle
    w = budget_cells
    a = n // 2 - w // 2
    sub = np.ascontiguousarray(W0[:, a:a + w, a:a + w])
    h = 1.0 / n
    Po = oracle.Problem(dim=2, nx=w, ny=w, x0=0, x1=w * h, y0=0, y1=w * h, bc=(1, 1, 1, 1), c1=0.01, c2=1.0,
                        cfl=0.5)
    nth = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    W, t = sub, 0.0
    nsteps = 2
    for _ in range(nsteps):
        W, t, _ = oracle.step(Po, W, t, nthreads=nth)
    el = time.perf_counter() - t0
    return {"value": w * w * nsteps / el / 1e6, "unit": "Mcell-updates/s", "cores": nth, "kind": "oracle",
            "sample": f"{nsteps} S2O4 steps of the centred {w}x{w} window of the 1024^2 Riemann problem "
                      f"(outflow window edges), FP64 C oracle, {nth} OpenMP threads, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile", type=int, default=-1, help="tile-shape index; -1 autotunes")
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--skip", default="", help="comma list of: fp32,batched,cpu,parity")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (each box has one GPU); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    skip = set(x for x in args.skip.split(",") if x)

    import torch  # device memory and streams; the compute is the HIP library
    from paper_2304_05572_amd import hgks as H
    from paper_2304_05572_amd import workloads as wl

    assert torch.cuda.is_available(), "no GPU visible"
    n = args.n
    W0, states = wl.riemann_2d(n, seed=args.seed)
    log(f"[bench] workload RP {n}^2 seed {args.seed} states {states}")
    cells = n * n

    res = {}
    for name, prec in (("fp64", H.FP64), ("fp32", H.FP32_BULK)):
        if name == "fp32" and "fp32" in skip:
            continue
        log(f"[bench] timing {name}: {args.warmup} warm-up + {args.steps} steps")
        el, flux_ms, stats, tile, prof = time_solver(H, [rp_problem(H, n)], [W0], prec, args.steps, args.warmup,
                                                     args.tile)
        res[name] = dict(seconds=el, flux_ms=flux_ms, stats=stats[0], tile=tile, prof=prof,
                         mcells=cells * args.steps / el / 1e6, ms_per_step=el / args.steps * 1e3)
        log(f"[bench] {name}: {res[name]['mcells']:.1f} Mcell-updates/s, {res[name]['ms_per_step']:.3f} ms/step, "
            f"flux kernel {flux_ms:.3f} ms/launch, tile {tile}, flagged x {stats[0]['flagged_x']:.4f}")

    batch = None
    if "batched" not in skip:
        sizes = wl.batch_sizes(args.batch, seed=args.seed)
        probs = [rp_problem(H, m) for m in sizes]
        bstates = [wl.riemann_2d(m, seed=args.seed * 1000 + k + 1)[0] for k, m in enumerate(sizes)]
        log(f"[bench] timing batched: {len(sizes)} problems, {sum(m * m for m in sizes)} cells")
        el, flux_ms, stats, tile, prof = time_solver(H, probs, bstates, H.FP32_BULK, args.steps, args.warmup,
                                                     args.tile)
        bcells = sum(m * m for m in sizes)
        batch = dict(mcells=bcells * args.steps / el / 1e6, ms_per_step=el / args.steps * 1e3, cells=bcells,
                     problems=len(sizes), min_n=min(sizes), max_n=max(sizes), tile=tile)
        log(f"[bench] batched: {batch['mcells']:.1f} Mcell-updates/s")
        del bstates

    parity = {}
    if "parity" not in skip:
        import oracle as O
        for name, prec in (("fp64", H.FP64), ("fp32", H.FP32_BULK)):
            if name in res:
                log(f"[bench] window parity {name}")
                parity[name] = window_l1(H, O, W0, n, prec)
    cpu = None
    if "cpu" not in skip:
        import oracle as O
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(H, O, W0, n)

    r = res["fp64"]
    gps = 2 * ((n + 1) * n * 2)  # two Gauss points on every x- and y-interface
    roof = None
    fl = FLOPS_PER_GP.get("fp64")
    traffic = read_profile_table("k_flux_traffic_rp1024_fp64.txt")
    if fl:
        achieved = fl * gps / (r["flux_ms"] * 1e-3) / 1e12
        tr = None
        if traffic.get("kernel_hash") == kernel_hash() and "bytes_per_launch" in traffic:
            tr = float(traffic["bytes_per_launch"])
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_VALU, "traffic": tr,
                "kernel": "k_flux (fused reconstruction + GKS flux, FP64)", "ms_per_launch": r["flux_ms"],
                "flops_per_launch": fl * gps}
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
                   "nx": n, "ny": n, "seed": args.seed, "tile": list(r["tile"]),
                   "flagged_fraction_x": r["stats"]["flagged_x"], "flagged_fraction_y": r["stats"]["flagged_y"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": {
            "fp64": {"value": r["mcells"], "ms_per_step": r["ms_per_step"], "flux_ms_per_launch": r["flux_ms"],
                     "l1_rel_vs_oracle": parity.get("fp64", (None, None))[0],
                     "linf_rel_vs_oracle": parity.get("fp64", (None, None))[1]},
        },
    }
    if "fp32" in res:
        f = res["fp32"]
        out["variants"]["fp32_bulk"] = {"value": f["mcells"], "ms_per_step": f["ms_per_step"],
                                        "flux_ms_per_launch": f["flux_ms"], "dtype": "f32 (f64 state/flags/CFL)",
                                        "l1_rel_vs_oracle": parity.get("fp32", (None, None))[0],
                                        "linf_rel_vs_oracle": parity.get("fp32", (None, None))[1],
                                        "speedup_vs_fp64": f["mcells"] / r["mcells"], "tile": list(f["tile"])}
    if batch:
        out["variants"]["batched"] = dict(batch, value=batch["mcells"], dtype="f32 (f64 state/flags/CFL)",
                                          workload=f"{batch['problems']} independent Riemann problems, N in "
                                                   f"[{batch['min_n']}, {batch['max_n']}], one launch per kernel")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
