"""Benchmark: short-range non-bonded MD on one MI355X.

Default workload (one JSON line): the 24,000-atom Ewald dynamics system (cubic
6.2 nm box, LJ sigma 0.30 nm / epsilon 0.5 kJ/mol, charges +/-0.4 e, Ewald
real-space beta 3.12 nm^-1, r_cut 1.0, r_list 1.1, 16 amu, 300 K Maxwell
velocities), relaxed by steepest descent, then velocity-Verlet steps at dt 2 fs
with the pair list rebuilt every 10 steps.  A "step" is one MD step: position
update, list rebuild when due, staging, force kernel, force gather, velocity
update -- the whole hot path, inputs resident in HBM.

    python bench.py [--steps K] [--warmup W] [--workload dynamics|ensemble|serve|large]

value = useful pair interactions/s (pairs with r < r_cut per step x steps / s).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s + ns/day (24k atoms); ensemble p50/p99 latency vs plain"
FP32_PEAK_TFLOPS = 157.3        # MI355X published FP32 vector peak (packed FP32)
FP32_PEAK_UNPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0

# Algorithmic flops per useful pair (plain formula: add/sub/mul = 1, FMA = 2,
# each rsqrt/exp/erfc = 1), force-only pass.
FLOPS_PER_PAIR = {"ewald": 36, "rf": 30, "none": 26}


def ns_per_day(steps_per_s: float, dt_ps: float) -> float:
    return steps_per_s * dt_ps * 1e-3 * 86400.0


def cpu_baseline(sysm, budget_s: float = 12.0):
    """Time the FP64 O(N^2) oracle on the host on a bounded sample of atoms of the
    same workload (its generator positions), as useful pair interactions/s."""
    import oracle
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    rng = np.random.default_rng(12345)
    rc2 = sysm.model.r_cut ** 2
    done_rows, pairs, elapsed = 0, 0, 0.0
    rows = 64
    order = rng.permutation(sysm.n)
    while elapsed < budget_s and done_rows < sysm.n:
        idx = np.sort(order[done_rows:done_rows + rows])
        t0 = time.perf_counter()
        oracle.forces_subset(sysm, idx, nthreads=nthreads)
        dt = time.perf_counter() - t0
        # partners within r_cut of each sampled atom (min image), counted outside the timing
        d = sysm.x[None, :, :] - sysm.x[idx][:, None, :]
        d -= np.round(d / sysm.box) * sysm.box
        r2 = (d * d).sum(-1)
        pairs += int((r2 < rc2).sum()) - len(idx)
        elapsed += dt
        done_rows += len(idx)
        rows = min(4096, rows * 2)
    # each row evaluates its pairs once (the oracle's full loop sees every pair from
    # both ends, half-weighted), so pair interactions/s = rows' partners / time
    return {"value": pairs / elapsed, "unit": "pair interactions/s", "cores": oracle.num_threads() if nthreads is None else nthreads,
            "kind": "oracle",
            "sample": f"{done_rows} of {sysm.n} atoms (all partners each, FP64 O(N) rows), {elapsed:.1f} s"}


def run_dynamics(args):
    import torch

    from paper_1506_00716_amd import inputs, nb

    ctx = nb.Context(0)
    sysm = inputs.dynamics_ewald(velocities=True)
    dt = 0.002
    s = nb.System(ctx, sysm, cluster=args.cluster, jtile=args.jtile)
    x, v, f = nb.device_state(sysm)
    # pre-relaxation of the literal lattice (steepest descent on the same force path)
    fmax, iters = s.minimize(x, f, n_iter=500, f_tol=1000.0, max_disp=0.002)
    v.copy_(torch.tensor(sysm.v, dtype=torch.float64, device="cuda:0"))
    s.step = 0
    s.build_pairlist(x)
    st = s.stats()
    s.set_build_checks(False)
    # warm-up steps (untimed)
    if args.warmup > 0:
        s.md_step(x, v, f, dt, args.warmup, nstlist=10, nstenergy=0)
    torch.cuda.synchronize()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.md_step(x, v, f, dt, args.steps, nstlist=10, nstenergy=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = s.timings()
    s.set_timing(False)
    wall = t1 - t0
    # useful pairs (r < r_cut) at the end of the run: one more build for the count
    s.build_pairlist(x)
    st_end = s.stats()
    useful = 0.5 * (st["pairs_rcut"] + st_end["pairs_rcut"])
    steps_per_s = args.steps / wall
    value = useful * args.steps / wall
    force_us = 1000.0 * tm["force_ms"] / max(1, tm["force_launches"])
    flops = FLOPS_PER_PAIR[sysm.model.coulomb] * useful
    achieved = flops / (force_us * 1e-6) / 1e12
    # energy drift over a separate short NVE leg (energies every 10 steps, not timed)
    tr = s.md_step(x, v, f, dt, 200, nstlist=10, nstenergy=10)
    t_ps = tr[:, 0] * dt
    drift = float(np.polyfit(t_ps, tr[:, 4] / sysm.n, 1)[0]) if len(tr) > 2 else float("nan")
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "24000-atom Ewald dynamics (6.2 nm box, rc 1.0, rlist 1.1, beta 3.12, "
                               "dt 2 fs, nstlist 10, FP32 forces, FP64 update)",
                   "n_atoms": sysm.n, "cluster": st["clusters"] and s.params.cluster or 8,
                   "jtile": s.params.jtile},
        "ns_per_day": ns_per_day(steps_per_s, dt),
        "useful_pairs_per_step": useful,
        "evaluated_pairs_per_step": st["evaluated_pairs"],
        "list_pairs_rlist": st["atom_pairs_rlist"],
        "force_kernel_us": force_us,
        "rebuild_us": 1000.0 * tm["build_ms"] / max(1, tm["builds"]),
        "nve_drift_kj_mol_ps_atom": drift,
        "relax": {"fmax": fmax, "iterations": iters},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "peak_unpacked": FP32_PEAK_UNPACKED_TFLOPS,
                     "frac_unpacked": achieved / FP32_PEAK_UNPACKED_TFLOPS,
                     "flops_per_pair": FLOPS_PER_PAIR[sysm.model.coulomb]},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inputs.dynamics_ewald(velocities=False), budget_s=args.cpu_budget)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="dynamics", choices=["dynamics"])
    ap.add_argument("--cluster", type=int, default=0)
    ap.add_argument("--jtile", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    res = run_dynamics(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
