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


# HBM bytes per launch of the force kernel on the default workload, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes over the MD steps, scaled by
# what the same counters read for a 512 MiB device copy (FETCH_SIZE reads half
# the copied bytes: x2.0; WRITE_SIZE reads them exactly: x1.0).  Valid only for
# the sources they were taken on (keyed by the SHA-256 of the force kernel's
# source followed by the list builder's, which sets the work items and so the
# partials written) and the default cluster size / j-tile; otherwise the
# traffic is reported as null.
TIMING_STRIDE = 7

FORCE_TRAFFIC = {
    "786f8f5986e925bc785c6b17270cd6ef96680f4a4041a4e3c9f2e73a0cd65c63":
        {"fetch_bytes": 2 * 1438.3 * 1024, "write_bytes": 8439.7 * 1024},
}


# HBM bytes per list rebuild on the default workload (the sum over the build's
# kernels of the calibrated FETCH_SIZE + WRITE_SIZE), keyed by the SHA-256 of
# the list builder's source; null for other sources.
BUILD_TRAFFIC = {
    "6d51a392c46240d24b512fdfd692eb28c711732e75759a82f68ea9a44c057499": 14.754e6,
}


def _src_hash(names):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1506_00716_amd", "csrc")
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# VALU counter FLOP per launch of the same kernel on the default workload:
# 64 x (ADD_F32 + MUL_F32 + TRANS_F32) + 128 x FMA_F32 wave instructions from
# one rocprofv3 --pmc pass (every lane of every issued instruction, masked-off
# pairs included), keyed like FORCE_TRAFFIC.
FORCE_VALU_FLOP = {
    "786f8f5986e925bc785c6b17270cd6ef96680f4a4041a4e3c9f2e73a0cd65c63": 588.6e6,
}


def force_kernel_counter_flop(cluster: int, jtile: int):
    f = FORCE_VALU_FLOP.get(_src_hash(("nb_force.hip", "nb_build.hip")))
    if f is None or cluster not in (0, 8) or jtile != 0:
        return None
    return f


def force_kernel_traffic(cluster: int, jtile: int):
    t = FORCE_TRAFFIC.get(_src_hash(("nb_force.hip", "nb_build.hip")))
    if t is None or cluster not in (0, 8) or jtile != 0:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def list_build_traffic(cluster: int, jtile: int):
    t = BUILD_TRAFFIC.get(_src_hash(("nb_build.hip",)))
    if t is None or cluster not in (0, 8) or jtile != 0:
        return None
    return t


def ns_per_day(steps_per_s: float, dt_ps: float) -> float:
    return steps_per_s * dt_ps * 1e-3 * 86400.0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, sysm, useful: int, nthreads: int, budget_s: float):
    """Whole force evaluations of the oracle until the budget is spent."""
    evals, elapsed = 0, 0.0
    while elapsed < budget_s:
        t0 = time.perf_counter()
        oracle.forces(sysm, nthreads=nthreads)
        elapsed += time.perf_counter() - t0
        evals += 1
    return useful * evals / elapsed, evals, elapsed


def cpu_baseline(sysm, budget_s: float = 12.0):
    """Time the FP64 O(N^2) oracle on the host: whole force evaluations of the
    same workload (its generator positions), repeated until the budget is spent,
    on every core this process may use and on one core, reported as useful pair
    interactions/s."""
    import oracle
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    # useful pairs (r < r_cut, min image) at these positions, counted outside the timing
    useful = int(oracle.pairs(sysm.x, sysm.box, sysm.model.r_cut, nthreads=nthreads).shape[0])
    rate, evals, elapsed = _oracle_rate(oracle, sysm, useful, nthreads, budget_s)
    rate1, evals1, elapsed1 = _oracle_rate(oracle, sysm, useful, 1, budget_s / 2)
    # the all-pairs loop tests every unordered pair once per evaluation
    checks = sysm.n * (sysm.n - 1) // 2
    return {"value": rate, "unit": "pair interactions/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{evals} full force evaluations of the {sysm.n}-atom system at its generator "
                      f"positions ({useful} pairs within r_cut each), {elapsed:.1f} s on {nthreads} threads",
            "pair_checks_per_s": rate * checks / useful,
            "single_thread": {"value": rate1, "cores": 1, "pair_checks_per_s": rate1 * checks / useful,
                              "sample": f"{evals1} full force evaluations, {elapsed1:.1f} s"},
            "cpu_model": cpu_model()}


def calibration_copy(mb: int):
    """A plain device copy of a known size: its FETCH_SIZE / WRITE_SIZE counters
    calibrate the per-dispatch HBM byte counts of the profiled kernels."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def list_build_bytes(n_atoms: int, st: dict) -> float:
    """Algorithmic bytes of one list build: read x (24 B/atom), write the staged
    slots and the atom permutation (20 B per slot + 4 B per atom), cluster
    bounding boxes and references (56 B per cluster), the bounding-box search
    (32 B per candidate cluster pair), the atom-pair prune (the candidate's M
    staged j-atoms, 16 B each) and the list write (24 B per kept entry)."""
    m = st["slots"] // max(1, st["groups"] * 8)
    return (24.0 * n_atoms + 20.0 * st["slots"] + 4.0 * n_atoms + 56.0 * st["clusters"]
            + 32.0 * st["candidates"] + 16.0 * m * st["candidates"] + 24.0 * st["entries"])


def timed_leg(s, x, v, f, dt, steps, nstenergy, marks=True):
    """K md_step steps between two synchronisations; with marks, HIP events
    bracket one of every TIMING_STRIDE force launches and rebuilds (a stride
    coprime with nstlist, so every step of the list period is sampled; each
    event record costs the stream a few microseconds)."""
    import torch
    s.set_timing(marks, every=TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.md_step(x, v, f, dt, steps, nstlist=10, nstenergy=nstenergy)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = s.timings()
    s.set_timing(False)
    return wall, tm


def run_dodecahedron_leg(ctx, nb, inputs, dt, steps, warmup):
    """16,800 atoms in a rhombic dodecahedron of image distance 6.2 nm (the
    24,000-atom cubic workload's model, density and image distance): relaxed,
    then `steps` timed velocity-Verlet steps with energies every 10 steps."""
    import torch
    sysm = inputs.dodecahedron_ewald(velocities=True)
    s = nb.System(ctx, sysm)
    x, v, f = nb.device_state(sysm)
    s.minimize(x, f, n_iter=500, f_tol=1000.0, max_disp=0.002)
    v.copy_(torch.tensor(sysm.v, dtype=torch.float64, device="cuda:0"))
    s.step = 0
    s.build_pairlist(x)
    st = s.stats()
    s.set_build_checks(False)
    s.md_step(x, v, f, dt, max(warmup, 10), nstlist=10, nstenergy=10)
    wall, tm = timed_leg(s, x, v, f, dt, steps, nstenergy=10)
    res = {"workload": "16800-atom Ewald dynamics in a rhombic dodecahedron (image distance 6.2 nm)",
           "n_atoms": sysm.n, "ms_per_step": 1000.0 * wall / steps, "ns_per_day": ns_per_day(steps / wall, dt),
           "pairs_per_s": st["pairs_rcut"] * steps / wall, "useful_pairs_per_step": st["pairs_rcut"],
           "force_kernel_us": 1000.0 * tm["force_ms"] / max(1, tm["force_launches"]),
           "rebuild_us": 1000.0 * tm["build_ms"] / max(1, tm["builds"]),
           "buffer_guard": s.buffer_stats()}
    s.close()
    return res


def run_pme_leg(ctx, nb, sysm, x0, v0, dt, steps):
    """Full Ewald: the 24,000-atom state with the reciprocal part by smooth PME
    (0.12 nm grid, order 4) on a stream of its own beside the pair kernel;
    `steps` velocity-Verlet steps with energies every 10 steps, and the PME
    evaluation alone."""
    import dataclasses

    import torch
    grid = nb.pme_grid_for(sysm.box)
    m = dataclasses.replace(sysm.model, pme_grid=grid, pme_order=4)
    h = nb.System(ctx, sysm, model=m)
    h.set_build_checks(False)
    x, v = x0.clone(), v0.clone()
    f = torch.zeros((sysm.n, 3), dtype=torch.float32, device=x.device)
    h.md_step(x, v, f, dt, 10, nstlist=10, nstenergy=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.md_step(x, v, f, dt, steps, nstlist=10, nstenergy=10)
    torch.cuda.synchronize()
    w = time.perf_counter() - t0
    fp = torch.zeros_like(f)
    for _ in range(5):
        h.pme_forces(x, fp, energies=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 200
    for _ in range(reps):
        h.pme_forces(x, fp, energies=False)
    torch.cuda.synchronize()
    wp = (time.perf_counter() - t0) / reps
    e_rec, _ = h.pme_forces(x, fp)
    h.close()
    return {"workload": "24000-atom full Ewald dynamics: pair part as the headline plus smooth PME "
                        f"(grid {grid[0]}x{grid[1]}x{grid[2]}, order 4, beta 3.12)",
            "grid": list(grid), "order": 4, "steps": steps, "ms_per_step": 1000.0 * w / steps,
            "ns_per_day": ns_per_day(steps / w, dt), "pme_us_per_evaluation": 1e6 * wp,
            "e_recip_self_background": e_rec}


def run_dynamics(args):
    import torch

    from paper_1506_00716_amd import inputs, nb

    ctx = nb.Context(0)
    if args.calib_copy_mb > 0:
        calibration_copy(args.calib_copy_mb)
    sysm = inputs.dynamics_ewald(velocities=True)
    dt = 0.002
    s = nb.System(ctx, sysm, cluster=args.cluster, jtile=args.jtile, fp32_reduce=args.fp32_reduce)
    x, v, f = nb.device_state(sysm)
    # pre-relaxation of the literal lattice (steepest descent on the same force path)
    fmax, iters = s.minimize(x, f, n_iter=500, f_tol=1000.0, max_disp=0.002)
    v.copy_(torch.tensor(sysm.v, dtype=torch.float64, device="cuda:0"))
    s.step = 0
    s.build_pairlist(x)
    st = s.stats()
    # capacity is checked once at the end of each call (an overflow makes the
    # call fail: the binding raises), not after every rebuild
    s.set_build_checks(False)
    # warm-up steps (untimed)
    if args.warmup > 0:
        s.md_step(x, v, f, dt, args.warmup, nstlist=10, nstenergy=10)
    torch.cuda.synchronize()
    # the workload as stated: energies and virial (FP64 reduction) every 10
    # steps, without timing events (the kernel times come from the next leg)
    wall, _ = timed_leg(s, x, v, f, dt, args.steps, nstenergy=10, marks=False)
    # the same number of steps without energy evaluations: every force launch is
    # then the force-only kernel, whose time the roofline uses
    wall0, tm0 = timed_leg(s, x, v, f, dt, args.steps, nstenergy=0)
    # useful pairs (r < r_cut) at the end of the run: one more build for the count
    s.build_pairlist(x)
    st_end = s.stats()
    useful = 0.5 * (st["pairs_rcut"] + st_end["pairs_rcut"])
    steps_per_s = args.steps / wall
    value = useful * args.steps / wall
    force_us = 1000.0 * tm0["force_ms"] / max(1, tm0["force_launches"])
    rebuild_us = 1000.0 * tm0["build_ms"] / max(1, tm0["builds"])
    flops = FLOPS_PER_PAIR[sysm.model.coulomb] * useful
    achieved = flops / (force_us * 1e-6) / 1e12
    cflop = force_kernel_counter_flop(args.cluster, args.jtile)
    counter_tflops = cflop / (force_us * 1e-6) / 1e12 if cflop else None
    lb_bytes = 0.5 * (list_build_bytes(sysm.n, st) + list_build_bytes(sysm.n, st_end))
    lb_gbs = lb_bytes / (rebuild_us * 1e-6) / 1e9
    # longer list lifetimes with the GPU's rolling prune, from the same state:
    # buffers sized from the largest displacement measured over 10 / 50 / 100
    # steps of this system (~0.06 / 0.10 / 0.14 nm: the relaxed lattice heats
    # to ~650 K) and the inner radius from ~0.025 nm per 4 steps
    lifetimes = {}
    x_l, v_l = x.clone(), v.clone()
    n_l = max(args.steps, 300)
    for nstlist, r_list, r_inner, nstprune in () if args.headline_only else ((10, 1.1, 0.0, 0), (10, 1.1, 1.03, 2),
                                               (50, 1.25, 1.06, 4), (100, 1.35, 1.06, 4)):
        m = inputs.Model(r_cut=sysm.model.r_cut, r_list=r_list, coulomb="ewald",
                         ewald_beta=sysm.model.ewald_beta)
        h = nb.System(ctx, sysm, model=m, r_inner=r_inner, nstprune=nstprune)
        h.set_build_checks(False)
        xx, vv, ff = x_l.clone(), v_l.clone(), torch.zeros_like(f)
        h.md_step(xx, vv, ff, dt, 10, nstlist=nstlist, nstenergy=10)  # list built, caches warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.md_step(xx, vv, ff, dt, n_l, nstlist=nstlist, nstenergy=10)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        gd = h.buffer_stats()
        lifetimes[f"nstlist{nstlist}_rlist{r_list}" + (f"_prune{r_inner}x{nstprune}" if r_inner else "")] = {
            "ms_per_step": 1000.0 * w / n_l, "ns_per_day": ns_per_day(n_l / w, dt),
            "pairs_per_s": useful * n_l / w, "steps": n_l,
            "unsafe_lifetimes": gd["unsafe_lifetimes"], "max_displacement_nm": gd["max_displacement"],
            "unsafe_prune_intervals": gd["unsafe_prune_intervals"],
            "prune_max_displacement_nm": gd["prune_max_displacement"]}
        h.close()
    # the paper's other box shape (Fig. 6): the same model and image distance in
    # a rhombic dodecahedron holds 16,800 atoms
    dodec = pme = None
    if not args.headline_only:
        dodec = run_dodecahedron_leg(ctx, nb, inputs, dt, max(args.steps, 300), args.warmup)
        progress("dodecahedron leg done")
        pme = run_pme_leg(ctx, nb, sysm, x_l, v_l, dt, n_l)
        progress("PME leg done")
    # NVE energy conservation: equilibrate to 1,000 steps after the velocities
    # were assigned, then 1,000 steps (2 ps) with energies every 10 steps
    done = args.warmup + 2 * args.steps
    if done < 1000:
        s.md_step(x, v, f, dt, 1000 - done, nstlist=10, nstenergy=0)
    tr = s.md_step(x, v, f, dt, 1000, nstlist=10, nstenergy=10)
    t_ps = tr[:, 0] * dt
    etot = tr[:, 4] / sysm.n
    drift = float(np.polyfit(t_ps, etot, 1)[0]) if len(tr) > 2 else float("nan")
    buf = s.buffer_stats()
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
                               "dt 2 fs, nstlist 10, FP32 forces, FP64 update, energies and virial "
                               "(FP64 reduction) every 10 steps)",
                   "n_atoms": sysm.n, "cluster": s.params.cluster or 8, "jtile": s.params.jtile,
                   "precision": "V32" if args.fp32_reduce else "V64r", "nstenergy": 10},
        "ns_per_day": ns_per_day(steps_per_s, dt),
        "forces_only_leg": {"ms_per_step": 1000.0 * wall0 / args.steps,
                            "value": useful * args.steps / wall0,
                            "ns_per_day": ns_per_day(args.steps / wall0, dt)},
        "useful_pairs_per_step": useful,
        "evaluated_pairs_per_step": st["evaluated_pairs"],
        "evaluated_over_useful": st["evaluated_pairs"] / useful,
        "list": {"entries": st["entries"], "cluster_pairs": st["cluster_pairs"], "items": st["items"],
                 "groups": st["groups"], "clusters": st["clusters"], "candidates": st["candidates"]},
        "list_pairs_rlist": st["atom_pairs_rlist"],
        "force_kernel_us": force_us,
        "rebuild_us": rebuild_us,
        "list_build": {"bound": "hbm", "achieved": lb_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": lb_gbs / HBM_PEAK_GBS, "algorithmic_bytes": lb_bytes,
                       "hbm_bytes": list_build_traffic(args.cluster, args.jtile)},
        "timed_launches": {"stride": TIMING_STRIDE, "force": tm0["force_launches"], "rebuilds": tm0["builds"]},
        "nve": {"drift_kj_mol_ps_atom": drift,
                "rms_fluct_kj_mol_atom": float(np.std(etot - np.polyval(np.polyfit(t_ps, etot, 1), t_ps))),
                "steps": 1000, "after_steps": max(1000, done),
                "max_rel_dev": float(np.max(np.abs(tr[:, 4] - tr[0, 4])) / abs(tr[0, 4]))},
        "list_lifetimes": lifetimes,
        "dodecahedron": dodec,
        "full_ewald_pme": pme,
        "buffer_guard": {"max_displacement_nm": buf["max_displacement"],
                         "unsafe_lifetimes": buf["unsafe_lifetimes"]},
        "ewald_fit_error": s.ewald_fit_error(),
        "relax": {"fmax": fmax, "iterations": iters},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": force_kernel_traffic(args.cluster, args.jtile), "traffic_unit": "HBM bytes per launch",
                     "peak_unpacked": FP32_PEAK_UNPACKED_TFLOPS,
                     "frac_unpacked": achieved / FP32_PEAK_UNPACKED_TFLOPS,
                     "flops_per_pair": FLOPS_PER_PAIR[sysm.model.coulomb],
                     "counter_achieved": counter_tflops,
                     "counter_frac": counter_tflops / FP32_PEAK_TFLOPS if counter_tflops else None,
                     "kernel": "force-only pass, 8x8 clusters"},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inputs.dynamics_ewald(velocities=False), budget_s=args.cpu_budget)
    return res


def relax_inplace(ctx, nb, sysm, n_iter=300, f_tol=1000.0):
    """Steepest-descent relaxation on the GPU force path; returns relaxed x (host)."""
    import torch
    g = nb.System(ctx, sysm)
    x = torch.tensor(sysm.x, dtype=torch.float64, device="cuda:0")
    f = torch.zeros((sysm.n, 3), dtype=torch.float32, device="cuda:0")
    g.minimize(x, f, n_iter=n_iter, f_tol=f_tol, max_disp=0.002)
    g.build_pairlist(x)
    useful = g.stats()["pairs_rcut"]
    out = x.cpu().numpy()
    g.close()
    return out, useful


def autotune_table(ctx, nb, inputs, sizes, dt=0.002):
    """(cluster, jtile) per size class, tuned once on a representative member of
    each class; a system's choice is then a function of its size only."""
    import torch
    edges = [1000, 2000, 4000, 8000, 16000, 32000]
    table = []
    for lo, hi in zip(edges, edges[1:]):
        n = int(round(math.sqrt(lo * hi) / 2)) * 2
        s = inputs.ensemble_member(10_000 + lo, n)
        x, _ = relax_inplace(ctx, nb, s, n_iter=100)
        s.x = x
        g = nb.System(ctx, s)
        xx = torch.tensor(x, dtype=torch.float64, device="cuda:0")
        f = torch.zeros((s.n, 3), dtype=torch.float32, device="cuda:0")
        c, j, us = g.autotune(xx, f, clusters=(4, 8), jtiles=(8, 16, 32, 64))
        table.append({"lo": lo, "hi": hi, "cluster": c, "jtile": j, "force_us": us})
        g.close()
    return table


def pick(table, n):
    for row in table:
        if row["lo"] <= n < row["hi"]:
            return row["cluster"], row["jtile"]
    return table[-1]["cluster"], table[-1]["jtile"]


def run_ensemble(args):
    """512 independent systems, batched (one launch per kernel per step, graph
    replay) vs 512 plain per-system md_step calls on the same GPU."""
    import torch

    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    dt = 0.002
    sizes = inputs.ensemble_sizes(args.n_systems)
    t_setup = time.perf_counter()
    tune = autotune_table(ctx, nb, inputs, sizes) if args.autotune else None
    members = []
    for k, n in enumerate(sizes):
        s = inputs.ensemble_member(k, n)
        s.x, useful = relax_inplace(ctx, nb, s, n_iter=args.relax_iter)
        c, j = pick(tune, n) if tune else (args.cluster, args.jtile)
        members.append((s, useful, c, j))
        if (k + 1) % 64 == 0:
            progress(f"{k + 1} members relaxed")
    setup_s = time.perf_counter() - t_setup
    useful_total = sum(m[1] for m in members)

    def fresh_state():
        out = []
        for s, useful, c, j in members:
            g = nb.System(ctx, s, cluster=c, jtile=j)
            x, v, f = nb.device_state(s)
            out.append((g, x, v, f))
        return out

    # plain: one system at a time, each with its own launches
    plain = fresh_state()
    for g, x, v, f in plain:
        g.md_step(x, v, f, dt, args.warmup, nstlist=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, x, v, f in plain:
        g.md_step(x, v, f, dt, args.steps, nstlist=10)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    progress(f"plain: {t_plain:.2f} s")
    xs_plain = [x.cpu().numpy() for _, x, _, _ in plain[:4]]
    for g, *_ in plain:
        g.close()
    del plain
    # batched
    batch = fresh_state()
    ens = nb.Ensemble(ctx, len(batch))
    for g, x, v, f in batch:
        ens.add(g, x, v, f)
    ens.step(args.warmup, dt, nstlist=10, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(args.steps, dt, nstlist=10, use_graph=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(a, x.cpu().numpy()) for a, (_, x, _, _) in zip(xs_plain, batch[:4]))
    ens.close()
    v_batch = useful_total * args.steps / t_batch
    v_plain = useful_total * args.steps / t_plain
    return {
        "metric": METRIC, "value": v_batch, "unit": "pair interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * t_batch / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched ensemble of {len(sizes)} systems, N log-uniform 1000-30000, RF rc 0.9, "
                               f"rlist 1.0, dt 2 fs, nstlist 10, {args.steps} steps", "total_atoms": int(sum(sizes))},
        "plain_value": v_plain, "batched_over_plain": v_batch / v_plain,
        "plain_ms_per_step": 1000.0 * t_plain / args.steps,
        "useful_pairs_per_step": useful_total, "alone_equals_batched_bitwise": bool(same),
        "autotune": tune, "setup_s": setup_s,
    }


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_serve(args):
    """Poisson stream of MD jobs through the continuous-batching server vs the same
    trace served one job at a time (FIFO), at several offered loads, plus a run
    with a small device-memory budget that forces queueing."""
    import torch

    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    dt = 0.002
    # capacity calibration: a batch of typical jobs, atom-steps/s
    cal = inputs.job_trace(24, rate=1.0, seed=505)
    srv = nb.Server(ctx, pool_bytes=int(args.pool_gib * (1 << 30)), max_slots=64, dt=dt)
    cal_sys = []
    for j in cal:
        s = inputs.job_system(j, seed=505)
        s.x, _ = relax_inplace(ctx, nb, s, n_iter=args.relax_iter)
        cal_sys.append(s)
    t0 = time.perf_counter()
    for s in cal_sys:
        srv.submit(s, 100)
    srv.wait_idle(600)
    cap = srv.stats()["atom_steps"] / (time.perf_counter() - t0)
    srv.close()
    progress(f"capacity {cap:.3e} atom-steps/s")
    # the trace's sizes and step counts do not depend on the rate: relax once
    base = inputs.job_trace(args.n_jobs, rate=1.0)
    mean_work = np.mean([j.n_atoms * j.n_steps for j in base])
    systems = []
    for j in base:
        s = inputs.job_system(j)
        s.x, _ = relax_inplace(ctx, nb, s, n_iter=args.relax_iter)
        systems.append(s)
    progress(f"{len(systems)} job systems relaxed")

    def serve(jobs, slots, pool_bytes):
        srv = nb.Server(ctx, pool_bytes=int(pool_bytes), max_slots=slots, dt=dt)
        t0 = time.perf_counter()
        ids = []
        for j, s in zip(jobs, systems):
            delay = j.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(s, j.n_steps))
        srv.wait_idle(3600)
        wall = time.perf_counter() - t0
        polls = [srv.poll(i) for i in ids]
        lat = np.array([q["t_done"] - q["t_submit"] for q in polls if q["state"] == "done"])
        st = srv.stats()
        out = {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
               "atom_steps_per_s": st["atom_steps"] / wall,
               "ns_per_day_aggregate": ns_per_day(st["atom_steps"] / wall / np.mean([j.n_atoms for j in jobs]), dt),
               "done": st["done"], "failed": st["failed"], "rejected": st["rejected"], "wall_s": wall}
        srv.close()
        return out

    results = {}
    for load in args.loads:
        jobs = inputs.job_trace(args.n_jobs, rate=load * cap / mean_work)
        for mode, slots in (("batched", 64), ("serial", 1)):
            results.setdefault(str(load), {})[mode] = serve(jobs, slots, args.pool_gib * (1 << 30))
            progress(f"load {load} {mode}: {results[str(load)][mode]}")
    small = {}
    if args.small_pool_gib > 0:
        jobs = inputs.job_trace(args.n_jobs, rate=args.loads[0] * cap / mean_work)
        small = serve(jobs, 64, args.small_pool_gib * (1 << 30))
        small["pool_gib"] = args.small_pool_gib
        progress(f"small pool: {small}")
    key = str(args.loads[0])
    b, s_ = results[key]["batched"], results[key]["serial"]
    return {
        "metric": METRIC, "value": b["p99_s"], "unit": "s (p99 job latency)", "n_gpus": 1,
        "steps": args.n_jobs, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served Poisson stream of {args.n_jobs} MD jobs, N log-uniform 2000-200000, "
                               f"steps U(100,5000), RF, loads {args.loads} of batched capacity",
                   "capacity_atom_steps_per_s": cap},
        "p50_s": b["p50_s"], "serial_p50_s": s_["p50_s"], "serial_p99_s": s_["p99_s"],
        "by_load": results, "small_pool": small,
    }


def run_large(args):
    """1M-atom slab (dense central slab, LB mixing, Ewald): list build and force
    kernel timings, and the precision study V64r vs V32 against the FP64 oracle
    on a sampled subset of atoms (forces) and on a 1/8-volume system (energies)."""
    import torch

    import oracle
    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    if args.calib_copy_mb > 0:
        calibration_copy(args.calib_copy_mb)
    out = {}
    sysm = inputs.slab_system()
    x = torch.tensor(sysm.x, dtype=torch.float64, device="cuda:0")
    f = torch.zeros((sysm.n, 3), dtype=torch.float32, device="cuda:0")
    rng = np.random.default_rng((3, 99))
    idx = np.sort(rng.choice(sysm.n, size=args.sample, replace=False))
    t0 = time.perf_counter()
    fr, _ = oracle.forces_subset(sysm, idx)
    t_oracle = time.perf_counter() - t0
    for name, fp32 in (("V64r", False), ("V32", True)):
        g = nb.System(ctx, sysm, fp32_reduce=fp32, force_fixed_bits=16)
        g.build_pairlist(x)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(5):
            g.build_pairlist(x)
        torch.cuda.synchronize()
        build_ms = 1000.0 * (time.perf_counter() - tb) / 5
        st = g.stats()
        g.compute_forces(x, f, energies=False)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        for _ in range(args.steps):
            g.compute_forces(x, f, energies=False)
        torch.cuda.synchronize()
        force_ms = 1000.0 * (time.perf_counter() - tf) / args.steps
        fg = f.cpu().numpy().astype(np.float64)
        err = float(np.sqrt(((fg[idx] - fr) ** 2).sum() / (fr ** 2).sum()))
        out[name] = {"force_rel_rms": err, "build_ms": build_ms, "force_call_ms": force_ms,
                     "useful_pairs": st["pairs_rcut"], "evaluated_pairs": st["evaluated_pairs"],
                     "pairs_per_s": st["pairs_rcut"] / (force_ms * 1e-3)}
        if name == "V64r":
            # the rebuilds of an MD run (FP32-pruned list, no exact test): 30
            # steps from rest with a tiny time step (the generator lattice is
            # not relaxed), 3 rebuilds timed with HIP events
            xm = x.clone()
            vm = torch.zeros_like(xm)
            g.set_build_checks(False)
            g.md_step(xm, vm, f, 1e-6, 10, nstlist=10, nstenergy=0)
            g.set_timing(True)
            g.md_step(xm, vm, f, 1e-6, 30, nstlist=10, nstenergy=0)
            tm = g.timings()
            g.set_timing(False)
            rb_us = 1000.0 * tm["build_ms"] / max(1, tm["builds"])
            lb = list_build_bytes(sysm.n, st)
            out[name]["md_rebuild_ms"] = rb_us / 1000.0
            out[name]["list_build"] = {"bound": "hbm", "achieved": lb / (rb_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": lb / (rb_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                       "algorithmic_bytes": lb}
        g.close()
    # energies on a 1/8-volume slab system (same densities), full oracle sum
    small = inputs.slab_system(n_atoms=125_000, box=21.5 / 2)
    t0 = time.perf_counter()
    _, er, _ = oracle.forces(small)
    t_small = time.perf_counter() - t0
    xs = torch.tensor(small.x, dtype=torch.float64, device="cuda:0")
    fs = torch.zeros((small.n, 3), dtype=torch.float32, device="cuda:0")
    for name, fp32 in (("V64r", False), ("V32", True)):
        g = nb.System(ctx, small, fp32_reduce=fp32, force_fixed_bits=16)
        g.build_pairlist(xs)
        e, _ = g.compute_forces(xs, fs)
        out[name]["energy_rel_err_125k"] = [float(abs(e[k] - er[k]) / abs(er[k])) for k in range(2)]
        g.close()
    v = out["V64r"]["pairs_per_s"]
    return {
        "metric": METRIC, "value": v, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": out["V64r"]["force_call_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1,000,000-atom slab (21.5 nm box, 1.5x density slab, LB mixing, Ewald beta 3.12, "
                               "rc 1.0, rlist 1.1), one force evaluation per step"},
        "precision": out, "oracle_sample_atoms": int(args.sample), "oracle_sample_s": t_oracle,
        "oracle_125k_s": t_small,
    }


def run_drift(args):
    """NVE energy conservation of the 24,000-atom Ewald workload, separated into
    its causes: integrator error (dt 2 fs against 1 fs over the same time),
    precision (V32 against V64r), missed pairs (every pair inside r_cut at the
    last step of a list lifetime checked against the pairs within r_list at
    that list's build, by the FP64 oracle), and the FP64 oracle's own drift on
    a 2,700-atom box of the same density and model (no list, FP64 forces) as the
    floor."""
    import torch

    import oracle
    from paper_1506_00716_amd import inputs, nb
    ctx = nb.Context(0)
    kb = inputs.KB
    out = {}

    def slope(tr, dt, n):
        t_ps = tr[:, 0] * dt
        e = tr[:, 4] / n
        p = np.polyfit(t_ps, e, 1)
        return float(p[0]), float(np.std(e - np.polyval(p, t_ps)))

    def temperature(tr, n):
        return float(np.mean(2.0 * tr[:, 3] / ((3 * n - 3) * kb)))

    sysm = inputs.dynamics_ewald(velocities=True)
    g = nb.System(ctx, sysm)
    x, v, f = nb.device_state(sysm)
    g.minimize(x, f, n_iter=500, f_tol=1000.0, max_disp=0.002)
    v.copy_(torch.tensor(sysm.v, dtype=torch.float64, device="cuda:0"))
    g.step = 0
    tr = g.md_step(x, v, f, 0.002, args.equil, nstlist=10, nstenergy=100)
    out["equilibration"] = {"steps": args.equil, "temperature_K_first": temperature(tr[:1], sysm.n),
                            "temperature_K_last": temperature(tr[-1:], sysm.n)}
    x0, v0 = x.clone(), v.clone()
    g.close()
    legs = {}
    for name, dt, steps, fp32 in (("V64r_dt2fs", 0.002, args.drift_steps, False),
                                  ("V64r_dt1fs", 0.001, 2 * args.drift_steps, False),
                                  ("V32_dt2fs", 0.002, args.drift_steps, True)):
        h = nb.System(ctx, sysm, fp32_reduce=fp32)
        xx, vv, ff = x0.clone(), v0.clone(), torch.zeros_like(f)
        t = h.md_step(xx, vv, ff, dt, steps, nstlist=10 if dt == 0.002 else 20, nstenergy=10)
        d, fl = slope(t, dt, sysm.n)
        legs[name] = {"drift_kj_mol_ps_atom": d, "rms_fluct_kj_mol_atom": fl, "ps": steps * dt,
                      "temperature_K": temperature(t, sysm.n), "buffer_guard": h.buffer_stats()}
        h.close()
    out["legs"] = legs
    # missed pairs: each list lifetime's last positions against its build positions
    h = nb.System(ctx, sysm)
    xx, vv, ff = x0.clone(), v0.clone(), torch.zeros_like(f)
    h.md_step(xx, vv, ff, 0.002, 1, nstlist=10)  # step 1: the list is built at step 0's positions
    missed, checked, lifetimes = 0, 0, 0
    x_build = x0.cpu().numpy()
    to_last = 8  # the first list serves steps 1-9, every later one steps k..k+9
    for _ in range(args.lifetimes):
        h.md_step(xx, vv, ff, 0.002, to_last, nstlist=10)  # to the lifetime's last step
        x_last = xx.cpu().numpy()
        inner = oracle.pairs(x_last, sysm.box, sysm.model.r_cut)
        listed = oracle.pairs(x_build, sysm.box, sysm.model.r_list)
        ki = inner[:, 0].astype(np.int64) * sysm.n + inner[:, 1]
        kl = listed[:, 0].astype(np.int64) * sysm.n + listed[:, 1]
        missed += int(np.setdiff1d(ki, kl, assume_unique=True).size)
        checked += int(ki.size)
        lifetimes += 1
        h.md_step(xx, vv, ff, 0.002, 1, nstlist=10)  # the rebuild step: x is then the build's positions
        x_build = xx.cpu().numpy()
        to_last = 9
    out["missed_pairs"] = {"lifetimes": lifetimes, "pairs_checked": checked, "missed": missed,
                           "note": "pairs inside r_cut at a list lifetime's last step that were not within "
                                   "r_list at that list's build (FP64 oracle)"}
    h.close()
    # the FP64 oracle's drift floor on a 2,700-atom box of the same density and model
    small = inputs.lattice_system(2700, 3.0, 6, inputs.MODEL_EWALD, velocities=True)
    gs = nb.System(ctx, small)
    xs, vs, fs = nb.device_state(small)
    gs.minimize(xs, fs, n_iter=500, f_tol=1000.0, max_disp=0.002)
    vs.copy_(torch.tensor(small.v, dtype=torch.float64, device="cuda:0"))
    gs.step = 0
    gs.md_step(xs, vs, fs, 0.002, args.equil, nstlist=10, nstenergy=0)
    small.x, small.v = xs.cpu().numpy(), vs.cpu().numpy()
    gs.close()
    gs = nb.System(ctx, small)
    xs, vs, fs = nb.device_state(small)
    tg = gs.md_step(xs, vs, fs, 0.002, args.floor_steps, nstlist=10, nstenergy=10)
    d_gpu, fl_gpu = slope(tg, 0.002, small.n)
    t0 = time.perf_counter()
    _, _, to = oracle.md(small, small.x, small.v, 0.002, args.floor_steps)
    t_or = time.perf_counter() - t0
    rows = np.arange(10, args.floor_steps + 1, 10)
    tro = np.column_stack([rows, to[rows - 1]])
    d_or, fl_or = slope(tro, 0.002, small.n)
    out["floor_2700"] = {"steps": args.floor_steps, "gpu_drift": d_gpu, "gpu_rms_fluct": fl_gpu,
                         "oracle_drift": d_or, "oracle_rms_fluct": fl_or, "oracle_s": t_or,
                         "temperature_K": temperature(tg, small.n), "gpu_buffer_guard": gs.buffer_stats()}
    gs.close()
    return {"metric": METRIC, "value": legs["V64r_dt2fs"]["drift_kj_mol_ps_atom"],
            "unit": "kJ/mol/ps/atom (NVE drift)", "n_gpus": 1, "steps": args.drift_steps, "warmup": args.equil,
            "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "24000-atom Ewald dynamics, NVE energy conservation study"}, "drift": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="dynamics", choices=["dynamics", "ensemble", "serve", "large", "drift"])
    ap.add_argument("--sample", type=int, default=50000)
    ap.add_argument("--calib-copy-mb", type=int, default=0)
    ap.add_argument("--n-systems", type=int, default=512)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--relax-iter", type=int, default=500)
    ap.add_argument("--n-jobs", type=int, default=400)
    ap.add_argument("--pool-gib", type=float, default=64.0)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.7])
    ap.add_argument("--small-pool-gib", type=float, default=0.0)
    ap.add_argument("--cluster", type=int, default=0)
    ap.add_argument("--jtile", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--fp32-reduce", action="store_true", help="precision variant V32")
    ap.add_argument("--equil", type=int, default=2000)
    ap.add_argument("--drift-steps", type=int, default=2000)
    ap.add_argument("--lifetimes", type=int, default=20)
    ap.add_argument("--floor-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="dynamics: only the headline legs (no list-lifetime, dodecahedron and PME legs; "
                         "for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ensemble":
        res = run_ensemble(args)
    elif args.workload == "serve":
        res = run_serve(args)
    elif args.workload == "large":
        res = run_large(args)
    elif args.workload == "drift":
        res = run_drift(args)
    else:
        res = run_dynamics(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
