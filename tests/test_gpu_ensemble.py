"""Batched ensembles and the job server: every member's result is bitwise the same
alone and in the batch (V64r fixed-point force sums); graph replay equals eager
launches; admission by memory budget; failure isolation."""
import time

import numpy as np
import pytest

from paper_1506_00716_amd import inputs

pytestmark = pytest.mark.gpu


def members(k=6, seed=0):
    sizes = [1000, 1500, 2300, 3100, 4200, 5000, 1200, 2600][:k]
    out = []
    for i, n in enumerate(sizes):
        s = inputs.ensemble_member(i, n, seed=70 + seed)
        out.append(s)
    return out


def alone(nbmod, ctx, s, steps, cluster=0, nstlist=10):
    import torch
    g = nbmod.System(ctx, s, cluster=cluster)
    x = torch.tensor(s.x, dtype=torch.float64, device=ctx.device)
    v = torch.tensor(s.v, dtype=torch.float64, device=ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=ctx.device)
    g.md_step(x, v, f, 0.002, steps, nstlist=nstlist)
    out = (x.cpu().numpy(), v.cpu().numpy())
    g.close()
    return out


def relaxed(nbmod, ctx, sysms):
    """Relax each generated lattice on the GPU (as the benchmark does) and return
    the systems with relaxed positions."""
    import torch
    out = []
    for s in sysms:
        g = nbmod.System(ctx, s)
        x = torch.tensor(s.x, dtype=torch.float64, device=ctx.device)
        f = torch.zeros((s.n, 3), dtype=torch.float32, device=ctx.device)
        g.minimize(x, f, n_iter=300, f_tol=1000.0, max_disp=0.002)
        s2 = inputs.System(box=s.box, x=x.cpu().numpy(), q=s.q, sigma=s.sigma, epsilon=s.epsilon,
                           mass=s.mass, model=s.model, v=s.v)
        g.close()
        out.append(s2)
    return out


@pytest.mark.parametrize("use_graph", [True, False])
def test_ensemble_equals_alone_bitwise(nbmod, gpu_ctx, use_graph):
    import torch
    sysms = relaxed(nbmod, gpu_ctx, members(6))
    clusters = [8, 4, 8, 4, 8, 8]
    ref = [alone(nbmod, gpu_ctx, s, 25, cluster=c) for s, c in zip(sysms, clusters)]
    ens = nbmod.Ensemble(gpu_ctx, 8)
    keep = []
    for s, c in zip(sysms, clusters):
        g = nbmod.System(gpu_ctx, s, cluster=c)
        x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
        v = torch.tensor(s.v, dtype=torch.float64, device=gpu_ctx.device)
        f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
        ens.add(g, x, v, f)
        keep.append((g, x, v, f))
    print(f"[ens] members={len(keep)} graph={use_graph}", flush=True)
    ens.step(12, 0.002, nstlist=10, use_graph=use_graph)
    ens.step(13, 0.002, nstlist=10, use_graph=use_graph)
    for (g, x, v, f), (xr, vr) in zip(keep, ref):
        assert np.array_equal(x.cpu().numpy(), xr)
        assert np.array_equal(v.cpu().numpy(), vr)
        assert g.step == 25
    ens.close()


def test_ensemble_energies_and_membership(nbmod, gpu_ctx):
    import torch
    sysms = relaxed(nbmod, gpu_ctx, members(4, seed=1))
    ens = nbmod.Ensemble(gpu_ctx, 4)
    keep = []
    for s in sysms:
        g = nbmod.System(gpu_ctx, s)
        x, v, f = nbmod.device_state(s)
        ens.add(g, x, v, f)
        keep.append((g, x, v, f, s))
    e = ens.step(10, 0.002, nstlist=10, energies=True)
    assert e.shape == (4, 3) and np.all(np.isfinite(e))
    # the same member alone gives the same energies
    g0, x0, v0, f0, s0 = keep[0]
    ens.remove(g0)
    assert ens.size() == 3
    ens.step(5, 0.002, nstlist=10)
    ref = alone(nbmod, gpu_ctx, s0, 10)
    assert np.array_equal(x0.cpu().numpy(), ref[0])
    ens.close()


def test_autotune_picks_a_candidate(nbmod, gpu_ctx):
    import torch
    s = relaxed(nbmod, gpu_ctx, members(1))[0]
    g = nbmod.System(gpu_ctx, s)
    x, v, f = nbmod.device_state(s)
    c, j, us = g.autotune(x, f, clusters=(4, 8), jtiles=(8, 16, 32))
    print("autotune", c, j, us)
    assert c in (4, 8) and j in (8, 16, 32) and us > 0


def test_server_results_equal_alone(nbmod, gpu_ctx):
    sysms = relaxed(nbmod, gpu_ctx, members(5, seed=2))
    steps = [37, 20, 55, 12, 41]
    ref = [alone(nbmod, gpu_ctx, s, n) for s, n in zip(sysms, steps)]
    srv = nbmod.Server(gpu_ctx, pool_bytes=1 << 30, max_slots=8)
    ids = []
    for k, (s, n) in enumerate(zip(sysms, steps)):
        print(f"[srv] submit job {k} N={s.n} steps={n}", flush=True)
        ids.append(srv.submit(s, n))
        time.sleep(0.003)  # arrivals while others run
    srv.wait_idle(120.0)
    for jid, s, (xr, vr) in zip(ids, sysms, ref):
        st = srv.poll(jid)
        assert st["state"] == "done", st
        x, v = srv.fetch(jid, s.n)
        assert np.array_equal(x, xr) and np.array_equal(v, vr)
        assert st["t_done"] >= st["t_admit"] >= st["t_submit"]
    stats = srv.stats()
    assert stats["done"] == 5 and stats["failed"] == 0
    srv.close()


def test_server_budget_queueing_and_rejection(nbmod, gpu_ctx):
    # three jobs of the same size and a budget that holds one job but not two
    sysms = relaxed(nbmod, gpu_ctx, [inputs.ensemble_member(k, 2000, seed=73) for k in range(3)])
    p = nbmod.make_params(sysms[0].n, sysms[0].box, sysms[0].model)
    job = int(nbmod.arena_bytes(p) * 1.25) + 60 * sysms[0].n + 4096
    srv = nbmod.Server(gpu_ctx, pool_bytes=int(1.5 * job), max_slots=4)
    ids = [srv.submit(s, 15) for s in sysms]
    big = inputs.ensemble_member(9, 30000, seed=74)
    jbig = srv.submit(big, 5)
    srv.wait_idle(120.0)
    for jid in ids:
        assert srv.poll(jid)["state"] == "done"
    assert srv.poll(jbig)["state"] == "rejected"
    # a budget for one job runs them one at a time
    t = sorted((srv.poll(j)["t_admit"], srv.poll(j)["t_done"]) for j in ids)
    for (a0, d0), (a1, d1) in zip(t, t[1:]):
        assert a1 >= d0 - 1e-6
    srv.close()


def test_server_isolates_a_failing_job(nbmod, gpu_ctx):
    sysms = relaxed(nbmod, gpu_ctx, members(3, seed=4))
    bad = sysms[1]
    x = bad.x.copy()
    x[1] = x[0]  # two atoms on top of each other: infinite pair force
    broken = inputs.System(box=bad.box, x=x, q=bad.q, sigma=bad.sigma, epsilon=bad.epsilon,
                           mass=bad.mass, model=bad.model, v=bad.v)
    ref0 = alone(nbmod, gpu_ctx, sysms[0], 30)
    srv = nbmod.Server(gpu_ctx, pool_bytes=1 << 30, max_slots=4)
    j0 = srv.submit(sysms[0], 30)
    j1 = srv.submit(broken, 30)
    j2 = srv.submit(sysms[2], 30)
    srv.wait_idle(120.0)
    assert srv.poll(j1)["state"] == "failed"
    assert srv.poll(j0)["state"] == "done" and srv.poll(j2)["state"] == "done"
    x0, v0 = srv.fetch(j0, sysms[0].n)
    assert np.array_equal(x0, ref0[0])
    srv.close()


# ---- batched and served members against the FP64 oracle ----------------------

def oracle_gap(s, x, v, steps):
    import oracle
    xo, vo, _ = oracle.md(s, s.x, s.v, 0.002, steps)
    return float(np.abs(x - xo).max()), float(np.abs(v - vo).max())


def test_batched_members_match_oracle(nbmod, gpu_ctx):
    # dense RF members (100 atoms/nm^3, relaxed) advanced 50 steps in one batch:
    # each stays on the FP64 oracle's own trajectory from the same start
    sysms = relaxed(nbmod, gpu_ctx, members(3, seed=5))
    ens = nbmod.Ensemble(gpu_ctx, 4)
    keep = []
    for s, c in zip(sysms, (8, 4, 8)):
        g = nbmod.System(gpu_ctx, s, cluster=c)
        x, v, f = nbmod.device_state(s)
        ens.add(g, x, v, f)
        keep.append((g, x, v, f, s))
    print("[ens] batched vs oracle", flush=True)
    ens.step(50, 0.002, nstlist=10, use_graph=True)
    for g, x, v, f, s in keep:
        ex, ev = oracle_gap(s, x.cpu().numpy(), v.cpu().numpy(), 50)
        print(f"N={s.n}: max |dx| {ex:.3e} nm, max |dv| {ev:.3e} nm/ps", flush=True)
        assert ex < 1e-5 and ev < 1e-3
    ens.close()


def test_served_jobs_match_oracle(nbmod, gpu_ctx):
    sysms = relaxed(nbmod, gpu_ctx, members(3, seed=6))
    steps = [50, 33, 47]
    srv = nbmod.Server(gpu_ctx, pool_bytes=1 << 30, max_slots=4)
    ids = [srv.submit(s, n) for s, n in zip(sysms, steps)]
    srv.wait_idle(120.0)
    for jid, s, n in zip(ids, sysms, steps):
        assert srv.poll(jid)["state"] == "done"
        x, v = srv.fetch(jid, s.n)
        ex, ev = oracle_gap(s, x, v, n)
        print(f"served N={s.n} steps={n}: max |dx| {ex:.3e} nm, max |dv| {ev:.3e} nm/ps", flush=True)
        assert ex < 1e-5 and ev < 1e-3
    srv.close()


# ---- a member whose list outgrows its arena -----------------------------------

def imploding(n=4096, box=7.0, rate=25.0, seed=77):
    """A dilute lattice with the velocity field v = -rate (x - L/2): within a
    list lifetime of 10 steps (0.02 ps) the atoms fall to about half their
    distance from the box centre, so the density there grows ~8x and the
    rebuild at step 10 needs more list capacity than the arena, sized for the
    mean density, holds."""
    s = inputs.lattice_system(n, box, seed, inputs.MODEL_RF, velocities=True, jitter=0.02)
    s.v = s.v - rate * (s.x - 0.5 * box)
    return s


def test_ensemble_overflow_rolls_back_the_batch(nbmod, gpu_ctx):
    import torch
    others = relaxed(nbmod, gpu_ctx, members(2, seed=8))
    bad = imploding()
    ref = [alone(nbmod, gpu_ctx, s, 25) for s in others]
    ens = nbmod.Ensemble(gpu_ctx, 4)
    keep = []
    for s in others + [bad]:
        g = nbmod.System(gpu_ctx, s)
        x, v, f = nbmod.device_state(s)
        ens.add(g, x, v, f)
        keep.append((g, x, v, f))
    print("[ens] overflow rollback", flush=True)
    with pytest.raises(nbmod.NbError) as exc:
        ens.step(25, 0.002, nstlist=10)
    assert exc.value.code == nbmod.NB_ERR_CAPACITY
    # every member stopped at the last full step before the failed rebuild
    assert [g.step for g, *_ in keep] == [9, 9, 9]
    # drop the member that overflowed; the others finish the run and equal
    # their runs alone bitwise
    ens.remove(keep[2][0])
    ens.step(16, 0.002, nstlist=10)
    for (g, x, v, f), (xr, vr) in zip(keep[:2], ref):
        assert g.step == 25
        assert np.array_equal(x.cpu().numpy(), xr) and np.array_equal(v.cpu().numpy(), vr)
    ens.close()


def test_server_grows_an_overflowing_job(nbmod, gpu_ctx):
    # the imploding job's list outgrows its arena at step 10: the server stops
    # the batch at step 9, moves that job to a larger block and continues; it
    # ends as its lone run does (which grows its arena at the same step), and
    # the other jobs end bitwise as alone
    others = relaxed(nbmod, gpu_ctx, members(2, seed=9))
    bad = imploding()
    steps = [30, 30, 12]  # (the imploding job stops two steps after its rebuild)
    ref = [alone(nbmod, gpu_ctx, s, n) for s, n in zip(others + [bad], steps)]
    srv = nbmod.Server(gpu_ctx, pool_bytes=1 << 30, max_slots=4)
    print("[srv] overflow regrow", flush=True)
    ids = [srv.submit(s, n) for s, n in zip(others + [bad], steps)]
    srv.wait_idle(120.0)
    for jid, s, (xr, vr) in zip(ids, others + [bad], ref):
        st = srv.poll(jid)
        assert st["state"] == "done", st
        x, v = srv.fetch(jid, s.n)
        assert np.array_equal(x, xr) and np.array_equal(v, vr)
    assert srv.stats()["failed"] == 0
    srv.close()
