"""Long-lifetime pair lists with dynamic pruning on the GPU (paper, Section
"Heterogeneous parallelization": the GPU prunes the list, which can then be kept
for many more steps with a larger buffer).

A cluster pair pruned at r_inner has no pair inside r_cut until two atoms have
moved (r_inner - r_cut)/2 each, so, while the guard counts no such interval,
the pruned run evaluates exactly the non-zero pair terms of the unpruned one and
must agree with it bitwise; forces at prune, non-prune and rebuild steps must
also match the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1506_00716_amd import inputs

pytestmark = pytest.mark.gpu


def relaxed_rf(nbmod, ctx, seed=1):
    import torch
    s = inputs.small_rf(velocities=True)
    g = nbmod.System(ctx, s)
    x = torch.tensor(s.x, dtype=torch.float64, device=ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=ctx.device)
    g.minimize(x, f, n_iter=500, f_tol=1000.0, max_disp=0.002)
    s.x = x.cpu().numpy()
    g.close()
    return s


def run(nbmod, ctx, s, steps, nstlist, r_list=None, r_inner=0.0, nstprune=0, nstenergy=0):
    import torch
    m = s.model if r_list is None else inputs.Model(r_cut=s.model.r_cut, r_list=r_list,
                                                    coulomb=s.model.coulomb, eps_rf=s.model.eps_rf)
    print(f"[prune] N={s.n} steps={steps} nstlist={nstlist} r_list={m.r_list} r_inner={r_inner} "
          f"nstprune={nstprune}", flush=True)
    g = nbmod.System(ctx, s, model=m, r_inner=r_inner, nstprune=nstprune)
    x = torch.tensor(s.x, dtype=torch.float64, device=ctx.device)
    v = torch.tensor(s.v, dtype=torch.float64, device=ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=ctx.device)
    tr = g.md_step(x, v, f, 0.002, steps, nstlist=nstlist, nstenergy=nstenergy)
    out = dict(x=x.cpu().numpy(), v=v.cpu().numpy(), f=f.cpu().numpy().astype(np.float64),
               tr=tr, guard=g.buffer_stats(), stats=g.stats())
    g.close()
    return out


def rel_rms(f, ref):
    return float(np.sqrt(((f - ref) ** 2).sum() / (ref ** 2).sum()))


@pytest.mark.parametrize("nstprune", [1, 2, 3])
def test_pruned_run_equals_unpruned_bitwise(nbmod, gpu_ctx, nstprune):
    s = relaxed_rf(nbmod, gpu_ctx)
    ref = run(nbmod, gpu_ctx, s, 60, 10)
    pr = run(nbmod, gpu_ctx, s, 60, 10, r_inner=0.95, nstprune=nstprune, nstenergy=10)
    print("guard", pr["guard"])
    assert pr["guard"]["unsafe_prune_intervals"] == 0
    assert pr["guard"]["prune_max_displacement"] > 0.0
    assert np.array_equal(pr["x"], ref["x"]) and np.array_equal(pr["v"], ref["v"])


def test_long_lifetime_list(nbmod, gpu_ctx):
    # a 50-step list lifetime with a 0.4 nm buffer (r_list 1.3), pruned to
    # r_inner 1.0 every 5 steps: bitwise the same run as the same long-lived
    # list without pruning, and forces on the oracle at the end of the run.
    # (The relaxed dense lattice heats up well above 300 K: atoms move up to
    # ~0.16 nm in 50 steps and ~0.03 nm in 5, so both buffers are sized for that.)
    s = relaxed_rf(nbmod, gpu_ctx)
    for steps in (53, 55, 100):  # ends: two steps after a prune, on a prune step, on a rebuild step
        full = run(nbmod, gpu_ctx, s, steps, 50, r_list=1.3)
        pr = run(nbmod, gpu_ctx, s, steps, 50, r_list=1.3, r_inner=1.0, nstprune=5)
        print(steps, "guard", pr["guard"], flush=True)
        assert full["guard"]["unsafe_lifetimes"] == 0
        assert pr["guard"]["unsafe_prune_intervals"] == 0
        assert np.array_equal(pr["x"], full["x"]) and np.array_equal(pr["v"], full["v"])
        assert np.array_equal(pr["f"], full["f"])
        fr, _, _ = oracle.forces(s, x=pr["x"])
        err = rel_rms(pr["f"], fr)
        print(steps, "force rel-RMS vs oracle", err, flush=True)
        assert err <= 1e-5


def test_prune_guard_counts_a_too_narrow_inner_radius(nbmod, gpu_ctx):
    # r_inner = r_cut leaves no margin: the first interval in which any atom
    # moves is counted (the run itself is not checked: it may miss pairs)
    s = relaxed_rf(nbmod, gpu_ctx)
    pr = run(nbmod, gpu_ctx, s, 20, 10, r_inner=s.model.r_cut, nstprune=2)
    assert pr["guard"]["unsafe_prune_intervals"] >= 1
