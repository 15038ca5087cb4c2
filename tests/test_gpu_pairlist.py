"""GPU pair list vs the oracle's exact pair set (bit-exact after canonical sort).

The cluster-pair list (paper, Section "SIMD parallelism") must cover exactly the
atom pairs within r_list; with M = N = 1 it is the plain Verlet list (same
section).  Every case compares the exported set with oracle.pairs on the same
FP64 positions.
"""
import numpy as np
import pytest

import oracle
from paper_1506_00716_amd import inputs

pytestmark = pytest.mark.gpu


def run_pairs(nbmod, ctx, sysm, x=None, cluster=0, model=None):
    import torch
    m = model or sysm.model
    s = nbmod.System(ctx, sysm, cluster=cluster, model=m)
    xx = torch.tensor(np.ascontiguousarray(sysm.x if x is None else x), dtype=torch.float64,
                      device=ctx.device)
    print(f"[pairlist] N={sysm.n} box={sysm.box.tolist()} M={cluster} rlist={m.r_list}", flush=True)
    s.build_pairlist(xx)
    p = s.export_pairs()
    st = s.stats()
    s.close()
    return p, st


def same_set(a, b):
    return a.shape == b.shape and np.array_equal(a, b)


@pytest.mark.parametrize("cluster", [1, 4, 8])
def test_small_rf_pair_set_exact(nbmod, gpu_ctx, cluster):
    s = inputs.small_rf()
    ref = oracle.pairs(s.x, s.box, s.model.r_list)
    got, st = run_pairs(nbmod, gpu_ctx, s, cluster=cluster)
    assert same_set(got, ref), (len(got), len(ref))
    assert st["atom_pairs_rlist"] == len(ref)


@pytest.mark.parametrize("n,box,rl,seed", [(50, (2.1, 2.1, 2.1), 1.0, 1),
                                           (301, (2.15, 2.2, 2.3), 1.07, 2),
                                           (1000, (2.15, 2.15, 2.15), 1.07, 3),
                                           (513, (3.0, 2.05, 2.5), 1.02, 4),
                                           (63, (4.0, 4.0, 4.0), 1.9, 5),
                                           (1, (3.0, 3.0, 3.0), 1.0, 6),
                                           (2, (3.0, 3.0, 3.0), 1.0, 7)])
@pytest.mark.parametrize("cluster", [1, 4, 8])
def test_tiny_boxes_rlist_near_half_box(nbmod, gpu_ctx, n, box, rl, seed, cluster):
    m = inputs.Model(r_cut=min(rl, 0.9), r_list=rl, coulomb="rf")
    s = inputs.tiny_random_system(n, box, seed, m)
    ref = oracle.pairs(s.x, s.box, rl)
    got, _ = run_pairs(nbmod, gpu_ctx, s, cluster=cluster)
    assert same_set(got, ref), (len(got), len(ref))


@pytest.mark.parametrize("cluster", [4, 8])
def test_any_periodic_image_and_permutation(nbmod, gpu_ctx, cluster):
    s = inputs.small_rf()
    rng = np.random.default_rng(17)
    x = s.x + rng.integers(-3, 4, size=s.x.shape) * s.box  # other images, as given
    ref = oracle.pairs(x, s.box, s.model.r_list)
    got, _ = run_pairs(nbmod, gpu_ctx, s, x=x, cluster=cluster)
    assert same_set(got, ref)
    perm = rng.permutation(s.n)
    sp = inputs.System(box=s.box, x=s.x[perm], q=s.q[perm], sigma=s.sigma[perm],
                       epsilon=s.epsilon[perm], mass=s.mass[perm], model=s.model)
    got_p, _ = run_pairs(nbmod, gpu_ctx, sp, cluster=cluster)
    mapped = np.sort(np.stack([perm[got_p[:, 0]], perm[got_p[:, 1]]], 1), axis=1)
    mapped = mapped[np.lexsort((mapped[:, 1], mapped[:, 0]))]
    assert same_set(mapped, oracle.pairs(s.x, s.box, s.model.r_list))


def test_dynamics_ewald_full_size_pair_set_exact(nbmod, gpu_ctx):
    s = inputs.dynamics_ewald(velocities=False)
    ref = oracle.pairs(s.x, s.box, s.model.r_list)
    got, st = run_pairs(nbmod, gpu_ctx, s)
    assert same_set(got, ref), (len(got), len(ref))
    # cluster-pair overhead: evaluated pair slots per useful pair within r_list
    assert st["evaluated_pairs"] > len(ref)


def test_slab_subregion_pair_set_exact(nbmod, gpu_ctx):
    # a 60k-atom slab (same densities as the 1M-atom system): dense and sparse columns
    s = inputs.slab_system(n_atoms=60_000, box=21.5 * (0.06 ** (1 / 3)))
    ref = oracle.pairs(s.x, s.box, s.model.r_list)
    got, _ = run_pairs(nbmod, gpu_ctx, s)
    assert same_set(got, ref), (len(got), len(ref))


def test_degenerate_dense_column(nbmod, gpu_ctx):
    # all atoms squeezed into a thin rod along z: one xy column far above the
    # average fill (exercises the large-column sort path)
    rng = np.random.default_rng(9)
    n = 6000
    x = np.stack([rng.uniform(0, 0.05, n), rng.uniform(0, 0.05, n), rng.uniform(0, 3.0, n)], 1)
    m = inputs.Model(r_cut=0.9, r_list=1.0, coulomb="rf")
    s = inputs.System(box=np.full(3, 3.0), x=x, q=np.zeros(n), sigma=np.full(n, 0.3),
                      epsilon=np.full(n, 0.5), mass=np.full(n, 16.0), model=m)
    ref = oracle.pairs(s.x, s.box, 1.0)
    got, _ = run_pairs(nbmod, gpu_ctx, s)
    assert same_set(got, ref), (len(got), len(ref))


@pytest.mark.parametrize("cluster", [4, 8])
def test_md_rebuilds_export_exact_and_same_forces(nbmod, gpu_ctx, cluster):
    # Lists built inside md_step keep the search's conservative FP32 atom-pair
    # prune; the exact masks are computed when the pairs are exported.  After
    # 20 steps with nstlist 10 the last rebuild is at the final positions: the export must be the exact set there, and the forces
    # must be those of a list built exactly at the same positions.
    import torch
    s = inputs.small_rf(velocities=True)
    dev = gpu_ctx.device
    g = nbmod.System(gpu_ctx, s, cluster=cluster)
    x = torch.tensor(s.x, dtype=torch.float64, device=dev)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=dev)
    g.minimize(x, f, n_iter=300, f_tol=1000.0, max_disp=0.002)
    v = torch.tensor(s.v, dtype=torch.float64, device=dev)
    g.step = 0
    g.md_step(x, v, f, 0.002, 20, nstlist=10)
    f_md = f.cpu().numpy().copy()
    xf = x.cpu().numpy()
    got = g.export_pairs()
    ref = oracle.pairs(xf, s.box, s.model.r_list)
    assert same_set(got, ref), (len(got), len(ref))
    h = nbmod.System(gpu_ctx, s, cluster=cluster)
    f2 = torch.zeros_like(f)
    h.build_pairlist(x)
    h.compute_forces(x, f2, energies=False)
    # the same pairs within r_cut; the lists' entries fall into other work items,
    # which regroups the FP32 register sums
    fa, fb = f2.cpu().numpy().astype(np.float64), f_md.astype(np.float64)
    assert np.sqrt(((fa - fb) ** 2).sum() / (fb ** 2).sum()) < 1e-6
    # exporting did not change the list the forces run on
    f3 = torch.zeros_like(f)
    g.compute_forces(x, f3, energies=False)
    assert np.array_equal(f3.cpu().numpy(), f_md)
    g.close()
    h.close()


@pytest.mark.parametrize("n,box,rl,seed", [(301, (2.15, 2.2, 2.3), 1.07, 2),
                                           (513, (3.0, 2.05, 2.5), 1.02, 4),
                                           (63, (4.0, 4.0, 4.0), 1.9, 5)])
@pytest.mark.parametrize("cluster", [1, 4, 8])
def test_tiny_boxes_md_build(nbmod, gpu_ctx, n, box, rl, seed, cluster):
    # The build md_step starts with (FP32 prune in the search, no exact test)
    # in boxes where r_list reaches near half the box, so a column meets its
    # own periodic images: every pair within r_list is listed exactly once
    # (exact export), and the forces equal those of an exact build up to the
    # regrouping of FP32 sums.
    import torch
    m = inputs.Model(r_cut=min(rl, 0.9), r_list=rl, coulomb="rf")
    s = inputs.tiny_random_system(n, box, seed, m, min_dist=0.15)
    dev = gpu_ctx.device
    print(f"[pairlist] md build N={s.n} box={s.box.tolist()} M={cluster} rlist={rl}", flush=True)
    g = nbmod.System(gpu_ctx, s, cluster=cluster)
    x = torch.tensor(s.x, dtype=torch.float64, device=dev)
    v = torch.zeros((s.n, 3), dtype=torch.float64, device=dev)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=dev)
    g.md_step(x, v, f, 0.002, 0, nstlist=10)
    got = g.export_pairs()
    ref = oracle.pairs(s.x, s.box, rl)
    assert same_set(got, ref), (len(got), len(ref))
    h = nbmod.System(gpu_ctx, s, cluster=cluster)
    f2 = torch.zeros_like(f)
    h.build_pairlist(x)
    h.compute_forces(x, f2, energies=False)
    fa, fb = f2.cpu().numpy().astype(np.float64), f.cpu().numpy().astype(np.float64)
    assert np.sqrt(((fa - fb) ** 2).sum() / max((fb ** 2).sum(), 1e-300)) < 1e-6
