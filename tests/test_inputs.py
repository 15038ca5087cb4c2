"""Seeded input generators: reproducibility, sizes, charge neutrality, densities."""
import numpy as np
import pytest

from paper_1506_00716_amd import inputs


def test_lattice_edge_integer():
    assert inputs.lattice_edge(2700) == 14
    assert inputs.lattice_edge(24000) == 29
    assert inputs.lattice_edge(27000) == 30
    assert inputs.lattice_edge(27001) == 31
    assert inputs.lattice_edge(1) == 1


def test_small_rf_reproducible_bitwise():
    a = inputs.small_rf(velocities=True)
    b = inputs.small_rf(velocities=True)
    assert a.n == 2700
    assert np.array_equal(a.x.view(np.uint64), b.x.view(np.uint64))
    assert np.array_equal(a.v.view(np.uint64), b.v.view(np.uint64))
    assert np.all(a.x >= 0.0) and np.all(a.x < 3.0)
    assert abs(a.q.sum()) == 0.0
    assert set(np.unique(a.q)) == {-0.4, 0.4}


def test_lattice_spacing_and_jitter_bounds():
    s = inputs.small_rf()
    n = 14
    a = 3.0 / n
    idx = np.arange(s.n)
    site = np.stack([(idx % n + 0.5) * a, ((idx // n) % n + 0.5) * a, (idx // (n * n) + 0.5) * a], 1)
    d = s.x - site
    d -= np.round(d / 3.0) * 3.0
    assert np.max(np.abs(d)) <= 0.05 + 1e-12
    assert np.max(np.abs(d)) > 0.049  # the jitter is actually applied


def test_maxwell_kinetic_energy_exact():
    s = inputs.dynamics_ewald(velocities=True)
    ke = 0.5 * np.sum(s.mass[:, None] * s.v ** 2)
    target = 0.5 * (3 * s.n - 3) * inputs.KB * 300.0
    assert abs(ke - target) < 1e-9 * target
    assert np.max(np.abs((s.mass[:, None] * s.v).sum(0))) < 1e-9


def test_slab_density_ratio_and_neutrality():
    s = inputs.slab_system(n_atoms=200_000, box=21.5 * (0.2 ** (1 / 3)))
    L = s.box[0]
    z = s.x[:, 2]
    in_slab = (z >= 0.35 * L) & (z < 0.65 * L)
    # jitter moves a few atoms across the faces; the ratio is taken from the lattice
    # assignment by region volume
    rho_slab = in_slab.sum() / (0.3 * L ** 3)
    rho_bulk = (~in_slab).sum() / (0.7 * L ** 3)
    assert abs(rho_slab / rho_bulk - 1.5) < 0.02
    assert abs(s.q.sum()) < 1e-9
    assert s.sigma.min() >= 0.25 and s.sigma.max() <= 0.35
    assert s.epsilon.min() >= 0.2 and s.epsilon.max() <= 1.0


def test_slab_counts_full_size():
    # region counts of the 1M-atom slab without drawing it: N = rho_b (0.7 + 0.45) V
    n, L = 1_000_000, 21.5
    rho_b = n / (1.15 * L ** 3)
    n_slab = int(round(1.5 * rho_b * 0.3 * L ** 3))
    assert n_slab == 391304
    assert n - n_slab == 608696
    assert abs(n_slab / (0.3 * L ** 3) / ((n - n_slab) / (0.7 * L ** 3)) - 1.5) < 1e-3


def test_ensemble_sizes():
    sz = inputs.ensemble_sizes()
    assert len(sz) == 512
    assert min(sz) >= 1000 and max(sz) <= 30000
    assert all(v % 2 == 0 for v in sz)
    assert sz == inputs.ensemble_sizes()
    m = inputs.ensemble_member(3, sz[3])
    assert abs(m.box[0] - (sz[3] / 100.0) ** (1 / 3)) < 1e-12
    assert abs(m.q.sum()) == 0.0


def test_job_trace():
    jobs = inputs.job_trace(400, rate=2.0)
    assert len(jobs) == 400
    assert jobs[0].arrival == 0.0
    assert all(b.arrival >= a.arrival for a, b in zip(jobs, jobs[1:]))
    assert all(2000 <= j.n_atoms <= 200000 and j.n_atoms % 2 == 0 for j in jobs)
    assert all(100 <= j.n_steps <= 5000 for j in jobs)
    gaps = np.diff([j.arrival for j in jobs])
    assert 0.35 < gaps.mean() < 0.7
