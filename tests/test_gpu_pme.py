"""GPU reciprocal-space Ewald (smooth PME) against the FP64 oracle.

The GPU path computes in FP64 except the charge grid (fixed point, 2^-34 e per
contribution) and the FP32 output forces, so against the oracle's smooth PME on
the same grid and spline order the forces agree to a few FP32 roundings:
|dF| <= 1e-6 |F| + 2e-6 rms(F) per component; energy and virial to 1e-8 of
their scale.  With the pair part (FP32 arithmetic), the full Ewald forces meet
the pair tests' relative RMS bound 1e-5.  Trajectories follow the oracle's for
short times, as in the pair-only dynamics tests.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.pme as PM
from paper_1506_00716_amd import inputs

pytestmark = pytest.mark.gpu


def ewald_model(grid, order=4, r_cut=0.8, r_list=0.9, beta=3.12):
    return inputs.Model(r_cut=r_cut, r_list=r_list, coulomb="ewald", ewald_beta=beta,
                        pme_grid=tuple(grid), pme_order=order)


def with_grid(s, grid, order=4):
    s.model = dataclasses.replace(s.model, pme_grid=tuple(grid), pme_order=order)
    return s


def lattice_of(s):
    return PM.box_matrix(s.box, s.box_off)


def oracle_recip(s):
    """(E_recip + E_self + E_background, F, Xi) of the oracle's smooth PME."""
    m = s.model
    L = lattice_of(s)
    return PM.ewald_total(s.x, s.q, L, m.ewald_beta, m.eps_r,
                          recip=PM.pme_recip(s.x, s.q, L, m.ewald_beta, m.pme_grid, m.pme_order, m.eps_r))


def gpu_pme(nbmod, ctx, s):
    import torch
    print(f"[pme] N={s.n} grid={s.model.pme_grid} order={s.model.pme_order}", flush=True)
    g = nbmod.System(ctx, s)
    x = torch.tensor(np.ascontiguousarray(s.x), dtype=torch.float64, device=ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=ctx.device)
    e, w = g.pme_forces(x, f)
    out = f.cpu().numpy().astype(np.float64)
    # without energies the same forces (asynchronous call)
    f2 = torch.zeros_like(f)
    g.pme_forces(x, f2, energies=False)
    assert torch.equal(f, f2)
    g.close()
    return e, out, w


def rect_case(n, box, grid, order, seed, net=0.0):
    s = inputs.tiny_random_system(n, box, seed, ewald_model(grid, order))
    s.q = s.q + net / n
    return s


def tric_case(n, box, off, grid, order, seed, net=0.0):
    s = inputs.random_triclinic_system(n, box, off, seed, ewald_model(grid, order))
    s.q = s.q + net / n
    return s


def dodec_case():
    box, off = inputs.dodecahedron_box(3.6)
    s = inputs.triclinic_lattice_system(14, box, off, 31, ewald_model((30, 30, 22)), n_atoms=2300)
    return s


def crowded_case(n, n_rod, box, grid, seed, rod_xy, rod_w):
    """Random charges with n_rod of them packed into a rod along c of width
    rod_w at (x, y) = rod_xy: their grid columns hold far more atoms than a
    column bucket (twice the mean occupancy + 16), so the spread also takes
    atoms from the overflow list."""
    s = rect_case(n, box, grid, 4, seed)
    rng = np.random.default_rng(seed + 1000)
    s.x = np.array(s.x, dtype=np.float64)
    s.x[:n_rod, 0] = rod_xy[0] + rod_w * rng.random(n_rod)
    s.x[:n_rod, 1] = rod_xy[1] + rod_w * rng.random(n_rod)
    return s


CASES = {
    "rectangular even grid": lambda: rect_case(1500, (3.0, 3.2, 3.4), (24, 26, 28), 4, 61),
    "rectangular odd grid order 6": lambda: rect_case(1499, (3.0, 3.2, 3.4), (25, 27, 29), 6, 62),
    "dodecahedron": dodec_case,
    "skewed, net charge, ragged": lambda: tric_case(1001, (2.6, 2.4, 2.5), (0.9, -0.6, 0.7), (21, 20, 23), 4, 63,
                                                    net=0.8),
    "grid at the spline order": lambda: tric_case(77, (2.1, 2.2, 2.3), (0.3, 0.2, -0.4), (4, 5, 6), 4, 64),
    "order 6, grid 6": lambda: rect_case(50, (2.0, 2.1, 2.2), (6, 7, 8), 6, 65),
    "one charge": lambda: rect_case(1, (2.0, 2.0, 2.0), (10, 11, 12), 4, 66, net=0.4),
    # lines longer than a wave (more than 64 half-complex points along c)
    "long lines": lambda: rect_case(500, (2.0, 3.0, 3.1), (8, 150, 151), 4, 67),
    "largest grid dimension (256)": lambda: rect_case(300, (2.0, 3.0, 3.2), (4, 256, 256), 4, 68),
    # column buckets overflow: a dense rod over a few columns among random atoms
    "crowded columns": lambda: crowded_case(700, 350, (3.0, 3.0, 3.0), (16, 16, 16), 69, (1.0, 1.5), 0.3),
    # every atom in one grid column (all but a bucket's worth overflow)
    "one column": lambda: crowded_case(200, 200, (3.0, 3.0, 3.0), (16, 16, 16), 70, (1.2, 2.0), 0.04),
}


@pytest.mark.parametrize("case", list(CASES), ids=list(CASES))
def test_pme_matches_oracle(nbmod, gpu_ctx, case):
    s = CASES[case]()
    Eo, Fo, Xo = oracle_recip(s)
    E, F, X = gpu_pme(nbmod, gpu_ctx, s)
    rms = float(np.sqrt(np.mean(Fo ** 2))) + 1e-30
    err = np.abs(F - Fo)
    print(case, "E", E, Eo, "max |dF|/rms", err.max() / rms)
    assert np.all(err <= 1e-6 * np.abs(Fo) + 2e-6 * rms)
    scale = abs(Eo) + abs(PM.ewald_self(s.q, s.model.ewald_beta))
    assert abs(E - Eo) <= 1e-8 * scale
    assert np.max(np.abs(X - Xo)) <= 1e-8 * scale


def test_pme_full_size_dodecahedron(nbmod, gpu_ctx):
    # the 16,800-atom dodecahedron workload on its 0.12 nm grid, every atom
    s = inputs.dodecahedron_ewald(velocities=False)
    with_grid(s, nbmod.pme_grid_for(s.box, s.box_off))
    Eo, Fo, Xo = oracle_recip(s)
    E, F, X = gpu_pme(nbmod, gpu_ctx, s)
    rms = float(np.sqrt(np.mean(Fo ** 2)))
    assert np.all(np.abs(F - Fo) <= 1e-6 * np.abs(Fo) + 2e-6 * rms)
    assert abs(E - Eo) <= 1e-8 * (abs(Eo) + abs(PM.ewald_self(s.q, s.model.ewald_beta)))


def full_ewald_oracle(s):
    fr, er, wr = oracle.forces(s)
    Ek, Fk, Xk = oracle_recip(s)
    return fr + Fk, np.array([er[0], er[1] + Ek]), wr + Xk


_FULL_24K = {}


def full_ewald_24k(nbmod):
    """The 24,000-atom workload on its 0.12 nm grid and its oracle (computed once)."""
    if not _FULL_24K:
        s = inputs.dynamics_ewald(velocities=False)
        with_grid(s, nbmod.pme_grid_for(s.box))
        _FULL_24K["s"] = s
        _FULL_24K["ref"] = full_ewald_oracle(s)
    return _FULL_24K["s"], _FULL_24K["ref"]


@pytest.mark.parametrize("fp32", [False, True], ids=["V64r", "V32"])
def test_full_ewald_forces_24k(nbmod, gpu_ctx, fp32):
    # the 24,000-atom workload: pair forces + reciprocal space through
    # nb_compute_forces, against oracle pair sum + oracle PME, in both
    # precision variants (V32: the gather sums the pair partials and the
    # reciprocal forces in FP32)
    import torch
    s, (fo, eo, wo) = full_ewald_24k(nbmod)
    print(f"[pme] full Ewald N={s.n} grid={s.model.pme_grid} fp32={fp32}", flush=True)
    g = nbmod.System(gpu_ctx, s, fp32_reduce=fp32)
    x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
    g.build_pairlist(x)
    e, w = g.compute_forces(x, f)
    fg = f.cpu().numpy().astype(np.float64)
    g.close()
    err = float(np.sqrt(((fg - fo) ** 2).sum() / (fo ** 2).sum()))
    print("rel-RMS", err, "E", e, eo)
    assert err <= 1e-5
    assert abs(e[0] - eo[0]) <= 1e-5 * abs(eo[0])
    assert abs(e[1] - eo[1]) <= 1e-5 * abs(eo[1])
    assert np.max(np.abs(w - wo)) <= 1e-5 * np.max(np.abs(wo))


def dilute_pme(n=400, box=(3.2, 3.3, 3.4), seed=51):
    m = ewald_model((28, 28, 30), r_cut=0.9, r_list=1.0)
    s = inputs.tiny_random_system(n, box, seed, m, min_dist=0.3)
    s.v = inputs.maxwell_velocities(np.random.default_rng(seed), s.mass, 300.0)
    return s


def oracle_md(s, n_steps, dt):
    """Velocity Verlet in FP64 with the oracle's full Ewald forces; rows
    (step, E_LJ, E_coul, E_kin, E_tot) after every step."""
    x, v = s.x.copy(), s.v.copy()
    m = s.mass[:, None]

    def forces(x):
        s2 = inputs.System(box=s.box, x=x, q=s.q, sigma=s.sigma, epsilon=s.epsilon, mass=s.mass,
                           model=s.model, box_off=s.box_off)
        return full_ewald_oracle(s2)

    f, e, _ = forces(x)
    rows = []
    for k in range(n_steps):
        v = v + 0.5 * dt * f / m
        x = x + dt * v
        f, e, _ = forces(x)
        v = v + 0.5 * dt * f / m
        ke = 0.5 * float(np.sum(m * v * v))
        rows.append([k + 1, e[0], e[1], ke, e[0] + e[1] + ke])
    return x, v, np.array(rows)


def test_pme_trajectory_matches_oracle(nbmod, gpu_ctx):
    import torch
    s = dilute_pme()
    xo, vo, tro = oracle_md(s, 30, 0.002)
    print(f"[pme] md N={s.n}", flush=True)
    g = nbmod.System(gpu_ctx, s)
    x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
    v = torch.tensor(s.v, dtype=torch.float64, device=gpu_ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
    tr = g.md_step(x, v, f, 0.002, 30, nstlist=10, nstenergy=1)
    g.close()
    assert np.max(np.abs(x.cpu().numpy() - xo)) < 1e-4
    assert np.max(np.abs(v.cpu().numpy() - vo)) < 1e-2
    assert np.array_equal(tr[:, 0], np.arange(1, 31))
    assert np.allclose(tr[:, 1:], tro[:, 1:], rtol=1e-4, atol=1e-3)


def test_pme_nve_energy_conservation_and_determinism(nbmod, gpu_ctx):
    import torch
    s = dilute_pme(n=600, box=(3.6, 3.6, 3.6), seed=52)
    with_grid(s, (30, 30, 30))
    runs = []
    for _ in range(2):
        print(f"[pme] nve N={s.n}", flush=True)
        g = nbmod.System(gpu_ctx, s)
        x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
        v = torch.tensor(s.v, dtype=torch.float64, device=gpu_ctx.device)
        f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
        tr = g.md_step(x, v, f, 0.002, 1000, nstlist=10, nstenergy=10)
        g.close()
        runs.append((x.cpu().numpy(), tr))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    tr = runs[0][1]
    e = tr[:, 4]
    drift = np.polyfit(tr[:, 0] * 0.002, e / s.n, 1)[0]
    print("drift kJ/mol/ps/atom", drift)
    assert abs(drift) < 1e-3
    assert np.max(np.abs(e - e[0])) < 2e-3 * np.abs(tr[:, 1:3]).sum(1).max()


def test_pme_trajectory_independent_of_calls_and_energy_steps(nbmod, gpu_ctx):
    # PME runs beside the list build on rebuild steps and on the context
    # stream otherwise; neither the arrangement, nor how the run is split into
    # calls, nor how often energies are asked for changes a bit of it
    import torch

    def run(splits, nstenergy):
        s = dilute_pme(n=500, seed=58)
        print(f"[pme] split {splits} nstenergy {nstenergy}", flush=True)
        g = nbmod.System(gpu_ctx, s)
        x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
        v = torch.tensor(s.v, dtype=torch.float64, device=gpu_ctx.device)
        f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
        for n in splits:
            g.md_step(x, v, f, 0.002, n, nstlist=10, nstenergy=nstenergy)
        g.close()
        return x.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy()

    ref = run((37,), 0)
    for splits, ne in (((37,), 1), ((1, 8, 1, 12, 15), 5)):
        for a, b in zip(ref, run(splits, ne)):
            assert np.array_equal(a, b)


def test_pme_with_dynamic_pruning_equals_unpruned_bitwise(nbmod, gpu_ctx):
    # on steps without a list build the pruning pass of the pair kernel runs
    # on the second stream beside PME; the pairs inside r_cut stay the same
    # while the prune guard holds, and so does every bit of the trajectory
    import torch

    def run(r_inner, nstprune):
        s = dilute_pme(n=500, seed=59)
        print(f"[pme] prune r_inner={r_inner} every {nstprune}", flush=True)
        g = nbmod.System(gpu_ctx, s, r_inner=r_inner, nstprune=nstprune)
        x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
        v = torch.tensor(s.v, dtype=torch.float64, device=gpu_ctx.device)
        f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
        g.md_step(x, v, f, 0.002, 40, nstlist=10, nstenergy=10)
        bs = g.buffer_stats()
        g.close()
        return x.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy(), bs

    ref = run(0.0, 0)
    pr = run(0.95, 2)
    assert pr[3]["unsafe_prune_intervals"] == 0
    for a, b in zip(ref[:3], pr[:3]):
        assert np.array_equal(a, b)


def test_pme_refused_where_there_is_no_pme_stage(nbmod, gpu_ctx):
    # the batched, served and allocation-free forms have no reciprocal stage:
    # a PME system is refused with NB_ERR_ARG, and the reciprocal call on a
    # system without PME is a state error
    s = rect_case(200, (2.2, 2.3, 2.4), (12, 12, 12), 4, 69)
    s.v = np.zeros_like(s.x)
    print(f"[pme] refusals N={s.n}", flush=True)
    g = nbmod.System(gpu_ctx, s)
    x, v, f = nbmod.device_state(s)
    ens = nbmod.Ensemble(gpu_ctx, 2)
    with pytest.raises(nbmod.NbError) as ei:
        ens.add(g, x, v, f)
    assert ei.value.code == nbmod.NB_ERR_ARG
    with pytest.raises(nbmod.NbError) as ei:
        nbmod.compute_forces_noalloc(gpu_ctx, s, x, f)
    assert ei.value.code == nbmod.NB_ERR_ARG
    srv = nbmod.Server(gpu_ctx, 64 << 20, max_slots=4)
    with pytest.raises(nbmod.NbError) as ei:
        srv.submit(s, 10)
    assert ei.value.code == nbmod.NB_ERR_ARG
    srv.close()
    ens.close()
    g.close()
    plain = inputs.tiny_random_system(200, (2.2, 2.3, 2.4), 69, ewald_model((12, 12, 12)))
    plain.model = dataclasses.replace(plain.model, pme_grid=None)
    h = nbmod.System(gpu_ctx, plain)
    with pytest.raises(nbmod.NbError) as ei:
        h.pme_forces(x, f)
    assert ei.value.code == nbmod.NB_ERR_STATE
    h.close()


def test_pme_trajectory_in_a_dodecahedron_matches_oracle(nbmod, gpu_ctx):
    # full Ewald dynamics (pair part + PME) in the skewed box: positions,
    # velocities and the energy rows against the oracle's velocity Verlet
    import torch
    box, off = inputs.dodecahedron_box(3.4)
    s = inputs.triclinic_lattice_system(10, box, off, 71, ewald_model((28, 28, 20), r_cut=0.9, r_list=1.0),
                                        n_atoms=900)
    s.v = inputs.maxwell_velocities(np.random.default_rng(71), s.mass, 300.0)
    dt, n = 0.002, 20
    xo, vo, tro = oracle_md(s, n, dt)
    print(f"[pme] dodecahedron md N={s.n}", flush=True)
    g = nbmod.System(gpu_ctx, s)
    x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
    v = torch.tensor(s.v, dtype=torch.float64, device=gpu_ctx.device)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=gpu_ctx.device)
    tr = g.md_step(x, v, f, dt, n, nstlist=10, nstenergy=1)
    g.close()
    assert np.max(np.abs(x.cpu().numpy() - xo)) < 1e-4
    assert np.max(np.abs(v.cpu().numpy() - vo)) < 1e-2
    assert np.allclose(tr[:, 1:], tro[:, 1:], rtol=1e-4, atol=1e-3)
