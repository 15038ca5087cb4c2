"""Pins of the reciprocal-space oracle (oracle/pme.py) to what the mathematics
fixes, independently of the oracle itself:

* B-spline weights: closed form of M_4, partition of unity, symmetry, and the
  derivative against finite differences; the moduli of order 4 in closed form.
* The direct Ewald sum: the Madelung constant of rock salt (real-space part
  from the C oracle, which its own pins fix), independence of the total energy,
  forces and virial from the splitting parameter beta (both with and without a
  net charge, so the self and background terms are pinned too), forces and
  virial against finite differences of the energy.
* Smooth PME: convergence to the direct sum as the grid is refined (fast for
  order 6), forces and virial against finite differences of the PME energy
  itself.

Every mistake planted at the end of this file (each in a copy of oracle/pme.py
loaded as a module of its own) fails at least one of these.  Nothing here runs
on a GPU.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.pme as PM
from paper_1506_00716_amd import inputs

MADELUNG_NACL = 1.747564594633182  # rock salt, per ion pair, at the nearest-neighbour distance


def _system(x, q, L, model):
    L = PM.box_matrix(L)
    n = x.shape[0]
    z = np.zeros(n)
    box_off = None
    if abs(L[1, 0]) + abs(L[2, 0]) + abs(L[2, 1]) > 0:
        box_off = np.array([L[1, 0], L[2, 0], L[2, 1]])
    return inputs.System(box=np.array([L[0, 0], L[1, 1], L[2, 2]]), x=np.ascontiguousarray(x), q=q,
                         sigma=z + 0.3, epsilon=z, mass=z + 1.0, model=model, box_off=box_off)


def _real(x, q, L, beta, rc):
    model = inputs.Model(r_cut=rc, r_list=rc, coulomb="ewald", ewald_beta=beta, pot_shift=False, epsilon=0.0)
    f, e, w = oracle.forces(_system(x, q, L, model), nthreads=2)
    return float(e[1]), f, w


def _random_charges(n, L, seed, net=0.0):
    rng = np.random.default_rng(seed)
    L = PM.box_matrix(L)
    s = rng.random((n, 3))
    x = s @ L
    q = rng.uniform(-1.0, 1.0, n)
    q -= q.mean()
    q += net / n
    return x, q


def _total(x, q, L, beta, rc, kmax, pm=PM):
    er, fr, wr = _real(x, q, L, beta, rc)
    ek, fk, wk = pm.ewald_recip(x, q, L, beta, kmax)
    eb, wb = pm.ewald_background(q, beta, PM.box_matrix(L))
    return er + ek + pm.ewald_self(q, beta) + eb, fr + fk, wr + wk + wb


# ---- B-splines -------------------------------------------------------------
def test_bspline_order4_closed_form(pm=PM):
    w = np.linspace(0.0, 0.999, 37)
    A, D = pm.bspline(w, 4)
    # M_4 on its four unit pieces, u = w + j
    ref = np.stack([w ** 3 / 6.0,
                    (-3 * w ** 3 + 3 * w ** 2 + 3 * w + 1) / 6.0,
                    (3 * w ** 3 - 6 * w ** 2 + 4) / 6.0,
                    (1 - w) ** 3 / 6.0], 1)
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-15)
    dref = np.stack([w ** 2 / 2.0, (-9 * w ** 2 + 6 * w + 3) / 6.0, (9 * w ** 2 - 12 * w) / 6.0,
                     -(1 - w) ** 2 / 2.0], 1)
    np.testing.assert_allclose(D, dref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [4, 5, 6, 8])
def test_bspline_partition_symmetry_derivative(p, pm=PM):
    w = np.random.default_rng(p).random(50) * 0.98 + 0.01
    A, D = pm.bspline(w, p)
    np.testing.assert_allclose(A.sum(1), 1.0, atol=1e-14)
    np.testing.assert_allclose(D.sum(1), 0.0, atol=1e-13)
    # M_p(u) = M_p(p - u): weight j at w equals weight p-1-j at 1-w
    A2, _ = pm.bspline(1.0 - w, p)
    np.testing.assert_allclose(A, A2[:, ::-1], atol=1e-14)
    # first moment: sum_j (w + j) M_p(w + j) = p / 2 (the spline's centre)
    np.testing.assert_allclose(((w[:, None] + np.arange(p)[None, :]) * A).sum(1), p / 2.0, atol=1e-13)
    h = 1e-6
    Ap, _ = pm.bspline(w + h, p)
    Am, _ = pm.bspline(w - h, p)
    np.testing.assert_allclose(D, (Ap - Am) / (2 * h), atol=1e-8)


@pytest.mark.parametrize("K", [16, 25, 52])
def test_moduli_order4_closed_form(K, pm=PM):
    # M_4 at the integers: 0, 1/6, 2/3, 1/6, so the sum is e^{2 i t} (2 + cos t)/3
    t = 2 * math.pi * np.arange(K) / K
    np.testing.assert_allclose(pm.bspline_moduli(K, 4), 9.0 / (2.0 + np.cos(t)) ** 2, rtol=1e-13)


# ---- direct Ewald sum ------------------------------------------------------
def test_madelung_constant_rock_salt(pm=PM):
    # 2 x 2 x 2 conventional cells of rock salt, lattice constant a: 64 ions of
    # charge +-1, nearest-neighbour distance a/2
    a = 0.5
    g = np.arange(4) * (a / 2)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    idx = np.rint(X / (a / 2)).astype(int)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    L = np.diag([2 * a] * 3)
    for beta in (9.5, 11.0):
        E, F, Xi = _total(X, q, L, beta, 0.49, 20, pm)
        ref = -(len(q) / 2) * MADELUNG_NACL * PM.F_COUL / (a / 2)
        assert E == pytest.approx(ref, rel=1e-9)
        assert np.abs(F).max() < 1e-6 * abs(ref)
        # cubic symmetry: isotropic virial, equal to E/6 for a 1/r potential
        # (1/2 dE/d(strain) with E homogeneous of degree -1 in lengths)
        np.testing.assert_allclose(Xi, -E / 6.0 * np.eye(3), atol=1e-8 * abs(E))


@pytest.mark.parametrize("box,net", [
    ((1.2, 1.3, 1.4), 0.0),
    ((1.2, 1.3, 1.4), 0.7),
    (np.array([[1.3, 0.0, 0.0], [0.3, 1.25, 0.0], [-0.2, 0.35, 1.35]]), 0.0),
])
def test_total_independent_of_beta(box, net, pm=PM):
    x, q = _random_charges(40, box, 11, net)
    rc = 0.56
    E1, F1, X1 = _total(x, q, box, 5.2 / rc, rc, 26, pm)
    E2, F2, X2 = _total(x, q, box, 6.0 / rc, rc, 30, pm)
    assert E1 == pytest.approx(E2, rel=1e-9, abs=1e-7)
    scale = np.abs(F1).max()
    np.testing.assert_allclose(F1, F2, atol=1e-8 * scale)
    np.testing.assert_allclose(X1, X2, atol=1e-8 * abs(E1) + 1e-7)


def test_recip_forces_and_virial_are_energy_derivatives(pm=PM):
    L = np.array([[1.1, 0.0, 0.0], [0.2, 1.0, 0.0], [0.15, -0.25, 1.2]])
    x, q = _random_charges(12, L, 5, 0.3)
    beta, kmax = 3.0, 7
    E, F, Xi = pm.ewald_recip(x, q, L, beta, kmax)
    h = 1e-6
    for i in (0, 5, 11):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd = -(pm.ewald_recip(xp, q, L, beta, kmax)[0] - pm.ewald_recip(xm, q, L, beta, kmax)[0]) / (2 * h)
            assert F[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    # affine strain of box and positions: 1/2 dE/d(strain) = Xi
    for a_, b_ in ((0, 0), (1, 2), (0, 1), (2, 2)):
        e = np.zeros((3, 3))
        e[a_, b_] += 0.5
        e[b_, a_] += 0.5
        T = lambda d: np.eye(3) + d * e
        Ep = pm.ewald_recip(x @ T(h).T, q, L @ T(h).T, beta, kmax)[0]
        Em = pm.ewald_recip(x @ T(-h).T, q, L @ T(-h).T, beta, kmax)[0]
        dEde = (Ep - Em) / (2 * h)
        assert Xi[a_, b_] == pytest.approx(0.5 * dEde, rel=1e-6, abs=1e-6)


# ---- smooth PME ------------------------------------------------------------
def test_pme_converges_to_direct_sum(pm=PM):
    L = np.array([[1.6, 0.0, 0.0], [0.3, 1.5, 0.0], [-0.25, 0.4, 1.7]])
    x, q = _random_charges(60, L, 8, 0.0)
    beta = 3.2
    E0, F0, X0 = pm.ewald_recip(x, q, L, beta, 14)
    errs = []
    for K in (12, 24):
        E, F, Xi = pm.pme_recip(x, q, L, beta, (K, K + 2, K + 4), order=4)
        errs.append(np.sqrt(np.mean((F - F0) ** 2)) / np.sqrt(np.mean(F0 ** 2)))
    # order-4 interpolation: the force error falls by about 2^4 when the spacing halves
    assert errs[1] < errs[0] / 8
    E, F, Xi = pm.pme_recip(x, q, L, beta, (48, 44, 50), order=6)
    assert E == pytest.approx(E0, rel=2e-7)
    np.testing.assert_allclose(F, F0, atol=2e-6 * np.abs(F0).max())
    np.testing.assert_allclose(Xi, X0, atol=2e-6 * abs(E0))


def test_pme_forces_and_virial_are_its_energy_derivatives(pm=PM):
    L = np.array([[1.0, 0.0, 0.0], [-0.2, 1.1, 0.0], [0.3, 0.1, 0.9]])
    x, q = _random_charges(10, L, 21, -0.4)
    beta, grid = 3.0, (10, 12, 9)
    E, F, Xi = pm.pme_recip(x, q, L, beta, grid, order=4)
    h = 1e-6
    for i in (0, 3, 9):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd = -(pm.pme_recip(xp, q, L, beta, grid)[0] - pm.pme_recip(xm, q, L, beta, grid)[0]) / (2 * h)
            assert F[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    for a_, b_ in ((0, 0), (1, 1), (0, 2), (1, 2)):
        e = np.zeros((3, 3))
        e[a_, b_] += 0.5
        e[b_, a_] += 0.5
        T = lambda d: np.eye(3) + d * e
        Ep = pm.pme_recip(x @ T(h).T, q, L @ T(h).T, beta, grid)[0]
        Em = pm.pme_recip(x @ T(-h).T, q, L @ T(-h).T, beta, grid)[0]
        assert Xi[a_, b_] == pytest.approx(0.5 * (Ep - Em) / (2 * h), rel=1e-6, abs=1e-6)


def test_pme_translation_by_a_grid_vector_is_exact(pm=PM):
    # moving every charge by one grid spacing along a lattice vector moves the
    # charge grid by one point: energy and forces are unchanged up to rounding
    L = np.array([[1.2, 0.0, 0.0], [0.25, 1.3, 0.0], [0.1, -0.3, 1.1]])
    x, q = _random_charges(30, L, 3, 0.0)
    grid = (12, 13, 11)
    E, F, _ = pm.pme_recip(x, q, L, 3.1, grid)
    for k in range(3):
        E2, F2, _ = pm.pme_recip(x + L[k] / grid[k], q, L, 3.1, grid)
        assert E2 == pytest.approx(E, rel=1e-12)
        np.testing.assert_allclose(F2, F, atol=1e-10 * np.abs(F).max())


# ---- planted mistakes ------------------------------------------------------
# (name, text in oracle/pme.py, replacement): each is loaded as a module of its
# own and must fail at least one of the pins above
PME_MUTANTS = [
    ("recip force factor 2 dropped", "F -= (2.0 * fel / V)", "F -= (fel / V)"),
    ("recip energy 1/(2 pi V) -> 1/(pi V)", "Em = fel / (2.0 * math.pi * V) * g * S2",
     "Em = fel / (math.pi * V) * g * S2"),
    ("gaussian exponent pi for pi^2", "g = np.exp(-math.pi ** 2 * m2 / beta ** 2) / m2",
     "g = np.exp(-math.pi * m2 / beta ** 2) / m2"),
    ("reciprocal vectors not transposed", "return np.linalg.inv(L).T", "return np.linalg.inv(L)"),
    ("self term sign", "return -F_COUL / eps_r * beta / math.sqrt(math.pi)", "return F_COUL / eps_r * beta / math.sqrt(math.pi)"),
    ("background factor 2", "math.pi * Q * Q / (2.0 * V * beta * beta)", "math.pi * Q * Q / (V * beta * beta)"),
    ("background virial dropped", "return E, -0.5 * E * np.eye(3)", "return E, 0.0 * np.eye(3)"),
    ("recip virial 1 + dropped", "w = Em * 2.0 * (1.0 + math.pi ** 2 * m2 / beta ** 2) / m2",
     "w = Em * 2.0 * (math.pi ** 2 * m2 / beta ** 2) / m2"),
    ("recip force cos/sin swapped", "t = (im[None, :] * c - re[None, :] * s)", "t = (re[None, :] * c - im[None, :] * s)"),
    ("bspline recursion (n - u) -> (n - 1 - u)", "out[:, j] = (u * here + (n - u) * left) / (n - 1)",
     "out[:, j] = (u * here + (n - 1 - u) * left) / (n - 1)"),
    ("bspline derivative sign", "D[:, j] = (Ap[:, j] if j < p - 1 else 0.0) - (Ap[:, j - 1] if j >= 1 else 0.0)",
     "D[:, j] = (Ap[:, j - 1] if j >= 1 else 0.0) - (Ap[:, j] if j < p - 1 else 0.0)"),
    ("spread to base + j", "idx.append((base[:, k][:, None] - np.arange(p)[None, :]) % K[k])",
     "idx.append((base[:, k][:, None] + np.arange(p)[None, :]) % K[k])"),
    ("moduli dropped", "/ (math.pi * V * m2) * B", "/ (math.pi * V * m2)"),
    ("moduli modulus not squared", "out[m] = 1.0 / abs(den) ** 2", "out[m] = 1.0 / abs(den)"),
    ("pme force grid scale dropped", "A[0][:, a] * A[1][:, b] * D[2][:, c]], 1) * Kf[None, :]",
     "A[0][:, a] * A[1][:, b] * D[2][:, c]], 1)"),
    ("pme force reciprocal transposed", "F -= fel * (q * cv)[:, None] * (du @ R)", "F -= fel * (q * cv)[:, None] * (du @ R.T)"),
    ("pme energy factor 1/2 dropped", "Em = 0.5 * fel * G * np.abs(FQ) ** 2", "Em = fel * G * np.abs(FQ) ** 2"),
    ("pme convolution normalisation", "conv = np.real(np.fft.ifftn(FQ * G)) * Q.size", "conv = np.real(np.fft.ifftn(FQ * G))"),
    ("pme virial sign", "Xi = -0.5 * (E * np.eye(3) - np.einsum", "Xi = -0.5 * (E * np.eye(3) + np.einsum"),
    ("pme frequencies unsigned", "h = [np.fft.fftfreq(K[k]) * K[k] for k in range(3)]",
     "h = [np.arange(K[k]) * 1.0 for k in range(3)]"),
]

_PINS = [
    (test_bspline_order4_closed_form, ()),
    (test_bspline_partition_symmetry_derivative, (4,)),
    (test_bspline_partition_symmetry_derivative, (5,)),
    (test_moduli_order4_closed_form, (25,)),
    (test_recip_forces_and_virial_are_energy_derivatives, ()),
    (test_madelung_constant_rock_salt, ()),
    (test_total_independent_of_beta, ((1.2, 1.3, 1.4), 0.7)),
    (test_pme_forces_and_virial_are_its_energy_derivatives, ()),
    (test_pme_converges_to_direct_sum, ()),
    (test_pme_translation_by_a_grid_vector_is_exact, ()),
]


@pytest.mark.parametrize("name,old,new", PME_MUTANTS, ids=[m[0] for m in PME_MUTANTS])
def test_pme_pins_catch_planted_mistake(name, old, new):
    import types
    src = open(PM.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("pme_mutant")
    exec(compile(src.replace(old, new), "pme_mutant", "exec"), mod.__dict__)
    for pin, args in _PINS:
        try:
            pin(*args, pm=mod)
        except Exception:
            return
    pytest.fail("no pin caught the planted mistake: " + name)
