"""Seeded synthetic inputs for the short-range non-bonded workloads.

This module only draws numbers: lattice sites, jitter, charges, Lennard-Jones
parameters, masses, Maxwell velocities, ensemble sizes and job arrival times.
It holds none of the method's arithmetic (no distances, pair tests, forces or
integration), so the FP64 oracle and the GPU library can both be fed from it
without sharing any computation.

The paper gives no benchmark inputs of its own (its systems are production
biomolecules, Section "Heterogeneous parallelization", Figs. 6-7); the
workloads here are synthetic stand-ins of the same scale (24k atoms as in the
RNAse box of Fig. 3/Fig. 6, up to 1M atoms, ensembles as in Section
"Ensemble simulations").  Every draw uses numpy's PCG64 ``default_rng`` and a
fixed draw order: sizes, then positions, then charges/LJ parameters, then
velocities.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Boltzmann constant in kJ mol^-1 K^-1 (units: nm, ps, amu, kJ/mol, e, K).
KB = 0.00831446261815324

# Model constants shared by every lattice workload: sigma 0.30 nm, epsilon
# 0.5 kJ/mol, charges +/-0.4 e, mass 16 amu, temperature 300 K.
SIGMA = 0.30
EPSILON = 0.5
CHARGE = 0.4
MASS = 16.0
TEMPERATURE = 300.0
JITTER = 0.05


@dataclasses.dataclass
class Model:
    """Interaction model of one workload (all lengths in nm)."""

    r_cut: float
    r_list: float
    coulomb: str  # "none" | "rf" | "ewald"
    eps_r: float = 1.0
    eps_rf: float = 0.0  # <= 0 means infinity
    ewald_beta: float = 0.0
    lj: str = "single"  # "single" | "lb"
    pot_shift: bool = True
    sigma: float = SIGMA
    epsilon: float = EPSILON
    # reciprocal-space Ewald by PME: grid points along a, b, c (None: off) and
    # the B-spline order
    pme_grid: Optional[Sequence[int]] = None
    pme_order: int = 4

    @property
    def c6(self) -> float:
        return 4.0 * self.epsilon * self.sigma ** 6

    @property
    def c12(self) -> float:
        return 4.0 * self.epsilon * self.sigma ** 12


@dataclasses.dataclass
class System:
    """One periodic rectangular system (FP64 host arrays)."""

    box: np.ndarray  # (3,)
    x: np.ndarray  # (N, 3), wrapped into [0, L)
    q: np.ndarray  # (N,)
    sigma: np.ndarray  # (N,)
    epsilon: np.ndarray  # (N,)
    mass: np.ndarray  # (N,)
    model: Model
    v: Optional[np.ndarray] = None  # (N, 3)
    seed: object = None
    # off-diagonal b_x, c_x, c_y of a lower-triangular (triclinic) box with
    # lattice vectors a = (box[0], 0, 0), b = (b_x, box[1], 0),
    # c = (c_x, c_y, box[2]); None: rectangular
    box_off: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


# ---------------------------------------------------------------------------
# Models of the five workloads
# ---------------------------------------------------------------------------
MODEL_RF = Model(r_cut=0.9, r_list=1.0, coulomb="rf", eps_rf=0.0)
MODEL_EWALD = Model(r_cut=1.0, r_list=1.1, coulomb="ewald", ewald_beta=3.12)
MODEL_EWALD_LB = Model(r_cut=1.0, r_list=1.1, coulomb="ewald", ewald_beta=3.12, lj="lb")
MODEL_RF_LB = Model(r_cut=1.0, r_list=1.1, coulomb="rf", eps_rf=0.0, lj="lb")


def lattice_edge(n_atoms: int) -> int:
    """Smallest n with n**3 >= n_atoms (integer arithmetic, no cube-root rounding)."""
    n = max(1, int(round(n_atoms ** (1.0 / 3.0))) - 1)
    while n ** 3 < n_atoms:
        n += 1
    return n


def _wrap(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    x = np.mod(x, box)
    # np.mod of a tiny negative number can round up to exactly L.
    x = np.where(x >= box, x - box, x)
    return x


def _lattice_positions(rng, n_atoms: int, box: float, jitter: float = JITTER) -> np.ndarray:
    """First n_atoms sites of an n^3 cubic lattice (site s = ix + n*iy + n^2*iz at
    ((ix+1/2)a, (iy+1/2)a, (iz+1/2)a)), plus i.i.d. U(-jitter, jitter) per
    coordinate drawn atom-major / xyz-minor, wrapped into [0, L)."""
    n = lattice_edge(n_atoms)
    a = box / n
    s = np.arange(n_atoms, dtype=np.int64)
    ix, iy, iz = s % n, (s // n) % n, s // (n * n)
    x = np.stack([(ix + 0.5) * a, (iy + 0.5) * a, (iz + 0.5) * a], axis=1)
    if jitter > 0.0:
        x = x + rng.uniform(-jitter, jitter, size=(n_atoms, 3))
    return _wrap(x, np.full(3, box))


def alternating_charges(n_atoms: int, charge: float = CHARGE) -> np.ndarray:
    q = np.full(n_atoms, charge)
    q[1::2] = -charge
    return q


def maxwell_velocities(rng, mass: np.ndarray, temperature: float = TEMPERATURE) -> np.ndarray:
    """Gaussian velocities at T, centre-of-mass velocity removed, rescaled so that
    the kinetic energy is exactly (3N-3)/2 k_B T."""
    n = mass.shape[0]
    sd = np.sqrt(KB * temperature / mass)
    v = rng.normal(0.0, 1.0, size=(n, 3)) * sd[:, None]
    vcom = (mass[:, None] * v).sum(axis=0) / mass.sum()
    v = v - vcom
    ke = 0.5 * float((mass[:, None] * v * v).sum())
    target = 0.5 * (3 * n - 3) * KB * temperature
    return v * math.sqrt(target / ke)


def lattice_system(n_atoms: int, box: float, seed, model: Model = MODEL_RF,
                   velocities: bool = False, jitter: float = JITTER) -> System:
    rng = np.random.default_rng(seed)
    x = _lattice_positions(rng, n_atoms, box, jitter)
    q = alternating_charges(n_atoms)
    sig = np.full(n_atoms, model.sigma)
    eps = np.full(n_atoms, model.epsilon)
    m = np.full(n_atoms, MASS)
    v = maxwell_velocities(rng, m) if velocities else None
    return System(box=np.full(3, float(box)), x=x, q=q, sigma=sig, epsilon=eps,
                  mass=m, model=model, v=v, seed=seed)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
def small_rf(velocities: bool = False) -> System:
    """2,700 atoms, cubic 3.0 nm box, RF eps_rf = inf, rc 0.9, rlist 1.0, seed 1."""
    return lattice_system(2700, 3.0, 1, MODEL_RF, velocities)


def dynamics_ewald(velocities: bool = True) -> System:
    """24,000 atoms, cubic 6.2 nm box, Ewald real space beta 3.12, rc 1.0,
    rlist 1.1, 16 amu, Maxwell 300 K, seed 2."""
    return lattice_system(24000, 6.2, 2, MODEL_EWALD, velocities)


def slab_system(n_atoms: int = 1_000_000, box: float = 21.5, seed=3,
                model: Model = MODEL_EWALD_LB) -> System:
    """Dense central slab z in [0.35L, 0.65L) at 1.5x the bulk density (30% of the
    volume), bulk elsewhere; sigma ~ U(0.25, 0.35), epsilon ~ U(0.2, 1.0),
    q ~ N(0, 0.3) shifted to zero net charge.  Each region is a jittered cubic
    lattice with N_R sites chosen without replacement."""
    rng = np.random.default_rng(seed)
    vol = box ** 3
    rho_b = n_atoms / (1.15 * vol)
    n_slab = int(round(1.5 * rho_b * 0.3 * vol))
    n_bulk = n_atoms - n_slab
    parts = []
    for (z0, h, nr) in ((0.35 * box, 0.3 * box, n_slab), (0.65 * box, 0.7 * box, n_bulk)):
        spacing = (box * box * h / nr) ** (1.0 / 3.0)
        nx = int(math.ceil(box / spacing))
        nz = int(math.ceil(h / spacing))
        ax, az = box / nx, h / nz
        n_sites = nx * nx * nz
        pick = np.sort(rng.choice(n_sites, size=nr, replace=False))
        ix, iy, iz = pick % nx, (pick // nx) % nx, pick // (nx * nx)
        xr = np.stack([(ix + 0.5) * ax, (iy + 0.5) * ax, z0 + (iz + 0.5) * az], axis=1)
        xr = xr + rng.uniform(-JITTER, JITTER, size=(nr, 3))
        parts.append(xr)
    x = _wrap(np.concatenate(parts, axis=0), np.full(3, box))
    sig = rng.uniform(0.25, 0.35, size=n_atoms)
    eps = rng.uniform(0.2, 1.0, size=n_atoms)
    q = rng.normal(0.0, 0.3, size=n_atoms)
    q = q - q.mean()
    m = np.full(n_atoms, MASS)
    return System(box=np.full(3, float(box)), x=x, q=q, sigma=sig, epsilon=eps,
                  mass=m, model=model, v=None, seed=seed)


def _even(v: float) -> int:
    return int(2 * round(v / 2.0))


def ensemble_sizes(n_systems: int = 512, lo: int = 1000, hi: int = 30000, seed: int = 4) -> List[int]:
    """Atom counts log-uniform in [lo, hi], rounded to the nearest even number."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_systems)
    return [_even(math.exp(t)) for t in u]


def ensemble_member(k: int, n_atoms: int, density: float = 100.0, seed: int = 4,
                    model: Model = MODEL_RF) -> System:
    """System k of the batched ensemble: L = (N/density)^(1/3), seed (seed, k)."""
    box = (n_atoms / density) ** (1.0 / 3.0)
    return lattice_system(n_atoms, box, [seed, k], model, velocities=True)


def ensemble(n_systems: int = 512, lo: int = 1000, hi: int = 30000, seed: int = 4) -> List[System]:
    return [ensemble_member(k, n, seed=seed) for k, n in enumerate(ensemble_sizes(n_systems, lo, hi, seed))]


@dataclasses.dataclass
class Job:
    job_id: int
    arrival: float  # seconds after the start of the trace
    n_atoms: int
    n_steps: int


def job_trace(n_jobs: int, rate: float, lo: int = 2000, hi: int = 200000,
              steps_lo: int = 100, steps_hi: int = 5000, seed: int = 5) -> List[Job]:
    """Poisson arrivals at `rate` jobs/s; sizes log-uniform in [lo, hi] (even);
    step counts uniform in {steps_lo..steps_hi}."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=n_jobs)
    steps = rng.integers(steps_lo, steps_hi + 1, size=n_jobs)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    t = np.cumsum(gaps) - gaps[0]
    return [Job(j, float(t[j]), _even(math.exp(u[j])), int(steps[j])) for j in range(n_jobs)]


def job_system(job: Job, density: float = 100.0, seed: int = 5) -> System:
    box = (job.n_atoms / density) ** (1.0 / 3.0)
    return lattice_system(job.n_atoms, box, [seed, job.job_id], MODEL_RF, velocities=True)


# ---------------------------------------------------------------------------
# Triclinic boxes (the paper also runs a rhombic dodecahedron, Fig. 6)
# ---------------------------------------------------------------------------
def dodecahedron_box(d: float):
    """Rhombic dodecahedron with image distance d (xy-square orientation):
    a = (d, 0, 0), b = (0, d, 0), c = (d/2, d/2, d/sqrt(2)); volume d^3/sqrt(2).
    Returns (diagonal, off-diagonal b_x, c_x, c_y)."""
    return (np.array([d, d, d / math.sqrt(2.0)]), np.array([0.0, 0.5 * d, 0.5 * d]))


def _lattice_matrix(box, box_off) -> np.ndarray:
    """Rows a, b, c of a lower-triangular box."""
    return np.array([[box[0], 0.0, 0.0], [box_off[0], box[1], 0.0], [box_off[1], box_off[2], box[2]]])


def triclinic_lattice_system(n_side: int, box, box_off, seed, model: Model = MODEL_EWALD,
                             n_atoms: Optional[int] = None, velocities: bool = False,
                             jitter: float = JITTER) -> System:
    """Sites (i + 1/2) a/n + (j + 1/2) b/n + (k + 1/2) c/n of the box's own
    lattice subdivided n times per vector (so the lattice is periodic in the
    triclinic box; for the dodecahedron it is face-centred cubic), the first
    n_atoms of them in (i + n j + n^2 k) order, plus i.i.d. U(-jitter, jitter)
    per coordinate; charges alternate +/-0.4, model sigma/epsilon, 16 amu."""
    rng = np.random.default_rng(seed)
    n = int(n_side)
    n_atoms = n ** 3 if n_atoms is None else int(n_atoms)
    s = np.arange(n_atoms, dtype=np.int64)
    frac = np.stack([(s % n + 0.5) / n, ((s // n) % n + 0.5) / n, (s // (n * n) + 0.5) / n], axis=1)
    box = np.asarray(box, dtype=np.float64)
    box_off = np.asarray(box_off, dtype=np.float64)
    x = frac @ _lattice_matrix(box, box_off)
    if jitter > 0.0:
        x = x + rng.uniform(-jitter, jitter, size=(n_atoms, 3))
    q = alternating_charges(n_atoms)
    sig = np.full(n_atoms, model.sigma)
    eps = np.full(n_atoms, model.epsilon)
    m = np.full(n_atoms, MASS)
    v = maxwell_velocities(rng, m) if velocities else None
    return System(box=box, x=x, q=q, sigma=sig, epsilon=eps, mass=m, model=model, v=v, seed=seed,
                  box_off=box_off)


def dodecahedron_ewald(velocities: bool = True) -> System:
    """16,800 atoms in a rhombic dodecahedron with the 6.2 nm image distance of
    the 24,000-atom cubic workload (volume 168.5 nm^3, 99.7 atoms/nm^3), its
    Ewald model, seed 7: the rectangular / dodecahedron pair of the paper's
    Fig. 6 (24k and 16.8k atoms)."""
    box, off = dodecahedron_box(6.2)
    return triclinic_lattice_system(26, box, off, 7, MODEL_EWALD, n_atoms=16800, velocities=velocities)


def random_triclinic_system(n_atoms: int, box, box_off, seed, model: Model) -> System:
    """Uniform random fractional coordinates in a triclinic box (no minimum
    distance: for pair-set tests), charges, LB parameters as tiny_random_system."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    box_off = np.asarray(box_off, dtype=np.float64)
    x = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) @ _lattice_matrix(box, box_off)
    q = 0.4 * np.where(rng.uniform(size=n_atoms) < 0.5, 1.0, -1.0)
    q = q - q.mean()
    sig = rng.uniform(0.25, 0.35, size=n_atoms)
    eps = rng.uniform(0.2, 1.0, size=n_atoms)
    m = np.full(n_atoms, MASS)
    return System(box=box, x=x, q=q, sigma=sig, epsilon=eps, mass=m, model=model, seed=seed, box_off=box_off)


def tiny_random_system(n_atoms: int, box: Sequence[float], seed, model: Model,
                       charge_scale: float = 0.4, min_dist: float = 0.0) -> System:
    """Uniform random positions (optionally with a minimum pair distance enforced by
    rejection), random +/- charges with zero net charge, per-atom sigma/epsilon
    spread around the model's values.  For small test systems only."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < n_atoms:
        p = rng.uniform(0.0, 1.0, size=3) * box
        tries += 1
        if min_dist > 0.0 and pts:
            arr = np.asarray(pts)
            d = arr - p
            d -= np.round(d / box) * box
            if np.min((d * d).sum(axis=1)) < min_dist * min_dist:
                if tries > 200000:
                    raise RuntimeError("cannot place atoms at this density")
                continue
        pts.append(p)
    x = _wrap(np.asarray(pts), box)
    q = charge_scale * np.where(rng.uniform(size=n_atoms) < 0.5, 1.0, -1.0)
    q = q - q.mean()
    sig = rng.uniform(0.25, 0.35, size=n_atoms)
    eps = rng.uniform(0.2, 1.0, size=n_atoms)
    m = np.full(n_atoms, MASS)
    return System(box=box, x=x, q=q, sigma=sig, epsilon=eps, mass=m, model=model, seed=seed)
