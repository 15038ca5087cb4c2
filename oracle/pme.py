"""FP64 reference for the reciprocal-space half of Ewald electrostatics.

TEST INFRASTRUCTURE ONLY, like the rest of this package: imported by the tests
and by the checks of the benchmark, never by the product library.

The paper splits electrostatics into the short-range pair part that the
cluster-pair kernel computes and a long-range lattice part done by
particle-mesh Ewald (PME): a 3D FFT on a charge grid (Section "Multi-level
parallelism" and Fig. 2; Section "Heterogeneous parallelization", where the CPU
does the lattice summation while the GPU does the pair forces).  The paper does
not restate the PME equations; they are those of smooth PME (Essmann et al.,
J. Chem. Phys. 103, 8577, 1995), which the paper's PME refers to.

Box: lattice vectors a, b, c are the rows of a 3x3 matrix L (the library's
boxes are lower triangular: a = (a_x,0,0), b = (b_x,b_y,0), c = (c_x,c_y,c_z)).
Reciprocal vectors a*, b*, c* are the rows of inv(L)^T, V = |det L|,
f = 138.935458 kJ mol^-1 nm e^-2 / eps_r, beta the splitting parameter (the
real-space pair term is f q_i q_j erfc(beta r)/r).  Virial convention as in the
pair code: Xi = -1/2 sum_pairs r_ij (x) F_ij, which equals 1/2 dE/d(strain).

Functions
  ewald_recip   the reciprocal-space energy by its definition, the direct sum
                over reciprocal lattice vectors m = h0 a* + h1 b* + h2 c*,
                0 < max|h_k| <= kmax:
                    E = f/(2 pi V) sum_m exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2,
                    S(m) = sum_j q_j exp(2 pi i m.r_j),
                with F_i = -dE/dr_i and the virial in closed form.
  ewald_self, ewald_background
                the constant self term -f beta/sqrt(pi) sum q^2 and, for a
                non-neutral box, the uniform neutralising background
                -f pi (sum q)^2 / (2 V beta^2) (with its virial).
  bspline       cardinal B-spline weights M_p(w + j), j = 0..p-1, and their
                derivatives, from the recursion that defines M_p.
  bspline_moduli  |b(m)|^2 of the exponential-spline interpolation.
  pme_recip     smooth PME: spread, FFT, influence function (left out at the
                Nyquist frequency of an even grid dimension), inverse FFT,
                gather with analytic spline derivatives.
"""
from __future__ import annotations

import math

import numpy as np

F_COUL = 138.935458


def box_matrix(box, box_off=None):
    """3x3 matrix of lattice rows from a diagonal (3,) and off-diagonals
    (b_x, c_x, c_y), or a 3x3 matrix passed through."""
    box = np.asarray(box, dtype=np.float64)
    if box.shape == (3, 3):
        return box.copy()
    off = np.zeros(3) if box_off is None else np.asarray(box_off, dtype=np.float64)
    return np.array([[box[0], 0.0, 0.0], [off[0], box[1], 0.0], [off[1], off[2], box[2]]])


def recip_matrix(L):
    """Rows a*, b*, c* with (row i of L) . (row j of the result) = delta_ij."""
    return np.linalg.inv(L).T


def ewald_self(q, beta, eps_r=1.0):
    """Self energy of the Gaussian screening charges (no force, no virial)."""
    q = np.asarray(q, dtype=np.float64)
    return -F_COUL / eps_r * beta / math.sqrt(math.pi) * float(np.sum(q * q))


def ewald_background(q, beta, L, eps_r=1.0):
    """(E, Xi) of the uniform background that neutralises a net charge."""
    V = abs(np.linalg.det(L))
    Q = float(np.sum(q))
    E = -F_COUL / eps_r * math.pi * Q * Q / (2.0 * V * beta * beta)
    # E scales as 1/V, so dE/d(strain_ab) = -E delta_ab
    return E, -0.5 * E * np.eye(3)


def ewald_recip(x, q, L, beta, kmax, eps_r=1.0):
    """(E, F [N,3], Xi [3,3]) of the reciprocal-space sum, term by term."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    L = box_matrix(L)
    R = recip_matrix(L)
    V = abs(np.linalg.det(L))
    fel = F_COUL / eps_r
    h = np.arange(-kmax, kmax + 1)
    H = np.stack(np.meshgrid(h, h, h, indexing="ij"), -1).reshape(-1, 3)
    H = H[np.any(H != 0, axis=1)]
    E = 0.0
    F = np.zeros_like(x)
    Xi = np.zeros((3, 3))
    for b0 in range(0, H.shape[0], 2048):
        m = H[b0:b0 + 2048].astype(np.float64) @ R  # [K,3]
        m2 = np.sum(m * m, axis=1)
        g = np.exp(-math.pi ** 2 * m2 / beta ** 2) / m2
        ph = 2.0 * math.pi * (x @ m.T)  # [N,K]
        c, s = np.cos(ph), np.sin(ph)
        re, im = q @ c, q @ s  # S(m) = re + i im
        S2 = re * re + im * im
        Em = fel / (2.0 * math.pi * V) * g * S2
        E += float(np.sum(Em))
        # d|S|^2/dr_i = 2 Re(conj(S) dS/dr_i), dS/dr_i = 2 pi i q_i m exp(i ph_i)
        #             = 4 pi q_i m (im cos ph_i - re sin ph_i)
        t = (im[None, :] * c - re[None, :] * s) * g[None, :]
        F -= (2.0 * fel / V) * q[:, None] * (t @ m)
        # under strain: V -> V (1 + tr e), m -> (1 - e^T) m, m.r unchanged, so
        # dE_m/de_ab = -E_m (delta_ab - 2 (1 + pi^2 m^2/beta^2) m_a m_b / m^2)
        w = Em * 2.0 * (1.0 + math.pi ** 2 * m2 / beta ** 2) / m2
        Xi += -0.5 * (float(np.sum(Em)) * np.eye(3) - (m * w[:, None]).T @ m)
    return E, F, Xi


# ---- smooth PME ------------------------------------------------------------
def bspline(w, p):
    """Weights A[:, j] = M_p(w + j) and derivatives D[:, j] = M_p'(w + j) for
    j = 0..p-1 and w in [0, 1), from M_2(u) = 1 - |u - 1| on [0, 2] and
        M_n(u) = (u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)) / (n - 1),
        M_n'(u) = M_{n-1}(u) - M_{n-1}(u - 1)."""
    w = np.asarray(w, dtype=np.float64)

    def M(n):
        """[N, n] array of M_n(w + j), j = 0..n-1 (zero outside the support)."""
        if n == 2:
            return np.stack([w, 1.0 - w], 1)
        prev = M(n - 1)
        out = np.zeros((w.shape[0], n))
        for j in range(n):
            u = w + j
            here = prev[:, j] if j < n - 1 else 0.0  # M_{n-1}(u)
            left = prev[:, j - 1] if j >= 1 else 0.0  # M_{n-1}(u - 1)
            out[:, j] = (u * here + (n - u) * left) / (n - 1)
        return out

    if p < 3:
        raise ValueError("spline order must be at least 3")
    A = M(p)
    Ap = M(p - 1)
    D = np.zeros_like(A)
    for j in range(p):
        D[:, j] = (Ap[:, j] if j < p - 1 else 0.0) - (Ap[:, j - 1] if j >= 1 else 0.0)
    return A, D


def bspline_moduli(K, p):
    """|b(m)|^2 = 1 / |sum_{j=0}^{p-1} M_p(j) exp(2 pi i m j / K)|^2, m = 0..K-1
    (the phase factor of b(m) drops out of the modulus).  Even orders only:
    odd orders have a zero denominator at m = K/2 for even K."""
    if p % 2:
        raise ValueError("even spline orders only")
    Mint, _ = bspline(np.zeros(1), p)  # M_p(0 + j)
    j = np.arange(p)
    out = np.zeros(K)
    for m in range(K):
        den = np.sum(Mint[0] * np.exp(2j * math.pi * m * j / K))
        out[m] = 1.0 / abs(den) ** 2
    return out


def pme_recip(x, q, L, beta, grid, order=4, eps_r=1.0):
    """(E, F [N,3], Xi [3,3]) of smooth PME on a grid[0] x grid[1] x grid[2]
    mesh along a, b, c with B-splines of the given (even) order."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    L = box_matrix(L)
    R = recip_matrix(L)
    V = abs(np.linalg.det(L))
    fel = F_COUL / eps_r
    K = [int(k) for k in grid]
    p = int(order)
    n = x.shape[0]
    # scaled fractional coordinates u_k = K_k (r . a*_k), taken modulo K_k
    u = (x @ R.T) * np.asarray(K, dtype=np.float64)[None, :]
    u = u - np.floor(u / np.asarray(K)[None, :]) * np.asarray(K)[None, :]
    base = np.floor(u).astype(np.int64)
    over = base >= np.asarray(K)[None, :]  # (u rounded up to K)
    base = np.where(over, base - np.asarray(K)[None, :], base)
    u = np.where(over, u - np.asarray(K)[None, :], u)
    w = u - base
    A, D, idx = [], [], []
    for k in range(3):
        a_k, d_k = bspline(w[:, k], p)
        A.append(a_k)
        D.append(d_k)
        # weight M_p(w + j) goes to grid point base - j: there u - point = w + j
        idx.append((base[:, k][:, None] - np.arange(p)[None, :]) % K[k])
    Q = np.zeros(K)
    for a in range(p):
        for b in range(p):
            for c in range(p):
                np.add.at(Q, (idx[0][:, a], idx[1][:, b], idx[2][:, c]), q * A[0][:, a] * A[1][:, b] * A[2][:, c])
    FQ = np.fft.fftn(Q)
    # m for every grid frequency (h in numpy's FFT order: 0..K/2-1, -K/2..-1)
    h = [np.fft.fftfreq(K[k]) * K[k] for k in range(3)]
    H0, H1, H2 = np.meshgrid(h[0], h[1], h[2], indexing="ij")
    m = H0[..., None] * R[0] + H1[..., None] * R[1] + H2[..., None] * R[2]
    m2 = np.sum(m * m, axis=-1)
    m2[0, 0, 0] = 1.0
    B = (bspline_moduli(K[0], p)[:, None, None] * bspline_moduli(K[1], p)[None, :, None]
         * bspline_moduli(K[2], p)[None, None, :])
    G = np.exp(-math.pi ** 2 * m2 / beta ** 2) / (math.pi * V * m2) * B
    G[0, 0, 0] = 0.0
    # the Nyquist frequency h = -K/2 of an even K has no partner +K/2 on the
    # grid, so in a skewed box G(m) would differ from G(-m) there: those
    # planes are left out, which keeps G symmetric (their terms carry
    # exp(-pi^2 m^2/beta^2) at |m| >= K/(2 L) and vanish as the grid is refined)
    for k, ax in enumerate(((slice(None), None, None), (None, slice(None), None), (None, None, slice(None)))):
        if K[k] % 2 == 0:
            nyq = np.zeros(K[k], bool)
            nyq[K[k] // 2] = True
            G = np.where(nyq[ax], 0.0, G)
    Em = 0.5 * fel * G * np.abs(FQ) ** 2
    E = float(np.sum(Em))
    w_vir = Em * 2.0 * (1.0 + math.pi ** 2 * m2 / beta ** 2) / m2
    Xi = -0.5 * (E * np.eye(3) - np.einsum("abcx,abc,abcy->xy", m, w_vir, m))
    # E = 1/2 sum_k Q(k) (theta * Q)(k) with theta the inverse transform of G:
    # conv = N_grid * ifft(G fft(Q)) is that convolution
    conv = np.real(np.fft.ifftn(FQ * G)) * Q.size
    F = np.zeros((n, 3))
    Kf = np.asarray(K, dtype=np.float64)
    for a in range(p):
        for b in range(p):
            for c in range(p):
                cv = conv[idx[0][:, a], idx[1][:, b], idx[2][:, c]]
                # dQ/du_k per unit charge, times du_k/dr = K_k a*_k
                du = np.stack([D[0][:, a] * A[1][:, b] * A[2][:, c],
                               A[0][:, a] * D[1][:, b] * A[2][:, c],
                               A[0][:, a] * A[1][:, b] * D[2][:, c]], 1) * Kf[None, :]
                F -= fel * (q * cv)[:, None] * (du @ R)
    return E, F, Xi


def ewald_total(x, q, L, beta, eps_r=1.0, recip=None):
    """Constant terms plus the given reciprocal part: (E, F, Xi) with E the
    reciprocal + self + background energy (the real-space pair part is
    oracle.forces)."""
    E, F, Xi = recip
    Eb, Xb = ewald_background(q, beta, box_matrix(L), eps_r)
    return E + ewald_self(q, beta, eps_r) + Eb, F, Xi + Xb
