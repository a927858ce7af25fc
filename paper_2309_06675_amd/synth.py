"""Seeded synthetic tight-binding models (inputs only; no Kubo-formula arithmetic).

This module is shared by the tests, the benchmark and the smoke check, and is
the only code the HIP path and the CPU oracle have in common.  It draws
hopping matrices t(R) and builds the special models used as pins; it never
evaluates a Bloch sum, an eigenproblem or a conductivity.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) mapped to (0, 1) and turned into
normals by the Box-Muller transform, so any language can regenerate the same
models from the seed.

Model recipe (the paper's inputs are Wannier models of bcc Fe that are not
available; these random models of the same structure stand in for them):
  * R runs over the cube {-L..L}^3 in lexicographic order (R_x slowest).
  * For every lexicographically positive R, t(R)_ij = (a + i b) exp(-|R|/lam)
    with a, b independent N(0, 1) and |R| Euclidean; t(-R) = t(R)^+.
  * t(0) = (X + X^+)/2 with X drawn the same way (decay factor 1).
"""

from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """The first ``count`` outputs of splitmix64 started from ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLD
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """Uniform doubles in the open interval (0, 1): ((z >> 11) + 1/2) / 2^53."""
    z = splitmix64(seed, count)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normals(seed: int, count: int) -> np.ndarray:
    """``count`` standard normals; pairs (u1, u2) -> r cos(th), r sin(th)."""
    m = (count + 1) // 2
    u = uniform01(seed, 2 * m)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    out = np.empty(2 * m)
    out[0::2] = r * np.cos(th)
    out[1::2] = r * np.sin(th)
    return out[:count]


@dataclasses.dataclass
class TBModel:
    """A tight-binding model: hoppings t [n_R, n, n] complex128 on lattice vectors R [n_R, 3]."""

    t: np.ndarray
    R: np.ndarray

    @property
    def n(self) -> int:
        return int(self.t.shape[1])

    @property
    def n_R(self) -> int:
        return int(self.t.shape[0])


def cube(L: int) -> np.ndarray:
    """All R in {-L..L}^3, lexicographic (R_x slowest), int32 [(2L+1)^3, 3]."""
    r = np.arange(-L, L + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.int32)


def _lex_positive(R: np.ndarray) -> np.ndarray:
    pos = np.zeros(len(R), bool)
    for i, v in enumerate(R):
        nz = v[v != 0]
        pos[i] = nz.size > 0 and nz[0] > 0
    return pos


def random_model(n: int, L: int, lam: float, seed: int) -> TBModel:
    """Random Hermitian model of the recipe above (complex Gaussian hoppings)."""
    R = cube(L)
    nR = len(R)
    index = {tuple(v): i for i, v in enumerate(R)}
    pos = np.nonzero(_lex_positive(R))[0]
    z = normals(seed, 2 * n * n * (len(pos) + 1))
    z = z.reshape(len(pos) + 1, n, n, 2)
    g = z[..., 0] + 1j * z[..., 1]
    t = np.zeros((nR, n, n), np.complex128)
    for a, i in enumerate(pos):
        d = np.exp(-np.linalg.norm(R[i].astype(float)) / lam)
        t[i] = g[a] * d
        t[index[tuple(-R[i])]] = t[i].conj().T
    x = g[len(pos)]
    t[index[(0, 0, 0)]] = 0.5 * (x + x.conj().T)
    return TBModel(t=t, R=R)


# ---------------------------------------------------------------------------
# Special models used as pins (closed forms and symmetries)
# ---------------------------------------------------------------------------

SX = np.array([[0, 1], [1, 0]], np.complex128)
SY = np.array([[0, -1j], [1j, 0]], np.complex128)
SZ = np.array([[1, 0], [0, -1]], np.complex128)


def qwz_model(u: float) -> TBModel:
    """Qi-Wu-Zhang lattice: H = sin kx sx + sin ky sy + (u + cos kx + cos ky) sz.

    t(0) = u sz, t(+x) = (sz - i sx)/2, t(+y) = (sz - i sy)/2, t(-R) = t(R)^+,
    with R_z = 0 (use a grid with N_z = 1)."""
    R = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0]], np.int32)
    tx = 0.5 * (SZ - 1j * SX)
    ty = 0.5 * (SZ - 1j * SY)
    t = np.stack([u * SZ, tx, tx.conj().T, ty, ty.conj().T])
    return TBModel(t=t, R=R)


def massive_dirac_lattice(m: float) -> TBModel:
    """H = sin kx sx + sin ky sy + m sz (at k = 0 a massive Dirac point)."""
    R = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0]], np.int32)
    tx = -0.5j * SX
    ty = -0.5j * SY
    t = np.stack([m * SZ, tx, tx.conj().T, ty, ty.conj().T])
    return TBModel(t=t, R=R)


def trs_model(n: int, L: int, lam: float, seed: int) -> TBModel:
    """Time-reversal-symmetric model: real t(R) with t(-R) = t(R)^T."""
    m = random_model(n, L, lam, seed)
    R = m.R
    index = {tuple(v): i for i, v in enumerate(R)}
    t = np.zeros_like(m.t)
    for i, v in enumerate(R):
        j = index[tuple(-v)]
        if i <= j:
            re = m.t[i].real.copy()
            if i == j:
                re = 0.5 * (re + re.T)
            t[i] = re
            t[j] = re.T
    return TBModel(t=t, R=R)


def direct_sum(a: TBModel, b: TBModel) -> TBModel:
    """Block-diagonal model t_a (+) t_b on the union of the R-sets."""
    keys: List[tuple] = []
    for v in list(map(tuple, a.R)) + list(map(tuple, b.R)):
        if v not in keys:
            keys.append(v)
    R = np.array(keys, np.int32)
    n = a.n + b.n
    t = np.zeros((len(R), n, n), np.complex128)
    ia = {tuple(v): i for i, v in enumerate(a.R)}
    ib = {tuple(v): i for i, v in enumerate(b.R)}
    for r, v in enumerate(keys):
        if v in ia:
            t[r, : a.n, : a.n] = a.t[ia[v]]
        if v in ib:
            t[r, a.n:, a.n:] = b.t[ib[v]]
    return TBModel(t=t, R=R)


def doubled(a: TBModel) -> TBModel:
    """t (x) I_2: every band exactly doubly degenerate."""
    t = np.einsum("rij,ab->riajb", a.t, np.eye(2)).reshape(a.n_R, 2 * a.n, 2 * a.n)
    return TBModel(t=t, R=a.R.copy())


def random_unitary(n: int, seed: int) -> np.ndarray:
    """A Haar-like unitary from the QR factorisation of a complex Gaussian matrix."""
    z = normals(seed, 2 * n * n).reshape(n, n, 2)
    q, r = np.linalg.qr(z[..., 0] + 1j * z[..., 1])
    d = np.diag(r)
    return q * (d / np.abs(d))


def rotate_orbitals(a: TBModel, W: np.ndarray) -> TBModel:
    """t(R) -> W t(R) W^+ (a change of orbital basis)."""
    return TBModel(t=np.ascontiguousarray(W @ a.t @ W.conj().T), R=a.R.copy())


def qwz_plane_model(u: float, plane: str) -> TBModel:
    """The Qi-Wu-Zhang lattice in the plane (a, b) = "xy", "yz" or "zx": its first axis
    carries the sin k sx hopping, its second the sin k sy one (use N = 1 along the third)."""
    axes = {"xy": (0, 1), "yz": (1, 2), "zx": (2, 0)}[plane]
    base = qwz_model(u)
    R = np.zeros_like(base.R)
    R[:, axes[0]] = base.R[:, 0]
    R[:, axes[1]] = base.R[:, 1]
    return TBModel(t=base.t.copy(), R=R)


def permute_axes(a: TBModel) -> TBModel:
    """Cyclic relabelling of the axes: the new y axis is the old x, new z the old y and new x
    the old z (R' = (R_z, R_x, R_y)); a grid (N0, N1, N2) becomes (N2, N0, N1)."""
    R = a.R[:, [2, 0, 1]].copy()
    return TBModel(t=a.t.copy(), R=R)


def conjugate(a: TBModel) -> TBModel:
    """t(R) -> t(R)*: H(k) -> H(-k)*, the time-reversal partner of a spinless block."""
    return TBModel(t=a.t.conj().copy(), R=a.R.copy())


def spin_qwz_pair(u_up: float, u_dn: float):
    """Spin-up QWZ(u_up) (+) the time-reversal partner of QWZ(u_dn) as the spin-down block,
    with s_z = (+1, +1, -1, -1): (model, spin diagonal)."""
    m = direct_sum(qwz_model(u_up), conjugate(qwz_model(u_dn)))
    return m, np.array([1.0, 1.0, -1.0, -1.0])


def swap_xy(a: TBModel) -> TBModel:
    """Exchange the x and y components of every lattice vector."""
    R = a.R.copy()
    R[:, [0, 1]] = R[:, [1, 0]]
    return TBModel(t=a.t.copy(), R=R)


# ---------------------------------------------------------------------------
# The five benchmark / parity workloads
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Workload:
    name: str
    models: List[TBModel]
    grid: tuple
    n_fermi: int
    eta: float
    kT: float
    eta_adjoint: float | None = None

    @property
    def n_k(self) -> int:
        return int(np.prod(self.grid))


def fermi_levels(emin: float, emax: float, n_fermi: int) -> np.ndarray:
    """n_fermi levels spread evenly over [emin, emax], ends included."""
    if n_fermi == 1:
        return np.array([0.5 * (emin + emax)])
    return np.linspace(emin, emax, n_fermi)


def cfg2_orbital_counts(count: int = 200) -> np.ndarray:
    """n_orb for the batched workload: uniform over {8, 12, ..., 64} (stream seed 2999)."""
    choices = np.arange(8, 65, 4)
    u = uniform01(2999, count)
    return choices[np.minimum((u * len(choices)).astype(int), len(choices) - 1)]


def workload(cfg: int, n_models: int | None = None) -> Workload:
    """Model(s) and parameters of workload ``cfg`` (model seed = 1000 cfg + index)."""
    if cfg == 0:
        return Workload("n8_R125_k20^3_F1_T0", [random_model(8, 2, 1.0, 0)], (20, 20, 20), 1,
                        1e-3, 0.0)
    if cfg == 1:
        return Workload("n32_R343_k100^3_F64_kT0.01", [random_model(32, 3, 1.5, 1000)],
                        (100, 100, 100), 64, 1e-3, 0.01)
    if cfg == 2:
        ns = cfg2_orbital_counts(200)
        if n_models is not None:
            ns = ns[:n_models]
        models = [random_model(int(n), 2, 1.0, 2000 + i) for i, n in enumerate(ns)]
        return Workload("200models_n8-64_R125_k32^3_F16_T0", models, (32, 32, 32), 16, 1e-3, 0.0)
    if cfg == 3:
        return Workload("adjoint_n32_R343_k64^3_F16_kT0.01", [random_model(32, 3, 1.5, 3000)],
                        (64, 64, 64), 16, 1e-2, 0.01, eta_adjoint=1e-2)
    if cfg == 4:
        return Workload("n128_R729_k128^3_F256_kT0.01", [random_model(128, 4, 2.0, 4000)],
                        (128, 128, 128), 256, 1e-3, 0.01, eta_adjoint=1e-2)
    raise ValueError(cfg)


def pack_models(models: Sequence[TBModel]) -> np.ndarray:
    """Concatenate the t arrays of several models, as the C ABI expects (complex128)."""
    return np.concatenate([m.t.reshape(-1) for m in models])
