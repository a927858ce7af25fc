"""Python harness for the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loads ``liboracle.so`` (built from ``kubo_oracle.c`` with gcc) through ctypes
and wraps its entry points with numpy arrays.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this module; the
HIP library and its Python binding never do.

Every function follows the definition written at the top of
``kubo_oracle.c``: the Kubo-formula anomalous Hall conductivity of the
paper's Eqs. (2)-(3), evaluated step by step as in its baseline listing
(Bloch sums, Hermitian eigensolve, rotation into the eigenbasis, band-pair
sum), with the Brillouin-zone measure stated under Eq. (1).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kubo_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.oracle_hk.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, _dp, _dp, _dp]
        L.oracle_eigh.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_bands_k.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, ctypes.c_double,
                                     _dp, _dp]
        L.oracle_ahc.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _ip, ctypes.c_long,
                                 ctypes.c_long, ctypes.c_int, _dp, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp, _dp, ctypes.c_int]
        L.oracle_ahc_tensor.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _ip, ctypes.c_long,
                                        ctypes.c_long, ctypes.c_int, _dp, ctypes.c_double,
                                        ctypes.c_double, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.oracle_ahc_gf.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _ip, ctypes.c_long,
                                    ctypes.c_long, ctypes.c_int, _dp, ctypes.c_double,
                                    ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int]
        L.oracle_band_range.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _ip, _dp, _dp,
                                        ctypes.c_int]
        L.oracle_ahc_grad.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _dp, _ip, ctypes.c_long,
                                      ctypes.c_long, ctypes.c_int, _dp, ctypes.c_double,
                                      ctypes.c_double, _dp, _dp, ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, kind):
    return a.ctypes.data_as(kind)


def _model(t, R):
    t = _c(t, np.complex128)
    R = _c(R, np.int32)
    nR, n, n2 = t.shape
    assert n == n2 and R.shape == (nR, 3)
    return t, R, n, nR


def hk(t, R, k):
    """H(k), v_x(k), v_y(k) at a real k (radians): step (1) of the listing."""
    t, R, n, nR = _model(t, R)
    k = _c(k, np.float64)
    H = np.zeros((n, n), np.complex128)
    vx = np.zeros_like(H)
    vy = np.zeros_like(H)
    lib().oracle_hk(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(k, _dp), _ptr(H, _dp),
                    _ptr(vx, _dp), _ptr(vy, _dp))
    return H, vx, vy


def eigh(A):
    """(E ascending, U, sweeps) of a Hermitian matrix by the oracle's Jacobi."""
    A = _c(A, np.complex128)
    n = A.shape[0]
    E = np.zeros(n)
    U = np.zeros((n, n), np.complex128)
    sw = lib().oracle_eigh(n, _ptr(A, _dp), _ptr(E, _dp), _ptr(U, _dp))
    return E, U, sw


def bands_k(t, R, k, eta):
    """(E_n, Omega_n) at one real k, Omega_n the broadened Berry curvature."""
    t, R, n, nR = _model(t, R)
    k = _c(k, np.float64)
    E = np.zeros(n)
    Om = np.zeros(n)
    rc = lib().oracle_bands_k(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(k, _dp), float(eta),
                              _ptr(E, _dp), _ptr(Om, _dp))
    if rc != 0:
        raise RuntimeError("oracle eigensolver did not converge")
    return E, Om


def ahc(t, R, grid, e_fermi, eta, kT, k_begin=0, k_count=None, nthreads=0, with_sabs=False):
    """sigma_xy[j] over a k-slab, normalised by the full grid (Eq. (2)-(3)).

    with_sabs: also return the rounding scale max(S_pair, S_band) per level, where
    S_pair = (1/N_k) sum |pair terms| and S_band = (1/N_k) sum_k sum_n f_n |Omega_n|."""
    t, R, n, nR = _model(t, R)
    grid = _c(grid, np.int32)
    Nk = int(np.prod(grid.astype(np.int64)))
    if k_count is None:
        k_count = Nk - k_begin
    EF = _c(np.atleast_1d(e_fermi), np.float64)
    nF = EF.size
    sig = np.zeros(nF)
    sabs = np.zeros(nF)
    sband = np.zeros(nF)
    rc = lib().oracle_ahc(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(grid, _ip), int(k_begin),
                          int(k_count), nF, _ptr(EF, _dp), float(eta), float(kT), _ptr(sig, _dp),
                          _ptr(sabs, _dp), _ptr(sband, _dp) if with_sabs else None,
                          int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle eigensolver did not converge")
    return (sig, np.maximum(sabs, sband)) if with_sabs else sig


TENSOR_COMPONENTS = ("xy", "yz", "zx", "spin_xy")


def ahc_tensor(t, R, grid, e_fermi, eta, kT, spin=None, k_begin=0, k_count=None, nthreads=0,
               with_sabs=False):
    """[4, nF]: sigma_xy, sigma_yz, sigma_zx and the spin Hall sigma (spin current
    (s v_x + v_x s)/2, field along y; zero when spin is None) over a k-slab, normalised by
    the full grid.  spin: the diagonal of s_z in the orbital basis (length n).
    with_sabs: also return the per-component rounding scale max(S_pair, S_band)."""
    t, R, n, nR = _model(t, R)
    grid = _c(grid, np.int32)
    Nk = int(np.prod(grid.astype(np.int64)))
    if k_count is None:
        k_count = Nk - k_begin
    EF = _c(np.atleast_1d(e_fermi), np.float64)
    nF = EF.size
    sp = None
    if spin is not None:
        sp = _c(spin, np.float64)
        assert sp.shape == (n,)
    sig = np.zeros((4, nF))
    sabs = np.zeros((4, nF))
    sband = np.zeros((4, nF))
    rc = lib().oracle_ahc_tensor(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(grid, _ip), int(k_begin),
                                 int(k_count), nF, _ptr(EF, _dp), float(eta), float(kT),
                                 _ptr(sp, _dp) if sp is not None else None, _ptr(sig, _dp),
                                 _ptr(sabs, _dp), _ptr(sband, _dp) if with_sabs else None,
                                 int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle eigensolver did not converge")
    return (sig, np.maximum(sabs, sband)) if with_sabs else sig


def ahc_gf(t, R, grid, e_fermi, gamma, omega, weight, k_begin=0, k_count=None, nthreads=0,
           with_sabs=False):
    """[nF]: the Green's-function form of sigma_xy (definition at the top of
    kubo_oracle.c) for a constant scattering rate gamma, with the half-line
    w-integral replaced by the caller's nodes `omega` (> 0) and weights `weight`;
    over a k-slab, normalised by the full grid.  with_sabs: also return the
    rounding scale (the same sum of |Tr| terms)."""
    t, R, n, nR = _model(t, R)
    grid = _c(grid, np.int32)
    Nk = int(np.prod(grid.astype(np.int64)))
    if k_count is None:
        k_count = Nk - k_begin
    EF = _c(np.atleast_1d(e_fermi), np.float64)
    om = _c(np.atleast_1d(omega), np.float64)
    wt = _c(np.atleast_1d(weight), np.float64)
    assert om.shape == wt.shape
    sig = np.zeros(EF.size)
    sabs = np.zeros(EF.size)
    rc = lib().oracle_ahc_gf(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(grid, _ip), int(k_begin),
                             int(k_count), EF.size, _ptr(EF, _dp), float(gamma), om.size,
                             _ptr(om, _dp), _ptr(wt, _dp), _ptr(sig, _dp), _ptr(sabs, _dp),
                             int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle: singular matrix in the Green's function")
    return (sig, sabs) if with_sabs else sig


def half_line_rule(m, scale=1.0):
    """Nodes and weights for the integral over w in (0, inf): Gauss-Legendre on
    u in (-1, 1) mapped by w = scale tan(pi (u + 1) / 4)."""
    u, c = np.polynomial.legendre.leggauss(int(m))
    th = 0.25 * np.pi * (u + 1.0)
    return scale * np.tan(th), scale * 0.25 * np.pi * c / np.cos(th) ** 2


def band_range(t, R, grid, nthreads=0):
    """(min, max) eigenvalue of H(k) over a grid."""
    t, R, n, nR = _model(t, R)
    grid = _c(grid, np.int32)
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    rc = lib().oracle_band_range(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(grid, _ip),
                                 ctypes.byref(lo), ctypes.byref(hi), int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle eigensolver did not converge")
    return lo.value, hi.value


def ahc_grad(t, R, grid, e_fermi, eta, kT, sigma_bar, k_begin=0, k_count=None, mode=0,
             nthreads=0):
    """dL/dRe t + i dL/dIm t for L = sum_j sigma_bar_j sigma_j (complex [n_R, n, n])."""
    t, R, n, nR = _model(t, R)
    grid = _c(grid, np.int32)
    Nk = int(np.prod(grid.astype(np.int64)))
    if k_count is None:
        k_count = Nk - k_begin
    EF = _c(np.atleast_1d(e_fermi), np.float64)
    sb = _c(np.atleast_1d(sigma_bar), np.float64)
    assert sb.size == EF.size
    G = np.zeros((nR, n, n), np.complex128)
    rc = lib().oracle_ahc_grad(n, nR, _ptr(R, _ip), _ptr(t, _dp), _ptr(grid, _ip), int(k_begin),
                               int(k_count), EF.size, _ptr(EF, _dp), float(eta), float(kT),
                               _ptr(sb, _dp), _ptr(G, _dp), int(mode), int(nthreads))
    if rc == -2:
        raise ValueError("the gradient needs eta > 0")
    if rc != 0:
        raise RuntimeError("oracle eigensolver did not converge")
    return G
