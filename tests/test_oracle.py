"""Pins for the CPU oracle: closed forms, invariants and brute force (no GPU).

Each test checks the oracle against something other than itself: a closed
form, a symmetry the paper's Eq. (3) implies, a library eigensolver, or a
finite difference.  The paper prints no worked numerical example, so no value
here is copied from it.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from paper_2309_06675_amd import synth as S

# ---------------------------------------------------------------------------
# Eigensolver (listing step 2) against LAPACK
# ---------------------------------------------------------------------------


def _herm(n, seed):
    z = S.normals(seed, 2 * n * n).reshape(n, n, 2)
    x = z[..., 0] + 1j * z[..., 1]
    return 0.5 * (x + x.conj().T)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 33, 150])
def test_jacobi_matches_lapack(oracle, n):
    H = _herm(n, 11 + n)
    E, U, sw = oracle.eigh(H)
    assert sw >= 0
    nrm = np.linalg.norm(H, 2)
    ref = sla.eigh(H, eigvals_only=True)
    assert np.max(np.abs(E - ref)) <= 1e-13 * max(nrm, 1.0)
    assert np.max(np.abs(H @ U - U * E)) <= 1e-13 * max(nrm, 1.0)
    assert np.max(np.abs(U.conj().T @ U - np.eye(n))) <= 1e-13


def test_jacobi_degenerate_and_diagonal(oracle):
    W = S.random_unitary(6, 5)
    lam = np.array([-1.0, -1.0, 0.5, 0.5, 0.5, 2.0])
    H = (W * lam) @ W.conj().T
    E, U, sw = oracle.eigh(H)
    assert sw >= 0
    assert np.allclose(E, np.sort(lam), atol=1e-13)
    assert np.max(np.abs(H @ U - U * E)) <= 1e-13
    D = np.diag([3.0, -2.0, 0.0, 1.0]).astype(complex)
    E, U, sw = oracle.eigh(D)
    assert sw == 0 and np.array_equal(E, [-2.0, 0.0, 1.0, 3.0])
    E, U, sw = oracle.eigh(np.zeros((3, 3), complex))
    assert sw == 0 and np.all(E == 0)


# ---------------------------------------------------------------------------
# Bloch sums (listing step 1)
# ---------------------------------------------------------------------------


def test_qwz_bloch_closed_form(oracle):
    u = 0.7
    m = S.qwz_model(u)
    for seed in range(5):
        kx, ky = (S.uniform01(100 + seed, 2) - 0.5) * 2 * np.pi
        H, vx, vy = oracle.hk(m.t, m.R, [kx, ky, 0.3])
        Hc = np.sin(kx) * S.SX + np.sin(ky) * S.SY + (u + np.cos(kx) + np.cos(ky)) * S.SZ
        vxc = np.cos(kx) * S.SX - np.sin(kx) * S.SZ
        vyc = np.cos(ky) * S.SY - np.sin(ky) * S.SZ
        assert np.allclose(H, Hc, atol=1e-14)
        assert np.allclose(vx, vxc, atol=1e-14)
        assert np.allclose(vy, vyc, atol=1e-14)


def test_velocity_is_k_derivative_and_hermitian(oracle):
    m = S.random_model(5, 2, 1.0, 77)
    k = np.array([0.3, -1.1, 2.0])
    H, vx, vy = oracle.hk(m.t, m.R, k)
    assert np.array_equal(H, H.conj().T)
    h = 1e-5
    for a, v in ((0, vx), (1, vy)):
        dk = np.zeros(3)
        dk[a] = h
        Hp = oracle.hk(m.t, m.R, k + dk)[0]
        Hm = oracle.hk(m.t, m.R, k - dk)[0]
        fd = (Hp - Hm) / (2 * h)
        assert np.max(np.abs(fd - v)) <= 1e-7 * np.max(np.abs(v))


def test_hermitian_projection_of_nonhermitian_input(oracle):
    """A non-Hermitian t enters through H = (Ht + Ht^+)/2, i.e. as its projection."""
    m = S.random_model(4, 1, 1.0, 5)
    z = S.normals(6, 2 * m.t.size).reshape(m.t.shape + (2,))
    junk = 0.3 * (z[..., 0] + 1j * z[..., 1])
    t2 = m.t + junk
    idx = {tuple(v): i for i, v in enumerate(m.R)}
    proj = np.stack([0.5 * (t2[i] + t2[idx[tuple(-v)]].conj().T) for i, v in enumerate(m.R)])
    k = [0.4, 0.9, -0.2]
    a = oracle.hk(t2, m.R, k)
    b = oracle.hk(proj, m.R, k)
    for x, y in zip(a, b):
        assert np.allclose(x, y, atol=1e-13)


# ---------------------------------------------------------------------------
# Per-k integrand (Eq. (3)) against the two-band closed form
# ---------------------------------------------------------------------------


def _d_and_derivs(u, kx, ky):
    d = np.array([np.sin(kx), np.sin(ky), u + np.cos(kx) + np.cos(ky)])
    dx = np.array([np.cos(kx), 0.0, -np.sin(kx)])
    dy = np.array([0.0, np.cos(ky), -np.sin(ky)])
    return d, dx, dy


@pytest.mark.parametrize("eta", [0.0, 1e-3, 0.4])
def test_two_band_curvature_closed_form(oracle, eta):
    u = -0.8
    m = S.qwz_model(u)
    for seed in range(6):
        kx, ky = (S.uniform01(200 + seed, 2) - 0.5) * 2 * np.pi
        E, Om = oracle.bands_k(m.t, m.R, [kx, ky, 0.0], eta)
        d, dx, dy = _d_and_derivs(u, kx, ky)
        nd = np.linalg.norm(d)
        trip = d @ np.cross(dx, dy)
        assert np.isclose(trip, np.cos(kx) + np.cos(ky) + u * np.cos(kx) * np.cos(ky))
        lower = 2.0 * trip / (nd * (4 * nd * nd + eta * eta))
        assert np.allclose(E, [-nd, nd], atol=1e-14)
        assert np.allclose(Om, [lower, -lower], rtol=1e-12, atol=1e-14)


def test_massive_dirac_point(oracle):
    for mass in (0.3, 1.0, -0.5):
        m = S.massive_dirac_lattice(mass)
        E, Om = oracle.bands_k(m.t, m.R, [0.0, 0.0, 0.0], 0.0)
        assert np.isclose(Om[0], np.sign(mass) * 0.5 / mass**2, rtol=1e-13)


@pytest.mark.parametrize("eta", [0.0, 1e-3, 0.5])
def test_curvature_sums_to_zero(oracle, eta):
    m = S.random_model(7, 1, 1.0, 31)
    for seed in range(3):
        k = (S.uniform01(300 + seed, 3) - 0.5) * 2 * np.pi
        E, Om = oracle.bands_k(m.t, m.R, k, eta)
        assert abs(Om.sum()) <= 1e-12 * np.abs(Om).sum()


# ---------------------------------------------------------------------------
# Brillouin-zone sum (Eq. (2)): quantised Chern number of the QWZ lattice
# ---------------------------------------------------------------------------


def _chern(u):
    return 0.5 * (np.sign(u + 2) - 2 * np.sign(u) + np.sign(u - 2))


@pytest.mark.parametrize("u", [-3.0, -1.5, -0.5, 0.5, 1.0, 1.5, 3.0])
def test_qwz_hall_conductivity_is_quantised(oracle, u):
    m = S.qwz_model(u)
    exact = -_chern(u) / (2 * np.pi)
    errs = []
    for N in (12, 24, 48, 96):
        s = oracle.ahc(m.t, m.R, (N, N, 1), [0.0], 0.0, 0.0)[0]
        errs.append(abs(s - exact))
    # the gapped integrand is analytic: the uniform sum converges exponentially
    assert errs[-1] <= 1e-10
    assert errs[1] <= errs[0] + 1e-15 and errs[2] <= errs[1] + 1e-15


def test_qwz_sign_follows_mass(oracle):
    s_pos = oracle.ahc(S.qwz_model(1.0).t, S.qwz_model(1.0).R, (64, 64, 1), [0.0], 0.0, 0.0)[0]
    s_neg = oracle.ahc(S.qwz_model(-1.0).t, S.qwz_model(-1.0).R, (64, 64, 1), [0.0], 0.0, 0.0)[0]
    assert np.isclose(s_pos, 1 / (2 * np.pi), atol=1e-10)
    assert np.isclose(s_neg, -1 / (2 * np.pi), atol=1e-10)


def test_qwz_broadening_shift_is_second_order(oracle):
    m = S.qwz_model(1.0)
    s0 = oracle.ahc(m.t, m.R, (48, 48, 1), [0.0], 0.0, 0.0)[0]
    d1 = abs(oracle.ahc(m.t, m.R, (48, 48, 1), [0.0], 1e-2, 0.0)[0] - s0)
    d2 = abs(oracle.ahc(m.t, m.R, (48, 48, 1), [0.0], 2e-2, 0.0)[0] - s0)
    assert d1 > 0 and 3.0 < d2 / d1 < 5.0


# ---------------------------------------------------------------------------
# Symmetries and exact identities of Eq. (2)-(3)
# ---------------------------------------------------------------------------

GRID = (5, 4, 3)


def _levels(m, oracle, nf=5):
    lo, hi = oracle.band_range(m.t, m.R, (4, 4, 4))
    return np.linspace(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo), nf)


@pytest.mark.parametrize("kT", [0.0, 0.05])
def test_time_reversal_gives_zero(oracle, kT):
    m = S.trs_model(6, 1, 1.0, 41)
    ef = _levels(m, oracle)
    s, sabs = oracle.ahc(m.t, m.R, (6, 6, 6), ef, 1e-3, kT, with_sabs=True)
    assert np.all(sabs > 0)
    assert np.all(np.abs(s) <= 1e-12 * sabs)


def test_empty_and_full_bands_give_zero(oracle):
    m = S.random_model(5, 1, 1.0, 51)
    lo, hi = oracle.band_range(m.t, m.R, GRID)
    s = oracle.ahc(m.t, m.R, GRID, [lo - 1.0, hi + 1.0], 1e-3, 0.0)
    assert np.array_equal(s, [0.0, 0.0])


def test_orbital_basis_invariance(oracle):
    m = S.random_model(6, 1, 1.0, 61)
    ef = _levels(m, oracle)
    W = S.random_unitary(6, 62)
    a, sabs = oracle.ahc(m.t, m.R, GRID, ef, 1e-2, 0.02, with_sabs=True)
    b = oracle.ahc(S.rotate_orbitals(m, W).t, m.R, GRID, ef, 1e-2, 0.02)
    assert np.all(np.abs(a - b) <= 1e-10 * np.maximum(np.abs(a), sabs))


def test_swapping_x_and_y_flips_sign(oracle):
    m = S.random_model(6, 1, 1.0, 71)
    ef = _levels(m, oracle)
    g = (5, 5, 3)  # N_x = N_y so the swapped grid is the same grid
    a, sabs = oracle.ahc(m.t, m.R, g, ef, 1e-2, 0.0, with_sabs=True)
    sw = S.swap_xy(m)
    b = oracle.ahc(sw.t, sw.R, g, ef, 1e-2, 0.0)
    assert np.all(np.abs(a + b) <= 1e-10 * np.maximum(np.abs(a), sabs))


def test_direct_sum_and_doubling(oracle):
    a = S.random_model(4, 1, 1.0, 81)
    b = S.random_model(3, 1, 1.0, 82)
    ef = np.array([-1.0, 0.0, 0.7])
    sa, abs_a = oracle.ahc(a.t, a.R, GRID, ef, 1e-2, 0.03, with_sabs=True)
    sb, abs_b = oracle.ahc(b.t, b.R, GRID, ef, 1e-2, 0.03, with_sabs=True)
    ab = S.direct_sum(a, b)
    sab = oracle.ahc(ab.t, ab.R, GRID, ef, 1e-2, 0.03)
    assert np.all(np.abs(sab - sa - sb) <= 1e-11 * (abs_a + abs_b))
    d = S.doubled(a)
    sd = oracle.ahc(d.t, d.R, GRID, ef, 1e-2, 0.03)
    assert np.all(np.abs(sd - 2 * sa) <= 1e-11 * abs_a)


def test_slabs_add_up(oracle):
    m = S.random_model(5, 1, 1.0, 91)
    ef = _levels(m, oracle, 3)
    full = oracle.ahc(m.t, m.R, GRID, ef, 1e-3, 0.01)
    parts = [oracle.ahc(m.t, m.R, GRID, ef, 1e-3, 0.01, k_begin=b, k_count=c)
             for b, c in ((0, 7), (7, 30), (37, 23))]
    assert np.allclose(sum(parts), full, rtol=1e-13, atol=1e-16)


def test_zero_temperature_limit(oracle):
    m = S.random_model(5, 1, 1.0, 95)
    ef = _levels(m, oracle, 3)
    a, sabs = oracle.ahc(m.t, m.R, GRID, ef, 1e-2, 0.0, with_sabs=True)
    b = oracle.ahc(m.t, m.R, GRID, ef, 1e-2, 1e-9)
    assert np.all(np.abs(a - b) <= 1e-6 * sabs)


def test_thread_count_does_not_change_result(oracle):
    m = S.random_model(4, 1, 1.0, 97)
    a = oracle.ahc(m.t, m.R, GRID, [0.1, 0.4], 1e-3, 0.01, nthreads=1)
    b = oracle.ahc(m.t, m.R, GRID, [0.1, 0.4], 1e-3, 0.01, nthreads=4)
    assert np.array_equal(a, b)


def test_brute_force_with_lapack_eigensolver(oracle):
    """The whole sum on a 3^3 grid with scipy's eigh in place of the Jacobi solver."""
    m = S.random_model(4, 1, 1.0, 99)
    g = (3, 3, 3)
    ef = np.array([-0.5, 0.3])
    eta, kT = 1e-2, 0.05
    tot = np.zeros(2)
    for f in range(27):
        i0, i1, i2 = f % 3, (f // 3) % 3, f // 9
        k = 2 * np.pi * np.array([i0 / 3, i1 / 3, i2 / 3])
        H, vx, vy = oracle.hk(m.t, m.R, k)
        E, U = sla.eigh(H)
        A = U.conj().T @ vx @ U
        B = U.conj().T @ vy @ U
        Om = -2 * np.array([sum(np.imag(A[a, b] * B[b, a]) / ((E[a] - E[b]) ** 2 + eta**2)
                                for b in range(4) if b != a) for a in range(4)])
        f_occ = 1 / (1 + np.exp((E[:, None] - ef[None, :]) / kT))
        tot -= (f_occ * Om[:, None]).sum(0)
    tot /= 27
    s, sabs = oracle.ahc(m.t, m.R, g, ef, eta, kT, with_sabs=True)
    assert np.all(np.abs(s - tot) <= 1e-11 * sabs)


def _brute_sigma(m, grid, flats, ef, eta, kT):
    """sigma over the listed flat k indices with the test's own k enumeration
    (f = i0 + N0 (i1 + N1 i2), k = 2 pi (i0/N0, i1/N1, i2/N2)), numpy Bloch sums and
    LAPACK's eigensolver; normalised by the full grid."""
    N0, N1, N2 = grid
    tot = np.zeros(len(ef))
    n = m.n
    for f in flats:
        i0, rest = f % N0, f // N0
        i1, i2 = rest % N1, rest // N1
        k = 2 * np.pi * np.array([i0 / N0, i1 / N1, i2 / N2])
        ph = np.exp(1j * (m.R @ k))
        Ht = np.einsum("r,rij->ij", ph, m.t)
        Xt = np.einsum("r,rij->ij", 1j * m.R[:, 0] * ph, m.t)
        Yt = np.einsum("r,rij->ij", 1j * m.R[:, 1] * ph, m.t)
        H, vx, vy = [(X + X.conj().T) / 2 for X in (Ht, Xt, Yt)]
        E, U = sla.eigh(H)
        A = U.conj().T @ vx @ U
        B = U.conj().T @ vy @ U
        g = 1.0 / ((E[:, None] - E[None, :]) ** 2 + eta**2)
        np.fill_diagonal(g, 0.0)
        Om = -2 * np.sum(np.imag(A * B.T) * g, axis=1)
        f_occ = 1 / (1 + np.exp((E[:, None] - ef[None, :]) / kT))
        tot -= (f_occ * Om[:, None]).sum(0)
    return tot / (N0 * N1 * N2)


def test_brute_force_on_a_non_cubic_grid_and_slab(oracle):
    """A 4 x 3 x 2 grid, and a slab of it, with k enumerated by the test: a mix-up of
    the axes or of the flat-index order in the oracle's grid handling changes the result
    (the model's hoppings differ along x, y and z)."""
    m = S.random_model(4, 1, 1.0, 1199)
    g = (4, 3, 2)
    ef = np.array([-0.6, 0.1, 0.9])
    eta, kT = 2e-2, 0.04
    full = _brute_sigma(m, g, range(24), ef, eta, kT)
    s, sabs = oracle.ahc(m.t, m.R, g, ef, eta, kT, with_sabs=True)
    assert np.all(np.abs(s - full) <= 1e-11 * sabs)
    part = _brute_sigma(m, g, range(5, 18), ef, eta, kT)
    sp, sabs_p = oracle.ahc(m.t, m.R, g, ef, eta, kT, k_begin=5, k_count=13, with_sabs=True)
    assert np.all(np.abs(sp - part) <= 1e-11 * sabs_p)
    # the axes matter here: the transposed grid gives a different sum
    other = oracle.ahc(m.t, m.R, (2, 3, 4), ef, eta, kT)
    assert np.max(np.abs(other - s)) > 1e-6 * np.max(sabs)


# ---------------------------------------------------------------------------
# Reference gradient
# ---------------------------------------------------------------------------

GG = (3, 3, 2)


def _fd(oracle, m, ef, eta, kT, sbar, entries, h=1e-6):
    out = []
    for (r, i, j, part) in entries:
        d = np.zeros_like(m.t)
        d[r, i, j] = h if part == 0 else 1j * h
        sp = oracle.ahc(m.t + d, m.R, GG, ef, eta, kT)
        sm = oracle.ahc(m.t - d, m.R, GG, ef, eta, kT)
        out.append(float(sbar @ (sp - sm)) / (2 * h))
    return np.array(out)


def _entries(m, count, seed):
    u = S.uniform01(seed, 4 * count).reshape(count, 4)
    return [(int(a * m.n_R), int(b * m.n), int(c * m.n), int(d * 2)) for a, b, c, d in u]


def test_gradient_matches_finite_differences(oracle):
    m = S.random_model(4, 1, 1.0, 111)
    ef = np.array([-0.4, 0.2, 0.9])
    sbar = np.array([0.7, -1.3, 0.4])
    eta, kT = 0.05, 0.05
    G = oracle.ahc_grad(m.t, m.R, GG, ef, eta, kT, sbar)
    ent = _entries(m, 12, 112)
    fd = _fd(oracle, m, ef, eta, kT, sbar, ent)
    an = np.array([G[r, i, j].real if p == 0 else G[r, i, j].imag for (r, i, j, p) in ent])
    scale = np.abs(G).max()
    assert np.all(np.abs(an - fd) <= 1e-6 * np.maximum(np.abs(fd), 1e-3 * scale))


def test_gradient_two_forms_agree_and_symmetry(oracle):
    m = S.random_model(5, 1, 1.0, 121)
    ef = np.array([-0.2, 0.5])
    sbar = np.array([1.0, 0.3])
    g0 = oracle.ahc_grad(m.t, m.R, GG, ef, 0.02, 0.04, sbar, mode=0)
    g1 = oracle.ahc_grad(m.t, m.R, GG, ef, 0.02, 0.04, sbar, mode=1)
    assert np.max(np.abs(g0 - g1)) <= 1e-9 * np.abs(g0).max()
    idx = {tuple(v): i for i, v in enumerate(m.R)}
    for i, v in enumerate(m.R):
        j = idx[tuple(-v)]
        assert np.max(np.abs(g0[j] - g0[i].conj().T)) <= 1e-12 * np.abs(g0).max()


def test_gradient_through_exact_degeneracy(oracle):
    a = S.random_model(3, 1, 1.0, 131)
    m = S.doubled(a)
    ef = np.array([0.1, 0.6])
    sbar = np.array([1.0, -0.5])
    eta, kT = 0.05, 0.05
    G = oracle.ahc_grad(m.t, m.R, GG, ef, eta, kT, sbar)
    assert np.all(np.isfinite(G))
    ent = _entries(m, 10, 132)
    fd = _fd(oracle, m, ef, eta, kT, sbar, ent)
    an = np.array([G[r, i, j].real if p == 0 else G[r, i, j].imag for (r, i, j, p) in ent])
    scale = np.abs(G).max()
    assert np.all(np.abs(an - fd) <= 1e-6 * np.maximum(np.abs(fd), 1e-3 * scale))


def test_gradient_requires_broadening(oracle):
    m = S.random_model(3, 1, 1.0, 141)
    with pytest.raises(ValueError):
        oracle.ahc_grad(m.t, m.R, GG, [0.0], 0.0, 0.01, [1.0])
