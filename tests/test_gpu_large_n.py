"""GPU parity of the large-n path (128 < n <= 512: a batch of k-points through the
Householder reduction, split-block bisection, tridiagonal eigenvectors, compact-WY
back-transformation and MFMA products, many workgroups per k-point) against the
oracle, through the C ABI."""

import numpy as np
import pytest

from paper_2309_06675_amd import kubo, synth

from _util import assert_sigma_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


def run(torch, models, grid, ef, eta, kT, slabs=None):
    plan = kubo.Plan(models, grid=grid, n_fermi=ef.shape[-1], flags=kubo.KUBO_F_FORWARD_ONLY,
                     slabs=slabs)
    t = kubo.to_device_t(models)
    efd = torch.from_numpy(np.ascontiguousarray(np.tile(ef, (len(models), 1)))).to("cuda")
    sig = plan.forward(t, efd, eta, kT)
    st = plan.device_status()
    assert st == kubo.KUBO_OK, kubo.kubo_status_string(st)
    return sig.cpu().numpy()


def _levels(oracle, m, nf):
    lo, hi = oracle.band_range(m.t, m.R, (2, 2, 1))
    return np.linspace(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo), nf)


@pytest.mark.parametrize("n,grid,kT", [(136, (3, 2, 2), 0.01), (200, (2, 2, 2), 0.0),
                                       (256, (2, 2, 1), 0.02)])
def test_large_n_parity(torch, oracle, n, grid, kT):
    m = synth.random_model(n, 1, 1.0, 9100 + n)
    ef = _levels(oracle, m, 5)
    print(f"case large n={n} grid={grid}", flush=True)
    got = run(torch, [m], grid, ef, 1e-3, kT)
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-3, kT, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"large n={n}")


def test_large_n_doubly_degenerate(torch, oracle):
    """t x I2: every band twice degenerate, so the tridiagonal matrix splits into blocks."""
    m = synth.doubled(synth.random_model(80, 1, 1.0, 9201))
    grid = (2, 2, 2)
    ef = _levels(oracle, m, 4)
    print(f"case large doubled n={m.n}", flush=True)
    got = run(torch, [m], grid, ef, 1e-2, 0.01)
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-2, 0.01, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"large doubled n={m.n}")


def test_large_n_mixed_plan_and_slab(torch, oracle):
    """A small and a large model in one plan, the large one on a slab of its grid."""
    small = synth.random_model(20, 1, 1.0, 9301)
    big = synth.random_model(150, 1, 1.0, 9302)
    grid = (4, 3, 2)
    ef = np.linspace(-2.0, 2.0, 4)
    slabs = [(0, -1), (5, 9)]
    print("case large mixed", flush=True)
    got = run(torch, [small, big], grid, ef, 1e-3, 0.01, slabs=slabs)
    ref0, s0 = oracle.ahc(small.t, small.R, grid, ef, 1e-3, 0.01, with_sabs=True)
    ref1, s1 = oracle.ahc(big.t, big.R, grid, ef, 1e-3, 0.01, k_begin=5, k_count=9,
                          with_sabs=True)
    assert_sigma_parity(got[0], ref0, s0, what="large mixed small n=20")
    assert_sigma_parity(got[1], ref1, s1, what="large mixed n=150 slab")


@pytest.mark.parametrize("parts,grid", [((150, 150), (1, 2, 2)), ((128, 128, 128, 128), (1, 1, 2))])
def test_large_n_rotated_direct_sum(torch, oracle, parts, grid):
    """n above 256, up to the 512 maximum: W (A (+) B (+) ...) W^+ with a random unitary W
    is a dense model whose sigma is exactly the sum of its blocks' (a k-independent change
    of orbital basis leaves every band's curvature unchanged, and bands of different
    blocks have no velocity matrix elements between them), so the oracle runs on the
    blocks alone."""
    blocks = [synth.random_model(p, 1, 1.0, 9400 + 10 * i + p) for i, p in enumerate(parts)]
    m = blocks[0]
    for b in blocks[1:]:
        m = synth.direct_sum(m, b)
    m = synth.rotate_orbitals(m, synth.random_unitary(m.n, 9499 + m.n))
    assert m.n == sum(parts)
    ranges = [oracle.band_range(b.t, b.R, (1, 1, 1)) for b in blocks]
    lo, hi = min(r[0] for r in ranges), max(r[1] for r in ranges)
    ef = np.linspace(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo), 5)
    print(f"case large rotated direct sum n={m.n} grid={grid}", flush=True)
    got = run(torch, [m], grid, ef, 1e-3, 0.01)
    ref = np.zeros(ef.size)
    sabs = np.zeros(ef.size)
    for b in blocks:
        r, s = oracle.ahc(b.t, b.R, grid, ef, 1e-3, 0.01, with_sabs=True)
        ref += r
        sabs += s
    assert_sigma_parity(got[0], ref, sabs, what=f"large rotated direct sum n={m.n}")


def test_large_n_ragged_batches(torch, oracle, monkeypatch):
    """KUBO_BIG_BATCH = 5 on 12 k-points: passes of 5, 5 and 2 k-points through the pipeline."""
    monkeypatch.setenv("KUBO_BIG_BATCH", "5")
    m = synth.random_model(136, 1, 1.0, 9500)
    grid = (3, 2, 2)
    ef = _levels(oracle, m, 4)
    print("case large ragged batches n=136", flush=True)
    got = run(torch, [m], grid, ef, 1e-3, 0.01)
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-3, 0.01, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what="large ragged batches n=136")
