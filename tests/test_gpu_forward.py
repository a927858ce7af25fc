"""GPU parity of the forward path (kubo_ahc through the C ABI) against the oracle."""

import os

import numpy as np
import pytest

from paper_2309_06675_amd import kubo, synth

from _util import assert_sigma_parity, slab_sample, workload_fermi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


def run_gpu(torch, models, grid, ef, eta, kT, slabs=None, flags=0, tiles=None):
    plan = kubo.Plan(models, grid=grid, n_fermi=ef.shape[-1], flags=flags, tiles=tiles,
                     slabs=slabs)
    t = kubo.to_device_t(models)
    efd = torch.from_numpy(np.ascontiguousarray(np.tile(ef, (len(models), 1))))
    efd = efd.to("cuda")
    sig = plan.forward(t, efd, eta, kT)
    st = plan.device_status()
    assert st == kubo.KUBO_OK, kubo.kubo_status_string(st)
    return sig.cpu().numpy(), plan


def test_cfg0_full_grid_parity(torch, oracle):
    wl = synth.workload(0)
    m = wl.models[0]
    ef = workload_fermi(0, wl)[0]
    print("case cfg0 full grid", flush=True)
    got, _ = run_gpu(torch, [m], wl.grid, ef, wl.eta, wl.kT)
    ref, sabs = oracle.ahc(m.t, m.R, wl.grid, ef, wl.eta, wl.kT, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what="cfg0")


@pytest.mark.parametrize("count,seed", [(600, 1), (257, 2)])
def test_cfg1_model_sampled_slab_parity(torch, oracle, count, seed):
    wl = synth.workload(1)
    m = wl.models[0]
    ef = workload_fermi(1, wl)[0]
    kb, kc = slab_sample(wl.n_k, count, seed)
    print(f"case cfg1 slab {kb}+{kc}", flush=True)
    got, _ = run_gpu(torch, [m], wl.grid, ef, wl.eta, wl.kT, slabs=[(kb, kc)])
    ref, sabs = oracle.ahc(m.t, m.R, wl.grid, ef, wl.eta, wl.kT, k_begin=kb, k_count=kc,
                           with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what="cfg1 slab")


@pytest.mark.parametrize("n,L,grid,kT", [(1, 1, (3, 2, 2), 0.0), (3, 1, (5, 3, 2), 0.02),
                                         (5, 2, (7, 2, 3), 0.0), (7, 1, (4, 4, 4), 0.05),
                                         (12, 1, (6, 3, 2), 0.01), (16, 1, (3, 3, 3), 0.0),
                                         (23, 2, (4, 3, 2), 0.03), (32, 1, (5, 2, 2), 0.01)])
def test_small_models_parity(torch, oracle, n, L, grid, kT):
    m = synth.random_model(n, L, 1.0, 500 + n)
    lo, hi = oracle.band_range(m.t, m.R, (3, 3, 3))
    ef = np.linspace(lo - 0.5, hi + 0.5, 7)
    print(f"case small n={n} grid={grid}", flush=True)
    got, _ = run_gpu(torch, [m], grid, ef, 1e-3, kT)
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-3, kT, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"n={n}")


@pytest.mark.parametrize("n,L,grid,kT", [(33, 1, (3, 2, 2), 0.02), (40, 1, (2, 3, 2), 0.0),
                                         (64, 1, (2, 2, 3), 0.01), (97, 1, (2, 2, 1), 0.02),
                                         (128, 1, (2, 1, 2), 0.01)])
def test_large_models_parity(torch, oracle, n, L, grid, kT):
    """The workgroup-per-k-point path (n > 32) against the oracle."""
    m = synth.random_model(n, L, 1.0, 600 + n)
    lo, hi = oracle.band_range(m.t, m.R, (2, 2, 2))
    ef = np.linspace(lo - 0.5, hi + 0.5, 6)
    print(f"case large n={n} grid={grid}", flush=True)
    got, _ = run_gpu(torch, [m], grid, ef, 1e-3, kT)
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-3, kT, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"n={n}")


@pytest.mark.parametrize("n,grid", [(5, (4, 3, 2)), (16, (3, 3, 2)), (32, (3, 2, 2))])
def test_workgroup_kernel_for_small_n(torch, oracle, n, grid):
    """Small n routed to the workgroup-per-k-point kernel (tile threads = 256)."""
    m = synth.random_model(n, 1, 1.0, 620 + n)
    lo, hi = oracle.band_range(m.t, m.R, (2, 2, 2))
    ef = np.linspace(lo, hi, 5)
    got, _ = run_gpu(torch, [m], grid, ef, 1e-3, 0.01, tiles=[(n, 256, 3)])
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-3, 0.01, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"wg n={n}")


@pytest.mark.parametrize("n", [6, 24])
def test_degenerate_spectrum_parity(torch, oracle, n):
    """t (x) I_2: every eigenvalue doubly degenerate (the clustered-spectrum path)."""
    m = synth.doubled(synth.random_model(n, 1, 1.0, 640 + n))
    ef = np.array([-1.0, 0.0, 1.3])
    got, _ = run_gpu(torch, [m], (3, 2, 2), ef, 1e-2, 0.02)
    ref, sabs = oracle.ahc(m.t, m.R, (3, 2, 2), ef, 1e-2, 0.02, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"doubled n={2 * n}")


@pytest.mark.parametrize("n,grid", [(40, (3, 2, 2)), (64, (2, 1, 2))])
def test_degenerate_spectrum_parity_workgroup_class(torch, oracle, n, grid):
    """t (x) I_2 at n = 80 and n = 128: every eigenvalue doubly degenerate, so the
    workgroup kernel for n > 64 takes its clustered-spectrum path (implicit QL with
    accumulated rotations, then the back-transformation)."""
    m = synth.doubled(synth.random_model(n, 1, 1.0, 6400 + n))
    lo, hi = oracle.band_range(m.t, m.R, (2, 2, 1))
    ef = np.linspace(lo, hi, 5)
    print(f"case doubled n={2 * n} grid={grid}", flush=True)
    got, _ = run_gpu(torch, [m], grid, ef, 1e-2, 0.02)
    ref, sabs = oracle.ahc(m.t, m.R, grid, ef, 1e-2, 0.02, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"doubled n={2 * n}")


@pytest.mark.parametrize("n", [12, 28])
def test_graded_spectrum_parity(torch, oracle, n):
    """Orbitals scaled over four decades (D t D): many eigenvalues far below the spectral
    radius, so the eigenvalue search keeps bracketing to the absolute tolerance instead of
    converging by Newton steps, and the twisted vectors see strongly graded pivots."""
    base = synth.random_model(n, 1, 1.0, 660 + n)
    d = 10.0 ** np.linspace(-3.0, 1.0, n)
    m = synth.TBModel(t=base.t * d[None, :, None] * d[None, None, :], R=base.R.copy())
    ef = np.array([-2.0, -1e-3, 0.0, 1e-3, 2.0])
    got, _ = run_gpu(torch, [m], (4, 3, 2), ef, 1e-3, 0.01)
    ref, sabs = oracle.ahc(m.t, m.R, (4, 3, 2), ef, 1e-3, 0.01, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"graded n={n}")


@pytest.mark.parametrize("u", [-1.0, 1.0, 3.0])
def test_qwz_quantised_on_gpu(torch, u):
    m = synth.qwz_model(u)
    exact = -0.5 * (np.sign(u + 2) - 2 * np.sign(u) + np.sign(u - 2)) / (2 * np.pi)
    got, _ = run_gpu(torch, [m], (96, 96, 1), np.array([0.0]), 0.0, 0.0)
    assert abs(got[0, 0] - exact) <= 1e-10


def test_time_reversal_zero_on_gpu(torch, oracle):
    m = synth.trs_model(8, 1, 1.0, 41)
    ef = np.linspace(-2.0, 2.0, 5)
    got, _ = run_gpu(torch, [m], (6, 6, 6), ef, 1e-3, 0.01)
    _, sabs = oracle.ahc(m.t, m.R, (6, 6, 6), ef, 1e-3, 0.01, with_sabs=True)
    assert np.all(np.abs(got[0]) <= 1e-12 * sabs)


def test_slabs_add_up_and_determinism(torch):
    m = synth.random_model(10, 1, 1.0, 77)
    ef = np.linspace(-3, 3, 9)
    grid = (9, 5, 4)
    full, _ = run_gpu(torch, [m], grid, ef, 1e-3, 0.01)
    again, _ = run_gpu(torch, [m], grid, ef, 1e-3, 0.01)
    assert np.array_equal(full, again)
    parts = sum(run_gpu(torch, [m], grid, ef, 1e-3, 0.01, slabs=[s])[0]
                for s in [(0, 13), (13, 50), (63, 117)])
    assert np.allclose(parts, full, rtol=1e-12, atol=1e-14)


def test_multi_model_plan_equals_single_plans(torch):
    ms = [synth.random_model(n, 1, 1.0, 900 + n) for n in (3, 8, 17, 30, 44)]
    ef = np.linspace(-2, 2, 4)
    grid = (6, 4, 3)
    both, _ = run_gpu(torch, ms, grid, ef, 1e-3, 0.02)
    for i, m in enumerate(ms):
        one, _ = run_gpu(torch, [m], grid, ef, 1e-3, 0.02)
        assert np.array_equal(one[0], both[i])


def test_many_chunks_equal_one_chunk(torch, monkeypatch):
    m = synth.random_model(16, 2, 1.0, 123)
    ef = np.linspace(-4, 4, 5)
    grid = (8, 6, 5)
    ref, _ = run_gpu(torch, [m], grid, ef, 1e-3, 0.01)
    monkeypatch.setenv("KUBO_CHUNK_MB", "1")
    got, _ = run_gpu(torch, [m], grid, ef, 1e-3, 0.01)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)


def test_graph_replay_matches_eager(torch):
    m = synth.random_model(12, 1, 1.0, 321)
    grid = (6, 5, 4)
    ef = torch.linspace(-2, 2, 6, dtype=torch.float64, device="cuda").reshape(1, 6)
    t = kubo.to_device_t([m])
    eager = kubo.Plan([m], grid=grid, n_fermi=6)
    ref = eager.forward(t, ef, 1e-3, 0.01).cpu().numpy()
    g = kubo.Plan([m], grid=grid, n_fermi=6, flags=kubo.KUBO_F_GRAPH)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = torch.empty(1, 6, dtype=torch.float64, device="cuda")
        for rep in range(4):
            out.fill_(float("nan"))
            g.forward(t, ef, 1e-3, 0.01, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), rep
            _ = (t * 2).sum()  # unrelated eager work between replays
    # new hopping values, same pointers: the graph sees them
    t2 = t * 1.5
    with torch.cuda.stream(s):
        t.copy_(t2)
        g.forward(t, ef, 1e-3, 0.01, out=out)
        torch.cuda.synchronize()
    ref2 = eager.forward(t, ef, 1e-3, 0.01).cpu().numpy()
    assert np.array_equal(out.cpu().numpy(), ref2)


def test_device_status_flags(torch):
    m = synth.random_model(8, 1, 1.0, 55)
    grid = (4, 3, 2)
    ef = torch.zeros(1, 1, dtype=torch.float64, device="cuda")
    t = kubo.to_device_t([m])
    capped = kubo.Plan([m], grid=grid, n_fermi=1, flags=kubo.KUBO_F_DEBUG_SWEEPCAP)
    capped.forward(t, ef, 1e-3, 0.0)
    assert capped.device_status() == kubo.KUBO_E_NOCONV
    plan = kubo.Plan([m], grid=grid, n_fermi=1)
    bad = t.clone()
    bad[3] = complex(float("nan"), 0.0)
    plan.forward(bad, ef, 1e-3, 0.0)
    assert plan.device_status() in (kubo.KUBO_E_NONFINITE, kubo.KUBO_E_NOCONV)
    plan.forward(t, ef, 1e-3, 0.0)
    assert plan.device_status() == kubo.KUBO_OK
