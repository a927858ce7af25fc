"""GPU parity of kubo_ahc_tensor (the Hall tensor xy, yz, zx and the spin Hall
conductivity in one pass) against the oracle, through the C ABI."""

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


def run_tensor(torch, models, grid, ef, eta, kT, spins=None, slabs=None, flags=0, tiles="auto"):
    plan = kubo.Plan(models, grid=grid, n_fermi=ef.shape[-1], flags=flags | kubo.KUBO_F_TENSOR,
                     slabs=slabs, tiles=tiles)
    t = kubo.to_device_t(models)
    efd = torch.from_numpy(np.ascontiguousarray(np.tile(ef, (len(models), 1)))).to("cuda")
    sp = None
    if spins is not None:
        sp = torch.from_numpy(np.concatenate(spins).astype(np.float64)).to("cuda")
    sig = plan.tensor(t, efd, eta, kT, spin=sp)
    st = plan.device_status()
    assert st == kubo.KUBO_OK, kubo.kubo_status_string(st)
    return sig.cpu().numpy(), plan, t, efd


def _spin(n, seed):
    """A spin diagonal of mixed signs and magnitudes."""
    return np.round(2.0 * synth.uniform01(seed, n) - 1.0, 3)


def _check(got, ref, sabs, what):
    for c, name in enumerate(kubo.TENSOR_COMPONENTS):
        assert_sigma_parity(got[c], ref[c], sabs[c], what=f"{what} {name}")


@pytest.mark.parametrize("n,grid,kT", [(3, (5, 3, 2), 0.02), (8, (4, 3, 3), 0.0),
                                       (13, (3, 4, 2), 0.01), (24, (3, 2, 3), 0.03),
                                       (32, (4, 2, 2), 0.01), (40, (2, 3, 2), 0.02),
                                       (64, (2, 2, 1), 0.0), (80, (2, 1, 2), 0.01)])
def test_tensor_and_spin_hall_parity(torch, oracle, n, grid, kT):
    """Every per-k kernel class: one wavefront at padded sizes 8, 16, 32, one workgroup for
    n <= 64 and for n <= 128."""
    m = synth.random_model(n, 1, 1.0, 7300 + n)
    spin = _spin(n, 7400 + n)
    lo, hi = oracle.band_range(m.t, m.R, (2, 2, 2))
    ef = np.linspace(lo - 0.3, hi + 0.3, 6)
    print(f"case tensor n={n} grid={grid}", flush=True)
    got, *_ = run_tensor(torch, [m], grid, ef, 1e-3, kT, spins=[spin])
    ref, sabs = oracle.ahc_tensor(m.t, m.R, grid, ef, 1e-3, kT, spin=spin, with_sabs=True)
    _check(got[0], ref, sabs, f"n={n}")


def test_xy_component_equals_kubo_ahc_and_spin_none_is_zero(torch):
    models = [synth.random_model(n, 1, 1.0, 7500 + n) for n in (6, 20, 36)]
    grid = (5, 4, 3)
    ef = np.linspace(-2.0, 2.0, 5)
    got, plan, t, efd = run_tensor(torch, models, grid, ef, 2e-3, 0.01)
    xy = plan.forward(t, efd, 2e-3, 0.01).cpu().numpy()
    assert np.array_equal(got[:, 0, :], xy)
    assert np.array_equal(got[:, 3, :], np.zeros_like(xy))


def test_cfg1_model_tensor_sampled_slab(torch, oracle):
    """The n_orb = 32 workload model (343 lattice vectors, 64 levels) on a slab of its
    100^3 grid, with a spin-up/spin-down split of the orbitals."""
    wl = synth.workload(1)
    m = wl.models[0]
    ef = workload_fermi(1, wl)[0]
    spin = np.repeat([1.0, -1.0], m.n // 2)
    kb, kc = slab_sample(wl.n_k, 160, 7601)
    print(f"case tensor cfg1 slab {kb}+{kc}", flush=True)
    got, *_ = run_tensor(torch, [m], wl.grid, ef, wl.eta, wl.kT, spins=[spin], slabs=[(kb, kc)])
    ref, sabs = oracle.ahc_tensor(m.t, m.R, wl.grid, ef, wl.eta, wl.kT, spin=spin, k_begin=kb,
                                  k_count=kc, with_sabs=True)
    _check(got[0], ref, sabs, "cfg1 slab")


@pytest.mark.parametrize("plane,comp,grid", [("yz", 1, (1, 96, 96)), ("zx", 2, (96, 1, 96))])
def test_qwz_in_other_planes_quantised_on_gpu(torch, plane, comp, grid):
    m = synth.qwz_plane_model(1.0, plane)
    got, *_ = run_tensor(torch, [m], grid, np.array([0.0]), 0.0, 0.0)
    assert abs(got[0, comp, 0] - 1.0 / (2 * np.pi)) <= 1e-10


def test_spin_split_qwz_pair_on_gpu(torch, oracle):
    """Spin Hall of QWZ(1) up and the time-reversal partner of QWZ(1.5) down: against the
    oracle at eta = 1e-3, and within O(eta^2) of the quantised 1/pi."""
    m, spin = synth.spin_qwz_pair(1.0, 1.5)
    ef = np.array([0.0])
    got, *_ = run_tensor(torch, [m], (64, 64, 1), ef, 1e-3, 0.0, spins=[spin])
    ref, sabs = oracle.ahc_tensor(m.t, m.R, (64, 64, 1), ef, 1e-3, 0.0, spin=spin,
                                  with_sabs=True)
    _check(got[0], ref, sabs, "spin QWZ pair")
    assert abs(got[0, 3, 0] - 1.0 / np.pi) <= 1e-5
    assert abs(got[0, 0, 0]) <= 1e-5


def test_doubled_model_with_opposite_spins(torch, oracle):
    """t (x) I_2 (every band doubly degenerate: the clustered-spectrum paths) with s_z = +1
    on one copy and -1 on the other, at n = 16 (one wavefront) and n = 48 (workgroup)."""
    for n in (8, 24):
        m = synth.doubled(synth.random_model(n, 1, 1.0, 7700 + n))
        spin = np.tile([1.0, -1.0], n)
        ef = np.array([-0.8, 0.1, 0.9])
        got, *_ = run_tensor(torch, [m], (3, 2, 2), ef, 1e-2, 0.02, spins=[spin])
        ref, sabs = oracle.ahc_tensor(m.t, m.R, (3, 2, 2), ef, 1e-2, 0.02, spin=spin,
                                      with_sabs=True)
        _check(got[0], ref, sabs, f"doubled n={2 * n}")


def test_time_reversal_tensor_zero_on_gpu(torch, oracle):
    m = synth.trs_model(10, 1, 1.0, 7801)
    ef = np.linspace(-2.0, 2.0, 5)
    got, *_ = run_tensor(torch, [m], (5, 4, 4), ef, 1e-3, 0.01)
    _, sabs = oracle.ahc_tensor(m.t, m.R, (5, 4, 4), ef, 1e-3, 0.01, with_sabs=True)
    assert np.all(np.abs(got[0, :3]) <= 1e-12 * sabs[:3])


def test_tensor_multi_model_graph_replay(torch, oracle):
    """Uneven models (both kernel families) in one plan, captured as a graph and replayed,
    against the eager plan and the oracle."""
    models = [synth.random_model(n, 1, 1.0, 7900 + n) for n in (5, 17, 30, 44)]
    spins = [_spin(m.n, 7950 + m.n) for m in models]
    grid = (4, 3, 2)
    ef = np.linspace(-1.5, 1.5, 4)
    eager, *_ = run_tensor(torch, models, grid, ef, 1e-3, 0.02, spins=spins)
    plan = kubo.Plan(models, grid=grid, n_fermi=4, flags=kubo.KUBO_F_TENSOR | kubo.KUBO_F_GRAPH)
    t = kubo.to_device_t(models)
    efd = torch.from_numpy(np.ascontiguousarray(np.tile(ef, (4, 1)))).to("cuda")
    sp = torch.from_numpy(np.concatenate(spins)).to("cuda")
    s = torch.cuda.Stream()
    out = torch.empty(4, 4, 4, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        for rep in range(3):
            out.fill_(float("nan"))
            plan.tensor(t, efd, 1e-3, 0.02, spin=sp, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), eager), rep
            _ = (t * 2).abs().sum()
    for i, m in enumerate(models):
        ref, sabs = oracle.ahc_tensor(m.t, m.R, grid, ef, 1e-3, 0.02, spin=spins[i],
                                      with_sabs=True)
        _check(eager[i], ref, sabs, f"multi n={m.n}")
