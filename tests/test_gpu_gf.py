"""GPU parity of kubo_ahc_gf (the Green's-function form of sigma_xy: one inverse of
(i (w + gamma) + E_F) - H(k) per k-point, Fermi level and quadrature node) against
the oracle, through the C ABI."""

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


def run_gf(torch, models, grid, ef, gamma, omega, weight, slabs=None, flags=0, tiles="auto"):
    plan = kubo.Plan(models, grid=grid, n_fermi=ef.shape[-1],
                     flags=flags | kubo.KUBO_F_FORWARD_ONLY, slabs=slabs, tiles=tiles)
    t = kubo.to_device_t(models)
    efd = torch.from_numpy(np.ascontiguousarray(np.tile(ef, (len(models), 1)))).to("cuda")
    om = torch.from_numpy(np.ascontiguousarray(omega, dtype=np.float64)).to("cuda")
    wt = torch.from_numpy(np.ascontiguousarray(weight, dtype=np.float64)).to("cuda")
    sig = plan.gf(t, efd, gamma, om, wt)
    st = plan.device_status()
    assert st == kubo.KUBO_OK, kubo.kubo_status_string(st)
    return sig.cpu().numpy(), plan, t, efd


def _levels(oracle, m, nf):
    lo, hi = oracle.band_range(m.t, m.R, (2, 2, 2))
    return np.linspace(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo), nf)


@pytest.mark.parametrize("n,grid,gamma", [(3, (5, 3, 2), 0.05), (8, (4, 3, 3), 0.0),
                                          (13, (3, 4, 2), 0.02), (24, (3, 2, 3), 0.1),
                                          (32, (4, 2, 2), 0.01)])
def test_gf_parity(torch, oracle, n, grid, gamma):
    """Padded sizes 8, 16 and 32 of the one-wavefront classes; gamma = 0 included."""
    m = synth.random_model(n, 1, 1.0, 8100 + n)
    ef = _levels(oracle, m, 4)
    om, w = oracle.half_line_rule(8, 0.8)
    print(f"case gf n={n} grid={grid} gamma={gamma}", flush=True)
    got, *_ = run_gf(torch, [m], grid, ef, gamma, om, w)
    ref, sabs = oracle.ahc_gf(m.t, m.R, grid, ef, gamma, om, w, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what=f"gf n={n} gamma={gamma}")


def test_gf_mixed_models_and_workgroup_tiles(torch, oracle):
    """Several models in one plan, some of them placed in the workgroup size class by the
    tile table: the kernel serves every item with n <= 32 whatever its class."""
    models = [synth.random_model(n, 1, 1.0, 8200 + n) for n in (5, 17, 30)]
    grid = (3, 3, 2)
    ef = np.linspace(-1.5, 1.5, 3)
    om, w = oracle.half_line_rule(6, 0.6)
    tiles = [(17, 256, 4), (30, 64, 2)]
    print("case gf mixed", flush=True)
    got, *_ = run_gf(torch, models, grid, ef, 0.03, om, w, tiles=tiles)
    for i, m in enumerate(models):
        ref, sabs = oracle.ahc_gf(m.t, m.R, grid, ef, 0.03, om, w, with_sabs=True)
        assert_sigma_parity(got[i], ref, sabs, what=f"gf mixed n={m.n}")


def test_gf_many_chunks(torch, oracle, monkeypatch):
    m = synth.random_model(12, 2, 1.0, 8301)
    grid = (6, 5, 4)
    ef = np.linspace(-1.0, 1.0, 3)
    om, w = oracle.half_line_rule(5, 0.5)
    monkeypatch.setenv("KUBO_CHUNK_MB", "1")
    print("case gf chunks", flush=True)
    got, *_ = run_gf(torch, [m], grid, ef, 0.02, om, w)
    monkeypatch.delenv("KUBO_CHUNK_MB")
    ref, sabs = oracle.ahc_gf(m.t, m.R, grid, ef, 0.02, om, w, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what="gf many chunks")


def test_gf_cfg1_model_sampled_slab(torch, oracle):
    """The n_orb = 32 workload model (343 lattice vectors) on a slab of its 100^3 grid."""
    wl = synth.workload(1)
    m = wl.models[0]
    ef = workload_fermi(1, wl)[0][::16]
    om, w = oracle.half_line_rule(6, 1.0)
    kb, kc = slab_sample(wl.n_k, 96, 8401)
    print(f"case gf cfg1 slab {kb}+{kc}", flush=True)
    got, *_ = run_gf(torch, [m], wl.grid, ef, 0.01, om, w, slabs=[(kb, kc)])
    ref, sabs = oracle.ahc_gf(m.t, m.R, wl.grid, ef, 0.01, om, w, k_begin=kb, k_count=kc,
                              with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what="gf cfg1 slab")


def test_gf_qwz_gap_is_quantised_and_matches(torch, oracle):
    """QWZ with the Fermi level in the gap at gamma = 0: the Chern number, as the
    eigenvalue form gives it, and the oracle element by element."""
    m = synth.qwz_model(1.0)
    grid = (32, 32, 1)
    om, w = oracle.half_line_rule(48, 1.0)
    ef = np.array([0.0, 0.3])
    print("case gf qwz", flush=True)
    got, *_ = run_gf(torch, [m], grid, ef, 0.0, om, w)
    ref, sabs = oracle.ahc_gf(m.t, m.R, grid, ef, 0.0, om, w, with_sabs=True)
    assert_sigma_parity(got[0], ref, sabs, what="gf qwz")
    assert np.all(np.abs(got[0] - 1.0 / (2 * np.pi)) < 1e-6)


def test_gf_zero_gamma_tracks_kubo_ahc(torch, oracle):
    """With gamma = 0 and a fine quadrature the GPU's Green's-function form and its
    eigenvalue form (eta = 0, kT = 0) agree to the quadrature error."""
    m = synth.random_model(10, 1, 1.0, 8501)
    grid = (4, 4, 3)
    ef = _levels(oracle, m, 3)
    om, w = oracle.half_line_rule(160, 1.0)
    print("case gf vs ahc", flush=True)
    got, plan, t, efd = run_gf(torch, [m], grid, ef, 0.0, om, w)
    ahc = plan.forward(t, efd, 0.0, 0.0).cpu().numpy()
    _, sabs = oracle.ahc(m.t, m.R, grid, ef, 0.0, 0.0, with_sabs=True)
    assert np.all(np.abs(got - ahc) <= 1e-7 * np.maximum(np.abs(ahc), sabs))
