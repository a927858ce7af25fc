"""The n_orb = 128 workload (729 lattice vectors, 128^3 grid, 256 Fermi levels):
sampled slabs of its full-grid plan against the oracle, forward and gradient."""

import numpy as np
import pytest

from paper_2309_06675_amd import kubo, synth

from _util import assert_grad_close, assert_sigma_parity, slab_sample, workload_fermi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


@pytest.fixture(scope="module")
def cfg4():
    wl = synth.workload(4)
    return wl, wl.models[0], workload_fermi(4, wl)[0]


@pytest.mark.parametrize("seed", [41, 42])
def test_cfg4_sampled_slab_forward(torch, oracle, cfg4, seed):
    wl, m, ef = cfg4
    kb, kc = slab_sample(wl.n_k, 16, seed)
    print(f"case cfg4 slab {kb}+{kc}", flush=True)
    plan = kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, slabs=[(kb, kc)])
    t = kubo.to_device_t([m])
    sig = plan.forward(t, torch.from_numpy(ef.reshape(1, -1).copy()).cuda(), wl.eta, wl.kT)
    assert plan.device_status() == kubo.KUBO_OK
    ref, sabs = oracle.ahc(m.t, m.R, wl.grid, ef, wl.eta, wl.kT, k_begin=kb, k_count=kc,
                           with_sabs=True)
    assert_sigma_parity(sig.cpu().numpy()[0], ref, sabs, what="cfg4 slab")


def test_cfg4_sampled_slab_gradient(torch, oracle, cfg4):
    wl, m, ef = cfg4
    kb, kc = slab_sample(wl.n_k, 2, 43)
    sbar = synth.normals(4343, wl.n_fermi)
    plan = kubo.Plan([m], grid=wl.grid, n_fermi=wl.n_fermi, slabs=[(kb, kc)])
    t = kubo.to_device_t([m])
    efd = torch.from_numpy(ef.reshape(1, -1).copy()).cuda()
    sb = torch.from_numpy(sbar.reshape(1, -1).copy()).cuda()
    g = plan.backward(t, efd, wl.eta_adjoint, wl.kT, sb).cpu().numpy()
    assert plan.device_status() == kubo.KUBO_OK
    ref = oracle.ahc_grad(m.t, m.R, wl.grid, ef, wl.eta_adjoint, wl.kT, sbar, k_begin=kb,
                          k_count=kc).reshape(-1)
    assert_grad_close(g, ref, 1e-8, "cfg4 slab")
