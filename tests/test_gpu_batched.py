"""The batched workload: many tight-binding models of uneven orbital count in one plan,
launched as one captured hipGraph, against the oracle and against per-model plans."""

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


def test_cfg2_models_sampled_slabs_parity(torch, oracle):
    """The first 12 models of the 200-model workload, 96-point slabs of their 32^3 grids,
    in one graph-captured plan with the tuned tiles."""
    wl = synth.workload(2, n_models=12)
    ef = workload_fermi(2, wl)
    slabs = [slab_sample(wl.n_k, 96, 4000 + i) for i in range(len(wl.models))]
    plan = kubo.Plan(wl.models, grid=wl.grid, n_fermi=wl.n_fermi, flags=kubo.KUBO_F_GRAPH,
                     slabs=slabs)
    t = kubo.to_device_t(wl.models)
    efd = torch.from_numpy(ef).to("cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sig = plan.forward(t, efd, wl.eta, wl.kT)
        torch.cuda.synchronize()
    assert plan.device_status() == kubo.KUBO_OK
    got = sig.cpu().numpy()
    for i, m in enumerate(wl.models):
        print(f"case cfg2 model {i} n={m.n} slab {slabs[i]}", flush=True)
        ref, sabs = oracle.ahc(m.t, m.R, wl.grid, ef[i], wl.eta, wl.kT, k_begin=slabs[i][0],
                               k_count=slabs[i][1], with_sabs=True)
        assert_sigma_parity(got[i], ref, sabs, what=f"cfg2 model {i} (n={m.n})")


def test_batched_equals_plain_full_grid(torch):
    """Batched and per-model plans give bitwise equal sigma on the full 32^3 grids."""
    ns = [8, 20, 32, 36, 52, 64]
    models = [synth.random_model(n, 2, 1.0, 2100 + n) for n in ns]
    grid = (32, 32, 32)
    ef = torch.linspace(-6.0, 6.0, 16, dtype=torch.float64, device="cuda")
    efd = ef.reshape(1, 16).repeat(len(models), 1).contiguous()
    t = kubo.to_device_t(models)
    batched = kubo.Plan(models, grid=grid, n_fermi=16, flags=kubo.KUBO_F_FORWARD_ONLY)
    sb = batched.forward(t, efd, 1e-3, 0.0).cpu().numpy()
    off = 0
    for i, m in enumerate(models):
        p = kubo.Plan([m], grid=grid, n_fermi=16)
        cnt = m.t.size
        one = p.forward(t[off:off + cnt], efd[i:i + 1].contiguous(), 1e-3, 0.0).cpu().numpy()
        off += cnt
        assert np.array_equal(one[0], sb[i]), f"model {i} (n={m.n})"


def test_batched_graph_replays(torch):
    models = [synth.random_model(n, 1, 1.0, 2200 + n) for n in (8, 24, 40)]
    grid = (6, 5, 4)
    efd = torch.linspace(-2, 2, 5, dtype=torch.float64, device="cuda").reshape(1, 5).repeat(3, 1)
    efd = efd.contiguous()
    t = kubo.to_device_t(models)
    ref = kubo.Plan(models, grid=grid, n_fermi=5).forward(t, efd, 1e-3, 0.01).cpu().numpy()
    g = kubo.Plan(models, grid=grid, n_fermi=5, flags=kubo.KUBO_F_GRAPH)
    s = torch.cuda.Stream()
    out = torch.empty(3, 5, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        for rep in range(3):
            out.fill_(float("nan"))
            g.forward(t, efd, 1e-3, 0.01, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), rep
            _ = (t * 3).abs().sum()


def test_forward_only_plan_rejects_backward(torch):
    m = synth.random_model(4, 1, 1.0, 2300)
    p = kubo.Plan([m], grid=(3, 2, 2), n_fermi=1, flags=kubo.KUBO_F_FORWARD_ONLY)
    t = kubo.to_device_t([m])
    ef = torch.zeros(1, 1, dtype=torch.float64, device="cuda")
    p.forward(t, ef, 1e-3, 0.0)
    with pytest.raises(kubo.KuboError):
        p.backward(t, ef, 1e-3, 0.0, torch.ones_like(ef))
