"""kubo_ahc_noalloc (the forward on the library's own static device workspace)
against kubo_ahc on a caller workspace, through the C ABI: two calls in a row,
the second on a smaller input, then the first plan again."""

import numpy as np
import pytest

from paper_2309_06675_amd import kubo, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


def _case(torch, models, grids, nf, seed):
    plan = kubo.Plan(models, grid=grids, n_fermi=nf, flags=kubo.KUBO_F_FORWARD_ONLY)
    assert plan.ws_bytes <= kubo.KUBO_NOALLOC_MAX_BYTES
    t = kubo.to_device_t(models)
    ef = np.sort(synth.normals(seed, len(models) * nf).reshape(len(models), nf), axis=1)
    efd = torch.from_numpy(ef).to("cuda")
    return plan, t, efd


def _noalloc(torch, case, eta, kT):
    plan, t, efd = case
    sig = torch.full((plan.n_models, plan.n_fermi), float("nan"), dtype=torch.float64,
                     device="cuda")
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = kubo.kubo_ahc_noalloc(plan.handle, t.data_ptr(), efd.data_ptr(), eta, kT,
                               sig.data_ptr(), status.data_ptr(), stream)
    assert st == kubo.KUBO_OK, kubo.kubo_status_string(st)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return sig.cpu().numpy()


def test_noalloc_matches_kubo_ahc_twice(torch):
    big = [synth.random_model(20, 1, 1.0, 7101), synth.random_model(40, 1, 1.0, 7102)]
    small = [synth.random_model(6, 1, 1.0, 7103)]
    a = _case(torch, big, [(12, 8, 6), (4, 3, 2)], 5, 7104)
    b = _case(torch, small, [(5, 4, 3)], 3, 7105)
    print("case noalloc: 2 models (n=20, 40), then 1 model (n=6), then the first again",
          flush=True)
    ref_a = a[0].forward(a[1], a[2], 1e-3, 0.01).cpu().numpy()
    ref_b = b[0].forward(b[1], b[2], 2e-3, 0.0).cpu().numpy()
    got_a = _noalloc(torch, a, 1e-3, 0.01)
    got_b = _noalloc(torch, b, 2e-3, 0.0)
    again_a = _noalloc(torch, a, 1e-3, 0.01)
    assert np.all(np.isfinite(ref_a)) and np.all(np.isfinite(ref_b))
    assert np.array_equal(got_a, ref_a)
    assert np.array_equal(got_b, ref_b)
    assert np.array_equal(again_a, ref_a)


def test_noalloc_rejects_plan_beyond_the_array(torch):
    m = synth.random_model(32, 1, 1.0, 7106)
    plan = kubo.Plan([m], grid=(64, 64, 64), n_fermi=8, flags=kubo.KUBO_F_FORWARD_ONLY)
    assert plan.ws_bytes > kubo.KUBO_NOALLOC_MAX_BYTES
    t = kubo.to_device_t([m])
    ef = torch.zeros(1, 8, dtype=torch.float64, device="cuda")
    sig = torch.empty(1, 8, dtype=torch.float64, device="cuda")
    st = kubo.kubo_ahc_noalloc(plan.handle, t.data_ptr(), ef.data_ptr(), 1e-3, 0.0,
                               sig.data_ptr(), 0, torch.cuda.current_stream().cuda_stream)
    assert st == kubo.KUBO_E_WORKSPACE
