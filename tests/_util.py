"""Shared helpers of the test suite (inputs and tolerances; no method arithmetic)."""

import json
import os

import numpy as np

from paper_2309_06675_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_RANGES = None


def band_range(cfg: int, model_index: int = 0):
    """[E_min, E_max] of a workload model, from the oracle-written fixture."""
    global _RANGES
    if _RANGES is None:
        with open(os.path.join(ROOT, "tests", "golden", "fermi_ranges.json")) as f:
            _RANGES = json.load(f)["ranges"]
    return _RANGES[str(cfg)][model_index]


def workload_fermi(cfg: int, wl=None):
    """Fermi levels [n_models, n_fermi] of workload cfg."""
    wl = wl or synth.workload(cfg)
    if cfg == 0:
        return np.zeros((1, 1))
    out = []
    for i in range(len(wl.models)):
        lo, hi = band_range(cfg, i)
        out.append(synth.fermi_levels(lo, hi, wl.n_fermi))
    return np.array(out)


# worst error/bound ratio of every parity comparison of the session; conftest
# writes them to parity_margins.json in the folder KUBO_MARGINS_DIR names (if set)
# at the end of the session
MARGINS = []


def record_margin(kind: str, what: str, ratio: float, rel: float):
    MARGINS.append({"kind": kind, "case": what, "err_over_bound": float(ratio), "rel": rel})


def assert_sigma_parity(got, ref, sabs, rel=1e-10, what=""):
    """|got - ref| <= rel * max(|ref|, S_abs) element by element.

    S_abs is the oracle's (1/N_k) sum of absolute band-pair terms, which keeps
    the test meaningful when sigma is small through cancellation."""
    got = np.asarray(got, float).reshape(-1)
    ref = np.asarray(ref, float).reshape(-1)
    sabs = np.asarray(sabs, float).reshape(-1)
    bound = rel * np.maximum(np.abs(ref), sabs)
    err = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
    record_margin("sigma", what, ratio.max() if ratio.size else 0.0, rel)
    print(f"parity {what}: max err/bound {ratio.max():.3e} (rel {rel:g})", flush=True)
    bad = np.nonzero(err > bound)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{what}: {bad.size} of {got.size} outside {rel:g}; first j={i}: "
                             f"got {got[i]!r} ref {ref[i]!r} sabs {sabs[i]!r}")


def slab_sample(nk: int, count: int, seed: int):
    """A deterministic pseudo-random slab (k_begin, k_count) of a grid of nk points."""
    u = synth.uniform01(seed, 1)[0]
    kb = int(u * (nk - count))
    return kb, count


def assert_grad_close(got, ref, rel, what=""):
    """|G - G_ref| <= rel * max(|G_ref|, 1e-3 max|G_ref|) entry by entry."""
    got = np.asarray(got).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    bound = rel * np.maximum(np.abs(ref), 1e-3 * scale)
    ratio = (err / bound).max() if bound.size and scale > 0 else (0.0 if err.max() == 0 else np.inf)
    record_margin("gradient", what, ratio, rel)
    print(f"gradient {what}: max err/bound {ratio:.3e} (rel {rel:g})", flush=True)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{what}: {bad.size} of {err.size} entries off; worst err/bound "
                           f"{ratio:.3e}")
