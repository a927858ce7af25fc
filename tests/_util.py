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


def assert_sigma_parity(got, ref, sabs, rel=1e-10, what=""):
    """|got - ref| <= rel * max(|ref|, S_abs) element by element.

    S_abs is the oracle's (1/N_k) sum of absolute band-pair terms, which keeps
    the test meaningful when sigma is small through cancellation."""
    got = np.asarray(got, float).reshape(-1)
    ref = np.asarray(ref, float).reshape(-1)
    sabs = np.asarray(sabs, float).reshape(-1)
    bound = rel * np.maximum(np.abs(ref), sabs)
    bad = np.nonzero(np.abs(got - ref) > bound)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{what}: {bad.size} of {got.size} outside {rel:g}; first j={i}: "
                             f"got {got[i]!r} ref {ref[i]!r} sabs {sabs[i]!r}")


def slab_sample(nk: int, count: int, seed: int):
    """A deterministic pseudo-random slab (k_begin, k_count) of a grid of nk points."""
    u = synth.uniform01(seed, 1)[0]
    kb = int(u * (nk - count))
    return kb, count
