"""Write fermi_ranges.json: the band range [E_min, E_max] of each workload model.

The Fermi levels of the workloads are spread evenly over the band range of
their model (n_fermi levels, ends included).  The range is taken over a
coarse 10^3 grid (6^3 for the n = 128 model) and computed by the CPU oracle
only.  Run from the repository root:  python tests/golden/make_fermi_ranges.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2309_06675_amd import synth as S  # noqa: E402


def main():
    out = {"grid": {"default": [10, 10, 10], "n128": [6, 6, 6]}, "ranges": {}}
    for cfg in (0, 1, 2, 3, 4):
        wl = S.workload(cfg)
        rng = []
        for m in wl.models:
            g = (6, 6, 6) if m.n >= 128 else (10, 10, 10)
            rng.append(list(O.band_range(m.t, m.R, g)))
        out["ranges"][str(cfg)] = rng
        print(cfg, wl.name, rng[:2], flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "fermi_ranges.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
