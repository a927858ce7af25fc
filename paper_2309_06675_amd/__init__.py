"""Kubo-formula anomalous Hall conductivity on MI355X (gfx950).

The compute path is the HIP library ``libkubo.so`` behind the C ABI declared
in ``include/kubo.h``; :mod:`paper_2309_06675_amd.kubo` is its thin Python
binding.  Import the binding explicitly; this package import itself loads
nothing native.
"""

__all__ = ["kubo", "synth"]
