"""MI355X-native plug-and-play ULA sampler (hot path of arXiv 2511.00870).

The compute path lives in the HIP library ``libpnpula.so`` (C ABI declared in
``include/pnpula.h``); :mod:`paper_2511_00870_amd.pnpula` is its thin ctypes
binding.  :mod:`paper_2511_00870_amd.workloads` builds seeded synthetic
inputs.  Importing the package loads nothing.
"""
__all__ = ["workloads", "accounting", "pnpula"]
