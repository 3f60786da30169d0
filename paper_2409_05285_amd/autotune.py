"""Choice of the boundary-compression kernel per lattice shape, measured on
the device and kept in a JSON cache.

The library has three kernels for the same compression (register-, LDS- and
workspace-resident; which ones apply depends on chi, D and the LDS size).
`tune` times every valid one on the caller's configurations through
peps_autotune_compression (the timing runs in the library) and returns the
descriptor with the fastest selected; the result is stored under a key of
the shape, precision and chain count, so later runs read it instead of
measuring again.
"""
from __future__ import annotations

import dataclasses
import json
import os

from . import _lib, api


def _key(desc, n):
    return (f"{desc.L1}x{desc.L2}_d{desc.d}_D{desc.D}_chi{desc.chi}_model{desc.model}"
            f"_prec{desc.precision}_n{n}")


def tune(desc: api.Desc, theta, configs, cache_path=None, repeats=2):
    """(descriptor with compress_kernel set, record).  record: {"best":
    kernel name, "ms": {kernel name: ms per boundary pass}, "cached": bool}."""
    n = configs.shape[0]
    key = _key(desc, n)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    rec = cache.get(key)
    if rec is None:
        best, ms = api.peps_autotune_compression(desc, theta, configs, repeats=repeats)
        rec = {"best": _lib.COMPRESS_NAMES[best], "ms": ms}
        if cache_path:
            cache[key] = rec
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
        cached = False
    else:
        cached = True
    code = {v: k for k, v in _lib.COMPRESS_NAMES.items()}[rec["best"]]
    return dataclasses.replace(desc, compress_kernel=code), dict(rec, cached=cached)
