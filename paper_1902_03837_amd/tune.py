"""Persisted autotuning of the batched chi0 launch (xo_chi0_autotune).

The tuner in the library times a grid of (column tiles per wave, transitions per
unit, persistent workgroups per CU) on a representative batch; this module keys
the winner by (precision, G-set bucket, transition bucket, frequencies) and keeps
it in a JSON file so later runs reuse it.
"""

from __future__ import annotations

import json
import os

from . import xo


def key(prec, ngs, nts, nw):
    ngb = 1 << max(int(max(ngs)) - 1, 1).bit_length()
    ntb = 1 << max(int(max(nts)) - 1, 1).bit_length()
    return f"{prec}:ng{ngb}:nt{ntb}:nw{nw}"


def tuned(items, omegas, prec, path=None, sample=3):
    """Tune on the first `sample` items (or reuse the cached result)."""
    k = key(prec, [it[0].shape[1] for it in items], [it[0].shape[0] for it in items], len(omegas))
    cache = {}
    if path and os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    if k in cache:
        return tuple(cache[k]["tune"]), cache[k]["ms"], True
    best, ms = xo.chi0_autotune(items[:sample], omegas, prec=prec)
    cache[k] = dict(tune=list(best), ms=ms, sample=min(sample, len(items)))
    if path:
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return best, ms, False
