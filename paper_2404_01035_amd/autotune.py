"""Tile-shape autotuner for the step kernels, with an on-disk cache.

The library times each candidate -- tile (bx, seg, vec) and steps per launch --
on the bound state itself (``mp_tune``: launches from the current buffer into
the other, repeated, with events on the stream) and keeps the fastest per step.  The choice is cached per
workload signature -- grid, phases, components, precision, potential,
anisotropy, the extended model, the anti-trapping current's form, batch
composition and device name -- in a JSON file, so later runs
of the same workload set the tile without timing.  Results never depend on the
tile (bitwise), only speed does.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

import numpy as np

from . import abi

CACHE_ENV = "MP_TUNE_CACHE"


def default_cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2404_01035_amd", "tiles.json")


def _extended(p) -> bool:
    """Whether p uses the extended model (the general kernels)."""
    return bool(p.potential == "obstacle_active" or any(
        np.any(np.asarray(v) != 0) for v in (p.Bt, p.Ct, p.A01, p.D01, p.tau_ab)))


def _one(p) -> list:
    return [p.dim, list(p.n), p.nphases, p.ncomp, bool(abs(p.delta).max() > 0), _extended(p)]


def signature(plist, device: str, antitrapping: int = 0) -> str:
    """Cache key of a single (len 1) or batched workload on ``device``
    (``antitrapping``: the state's mp_get_antitrapping value; it selects other kernels)."""
    p0 = plist[0]
    body = {
        "kind": "batch" if len(plist) > 1 else "single",
        "precision": p0.precision,
        "potential": p0.potential,
        "device": device,
        "antitrapping": int(antitrapping),
    }
    if len(plist) == 1:
        body["grid"] = _one(p0)
    else:
        h = hashlib.sha1(json.dumps([_one(p) for p in plist]).encode()).hexdigest()[:16]
        body["members"] = f"{len(plist)}:{h}"
    return json.dumps(body, sort_keys=True)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tiles.")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(st, plist, stream: int, device: str, reps: int = 10, cache: str | None = None,
         force: bool = False) -> dict:
    """Pick and set the tile of bound state ``st`` (built from ``plist``).

    Returns {"bx", "seg", "vec", "fuse", "source": "cache" | "timed",
    "ms": {"bx,seg,vec,fuse": ms per step}}.
    """
    path = cache or default_cache_path()
    key = signature(plist, device, abi.mp_get_antitrapping(st))
    data = _load(path)
    hit = data.get(key)
    if hit and not force:
        abi.mp_set_fusion(st, hit["fuse"])
        abi.mp_set_tile(st, hit["bx"], hit["seg"], hit["vec"])
        return dict(hit, source="cache")
    cand = abi.mp_tune_candidates(st)
    ms, best = abi.mp_tune(st, cand, reps, stream)
    rec = {
        "bx": cand[best][0],
        "seg": cand[best][1],
        "vec": cand[best][2],
        "fuse": cand[best][3],
        "ms": {",".join(map(str, c)): t for c, t in zip(cand, ms)},
    }
    data[key] = rec
    _store(path, data)
    return dict(rec, source="timed")
