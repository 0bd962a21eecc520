"""Autotuner of the batched ensemble's launch shape.

Times a short run of every candidate launch shape (elements per workgroup for
K = 4 and K = 8, i.e. the LDS tile of the analyse and residual kernels; a
persistent grid of n workgroups per compute unit or one workgroup per tile;
XCD-contiguous tile ranges or not; the register budget of the analyse kernel,
3 or 4 wavefronts per SIMD) on a scratch copy of the
ensemble state, keeps the fastest and caches the choice as JSON, keyed by the
device and the ensemble's element counts per K.  The cache file is
$SEDG_TUNING_CACHE, else ~/.cache/sedg/batch_tuning.json.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

def _candidates():
    """One workgroup per tile: the two element-per-workgroup tiles x XCD remap on/off x
    the register budget of the analyse kernel (3 or 4 waves per SIMD); persistent grids
    of 2-8 workgroups per CU at the default budget."""
    out = []
    for epb4, epb8 in ((4, 1), (8, 2)):
        for xcd in (1, 0):
            for wa in (3, 4):
                out.append(dict(epb4=epb4, epb8=epb8, blocks_per_cu=0, xcd_map=xcd, waves_analyse=wa,
                                waves_residual=3))
    for epb4, epb8, bpc in ((4, 1, 4), (4, 1, 8), (8, 2, 2), (8, 2, 4)):
        out.append(dict(epb4=epb4, epb8=epb8, blocks_per_cu=bpc, xcd_map=1, waves_analyse=3, waves_residual=3))
    return out


CANDIDATES = _candidates()


def cache_path() -> str:
    return os.environ.get("SEDG_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sedg",
                                                            "batch_tuning.json"))


def signature(batch) -> str:
    """Device name plus the ensemble's element counts per K (order independent)."""
    counts = {}
    for m in batch.meshes:
        counts[m.K] = counts.get(m.K, 0) + m.nel
    text = json.dumps([torch.cuda.get_device_name(), sorted(counts.items()), len(batch.meshes), CANDIDATES])
    return hashlib.sha1(text.encode()).hexdigest()[:16]


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time(batch, u0, steps):
    u = u0.clone()
    batch.rk_step(u, 1)                      # capture the step graph
    batch.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    batch.rk_step(u, steps)
    e1.record()
    torch.cuda.synchronize()
    batch.check()
    return e0.elapsed_time(e1) / steps


def tune(batch, u, steps: int = 2, use_cache: bool = True, candidates=None):
    """Pick and set the fastest launch shape for `batch` (state u is not modified).
    Returns (tuning, {candidate index: ms per step}, from_cache)."""
    key = signature(batch)
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        batch.set_tuning(**cache[key]["tuning"])
        return cache[key]["tuning"], cache[key].get("timings", {}), True
    cands = candidates or CANDIDATES
    timings = {}
    for i, c in enumerate(cands):
        batch.set_tuning(**c)
        timings[i] = _time(batch, u, steps)
    best = min(timings, key=timings.get)
    batch.set_tuning(**cands[best])
    entry = {"tuning": cands[best], "timings": {str(i): t for i, t in timings.items()},
             "candidates": cands}
    if use_cache:
        cache[key] = entry
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return cands[best], timings, False
