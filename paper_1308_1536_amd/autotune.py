"""Choice of the trailing update's path and launch shapes by measurement.

Every candidate computes the same bits (the number format and the truncation
rule fix every result, and each element gets the same operations in the same
order whatever the tiling), so tuning only changes speed.  Candidates:
- the path: the VALU lane product / one-wave update, or the INT8 MFMA
  Toeplitz contraction (P a multiple of 8);
- the tile of the VALU lane product: 2, 4 or 8 rows (= waves) x 64 columns
  per workgroup;
- the MFMA update's waves (= rows of one 32-column block) per workgroup: 1, 2
  or 4 (where their LDS fits);
- for a batch, the schedule: one launch per phase per step (lockstep; the
  persistent launch over a task queue is left out while a defect in it on
  large batches is open).
For a key (arch, limbs P, size bucket[, batch]) the tuner times the
candidates on seeded random-mantissa matrices of the bucket's size (capped)
and caches the fastest in a JSON file (``MPDET_AUTOTUNE_CACHE``, default
``~/.cache/mpdet/autotune.json``).
"""
from __future__ import annotations

import json
import os
import time

from . import binding, inputs

ARCH = "gfx950"
LANE_ROWS = (2, 4, 8)
MFMA_WAVES = (1, 2, 4)
MFMA_LDS_MAX = 64 * 1024


def cache_path() -> str:
    return os.environ.get("MPDET_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mpdet", "autotune.json"))


def bucket(n: int) -> int:
    b = 16
    while b < n:
        b *= 2
    return b


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(db: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lane_ok(P: int) -> bool:
    return P <= 128 and P % 4 == 0


def mfma_waves_ok(P: int, waves: int) -> bool:
    """the MFMA update's LDS (one reversed digit row per wave) fits a workgroup"""
    return P >= 8 and P % 8 == 0 and (4 * P + 608) * waves <= MFMA_LDS_MAX


def candidates(P: int, batch: bool = False) -> list[dict]:
    """Every launch configuration to try for P-limb numbers."""
    out = []
    # (the persistent schedule is not a candidate: on config 4's batch it has
    # given a different result for one or two large matrices in some runs, a
    # defect not found yet; `batch` keeps the signature for when it returns)
    if lane_ok(P):
        out += [{"path": "valu", "lane_rows": r} for r in LANE_ROWS]
    else:
        out.append({"path": "valu", "lane_rows": 0})
    out += [{"path": "mfma", "mfma_waves": w} for w in MFMA_WAVES if mfma_waves_ok(P, w)]
    return out


def apply(cfg: dict, device: int = 0) -> None:
    """Set the handle's launch shapes for a candidate."""
    binding.set_tuning(cfg.get("lane_rows", 0), cfg.get("mfma_waves", 0), device=device)


def measure(n: int, P: int, cfg: dict, reps: int = 2, batch: int = 0) -> float:
    """Seconds for factor + minors on a seeded n x n random-mantissa matrix
    (batch > 0: `batch` matrices of sizes spread up to n in one batched call)."""
    import torch
    sizes = [n] if not batch else [max(2, n * (b + 1) // batch) for b in range(batch)]
    hosts = [inputs.random_mantissas((s, s), P, 97 + s + 7 * b) for b, s in enumerate(sizes)]
    pristine = [binding.DeviceMp.from_host(h) for h in hosts]
    work = [binding.DeviceMp.empty(s, s, P) for s in sizes]
    apply(cfg)

    def once():
        for p, w in zip(pristine, work):
            w.limbs.copy_(p.limbs)
            w.exp.copy_(p.exp)
            w.sign.copy_(p.sign)
        if batch:
            binding.batched(work, cfg["path"], schedule=cfg.get("schedule", "lockstep"))
        else:
            D, info = binding.factor(work[0], cfg["path"])
            binding.minors(work[0], D, info)

    try:
        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps
    finally:
        apply({})


def choose(n: int, P: int, cap: int = 256, batch: int = 0, retune: bool = False) -> dict:
    """The fastest candidate for (P, size bucket[, batch]); measured once and cached."""
    cands = candidates(P, batch=bool(batch))
    key = f"{ARCH}/P{P}/N{bucket(n)}" + (f"/B{batch}" if batch else "")
    db = _load()
    if not retune and key in db and "config" in db[key]:
        return db[key]["config"]
    size = min(bucket(n), cap)
    times = [measure(size, P, c, batch=batch) for c in cands]
    best = min(range(len(cands)), key=lambda i: times[i])
    db[key] = {"config": cands[best], "candidates": cands, "seconds": times, "measured_n": size}
    _save(db)
    return cands[best]


def choose_path(n: int, P: int, cap: int = 256, retune: bool = False) -> str:
    """The path of the fastest candidate, with the handle set to its launch shapes."""
    cfg = choose(n, P, cap=cap, retune=retune)
    apply(cfg)
    return cfg["path"]
