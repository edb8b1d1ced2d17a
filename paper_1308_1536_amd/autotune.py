"""Choice of the trailing-update path by measurement.

Every path computes the same bits (the number format and the truncation rule
fix every result), so the choice only affects speed.  For a key (arch, limbs P,
size bucket) the tuner times the candidate paths on a seeded random-mantissa
matrix of the bucket's size (capped) and caches the fastest in a JSON file
(``MPDET_AUTOTUNE_CACHE``, default ``~/.cache/mpdet/autotune.json``).
"""
from __future__ import annotations

import json
import os
import time

from . import binding, inputs

ARCH = "gfx950"


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


def candidates(P: int) -> list[str]:
    return ["valu", "mfma"] if P >= 8 and P % 8 == 0 else ["valu"]


def measure(n: int, P: int, path: str, reps: int = 2) -> float:
    """Seconds for factor + minors on a seeded n x n random-mantissa matrix."""
    import torch
    A = inputs.random_mantissas((n, n), P, 97 + n)
    pristine = binding.DeviceMp.from_host(A)
    work = binding.DeviceMp.empty(n, n, P)
    D = binding.DeviceMp.empty(1, n, P)
    c = binding.DeviceMp.empty(1, n, P)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def once():
        work.limbs.copy_(pristine.limbs)
        work.exp.copy_(pristine.exp)
        work.sign.copy_(pristine.sign)
        binding.factor(work, path, D=D, info=info)
        binding.minors(work, D, info, c=c)

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        once()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def choose_path(n: int, P: int, cap: int = 256, retune: bool = False) -> str:
    cands = candidates(P)
    if len(cands) == 1:
        return cands[0]
    key = f"{ARCH}/P{P}/N{bucket(n)}"
    db = _load()
    if not retune and key in db:
        return db[key]["path"]
    size = min(bucket(n), cap)
    times = {p: measure(size, P, p) for p in cands}
    best = min(times, key=times.get)
    db[key] = {"path": best, "seconds": times, "measured_n": size}
    _save(db)
    return best
