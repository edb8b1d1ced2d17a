"""Loss of accuracy by comparing precisions (the method of Sec. 4.3).

The paper estimates how many digits Gaussian elimination loses by computing
the same normalised minors at two precisions and counting the digits on
which they agree, as a function of the matrix size N; the agreement decays
linearly, and the slope of a least-squares line through it is the loss per
row operation.  Here the normalised minors of every leading block come from
one run (mp_det_all_minors, then mp_det_normalize_minors: row r holds
delta_{r+1, n} = c_n / c_1 of the leading (r+1) x (r+1) block), at p and at
2p bits on the same exact input (each precision truncates the same rationals),
so one pair of runs gives the agreement for every N <= N_max.

Only the comparison and the line fit run on the host; every number compared
comes from the library's kernels.
"""
from __future__ import annotations

import math

import numpy as np


def agreement_bits(a_limbs, a_exp, a_sign, b_limbs, b_exp, b_sign) -> float:
    """Bits on which x (p = 32 * len(a_limbs) bits) agrees with y (any
    precision): log2(|y| / |x - y|), computed exactly; capped at x's
    precision (equal values or x = y = 0), 0 when exactly one of them is 0."""
    Pa, Pb = len(a_limbs), len(b_limbs)
    ma = int.from_bytes(np.ascontiguousarray(a_limbs, "<u4").tobytes(), "little")
    mb = int.from_bytes(np.ascontiguousarray(b_limbs, "<u4").tobytes(), "little")
    cap = float(32 * Pa)
    if ma == 0 and mb == 0:
        return cap
    if ma == 0 or mb == 0:
        return 0.0
    # x = +-ma 2^(ea - 32 Pa), y = +-mb 2^(eb - 32 Pb), on a common scale
    sa, sb = int(a_exp) - 32 * Pa, int(b_exp) - 32 * Pb
    E = min(sa, sb)
    A = (-1 if a_sign else 1) * (ma << (sa - E))
    B = (-1 if b_sign else 1) * (mb << (sb - E))
    d = abs(A - B)
    if d == 0:
        return cap
    # math.log2 takes integers of any size; disagreement beyond |y| counts as 0
    return max(0.0, min(cap, math.log2(abs(B)) - math.log2(d)))


def row_agreement(C_lo, C_hi, r: int) -> tuple[float, float]:
    """(smallest, mean) agreement over entries 0..r of row r of two
    normalised-minors arrays (host containers, [rows][cols] numbers)."""
    vals = [agreement_bits(C_lo.limbs[r, i], C_lo.exp[r, i], C_lo.sign[r, i],
                           C_hi.limbs[r, i], C_hi.exp[r, i], C_hi.sign[r, i]) for i in range(r + 1)]
    return min(vals), float(np.mean(vals))


def fit_line(x, y) -> tuple[float, float]:
    """Least-squares line y = slope * x + intercept."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    A = np.vstack([x, np.ones_like(x)]).T
    (slope, intercept), *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(slope), float(intercept)


def normalised_all_minors(A_host, path: str = "auto"):
    """Factor A on the GPU, then every leading block's last-column minors and
    their normalisation (row r: delta_{r+1, n} = c_n / c_1).  Returns the host
    container and the factorisation's info."""
    import torch

    from . import binding
    A = binding.DeviceMp.from_host(A_host)
    D, info = binding.factor(A, path)
    C = binding.all_minors(A, D, info)
    Dn = binding.normalize_minors(C)
    torch.cuda.synchronize()
    return Dn.to_host(), int(info.item())


def report(make_input, n_max: int, P: int, rows=None, path: str = "auto") -> dict:
    """Agreement between p = 32P and 2p bits of the normalised minors of every
    leading block up to n_max: per block size N (rows r = N - 1) the smallest
    and mean agreement in bits over n = 1..N, and a line fitted through the
    smallest (bits lost per row operation = -slope).  make_input(n, P) gives
    the n x n input at P limbs from the same exact values for every P."""
    lo, info_lo = normalised_all_minors(make_input(n_max, P), path)
    hi, info_hi = normalised_all_minors(make_input(n_max, 2 * P), path)
    if info_lo != 0 or info_hi != 0:
        raise ArithmeticError(f"elimination stopped (info {info_lo} at p, {info_hi} at 2p)")
    rows = list(rows) if rows is not None else sorted(set(np.linspace(1, n_max - 1, 24).astype(int).tolist()))
    N, mins, means = [], [], []
    for r in rows:
        mn, me = row_agreement(lo, hi, r)
        N.append(r + 1)
        mins.append(mn)
        means.append(me)
    slope, intercept = fit_line(N, mins)
    return {"bits": 32 * P, "N": N, "min_agree_bits": mins, "mean_agree_bits": means,
            "fit": {"slope_bits_per_row": slope, "intercept_bits": intercept,
                    "bits_lost_per_row_operation": -slope}}


def main(argv=None) -> None:
    """python -m paper_1308_1536_amd.accuracy --kind hilbert|cauchy --n N --limbs P
    prints the report as one JSON line (p = 32P bits against 2p)."""
    import argparse
    import json

    from . import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--kind", choices=["hilbert", "cauchy"], default="cauchy")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--limbs", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1308_0200)
    ap.add_argument("--points", type=int, default=24)
    a = ap.parse_args(argv)
    if a.kind == "hilbert":
        make = inputs.hilbert
    else:  # the nearly singular Cauchy generator of config 2 (nodes on [0, 1000])
        def make(n, P):
            return inputs.cauchy_dyadic(n, P, a.seed)[0]
    rows = sorted(set(np.linspace(1, a.n - 1, a.points).astype(int).tolist()))
    r = report(make, a.n, a.limbs, rows=rows)
    r["kind"] = a.kind
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
