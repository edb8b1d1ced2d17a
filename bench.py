#!/usr/bin/env python3
"""Throughput of the multiprecision determinant hot path on one MI355X.

The default workload is configuration 3: one N=2048 Cauchy matrix of
32768-bit numbers on the INT8-MFMA path.  Its whole solve -- Gaussian
elimination without pivoting (every D_k and det), then the last-column minors
-- takes tens of seconds, so one timed solve is split into K consecutive
segments of about equal trailing-update work: step s runs elimination steps
b_s .. b_{s+1}-1 in place, the last step also the minors, and the K steps
together are exactly one time to solution (the copy of the pristine matrix
into the work buffer is inside the first step).  The W warm-up steps are the
first W segments of a throwaway solve.

    python bench.py [--steps K] [--warmup W] [--config 3] [--path auto|valu|mfma]

Configurations 1, 2 and 4 keep whole passes as steps: one step is the whole
path over every matrix of the workload.  Configuration 5 is timed in part
(--factor-steps).

Prints ONE JSON line.  `value` is algorithmic 8-bit limb MACs per second:
U(N) * (p/8)^2 per matrix, U(N) = (N-1)N(2N-1)/6 trailing updates, divided by
the wall time.  `roofline` describes the dominant kernel, timed live with HIP
events on its launch stream during the timed steps; `cpu_baseline` times the
CPU oracle on a bounded leading block of the first matrix (same unit), which
also checks the GPU's D_1..D_K bit for bit (prefix property of elimination
without pivoting).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks (dense) and the derived integer-VALU rate.
PEAK_INT8_MFMA_TOPS = 5.0e15           # int8 ops/s; a MAC is 2 ops
PEAK_INT8_MAC = PEAK_INT8_MFMA_TOPS / 2
# v_mad_u64_u32 (32x32->64 multiply-add) issues at the rate of the float64
# FMA (78.6 TFLOP/s = 39.3e12 FMA/s): 64 lanes per clock per CU -> 256 CUs * 64
# * 2.4 GHz.  bench also reports the rate its probe kernel measures.
PEAK_VALU_MAC32 = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12                      # bytes/s


def FINISH_BYTES(P: int) -> int:
    """HBM bytes the finish must move per element update: read a_ij (4P limb
    bytes + 8 exponent + 4 sign) and the product record (4(P+1)), write a_ij."""
    return 2 * (4 * P + 12) + 4 * (P + 1)

METRIC = "time to det+all D_k+last-col minors at (N,bits); limb-MAC/s vs INT8 MFMA peak"
DEFAULT_PATH = {1: "valu", 2: "valu", 3: "mfma", 4: "auto", 5: "mfma"}


def workload(cfg: int):
    from paper_1308_1536_amd import inputs
    if cfg == 1:
        c = inputs.config_c1()
        return ("config 1: N=64, 1024-bit: integer-node Cauchy + random integers in [-1000,1000]",
                [("cauchy", c["cauchy"][0]), ("randint", c["randint"][0])])
    if cfg == 2:
        c = inputs.config_c2()
        return ("config 2: N=512, 4096-bit: dyadic Cauchy (nodes on [0,1000], delta in [1e-6,1e-3]) "
                "+ random mantissas (exp in [-4,4])",
                [("cauchy", c["cauchy"][0]), ("randmant", c["randmant"])])
    if cfg == 3:
        c = inputs.config_c3()
        return ("config 3: N=2048, 32768-bit: interlaced dyadic Cauchy on [0,1000]",
                [("cauchy", c["cauchy"][0])])
    if cfg == 4:
        return ("config 4: 256 matrices, N uniform in [16,384], 2048-bit, half random mantissas / half "
                "dyadic Cauchy, one batched elimination", inputs.config_c4())
    if cfg == 5:
        c = inputs.config_c5()
        return ("config 5: N=6144, 32768-bit: dyadic Cauchy, sorted nodes on [0,10000] (155 GB)",
                [("cauchy", c["cauchy"][0])])
    raise SystemExit(f"bench.py: config {cfg} is not a single-GPU bench workload")


def mfma_copies(P: int) -> int:
    """shifted LDS copies of the digit row the MFMA update keeps per wave (its
    template argument): 4 where two waves' copies fit 64 KB"""
    lr = 4 * P + 608
    return 4 if 4 * lr * 2 <= 64 * 1024 else 1


def lane_issued_mac32(P: int) -> int:
    """v_mad_u64_u32 the VALU lane product issues per element update: radix-2^28
    digits, Comba blocks of 8 columns from the first column it forms (the
    truncated product), steps padded to whole blocks of 8 -- a wave's rare
    second, whole product is not counted.  The algorithmic figure is P^2."""
    nd = (32 * P + 27) // 28
    c0 = (32 * (P - 1) - 68) // 28
    c0 = c0 if c0 >= 8 else 0
    steps = 0
    for r0 in range(c0, 2 * nd, 8):
        alo, ahi = max(0, r0 - nd + 1), min(r0 + 7, nd - 1)
        steps += (ahi - alo + 8) // 8 * 8  # padded to whole blocks of 8 steps
    return 8 * steps


def mfma_issued_mac8(P: int) -> int:
    """int8 MACs the MFMA update issues per element update: every K-step of a
    chunk is 8 MFMAs of 32x32x32, 8 * 32 * 32 MACs per column, over the chunks
    from the first one formed (the truncated product); a wave's rare second,
    whole product is not counted.  The algorithmic figure is (4P)^2."""
    P8 = 4 * P
    rb = 0 if P8 >= 1 << 15 else max(0, (4 * P - 11) // 32 * 32)
    steps = 0
    for chunk in range((2 * P8 - rb + 255) // 256):
        r0 = rb + 256 * chunk
        c_lo = r0 - 31 - P8
        c_lo = 0 if c_lo <= 0 else (c_lo + 31) & ~31
        steps += (min(P8, r0 + 224) - c_lo) // 32 + 1
    return steps * 8 * 32 * 32


def issued(kind: str, P: int, frac: float) -> dict:
    """What the kernel multiplies per update next to the algorithmic figure,
    and the share of the unit's peak those issued multiply-adds take."""
    if kind == "alu":
        n, alg = lane_issued_mac32(P), P * P
    else:
        n, alg = mfma_issued_mac8(P), 16 * P * P
    return {"issued_per_update": n, "issued_over_algorithmic": n / alg, "issued_frac": frac * n / alg}


def kernel_source_sha256() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1308_1536_amd", "csrc", "*"))):
        if f.endswith((".h", ".hip")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def load_traffic(cfg: int) -> dict:
    """profiles/traffic_config<cfg>.json (per-launch HBM bytes measured with
    rocprofv3 counters), keyed by kernel -- empty when absent or when the
    kernel sources have changed since the counters were taken"""
    path = os.path.join(ROOT, "profiles", f"traffic_config{cfg}.json")
    try:
        with open(path) as fh:
            db = json.load(fh)
    except (OSError, ValueError):
        return {}
    if db.get("source_sha256") != kernel_source_sha256():
        return {}
    return db.get("kernels", {})


def cached_workload(cfg: int, cache: str | None):
    """workload(cfg), with the generated matrices stored as .npy files under
    `cache` (numpy's own format, loaded without pickle)."""
    import numpy as np

    from paper_1308_1536_amd.inputs import MpArray
    if cache is None:
        return workload(cfg)
    root = os.path.join(cache, f"config{cfg}")
    index = os.path.join(root, "index.json")
    if os.path.exists(index):
        with open(index) as fh:
            meta = json.load(fh)
        mats = []
        for k, name in enumerate(meta["names"]):
            parts = [np.load(os.path.join(root, f"{k}_{f}.npy"), allow_pickle=False)
                     for f in ("limbs", "exp", "sign")]
            mats.append((name, MpArray(*parts)))
        return meta["desc"], mats
    desc, mats = workload(cfg)
    os.makedirs(root, exist_ok=True)
    for k, (_, m) in enumerate(mats):
        for f in ("limbs", "exp", "sign"):
            np.save(os.path.join(root, f"{k}_{f}.npy"), getattr(m, f), allow_pickle=False)
    with open(index, "w") as fh:
        json.dump({"desc": desc, "names": [nm for nm, _ in mats]}, fh)
    return desc, mats


def unit_work(mats):
    from paper_1308_1536_amd.inputs import limb_macs_int8, u_count
    macs = sum(limb_macs_int8(m.exp.shape[0], m.limbs.shape[-1]) for _, m in mats)
    upd = sum(u_count(m.exp.shape[0]) for _, m in mats)
    return macs, upd


# Cauchy matrices of the workloads, by configuration and matrix name: the
# generator's node parameters, for the closed-form checks
CAUCHY_NODES = {2: {"cauchy": (512, 2, 0.0, 1000.0)}, 3: {"cauchy": (2048, 3, 0.0, 1000.0)},
                5: {"cauchy": (6144, 5, 0.0, 10000.0)}}


def _mp_int(limbs, e, s, P):
    """(-1)^s m 2^(e - 32P) as (signed integer m, exponent e - 32P)"""
    import numpy as np
    m = int.from_bytes(np.ascontiguousarray(limbs, "<u4").tobytes(), "little")
    return (-m if s else m), int(e) - 32 * P


def _rel_err_bits(got, exact):
    """log2(|got - exact| / |exact|) for Fractions (-inf when equal)"""
    import math
    d = abs(got - exact)
    if d == 0:
        return float("-inf")
    return math.log2(d.numerator) - math.log2(d.denominator) - (math.log2(abs(exact.numerator))
                                                                - math.log2(exact.denominator))


def all_minors_invariant_bits(A_host, C_host, D_host, rows):
    """Exact check of sampled rows of the minors of every leading block:
    sum_{i<=r} C[r][i] a_ir = D_{r+1} for the leading (r+1) x (r+1) block
    (Sec. 3 per block), as log2(|sum - D| / sum |terms|); the worst row."""
    import math
    P = A_host.limbs.shape[-1]
    worst = float("-inf")
    for r in rows:
        terms = []
        for i in range(r + 1):
            mc, ec = _mp_int(C_host.limbs[r, i], C_host.exp[r, i], C_host.sign[r, i], P)
            ma, ea = _mp_int(A_host.limbs[i, r], A_host.exp[i, r], A_host.sign[i, r], P)
            terms.append((mc * ma, ec + ea))
        md, ed = _mp_int(D_host.limbs[r], D_host.exp[r], D_host.sign[r], P)
        emin = min([e for _, e in terms] + [ed])
        S = sum(v << (e - emin) for v, e in terms)
        absS = sum(abs(v) << (e - emin) for v, e in terms)
        diff = abs(S - (md << (ed - emin)))
        if diff:
            worst = max(worst, math.log2(diff) - math.log2(absS))
    return worst


def full_size_checks(cfg, name, A_host, LU_dev, D_host, c_host, size, steps_done=None):
    """Exact checks at the workload's full size (no oracle run needed):
    - Cauchy matrices: sampled pivots u_kk against the closed form
      u_kk = prod_{i<k} (x_k - x_i)(y_i - y_k) / ((x_k - y_k) prod_{i<k} (x_i - y_k)(x_k - y_i)),
      evaluated exactly; reported as the largest relative error in bits;
    - after a whole factorisation: the minors' invariant sum_i c_i a_iN = det(A)
      (exact products and sum), reported relative to sum_i |c_i a_iN| in bits."""
    import math
    from fractions import Fraction

    from paper_1308_1536_amd import inputs
    N, P = A_host.exp.shape[0], A_host.limbs.shape[-1]
    out = {}
    spec = CAUCHY_NODES.get(cfg, {}).get(name)
    if spec is not None:
        n0, sc, lo, hi = spec
        x, y = inputs.dyadic_nodes(n0, inputs.config_seed(sc), lo, hi)
        x, y = [Fraction(v) for v in x[:N]], [Fraction(v) for v in y[:N]]
        F = max(max(v.denominator for v in x + y).bit_length() - 1, 0)
        X = [int(v * (1 << F)) for v in x]
        Y = [int(v * (1 << F)) for v in y]
        last = N if steps_done is None else min(N, steps_done + 1)
        ks = sorted(set([0, 1, 2, last - 1] + [int(round(t * (last - 1) / 40)) for t in range(41)]))
        import torch
        idx = torch.tensor(ks, device=LU_dev.limbs.device)
        dl = LU_dev.limbs[idx, idx].cpu().numpy().view("uint32")
        de = LU_dev.exp[idx, idx].cpu().numpy()
        ds = LU_dev.sign[idx, idx].cpu().numpy()
        worst = float("-inf")
        for t, k in enumerate(ks):
            num, den = 1, X[k] - Y[k]
            for i in range(k):
                num *= (X[k] - X[i]) * (Y[i] - Y[k])
                den *= (X[i] - Y[k]) * (X[k] - Y[i])
            exact = Fraction(num << F, den)
            m, e = _mp_int(dl[t], de[t], ds[t], P)
            got = Fraction(m) * (Fraction(2) ** e)
            worst = max(worst, _rel_err_bits(got, exact))
        out["cauchy_pivots_checked"] = len(ks)
        out["cauchy_pivot_max_rel_err_bits"] = worst
        out["cauchy_pivot_bits_lost"] = worst + 32 * P if worst != float("-inf") else 0.0
    if c_host is not None and steps_done is None:
        terms = []
        for i in range(N):
            mc, ec = _mp_int(c_host.limbs[i], c_host.exp[i], c_host.sign[i], P)
            ma, ea = _mp_int(A_host.limbs[i, N - 1], A_host.exp[i, N - 1], A_host.sign[i, N - 1], P)
            terms.append((mc * ma, ec + ea))
        md, ed = _mp_int(D_host.limbs[N - 1], D_host.exp[N - 1], D_host.sign[N - 1], P)
        emin = min([e for _, e in terms] + [ed])
        S = sum(v << (e - emin) for v, e in terms)
        absS = sum(abs(v) << (e - emin) for v, e in terms)
        diff = abs(S - (md << (ed - emin)))
        out["minors_invariant_rel_err_bits"] = (math.log2(diff) - math.log2(absS)) if diff else float("-inf")
    return out


def minors_invariant(lastcol, D_host, c_host, N: int, P: int) -> dict:
    """sum_i c_i a_iN = det(A) = D_N, exactly, relative to sum_i |c_i a_iN| in
    bits (lastcol: the input's last column as an N x 1 host array)."""
    import math
    terms = []
    for i in range(N):
        mc, ec = _mp_int(c_host.limbs[i], c_host.exp[i], c_host.sign[i], P)
        ma, ea = _mp_int(lastcol.limbs[i, 0], lastcol.exp[i, 0], lastcol.sign[i, 0], P)
        terms.append((mc * ma, ec + ea))
    md, ed = _mp_int(D_host.limbs[N - 1], D_host.exp[N - 1], D_host.sign[N - 1], P)
    emin = min([e for _, e in terms] + [ed])
    S = sum(v << (e - emin) for v, e in terms)
    absS = sum(abs(v) << (e - emin) for v, e in terms)
    diff = abs(S - (md << (ed - emin)))
    return {"minors_invariant_rel_err_bits": (math.log2(diff) - math.log2(absS)) if diff else float("-inf")}


def cpu_baseline(A, gpu_D, budget_s: float):
    """Time the oracle (factor + minors) on the leading K x K block of A, K
    grown until one run takes at least a third of the budget (or K = N)."""
    import numpy as np

    import oracle
    from paper_1308_1536_amd.inputs import MpArray, limb_macs_int8
    oracle.build(force=False)
    N, P = A.exp.shape[0], A.limbs.shape[-1]
    threads = oracle.default_threads()
    K = min(N, 32)
    while True:
        sub = MpArray(A.limbs[:K, :K].copy(), A.exp[:K, :K].copy(), A.sign[:K, :K].copy())
        t0 = time.perf_counter()
        f, c = oracle.det_pipeline(sub, threads)
        dt = time.perf_counter() - t0
        if dt >= budget_s / 3 or K == N:
            break
        # time ~ K^3: aim at the budget
        scale = (budget_s / 2 / max(dt, 1e-3)) ** (1 / 3)
        K = min(N, max(K + 8, int(K * min(scale, 2.5))))
    prefix_ok = bool(np.array_equal(gpu_D.limbs[:K], f.D.limbs) and np.array_equal(gpu_D.exp[:K], f.D.exp)
                     and np.array_equal(gpu_D.sign[:K], f.D.sign))
    return {"value": limb_macs_int8(K, P) / dt, "unit": "limb-MAC/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle factor+D_k+minors on the leading {K}x{K} block of the first matrix "
                      f"({32 * P}-bit), {dt:.2f} s wall",
            "seconds": dt, "prefix_D_bit_exact": prefix_ok}


def bench_elimination_steps(args):
    """--factor-steps K: time elimination steps W .. W+K-1 of the workload's
    first matrix in place (mp_det_factor_steps; the first W steps run untimed,
    with the workspace allocation), for matrices too large to repeat whole
    steps of the path on (configuration 5: 155 GB, about 13 minutes a
    factorisation).  With --warmup 0 and K = N the run is the whole
    factorisation, then the minors: its time is the time to solution and the
    minors' invariant is checked exactly.  The JSON line is marked as a partial run: `value` is the
    algorithmic limb-MACs of the K timed elimination steps over their time,
    and `extrapolated_factor_s` scales each kernel's time to the whole
    factorisation by its work (trailing-block kernels by the sum of m^2, the
    multipliers by the sum of m, the pivot by the step count).  The oracle on a
    leading block checks D_1..D_K' bit for bit (prefix property)."""
    import numpy as np

    from paper_1308_1536_amd.inputs import MpArray
    desc, mats = cached_workload(args.config, args.input_cache)
    name, Ah = mats[0]
    N, P = Ah.exp.shape[0], Ah.limbs.shape[-1]
    W = max(0, min(args.warmup, N))
    K = max(1, min(args.factor_steps, N - W))
    lead = min(N, 64)
    Alead = MpArray(Ah.limbs[:lead, :lead].copy(), Ah.exp[:lead, :lead].copy(), Ah.sign[:lead, :lead].copy())
    whole = W == 0 and K == N  # the whole factorisation: the minors and their invariant follow
    # the last column, for the minors' invariant sum_i c_i a_iN = det (the
    # factorisation overwrites A on the device)
    lastcol = MpArray(Ah.limbs[:, N - 1:].copy(), Ah.exp[:, N - 1:].copy(), Ah.sign[:, N - 1:].copy())
    print(f"[bench] {desc}: uploading", file=sys.stderr, flush=True)

    import torch

    from paper_1308_1536_amd import binding
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    A = binding.DeviceMp.from_host(Ah)
    # the pivot check needs only the shape and P of the host matrix
    Alead_full = MpArray(np.zeros((N, 0, P), np.uint32), np.zeros((N, N), np.int64)[:, :0],
                         np.zeros((N, 0), np.int32))
    del Ah, mats
    D = binding.DeviceMp.empty(1, N, P)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    path = args.path or DEFAULT_PATH.get(args.config, "mfma")
    torch.cuda.synchronize()
    binding.factor_steps(A, D, info, 0, W, path)
    torch.cuda.synchronize()
    print(f"[bench] {W} untimed steps done", file=sys.stderr, flush=True)
    binding.profile_begin()
    t0 = time.perf_counter()
    chunk = 8  # report progress every few steps (each is ~1 s at N = 6144, 32K bits)
    for k0 in range(W, W + K, chunk):
        binding.factor_steps(A, D, info, k0, min(W + K, k0 + chunk), path)
        torch.cuda.synchronize()
        print(f"[bench] elimination steps {k0}..{min(W + K, k0 + chunk) - 1} done", file=sys.stderr, flush=True)
    c = None
    if whole:
        c = binding.minors(A, D, info)
        torch.cuda.synchronize()
        print("[bench] minors done", file=sys.stderr, flush=True)
    secs = time.perf_counter() - t0
    prof = binding.profile_end()
    if int(info.item()) != 0:
        raise SystemExit(f"bench.py: factorisation reported info {int(info.item())}")
    ms_ = [N - k - 1 for k in range(W, W + K)]
    all_m = [N - k - 1 for k in range(N)]
    s2, s2all = sum(m * m for m in ms_), sum(m * m for m in all_m)
    s1, s1all = sum(ms_), sum(all_m)
    P8 = 4 * P
    macs = s2 * P8 * P8
    ext = 0.0
    for kname, (kms, _) in prof.items():
        if kname in ("update_mfma", "update_valu", "update_finish", "mfma_prep"):
            ext += kms / 1e3 * s2all / s2
        elif kname == "divide":
            ext += kms / 1e3 * s1all / s1
        elif kname == "pivot_divide":
            ext += kms / 1e3 * N / K
    roof = None
    upd_key = "update_mfma" if prof.get("update_mfma", (0, 0))[1] else "update_valu"
    if prof.get(upd_key, (0, 0))[1]:
        kms, kn = prof[upd_key]
        if upd_key == "update_mfma":
            mp = binding.measure_peak("mfma_i8")
            ach = macs / (kms / 1e3)
            roof = {"bound": "mfma", "achieved": 2 * ach / 1e12, "peak": PEAK_INT8_MFMA_TOPS / 1e12,
                    "unit": "TOP/s", "frac": ach / PEAK_INT8_MAC, "kernel": f"k_update_mfma<{mfma_copies(P)}>",
                    "measured_peak": 2 * mp / 1e12, "frac_of_measured_peak": ach / mp,
                    "measured_clock_ghz": binding.measure_peak("mfma_clock") / 1e9, "traffic": None,
                    "avg_launch_ms": kms / kn, "launches": kn}
            roof.update(issued("mfma", P, roof["frac"]))
        else:
            ach = s2 * P * P / (kms / 1e3)
            roof = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_VALU_MAC32 / 1e12, "unit": "Tmac32/s",
                    "frac": ach / PEAK_VALU_MAC32, "kernel": "k_update_valu", "traffic": None,
                    "avg_launch_ms": kms / kn, "launches": kn}
    what = (f"{desc} -- the whole factorisation and the minors, one pass" if whole else
            f"{desc} -- elimination steps {W}..{W + K - 1} of {N - 1} only (partial run)")
    out = {"metric": METRIC, "value": macs / secs, "unit": "limb-MAC/s", "n_gpus": 1, "steps": 1, "warmup": W,
           "ms_per_step": secs * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "i8" if path == "mfma" else "u32", "data": "synthetic",
           "config": {"workload": what, "N": N, "bits": 32 * P, "matrices": 1, "path": path,
                      "partial": not whole, "elimination_steps_timed": K, "limb_macs_timed": macs},
           "roofline": roof, "kernel_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]}}
    if whole:
        out["time_to_solution_s"] = secs
    else:
        out["extrapolated_factor_s"] = ext
    if not args.no_checks:
        chk = full_size_checks(args.config, name, Alead_full, A, None, None, 0, steps_done=W + K)
        if whole:
            # the minors' invariant, exactly: last column against c and D_N
            chk.update(minors_invariant(lastcol, D.row(0), c.row(0), N, P))
        out["full_size_checks"] = {name: chk}
    if not args.no_cpu_baseline:
        Dh = D.row(0)
        done = W + K
        sub = MpArray(Alead.limbs[:min(lead, done), :min(lead, done)],
                      Alead.exp[:min(lead, done), :min(lead, done)],
                      Alead.sign[:min(lead, done), :min(lead, done)])
        out["cpu_baseline"] = cpu_baseline(sub, Dh, args.cpu_budget)
    print(json.dumps(out), flush=True)


def bench_all_minors(args, mats, work, Ds, cs, binfo, infos, P):
    """mp_det_all_minors on every factored matrix: wall time per pass over the
    workload (the matrices at once on separate streams and handles), the VALU
    rate of its row sweeps (N^3/6 - N/6 multiply-subtracts of P-limb numbers,
    P^2 32-bit MACs each, timed live with HIP events over the calls made one
    after another; avg_launch_ms is that time over the sweep launches), row
    N-1 against mp_det_minors bit for bit, and the exact invariant on sampled
    rows."""
    import torch

    from paper_1308_1536_amd import binding
    Cs = [binding.DeviceMp.empty(w.rows, w.rows, P, w.limbs.device) for w in work]
    info_of = [binfo[b:b + 1] if binfo is not None else infos[b] for b in range(len(work))]
    # independent matrices run concurrently, as in bench_backward
    S = min(int(os.environ.get("MPDET_BWD_STREAMS", "16")), len(work))
    streams = [torch.cuda.Stream() for _ in range(S)]
    handles = [binding.Handle(work[0].limbs.device.index or 0) for _ in range(S)]

    def run(concurrent=True):
        torch.cuda.synchronize()
        for b, (w, D, C, inf) in enumerate(zip(work, Ds, Cs, info_of)):
            if concurrent:
                binding.all_minors(w, D, inf, C, stream=streams[b % S], h=handles[b % S])
            else:
                binding.all_minors(w, D, inf, C)
        torch.cuda.synchronize()

    run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # kernel time of one pass, one matrix after another on the shared handle
    binding.profile_begin()
    run(concurrent=False)
    prof = binding.profile_end()
    kms, _ = prof["all_minors"]
    ops = sum((w.rows ** 3 - w.rows) // 6 for w in work)
    lane = P <= 128 and P % 4 == 0  # the sweeps run on the lane product and the tile finish
    launches = sum(w.rows - 1 for w in work) * (2 if lane else 1)
    rate = ops * P * P / (kms / 1e3)
    mp = binding.measure_peak("mad64")
    last_same = all(torch.equal(C.limbs[-1], c.limbs[0]) and torch.equal(C.exp[-1], c.exp[0])
                    and torch.equal(C.sign[-1], c.sign[0]) for C, c in zip(Cs, cs))
    checks = {}
    if not args.no_checks:
        for (nm, m), C, D in zip(mats, Cs, Ds):
            n = m.exp.shape[0]
            rows = sorted(set([0, 1, n // 3, (2 * n) // 3, n - 2, n - 1]) & set(range(n)))
            checks[nm] = {"rows": rows, "max_rel_err_bits": all_minors_invariant_bits(m, C.to_host(), D.row(0),
                                                                                      rows)}
    return {"ms_per_pass": ms, "streams": S, "multiply_subtracts": ops,
            "roofline": {"bound": "alu", "kernel": "k_prod_lane_r1 + k_finish_r1" if lane else "k_adj_w",
                         "achieved": rate / 1e12,
                         "peak": PEAK_VALU_MAC32 / 1e12, "unit": "Tmac32/s", "frac": rate / PEAK_VALU_MAC32,
                         "measured_peak": mp / 1e12, "frac_of_measured_peak": rate / mp,
                         "avg_launch_ms": kms / launches, "launches": launches},
            "last_row_equals_minors": bool(last_same), "invariant_checks": checks}


def adjugate_column_bits(A_host, adjT_host, det_host, cols):
    """Exact check of sampled columns of adj(A)^T: Laplace expansion along
    column j, sum_i adjT[i][j] a_ij = det(A), as log2(|sum - det| / sum |terms|);
    the worst column."""
    import math
    P = A_host.limbs.shape[-1]
    N = A_host.exp.shape[0]
    md, ed = _mp_int(det_host.limbs, det_host.exp, det_host.sign, P)
    worst = float("-inf")
    for j in cols:
        terms = []
        for i in range(N):
            mc, ec = _mp_int(adjT_host.limbs[i, j], adjT_host.exp[i, j], adjT_host.sign[i, j], P)
            ma, ea = _mp_int(A_host.limbs[i, j], A_host.exp[i, j], A_host.sign[i, j], P)
            terms.append((mc * ma, ec + ea))
        emin = min([e for _, e in terms] + [ed])
        S = sum(v << (e - emin) for v, e in terms)
        absS = sum(abs(v) << (e - emin) for v, e in terms)
        diff = abs(S - (md << (ed - emin)))
        if diff:
            worst = max(worst, math.log2(diff) - math.log2(absS))
    return worst


def bench_backward(args, mats, work, Ds, cs, binfo, infos, P):
    """The determinant's backward, adj(A)^T = d det / d A (mp_det_adjugate), on
    every factored matrix (several matrices at once on separate streams and
    handles): wall time per pass over the workload, the VALU rate of its
    multiply-adds over that time (2N^3/3 of P-limb numbers per matrix: the
    row sweeps of L^-1, the back substitution and the accumulation, P^2
    32-bit MACs each), column N against the minors bit for bit, and Laplace's
    expansion along sampled columns evaluated exactly."""
    import torch

    from paper_1308_1536_amd import binding
    outs = [binding.DeviceMp.empty(w.rows, w.rows, P, w.limbs.device) for w in work]
    info_of = [binfo[b:b + 1] if binfo is not None else infos[b] for b in range(len(work))]
    # independent matrices run concurrently: S streams (default priority),
    # each with a handle (workspace) of its own; config 4 measured 8.17 s per
    # pass on 1 stream, 4.48 s on 4, 3.59 s on 8, 3.16 s on 16
    S = min(int(os.environ.get("MPDET_BWD_STREAMS", "16")), len(work))
    persistent = args.backward_schedule == "persistent" and binfo is not None
    if persistent:
        S = 1
    streams = [torch.cuda.Stream() for _ in range(S)]
    handles = [binding.Handle(work[0].limbs.device.index or 0) for _ in range(S)]
    status = torch.zeros(len(work), dtype=torch.int32, device=work[0].limbs.device)

    def run():
        torch.cuda.synchronize()
        if persistent:  # every matrix's backward in one persistent launch
            binding.adjugate_batched(work, Ds, binfo, outs, status)
        else:
            for b, (w, D, t, inf) in enumerate(zip(work, Ds, outs, info_of)):
                binding.adjugate(w, D, inf, t, stream=streams[b % S], h=handles[b % S])
        torch.cuda.synchronize()

    run()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ops = sum(2 * w.rows ** 3 // 3 for w in work)
    rate = ops * P * P / (ms / 1e3)
    mp = binding.measure_peak("mad64")
    last_same = all(torch.equal(t.limbs[:, -1], c.limbs[0]) and torch.equal(t.exp[:, -1], c.exp[0])
                    and torch.equal(t.sign[:, -1], c.sign[0]) for t, c in zip(outs, cs))
    checks = {}
    if not args.no_checks:
        order = sorted(range(len(mats)), key=lambda b: mats[b][1].exp.shape[0])
        for b in sorted(set([order[0], order[len(order) // 2], order[-1]])):
            nm, m = mats[b]
            n = m.exp.shape[0]
            cols = sorted(set([0, n // 2, n - 1]))
            Dh = Ds[b].row(0)
            from paper_1308_1536_amd.binding import HostMp
            det = HostMp(Dh.limbs[n - 1], Dh.exp[n - 1], Dh.sign[n - 1])
            checks[f"{b}:{nm}:N={n}"] = {"cols": cols,
                                         "max_rel_err_bits": adjugate_column_bits(m, outs[b].to_host(), det, cols)}
    lane = P <= 128 and P % 4 == 0
    if persistent and status.any():
        raise SystemExit(f"bench.py: batched backward status {status.cpu().tolist()}")
    kern = "k_persist_adj" if persistent else ("k_prod_lane_r1 + k_finish_r1" if lane else "k_adj_w")
    return {"ms_per_pass": ms, "multiply_adds": ops,
            "schedule": "persistent" if persistent else f"one call per matrix on {S} streams",
            "roofline": {"bound": "alu", "kernel": kern,
                         "achieved": rate / 1e12, "peak": PEAK_VALU_MAC32 / 1e12, "unit": "Tmac32/s",
                         "frac": rate / PEAK_VALU_MAC32, "measured_peak": mp / 1e12,
                         "frac_of_measured_peak": rate / mp, "streams": S},
            "last_column_equals_minors": bool(last_same), "laplace_checks": checks}


# configurations whose one matrix is timed as K segments of a single solve
SEGMENTED = {3}


def segment_bounds(N: int, K: int) -> list[int]:
    """Elimination-step boundaries 0 = b_0 < b_1 < ... < b_K = N that split one
    solve into K segments of about equal trailing-update work (sum of m^2 over
    the steps, m = N - k - 1 the trailing block's order at step k)."""
    K = max(1, min(K, N))
    w = [(N - k - 1) ** 2 for k in range(N)]
    total = max(1, sum(w))
    b, cum, s = [0], 0, 1
    for k in range(N):
        cum += w[k]
        if s < K and cum * K >= total * s:
            b.append(k + 1)
            s += 1
    b.append(N)
    # strictly increasing, K segments, each at least one step
    for t in range(1, K):
        b[t] = max(b[t], b[t - 1] + 1)
    for t in range(K - 1, 0, -1):
        b[t] = min(b[t], b[t + 1] - 1)
    assert len(b) == K + 1 and all(b[t] < b[t + 1] for t in range(K))
    return b


def compare_paths_on_block(Ah, L: int, paths=("mfma", "valu"), reps: int = 1):
    """Factor + minors of the leading L x L block on each update path: the time
    of one whole solve on each, and whether LU, every D_k and every minor have
    the same bits."""
    import torch

    from paper_1308_1536_amd import binding
    from paper_1308_1536_amd.inputs import MpArray
    blk = MpArray(Ah.limbs[:L, :L].copy(), Ah.exp[:L, :L].copy(), Ah.sign[:L, :L].copy())
    pristine = binding.DeviceMp.from_host(blk)
    out = {"size": L, "paths": {}}
    results = []
    for path in paths:
        w = binding.DeviceMp.empty(L, L, pristine.P)
        D = binding.DeviceMp.empty(1, L, pristine.P)
        c = binding.DeviceMp.empty(1, L, pristine.P)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        times = []
        for _ in range(reps + 1):  # the first run also allocates the path's workspace
            for t, f in zip((w.limbs, w.exp, w.sign), (pristine.limbs, pristine.exp, pristine.sign)):
                t.copy_(f)
            info.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            binding.factor(w, path, D=D, info=info)
            binding.minors(w, D, info, c=c)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        print(f"[bench] leading {L}x{L} block on the {path} path: {min(times[1:]):.3f} s", file=sys.stderr,
              flush=True)
        out["paths"][path] = {"seconds": min(times[1:]), "info": int(info.item())}
        results.append((w, D, c))
    same = all(torch.equal(a, b) for (w0, D0, c0) in results[:1] for (w1, D1, c1) in results[1:]
               for a, b in zip((w0.limbs, w0.exp, w0.sign, D0.limbs, D0.exp, D0.sign, c0.limbs, c0.exp, c0.sign),
                               (w1.limbs, w1.exp, w1.sign, D1.limbs, D1.exp, D1.sign, c1.limbs, c1.exp, c1.sign)))
    out["same_bits_LU_D_minors"] = bool(same)
    t = {p: out["paths"][p]["seconds"] for p in paths}
    if "mfma" in t and "valu" in t:
        out["valu_over_mfma_time"] = t["valu"] / t["mfma"]
    return out


def bench_segmented(args):
    """One whole solve of the workload's matrix, timed as K segments (see the
    module docstring)."""
    import numpy as np

    from paper_1308_1536_amd.inputs import MpArray, limb_macs_int8, u_count
    desc, mats = cached_workload(args.config, args.input_cache)
    name, Ah = mats[0]
    if args.size:
        Ah = MpArray(Ah.limbs[:args.size, :args.size].copy(), Ah.exp[:args.size, :args.size].copy(),
                     Ah.sign[:args.size, :args.size].copy())
        desc += f" -- leading {args.size}x{args.size} block"
    N, P = Ah.exp.shape[0], Ah.limbs.shape[-1]
    K = max(1, min(args.steps, N))
    W = max(0, min(args.warmup, K))
    b = segment_bounds(N, K)
    print(f"[bench] {desc}: {K} segments {b}", file=sys.stderr, flush=True)

    import torch

    from paper_1308_1536_amd import binding
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pristine = binding.DeviceMp.from_host(Ah)
    work = binding.DeviceMp.empty(N, N, P)
    D = binding.DeviceMp.empty(1, N, P)
    c = binding.DeviceMp.empty(1, N, P)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    path = args.path or DEFAULT_PATH[args.config]
    binding.set_overlap(args.overlap)

    def reset():
        for t, f in zip((work.limbs, work.exp, work.sign), (pristine.limbs, pristine.exp, pristine.sign)):
            t.copy_(f)
        info.zero_()

    def segment(s):
        binding.factor_steps(work, D, info, b[s], b[s + 1], path)
        if s == K - 1:
            binding.minors(work, D, info, c=c)

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # warm-up: the first W segments of a throwaway solve (allocates the workspace)
    reset()
    for s in range(W):
        segment(s)
        torch.cuda.synchronize()
        print(f"[bench] warm-up step {s + 1}/{W} done", file=sys.stderr, flush=True)

    # the timed solve; per-kernel HIP events on the launch stream throughout
    torch.cuda.synchronize()
    binding.profile_begin()
    seg_s = []
    t0 = time.perf_counter()
    for s in range(K):
        ts = time.perf_counter()
        if s == 0:
            reset()
        segment(s)
        torch.cuda.synchronize()
        seg_s.append(time.perf_counter() - ts)
        print(f"[bench] step {s + 1}/{K} (elimination steps {b[s]}..{b[s + 1] - 1}"
              f"{' + minors' if s == K - 1 else ''}) {seg_s[-1]:.2f} s", file=sys.stderr, flush=True)
    secs = time.perf_counter() - t0
    prof = binding.profile_end()
    if int(info.item()) != 0:
        raise SystemExit(f"bench.py: factorisation reported info {int(info.item())}")
    macs, upd = limb_macs_int8(N, P), u_count(N)
    value = macs / secs

    traffic_db = load_traffic(args.config)

    def traffic(kernel):
        t = traffic_db.get(kernel)
        if t is None:
            return None
        return {"bytes_per_launch": t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"],
                "fetch_bytes_per_launch": t["fetch_bytes_per_launch"],
                "write_bytes_per_launch": t["write_bytes_per_launch"]}

    roof, other = None, {}
    if prof["update_mfma"][1]:
        kms, kn = prof["update_mfma"]
        mp = binding.measure_peak("mfma_i8")
        ach = macs / (kms / 1e3)
        # above 256 limbs the update launch finishes its own products (no finish launch)
        fused = P > 256 and not prof["update_finish"][1]
        kern = f"k_update_mfma<{mfma_copies(P)}>" + (" with the finish" if fused else "")
        roof = {"bound": "mfma", "achieved": 2 * ach / 1e12, "peak": PEAK_INT8_MFMA_TOPS / 1e12, "unit": "TOP/s",
                "frac": ach / PEAK_INT8_MAC, "kernel": kern, "measured_peak": 2 * mp / 1e12,
                "frac_of_measured_peak": ach / mp, "measured_clock_ghz": binding.measure_peak("mfma_clock") / 1e9,
                "traffic": traffic(kern), "avg_launch_ms": kms / kn, "launches": kn}
        roof.update(issued("mfma", P, roof["frac"]))
    elif prof["update_valu"][1]:
        kms, kn = prof["update_valu"]
        ach = upd * P * P / (kms / 1e3)
        kern = "k_prod_lane" if (P <= 128 and P % 4 == 0) else "k_update_valu"
        roof = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_VALU_MAC32 / 1e12, "unit": "Tmac32/s",
                "frac": ach / PEAK_VALU_MAC32, "kernel": kern, "traffic": traffic(kern), "avg_launch_ms": kms / kn,
                "launches": kn}
    if prof["update_finish"][1]:
        kms, kn = prof["update_finish"]
        ach = upd * FINISH_BYTES(P) / (kms / 1e3)
        kern = "k_finish" + ("<true>" if P > 256 else "<false>")
        other["update_finish"] = {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                  "frac": ach / PEAK_HBM, "kernel": kern, "traffic": traffic(kern),
                                  "avg_launch_ms": kms / kn, "launches": kn}
    if roof is None:
        raise SystemExit("bench.py: no trailing-update launches were timed")
    roof["other_update_kernels"] = other
    roof["kernel_s_per_solve"] = {k: round(v[0] / 1e3, 3) for k, v in prof.items() if v[1]}

    out = {"metric": METRIC, "value": value, "unit": "limb-MAC/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": secs * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "i8" if prof["update_mfma"][1] else "u32", "data": "synthetic",
           "config": {"workload": desc, "N": N, "bits": 32 * P, "matrices": 1, "path": path,
                      "step": "one of K consecutive segments of one whole solve (elimination steps b_s..b_{s+1}-1; "
                              "the last also runs the minors): the K steps are one time to solution",
                      "segment_bounds": b, "segment_seconds": [round(v, 3) for v in seg_s],
                      "time_to_solution_s": secs, "updates": upd, "limb_macs": macs,
                      "overlap_panels": args.overlap},
           "end_to_end_frac_of_int8_peak": value / PEAK_INT8_MAC,
           "roofline": roof}
    Dh, ch = D.row(0), c.row(0)
    if not args.no_cpu_baseline:
        lead = min(N, 256)
        sub = MpArray(Ah.limbs[:lead, :lead].copy(), Ah.exp[:lead, :lead].copy(), Ah.sign[:lead, :lead].copy())
        out["cpu_baseline"] = cpu_baseline(sub, Dh, args.cpu_budget)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    if not args.no_checks:
        out["full_size_checks"] = {name: full_size_checks(args.config, name, Ah, work, Dh, ch, args.size)}
        print("[bench] full-size checks done", file=sys.stderr, flush=True)
    del work, pristine
    torch.cuda.empty_cache()
    if args.compare != "none" and args.compare_size > 0:
        other_path = "valu" if path == "mfma" else "mfma"
        out["comparison"] = compare_paths_on_block(Ah, min(N, args.compare_size), (path, other_path))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 10 segments of one solve for configuration 3, 3 passes otherwise)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 2 for 3, 1 otherwise)")
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--path", default=None, choices=["auto", "valu", "mfma", "tuned"],
                    help="trailing-update path (default: the configuration's own -- VALU for the plain "
                         "configurations 1 and 2, MFMA for 3, auto for the batched 4)")
    ap.add_argument("--compare", default="default", choices=["default", "none", "valu", "mfma"],
                    help="also time the other update path on the same workload and check that it gives the "
                         "same bits (default: MFMA beside the VALU path of configuration 2)")
    ap.add_argument("--compare-size", type=int, default=256, metavar="L",
                    help="configuration 3: time both update paths on the leading L x L block and compare their "
                         "bits (0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--input-cache", default=None, metavar="DIR",
                    help="load the workload's generated matrices from DIR (.npy files), generating and "
                         "saving them there first if absent")
    ap.add_argument("--size", type=int, default=0, metavar="N",
                    help="use the leading N x N block of every matrix (a scaling study, not the configuration's "
                         "workload; the JSON line says so)")
    ap.add_argument("--per-matrix", action="store_true",
                    help="factor the workload's matrices one after another instead of in one batched call")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed region, copy MIB MiB device-to-device once (a kernel of known "
                         "traffic for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the exact full-size checks (Cauchy pivots against their closed form, the "
                         "minors' invariant sum_i c_i a_iN = det)")
    ap.add_argument("--all-minors", action="store_true",
                    help="after the timed factorisations, also time mp_det_all_minors (the last-column minors "
                         "of every leading block) on each matrix and check its rows")
    ap.add_argument("--backward", action="store_true",
                    help="after the timed factorisations, also time the determinant's backward "
                         "(mp_det_adjugate, adj(A)^T) on each matrix and check it")
    ap.add_argument("--schedule", default="auto", choices=["auto", "persistent", "lockstep"],
                    help="schedule of a batched call (configs 2 and 4): one persistent launch over a task "
                         "queue, or one launch per phase per step (lockstep, the default)")
    ap.add_argument("--overlap", type=int, default=0, metavar="S",
                    help="MFMA path: S row panels per step, each panel's finish on a second stream beside the "
                         "next panel's update (0: off)")
    ap.add_argument("--backward-schedule", default="persistent", choices=["persistent", "streams"],
                    help="--backward on a batch: one persistent launch over every matrix "
                         "(mp_det_adjugate_batched) or one mp_det_adjugate call per matrix on 16 streams")
    ap.add_argument("--factor-steps", type=int, default=0, metavar="K",
                    help="time only K elimination steps of the first matrix, after --warmup untimed ones "
                         "(a partial run for matrices too large to repeat the path on; default for config 5: 24)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU (the method's single-GPU share); "
              "--gpus must be 1", file=sys.stderr, flush=True)
        sys.exit(2)
    if args.config == 5 and not args.factor_steps:
        args.factor_steps = 24
    seg = args.config in SEGMENTED and not args.factor_steps
    if args.steps is None:
        args.steps = 10 if seg else (24 if args.factor_steps else 3)
    if args.warmup is None:
        args.warmup = 2 if seg else (1 if not args.factor_steps else 0)
    if args.factor_steps:
        bench_elimination_steps(args)
        return
    if seg:
        bench_segmented(args)
        return

    # inputs first: the generator may fork worker processes, which must
    # happen before this process touches the GPU
    desc, mats = cached_workload(args.config, args.input_cache)
    if args.size:
        from paper_1308_1536_amd.inputs import MpArray
        mats = [(nm, MpArray(m.limbs[:args.size, :args.size].copy(), m.exp[:args.size, :args.size].copy(),
                             m.sign[:args.size, :args.size].copy())) for nm, m in mats]
        desc += f" -- leading {args.size}x{args.size} blocks"
    print(f"[bench] {desc}", file=sys.stderr, flush=True)

    import torch

    from paper_1308_1536_amd import binding
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    pristine = [binding.DeviceMp.from_host(m) for _, m in mats]
    work = [binding.DeviceMp.empty(p.rows, p.cols, p.P, dev) for p in pristine]
    Ds = [binding.DeviceMp.empty(1, p.rows, p.P, dev) for p in pristine]
    cs = [binding.DeviceMp.empty(1, p.rows, p.P, dev) for p in pristine]
    infos = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in pristine]
    path = args.path or DEFAULT_PATH[args.config]
    compare = args.compare
    if compare == "default":
        compare = "mfma" if (args.config == 2 and path == "valu") else "none"

    # several matrices go through one batched call (the same kernels, every
    # phase of a step launched once for all of them)
    batched = len(pristine) > 1 and not args.per_matrix
    if batched:
        binfo = torch.zeros(len(pristine), dtype=torch.int32, device=dev)

    def step(path=path):
        for p, w in zip(pristine, work):
            w.limbs.copy_(p.limbs)
            w.exp.copy_(p.exp)
            w.sign.copy_(p.sign)
        if batched:
            binding.batched(work, path, minors=True, Ds=Ds, cs=cs, info=binfo, schedule=args.schedule)
            return
        for w, D, c, info in zip(work, Ds, cs, infos):
            binding.factor(w, path, D=D, info=info)
            binding.minors(w, D, info, c=c)

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
        torch.cuda.synchronize()
        print(f"[bench] step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    bad = ([int(v) for v in binfo.cpu().tolist() if v] if batched else
           [int(i.item()) for i in infos if int(i.item()) != 0])
    if bad:
        raise SystemExit(f"bench.py: factorisation reported info {bad}")
    macs, upd = unit_work(mats)
    value = macs / (ms / 1e3)

    # live per-kernel timing with HIP events on the launch stream (one extra step)
    binding.profile_begin()
    step()
    prof = binding.profile_end()
    P = mats[0][1].limbs.shape[-1]

    peaks = {}
    traffic_db = load_traffic(args.config)

    def measured_traffic(kernel):
        """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE counter
        passes, if they were taken on the current kernel sources, else None"""
        t = traffic_db.get(kernel)
        if t is None:
            return None
        return {"bytes_per_launch": t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"],
                "fetch_bytes_per_launch": t["fetch_bytes_per_launch"],
                "write_bytes_per_launch": t["write_bytes_per_launch"]}

    def kname_of(single):
        """the kernel's symbol as launched: the batched variants carry k_batch_"""
        return "k_batch_" + single[2:] if batched else single

    def measured_peak(kind):
        """the unit's throughput measured on this GPU (probe kernel), multiply-adds/s"""
        if kind not in peaks:
            peaks[kind] = binding.measure_peak(kind)
        return peaks[kind]

    def roofline(kname):
        """Algorithmic work of every launch of `kname` in one step over its
        total event time: MFMA int8 MACs, VALU 32x32->64 MACs, or the finish's
        HBM bytes (read a_ij and the product record, write a_ij)."""
        kms, kn = prof[kname]
        secs = kms / 1e3
        if kname == "batch_persistent":
            # the whole batch in one launch: every phase of every step inside it
            achieved = upd * P * P / secs
            mp = measured_peak("mad64")
            r = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_MAC32 / 1e12,
                 "unit": "Tmac32/s", "frac": achieved / PEAK_VALU_MAC32, "kernel": "k_persist",
                 "measured_peak": mp / 1e12, "frac_of_measured_peak": achieved / mp,
                 "note": "one launch holds the products, the finish, the multipliers, the pivots and the "
                         "minors of every matrix"}
            if P <= 128 and P % 4 == 0:
                r.update(issued("alu", P, r["frac"]))
        elif kname == "update_valu":
            achieved = upd * P * P / secs
            mp = measured_peak("mad64")
            r = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_MAC32 / 1e12,
                 "unit": "Tmac32/s", "frac": achieved / PEAK_VALU_MAC32,
                 "kernel": kname_of("k_prod_lane" if (P <= 128 and P % 4 == 0) else "k_update_valu"),
                 "measured_peak": mp / 1e12, "frac_of_measured_peak": achieved / mp}
            if P <= 128 and P % 4 == 0:
                r.update(issued("alu", P, r["frac"]))
        elif kname == "update_mfma":
            achieved = macs / secs
            mp = measured_peak("mfma_i8")
            r = {"bound": "mfma", "achieved": 2 * achieved / 1e12, "peak": PEAK_INT8_MFMA_TOPS / 1e12,
                 "unit": "TOP/s", "frac": achieved / PEAK_INT8_MAC,
                 "kernel": kname_of("k_update_mfma") + f"<{mfma_copies(P)}>",
                 "measured_peak": 2 * mp / 1e12, "frac_of_measured_peak": achieved / mp}
            r.update(issued("mfma", P, r["frac"]))
        else:
            achieved = upd * FINISH_BYTES(P) / secs
            r = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                 "frac": achieved / PEAK_HBM, "kernel": kname_of("k_finish") + ("<true>" if P > 256 else "<false>")}
        r.update({"traffic": measured_traffic(r["kernel"]), "avg_launch_ms": kms / kn, "launches": kn})
        return r

    cands = [k for k in ("update_valu", "update_mfma", "update_finish", "batch_persistent") if prof[k][1] > 0]
    if not cands:
        raise SystemExit("bench.py: no trailing-update launches were timed")
    dom = max(cands, key=lambda k: prof[k][0])
    roof = roofline(dom)
    roof["other_update_kernels"] = {k: roofline(k) for k in cands if k != dom}
    roof["kernel_ms_per_step"] = {k: round(v[0], 3) for k, v in prof.items() if v[1]}

    out = {"metric": METRIC, "value": value, "unit": "limb-MAC/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "i8" if prof["update_mfma"][1] > 0 else "u32", "data": "synthetic",
           "config": {"workload": desc, "N": int(max(m.exp.shape[0] for _, m in mats)), "bits": 32 * P,
                      "matrices": len(mats), "path": path, "batched": batched,
                      "schedule": (("persistent" if prof["batch_persistent"][1] > 0 else "lockstep")
                                   if batched else None), "updates_per_step": upd,
                      "limb_macs_per_step": macs},
           "roofline": roof}
    if not args.no_cpu_baseline:
        first = max(range(len(mats)), key=lambda b: mats[b][1].exp.shape[0]) if batched else 0
        gpu_D = Ds[first].row(0)
        out["cpu_baseline"] = cpu_baseline(mats[first][1], gpu_D, args.cpu_budget)
    if not args.no_checks:
        # exact checks of the whole run's outputs (the work buffers hold the
        # last step's factorisation)
        checks = {}
        for b, (nm, m) in enumerate(mats):
            if args.config in CAUCHY_NODES or m.exp.shape[0] <= 600:
                r = full_size_checks(args.config, nm, m, work[b], Ds[b].row(0), cs[b].row(0), args.size)
                if r:
                    checks[nm] = r
        print("[bench] full-size checks done", file=sys.stderr, flush=True)
        out["full_size_checks"] = checks
    if args.all_minors:
        out["all_minors"] = bench_all_minors(args, mats, work, Ds, cs, binfo if batched else None, infos, P)
    if args.backward:
        out["backward"] = bench_backward(args, mats, work, Ds, cs, binfo if batched else None, infos, P)
    if compare != "none":
        # the other update path on the same inputs: its time, and whether every
        # D_k and minor it returns has the same bits
        saved = [tuple(t.clone() for t in (D.limbs, D.exp, D.sign, c.limbs, c.exp, c.sign)) for D, c in zip(Ds, cs)]
        step(compare)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            step(compare)
            torch.cuda.synchronize()
            print(f"[bench] {compare} step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
        cms = (time.perf_counter() - t0) * 1e3 / args.steps
        same = all(torch.equal(a, b) for sv, D, c in zip(saved, Ds, cs)
                   for a, b in zip(sv, (D.limbs, D.exp, D.sign, c.limbs, c.exp, c.sign)))
        out["comparison"] = {"path": compare, "ms_per_step": cms, "value": macs / (cms / 1e3),
                             "measured_over_compared_time": ms / cms, "same_bits_D_and_minors": bool(same)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
