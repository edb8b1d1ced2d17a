"""Batched launches (many matrices of uneven n in lockstep): bit-identical to
single-matrix calls and to the oracle; a matrix with a zero pivot reports its
own info without disturbing the others."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def run_batch(hosts, path):
    import torch
    from paper_1308_1536_amd import binding
    mats = [binding.DeviceMp.from_host(h) for h in hosts]
    Ds, cs, info = binding.batched(mats, path)
    torch.cuda.synchronize()
    return ([m.to_host() for m in mats], [d.row(0) for d in Ds], [c.row(0) for c in cs],
            info.cpu().numpy())


@pytest.mark.parametrize("path,P", [("valu", 3), ("mfma", 8), ("auto", 16)])
def test_batch_matches_single_and_oracle(path, P):
    rng = np.random.default_rng(P)
    sizes = [1, 2, 5, 17, 40, 33, 9, 64, 3]
    hosts = []
    for b, n in enumerate(sizes):
        if b % 2:
            hosts.append(inputs.cauchy_dyadic(n, P, 90 + b)[0])
        else:
            hosts.append(inputs.random_mantissas((n, n), P, 70 + b))
    say(f"[batch] path={path} P={P} sizes={sizes}")
    LUs, Ds, cs, info = run_batch(hosts, path)
    assert not info.any()
    for b, h in enumerate(hosts):
        f, c = oracle.det_pipeline(h)
        assert_same(Ds[b], f.D, f"batch D[{b}]")
        assert_same(LUs[b], f.LU, f"batch LU[{b}]")
        assert_same(cs[b], c, f"batch c[{b}]")
    if path != "valu":
        LU1, D1, c1, i1 = gpu_det(hosts[7], path)
        assert_same(Ds[7], D1, "batch vs single D")
        assert_same(cs[7], c1, "batch vs single c")


def test_batch_poisoned_matrix_is_isolated():
    P = 8
    good = [inputs.random_mantissas((n, n), P, 300 + n) for n in (12, 30, 7)]
    bad = inputs.random_mantissas((20, 20), P, 301)
    bad.limbs[0, 0] = 0
    bad.exp[0, 0] = 0
    bad.sign[0, 0] = 0  # zero first pivot
    hosts = [good[0], bad, good[1], good[2]]
    say("[batch] poisoned")
    LUs, Ds, cs, info = run_batch(hosts, "auto")
    assert list(info) == [0, 1, 0, 0]
    assert not Ds[1].limbs.any() and not cs[1].limbs.any()
    for b in (0, 2, 3):
        f, c = oracle.det_pipeline(hosts[b])
        assert_same(Ds[b], f.D, f"good D[{b}]")
        assert_same(cs[b], c, f"good c[{b}]")


def test_batch_config4_sample():
    """A slice of config 4 (2048-bit, uneven n, half Cauchy half random)."""
    batch = inputs.config_c4(count=8)
    hosts = [m for _, m in batch if m.exp.shape[0] <= 200][:4]
    say(f"[batch] config-4 sample sizes {[h.exp.shape[0] for h in hosts]}")
    LUs, Ds, cs, info = run_batch(hosts, "auto")
    assert not info.any()
    for b, h in enumerate(hosts[:2]):
        f, c = oracle.det_pipeline(h)
        assert_same(Ds[b], f.D, f"c4 D[{b}]")
        assert_same(cs[b], c, f"c4 c[{b}]")


def test_autotuner_choice_does_not_change_bits(tmp_path, monkeypatch):
    """The tuner only picks among bit-identical paths; its cache round-trips."""
    from paper_1308_1536_amd import autotune
    monkeypatch.setenv("MPDET_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    P = 16
    try:
        path = autotune.choose_path(40, P, cap=48)
        assert path in ("valu", "mfma")
        assert autotune.choose_path(40, P) == path  # cached
        A = inputs.random_mantissas((30, 30), P, 9)
        b = gpu_det(A, path)
    finally:
        autotune.apply({})
    a = gpu_det(A, "valu")
    for x, y in zip(a[:3], b[:3]):
        assert_same(x, y, "tuned path vs valu")


def _mixed_batch(sizes, P, seed):
    hosts = []
    for b, n in enumerate(sizes):
        if b % 2:
            hosts.append(inputs.cauchy_dyadic(n, P, seed + b)[0])
        else:
            hosts.append(inputs.random_mantissas((n, n), P, seed + b))
    return hosts


def _run_schedule(hosts, schedule, path="valu"):
    import torch
    from paper_1308_1536_amd import binding
    mats = [binding.DeviceMp.from_host(h) for h in hosts]
    Ds, cs, info = binding.batched(mats, path, schedule=schedule)
    torch.cuda.synchronize()
    return ([m.to_host() for m in mats], [d.row(0) for d in Ds], [c.row(0) for c in cs], info.cpu().numpy())


@pytest.mark.parametrize("P", [64, 16, 6])
def test_persistent_launch_matches_lockstep_and_oracle(P):
    """One persistent launch over the task queue against one launch per phase
    per step: the same bits for every matrix (lane product at 64 and 16
    limbs, the one-wave update at 6), and the oracle on three of them."""
    sizes = [48, 17, 1, 2, 33, 90, 64, 5, 3, 71]
    hosts = _mixed_batch(sizes, P, 4100 + P)
    say(f"[persistent] P={P} sizes={sizes}")
    a = _run_schedule(hosts, "persistent")
    b = _run_schedule(hosts, "lockstep")
    assert not a[3].any() and not b[3].any()
    for i in range(len(sizes)):
        assert_same(a[0][i], b[0][i], f"LU[{i}]")
        assert_same(a[1][i], b[1][i], f"D[{i}]")
        assert_same(a[2][i], b[2][i], f"c[{i}]")
    for i in (0, 2, 4):
        f, c = oracle.det_pipeline(hosts[i])
        assert_same(a[1][i], f.D, f"oracle D[{i}]")
        assert_same(a[2][i], c, f"oracle c[{i}]")


def test_persistent_launch_expired_wait_drains():
    """A wait limit of zero makes the first wait that is not already satisfied
    expire: the launch skips every later ticket, ends normally, and the
    matrices it did not finish report info = -2; with the limit restored the
    same batch gives the lockstep bits."""
    from paper_1308_1536_amd import binding
    hosts = _mixed_batch([120, 80, 40, 9], 16, 4300)
    say("[persistent] wait limit 0")
    binding.set_wait_limit(0.0)
    try:
        a = _run_schedule(hosts, "persistent")
    finally:
        binding.set_wait_limit(10.0)
    assert set(a[3].tolist()) <= {0, -2}
    assert (a[3] == -2).any()
    say("[persistent] wait limit restored")
    b = _run_schedule(hosts, "persistent")
    c = _run_schedule(hosts, "lockstep")
    assert not b[3].any()
    for i in range(len(hosts)):
        assert_same(b[1][i], c[1][i], f"D[{i}]")
        assert_same(b[2][i], c[2][i], f"c[{i}]")
        assert_same(b[0][i], c[0][i], f"LU[{i}]")
    # the matrices that finished before the abort hold correct results
    for i in np.flatnonzero(a[3] == 0):
        assert_same(a[1][i], c[1][i], f"finished D[{i}]")


def test_persistent_refuses_mfma():
    import torch
    from paper_1308_1536_amd import binding
    mats = [binding.DeviceMp.from_host(inputs.random_mantissas((8, 8), 8, 1))]
    with pytest.raises(binding.MpdetError) as e:
        binding.batched(mats, "mfma", schedule="persistent")
    assert e.value.status == binding.MPDET_ENOTSUP
    torch.cuda.synchronize()
