"""Every launch configuration the autotuner may pick gives the same bits:
the lane product's tile (2, 4, 8 rows), the MFMA update's waves per workgroup
(1, 2, 4), on a single factorisation, on a batch, and on the rank-1 updates
of the backward; and the tuner's choice round-trips through its cache."""
import pytest

import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _restore():
    yield
    from paper_1308_1536_amd import binding
    binding.set_tuning(0, 0)


@pytest.mark.parametrize("P,n", [(64, 45), (16, 70), (128, 33)])
@pytest.mark.parametrize("rows", [2, 4, 8])
def test_lane_rows_same_bits(P, n, rows):
    from paper_1308_1536_amd import binding
    A = inputs.random_mantissas((n, n), P, 6100 + n)
    say(f"[tuning] lane rows={rows} P={P} n={n}")
    binding.set_tuning(lane_rows=rows)
    LU, D, c, info = gpu_det(A, "valu")
    f, cw = oracle.det_pipeline(A)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")


@pytest.mark.parametrize("P,n", [(16, 70), (264, 21), (1024, 40)])
@pytest.mark.parametrize("waves", [1, 2, 4])
def test_mfma_waves_same_bits(P, n, waves):
    from paper_1308_1536_amd import autotune, binding
    if not autotune.mfma_waves_ok(P, waves):
        pytest.skip("LDS of that many waves does not fit")
    A = inputs.random_mantissas((n, n), P, 6200 + n)
    say(f"[tuning] mfma waves={waves} P={P} n={n}")
    binding.set_tuning(mfma_waves=waves)
    LU, D, c, info = gpu_det(A, "mfma")
    f, cw = oracle.det_pipeline(A)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")


@pytest.mark.parametrize("cfg", [{"lane_rows": 2, "path": "valu"}, {"lane_rows": 8, "path": "valu"},
                                 {"mfma_waves": 1, "path": "mfma"}, {"mfma_waves": 4, "path": "mfma"}])
def test_batched_and_backward_under_tuning(cfg):
    import torch
    from paper_1308_1536_amd import autotune, binding
    P = 16
    sizes = [30, 5, 47, 1, 18]
    hosts = [inputs.random_mantissas((n, n), P, 6300 + n) for n in sizes]
    say(f"[tuning] batch {cfg}")
    autotune.apply(cfg)
    mats = [binding.DeviceMp.from_host(h) for h in hosts]
    Ds, cs, info = binding.batched(mats, cfg["path"])
    adj = [binding.adjugate(m, d, info[b:b + 1]) for b, (m, d) in enumerate(zip(mats, Ds))]
    torch.cuda.synchronize()
    assert not info.cpu().numpy().any()
    for b in (0, 2):
        f, c = oracle.det_pipeline(hosts[b])
        assert_same(Ds[b].row(0), f.D, f"D[{b}]")
        assert_same(cs[b].row(0), c, f"c[{b}]")
        assert_same(adj[b].to_host(), oracle.adjugate_t(f), f"adjT[{b}]")


def test_autotuner_choice_is_cached_and_exact(tmp_path, monkeypatch):
    from paper_1308_1536_amd import autotune, binding
    monkeypatch.setenv("MPDET_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = autotune.choose(40, 16, cap=48)
    assert cfg in autotune.candidates(16)
    assert autotune.choose(40, 16) == cfg  # from the cache
    A = inputs.random_mantissas((30, 30), 16, 9)
    want = gpu_det(A, "valu")
    autotune.apply(cfg)
    got = gpu_det(A, cfg["path"])
    for x, y in zip(got[:3], want[:3]):
        assert_same(x, y, "tuned vs default")
