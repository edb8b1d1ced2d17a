"""The step-serial kernels (pivot reciprocal and D_k, the multipliers, the
minors sweeps) as teams of waves: above about 224 limbs the waves of one
workgroup share the digit-column windows of each product.  Which wave forms
a window cannot change a bit, so every team size gives the oracle's bits;
the teams' bounded waits turn into info = -2 when they run out (a wait
limit of zero makes every wait that is not already satisfied run out)."""
import pytest

import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu


def team_waves(P):
    """Waves per workgroup of the step-serial kernels (the library's rule,
    restated for the test labels): one per round of 64 windows of 8 radix-2^28
    digit columns of a P x P product, at most 4."""
    cols = (64 * P + 27) // 28
    rounds = ((cols + 7) // 8 + 63) // 64
    return max(1, min(4, rounds))


@pytest.mark.parametrize("P", [224, 232, 520, 1024])
@pytest.mark.parametrize("path", ["mfma", "valu"])
def test_team_sizes_against_oracle(P, path):
    """One wave (224 limbs), two (232), three (520) and four (1024), on both
    update paths, with several rows per step and the minors."""
    N = 12 if path == "valu" else 20
    A = inputs.random_mantissas((N, N), P, 7100 + P)
    say(f"[teams] path={path} P={P} N={N} waves={team_waves(P)}")
    LU, D, c, info = gpu_det(A, path)
    f, cw = oracle.det_pipeline(A)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")


def test_team_extend_against_oracle():
    """Growing a factorisation (the new rows' multipliers) with teams of two."""
    from test_gpu_extend import _grown
    A = inputs.random_mantissas((21, 21), 264, 7300)
    say("[teams] extend P=264 n=21 cuts=[9]")
    LU, D, c, info = _grown(A, [9], "mfma")
    f, cw = oracle.det_pipeline(A)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")


def test_team_waits_run_out_into_info():
    """Wait limit zero: the factorisation (teams of four) stops with
    info = -2, and so do the minors of a good factorisation; with the limit
    restored both give the oracle's bits again."""
    import torch

    from paper_1308_1536_amd import binding
    P, N = 1024, 10
    A_host = inputs.random_mantissas((N, N), P, 7400)
    f, cw = oracle.det_pipeline(A_host)
    say("[teams] factor with wait limit 0")
    binding.set_wait_limit(0.0)
    try:
        A = binding.DeviceMp.from_host(A_host)
        D, info = binding.factor(A, "mfma")
        torch.cuda.synchronize()
        assert int(info.item()) == -2
    finally:
        binding.set_wait_limit(10.0)
    say("[teams] minors with wait limit 0")
    A = binding.DeviceMp.from_host(A_host)
    D, info = binding.factor(A, "mfma")
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    binding.set_wait_limit(0.0)
    try:
        binding.minors(A, D, info)
        torch.cuda.synchronize()
        assert int(info.item()) == -2
    finally:
        binding.set_wait_limit(10.0)
    say("[teams] limit restored")
    LU, D2, c, info2 = gpu_det(A_host, "mfma")
    assert info2 == 0
    assert_same(D2, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")


@pytest.mark.parametrize("P", [8, 64, 264, 1024])
def test_long_division_fallback_against_oracle(P):
    """Every multiplier by long division (the shared reciprocal's fallback),
    on the general layout (8 limbs) and the divide's lean one (64, 264 with a
    team of two, 1024 with four): the oracle's bits, and the same bits as the
    reciprocal path."""
    from paper_1308_1536_amd import binding
    N = 14
    A = inputs.random_mantissas((N, N), P, 7500 + P)
    say(f"[long division] P={P} N={N}")
    binding.set_long_division(True)
    try:
        LU, D, c, info = gpu_det(A, "mfma" if P % 8 == 0 and P > 64 else "valu")
    finally:
        binding.set_long_division(False)
    f, cw = oracle.det_pipeline(A)
    assert info == f.info == 0
    assert_same(D, f.D, "D")
    assert_same(LU, f.LU, "LU")
    assert_same(c, cw, "c")
