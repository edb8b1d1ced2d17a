"""The p-versus-2p accuracy report (Sec. 4.3 method) on the GPU: normalised
minors of every leading block at p and 2p bits from the same exact input;
the agreement falls with N (Hilbert: steeply, as its conditioning grows),
and the line fit gives a positive loss per row operation."""
import pytest

from gpu_util import say
from paper_1308_1536_amd import accuracy, inputs

pytestmark = pytest.mark.gpu


def test_hilbert_loses_bits_linearly():
    say("[accuracy] hilbert n=40 at 512 / 1024 bits")
    r = accuracy.report(inputs.hilbert, 40, 16, rows=range(3, 40, 4))
    mins = r["min_agree_bits"]
    assert mins[0] > mins[-1] + 50           # the agreement falls with N
    assert 1.0 < r["fit"]["bits_lost_per_row_operation"] < 10.0
    assert all(a >= b - 8 for a, b in zip(mins, mins[1:]))  # roughly monotone


def test_cauchy_config2_generator_keeps_most_bits():
    say("[accuracy] cauchy n=48 at 1024 / 2048 bits")
    mk = lambda n, P: inputs.cauchy_dyadic(n, P, 77)[0]  # noqa: E731
    r = accuracy.report(mk, 48, 32, rows=range(5, 48, 6))
    assert min(r["min_agree_bits"]) > 1024 - 200
    assert r["mean_agree_bits"][0] >= r["min_agree_bits"][0]
