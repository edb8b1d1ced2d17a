"""GPU parity: the HIP path through the C-ABI against the CPU oracle, bit for
bit (det, every D_k, the factors and the last-column minors), on seeded
inputs that span several wave blocks of limbs and ragged sizes, plus the
degenerate cases (zero pivots, exponent overflow, N = 1, empty)."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same, gpu_det, say
from paper_1308_1536_amd import inputs

pytestmark = pytest.mark.gpu

PATHS = ["valu", "mfma"]


def check_against_oracle(A, path, what, ld=None):
    from paper_1308_1536_amd import binding
    P = A.limbs.shape[-1]
    say(f"[parity] {what} path={path} N={A.exp.shape[0]} P={P}")
    if path == "mfma" and (P % 8 != 0 or P < 8):
        with pytest.raises(binding.MpdetError) as e:
            gpu_det(A, path, ld=ld)
        assert e.value.status == binding.MPDET_ENOTSUP
        return None, None, None, None
    LU, D, c, info = gpu_det(A, path, ld=ld)
    f, cw = oracle.det_pipeline(A)
    assert info == f.info, (what, info, f.info)
    assert_same(D, f.D, f"{what} D")
    assert_same(LU, f.LU, f"{what} LU")
    if cw is not None:  # complete factors: info 0, or info n (only u_nn = 0)
        assert_same(c, cw, f"{what} c")
    return LU, D, c, info


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N,P", [(1, 2), (2, 2), (3, 3), (5, 2), (17, 4), (40, 8), (65, 3),
                                 (33, 64), (12, 65), (9, 130)])
def test_random_mantissas(path, N, P):
    A = inputs.random_mantissas((N, N), P, 1000 + 7 * N + P)
    check_against_oracle(A, path, f"randmant N={N} P={P}")


@pytest.mark.parametrize("path", PATHS)
def test_wide_exponent_range(path):
    """Exponent gaps far beyond p exercise the sticky/clamp paths."""
    A = inputs.random_mantissas((24, 24), 8, 77, emin=-3000, emax=3000)
    check_against_oracle(A, path, "wide exponents")


@pytest.mark.parametrize("path", PATHS)
def test_cancellation_heavy(path):
    """Nearly equal rows: the updates cancel to a few bits and renormalise."""
    P = 8
    base = inputs.random_mantissas((1, 20), P, 5)
    A = inputs.random_mantissas((20, 20), P, 6)
    for i in range(20):
        A.limbs[i] = base.limbs[0]
        A.exp[i] = base.exp[0]
        A.sign[i] = base.sign[0]
        A.limbs[i, :, 0] ^= np.uint32(i + 1)  # differ in the last bits only
        A.limbs[i, i, 1] ^= np.uint32(1 << (i % 31))
    check_against_oracle(A, path, "cancellation")


@pytest.mark.parametrize("path", PATHS)
def test_config1(path):
    """Config 1 (N=64, 1024 bits): integer-node Cauchy and random integers."""
    cfg = inputs.config_c1()
    check_against_oracle(cfg["cauchy"][0], path, "C1 cauchy")
    check_against_oracle(cfg["randint"][0], path, "C1 randint")


@pytest.mark.parametrize("path", PATHS)
def test_cauchy_hilbert_exact(path):
    check_against_oracle(inputs.cauchy_dyadic(48, 8, 3)[0], path, "dyadic cauchy")
    check_against_oracle(inputs.hilbert(30, 8), path, "hilbert")
    check_against_oracle(inputs.triangular_product(40, 8, 9)[0], path, "exact L*U")


@pytest.mark.parametrize("path", PATHS)
def test_padded_leading_dimension(path):
    A = inputs.random_mantissas((19, 19), 16, 31)
    check_against_oracle(A, path, "ld=27", ld=27)


@pytest.mark.parametrize("path", PATHS)
def test_zero_pivots(path):
    P = 2
    # a_11 = 0
    P = 8 if path == "mfma" else 2
    A = inputs.from_values([[0, 1, 2], [3, 4, 5], [6, 7, 9]], P)
    _, D, _, info = check_against_oracle(A, path, "zero pivot 1")
    assert info == 1 and not D.limbs.any()
    # exactly singular leading 5x5 block inside a 12x12 matrix (L U with u_55 = 0)
    A, L, U = inputs.triangular_product(12, P, 4)
    U[4, 4] = 0
    A = inputs.from_values((L.astype(object) @ U.astype(object)), P)
    _, D, _, info = check_against_oracle(A, path, "zero pivot 5")
    assert info == 5


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [2, 9, 40])
def test_singular_last_pivot(path, N):
    """Only u_nn is zero: info = n, D_n = 0, and the last-column minors are
    still the oracle's (they never divide by u_nn)."""
    P = 8
    A, L, U = inputs.triangular_product(N, P, 40 + N)
    U[N - 1, N - 1] = 0
    A = inputs.from_values((L.astype(object) @ U.astype(object)), P)
    _, D, c, info = check_against_oracle(A, path, f"singular last pivot N={N}")
    assert info == N and not D.limbs[N - 1].any() and c.limbs.any()


@pytest.mark.parametrize("P", [264, 520])
def test_zero_pivot_and_overflow_large_p(P):
    """At P > 256 the MFMA path runs each pivot in a launch of its own (no
    look-ahead inside the finish): a zero pivot at step 5 and an exponent
    overflow at step 2 must stop the factorisation with the oracle's info, D
    and factors."""
    A, L, U = inputs.triangular_product(12, P, 4)
    U[4, 4] = 0
    A = inputs.from_values((L.astype(object) @ U.astype(object)), P)
    _, D, _, info = check_against_oracle(A, "mfma", f"zero pivot 5 P={P}")
    assert info == 5
    B = inputs.from_values([[1, 0, 0], [0, 1, 0], [0, 0, 1]], P)
    B.exp[0, 0] = 2 ** 61
    B.exp[1, 1] = 2 ** 61 + 5
    B.exp[2, 2] = 2 ** 61
    say(f"[parity] overflow P={P}")
    _, D, _, info = gpu_det(B, "mfma")
    f = oracle.factor(B)
    assert info == f.info == -1
    assert_same(D, f.D, "overflow D")


@pytest.mark.parametrize("path", PATHS)
def test_exponent_overflow(path):
    P = 8 if path == "mfma" else 2
    A = inputs.from_values([[1, 0, 0], [0, 1, 0], [0, 0, 1]], P)
    A.exp[0, 0] = 2 ** 61
    A.exp[1, 1] = 2 ** 61 + 5
    A.exp[2, 2] = 2 ** 61
    say("[parity] overflow")
    _, D, _, info = gpu_det(A, path)
    f = oracle.factor(A)
    assert info == f.info == -1
    assert_same(D, f.D, "overflow D")


def test_empty_matrix():
    import torch
    from paper_1308_1536_amd import binding
    A = binding.DeviceMp.empty(0, 0, 4)
    D, info = binding.factor(A, "valu")
    torch.cuda.synchronize()
    assert int(info.item()) == 0


def test_to_f64_matches_oracle():
    import torch
    from paper_1308_1536_amd import binding
    x = inputs.random_mantissas((7, 9), 6, 12, emin=-50, emax=50)
    x.limbs[0, 0] = 0
    x.exp[0, 0] = 0
    x.sign[0, 0] = 0
    xd = binding.DeviceMp.from_host(x)
    mant, e = binding.to_f64(xd)
    torch.cuda.synchronize()
    wm, we = oracle.to_f64(x)
    assert np.array_equal(mant.cpu().numpy(), wm)
    assert np.array_equal(e.cpu().numpy(), we)


def test_to_f64_scaled_matches_ldexp():
    """mp_to_f64_scaled against numpy's ldexp of the oracle's (mantissa,
    exponent): normal, subnormal (one rounding), underflow to zero and
    overflow to inf."""
    import torch
    from paper_1308_1536_amd import binding
    x = inputs.random_mantissas((6, 11), 5, 77, emin=-1200, emax=1200)
    x.limbs[1, 2] = 0
    x.exp[1, 2] = 0
    x.sign[1, 2] = 0
    x.exp[0, :] = [-1021, -1022, -1030, -1060, -1073, -1074, -1075, -1076, 1023, 1024, 1025]
    xd = binding.DeviceMp.from_host(x)
    wm, we = oracle.to_f64(x)
    for sh in (0, 5, -7, 3000, -3000):
        got = binding.to_f64_scaled(xd, torch.tensor([sh], dtype=torch.int64, device="cuda"))
        torch.cuda.synchronize()
        want = np.ldexp(wm, np.clip(we - sh, -2200, 2200))
        g = got.cpu().numpy()
        assert np.array_equal(g, want), (sh, np.argwhere(g != want)[:4])


@pytest.mark.parametrize("N,P", [(3, 8), (33, 8), (40, 16), (37, 24), (66, 32), (20, 40), (70, 64),
                                 (35, 128), (9, 256), (70, 264), (20, 520), (10, 1024)])
def test_mfma_shapes(N, P):
    """MFMA path: ragged column blocks (N-k-1 not a multiple of 32), partial
    product chunks (2*P8 not a multiple of 256) and several chunk counts."""
    A = inputs.random_mantissas((N, N), P, 4000 + 13 * N + P)
    check_against_oracle(A, "mfma", f"mfma shape N={N} P={P}")


@pytest.mark.parametrize("N,P", [(20, 264), (20, 520), (10, 1024)])
def test_valu_large_limbs(N, P):
    """VALU path (one wave per element update) at the MFMA path's large limb
    counts, on the same inputs as test_mfma_shapes: both paths must give the
    oracle's bits, so they agree with each other at 32768 bits too."""
    A = inputs.random_mantissas((N, N), P, 4000 + 13 * N + P)
    check_against_oracle(A, "valu", f"valu shape N={N} P={P}")


@pytest.mark.parametrize("setting", [0, 1])
@pytest.mark.parametrize("case", ["wide_exponents", "limb_shifts", "cancellation", "zero_entries", "zero_pivot",
                                  "patterns"])
def test_streaming_finish_cases(case, setting):
    """P > 256 takes the streaming finish (chunked a_ij, intermediate kept in
    the record buffer): the sticky, cancellation, 0 - t and zero-pivot cases,
    and operands a few limbs apart (so that the last chunks of a wave need the
    range checks the others skip), with the finish inside the update launch
    (setting 0) and in a launch of its own (setting 1)."""
    from paper_1308_1536_amd import binding
    P, N = 264, 22
    if case == "wide_exponents":
        A = inputs.random_mantissas((N, N), P, 91, emin=-30000, emax=30000)
    elif case == "limb_shifts":
        P, N = 520, 40
        A = inputs.random_mantissas((N, N), P, 97, emin=-200, emax=200)
    elif case == "cancellation":
        base = inputs.random_mantissas((1, N), P, 92)
        A = inputs.random_mantissas((N, N), P, 93)
        for i in range(N):
            A.limbs[i] = base.limbs[0]
            A.exp[i] = base.exp[0]
            A.sign[i] = base.sign[0]
            A.limbs[i, :, 0] ^= np.uint32(i + 1)
            A.limbs[i, i, 5 + i] ^= np.uint32(1 << (i % 31))
    elif case == "zero_entries":
        A = inputs.random_mantissas((N, N), P, 94)
        for i in range(N):
            for j in range(N):
                if i != j and (i * 7 + j * 3) % 5 == 0:
                    A.limbs[i, j] = 0
                    A.exp[i, j] = 0
                    A.sign[i, j] = 0
    elif case == "patterns":
        # powers of two and all-ones mantissas with equal exponents: sums and
        # differences whose top limbs are all ones or a single bit, where the
        # length of the intermediate cannot be read off its top limbs
        A = inputs.random_mantissas((N, N), P, 95, emin=0, emax=1)
        pats = [np.full(P, 0xFFFFFFFF, np.uint32), np.zeros(P, np.uint32), np.zeros(P, np.uint32)]
        pats[1][P - 1] = 0x80000000
        pats[2][P - 1] = 0x80000000
        pats[2][: P - 1] = 0xFFFFFFFF
        rng = np.random.default_rng(96)
        for i in range(N):
            for j in range(N):
                if (i * 5 + j) % 3:
                    A.limbs[i, j] = pats[int(rng.integers(0, 3))]
                    A.exp[i, j] = int(rng.integers(0, 2))
    else:
        A, L, U = inputs.triangular_product(12, P, 8)
        U[6, 6] = 0
        A = inputs.from_values((L.astype(object) @ U.astype(object)), P)
    binding.set_overlap(setting)
    try:
        check_against_oracle(A, "mfma", f"streaming finish {case} (overlap setting {setting})")
    finally:
        binding.set_overlap(0)


@pytest.mark.parametrize("path", ["valu", "mfma"])
def test_tile_finish_patterns(path):
    """The LDS-tile finish (P <= 256) on powers of two and all-ones mantissas
    with equal exponents: intermediates whose length the top limbs leave open."""
    P, N = 64, 30
    A = inputs.random_mantissas((N, N), P, 97, emin=0, emax=1)
    pats = [np.full(P, 0xFFFFFFFF, np.uint32), np.zeros(P, np.uint32), np.zeros(P, np.uint32)]
    pats[1][P - 1] = 0x80000000
    pats[2][P - 1] = 0x80000000
    pats[2][: P - 1] = 0xFFFFFFFF
    rng = np.random.default_rng(98)
    for i in range(N):
        for j in range(N):
            if (i * 7 + j) % 3:
                A.limbs[i, j] = pats[int(rng.integers(0, 3))]
                A.exp[i, j] = int(rng.integers(0, 2))
    check_against_oracle(A, path, "tile finish patterns")


@pytest.mark.parametrize("path,P", [("valu", 16), ("valu", 32), ("valu", 64), ("valu", 128),
                                    ("mfma", 72), ("mfma", 128), ("mfma", 264), ("mfma", 1024)])
def test_short_product_guard(path, P):
    """Both product kernels form only the columns the kept limbs need and redo
    the whole product when the guard bits below those limbs cannot rule out a
    carry (all ones) or, with the MFMA path's signed digits, a borrow (all
    zeros).  Step 0 with a_00 = 1 (so l_i = a_i0 exactly) multiplies
    all-ones mantissas by 2^(p-1) + 1 (bits below the kept limbs all ones; in
    balanced digits the skipped part is -1, a borrow) and by all-ones ones
    (a carry from the skipped columns)."""
    N = 24 if P <= 264 else 10
    say(f"[short product guard] {path} P={P}")
    A = inputs.random_mantissas((N, N), P, 300 + P)
    ones = np.full(P, 0xFFFFFFFF, np.uint32)
    top1 = np.zeros(P, np.uint32)
    top1[P - 1], top1[0] = 0x80000000, 1
    A.limbs[0, 0, :] = 0
    A.limbs[0, 0, P - 1] = 0x80000000
    A.exp[0, 0], A.sign[0, 0] = 1, 0
    for i in range(1, N):
        A.limbs[i, 0] = ones if i % 3 else top1
        A.limbs[0, i] = top1 if i % 2 else ones
    check_against_oracle(A, path, f"short product guard P={P}")


def test_mfma_digit_carry_extremes():
    """Bytes 0x7F/0x80/0xFF patterns drive every balanced-digit carry case."""
    P = 16
    N = 20
    A = inputs.random_mantissas((N, N), P, 55)
    pats = [0x7F7F7F7F, 0x80808080, 0xFFFFFFFF, 0x7F80FF7F, 0x00000000, 0x807F0080]
    for i in range(N):
        for j in range(N):
            if (i + j) % 3 == 0:
                A.limbs[i, j, :] = np.uint32(pats[(i * N + j) % len(pats)])
                A.limbs[i, j, -1] |= np.uint32(0x80000000)
    check_against_oracle(A, "mfma", "digit extremes")


def test_mfma_carry_into_zero_limbs():
    """Step 0 multiplies a_i0 (a_00 = 1, so l_i = a_i0 exactly; its low 12
    bytes are 0xFF, balanced digits -1, 0, ..., 0) by a_0j (low limbs
    1, 0, 0): the product's signed column sums are -1 then zeros, so a borrow
    has to run into a zero limb -- the case the update's one-level carry
    shortcut cannot take and hands to the limb-by-limb resolution."""
    P, N = 64, 24
    A = inputs.random_mantissas((N, N), P, 61)
    A.limbs[0, 0, :] = 0
    A.limbs[0, 0, P - 1] = np.uint32(0x80000000)
    A.exp[0, 0] = 1
    A.sign[0, 0] = 0
    for i in range(1, N):
        A.limbs[i, 0, :3] = np.uint32(0xFFFFFFFF)
    for j in range(1, N):
        A.limbs[0, j, 0] = np.uint32(1)
        A.limbs[0, j, 1:3] = 0
    check_against_oracle(A, "mfma", "borrow into zero limbs")


@pytest.mark.parametrize("P", [32, 64, 128, 264])
def test_mfma_sparse_bytes(P):
    """Mantissas made mostly of 0x00 and 0xFF bytes: long zero runs, negative
    column sums and all-ones limbs throughout the products."""
    N = 28
    rng = np.random.default_rng(62 + P)
    A = inputs.random_mantissas((N, N), P, 63 + P)
    choice = rng.choice(5, size=(N, N, 4 * P), p=[0.70, 0.15, 0.05, 0.05, 0.05])
    vals = np.array([0x00, 0xFF, 0x01, 0x80, 0x00], dtype=np.uint8)[choice]
    rnd = rng.integers(0, 256, size=(N, N, 4 * P), dtype=np.uint16).astype(np.uint8)
    vals = np.where(choice == 4, rnd, vals)
    A.limbs[...] = np.ascontiguousarray(vals).view(np.uint32).reshape(N, N, P)
    A.limbs[..., P - 1] |= np.uint32(0x80000000)
    check_against_oracle(A, "mfma", f"sparse bytes P={P}")


def test_mfma_equals_valu_config2_sized():
    """Both paths on the same config-2-sized numbers (4096-bit), N=100."""
    c = inputs.config_c2(N=100)
    for name in ("cauchy", "randmant"):
        A = c[name][0] if name == "cauchy" else c[name]
        check_against_oracle(A, "mfma", f"C2-sized {name}")
        a = gpu_det(A, "valu")
        b = gpu_det(A, "mfma")
        for x, y, w in ((a[0], b[0], "LU"), (a[1], b[1], "D"), (a[2], b[2], "c")):
            assert_same(x, y, f"valu vs mfma {name} {w}")
