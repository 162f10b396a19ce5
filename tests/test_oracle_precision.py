"""Pins of the oracle's reduced-precision Schur product.

The precision form rounds the eliminated rows ``F`` to fp32, or to bf16 by
way of fp32 (round to nearest, ties to even), multiplies with fp32
accumulation and subtracts the product from the fp64 block (Eq. elim with a
reduced-precision ``F^T F``).  These tests fix the rounding against IEEE
definitions worked out by hand and against torch's own bfloat16 conversion,
the product against exactly representable cases and the fp32 accumulation
error bound, and the factor built with it against the dense solve.
"""
import numpy as np
import pytest

from oracle import build_tree, factor, solve
from oracle.hsolver import round_bf16, schur_product
from synth import laplace2d, lognormal_field, rhs, slab_scalar, slab_vector


def _f32(bits):
    return np.array([bits], dtype=np.uint32).view(np.float32)[0]


def _bits(x):
    return int(np.asarray(x, dtype=np.float32).reshape(1).view(np.uint32)[0])


def test_round_bf16_ties_to_even():
    # bf16 keeps 7 fraction bits: next to 1 the spacing is 2^-7
    assert round_bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0  # tie, even neighbour 1
    assert round_bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6  # tie, even is up
    assert round_bf16(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7  # above the tie
    assert round_bf16(np.float32(1.0 + 2.0 ** -8 - 2.0 ** -20)) == 1.0  # below the tie
    assert round_bf16(np.float32(-(1.0 + 3 * 2.0 ** -8))) == -(1.0 + 2.0 ** -6)  # sign kept
    assert round_bf16(np.float32(-(1.0 + 2.0 ** -8))) == -1.0
    for v in (0.0, 1.5, -2.25, 2.0 ** -126, 3.0 * 2.0 ** 100):  # representable: unchanged
        assert round_bf16(np.float32(v)) == np.float32(v)
    assert _bits(round_bf16(np.float32(-0.0))) == 0x80000000


def test_round_bf16_extremes():
    bf16_max = _f32(0x7F7F0000)  # (2 - 2^-7) * 2^127
    assert _bits(round_bf16(_f32(0x7F7F7FFF))) == 0x7F7F0000  # just below the tie: down to max
    assert _bits(round_bf16(_f32(0x7F7F8000))) == 0x7F800000  # tie, odd max: up to infinity
    assert _bits(round_bf16(_f32(0x7F7FFFFF))) == 0x7F800000  # fp32 max overflows
    assert round_bf16(bf16_max) == bf16_max
    assert _bits(round_bf16(_f32(0xFF7F8000))) == 0xFF800000  # negative overflow
    assert _bits(round_bf16(_f32(0x7F800000))) == 0x7F800000  # infinity stays
    # subnormals: the same rule on the raw bits
    assert _bits(round_bf16(_f32(0x00008000))) == 0x00000000
    assert _bits(round_bf16(_f32(0x00018000))) == 0x00020000
    assert _bits(round_bf16(_f32(0x00010001))) == 0x00010000


def test_round_bf16_goes_through_fp32():
    # reading of the precision form: fp64 -> fp32 -> bf16, both to nearest
    # even.  1 + 2^-8 + 2^-30 rounds to 1 + 2^-8 in fp32 (2^-30 is below half
    # an fp32 ulp), which is then a bf16 tie that goes to 1; rounding the
    # double directly would give 1 + 2^-7
    assert round_bf16(np.array([1.0 + 2.0 ** -8 + 2.0 ** -30]))[0] == 1.0


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    # hand-picked ties and near-ties
    base = rng.integers(0, 0x7F000000, 2000, dtype=np.uint32) & np.uint32(0xFFFF0000)
    ties = np.concatenate([base | 0x8000, base | 0x7FFF, base | 0x8001]).astype(np.uint32).view(np.float32)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = round_bf16(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_schur_product_f32_exact_and_rounded():
    rng = np.random.default_rng(3)
    # small integers: every product and partial sum is exact in fp32
    Fp = rng.integers(-64, 65, size=(40, 7)).astype(np.float64)
    Fq = rng.integers(-64, 65, size=(40, 5)).astype(np.float64)
    for prec in ("f32", "bf16"):
        out = schur_product(Fp, Fq, prec)
        assert out.dtype == np.float64
        assert np.array_equal(out, Fp.T @ Fq)
    # 1 + 2^-30 is 1 in fp32: the product sums m ones exactly
    m = 33
    F = np.full((m, 2), 1.0 + 2.0 ** -30)
    assert np.array_equal(schur_product(F, F, "f32"), np.full((2, 2), float(m)))
    assert not np.array_equal(schur_product(F, F, "f64"), np.full((2, 2), float(m)))


def test_schur_product_bf16_rounds_inputs():
    # 1 + 3*2^-8 rounds to 1 + 2^-6 in bf16; m products of that square are
    # exact in fp32 for m = 9 (9 * (1 + 2^-5 + 2^-12) needs 17 bits)
    m = 9
    F = np.full((m, 3), 1.0 + 3 * 2.0 ** -8)
    want = m * (1.0 + 2.0 ** -6) ** 2
    assert np.array_equal(schur_product(F, F, "bf16"), np.full((3, 3), want))
    # f32 keeps 1 + 3*2^-8 exactly
    assert np.array_equal(schur_product(F, F, "f32"), np.full((3, 3), m * (1.0 + 3 * 2.0 ** -8) ** 2))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_schur_product_accumulation_bound(prec):
    # fp32 accumulation of exactly rounded inputs: |computed - exact| <=
    # gamma_m |a|^T |b| with gamma_m = m u / (1 - m u), u = 2^-24 (the
    # textbook bound for a recursive dot product; blocked sums obey it too)
    rng = np.random.default_rng(5)
    m = 300
    Fp = rng.standard_normal((m, 16))
    Fq = rng.standard_normal((m, 12))
    a = Fp.astype(np.float32).astype(np.float64) if prec == "f32" else round_bf16(Fp).astype(np.float64)
    b = Fq.astype(np.float32).astype(np.float64) if prec == "f32" else round_bf16(Fq).astype(np.float64)
    exact = a.T @ b  # the rounded inputs' exact product (fp64 is exact enough here)
    u = 2.0 ** -24
    gam = m * u / (1 - m * u)
    got = schur_product(Fp, Fq, prec)
    assert np.all(np.abs(got - exact) <= gam * (np.abs(a).T @ np.abs(b)) + 1e-300)
    if prec == "bf16":
        # the inputs were really rounded: their rounding (2^-9 relative)
        # moves the product by more than the accumulation bound somewhere
        assert np.max(np.abs(Fp.T @ Fq - exact) - gam * (np.abs(a).T @ np.abs(b))) > 0


CASES = [
    (lambda: laplace2d(16), 16),
    (lambda: slab_scalar(8, 8, 4, 1e3, lognormal_field((8, 8, 4), seed=3)), 16),
    (lambda: slab_vector(6, 6, 3, 1e2), 16),
]


@pytest.mark.parametrize("prec,bound", [("f32", 1e-4), ("bf16", 5e-2)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_reduced_precision_factor_without_truncation(case, prec, bound):
    # tol = 0 makes the factor an exact block Cholesky except for the
    # rounding of the Schur products: M^{-1} b stays close to A^{-1} b (within
    # cond(A) times the product's relative rounding) but is no longer exact
    # to fp64 rounding
    mk, leaf = CASES[case]
    pr = mk()
    T = build_tree(pr.grid, leaf)
    F = factor(pr.rowptr, pr.col, pr.val, T, 0.0, gemm_prec=prec)
    b = rhs(pr.n, 1)
    Ad = pr.scipy().toarray()
    xe = np.linalg.solve(Ad, b)
    x = solve(F, b)
    err = np.linalg.norm(x - xe) / np.linalg.norm(xe)
    u = 2.0 ** -24 if prec == "f32" else 2.0 ** -9
    assert err <= bound
    assert err <= 64 * u * np.linalg.cond(Ad)
    assert err > 1e-13  # the reduced product is really used
