"""Pins of oracle.quantize, the reference of every reduced-precision parity
test: BF16 and FP16 rounding to nearest with ties to even, checked against
hand-worked values (both tie directions, values just past a tie, the largest
finite values and overflow, subnormals) and against an independent
implementation (torch's CPU casts)."""
import numpy as np
import pytest

import oracle


def bits(x):
    return np.array(x, np.float32).view(np.uint32)


def from_bits(u):
    return np.array(u, np.uint32).view(np.float32)


def test_bf16_hand_worked():
    q = lambda v: oracle.quantize(np.array(v, np.float32), "bf16")  # noqa: E731
    # BF16 keeps 7 fraction bits: the spacing at 1 is 2^-7
    assert q([1.0]).tolist() == [1.0]
    assert q([1 + 2.0 ** -8]).tolist() == [1.0]                         # tie, down to the even 1.0
    assert q([1 + 3 * 2.0 ** -8]).tolist() == [1 + 2.0 ** -6]           # tie, up to the even neighbour
    assert q([1 + 2.0 ** -8 + 2.0 ** -20]).tolist() == [1 + 2.0 ** -7]  # just past the tie
    assert q([1 + 2.0 ** -8 - 2.0 ** -20]).tolist() == [1.0]            # just before it
    assert q([0.0, 0.5, 0.25]).tolist() == [0.0, 0.5, 0.25]
    # largest finite BF16 stays, the largest FP32 rounds up to infinity
    big = from_bits([0x7F7F0000, 0x7F7FFFFF, 0x7F7F7FFF, 0x7F7F8000])
    out = bits(q(big))
    assert out.tolist() == [0x7F7F0000, 0x7F800000, 0x7F7F0000, 0x7F800000]
    # subnormals: the same rule on the raw bits
    sub = from_bits([0x00010000, 0x00018000, 0x00028000, 0x00018001, 0x00007FFF, 0x00002000])
    assert bits(q(sub)).tolist() == [0x00010000, 0x00020000, 0x00020000, 0x00020000, 0, 0]


def test_f16_hand_worked():
    q = lambda v: oracle.quantize(np.array(v, np.float32), "f16")  # noqa: E731
    # FP16 keeps 10 fraction bits: the spacing at 1 is 2^-10
    assert q([1 + 2.0 ** -11]).tolist() == [1.0]
    assert q([1 + 3 * 2.0 ** -11]).tolist() == [1 + 2.0 ** -9]
    assert q([1 + 2.0 ** -11 + 2.0 ** -20]).tolist() == [1 + 2.0 ** -10]
    assert q([65504.0]).tolist() == [65504.0]                          # largest finite
    with np.errstate(over="ignore"):
        assert np.isinf(q([65520.0]))[0]                               # tie to the even 2^16 = overflow
    assert q([65519.0]).tolist() == [65504.0]
    assert q([2.0 ** -24]).tolist() == [2.0 ** -24]                    # smallest subnormal
    assert q([2.0 ** -25]).tolist() == [0.0]                           # tie to even 0
    assert q([3 * 2.0 ** -25]).tolist() == [2.0 ** -23]                # tie to even 2 * 2^-24
    assert q([2.0 ** -25 + 2.0 ** -40]).tolist() == [2.0 ** -24]


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_matches_torch_cast(storage):
    torch = pytest.importorskip("torch")
    rs = np.random.default_rng(5)
    # values of the images (non-negative, [0, 1] and beyond), every exponent,
    # and every bit pattern of the 16 bits a BF16 rounding drops
    a = np.concatenate([
        rs.uniform(0, 1, 100000).astype(np.float32),
        (rs.uniform(1, 2, 20000) * 2.0 ** rs.integers(-149, 128, 20000)).astype(np.float32),
        from_bits((0x3F800000 + np.arange(1 << 16)).astype(np.uint32)),
        from_bits(rs.integers(0, 0x7F800000, 50000).astype(np.uint32)),
    ])
    a = a[np.isfinite(a)]
    dt = torch.bfloat16 if storage == "bf16" else torch.float16
    ref = torch.from_numpy(a).to(dt).to(torch.float32).numpy()
    with np.errstate(over="ignore"):
        got = oracle.quantize(a, storage)
    np.testing.assert_array_equal(bits(got), bits(ref))


def test_f32_is_identity():
    a = np.random.default_rng(6).uniform(0, 1, 1000).astype(np.float32)
    np.testing.assert_array_equal(oracle.quantize(a, "f32"), a)
