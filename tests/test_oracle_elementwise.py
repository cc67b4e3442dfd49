"""Pins of the oracle's element operators against library routines and
hand-worked values (none of these re-types the oracle's own formula)."""
import numpy as np
import pytest
import torch

from oracle import elementwise as ew


def _torch_bf16_bits(f32: np.ndarray) -> np.ndarray:
    t = torch.from_numpy(np.ascontiguousarray(f32, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def test_bf16_rne_matches_torch_random():
    rng = np.random.default_rng(1)
    bits = rng.integers(0, 2**32, size=200000, dtype=np.uint64).astype(np.uint32)
    f = bits.view(np.float32)
    f = f[~np.isnan(f)]
    np.testing.assert_array_equal(ew.f32_to_bf16_rne(f), _torch_bf16_bits(f))


def test_bf16_rne_hand_cases():
    # 1 + 2^-8 is exactly halfway between bf16 1.0 (0x3F80) and 1+2^-7 (0x3F81): tie -> even 0x3F80
    # 1 + 3*2^-8 is halfway between 0x3F81 and 0x3F82: tie -> even 0x3F82
    # 1 + 2^-8 + 2^-20 is above the tie: rounds up to 0x3F81
    cases = [(1.0 + 2**-8, 0x3F80), (1.0 + 3 * 2**-8, 0x3F82), (1.0 + 2**-8 + 2**-20, 0x3F81),
             (-1.0 - 2**-8, 0xBF80), (0.0, 0x0000), (-0.0, 0x8000),
             (float(np.finfo(np.float32).max), 0x7F80)]   # rounds past bf16 max -> +inf
    for v, want in cases:
        got = int(ew.f32_to_bf16_rne(np.array([v], dtype=np.float32))[0])
        assert got == want, (v, hex(got), hex(want))
    # subnormal fp32 values round like any other: compare with torch
    sub = np.array([1e-40, -3e-39, 9.2e-41], dtype=np.float32)
    np.testing.assert_array_equal(ew.f32_to_bf16_rne(sub), _torch_bf16_bits(sub))


def test_bf16_widening_is_exact():
    u = np.arange(0, 2**16, dtype=np.uint32).astype(np.uint16)
    f = ew.bf16_to_f32(u)
    t = torch.from_numpy(u.view(np.int16).copy()).view(torch.bfloat16).to(torch.float32).numpy()
    ok = ~np.isnan(t)
    np.testing.assert_array_equal(f[ok].view(np.uint32), t[ok].view(np.uint32))


def test_bf16_sum_is_fp32_add_then_rne():
    rng = np.random.default_rng(2)
    a = _torch_bf16_bits(rng.uniform(-4, 4, 5000).astype(np.float32))
    b = _torch_bf16_bits(rng.uniform(-4, 4, 5000).astype(np.float32))
    ta = torch.from_numpy(a.view(np.int16).copy()).view(torch.bfloat16).float()
    tb = torch.from_numpy(b.view(np.int16).copy()).view(torch.bfloat16).float()
    want = (ta + tb).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ew.combine("sum", "bfloat16", a, b), want)


def test_fp32_sum_matches_torch():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(10000).astype(np.float32) * np.float32(1e3)
    b = rng.standard_normal(10000).astype(np.float32)
    want = (torch.from_numpy(a) + torch.from_numpy(b)).numpy()
    np.testing.assert_array_equal(ew.combine("sum", "float32", a, b).view(np.uint32), want.view(np.uint32))


def test_int32_sum_wraps():
    a = np.array([2**31 - 1, -2**31, 5, -7], dtype=np.int32)
    b = np.array([1, -1, 2**31 - 1, 3], dtype=np.int32)
    got = ew.combine("sum", "int32", a, b)
    assert got.tolist() == [-2**31, 2**31 - 1, -2**31 + 4, -4]


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_max_prefers_positive_zero_and_is_commutative(dtype):
    if dtype == "float32":
        pz, nz = np.array([0.0], np.float32), np.array([-0.0], np.float32)
        view = np.uint32
    else:
        pz, nz = np.array([0x0000], np.uint16), np.array([0x8000], np.uint16)
        view = np.uint16
    for x, y in ((pz, nz), (nz, pz)):
        r = ew.combine("max", dtype, x, y)
        assert r.view(view)[0] == pz.view(view)[0]
    r = ew.combine("max", dtype, nz, nz)
    assert r.view(view)[0] == nz.view(view)[0]


def test_max_matches_numpy_on_nonzero_values():
    rng = np.random.default_rng(4)
    a = rng.standard_normal(1000).astype(np.float32)
    b = rng.standard_normal(1000).astype(np.float32)
    np.testing.assert_array_equal(ew.combine("max", "float32", a, b), np.maximum(a, b))
    ai = rng.integers(-2**31, 2**31, 1000, dtype=np.int64).astype(np.int32)
    bi = rng.integers(-2**31, 2**31, 1000, dtype=np.int64).astype(np.int32)
    np.testing.assert_array_equal(ew.combine("max", "int32", ai, bi), np.maximum(ai, bi))
