"""Pins for the oracle's Sec. 2.A arithmetic: eta(T) and the storage codes of eta - 1.

The codes are checked against independent implementations: NumPy's float32 -> float16
conversion, and round-to-nearest-even on float32 bit patterns for bfloat16.
"""

import numpy as np
import pytest

import oracle

RHO0G, T0 = 2.7e-4, 293.0


def _values(rng, n=20000):
    v = np.concatenate([
        rng.uniform(-3e4, 3e4, n),
        rng.uniform(-1.0, 1.0, n),
        rng.standard_normal(n) * 1e-5,       # fp16 subnormal range
        np.ldexp(rng.integers(1, 2**13, n), -24).astype(np.float64),  # exact small ints * 2^-24
        np.array([0.0, -0.0, 65504.0, 2.0**-14, 2.0**-24, 1.0 + 2.0**-11, 1.0 + 3 * 2.0**-11]),
    ])
    return v.astype(np.float32)


def test_f16_codes_match_numpy_conversion():
    x = _values(np.random.default_rng(0))
    codes = oracle.encode(x, oracle.CODE_F16, 1.0, 0.0)
    ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(codes, ref)


def _bf16_rne_bits(x32: np.ndarray) -> np.ndarray:
    b = x32.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((b >> 16) & 1)
    return ((b + bias) >> 16).astype(np.uint16)


def test_bf16_codes_match_bit_rounding():
    x = _values(np.random.default_rng(1))
    codes = oracle.encode(x, oracle.CODE_BF16, 1.0, 0.0)
    assert np.array_equal(codes, _bf16_rne_bits(x))


def test_ties_round_to_even():
    # 1 + 2^-11 lies halfway between two fp16 neighbours: ties go to the even mantissa
    x = np.array([1.0 + 2.0**-11, 1.0 + 3 * 2.0**-11], np.float32)
    q = oracle.decode(oracle.encode(x, oracle.CODE_F16), oracle.CODE_F16)
    assert q[0] == 1.0 and q[1] == 1.0 + 2 * 2.0**-10


@pytest.mark.parametrize("code", [oracle.CODE_F16, oracle.CODE_BF16])
def test_scaled_offset_codes_and_decode(code):
    rng = np.random.default_rng(2)
    delta = (RHO0G * T0 / rng.uniform(293.0, 303.0, 5000)).astype(np.float32)
    c, s = 2.7e-4, 2.0**30
    codes = oracle.encode(delta, code, s, c)
    # the code is the one rounding of the binary32 value (delta - c) * s
    t = (delta - np.float32(c)) * np.float32(s)
    if code == oracle.CODE_F16:
        assert np.array_equal(codes, t.astype(np.float16).view(np.uint16))
        back = t.astype(np.float16).astype(np.float64)
    else:
        assert np.array_equal(codes, _bf16_rne_bits(t))
        back = (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    dec = oracle.decode(codes, code, s, c)
    assert np.array_equal(dec, np.float64(np.float32(c)) + back / s)
    # decoded value within half a code quantum of the binary32 input
    ulp_bits = 10 if code == oracle.CODE_F16 else 7
    quantum = np.ldexp(1.0, np.frexp(np.abs(t.astype(np.float64)))[1] - 1 - ulp_bits) / s
    assert np.all(np.abs(dec - (np.float64(np.float32(c)) + t.astype(np.float64) / s)) <= 0.5 * quantum + 1e-30)


def test_f32_codes_identity():
    rng = np.random.default_rng(3)
    x = rng.uniform(2.6e-4, 2.8e-4, 1000).astype(np.float32)
    assert np.array_equal(oracle.encode(x, oracle.CODE_F32, 1.0, 0.0), x)
    assert np.array_equal(oracle.decode(x, oracle.CODE_F32, 1.0, 0.0), x.astype(np.float64))


def test_eta_of_temperature_fixed_points():
    # eta(T0) = 1 + rho0 G (ideal gas at ambient temperature); delta * T constant
    T = np.array([T0, 2 * T0, 0.5 * T0, 300.0], np.float32)
    d = oracle.delta_from_temperature(T, RHO0G, T0)
    assert d[0] == pytest.approx(RHO0G, rel=1e-15)
    assert d[1] == pytest.approx(RHO0G / 2, rel=1e-15)
    assert d[2] == pytest.approx(2 * RHO0G, rel=1e-15)
    assert np.allclose(d * T.astype(np.float64), RHO0G * T0, rtol=1e-15)
    # hotter air is less dense: lower refractive index
    Ts = np.linspace(280.0, 320.0, 50).astype(np.float32)
    assert np.all(np.diff(oracle.delta_from_temperature(Ts)) < 0)


def test_eta_binary32_path():
    rng = np.random.default_rng(4)
    T = rng.uniform(290.0, 310.0, 10000).astype(np.float32)
    d32 = oracle.delta_from_temperature_f32(T, RHO0G, T0)
    ref = np.float32(RHO0G) * (np.float32(T0) / T)  # NumPy binary32, two roundings
    assert d32.dtype == np.float32 and np.array_equal(d32, ref)
    d64 = oracle.delta_from_temperature(T, RHO0G, T0)
    # two binary32 roundings plus the rounding of the constant: within 3 ulp
    assert np.all(np.abs(d32.astype(np.float64) - d64) <= 3 * np.spacing(d32).astype(np.float64))
