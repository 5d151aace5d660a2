"""Pins of the e4m3 quantiser against the OCP E4M3 definition."""
import numpy as np

from oracle import quant


def test_named_values():
    # largest normal 448 = 0.1111.110, smallest subnormal 2^-9 = 0.0000.001,
    # smallest normal 2^-6 = 0.0001.000, 1.0 = 0.0111.000
    assert quant.e4m3_code([448.0]).tolist() == [0x7E]
    assert quant.e4m3_code([2.0 ** -9]).tolist() == [0x01]
    assert quant.e4m3_code([2.0 ** -6]).tolist() == [0x08]
    assert quant.e4m3_code([1.0]).tolist() == [0x38]
    assert quant.e4m3_code([-1.0]).tolist() == [0xB8]
    assert quant.e4m3_code([0.0]).tolist() == [0x00]


def test_every_code_round_trips():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = quant.e4m3_decode(codes)
    back = quant.e4m3_code(vals)
    # +0 and -0 are distinct codes; every other value maps back to itself
    assert np.array_equal(back, codes)
    # 126 positive finite values besides zero, strictly increasing
    pos = np.sort(vals[vals > 0])
    assert len(pos) == 126 and np.all(np.diff(pos) > 0)


def test_round_to_nearest_even_and_saturation():
    # 17 lies halfway between 16 (mantissa 0) and 18 (mantissa 1): even wins
    assert quant.e4m3_value([17.0]).tolist() == [16.0]
    assert quant.e4m3_value([19.0]).tolist() == [20.0]
    assert quant.e4m3_value([17.01]).tolist() == [18.0]
    # halfway between subnormals 2^-9 and 2*2^-9
    assert quant.e4m3_value([1.5 * 2.0 ** -9]).tolist() == [2 * 2.0 ** -9]
    assert quant.e4m3_value([500.0, -1e9]).tolist() == [448.0, -448.0]
    # relative error of normal values at most 2^-4
    x = np.random.default_rng(0).uniform(2.0 ** -6, 448, 10000)
    assert np.max(np.abs(quant.e4m3_value(x) - x) / x) <= 2.0 ** -4


def test_block_scaling():
    x = np.random.default_rng(1).standard_normal((128, 128)).astype(np.float32)
    s, c = quant.quantize_block(x)
    assert s == np.float32(np.max(np.abs(x)) / np.float32(448))
    assert quant.e4m3_decode(c).max() <= 448
    err = np.linalg.norm(quant.e4m3_decode(c) * s - x) / np.linalg.norm(x)
    assert err < 0.05
    s2, c1, c2 = quant.quantize_block(x, residual=True)
    err2 = np.linalg.norm((quant.e4m3_decode(c1) + quant.e4m3_decode(c2) / 16) * s2 - x) / np.linalg.norm(x)
    assert err2 < err / 8
    s0, c0 = quant.quantize_block(np.zeros((4, 4)))
    assert s0 == 1.0 and not c0.any()
