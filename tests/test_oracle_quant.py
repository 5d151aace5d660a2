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


def test_block_scale_is_the_smallest_sufficient_power_of_two():
    # worked cases: 448 fits 448 * 2^0; the next float32 above it needs 2^1;
    # 224 = 448 / 2 fits 2^-1; 1 needs 2^-8 (448 * 2^-9 = 0.875 < 1)
    assert quant.block_scale(np.float32(448.0)) == 1.0
    assert quant.block_scale(np.nextafter(np.float32(448.0), np.float32(1e9))) == 2.0
    assert quant.block_scale(np.float32(224.0)) == 0.5
    assert quant.block_scale(np.float32(1.0)) == 2.0 ** -8
    assert quant.block_scale(np.float32(0.0)) == 1.0
    assert quant.block_scale(np.float32(1e-40)) == np.float32(2.0 ** -122)   # the floor
    rng = np.random.default_rng(2)
    for amax in np.exp(rng.uniform(-60, 60, 2000)).astype(np.float32):
        s = float(quant.block_scale(amax))
        m, _ = np.frexp(s)
        assert m == 0.5                                  # a power of two
        assert amax <= 448 * s and amax > 448 * s / 2    # and the smallest one


def test_block_scaling():
    x = np.random.default_rng(1).standard_normal((128, 128)).astype(np.float32)
    s, c = quant.quantize_block(x)
    assert s == quant.block_scale(np.max(np.abs(x)))
    assert quant.e4m3_decode(c).max() <= 448
    err = np.linalg.norm(quant.e4m3_decode(c) * s - x) / np.linalg.norm(x)
    assert err < 0.05
    s2, c1, c2 = quant.quantize_block(x, residual=True)
    err2 = np.linalg.norm((quant.e4m3_decode(c1) + quant.e4m3_decode(c2) / 16) * s2 - x) / np.linalg.norm(x)
    assert err2 < err / 8
    s0, c0 = quant.quantize_block(np.zeros((4, 4)))
    assert s0 == 1.0 and not c0.any()


def test_coded_block_fp32_is_the_block_sum_on_integers():
    # On integer operands every float32 addition is exact, so the float32
    # coded block must equal the float64 encode (the plain sum of the member
    # blocks, Sec. III-A's XOR read as a real sum), including the zero rows
    # of a ragged last block (M = 7 Mb + 11 here) and members in any order.
    from oracle import codes as ocodes
    from oracle import pipeline
    rng = np.random.default_rng(3)
    kb, Mb, K = 8, 16, 40
    M = (kb - 1) * Mb + 11   # Mb = ceil(M / kb) = 16, the last block ragged
    A = rng.integers(-8, 9, size=(M, K)).astype(np.float32)
    cols = [[(0, 3), (7,)], [(1, 6, 7), (2, 4, 5, 6)], [(5,), (0, 1, 2, 3, 4, 5, 6, 7)],
            [(6, 7), (3,)]]
    code = ocodes.Code("array", n=4, k=4, b=2, columns=cols)
    ref = pipeline.encode(A, code, range(8))
    for g, _, members in code.symbols():
        got = quant.coded_block_fp32(A, Mb, list(reversed(members)), M)
        assert got.dtype == np.float32 and got.shape == (Mb, K)
        assert np.array_equal(got.astype(np.float64), ref[g]), g


def test_coded_block_fp32_adds_members_in_ascending_order():
    # Order pin, worked by hand: blocks 0, 1, 2 hold 2^24, 1 and -2^24.
    # Ascending order: 2^24 + 1 rounds (ties to even) to 2^24, minus 2^24
    # gives 0.  Descending order would give -2^24 + 1 (exact) + 2^24 = 1.
    A = np.array([[2.0 ** 24], [1.0], [-(2.0 ** 24)]], dtype=np.float32)
    got = quant.coded_block_fp32(A, 1, [2, 0, 1], 3)
    assert got.tolist() == [[0.0]]
