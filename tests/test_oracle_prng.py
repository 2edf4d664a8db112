"""Pins of the ChaCha20 streams and samplers: the RFC 8439 test vectors of the quarter
round and the block function, the CDT table's properties (monotone, symmetric about
zero, no threshold within 2^-20 of an integer so any >= 90-bit evaluation agrees), and
the samplers' ranges and moments."""
import numpy as np

from oracle import prng


def test_quarter_round_rfc8439_vector():
    # RFC 8439 section 2.1.1
    assert prng.quarter_round(0x11111111, 0x01020304, 0x9B8D6F43, 0x01234567) == \
        (0xEA2A92F4, 0xCB1CF8CE, 0x4581472E, 0x5881C4BB)


def test_block_function_rfc8439_vector():
    # RFC 8439 section 2.3.2: key 00..1f, nonce 00 00 00 09 00 00 00 4a 00 00 00 00, counter 1
    key = bytes(range(32))
    nonce = bytes.fromhex("000000090000004a00000000")
    want = bytes.fromhex(
        "10f1e7e4d13b5915500fdd1fa32071c4c7d1f4c733c068030422aa9ac3d46c4e"
        "d2826446079faa0914c2d705d98b02a2b5129cd1de164eb9cbd083e8a2503c4e")
    assert prng.block(key, 1, nonce) == want


def test_cdt_table_properties():
    from decimal import Decimal, getcontext
    t = prng.cdt_thresholds()
    assert len(t) == 38 and all(a < b for a, b in zip(t, t[1:]))
    # symmetric: T_k + T_{-k-1} = 2^64 up to the floors
    for k in range(19):
        assert abs(t[k] + t[37 - k] - 2 ** 64) <= 1
    # margin: 2^64 CDF(k) is never within 2^-20 of an integer
    getcontext().prec = 80
    rho = [(-(Decimal(k) ** 2) / (2 * Decimal("3.2") ** 2)).exp() for k in range(-19, 20)]
    total, acc = sum(rho), Decimal(0)
    for r in rho[:-1]:
        acc += r
        v = acc / total * Decimal(2) ** 64
        frac = v - int(v)
        assert Decimal(2) ** -20 < frac < 1 - Decimal(2) ** -20


def test_samplers_ranges_and_moments():
    st = prng.Stream(7, prng.P_ENC_E, 3)
    g = prng.gaussian(st, 4000)
    assert max(abs(x) for x in g) <= 19
    assert abs(np.mean(g)) < 0.25 and abs(np.std(g) - 3.2) < 0.2
    t = prng.ternary(prng.Stream(7, prng.P_SECRET, 0), 3000)
    assert set(t) == {-1, 0, 1}
    q = 1099510054913
    u = prng.uniform(prng.Stream(7, prng.P_ENC_A, (5 << 32) | 1), q, 2000)
    assert all(0 <= x < q for x in u) and abs(np.mean(u) / q - 0.5) < 0.03
    # streams are independent of one another and reproducible
    assert prng.Stream(1, 2, 3).next() == prng.Stream(1, 2, 3).next() != prng.Stream(1, 2, 4).next()
