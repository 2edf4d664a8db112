"""The library's client-side samplers against the oracle's, on the host (no GPU): every
ChaCha20 stream value and sample bit-equal, the Gaussian table identical, and bad
arguments reported as errors."""
import os

import pytest

from oracle import prng


@pytest.fixture(scope="module")
def bcn():
    from paper_2402_01296_amd import bcn
    if not os.path.exists(bcn.LIB_PATH):
        from paper_2402_01296_amd import build
        build.build()
    return bcn


def test_gaussian_table_identical(bcn):
    assert bcn.gaussian_table() == prng.cdt_thresholds()


@pytest.mark.parametrize("seed,purpose,index", [(0, 1, 0), (31, 3, (7 << 32) | 5), (2 ** 64 - 1, 5, 2 ** 63 + 9),
                                                (123456789, 2, (1 << 32) | 11)])
def test_samples_bit_equal(bcn, seed, purpose, index):
    n = 517      # not a multiple of the 8 values of a block
    assert [int(x) for x in bcn.sample(bcn.BCN_SAMPLE_TERNARY, seed, purpose, index, n)] == \
        prng.ternary(prng.Stream(seed, purpose, index), n)
    assert [int(x) for x in bcn.sample(bcn.BCN_SAMPLE_GAUSSIAN, seed, purpose, index, n)] == \
        prng.gaussian(prng.Stream(seed, purpose, index), n)
    for q in (65537, 1099510054913, 2 ** 62):
        assert [int(x) for x in bcn.sample(bcn.BCN_SAMPLE_UNIFORM, seed, purpose, index, n, q)] == \
            prng.uniform(prng.Stream(seed, purpose, index), q, n)


def test_key_stream_layout(bcn):
    """The key-switching randomness of key k, digit j, prime i is the stream
    (seed, KSK_A, k << 32 | j (L+K) + i): spot-check one digit against the oracle's layout."""
    moduli = [1099510054913, 1099507695617, 1099506515969]
    a, e = prng.ksk_randomness(9, 25, moduli, 2, 64)
    for j in range(2):
        for i, q in enumerate(moduli):
            got = bcn.sample(bcn.BCN_SAMPLE_UNIFORM, 9, bcn.BCN_PURPOSE_KSK_A, (25 << 32) | (j * 3 + i), 64, q)
            assert [int(x) for x in got] == a[j][i]
        got = bcn.sample(bcn.BCN_SAMPLE_GAUSSIAN, 9, bcn.BCN_PURPOSE_KSK_E, (25 << 32) | j, 64)
        assert [int(x) for x in got] == e[j]


def test_bad_arguments(bcn):
    with pytest.raises(bcn.BcnError):
        bcn.sample(7, 1, 1, 0, 4)
    with pytest.raises(bcn.BcnError):
        bcn.sample(bcn.BCN_SAMPLE_UNIFORM, 1, 1, 0, 4, 1)
    with pytest.raises(bcn.BcnError):
        bcn.sample(bcn.BCN_SAMPLE_UNIFORM, 1, 1, 0, 4, 2 ** 62 + 1)
    assert len(bcn.sample(bcn.BCN_SAMPLE_TERNARY, 1, 1, 0, 0)) == 0
