"""Pins of the CRT batch encoder: decode(encode(v)) = v, slot-wise products,
rotation by the automorphism X -> X^(3^r) (the appendix's Rot: left shift by r
of each row), and a direct power-sum evaluation on tiny sizes."""
import numpy as np
import pytest

from oracle import ring
from oracle.encoder import BatchEncoder


@pytest.mark.parametrize("n,t", [(8, 17), (16, 97), (64, 257), (1024, 65537)])
def test_roundtrip_and_products(n, t):
    enc = BatchEncoder(n, t)
    rng = np.random.default_rng(n)
    u = rng.integers(0, t, n)
    v = rng.integers(0, t, n)
    mu, mv = enc.encode(u), enc.encode(v)
    assert (enc.decode(mu) == u).all()
    prod = ring.reduce(ring.negacyclic_mul(mu, mv), t)
    assert (enc.decode(prod) == u * v % t).all()
    summ = [(a + b) % t for a, b in zip(mu, mv)]
    assert (enc.decode(summ) == (u + v) % t).all()


@pytest.mark.parametrize("n,t", [(16, 97), (64, 257)])
def test_rotation_is_rowwise_left_shift(n, t):
    enc = BatchEncoder(n, t)
    v = np.arange(n) % t
    m = enc.encode(v)
    half = n // 2
    for r in (1, 2, 3, half - 1):
        rot = ring.reduce(ring.automorphism(m, pow(3, r, 2 * n)), t)
        got = enc.decode(rot)
        want = np.concatenate([np.roll(v[:half], -r), np.roll(v[half:], -r)])
        assert (got == want).all()
    # X -> X^(-1) swaps the two rows
    sw = enc.decode(ring.reduce(ring.automorphism(m, 2 * n - 1), t))
    assert (sw == np.concatenate([v[half:], v[:half]])).all()


def test_exponents_cover_odd_residues_and_direct_evaluation():
    n, t = 8, 17
    enc = BatchEncoder(n, t)
    assert sorted(enc.exponent.tolist()) == list(range(1, 2 * n, 2))
    assert pow(enc.zeta, n, t) == t - 1
    v = [3, 1, 4, 1, 5, 9, 2, 6]
    m = enc.encode(v)
    for s in range(n):
        x = pow(enc.zeta, int(enc.exponent[s]), t)
        assert sum(mk * pow(x, k, t) for k, mk in enumerate(m)) % t == v[s]
