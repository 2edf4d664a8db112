"""Pins of the oracle's number theory and ring arithmetic against definitions
and closed forms that do not share its code paths."""
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import nt, ring


def _sieve(n):
    s = bytearray([1]) * (n + 1)
    s[0] = s[1] = 0
    for i in range(2, int(n ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = bytearray(len(s[i * i::i]))
    return s


def test_is_prime_matches_sieve():
    s = _sieve(20000)
    for n in range(20000):
        assert nt.is_prime(n) == bool(s[n]), n


def test_ntt_primes_rule():
    # the largest primes below 2^bits that are 1 mod 2N, in order, none skipped
    for bits, two_n, count in [(20, 64, 4), (30, 8192, 3), (36, 16384, 2)]:
        ps = nt.ntt_primes(bits, two_n, count)
        assert ps == sorted(ps, reverse=True)
        top = (1 << bits) - 1
        cand = [p for p in range(top - top % two_n + 1, ps[-1] - 1, -two_n) if p < (1 << bits)]
        primes = [p for p in cand if nt.is_prime(p)]
        assert primes[:count] == ps
        for p in ps:
            assert (p - 1) % two_n == 0 and p.bit_length() == bits


def test_negacyclic_root_is_smallest_primitive():
    for q, n in [(17, 8), (97, 16), (193, 32), (257, 64), (65537, 4096), (12289, 1024)]:
        psi = nt.negacyclic_root(q, n)
        assert pow(psi, n, q) == q - 1
        assert pow(psi, 2 * n, q) == 1
        for x in range(2, psi):
            assert pow(x, n, q) != q - 1
        assert psi == nt.negacyclic_root_search(q, n)


def test_crt_and_centered():
    rnd = random.Random(1)
    mods = [97, 193, 257, 65537]
    M = 97 * 193 * 257 * 65537
    for _ in range(200):
        x = rnd.randrange(M)
        assert nt.crt([x % m for m in mods], mods) == x
        c = nt.centered(x, M)
        assert -M / 2 < c < M / 2 and (c - x) % M == 0
    import math
    for a in range(-40, 41):
        for b in (1, 3, 5, 7, 65537):
            f = Fraction(a, b)
            near = math.floor(f + Fraction(1, 2))
            assert nt.round_div(a, b) == near
            assert abs(f - near) <= Fraction(1, 2)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
def test_negacyclic_mul_matches_schoolbook(n):
    rnd = random.Random(n)
    for bits in (1, 8, 40, 300):
        a = [rnd.randrange(-(1 << bits), 1 << bits) for _ in range(n)]
        b = [rnd.randrange(-(1 << bits), 1 << bits) for _ in range(n)]
        assert ring.negacyclic_mul(a, b) == ring.schoolbook_mul(a, b)
    assert ring.negacyclic_mul([0] * n, [1] * n) == [0] * n


def test_x_to_the_n_is_minus_one():
    for n in (8, 64, 1024):
        x = [0] * n
        x[n - 1] = 1                         # X^(N-1)
        y = [0] * n
        y[1] = 1                             # X
        assert ring.negacyclic_mul(x, y) == [-1] + [0] * (n - 1)


def test_automorphism_is_ring_homomorphism():
    rnd = random.Random(3)
    n = 32
    a = [rnd.randrange(-50, 50) for _ in range(n)]
    b = [rnd.randrange(-50, 50) for _ in range(n)]
    for k in (1, 3, 5, 9, 2 * n - 1, 27):
        lhs = ring.automorphism(ring.negacyclic_mul(a, b), k)
        rhs = ring.negacyclic_mul(ring.automorphism(a, k), ring.automorphism(b, k))
        assert lhs == rhs
    assert ring.automorphism(a, 1) == a
    assert ring.automorphism(ring.automorphism(a, 3), 5) == ring.automorphism(a, 15)
    # X -> X^k sends X^i to +-X^(ik mod N): check one monomial by hand
    mono = [0] * n
    mono[7] = 1
    out = ring.automorphism(mono, 5)          # X^35 = X^32 * X^3 = -X^3
    assert out[3] == -1 and sum(abs(v) for v in out) == 1


@pytest.mark.parametrize("n,q", [(8, 17), (16, 97), (32, 193), (64, 257)])
def test_ntt_convolution_theorem(n, q):
    psi = nt.negacyclic_root(q, n)
    rnd = random.Random(n)
    a = [rnd.randrange(q) for _ in range(n)]
    b = [rnd.randrange(q) for _ in range(n)]
    prod = ring.reduce(ring.schoolbook_mul(a, b), q)
    fa, fb, fp = ring.ntt(a, q, psi), ring.ntt(b, q, psi), ring.ntt(prod, q, psi)
    assert fp == [x * y % q for x, y in zip(fa, fb)]
    # linearity, monomials (closed form), single-output evaluator
    c = [(3 * x + 5 * y) % q for x, y in zip(a, b)]
    assert ring.ntt(c, q, psi) == [(3 * x + 5 * y) % q for x, y in zip(fa, fb)]
    m = 5
    mono = [0] * n
    mono[m] = 1
    assert ring.ntt(mono, q, psi) == [pow(psi, (2 * j + 1) * m, q) for j in range(n)]
    assert all(ring.ntt_at(a, q, psi, j) == fa[j] for j in range(n))
    # the N points are distinct, so the transform is invertible
    assert len({pow(psi, 2 * j + 1, q) for j in range(n)}) == n


def test_lift_c_range_and_congruence():
    m = 1_000_003
    xs = list(range(0, m, 9973)) + [m - 1, (m - 1) // 2, (m + 1) // 2]
    ys = ring.lift_c(xs, m)
    for x, y in zip(xs, ys):
        assert -m / 2 < y < m / 2 and (x - y) % m == 0
