"""Pins of the CKKS oracle (the paper's scheme, appendix "CKKS Scheme"): the encoder
against direct polynomial evaluation at the roots of X^N + 1, slot rotation and slot
products through the ring, exact encryption and tensor identities, and the homomorphic
operations' decrypted slots within their error bounds."""
import cmath

import numpy as np
import pytest

import synthetic
from oracle import bfv, ckks, params, ring


def _horner(m, x):
    acc = 0j
    for c in reversed(m):
        acc = acc * x + c
    return acc


@pytest.mark.parametrize("n", [8, 16, 32])
def test_encode_evaluates_to_the_slots(n):
    """m = encode(z): m(zeta^(5^i)) = Delta z_i and m(zeta^(-5^i)) = Delta conj(z_i), up to the
    coefficient rounding (|error| <= N/2), by Horner evaluation at the complex roots."""
    rng = np.random.default_rng(n)
    z = rng.normal(size=n // 2) + 1j * rng.normal(size=n // 2)
    scale = 2.0 ** 20
    m = ckks.encode(z, scale, n)
    assert all(isinstance(c, int) for c in m)
    for i in range(n // 2):
        e = pow(5, i, 2 * n)
        root = cmath.exp(1j * cmath.pi * e / n)
        assert abs(_horner(m, root) - scale * z[i]) <= n / 2
        assert abs(_horner(m, root.conjugate()) - scale * np.conj(z[i])) <= n / 2


def test_slot_exponents_cover_half_the_odd_residues():
    n = 64
    e = ckks.slot_exponents(n)
    both = set(e) | {(2 * n - x) % (2 * n) for x in e}
    assert len(set(e)) == n // 2 and both == set(range(1, 2 * n, 2))


@pytest.mark.parametrize("r", [1, 3, -2])
def test_rotation_and_product_through_the_ring(r):
    """decode(sigma_{5^r} m) = z shifted left by r; decode(m1 m2) = z1 z2 at scale Delta^2."""
    n = 64
    rng = np.random.default_rng(5)
    z1 = rng.uniform(-1, 1, n // 2)
    z2 = rng.uniform(-1, 1, n // 2)
    scale = 2.0 ** 24
    m1, m2 = ckks.encode(z1, scale, n), ckks.encode(z2, scale, n)
    rot = ring.automorphism(m1, ckks.galois_element(params.make("x", n, 30, 1, 1, 1, 65537), r))
    assert np.abs(ckks.decode(rot, scale, n) - np.roll(z1, -r)).max() <= n / scale
    prod = ring.negacyclic_mul(m1, m2)
    assert np.abs(ckks.decode(prod, scale * scale, n) - z1 * z2).max() <= 4 * n / scale


def _env(pname="t1k", seed=17):
    prm = params.get(pname)
    s = [int(x) for x in synthetic.ternary_secret(seed, prm.n)]
    moduli = list(prm.q) + list(prm.p)
    d = prm.dnum(prm.L)

    def rnd(key_id):
        a = [synthetic.uniform_residues(seed, "ksk_a", (key_id, j), moduli, prm.n) for j in range(d)]
        e = [synthetic.gaussian_error(seed, "ksk_e", (key_id, j), prm.n) for j in range(d)]
        return a, e
    rk = bfv.relin_key(prm, s, *rnd(0))
    return prm, s, rk, rnd


def _enc(prm, s, z, scale, idx, level=None):
    level = prm.L if level is None else level
    m = ckks.encode(z, scale, prm.n)
    a = synthetic.uniform_residues(9, "enc_a", (idx,), prm.q[:level], prm.n)
    e = synthetic.gaussian_error(9, "enc_e", (idx,), prm.n)
    return ckks.encrypt(prm, s, m, a, e, level), m, e


def test_decrypt_is_message_plus_error_exactly():
    prm, s, rk, rnd = _env()
    z = np.linspace(-1, 1, prm.n // 2)
    ct, m, e = _enc(prm, s, z, 2.0 ** 30, 0)
    assert ckks.decrypt(prm, s, ct) == [int(a) + int(b) for a, b in zip(m, e)]


def test_tensor_is_the_square_of_the_decryption_mod_q():
    """d0 + d1 s + d2 s^2 = (c0 + c1 s)^2 mod Q_l (exact ring identity)."""
    prm, s, rk, rnd = _env()
    ct, _, _ = _enc(prm, s, np.full(prm.n // 2, 0.5), 2.0 ** 20, 1)
    Q = prm.Q(ct.level)
    d0, d1, d2 = ckks.tensor(prm, ct, ct)
    s2 = ring.negacyclic_mul(s, s)
    lhs = [(a + b + c) % Q for a, b, c in zip(d0, ring.negacyclic_mul(d1, s), ring.negacyclic_mul(d2, s2))]
    x = [(a + b) % Q for a, b in zip(ct.c0, ring.negacyclic_mul(ct.c1, s))]
    assert lhs == ring.reduce(ring.negacyclic_mul(x, x), Q)


def test_homomorphic_ops_decode_within_bounds():
    """Mult(c1,c2) + relinearisation + rescale, Mult(c,u), Add(c,u), Rot(c,r): decrypted slots
    equal the slot-wise results within the encoding, encryption and key-switching errors."""
    prm, s, rk, rnd = _env()
    n = prm.n
    rng = np.random.default_rng(1)
    z1 = rng.uniform(-1, 1, n // 2)
    u = rng.uniform(-1, 1, n // 2)
    scale = float(prm.q[prm.L - 1])          # the scale that rescaling by q_L returns to
    ct, _, _ = _enc(prm, s, z1, scale, 2)
    sq = ckks.rescale(prm, ckks.square_relin(prm, ct, rk))
    got = ckks.decode(ckks.decrypt(prm, s, sq), scale * scale / prm.q[prm.L - 1], n)
    assert np.abs(got - z1 * z1).max() < 1e-4
    mp = ckks.rescale(prm, ckks.mul_plain(prm, ct, ckks.encode(u, scale, n)))
    got = ckks.decode(ckks.decrypt(prm, s, mp), scale * scale / prm.q[prm.L - 1], n)
    assert np.abs(got - z1 * u).max() < 1e-4
    ap = ckks.add_plain(prm, ct, ckks.encode(u, scale, n))
    assert np.abs(ckks.decode(ckks.decrypt(prm, s, ap), scale, n) - (z1 + u)).max() < 1e-4
    for r in (1, 5):
        gk = ckks.galois_key(prm, s, r, *rnd(1000 + r))
        rt = ckks.rotate(prm, ct, r, gk)
        assert np.abs(ckks.decode(ckks.decrypt(prm, s, rt), scale, n) - np.roll(z1, -r)).max() < 1e-4


def test_real_network_is_the_integer_network_on_integers():
    """With pixel scale 1, weight scale 1 and the features replaced by their quantised
    integers, the real-valued network equals the integer network (to FP64 rounding: the
    values reach 10^22)."""
    from oracle import ckks_network, network
    from synthetic import workloads as W
    name = "cfg3_ckks_small"
    inp = W.make_inputs(name)
    q = dict(inp, features=[None if f is None else network.quantise(f).astype(np.float64) for f in inp["features"]])
    got = ckks_network.run(name, q, pixel_scale=1.0, wscale=1.0)
    want = np.asarray(network.run(name, inp), dtype=np.float64)
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=1e-12, atol=0)
