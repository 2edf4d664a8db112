"""Seeded keys and encryptions: the library draws the secret key, the key-switching
keys and the encryptions from its own ChaCha20 streams; every key and ciphertext is
bit-equal to the oracle's built from the oracle's streams (CKKS: the mask part
exactly, the body within the encoder's one unit)."""
import numpy as np
import pytest

from oracle import bfv, ckks, params, prng
from oracle.encoder import BatchEncoder

from gpu_util import context, torch_cuda

pytestmark = pytest.mark.gpu


def _key_rns(prm, key):
    moduli = list(prm.q) + list(prm.p)
    return np.stack([np.stack([bfv.to_rns(part, moduli) for part in pair]) for pair in key.parts])


def test_seeded_keys_and_encryption_bfv():
    torch_cuda()
    from paper_2402_01296_amd import bcn
    prm, ctx = context("t2k")
    seed = 2024
    s = prng.secret(seed, prm.n)
    sk = ctx.secret_key_seeded(seed)
    ek = ctx.eval_keys()
    moduli = list(prm.q) + list(prm.p)
    d = prm.dnum(prm.L)
    ctx.keygen_seeded(sk, ek, bcn.BCN_KEY_RELIN, 0, seed)
    a, e = prng.ksk_randomness(seed, 0, moduli, d, prm.n)
    want = _key_rns(prm, bfv.relin_key(prm, s, a, e))
    assert (ctx.export_key(ek, bcn.BCN_KEY_RELIN) == want).all()
    for r in (3, -2):
        ctx.keygen_seeded(sk, ek, bcn.BCN_KEY_ROTATION, r, seed)
        a, e = prng.ksk_randomness(seed, bfv.galois_element(prm, r), moduli, d, prm.n)
        want = _key_rns(prm, bfv.galois_key(prm, s, r, a, e))
        assert (ctx.export_key(ek, bcn.BCN_KEY_ROTATION, r) == want).all(), "rotation %d" % r
    enc = BatchEncoder(prm.n, prm.t)
    rng = np.random.default_rng(4)
    for level, first in ((prm.L, 5), (1, 0)):
        slots = rng.integers(-(prm.t // 2), prm.t // 2, (2, prm.n))
        ct = ctx.encrypt_seeded(sk, slots, seed, first, level)
        got = ctx.export(ct)
        for i in range(2):
            a, e = prng.enc_randomness(seed, first + i, prm.q[:level], prm.n)
            oc = bfv.encrypt(prm, s, enc.encode(slots[i]), a, e, level)
            assert (got[i] == bfv.ct_to_rns(prm, oc)).all(), "ciphertext %d level %d" % (first + i, level)
        assert (ctx.decrypt(sk, ct) == slots).all()


def test_seeded_encryption_ckks():
    torch_cuda()
    from paper_2402_01296_amd import bcn
    prm = params.get("t2k3")
    ctx = bcn.Context(prm.n, prm.q[0].bit_length(), prm.L, prm.K, prm.alpha, 0, ckks=True)
    seed = 77
    s = prng.secret(seed, prm.n)
    sk = ctx.secret_key_seeded(seed)
    z = np.random.default_rng(8).uniform(-1, 1, (2, prm.n // 2))
    scale, level = 2.0 ** 30, 3
    ct = ctx.ckks_encrypt_seeded(sk, z, scale, seed, 0, level)
    got = ctx.export(ct)
    Q = prm.Q(level)
    for i in range(2):
        a, e = prng.enc_randomness(seed, i, prm.q[:level], prm.n)
        oc = ckks.encrypt(prm, s, ckks.encode(z[i], scale, prm.n), a, e, level)
        want = bfv.ct_to_rns(prm, oc)
        assert (got[i, 1] == want[1]).all()
        diff = [(x - y) % Q for x, y in zip(bfv.from_rns(got[i, 0], prm.q[:level]), oc.c0)]
        assert all(v <= 1 or v >= Q - 1 for v in diff)
    back = ctx.ckks_decrypt(sk, ct, scale)
    assert np.abs(back - z).max() < 1e-4
