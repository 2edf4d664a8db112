"""CKKS on the GPU against the CKKS oracle: the encoder within one unit of the
oracle's rounding, secret-key encryption, and bit-exact ring operations (the
exact tensor with relinearisation and rescale, rotations with k = 5^r, plaintext
multiply and add) on the same inputs."""
import numpy as np
import pytest

import synthetic
from oracle import bfv, ckks, params

from gpu_util import key_randomness, oracle_ct, random_ct_residues, torch_cuda

pytestmark = pytest.mark.gpu


def _ctx(pname):
    from paper_2402_01296_amd import bcn
    prm = params.get(pname)
    ctx = bcn.Context(prm.n, prm.q[0].bit_length(), prm.L, prm.K, prm.alpha, 0, ckks=True)
    assert ctx.q == list(prm.q) and ctx.p_primes == list(prm.p)
    return prm, ctx


def _centred(res, prm, level):
    vals = bfv.from_rns(res, prm.q[:level])
    Q = prm.Q(level)
    return np.array([v - Q if 2 * v > Q else v for v in vals], dtype=object)


@pytest.mark.parametrize("pname", ["t2k3", "cfg3"])
def test_encoder_within_one_unit_of_the_oracle(pname):
    torch = torch_cuda()
    prm, ctx = _ctx(pname)
    rng = np.random.default_rng(7)
    z = rng.uniform(-1, 1, (2, prm.n // 2))
    scale = 2.0 ** 30
    level = 2
    got = ctx.ckks_encode(torch.from_numpy(z).cuda(), level, scale).cpu().numpy().astype(np.uint64)
    for i in range(2):
        want = np.array(ckks.encode(z[i], scale, prm.n), dtype=object)
        g = _centred(got[i], prm, level)
        diff = np.abs((g - want).astype(np.int64))
        assert diff.max() <= 1
        assert (diff != 0).mean() < 1e-3


def _keys(prm, ctx, seed, steps=()):
    from paper_2402_01296_amd import bcn
    s = synthetic.ternary_secret(seed, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    a, e = key_randomness(prm, seed, 0)
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    rk = bfv.relin_key(prm, [int(x) for x in s], a, e)
    gks = {}
    for r in steps:
        a, e = key_randomness(prm, seed, 1000 + r)
        ctx.keygen(sk, ek, bcn.BCN_KEY_ROTATION, r, np.stack(a), np.stack(e))
        gks[r] = ckks.galois_key(prm, [int(x) for x in s], r, a, e)
    return [int(x) for x in s], sk, ek, rk, gks


def test_encrypt_matches_the_oracle_up_to_the_encoding():
    torch = torch_cuda()
    prm, ctx = _ctx("t2k3")
    s, sk, ek, rk, _ = _keys(prm, ctx, 61)
    z = np.random.default_rng(3).uniform(-1, 1, (1, prm.n // 2))
    scale, level = 2.0 ** 35, prm.L
    a = np.stack([synthetic.uniform_residues(8, "enc_a", (0,), prm.q[:level], prm.n)])
    e = np.stack([synthetic.gaussian_error(8, "enc_e", (0,), prm.n)])
    ct = ctx.ckks_encrypt(sk, z, scale, a, e, level)
    got = ctx.export(ct)[0]
    enc_gpu = _centred(ctx.ckks_encode(torch.from_numpy(z).cuda(), level, scale).cpu().numpy().astype(np.uint64)[0],
                       prm, level)
    m = ckks.encode(z[0], scale, prm.n)
    ref = ckks.encrypt(prm, s, m, a[0], e[0], level)
    assert (got[1] == bfv.to_rns(ref.c1, prm.q[:level])).all()
    # part 0 differs from the oracle's exactly by the encodings' difference (rarely nonzero)
    d = _centred(got[0], prm, level) - np.array(ring_c(ref.c0, prm.Q(level)), dtype=object)
    assert (d == enc_gpu - np.array(m, dtype=object)).all()
    dec = ctx.ckks_decrypt(sk, ct, scale)
    assert np.abs(dec[0] - z[0]).max() < 1e-6


def ring_c(c, Q):
    return [v - Q if 2 * v > Q else v for v in c]


@pytest.mark.parametrize("pname", ["t2k3", "t1k"])
def test_square_relin_rescale_bit_exact(pname):
    torch_cuda()
    prm, ctx = _ctx(pname)
    s, sk, ek, rk, _ = _keys(prm, ctx, 62)
    level = prm.L
    res = random_ct_residues(prm, level, 3, 71)
    out = ctx.export(ctx.ckks_square_relin_rescale(ek, ctx.import_(res)))
    for i in range(3):
        ref = ckks.rescale(prm, ckks.square_relin(prm, oracle_ct(prm, res[i]), rk))
        assert (out[i] == bfv.ct_to_rns(prm, ref)).all(), "ciphertext %d" % i


def test_rotation_bit_exact():
    torch_cuda()
    prm, ctx = _ctx("t2k3")
    steps = [1, 5, -3]
    s, sk, ek, rk, gks = _keys(prm, ctx, 63, steps)
    level = prm.L - 1            # a partial last digit (two-prime digits over five primes)
    res = random_ct_residues(prm, level, 2, 72)
    got = ctx.export(ctx.rotate(ek, ctx.import_(res), steps).reshape(2 * len(steps), 2, level, prm.n))
    for i in range(2):
        for k, r in enumerate(steps):
            ref = ckks.rotate(prm, oracle_ct(prm, res[i]), r, gks[r])
            assert (got[i * len(steps) + k] == bfv.ct_to_rns(prm, ref)).all(), "ct %d step %d" % (i, r)


def test_plain_multiply_and_add_bit_exact():
    torch = torch_cuda()
    prm, ctx = _ctx("t2k3")
    level = 3
    res = random_ct_residues(prm, level, 2, 73)
    m = np.random.default_rng(4).integers(-2 ** 20, 2 ** 20, prm.n)
    mres = bfv.to_rns([int(x) for x in m], prm.q[:level])
    pt = torch.from_numpy(mres.astype(np.float64))[None].cuda()
    pt_ntt = pt.clone()
    ctx.ntt(pt_ntt, 0)
    got = ctx.export(ctx.ckks_mul_plain(ctx.import_(res), pt_ntt[0]))
    ct = ctx.import_(res)
    ctx.ckks_add_plain(ct, pt.expand(2, -1, -1).contiguous())
    got_add = ctx.export(ct)
    for i in range(2):
        oc = oracle_ct(prm, res[i])
        assert (got[i] == bfv.ct_to_rns(prm, ckks.mul_plain(prm, oc, [int(x) for x in m]))).all()
        assert (got_add[i] == bfv.ct_to_rns(prm, ckks.add_plain(prm, oc, [int(x) for x in m]))).all()


def test_decode_of_an_oracle_ciphertext():
    """The GPU's decryption and decoding of a ciphertext the oracle encrypted."""
    torch_cuda()
    prm, ctx = _ctx("t2k3")
    s, sk, ek, rk, _ = _keys(prm, ctx, 64)
    z = np.random.default_rng(5).uniform(-1, 1, prm.n // 2)
    scale, level = 2.0 ** 38, prm.L
    a = synthetic.uniform_residues(9, "enc_a", (1,), prm.q[:level], prm.n)
    e = synthetic.gaussian_error(9, "enc_e", (1,), prm.n)
    oc = ckks.encrypt(prm, s, ckks.encode(z, scale, prm.n), a, e, level)
    got = ctx.ckks_decrypt(sk, ctx.import_(bfv.ct_to_rns(prm, oc)[None]), scale)[0]
    want = np.real(ckks.decode(ckks.decrypt(prm, s, oc), scale, prm.n))
    assert np.abs(got - want).max() < 1e-9
    assert np.abs(got - z).max() < 1e-6


@pytest.mark.parametrize("name", ["cfg3_ckks_small", "cfg3_ckks"])
def test_ckks_branch_decrypts_to_the_real_network(name):
    """The CIFAR-shaped branch under CKKS: decrypted outputs equal the FP64 real-valued
    network within 1e-6 relative to its largest output (the scheme's approximation error;
    the inputs are encoded at 2^30 and the last scale is about 2^56)."""
    torch_cuda()
    from oracle import ckks_network
    from paper_2402_01296_amd.ckks_workload import CkksSession
    g = CkksSession(name)
    out, scale = g.run(g.encrypt_inputs())
    got = g.output_values(out, scale)
    want = ckks_network.run(name, g.inputs)
    assert got.shape == want.shape
    assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()
