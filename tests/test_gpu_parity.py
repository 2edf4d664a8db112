"""GPU parity of each step of the hot path against the oracle, bit-exact on
every coefficient (the arithmetic is exact, so the tolerance is zero)."""
import numpy as np
import pytest

import synthetic
from oracle import bfv, nt, ring
from oracle.encoder import BatchEncoder

from gpu_util import context, key_randomness, oracle_ct, random_ct_residues, torch_cuda

pytestmark = pytest.mark.gpu


def _bitrev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2)


def _ntt_word_index(p, bits):
    """Transform index held at storage word p (index i is stored at (i mod 16) * N/16 + i // 16)."""
    return (p % (1 << (bits - 4))) * 16 + p // (1 << (bits - 4))


@pytest.mark.parametrize("pname", ["t1k", "t2k"])
def test_ntt_forward_is_the_definition(pname):
    torch = torch_cuda()
    prm, ctx = context(pname)
    n = prm.n
    bits = n.bit_length() - 1
    primes = ctx.primes                     # Q, P, aux, t
    x = np.stack([synthetic.test_poly(7, i, [q], n)[0] for i, q in enumerate(primes)])
    d = torch.from_numpy(x.astype(np.float64))[None].cuda()
    ctx.ntt(d, 0)
    got = d.cpu().numpy()[0].astype(np.uint64)
    perm = np.array([_bitrev(_ntt_word_index(p, bits), bits) for p in range(n)])
    for i, q in enumerate(primes):
        ref = np.array(ring.ntt([int(v) for v in x[i]], q, nt.negacyclic_root(q, n)), dtype=np.uint64)
        assert (got[i] == ref[perm]).all(), "limb %d (q=%d)" % (i, q)
    ctx.ntt(d, 0, inverse=True)
    assert (d.cpu().numpy()[0].astype(np.uint64) == x).all()


def test_ntt_full_size_sampled():
    torch = torch_cuda()
    prm, ctx = context("cfg3")
    n = prm.n
    bits = n.bit_length() - 1
    x = synthetic.test_poly(9, 0, ctx.q, n)
    d = torch.from_numpy(x.astype(np.float64))[None].cuda()
    ctx.ntt(d, 0)
    got = d.cpu().numpy()[0].astype(np.uint64)
    rng = np.random.default_rng(0)
    for i, q in enumerate(ctx.q[:2]):
        psi = nt.negacyclic_root(q, n)
        xi = [int(v) for v in x[i]]
        for pos in rng.integers(0, n, 6):
            assert int(got[i, pos]) == ring.ntt_at(xi, q, psi, _bitrev(_ntt_word_index(int(pos), bits), bits))
    ctx.ntt(d, 0, inverse=True)
    assert (d.cpu().numpy()[0].astype(np.uint64) == x).all()


@pytest.fixture(scope="module")
def env_t1k():
    torch_cuda()
    prm, ctx = context("t1k")
    s = synthetic.ternary_secret(31, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    a, e = key_randomness(prm, 31, 0)
    from paper_2402_01296_amd import bcn
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    rk = bfv.relin_key(prm, [int(v) for v in s], a, e)
    return dict(prm=prm, ctx=ctx, s=[int(v) for v in s], sk=sk, ek=ek, rk=rk, enc=BatchEncoder(prm.n, prm.t))


@pytest.fixture(scope="module")
def env_t2k():
    torch_cuda()
    prm, ctx = context("t2k")
    s = synthetic.ternary_secret(32, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    from paper_2402_01296_amd import bcn
    a, e = key_randomness(prm, 32, 0)
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    rk = bfv.relin_key(prm, [int(v) for v in s], a, e)
    gk = {}
    for r in (1, 3, 16, 100):
        a, e = key_randomness(prm, 32, 1000 + r)
        ctx.keygen(sk, ek, bcn.BCN_KEY_ROTATION, r, np.stack(a), np.stack(e))
        gk[r] = bfv.galois_key(prm, [int(v) for v in s], r, a, e)
    return dict(prm=prm, ctx=ctx, s=[int(v) for v in s], sk=sk, ek=ek, rk=rk, gk=gk, enc=BatchEncoder(prm.n, prm.t))


def _key_rns(prm, key):
    moduli = list(prm.q) + list(prm.p)
    return np.stack([np.stack([bfv.to_rns(part, moduli) for part in pair]) for pair in key.parts])


def test_relin_key_parity(env_t1k):
    ev = env_t1k
    from paper_2402_01296_amd import bcn
    got = ev["ctx"].export_key(ev["ek"], bcn.BCN_KEY_RELIN)
    assert (got == _key_rns(ev["prm"], ev["rk"])).all()


def test_rotation_key_parity(env_t2k):
    ev = env_t2k
    from paper_2402_01296_amd import bcn
    got = ev["ctx"].export_key(ev["ek"], bcn.BCN_KEY_ROTATION, 3)
    assert (got == _key_rns(ev["prm"], ev["gk"][3])).all()


@pytest.mark.parametrize("envname", ["env_t1k", "env_t2k"])
def test_encrypt_decrypt_parity(envname, request):
    ev = request.getfixturevalue(envname)
    prm, ctx = ev["prm"], ev["ctx"]
    rng = np.random.default_rng(3)
    for level in (prm.L, 1):
        slots = rng.integers(-(prm.t // 2), prm.t // 2, (3, prm.n))
        q = list(prm.q[:level])
        a = np.stack([synthetic.uniform_residues(5, "enc_a", (i,), q, prm.n) for i in range(3)])
        e = np.stack([synthetic.gaussian_error(5, "enc_e", (i,), prm.n) for i in range(3)])
        ct = ctx.encrypt(ev["sk"], slots, a, e, level)
        got = ctx.export(ct)
        for i in range(3):
            oc = bfv.encrypt(prm, ev["s"], ev["enc"].encode(slots[i]), a[i], e[i], level)
            assert (got[i] == bfv.ct_to_rns(prm, oc)).all(), "ciphertext %d level %d" % (i, level)
        assert (ctx.decrypt(ev["sk"], ct) == slots).all()


def test_import_export_roundtrip(env_t1k):
    ev = env_t1k
    res = random_ct_residues(ev["prm"], 2, 3, 11)
    assert (ev["ctx"].export(ev["ctx"].import_(res)) == res).all()


@pytest.mark.parametrize("n_in,n_out,bound", [(37, 19, 31), (7, 100, 15), (300, 3, 1000)])
def test_mac_parity(env_t1k, n_in, n_out, bound):
    # (7, 100): two 64-row tiles, the second partial, column count not a multiple of 4;
    # (300, 3): large weights force partial reductions inside the accumulation
    ev = env_t1k
    prm, ctx = ev["prm"], ev["ctx"]
    level = prm.L
    res = random_ct_residues(prm, level, n_in, 12)
    w = np.random.default_rng(4).integers(-bound, bound + 1, (n_out, n_in)).astype(np.int32)
    w[min(3, n_out - 1)] = 0                   # an all-zero row
    w[:, min(5, n_in - 1)] = 0                 # an unused input
    out = ctx.export(ctx.mac(ctx.import_(res), w))
    cts = [oracle_ct(prm, r) for r in res]
    for o in range(n_out):
        ref = bfv.ct_to_rns(prm, bfv.mac(prm, cts, w[o]))
        assert (out[o] == ref).all(), "output %d" % o


@pytest.mark.parametrize("tile", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("regime", ["uncentred", "centred"])
def test_mac_parity_every_tile(env_t1k, tile, regime, monkeypatch):
    """Each compiled output-tile width, on the uncentred path (a tile's sum of |w| (q-1) fits
    2^53) and on the centred path with partial reductions (it does not)."""
    ev = env_t1k
    prm, ctx = ev["prm"], ev["ctx"]
    level = prm.L
    # one full tile and a partial one; centred: |w| up to 30000 makes a tile's sum of |w| (q-1)
    # exceed 2^53 and forces a partial reduction every few inputs
    n_out = tile + 3
    n_in, bound = (37, 15) if regime == "uncentred" else (13, 30000)
    res = random_ct_residues(prm, level, n_in, 20 + tile)
    w = np.random.default_rng(tile).integers(-bound, bound + 1, (n_out, n_in)).astype(np.int32)
    w[2] = 0
    monkeypatch.setenv("BCN_MAC_TILE", str(tile))
    out = ctx.export(ctx.mac(ctx.import_(res), w))
    cts = [oracle_ct(prm, r) for r in res]
    for o in range(n_out):
        ref = bfv.ct_to_rns(prm, bfv.mac(prm, cts, w[o]))
        assert (out[o] == ref).all(), "tile %d output %d" % (tile, o)


def test_plain_ops_parity(env_t1k):
    ev = env_t1k
    prm, ctx, enc = ev["prm"], ev["ctx"], ev["enc"]
    res = random_ct_residues(prm, 2, 2, 13)
    rng = np.random.default_rng(5)
    slots = rng.integers(-300, 300, (2, prm.n))
    ct = ctx.import_(res)
    ctx.add_plain(ct, slots)
    got = ctx.export(ct)
    for i in range(2):
        ref = bfv.add_plain(prm, oracle_ct(prm, res[i]), enc.encode(slots[i]))
        assert (got[i] == bfv.ct_to_rns(prm, ref)).all()
    mslots = rng.integers(-20, 21, prm.n)
    got = ctx.export(ctx.mul_plain(ctx.import_(res), mslots))
    for i in range(2):
        ref = bfv.mul_plain(prm, oracle_ct(prm, res[i]), enc.encode(mslots))
        assert (got[i] == bfv.ct_to_rns(prm, ref)).all()


@pytest.mark.parametrize("envname", ["env_t1k", "env_t2k"])
@pytest.mark.parametrize("modsw", [False, True])
def test_square_relin_parity(envname, modsw, request):
    ev = request.getfixturevalue(envname)
    prm, ctx = ev["prm"], ev["ctx"]
    for level in sorted({prm.L, 2}):
        res = random_ct_residues(prm, level, 3, 20 + level)
        got = ctx.export(ctx.square_relin(ev["ek"], ctx.import_(res), modswitch=modsw))
        for i in range(3):
            ref = bfv.square(prm, oracle_ct(prm, res[i]), ev["rk"])
            if modsw:
                ref = bfv.modswitch(prm, ref)
            assert (got[i] == bfv.ct_to_rns(prm, ref)).all(), "ct %d level %d" % (i, level)


def test_modswitch_parity(env_t2k):
    ev = env_t2k
    prm, ctx = ev["prm"], ev["ctx"]
    res = random_ct_residues(prm, prm.L, 3, 30)
    got = ctx.export(ctx.modswitch(ctx.import_(res)))
    for i in range(3):
        ref = bfv.modswitch(prm, oracle_ct(prm, res[i]))
        assert (got[i] == bfv.ct_to_rns(prm, ref)).all()


@pytest.mark.parametrize("level", [4, 3])
def test_rotation_parity_hoisted(env_t2k, level):
    ev = env_t2k
    prm, ctx = ev["prm"], ev["ctx"]
    res = random_ct_residues(prm, level, 2, 40 + level)
    steps = [1, 3, 16, 100]
    got = ctx.export(ctx.rotate(ev["ek"], ctx.import_(res), steps).reshape(-1, 2, level, prm.n))
    for i in range(2):
        ct = oracle_ct(prm, res[i])
        for si, r in enumerate(steps):
            ref = bfv.rotate(prm, ct, r, ev["gk"][r])
            assert (got[i * len(steps) + si] == bfv.ct_to_rns(prm, ref)).all(), "ct %d step %d" % (i, r)


def test_rotate_sum_parity(env_t2k):
    ev = env_t2k
    prm, ctx = ev["prm"], ev["ctx"]
    from paper_2402_01296_amd import bcn
    # span 4: baby step 1, giant step 2
    assert bcn.rotate_sum_steps(4) == [1, 2]
    a, e = key_randomness(prm, 32, 1002)
    ctx.keygen(ev["sk"], ev["ek"], bcn.BCN_KEY_ROTATION, 2, np.stack(a), np.stack(e))
    gks = {1: ev["gk"][1], 2: bfv.galois_key(prm, ev["s"], 2, a, e)}
    res = random_ct_residues(prm, prm.L, 2, 50)
    ct = ctx.import_(res)
    ctx.rotate_sum(ev["ek"], ct, 4)
    got = ctx.export(ct)
    for i in range(2):
        c = bfv.rotate_sum(prm, oracle_ct(prm, res[i]), 4, gks)
        assert (got[i] == bfv.ct_to_rns(prm, c)).all()


def test_errors_are_reported(env_t1k):
    from paper_2402_01296_amd import bcn
    ev = env_t1k
    ctx = ev["ctx"]
    res = random_ct_residues(ev["prm"], 1, 1, 60)
    ct = ctx.import_(res)
    with pytest.raises(bcn.BcnError) as ei:
        ctx.modswitch(ct)                        # one prime left
    assert ei.value.code == -2
    with pytest.raises(bcn.BcnError) as ei:
        ctx.rotate(ev["ek"], ct, [5])            # no Galois key for step 5
    assert ei.value.code == -3
    bad = res.copy()
    bad[0, 0, 0, 0] = ev["prm"].q[0]             # residue not below its prime
    with pytest.raises(bcn.BcnError):
        ctx.import_(bad)


@pytest.mark.parametrize("pname", ["t1k", "cfg2", "cfg3"])
@pytest.mark.parametrize("persist", ["0", "1"])
def test_transform_shapes_agree(pname, persist, monkeypatch):
    """Every transform shape (registers per thread, per-limb or persistent prefetching kernel)
    the autotuner may pick computes the same exact transform."""
    torch = torch_cuda()
    from oracle import params
    from paper_2402_01296_amd import bcn
    spec = params.get(pname)
    monkeypatch.setenv("BCN_NTT_PERSIST", persist)
    outs = []
    for loge in (3, 4, 5):
        monkeypatch.setenv("BCN_NTT_LOGE", str(loge))
        ctx = bcn.Context(spec.n, spec.q[0].bit_length(), spec.L, spec.K, spec.alpha, spec.t)
        x = np.stack([synthetic.test_poly(3, i, ctx.q, spec.n) for i in range(700)])
        d = torch.from_numpy(x.astype(np.float64)).cuda()
        ctx.ntt(d, 0)
        f = d.cpu().numpy().copy()
        ctx.ntt(d, 0, inverse=True)
        assert (d.cpu().numpy().astype(np.uint64) == x).all()
        outs.append(f)
        ctx.close()
    assert all((o == outs[0]).all() for o in outs)


@pytest.mark.parametrize("pname", ["t1k", "cfg2", "cfg3"])
def test_transform_cross_lane_exchange_agrees(pname, monkeypatch):
    """The transform whose row-transpose exchanges run on cross-lane moves (DPP quad permutations
    and the swizzle unit instead of LDS words) computes the same exact transform, forward and
    inverse, as the LDS exchange."""
    torch = torch_cuda()
    from oracle import params
    from paper_2402_01296_amd import bcn
    spec = params.get(pname)
    for k, v in (("BCN_NTT_PERSIST", "0"), ("BCN_NTT_LOGE", "4"), ("BCN_NTT_PREFETCH", "0")):
        monkeypatch.setenv(k, v)
    outs = []
    for xl in ("0", "1"):
        monkeypatch.setenv("BCN_NTT_XLANE", xl)
        ctx = bcn.Context(spec.n, spec.q[0].bit_length(), spec.L, spec.K, spec.alpha, spec.t)
        x = np.stack([synthetic.test_poly(5, i, ctx.q, spec.n) for i in range(300)])
        d = torch.from_numpy(x.astype(np.float64)).cuda()
        ctx.ntt(d, 0)
        f = d.cpu().numpy().copy()
        ctx.ntt(d, 0, inverse=True)
        assert (d.cpu().numpy().astype(np.uint64) == x).all()
        outs.append(f)
        ctx.close()
    assert (outs[0] == outs[1]).all()


# (parameter set, fused square, key-switch mode, square transform shape); key-switch modes:
# 0 four kernels, 1 one fused kernel, 2 digits+NTT and inner product+INTT
_SQUARE_PATHS = [(p, fs, km, lg) for p in ("t1k", "t2k")
                 for fs, km, lg in (("0", "0", ""), ("1", "0", "3"), ("1", "0", "4"), ("0", "1", ""),
                                    ("1", "1", "3"), ("1", "1", "4"), ("0", "2", ""), ("1", "2", "3"),
                                    ("1", "2", "4"))]
_SQUARE_PATHS += [("cfg2", "0", "0", ""), ("cfg2", "1", "1", "4"), ("cfg2", "1", "1", "5"), ("cfg2", "1", "2", "4"),
                  ("cfg2", "1", "2", "5")]
# ModDown scaling and rounding d0, d1 itself (default) or taking them from the scale-and-round kernel
_SQUARE_PATHS = [sp + ("1",) for sp in _SQUARE_PATHS]
_SQUARE_PATHS += [("t1k", "1", "2", "4", "0"), ("t2k", "1", "2", "4", "0"), ("t1k", "0", "0", "", "0"),
                  ("cfg2", "1", "2", "4", "0")]


@pytest.mark.parametrize("pname,fuse_sq,ks_mode,sq_loge,fuse_md", _SQUARE_PATHS)
def test_square_paths_agree(pname, fuse_sq, ks_mode, sq_loge, fuse_md, monkeypatch):
    """Fused (each transform shape) and unfused square, every key-switching path, and ModDown with
    or without the scale-and-round of d0, d1 folded in, give the oracle's exact ciphertexts."""
    torch_cuda()
    from oracle import params
    from paper_2402_01296_amd import bcn
    monkeypatch.setenv("BCN_FUSE_SQUARE", fuse_sq)
    monkeypatch.setenv("BCN_KS_MODE", ks_mode)
    monkeypatch.setenv("BCN_FUSE_MODDOWN", fuse_md)
    if sq_loge:
        monkeypatch.setenv("BCN_SQUARE_LOGE", sq_loge)
    prm, ctx = context(pname)
    s = synthetic.ternary_secret(31, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    a, e = key_randomness(prm, 31, 0)
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    rk = bfv.relin_key(prm, [int(v) for v in s], a, e)
    res = random_ct_residues(prm, prm.L, 2, 77)
    got = ctx.export(ctx.square_relin(ek, ctx.import_(res), modswitch=True))
    for i in range(2):
        ref = bfv.modswitch(prm, bfv.square(prm, oracle_ct(prm, res[i]), rk))
        assert (got[i] == bfv.ct_to_rns(prm, ref)).all()


@pytest.mark.parametrize("span", [2, 8, 32])
def test_rotate_sum_spans(span):
    """Rotate-and-sum over one round (span 2) and two rounds (baby and giant steps), at the top
    level and at a level whose last key-switching digit holds one prime, bit-equal to the oracle."""
    torch_cuda()
    from paper_2402_01296_amd import bcn
    prm, ctx = context("t2k")
    s = synthetic.ternary_secret(33, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    gk = {}
    for r in bcn.rotate_sum_steps(span):
        a, e = key_randomness(prm, 33, 1000 + r)
        ctx.keygen(sk, ek, bcn.BCN_KEY_ROTATION, r, np.stack(a), np.stack(e))
        gk[r] = bfv.galois_key(prm, [int(v) for v in s], r, a, e)
    for level in (prm.L, 3):
        res = random_ct_residues(prm, level, 2, 90 + level)
        ct = ctx.import_(res)
        ctx.rotate_sum(ek, ct, span)
        got = ctx.export(ct)
        for i in range(2):
            c = bfv.rotate_sum(prm, oracle_ct(prm, res[i]), span, gk)
            assert (got[i] == bfv.ct_to_rns(prm, c)).all(), "ct %d level %d" % (i, level)


@pytest.mark.parametrize("ks_mode", ["0", "2"])
@pytest.mark.parametrize("pname", ["t1k", "t2k"])
def test_rotation_hoisted_paths_agree(pname, ks_mode, monkeypatch):
    """Hoisted rotations (one digit decomposition per source, several Galois keys) through the
    four-kernel and two-kernel key-switching paths, against the oracle."""
    torch_cuda()
    from paper_2402_01296_amd import bcn
    monkeypatch.setenv("BCN_KS_MODE", ks_mode)
    prm, ctx = context(pname)
    s = synthetic.ternary_secret(35, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    steps = [1, 5, 64]
    gk = {}
    for r in steps:
        a, e = key_randomness(prm, 35, 1000 + r)
        ctx.keygen(sk, ek, bcn.BCN_KEY_ROTATION, r, np.stack(a), np.stack(e))
        gk[r] = bfv.galois_key(prm, [int(v) for v in s], r, a, e)
    level = prm.L
    res = random_ct_residues(prm, level, 3, 95)
    got = ctx.export(ctx.rotate(ek, ctx.import_(res), steps).reshape(-1, 2, level, prm.n))
    for i in range(3):
        c = oracle_ct(prm, res[i])
        for si, r in enumerate(steps):
            ref = bfv.rotate(prm, c, r, gk[r])
            assert (got[i * len(steps) + si] == bfv.ct_to_rns(prm, ref)).all(), "ct %d step %d" % (i, r)


@pytest.mark.parametrize("pname,loge", [("t1k", "3"), ("t1k", "4"), ("t2k", "3"), ("t2k", "4"), ("cfg2", "5")])
def test_two_kernel_key_switch_shapes_agree(pname, loge, monkeypatch):
    """The two-kernel key switch at every transform shape the autotuner may pick for it:
    relinearisation (square) and hoisted rotations against the oracle."""
    torch_cuda()
    from paper_2402_01296_amd import bcn
    monkeypatch.setenv("BCN_KS_MODE", "2")
    monkeypatch.setenv("BCN_KS_LOGE", loge)
    prm, ctx = context(pname)
    s = synthetic.ternary_secret(37, prm.n)
    sk = ctx.secret_key(s)
    ek = ctx.eval_keys()
    a, e = key_randomness(prm, 37, 0)
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    rk = bfv.relin_key(prm, [int(v) for v in s], a, e)
    res = random_ct_residues(prm, prm.L, 2, 97)
    got = ctx.export(ctx.square_relin(ek, ctx.import_(res), modswitch=False))
    for i in range(2):
        assert (got[i] == bfv.ct_to_rns(prm, bfv.square(prm, oracle_ct(prm, res[i]), rk))).all()
    steps = [1, 7]
    gk = {}
    for r in steps:
        a, e = key_randomness(prm, 37, 1000 + r)
        ctx.keygen(sk, ek, bcn.BCN_KEY_ROTATION, r, np.stack(a), np.stack(e))
        gk[r] = bfv.galois_key(prm, [int(v) for v in s], r, a, e)
    got = ctx.export(ctx.rotate(ek, ctx.import_(res), steps).reshape(-1, 2, prm.L, prm.n))
    for i in range(2):
        c = oracle_ct(prm, res[i])
        for si, r in enumerate(steps):
            assert (got[i * len(steps) + si] == bfv.ct_to_rns(prm, bfv.rotate(prm, c, r, gk[r]))).all()
