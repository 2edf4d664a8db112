"""Pins of the oracle's BFV against the appendix identities (CKKS Scheme
section: D(Add(c,u)) = D(c)+u, D(Add(c1,c2)) = D(c1)+D(c2), D(Mult(c,u)) =
D(c)*u, D(Mult(c1,c2)) = D(c1)*D(c2), D(Rot(c,r)) = <D(c)>_r), against an
independent evaluation of the exact definitions (schoolbook products and
Fraction rounding), and against the noise-budget invariant."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synthetic
from oracle import bfv, nt, params, ring
from oracle.encoder import BatchEncoder

PRM = params.get("t1k")        # N=1024, 3 x 36-bit, P 1 x 36-bit, t=65537
PRM2 = params.get("t2k")       # N=2048, 4 x 40-bit, P 2 x 40-bit, alpha=2


class Ctx:
    def __init__(self, prm, seed=11):
        self.prm = prm
        self.enc = BatchEncoder(prm.n, prm.t)
        self.s = [int(x) for x in synthetic.ternary_secret(seed, prm.n)]
        self.seed = seed
        self.count = 0
        self.moduli = list(prm.q) + list(prm.p)

    def rand_key(self, kid):
        d = self.prm.dnum(self.prm.L)
        a = [synthetic.uniform_residues(self.seed, "ksk_a", (kid, j), self.moduli, self.prm.n) for j in range(d)]
        e = [synthetic.gaussian_error(self.seed, "ksk_e", (kid, j), self.prm.n) for j in range(d)]
        return a, e

    def encrypt(self, v, level=None):
        level = self.prm.L if level is None else level
        self.count += 1
        a = synthetic.uniform_residues(self.seed, "enc_a", (self.count,), self.prm.q[:level], self.prm.n)
        e = synthetic.gaussian_error(self.seed, "enc_e", (self.count,), self.prm.n)
        return bfv.encrypt(self.prm, self.s, self.enc.encode(v), a, e, level)

    def dec(self, ct):
        return self.enc.decode(bfv.decrypt(self.prm, self.s, ct))

    def budget(self, ct, v):
        return bfv.noise_budget(self.prm, self.s, ct, self.enc.encode(v))


@pytest.fixture(scope="module")
def cx():
    c = Ctx(PRM)
    a, e = c.rand_key(0)
    c.rk = bfv.relin_key(PRM, c.s, a, e)
    return c


@pytest.fixture(scope="module")
def cx2():
    c = Ctx(PRM2, seed=12)
    a, e = c.rand_key(0)
    c.rk = bfv.relin_key(PRM2, c.s, a, e)
    c.gk = {}
    for r in (1, 5, 100):
        a, e = c.rand_key(1000 + r)
        c.gk[r] = bfv.galois_key(PRM2, c.s, r, a, e)
    return c


def _vec(prm, seed):
    return np.random.default_rng(seed).integers(0, prm.t, prm.n)


def test_encrypt_decrypt_all_levels(cx):
    t = PRM.t
    for level in range(1, PRM.L + 1):
        v = _vec(PRM, level)
        ct = cx.encrypt(v, level)
        assert ct.level == level
        assert (cx.dec(ct) == v).all()
        b = cx.budget(ct, v)
        # fresh noise: |t*e + rounding| <= t*(19 + 1/2) -> budget >= log2(Q/(2*t*19.5)) - 1 bit slack
        assert b >= math.log2(PRM.Q(level) / (2 * t * 19.5)) - 1


def test_encryption_matches_independent_evaluation(cx):
    # c0 = -a*s + e + round(Q*m/t) recomputed with schoolbook product and Fractions on N=8
    prm = params.make("tiny", 8, 30, 2, 1, 1, 17, insecure=True)
    s = [1, 0, -1, 1, 1, 0, 0, -1]
    a_res = synthetic.uniform_residues(5, "enc_a", (0,), prm.q, 8)
    e = [2, -1, 0, 3, -4, 0, 1, 0]
    m = [0, 16, 3, 8, 9, 1, 0, 5]
    ct = bfv.encrypt(prm, s, m, a_res, e)
    Q = prm.Q(2)
    a = [nt.crt([int(a_res[0][i]), int(a_res[1][i])], prm.q) for i in range(8)]
    assert ct.c1 == a
    as_ = ring.schoolbook_mul(a, s)
    for i in range(8):
        want = -as_[i] + e[i] + math.floor(Fraction(Q * m[i], 17) + Fraction(1, 2))
        assert ct.c0[i] == want % Q


def test_add_identities(cx):
    t = PRM.t
    u, v, w = _vec(PRM, 1), _vec(PRM, 2), _vec(PRM, 3)
    cu, cv = cx.encrypt(u), cx.encrypt(v)
    assert (cx.dec(bfv.add(PRM, cu, cv)) == (u + v) % t).all()
    assert (cx.dec(bfv.add_plain(PRM, cu, cx.enc.encode(w))) == (u + w) % t).all()
    assert (cx.dec(bfv.mul_scalar(PRM, cu, -7)) == (-7 * u) % t).all()
    assert (cx.dec(bfv.mac(PRM, [cu, cv], [3, -2])) == (3 * u - 2 * v) % t).all()


def test_mul_plain_identity(cx):
    t = PRM.t
    u = _vec(PRM, 4)
    w = np.random.default_rng(9).integers(-20, 21, PRM.n)
    out = bfv.mul_plain(PRM, cx.encrypt(u), cx.enc.encode(w))
    assert (cx.dec(out) == (u * w) % t).all()


def test_tensor_is_the_exact_definition():
    # independent evaluation on N=8: schoolbook products over Z and Fraction rounding
    prm = params.make("tiny", 8, 30, 2, 1, 1, 17, insecure=True)
    Q, t = prm.Q(2), prm.t
    rng = np.random.default_rng(3)
    a = bfv.Ct([int(x) for x in rng.integers(0, Q, 8)], [int(x) for x in rng.integers(0, Q, 8)], 2)
    b = bfv.Ct([int(x) for x in rng.integers(0, Q, 8)], [int(x) for x in rng.integers(0, Q, 8)], 2)
    d = bfv.tensor(prm, a, b)

    def cl(x):
        x %= Q
        return x - Q if x > Q // 2 else x

    A0, A1 = [cl(x) for x in a.c0], [cl(x) for x in a.c1]
    B0, B1 = [cl(x) for x in b.c0], [cl(x) for x in b.c1]
    e0 = ring.schoolbook_mul(A0, B0)
    e1 = [x + y for x, y in zip(ring.schoolbook_mul(A0, B1), ring.schoolbook_mul(A1, B0))]
    e2 = ring.schoolbook_mul(A1, B1)
    for got, ex in zip(d, (e0, e1, e2)):
        want = [math.floor(Fraction(t * x, Q) + Fraction(1, 2)) % Q for x in ex]
        assert got == want


def test_mult_relin_identity_and_budget(cx):
    t = PRM.t
    u, v = _vec(PRM, 5), _vec(PRM, 6)
    cu, cv = cx.encrypt(u), cx.encrypt(v)
    prod = bfv.multiply(PRM, cu, cv, cx.rk)
    assert (cx.dec(prod) == u * v % t).all()
    sq = bfv.square(PRM, cu, cx.rk)
    assert (cx.dec(sq) == u * u % t).all()
    # budget never increases through an operation
    b0 = cx.budget(cu, u)
    b1 = cx.budget(sq, u * u % t)
    assert 0 < b1 < b0


def test_key_switch_correctness(cx):
    # KS with the relinearisation key maps d2 under s^2 to a pair under s:
    # k0 + k1*s = d2*s^2 + small (mod Q)
    prm = PRM
    Q = prm.Q(prm.L)
    x = bfv.from_rns(synthetic.test_poly(8, 0, prm.q, prm.n), prm.q)
    k0, k1 = bfv.key_switch(prm, x, cx.rk, prm.L)
    s2 = ring.negacyclic_mul(cx.s, cx.s)
    lhs = [(a + b) % Q for a, b in zip(k0, ring.negacyclic_mul(k1, cx.s))]
    rhs = ring.reduce(ring.negacyclic_mul(x, s2), Q)
    err = max(abs(nt.centered(a - b, Q)) for a, b in zip(lhs, rhs))
    # error = sum_j D_j e_j / P + rounding: far below Q
    assert err < 2 ** 30


def test_rotation_identity_and_hoisting(cx2):
    prm, t = PRM2, PRM2.t
    v = _vec(prm, 7)
    ct = cx2.encrypt(v)
    half = prm.n // 2
    single = {}
    for r in (1, 5, 100):
        out = bfv.rotate(prm, ct, r, cx2.gk[r])
        want = np.concatenate([np.roll(v[:half], -r), np.roll(v[half:], -r)])
        assert (cx2.dec(out) == want).all()
        single[r] = out
    hoisted = bfv.rotate_hoisted(prm, ct, [1, 5, 100], [cx2.gk[r] for r in (1, 5, 100)])
    for r, h in zip((1, 5, 100), hoisted):
        assert h.c0 == single[r].c0 and h.c1 == single[r].c1


def test_rotation_at_partial_digit_level(cx2):
    # alpha = 2, level 3: the second digit has one prime left
    prm = PRM2
    v = _vec(prm, 8)
    ct = cx2.encrypt(v, level=3)
    out = bfv.rotate(prm, ct, 1, cx2.gk[1])
    half = prm.n // 2
    want = np.concatenate([np.roll(v[:half], -1), np.roll(v[half:], -1)])
    assert (cx2.dec(out) == want).all()


def test_modswitch_preserves_plaintext_and_is_exact_rounding(cx):
    prm, t = PRM, PRM.t
    u = _vec(prm, 9)
    ct = cx.encrypt(u)
    ms = bfv.modswitch(prm, ct)
    assert ms.level == prm.L - 1
    assert (cx.dec(ms) == u).all()
    ql = prm.q[prm.L - 1]
    for i in range(0, prm.n, 97):
        x = ct.c0[i]
        assert ms.c0[i] == math.floor(Fraction(x, ql) + Fraction(1, 2)) % prm.Q(prm.L - 1)


def test_budget_zero_means_failure():
    # one 30-bit prime: a fresh ciphertext decrypts, its square cannot
    prm = params.make("onelimb", 1024, 30, 1, 1, 1, 65537, insecure=True)
    c = Ctx(prm, seed=21)
    a, e = c.rand_key(0)
    rk = bfv.relin_key(prm, c.s, a, e)
    v = _vec(prm, 10)
    ct = c.encrypt(v)
    assert c.budget(ct, v) > 0 and (c.dec(ct) == v).all()
    sq = bfv.square(prm, ct, rk)
    want = v * v % prm.t
    assert c.budget(sq, want) <= 0
    assert not (c.dec(sq) == want).all()


# ---------------------------------------------------------------- bit-level known answers
#
# The decryption identities above cannot see a +-1 slip in a rounding or a
# different (but still valid) choice of digit representative: every such
# variant still decrypts correctly.  The tests below recompute the exact
# outputs from the definitions alone (appendix "CKKS Scheme": Mult(c1,c2) and
# Rot(c,r), whose key switch is
#     D_j = centred [x]_{Q_j},  u = sum_j D_j * key_j over Z[X]/(X^N+1),
#     KS = nearest integer to u / P, reduced mod Q_l;
# and Mult(c,u) multiplies by the centred lift of u mod t), with schoolbook
# products and Fraction rounding, never through the oracle's own helpers.

def _centred(x, m):
    r = x % m
    return r - m if 2 * r > m else r


def _schoolbook(a, b):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    return c


def _nearest(num, den):
    return math.floor(Fraction(num, den) + Fraction(1, 2))


def _ks_by_definition(prm, x, key, level):
    Q = 1
    for q in prm.q[:level]:
        Q *= q
    P = 1
    for p in prm.p:
        P *= p
    out = []
    for part in (0, 1):
        u = [0] * prm.n
        ndig = -(-level // prm.alpha)
        for j in range(ndig):
            Qj = 1
            for q in prm.q[j * prm.alpha:min((j + 1) * prm.alpha, level)]:
                Qj *= q
            D = [_centred(v, Qj) for v in x]
            k = [v % (Q * P) for v in key.parts[j][part]]
            u = [a + b for a, b in zip(u, _schoolbook(D, k))]
        out.append([_nearest(v, P) % Q for v in u])
    return out


def _tiny_key(prm, seed):
    rng = np.random.default_rng(seed)
    QP = prm.Q(prm.L) * prm.P
    parts = []
    for _ in range(prm.dnum(prm.L)):
        parts.append(([int(v) for v in rng.integers(0, 2 ** 62, prm.n)],
                      [int(v) for v in rng.integers(0, 2 ** 62, prm.n)]))
    # spread the key words over all of [0, QP)
    parts = [([(v * 0x9E3779B97F4A7C15 + 12345) % QP for v in b], [(v * 0xC2B2AE3D27D4EB4F + 777) % QP for v in a])
             for b, a in parts]
    return bfv.KSKey(parts)


KS_SHAPES = [
    # (L, K, alpha, level): one-prime digits; two special primes; alpha = 2 with a
    # full and with a partial (one prime left) last digit
    (2, 1, 1, 2),
    (3, 2, 1, 3),
    (4, 1, 2, 4),
    (3, 2, 2, 3),
    (3, 2, 2, 2),
]


@pytest.mark.parametrize("L,K,alpha,level", KS_SHAPES)
def test_key_switch_known_answer(L, K, alpha, level):
    prm = params.make("ks%d%d%d" % (L, K, alpha), 8, 30, L, K, alpha, 17, insecure=True)
    key = _tiny_key(prm, 100 + L * 10 + K)
    rng = np.random.default_rng(7 + level)
    Q = prm.Q(level)
    x = [int(v) % Q for v in rng.integers(0, 2 ** 62, 8) * 0x9E3779B9]
    x = [(v * 0xD6E8FEB86659FD93 + 99) % Q for v in x]
    got = bfv.key_switch(prm, x, key, level)
    want = _ks_by_definition(prm, x, key, level)
    assert list(got[0]) == want[0] and list(got[1]) == want[1]
    # the rounding is visible: floor(u/P) differs from round(u/P) somewhere
    u_floor_differs = False
    P = prm.P
    for part in (0, 1):
        u = [0] * 8
        for j in range(prm.dnum(level)):
            Qj = 1
            for q in prm.digit_primes(j, level):
                Qj *= q
            D = [_centred(v, Qj) for v in x]
            u = [a + b for a, b in zip(u, _schoolbook(D, [v % (Q * P) for v in key.parts[j][part]]))]
        u_floor_differs |= any((v // P) % Q != _nearest(v, P) % Q for v in u)
    assert u_floor_differs


def test_key_switch_digits_are_centred():
    # the same switch with digits taken in [0, Q_j) gives a different result:
    # the known answer above fixes the representative
    prm = params.make("ks212", 8, 30, 2, 1, 1, 17, insecure=True)
    key = _tiny_key(prm, 5)
    Q = prm.Q(2)
    x = [(i * 0x1F123BB5 + 3) * 0x9E3779B97F4A7C15 % Q for i in range(8)]
    got = bfv.key_switch(prm, x, key, 2)
    P = prm.P
    alt = []
    for part in (0, 1):
        u = [0] * 8
        for j in range(2):
            qj = prm.q[j]
            D = [v % qj for v in x]
            u = [a + b for a, b in zip(u, _schoolbook(D, [v % (Q * P) for v in key.parts[j][part]]))]
        alt.append([_nearest(v, P) % Q for v in u])
    assert list(got[0]) != alt[0] or list(got[1]) != alt[1]


def test_rotation_known_answer():
    # Rot(c, r) = (sigma_k c0 + KS(sigma_k c1)_0, KS(sigma_k c1)_1), k = 3^r mod 2N,
    # sigma_k(X^i) = (-1)^floor(ik/N) X^(ik mod N); one rotation alone and hoisted
    prm = params.make("rot", 8, 30, 3, 2, 2, 17, insecure=True)
    key = _tiny_key(prm, 31)
    Q = prm.Q(3)
    c0 = [(i * 0x2545F4914F6CDD1D + 17) % Q for i in range(8)]
    c1 = [(i * 0x9E3779B97F4A7C15 + 5) % Q for i in range(8)]
    ct = bfv.Ct(c0, c1, 3)
    r = 1
    k = pow(3, r, 16)

    def sigma(a):
        out = [0] * 8
        for i, v in enumerate(a):
            e = i * k
            sign = -1 if (e // 8) % 2 else 1
            out[e % 8] += sign * v
        return out

    s0, s1 = sigma(c0), sigma(c1)
    ks = _ks_by_definition(prm, [v % Q for v in s1], key, 3)
    want0 = [(a + b) % Q for a, b in zip(s0, ks[0])]
    want1 = ks[1]
    for got in (bfv.rotate(prm, ct, r, key), bfv.rotate_hoisted(prm, ct, [r], [key])[0]):
        assert list(got.c0) == want0 and list(got.c1) == want1


def test_mul_plain_known_answer():
    # Mult(c, u) multiplies by the centred lift of u mod t: a plaintext coefficient
    # m > t/2 acts as the negative integer m - t (not as m)
    prm = params.make("pm", 8, 30, 2, 1, 1, 17, insecure=True)
    Q, t = prm.Q(2), prm.t
    c0 = [(i * 0x2545F4914F6CDD1D + 1) % Q for i in range(8)]
    c1 = [(i * 0x9E3779B97F4A7C15 + 2) % Q for i in range(8)]
    m = [16, 0, 9, 3, 8, 12, 1, 15]          # 16, 9, 12, 15 > t/2
    got = bfv.mul_plain(prm, bfv.Ct(c0, c1, 2), m)
    lifted = [v - t if 2 * v > t else v for v in m]
    assert lifted[0] == -1 and lifted[2] == -8
    assert list(got.c0) == [v % Q for v in _schoolbook(c0, lifted)]
    assert list(got.c1) == [v % Q for v in _schoolbook(c1, lifted)]
    uncentred = [v % Q for v in _schoolbook(c0, m)]
    assert list(got.c0) != uncentred


def test_modswitch_known_answer_every_coefficient():
    # c' = nearest integer to c / q_l, mod Q_{l-1}, on every coefficient of both parts
    prm = params.make("ms", 8, 30, 3, 1, 1, 17, insecure=True)
    Q = prm.Q(3)
    c0 = [(i * 0x2545F4914F6CDD1D + 11) % Q for i in range(8)]
    c1 = [(i * 0x9E3779B97F4A7C15 + 13) % Q for i in range(8)]
    got = bfv.modswitch(prm, bfv.Ct(c0, c1, 3))
    ql, Qn = prm.q[2], prm.Q(2)
    assert list(got.c0) == [_nearest(v, ql) % Qn for v in c0]
    assert list(got.c1) == [_nearest(v, ql) % Qn for v in c1]


def _sigma_signed(a, k):
    n = len(a)
    out = [0] * n
    for i, v in enumerate(a):
        e = i * k
        out[e % n] += -v if (e // n) % 2 else v
    return out


@pytest.mark.parametrize("level", [3, 2])
def test_deferred_moddown_conv_known_answer(level):
    # A weighted sum of rotations kept over Q_l P, times a plaintext, then one ModDown:
    #   tap(c, 0) = (P c0, P c1);  tap(c, r) = (P sigma_k(c0) + u0, u1),
    #   u_k = sum_j D_j(sigma_k(c1)) * key_r,j[k]  (D_j centred mod Q_j, schoolbook over Z);
    #   out = nearest((lift_c(m) * sum w tap) / P) mod Q_l, every coefficient of both parts.
    prm = params.make("dh", 8, 30, 3, 2, 2, 17, insecure=True)
    Q, P = prm.Q(level), prm.P
    QP = Q * P
    keys = {1: _tiny_key(prm, 41), 3: _tiny_key(prm, 43)}
    cts = []
    for c in range(2):
        c0 = [(i * 0x2545F4914F6CDD1D + 17 + 101 * c) % Q for i in range(8)]
        c1 = [(i * 0x9E3779B97F4A7C15 + 5 + 37 * c) % Q for i in range(8)]
        cts.append(bfv.Ct(c0, c1, level))
    steps = [0, 1, 3]
    w = {(0, 0): 3, (0, 1): -2, (0, 3): 5, (1, 0): -7, (1, 1): 4, (1, 3): 1}
    m = [1, 0, 16, 3, 0, 9, 1, 15]

    def tap(ct, r):
        if r == 0:
            return [(P * v) % QP for v in ct.c0], [(P * v) % QP for v in ct.c1]
        k = pow(3, r, 16)
        s0, s1 = _sigma_signed(ct.c0, k), [v % Q for v in _sigma_signed(ct.c1, k)]
        u = []
        for part in (0, 1):
            acc = [0] * 8
            for j in range(prm.dnum(level)):
                Qj = 1
                for q in prm.q[j * prm.alpha:min((j + 1) * prm.alpha, level)]:
                    Qj *= q
                D = [_centred(v, Qj) for v in s1]
                acc = [a + b for a, b in zip(acc, _schoolbook(D, [v % QP for v in keys[r].parts[j][part]]))]
            u.append(acc)
        return [(P * a + b) % QP for a, b in zip(s0, u[0])], [v % QP for v in u[1]]

    A = [[0] * 8, [0] * 8]
    for c in range(2):
        for r in steps:
            t0, t1 = tap(cts[c], r)
            A[0] = [a + w[(c, r)] * b for a, b in zip(A[0], t0)]
            A[1] = [a + w[(c, r)] * b for a, b in zip(A[1], t1)]
    lifted = [v - 17 if 2 * v > 17 else v for v in m]
    want = [[_nearest(v % QP, P) % Q for v in _schoolbook([a % QP for a in part], lifted)] for part in A]

    exts = {c: bfv.rotations_extended(prm, cts[c], steps, [None, keys[1], keys[3]]) for c in range(2)}
    terms = [exts[c][i] for c in range(2) for i in range(3)]
    ws = [w[(c, r)] for c in range(2) for r in steps]
    acc = bfv.mac_extended(prm, terms, ws, level)
    got = bfv.mod_down_ct(prm, bfv.mul_plain_extended(prm, acc, m, level), level)
    assert list(got.c0) == want[0] and list(got.c1) == want[1]
    # the single rounding is visible: ModDown per rotation before the sum gives another result
    per = []
    for c in range(2):
        rots = bfv.rotate_hoisted(prm, cts[c], [1, 3], [keys[1], keys[3]])
        per += [cts[c]] + rots
    alt = bfv.mul_plain(prm, bfv.mac(prm, per, ws), m)
    assert list(alt.c0) != want[0] or list(alt.c1) != want[1]


def test_mod_down_is_exact_on_multiples_of_p():
    prm = params.make("md", 8, 30, 3, 2, 1, 17, insecure=True)
    Q, P = prm.Q(3), prm.P
    x = [(i * 0x9E3779B97F4A7C15 + 3) % Q for i in range(8)]
    assert bfv.mod_down(prm, [(P * v) % (Q * P) for v in x], 3) == x
    # and rounds to nearest: P x + y with |y| < P/2 maps to x
    ys = [P // 2 - 1, -(P // 2) + 1, 1, -1, 0, 5, P // 3, -(P // 3)]
    assert bfv.mod_down(prm, [(P * v + y) % (Q * P) for v, y in zip(x, ys)], 3) == x


def test_rotate_sum_known_answer():
    # sum_{r < 8} Rot(c, r) as baby steps {0,1,2,3} then giant steps {0,4}, each round's taps
    # kept over Q P (by definition, schoolbook) and rounded once; and the library's step list
    prm = params.make("rs", 8, 30, 3, 2, 2, 17, insecure=True)
    assert bfv.rotate_sum_steps(8) == [[1, 2, 3], [4]]
    assert bfv.rotate_sum_steps(2) == [[1], []]
    assert bfv.rotate_sum_steps(256) == [list(range(1, 16)), [16 * j for j in range(1, 16)]]
    keys = {r: _tiny_key(prm, 60 + r) for r in (1, 2, 3, 4)}
    level = 3
    Q, P = prm.Q(level), prm.P
    QP = Q * P
    c0 = [(i * 0x2545F4914F6CDD1D + 7) % Q for i in range(8)]
    c1 = [(i * 0x9E3779B97F4A7C15 + 9) % Q for i in range(8)]

    def round_(c0, c1, steps):
        A0 = [(P * v) % QP for v in c0]
        A1 = [(P * v) % QP for v in c1]
        for r in steps:
            k = pow(3, r, 16)
            s0, s1 = _sigma_signed(c0, k), [v % Q for v in _sigma_signed(c1, k)]
            for part, acc in ((0, A0), (1, A1)):
                u = [0] * 8
                for j in range(prm.dnum(level)):
                    Qj = 1
                    for q in prm.q[j * prm.alpha:min((j + 1) * prm.alpha, level)]:
                        Qj *= q
                    D = [_centred(v, Qj) for v in s1]
                    u = [a + b for a, b in zip(u, _schoolbook(D, [v % QP for v in keys[r].parts[j][part]]))]
                if part == 0:
                    u = [a + P * b for a, b in zip(u, s0)]
                for i in range(8):
                    acc[i] += u[i]
        return [_nearest(v % QP, P) % Q for v in A0], [_nearest(v % QP, P) % Q for v in A1]

    w0, w1 = round_(c0, c1, [1, 2, 3])
    w0, w1 = round_(w0, w1, [4])
    got = bfv.rotate_sum(prm, bfv.Ct(c0, c1, level), 8, keys)
    assert list(got.c0) == w0 and list(got.c1) == w1


def test_deferred_relinearisation_identity(cx):
    # relinearising after a weighted sum of unrelinearised squares (and a modulus switch of all
    # three parts) decrypts to the same slots as squaring, relinearising and summing:
    # D = sum_i w_i u_i^2 mod t; the three-part product decrypts as d0 + d1 s + d2 s^2
    prm, t = PRM, PRM.t
    us = [_vec(prm, 40 + i) for i in range(3)]
    ws = [3, -5, 7]
    sq3 = [bfv.modswitch3(prm, bfv.square_unrelinearised(prm, cx.encrypt(u))) for u in us]
    assert sq3[0].level == prm.L - 1
    # the three-part product decrypts directly (s^2 term) before any relinearisation
    Q = prm.Q(sq3[0].level)
    s2 = ring.negacyclic_mul(cx.s, cx.s)
    ph = [(a + b + c) % Q for a, b, c in zip(sq3[0].c0, ring.negacyclic_mul(sq3[0].c1, cx.s),
                                           ring.negacyclic_mul(sq3[0].c2, s2))]
    m0 = [nt.round_div(t * x, Q) % t for x in ph]
    assert (cx.enc.decode(m0) == us[0] * us[0] % t).all()
    out = bfv.relinearize3(prm, bfv.mac3(prm, sq3, ws), cx.rk)
    want = sum(w * (u * u % t) for w, u in zip(ws, us)) % t
    assert (cx.dec(out) == want).all()


def test_modswitch3_known_answer_every_coefficient():
    # each of the three parts: nearest integer to c / q_l, mod Q_{l-1}
    prm = params.make("ms3", 8, 30, 3, 1, 1, 17, insecure=True)
    Q = prm.Q(3)
    ql = prm.q[2]
    parts = [[(i * 0x9E3779B97F4A7C15 + 13 * p) % Q for i in range(8)] for p in range(3)]
    got = bfv.modswitch3(prm, bfv.Ct3(*parts, 3))
    for p, part in enumerate((got.c0, got.c1, got.c2)):
        assert list(part) == [math.floor(Fraction(x, ql) + Fraction(1, 2)) % prm.Q(2) for x in parts[p]]
