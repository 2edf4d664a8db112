"""Pins of the oracle's network and homomorphic programs: Dec(Eval(c)) equals
the integer-quantised network mod t (the spec property check), the
network against brute force, and the workload-1 noise floor."""
import numpy as np
import pytest

from oracle import bfv, network, programs
from synthetic import workloads as W


def test_quantise_fp32_rounding():
    f = np.array([0.0625, 0.1875, -0.0625, -0.1875, 15.9, -15.9, 100.0, 1e-8], dtype=np.float32)
    # 8f = 0.5, 1.5, -0.5, -1.5 round half to even; clamp at +-127
    assert network.quantise(f).tolist() == [0, 2, 0, -2, 127, -127, 127, 0]


def test_conv_and_dense_against_brute_force():
    rng = np.random.default_rng(0)
    x = rng.integers(0, 256, (2, 9, 9))
    w = rng.integers(-7, 8, (3, 2, 3, 3))
    for stride, pad in [(1, 0), (2, 1), (2, 0)]:
        out = network.conv2d(x.astype(object), w, stride, pad)
        H = 9
        oh = (H + 2 * pad - 3) // stride + 1
        for o in range(3):
            for i in range(oh):
                for j in range(oh):
                    acc = 0
                    for c in range(2):
                        for di in range(3):
                            for dj in range(3):
                                y, xx = stride * i + di - pad, stride * j + dj - pad
                                if 0 <= y < H and 0 <= xx < H:
                                    acc += int(x[c, y, xx]) * int(w[o, c, di, dj])
                    assert out[o, i, j] == acc
    v = rng.integers(-100, 100, 17)
    wd = rng.integers(-15, 16, (4, 17))
    assert network.dense(v.astype(object), wd).tolist() == [sum(int(a) * int(b) for a, b in zip(row, v)) for row in wd]


@pytest.mark.parametrize("name", ["cfg1", "cfg2_small", "cfg3"])
def test_mod_t_network_equals_exact_network(name):
    inp = W.make_inputs(name)
    t = 65537
    imgs = [0, 1, 2] if W.WORKLOADS[name]["batch"] > 1 else None
    exact = network.run(name, inp, imgs)
    red = network.run_mod_t(name, inp, t, imgs)
    ex = np.vectorize(lambda z: int(z) % t)(exact)
    assert (np.where(2 * ex > t, ex - t, ex) == red).all()


@pytest.mark.parametrize("name", ["cfg1_small", "cfg2_small", "cfg3_small", "cfg3_bhw_small"])
def test_dec_eval_equals_network(name):
    S = programs.OracleSession(name)
    out = S.run(S.encrypt_inputs())
    got = S.output_values(out)
    want = network.run_mod_t(name, S.inputs, S.prm.t)
    assert got.shape == want.shape
    assert (got == want).all()


def test_workload1_first_layer_and_noise_floor():
    S = programs.OracleSession("cfg1")
    cts = S.encrypt_inputs()
    li = 0
    info = S.plan["layers"][li]
    # linear part of layer 1 (rotations, scalar MAC, mask) decrypts to the conv
    w = S.inputs["weights"][li]
    rots = bfv.rotate_hoisted(S.prm, cts[0], [o for o in info["offsets"] if o],
                              [S.gk[o] for o in info["offsets"] if o])
    table = dict(zip([o for o in info["offsets"] if o], rots))
    table[0] = cts[0]
    mask = S.enc.encode(S.mask_slots(li))
    conv = network.first_layer_linear("cfg1", S.inputs, t=S.prm.t)[0]
    A = bfv.mac(S.prm, [table[o] for o in info["offsets"]], [int(x) for x in w[0, 0].reshape(-1)])
    A = bfv.mul_plain(S.prm, A, mask)
    slots = S.decrypt_slots(A)
    want = np.zeros(S.prm.n, dtype=np.int64)
    want[info["out_slots"]] = conv[0].reshape(-1)
    t = S.prm.t
    want = np.where(2 * (want % t) > t, want % t - t, want % t)
    assert (slots == want).all()
    # after the square the 60-bit modulus has no budget left: decryption fails
    sq = bfv.square(S.prm, A, S.rk)
    m_exp = S.enc.encode(want * want % t)
    assert bfv.noise_budget(S.prm, S.s, sq, m_exp) <= 0
