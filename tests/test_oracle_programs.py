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


@pytest.mark.parametrize("name", ["cfg1_small", "cfg2_small", "cfg3_small", "cfg3_bhw_small", "cfg2_bi_small", "fc_diag_small", "cfg3_pool_small"])
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


def test_plain_reference_conv_is_the_integer_conv():
    """The plaintext-side reference's convolution equals the integer network's convolution
    (brute-force definition) on integer inputs, bias zero."""
    from oracle import plain
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (2, 3, 11, 11))
    w = rng.integers(-7, 8, (4, 3, 5, 5))
    for stride, pad in [(1, 0), (2, 1)]:
        got = plain._conv(x.astype(np.float64), w.astype(np.float64), None, stride, pad)
        want = np.stack([network.conv2d(x[b].astype(object), w, stride, pad) for b in range(2)]).astype(np.float64)
        assert (got == want).all()


def test_plain_branch_fp32_matches_fp64_reference():
    """The FP32 plaintext side (torch ops, here on the CPU) against the FP64 reference:
    resize = centre crop aligned with ciphertext layer 1, CRot, plaintext neurons."""
    torch = pytest.importorskip("torch")
    from oracle import plain
    from paper_2402_01296_amd import plain_branch
    name = "cfg2_bi_small"
    inp = W.make_inputs(name)
    ref = plain.run(name, inp)

    class OnCpu(plain_branch.PlainBranch):
        def __init__(self, nm, params):
            self.torch = torch
            self.wl = W.WORKLOADS[nm]
            self.p = self.wl["plain"]
            self.sp = W.plain_shapes(nm)
            self.w = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32))
                      for k, v in params.items() if k != "noise"}

    out = OnCpu(name, inp["plain"])(torch.from_numpy(inp["images"]), torch.from_numpy(inp["plain"]["noise"]))
    for k in ("z1", "u1", "u2"):
        a = out[k].numpy().astype(np.float64)
        assert a.shape == ref[k].shape
        assert np.abs(a - ref[k]).max() <= 1e-5 * max(1.0, np.abs(ref[k]).max()), k
    # the centre crop of layer 1 lines up with ciphertext layer 1's outputs: output (i, j) of both
    # convolutions is centred on the same image pixel
    sp = W.plain_shapes(name)
    wl = W.WORKLOADS[name]
    lay, p = wl["layers"][0], wl["plain"]
    y0 = wl["crop"][0]
    for i in (0, sp["out_hw"] - 1):
        c_cipher = y0 + lay["stride"] * i - lay["pad"] + lay["k"] // 2
        c_plain = p["stride1"] * (i + sp["resize"]) - p["pad1"] + p["k1"] // 2
        assert c_cipher == c_plain
