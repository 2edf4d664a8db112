"""Parity at the workloads' full sizes, in the configuration bench.py times:
sampled output ciphertexts against the oracle (computed one by one), and the
any-size property Dec(Eval(c)) = integer network mod t over every image."""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import bfv, network, programs

from gpu_util import export_rows, oracle_rows, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    """Oracle digests of every ciphertext of a workload at full size (written by
    tests/golden/make_fullsize_digests.py from the oracle alone)."""
    path = os.path.join(GOLDEN, "%s_fullsize.json" % name)
    if not os.path.exists(path):
        pytest.skip("no oracle digests for %s" % name)
    with open(path) as f:
        return json.load(f)


def _digests(ctx, ct):
    got = export_rows(ctx, ct)
    return [hashlib.sha256(np.ascontiguousarray(got[k], dtype="<u8").tobytes()).hexdigest()
            for k in range(got.shape[0])]


def _check_every_layer(g, ct, gold):
    """Runs the session's layers from `ct`, comparing every ciphertext with the oracle's digests."""
    layers = gold["layers"]
    assert len(layers) == len(g.layers) + 1
    assert _digests(g.ctx, ct) == layers[0]["digests"], "encrypted inputs"
    for li, lay in enumerate(g.layers):
        ct = lay(g.ek, ct, g.features[li])
        want = layers[li + 1]["digests"]
        got = _digests(g.ctx, ct)
        assert ct.shape[2] == layers[li + 1]["level"]
        bad = [k for k in range(len(want)) if got[k] != want[k]]
        assert len(got) == len(want) and not bad, "layer %d: outputs %s differ from the oracle" % (li + 1, bad[:8])
    return ct


@pytest.fixture(scope="module")
def cfg2_gpu():
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg2")
    g.autotune()
    ct = g.encrypt_inputs()
    return g, ct


def test_cfg2_full_every_ciphertext_matches_oracle(cfg2_gpu):
    """Every ciphertext of every layer at full size (245 conv outputs, 100 dense outputs at the
    autotuned MAC tile, 10 dense outputs at theirs) bit-exact against the oracle's digests."""
    g, ct = cfg2_gpu
    _check_every_layer(g, ct, _golden("cfg2"))


def test_cfg2_full_decrypts_to_network(cfg2_gpu):
    g, ct = cfg2_gpu
    out = g.run(ct)
    vals = g.output_values(out)
    want = network.run_mod_t("cfg2", g.inputs, g.ctx.t)
    assert vals.shape == (8192, 10)
    assert (vals == want).all()


def test_cfg2_full_first_layer_sampled(cfg2_gpu):
    g, ct = cfg2_gpu
    first = g.layers[0](g.ek, ct, g.features[0])
    got = export_rows(g.ctx, first)
    O = programs.OracleSession("cfg2", with_galois=False)
    # outputs (o, i, j) = (0, 0, 0) (touches the zero padding) and (4, 3, 5)
    samples = [0, (4 * 7 + 3) * 7 + 5]
    need = set()
    for idx in samples:
        o, rem = divmod(idx, 49)
        i, j = divmod(rem, 7)
        for di in range(5):
            for dj in range(5):
                y, x = 2 * i + di - 1, 2 * j + dj - 1
                if 0 <= y < 16 and 0 <= x < 16:
                    need.add(y * 16 + x)
    cts = O.encrypt_inputs(sorted(need))
    gin = g.ctx.export(ct[sorted(need)[:2]])
    for k, i in enumerate(sorted(need)[:2]):
        assert (gin[k] == bfv.ct_to_rns(O.prm, cts[i])).all(), "input %d" % i
    ref = O.conv_batch(0, cts, outputs=samples)
    for idx in samples:
        assert (got[idx] == oracle_rows(O.prm, ref[idx])).all(), "output %d" % idx


def test_cfg1_full_program_parity():
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg1")
    O = programs.OracleSession("cfg1")
    ct = g.encrypt_inputs()
    out = g.run(ct)
    ref = O.run(O.encrypt_inputs())
    got = g.ctx.export(out)
    assert got.shape[0] == len(ref) == 10
    for k in range(10):
        assert (got[k] == bfv.ct_to_rns(O.prm, ref[k])).all(), "output %d" % k


def test_cfg1d_full_decrypts_to_network():
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg1d")
    out = g.run(g.encrypt_inputs())
    vals = g.output_values(out)
    want = network.run_mod_t("cfg1d", g.inputs, g.ctx.t)
    assert (vals == want).all()


@pytest.fixture(scope="module")
def cfg3_gpu():
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg3")
    g.autotune()
    return g, g.encrypt_inputs()


def test_cfg3_full_every_ciphertext_matches_oracle(cfg3_gpu):
    """Every ciphertext of the CIFAR-shaped branch at N = 16384 bit-exact against the oracle's
    digests: layer 1 (24 hoisted rotations, MAC, mask, features, square, relinearisation, modulus
    switch), layer 2 (256 hoisted rotations at five primes with a one-prime last digit, MAC, mask,
    features, square, relinearisation, modulus switch, rotate-and-sum over 128 slots) and the
    dense outputs."""
    g, ct = cfg3_gpu
    _check_every_layer(g, ct, _golden("cfg3"))


def test_cfg3_full_decrypts_to_network(cfg3_gpu):
    g, ct = cfg3_gpu
    out = g.run(ct)
    vals = g.output_values(out)
    want = network.run_mod_t("cfg3", g.inputs, g.ctx.t)
    assert (vals == want).all()


def test_cfg3_bhw_full_decrypts_to_network():
    """BHW packing at full size: 64 CIFAR-shaped images per ciphertext; every image's ten
    outputs equal its integer network mod t."""
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg3_bhw")
    out = g.run(g.encrypt_inputs())
    vals = g.output_values(out)
    want = network.run_mod_t("cfg3_bhw", g.inputs, g.ctx.t)
    assert vals.shape == (64, 10)
    assert (vals == want).all()


def test_cfg2_bi_full_decrypts_to_network():
    """The whole bi-CryptoNets model on 8192 MNIST-shaped images (plaintext branch on a side
    stream, ciphertext branch, feature integration): Dec(Eval) equals the integer network for
    every image, on five 36-bit primes."""
    torch = torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg2_bi")
    g.autotune()
    images, noise = g.plain_inputs(g.inputs)
    out = g.run_bi(g.encrypt_inputs(), images, noise, torch.cuda.Stream())
    vals = g.output_values(out)
    want = network.run_mod_t("cfg2_bi", g.inputs, g.ctx.t)
    assert vals.shape == (8192, 10)
    assert (vals == want).all()


@pytest.mark.parametrize("name", ["fc_diag", "cfg3_pool"])
def test_diag_fc_and_pooling_full_decrypt_to_network(name):
    """At N = 16384: the diagonal-method fully connected branch (144 -> 32 -> 10, 175 and 41
    hoisted rotations) and the CIFAR-shaped branch with a local sum-pooling layer."""
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession(name)
    out = g.run(g.encrypt_inputs())
    vals = g.output_values(out)
    want = network.run_mod_t(name, g.inputs, g.ctx.t)
    assert (vals == want).all()
