"""Parity at the workloads' full sizes, in the configuration bench.py times:
sampled output ciphertexts against the oracle (computed one by one), and the
any-size property Dec(Eval(c)) = integer network mod t over every image."""
import numpy as np
import pytest

from oracle import bfv, network, programs

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg2_gpu():
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg2")
    g.autotune()
    ct = g.encrypt_inputs()
    return g, ct


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
    got = g.ctx.export(first)
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
        assert (got[idx] == bfv.ct_to_rns(O.prm, ref[idx])).all(), "output %d" % idx


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


def test_cfg3_full_decrypts_to_network():
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg3")
    g.autotune()
    out = g.run(g.encrypt_inputs())
    vals = g.output_values(out)
    want = network.run_mod_t("cfg3", g.inputs, g.ctx.t)
    assert (vals == want).all()


@pytest.mark.slow
def test_cfg3_full_first_layer_sampled():
    """One output channel of the first CIFAR-shaped layer (24 hoisted rotations at N = 16384,
    MAC, mask, features, square, relinearisation, modulus switch) against the oracle."""
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession("cfg3")
    ct = g.encrypt_inputs()
    first = g.layers[0](g.ek, ct, g.features[0])
    got = g.ctx.export(first[5:6])[0]
    O = programs.OracleSession("cfg3", with_galois=False)
    for r in O.plan["layers"][0]["offsets"]:
        if r:
            O.galois(r)
    cts = O.encrypt_inputs()
    ref = O.conv_hw(0, cts, outputs=[5])[5]
    assert (got == bfv.ct_to_rns(O.prm, ref)).all()
