"""The CIFAR-shaped ciphertext branch under CKKS, the paper's scheme (section
"Experiments": CKKS with N = 2^14), driven through the library's CKKS calls.

Client-side placement: channel c of the crop holds pixel (y, x) / 255 at slot
row*y + x.  Per HW convolution (appendix "Implementation Details"): hoisted
rotations by the kernel offsets, a multiply-accumulate with the integer weights
W (real weights W / 2^wbits: the scale grows by 2^wbits), the mask of the valid
outputs encoded at scale q_level and rescaled away, the plaintext-branch features
encoded at the ciphertext's scale and added, then the square with
relinearisation and rescale.  The global sum runs after the scalar dense layer
(both linear).  The scale of every ciphertext is tracked here on the host; all
arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

import synthetic
from synthetic import workloads as W

from . import bcn


class CkksSession:
    def __init__(self, name: str, seeds=None, device: int = 0):
        import torch
        self.torch = torch
        self.name = name
        self.wl = W.WORKLOADS[name]
        assert self.wl.get("scheme") == "ckks" and self.wl["packing"] == "hw"
        self.seeds = dict(W.SEEDS if seeds is None else seeds)
        spec = W.PARAMS[self.wl["params"]]
        self.ctx = bcn.Context(spec["n"], spec["bits"], spec["L"], spec["K"], spec["alpha"], 0, device, ckks=True)
        self.n = spec["n"]
        self.inputs = W.make_inputs(name, self.seeds)
        self.s = synthetic.ternary_secret(self.seeds["keys"], self.n)
        self.sk = self.ctx.secret_key(self.s)
        self.ek = self.ctx.eval_keys()
        self._geometry()
        self._keygen()

    # ------------------------------------------------------------ layout
    def _geometry(self):
        wl, n = self.wl, self.n
        row = wl["crop"][1]
        shapes = W.layer_shapes(self.name)
        ps = 1
        self.layers = []
        moved = 0
        steps = set()
        for li, lay in enumerate(wl["layers"]):
            info = dict(lay, li=li)
            if lay["kind"] == "conv":
                offs = [ps * (row * di + dj) for di in range(lay["k"]) for dj in range(lay["k"])]
                info["offsets"] = offs
                steps.update(o for o in offs if o)
                ps *= lay["stride"]
                _, oh, ow = shapes[li][1]
                info["out_slots"] = [ps * (row * i + j) for i in range(oh) for j in range(ow)]
                mask = np.zeros((1, n // 2))
                mask[0, info["out_slots"]] = 1.0
                info["mask"] = self.torch.from_numpy(mask).cuda()
                if lay.get("sum"):
                    last = max(info["out_slots"])
                    moved = 1
                    while moved < last + 1:
                        moved *= 2
                    steps.update(bcn.rotate_sum_steps(moved))
            else:
                info["sum_span"] = moved
                moved = 0
            self.layers.append(info)
        self.steps = sorted(steps)

    def _keygen(self):
        moduli = self.ctx.q + self.ctx.p_primes
        d = self.ctx.dnum()

        def rnd(key_id):
            a = np.stack([synthetic.uniform_residues(self.seeds["keys"], "ksk_a", (key_id, j), moduli, self.n)
                          for j in range(d)])
            e = np.stack([synthetic.gaussian_error(self.seeds["keys"], "ksk_e", (key_id, j), self.n)
                          for j in range(d)])
            return a, e
        self.ctx.keygen(self.sk, self.ek, bcn.BCN_KEY_RELIN, 0, *rnd(W.RELIN_KEY_ID))
        for r in self.steps:
            self.ctx.keygen(self.sk, self.ek, bcn.BCN_KEY_ROTATION, r, *rnd(W.rotation_key_id(r)))

    # ------------------------------------------------------------ client
    def input_slots(self):
        y0, size = self.wl["crop"]
        crop = self.inputs["images"][0, :, y0:y0 + size, y0:y0 + size].astype(np.float64) / 255.0
        out = np.zeros((crop.shape[0], self.n // 2))
        out[:, :size * size] = crop.reshape(crop.shape[0], -1)
        return out

    def encrypt_inputs(self):
        slots = self.input_slots()
        q = self.ctx.q
        a = np.stack([synthetic.uniform_residues(self.seeds["enc"], "enc_a", (i,), q, self.n)
                      for i in range(len(slots))])
        e = np.stack([synthetic.gaussian_error(self.seeds["enc"], "enc_e", (i,), self.n) for i in range(len(slots))])
        return self.ctx.ckks_encrypt(self.sk, slots, 2.0 ** self.wl["scale_bits"], a, e)

    def output_values(self, ct, scale):
        return self.ctx.ckks_decrypt(self.sk, ct, scale)[:, 0][None, :]

    # ------------------------------------------------------------ server
    def feature_slots(self, li):
        info = self.layers[li]
        f = np.asarray(self.inputs["features"][li], dtype=np.float64)    # [C][oh][ow]
        out = np.zeros((f.shape[0], self.n // 2))
        out[:, info["out_slots"]] = f.reshape(f.shape[0], -1)
        return self.torch.from_numpy(out).cuda()

    def run(self, ct):
        """Evaluates every layer; returns (output ciphertexts, their scale)."""
        ctx, ek = self.ctx, self.ek
        wb = 2.0 ** self.wl["wbits"]
        scale = 2.0 ** self.wl["scale_bits"]
        level = ct.shape[2]
        for info in self.layers:
            w = self.inputs["weights"][info["li"]]
            if info["kind"] == "conv":
                offs = info["offsets"]
                nz = [o for o in offs if o]
                rot = ctx.rotate(ek, ct, nz)                           # [C][len(nz)][2][level][N]
                taps = self.torch.cat([ct[:, None], rot], dim=1)       # tap 0 = offset 0
                order = [0] + [1 + nz.index(o) for o in offs if o]
                C = ct.shape[0]
                k2 = len(offs)
                Wm = np.zeros((w.shape[0], C * k2), dtype=np.int32)
                for t, o in enumerate(offs):
                    tap = 0 if o == 0 else 1 + nz.index(o)
                    Wm[:, np.arange(C) * k2 + tap] = w[:, :, t // info["k"], t % info["k"]]
                ct = ctx.mac(taps.reshape(C * k2, 2, level, self.n).contiguous(), Wm)
                scale *= wb
                ql = float(ctx.q[level - 1])
                mask = ctx.ckks_encode(info["mask"], level, ql, ntt=True)
                ct = ctx.modswitch(ctx.ckks_mul_plain(ct, mask[0]))  # scale * ql / ql
                level -= 1
                if info.get("features"):
                    ctx.ckks_add_plain(ct, ctx.ckks_encode(self.feature_slots(info["li"]), level, scale))
                if info.get("square"):
                    ct = ctx.ckks_square_relin_rescale(ek, ct)
                    scale = scale * scale / float(ctx.q[level - 1])
                    level -= 1
            else:
                ct = ctx.mac(ct, w)
                scale *= wb
                if info["sum_span"]:
                    ctx.rotate_sum(ek, ct, info["sum_span"])
        return ct, scale
