"""Drives a synthetic workload through the HIP library: keys, encryption,
layer-by-layer evaluation of the ciphertext branch, decryption.

Slot layouts (client-side data placement):
  batch packing: one ciphertext per crop pixel (c, y, x); slot b = image b.
  HW packing: one ciphertext per channel; crop pixel (y, x) at slot row*y + x
  of slot row 0, with row the crop width.
  BHW packing: HW packing of `batch` images per ciphertext, image b's block
  starting at slot image_base(b, block, N).
Every homomorphic step is a call into libbcn.
"""
from __future__ import annotations

import numpy as np

import synthetic
from synthetic import workloads as W

from . import bcn


def layer_descs(name: str):
    """Layer descriptions of a workload's ciphertext branch (dicts for bcn.Layer)."""
    wl = W.WORKLOADS[name]
    shapes = W.layer_shapes(name)
    hw = wl["packing"] in ("hw", "bhw")
    bhw = dict(batch=wl["batch"], block=wl["block"]) if wl["packing"] == "bhw" else {}
    row = wl["crop"][1]
    ps = 1
    spatial = True
    moved_span = 0
    out = []
    for li, lay in enumerate(wl["layers"]):
        (inp, outp) = shapes[li]
        d = dict(square=lay.get("square", False), modswitch=lay.get("square", False), batch=wl["batch"])
        if lay["kind"] == "pool":
            c, h, w = inp
            d.update(kind=bcn.BCN_POOL, packing=bcn.BCN_PACK_HW, in_c=c, in_h=h, in_w=w, out_c=c, k=lay["k"],
                     stride=lay["stride"], pad=0, row=row, pos_stride=ps, **bhw)
            ps *= lay["stride"]
        elif lay["kind"] == "dense" and lay.get("method") == "diag":
            # diagonal method: inputs at slots 0..n1-1 (the crop, or the previous diagonal layer)
            if li == 0:
                c, h, w = wl["image"][0], wl["crop"][1], wl["crop"][1]
            else:
                c, h, w = 1, 1, out[-1]["out_c"]
            d.update(kind=bcn.BCN_DENSE, packing=bcn.BCN_PACK_HW, method=bcn.BCN_DENSE_DIAGONAL, in_c=c, in_h=h,
                     in_w=w, out_c=lay["out"], row=row, pos_stride=1)
            spatial = False
        elif lay["kind"] == "conv":
            c, h, w = inp
            # with sum_after_dense the global sum runs after the next (scalar) dense layer
            conv_sum = lay.get("sum", False) and not (hw and wl.get("sum_after_dense"))
            d.update(kind=bcn.BCN_CONV2D, packing=bcn.BCN_PACK_HW if hw else bcn.BCN_PACK_BATCH,
                     in_c=c, in_h=h, in_w=w, out_c=lay["out"], k=lay["k"], stride=lay["stride"],
                     pad=lay["pad"], row=row, pos_stride=ps, features=lay.get("features", False),
                     sum=conv_sum)
            if hw:
                d.update(bhw)
            if hw:
                ps *= lay["stride"]
                if lay.get("sum"):
                    spatial = False
                    if not conv_sum:
                        oh, ow = outp[1], outp[2]
                        last = ps * (row * (oh - 1) + ow - 1)
                        moved_span = 1
                        while moved_span < last + 1:
                            moved_span *= 2
        else:
            if hw and spatial:
                c, h, w = shapes[li - 1][1]
                d.update(kind=bcn.BCN_DENSE, packing=bcn.BCN_PACK_HW, in_c=c, in_h=h, in_w=w,
                         out_c=lay["out"], row=row, pos_stride=ps, **bhw)
                spatial = False
            else:
                d.update(kind=bcn.BCN_DENSE, packing=bcn.BCN_PACK_BATCH, in_c=inp[0], in_h=1, in_w=1,
                         out_c=lay["out"], batch=max(1, wl["batch"]), sum=moved_span,
                         features=bool(lay.get("features")))
                moved_span = 0
        # a square followed by a scalar dense layer (slot batching, or the dense layer a global sum
        # was moved after) leaves its products unrelinearised; the dense layer sums over the three
        # parts and relinearises its outputs
        if (out and out[-1].get("square") and not out[-1].get("sum") and d["kind"] == bcn.BCN_DENSE
                and d["packing"] == bcn.BCN_PACK_BATCH):
            out[-1]["defer_relin"] = True
            d["in_parts"] = 3
        out.append(d)
    return out


class GpuSession:
    """Keys, encryptions and evaluation of one workload on the GPU.

    The model part (context, keys, prepared layers) is shared by every request
    of the workload; request_inputs() / encrypt_request() give independent
    requests their own images, features and encryption randomness.
    """

    def __init__(self, name: str, seeds=None, device: int = 0):
        import torch
        self.torch = torch
        self.name = name
        self.wl = W.WORKLOADS[name]
        self.seeds = dict(W.SEEDS if seeds is None else seeds)
        spec = W.PARAMS[self.wl["params"]]
        self.ctx = bcn.Context(spec["n"], spec["bits"], spec["L"], spec["K"], spec["alpha"], spec["t"], device)
        n = spec["n"]
        self.n = n
        self.s = synthetic.ternary_secret(self.seeds["keys"], n)
        self.sk = self.ctx.secret_key(self.s)
        self.ek = self.ctx.eval_keys()
        self.inputs = W.make_inputs(name, self.seeds)
        self.plain = None
        if "plain" in self.inputs:
            from .plain_branch import PlainBranch
            self.plain = PlainBranch(name, self.inputs["plain"])
            self.inputs = self.with_plain(self.inputs)
        self.descs = layer_descs(name)
        for d, w in zip(self.descs, self.inputs["weights"]):
            d["weights"] = w
        self.layers = []
        level = self.ctx.L
        for d in self.descs:
            lay = self.ctx.layer(d, level)
            self.layers.append(lay)
            level = lay.level_out
        self.features = self.request_features(self.inputs)
        self.steps = sorted({s for lay in self.layers for s in lay.steps})
        self._keygen()

    def autotune(self) -> str:
        """Measured choice of transform shape and MAC tile sizes (results unchanged)."""
        report = self.ctx.autotune()
        for lay in self.layers:
            report += self.ctx.autotune_layer(lay)
        return report

    def key_randomness(self, key_id: int):
        moduli = self.ctx.q + self.ctx.p_primes
        d = self.ctx.dnum()
        a = np.stack([synthetic.uniform_residues(self.seeds["keys"], "ksk_a", (key_id, j), moduli, self.n)
                      for j in range(d)])
        e = np.stack([synthetic.gaussian_error(self.seeds["keys"], "ksk_e", (key_id, j), self.n) for j in range(d)])
        return a, e

    def _keygen(self):
        a, e = self.key_randomness(W.RELIN_KEY_ID)
        self.ctx.keygen(self.sk, self.ek, bcn.BCN_KEY_RELIN, 0, a, e)
        for r in self.steps:
            a, e = self.key_randomness(W.rotation_key_id(r))
            self.ctx.keygen(self.sk, self.ek, bcn.BCN_KEY_ROTATION, r, a, e)

    # ------------------------------------------------------------ plaintext side
    def plain_inputs(self, inputs):
        """Device images and perturbation of a request (for the plaintext branch)."""
        torch = self.torch
        return (torch.from_numpy(np.ascontiguousarray(inputs["images"])).cuda(),
                torch.from_numpy(np.ascontiguousarray(inputs["plain"]["noise"])).cuda())

    def with_plain(self, inputs):
        """inputs with the plaintext side's FP32 outputs (computed on the GPU) in the feature
        slots it feeds (host copies: the integer network reads them too)."""
        outs = self.plain(*self.plain_inputs(inputs))
        return W.with_plain_features(inputs, self.name, {k: v.cpu().numpy() for k, v in outs.items()})

    # ------------------------------------------------------------ inputs
    def input_slots(self) -> np.ndarray:
        wl, n = self.wl, self.n
        y0, size = wl["crop"]
        crop = self.inputs["images"][:, :, y0:y0 + size, y0:y0 + size].astype(np.int64)
        if wl["packing"] == "batch":
            b = crop.shape[0]
            flat = crop.reshape(b, -1).T
            out = np.zeros((flat.shape[0], n), dtype=np.int64)
            out[:, :b] = flat
            return out
        c = crop.shape[1]
        out = np.zeros((c, n), dtype=np.int64)
        for b, base in enumerate(self.image_bases()):
            for ch in range(c):
                out[ch, base:base + size * size] = crop[b, ch].reshape(-1)
        return out

    def image_bases(self):
        """First slot of each image's block (HW: one image at slot 0)."""
        if self.wl["packing"] != "bhw":
            return [0]
        return [W.image_base(b, self.wl["block"], self.n) for b in range(self.wl["batch"])]

    def encryption_randomness(self, indices, level=None):
        level = self.ctx.L if level is None else level
        q = self.ctx.q[:level]
        a = np.stack([synthetic.uniform_residues(self.seeds["enc"], "enc_a", (i,), q, self.n) for i in indices])
        e = np.stack([synthetic.gaussian_error(self.seeds["enc"], "enc_e", (i,), self.n) for i in indices])
        return a, e

    def encrypt_inputs(self):
        slots = self.input_slots()
        a, e = self.encryption_randomness(range(len(slots)))
        return self.ctx.encrypt(self.sk, slots, a, e)

    # ------------------------------------------------------------ evaluation
    def run(self, ct, upto=None):
        """Evaluates the layers (all, or the first ``upto``); returns the last output batch."""
        for li, lay in enumerate(self.layers[:upto]):
            ct = lay(self.ek, ct, self.features[li])
        return ct

    def run_bi(self, ct, images, noise, side_stream):
        """The whole bi-CryptoNets model for one request: the plaintext branch on `side_stream`
        in parallel with the ciphertext branch on the current stream.  Ciphertext layer 1 waits
        for z1 only; the integration layers wait for u1, u2.  Returns the output ciphertexts."""
        torch = self.torch
        cur = torch.cuda.current_stream()
        side_stream.wait_stream(cur)
        with torch.cuda.stream(side_stream):
            h1, z1 = self.plain.first(images, noise)
            ev1 = torch.cuda.Event()
            ev1.record(side_stream)
            u1, u2 = self.plain.rest(h1)
            ev2 = torch.cuda.Event()
            ev2.record(side_stream)
        feats = {}
        for li, key in W.plain_feature_layers(self.name).items():
            feats[li] = key
        out = {"z1": z1.reshape(z1.shape[0], -1), "u1": u1, "u2": u2}
        for li, lay in enumerate(self.layers):
            f = self.features[li]
            if li in feats:
                cur.wait_event(ev1 if feats[li] == "z1" else ev2)
                f = out[feats[li]]
            ct = lay(self.ek, ct, f)
        # the side stream's tensors were used on this stream
        for t in (z1, u1, u2):
            t.record_stream(cur)
        return ct

    # ------------------------------------------------------------ independent requests
    def request_seeds(self, rid: int) -> dict:
        """Seeds of request rid: the model's keys and weights, the request's own data."""
        s = dict(self.seeds)
        s.update(images=100000 + rid, features=200000 + rid, enc=300000 + rid)
        return s

    def request_inputs(self, rid: int):
        inputs = W.make_inputs(self.name, self.request_seeds(rid))
        return self.with_plain(inputs) if self.plain is not None else inputs

    def request_slots(self, inputs) -> np.ndarray:
        saved = self.inputs
        self.inputs = inputs
        try:
            return self.input_slots()
        finally:
            self.inputs = saved

    def request_features(self, inputs):
        """Device feature tensors of one request, per layer (None where a layer has none)."""
        out = []
        for f in inputs["features"]:
            if f is None:
                out.append(None)
            elif self.wl["packing"] == "batch":
                out.append(self.torch.from_numpy(np.ascontiguousarray(f.reshape(f.shape[0], -1))).cuda())
            elif self.wl["packing"] == "bhw":
                # per image [batch][C][h][w] -> the layer's [C][batch][h][w]
                out.append(self.torch.from_numpy(np.ascontiguousarray(f.transpose(1, 0, 2, 3))).cuda())
            else:
                out.append(self.torch.from_numpy(np.ascontiguousarray(f)).cuda())
        return out

    def encrypt_request(self, rid: int, inputs=None):
        inputs = self.request_inputs(rid) if inputs is None else inputs
        slots = self.request_slots(inputs)
        seeds = self.request_seeds(rid)
        q = self.ctx.q
        a = np.stack([synthetic.uniform_residues(seeds["enc"], "enc_a", (i,), q, self.n) for i in range(len(slots))])
        e = np.stack([synthetic.gaussian_error(seeds["enc"], "enc_e", (i,), self.n) for i in range(len(slots))])
        return self.ctx.encrypt(self.sk, slots, a, e)

    def run_batch(self, ct, features, n_requests):
        """All layers over n_requests stacked requests (features: per layer, stacked or None)."""
        for li, lay in enumerate(self.layers):
            ct = lay.batch(self.ek, ct, n_requests, features[li])
        return ct

    def n_inputs(self) -> int:
        return self.layers[0].n_in

    def n_outputs(self) -> int:
        return self.layers[-1].n_out

    def output_values(self, ct) -> np.ndarray:
        vals = self.ctx.decrypt(self.sk, ct)
        last = self.wl["layers"][-1]
        if last.get("method") == "diag":
            return vals[0, :last["out"]][None, :]
        if self.wl["packing"] == "batch":
            return vals[:, :self.wl["batch"]].T
        return vals[:, self.image_bases()].T
