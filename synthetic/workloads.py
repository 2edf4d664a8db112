"""Workload recipes: shapes, crops, value ranges and seeds of the synthetic inputs.

Descriptive data only (no scheme arithmetic).  The sensitive segment is the
central crop of each image (the paper's experiments encrypt the central part
of the image; section "Our bi-CryptoNets", Experiments section).  Images stand
in for MNIST (28x28x1) and CIFAR (32x32x3): uniform uint8 of the same shape,
never dataset items.

Layer entries:
  conv  : out channels, kernel k, stride, pad, weight bound, features?, square?
  pool  : local sum pooling, window k, stride (no weights; appendix "Implementation
          Details", pooling layer), channel by channel
  dense : out units, weight bound, square?; method "diag" (HW packing, input
          values at slots 0..n1-1 of each channel) uses the diagonal method of the
          appendix's fully connected layer: n1 + n2 - 1 rotations of the input (steps
          1 - n2 .. n1 - 1), each multiplied by one weight vector, summed; outputs at
          slots 0..n2-1
  For 'hw' packing a conv output (y, x) lives at the slot of its top-left tap,
  so a strided conv leaves its outputs spread at the stride; 'sum' on a layer
  asks for a global sum of each output map (sum pooling over all positions).
  'bhw' packing (appendix "Implementation Details", BHW packing) puts `batch`
  images' h x w crops into one ciphertext per channel: image b's block starts
  at slot image_base(b, block, N) and is laid out as in 'hw' packing.

A workload with a 'plain' entry is the whole bi-CryptoNets model (section "Our
bi-CryptoNets"): an FP32 plaintext branch on the image with the sensitive crop
zeroed and the rest perturbed, whose layer-1 map is resized (centre crop) and
channel-rotated (1x1 mix) into the features of ciphertext layer 1 (features =
"plain"), and a two-layer feature integration whose ciphertext neurons are the
last two dense layers (integration 1, 2): their plaintext-branch terms
W_p1 x_p + b_1 and W_p2 x_p^<1> + b_2 enter as features, x_p^<1> being the
plaintext neurons (section "The feature integration").
"""
from __future__ import annotations

SEEDS = dict(keys=1, enc=2, weights=3, images=4, features=5)

# Parameter sets: ring degree, prime size, ciphertext primes L, special primes
# K, primes per key-switching digit, plaintext modulus t.
PARAMS = {
    # the three workloads
    "cfg1": dict(n=4096, bits=30, L=2, K=1, alpha=1, t=65537),
    "cfg2": dict(n=8192, bits=36, L=4, K=2, alpha=2, t=1032193),
    "cfg3": dict(n=16384, bits=40, L=6, K=2, alpha=2, t=65537),
    # workload 1 with five primes so that its output still decrypts (insecure)
    "cfg1d": dict(n=4096, bits=30, L=5, K=1, alpha=1, t=65537, insecure=True),
    # reduced sizes for tests the oracle finishes in seconds (insecure)
    "t1k": dict(n=1024, bits=36, L=3, K=1, alpha=1, t=65537, insecure=True),
    "t2k": dict(n=2048, bits=40, L=4, K=2, alpha=2, t=65537, insecure=True),
    "t1k5": dict(n=1024, bits=30, L=5, K=1, alpha=1, t=65537, insecure=True),
    "t2k3": dict(n=2048, bits=40, L=6, K=2, alpha=2, t=65537, insecure=True),
    "t4k": dict(n=4096, bits=36, L=4, K=1, alpha=1, t=40961, insecure=True),
    # the MNIST-shaped branch plus the feature-integration layers: one more prime of noise budget
    "cfg2i": dict(n=8192, bits=36, L=5, K=1, alpha=1, t=1032193),
}

# key ids of the key-switching-key randomness streams
RELIN_KEY_ID = 0


def rotation_key_id(step: int) -> int:
    return 1000 + step

WORKLOADS = {
    # one 28x28 image, HW packing, central 12x12 crop
    # (two 30-bit limbs leave no noise budget after the square: the output does not decrypt)
    "cfg1": dict(params="cfg1", packing="hw", batch=1, image=(1, 28, 28), crop=(8, 12), decrypts=False,
                 layers=[dict(kind="conv", out=5, k=5, stride=2, pad=0, bound=7, features=False, square=True),
                         dict(kind="dense", out=10, bound=7, square=False)]),
    # same network on five limbs, so the output still decrypts (insecure, test only)
    "cfg1d": dict(params="cfg1d", packing="hw", batch=1, image=(1, 28, 28), crop=(8, 12),
                  layers=[dict(kind="conv", out=5, k=5, stride=2, pad=0, bound=7, features=False, square=True),
                          dict(kind="dense", out=10, bound=7, square=False)]),
    # 8192 28x28 images, one image per slot, central 16x16 crop
    "cfg2": dict(params="cfg2", packing="batch", batch=8192, image=(1, 28, 28), crop=(6, 16),
                 layers=[dict(kind="conv", out=5, k=5, stride=2, pad=1, bound=15, features=True, square=True),
                         dict(kind="dense", out=100, bound=15, square=True),
                         dict(kind="dense", out=10, bound=15, square=False)]),
    # one 32x32x3 image, HW packing (one channel per ciphertext), central 16x16 crop.
    # sum_after_dense: the HE program applies the dense layer's scalar weights to the 64 channel
    # ciphertexts first and rotates-and-sums the 10 results (10 x 8 rotations instead of 64 x 8);
    # global sum and dense are linear, so the network is the same
    "cfg3": dict(params="cfg3", packing="hw", batch=1, image=(3, 32, 32), crop=(8, 16), sum_after_dense=True,
                 layers=[dict(kind="conv", out=32, k=3, stride=1, pad=0, bound=31, features=True, square=True),
                         dict(kind="conv", out=64, k=3, stride=2, pad=0, bound=31, features=True, square=True,
                              sum=True),
                         dict(kind="dense", out=10, bound=31, square=False)]),
    # reduced variants the oracle finishes in seconds (same layer kinds)
    "cfg2_small": dict(params="t1k", packing="batch", batch=1024, image=(1, 28, 28), crop=(6, 16),
                       layers=[dict(kind="conv", out=2, k=5, stride=2, pad=1, bound=15, features=True, square=True),
                               dict(kind="dense", out=7, bound=15, square=True),
                               dict(kind="dense", out=3, bound=15, square=False)]),
    "cfg1_small": dict(params="t1k5", packing="hw", batch=1, image=(1, 28, 28), crop=(8, 12),
                       layers=[dict(kind="conv", out=2, k=5, stride=2, pad=0, bound=7, features=False, square=True),
                               dict(kind="dense", out=3, bound=7, square=False)]),
    # CIFAR-shaped branch with BHW packing: 64 images per ciphertext, one 256-slot block per image
    "cfg3_bhw": dict(params="cfg3", packing="bhw", batch=64, block=256, image=(3, 32, 32), crop=(8, 16),
                     sum_after_dense=True,
                     layers=[dict(kind="conv", out=32, k=3, stride=1, pad=0, bound=31, features=True, square=True),
                             dict(kind="conv", out=64, k=3, stride=2, pad=0, bound=31, features=True, square=True,
                                  sum=True),
                             dict(kind="dense", out=10, bound=31, square=False)]),
    # the whole bi-CryptoNets model on the MNIST-shaped batch (ciphertext branch as in cfg2)
    "cfg2_bi": dict(params="cfg2i", packing="batch", batch=8192, image=(1, 28, 28), crop=(6, 16),
                    plain=dict(ch1=8, k1=5, stride1=2, pad1=1, ch2=8, k2=3, stride2=2, noise=16.0),
                    layers=[dict(kind="conv", out=5, k=5, stride=2, pad=1, bound=15, features="plain", square=True),
                            dict(kind="dense", out=100, bound=15, square=True),
                            dict(kind="dense", out=10, bound=15, square=False),
                            dict(kind="dense", out=8, bound=7, features="plain", square=True, integration=1),
                            dict(kind="dense", out=10, bound=7, features="plain", square=False, integration=2)]),
    "cfg2_bi_small": dict(params="t1k5", packing="batch", batch=512, image=(1, 28, 28), crop=(6, 16),
                          plain=dict(ch1=4, k1=5, stride1=2, pad1=1, ch2=4, k2=3, stride2=2, noise=16.0),
                          layers=[dict(kind="conv", out=2, k=5, stride=2, pad=1, bound=15, features="plain",
                                       square=True),
                                  dict(kind="dense", out=7, bound=15, square=True),
                                  dict(kind="dense", out=3, bound=15, square=False),
                                  dict(kind="dense", out=4, bound=7, features="plain", square=True, integration=1),
                                  dict(kind="dense", out=3, bound=7, features="plain", square=False,
                                       integration=2)]),
    # a fully connected branch on one HW-packed 12x12 MNIST-shaped crop by the diagonal method
    # (on the N = 16384 parameters: each weight-vector product costs about log2(N t / 2) bits of
    # noise budget, two of them need more than four 36-bit primes)
    "fc_diag": dict(params="cfg3", packing="hw", batch=1, image=(1, 28, 28), crop=(8, 12),
                    layers=[dict(kind="dense", out=32, bound=7, square=True, method="diag"),
                            dict(kind="dense", out=10, bound=7, square=False, method="diag")]),
    "fc_diag_small": dict(params="t2k3", packing="hw", batch=1, image=(1, 28, 28), crop=(10, 8),
                          layers=[dict(kind="dense", out=16, bound=7, square=True, method="diag"),
                                  dict(kind="dense", out=4, bound=7, square=False, method="diag")]),
    # the CIFAR-shaped branch with a local sum-pooling layer between the convolutions
    "cfg3_pool": dict(params="cfg3", packing="hw", batch=1, image=(3, 32, 32), crop=(8, 16), sum_after_dense=True,
                      layers=[dict(kind="conv", out=32, k=3, stride=1, pad=0, bound=31, features=True, square=True),
                              dict(kind="pool", k=2, stride=2),
                              dict(kind="conv", out=64, k=3, stride=1, pad=0, bound=31, features=True, square=True,
                                   sum=True),
                              dict(kind="dense", out=10, bound=31, square=False)]),
    "cfg3_pool_small": dict(params="t2k3", packing="hw", batch=1, image=(3, 32, 32), crop=(8, 16),
                            sum_after_dense=True,
                            layers=[dict(kind="conv", out=3, k=3, stride=1, pad=0, bound=31, features=True,
                                         square=True),
                                    dict(kind="pool", k=2, stride=2),
                                    dict(kind="conv", out=2, k=3, stride=1, pad=0, bound=31, features=True,
                                         square=True, sum=True),
                                    dict(kind="dense", out=3, bound=31, square=False)]),
    # the CIFAR-shaped branch under CKKS (the paper's scheme): real inputs (pixel / 255), real
    # weights W / 2^wbits (W the integer weights above), real FP32 features added unquantised;
    # inputs encrypted at scale 2^scale_bits, each mask and square followed by a rescale
    "cfg3_ckks": dict(params="cfg3", scheme="ckks", packing="hw", batch=1, image=(3, 32, 32), crop=(8, 16),
                      sum_after_dense=True, scale_bits=30, wbits=8,
                      layers=[dict(kind="conv", out=32, k=3, stride=1, pad=0, bound=31, features=True, square=True),
                              dict(kind="conv", out=64, k=3, stride=2, pad=0, bound=31, features=True, square=True,
                                   sum=True),
                              dict(kind="dense", out=10, bound=31, square=False)]),
    "cfg3_ckks_small": dict(params="t2k3", scheme="ckks", packing="hw", batch=1, image=(3, 32, 32), crop=(8, 16),
                            sum_after_dense=True, scale_bits=30, wbits=8,
                            layers=[dict(kind="conv", out=3, k=3, stride=1, pad=0, bound=31, features=True,
                                         square=True),
                                    dict(kind="conv", out=2, k=3, stride=2, pad=0, bound=31, features=True,
                                         square=True, sum=True),
                                    dict(kind="dense", out=3, bound=31, square=False)]),
    "cfg3_small": dict(params="t2k3", packing="hw", batch=1, image=(3, 32, 32), crop=(8, 16), sum_after_dense=True,
                       layers=[dict(kind="conv", out=3, k=3, stride=1, pad=0, bound=31, features=True, square=True),
                               dict(kind="conv", out=2, k=3, stride=2, pad=0, bound=31, features=True, square=True,
                                    sum=True),
                               dict(kind="dense", out=3, bound=31, square=False)]),
    "cfg3_bhw_small": dict(params="t2k3", packing="bhw", batch=8, block=256, image=(3, 32, 32), crop=(8, 16),
                           sum_after_dense=True,
                           layers=[dict(kind="conv", out=3, k=3, stride=1, pad=0, bound=31, features=True,
                                        square=True),
                                   dict(kind="conv", out=2, k=3, stride=2, pad=0, bound=31, features=True,
                                        square=True, sum=True),
                                   dict(kind="dense", out=3, bound=31, square=False)]),
}


def image_base(b: int, block: int, n: int) -> int:
    """First slot of image b's block in BHW packing: blocks fill slot row 0, then row 1."""
    per_row = (n // 2) // block
    return (b % per_row) * block + (b // per_row) * (n // 2)


def layer_shapes(name: str):
    """(in_shape, out_shape) per layer as (channels, height, width) or (units,)."""
    w = WORKLOADS[name]
    c = w["image"][0]
    h = wd = w["crop"][1]
    shapes = []
    cur = (c, h, wd)
    for lay in w["layers"]:
        if lay["kind"] == "pool":
            ci, hi, wi = cur
            out = (ci, (hi - lay["k"]) // lay["stride"] + 1, (wi - lay["k"]) // lay["stride"] + 1)
            shapes.append((cur, out))
            cur = out
        elif lay["kind"] == "conv":
            ci, hi, wi = cur
            oh = (hi + 2 * lay["pad"] - lay["k"]) // lay["stride"] + 1
            ow = (wi + 2 * lay["pad"] - lay["k"]) // lay["stride"] + 1
            out = (lay["out"], oh, ow)
            if lay.get("sum"):
                out_after = (lay["out"],)
            else:
                out_after = out
            shapes.append((cur, out))
            cur = out_after
        else:
            n_in = 1
            for d in cur:
                n_in *= d
            out = (lay["out"],)
            shapes.append(((n_in,), out))
            cur = out
    return shapes


def weight_shape(name: str, li: int):
    lay = WORKLOADS[name]["layers"][li]
    (cin, *rest), out = layer_shapes(name)[li]
    if lay["kind"] == "conv":
        return (lay["out"], cin, lay["k"], lay["k"])
    return (lay["out"], cin if not rest else cin * rest[0] * rest[1])


def feature_shape(name: str, li: int):
    """Per-image feature map shape (out channels, out h, out w) of a conv layer with features."""
    return layer_shapes(name)[li][1]


def plain_shapes(name: str):
    """Shapes of the FP32 plaintext-branch and integration parameters, and its map sizes."""
    w = WORKLOADS[name]
    p = w["plain"]
    c, h, _ = w["image"]
    s1 = (h + 2 * p["pad1"] - p["k1"]) // p["stride1"] + 1
    s2 = (s1 - p["k2"]) // p["stride2"] + 1
    out1 = w["layers"][0]["out"]
    oh = layer_shapes(name)[0][1][1]
    n_half = [lay for lay in w["layers"] if lay.get("integration") == 1][0]["out"]
    n_out = [lay for lay in w["layers"] if lay.get("integration") == 2][0]["out"]
    n_p = p["ch2"] * s2 * s2
    return dict(
        tensors=dict(w1=(p["ch1"], c, p["k1"], p["k1"]), b1=(p["ch1"],), crot=(out1, p["ch1"]),
                     w2=(p["ch2"], p["ch1"], p["k2"], p["k2"]), b2=(p["ch2"],),
                     wpp=(n_half, n_p), bpp=(n_half,), wpc=(n_half, n_p), bpc=(n_half,),
                     wo=(n_out, n_half), bo=(n_out,)),
        fan_in=dict(w1=c * p["k1"] ** 2, crot=p["ch1"], w2=p["ch1"] * p["k2"] ** 2, wpp=n_p, wpc=n_p, wo=n_half),
        # weights uniform in +-gain/sqrt(fan_in): the features reach a few units before quantisation
        gain=dict(w1=1.0, crot=16.0, w2=1.0, wpp=4.0, wpc=16.0, wo=16.0),
        s1=s1, s2=s2, n_p=n_p, resize=(s1 - oh) // 2, out_hw=oh)


def plain_feature_layers(name: str) -> dict:
    """Layer index -> which plaintext-side output feeds it: 'z1' (ciphertext layer 1),
    'u1' / 'u2' (the two integration layers)."""
    out = {}
    for li, lay in enumerate(WORKLOADS[name]["layers"]):
        if lay.get("features") == "plain":
            out[li] = {None: "z1", 1: "u1", 2: "u2"}[lay.get("integration")]
    return out


def with_plain_features(inputs: dict, name: str, outs: dict) -> dict:
    """A copy of inputs whose plaintext-fed feature slots hold the given FP32 arrays
    (outs: 'z1', 'u1', 'u2' -> [B][...] arrays)."""
    feats = list(inputs["features"])
    for li, key in plain_feature_layers(name).items():
        feats[li] = outs[key]
    return dict(inputs, features=feats)


def make_inputs(name: str, seeds=SEEDS):
    """All raw inputs of a workload: images, weights and features.  Features that the
    plaintext branch produces (features = "plain") are left None; inputs["plain"] then
    holds that branch's FP32 parameters and perturbation."""
    from . import images as _images, int_weights, features as _features, float_weights, perturbation
    w = WORKLOADS[name]
    c, h, wd = w["image"]
    imgs = _images(seeds["images"], w["batch"], h, wd, c)
    weights, feats = [], []
    plain = None
    if "plain" in w:
        ps = plain_shapes(name)
        plain = {}
        for i, (k, shape) in enumerate(sorted(ps["tensors"].items())):
            fan = ps["fan_in"].get(k)
            plain[k] = float_weights(seeds["weights"], i, shape, ps["gain"][k] / fan ** 0.5 if fan else 0.1)
        plain["noise"] = perturbation(seeds["images"], (w["batch"], c, h, wd), w["plain"]["noise"])
    for li, lay in enumerate(w["layers"]):
        if lay["kind"] == "pool":
            weights.append(None)
            feats.append(None)
            continue
        weights.append(int_weights(seeds["weights"], li, weight_shape(name, li), lay["bound"]))
        if lay.get("features") == "plain":
            feats.append(None)
        elif lay.get("features"):
            fs = feature_shape(name, li)
            shape = (w["batch"],) + fs if w["packing"] in ("batch", "bhw") else fs
            feats.append(_features(seeds["features"], li, shape))
        else:
            feats.append(None)
    out = dict(images=imgs, weights=weights, features=feats)
    if plain is not None:
        out["plain"] = plain
    return out
