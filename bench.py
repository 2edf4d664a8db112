#!/usr/bin/env python3
"""Throughput of the encrypted ciphertext branch of bi-CryptoNets on one MI355X.

A step is one homomorphic evaluation of the whole ciphertext branch over one
batch: for the default workload (MNIST-shaped slot-batched inference: N=8192,
four 36-bit primes, t=1032193, 8192 images, one image per slot, 16x16
sensitive crop) that is conv 5x5/2 (5 maps) + feature injection + square +
relinearisation + modulus switch, dense 100 + square + relinearisation +
modulus switch, dense 10.  Inputs (ciphertexts, features, keys) are resident
in HBM before the timed region.

Prints one JSON line.  `value` is encrypted inferences (images) per second.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector peak in lane operations: 256 CUs x 64 FP64 lanes per clock x 2.4 GHz (the published
# 78.6 TFLOP/s counts each fused multiply-add as two flops; every FP64 instruction here counts one)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
WORKLOAD_TEXT = {
    "cfg2": "MNIST-shaped slot-batched inference: N=8192, 4x36-bit primes, t=1032193, 8192 images/batch, "
            "conv5x5s2(5)+features+square, dense100+square, dense10",
    "cfg1": "tiny HW-packed branch: N=4096, 2x30-bit primes, t=65537, one 28x28 image",
    "cfg3": "CIFAR-shaped HW-packed branch: N=16384, 6x40-bit primes, dnum=3, one 32x32x3 image",
    "cfg2_bi": "whole bi-CryptoNets model on the MNIST-shaped batch: FP32 plaintext branch (side stream) + "
               "ciphertext branch as cfg2 + two feature-integration layers; N=8192, 5x36-bit primes, 8192 images",
    "cfg3_bhw": "CIFAR-shaped branch with BHW packing: N=16384, 6x40-bit primes, dnum=3, 64 32x32x3 images "
                "per ciphertext (one 256-slot block each)",
}


def _schemes():
    from synthetic import workloads as W
    return {k: v.get("scheme", "bfv") for k, v in W.WORKLOADS.items()}


W_SCHEME = _schemes()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of the step captured as one hipGraph instead of eager launches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--kernel", choices=["ntt"], default=None,
                    help="microbenchmark one kernel on the workload's shapes instead of the whole step")
    ap.add_argument("--mix", type=int, default=0,
                    help="batched uneven workload: this many requests drawn from the three parameter sets")
    ap.add_argument("--serve", action="store_true",
                    help="serving loop: Poisson arrivals at --rates, continuous batching vs unbatched")
    ap.add_argument("--rates", default="50,200,800")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-legs", action="store_true",
                    help="only the headline workload (no CIFAR-shaped, transform or serving legs)")
    ap.add_argument("--legs-rates", default="50,200,800", help="Poisson rates of the serving leg")
    ap.add_argument("--legs-requests", type=int, default=600, help="requests per rate in the serving leg")
    return ap.parse_args()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE summaries
    under profiles/ (a `<!-- traffic: {...} -->` record, already scaled by the plain-copy
    calibration).  None when no record exists or the kernel's source changed since the
    counters were taken (the record carries the source file's SHA-256)."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            text = f.read()
        for m in re.finditer(r"<!-- traffic: (\{.*?\}) -->", text):
            rec = json.loads(m.group(1))
            if rec.get("kernel") != kernel or rec.get("workload") != workload:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src):
                continue
            with open(src, "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
                    continue          # taken from an older version of the kernel: stale
            return {"bytes_per_launch": rec["bytes_per_launch"], "read": rec.get("read_bytes_per_launch"),
                    "write": rec.get("write_bytes_per_launch"), "profile": os.path.relpath(path, ROOT)}
    return None


def copy_calibration():
    import torch
    n = 1 << 27                                   # 1 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def ntt_microbench(args):
    """Forward + inverse transforms of the square's batch shape (limbs over Q + aux primes)."""
    import numpy as np
    import torch

    from paper_2402_01296_amd import bcn
    from synthetic import workloads as W
    spec = W.PARAMS[W.WORKLOADS[args.workload]["params"]]
    ctx = bcn.Context(spec["n"], spec["bits"], spec["L"], spec["K"], spec["alpha"], spec["t"])
    tuning = None if args.no_autotune else ctx.autotune()
    nl = ctx.n_q + ctx.n_aux
    polys = 490                                   # 245 ciphertexts x 2 parts, as in the first square
    x = torch.zeros((polys, nl, spec["n"]), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        ctx.ntt(x, 0)
        ctx.ntt(x, 0, inverse=True)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.ntt(x, 0)
        ctx.ntt(x, 0, inverse=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ctx.profile(False)
    prof = ctx.profile_read()
    limb_ntts = 2 * polys * nl * args.steps
    out = {"kernel": "ntt", "n": spec["n"], "limbs_per_launch": polys * nl, "steps": args.steps,
           "limb_ntts_per_s": limb_ntts / total, "tuning": tuning}
    for k, (la, ms, by, ops) in prof.items():
        out[k] = {"launches": la, "avg_launch_us": ms * 1000.0 / la, "gbs": by / (ms * 1e-3) / 1e9,
                  "frac_of_hbm_peak": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "fp64_tops": ops / (ms * 1e-3) / 1e12, "frac_of_alu_peak": ops / (ms * 1e-3) / 1e12 / ALU_PEAK_TOPS}
    print(json.dumps(out), flush=True)


def mix_bench(args):
    """Requests/s of the batched path (stacked per parameter set, concurrent streams, hipGraphs)
    against the per-request launch loop on the same requests."""
    import torch

    from paper_2402_01296_amd.batch import Mix
    t0 = time.perf_counter()
    m = Mix(args.mix, autotune=not args.no_autotune)
    setup = time.perf_counter() - t0
    counts = {k: len(g) for k, g in m.groups.items()}
    print("bench: mix ready %s in %.1fs" % (counts, setup), file=sys.stderr, flush=True)
    chunks = {"cfg2": 8, "cfg3": 16}
    # per-request loop
    m.run_per_request()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        alone = m.run_per_request()
    t_alone = (time.perf_counter() - t0) / args.steps
    print("bench: per-request loop %.3f s" % t_alone, file=sys.stderr, flush=True)
    m.run_batched(chunks)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = m.run_batched(chunks)
    t_batched = (time.perf_counter() - t0) / args.steps
    print("bench: batched %.3f s" % t_batched, file=sys.stderr, flush=True)
    per_group = {}
    for name, grp in m.groups.items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(len(grp)):
            grp.run_alone(k)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        t0 = time.perf_counter()
        grp.run_batched(chunks.get(name))
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        per_group[name] = {"requests": len(grp), "alone_s": round(ta, 4), "batched_s": round(tb, 4)}
    m.capture(chunks)
    m.run_batched(graphs=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outg = m.run_batched(graphs=True)
    t_graph = (time.perf_counter() - t0) / args.steps
    same = all(bool((alone[r] == m.request_output(outg, r)).all()) for r in range(len(m.names)))
    # the transform phase of the whole mix: one persistent launch over the uneven (N, limbs) work
    # list against per-group launches on their streams (the autotuner keeps the faster)
    tp_multi = m.transform_phase(multi=True)
    tp_streams = m.transform_phase(multi=False)
    print("bench: transform phase multi %.3f ms, per-group streams %.3f ms" % (tp_multi, tp_streams),
          file=sys.stderr, flush=True)
    n = len(m.names)
    print(json.dumps({
        "metric": "encrypted inferences/sec (batched uneven mix)",
        "value": round(n / t_graph, 2), "unit": "requests/s", "n_gpus": 1, "steps": args.steps,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%d requests drawn uniformly from (N, limbs) in {(4096,2), (8192,4), (16384,6)}"
                               % n, "counts": counts, "chunks": chunks},
        "per_request_loop": {"requests_per_s": round(n / t_alone, 2), "s_per_mix": round(t_alone, 4)},
        "batched_eager": {"requests_per_s": round(n / t_batched, 2), "s_per_mix": round(t_batched, 4)},
        "batched_graphs": {"requests_per_s": round(n / t_graph, 2), "s_per_mix": round(t_graph, 4)},
        "speedup_vs_per_request": round(t_alone / t_graph, 2),
        "per_group": per_group,
        "bit_identical_alone_vs_batched": same,
        "transform_phase": {"work": "forward + inverse transform of every request's input ciphertexts",
                            "one_persistent_launch_ms": round(tp_multi, 3),
                            "per_group_streams_ms": round(tp_streams, 3),
                            "chosen": "one persistent launch" if tp_multi < tp_streams else "per-group streams"},
    }), flush=True)


def serve_bench(args):
    """p50/p99 latency and sustained throughput under Poisson arrivals, continuous batching
    against the unbatched path (one request per launch group), same arrival trace."""
    from paper_2402_01296_amd.serve import Server, poisson_arrivals
    t0 = time.perf_counter()
    srv = Server(autotune=not args.no_autotune, max_batch={"cfg1": 64, "cfg2": 8, "cfg3": 16})
    print("bench: server ready in %.1fs, keys %.1f MB, per-request bytes %s" % (
        time.perf_counter() - t0, srv.key_bytes / 1e6, {k: round(v / 1e6, 1) for k, v in srv.req_bytes.items()}),
        file=sys.stderr, flush=True)
    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        arr = poisson_arrivals(rate, args.serve_requests)
        row = {"rate": rate, "requests": len(arr)}
        for label, mb in (("batched", None), ("unbatched", {n: 1 for n in srv.mix})):
            r = srv.serve(arr, max_batch=mb)
            row[label] = {"p50_ms": round(r["p50_ms"], 3), "p99_ms": round(r["p99_ms"], 3),
                          "throughput": round(r["throughput"], 1), "batches": r["batches"],
                          "mean_batch": {k: round(v, 2) for k, v in r["mean_batch"].items()}}
            print("bench: rate %g %s p50 %.2f ms p99 %.2f ms %.1f req/s" % (
                rate, label, r["p50_ms"], r["p99_ms"], r["throughput"]), file=sys.stderr, flush=True)
        results.append(row)
    top = results[-1]["batched"]
    print(json.dumps({
        "metric": "encrypted inferences/sec + p50/p99 latency (serving)",
        "value": top["throughput"], "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Poisson arrivals, uniform mix of (N, limbs) in {(4096,2), (8192,4), (16384,6)}, "
                               "HBM budget 200 GB", "max_batch": srv.max_batch},
        "rates": results,
    }), flush=True)


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


# oracle state shared with forked workers of the all-core leg (set before the pool forks)
_ORACLE = {}


def _oracle_output(task):
    """One output ciphertext of one layer of the MNIST-shaped step, computed by the oracle."""
    from oracle import bfv
    O, w, feats, cts = _ORACLE["O"], _ORACLE["w"], _ORACLE["feats"], _ORACLE["cts"]
    prm = O.prm
    layer, idx = task
    t0 = time.perf_counter()
    if layer == 0:
        c, y, x = idx
        ct = bfv.mac(prm, cts[0], w[0][c, 0].reshape(-1))
        ct = bfv.add_plain(prm, ct, O.enc.encode(feats[:, c, y, x]))
        bfv.modswitch(prm, bfv.square(prm, ct, O.rk))
    elif layer == 1:
        ct = bfv.mac(prm, cts[1], w[1][idx])
        bfv.modswitch(prm, bfv.square(prm, ct, O.rk))
    else:
        bfv.mac(prm, cts[2], w[2][idx])
    return layer, time.perf_counter() - t0


def cpu_baseline(workload: str, workers: int):
    """The oracle on a bounded sample of one step, scaled to inferences/s, on one core and on
    `workers` cores (a process pool over independent output ciphertexts).

    Sample: output ciphertexts of the three layers (conv outputs with their feature add,
    square, relinearisation and modulus switch; dense-100 outputs with square and modulus
    switch; dense-10 outputs) on random ciphertexts of the right level.  The step time is
    each layer's time per output times its number of outputs (245, 100, 10).  Runs before
    the GPU is touched, so the pool may fork.
    """
    import multiprocessing as mp

    import synthetic
    from oracle import network, programs
    from oracle import bfv
    from synthetic import workloads as W

    assert workload == "cfg2"
    t_all = time.perf_counter()
    O = programs.OracleSession(workload, with_galois=False)
    prm = O.prm

    def rand_cts(level, count, seed):
        out = []
        for i in range(count):
            r0 = synthetic.test_poly(seed, 2 * i, prm.q[:level], prm.n)
            r1 = synthetic.test_poly(seed, 2 * i + 1, prm.q[:level], prm.n)
            out.append(bfv.Ct(bfv.from_rns(r0, prm.q[:level]), bfv.from_rns(r1, prm.q[:level]), level))
        return out

    _ORACLE.update(O=O, w=O.inputs["weights"], feats=network.quantise(O.inputs["features"][0]),
                   cts=[rand_cts(prm.L, 25, 101), rand_cts(prm.L - 1, 245, 102), rand_cts(prm.L - 2, 100, 103)])
    shapes = W.layer_shapes(workload)
    n_out = [shapes[0][1][0] * shapes[0][1][1] * shapes[0][1][2], shapes[1][1][0], shapes[2][1][0]]
    batch = W.WORKLOADS[workload]["batch"]
    setup_s = time.perf_counter() - t_all
    # one core: 3 + 3 + 10 outputs
    single = [(0, (0, 3, 3)), (0, (2, 0, 5)), (0, (4, 6, 1)), (1, 0), (1, 41), (1, 99)] + [(2, o) for o in range(10)]
    per = {0: [], 1: [], 2: []}
    for task in single:
        layer, dt = _oracle_output(task)
        per[layer].append(dt)
    t1 = [sum(v) / len(v) for v in (per[0], per[1], per[2])]
    step1 = sum(n * t for n, t in zip(n_out, t1))
    sampled1 = sum(sum(v) for v in per.values())
    out = {
        "value": batch / step1, "unit": "encrypted inferences/s (images)", "cores": 1, "kind": "oracle",
        "requests_per_s": 1.0 / step1,
        "sample": "one core: 3 + 3 + 10 output ciphertexts of the three layers on random ciphertexts of the "
                  "right level (%.1f s of oracle work; per output: layer1 %.2fs, layer2 %.2fs, layer3 %.3fs), "
                  "scaled by the outputs per layer (%d, %d, %d) to one step of %d images: %.0f s/step"
                  % (sampled1, t1[0], t1[1], t1[2], n_out[0], n_out[1], n_out[2], batch, step1),
    }
    model, ncpu, avail = _host_cpu()
    out["host"] = {"cpu_model": model, "nproc": ncpu, "cpus_available": avail}
    if workers > 1:
        # all cores: `workers` outputs of each of the two big layers and all ten dense-10 outputs,
        # each layer's tasks run together on the pool; per-output time = wall time / outputs
        ctx = mp.get_context("fork")
        tasks = {0: [(0, (k % 5, (k // 5) % 7, (3 * k) % 7)) for k in range(workers)],
                 1: [(1, (17 * k) % 100) for k in range(workers)],
                 2: [(2, o) for o in range(10)]}
        wall = {}
        with ctx.Pool(workers) as pool:
            pool.map(_oracle_output, [(2, 0)] * workers)          # start the workers
            for layer in (0, 1, 2):
                t0 = time.perf_counter()
                pool.map(_oracle_output, tasks[layer], chunksize=1)
                wall[layer] = (time.perf_counter() - t0) / len(tasks[layer])
        stepw = sum(n * wall[k] for k, n in enumerate(n_out))
        out["all_cores"] = {
            "value": batch / stepw, "requests_per_s": 1.0 / stepw, "cores": workers,
            "sample": "%d worker processes (fork) over %d + %d + 10 independent output ciphertexts; per output "
                      "wall time: layer1 %.3fs, layer2 %.3fs, layer3 %.4fs; %.0f s/step"
                      % (workers, workers, workers, wall[0], wall[1], wall[2], stepw)}
        # the reported baseline is the all-core figure
        out["single_core"] = {"value": out["value"], "requests_per_s": out["requests_per_s"]}
        out["value"] = out["all_cores"]["value"]
        out["requests_per_s"] = out["all_cores"]["requests_per_s"]
        out["cores"] = workers
    out["sample"] += "; setup %.1fs, total wall %.1fs" % (setup_s, time.perf_counter() - t_all)
    _ORACLE.clear()
    return out


def run_workload(name: str, steps: int, warmup: int, autotune: bool = True, graph: bool = False,
                 verify: bool = True, log_prefix: str = "bench"):
    """Times `steps` steps (one request each) of a workload's whole ciphertext branch, then an
    instrumented pass with per-kernel launch timing; returns the measurements."""
    import torch

    from paper_2402_01296_amd.workload import GpuSession
    from synthetic import workloads as W

    wl = W.WORKLOADS[name]
    g = GpuSession(name)
    tuning = g.autotune() if autotune else None
    for ln in (tuning or "").splitlines():
        print("%s: %s autotune %s" % (log_prefix, name, ln), file=sys.stderr, flush=True)
    ct_in = g.encrypt_inputs()
    torch.cuda.synchronize()
    print("%s: %s keys+encryption ready, %d input ciphertexts" % (log_prefix, name, ct_in.shape[0]),
          file=sys.stderr, flush=True)

    if g.plain is not None:
        # the whole model: the plaintext branch on a side stream, in parallel with the HE layers
        images, noise = g.plain_inputs(g.inputs)
        side = torch.cuda.Stream()

        def step():
            return g.run_bi(ct_in, images, noise, side)
    else:
        def step():
            return g.run(ct_in)

    for _ in range(max(2, warmup)):
        out = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eager_out = step()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1000.0 / steps
    eager_step = step
    graph_ok = None
    if graph:
        # the whole step captured once as a hipGraph and replayed, checked against the eager result
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            graph_out = step()
        cg.replay()
        torch.cuda.synchronize()
        graph_ok = bool(torch.equal(graph_out, eager_out))
        if not graph_ok:
            raise RuntimeError("captured step differs from the eager step")

        def step():  # noqa: F811
            cg.replay()
            return graph_out
        for _ in range(warmup):
            out = step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        out = step()
        ends[i].record()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    lat = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    ms_per_step = total * 1000.0 / steps
    print("%s: %s timed %d steps, %.3f ms/step" % (log_prefix, name, steps, ms_per_step), file=sys.stderr, flush=True)

    # instrumented eager pass over the same steps: per-kernel launch durations (library hipEvents
    # around each launch, on the launch stream)
    g.ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eager_step()
    torch.cuda.synchronize()
    inst_ms = (time.perf_counter() - t0) * 1000.0 / steps
    g.ctx.profile(False)
    prof = g.ctx.profile_read()
    kern = {}
    for k, (la, ms, by, ops) in prof.items():
        sec = ms * 1e-3
        kern[k] = dict(launches=la, ms=ms, bytes=by, ops=ops,
                       gbs=by / sec / 1e9 if sec > 0 else 0.0, tops=ops / sec / 1e12 if sec > 0 else 0.0)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    roof = roofline(kern[dom], dom, name)
    # transform-bearing kernels: the plain transforms and the kernels that run transforms inside
    tk = [k for k in kern if k.startswith("ntt") or k in ("square_fused", "ks_intt", "ks_fused")]
    t_bytes = sum(kern[k]["bytes"] for k in tk)
    t_ms = sum(kern[k]["ms"] for k in tk)
    verified = None
    if not wl.get("decrypts", True):
        verified = "n/a: two 30-bit limbs leave no noise budget after the square, so the output does not decrypt"
    elif verify:
        from oracle import network   # test-only check of this run's outputs
        vals = g.output_values(out)
        want = network.run_mod_t(name, g.inputs, g.ctx.t)
        verified = bool((vals == want).all())
    res = {
        "workload": WORKLOAD_TEXT.get(name, name), "name": name, "n": g.n, "limbs": g.ctx.L,
        "images_per_request": wl["batch"], "steps": steps, "ms_per_step": round(ms_per_step, 3),
        "requests_per_s": round(steps / total, 3), "images_per_s": round(wl["batch"] * steps / total, 1),
        "step_time_ms": {"p50": round(statistics.median(lat), 3),
                         "p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 3),
                         "note": "device time of one step (one request) back to back, not a served latency"},
        "transform_kernels": {"kernels": sorted(tk),
                              "gbs": round(t_bytes / (t_ms * 1e-3) / 1e9, 1) if t_ms else None,
                              "frac_of_hbm_peak": round(t_bytes / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if t_ms
                              else None,
                              "ms_per_step": round(t_ms / steps, 3)},
        "roofline": roof,
        "kernels": {k: {"ms_per_step": round(v["ms"] / steps, 3), "launches": v["launches"],
                        "gbs": round(v["gbs"], 1), "fp64_tops": round(v["tops"], 3)}
                    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])},
        "instrumented_ms_per_step": round(inst_ms, 3),
        "timed_as": "hipGraph replay of the whole step" if graph else "eager launches",
        "eager_ms_per_step": round(eager_ms, 3),
        "graph_matches_eager": graph_ok,
        "autotune": [ln for ln in (tuning or "").splitlines() if "chosen" in ln],
        "verified_vs_integer_network": verified,
    }
    del g, ct_in, out, eager_out
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def run_ckks_workload(name: str, steps: int, warmup: int, autotune: bool = True, verify: bool = True):
    """The CIFAR-shaped branch under CKKS (the paper's scheme): requests/s of one image, the
    per-kernel split, and the decrypted outputs against the FP64 real-valued network."""
    import numpy as np
    import torch

    from paper_2402_01296_amd.ckks_workload import CkksSession
    g = CkksSession(name)
    tuning = g.ctx.autotune() if autotune else None
    ct_in = g.encrypt_inputs()
    for _ in range(max(2, warmup)):
        out, scale = g.run(ct_in)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out, scale = g.run(ct_in)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    print("bench: %s timed %d steps, %.3f ms/step" % (name, steps, total * 1e3 / steps), file=sys.stderr, flush=True)
    g.ctx.profile(True)
    for _ in range(steps):
        g.run(ct_in)
    torch.cuda.synchronize()
    g.ctx.profile(False)
    kern = {}
    for k, (la, ms, by, ops) in g.ctx.profile_read().items():
        sec = ms * 1e-3
        kern[k] = dict(launches=la, ms=ms, bytes=by, ops=ops,
                       gbs=by / sec / 1e9 if sec > 0 else 0.0, tops=ops / sec / 1e12 if sec > 0 else 0.0)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    err = None
    if verify:
        from oracle import ckks_network   # test-only check of this run's outputs
        want = ckks_network.run(name, g.inputs)
        got = g.output_values(out, scale)
        err = float(np.abs(got - want).max() / np.abs(want).max())
    res = {"workload": "CIFAR-shaped branch under CKKS (the paper's scheme): N=16384, 6x40-bit primes, dnum=3, "
                       "one 32x32x3 image, inputs at scale 2^30, real weights W/2^8, real features",
           "name": name, "ms_per_step": round(total * 1e3 / steps, 3), "requests_per_s": round(steps / total, 3),
           "roofline": roofline(kern[dom], dom, name),
           "kernels": {k: {"ms_per_step": round(v["ms"] / steps, 3), "launches": v["launches"],
                           "gbs": round(v["gbs"], 1), "fp64_tops": round(v["tops"], 3)}
                       for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])},
           "autotune": [ln for ln in (tuning or "").splitlines() if "chosen" in ln],
           "max_error_vs_real_network": err,
           "error_bound": 1e-6}
    del g, ct_in, out
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def roofline(d: dict, kernel: str, workload: str):
    """The kernel's bound is the larger of its two floors: algorithmic bytes at the HBM peak and
    algorithmic FP64 operations at the vector peak; achieved = algorithmic units / launch time."""
    hbm_floor = d["bytes"] / (HBM_PEAK_GBS * 1e9)
    alu_floor = d["ops"] / (ALU_PEAK_TOPS * 1e12)
    la = max(1, d["launches"])
    if alu_floor > hbm_floor:
        roof = {"kernel": kernel, "bound": "alu", "achieved": round(d["tops"], 3), "peak": round(ALU_PEAK_TOPS, 3),
                "unit": "T fp64 op/s", "frac": round(d["tops"] / ALU_PEAK_TOPS, 4)}
    else:
        roof = {"kernel": kernel, "bound": "hbm", "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(d["gbs"] / HBM_PEAK_GBS, 4)}
    traffic = measured_traffic(kernel, workload)
    roof.update({
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "traffic_unit": "bytes per launch (HBM read + write, rocprofv3 counters)",
        "traffic_over_algorithmic": round(traffic["bytes_per_launch"] / (d["bytes"] / la), 3) if traffic else None,
        "traffic_profile": traffic["profile"] if traffic else None,
        "launches": d["launches"],
        "avg_launch_us": round(d["ms"] * 1000.0 / la, 2),
        "bytes_per_launch": d["bytes"] / la,
        "fp64_ops_per_launch": d["ops"] / la,
        "hbm_gbs": round(d["gbs"], 1),
        "hbm_frac": round(d["gbs"] / HBM_PEAK_GBS, 4),
        "alu_frac": round(d["tops"] / ALU_PEAK_TOPS, 4),
    })
    return roof


def ntt_leg(workload: str, steps: int, autotune: bool = True):
    """Plain forward + inverse limb transforms on the square's batch shape (HBM GB/s vs peak)."""
    import torch

    from paper_2402_01296_amd import bcn
    from synthetic import workloads as W
    spec = W.PARAMS[W.WORKLOADS[workload]["params"]]
    ctx = bcn.Context(spec["n"], spec["bits"], spec["L"], spec["K"], spec["alpha"], spec["t"])
    if autotune:
        ctx.autotune()
    nl = ctx.n_q + ctx.n_aux
    polys = 490
    x = torch.zeros((polys, nl, spec["n"]), dtype=torch.float64, device="cuda")
    for _ in range(2):
        ctx.ntt(x, 0)
        ctx.ntt(x, 0, inverse=True)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(steps):
        ctx.ntt(x, 0)
        ctx.ntt(x, 0, inverse=True)
    torch.cuda.synchronize()
    ctx.profile(False)
    out = {"n": spec["n"], "limb_transforms_per_launch": polys * nl}
    for k, (la, ms, by, ops) in ctx.profile_read().items():
        out[k] = {"launches": la, "avg_launch_us": round(ms * 1000.0 / la, 2),
                  "gbs": round(by / (ms * 1e-3) / 1e9, 1),
                  "frac_of_hbm_peak": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "limb_transforms_per_s": round(polys * nl * la / (ms * 1e-3), 1)}
    del x, ctx
    torch.cuda.empty_cache()
    return out


def serving_leg(rates, n_requests: int, autotune: bool = True, window_ms: float = None):
    from paper_2402_01296_amd.serve import Server, poisson_arrivals
    t0 = time.perf_counter()
    srv = Server(autotune=autotune, max_batch={"cfg1": 64, "cfg2": 8, "cfg3": 16})
    if window_ms is not None:
        srv.window = window_ms * 1e-3
    print("bench: server ready in %.1fs, keys %.1f MB, per-request bytes %s" % (
        time.perf_counter() - t0, srv.key_bytes / 1e6, {k: round(v / 1e6, 1) for k, v in srv.req_bytes.items()}),
        file=sys.stderr, flush=True)
    rows = []
    for rate in rates:
        arr = poisson_arrivals(rate, n_requests)
        row = {"rate": rate, "requests": len(arr)}
        for label, mb in (("batched", None), ("unbatched", {n: 1 for n in srv.mix})):
            r = srv.serve(arr, max_batch=mb, window=None if mb is None else 0.0)
            row[label] = {"p50_ms": round(r["p50_ms"], 3), "p99_ms": round(r["p99_ms"], 3),
                          "throughput": round(r["throughput"], 1), "batches": r["batches"],
                          "mean_batch": {k: round(v, 2) for k, v in r["mean_batch"].items()}}
            print("bench: rate %g %s p50 %.2f ms p99 %.2f ms %.1f req/s" % (
                rate, label, r["p50_ms"], r["p99_ms"], r["throughput"]), file=sys.stderr, flush=True)
        rows.append(row)
    info = {"max_batch": srv.max_batch, "window_ms": srv.window * 1e3, "depth": srv.depth,
            "hbm_budget_gb": srv.budget / 1e9, "key_bytes": srv.key_bytes,
            "request_bytes": srv.req_bytes, "request_bytes_fixed": srv.req_fixed,
            "admission": "per-request bytes measured: arena high-water + torch peak of batches of 1 and 2"}
    srv.close()
    return rows, info


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.kernel == "ntt":
        ntt_microbench(args)
        return
    if args.mix:
        mix_bench(args)
        return
    if args.serve:
        serve_bench(args)
        return
    if W_SCHEME.get(args.workload) == "ckks":
        print(json.dumps(run_ckks_workload(args.workload, args.steps, args.warmup, not args.no_autotune,
                                           not args.no_verify)), flush=True)
        return
    # the oracle baseline runs first, before anything touches the GPU (its pool forks)
    cpu = None
    if not args.no_cpu_baseline and args.workload == "cfg2":
        print("bench: timing the oracle sample on the host", file=sys.stderr, flush=True)
        _, _, avail = _host_cpu()
        cpu = cpu_baseline(args.workload, workers=min(16, avail))
        print("bench: oracle baseline %.1f images/s on %d cores" % (cpu["value"], cpu["cores"]),
              file=sys.stderr, flush=True)
    head = run_workload(args.workload, args.steps, args.warmup, autotune=not args.no_autotune, graph=args.graph,
                        verify=not args.no_verify)
    legs = {}
    if not args.no_legs:
        other = "cfg3" if args.workload != "cfg3" else "cfg2"
        legs[other] = run_workload(other, max(5, args.steps // 2), args.warmup, autotune=not args.no_autotune,
                                   verify=not args.no_verify)
        legs["cfg3_bhw"] = run_workload("cfg3_bhw", max(5, args.steps // 2), args.warmup,
                                        autotune=not args.no_autotune, verify=not args.no_verify)
        legs["cfg2_bi"] = run_workload("cfg2_bi", max(5, args.steps // 2), args.warmup,
                                       autotune=not args.no_autotune, verify=not args.no_verify)
        legs["cfg3_ckks"] = run_ckks_workload("cfg3_ckks", max(5, args.steps // 2), args.warmup,
                                              autotune=not args.no_autotune, verify=not args.no_verify)
        legs["ntt_" + args.workload] = ntt_leg(args.workload, max(5, args.steps // 2), not args.no_autotune)
        rows, info = serving_leg([float(r) for r in args.legs_rates.split(",")], args.legs_requests,
                                 autotune=not args.no_autotune)
        legs["serving"] = {"rates": rows, **info}
    served = None
    if "serving" in legs:
        r0 = legs["serving"]["rates"][0]
        served = {"rate_req_per_s": r0["rate"], "p50": r0["batched"]["p50_ms"], "p99": r0["batched"]["p99_ms"],
                  "unbatched_p50": r0["unbatched"]["p50_ms"], "unbatched_p99": r0["unbatched"]["p99_ms"],
                  "note": "served end-to-end latency (arrival to completion) under Poisson arrivals of the "
                          "mixed workload"}
    line = {
        "metric": "encrypted inferences/sec + p50/p99 latency; NTT HBM GB/s vs peak",
        "value": head["requests_per_s"],
        "unit": "encrypted inferences/s (requests)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "name": head["name"], "n": head["n"], "limbs": head["limbs"],
                   "images_per_request": head["images_per_request"]},
        "images_per_s": head["images_per_s"],
        "latency_ms": served,
        "step_time_ms": head["step_time_ms"],
        "roofline": head["roofline"],
        "transform_kernels": head["transform_kernels"],
        "kernels": head["kernels"],
        "instrumented_ms_per_step": head["instrumented_ms_per_step"],
        "timed_as": head["timed_as"],
        "eager_ms_per_step": head["eager_ms_per_step"],
        "graph_matches_eager": head["graph_matches_eager"],
        "autotune": head["autotune"],
        "verified_vs_integer_network": head["verified_vs_integer_network"],
        "legs": legs,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
