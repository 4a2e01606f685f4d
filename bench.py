#!/usr/bin/env python3
"""Benchmark: decoded queries/s of the block-compressed neural material decode
(fetch + BC6H unpack + trilinear filter + MLP) on one MI355X.

Workload (the full-frame case): four 2048x2048 BC6H feature pyramids with full
mip chains (12 levels, modes uniform over all 14, endpoints bounded so every
texel is below 1.0), decoder MLP 12-32-32-10, and the 3840x2160 queries of a
perspective ground plane in scanline order with LOD from analytic uv
derivatives. Synthetic seeded data; no trained weights exist for it.

One step = one decode of the whole frame with textures, MLP and queries
already resident in HBM, issued as its two calls (bcf_unpack, then
bcf_decode_unpacked) so that HIP events time each kernel; the step time is
the median over the timed steps. The headline value is the FP16-MFMA rate;
the plain FP32 rate is timed on the same inputs. The FP16 output is compared
with the FP32 output over the whole frame, and (in the CPU-baseline leg) both
with the fp64 oracle on the oracle's sample; the rate is reported only when
FP16 stays within 2e-3 of both. The same decode of full-range random blocks
(variant R) and of the frame's queries in shuffled order (seed 4, no image
structure) are timed alongside.

The roofline prices the dominant kernel on the path's algorithmic bytes:
12 (query) + 4c (output) + 16 U / N (every distinct BC6H block the frame's
footprints touch, read once) per query.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded queries/s (fetch+BC6H+MLP), FP16-MFMA vs FP32 at ≤2e-3 abs err"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _footprints(textures, queries):
    """For each distinct pyramid geometry ((w, h), levels, bias) and each level:
    how many pyramids share it, the level's size, and the integer tap
    coordinates (x0, y0) of every query footprint that reads the level
    (eq. 9 at s_i = s + b_i, texel centres at (i + 1/2)/w, wrap addressing)."""
    u = queries[:, 0].astype(np.float64)
    v = queries[:, 1].astype(np.float64)
    s = queries[:, 2].astype(np.float64)
    u -= np.floor(u)
    v -= np.floor(v)
    counts = {}
    for t in textures:                      # pyramids of one geometry touch the same positions
        counts[t] = counts.get(t, 0) + 1
    for ((w0, h0), levels, bias), times in counts.items():
        si = np.clip(s + bias, 0, levels - 1)
        l0 = np.floor(si).astype(np.int64)
        l1 = np.minimum(l0 + 1, levels - 1)
        for lev in range(levels):
            w, h = max(w0 >> lev, 1), max(h0 >> lev, 1)
            sel = (l0 == lev) | (l1 == lev)
            if not sel.any():
                continue
            x0 = np.floor(u[sel] * w - 0.5).astype(np.int64)
            y0 = np.floor(v[sel] * h - 0.5).astype(np.int64)
            yield times, w, h, x0, y0


def unique_blocks(textures, queries):
    """Distinct (pyramid, level, block) the trilinear footprints of `queries`
    touch: the BC6H blocks a decode must read at least once."""
    total = 0
    for times, w, h, x0, y0 in _footprints(textures, queries):
        bx, by = (w + 3) // 4, (h + 3) // 4
        mark = np.zeros(bx * by, bool)
        for dx in (0, 1):
            for dy in (0, 1):
                mark[(((y0 + dy) % h) // 4) * bx + ((x0 + dx) % w) // 4] = True
        total += times * int(mark.sum())
    return total


def unique_texels(textures, queries):
    """Distinct (pyramid, level, texel) the footprints touch: the unpacked
    texels the filter kernel must read at least once."""
    total = 0
    for times, w, h, x0, y0 in _footprints(textures, queries):
        mark = np.zeros(w * h, bool)
        for dx in (0, 1):
            for dy in (0, 1):
                mark[((y0 + dy) % h) * w + (x0 + dx) % w] = True
        total += times * int(mark.sum())
    return total


def all_blocks(textures):
    return sum(sum(((max(w >> l, 1) + 3) // 4) * ((max(h >> l, 1) + 3) // 4) for l in range(L))
               for (w, h), L, _ in textures)


FRAME_SOURCES = ("api.cpp", "bc6h_device.hpp", "filter_device.hpp", "frame_f16.hip", "frame_kernels.hpp",
                 "internal.hpp", "kernels.hip", "mlp_device.hpp")


def sources_digest():
    """Digest of the sources the filter kernel is built from: counter figures
    taken from another version of the kernel do not apply."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2311_16121_amd", "csrc")
    for name in FRAME_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_frame_fp16_frame4k_traffic.md")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batch_batch64_traffic.md")


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch of the kernel a committed counter summary covers
    (k_frame FP16 on frame4k by default), or None when it is missing or was
    taken from other kernel sources."""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("sources_digest") != sources_digest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """The host's logical CPU count, the CPUs this process may use, and the model name."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(material, queries, budget_s, gpu_outputs=None):
    """The CPU oracle on the GPU host's cores: all threads the process may use
    (at most 16) on a bounded seeded sample of the workload's queries, the
    median of 3 runs; and one thread on the first 2^20 queries of the
    workload (median of 3). When `gpu_outputs` ({name: host array [n, c]}) is
    given, also the largest difference of each from the oracle on the
    all-cores sample."""
    import statistics

    import oracle
    import synth
    host_mat = oracle.Material.from_synth(material)
    threads = oracle.default_threads()
    pick = synth.rng(synth.SEED_SHUFFLE).permutation(len(queries))
    n = 2048
    t = time.perf_counter()
    oracle.decode(host_mat, queries[pick[:n]], n_threads=threads)
    dt = time.perf_counter() - t
    n = int(min(len(pick), max(n, n * (budget_s / 6) / max(dt, 1e-6))))
    runs = []
    for _ in range(3):
        t = time.perf_counter()
        ref = oracle.decode(host_mat, queries[pick[:n]], n_threads=threads)
        runs.append(time.perf_counter() - t)
    dt = statistics.median(runs)
    prefix = min(len(queries), 1 << 20)
    one = []
    for _ in range(3):
        t = time.perf_counter()
        oracle.decode(host_mat, queries[:prefix], n_threads=1)
        one.append(time.perf_counter() - t)
    out = {"value": n / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} queries drawn without replacement (seed {synth.SEED_SHUFFLE}) from the same "
                     f"workload; median of 3 runs ({', '.join(f'{r:.2f}' for r in runs)} s) on {threads} threads",
           "single_core": {"value": prefix / statistics.median(one), "unit": "queries/s",
                           "sample": f"the first {prefix} queries, one thread, median of 3 runs "
                                     f"({', '.join(f'{r:.2f}' for r in one)} s)"},
           "host": host_cpu()}
    if gpu_outputs:
        out["gpu_vs_oracle_max_abs"] = {k: float(np.abs(v[pick[:n]] - ref).max()) for k, v in gpu_outputs.items()}
    return out


def bench_batch(args):
    """64 materials (base 512..4096^2, four pyramids each, full chains), MLP
    12-32-32-10 FP16 each, query counts log-uniform in [2^14, 2^22], u, v
    uniform, s uniform over each chain. A step unpacks the blocks the queries
    touch and decodes every query in one persistent launch, replayed from a
    graph."""
    import torch

    import paper_2311_16121_amd as bcf
    import synth

    spec = synth.batch_spec()
    pool = synth.block_pool()
    log(f"generating {spec.n_materials} materials, {sum(spec.counts)} queries")
    mats, qparts, hosts, hqs, alg_blocks = [], [], [], [], 0
    for k in range(spec.n_materials):
        m = synth.batch_material(spec, k, pool)
        mats.append(bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params))
        q = synth.batch_queries(spec, k)
        geo = [((r, r), L, b) for r, L, b in zip(m.res, m.levels, m.lod_bias)]
        alg_blocks += unique_blocks(geo, q)
        qparts.append(torch.from_numpy(q).cuda())
        if not args.no_cpu_baseline:
            hosts.append(m)
            hqs.append(q)
        del m
    qd = torch.cat(qparts)
    del qparts
    n = qd.shape[0]
    offsets = torch.from_numpy(spec.offsets().astype(np.int32)).cuda()
    batch = bcf.Batch(mats, bcf.Precision.FP16)
    out = torch.empty((n, spec.dims[-1]), dtype=torch.float32, device="cuda")
    batch.unpack()
    log("tuning")
    plan, tuned_ms = batch.tune(qd, offsets, out=out)
    stream = torch.cuda.current_stream()

    # per-call times with events (eager): the whole unpack (for reference),
    # the unpack of the blocks the queries touch, the decode
    def eager(steps):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        for e in ev:
            e[0].record(stream)
            batch.unpack(stream)
            e[1].record(stream)
            batch.unpack_touched(qd, offsets, stream)
            e[2].record(stream)
            batch.decode(qd, offsets, out=out, plan=plan, stream=stream)
            e[3].record(stream)
        torch.cuda.synchronize()
        return tuple(sum(e[i].elapsed_time(e[i + 1]) for e in ev) / steps for i in range(3))

    eager(args.warmup)
    unpack_ms, touched_ms, decode_ms = eager(args.steps)
    # the step as one graph: unpack the touched blocks, decode
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            batch.unpack_touched(qd, offsets)
            batch.decode(qd, offsets, out=out, plan=plan)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        graph.replay()
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    c = spec.dims[-1]
    step_bytes = n * 12 + n * 4 * c + 16 * alg_blocks     # queries, outputs, every touched block once
    blocks = sum(4 * synth.chain_blocks(r, r, synth.full_levels(r, r)) for r in spec.res)
    unpack_bytes = blocks * (16 + 16 * 6)          # every block in, its 16 texels' (r, g, b) halves out
    achieved = step_bytes / (decode_ms * 1e-3) / 1e9
    line = {
        "metric": "decoded queries/s, 64 materials per graph-captured step: unpack of the touched blocks, one "
                  "persistent decode launch (FP16-MFMA MLP)",
        "value": n / (ms * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "batch64: 64 materials, base 512..4096^2 (4 pyramids, full chains), MLP 12-32-32-10 "
                               "FP16 per material, queries log-uniform in [2^14, 2^22] per material",
                   "queries": n, "materials": spec.n_materials, "texture_bytes": blocks * 16,
                   "plan": {"workgroups": plan[0], "interleave": plan[1], "run": plan[2], "waves": plan[3],
                            "tuned_decode_ms": tuned_ms}},
        "roofline": {"bound": "hbm", "kernel": "k_batch (fp16)", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(BATCH_TRAFFIC_FILE),
                     "alg_bytes_per_launch": step_bytes, "launch_ms": decode_ms},
        "kernels": {"unpack_all": {"launch_ms": unpack_ms, "alg_bytes": unpack_bytes,
                                   "achieved": unpack_bytes / (unpack_ms * 1e-3) / 1e9,
                                   "note": "every block of every material; not part of the step"},
                    "unpack_touched": {"ms": touched_ms, "blocks": alg_blocks,
                                       "note": "clear + item prefix + mark + unpack launches"},
                    "decode": {"launch_ms": decode_ms},
                    "step": {"bound": "hbm", "achieved": step_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                             "frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "launch_ms": ms}},
        "counts": {"unique_blocks": alg_blocks, "all_blocks": blocks},
    }
    if not args.no_cpu_baseline:
        # the oracle on rows spread over every material, timed; the graph's
        # output on the same rows compared with it
        import oracle
        log("cpu baseline")
        got = out.cpu().numpy()
        offs = spec.offsets()
        threads = oracle.default_threads()
        rows, worst, dt = 0, 0.0, 0.0
        for k, (m, q) in enumerate(zip(hosts, hqs)):
            pick = np.unique(np.linspace(0, len(q) - 1, 2048).astype(np.int64))
            t0 = time.perf_counter()
            ref = oracle.decode(oracle.Material.from_synth(m), q[pick], n_threads=threads)
            dt += time.perf_counter() - t0
            rows += len(pick)
            worst = max(worst, float(np.abs(got[offs[k] + pick] - ref).max()))
        line["cpu_baseline"] = {"value": rows / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
                                "sample": f"{rows} rows, 2048 spread over each material's range; {dt:.1f} s",
                                "host": host_cpu(), "gpu_vs_oracle_max_abs": {"fp16": worst}}
        line["check"] = {"rows": rows, "max_abs_err_vs_oracle": worst, "bar": 2e-3, "ok": worst <= 2e-3}
        if worst > 2e-3:
            line["value"] = None
    print(json.dumps(line), flush=True)


def bench_train(args):
    """One training step (Section 5.1) per timed step: the straight-through
    forward of four 1024^2 trainable pyramids (full chains, LOD bias -1 against
    the 2048^2 reference), MLP 12-32-32-10, on 2^20 random (u, v, s) samples;
    the mean squared error against the procedural reference sampled bicubically
    on two mips; the backward to every block parameter and weight; one Adam
    update."""
    import torch

    import paper_2311_16121_amd as bcf
    import synth

    dims = (12, 32, 32, 10)
    n = 1 << 20
    log("generating the reference and the trainable pyramids")
    ends, idxs, parts, L, params = synth.train_problem(1024, dims)
    chain = synth.procedural_target(2048)
    q = synth.uniform_queries(n, synth.rng(synth.SEED_QUERIES), float(len(chain) - 1))
    target = torch.from_numpy(synth.sample_target(chain, q)).cuda()
    del chain
    qd = torch.from_numpy(q).cuda()
    geo = bcf.TrainGeometry([1024] * 4, [L] * 4, [torch.from_numpy(p).cuda() for p in parts], dims, [-1.0] * 4,
                            straight_through=True)
    leaves = [torch.from_numpy(e).cuda().requires_grad_(True) for e in ends] + \
             [torch.from_numpy(x).cuda().requires_grad_(True) for x in idxs]
    w = torch.from_numpy(params).cuda().requires_grad_(True)
    # torch's fused Adam: one kernel per step for every parameter tensor
    opt = torch.optim.Adam([{"params": leaves, "lr": 0.02}, {"params": [w], "lr": 2e-3}], fused=True)

    def step():
        out = bcf.train_decode(geo, leaves[:4], leaves[4:], w, qd)
        loss = torch.nn.functional.mse_loss(out, target)
        opt.zero_grad()
        loss.backward()
        opt.step()
        return loss

    losses = [float(step())]
    for _ in range(max(args.warmup - 1, 0)):
        step()
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        loss = step()
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    losses.append(float(loss))
    # the two native calls alone
    with torch.no_grad():
        e = [x.detach() for x in leaves]
        go = torch.randn((n, dims[-1]), device="cuda")
        t0, t1, t2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        bcf.train_forward(geo, e[:4], e[4:], w.detach(), qd)
        bcf.train_backward(geo, e[:4], e[4:], w.detach(), qd, go)
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(5):
            bcf.train_forward(geo, e[:4], e[4:], w.detach(), qd)
        t1.record(stream)
        for _ in range(5):
            bcf.train_backward(geo, e[:4], e[4:], w.detach(), qd, go)
        t2.record(stream)
        torch.cuda.synchronize()
    line = {
        "metric": "training samples/s (straight-through forward + backward + Adam)",
        "value": n / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "train: 4 x 1024^2 trainable BC6H pyramids (11 levels, two-subset 6-bit endpoint / "
                               "3-bit index blocks), MLP 12-32-32-10, batch 2^20, procedural 2048^2 10-channel "
                               "reference", "batch": n,
                   "parameters": int(sum(x.numel() for x in leaves) + w.numel())},
        "loss": {"first": losses[0], "last": losses[-1]},
        "kernels": {"train_forward_ms": t0.elapsed_time(t1) / 5, "train_backward_ms": t1.elapsed_time(t2) / 5},
    }
    if not args.no_cpu_baseline:
        # the fp64 training oracle (forward and backward) on a sample of the
        # batch at the trained parameters, timed; the GPU's forward and
        # gradients on the same sample compared with it
        from oracle import train as T
        log("cpu baseline")
        k = 1 << 15
        qs = q[:k]
        ends_h = [x.detach().cpu().numpy() for x in leaves[:4]]
        idxs_h = [x.detach().cpu().numpy() for x in leaves[4:]]
        w_h = w.detach().cpu().numpy()
        go_s = synth.rng(78).standard_normal((k, dims[-1])).astype(np.float32)
        texs = [T.TrainTexture(1024, 1024, L, e, x, p_, -1.0) for e, x, p_ in zip(ends_h, idxs_h, parts)]
        t0_ = time.perf_counter()
        val, r_end, r_idx, r_par = T.gradients(texs, dims, w_h, qs, go_s, ste=True)
        dt = time.perf_counter() - t0_
        with torch.no_grad():
            qsd = torch.from_numpy(qs).cuda()
            fwd = bcf.train_forward(geo, e[:4], e[4:], w.detach(), qsd).cpu().numpy()
            g_e, g_i, g_p = bcf.train_backward(geo, e[:4], e[4:], w.detach(), qsd, torch.from_numpy(go_s).cuda())
        f_err = float(np.abs(fwd - val).max())
        p_err = float(np.abs(g_p.cpu().numpy() - r_par).max() / np.abs(r_par).max())
        b_err = max(float(np.abs(a.cpu().numpy() - b).max() / max(np.abs(b).max(), 1e-30))
                    for a, b in zip(g_e + g_i, r_end + r_idx))
        line["cpu_baseline"] = {"value": k / dt, "unit": "samples/s", "cores": torch.get_num_threads(),
                                "kind": "oracle", "sample": f"the first {k} samples of the batch, forward and "
                                f"backward in binary64 (torch on the CPU); {dt:.1f} s", "host": host_cpu()}
        line["check"] = {"samples": k, "forward_max_abs_err": f_err, "param_grad_rel_err": p_err,
                         "block_grad_rel_err": b_err, "bars": {"forward": 1e-5, "grad_rel": 2e-4},
                         "ok": f_err <= 1e-5 and p_err <= 2e-4 and b_err <= 2e-4}
    print(json.dumps(line), flush=True)


def bench_sweep(args):
    """Every MLP precision on the precision-sweep workload: 4 x 256^2 pyramids
    (bounded blocks), MLP 12-64-64-10, 2^24 uniform queries. One line, the
    FP8 rate as the value; each precision's rate and its MLP's share of the
    MFMA peak alongside (errors: tests/test_gpu_precision_sweep.py)."""
    import torch

    import paper_2311_16121_amd as bcf
    import synth

    wl = synth.WORKLOADS["sweep"]
    m = synth.workload_material(wl, variant="B")
    q = synth.workload_queries(wl)
    mat = bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params)
    qd = torch.from_numpy(q).cuda()
    calib = synth.uniform_queries(1 << 16, synth.rng(1234), wl.s_max)
    mat.set_act_absmax(bcf.calibrate(mat, torch.from_numpy(calib).cuda()))
    n = len(q)
    out = torch.empty((n, m.dims[-1]), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    flops = 2 * sum(a * b for a, b in zip(m.dims[:-1], m.dims[1:])) * n      # MLP multiply-adds x 2
    peaks = {"FP32": FP32_VECTOR_PEAK_TFLOPS, "FP32_MFMA": 157.3, "FP16": 2500.0, "BF16": 2500.0, "FP8": 5000.0}   # TFLOP/s
    rates = {}
    for name in ("FP32", "FP32_MFMA", "FP16", "BF16", "FP8"):
        prec = bcf.Precision[name]
        ws = bcf.prepare(mat, prec)
        bcf.unpack(mat, ws)
        for _ in range(args.warmup):
            bcf.decode_unpacked(mat, ws, qd, prec, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            bcf.decode_unpacked(mat, ws, qd, prec, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        rates[name] = {"queries_per_s": n / (ms * 1e-3), "ms": ms,
                       "mlp_tflops": flops / (ms * 1e-3) / 1e12,
                       "mlp_frac_of_peak": flops / (ms * 1e-3) / 1e12 / peaks[name]}
        del ws
    line = {
        "metric": "decoded queries/s per MLP precision (filter + MLP from unpacked texels)",
        "value": rates["FP8"]["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rates["FP8"]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp8", "data": "synthetic",
        "config": {"workload": "sweep: 4 x 256^2 BC6H pyramids (9 levels, bounded), MLP 12-64-64-10, "
                               "2^24 uniform queries", "queries": n},
        "precisions": rates,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="frame4k: skip the shuffled-order and variant-R timings")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain copy of this many MiB (to scale memory counters)")
    ap.add_argument("--workload", default="frame4k", choices=("frame4k", "batch64", "train", "sweep"),
                    help="frame4k: the full-frame decode (default); batch64: 64 materials in one launch; "
                         "train: a straight-through training step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(queries shard across GPUs with no communication; the figure reported is one GPU's).", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "train":
        return bench_train(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    return bench_frame(args)


def bench_frame(args):
    """The headline line: frame4k decoded with the FP16-MFMA MLP, the plain
    FP32 MLP beside it, and the R-variant and shuffled-order rates."""
    import statistics

    import torch

    import paper_2311_16121_amd as bcf
    import synth

    wl = synth.WORKLOADS["frame4k"]
    log("generating workload")
    m = synth.workload_material(wl, variant="B")
    q = synth.workload_queries(wl)
    n = len(q)
    c = m.dims[-1]
    mat = bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params)
    qd = torch.from_numpy(q).cuda()
    stream = torch.cuda.current_stream()
    p16, p32 = bcf.Precision.FP16, bcf.Precision.FP32

    def run(mt, ws, queries, p, steps, grid_width, out):
        """`steps` whole decodes, each as its two calls (unpack, then filter +
        MLP) with HIP events around each on the launch stream; per-step
        medians and means in ms."""
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        for e in ev:
            e[0].record(stream)
            bcf.unpack(mt, ws, stream)
            e[1].record(stream)
            bcf.decode_unpacked(mt, ws, queries, p, grid_width=grid_width, out=out, stream=stream)
            e[2].record(stream)
        torch.cuda.synchronize()
        step = [e[0].elapsed_time(e[2]) for e in ev]
        unpack = [e[0].elapsed_time(e[1]) for e in ev]
        frame = [e[1].elapsed_time(e[2]) for e in ev]
        return {"step": statistics.median(step), "step_mean": statistics.fmean(step),
                "unpack": statistics.median(unpack), "unpack_mean": statistics.fmean(unpack),
                "frame": statistics.median(frame), "frame_mean": statistics.fmean(frame)}

    if args.copy_probe:
        # a plain copy of known size, for scaling memory counters (profiling runs only)
        src = torch.ones(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read, {args.copy_probe} MiB written")
        del src, dst

    out = {p: torch.empty((n, c), dtype=torch.float32, device="cuda") for p in (p16, p32)}
    ws = {p: bcf.prepare(mat, p) for p in out}
    log("warmup")
    for p in out:
        run(mat, ws[p], qd, p, args.warmup, 3840, out[p])
    log("timing")
    t = {p: run(mat, ws[p], qd, p, args.steps, 3840, out[p]) for p in out}
    diff16 = float((out[p16] - out[p32]).abs().max().item())
    # the outputs the oracle checks (copied only when the CPU leg runs)
    host_out = None if args.no_cpu_baseline else {"fp16": out[p16].cpu().numpy(), "fp32": out[p32].cpu().numpy()}

    # the same frame in shuffled order (no image structure), and full-range random blocks
    extra = {}
    if not args.no_variants:
        log("shuffled order")
        perm = torch.from_numpy(synth.rng(synth.SEED_SHUFFLE).permutation(n)).cuda()
        qs = qd[perm].contiguous()
        o = torch.empty((n, c), dtype=torch.float32, device="cuda")
        run(mat, ws[p16], qs, p16, args.warmup, 0, o)
        ts = run(mat, ws[p16], qs, p16, args.steps, 0, o)
        same = bool(torch.equal(o, out[p16][perm]))
        extra["shuffled"] = {"queries_per_s": n / (ts["step"] * 1e-3), "ms_per_step": ts["step"],
                             "frame_ms": ts["frame"], "unpack_ms": ts["unpack"],
                             "outputs_equal_scanline_rows": same,
                             "order": f"the frame's queries permuted (seed {synth.SEED_SHUFFLE}), grid_width 0"}
        del qs, o, perm
        log("variant R")
        mr = synth.workload_material(wl, variant="R")
        matr = bcf.Material.from_host(mr.textures, mr.res, mr.levels, mr.dims, mr.params)
        wsr = bcf.prepare(matr, p16)
        o = torch.empty((n, c), dtype=torch.float32, device="cuda")
        run(matr, wsr, qd, p16, args.warmup, 3840, o)
        tr = run(matr, wsr, qd, p16, args.steps, 3840, o)
        extra["variant_R"] = {"queries_per_s": n / (tr["step"] * 1e-3), "ms_per_step": tr["step"],
                              "frame_ms": tr["frame"], "unpack_ms": tr["unpack"],
                              "blocks": "every bit uniform except the mode code (uniform over the 14 modes); "
                                        "texels up to 65504, so speed only"}
        del matr, wsr, o, mr

    # algorithmic work
    geo = [((r, r), L, b) for r, L, b in zip(m.res, m.levels, m.lod_bias)]
    U, T, NB = unique_blocks(geo, q), unique_texels(geo, q), all_blocks(geo)
    step_bytes = n * 12 + n * 4 * c + 16 * U           # the path: queries, outputs, touched blocks once
    scratch_bytes = n * 12 + n * 4 * c + 6 * T         # the filter kernel's own reads: unpacked texels once
    unpack_bytes = NB * (16 + 16 * 6)                  # every block in, its 16 texels' (r, g, b) halves out
    mlp_flops = 2 * sum(x * y for x, y in zip(m.dims[:-1], m.dims[1:])) * n     # MLP multiply-adds x 2

    def roof(kernel, nbytes, kms, traffic=None):
        achieved = nbytes / (kms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "alg_bytes_per_launch": nbytes,
                "launch_ms": kms}

    def roof_flops(kernel, bound, flops, kms, peak):
        achieved = flops / (kms * 1e-3) / 1e12
        return {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None, "alg_flops_per_launch": flops, "launch_ms": kms}

    line = {
        "metric": METRIC,
        "value": None,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t[p16]["step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {
            "workload": "frame4k: 4 x 2048^2 BC6H pyramids, 12 levels, modes uniform over 14, bounded "
                        "endpoints; MLP 12-32-32-10; 3840x2160 perspective ground-plane queries",
            "queries": n,
            "grid_width": 3840,
            "precision": "fp16 MFMA MLP, fp32 filter, exact integer BC6H",
        },
        "step_ms_mean": t[p16]["step_mean"],
        "fp16_max_abs_diff_vs_fp32": diff16,
        "fp32_value": n / (t[p32]["step"] * 1e-3),
        "fp32_ms_per_step": t[p32]["step"],
        # the dominant kernel (filter + MLP, FP16) priced on the path's algorithmic bytes
        "roofline": roof("k_frame (fp16)", step_bytes, t[p16]["frame_mean"], measured_traffic()),
        "kernels": {
            "step_fp16": roof("whole step (unpack + filter + MLP)", step_bytes, t[p16]["step_mean"]),
            "frame_fp16_own_reads": roof("k_frame (fp16), priced on its own reads (unpacked texels)",
                                         scratch_bytes, t[p16]["frame_mean"]),
            "unpack": roof("k_predecode", unpack_bytes, t[p16]["unpack_mean"]),
            "mlp_fp16_mfma": roof_flops("k_frame (fp16): the MLP's FLOPs against the fp16 MFMA peak", "mfma",
                                        mlp_flops, t[p16]["frame_mean"], 2500.0),
            "frame_fp32": roof_flops("k_frame (fp32)", "alu", mlp_flops, t[p32]["frame_mean"],
                                     FP32_VECTOR_PEAK_TFLOPS),
        },
        "peaks_note": "HBM 8 TB/s; fp16 dense MFMA 2.5 PFLOP/s; fp32 vector ALU 78.6 TFLOP/s without packed "
                      "fp32 (256 CUs x 64 lanes x 2 FLOP x 2.4 GHz; the 157.3 TFLOP/s spec figure needs packed "
                      "fp32, which this build does not emit)",
        "counts": {"unique_blocks": U, "unique_texels": T, "all_blocks": NB},
        **extra,
    }
    ok = diff16 <= 2e-3
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cb = cpu_baseline(m, q, args.cpu_budget, host_out)
        line["cpu_baseline"] = cb
        ok = ok and cb["gpu_vs_oracle_max_abs"]["fp16"] <= 2e-3
    line["value"] = n / (t[p16]["step"] * 1e-3) if ok else None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
