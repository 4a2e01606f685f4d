"""GPU tests of the batched decode (bcf_*_batch): many materials with different
pyramid sizes and uneven query counts in one persistent launch.

Bars:
  * every row equals, bit for bit, the single-material decode of the same
    material at the same precision (the per-query arithmetic is the same);
  * sampled rows against the oracle: FP32 <= 1e-5, FP16 <= 2e-3 absolute
    (bounded-feature materials);
  * rows that no material covers are left untouched;
  * graph replays equal the eager decode of the queries present at replay time;
  * after unpacking only the blocks the queries touch (on a workspace whose
    other texels are NaN), the decode equals the single-material decodes.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bcf():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_16121_amd as bcf
    return bcf


def log(msg):
    print(msg, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


DIMS = (12, 32, 32, 10)
# (sizes per pyramid, levels per pyramid, query count, signed)
SHAPES = [
    ([64] * 4, [7] * 4, 3000, False),
    ([(128, 32)] * 4, [8] * 4, 0, False),                 # no queries
    ([256] * 4, [9] * 4, 12345, False),
    ([64, 32, 64, 16], [7, 6, 5, 5], 65, False),           # pyramids of different sizes
    ([32] * 4, [6] * 4, 1, False),
    ([128] * 4, [8] * 4, 4096, True),                      # signed features
    ([16] * 4, [5] * 4, 64, False),
]


# every material's pyramids share one geometry: the pipelined batch loop
SHARED_SHAPES = [sh for sh in SHAPES if len(set(map(str, sh[0]))) == 1 and len(set(sh[1])) == 1]


def make_batch(bcf, shapes=SHAPES, seed=61, dims=DIMS):
    g = synth.rng(seed)
    host, mats, qs = [], [], []
    for k, (sizes, levels, n, signed) in enumerate(shapes):
        sz = [(s, s) if isinstance(s, int) else s for s in sizes]
        texs = [synth.bounded_blocks(synth.chain_blocks(w, h, L), g, signed=signed).reshape(-1)
                for (w, h), L in zip(sz, levels)]
        params = synth.mlp_params(dims, g)
        host.append(oracle.Material(texs, sz, levels, dims, params, [0.0] * len(sz), signed))
        mats.append(bcf.Material.from_host(texs, sz, levels, dims, params, signed=signed))
        qs.append(synth.uniform_queries(n, g, float(max(levels) - 1)))
    offsets = np.concatenate([[0], np.cumsum([len(q) for q in qs])]).astype(np.int32)
    return host, mats, qs, offsets


@pytest.mark.parametrize("shared_only", [False, True])
@pytest.mark.parametrize("precision", ["FP16", "FP32"])
def test_batch_equals_single_material_decodes(bcf, precision, shared_only):
    shapes = SHARED_SHAPES if shared_only else SHAPES
    host, mats, qs, offsets = make_batch(bcf, shapes)
    prec = bcf.Precision[precision]
    batch = bcf.Batch(mats, prec)
    batch.unpack()
    q_all = dev(np.concatenate(qs))
    out = batch.decode(q_all, dev(offsets)).cpu().numpy()
    for k, m in enumerate(mats):
        if len(qs[k]) == 0:
            continue
        ws = bcf.prepare(m, prec)
        ref = bcf.decode(m, ws, dev(qs[k]), prec).cpu().numpy()
        got = out[offsets[k]: offsets[k + 1]]
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), k
    # and sampled rows against the oracle
    bar = 1e-5 if precision == "FP32" else 2e-3
    for k in ((0, 2, 4) if shared_only else (0, 2, 3, 5)):
        pick = np.unique(np.linspace(0, len(qs[k]) - 1, 300).astype(int))
        ref = oracle.decode(host[k], qs[k][pick])
        err = np.abs(out[offsets[k] + pick] - ref).max()
        log(f"batch {precision} material {k}: max abs err {err:.3e}")
        assert err <= bar


@pytest.mark.parametrize("n_pyr", [2, 3])
def test_batch_of_fewer_pyramids_equals_single_decodes(bcf, n_pyr):
    # materials of two or three pyramids (one geometry per material, so the
    # shared-footprint path without the four-pyramid interleaved scratch, and
    # one of differing sizes), 3 * n_pyr MLP inputs
    dims = (3 * n_pyr, 32, 10)
    shapes = [([64] * n_pyr, [7] * n_pyr, 2000, False), ([(128, 32)] * n_pyr, [8] * n_pyr, 777, False),
              ([64, 32, 16][:n_pyr], [7, 6, 5][:n_pyr], 300, False)]
    host, mats, qs, offsets = make_batch(bcf, shapes, seed=67, dims=dims)
    for precision in ("FP16", "FP32"):
        prec = bcf.Precision[precision]
        batch = bcf.Batch(mats, prec)
        batch.unpack()
        out = batch.decode(dev(np.concatenate(qs)), dev(offsets)).cpu().numpy()
        for k, m in enumerate(mats):
            ref = bcf.decode(m, bcf.prepare(m, prec), dev(qs[k]), prec).cpu().numpy()
            assert np.array_equal(out[offsets[k]: offsets[k + 1]].view(np.uint32), ref.view(np.uint32)), (k, precision)
        err = np.abs(out[: offsets[1]] - oracle.decode(host[0], qs[0])).max()
        assert err <= (1e-5 if precision == "FP32" else 2e-3), (precision, err)


def test_batch_offsets_are_clamped_and_uncovered_rows_untouched(bcf):
    host, mats, qs, _ = make_batch(bcf, SHAPES[:3], seed=62)
    batch = bcf.Batch(mats, bcf.Precision.FP16)
    batch.unpack()
    n_total = 5000
    q_all = dev(synth.uniform_queries(n_total, synth.rng(63), 6.0))
    sentinel = torch.full((n_total, DIMS[-1]), float("nan"), device="cuda")
    ws = [bcf.prepare(m, bcf.Precision.FP16) for m in mats]

    def single(k, a, b):
        return bcf.decode(mats[k], ws[k], q_all[a:b], bcf.Precision.FP16).cpu().numpy()

    # material 0 rows 100..1099; material 1 a decreasing pair (empty);
    # material 2 rows 900..3999; rows outside stay untouched
    o = batch.decode(q_all, dev(np.array([100, 1100, 900, 4000], np.int32)), out=sentinel.clone()).cpu().numpy()
    covered = np.zeros(n_total, bool)
    covered[100:1100] = True
    covered[900:4000] = True
    assert np.isnan(o[~covered]).all()
    assert np.array_equal(o[100:900].view(np.uint32), single(0, 100, 900).view(np.uint32))
    assert np.array_equal(o[1100:4000].view(np.uint32), single(2, 1100, 4000).view(np.uint32))
    # an offset far past n_total is clamped to it
    o = batch.decode(q_all, dev(np.array([4000, 4500, 4600, 2 ** 31 - 1], np.int32)),
                     out=sentinel.clone()).cpu().numpy()
    assert np.isnan(o[:4000]).all()
    assert np.array_equal(o[4000:4500].view(np.uint32), single(0, 4000, 4500).view(np.uint32))
    assert np.array_equal(o[4600:].view(np.uint32), single(2, 4600, 5000).view(np.uint32))


@pytest.mark.parametrize("shared_only", [False, True])
def test_batch_plans_agree_and_tuner_returns_one(bcf, shared_only):
    host, mats, qs, offsets = make_batch(bcf, SHARED_SHAPES if shared_only else SHAPES, seed=64)
    batch = bcf.Batch(mats, bcf.Precision.FP16)
    batch.unpack()
    q_all, offs = dev(np.concatenate(qs)), dev(offsets)
    ref = batch.decode(q_all, offs).cpu().numpy()
    for plan in ((8, 0), (8, 1), (256, 0), (4096, 1), (1000, 0), (8, 1, 4, 2), (512, 1, 2, 2), (64, 0, 1, 2),
                 (3000, 1, 64, 4), (16, 1, 3, 4)):
        got = batch.decode(q_all, offs, plan=plan).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), plan
    plan, ms = batch.tune(q_all, offs)
    log(f"tuned plan {plan}: {ms:.4f} ms")
    workgroups, interleave, run, waves = plan
    assert waves in (2, 4) and workgroups * waves in (1024, 2048, 4096, 8192, 16384) and ms > 0
    assert (interleave, run) in ((0, 1), (1, 1), (1, 2), (1, 4))
    got = batch.decode(q_all, offs, plan=plan).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def special_queries(n, g, top):
    """Uniform queries with wrap, clamp and NaN cases mixed in."""
    q = synth.uniform_queries(n, g, top)
    k = min(n, 12)
    q[:k] = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, top], [-0.25, 1.75, -3.0], [0.999999, 0.5, 99.0],
                      [0.5, 0.0, 0.5], [3.5, -2.25, 1.0], [np.nan, 0.5, 1.0], [0.5, 0.5, np.nan],
                      [0.0, 0.999, top + 0.5], [1e-7, 1e-7, 0.999], [0.75, 0.125, 2.5], [0.5, 0.5, 0.0]],
                     np.float32)[:k]
    return q


@pytest.mark.parametrize("precision", ["FP16", "FP32"])
def test_touched_unpack_equals_full_unpack(bcf, precision):
    # a workspace of all-ones bytes: every texel the touched unpack leaves
    # alone is a NaN half, so a decode that read one would not match
    host, mats, qs, offsets = make_batch(bcf, seed=68)
    g = synth.rng(69)
    qs = [special_queries(len(q), g, float(max(levels) - 1)) for q, (_, levels, _, _) in zip(qs, SHAPES)]
    prec = bcf.Precision[precision]
    batch = bcf.Batch(mats, prec, ws_fill=0xFF)
    q_all, offs = dev(np.concatenate(qs)), dev(offsets)
    batch.unpack_touched(q_all, offs)
    out = batch.decode(q_all, offs).cpu().numpy()
    for k, m in enumerate(mats):
        if len(qs[k]) == 0:
            continue
        ref = bcf.decode(m, bcf.prepare(m, prec), dev(qs[k]), prec).cpu().numpy()
        got = out[offsets[k]: offsets[k + 1]]
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), k
    # a second, smaller set of queries after the first
    qs2 = [q[: len(q) // 3] for q in qs]
    offsets2 = np.concatenate([[0], np.cumsum([len(q) for q in qs2])]).astype(np.int32)
    q2 = dev(np.concatenate(qs2))
    batch.unpack_touched(q2, dev(offsets2))
    out2 = batch.decode(q2, dev(offsets2)).cpu().numpy()
    assert np.array_equal(out2.view(np.uint32), out[np.concatenate(
        [np.arange(offsets[k], offsets[k] + len(qs2[k])) for k in range(len(qs))])].view(np.uint32))
    log(f"touched unpack {precision}: every material equals its single decode")


def test_touched_unpack_with_clamped_offsets(bcf):
    host, mats, qs, _ = make_batch(bcf, SHAPES[:3], seed=70)
    batch = bcf.Batch(mats, bcf.Precision.FP16, ws_fill=0xFF)
    n_total = 5000
    q_all = dev(synth.uniform_queries(n_total, synth.rng(71), 6.0))
    ws = [bcf.prepare(m, bcf.Precision.FP16) for m in mats]
    offs = dev(np.array([100, 1100, 900, 2 ** 31 - 1], np.int32))
    batch.unpack_touched(q_all, offs)
    o = batch.decode(q_all, offs).cpu().numpy()
    ref0 = bcf.decode(mats[0], ws[0], q_all[100:900], bcf.Precision.FP16).cpu().numpy()
    ref2 = bcf.decode(mats[2], ws[2], q_all[1100:5000], bcf.Precision.FP16).cpu().numpy()
    assert np.array_equal(o[100:900].view(np.uint32), ref0.view(np.uint32))
    assert np.array_equal(o[1100:5000].view(np.uint32), ref2.view(np.uint32))


def test_batch_graph_capture_replays(bcf):
    host, mats, qs, offsets = make_batch(bcf, seed=65)
    batch = bcf.Batch(mats, bcf.Precision.FP16)
    q_static = dev(np.concatenate(qs))
    offs = dev(offsets)
    out_static = torch.empty((q_static.shape[0], DIMS[-1]), device="cuda")
    batch.unpack()
    batch.decode(q_static, offs, out=out_static)            # warm-up outside capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            batch.unpack()
            batch.decode(q_static, offs, out=out_static)
    torch.cuda.synchronize()
    # the touched unpack in a graph of its own, on a workspace of all-ones bytes
    tbatch = bcf.Batch(mats, bcf.Precision.FP16, ws_fill=0xFF)
    tout = torch.empty_like(out_static)
    tbatch.unpack_touched(q_static, offs)
    tbatch.decode(q_static, offs, out=tout)
    torch.cuda.synchronize()
    tgraph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(tgraph, stream=side):
            tbatch.unpack_touched(q_static, offs)
            tbatch.decode(q_static, offs, out=tout)
    torch.cuda.synchronize()
    g = synth.rng(66)
    a = torch.randn(512, 512, device="cuda")
    for replay in range(4):
        fresh = dev(synth.uniform_queries(q_static.shape[0], g, 6.0))
        q_static.copy_(fresh)
        b = a @ a                                           # eager work between replays
        graph.replay()
        tgraph.replay()
        torch.cuda.synchronize()
        eager = batch.decode(fresh, offs).cpu().numpy()
        assert np.array_equal(out_static.cpu().numpy().view(np.uint32), eager.view(np.uint32)), replay
        assert np.array_equal(tout.cpu().numpy().view(np.uint32), eager.view(np.uint32)), replay
        assert torch.isfinite(b).all()
    log("graph: 4 replays equal the eager decode (full and touched unpack)")
