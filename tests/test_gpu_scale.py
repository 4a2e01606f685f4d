"""GPU parity at the configured sizes of the batched-serving and training
workloads, in the launch configuration bench.py times.

* batch64: 64 materials with base resolution drawn from {512, 1024, 2048,
  4096}^2 (four pyramids each, full chains; the 4096^2 ones use 716 MB
  position-interleaved texel scratches), MLP 12-32-32-10 per material, query
  counts log-uniform in [2^14, 2^22] (54.3M queries), decoded in one launch
  with the autotuned plan. Sampled rows of every material against the FP64
  oracle (FP16 <= 2e-3, FP32 <= 1e-5 absolute), the first and last row of
  every material included, and the largest 4096^2 material's rows against its
  own single-material decode, bit for bit.
* train: four 1024^2 trainable pyramids (11 levels, LOD bias -1 against a
  2048^2 reference), MLP 12-32-32-10, a batch of 2^20 uniform samples. The
  straight-through forward over the whole batch against oracle/train.py
  (<= 1e-5 absolute), the continuous forward likewise, and the gradients:
  MLP parameters within 2e-4 of max |grad|, block parameters per pyramid and
  level within 2e-4 of that level's max |grad| (the fine levels' gradients
  are far smaller than the coarse ones', so each level has its own scale).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import train as T

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


def sample_rows(n, per=320):
    """`per` rows spread over [0, n), the first and the last included."""
    if n == 0:
        return np.zeros(0, np.int64)
    return np.unique(np.concatenate([np.linspace(0, n - 1, per).astype(np.int64), [0, n - 1]]))


def test_batch64_at_configured_scale(bcf):
    spec = synth.batch_spec()
    pool = synth.block_pool()
    host, mats, qs = [], [], []
    for k in range(spec.n_materials):
        m = synth.batch_material(spec, k, pool)
        host.append(oracle.Material.from_synth(m))
        mats.append(bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params))
        qs.append(synth.batch_queries(spec, k))
    offsets = spec.offsets()
    n = int(offsets[-1])
    log(f"batch64: {spec.n_materials} materials, {n} queries, resolutions {sorted(set(spec.res))}")
    assert 4096 in spec.res and n > 5e7
    qd = dev(np.concatenate(qs))
    offs = dev(offsets.astype(np.int32))
    picks = [sample_rows(len(q)) for q in qs]
    refs = [oracle.decode(host[k], qs[k][picks[k]]) for k in range(spec.n_materials)]
    log(f"oracle: {sum(len(p) for p in picks)} sampled rows")
    big = int(np.argmax([len(q) if r == 4096 else -1 for q, r in zip(qs, spec.res)]))
    for precision, bar in (("FP16", 2e-3), ("FP32", 1e-5)):
        prec = bcf.Precision[precision]
        batch = bcf.Batch(mats, prec)
        batch.unpack()
        out = torch.empty((n, spec.dims[-1]), dtype=torch.float32, device="cuda")
        plan, ms = batch.tune(qd, offs, out=out)
        batch.decode(qd, offs, out=out, plan=plan)
        got = out.cpu().numpy()
        worst = 0.0
        for k in range(spec.n_materials):
            err = float(np.abs(got[offsets[k] + picks[k]] - refs[k]).max()) if len(picks[k]) else 0.0
            worst = max(worst, err)
            assert err <= bar, (precision, k, spec.res[k], err)
        log(f"batch64 {precision} plan {plan} ({ms:.3f} ms): max abs err {worst:.3e} over "
            f"{sum(len(p) for p in picks)} rows")
        # the largest 4096^2 material against its own decode
        ws = bcf.prepare(mats[big], prec)
        single = bcf.decode(mats[big], ws, qd[offsets[big]: offsets[big + 1]], prec).cpu().numpy()
        assert np.array_equal(got[offsets[big]: offsets[big + 1]].view(np.uint32), single.view(np.uint32))
        del batch, out, ws
        torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def train_problem():
    dims = (12, 32, 32, 10)
    ends, idxs, parts, L, params = synth.train_problem(1024, dims)
    n = 1 << 20
    q = synth.uniform_queries(n, synth.rng(synth.SEED_QUERIES), float(L))     # s over the 2048^2 chain
    go = synth.rng(77).standard_normal((n, dims[-1])).astype(np.float32)
    texs = [T.TrainTexture(1024, 1024, L, e, x, p, -1.0) for e, x, p in zip(ends, idxs, parts)]
    return texs, dims, params, q, go


def to_gpu(bcf, texs, dims, params, ste):
    geo = bcf.TrainGeometry([(t.width, t.height) for t in texs], [t.levels for t in texs],
                            [dev(t.partitions) for t in texs], dims, [t.lod_bias for t in texs],
                            straight_through=ste)
    return geo, [dev(t.endpoints) for t in texs], [dev(t.indices) for t in texs], dev(params)


def test_train_forward_at_configured_scale_continuous(bcf, train_problem):
    texs, dims, params, q, _ = train_problem
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, False)
    got = bcf.train_forward(geo, ends, idxs, p, dev(q)).cpu().numpy().astype(np.float64)
    ref = T.forward(texs, dims, params, q, False).detach().numpy()
    err = np.abs(got - ref).max()
    log(f"train 4 x 1024^2, 2^20 samples, continuous forward: max abs err {err:.3e}")
    assert err <= 1e-5


def test_train_step_at_configured_scale_straight_through(bcf, train_problem):
    texs, dims, params, q, go = train_problem
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, True)
    qd = dev(q)
    got = bcf.train_forward(geo, ends, idxs, p, qd).cpu().numpy().astype(np.float64)
    g_end, g_idx, g_par = bcf.train_backward(geo, ends, idxs, p, qd, dev(go))
    torch.cuda.synchronize()
    val, r_end, r_idx, r_par = T.gradients(texs, dims, params, q, go, ste=True)
    err = np.abs(got - val).max()
    log(f"train 4 x 1024^2, 2^20 samples, straight-through forward: max abs err {err:.3e}")
    assert err <= 1e-5
    gp = g_par.cpu().numpy().astype(np.float64)
    rel = np.abs(gp - r_par).max() / np.abs(r_par).max()
    log(f"  MLP parameter gradients: max err {rel:.2e} of max |grad|")
    assert rel <= 2e-4
    for t, tex in enumerate(texs):
        ge = g_end[t].cpu().numpy().astype(np.float64)
        gi = g_idx[t].cpu().numpy().astype(np.float64)
        worst = []
        for level, (first, bx, by, _, _) in enumerate(tex.level_blocks()):
            sl = slice(first, first + bx * by)
            for name, a, b in (("endpoints", ge[sl], r_end[t][sl]), ("indices", gi[sl], r_idx[t][sl])):
                scale = np.abs(b).max()
                e = np.abs(a - b).max() / scale if scale > 0 else np.abs(a).max()
                worst.append(e)
                assert e <= 2e-4, (t, level, name, e, scale)
        log(f"  pyramid {t}: block gradients, worst level error {max(worst):.2e} of that level's max |grad|")
