"""GPU parity of the training-time decode (bcf_train_forward / bcf_train_backward)
against the FP64 oracle of oracle/train.py, finite differences on the
continuous path, and the straight-through forward against the product decode
of the exported blocks.

Bars:
  * forward: |gpu - oracle| <= 1e-5 absolute (features below 1: endpoints in [0, 31]).
  * gradients: |gpu - oracle| <= 2e-4 * max|oracle| per tensor (binary32 with
    float-atomic sums against binary64), excluding in continuous mode the
    blocks with a texel within 0.05 of a step of eq. (8)'s slope.
  * finite differences (continuous mode, binary32 forward, fp64 sums):
    within 3% of the analytic derivatives, per block-parameter coordinate and
    along directions in the MLP parameters. The loss is piecewise linear (ReLU,
    eq. (8)), so a step that crosses a ReLU kink of one of the queries the
    block feeds moves the difference quotient by up to about a percent; the
    exact check is the one against the binary64 oracle above.
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


def problem(seed, res=32, levels=6, n=3000, dims=(12, 32, 32, 10), ste=False, n_tex=4, e_hi=31.0):
    g = synth.rng(seed)
    sizes = [res if isinstance(res, int) else res[i] for i in range(n_tex)]
    texs = []
    for i in range(n_tex):
        w, h = (sizes[i], sizes[i]) if isinstance(sizes[i], int) else sizes[i]
        nb = synth.chain_blocks(w, h, levels)
        texs.append(T.TrainTexture(w, h, levels,
                                   endpoints=g.uniform(0.0, e_hi, (nb, 4, 3)).astype(np.float32),
                                   indices=g.uniform(0.0, 1.0, (nb, 16)).astype(np.float32),
                                   partitions=g.integers(0, 32, nb).astype(np.uint8),
                                   lod_bias=0.0))
    params = synth.mlp_params(dims, g).astype(np.float32)
    q = synth.uniform_queries(n, g, levels - 1.0)
    go = g.standard_normal((n, dims[-1])).astype(np.float32)
    return texs, dims, params, q, go


def to_gpu(bcf, texs, dims, params, ste):
    geo = bcf.TrainGeometry([(t.width, t.height) for t in texs], [t.levels for t in texs],
                            [dev(t.partitions) for t in texs], dims, [t.lod_bias for t in texs],
                            straight_through=ste)
    ends = [dev(t.endpoints) for t in texs]
    idxs = [dev(t.indices) for t in texs]
    return geo, ends, idxs, dev(params)


@pytest.mark.parametrize("ste", [False, True])
def test_forward_matches_oracle(bcf, ste):
    texs, dims, params, q, _ = problem(401 + ste, ste=ste)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, ste)
    got = bcf.train_forward(geo, ends, idxs, p, dev(q)).cpu().numpy().astype(np.float64)
    ref = T.forward(texs, dims, params, q, ste).detach().numpy()
    err = np.abs(got - ref).max()
    log(f"train forward ste={ste}: max abs err {err:.3e}")
    assert err <= 1e-5


def kink_blocks(tex):
    y = T.continuous_y(tex)
    d = np.abs((y - 1.0) / 1024.0 - np.round((y - 1.0) / 1024.0)) * 1024.0
    return (d < 0.05).any(axis=(1, 2))


@pytest.mark.parametrize("ste", [False, True])
@pytest.mark.parametrize("shape", [dict(dims=(12, 32, 32, 10)), dict(dims=(12, 16, 9)),
                                   dict(dims=(6, 16, 16, 16, 4), n_tex=2, res=(32, 64)),
                                   dict(dims=(12, 32, 32, 32, 10), levels=4)])
def test_gradients_match_oracle(bcf, ste, shape):
    kw = dict(shape)
    if "res" in kw and isinstance(kw["res"], tuple):
        kw["res"] = [kw["res"][i % 2] for i in range(kw.get("n_tex", 4))]
    texs, dims, params, q, go = problem(411 + ste, ste=ste, **kw)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, ste)
    g_end, g_idx, g_par = bcf.train_backward(geo, ends, idxs, p, dev(q), dev(go))
    torch.cuda.synchronize()
    _, r_end, r_idx, r_par = T.gradients(texs, dims, params, q, go, ste)

    def close(name, got, ref, keep=None):
        got = got.cpu().numpy().astype(np.float64)
        if keep is not None:
            got, ref = got[keep], ref[keep]
        scale = max(np.abs(ref).max(), 1e-30)
        err = np.abs(got - ref).max() / scale
        log(f"  ste={ste} dims={dims} {name}: max err {err:.2e} of max |grad| {scale:.3e}")
        assert err <= 2e-4, name

    close("params", g_par, r_par)
    for t in range(len(texs)):
        keep = None if ste else ~kink_blocks(texs[t])
        close(f"endpoints[{t}]", g_end[t], r_end[t], keep)
        close(f"indices[{t}]", g_idx[t], r_idx[t], keep)


def test_continuous_finite_differences(bcf):
    # eq. (8) as printed is exact at integer y but steps by half a unit of the
    # half's last place at y = 1024 k + 1 between integers, so the differences
    # are taken per coordinate on blocks whose texels stay clear of those
    # points, and along a direction in the (smooth) MLP parameters
    texs, dims, params, q, go = problem(421, n=4000)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, False)
    qd, god = dev(q), dev(go)
    g_end, g_idx, g_par = bcf.train_backward(geo, ends, idxs, p, qd, god)
    g = synth.rng(422)

    def loss(e, x, pp):
        out = bcf.train_forward(geo, e, x, pp, qd)
        return float((out.double() * god.double()).sum())

    def clear_blocks(tex, margin):
        y = T.continuous_y(tex)
        d = np.abs((y - 1.0) / 1024.0 - np.round((y - 1.0) / 1024.0)) * 1024.0
        return np.nonzero((d > margin).all(axis=(1, 2)))[0]

    checked = 0
    for trial in range(12):
        t = int(g.integers(len(texs)))
        blocks = clear_blocks(texs[t], 16.0)
        b = int(blocks[g.integers(len(blocks))])
        j, c, k = int(g.integers(4)), int(g.integers(3)), int(g.integers(16))
        # a step moves y by at most a 1024 h (endpoint) or a 31744 h (index): < 16
        for kind, h in (("endpoint", 1e-2), ("index", 1e-3)):
            def bumped(sign):
                e2 = [e.clone() for e in ends]
                x2 = [x.clone() for x in idxs]
                if kind == "endpoint":
                    e2[t][b, j, c] += sign * h
                else:
                    x2[t][b, k] += sign * h
                return loss(e2, x2, p)
            fd = (bumped(1.0) - bumped(-1.0)) / (2 * h)
            an = float(g_end[t][b, j, c] if kind == "endpoint" else g_idx[t][b, k])
            if abs(an) < 1e-3 and abs(fd) < 1e-3:
                continue                        # the block feeds no query
            log(f"{kind} t={t} b={b}: fd {fd:.6e} analytic {an:.6e}")
            assert abs(fd - an) <= 0.03 * abs(an) + 2e-4
            checked += 1
    assert checked >= 8
    for trial in range(3):
        # every weight moves at once: a small step keeps the number of ReLU
        # kinks crossed (by any of the 4,000 queries) small
        dp = dev(0.05 * g.standard_normal(p.shape).astype(np.float32))
        h = 1e-3
        fd = (loss(ends, idxs, p + h * dp) - loss(ends, idxs, p - h * dp)) / (2 * h)
        an = float((g_par.double() * dp.double()).sum())
        log(f"MLP direction {trial}: fd {fd:.6e} analytic {an:.6e}")
        assert abs(fd - an) <= 0.03 * abs(an)


def test_ste_forward_equals_product_decode_of_exported_blocks(bcf):
    # quantise, export as BC6H mode-10 blocks, decode with bcf_decode (FP32)
    from test_oracle_train import export_block
    texs, dims, params, q, _ = problem(431, res=32, levels=6, n=5000)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, True)
    got = bcf.train_forward(geo, ends, idxs, p, dev(q)).cpu().numpy()
    chains = []
    for t in texs:
        eq = np.clip(np.round(t.endpoints.astype(np.float64)), 0, 63).astype(np.int64)
        iq = np.clip(np.round(np.float32(7) * t.indices), 0, 7).astype(np.int64)
        chains.append(np.concatenate([export_block(eq[i], iq[i], t.partitions[i]) for i in range(len(eq))]))
    mat = bcf.Material.from_host(chains, [(t.width, t.height) for t in texs], [t.levels for t in texs],
                                 dims, params)
    ws = bcf.prepare(mat, bcf.Precision.FP32)
    dec = bcf.decode(mat, ws, dev(q), bcf.Precision.FP32).cpu().numpy()
    err = np.abs(got - dec).max()
    log(f"straight-through forward vs decode of the exported blocks: max abs diff {err:.3e}")
    assert err <= 1e-5


def test_autograd_function_and_a_few_training_steps(bcf):
    texs, dims, params, q, _ = problem(441, res=32, levels=6, n=8192, ste=True)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, True)
    leaves = [e.clone().requires_grad_(True) for e in ends] + [x.clone().requires_grad_(True) for x in idxs]
    pp = p.clone().requires_grad_(True)
    qd = dev(q)
    target = torch.rand((len(q), dims[-1]), device="cuda") * 0.5
    n = len(texs)
    out = bcf.train_decode(geo, leaves[:n], leaves[n:], pp, qd)
    loss = torch.mean((out - target) ** 2)
    loss.backward()
    go = (2.0 / out.numel()) * (out.detach() - target)
    g_end, g_idx, g_par = bcf.train_backward(geo, ends, idxs, p, qd, go)
    assert torch.allclose(pp.grad, g_par, rtol=1e-3, atol=1e-7 * float(g_par.abs().max()))
    for a, b in zip(leaves, g_end + g_idx):
        assert torch.allclose(a.grad, b, rtol=1e-3, atol=1e-6 * float(b.abs().max() + 1e-30))
    # Adam on features and weights lowers the loss (straight-through path)
    opt = torch.optim.Adam([{"params": leaves, "lr": 0.05}, {"params": [pp], "lr": 3e-3}])
    losses = []
    for _ in range(30):
        opt.zero_grad()
        out = bcf.train_decode(geo, leaves[:n], leaves[n:], pp, qd)
        loss = torch.mean((out - target) ** 2)
        loss.backward()
        opt.step()
        losses.append(float(loss))
    log(f"training losses: {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]


def special_train_queries(g, n, s_max):
    """Queries on and around the 64 x 64 cells the backward sorts its samples
    into, wrapped from outside [0, 1), and at the ends of the LOD range."""
    k = g.integers(0, 65, (n, 2)).astype(np.float64) / 64.0
    eps = g.choice([0.0, 1e-7, -1e-7, 3e-5, -3e-5], (n, 2))
    shift = g.choice([0.0, 1.0, -1.0, 7.0, -3.0], (n, 2))
    q = np.empty((n, 3), np.float32)
    q[:, :2] = (k + eps + shift).astype(np.float32)
    q[:, 2] = g.choice([0.0, -1.0, s_max, s_max + 2.0, 0.5, 1.0], n) + g.uniform(0, 1, n) * (g.random(n) < 0.5)
    return q


@pytest.mark.parametrize("res,levels", [(64, 7), (256, 9), ([(128, 32), (32, 128), (64, 64), (128, 128)], 6)])
def test_gradients_on_cell_edges_and_wrapped_queries(bcf, res, levels):
    """The scatter's LDS windows cover a cell's footprint; queries on the cell
    edges, wrapped from far outside [0, 1) and clamped in LOD take the same
    gradients as the oracle (bars as above)."""
    g = synth.rng(451 + levels)
    n_tex = 4
    texs, dims, params, _, _ = problem(452 + levels, res=res, levels=levels, n=10, ste=True)
    q = special_train_queries(g, 4000, levels - 1.0)
    go = g.standard_normal((len(q), dims[-1])).astype(np.float32)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, True)
    g_end, g_idx, g_par = bcf.train_backward(geo, ends, idxs, p, dev(q), dev(go))
    torch.cuda.synchronize()
    _, r_end, r_idx, r_par = T.gradients(texs, dims, params, q, go, True)
    for name, got, ref in [("params", g_par, r_par)] + \
            [(f"endpoints[{t}]", g_end[t], r_end[t]) for t in range(n_tex)] + \
            [(f"indices[{t}]", g_idx[t], r_idx[t]) for t in range(n_tex)]:
        got = got.cpu().numpy().astype(np.float64)
        scale = max(np.abs(ref).max(), 1e-30)
        err = np.abs(got - ref).max() / scale
        log(f"  res={res} {name}: max err {err:.2e} of max |grad| {scale:.3e}")
        assert err <= 2e-4, name


def test_backward_over_several_sort_batches_is_additive(bcf):
    """More than 2^20 samples are sorted and scattered 2^20 at a time; the
    gradient of the whole batch equals the sum of its two parts' gradients."""
    texs, dims, params, q, go = problem(461, res=64, levels=7, n=(1 << 20) + 5000, ste=True)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, True)
    qd, gd = dev(q), dev(go)
    whole = bcf.train_backward(geo, ends, idxs, p, qd, gd)
    a = bcf.train_backward(geo, ends, idxs, p, qd[:1 << 20], gd[:1 << 20])
    b = bcf.train_backward(geo, ends, idxs, p, qd[1 << 20:], gd[1 << 20:])
    torch.cuda.synchronize()
    def flat(r):
        return [*r[0], *r[1], r[2]]
    for w, x, y in zip(flat(whole), flat(a), flat(b)):
        ref = (x + y).double()
        err = float((w.double() - ref).abs().max() / max(float(ref.abs().max()), 1e-30))
        log(f"  additive: max err {err:.2e}")
        assert err <= 2e-4


def test_gradients_when_the_scatter_windows_overflow(bcf):
    """Two 2048^2 pyramids: the scatter's LDS windows of a cell hold every level
    of the first pyramid but not level 0 of the second, whose taps then go
    straight to memory; the gradients still match the oracle (bars as above)."""
    texs, dims, params, q, go = problem(471, res=2048, levels=12, n=1 << 18, dims=(6, 16, 16, 4), ste=True,
                                        n_tex=2)
    geo, ends, idxs, p = to_gpu(bcf, texs, dims, params, True)
    g_end, g_idx, g_par = bcf.train_backward(geo, ends, idxs, p, dev(q), dev(go))
    torch.cuda.synchronize()
    _, r_end, r_idx, r_par = T.gradients(texs, dims, params, q, go, True)
    gp = g_par.cpu().numpy().astype(np.float64)
    assert np.abs(gp - r_par).max() <= 2e-4 * np.abs(r_par).max(), "params"
    # per level: level 0's gradients are far smaller than the coarse levels'
    for t, tex in enumerate(texs):
        ge = g_end[t].cpu().numpy().astype(np.float64)
        gi = g_idx[t].cpu().numpy().astype(np.float64)
        for level, (first, bx, by, _, _) in enumerate(tex.level_blocks()):
            sl = slice(first, first + bx * by)
            for name, a, b in (("endpoints", ge[sl], r_end[t][sl]), ("indices", gi[sl], r_idx[t][sl])):
                scale = np.abs(b).max()
                err = np.abs(a - b).max() / scale if scale > 0 else np.abs(a).max()
                assert err <= 2e-4, (t, level, name, err, scale)
        log(f"  2 x 2048^2 pyramid {t}: block gradients within 2e-4 of each level's max |grad|")
