"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars:
  * BC6H halves: bit-exact (integer work).
  * FP32 decode: |gpu - oracle| <= 1e-5 absolute on bounded-feature materials
    (every texel < 1), and <= 1e-5 relative to the row's feature magnitude on
    full-range random blocks.
  * FP32-on-MFMA decode: same bars as FP32.
  * FP16-MFMA decode: max abs error <= 2e-3 on bounded materials.
  * BF16-MFMA decode: max abs error <= 2e-2 on bounded materials (8-bit
    significand; reported, not a paper target).
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def log(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# blocks

@pytest.mark.parametrize("signed", [False, True])
def test_decode_blocks_bit_exact(bcf, signed):
    g = synth.rng(50 + signed)
    blocks = np.concatenate([synth.random_mode_blocks(200000, g), synth.reserved_blocks(5000, g),
                             synth.bounded_blocks(20000, g), synth.random_mode_blocks(77, g)])
    log(f"decode_blocks signed={signed} n={len(blocks)}")
    got = bcf.decode_blocks(dev(blocks), signed=signed).cpu().numpy().view(np.uint16)
    ref = oracle.decode_blocks(blocks, signed)
    assert np.array_equal(got, ref)


def test_decode_blocks_empty_and_one(bcf):
    out = bcf.decode_blocks(torch.zeros((0, 16), dtype=torch.uint8, device="cuda"))
    assert out.shape == (0, 16, 3)
    g = synth.rng(3)
    b = synth.random_mode_blocks(1, g)
    got = bcf.decode_blocks(dev(b)).cpu().numpy().view(np.uint16)
    assert np.array_equal(got, oracle.decode_blocks(b))


# ---------------------------------------------------------------------------
# whole decode

def make(res, levels, dims, variant, n_tex=4, seed=1, bias=None, modes=synth.ALL_MODES, signed=False):
    g = synth.rng(seed)
    if isinstance(res, int):
        res = [res] * n_tex
    sizes = [(r, r) if isinstance(r, int) else r for r in res]
    lv = levels if isinstance(levels, list) else [levels] * n_tex
    texs = []
    for (w, h), L in zip(sizes, lv):
        n = synth.chain_blocks(w, h, L)
        if variant == "R":
            blk = synth.random_mode_blocks(n, g, modes)
        else:
            blk = synth.bounded_blocks(n, g, modes, signed=signed)
        texs.append(blk.reshape(-1))
    params = synth.mlp_params(dims, synth.rng(seed + 1))
    bias = bias or [0.0] * n_tex
    host = oracle.Material(texs, sizes, lv, dims, params, bias, signed)
    return texs, sizes, lv, params, bias, host


def run_gpu(bcf, texs, sizes, lv, dims, params, bias, q, precision, grid_width=0, signed=False):
    mat = bcf.Material.from_host(texs, sizes, lv, dims, params, bias, signed)
    ws = bcf.prepare(mat, precision)
    out = bcf.decode(mat, ws, dev(q), precision, grid_width)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def check(bcf, texs, sizes, lv, dims, params, bias, host, q, precision, atol, rel=False, grid_width=0,
          signed=False):
    got = run_gpu(bcf, texs, sizes, lv, dims, params, bias, q, precision, grid_width, signed)
    ref = oracle.decode(host, q)
    err = np.abs(got - ref)
    if rel:
        scale = np.maximum(1.0, np.abs(oracle.sample(host, q)).max(axis=1))[:, None]
        err = err / scale
    log(f"  {precision!r}: max err {err.max():.3e} (bar {atol:g}{' rel' if rel else ''})")
    assert np.isfinite(got).all()
    assert err.max() <= atol
    return got, ref


@pytest.mark.parametrize("precision,atol", [("FP32", 1e-5), ("FP32_MFMA", 1e-5), ("FP16", 2e-3),
                                            ("BF16", 2e-2)])
def test_tiny_workload_bounded(bcf, precision, atol):
    # 4 x 256^2 pyramids (9 levels), MLP 12-16-16-9, 65,536 uniform queries,
    # plus a ragged tail (65,536 + 77)
    texs, sizes, lv, params, bias, host = make(256, 9, (12, 16, 16, 9), "B")
    q = synth.uniform_queries(65536 + 77, synth.rng(3), 8.0)
    log(f"tiny bounded {precision}")
    check(bcf, texs, sizes, lv, (12, 16, 16, 9), params, bias, host, q, bcf.Precision[precision], atol)


@pytest.mark.parametrize("precision", ["FP32", "FP32_MFMA"])
def test_tiny_workload_random_modes_full_range(bcf, precision):
    texs, sizes, lv, params, bias, host = make(256, 9, (12, 16, 16, 9), "R")
    q = synth.uniform_queries(65536, synth.rng(3), 8.0)
    log(f"tiny R {precision}")
    check(bcf, texs, sizes, lv, (12, 16, 16, 9), params, bias, host, q, bcf.Precision[precision], 1e-5,
          rel=True)


@pytest.mark.parametrize("dims", [(12, 32, 32, 10), (12, 64, 64, 10), (12, 16, 4), (12, 20, 7, 33, 16)])
@pytest.mark.parametrize("precision,atol", [("FP32", 1e-5), ("FP16", 2e-3), ("FP32_MFMA", 1e-5)])
def test_mlp_shapes(bcf, dims, precision, atol):
    texs, sizes, lv, params, bias, host = make(64, 7, dims, "B", seed=11)
    q = synth.uniform_queries(4099, synth.rng(5), 7.0)
    log(f"mlp {dims} {precision}")
    check(bcf, texs, sizes, lv, dims, params, bias, host, q, bcf.Precision[precision], atol)


@pytest.mark.parametrize("precision,atol", [("FP32", 1e-5), ("FP16", 2e-3)])
def test_fewer_textures_non_square_bias_small_levels(bcf, precision, atol):
    # 3 pyramids: 64x16 (7 levels, down to 1x1), 8x32 (6), 4x4 (3); biases
    dims = (9, 16, 16, 5)
    texs, sizes, lv, params, bias, host = make([(64, 16), (8, 32), (4, 4)], [7, 6, 3], dims, "B",
                                               n_tex=3, seed=21, bias=[0.0, -0.75, 1.5])
    g = synth.rng(6)
    q = synth.uniform_queries(3001, g, 8.0)
    q[:500, :2] += g.integers(-3, 4, size=(500, 2)).astype(np.float32)     # whole periods
    q[500:600, 2] = -2.0                                                      # below level 0
    q[600:700, 2] = 30.0                                                      # above the top level
    log(f"mixed pyramids {precision}")
    check(bcf, texs, sizes, lv, dims, params, bias, host, q, bcf.Precision[precision], atol)


@pytest.mark.parametrize("rw,rh,L", [(32, 32, 6), (256, 64, 9)])
def test_texel_centres_reproduce_texels_on_gpu(bcf, rw, rh, L):
    # FP32 path with an identity MLP 3 -> 3 -> 3 (identity weights, zero
    # biases; the ReLU passes the non-negative UF16 features): outputs are the
    # filtered features, and at texel centres of integer levels the texels.
    # 256 x 64: levels of several unpack workgroups, block rows of 64 blocks,
    # and levels 2, 1 and 1 texel high under wider ones.
    g = synth.rng(9)
    tex = synth.bounded_blocks(synth.chain_blocks(rw, rh, L), g).reshape(-1)
    eye = np.concatenate([np.eye(3).ravel(), np.zeros(3)])
    params = np.concatenate([eye, eye]).astype(np.float32)
    host = oracle.Material([tex], [(rw, rh)], [L], (3, 3, 3), params)
    qs = []
    for l in range(L):
        w, h = max(rw >> l, 1), max(rh >> l, 1)
        jj, ii = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        qs.append(np.stack([(ii + 0.5) / w, (jj + 0.5) / h, np.full(ii.shape, l)], -1).reshape(-1, 3))
    q = np.concatenate(qs).astype(np.float32)
    got = run_gpu(bcf, [tex], [(rw, rh)], [L], (3, 3, 3), params, [0.0], q, bcf.Precision.FP32)
    assert np.array_equal(got, oracle.sample(host, q))


def test_empty_query_set(bcf):
    texs, sizes, lv, params, bias, host = make(16, 5, (12, 16, 10), "B")
    mat = bcf.Material.from_host(texs, sizes, lv, (12, 16, 10), params, bias)
    ws = bcf.prepare(mat, bcf.Precision.FP16)
    out = bcf.decode(mat, ws, torch.zeros((0, 3), device="cuda"), bcf.Precision.FP16)
    torch.cuda.synchronize()
    assert out.shape == (0, 10)


def test_non_finite_queries_are_memory_safe(bcf):
    texs, sizes, lv, params, bias, host = make(32, 6, (12, 16, 10), "B")
    q = synth.uniform_queries(1000, synth.rng(8), 6.0)
    q[::7, 0] = np.nan
    q[1::7, 1] = np.inf
    q[2::7, 2] = np.nan
    q[3::7, 0] = -np.inf
    q[4::7, 2] = np.inf
    q[5::7, :2] = 3.0e38
    for p in ("FP32", "FP16"):
        got = run_gpu(bcf, texs, sizes, lv, (12, 16, 10), params, bias, q, bcf.Precision[p])
        ok = np.isfinite(q).all(axis=1) & (np.abs(q[:, :2]) < 1e6).all(axis=1)
        ref = oracle.decode(host, q[ok])
        assert np.abs(got[ok] - ref).max() <= (1e-5 if p == "FP32" else 2e-3)


@pytest.mark.parametrize("precision,atol", [("FP32", 1e-5), ("FP16", 2e-3), ("FP32_MFMA", 1e-5)])
def test_signed_pyramids(bcf, precision, atol):
    # BC6H_SF16 pyramids with texels in (-1, 1)
    dims = (12, 32, 32, 10)
    texs, sizes, lv, params, bias, host = make(128, 8, dims, "B", seed=31, signed=True)
    q = synth.uniform_queries(20011, synth.rng(7), 8.0)
    log(f"signed {precision}")
    check(bcf, texs, sizes, lv, dims, params, bias, host, q, bcf.Precision[precision], atol, signed=True)


# ---------------------------------------------------------------------------
# fp8 (OCP e4m3, per-layer weight scales, static activation scales from a
# calibration batch)

def test_fp8_tracks_the_oracle(bcf):
    dims = (12, 32, 32, 10)
    texs, sizes, lv, params, bias, host = make(128, 8, dims, "B", seed=41)
    mat = bcf.Material.from_host(texs, sizes, lv, dims, params, bias)
    calib = synth.uniform_queries(50000, synth.rng(42), 8.0)
    absmax = bcf.calibrate(mat, dev(calib))
    torch.cuda.synchronize()
    a = absmax.cpu().numpy()
    # the calibration's layer-0 maximum is the largest filtered feature seen
    feats = oracle.sample(host, calib)
    assert abs(a[0] - np.abs(feats).max()) <= 1e-5
    assert (a > 0).all()
    mat.set_act_absmax(absmax)
    ws = bcf.prepare(mat, bcf.Precision.FP8)
    q = synth.uniform_queries(20000, synth.rng(43), 8.0)
    got = bcf.decode(mat, ws, dev(q), bcf.Precision.FP8).cpu().numpy().astype(np.float64)
    ref = oracle.decode(host, q)
    err = np.abs(got - ref)
    scale = np.abs(ref).max()
    log(f"fp8: max abs err {err.max():.3e}, mean {err.mean():.3e}, output scale {scale:.3f}")
    assert np.isfinite(got).all()
    # e4m3 keeps 3 significand bits: errors of a few percent of the output range
    assert err.mean() <= 0.02 * scale
    assert err.max() <= 0.15 * scale


# ---------------------------------------------------------------------------
# the full-frame workload in the launch configuration the benchmark times

def test_full_frame_sampled_outputs(bcf):
    wl = synth.WORKLOADS["frame4k"]
    m = synth.workload_material(wl, variant="B")
    q = synth.workload_queries(wl)
    host = oracle.Material.from_synth(m)
    mat = bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params)
    qd = dev(q)
    pick = np.sort(synth.rng(77).choice(len(q), size=20000, replace=False))
    # include the frame's first and last rows and the last query
    pick = np.unique(np.concatenate([pick, np.arange(64), np.arange(len(q) - 64, len(q))]))
    ref = oracle.decode(host, q[pick])
    for p, bar in (("FP32", 1e-5), ("FP16", 2e-3), ("FP32_MFMA", 1e-5), ("BF16", 2e-2)):
        prec = bcf.Precision[p]
        ws = bcf.prepare(mat, prec)
        bcf.unpack(mat, ws)                  # the two calls the benchmark times
        out = bcf.decode_unpacked(mat, ws, qd, prec, grid_width=3840)
        got = out[torch.from_numpy(pick).cuda()].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref).max()
        log(f"frame4k {p}: max abs err {err:.3e} on {len(pick)} sampled queries")
        assert err <= bar
        del ws, out


def test_unpack_then_decode_unpacked_equals_decode(bcf):
    texs, sizes, lv, params, bias, host = make(64, 7, (12, 32, 32, 10), "B", seed=21)
    q = synth.uniform_queries(5000, synth.rng(22), 6.0)
    mat = bcf.Material.from_host(texs, sizes, lv, (12, 32, 32, 10), params, bias)
    qd = dev(q)
    for p in ("FP32", "FP16"):
        prec = bcf.Precision[p]
        ws = bcf.prepare(mat, prec)
        whole = bcf.decode(mat, ws, qd, prec).cpu().numpy()
        ws2 = bcf.prepare(mat, prec)
        ws2.fill_(0xFF)                      # garbage everywhere, then prepare again
        ws2.copy_(bcf.prepare(mat, prec))
        bcf.unpack(mat, ws2)
        a = bcf.decode_unpacked(mat, ws2, qd, prec).cpu().numpy()
        b = bcf.decode_unpacked(mat, ws2, qd[:1234], prec).cpu().numpy()   # one unpack, two decodes
        assert np.array_equal(whole.view(np.uint32), a.view(np.uint32))
        assert np.array_equal(whole[:1234].view(np.uint32), b.view(np.uint32))
    # unpack takes no precision: its texels sit where every precision's layout reads them
    ws16 = bcf.prepare(mat, bcf.Precision.FP16)
    bcf.unpack(mat, ws16)
    got = bcf.decode_unpacked(mat, ws16, qd, bcf.Precision.FP16).cpu().numpy().astype(np.float64)
    assert np.abs(got - oracle.decode(host, q)).max() <= 2e-3


def test_workspace_prepared_for_another_precision_or_material_is_rejected(bcf):
    # bcf_prepare tags the workspace (host record and device header): a
    # decode at another precision, or of another material, is an argument
    # error before any launch
    texs, sizes, lv, params, bias, host = make(32, 6, (12, 16, 9), "B", seed=23)
    mat = bcf.Material.from_host(texs, sizes, lv, (12, 16, 9), params, bias)
    other = bcf.Material.from_host(texs, sizes, lv, (12, 16, 9), params, bias)   # same geometry, other buffers
    qd = dev(synth.uniform_queries(100, synth.rng(24), 5.0))
    ws = bcf.prepare(mat, bcf.Precision.FP16)
    header = ws[:48].cpu().numpy()
    assert bytes(header[:4]) == b"BCFW" and header[8:12].view(np.uint32)[0] == int(bcf.Precision.FP16)
    bcf.decode(mat, ws, qd, bcf.Precision.FP16)
    with pytest.raises(bcf.BcfError, match="precision"):
        bcf.decode(mat, ws, qd, bcf.Precision.FP32)
    with pytest.raises(bcf.BcfError, match="another material"):
        bcf.decode(other, ws, qd, bcf.Precision.FP16)
    with pytest.raises(bcf.BcfError, match="another material"):
        bcf.unpack(other, ws)
    # preparing again re-tags it
    ws2 = bcf.prepare(other, bcf.Precision.FP32)
    a = bcf.decode(other, ws2, qd, bcf.Precision.FP32).cpu().numpy()
    assert np.abs(a - oracle.decode(host, qd.cpu().numpy())).max() <= 1e-5


@pytest.mark.parametrize("dims", [(12, 32, 32, 10), (12, 16, 9)])
def test_grid_width_does_not_change_results(bcf, dims):
    # 16x4 tiles over images with ragged right and bottom edges, widths that
    # are and are not multiples of 16 (and narrower than a tile), rows whose
    # byte length is and is not a multiple of 16 (16-byte and 4-byte stores),
    # against the plain run of consecutive queries
    texs, sizes, lv, params, bias, host = make(64, 7, dims, "B", seed=31)
    mat = bcf.Material.from_host(texs, sizes, lv, dims, params, bias)
    g = synth.rng(32)
    # (53, 64 and 37 columns: 10, 16 and 34 tile rows, strips of 1, 2 and 4
    # tile rows per XCD; 256, 270 and 999 columns: fewer tile rows than XCDs,
    # items round-robin)
    for n, width in ((53 * 37 + 17, 53), (4096, 64), (3000, 8), (999, 999), (5000, 37), (70, 9),
                     (256 * 20, 256), (270 * 9 + 5, 270)):
        q = synth.uniform_queries(n, g, 6.0)
        qd = dev(q)
        for p in ("FP32", "FP16"):
            prec = bcf.Precision[p]
            ws = bcf.prepare(mat, prec)
            flat = bcf.decode(mat, ws, qd, prec).cpu().numpy()
            tiled = bcf.decode(mat, ws, qd, prec, grid_width=width).cpu().numpy()
            assert np.array_equal(flat.view(np.uint32), tiled.view(np.uint32)), (n, width, p)


@pytest.mark.parametrize("dims", [(12, 32, 32, 10), (12, 16, 9)])
def test_output_view_writes_only_its_rows(bcf, dims):
    # `out` a view into a larger NaN-filled buffer, at offsets that keep and
    # that break 16-byte alignment: the decode writes exactly its own rows
    # (the dropped out-of-range stores of partial work items never land past
    # the view) and equals the decode into a fresh buffer
    texs, sizes, lv, params, bias, host = make(64, 7, dims, "B", seed=33)
    mat = bcf.Material.from_host(texs, sizes, lv, dims, params, bias)
    g = synth.rng(34)
    c = dims[-1]
    for n, width, lead in ((4096, 64, 4), (53 * 37 + 17, 53, 1), (1000, 0, 3), (1000, 0, 4), (1001, 0, 2),
                           (999, 999, 8)):
        q = dev(synth.uniform_queries(n, g, 6.0))
        for p in ("FP32", "FP16"):
            prec = bcf.Precision[p]
            ws = bcf.prepare(mat, prec)
            ref = bcf.decode(mat, ws, q, prec, grid_width=width).cpu().numpy()
            big = torch.full((lead + n + 70, c), float("nan"), device="cuda")
            bcf.decode(mat, ws, q, prec, grid_width=width, out=big[lead: lead + n])
            got = big.cpu().numpy()
            assert np.isnan(got[:lead]).all() and np.isnan(got[lead + n:]).all(), (n, width, lead, p)
            assert np.array_equal(got[lead: lead + n].view(np.uint32), ref.view(np.uint32)), (n, width, lead, p)


def test_query_counts_beyond_one_launch(bcf):
    # One launch takes at most 2^25 queries (32-bit byte offsets: 2^25 rows of
    # 16 fp32 outputs are 2 GiB). 2^25 + 4097 queries with 16 outputs run as
    # a launch of exactly that maximum and a ragged one: sampled rows on both
    # sides of the boundary against the oracle, and the whole call bit-equal
    # to the two halves decoded on their own and to the call with a declared
    # image width (too many queries for tiles: the same runs)
    dims = (12, 16, 16, 16)
    texs, sizes, lv, params, bias, host = make(256, 9, dims, "B", seed=41)
    mat = bcf.Material.from_host(texs, sizes, lv, dims, params, bias)
    n0 = 1 << 25
    n = n0 + 4097
    q = synth.uniform_queries(n, synth.rng(42), 8.0)
    qd = dev(q)
    pick = np.unique(np.concatenate([synth.rng(43).choice(n, size=3000, replace=False),
                                     np.arange(64), np.arange(n0 - 70, n0 + 70), np.arange(n - 70, n)]))
    ref = oracle.decode(host, q[pick])
    pick_d = torch.from_numpy(pick).cuda()
    for p, bar in (("FP32", 1e-5), ("FP16", 2e-3)):
        prec = bcf.Precision[p]
        ws = bcf.prepare(mat, prec)
        log(f"{p}: {n} queries")
        whole = bcf.decode(mat, ws, qd, prec)
        got = whole[pick_d].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref).max()
        log(f"  max abs err {err:.3e} on {len(pick)} sampled queries")
        assert np.isfinite(got).all() and err <= bar
        head = bcf.decode(mat, ws, qd[:n0], prec)
        assert torch.equal(whole[:n0].view(torch.int32), head.view(torch.int32))
        del head
        tail = bcf.decode(mat, ws, qd[n0:], prec)
        assert torch.equal(whole[n0:].view(torch.int32), tail.view(torch.int32))
        tiled = bcf.decode(mat, ws, qd, prec, grid_width=4096)
        assert torch.equal(tiled.view(torch.int32), whole.view(torch.int32))
        del ws, whole, tail, tiled
        torch.cuda.empty_cache()
