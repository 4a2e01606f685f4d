"""GPU tests of the decode over coherent image queries: a perspective ground
plane at several texture scales (the plane wraps, magnifies, and minifies
down to levels of one or two texels), with one to four pyramids of a shared
geometry, unsigned and signed. The same queries are decoded as an image
(16x4 tiles), as runs of 64 consecutive queries, and in shuffled order with
no image structure: the three must be bit-identical (the order in which work
items visit the queries does not change any result), and sampled rows must
match the FP64 oracle (FP32 <= 1e-5, FP16 <= 2e-3 on bounded blocks)."""
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


def plane(width, height, res, scale, s_shift):
    """Perspective ground-plane queries with u, v scaled by `scale` (wrapping)
    and s shifted by `s_shift` (clamped at 0 by the decoder)."""
    q = synth.perspective_queries(width, height, res, s_max=20.0).astype(np.float64)
    q[:, 0] = (q[:, 0] * scale) % 1.0
    q[:, 1] = (q[:, 1] * scale) % 1.0
    q[:, 2] = q[:, 2] + np.log2(scale) + s_shift
    q = q.astype(np.float32)
    q[:, :2][q[:, :2] >= 1.0] = 0.0
    return q


CASES = [
    # (n pyramids, base resolution, levels, image width, height, uv scale, s shift, signed)
    (4, 256, 9, 640, 360, 1.0, 0.0, False),       # about a texel per pixel, LOD 0..5
    (4, 256, 9, 333, 97, 3.0, 0.0, False),        # the plane wraps three times; ragged tiles
    (4, 256, 9, 320, 180, 0.25, -2.0, False),     # magnified: level 0 only (s clamped)
    (4, 256, 9, 200, 120, 1.0, 6.0, False),       # minified to the last levels (2x2, 1x1 texels)
    (2, 128, 8, 256, 128, 1.0, 0.0, False),       # two pyramids
    (1, 512, 10, 300, 200, 2.0, 0.0, False),      # one pyramid
    (3, 256, 9, 256, 144, 1.0, 0.0, True),        # three signed pyramids
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-{c[3]}x{c[4]}-s{c[5]}-{c[6]}" for c in CASES])
def test_image_runs_and_shuffled_orders_agree_with_each_other_and_the_oracle(bcf, case):
    n_pyr, res, levels, width, height, scale, shift, signed = case
    dims = (3 * n_pyr, 32, 32, 10)
    g = synth.rng(700 + n_pyr + res)
    texs = [synth.bounded_blocks(synth.chain_blocks(res, res, levels), g, signed=signed).reshape(-1)
            for _ in range(n_pyr)]
    params = synth.mlp_params(dims, g)
    host = oracle.Material(texs, [res] * n_pyr, [levels] * n_pyr, dims, params, [0.0] * n_pyr, signed)
    mat = bcf.Material.from_host(texs, [res] * n_pyr, [levels] * n_pyr, dims, params, signed=signed)
    q = plane(width, height, res, scale, shift)
    n = len(q)
    perm = synth.rng(701).permutation(n)
    pick = np.unique(np.concatenate([np.linspace(0, n - 1, 1500).astype(np.int64), [0, n - 1]]))
    ref = oracle.decode(host, q[pick])
    for precision, bar in (("FP32", 1e-5), ("FP16", 2e-3)):
        prec = bcf.Precision[precision]
        ws = bcf.prepare(mat, prec)
        image = bcf.decode(mat, ws, dev(q), prec, grid_width=width).cpu().numpy()
        runs = bcf.decode(mat, ws, dev(q), prec).cpu().numpy()              # 64 consecutive queries per item
        shuffled = bcf.decode(mat, ws, dev(q[perm]), prec).cpu().numpy()
        assert np.array_equal(image.view(np.uint32), runs.view(np.uint32)), precision
        assert np.array_equal(image[perm].view(np.uint32), shuffled.view(np.uint32)), precision
        err = np.abs(image[pick] - ref).max()
        print(f"{case} {precision}: max abs err {err:.3e}", flush=True)
        assert err <= bar
