"""bcf_decode_noalloc (the library's own per-GPU workspace) against bcf_decode
with a caller workspace prepared by bcf_prepare: the same kernels, so every
output is bit-identical. Two calls in a row, the second on a smaller material
with fewer queries, so that the second call runs over what the first left in
the shared array; at two precisions and with and without an image width. A
material whose workspace exceeds the array is refused before any launch."""
import numpy as np
import pytest

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


def material(bcf, res, levels, dims, seed):
    m = synth.make_material([res] * 4, [levels] * 4, dims, variant="B", seed_tex=seed, seed_mlp=seed + 1)
    return bcf.Material.from_host(m.textures, m.res, m.levels, m.dims, m.params)


@pytest.mark.parametrize("precision", ["FP16", "FP32"])
def test_noalloc_equals_decode_with_a_prepared_workspace(bcf, precision):
    prec = bcf.Precision[precision]
    cases = [  # (res, levels, dims, queries, grid_width), the second smaller than the first
        (512, 10, (12, 32, 32, 10), 120_000, 400),
        (64, 7, (12, 16, 9), 3_001, 0),
    ]
    for k, (res, levels, dims, n, gw) in enumerate(cases):
        mat = material(bcf, res, levels, dims, 900 + 10 * k)
        q = synth.uniform_queries(n, synth.rng(901 + 10 * k), levels - 1.0)
        qd = dev(q)
        print(f"noalloc {precision} call {k}: {res}^2 x 4, MLP {dims}, {n} queries, grid_width {gw}", flush=True)
        got = bcf.decode_noalloc(mat, qd, prec, grid_width=gw).cpu().numpy()
        ref = bcf.decode(mat, bcf.prepare(mat, prec), qd, prec, grid_width=gw).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (precision, k)


def test_noalloc_refuses_a_material_beyond_its_workspace(bcf):
    # 4 x 2048^2 needs about 180 MB of texel scratch; the library's array holds 64 MiB
    mat = material(bcf, 2048, 12, (12, 32, 32, 10), 950)
    assert bcf.workspace_bytes(mat, bcf.Precision.FP16) > 64 << 20
    q = dev(synth.uniform_queries(100, synth.rng(951), 5.0))
    out = torch.full((100, 10), 7.0, device="cuda")
    with pytest.raises(bcf.BcfError, match="status 2.*workspace"):
        bcf.decode_noalloc(mat, q, bcf.Precision.FP16, out=out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
