"""The input generators behind the batch and training workloads: shapes,
ranges, determinism, and the reference sampler's exactness on what bicubic
filtering must reproduce (constants and texel centres at integer levels)."""
import numpy as np

import synth


def test_batch_spec_matches_its_description():
    s = synth.batch_spec()
    assert s.n_materials == 64 and set(s.res) <= {512, 1024, 2048, 4096}
    assert min(s.counts) >= 2 ** 14 and max(s.counts) <= 2 ** 22
    assert s.offsets()[-1] == sum(s.counts) and synth.batch_spec() == s
    m = synth.batch_material(s, 3)
    r = s.res[3]
    assert m.res == [r] * 4 and m.levels == [synth.full_levels(r, r)] * 4
    assert all(len(t) == 16 * synth.chain_blocks(r, r, m.levels[0]) for t in m.textures)
    q = synth.batch_queries(s, 3)
    assert q.shape == (s.counts[3], 3) and q[:, 2].max() <= m.levels[0] - 1


def test_procedural_target_levels_and_ranges():
    chain = synth.procedural_target(64)
    assert [c.shape for c in chain] == [(64 >> l, 64 >> l, 10) for l in range(7)]
    assert chain[0].min() >= 0.0 and chain[0].max() <= 1.0
    # every level is the 2x2 box average of the one below
    np.testing.assert_allclose(chain[1][3, 5], chain[0][6:8, 10:12].mean(axis=(0, 1)), rtol=1e-6)
    assert np.array_equal(synth.procedural_target(64)[0], chain[0])


def test_reference_sampler_reproduces_texels_and_constants():
    chain = synth.procedural_target(32)
    # at a texel centre of an integer level the Catmull-Rom weights are (0, 1, 0, 0)
    q = np.array([[(5 + 0.5) / 32, (9 + 0.5) / 32, 0.0], [(2 + 0.5) / 8, (7 + 0.5) / 8, 2.0]], np.float32)
    got = synth.sample_target(chain, q)
    np.testing.assert_allclose(got[0], chain[0][9, 5], rtol=1e-6)
    np.testing.assert_allclose(got[1], chain[2][7, 2], rtol=1e-6)
    # a constant image is reproduced anywhere (the weights sum to one)
    flat = [np.full_like(c, 0.25) for c in chain]
    q = synth.uniform_queries(1000, synth.rng(9), 5.0)
    np.testing.assert_allclose(synth.sample_target(flat, q), 0.25, rtol=1e-6)


def test_train_problem_shapes():
    ends, idxs, parts, L, params = synth.train_problem(64, (12, 16, 10))
    nb = synth.chain_blocks(64, 64, L)
    assert L == 7 and all(e.shape == (nb, 4, 3) for e in ends) and all(x.shape == (nb, 16) for x in idxs)
    assert all(p.max() < 32 for p in parts) and params.size == 12 * 16 + 16 + 16 * 10 + 10
