"""Pins of the oracle's trilinear filter (eq. 9 with the per-texture scale of
eq. 10) and of its decoder MLP (eq. 3).

Filter pins: reproduction of texels at texel centres of integer scales,
constants, midpoints, wrap addressing at the texture edge, the lerp between
the two levels, scale clamping, the LOD bias, small levels stored in one
block, and an exact rational recomputation on tiny textures. MLP pin: numpy's
float64 matmul on the same inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import bc6h_pack

G = synth.rng(7)


def level_texels(tex, res_w, res_h, level):
    """Decoded texels of one level as float64 [h, w, 3] (via the oracle's block
    decoder, which the BC6H pins cover)."""
    w, h = max(res_w >> level, 1), max(res_h >> level, 1)
    bx, by = (w + 3) // 4, (h + 3) // 4
    off = oracle.texture_bytes(res_w, res_h, level)
    blocks = np.frombuffer(tex[off: off + 16 * bx * by].tobytes(), np.uint8).reshape(-1, 16)
    dec = oracle.decode_blocks(blocks).view(np.float16).astype(np.float64)
    dec = dec.reshape(by, bx, 4, 4, 3).transpose(0, 2, 1, 3, 4).reshape(4 * by, 4 * bx, 3)
    return dec[:h, :w]


def one_texture_material(tex, w, h, levels, bias=0.0):
    dims = (3, 3)
    params = np.concatenate([np.eye(3).ravel(), np.zeros(3)]).astype(np.float32)
    return oracle.Material([tex], [(w, h)], [levels], dims, params, [bias])


@pytest.mark.parametrize("w,h", [(16, 16), (32, 8), (8, 32)])
def test_texel_centres_reproduce_texels(w, h):
    levels = max(w, h).bit_length()
    n = synth.chain_blocks(w, h, levels)
    tex = synth.bounded_blocks(n, G).reshape(-1)
    mat = one_texture_material(tex, w, h, levels)
    for l in range(levels):
        lw, lh = max(w >> l, 1), max(h >> l, 1)
        ref = level_texels(tex, w, h, l)
        jj, ii = np.meshgrid(np.arange(lh), np.arange(lw), indexing="ij")
        q = np.stack([(ii + 0.5) / lw, (jj + 0.5) / lh, np.full(ii.shape, l)], -1)
        got = oracle.sample(mat, q.reshape(-1, 3).astype(np.float32)).reshape(lh, lw, 3)
        assert np.array_equal(got, ref), l


def test_constant_texture_returns_the_constant():
    res, levels = 16, 5
    n = synth.chain_blocks(res, res, levels)
    blk = bc6h_pack.pack(11, dict(rw=300, gw=200, bw=100, rx=300, gx=200, bx=100), [0] * 16)
    tex = np.frombuffer(blk * n, np.uint8)
    mat = one_texture_material(tex, res, res, levels)
    c = level_texels(tex, res, res, 0)[0, 0]
    q = synth.uniform_queries(4000, G, s_max=6.0)
    got = oracle.sample(mat, q)
    assert np.allclose(got, c[None, :], rtol=1e-15, atol=0)


def test_midpoints_and_wrap_at_the_edge():
    res, levels = 16, 5
    tex = synth.bounded_blocks(synth.chain_blocks(res, res, levels), G).reshape(-1)
    mat = one_texture_material(tex, res, res, levels)
    for l in range(levels - 2):
        w = res >> l
        T = level_texels(tex, res, res, l)
        j = 3 % w
        vj = (j + 0.5) / w
        # halfway between the centres of texels i and i+1 in x
        for i in range(w - 1):
            got = oracle.sample(mat, np.array([[(i + 1.0) / w, vj, l]], np.float32))[0]
            assert np.array_equal(got, 0.5 * T[j, i] + 0.5 * T[j, i + 1])
        # u = 0 lies halfway between the last and the first texel (wrap)
        got = oracle.sample(mat, np.array([[0.0, vj, l]], np.float32))[0]
        assert np.array_equal(got, 0.5 * T[j, w - 1] + 0.5 * T[j, 0])
        # v = 0 likewise in y
        ui = (1 + 0.5) / w
        got = oracle.sample(mat, np.array([[ui, 0.0, l]], np.float32))[0]
        assert np.array_equal(got, 0.5 * T[w - 1, 1] + 0.5 * T[0, 1])
        # whole periods do not matter (values exact in binary32)
        q = np.array([[0.3125, 0.6875, l + 0.25], [1.3125, -0.3125, l + 0.25],
                      [-2.6875, 3.6875, l + 0.25]], np.float32)
        got = oracle.sample(mat, q)
        assert np.array_equal(got[1], got[0]) and np.array_equal(got[2], got[0])


def test_level_lerp_clamps_and_bias():
    res, levels = 32, 6
    tex = synth.bounded_blocks(synth.chain_blocks(res, res, levels), G).reshape(-1)
    mat = one_texture_material(tex, res, res, levels)
    q = synth.uniform_queries(500, G, s_max=1.0)
    for k in range(levels - 1):
        at = lambda s: oracle.sample(mat, np.c_[q[:, :2], np.full(len(q), s, np.float32)])
        a, b, mid = at(k), at(k + 1), at(k + 0.25)
        assert np.allclose(mid, 0.75 * a + 0.25 * b, rtol=1e-13, atol=1e-15)
    top = lambda s: oracle.sample(mat, np.c_[q[:, :2], np.full(len(q), s, np.float32)])
    assert np.array_equal(top(levels - 1), top(levels + 2.5))      # upper clamp, l1 = l0
    assert np.array_equal(top(0.0), top(-3.0))                     # lower clamp
    # b_i of eq. (10) shifts the scale of its own texture only
    biased = one_texture_material(tex, res, res, levels, bias=1.5)
    qs = np.c_[q[:, :2], np.full(len(q), 0.75, np.float32)]
    assert np.array_equal(oracle.sample(biased, qs), top(2.25))


def test_small_levels_use_the_top_left_texels_of_one_block():
    res, levels = 8, 4                         # levels 8x8, 4x4, 2x2, 1x1
    tex = synth.bounded_blocks(synth.chain_blocks(res, res, levels), G).reshape(-1)
    mat = one_texture_material(tex, res, res, levels)
    off2 = oracle.texture_bytes(res, res, 2)
    dec = oracle.decode_blocks(tex[off2: off2 + 16].reshape(1, 16))[0]
    dec = dec.view(np.float16).astype(np.float64)
    for ty in range(2):
        for tx in range(2):
            got = oracle.sample(mat, np.array([[(tx + 0.5) / 2, (ty + 0.5) / 2, 2]], np.float32))[0]
            assert np.array_equal(got, dec[ty * 4 + tx])
    off3 = oracle.texture_bytes(res, res, 3)
    dec3 = oracle.decode_blocks(tex[off3: off3 + 16].reshape(1, 16))[0].view(np.float16)
    got = oracle.sample(mat, np.array([[0.123, 0.877, 3]], np.float32))[0]
    assert np.array_equal(got, dec3[0].astype(np.float64))


def _exact_trilinear(T, u, v, s, levels):
    """Eq. (9) in exact rational arithmetic, as a sum over the eight texels of
    the two levels around s with product weights."""
    u, v, s = Fraction(float(u)), Fraction(float(v)), Fraction(float(s))
    s = min(max(s, 0), levels - 1)
    l0 = int(s)
    l1 = min(l0 + 1, levels - 1)
    lam = s - l0
    total = [Fraction(0)] * 3
    for level, lw in ((l0, 1 - lam), (l1, lam)):
        tex = T[level]
        h, w = tex.shape[:2]
        x = u * w - Fraction(1, 2)
        y = v * h - Fraction(1, 2)
        x0, y0 = x.__floor__(), y.__floor__()
        for dy in (0, 1):
            for dx in (0, 1):
                wx = (x - x0) if dx else (1 - (x - x0))
                wy = (y - y0) if dy else (1 - (y - y0))
                texel = tex[(y0 + dy) % h, (x0 + dx) % w]
                for c in range(3):
                    total[c] += lw * wx * wy * Fraction(float(texel[c]))
    return np.array([float(t) for t in total])


def test_exact_rational_recomputation_on_tiny_textures():
    for res in (4, 8):
        levels = res.bit_length()
        tex = synth.bounded_blocks(synth.chain_blocks(res, res, levels), G).reshape(-1)
        mat = one_texture_material(tex, res, res, levels)
        T = [level_texels(tex, res, res, l) for l in range(levels)]
        q = synth.uniform_queries(300, G, s_max=levels + 0.5)
        q[:, 2] -= 0.25                        # some scales below zero
        got = oracle.sample(mat, q)
        for i in range(len(q)):
            ref = _exact_trilinear(T, q[i, 0], q[i, 1], q[i, 2], levels)
            assert np.allclose(got[i], ref, rtol=1e-14, atol=1e-300), (i, q[i])


def test_mlp_matches_numpy_float64():
    dims = (12, 32, 32, 10)
    params = synth.mlp_params(dims, G)
    mat = oracle.Material([np.zeros(16, np.uint8)] * 4, [4] * 4, [1] * 4, dims, params)
    z = G.normal(size=(1000, 12))
    got = oracle.mlp(mat, z)
    h, p = z, 0
    for l, (n_in, n_out) in enumerate(zip(dims[:-1], dims[1:])):
        W = params[p: p + n_in * n_out].astype(np.float64).reshape(n_out, n_in)
        b = params[p + n_in * n_out: p + n_in * n_out + n_out].astype(np.float64)
        p += n_in * n_out + n_out
        h = h @ W.T + b
        if l < len(dims) - 2:
            h = np.maximum(h, 0.0)
    assert np.allclose(got, h, rtol=1e-13, atol=1e-13)


def test_decode_is_mlp_of_concatenated_samples():
    w = synth.WORKLOADS["tiny"]
    m = synth.make_material([16] * 4, [5] * 4, w.dims, variant="B")
    mat = oracle.Material.from_synth(m)
    q = synth.uniform_queries(2000, G, s_max=4.5)
    feats = oracle.sample(mat, q, n_threads=3)
    assert feats.shape == (2000, 12)
    # layer order: T_0.rgb, T_1.rgb, T_2.rgb, T_3.rgb
    for i in range(4):
        one = oracle.Material([m.textures[i]], [16], [5], (3, 3),
                              np.concatenate([np.eye(3).ravel(), np.zeros(3)]).astype(np.float32))
        assert np.array_equal(oracle.sample(one, q), feats[:, 3 * i: 3 * i + 3])
    out = oracle.decode(mat, q, n_threads=4)
    assert np.array_equal(out, oracle.mlp(mat, feats))
