"""Pins of the FP64 training-decode oracle (oracle/train.py) against facts
outside it: the exact BC6H decode of the exported block (a separate oracle
routine reading bits a separate packer wrote), numpy's IEEE half conversion,
closed forms of eqs. (6)-(8), and central finite differences in binary64."""
import numpy as np
import pytest

import oracle
import synth
from oracle import train as T
from synth import bc6h_pack

torch = pytest.importorskip("torch")


def random_texture(g, w, h, levels, lo=1.0, hi=62.0):
    nb = synth.chain_blocks(w, h, levels)
    return T.TrainTexture(
        w, h, levels,
        endpoints=g.uniform(lo, hi, (nb, 4, 3)).astype(np.float32),
        indices=g.uniform(0.0, 1.0, (nb, 16)).astype(np.float32),
        partitions=g.integers(0, 32, nb).astype(np.uint8))


def export_block(eq, iq, k):
    """Encode quantised mode-10 parameters as a BC6H block (Section 5.2's
    export): the anchors' index top bit must be zero, which swapping the
    subset's endpoints and mirroring its indices (i -> 7 - i) achieves without
    changing any decoded texel (the 3-bit weights satisfy w_{7-i} = 64 - w_i)."""
    mask, anchor = oracle.partition(int(k))
    eq = eq.copy()
    iq = iq.copy()
    for sub, at in ((0, 0), (1, anchor)):
        if iq[at] >= 4:
            members = [t for t in range(16) if ((mask >> t) & 1) == sub]
            eq[[2 * sub, 2 * sub + 1]] = eq[[2 * sub + 1, 2 * sub]]
            iq[members] = 7 - iq[members]
    fields = {ch + name: int(eq[j, c]) for j, name in enumerate("wxyz") for c, ch in enumerate("rgb")}
    fields["d"] = int(k)
    return np.frombuffer(bc6h_pack.pack(10, fields, iq), np.uint8)


def test_ste_forward_is_the_exported_blocks_exact_decode():
    g = synth.rng(301)
    n = 3000
    ends = g.uniform(-0.6, 63.6, (n, 4, 3)).astype(np.float32)        # includes clamped values
    ends[:50] = np.round(ends[:50])                                   # exact integers, 0 and 63 too
    idx = g.uniform(-0.05, 1.05, (n, 16)).astype(np.float32)
    parts = g.integers(0, 32, n).astype(np.uint8)
    got = T.block_texels(torch.from_numpy(ends.astype(np.float64)), torch.from_numpy(idx.astype(np.float64)),
                         parts, ste=True).detach().numpy()
    eq = np.clip(np.round(ends.astype(np.float64)), 0, 63).astype(np.int64)
    iq = np.clip(np.round(np.float32(7) * idx), 0, 7).astype(np.int64)
    blocks = np.stack([export_block(eq[i], iq[i], parts[i]) for i in range(n)])
    halves = oracle.decode_blocks(blocks)                              # [n, 16, 3] bit patterns
    ref = halves.view(np.float16).astype(np.float64)
    assert np.array_equal(got, ref)


def test_constant_blocks_closed_form():
    # all four endpoints equal e: eq. (6) gives 1024 e + 512 exactly (b = 6) and
    # a (1024 e + 512) = 496 e + 248 is an integer, so eq. (8) must return the
    # IEEE half whose bits are 496 e + 248, for any indices
    g = synth.rng(302)
    e = np.arange(1, 63)
    ends = np.repeat(e[:, None, None], 4, 1).repeat(3, 2).astype(np.float64)
    idx = g.uniform(0, 1, (len(e), 16))
    parts = g.integers(0, 32, len(e))
    bits = (496 * e + 248).astype(np.uint16)
    want = np.repeat(bits.view(np.float16).astype(np.float64)[:, None], 16, 1)
    for ste in (False, True):
        got = T.block_texels(torch.from_numpy(ends), torch.from_numpy(idx), parts, ste).detach().numpy()
        for c in range(3):
            np.testing.assert_array_equal(got[:, :, c], want)


def test_continuous_matches_exact_decode_within_the_format_floors():
    # at integer endpoints in [1, 62] and x = w_i / 64 the continuous chain and
    # the integer decode differ only by the blend's and the finish's floors:
    # |y - y_int| < 1.25, i.e. within 1.25 steps of eq. (8)'s slope
    g = synth.rng(303)
    n = 4000
    ends = g.integers(1, 63, (n, 4, 3)).astype(np.float64)
    iq = g.integers(0, 8, (n, 16))
    wts = np.floor(64.0 * np.arange(8) / 7.0 + 0.5)
    x_exact = wts[iq] / 64.0
    x_index = (iq / 7.0).astype(np.float32)                          # rounds back to iq
    parts = g.integers(0, 32, n)
    cont = T.block_texels(torch.from_numpy(ends), torch.from_numpy(x_exact), parts, False).numpy()
    exact = T.block_texels(torch.from_numpy(ends), torch.from_numpy(x_index.astype(np.float64)), parts,
                           True).detach().numpy()
    y_bits = np.array(exact, np.float16).view(np.uint16).astype(np.float64)
    slope = T.half_slope(torch.from_numpy(y_bits)).numpy()
    assert np.all(np.abs(cont - exact) <= 1.25 * slope * 2 + 1e-18)


def test_half_value_is_ieee_half_and_slope_steps():
    y = np.arange(0, 31744, dtype=np.float64)
    got = T.half_value(torch.from_numpy(y)).numpy()
    np.testing.assert_array_equal(got, y.astype(np.uint16).view(np.float16).astype(np.float64))
    s = T.half_slope(torch.from_numpy(y[1:])).numpy()
    np.testing.assert_allclose(s, np.diff(got), rtol=0, atol=0)


def small_problem(seed, ste, res=16, levels=5, n=200, dims=(12, 8, 8, 5)):
    g = synth.rng(seed)
    texs = [random_texture(g, res, res, levels) for _ in range(4)]
    params = synth.mlp_params(dims, g)
    q = synth.uniform_queries(n, g, levels - 1.0)
    go = g.standard_normal((n, dims[-1]))
    return texs, dims, params, q, go


def test_continuous_gradients_match_central_differences():
    texs, dims, params, q, go = small_problem(304, ste=False)
    val, d_end, d_idx, d_par = T.gradients(texs, dims, params, q, go, ste=False)
    g = synth.rng(305)

    def loss(tx, p):
        return float((T.forward(tx, dims, p, q, False).detach().numpy() * go).sum())

    def check(analytic, bump):
        eps = 1e-5
        plus, minus = bump(eps), bump(-eps)
        fd = (plus - minus) / (2 * eps)
        assert abs(fd - analytic) <= 1e-6 * max(1.0, abs(analytic)), (fd, analytic)

    import copy
    for _ in range(12):
        t = int(g.integers(4))
        b = int(g.integers(len(texs[t].partitions)))
        j, c = int(g.integers(4)), int(g.integers(3))

        def bump_e(eps, t=t, b=b, j=j, c=c):
            tx = copy.deepcopy(texs)
            tx[t].endpoints = tx[t].endpoints.astype(np.float64)
            tx[t].endpoints[b, j, c] += eps
            return loss(tx, params)
        check(d_end[t][b, j, c], bump_e)
        k = int(g.integers(16))

        def bump_x(eps, t=t, b=b, k=k):
            tx = copy.deepcopy(texs)
            tx[t].indices = tx[t].indices.astype(np.float64)
            tx[t].indices[b, k] += eps
            return loss(tx, params)
        check(d_idx[t][b, k], bump_x)
        i = int(g.integers(len(params)))

        def bump_p(eps, i=i):
            p = np.asarray(params, np.float64).copy()
            p[i] += eps
            return loss(texs, p)
        check(d_par[i], bump_p)


def test_ste_gradient_is_the_surrogate_slope():
    # with one block, one query at a texel centre of level 0 and an identity
    # readout, d G / d e_A = slope(y) * a * 1024 * (1 - w_i / 64) on that texel
    g = synth.rng(306)
    tex = random_texture(g, 4, 4, 1)
    zeros = [T.TrainTexture(4, 4, 1, np.full((1, 4, 3), 1.0, np.float32), np.zeros((1, 16), np.float32),
                            np.zeros(1, np.uint8)) for _ in range(3)]
    dims = (12, 3)
    W = np.zeros((3, 12))
    W[0, 0] = 1.0                                                     # red of pyramid 0
    params = np.concatenate([W.ravel(), np.zeros(3)])
    tx, ty = 2, 1
    q = np.array([[(tx + 0.5) / 4, (ty + 0.5) / 4, 0.0]], np.float32)
    go = np.array([[1.0, 0.0, 0.0]])
    _, d_end, d_idx, _ = T.gradients([tex] + zeros, dims, params, q, go, ste=True)
    t = ty * 4 + tx
    mask, _ = oracle.partition(int(tex.partitions[0]))
    sub = (mask >> t) & 1
    iq = int(np.clip(np.round(np.float32(7) * tex.indices[0, t]), 0, 7))
    w = np.floor(64.0 * iq / 7.0 + 0.5) / 64.0
    texel = T.block_texels(torch.from_numpy(tex.endpoints.astype(np.float64)),
                           torch.from_numpy(tex.indices.astype(np.float64)), tex.partitions, True)
    y_bits = float(np.array(texel.detach().numpy()[0, t, 0], np.float16).view(np.uint16))
    slope = float(T.half_slope(torch.tensor(y_bits, dtype=torch.float64)))
    expect_a = slope * T.A_UNSIGNED * 1024.0 * (1.0 - w)
    expect_b = slope * T.A_UNSIGNED * 1024.0 * w
    assert d_end[0][0, 2 * sub, 0] == pytest.approx(expect_a, rel=1e-12)
    assert d_end[0][0, 2 * sub + 1, 0] == pytest.approx(expect_b, rel=1e-12)
    # nothing flows to the other channels, the other subset or other texels' indices
    assert np.count_nonzero(d_end[0][0, :, 1:]) == 0
    assert np.count_nonzero(d_idx[0][0]) == 1
