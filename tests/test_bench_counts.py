"""bench.py's algorithmic-byte counts (distinct blocks and texels the
trilinear footprints touch) against a brute-force enumeration, query by
query, on small cases."""
import math
import sys

import numpy as np

import synth


def bench():
    sys.argv = ["bench.py"]
    import bench as b
    return b


def brute(geo, queries):
    blocks, texels = set(), set()
    for k, ((w0, h0), levels, bias) in enumerate(geo):
        for u, v, s in queries.astype(np.float64):
            u -= math.floor(u)
            v -= math.floor(v)
            si = min(max(s + bias, 0.0), levels - 1)
            l0 = int(math.floor(si))
            for lev in {l0, min(l0 + 1, levels - 1)}:
                w, h = max(w0 >> lev, 1), max(h0 >> lev, 1)
                x0, y0 = math.floor(u * w - 0.5), math.floor(v * h - 0.5)
                for dx in (0, 1):
                    for dy in (0, 1):
                        x, y = (x0 + dx) % w, (y0 + dy) % h
                        texels.add((k, lev, x, y))
                        blocks.add((k, lev, x // 4, y // 4))
    return len(blocks), len(texels)


def test_unique_counts_match_brute_force():
    b = bench()
    g = synth.rng(5)
    for geo in ([((16, 16), 5, 0.0)] * 4, [((32, 8), 6, 0.0), ((8, 8), 4, 0.5), ((16, 16), 5, -1.0)]):
        q = synth.uniform_queries(300, g, 6.0)
        nb, nt = brute(geo, q)
        assert b.unique_blocks(geo, q) == nb
        assert b.unique_texels(geo, q) == nt


def test_all_blocks_counts_every_level():
    b = bench()
    geo = [((2048, 2048), 12, 0.0)] * 4
    assert b.all_blocks(geo) == 4 * synth.chain_blocks(2048, 2048, 12) == 1398108
