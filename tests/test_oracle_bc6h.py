"""Pins of the oracle's BC6H decoder.

Against the paper: the unsigned output range stated with eq. (7), the
continuous unquantise / interpolate / scale chain of eqs. (6)-(7) for the
exported format (6-bit endpoints, 3-bit indices, Section "Real-time
Decoding"), and the half reinterpretation of eq. (8).

Against the format itself: mode codes, reserved codes, partition/anchor
invariants, interpolation invariants, and a round trip through the input
packer (an independent transcription of the layouts).

The black-box comparison with Pillow's BC6H reader lives in
test_oracle_pillow.py.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import bc6h_pack

G = synth.rng(20231116)


def halves(h):
    return np.asarray(h, np.uint16).view(np.float16).astype(np.float64)


def test_valid_codes_and_reserved_codes():
    for mode, (code, width) in bc6h_pack.MODE_CODE.items():
        for hi in range(8 if width == 5 else 64):
            blk = bytearray(G.integers(0, 256, 16, dtype=np.uint8).tobytes())
            blk[0] = (hi << width | code) & 0xFF
            assert oracle.decode_block(bytes(blk))[0] == mode
    blocks = synth.reserved_blocks(2000, G)
    out = oracle.decode_blocks(blocks)
    assert not out.any()
    for b in blocks[:50]:
        assert oracle.decode_block(b.tobytes())[0] == 0


def test_unsigned_output_range():
    # eq. (7): y lies in [-31743, 31743]; the unsigned format never sets the
    # sign bit and reaches at most 0x7BFF (65504, the largest finite half)
    blocks = synth.random_mode_blocks(50000, G)
    out = oracle.decode_blocks(blocks)
    assert (out & 0x8000).max() == 0
    assert out.max() <= 0x7BFF
    assert out.max() == 0x7BFF            # random bits hit the top endpoint code


@pytest.mark.parametrize("mode,bits", [(11, 10), (12, 11), (13, 12), (14, 16), (10, 6)])
def test_constant_blocks_follow_eq6(mode, bits):
    # Equal endpoints (zero deltas in transformed modes): every texel is the
    # unquantised endpoint scaled by a = 31/64. Read with a scaling the whole
    # unquantised value, eq. (6) gives a (2^16 e + 2^15) / 2^b; the format
    # rounds down twice, so the decoded integer lies less than 1.5 below it.
    # The extremes follow the format: e = 0 gives 0 and the top code gives
    # the largest value 31743.
    cap = 1 << bits
    step = max(1, cap // 4000)
    for e in list(range(0, cap, step)) + [cap - 1]:
        fields = {"rw": e, "gw": e, "bw": e}
        if mode == 11:                       # untransformed: x stores e itself
            fields.update(rx=e, gx=e, bx=e)
        if mode == 10:
            fields.update(rx=e, gx=e, bx=e, ry=e, gy=e, by=e, rz=e, gz=e, bz=e,
                          d=int(G.integers(0, 32)))
        idx = G.integers(0, 8 if mode <= 10 else 16, 16)
        idx[0] >>= 1
        if mode <= 10:
            idx[bc6h_pack.ANCHOR2[fields["d"]]] >>= 1
        m, out = oracle.decode_block(bc6h_pack.pack(mode, fields, idx))
        assert m == mode
        assert (out == out[0, 0]).all(), e
        y = int(out[0, 0])
        if e == 0:
            assert y == 0
        elif e == cap - 1:
            assert y == 31743
        else:
            eq6 = 31 / 64 * (2 ** 16 * e + 2 ** 15) / 2 ** bits
            assert 0 <= eq6 - y < 1.5, (e, y, eq6)


def test_exported_mode_follows_eqs_6_to_8():
    # The paper exports every block with 6-bit endpoints and 3-bit indices,
    # the two-subset untransformed mode 10. Continuous chain of eqs. (6)-(7):
    # e_bar = a (2^16 e + 2^15) / 2^6, y = e_bar_1 + x (e_bar_2 - e_bar_1) with
    # x = w_i / 64 (the 3-bit weights), then eq. (8) reinterprets y as a half.
    # The format rounds the blend to nearest and the scaled value down, so the
    # decoded integer lies in (y - 1.25, y + 0.25].
    weights = [0, 9, 18, 27, 37, 46, 55, 64]
    blocks = synth.random_mode_blocks(3000, G, modes=(10,))
    for blk in blocks:
        m, out = oracle.decode_block(blk.tobytes())
        f = oracle.block_fields(blk.tobytes())
        bits = int.from_bytes(blk.tobytes(), "little")
        p, part = 82, f["d"]
        mask = [0xCCCC, 0x8888, 0xEEEE, 0xECC8, 0xC880, 0xFEEC, 0xFEC8, 0xEC80,
                0xC800, 0xFFEC, 0xFE80, 0xE800, 0xFFE8, 0xFF00, 0xFFF0, 0xF000,
                0xF710, 0x008E, 0x7100, 0x08CE, 0x008C, 0x7310, 0x3100, 0x8CCE,
                0x088C, 0x3110, 0x6666, 0x366C, 0x17E8, 0x0FF0, 0x718E, 0x399C][part]
        for t in range(16):
            nb = 3 - (t == 0 or t == bc6h_pack.ANCHOR2[part])
            i = (bits >> p) & ((1 << nb) - 1)
            p += nb
            s = (mask >> t) & 1
            x = weights[i] / 64
            for c, ch in enumerate("rgb"):
                e1 = f[ch + ("w" if s == 0 else "y")]
                e2 = f[ch + ("x" if s == 0 else "z")]
                ebar = [31 / 64 * (2 ** 16 * e + 2 ** 15) / 64 for e in (e1, e2)]
                for k, e in enumerate((e1, e2)):     # format's special codes
                    if e == 0:
                        ebar[k] = 0.0
                    elif e == 63:
                        ebar[k] = 31 / 64 * 0xFFFF
                y = ebar[0] + x * (ebar[1] - ebar[0])
                got = int(out[t, c])
                assert -0.25 <= y - got < 1.25, (t, c, y, got)
                # eq. (8) closed form of the reinterpretation
                h = max((got - 1) // 1024 - 1, 0)
                assert halves(got) == 2.0 ** (h - 14) * (got / 1024 - h)


def test_partition_table_invariants():
    # every partition: texel 0 in subset 0, its subset-1 anchor in subset 1,
    # all 32 masks distinct; decode a block whose subsets decode to 0 and to
    # a bright constant with all indices 0 and read the mask back
    seen = set()
    for part in range(32):
        e = 40
        f = dict(rw=0, gw=0, bw=0, rx=0, gx=0, bx=0, ry=e, gy=e, by=e, rz=e, gz=e, bz=e, d=part)
        m, out = oracle.decode_block(bc6h_pack.pack(10, f, [0] * 16))
        mask = sum(1 << t for t in range(16) if out[t, 0] != 0)
        assert not mask & 1
        assert mask >> bc6h_pack.ANCHOR2[part] & 1
        assert (out[:, 0] == 0).sum() + (out[:, 0] == out.max()).sum() == 16
        seen.add(mask)
    assert len(seen) == 32


def test_anchor_texels_carry_one_bit_fewer():
    # With every stored index bit set, ordinary texels read the top index and
    # the two anchors (texel 0 and the subset-1 anchor) read the top index
    # with its high bit cleared (3 for 3-bit indices).
    for part in range(32):
        f = dict(rw=0, gw=0, bw=0, rx=63, gx=63, bx=63, ry=0, gy=0, by=0, rz=62, gz=62, bz=62, d=part)
        blk = int.from_bytes(bc6h_pack.pack(10, f, [0] * 16), "little")
        blk |= ((1 << 46) - 1) << 82
        m, out = oracle.decode_block(blk.to_bytes(16, "little"))
        ref = {}
        for i in range(8):
            idx = [i] * 16
            idx[0] = min(i, 3)
            idx[bc6h_pack.ANCHOR2[part]] = min(i, 3)
            ref[i] = oracle.decode_block(bc6h_pack.pack(10, f, idx))[1]
        anchor = bc6h_pack.ANCHOR2[part]
        for t in range(16):
            want = ref[3][t] if t in (0, anchor) else ref[7][t]
            assert (out[t] == want).all(), (part, t)


@pytest.mark.parametrize("mode", range(1, 15))
def test_interpolation_invariants(mode):
    # index 0 reproduces the subset's first endpoint and the top index its
    # second one (weights 0 and 64); texel values are monotone in the index
    blocks = synth.bounded_blocks(200, G, modes=(mode,))
    two = mode <= 10
    width = 3 if two else 4
    for blk in blocks:
        f = oracle.block_fields(blk.tobytes())
        f = {k: v for k, v in f.items() if k != "mode"}
        anchor = bc6h_pack.ANCHOR2[f["d"]] if two else -1
        lo = oracle.decode_block(bc6h_pack.pack(mode, f, [0] * 16))[1].astype(np.int64)
        prev = lo
        for i in range(1, 1 << width):
            idx = [i] * 16
            for t in (0, anchor):
                if t >= 0:
                    idx[t] = min(i, (1 << (width - 1)) - 1)
            cur = oracle.decode_block(bc6h_pack.pack(mode, f, idx))[1].astype(np.int64)
            top = cur
            # along the segment every channel moves monotonically one way
            d_prev, d_cur = np.sign(prev - lo), np.sign(cur - prev)
            assert ((d_prev * d_cur) >= 0).all()
            prev = cur
        # swapping each subset's endpoints swaps the ends of the segment
        g = dict(f)
        keys = [("w", "x")] + ([("y", "z")] if two else [])
        for a, b in keys:
            for ch in "rgb":
                if mode in (10, 11):
                    g[ch + a], g[ch + b] = f[ch + b], f[ch + a]
        if mode in (10, 11):
            swapped = oracle.decode_block(bc6h_pack.pack(mode, g, [0] * 16))[1].astype(np.int64)
            free = [t for t in range(16) if t not in (0, anchor)]
            assert (swapped[free] == top[free]).all()


def test_packer_round_trip_recovers_fields():
    # two independent transcriptions of every layout agree field by field
    for mode in range(1, 15):
        shape = bc6h_pack.MODE_SHAPE[mode]
        for _ in range(300):
            f = {}
            for ch, wbits in zip("rgb", [shape[0]] * 3):
                f[ch + "w"] = int(G.integers(0, 1 << wbits))
            for j, name in enumerate("xyz"[: 2 * shape[3] - 1]):
                for c, ch in enumerate("rgb"):
                    f[ch + name] = int(G.integers(0, 1 << shape[1][c]))
            f["d"] = int(G.integers(0, 32)) if shape[3] == 2 else 0
            got = oracle.block_fields(bc6h_pack.pack(mode, f, [0] * 16))
            assert got["mode"] == mode
            for k, v in f.items():
                assert got[k] == v, (mode, k, v, got[k])


# ---------------------------------------------------------------------------
# signed format (BC6H_SF16)

@pytest.mark.parametrize("mode,bits", [(11, 10), (12, 11), (13, 12), (10, 6)])
def test_signed_constant_blocks_follow_eq6(mode, bits):
    # eq. (6) with a = 31/32 for the signed format: a constant block of code e
    # (two's complement of `bits`) decodes to sign(e) a (2^16 |e| + 2^15) / 2^b
    # within 1.5 below in magnitude, with the half's sign bit for e < 0. Zero
    # gives 0; magnitudes at the top code saturate to 31743.
    half = 1 << (bits - 1)
    step = max(1, half // 1500)
    for e in list(range(-half + 1, half, step)) + [half - 1, -(half - 1)]:
        s = e & ((1 << bits) - 1)
        fields = {"rw": s, "gw": s, "bw": s}
        if mode == 11:
            fields.update(rx=s, gx=s, bx=s)
        if mode == 10:
            fields.update(rx=s, gx=s, bx=s, ry=s, gy=s, by=s, rz=s, gz=s, bz=s, d=3)
        m, out = oracle.decode_block(bc6h_pack.pack(mode, fields, [0] * 16), signed=True)
        assert m == mode and (out == out[0, 0]).all()
        y = int(out[0, 0])
        mag, neg = y & 0x7FFF, bool(y & 0x8000)
        if e == 0:
            assert y == 0
        elif abs(e) >= half - 1:
            assert mag == 31743 and neg == (e < 0)
        else:
            eq6 = 31 / 32 * (2 ** 16 * abs(e) + 2 ** 15) / 2 ** bits
            assert 0 <= eq6 - mag < 1.5, (e, y, eq6)
            assert neg == (e < 0)


@pytest.mark.parametrize("mode", range(1, 15))
def test_signed_negation_symmetry(mode):
    # Negating every endpoint (the stored base and every stored delta, in two's
    # complement of their widths) negates every texel; the blend's rounding to
    # nearest with ties up can shift a magnitude by one unit.
    g = synth.rng(600 + mode)
    blocks = synth.bounded_blocks(300, g, modes=(mode,), signed=True)
    bits, widths, transformed, subsets = bc6h_pack.MODE_SHAPE[mode]
    checked = 0
    for blk in blocks:
        f = oracle.block_fields(blk.tobytes())
        # the most negative stored delta has no positive counterpart
        if transformed and any(f[ch + name] == 1 << (widths[i] - 1)
                               for i, ch in enumerate("rgb") for name in "xyz"[: 2 * subsets - 1]):
            continue
        checked += 1
        neg = {}
        for ch_i, ch in enumerate("rgb"):
            neg[ch + "w"] = (-f[ch + "w"]) & ((1 << bits) - 1)
            for name in "xyz"[: 2 * subsets - 1]:
                w = widths[ch_i] if transformed else bits
                neg[ch + name] = (-f[ch + name]) & ((1 << w) - 1)
        neg["d"] = f["d"]
        bits_in = int.from_bytes(blk.tobytes(), "little")
        header = bc6h_pack.header_bits(mode)
        idx = bits_in >> header
        p = int.from_bytes(bc6h_pack.pack(mode, neg, [0] * 16), "little")
        p |= idx << header
        a = oracle.decode_block(blk.tobytes(), signed=True)[1].astype(np.int64)
        b = oracle.decode_block(p.to_bytes(16, "little"), signed=True)[1].astype(np.int64)
        ma, mb = a & 0x7FFF, b & 0x7FFF
        assert (np.abs(ma - mb) <= 1).all()
        nz = (ma > 1) & (mb > 1)
        assert ((a[nz] & 0x8000) != (b[nz] & 0x8000)).all()
    assert checked > 100
