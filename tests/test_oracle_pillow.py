"""Black-box pin of the oracle's BC6H layouts against Pillow's DDS reader.

Pillow decodes BC6H_UF16 (DXGI format 95) and BC6H_SF16 (96) to 8-bit RGB.
It is run only; its decoder is never read. Characterised from outside:

* it maps a decoded half value v to floor(clamp(v, 0, 1) * 255);
* it blends endpoints as ((64 - w) A + w B) >> 6, without the +32 rounding
  term of the format definition, so it can read one 8-bit step lower.

The term provably cannot matter when every unquantised endpoint is a multiple
of 64: with endpoint precision b <= 9 the unquantised value of a code e other
than the top code is 2^(16-b) e + 2^(15-b) (or 0), a multiple of 64, and the
bounded generator never emits the top code. Those cases must agree exactly;
everywhere else the oracle may exceed Pillow by one 8-bit step, rarely. A
misplaced bit in any header map, partition, anchor, index width or weight
would show as differences far larger than one step.
"""
import io
import struct

import numpy as np
import pytest

import oracle
import synth

PIL = pytest.importorskip("PIL.Image")

LOW_PRECISION_MODES = (2, 6, 7, 8, 9, 10)          # endpoint precision <= 9 bits


def dds(blocks: bytes, w: int, h: int, signed: bool = False) -> bytes:
    flags = 0x1 | 0x2 | 0x4 | 0x1000
    pf = struct.pack("<II4sIIIII", 32, 0x4, b"DX10", 0, 0, 0, 0, 0)
    hdr = struct.pack("<IIIIIII", 124, flags, h, w, len(blocks), 0, 1) + b"\0" * 44 + pf
    hdr += struct.pack("<IIIII", 0x1000, 0, 0, 0, 0)
    dx10 = struct.pack("<IIIII", 96 if signed else 95, 3, 0, 1, 0)
    return b"DDS " + hdr + dx10 + blocks


def pillow_decode(blocks: np.ndarray, signed: bool = False) -> np.ndarray:
    """[n, 16] blocks -> Pillow's 8-bit texels [n, 16, 3] (n a multiple of 64)."""
    n = blocks.shape[0]
    bw = 64
    bh = n // bw
    im = PIL.open(io.BytesIO(dds(blocks.tobytes(), 4 * bw, 4 * bh, signed)))
    im.load()
    a = np.asarray(im.convert("RGB")).astype(np.int64)
    return a.reshape(bh, 4, bw, 4, 3).transpose(0, 2, 1, 3, 4).reshape(n, 16, 3)


def oracle_8bit(blocks: np.ndarray, signed: bool = False) -> np.ndarray:
    h = oracle.decode_blocks(blocks, signed)
    v = h.view(np.float16).astype(np.float64)
    return np.floor(np.clip(v, 0.0, 1.0) * 255.0).astype(np.int64)


def compare(blocks, exact, signed=False):
    ref = pillow_decode(blocks, signed)
    got = oracle_8bit(blocks, signed)
    d = got - ref
    if exact:
        assert not d.any(), int((d != 0).sum())
    else:
        assert set(np.unique(d)) <= {0, 1}, np.unique(d)
        assert (d != 0).mean() < 0.02
    return ref


@pytest.mark.parametrize("mode", range(1, 15))
def test_bounded_blocks_match_pillow(mode):
    g = synth.rng(100 + mode)
    blocks = synth.bounded_blocks(64 * 64, g, modes=(mode,))
    ref = compare(blocks, mode in LOW_PRECISION_MODES)
    # the comparison is informative: most texels land strictly inside (0, 255)
    assert ((ref > 0) & (ref < 255)).mean() > 0.4


@pytest.mark.parametrize("mode", range(1, 15))
def test_single_bit_flips_match_pillow(mode):
    # Flip every bit of the block, one at a time, on bounded base blocks: a
    # misplaced header bit, partition bit or index bit changes different
    # texels or channels in the oracle than in Pillow.
    g = synth.rng(200 + mode)
    base = synth.bounded_blocks(64, g, modes=(mode,))
    code_bits = 2 if mode <= 2 else 5
    flipped = []
    for p in range(code_bits, 128):
        b = base.copy()
        b[:, p >> 3] ^= np.uint8(1 << (p & 7))
        flipped.append(b)
    compare(np.concatenate(flipped), exact=False)


def test_random_bits_all_modes_and_reserved_codes_match_pillow():
    g = synth.rng(300)
    blocks = np.concatenate([synth.random_mode_blocks(64 * 32, g),
                             synth.reserved_blocks(64 * 4, g)])
    ref = pillow_decode(blocks)
    got = oracle_8bit(blocks)
    d = got - ref
    assert set(np.unique(d)) <= {0, 1}
    assert (d != 0).mean() < 0.01
    assert not ref[-64 * 4:].any()           # reserved codes decode to zero


@pytest.mark.parametrize("mode", range(1, 15))
def test_signed_bounded_blocks_match_pillow(mode):
    # BC6H_SF16 on non-negative bounded endpoints: the signed unquantisation
    # and the 31/32 scale. Pillow's signed reader gives values with no simple
    # characterisation once a blend mixes signs, so full-range signed blocks
    # are not compared against it.
    g = synth.rng(400 + mode)
    blocks = synth.bounded_blocks(64 * 64, g, modes=(mode,))
    compare(blocks, mode in LOW_PRECISION_MODES, signed=True)


ENDPOINT_FIELDS = {c + f for c in "rgb" for f in "wxyz"}


@pytest.mark.parametrize("mode", range(1, 15))
def test_every_endpoint_bit_matches_pillow_at_full_precision(mode):
    # With every index 0 or the largest, each texel shows one endpoint
    # unblended (weights 0 and 64), where Pillow's blend and the format's agree
    # exactly, so any block decodes identically at 8 bits in both readers.
    # Flipping one endpoint bit moves an endpoint by one unit of that bit; for
    # the low-order bits of the wide fields (mode 14's rw[3:0], the deltas,
    # the low bits of modes 12 and 13) the texel then crosses an 8-bit step
    # only when it sat just below one, so the two readers must agree on which
    # flips cross: a swapped or misplaced low bit changes which texels cross.
    from synth.bc6h_pack import POSITIONS
    g = synth.rng(500 + mode)
    base = synth.bounded_blocks(2048, g, modes=(mode,), extreme_indices=True)
    ref_base = oracle_8bit(base)
    assert np.array_equal(pillow_decode(base), ref_base)
    flipped, fields = [], []
    for p, (name, k) in enumerate(POSITIONS[mode]):
        if name not in ENDPOINT_FIELDS:
            continue                        # mode code, partition: covered by the flip test above
        b = base.copy()
        b[:, p >> 3] ^= np.uint8(1 << (p & 7))
        flipped.append(b)
        fields.append((name, k))
    flipped = np.concatenate(flipped)
    ref = pillow_decode(flipped)
    got = oracle_8bit(flipped)
    assert np.array_equal(got, ref), int((got != ref).sum())
    # the check is informative for every low-order bit: enough flips cross a step
    crossed = (ref.reshape(len(fields), -1, 16, 3) != ref_base[None]).sum(axis=(1, 2, 3))
    low = [(f, c) for f, c in zip(fields, crossed) if f[1] < 4]
    assert low and all(c >= 16 for _, c in low), low
