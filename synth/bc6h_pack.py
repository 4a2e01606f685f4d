"""BC6H block *packer* used only to synthesise inputs.

It places given field values and texel indices at the bit positions the
public BC6H format definition assigns them. It does no decoding arithmetic (no
transform, unquantisation, interpolation or half conversion); the decoders
live in the oracle and in the GPU library, each with its own transcription of
the layout. This file is a third, independent transcription, written as the
definition's layout strings, so a packer -> decoder round trip compares two
transcriptions against each other.
"""
from __future__ import annotations

import re

import numpy as np

# Header layout per 1-based mode, from block bit 0 upward, in the definition's
# notation: f[a:b] is |a-b|+1 consecutive bits, the lowest holding bit b.
LAYOUTS = {
    1: "m[1:0] gy[4] by[4] bz[4] rw[9:0] gw[9:0] bw[9:0] rx[4:0] gz[4] gy[3:0] gx[4:0] bz[0] "
       "gz[3:0] bx[4:0] bz[1] by[3:0] ry[4:0] bz[2] rz[4:0] bz[3] d[4:0]",
    2: "m[1:0] gy[5] gz[4] gz[5] rw[6:0] bz[0] bz[1] by[4] gw[6:0] by[5] bz[2] gy[4] bw[6:0] "
       "bz[3] bz[5] bz[4] rx[5:0] gy[3:0] gx[5:0] gz[3:0] bx[5:0] by[3:0] ry[5:0] rz[5:0] d[4:0]",
    3: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[4:0] rw[10] gy[3:0] gx[3:0] gw[10] bz[0] gz[3:0] "
       "bx[3:0] bw[10] bz[1] by[3:0] ry[4:0] bz[2] rz[4:0] bz[3] d[4:0]",
    4: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[3:0] rw[10] gz[4] gy[3:0] gx[4:0] gw[10] gz[3:0] "
       "bx[3:0] bw[10] bz[1] by[3:0] ry[3:0] bz[0] bz[2] rz[3:0] gy[4] bz[3] d[4:0]",
    5: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[3:0] rw[10] by[4] gy[3:0] gx[3:0] gw[10] bz[0] "
       "gz[3:0] bx[4:0] bw[10] by[3:0] ry[3:0] bz[1] bz[2] rz[3:0] bz[4] bz[3] d[4:0]",
    6: "m[4:0] rw[8:0] by[4] gw[8:0] gy[4] bw[8:0] bz[4] rx[4:0] gz[4] gy[3:0] gx[4:0] bz[0] "
       "gz[3:0] bx[4:0] bz[1] by[3:0] ry[4:0] bz[2] rz[4:0] bz[3] d[4:0]",
    7: "m[4:0] rw[7:0] gz[4] by[4] gw[7:0] bz[2] gy[4] bw[7:0] bz[3] bz[4] rx[5:0] gy[3:0] "
       "gx[4:0] bz[0] gz[3:0] bx[4:0] bz[1] by[3:0] ry[5:0] rz[5:0] d[4:0]",
    8: "m[4:0] rw[7:0] bz[0] by[4] gw[7:0] gy[5] gy[4] bw[7:0] gz[5] bz[4] rx[4:0] gz[4] "
       "gy[3:0] gx[5:0] gz[3:0] bx[4:0] bz[1] by[3:0] ry[4:0] bz[2] rz[4:0] bz[3] d[4:0]",
    9: "m[4:0] rw[7:0] bz[1] by[4] gw[7:0] by[5] gy[4] bw[7:0] bz[5] bz[4] rx[4:0] gz[4] "
       "gy[3:0] gx[4:0] bz[0] gz[3:0] bx[5:0] by[3:0] ry[4:0] bz[2] rz[4:0] bz[3] d[4:0]",
    10: "m[4:0] rw[5:0] gz[4] bz[0] bz[1] by[4] gw[5:0] gy[5] by[5] bz[2] gy[4] bw[5:0] gz[5] "
        "bz[3] bz[5] bz[4] rx[5:0] gy[3:0] gx[5:0] gz[3:0] bx[5:0] by[3:0] ry[5:0] rz[5:0] d[4:0]",
    11: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[9:0] gx[9:0] bx[9:0]",
    12: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[8:0] rw[10] gx[8:0] gw[10] bx[8:0] bw[10]",
    13: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[7:0] rw[10:11] gx[7:0] gw[10:11] bx[7:0] bw[10:11]",
    14: "m[4:0] rw[9:0] gw[9:0] bw[9:0] rx[3:0] rw[10:15] gx[3:0] gw[10:15] bx[3:0] bw[10:15]",
}

# Mode code and its width in bits.
MODE_CODE = {1: (0x00, 2), 2: (0x01, 2), 3: (0x02, 5), 4: (0x06, 5), 5: (0x0A, 5),
             6: (0x0E, 5), 7: (0x12, 5), 8: (0x16, 5), 9: (0x1A, 5), 10: (0x1E, 5),
             11: (0x03, 5), 12: (0x07, 5), 13: (0x0B, 5), 14: (0x0F, 5)}
RESERVED_CODES = (0x13, 0x17, 0x1B, 0x1F)

# (endpoint bits, stored widths of x/y/z per channel, transformed, subsets)
MODE_SHAPE = {1: (10, (5, 5, 5), True, 2), 2: (7, (6, 6, 6), True, 2),
              3: (11, (5, 4, 4), True, 2), 4: (11, (4, 5, 4), True, 2),
              5: (11, (4, 4, 5), True, 2), 6: (9, (5, 5, 5), True, 2),
              7: (8, (6, 5, 5), True, 2), 8: (8, (5, 6, 5), True, 2),
              9: (8, (5, 5, 6), True, 2), 10: (6, (6, 6, 6), False, 2),
              11: (10, (10, 10, 10), False, 1), 12: (11, (9, 9, 9), True, 1),
              13: (12, (8, 8, 8), True, 1), 14: (16, (4, 4, 4), True, 1)}

# Texel of subset 1 that stores one index bit fewer, per partition.
ANCHOR2 = (15,) * 17 + (2, 8, 2, 2, 8, 8, 15, 2, 8, 2, 2, 8, 8, 2, 2)

_TOKEN = re.compile(r"([a-z]+)\[(\d+)(?::(\d+))?\]")


def _positions(mode: int):
    """[(field, field_bit)] for block bits 0, 1, 2, ... of the header."""
    out = []
    for name, a, b in _TOKEN.findall(LAYOUTS[mode]):
        a = int(a)
        b = int(b) if b else a
        step = 1 if a >= b else -1
        out.extend((name, k) for k in range(b, a + step, step))
    return out


POSITIONS = {m: _positions(m) for m in LAYOUTS}


def pack(mode: int, fields: dict, indices) -> bytes:
    """Place `fields` (stored values: rw, gw, ..., bz, d) and 16 texel indices.

    Stored values are what the block holds: deltas for transformed modes.
    Index bits above a texel's stored width must be zero (the anchors)."""
    code, _ = MODE_CODE[mode]
    vals = {k: int(v) for k, v in fields.items()}
    vals["m"] = code
    bits = 0
    pos = 0
    for name, k in POSITIONS[mode]:
        bits |= ((vals.get(name, 0) >> k) & 1) << pos
        pos += 1
    subsets = MODE_SHAPE[mode][3]
    width = 3 if subsets == 2 else 4
    anchor = ANCHOR2[vals.get("d", 0)] if subsets == 2 else -1
    for t in range(16):
        nb = width - (t == 0 or t == anchor)
        idx = int(indices[t])
        if idx >> nb:
            raise ValueError(f"index {idx} of texel {t} does not fit {nb} bits")
        bits |= idx << pos
        pos += nb
    assert pos == 128, (mode, pos)
    return bits.to_bytes(16, "little")


def header_bits(mode: int) -> int:
    return len(POSITIONS[mode])
