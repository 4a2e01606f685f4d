"""Pins of the oracle's half conversion, block layout bookkeeping and mip-chain
sizes against values fixed by IEEE 754, by the paper and by the BC6H format."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from synth import bc6h_pack

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_half_to_double_matches_numpy_float16_for_every_pattern():
    # library routine: numpy's IEEE binary16 -> binary64
    pats = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ref = pats.view(np.float16).astype(np.float64)
    got = np.array([oracle.half_to_double(int(p)) for p in pats])
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


def test_half_cast_closed_form_eq8():
    # eq. (8): the bit reinterpretation of y in [0, 31743] as a half equals
    # 2^(h(y)-14) (y/1024 - h(y)), h(y) = max(floor((y-1)/1024) - 1, 0).
    for y in range(0, 31744):
        h = max((y - 1) // 1024 - 1, 0)
        w = Fraction(2) ** (h - 14) * (Fraction(y, 1024) - h)
        assert Fraction(oracle.half_to_double(y)) == w, y


def test_half_sign_symmetry():
    for y in range(0, 31744, 7):
        assert oracle.half_to_double(y | 0x8000) == -oracle.half_to_double(y)


@pytest.mark.parametrize("mode", range(1, 15))
def test_every_mode_spends_exactly_128_bits(mode):
    total, header, index = oracle.mode_bit_budget(mode)
    assert total == 128
    # two-subset modes: 77 endpoint + 5 partition bits, then 46 index bits;
    # one-subset modes: 60 endpoint bits, then 63 index bits
    assert (header, index) == ((82, 46) if mode <= 10 else (65, 63))
    # the independent transcription in the input packer agrees on the header size
    assert bc6h_pack.header_bits(mode) == header


def test_invalid_mode_numbers_have_no_budget():
    assert oracle.mode_bit_budget(0)[0] == -1
    assert oracle.mode_bit_budget(15)[0] == -1


def test_table2_sizes_from_table1_chains():
    spec = json.load(open(os.path.join(GOLDEN, "table2_sizes.json")))
    for name, cfg in spec["configs"].items():
        total = 0
        for res, mips in cfg["textures"]:
            # Table 1's chains end at a single 4x4 block: mips = log2(res) - 1
            assert mips == res.bit_length() - 1 - 1, (name, res, mips)
            total += oracle.texture_bytes(res, res, mips)
        assert round(total / 2 ** 20, 2) == cfg["size_mb"], (name, total)


def test_texture_bytes_counts_small_levels_as_one_block():
    # 8x8 with 4 levels: 2x2 blocks, then 4x4, 2x2 and 1x1 texels -> 1 block each
    assert oracle.texture_bytes(8, 8, 4) == 16 * (4 + 1 + 1 + 1)
    assert oracle.texture_bytes(2048, 2048, 12) == 5592432
    assert oracle.texture_bytes(256, 256, 9) == 87408
    assert oracle.texture_bytes(16, 4, 5) == 16 * (4 + 2 + 1 + 1 + 1)
    assert synth.chain_blocks(2048, 2048, 12) * 16 == 5592432
