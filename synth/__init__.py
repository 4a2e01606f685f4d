"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

Holds no decode arithmetic: only random draws, BC6H bit placement (see
`bc6h_pack`), and the renderer-side geometry that produces query (u, v, s)
streams. Both the oracle and the GPU library consume these arrays; neither is
imported here.

Workload shapes follow the paper: four square power-of-two feature pyramids
of three channels (Section "Model structure", Table 1), a small ReLU MLP with
12 inputs (Section "Model configuration"), and full-screen query counts
(Section "Decoding performance", Table 3). The paper's trained features and
its material dataset are not available, so random blocks stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import bc6h_pack
from .bc6h_pack import ANCHOR2, MODE_CODE, MODE_SHAPE, POSITIONS, RESERVED_CODES

SEED_TEXTURES, SEED_MLP, SEED_QUERIES, SEED_SHUFFLE = 1, 2, 3, 4
ALL_MODES = tuple(range(1, 15))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# mip chains

def level_dim(d: int, level: int) -> int:
    return max(d >> level, 1)


def level_blocks(w: int, h: int, level: int) -> tuple[int, int]:
    """(blocks across, blocks down) of one level."""
    return (level_dim(w, level) + 3) // 4, (level_dim(h, level) + 3) // 4


def chain_blocks(w: int, h: int, levels: int) -> int:
    return sum(bx * by for bx, by in (level_blocks(w, h, l) for l in range(levels)))


def full_levels(w: int, h: int) -> int:
    return max(w, h).bit_length()


# --------------------------------------------------------------------------
# blocks

def random_mode_blocks(n: int, g: np.random.Generator, modes=ALL_MODES) -> np.ndarray:
    """Variant R: every bit uniform except the mode code, drawn uniformly from
    `modes` (raw random bytes would make modes 1 and 2 a quarter each and give
    reserved codes an eighth of the blocks)."""
    out = g.integers(0, 256, size=(n, 16), dtype=np.uint8)
    pick = np.asarray(modes)[g.integers(0, len(modes), size=n)]
    for m in modes:
        code, width = MODE_CODE[m]
        sel = pick == m
        keep = np.uint8((0xFF << width) & 0xFF)
        out[sel, 0] = (out[sel, 0] & keep) | np.uint8(code)
    return out


def reserved_blocks(n: int, g: np.random.Generator) -> np.ndarray:
    out = g.integers(0, 256, size=(n, 16), dtype=np.uint8)
    codes = np.asarray(RESERVED_CODES, np.uint8)[g.integers(0, 4, size=n)]
    out[:, 0] = (out[:, 0] & np.uint8(0xE0)) | codes
    return out


def pack_many(mode: int, fields: dict, indices: np.ndarray) -> np.ndarray:
    """Vectorised `bc6h_pack.pack` for n blocks of one mode."""
    n = indices.shape[0]
    code, _ = MODE_CODE[mode]
    bits = np.zeros((n, 128), np.uint8)
    vals = {k: np.asarray(v, np.int64) for k, v in fields.items()}
    vals["m"] = np.full(n, code, np.int64)
    pos = 0
    for name, k in POSITIONS[mode]:
        if name in vals:
            bits[:, pos] = (vals[name] >> k) & 1
        pos += 1
    subsets = MODE_SHAPE[mode][3]
    width = 3 if subsets == 2 else 4
    anchor = np.asarray(ANCHOR2)[vals["d"]] if subsets == 2 else np.full(n, -1)
    col = np.full(n, pos, np.int64)
    rows = np.arange(n)
    for t in range(16):
        nb = width - ((t == 0) | (anchor == t)).astype(np.int64)
        idx = indices[:, t].astype(np.int64)
        for j in range(width):
            live = j < nb
            bits[rows[live], col[live] + j] = (idx[live] >> j) & 1
        col += nb
    assert np.all(col == 128)
    return np.packbits(bits, axis=1, bitorder="little")


def bounded_blocks(n: int, g: np.random.Generator, modes=ALL_MODES,
                   fraction: float = 0.48, signed: bool = False) -> np.ndarray:
    """Variant B: every endpoint is drawn below cap = floor(fraction * 2^bits)
    of its mode's precision, so every decoded UF16 texel stays below 1.0 and
    absolute error targets are meaningful. Transformed modes draw each other
    endpoint within the signed delta range of the base endpoint and store the
    delta; partitions and indices are uniform.

    signed=True draws endpoints in (-cap, cap) with cap = floor(fraction *
    2^(bits-1)) and stores them as two's complement of the mode's precision,
    so every decoded SF16 texel lies in (-1, 1)."""
    pick = np.asarray(modes)[g.integers(0, len(modes), size=n)]
    out = np.empty((n, 16), np.uint8)
    for m in modes:
        sel = np.nonzero(pick == m)[0]
        k = len(sel)
        if k == 0:
            continue
        bits, widths, transformed, subsets = MODE_SHAPE[m]
        cap = int(np.floor(fraction * (1 << (bits - 1 if signed else bits))))
        low = -cap + 1 if signed else 0
        wrap = (1 << bits) - 1
        fields = {}
        n_ep = 2 * subsets
        for c, ch in enumerate("rgb"):
            base = g.integers(low, cap, size=k)
            fields[ch + "w"] = base & wrap
            for j, name in enumerate("xyz"[: n_ep - 1]):
                if transformed:
                    half = 1 << (widths[c] - 1)
                    lo = np.maximum(low, base - half)
                    hi = np.minimum(cap - 1, base + half - 1)
                    target = lo + (g.random(k) * (hi - lo + 1)).astype(np.int64)
                    fields[ch + name] = (target - base) & ((1 << widths[c]) - 1)
                else:
                    fields[ch + name] = g.integers(low, cap, size=k) & wrap
        width = 3 if subsets == 2 else 4
        fields["d"] = g.integers(0, 32, size=k) if subsets == 2 else np.zeros(k, np.int64)
        idx = g.integers(0, 1 << width, size=(k, 16))
        idx[:, 0] >>= 1                                   # texel 0 drops its top bit
        if subsets == 2:
            anchor = np.asarray(ANCHOR2)[fields["d"]]
            idx[np.arange(k), anchor] >>= 1
        out[sel] = pack_many(m, fields, idx)
    return out


def texture_chain(res: int, levels: int, g: np.random.Generator, variant: str = "R",
                  modes=ALL_MODES) -> np.ndarray:
    """All blocks of one full chain, levels concatenated, as uint8 [bytes]."""
    n = chain_blocks(res, res, levels)
    if variant == "R":
        blocks = random_mode_blocks(n, g, modes)
    elif variant == "B":
        blocks = bounded_blocks(n, g, modes)
    else:
        raise ValueError(variant)
    return blocks.reshape(-1)


# --------------------------------------------------------------------------
# decoder MLP

def mlp_params(dims, g: np.random.Generator) -> np.ndarray:
    """Per layer W[out][in] row-major then b[out], float32, both N(0, 1/fan_in)."""
    parts = []
    for n_in, n_out in zip(dims[:-1], dims[1:]):
        sd = 1.0 / np.sqrt(n_in)
        parts.append(g.normal(0.0, sd, size=n_out * n_in))
        parts.append(g.normal(0.0, sd, size=n_out))
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------
# queries

def uniform_queries(n: int, g: np.random.Generator, s_max: float) -> np.ndarray:
    q = np.empty((n, 3), np.float32)
    q[:, 0] = g.random(n, dtype=np.float32)
    q[:, 1] = g.random(n, dtype=np.float32)
    q[:, 2] = (g.random(n) * s_max).astype(np.float32)
    return q


def perspective_queries(width: int = 3840, height: int = 2160, tex_res: int = 2048,
                        pitch_deg: float = 40.0, fov_y_deg: float = 60.0,
                        s_max: float = 11.0) -> np.ndarray:
    """Full-screen queries of a textured ground plane, in scanline order.

    Camera one unit above the plane, pitched down by `pitch_deg`, vertical
    field of view `fov_y_deg`, square pixels. Each pixel centre's ray hits the
    plane at world (X, Y); (u, v) = (X, Y) / tau wrapped to [0, 1) in binary64,
    with tau chosen so the bottom-centre pixel maps to about one level-0 texel.
    s = log2 of the larger column norm of d(u*tex_res, v*tex_res)/d(px, py),
    from the analytic Jacobian of the plane mapping (the rule of eq. 10 with
    the texture-to-screen bias folded in), clamped to [0, s_max]."""
    p = np.deg2rad(pitch_deg)
    T = np.tan(np.deg2rad(fov_y_deg) / 2)
    aspect = width / height
    px = np.arange(width, dtype=np.float64) + 0.5
    py = np.arange(height, dtype=np.float64) + 0.5
    a = (2 * px / width - 1) * T * aspect               # right component of the ray
    b = (1 - 2 * py / height) * T                       # up component of the ray
    da_dpx = 2 * T * aspect / width
    db_dpy = -2 * T / height
    D = np.sin(p) - b * np.cos(p)                       # -(ray z), > 0 below horizon
    if np.any(D <= 0):
        raise ValueError("view reaches the horizon")
    Y = (b * np.sin(p) + np.cos(p)) / D                 # per row
    dX_dpx = da_dpx / D                                 # per row
    dY_dpy = db_dpy / D ** 2                            # per row
    # bottom-centre pixel: one texel per pixel
    bottom = height - 1
    tau = tex_res * max(abs(dX_dpx[bottom]), abs(dY_dpy[bottom]))
    X = a[None, :] / D[:, None]
    dX_dpy = a[None, :] * np.cos(p) * db_dpy / D[:, None] ** 2
    col_x = np.abs(dX_dpx)[:, None] * np.ones((1, width))
    col_y = np.sqrt(dX_dpy ** 2 + dY_dpy[:, None] ** 2)
    lod = np.log2(np.maximum(col_x, col_y) * tex_res / tau)
    q = np.empty((height, width, 3), np.float32)
    u = X / tau
    v = np.broadcast_to((Y / tau)[:, None], (height, width))
    q[..., 0] = (u - np.floor(u)).astype(np.float32)
    q[..., 1] = (v - np.floor(v)).astype(np.float32)
    q[..., 2] = np.clip(lod, 0.0, s_max).astype(np.float32)
    # a value that rounds up to 1.0f wraps to 0.0
    q[..., 0][q[..., 0] >= 1.0] = 0.0
    q[..., 1][q[..., 1] >= 1.0] = 0.0
    return q.reshape(-1, 3)


# --------------------------------------------------------------------------
# named workloads

@dataclass
class Material:
    """Host arrays of one material: 3-channel BC6H pyramids + decoder MLP."""
    textures: list                       # uint8 [bytes] per texture
    res: list                            # square base resolution per texture
    levels: list
    dims: tuple
    params: np.ndarray                   # float32
    lod_bias: list = field(default_factory=list)
    signed: bool = False

    def __post_init__(self):
        if not self.lod_bias:
            self.lod_bias = [0.0] * len(self.textures)


def make_material(res, levels, dims, variant="R", modes=ALL_MODES,
                  seed_tex=SEED_TEXTURES, seed_mlp=SEED_MLP) -> Material:
    gt = rng(seed_tex)
    n_tex = len(res)
    texs = [texture_chain(res[i], levels[i], gt, variant, modes) for i in range(n_tex)]
    params = mlp_params(dims, rng(seed_mlp))
    return Material(texs, list(res), list(levels), tuple(dims), params)


@dataclass(frozen=True)
class Workload:
    name: str
    res: int
    levels: int
    dims: tuple
    n_queries: int
    kind: str                 # "uniform" or "perspective"
    s_max: float = 8.0
    grid_width: int = 0       # row length of a 2D query grid, 0 if none


WORKLOADS = {
    # 4 x 256^2, 9 levels; MLP 12-16-16-9; 65,536 uniform queries, s in [0, 8]
    "tiny": Workload("tiny", 256, 9, (12, 16, 16, 9), 65536, "uniform", 8.0),
    # 4 x 2048^2, 12 levels; MLP 12-32-32-10; 3840x2160 perspective ground plane
    "frame4k": Workload("frame4k", 2048, 12, (12, 32, 32, 10), 3840 * 2160,
                        "perspective", 11.0, 3840),
    # textures of "tiny"; MLP 12-64-64-10; 2^24 uniform queries
    "sweep": Workload("sweep", 256, 9, (12, 64, 64, 10), 1 << 24, "uniform", 8.0),
}


def workload_material(w: Workload, variant="R", modes=ALL_MODES) -> Material:
    return make_material([w.res] * 4, [w.levels] * 4, w.dims, variant, modes)


def workload_queries(w: Workload, n: int | None = None) -> np.ndarray:
    if w.kind == "perspective":
        q = perspective_queries(3840, 2160, w.res, s_max=w.s_max)
        return q if n is None else q[:n]
    return uniform_queries(w.n_queries if n is None else n, rng(SEED_QUERIES), w.s_max)


def shuffled(q: np.ndarray) -> np.ndarray:
    return q[rng(SEED_SHUFFLE).permutation(len(q))]
