"""FP64 reference of the training-time decode and its gradients.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests are its
only users; the product package never imports it and shares no code with it.

What it computes (Section 4.2, "Trainable BC6 decompression"; Section 4.3;
Section 5.1): every block of every level of a feature pyramid holds
continuous parameters for the two-subset BC6H mode the features are exported
in (Section 5.2: 6-bit endpoints, 3-bit indices) with a fixed partition k:

  endpoints e[j][c], j = 0..3 (e_1..e_4 of eq. 7), in quantised units [0, 63]
  indices   x[t],    t = 0..15 (texel t at x = t & 3, y = t >> 2), in [0, 1]

Texel t of subset sigma = bit t of partition mask k takes the endpoint pair
(e_{2 sigma}, e_{2 sigma + 1}). Two ways to turn parameters into a texel:

* continuous (the paper's simulated decompression):
      ebar = (2^16 e + 2^15) / 2^6                        eq. (6), a applied below
      y    = a (ebar_A + x (ebar_B - ebar_A)),  a = 31/64  eq. (7) (reading: x in [0, 1])
      w    = 2^(h(y) - 14) (y / 1024 - h(y))               eq. (8)
  differentiable almost everywhere; the slope of eq. (8) changes where
  h(y) = max(floor((y - 1) / 1024) - 1, 0) steps.

* straight-through (the exported block): the forward value is the exact
  format decode of the quantised block (endpoints rounded to integers in
  [0, 63], indices to i = round(7 x) in [0, 7], blended with the format's
  weight omega_i / 64); the gradient is that of the continuous chain above
  evaluated at the quantised point (e rounded, x = omega_i / 64) with the
  rounding taken as the identity, and eq. (8)'s slope taken at the decoded
  half's bit pattern.

Then trilinear filtering (eq. 9, s_i = s + b_i of eq. 10, texel centres at
(i + 1/2)/w, wrap addressing), concatenation and the ReLU MLP (eq. 3), all in
binary64. Gradients come from torch's reverse-mode differentiation of this
forward, a library primitive applied to the definition.

Where floating point decides an integer the decision is taken in binary32, as
the GPU takes it: round(7 x) is evaluated on the binary32 product.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

A_UNSIGNED = 31.0 / 64.0
ENDPOINT_BITS = 6
INDEX_BITS = 3
INDEX_MAX = (1 << INDEX_BITS) - 1
ENDPOINT_MAX = (1 << ENDPOINT_BITS) - 1


def _torch():
    import torch
    return torch


def partition_masks() -> np.ndarray:
    """The 32 two-subset masks, from the oracle's own table."""
    from . import partition
    return np.array([partition(k)[0] for k in range(32)], np.int64)


def level_dim(d: int, level: int) -> int:
    return max(d >> level, 1)


@dataclass
class TrainTexture:
    """One feature pyramid with continuous block parameters (host arrays).

    endpoints:  float32 [n_blocks, 4, 3]   (e_1..e_4, r g b), all levels back to back
    indices:    float32 [n_blocks, 16]
    partitions: uint8   [n_blocks]
    """
    width: int
    height: int
    levels: int
    endpoints: np.ndarray
    indices: np.ndarray
    partitions: np.ndarray
    lod_bias: float = 0.0

    def level_blocks(self):
        """(first block, blocks across, blocks down, w, h) per level."""
        out, first = [], 0
        for l in range(self.levels):
            w, h = level_dim(self.width, l), level_dim(self.height, l)
            bx, by = (w + 3) // 4, (h + 3) // 4
            out.append((first, bx, by, w, h))
            first += bx * by
        return out


# ---------------------------------------------------------------------------
# eq. (8): a half bit pattern y as a real number

def half_value(y):
    """eq. (8) for y in [0, 31743] (torch tensor; h(y) is held constant)."""
    torch = _torch()
    h = torch.clamp(torch.floor((y.detach() - 1.0) / 1024.0) - 1.0, min=0.0)
    return torch.pow(2.0, h - 14.0) * (y / 1024.0 - h)


def half_slope(y_bits):
    """d w / d y of eq. (8) at integer bit patterns y_bits: 2^(h(y) - 24)."""
    torch = _torch()
    h = torch.clamp(torch.floor((y_bits - 1.0) / 1024.0) - 1.0, min=0.0)
    return torch.pow(2.0, h - 24.0)


# ---------------------------------------------------------------------------
# block parameters -> texels

def _unquantise_exact(e):
    """The format's integer unquantisation of a 6-bit unsigned endpoint."""
    torch = _torch()
    v = torch.div((e << 16) + 0x8000, 1 << ENDPOINT_BITS, rounding_mode="floor")
    v = torch.where(e == 0, torch.zeros_like(v), v)
    return torch.where(e == ENDPOINT_MAX, torch.full_like(v, 0xFFFF), v)


def _weights3():
    torch = _torch()
    # the format's 3-bit interpolation weights, round(64 i / 7)
    return torch.tensor([int(np.floor(64.0 * i / 7.0 + 0.5)) for i in range(8)], dtype=torch.int64)


def block_texels(endpoints, indices, partitions, ste: bool):
    """[n, 4, 3] endpoints and [n, 16] indices (fp64 tensors, possibly
    requiring grad) and [n] partitions -> texel values [n, 16, 3] (fp64)."""
    torch = _torch()
    masks = torch.from_numpy(partition_masks())[torch.as_tensor(partitions, dtype=torch.int64)]
    t = torch.arange(16)
    sigma = (masks[:, None] >> t[None, :]) & 1                       # [n, 16]
    ia = (2 * sigma)[:, :, None].expand(-1, -1, 3)                   # endpoint index of A
    e_a = torch.gather(endpoints, 1, ia)                             # [n, 16, 3]
    e_b = torch.gather(endpoints, 1, ia + 1)
    x = indices[:, :, None]
    if not ste:
        ebar_a = (65536.0 * e_a + 32768.0) / 64.0
        ebar_b = (65536.0 * e_b + 32768.0) / 64.0
        y = A_UNSIGNED * (ebar_a + x * (ebar_b - ebar_a))
        return half_value(y)
    # straight-through: forward = exact decode of the quantised block
    eq = torch.clamp(torch.round(endpoints.detach()), 0, ENDPOINT_MAX)
    x32 = torch.from_numpy((np.float32(INDEX_MAX) * indices.detach().numpy().astype(np.float32)))
    iq = torch.clamp(torch.round(x32.to(torch.float64)), 0, INDEX_MAX)       # [n, 16]
    eqa = torch.gather(eq, 1, ia).to(torch.int64)
    eqb = torch.gather(eq, 1, ia + 1).to(torch.int64)
    wgt = _weights3()[iq.to(torch.int64)][:, :, None]
    v = torch.div((64 - wgt) * _unquantise_exact(eqa) + wgt * _unquantise_exact(eqb) + 32, 64,
                  rounding_mode="floor")
    y_bits = torch.div(v * 31, 64, rounding_mode="floor").to(torch.float64)
    w_exact = half_value(y_bits).detach()
    # surrogate: the continuous chain at the quantised point, rounding as identity
    e_s = endpoints + (eq - endpoints).detach()
    x_s = indices + (_weights3()[iq.to(torch.int64)].to(torch.float64) / 64.0 - indices).detach()
    es_a = torch.gather(e_s, 1, ia)
    es_b = torch.gather(e_s, 1, ia + 1)
    xs = x_s[:, :, None]
    y_s = A_UNSIGNED * ((65536.0 * es_a + 32768.0) / 64.0
                        + xs * (65536.0 * (es_b - es_a) / 64.0))
    return w_exact + half_slope(y_bits) * (y_s - y_s.detach())


def level_images(tex: TrainTexture, endpoints, indices, ste: bool):
    """Texel images [h_l, w_l, 3] per level (levels below 4x4 use the
    top-left texels of their one block)."""
    torch = _torch()
    texels = block_texels(endpoints, indices, tex.partitions, ste)     # [n, 16, 3]
    imgs = []
    for first, bx, by, w, h in tex.level_blocks():
        yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        blk = first + (yy >> 2) * bx + (xx >> 2)
        tix = (yy & 3) * 4 + (xx & 3)
        imgs.append(texels[torch.from_numpy(blk.ravel()), torch.from_numpy(tix.ravel())].reshape(h, w, 3))
    return imgs


# ---------------------------------------------------------------------------
# eq. (9) / (10) and eq. (3)

def trilinear(tex: TrainTexture, imgs, queries: np.ndarray):
    """T_i(u, v, s_i) [n, 3] in binary64 from per-level texel images."""
    torch = _torch()
    q = queries.astype(np.float64)
    u = q[:, 0] - np.floor(q[:, 0])
    v = q[:, 1] - np.floor(q[:, 1])
    si = np.clip(q[:, 2] + tex.lod_bias, 0.0, tex.levels - 1)
    si = np.where(np.isfinite(si), si, 0.0)
    l0 = np.floor(si).astype(np.int64)
    l1 = np.minimum(l0 + 1, tex.levels - 1)
    lam = torch.from_numpy(si - l0)[:, None]
    out = torch.zeros((len(q), 3), dtype=torch.float64)

    def bilinear(level, sel):
        img = imgs[level]
        h, w = img.shape[0], img.shape[1]
        x = u[sel] * w - 0.5
        y = v[sel] * h - 0.5
        x0, y0 = np.floor(x), np.floor(y)
        fx = torch.from_numpy(x - x0)[:, None]
        fy = torch.from_numpy(y - y0)[:, None]
        x0 = x0.astype(np.int64)
        y0 = y0.astype(np.int64)
        xa, xb = torch.from_numpy(x0 % w), torch.from_numpy((x0 + 1) % w)
        ya, yb = torch.from_numpy(y0 % h), torch.from_numpy((y0 + 1) % h)
        return ((1 - fx) * (1 - fy) * img[ya, xa] + fx * (1 - fy) * img[ya, xb]
                + (1 - fx) * fy * img[yb, xa] + fx * fy * img[yb, xb])

    for level in range(tex.levels):
        s0 = l0 == level
        if s0.any():
            idx = torch.from_numpy(np.nonzero(s0)[0])
            out = out.index_add(0, idx, (1 - lam[idx]) * bilinear(level, s0))
        s1 = l1 == level
        if s1.any():
            idx = torch.from_numpy(np.nonzero(s1)[0])
            out = out.index_add(0, idx, lam[idx] * bilinear(level, s1))
    return out


def mlp(dims, params, z):
    """eq. (3)'s f_eta: ReLU after every layer but the last; params holds per
    layer W[out][in] row-major, then b[out]."""
    torch = _torch()
    off = 0
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        W = params[off: off + n_in * n_out].reshape(n_out, n_in)
        off += n_in * n_out
        b = params[off: off + n_out]
        off += n_out
        z = z @ W.T + b
        if l < len(dims) - 2:
            z = torch.relu(z)
    return z


def forward(textures, dims, params, queries, ste: bool, leaves=None):
    """G(u, v, s) [n, dims[-1]] in binary64. `leaves` (optional) supplies the
    fp64 tensors to differentiate against: ([endpoints], [indices], params)."""
    torch = _torch()
    if leaves is None:
        leaves = ([torch.from_numpy(t.endpoints.astype(np.float64)) for t in textures],
                  [torch.from_numpy(t.indices.astype(np.float64)) for t in textures],
                  torch.from_numpy(np.asarray(params, np.float64)))
    ends, idxs, p = leaves
    feats = [trilinear(t, level_images(t, e, x, ste), queries) for t, e, x in zip(textures, ends, idxs)]
    return mlp(dims, p, torch.cat(feats, dim=1))


def gradients(textures, dims, params, queries, grad_out, ste: bool):
    """Vector-Jacobian product of forward() with grad_out [n, c]:
    (forward value, [d endpoints], [d indices], d params) as float64 arrays."""
    torch = _torch()
    ends = [torch.from_numpy(t.endpoints.astype(np.float64)).requires_grad_(True) for t in textures]
    idxs = [torch.from_numpy(t.indices.astype(np.float64)).requires_grad_(True) for t in textures]
    p = torch.from_numpy(np.asarray(params, np.float64)).requires_grad_(True)
    g = forward(textures, dims, params, queries, ste, (ends, idxs, p))
    go = torch.from_numpy(np.asarray(grad_out, np.float64))
    grads = torch.autograd.grad((g * go).sum(), ends + idxs + [p], allow_unused=True)
    n = len(textures)

    def arr(x, like):
        return np.zeros(like.shape) if x is None else x.numpy()
    return (g.detach().numpy(), [arr(x, e) for x, e in zip(grads[:n], ends)],
            [arr(x, i) for x, i in zip(grads[n:2 * n], idxs)], arr(grads[2 * n], p))


def continuous_y(tex: TrainTexture) -> np.ndarray:
    """The continuous chain's y (eq. 7 times a) for every texel [n, 16, 3],
    to keep checks away from eq. (8)'s slope steps."""
    masks = partition_masks()[tex.partitions.astype(np.int64)]
    sigma = (masks[:, None] >> np.arange(16)[None, :]) & 1
    e = tex.endpoints.astype(np.float64)
    e_a = np.take_along_axis(e, (2 * sigma)[:, :, None].repeat(3, 2), 1)
    e_b = np.take_along_axis(e, (2 * sigma + 1)[:, :, None].repeat(3, 2), 1)
    x = tex.indices.astype(np.float64)[:, :, None]
    ebar_a = (65536.0 * e_a + 32768.0) / 64.0
    ebar_b = (65536.0 * e_b + 32768.0) / 64.0
    return A_UNSIGNED * (ebar_a + x * (ebar_b - ebar_a))
