"""ctypes binding of libbcf.so (include/bcf.h).

Argument marshalling only: every step of the decode runs in the library's HIP
kernels. torch provides device memory and the current stream. There is no
fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import enum
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG, "libbcf.so")
ABI_VERSION = 2


class Precision(enum.IntEnum):
    FP32 = 0
    FP16 = 1
    BF16 = 2
    FP8 = 3
    FP32_MFMA = 4


class BcfError(RuntimeError):
    pass


class _Texture(C.Structure):
    _fields_ = [("blocks", C.c_void_p), ("width", C.c_uint32), ("height", C.c_uint32),
                ("levels", C.c_uint32), ("lod_bias", C.c_float)]


class _Material(C.Structure):
    _fields_ = [("n_textures", C.c_uint32), ("textures", C.POINTER(_Texture)),
                ("n_layers", C.c_uint32), ("dims", C.POINTER(C.c_uint32)),
                ("params", C.c_void_p), ("is_signed", C.c_uint32), ("act_absmax", C.c_void_p)]


class _BatchPlan(C.Structure):
    _fields_ = [("workgroups", C.c_uint32), ("interleave", C.c_uint32), ("run", C.c_uint32),
                ("waves", C.c_uint32)]


class _TrainTexture(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("levels", C.c_uint32),
                ("lod_bias", C.c_float), ("endpoints", C.c_void_p), ("indices", C.c_void_p),
                ("partitions", C.c_void_p)]


class _TrainMaterial(C.Structure):
    _fields_ = [("n_textures", C.c_uint32), ("textures", C.POINTER(_TrainTexture)),
                ("n_layers", C.c_uint32), ("dims", C.POINTER(C.c_uint32)), ("params", C.c_void_p),
                ("straight_through", C.c_uint32)]


def _load():
    if not os.path.exists(LIBRARY):
        raise ImportError(f"{LIBRARY} is not built; run `python paper_2311_16121_amd/build.py`")
    L = C.CDLL(LIBRARY)
    L.bcf_abi_version.restype = C.c_int
    L.bcf_last_error.restype = C.c_char_p
    L.bcf_texture_bytes.restype = C.c_size_t
    L.bcf_texture_bytes.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
    L.bcf_prepare.restype = C.c_int
    L.bcf_prepare.argtypes = [C.POINTER(_Material), C.c_int, C.c_void_p, C.POINTER(C.c_size_t), C.c_void_p]
    L.bcf_decode.restype = C.c_int
    L.bcf_decode.argtypes = [C.POINTER(_Material), C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                             C.c_uint32, C.c_void_p, C.c_void_p]
    L.bcf_unpack.restype = C.c_int
    L.bcf_unpack.argtypes = [C.POINTER(_Material), C.c_void_p, C.c_void_p]
    L.bcf_decode_unpacked.restype = C.c_int
    L.bcf_decode_unpacked.argtypes = [C.POINTER(_Material), C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_uint32, C.c_void_p, C.c_void_p]
    L.bcf_calibrate.restype = C.c_int
    L.bcf_calibrate.argtypes = [C.POINTER(_Material), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                C.c_void_p]
    L.bcf_batch_workspace_size.restype = C.c_int
    L.bcf_batch_workspace_size.argtypes = [C.POINTER(_Material), C.c_uint32, C.c_int, C.POINTER(C.c_size_t)]
    L.bcf_prepare_batch.restype = C.c_int
    L.bcf_prepare_batch.argtypes = [C.POINTER(_Material), C.c_uint32, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]
    L.bcf_unpack_batch.restype = C.c_int
    L.bcf_unpack_batch.argtypes = [C.POINTER(_Material), C.c_uint32, C.c_void_p, C.c_void_p]
    L.bcf_unpack_batch_touched.restype = C.c_int
    L.bcf_unpack_batch_touched.argtypes = [C.POINTER(_Material), C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_uint32, C.c_void_p]
    L.bcf_decode_batch.restype = C.c_int
    L.bcf_decode_batch.argtypes = [C.POINTER(_Material), C.c_uint32, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_uint32, C.c_void_p, C.POINTER(_BatchPlan), C.c_void_p]
    L.bcf_tune_batch.restype = C.c_int
    L.bcf_tune_batch.argtypes = [C.POINTER(_Material), C.c_uint32, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_uint32, C.c_void_p, C.POINTER(_BatchPlan), C.POINTER(C.c_float), C.c_void_p]
    L.bcf_train_workspace_size.restype = C.c_int
    L.bcf_train_workspace_size.argtypes = [C.POINTER(_TrainMaterial), C.POINTER(C.c_size_t)]
    L.bcf_train_forward.restype = C.c_int
    L.bcf_train_forward.argtypes = [C.POINTER(_TrainMaterial), C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p, C.c_void_p]
    L.bcf_train_backward.restype = C.c_int
    L.bcf_train_backward.argtypes = [C.POINTER(_TrainMaterial), C.c_void_p, C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.c_void_p, C.c_void_p]
    L.bcf_decode_noalloc.restype = C.c_int
    L.bcf_decode_noalloc.argtypes = [C.POINTER(_Material), C.c_int, C.c_void_p, C.c_size_t, C.c_uint32,
                                     C.c_void_p, C.c_void_p]
    L.bcf_decode_blocks.restype = C.c_int
    L.bcf_decode_blocks.argtypes = [C.c_void_p, C.c_size_t, C.c_uint32, C.c_void_p, C.c_void_p]
    if L.bcf_abi_version() != ABI_VERSION:
        raise ImportError(f"libbcf ABI {L.bcf_abi_version()}, binding expects {ABI_VERSION}")
    return L


lib = _load()

EXPORTED = ("bcf_abi_version", "bcf_last_error", "bcf_texture_bytes", "bcf_prepare",
            "bcf_decode", "bcf_unpack", "bcf_decode_unpacked", "bcf_calibrate", "bcf_decode_blocks",
            "bcf_decode_noalloc",
            "bcf_batch_workspace_size", "bcf_prepare_batch", "bcf_unpack_batch", "bcf_unpack_batch_touched",
            "bcf_decode_batch",
            "bcf_tune_batch", "bcf_train_workspace_size", "bcf_train_forward", "bcf_train_backward")


def _check(status: int, what: str):
    if status != 0:
        raise BcfError(f"{what}: status {status}: {lib.bcf_last_error().decode()}")


def abi_version() -> int:
    return lib.bcf_abi_version()


def texture_bytes(width: int, height: int, levels: int) -> int:
    return int(lib.bcf_texture_bytes(width, height, levels))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Material:
    """A material on the device: BC6H pyramids + decoder MLP parameters.

    textures: list of uint8 device tensors (each a full level chain)
    sizes:    list of (width, height) or int (square)
    levels:   list of level counts
    dims:     MLP sizes (dims[0] = 3 * len(textures))
    params:   float32 device tensor, per layer W[out][in] then b[out]
    """

    def __init__(self, textures, sizes, levels, dims, params, lod_bias=None, signed=False):
        import torch
        n = len(textures)
        self.textures = [t.contiguous() for t in textures]
        self.params = params.contiguous()
        for t in self.textures:
            if t.dtype != torch.uint8 or not t.is_cuda:
                raise TypeError("textures must be uint8 device tensors")
        if self.params.dtype != torch.float32 or not self.params.is_cuda:
            raise TypeError("params must be a float32 device tensor")
        self.sizes = [(s, s) if isinstance(s, int) else tuple(s) for s in sizes]
        self.levels = list(levels)
        self.dims = tuple(int(d) for d in dims)
        self.signed = bool(signed)
        bias = list(lod_bias) if lod_bias is not None else [0.0] * n
        self._tex = (_Texture * n)()
        for i in range(n):
            w, h = self.sizes[i]
            self._tex[i] = _Texture(self.textures[i].data_ptr(), w, h, self.levels[i], float(bias[i]))
        self._dims = (C.c_uint32 * len(self.dims))(*self.dims)
        self.act_absmax = None
        self.c = _Material(n, self._tex, len(self.dims) - 1, self._dims, self.params.data_ptr(),
                           int(self.signed), None)

    def set_act_absmax(self, absmax):
        """Per-layer largest input magnitudes (device float32 [n_layers]) for BCF_FP8."""
        import torch
        a = absmax.contiguous()
        if a.dtype != torch.float32 or not a.is_cuda or a.numel() != len(self.dims) - 1:
            raise TypeError("act_absmax must be a float32 device tensor with one entry per layer")
        self.act_absmax = a
        self.c.act_absmax = a.data_ptr()

    @classmethod
    def from_host(cls, textures, sizes, levels, dims, params, lod_bias=None, signed=False,
                  device="cuda"):
        import numpy as np
        import torch
        tex = [torch.from_numpy(np.ascontiguousarray(t, np.uint8)).to(device) for t in textures]
        p = torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(device)
        return cls(tex, sizes, levels, dims, p, lod_bias, signed)

    @property
    def out_dim(self) -> int:
        return self.dims[-1]


def workspace_bytes(mat: Material, precision=Precision.FP32) -> int:
    n = C.c_size_t(0)
    _check(lib.bcf_prepare(C.byref(mat.c), int(precision), None, C.byref(n), None), "bcf_prepare(size)")
    return n.value


def prepare(mat: Material, precision=Precision.FP32, stream=None):
    """Allocate (torch) and fill the workspace for `precision`."""
    import torch
    nbytes = workspace_bytes(mat, precision)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=mat.params.device)
    off = (-ws.data_ptr()) % 256
    ws = ws[off: off + nbytes]
    n = C.c_size_t(nbytes)
    _check(lib.bcf_prepare(C.byref(mat.c), int(precision), C.c_void_p(ws.data_ptr()), C.byref(n),
                           _stream(stream)), "bcf_prepare")
    return ws


def _queries(queries):
    import torch
    q = queries.contiguous()
    if q.dtype != torch.float32 or q.dim() != 2 or q.shape[1] != 3 or not q.is_cuda:
        raise TypeError("queries must be a float32 device tensor of shape [n, 3]")
    return q


def _out(mat: Material, q, out):
    import torch
    if out is None:
        return torch.empty((q.shape[0], mat.out_dim), dtype=torch.float32, device=q.device)
    if (out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous()
            or tuple(out.shape) != (q.shape[0], mat.out_dim)):
        raise TypeError(f"out must be a contiguous float32 device tensor of shape [{q.shape[0]}, {mat.out_dim}]")
    return out


def decode(mat: Material, ws, queries, precision=Precision.FP32, grid_width: int = 0, out=None,
           stream=None):
    """queries: float32 device tensor [n, 3] (u, v, s) -> out [n, dims[-1]] float32."""
    q = _queries(queries)
    out = _out(mat, q, out)
    _check(lib.bcf_decode(C.byref(mat.c), int(precision), C.c_void_p(ws.data_ptr()),
                          C.c_void_p(q.data_ptr()), q.shape[0], grid_width, C.c_void_p(out.data_ptr()),
                          _stream(stream)), "bcf_decode")
    return out


def decode_noalloc(mat: Material, queries, precision=Precision.FP32, grid_width: int = 0, out=None,
                   stream=None):
    """decode() in the library's own per-GPU workspace (bcf_decode_noalloc):
    no workspace argument, nothing allocated by the library; `out` may be
    passed so that nothing is allocated here either."""
    q = _queries(queries)
    out = _out(mat, q, out)
    _check(lib.bcf_decode_noalloc(C.byref(mat.c), int(precision), C.c_void_p(q.data_ptr()), q.shape[0],
                                  grid_width, C.c_void_p(out.data_ptr()), _stream(stream)), "bcf_decode_noalloc")
    return out


def unpack(mat: Material, ws, stream=None):
    """Unpack every block of the material into the texel scratch of `ws`."""
    _check(lib.bcf_unpack(C.byref(mat.c), C.c_void_p(ws.data_ptr()), _stream(stream)), "bcf_unpack")


def decode_unpacked(mat: Material, ws, queries, precision=Precision.FP32, grid_width: int = 0, out=None,
                    stream=None):
    """decode() from the texels a previous unpack() left in `ws`."""
    q = _queries(queries)
    out = _out(mat, q, out)
    _check(lib.bcf_decode_unpacked(C.byref(mat.c), int(precision), C.c_void_p(ws.data_ptr()),
                                   C.c_void_p(q.data_ptr()), q.shape[0], grid_width,
                                   C.c_void_p(out.data_ptr()), _stream(stream)), "bcf_decode_unpacked")
    return out


def calibrate(mat: Material, queries, stream=None):
    """Largest input magnitude of every MLP layer over `queries` (plain fp32
    decode); returns a float32 device tensor [n_layers] for set_act_absmax."""
    import torch
    q = _queries(queries)
    ws = prepare(mat, Precision.FP32, stream)
    absmax = torch.empty(len(mat.dims) - 1, dtype=torch.float32, device=q.device)
    _check(lib.bcf_calibrate(C.byref(mat.c), C.c_void_p(ws.data_ptr()), C.c_void_p(q.data_ptr()),
                             q.shape[0], C.c_void_p(absmax.data_ptr()), _stream(stream)), "bcf_calibrate")
    return absmax


def decode_blocks(blocks, signed: bool = False, stream=None):
    """blocks: uint8 device tensor [n, 16] -> int16 device tensor [n, 16, 3] of half bit patterns."""
    import torch
    b = blocks.contiguous()
    if b.dtype != torch.uint8 or not b.is_cuda:
        raise TypeError("blocks must be a uint8 device tensor")
    n = b.numel() // 16
    out = torch.empty((n, 16, 3), dtype=torch.int16, device=b.device)
    _check(lib.bcf_decode_blocks(C.c_void_p(b.data_ptr()), n, int(signed), C.c_void_p(out.data_ptr()),
                                 _stream(stream)), "bcf_decode_blocks")
    return out


# ---------------------------------------------------------------------------
# many materials in one launch (include/bcf.h, bcf_*_batch)

class Batch:
    """Materials served together: one workspace, one persistent decode launch.

    materials: list of Material (one MLP shape); precision FP16 or FP32.
    """

    def __init__(self, materials, precision=Precision.FP16, stream=None, ws_fill=None):
        """ws_fill: a byte written over the whole workspace before it is
        prepared (lets a test see which texels an unpack wrote)."""
        import torch
        self.materials = list(materials)
        self.precision = Precision(precision)
        n = len(self.materials)
        self.c = (_Material * n)(*[m.c for m in self.materials])
        nbytes = C.c_size_t(0)
        _check(lib.bcf_batch_workspace_size(self.c, n, int(self.precision), C.byref(nbytes)),
               "bcf_batch_workspace_size")
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.materials[0].params.device)
        if ws_fill is not None:
            ws.fill_(int(ws_fill))
        off = (-ws.data_ptr()) % 256
        self.ws = ws[off: off + nbytes.value]
        _check(lib.bcf_prepare_batch(self.c, n, int(self.precision), C.c_void_p(self.ws.data_ptr()),
                                     nbytes.value, _stream(stream)), "bcf_prepare_batch")
        self.out_dim = self.materials[0].out_dim

    def __len__(self):
        return len(self.materials)

    def unpack(self, stream=None):
        _check(lib.bcf_unpack_batch(self.c, len(self), C.c_void_p(self.ws.data_ptr()), _stream(stream)),
               "bcf_unpack_batch")

    def unpack_touched(self, queries, offsets, stream=None):
        """Unpacks only the blocks these queries read (then decode() with the
        same queries and offsets)."""
        q = _queries(queries)
        offs = self._offsets(offsets)
        _check(lib.bcf_unpack_batch_touched(self.c, len(self), C.c_void_p(self.ws.data_ptr()),
                                            C.c_void_p(q.data_ptr()), C.c_void_p(offs.data_ptr()), q.shape[0],
                                            _stream(stream)), "bcf_unpack_batch_touched")

    @staticmethod
    def _offsets(offsets):
        import torch
        if offsets.dtype != torch.int32 or not offsets.is_cuda or not offsets.is_contiguous():
            raise TypeError("offsets must be a contiguous int32 device tensor (read as uint32)")
        return offsets

    def decode(self, queries, offsets, out=None, plan=None, stream=None):
        """queries [n, 3] (all materials, concatenated), offsets int32 device
        [n_materials + 1] -> out [n, out_dim]."""
        import torch
        q = _queries(queries)
        offs = self._offsets(offsets)
        if out is None:
            out = torch.empty((q.shape[0], self.out_dim), dtype=torch.float32, device=q.device)
        p = None if plan is None else C.byref(_BatchPlan(*plan))
        _check(lib.bcf_decode_batch(self.c, len(self), int(self.precision), C.c_void_p(self.ws.data_ptr()),
                                    C.c_void_p(q.data_ptr()), C.c_void_p(offs.data_ptr()), q.shape[0],
                                    C.c_void_p(out.data_ptr()), p, _stream(stream)), "bcf_decode_batch")
        return out

    def tune(self, queries, offsets, out=None, stream=None):
        """Times the candidate launch shapes; returns ((workgroups, interleave,
        run, waves), ms). A plan for decode() is such a tuple (trailing
        entries may be left out: run 1, waves 4)."""
        import torch
        q = _queries(queries)
        offs = self._offsets(offsets)
        if out is None:
            out = torch.empty((q.shape[0], self.out_dim), dtype=torch.float32, device=q.device)
        best = _BatchPlan()
        ms = C.c_float(0)
        _check(lib.bcf_tune_batch(self.c, len(self), int(self.precision), C.c_void_p(self.ws.data_ptr()),
                                  C.c_void_p(q.data_ptr()), C.c_void_p(offs.data_ptr()), q.shape[0],
                                  C.c_void_p(out.data_ptr()), C.byref(best), C.byref(ms), _stream(stream)),
               "bcf_tune_batch")
        return (best.workgroups, best.interleave, best.run, best.waves), ms.value


# ---------------------------------------------------------------------------
# training-time decode (include/bcf.h, bcf_train_*)

class TrainGeometry:
    """Everything about a trainable material except its trainable tensors:
    pyramid sizes and level counts, the fixed partition ids (uint8 device
    tensors, one per pyramid), MLP dims, LOD biases and the rounding mode."""

    def __init__(self, sizes, levels, partitions, dims, lod_bias=None, straight_through=False):
        import torch
        self.sizes = [(s, s) if isinstance(s, int) else tuple(s) for s in sizes]
        self.levels = list(levels)
        self.partitions = [p.contiguous() for p in partitions]
        for p in self.partitions:
            if p.dtype != torch.uint8 or not p.is_cuda:
                raise TypeError("partitions must be uint8 device tensors")
        self.dims = tuple(int(d) for d in dims)
        self.lod_bias = list(lod_bias) if lod_bias is not None else [0.0] * len(self.sizes)
        self.straight_through = bool(straight_through)

    def struct(self, endpoints, indices, params):
        n = len(self.sizes)
        tex = (_TrainTexture * n)()
        for i in range(n):
            w, h = self.sizes[i]
            tex[i] = _TrainTexture(w, h, self.levels[i], float(self.lod_bias[i]), endpoints[i].data_ptr(),
                                   indices[i].data_ptr(), self.partitions[i].data_ptr())
        dims = (C.c_uint32 * len(self.dims))(*self.dims)
        m = _TrainMaterial(n, tex, len(self.dims) - 1, dims, params.data_ptr(), int(self.straight_through))
        m._keep = (tex, dims)
        return m

    def workspace(self, m, device):
        import torch
        nbytes = C.c_size_t(0)
        _check(lib.bcf_train_workspace_size(C.byref(m), C.byref(nbytes)), "bcf_train_workspace_size")
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        return ws[off: off + nbytes.value]


def _check_train_tensors(geo, endpoints, indices, params):
    import torch
    for t in list(endpoints) + list(indices) + [params]:
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise TypeError("trainable tensors must be contiguous float32 device tensors")
    if len(endpoints) != len(geo.sizes) or len(indices) != len(geo.sizes):
        raise ValueError("one endpoints and one indices tensor per pyramid")


def train_forward(geo: TrainGeometry, endpoints, indices, params, queries, stream=None):
    """G(u, v, s) [n, dims[-1]] from the current trainable tensors (no autograd)."""
    import torch
    _check_train_tensors(geo, endpoints, indices, params)
    q = _queries(queries)
    m = geo.struct(endpoints, indices, params)
    ws = geo.workspace(m, q.device)
    out = torch.empty((q.shape[0], geo.dims[-1]), dtype=torch.float32, device=q.device)
    _check(lib.bcf_train_forward(C.byref(m), C.c_void_p(ws.data_ptr()), C.c_void_p(q.data_ptr()), q.shape[0],
                                 C.c_void_p(out.data_ptr()), _stream(stream)), "bcf_train_forward")
    return out


def train_backward(geo: TrainGeometry, endpoints, indices, params, queries, grad_out, stream=None):
    """(d endpoints list, d indices list, d params) for dL/dG = grad_out."""
    import torch
    _check_train_tensors(geo, endpoints, indices, params)
    q = _queries(queries)
    go = grad_out.contiguous()
    if go.dtype != torch.float32 or tuple(go.shape) != (q.shape[0], geo.dims[-1]):
        raise TypeError("grad_out must be float32 [n, dims[-1]]")
    m = geo.struct(endpoints, indices, params)
    ws = geo.workspace(m, q.device)
    g_end = [torch.empty_like(e) for e in endpoints]
    g_idx = [torch.empty_like(x) for x in indices]
    g_par = torch.empty_like(params)
    n = len(endpoints)
    ge = (C.c_void_p * n)(*[t.data_ptr() for t in g_end])
    gi = (C.c_void_p * n)(*[t.data_ptr() for t in g_idx])
    _check(lib.bcf_train_backward(C.byref(m), C.c_void_p(ws.data_ptr()), C.c_void_p(q.data_ptr()), q.shape[0],
                                  C.c_void_p(go.data_ptr()), ge, gi, C.c_void_p(g_par.data_ptr()),
                                  _stream(stream)), "bcf_train_backward")
    return g_end, g_idx, g_par


_TRAIN_FN = None


def _train_function():
    global _TRAIN_FN
    if _TRAIN_FN is None:
        import torch

        class TrainDecode(torch.autograd.Function):
            """G(u, v, s) as a differentiable function of the block parameters
            and the MLP parameters; backward runs the library's kernels."""

            @staticmethod
            def forward(ctx, geo, queries, params, *leaves):
                n = len(geo.sizes)
                ends, idxs = list(leaves[:n]), list(leaves[n:])
                ctx.geo = geo
                ctx.save_for_backward(queries, params, *leaves)
                return train_forward(geo, ends, idxs, params, queries)

            @staticmethod
            def backward(ctx, grad_out):
                geo = ctx.geo
                queries, params, *leaves = ctx.saved_tensors
                n = len(geo.sizes)
                g_end, g_idx, g_par = train_backward(geo, leaves[:n], leaves[n:], params, queries,
                                                     grad_out.contiguous())
                return (None, None, g_par, *g_end, *g_idx)

        _TRAIN_FN = TrainDecode
    return _TRAIN_FN


def train_decode(geo: TrainGeometry, endpoints, indices, params, queries):
    """Differentiable training-time decode: a torch.autograd.Function whose
    backward is bcf_train_backward (gradients for endpoints, indices and
    params; none for the queries)."""
    return _train_function().apply(geo, queries, params, *endpoints, *indices)
