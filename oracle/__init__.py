"""ctypes binding of the plain CPU oracle (bcf_oracle.c).

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only permitted users; the product package never
imports this module and shares no code with it.

Everything the oracle computes is binary64 on the host: BC6H decode written
from the format definition, trilinear filtering (eq. 9) at the per-texture
scale of eq. (10), and the decoder MLP of eq. (3).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "bcf_oracle.c")
LIBRARY = os.path.join(HERE, "liboracle.so")


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
           SOURCE, "-o", LIBRARY, "-lm"]
    subprocess.run(cmd, check=True)
    return LIBRARY


class _Texture(C.Structure):
    _fields_ = [("blocks", C.c_void_p), ("width", C.c_uint32), ("height", C.c_uint32),
                ("levels", C.c_uint32), ("lod_bias", C.c_double)]


class _Material(C.Structure):
    _fields_ = [("n_textures", C.c_uint32), ("textures", C.POINTER(_Texture)),
                ("n_layers", C.c_uint32), ("dims", C.POINTER(C.c_uint32)),
                ("params", C.c_void_p), ("is_signed", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build()
        L = C.CDLL(LIBRARY)
        L.bcfo_half_to_double.restype = C.c_double
        L.bcfo_half_to_double.argtypes = [C.c_uint16]
        L.bcfo_decode_block.restype = C.c_int
        L.bcfo_decode_block.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.bcfo_decode_blocks.restype = None
        L.bcfo_decode_blocks.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        L.bcfo_block_fields.restype = C.c_int
        L.bcfo_block_fields.argtypes = [C.c_void_p, C.c_void_p]
        L.bcfo_partition.restype = C.c_int
        L.bcfo_partition.argtypes = [C.c_int, C.POINTER(C.c_uint16), C.POINTER(C.c_int)]
        L.bcfo_mode_bit_budget.restype = C.c_int
        L.bcfo_mode_bit_budget.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.bcfo_texture_bytes.restype = C.c_size_t
        L.bcfo_texture_bytes.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        for name in ("bcfo_sample", "bcfo_decode"):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = [C.POINTER(_Material), C.c_void_p, C.c_size_t, C.c_void_p, C.c_int]
        L.bcfo_mlp.restype = None
        L.bcfo_mlp.argtypes = [C.POINTER(_Material), C.c_void_p, C.c_size_t, C.c_void_p]
        _lib = L
    return _lib


def half_to_double(h: int) -> float:
    return lib().bcfo_half_to_double(int(h))


def decode_block(block, signed: bool = False):
    """One 16-byte block -> (mode number or 0, uint16 [16, 3] half bit patterns)."""
    b = np.ascontiguousarray(np.frombuffer(bytes(block), np.uint8))
    out = np.zeros((16, 3), np.uint16)
    mode = lib().bcfo_decode_block(b.ctypes.data, int(signed), out.ctypes.data)
    return mode, out


def decode_blocks(blocks: np.ndarray, signed: bool = False) -> np.ndarray:
    b = np.ascontiguousarray(blocks, np.uint8).reshape(-1, 16)
    out = np.zeros((b.shape[0], 16, 3), np.uint16)
    lib().bcfo_decode_blocks(b.ctypes.data, b.shape[0], int(signed), out.ctypes.data)
    return out


def block_fields(block) -> dict:
    b = np.ascontiguousarray(np.frombuffer(bytes(block), np.uint8))
    f = np.zeros(14, np.int32)
    lib().bcfo_block_fields(b.ctypes.data, f.ctypes.data)
    names = ["rw", "gw", "bw", "rx", "gx", "bx", "ry", "gy", "by", "rz", "gz", "bz", "d", "mode"]
    return {k: int(v) for k, v in zip(names, f)}


def partition(k: int):
    """(mask, anchor) of two-subset partition k: mask bit t puts texel t in subset 1."""
    mask, anchor = C.c_uint16(0), C.c_int(0)
    if lib().bcfo_partition(k, C.byref(mask), C.byref(anchor)) != 0:
        raise ValueError(f"partition {k} out of range")
    return int(mask.value), int(anchor.value)


def mode_bit_budget(mode: int):
    h, i = C.c_int(), C.c_int()
    total = lib().bcfo_mode_bit_budget(mode, C.byref(h), C.byref(i))
    return total, h.value, i.value


def texture_bytes(w: int, h: int, levels: int) -> int:
    return int(lib().bcfo_texture_bytes(w, h, levels))


class Material:
    """Keeps the ctypes view of a material and the arrays it points into alive."""

    def __init__(self, textures, res, levels, dims, params, lod_bias=None, signed=False):
        n = len(textures)
        self._blocks = [np.ascontiguousarray(t, np.uint8) for t in textures]
        self._tex = (_Texture * n)()
        bias = lod_bias if lod_bias is not None else [0.0] * n
        for i in range(n):
            r = res[i]
            w, h = (r, r) if np.isscalar(r) else r
            self._tex[i] = _Texture(self._blocks[i].ctypes.data, w, h, levels[i], float(bias[i]))
        self._dims = np.ascontiguousarray(dims, np.uint32)
        self._params = np.ascontiguousarray(params, np.float32)
        self.dims = tuple(int(d) for d in dims)
        self.c = _Material(n, self._tex, len(dims) - 1,
                           self._dims.ctypes.data_as(C.POINTER(C.c_uint32)),
                           self._params.ctypes.data, int(signed))

    @classmethod
    def from_synth(cls, m):
        return cls(m.textures, m.res, m.levels, m.dims, m.params, m.lod_bias, m.signed)


# Threads used when the caller does not say: the CPUs this process may run on,
# at most 16 (the host share of one GPU on the GPU machines).
MAX_THREADS = 16


def default_threads() -> int:
    return max(1, min(MAX_THREADS, len(os.sched_getaffinity(0))))


def _threads(n_threads):
    return n_threads if n_threads else default_threads()


def sample(mat: Material, queries: np.ndarray, n_threads: int = 0) -> np.ndarray:
    q = np.ascontiguousarray(queries, np.float32).reshape(-1, 3)
    out = np.zeros((q.shape[0], 3 * len(mat._blocks)), np.float64)
    lib().bcfo_sample(C.byref(mat.c), q.ctypes.data, q.shape[0], out.ctypes.data,
                      _threads(n_threads))
    return out


def mlp(mat: Material, z: np.ndarray) -> np.ndarray:
    z = np.ascontiguousarray(z, np.float64).reshape(-1, mat.dims[0])
    out = np.zeros((z.shape[0], mat.dims[-1]), np.float64)
    lib().bcfo_mlp(C.byref(mat.c), z.ctypes.data, z.shape[0], out.ctypes.data)
    return out


def decode(mat: Material, queries: np.ndarray, n_threads: int = 0) -> np.ndarray:
    q = np.ascontiguousarray(queries, np.float32).reshape(-1, 3)
    out = np.zeros((q.shape[0], mat.dims[-1]), np.float64)
    lib().bcfo_decode(C.byref(mat.c), q.ctypes.data, q.shape[0], out.ctypes.data,
                      _threads(n_threads))
    return out
