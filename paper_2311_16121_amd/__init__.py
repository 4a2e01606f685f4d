"""Block-compressed neural material decode on AMD Instinct MI355X (gfx950).

Per query (u, v, s): fetch the BC6H blocks of every feature pyramid, unpack
them to half texels, filter trilinearly (eq. 9 at s_i = s + b_i, eq. 10),
concatenate, and run the decoder MLP (eq. 3) -- all in HIP kernels behind
the C ABI of include/bcf.h. This package is the thin Python binding.
"""
from ._lib import (ABI_VERSION, EXPORTED, BcfError, Batch, Material, Precision, TrainGeometry, abi_version,
                   calibrate, decode, decode_blocks, decode_noalloc, decode_unpacked, lib, prepare, texture_bytes,
                   train_backward, train_decode, train_forward, unpack, workspace_bytes)

__all__ = ["ABI_VERSION", "EXPORTED", "BcfError", "Batch", "Material", "Precision", "TrainGeometry", "abi_version",
           "calibrate", "decode", "decode_blocks", "decode_noalloc", "decode_unpacked", "lib", "prepare",
           "texture_bytes",
           "train_backward", "train_decode", "train_forward", "unpack", "workspace_bytes"]
