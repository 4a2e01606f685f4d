"""The C ABI on the CPU: the library loads, exports every symbol include/bcf.h
declares, and rejects invalid arguments with status codes before touching the
GPU (validation never dereferences device pointers, so fake aligned addresses
suffice here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bcf():
    import paper_2311_16121_amd as bcf
    return bcf


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bcf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcf_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(bcf):
    names = declared_functions()
    assert set(names) == set(bcf.EXPORTED)
    for name in names:
        assert hasattr(bcf.lib, name), name


def test_abi_version(bcf):
    assert bcf.abi_version() == 2


def test_texture_bytes_matches_oracle_and_rejects_bad_sizes(bcf):
    for w, h, L in [(2048, 2048, 12), (256, 256, 9), (64, 16, 7), (8, 32, 6), (1, 1, 1), (512, 512, 8)]:
        assert bcf.texture_bytes(w, h, L) == oracle.texture_bytes(w, h, L)
    for w, h, L in [(3, 4, 1), (4, 4, 0), (4, 4, 4), (0, 4, 1), (65536, 4, 1)]:
        assert bcf.texture_bytes(w, h, L) == 0


FAKE = 1 << 20          # an aligned, non-null address never dereferenced here


def material(bcf, n_tex=4, res=256, levels=9, dims=(12, 16, 16, 9), blocks=FAKE, params=FAKE,
             signed=0, bias=0.0):
    from paper_2311_16121_amd._lib import _Material, _Texture
    tex = (_Texture * max(n_tex, 1))()
    for i in range(n_tex):
        w, h = (res, res) if isinstance(res, int) else res
        tex[i] = _Texture(blocks, w, h, levels, bias)
    d = (C.c_uint32 * len(dims))(*dims)
    m = _Material(n_tex, tex, len(dims) - 1, d, params, signed, None)
    m._keep = (tex, d)
    return m


def size_query(bcf, m, precision=0):
    n = C.c_size_t(0)
    st = bcf.lib.bcf_prepare(C.byref(m), precision, None, C.byref(n), None)
    return st, n.value, bcf.lib.bcf_last_error().decode()


def test_valid_material_size_query(bcf):
    # four 256^2 pyramids of one geometry: 87,381 texel positions per pyramid
    # chain, packed four pyramids to a 24-byte position
    st, n, _ = size_query(bcf, material(bcf))
    assert st == 0 and n > 87381 * 24
    for p in (1, 2, 4):
        assert size_query(bcf, material(bcf), p)[0] == 0


@pytest.mark.parametrize("kwargs,status,msg", [
    (dict(n_tex=0), 1, "n_textures"),
    (dict(n_tex=5, dims=(15, 16, 9)), 1, "n_textures"),
    (dict(blocks=0), 1, "blocks is NULL"),
    (dict(blocks=FAKE + 8), 1, "16-byte"),
    (dict(res=(300, 256)), 1, "power-of-two"),
    (dict(levels=10), 1, "levels"),
    (dict(levels=0), 1, "levels"),
    (dict(dims=(11, 16, 9)), 1, "dims[0]"),
    (dict(dims=(12, 9)), 2, "n_layers"),
    (dict(dims=(12, 65, 9)), 2, "hidden"),
    (dict(dims=(12, 16, 17)), 2, "output"),
    (dict(params=0), 1, "params"),
    (dict(signed=2), 1, "is_signed"),
    (dict(bias=float("nan")), 1, "lod_bias"),
])
def test_invalid_materials_are_rejected(bcf, kwargs, status, msg):
    st, _, err = size_query(bcf, material(bcf, **kwargs))
    assert st == status
    assert msg in err


def test_unsupported_precision_and_null_arguments(bcf):
    m = material(bcf)
    assert size_query(bcf, m, 3)[0] == 0              # fp8 size query needs no scales
    n = C.c_size_t(1 << 40)
    assert bcf.lib.bcf_prepare(C.byref(m), 3, C.c_void_p(FAKE), C.byref(n), None) == 1
    assert "act_absmax" in bcf.lib.bcf_last_error().decode()
    st, _, err = size_query(bcf, m, 99)
    assert st == 2 and "precision" in err
    assert bcf.lib.bcf_prepare(None, 0, None, C.byref(C.c_size_t()), None) == 1
    assert bcf.lib.bcf_prepare(C.byref(m), 0, None, None, None) == 1
    # workspace too small / misaligned
    n = C.c_size_t(100)
    assert bcf.lib.bcf_prepare(C.byref(m), 0, C.c_void_p(FAKE), C.byref(n), None) == 1
    assert "workspace" in bcf.lib.bcf_last_error().decode()
    n = C.c_size_t(1 << 40)
    assert bcf.lib.bcf_prepare(C.byref(m), 0, C.c_void_p(FAKE + 16), C.byref(n), None) == 1
    # decode: n == 0 is a no-op that touches nothing
    assert bcf.lib.bcf_decode(C.byref(m), 0, None, None, 0, 0, None, None) == 0
    assert bcf.lib.bcf_decode(C.byref(m), 0, None, C.c_void_p(FAKE), 5, 0, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode(C.byref(m), 0, C.c_void_p(FAKE), None, 5, 0, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode(C.byref(m), 0, C.c_void_p(FAKE), C.c_void_p(FAKE), 5, 0, None, None) == 1
    assert bcf.lib.bcf_decode(C.byref(m), 0, C.c_void_p(FAKE), C.c_void_p(FAKE + 2), 5, 0,
                              C.c_void_p(FAKE), None) == 1
    # the two halves of decode
    assert bcf.lib.bcf_unpack(C.byref(m), None, None) == 1
    assert bcf.lib.bcf_unpack(C.byref(m), C.c_void_p(FAKE + 16), None) == 1
    assert bcf.lib.bcf_unpack(C.byref(material(bcf, levels=0)), C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode_unpacked(C.byref(m), 0, None, None, 0, 0, None, None) == 0
    assert bcf.lib.bcf_decode_unpacked(C.byref(m), 0, None, C.c_void_p(FAKE), 5, 0, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode_unpacked(C.byref(m), 99, C.c_void_p(FAKE), C.c_void_p(FAKE), 5, 0,
                                       C.c_void_p(FAKE), None) == 2
    # calibrate
    assert bcf.lib.bcf_calibrate(C.byref(m), None, C.c_void_p(FAKE), 5, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_calibrate(C.byref(m), C.c_void_p(FAKE), C.c_void_p(FAKE), 5, None, None) == 1
    assert bcf.lib.bcf_calibrate(C.byref(m), C.c_void_p(FAKE), None, 5, C.c_void_p(FAKE), None) == 1
    # decode_blocks
    assert bcf.lib.bcf_decode_blocks(None, 0, 0, None, None) == 0
    assert bcf.lib.bcf_decode_blocks(None, 4, 0, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode_blocks(C.c_void_p(FAKE + 4), 4, 0, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode_blocks(C.c_void_p(FAKE), 4, 2, C.c_void_p(FAKE), None) == 1


def test_error_text_is_thread_local(bcf):
    import threading
    size_query(bcf, material(bcf, n_tex=0))
    seen = {}

    def other():
        size_query(bcf, material(bcf, levels=0))
        seen["other"] = bcf.lib.bcf_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert "levels" in seen["other"]
    assert "n_textures" in bcf.lib.bcf_last_error().decode()


def train_material(bcf, n_tex=4, res=32, levels=6, dims=(12, 32, 32, 10), ste=0, ptr=FAKE, bias=0.0):
    from paper_2311_16121_amd._lib import _TrainMaterial, _TrainTexture
    tex = (_TrainTexture * max(n_tex, 1))()
    for i in range(n_tex):
        w, h = (res, res) if isinstance(res, int) else res
        tex[i] = _TrainTexture(w, h, levels, bias, ptr, ptr, ptr)
    d = (C.c_uint32 * len(dims))(*dims)
    m = _TrainMaterial(n_tex, tex, len(dims) - 1, d, FAKE, ste)
    m._keep = (tex, d)
    return m


def test_train_workspace_size(bcf):
    n = C.c_size_t(0)
    assert bcf.lib.bcf_train_workspace_size(C.byref(train_material(bcf)), C.byref(n)) == 0
    texels = 4 * sum(max(32 >> l, 1) ** 2 for l in range(6))
    # two texel images, then the backward's sample sort: 2^20 sorted indices,
    # two tables of 64 x 64 cells and 12 floats of dL/dz per sample; then the
    # forward's MLP operands (a few KiB, 256-byte aligned)
    base = 2 * ((texels * 16 + 255) // 256 * 256) + 4 * 2 ** 20 + 2 * 4 * 64 * 64 + 48 * 2 ** 20
    assert n.value % 256 == 0 and 1024 <= n.value - base <= 64 * 1024


@pytest.mark.parametrize("kwargs,status,msg", [
    (dict(n_tex=0), 1, "n_textures"),
    (dict(res=(48, 32)), 1, "power-of-two"),
    (dict(levels=7), 1, "levels"),
    (dict(ptr=0), 1, "NULL"),
    (dict(ste=2), 1, "straight_through"),
    (dict(dims=(12, 64, 10)), 2, "16 or 32"),
    (dict(dims=(12, 32, 16, 10)), 2, "16 or 32"),
    (dict(dims=(9, 32, 10)), 1, "dims[0]"),
    (dict(dims=(12, 32, 17)), 2, "output"),
    (dict(dims=(12, 10)), 2, "n_layers"),
    (dict(bias=float("inf")), 1, "lod_bias"),
])
def test_train_material_validation(bcf, kwargs, status, msg):
    n = C.c_size_t(0)
    st = bcf.lib.bcf_train_workspace_size(C.byref(train_material(bcf, **kwargs)), C.byref(n))
    assert st == status
    assert msg in bcf.lib.bcf_last_error().decode()


def test_train_call_argument_checks(bcf):
    m = train_material(bcf)
    assert bcf.lib.bcf_train_workspace_size(C.byref(m), None) == 1
    # forward: n == 0 touches nothing
    assert bcf.lib.bcf_train_forward(C.byref(m), None, None, 0, None, None) == 0
    assert bcf.lib.bcf_train_forward(C.byref(m), C.c_void_p(FAKE + 8), C.c_void_p(FAKE), 5, C.c_void_p(FAKE),
                                     None) == 1
    assert bcf.lib.bcf_train_forward(C.byref(m), C.c_void_p(FAKE), None, 5, C.c_void_p(FAKE), None) == 1
    ptrs = (C.c_void_p * 4)(*([FAKE] * 4))
    nulls = (C.c_void_p * 4)(FAKE, FAKE, 0, FAKE)
    args = [C.byref(m), C.c_void_p(FAKE), C.c_void_p(FAKE), 5, C.c_void_p(FAKE)]
    assert bcf.lib.bcf_train_backward(*args, None, ptrs, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_train_backward(*args, ptrs, nulls, C.c_void_p(FAKE), None) == 1
    assert "texture 2" in bcf.lib.bcf_last_error().decode()
    assert bcf.lib.bcf_train_backward(*args, ptrs, ptrs, None, None) == 1


def test_batch_validation(bcf):
    from paper_2311_16121_amd._lib import _Material
    mats = [material(bcf), material(bcf, res=(64, 16), levels=5), material(bcf, n_tex=2, dims=(6, 16, 16, 9))]
    arr = (_Material * 3)(*mats)
    n = C.c_size_t(0)
    # dims differ between material 0 and 2
    assert bcf.lib.bcf_batch_workspace_size(arr, 3, 1, C.byref(n)) == 1
    assert "material 2" in bcf.lib.bcf_last_error().decode()
    assert bcf.lib.bcf_batch_workspace_size(arr, 2, 1, C.byref(n)) == 0
    two = n.value
    single = C.c_size_t(0)
    assert bcf.lib.bcf_batch_workspace_size(arr, 1, 1, C.byref(single)) == 0
    assert two > single.value > 0
    # precisions other than FP16 / FP32, an empty batch, a bad member
    assert bcf.lib.bcf_batch_workspace_size(arr, 2, 2, C.byref(n)) == 2
    assert bcf.lib.bcf_batch_workspace_size(arr, 0, 1, C.byref(n)) == 1
    bad = (_Material * 2)(mats[0], material(bcf, levels=0))
    assert bcf.lib.bcf_batch_workspace_size(bad, 2, 0, C.byref(n)) == 1
    assert "material 1" in bcf.lib.bcf_last_error().decode()
    # decode argument checks
    assert bcf.lib.bcf_decode_batch(arr, 2, 1, C.c_void_p(FAKE), C.c_void_p(FAKE), None, 10,
                                    C.c_void_p(FAKE), None, None) == 1
    assert bcf.lib.bcf_decode_batch(arr, 2, 1, C.c_void_p(FAKE + 8), C.c_void_p(FAKE), C.c_void_p(FAKE), 10,
                                    C.c_void_p(FAKE), None, None) == 1
    assert bcf.lib.bcf_decode_batch(arr, 2, 1, C.c_void_p(FAKE), None, C.c_void_p(FAKE), 10,
                                    C.c_void_p(FAKE), None, None) == 1
    assert bcf.lib.bcf_prepare_batch(arr, 2, 1, C.c_void_p(FAKE), 100, None) == 1
    assert "workspace" in bcf.lib.bcf_last_error().decode()
    # launch shapes outside what the kernels take
    from paper_2311_16121_amd._lib import _BatchPlan
    for plan, msg in (((0, 1, 1, 3), "waves"), ((0, 1, 65, 4), "run")):
        p = _BatchPlan(*plan)
        assert bcf.lib.bcf_decode_batch(arr, 2, 1, C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), 10,
                                        C.c_void_p(FAKE), C.byref(p), None) == 1
        assert msg in bcf.lib.bcf_last_error().decode()
    # the touched-blocks unpack: argument checks before any launch
    touched = bcf.lib.bcf_unpack_batch_touched
    assert touched(arr, 2, C.c_void_p(FAKE), C.c_void_p(FAKE), None, 10, None) == 1
    assert "offsets" in bcf.lib.bcf_last_error().decode()
    assert touched(arr, 2, C.c_void_p(FAKE), C.c_void_p(FAKE + 2), C.c_void_p(FAKE), 10, None) == 1
    assert "queries" in bcf.lib.bcf_last_error().decode()
    assert touched(arr, 2, C.c_void_p(FAKE + 8), C.c_void_p(FAKE), C.c_void_p(FAKE), 10, None) == 1
    assert "workspace" in bcf.lib.bcf_last_error().decode()
    assert touched(arr, 2, C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), 10, None) == 1
    assert "bcf_prepare_batch" in bcf.lib.bcf_last_error().decode()
    assert touched(arr, 0, C.c_void_p(FAKE), C.c_void_p(FAKE), C.c_void_p(FAKE), 10, None) == 1


def test_workspace_not_filled_by_prepare_is_rejected(bcf):
    # The library remembers, per workspace address, what bcf_prepare filled it
    # for; an address it never prepared is an argument error, found on the
    # host before any launch.
    m = material(bcf)
    ws = C.c_void_p(FAKE + (1 << 16))
    calls = [
        ("bcf_decode", lambda: bcf.lib.bcf_decode(C.byref(m), 1, ws, C.c_void_p(FAKE), 5, 0, C.c_void_p(FAKE), None)),
        ("bcf_decode_unpacked", lambda: bcf.lib.bcf_decode_unpacked(C.byref(m), 1, ws, C.c_void_p(FAKE), 5, 0,
                                                                    C.c_void_p(FAKE), None)),
        ("bcf_unpack", lambda: bcf.lib.bcf_unpack(C.byref(m), ws, None)),
        ("bcf_calibrate", lambda: bcf.lib.bcf_calibrate(C.byref(m), ws, C.c_void_p(FAKE), 5, C.c_void_p(FAKE), None)),
    ]
    for name, call in calls:
        assert call() == 1, name
        assert "not filled by bcf_prepare" in bcf.lib.bcf_last_error().decode(), name
    from paper_2311_16121_amd._lib import _Material
    arr = (_Material * 2)(material(bcf), material(bcf, res=(64, 16), levels=5))
    assert bcf.lib.bcf_unpack_batch(arr, 2, ws, None) == 1
    assert "not filled by bcf_prepare_batch" in bcf.lib.bcf_last_error().decode()
    assert bcf.lib.bcf_decode_batch(arr, 2, 1, ws, C.c_void_p(FAKE), C.c_void_p(FAKE), 10,
                                    C.c_void_p(FAKE), None, None) == 1
    assert "not filled by bcf_prepare_batch" in bcf.lib.bcf_last_error().decode()


def test_noalloc_refuses_oversized_materials_and_bad_arguments_before_any_launch(bcf):
    big = material(bcf, res=2048, levels=12, dims=(12, 32, 32, 10))
    assert bcf.lib.bcf_decode_noalloc(C.byref(big), 1, C.c_void_p(FAKE), 5, 0, C.c_void_p(FAKE), None) == 2
    err = bcf.lib.bcf_last_error().decode()
    assert "workspace" in err and str(64 << 20) in err
    m = material(bcf)
    assert bcf.lib.bcf_decode_noalloc(C.byref(m), 1, None, 0, 0, None, None) == 0          # n == 0: no-op
    assert bcf.lib.bcf_decode_noalloc(C.byref(m), 1, None, 5, 0, C.c_void_p(FAKE), None) == 1
    assert bcf.lib.bcf_decode_noalloc(C.byref(m), 1, C.c_void_p(FAKE), 5, 0, None, None) == 1
    assert bcf.lib.bcf_decode_noalloc(C.byref(m), 3, C.c_void_p(FAKE), 5, 0, C.c_void_p(FAKE), None) == 1
    assert "act_absmax" in bcf.lib.bcf_last_error().decode()
    assert bcf.lib.bcf_decode_noalloc(C.byref(m), 99, C.c_void_p(FAKE), 5, 0, C.c_void_p(FAKE), None) == 2
