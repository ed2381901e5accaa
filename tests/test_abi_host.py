"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and validates arguments before touching the device.  No GPU needed:
none of these calls reaches a HIP runtime function."""
import ctypes
import os
import re

import pytest

from paper_1409_7474_amd import lse

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lse.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(lse_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_binding_exports():
    assert sorted(lse.EXPORTS) == declared_functions()


def test_library_exports_every_declared_symbol():
    lib = lse.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_version():
    assert lse.status_str(0) == "LSE_OK"
    assert lse.status_str(-2) == "LSE_ERR_BAD_VALUE"
    assert lse.lse_version() >= 100


def test_params_default():
    p = lse.lse_params_default(256, 300, 4)
    assert (p.height, p.width, p.bands, p.term, p.order) == (256, 300, 4, 0, 0)
    assert p.dt == 15.0 and p.sigma == 1.0 and p.ksize == 7 and p.ksize_img == 9
    assert p.edge_scale == 255.0 and p.reinit_every == 1


def test_workspace_bytes_scales_with_image():
    small = lse.lse_workspace_bytes(lse.make_params(256, 256, 1))
    big = lse.lse_workspace_bytes(lse.make_params(4096, 4096, 4, sigma=1.5, ksize=11))
    assert small > 256 * 256 * 4
    # image (16 B/px) + two bit planes (1/4 B/px) + fixed overhead
    assert 4096 * 4096 * 16 < big < 4096 * 4096 * 16.5 + 65536
    edge = lse.lse_workspace_bytes(lse.make_params(1000, 1000, 3, term="edge"))
    # edge map g (4 B/px) + two bit planes: the fused edge map needs no scratch planes
    assert 1000 * 1000 * 4 < edge < 1000 * 1000 * 4.5 + 65536


@pytest.mark.parametrize("field,value", [
    ("height", 1), ("width", 0), ("bands", 0), ("bands", 5), ("term", 7), ("dt", 0.0),
    ("dt", float("nan")), ("sigma", -1.0), ("ksize", 8), ("ksize", 33), ("image_dtype", 9),
])
def test_invalid_params_rejected(field, value):
    p = lse.make_params(64, 64, 1)
    setattr(p, field, value)
    assert lse.lse_workspace_bytes(p) == 0
    ctx = ctypes.c_void_p()
    st = lse.load().lse_init(ctypes.byref(p), 16, 16, 256, 1 << 30, None, ctypes.byref(ctx))
    assert st == lse.LSE_ERR_INVALID_ARG and not ctx.value


def test_huge_image_rejected():
    p = lse.make_params(65536, 65536, 1)
    assert lse.lse_workspace_bytes(p) == 0


def test_storage_type_sizes_workspace():
    # The resident image (region) or edge map (edge) takes 2 bytes per value
    # with 16-bit storage; everything else is the same.
    for term, nb in (("region", 4), ("edge", 1)):
        sizes = {st: lse.lse_workspace_bytes(lse.make_params(512, 512, 4, term=term, storage=st))
                 for st in ("f32", "f16", "bf16")}
        assert sizes["f16"] == sizes["bf16"]
        assert sizes["f32"] - sizes["f16"] == 512 * 512 * nb * 2


def test_16bit_storage_allows_larger_images():
    # 32-bit byte offsets bound the resident copy: 2^28 pixels x 4 bands x 4 B
    # is out of range in FP32 but fits at 2 bytes per value.
    p32 = lse.make_params(16384, 16384, 4, storage="f32")
    p16 = lse.make_params(16384, 16384, 4, storage="f16")
    assert lse.lse_workspace_bytes(p32) == 0
    assert lse.lse_workspace_bytes(p16) > 0


def test_variant_modes_are_valid():
    # listing order, reinitialisation schedules and the intensity-only term
    # are implemented; they keep a continuous LSF plane in the workspace
    # (the binary-state path instead keeps, per 96 x 48 step tile, 64 bytes
    # of all-inside region sums and 64 bytes of the tile's latest
    # contribution, three one-bit-per-tile schedule masks and a visit list of
    # 1 + tiles ints; two tiles here: four 256-byte pieces)
    base = lse.lse_workspace_bytes(lse.make_params(64, 64, 4))
    for kw in ({"order": "listing"}, {"reinit_every": 0}, {"reinit_every": 3}):
        n = lse.lse_workspace_bytes(lse.make_params(64, 64, 4, **kw))
        assert n == base - 4 * 256 + 2 * 64 * 64 * 4, kw
    gray = lse.lse_workspace_bytes(lse.make_params(64, 64, 4, term="region_intensity"))
    assert gray < base  # one stored value per pixel, no normaliser boxes


def test_edge_term_requires_reinitialisation():
    p = lse.make_params(64, 64, 1, term="edge", reinit_every=0)
    assert lse.lse_workspace_bytes(p) == 0
    ctx = ctypes.c_void_p()
    st = lse.load().lse_init(ctypes.byref(p), 16, 16, 256, 1 << 30, None, ctypes.byref(ctx))
    assert st == lse.LSE_ERR_INVALID_ARG
    assert lse.lse_workspace_bytes(lse.make_params(64, 64, 1, term="edge", reinit_every=4)) > 0


def test_init_pointer_and_workspace_checks():
    lib = lse.load()
    p = lse.make_params(64, 64, 1)
    need = lse.lse_workspace_bytes(p)
    ctx = ctypes.c_void_p()
    assert lib.lse_init(ctypes.byref(p), None, 16, 256, need, None, ctypes.byref(ctx)) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_init(ctypes.byref(p), 16, None, 256, need, None, ctypes.byref(ctx)) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_init(ctypes.byref(p), 18, 16, 256, need, None, ctypes.byref(ctx)) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_init(ctypes.byref(p), 16, 16, 260, need, None, ctypes.byref(ctx)) == lse.LSE_ERR_WORKSPACE
    assert lib.lse_init(ctypes.byref(p), 16, 16, 256, need - 1, None, ctypes.byref(ctx)) == lse.LSE_ERR_WORKSPACE
    assert lib.lse_init(ctypes.byref(p), 16, 16, None, need, None, ctypes.byref(ctx)) == lse.LSE_ERR_WORKSPACE
    assert lib.lse_init(None, 16, 16, 256, need, None, ctypes.byref(ctx)) == lse.LSE_ERR_INVALID_ARG


def test_null_context_calls_fail_cleanly():
    lib = lse.load()
    assert lib.lse_step(None, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_run(None, 3, 0, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_mask(None, 16, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_lsf(None, 16, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_set_mask(None, 16, 0, 0, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_set_lsf(None, 16, None, 0, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_edge_map(None, 16, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_stats(None, None, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_profile(None, 1) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_profile(None, 8) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_profile(None, 1 | (3 << 8)) == lse.LSE_ERR_INVALID_ARG  # valid flags, no context
    assert lib.lse_step_bytes_per_pixel(None) == 0.0
    lib.lse_destroy(None)


def test_batch_argument_checks():
    lib = lse.load()
    assert lib.lse_batch_bytes(None, 0) == 0
    assert lib.lse_batch_bytes(None, 3) == 0
    out = ctypes.c_void_p()
    assert lib.lse_batch_create(None, 1, None, 256, 1 << 20, None, ctypes.byref(out)) == lse.LSE_ERR_INVALID_ARG
    assert not out.value
    arr = (ctypes.c_void_p * 2)(None, None)
    assert lib.lse_batch_create(arr, 2, None, 256, 1 << 20, None, ctypes.byref(out)) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_batch_create(arr, 0, None, 256, 1 << 20, None, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_batch_run(None, 3, 0, 0, None) == lse.LSE_ERR_INVALID_ARG
    lib.lse_batch_destroy(None)


def test_static_solve_argument_checks():
    """lse_solve_static rejects bad arguments and images beyond its fixed
    workspace on the host, before any HIP call."""
    lib = lse.load()
    small = lse.make_params(64, 64, 1)
    big = lse.make_params(2100, 2100, 4)
    assert lse.lse_workspace_bytes(small) <= lse.STATIC_WORKSPACE_BYTES < lse.lse_workspace_bytes(big)
    P = ctypes.byref
    assert lib.lse_solve_static(P(big), 16, 16, 10, 0, 16, None, None) == lse.LSE_ERR_WORKSPACE
    assert lib.lse_solve_static(P(small), 16, 16, -1, 0, 16, None, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_solve_static(P(small), 16, 16, 10, 0, None, None, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_solve_static(P(small), 16, 16, 10, 0, 16, 18, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_solve_static(None, 16, 16, 10, 0, 16, None, None) == lse.LSE_ERR_INVALID_ARG
    bad = lse.make_params(64, 64, 1)
    bad.dt = -1.0
    assert lib.lse_solve_static(P(bad), 16, 16, 10, 0, 16, None, None) == lse.LSE_ERR_INVALID_ARG


def test_tuning_table_host_side():
    """The autotuner's table: set, look up by family and size class, clear;
    invalid variants and parameters are refused.  No GPU call is involved."""
    lse.lse_tuning_clear()
    p = lse.make_params(1000, 1100, 4, term="edge", ksize=11)
    t = lse.lse_tuning_lookup(p)
    assert (t.variant, t.candidates, t.tile_rows, t.tile_cols) == (0, 0, 64, 96)
    assert t.size_class == 2  # side ~1049 rounds to 1024
    lse.lse_tuning_set(p, 2)
    assert lse.lse_tuning_lookup(p).tile_rows == 80
    # same family and size class, other size: same entry; other class: none
    assert lse.lse_tuning_lookup(lse.make_params(900, 1200, 4, term="edge", ksize=11)).variant == 2
    assert lse.lse_tuning_lookup(lse.make_params(2048, 2048, 4, term="edge", ksize=11)).variant == 0
    # other family (band count does not matter for the edge term, the radius does)
    assert lse.lse_tuning_lookup(lse.make_params(1000, 1100, 1, term="edge", ksize=11)).variant == 2
    assert lse.lse_tuning_lookup(lse.make_params(1000, 1100, 4, term="edge", ksize=13)).variant == 0
    r = lse.make_params(1000, 1100, 4, ksize=11)
    lse.lse_tuning_set(r, 1)
    t = lse.lse_tuning_lookup(r)
    assert (t.variant, t.tile_rows, t.waves_per_simd) == (1, 48, 3)
    lib = lse.load()
    assert lib.lse_tuning_set(ctypes.byref(p), 3) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_tuning_set(ctypes.byref(p), -1) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_tuning_set(None, 0) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_tuning_lookup(None, None) == lse.LSE_ERR_INVALID_ARG
    assert lib.lse_ctx_tuning(None, None) == lse.LSE_ERR_INVALID_ARG
    out = lse.lse_tuning_t()
    assert lib.lse_autotune(ctypes.byref(p), 16, 16, 256, 1 << 30, 0, None, ctypes.byref(out)) == \
        lse.LSE_ERR_INVALID_ARG  # no iterations
    lse.lse_tuning_clear()
    assert lse.lse_tuning_lookup(p).variant == 0
