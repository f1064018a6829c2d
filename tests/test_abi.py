"""The C-ABI library loads and exports every entry point that include/lens.h
declares, and rejects bad host-side arguments before touching the device.
No GPU is needed: no call here reaches a kernel launch."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lens.h")
LIB = os.path.join(ROOT, "paper_1902_03252_amd", "liblens.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lens_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblens.so is not built (python -m paper_1902_03252_amd.build)")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("lens_create", "lens_destroy", "lens_deflect", "lens_source_positions", "lens_image_chi2",
              "lens_dls_dos", "lens_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lens_[a-z0-9_]+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        getattr(lib, n)


def test_python_binding_covers_the_boundary():
    from paper_1902_03252_amd import _lib as L
    assert set(L.EXPORTS) == set(declared())


def test_strerror(lib):
    lib.lens_strerror.restype = C.c_char_p
    assert lib.lens_strerror(0) == b"ok"
    assert b"invalid" in lib.lens_strerror(1)
    assert b"capacity" in lib.lens_strerror(3)
    assert b"no-allocation" in lib.lens_strerror(4)


def test_host_validation_rejects_before_any_device_call(lib):
    from paper_1902_03252_amd import _lib as L
    L._lib = None
    L.load(LIB)
    lb = L._lib
    ctx = C.c_void_p(1)  # never dereferenced: validation fails first
    pot = L.LensPotentials(-1, None, None, None, None, None, None, None)
    grid = L.LensGrid(0.0, 0.0, 1.0, 16, 16)
    buf = C.c_void_p(8)
    assert lb.lens_deflect(None, C.byref(pot), C.byref(grid), 0, buf, buf, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_deflect(ctx, C.byref(pot), C.byref(grid), 0, buf, buf, None, None) == L.LENS_ERR_INVALID
    pot = L.LensPotentials(1, None, None, None, None, None, None, None)  # null parameter rows
    assert lb.lens_deflect(ctx, C.byref(pot), C.byref(grid), 0, buf, buf, None, None) == L.LENS_ERR_INVALID
    pot = L.LensPotentials(0, None, None, None, None, None, None, None)
    for g in (L.LensGrid(0, 0, 1.0, 1, 16), L.LensGrid(0, 0, 0.0, 16, 16), L.LensGrid(0, 0, float("nan"), 16, 16),
              L.LensGrid(float("inf"), 0, 1.0, 16, 16), L.LensGrid(0, 0, 1.0, 16, 70000)):
        assert lb.lens_deflect(ctx, C.byref(pot), C.byref(g), 0, buf, buf, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_deflect(ctx, C.byref(pot), C.byref(grid), 7, buf, buf, None, None) == L.LENS_ERR_INVALID
    obs = L.LensObs(0, 0, buf, buf, buf, buf, buf)  # no systems
    opts = L.LensChi2Opts(2, 0, 0.0, 16, 0, 0)
    out = L.LensChi2Out(buf, buf, buf, buf, buf, buf, buf)
    assert lb.lens_image_chi2(ctx, C.byref(pot), C.byref(grid), C.byref(obs), C.byref(opts), C.byref(out),
                              None) == L.LENS_ERR_INVALID
    obs = L.LensObs(1, 2, buf, buf, buf, buf, buf)
    for o in (L.LensChi2Opts(1, 0, 0.0, 16, 0, 0),          # FP32 is a field-only precision
              L.LensChi2Opts(2, 0, 0.0, 0, 0, 0),           # no hit capacity
              L.LensChi2Opts(2, 0, 0.0, 1 << 20, 0, 0),     # beyond the sortable hit list
              L.LensChi2Opts(2, 1, -1.0, 16, 0, 0),         # negative literal threshold
              L.LensChi2Opts(2, 5, 0.0, 16, 0, 0),          # unknown fallback mode
              L.LensChi2Opts(2, 0, 0.0, 16, 3, 0),          # nodes per thread not a power of two
              L.LensChi2Opts(2, 0, 0.0, 16, 0, 9)):         # unknown tile shape
        assert lb.lens_image_chi2(ctx, C.byref(pot), C.byref(grid), C.byref(obs), C.byref(o), C.byref(out),
                                  None) == L.LENS_ERR_INVALID
    out_null = L.LensChi2Out(None, buf, buf, buf, buf, buf, buf)
    assert lb.lens_image_chi2(ctx, C.byref(pot), C.byref(grid), C.byref(obs), C.byref(opts), C.byref(out_null),
                              None) == L.LENS_ERR_INVALID
    # the no-allocation entry point checks the same arguments first (no device call)
    for o in (L.LensChi2Opts(1, 0, 0.0, 16, 0, 0), L.LensChi2Opts(2, 0, 0.0, 0, 0, 0)):
        assert lb.lens_image_chi2_noalloc(C.byref(pot), C.byref(grid), C.byref(obs), C.byref(o), C.byref(out),
                                          None) == L.LENS_ERR_INVALID
    assert lb.lens_image_chi2_noalloc(C.byref(pot), C.byref(grid), C.byref(obs), C.byref(opts), C.byref(out_null),
                                      None) == L.LENS_ERR_INVALID
    # batched entry point: sample layout and per-sample limits
    bout = L.LensBatchOut(buf, buf, buf, buf, buf)
    pot2 = L.LensPotentials(4, buf, buf, buf, buf, buf, buf, buf)
    grids = (L.LensGrid * 2)(grid, grid)

    def batched(off, o=opts, n=2, g=grids, ob=obs, out_=bout):
        offs = (C.c_int32 * len(off))(*off)
        return lb.lens_image_chi2_batched(ctx, C.byref(pot2), n, offs, g, C.byref(ob), C.byref(o), C.byref(out_),
                                          None)

    assert batched([0, 1, 3]) == L.LENS_ERR_INVALID          # last offset is not P
    assert batched([1, 2, 4]) == L.LENS_ERR_INVALID          # first offset is not 0
    assert batched([0, 3, 2, 4], n=3) == L.LENS_ERR_INVALID  # decreasing
    assert batched([0, 4], n=0) == L.LENS_ERR_INVALID        # no samples
    assert batched([0, 2, 4], g=(L.LensGrid * 2)(grid, L.LensGrid(0, 0, 1.0, 1, 16))) == L.LENS_ERR_INVALID
    assert batched([0, 2, 4], o=L.LensChi2Opts(2, 0, 0.0, 2048, 0, 0)) == L.LENS_ERR_INVALID  # > 1024 per sample
    assert batched([0, 2, 4], o=L.LensChi2Opts(1, 0, 0.0, 16, 0, 0)) == L.LENS_ERR_INVALID   # FP32
    assert batched([0, 2, 4], o=L.LensChi2Opts(2, 0, 0.0, 16, 8, 0)) == L.LENS_ERR_INVALID   # 8 nodes/thread
    assert batched([0, 2, 4], ob=L.LensObs(1, 2000, buf, buf, buf, buf, buf)) == L.LENS_ERR_INVALID
    assert batched([0, 2, 4], out_=L.LensBatchOut(buf, buf, None, buf, buf)) == L.LENS_ERR_INVALID
    # backward form
    assert lb.lens_deflect_backward(ctx, C.byref(pot2), C.byref(grid), 2, buf, buf, buf, None, None) == \
        L.LENS_ERR_INVALID  # mixed is not a backward precision
    assert lb.lens_deflect_backward(ctx, C.byref(pot2), C.byref(grid), 0, None, buf, buf, None, None) == \
        L.LENS_ERR_INVALID
    assert lb.lens_deflect_backward(ctx, C.byref(pot2), C.byref(grid), 1, buf, buf, None, None, None) == \
        L.LENS_ERR_INVALID
    assert lb.lens_src_chi2(ctx, C.byref(pot2), C.byref(obs), None, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_src_chi2(ctx, C.byref(pot2), C.byref(L.LensObs(0, 0, buf, buf, buf, buf, buf)), buf, None,
                            None) == L.LENS_ERR_INVALID
    assert lb.lens_src_chi2_backward(ctx, C.byref(pot2), C.byref(obs), None, None, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_dls_dos(ctx, 0.3, buf, 1, 0.5, 0.7, buf, None) == L.LENS_ERR_INVALID  # not flat
    # the paper's mixed-precision gradient
    mo = L.LensMixedOpts(1, 400, 20, 0.0092, 0.0104)
    assert lb.lens_deflect_mixed(ctx, C.byref(pot2), C.byref(grid), None, buf, buf, None, buf, None) == \
        L.LENS_ERR_INVALID
    assert lb.lens_deflect_mixed(ctx, C.byref(pot2), C.byref(grid), C.byref(mo), buf, buf, None, None, None) == \
        L.LENS_ERR_INVALID  # no stats
    for bad in (L.LensMixedOpts(5, 400, 20, 0.0092, 0.0104),       # more cluster halos than potentials
                L.LensMixedOpts(-1, 400, 20, 0.0092, 0.0104),
                L.LensMixedOpts(1, -4, 20, 0.0092, 0.0104),
                L.LensMixedOpts(1, 400, 20, float("nan"), 0.0104),
                L.LensMixedOpts(1, 400, 20, 0.0092, -1.0)):
        assert lb.lens_deflect_mixed(ctx, C.byref(pot2), C.byref(grid), C.byref(bad), buf, buf, None, buf,
                                     None) == L.LENS_ERR_INVALID
    # NFW deflection
    nfw = L.LensNfw(2, buf, buf, buf, buf, buf, buf)
    assert lb.lens_deflect_nfw(ctx, None, C.byref(grid), 0, buf, buf, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_deflect_nfw(ctx, C.byref(L.LensNfw(2, buf, buf, buf, buf, None, buf)), C.byref(grid), 0, buf,
                               buf, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_deflect_nfw(ctx, C.byref(L.LensNfw(-1, None, None, None, None, None, None)), C.byref(grid), 0,
                               buf, buf, None, None) == L.LENS_ERR_INVALID
    assert lb.lens_deflect_nfw(ctx, C.byref(nfw), C.byref(grid), 2, buf, buf, None, None) == L.LENS_ERR_INVALID
    # sampler steps
    assert lb.lens_hmc_step(ctx, buf, 0, C.byref(obs), buf, 5, buf, buf, buf, buf, None) == L.LENS_ERR_INVALID
    assert lb.lens_hmc_step(ctx, buf, 3, C.byref(obs), buf, 0, buf, buf, buf, buf, None) == L.LENS_ERR_INVALID
    assert lb.lens_hmc_step(ctx, buf, 3, C.byref(obs), buf, 1001, buf, buf, buf, buf, None) == L.LENS_ERR_INVALID
    assert lb.lens_hmc_step(ctx, buf, 3, C.byref(obs), buf, 5, None, buf, buf, buf, None) == L.LENS_ERR_INVALID
    assert lb.lens_mh_step_batched(ctx, buf, 0, 3, C.byref(grid), C.byref(obs), C.byref(opts), buf, buf, buf, buf,
                                   buf, None) == L.LENS_ERR_INVALID
    assert lb.lens_mh_step_batched(ctx, buf, 2, 3, C.byref(grid), C.byref(obs), C.byref(opts), buf, None, buf, buf,
                                   buf, None) == L.LENS_ERR_INVALID
    assert lb.lens_mh_step_batched(ctx, buf, 2, 3, C.byref(L.LensGrid(0, 0, -1.0, 16, 16)), C.byref(obs),
                                   C.byref(opts), buf, buf, buf, buf, buf, None) == L.LENS_ERR_INVALID
    # autotuning: argument checks that fail before the context is used
    t, npl = C.c_int32(), C.c_int32()
    assert lb.lens_autotune_chi2(ctx, C.byref(pot2), C.byref(grid), C.byref(obs), C.byref(opts), C.byref(out), 0,
                                 None, None, None) == L.LENS_ERR_INVALID  # no repetitions
    assert lb.lens_autotune_lookup(None, 2, 0, 16, 4, C.byref(t), C.byref(npl)) == L.LENS_ERR_INVALID
    assert lb.lens_autotune_lookup(ctx, 2, 2, 16, 4, C.byref(t), C.byref(npl)) == L.LENS_ERR_INVALID
    assert lb.lens_autotune_lookup(ctx, 2, 0, 0, 4, C.byref(t), C.byref(npl)) == L.LENS_ERR_INVALID
    assert lb.lens_autotune_save(ctx, None) == L.LENS_ERR_INVALID
    assert lb.lens_autotune_load(None, b"/nonexistent") == L.LENS_ERR_INVALID
    assert lb.lens_create(None, 0) == L.LENS_ERR_INVALID
