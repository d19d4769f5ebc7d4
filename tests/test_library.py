"""The C-ABI library builds, loads and exports every function the header declares
(no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "azrbf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(azrbf_[a-z_A-Z]+)\s*\(", src)))


def _lib_path():
    from paper_2308_14490_amd import azrbf
    if not os.path.exists(azrbf.LIB_PATH):
        from paper_2308_14490_amd import build
        build.build(verbose=False)
    return azrbf.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["azrbf_plan", "azrbf_apply_A", "azrbf_apply_Zstar", "azrbf_apply_AZstar", "azrbf_plan_dims", "azrbf_solve", "azrbf_factor",
                 "azrbf_destroy", "azrbf_strerror", "azrbf_footprint_bytes", "azrbf_solve_many",
                 "azrbf_solve_batched"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    # RTLD_NOW: every undefined symbol of the library fails the load here
    lib = ctypes.CDLL(_lib_path(), mode=os.RTLD_NOW | os.RTLD_GLOBAL)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2308_14490_amd import azrbf
    assert set(_declared()) == set(azrbf.EXPORTS)


def test_strerror_and_footprint_without_gpu():
    from paper_2308_14490_amd import azrbf
    lib = azrbf._lib()
    assert lib.azrbf_strerror(0) == b"ok"
    assert b"invalid" in lib.azrbf_strerror(-1)
    pr = azrbf._Problem()
    pr.dim, pr.n, pr.s, pr.T, pr.k = 1, 65536, 2, 1.0, 32
    assert lib.azrbf_footprint_bytes(ctypes.byref(pr), 64) > 8 * 65536 * 64
    pr.n = 0
    assert lib.azrbf_footprint_bytes(ctypes.byref(pr), 64) == -1


def test_plan_rejects_bad_arguments_before_touching_the_gpu():
    import numpy as np
    from paper_2308_14490_amd import azrbf
    lib = azrbf._lib()
    mask = np.ones(64, dtype=np.uint8)
    h = ctypes.c_void_p()
    # any count from 16 on is planned (powers of two, mixed radix, Bluestein); below 16 is not
    for field, val, code in [("n", 8, azrbf.EUNSUPPORTED), ("n", 15, azrbf.EUNSUPPORTED), ("s", 5, azrbf.EUNSUPPORTED),
                             ("dim", 3, azrbf.EINVAL), ("tau", 0.0, azrbf.EINVAL),
                             ("n", 1 << 21, azrbf.EUNSUPPORTED)]:
        pr = azrbf._Problem()
        pr.dim, pr.n, pr.s, pr.T, pr.eps, pr.tau, pr.tauZ = 1, 32, 2, 1.0, 8.0, 1e-12, 1e-12
        pr.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        setattr(pr, field, val)
        assert lib.azrbf_plan(ctypes.byref(pr), None, ctypes.byref(h)) == code
    # n = 2^20 with s = 4: a column pass would need 512 threads for the 4 phases
    big = np.ones(4 << 20, dtype=np.uint8)
    pr = azrbf._Problem()
    pr.dim, pr.n, pr.s, pr.T, pr.eps, pr.tau, pr.tauZ = 1, 1 << 20, 4, 1.0, 8.0, 1e-12, 1e-12
    pr.mask = big.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert lib.azrbf_plan(ctypes.byref(pr), None, ctypes.byref(h)) == azrbf.EUNSUPPORTED


def test_plan_rejects_neumann_points_without_unit_normals():
    """Neumann rows need a unit outward normal at every Neumann point; the
    checks run on the host before any GPU call."""
    import numpy as np
    from paper_2308_14490_amd import azrbf
    lib = azrbf._lib()
    mask = np.ones(64, dtype=np.uint8)
    bp = np.array([-1.0, 1.0])
    h = ctypes.c_void_p()
    for types, normals in [([1, 0], None), ([0, 1], [-1.0, 0.5]), ([2, 0], [-1.0, 1.0]),
                           ([1, 0], [np.nan, 1.0])]:
        pr = azrbf._Problem()
        pr.dim, pr.n, pr.s, pr.T, pr.eps, pr.tau, pr.tauZ = 1, 32, 2, 1.0, 8.0, 1e-12, 1e-12
        pr.op = azrbf.OP_BVP
        pr.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        pr.nb = 2
        pr.bpts = bp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        t = np.array(types, dtype=np.uint8)
        pr.btype = t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        nv = None if normals is None else np.array(normals, dtype=np.float64)
        pr.bnormal = None if nv is None else nv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        assert lib.azrbf_plan(ctypes.byref(pr), None, ctypes.byref(h)) == azrbf.EINVAL


def test_tune_table_round_trip_and_validation():
    """The tile-shape table is host state: loading validates every line."""
    from paper_2308_14490_amd import azrbf
    azrbf.tune_load({"e1_256x256_s2": (8, 4, 16)})
    assert azrbf.tune_table()["e1_256x256_s2"] == (8, 4, 16)
    lib = azrbf._lib()
    assert lib.azrbf_tune_load(b"e1_256x256_s2 3 4 16\n") == azrbf.EINVAL      # C not a power of two
    assert lib.azrbf_tune_load(b"e1_256x256_s2 32 4 16\n") == azrbf.EINVAL     # 32 x 16 threads > 256
    assert lib.azrbf_tune_load(b"e1_1024x64_s2 2 2 16\n") == azrbf.EINVAL      # N1 out of range
    assert lib.azrbf_tune_load(b"e1_4096x512_s2 1 2 16\n") == azrbf.EINVAL     # N1 out of range
    assert lib.azrbf_tune_load(b"e1_2048x512_s2 2 2 8\n") == 0                  # a 2^20 transform
    assert lib.azrbf_tune_load(b"garbage\n") == azrbf.EINVAL
    # TSQR tiles: rows per block 256 RPT with k RPT <= 128 (k = 16 from RPT 2)
    assert lib.azrbf_tune_load(b"t32_65537 512 0 0\nt64_32937 256 0 0\nt16_4097 2048 0 0\n") == azrbf.OK
    assert lib.azrbf_tune_load(b"t32_65537 2048 0 0\n") == azrbf.EINVAL     # 32 x 8 doubles per thread
    assert lib.azrbf_tune_load(b"t16_4097 256 0 0\n") == azrbf.EINVAL       # not instantiated
    assert lib.azrbf_tune_load(b"t48_4097 512 0 0\n") == azrbf.EINVAL       # width
    assert lib.azrbf_tune_load(b"t32_4097 768 0 0\n") == azrbf.EINVAL       # RPT not a power of two
    assert lib.azrbf_tune_load(b"t32_4097x 512 0 0\n") == azrbf.EINVAL      # key
    assert lib.azrbf_tune_load(b"t32_4097 512 1 0\n") == azrbf.EINVAL
    assert lib.azrbf_tune_load(b"e2_128x128_s2 16 16 8\ne2_64x64_s2 4 8 2\n") == 0
    t = azrbf.tune_table()
    assert t["e2_128x128_s2"] == (16, 16, 8) and t["e2_64x64_s2"] == (4, 8, 2)


def test_grouped_and_multi_plan_solves_check_arguments_before_touching_the_gpu():
    """The argument checks that need no device: a negative count or one past
    the grid's entry axis is EINVAL, an empty call is OK, missing arrays are
    EINVAL."""
    from paper_2308_14490_amd import azrbf
    lib = azrbf._lib()
    null = ctypes.c_void_p()
    for f in (lib.azrbf_solve_batched, lib.azrbf_solve_many):
        assert f(-1, None, None, None, None, None, None, None, null) == azrbf.EINVAL
        assert f(0, None, None, None, None, None, None, None, null) == azrbf.OK
        assert f(3, None, None, None, None, None, None, None, null) == azrbf.EINVAL
    assert lib.azrbf_solve_batched(65536, None, None, None, None, None, None, None, null) == azrbf.EINVAL
