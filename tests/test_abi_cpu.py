"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/fvr.h declares, validates grids on the host, and its own
marching-cubes table generator agrees byte for byte with the oracle's
independently written one."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1712_03084_amd as fvr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvr.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(fvr_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(fvr.library_path())
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_check_grid_statuses():
    ok = (-1, -1, -1, 1, 1, 1)
    assert fvr.check_grid((64, 64, 64), ok) == 0
    assert fvr.check_grid((96, 160, 192), ok) == 0
    assert fvr.check_grid((32, 64, 32), ok) == 0
    assert fvr.check_grid((512, 8, 10), ok) == 0
    assert fvr.check_grid((7, 64, 64), ok) == -1        # odd
    assert fvr.check_grid((6, 64, 64), ok) == -1        # below 8
    assert fvr.check_grid((14, 64, 64), ok) == -2       # 7 is not a factor allowed
    assert fvr.check_grid((1024, 64, 64), ok) == -2     # above 512
    assert fvr.check_grid((64, 64, 64), (0, 0, 0, 1, 0, 1)) == -1   # empty extent
    assert fvr.check_grid((64, 64, 64), (0, 0, 0, 1, float("nan"), 1)) == -1


def test_check_frame_point_count_cap_and_pointers():
    """A frame is refused on the host, before any launch, when its point
    count exceeds what 32-bit coordinate indices (3 i) can address."""
    ok = (-1, -1, -1, 1, 1, 1)
    cap = 715827882
    assert cap == (2 ** 31 - 1) // 3
    assert fvr.check_frame(cap, (64, 64, 64), ok) == 0
    assert fvr.check_frame(cap + 1, (64, 64, 64), ok) == -1
    assert fvr.check_frame(2 ** 31, (64, 64, 64), ok) == -1
    assert fvr.check_frame(-1, (64, 64, 64), ok) == -1
    assert fvr.check_frame(0, (64, 64, 64), ok, points_ptr=0, normals_ptr=0) == 0
    assert fvr.check_frame(10, (64, 64, 64), ok, points_ptr=0) == -1
    assert fvr.check_frame(10, (64, 64, 64), ok, normals_ptr=0) == -1
    assert fvr.check_frame(10, (14, 64, 64), ok) == -2


def test_mc_table_identical_to_oracle_generator():
    c_gpu, e_gpu = fvr.mc_table()
    c_orc, e_orc = oracle.mc_table()
    assert np.array_equal(c_gpu, c_orc)
    assert np.array_equal(e_gpu, e_orc)


def test_check_frame_option_bits():
    """Spectrum storages: one at a time, on any supported grid."""
    ok = (-1, -1, -1, 1, 1, 1)
    bf16, fp16, nearest = 2, 4, 1
    for opt in (0, bf16, fp16, nearest, nearest | bf16, nearest | fp16):
        assert fvr.check_frame(10, (64, 64, 64), ok, options=opt) == 0
    assert fvr.check_frame(10, (64, 64, 64), ok, options=bf16 | fp16) == -1
    assert fvr.check_frame(10, (64, 64, 64), ok, options=8) == -1
    for dims in ((48, 64, 64), (64, 96, 64), (64, 64, 512), (16, 256, 128)):
        for opt in (0, bf16, fp16):
            assert fvr.check_frame(10, dims, ok, options=opt) == 0
    for dims in ((56, 64, 64), (64, 64, 1024)):  # unsupported lengths stay unsupported
        for opt in (0, bf16, fp16):
            assert fvr.check_frame(10, dims, ok, options=opt) == -2


def test_status_strings_and_null_context():
    lib = fvr.load_library()
    names = set()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.fvr_status_string(s) and lib.fvr_status_string(s) != b"unknown status"
        names.add(lib.fvr_status_string(s))
    assert len(names) == 7
    assert fvr.STATUS[-6] == "FVR_E_RANGE"
    assert lib.fvr_reconstruct(None, None, None) == -1
    assert lib.fvr_last_error(None)


def test_entry_points_fail_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(fvr, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fvr, "_lib", None)
    with pytest.raises(fvr.FvrUnavailable):
        fvr.load_library()


def test_bench_covers_every_timed_kernel():
    """bench.py prices and fingerprints each launch the library can time."""
    import bench
    lib = fvr.load_library()
    names = {lib.fvr_timing_name(i).decode() for i in range(lib.fvr_timing_count())}
    assert names >= {"splat_fft_x", "fft_yx_inv", "mc_classify"}
    assert names <= set(bench.KERNEL_SOURCES), names - set(bench.KERNEL_SOURCES)
    priced = set(bench.kernel_alg_bytes((256, 256, 256), 700_000, 40_000, 80_000))
    assert priced <= names, priced - names
    assert names - priced <= {"prep", "mc_scan"}, names - priced


def test_tuning_set_get_and_validation():
    """Plan parameters set for a grid shape come back from fvr_get_tuning;
    parameters that do not fit the kernels are refused; clearing restores
    the defaults (host-only calls)."""
    from paper_1712_03084_amd import autotune as at
    d = (96, 160, 192)
    default = at.get_tuning(d)
    assert default["radices"][0] == [8, 4, 3] and default["radices"][1] == [8, 4, 5]
    t = {"radices": [[3, 8, 4], [], [2, 4, 8, 3]], "splat_tile": [2, 2]}
    at.set_tuning(d, t)
    got = at.get_tuning(d)
    assert got["radices"][0] == [3, 8, 4] and got["radices"][1] == [8, 4, 5]
    assert got["radices"][2] == [2, 4, 8, 3] and got["splat_tile"] == [2, 2]
    for bad in ({"radices": [[8, 4, 4], [], []]},            # product is not Nx
                {"radices": [[6, 16], [], []]},               # radix outside {2,3,4,5,8}
                {"radices": [[], [], []], "splat_tile": [1, 3]},    # odd row count
                {"radices": [[], [], []], "splat_tile": [16, 4]},   # 64 rows x 96 > 2048 voxels
                {"radices": [[2] * 5 + [3], [], []]}):        # fine (6 stages): accepted
        if bad.get("radices")[0] == [2] * 5 + [3]:
            at.set_tuning(d, bad)
            continue
        with pytest.raises(fvr.FvrError):
            at.set_tuning(d, bad)
    at.set_tuning(d, None)
    assert at.get_tuning(d) == default
    cand = at.candidates((96, 128, 160))
    assert [8, 4, 3] in cand["radices"][0] and [3, 4, 8] in cand["radices"][0]
    assert cand["radices"][1] == [[8, 8, 2]]          # y = 128 runs a fixed pencil
    assert [4, 4] in cand["splat_tile"]
