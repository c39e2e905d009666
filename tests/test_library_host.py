"""Host-side checks of the HIP library (no GPU needed): the C ABI loads and
exports every symbol include/air.h declares, the Joseph index tables match
the oracle's brute-force scan bit for bit, and argument validation rejects
bad calls before any GPU work is queued."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from synth.quality import paper_geometry
from synth.configs import Geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def air():
    from paper_1310_1434_amd import air
    return air


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "air.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(air_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_are_exported(air):
    names = _declared_functions()
    assert len(names) >= 13
    out = subprocess.run(["nm", "-D", "--defined-only", air.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (air_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(air.lib, n)
    assert set(names) == set(air.SIGNATURES)


def test_library_is_gfx950_code(air):
    """The library carries gfx950 device code (no other target)."""
    blob = open(air.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob
    assert b"amdgcn-amd-amdhsa--gfx942" not in blob and b"amdgcn-amd-amdhsa--gfx90a" not in blob


def _geoms():
    return {
        "c1": synth.workload("c1").geom,
        "c2": synth.workload("c2").geom,
        "c2_25": synth.workload("c2_25").geom,
        "ragged_fan": Geometry("fan", n=100, pixel=1.1, n_views=37, n_bins=150, bin=1.3, sod=400.0, sdd=700.0),
        "wide_detector": Geometry("parallel", n=20, pixel=1.0, n_views=11, n_bins=61, bin=1.0),
        # the paper-shaped scan (Materials: 350 x 350 at 1 mm, 528 detector
        # pixels, 800 views or the 25% subset of 200)
        "paper_800": paper_geometry(1),
        "paper_200": paper_geometry(4),
    }


@pytest.mark.parametrize("name", list(_geoms()))
def test_tables_bit_exact_against_oracle_scan(air, orc, name):
    g = _geoms()[name]
    axis, lo, hi = air.host_tables(g)
    oa, olo, ohi = orc.tables(orc.Geom(g))
    np.testing.assert_array_equal(axis, oa)
    np.testing.assert_array_equal(lo, olo)
    np.testing.assert_array_equal(hi, ohi)
    if name == "wide_detector":
        assert (hi < lo).any()     # rays that miss the image are present and empty


def test_tables_bit_exact_large(air, orc):
    g = synth.workload("c5").geom
    axis, lo, hi = air.host_tables(g)
    oa, olo, ohi = orc.tables(orc.Geom(g))
    assert np.array_equal(axis, oa) and np.array_equal(lo, olo) and np.array_equal(hi, ohi)


def _create(air, g, max_batch=1, prec=0, flags=0):
    st, keep = air._geometry_struct(g)
    h = ctypes.c_void_p()
    rc = air.lib.air_plan_create(ctypes.byref(st), max_batch, prec, flags, ctypes.byref(h))
    return rc, h


def test_plan_argument_validation(air):
    base = Geometry("fan", n=64, pixel=1.0, n_views=10, n_bins=90, bin=1.0, sod=300.0, sdd=500.0)
    import dataclasses
    bad = [
        (dataclasses.replace(base, n=0), air.AIR_E_INVALID),
        (dataclasses.replace(base, n_bins=0), air.AIR_E_INVALID),
        (dataclasses.replace(base, pixel=0.0), air.AIR_E_INVALID),
        (dataclasses.replace(base, sod=600.0), air.AIR_E_INVALID),        # sod >= sdd
        (dataclasses.replace(base, sod=40.0, sdd=500.0), air.AIR_E_UNSUPPORTED),   # image reaches the source
        (dataclasses.replace(base, n=20000, sod=1e5, sdd=2e5), air.AIR_E_UNSUPPORTED),
        (dataclasses.replace(base, n_bins=9000), air.AIR_E_UNSUPPORTED),
    ]
    for g, want in bad:
        rc, h = _create(air, g)
        assert rc == want, (g, rc, air.lib.air_last_error())
        assert not h.value
    assert _create(air, base, max_batch=0)[0] == air.AIR_E_INVALID
    assert _create(air, base, prec=7)[0] == air.AIR_E_INVALID
    for bad_flags in (3, 15, 32, 1 << 31, 16 | 3):
        assert _create(air, base, flags=bad_flags)[0] == air.AIR_E_INVALID, bad_flags
    for good in (0, 1, 2, 16, 17, 18):
        rc, h = _create(air, base, flags=good)
        assert rc == air.AIR_OK, (good, air.lib.air_last_error())
        air.lib.air_plan_destroy(h)

    class NonUnit:
        beam, n, pixel, n_views, n_bins, bin, sod, sdd = "parallel", 8, 1.0, 2, 9, 1.0, 0.0, 0.0
        view_cos = np.array([1.0, 0.5])
        view_sin = np.array([0.0, 0.5])

    assert _create(air, NonUnit())[0] == air.AIR_E_INVALID
    assert b"unit" in air.lib.air_last_error()


def test_calls_on_an_unbound_plan_fail_without_touching_the_gpu(air):
    rc, h = _create(air, synth.workload("c1").geom, max_batch=2)
    assert rc == air.AIR_OK
    try:
        dummy = ctypes.c_void_p(0x1000)
        assert air.lib.air_project(h, dummy, dummy, 1, None) == air.AIR_E_INVALID
        assert b"workspace" in air.lib.air_last_error()
        size = ctypes.c_size_t()
        assert air.lib.air_plan_workspace_size(h, ctypes.byref(size)) == air.AIR_OK
        assert size.value > 180 * 185 * 16
        # misaligned or short workspaces are refused before any copy
        assert air.lib.air_plan_bind_workspace(h, ctypes.c_void_p(0x1008), size.value, None) == air.AIR_E_INVALID
        assert air.lib.air_plan_bind_workspace(h, ctypes.c_void_p(0x1000), size.value - 1, None) == air.AIR_E_NOMEM
        assert air.lib.air_plan_bind_workspace(h, None, size.value, None) == air.AIR_E_INVALID
        s1, s3 = ctypes.c_size_t(), ctypes.c_size_t()
        assert air.lib.air_solve_workspace_size(h, 1, ctypes.byref(s1)) == air.AIR_OK
        assert air.lib.air_solve_workspace_size(h, 3, ctypes.byref(s3)) == air.AIR_OK
        assert s1.value < s3.value <= 4 * s1.value      # (3 images hold grouped buffers for 4)
        assert air.lib.air_solve_workspace_size(h, 0, ctypes.byref(s1)) == air.AIR_E_INVALID
    finally:
        air.lib.air_plan_destroy(h)


def test_oracle_and_library_share_no_code():
    """Neither side imports, includes or links the other."""
    pkg = os.path.join(ROOT, "paper_1310_1434_amd")
    bad_pkg = re.compile(r"^\s*(import oracle|from oracle|#include\s+\"oracle)|liboracle", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h", ".cuh")):
                assert not bad_pkg.search(open(os.path.join(dirpath, f)).read()), f
    bad_orc = re.compile(r"^\s*(import paper_1310_1434_amd|from paper_1310_1434_amd|#include\s+\"air)|libair", re.M)
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            assert not bad_orc.search(open(os.path.join(ROOT, "oracle", f)).read()), f
