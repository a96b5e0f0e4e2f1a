"""The C-ABI library loads on the CPU host and exports every symbol that
include/fgcg.h declares; the Python binding declares the same set.  No compute
calls (no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2305_13081_amd import build, fgcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fgcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fgcg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fgcg.LIB_PATH):
        build.build_library()
    return ctypes.CDLL(fgcg.LIB_PATH)


def test_header_declares_entry_points():
    syms = declared_symbols()
    for need in ("fgcg_create", "fgcg_mech_solve", "fgcg_phasefield_solve", "fgcg_diffusion_step",
                 "fgcg_staggered_step", "fgcg_destroy"):
        assert need in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_header():
    assert sorted(fgcg.EXPORTS) == declared_symbols()


def test_binding_loads_and_reports_errors(lib):
    L = fgcg.load_library()
    assert L.fgcg_strerror(-3).decode() == "CG breakdown"
    # NULL arguments are rejected on the host before any device work
    assert L.fgcg_create(None, None, None) == -1
    assert L.fgcg_mech_solve(None, None, None, 0.0, None, None, 1e-8, 10, None, None, None, None, None) == -1
    us = ctypes.c_double()
    assert L.fgcg_time_pass(None, 0, 10, ctypes.byref(us)) == -1


def test_create_rejects_bad_grids_without_gpu(lib):
    L = fgcg.load_library()
    out = ctypes.c_void_p()
    g = fgcg.Grid(2, (ctypes.c_int * 3)(100, 64, 1), 1.0, 0)  # 100 is not 2^a 3^b
    assert L.fgcg_create(ctypes.byref(g), None, ctypes.byref(out)) == -1
    g = fgcg.Grid(2, (ctypes.c_int * 3)(64, 64, 1), -1.0, 0)
    assert L.fgcg_create(ctypes.byref(g), None, ctypes.byref(out)) == -2
    g = fgcg.Grid(3, (ctypes.c_int * 3)(64, 64, 1024), 1.0, 0)  # 3D axes stop at 512
    assert L.fgcg_create(ctypes.byref(g), None, ctypes.byref(out)) == -1
    g = fgcg.Grid(3, (ctypes.c_int * 3)(64, 100, 64), 1.0, 0)
    assert L.fgcg_create(ctypes.byref(g), None, ctypes.byref(out)) == -1
    g = fgcg.Grid(4, (ctypes.c_int * 3)(64, 64, 64), 1.0, 0)
    assert L.fgcg_create(ctypes.byref(g), None, ctypes.byref(out)) == -1


def header_enum(prefix):
    """Name -> value of the enum constants of include/fgcg.h with a prefix."""
    text = open(os.path.join(ROOT, "include", "fgcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return {m.group(1): int(m.group(2)) for m in re.finditer(rf"\b({prefix}[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}


def test_binding_options_match_header():
    """Every context option of the header has a binding name with the same
    value, and no binding name points at a value the header lacks."""
    hdr = header_enum("FGCG_OPT_")
    assert sorted(hdr.values()) == sorted(fgcg.Context.OPTIONS.values())
    by_value = {v: k for k, v in fgcg.Context.OPTIONS.items()}
    for name, v in hdr.items():
        words = name[len("FGCG_OPT_"):].lower()
        assert by_value[v].replace("_", "") .startswith(words.replace("_", "")[:4]), (name, by_value[v])


def test_binding_status_and_precision_constants_match_header():
    for name, v in header_enum("FGCG_E").items():
        assert getattr(fgcg, name) == v, name
    assert fgcg.FGCG_OK == header_enum("FGCG_O")["FGCG_OK"]
    prec = header_enum("FGCG_FP")
    assert (fgcg.FP64, fgcg.FP32_MIXED) == (prec["FGCG_FP64"], prec["FGCG_FP32_MIXED"])
