"""The C-ABI library loads and exports every entry point declared in
include/demrx.h; argument validation happens on the host (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2311_03908_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "demrx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    decl = _declared()
    assert set(decl) == set(capi.EXPORTS), (decl, capi.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libdemrx.so not built")
    L = C.CDLL(capi.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_struct_layouts_match_header_sizes():
    # sizes implied by the C declarations (x86-64 / gfx950 host ABI)
    assert C.sizeof(capi.DemBed) == 4 + 4 + 24 + 24 + 8 + 24 + 8 + 12 + 4 + 48 + 8
    assert C.sizeof(capi.DemOre) == 8 * 3 + 32 + 8 + 8
    assert C.sizeof(capi.DemParcels) == 18 * 8
    assert C.sizeof(capi.DemGas) == 11 * 8
    assert C.sizeof(capi.DemSources) == 15 * 8
    assert C.sizeof(capi.DemStats) == 6 * 8 + 8 + 4 + 4 + 8 + 8 + 8 * 4


def test_host_validation_rejects_null_and_bad_arguments():
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libdemrx.so not built")
    L = capi.load()
    h = C.c_void_p()
    assert L.dem_init(None, None, 10, None, C.byref(h)) == -1
    assert b"null" in L.dem_last_error(None)
    P = capi.DemParams()
    pc = capi.DemParcels()
    assert L.dem_init(C.byref(P), C.byref(pc), 0, None, C.byref(h)) == -1
    P.precision = 7
    assert L.dem_init(C.byref(P), C.byref(pc), 4, None, C.byref(h)) == -1
    # every call on a null context is rejected
    assert L.dem_step(None, 1, None) == -1
    assert L.dem_sync(None) == -1
    assert L.dem_pairs(None, None, 0, None) == -1
    xin = (C.c_double * 2)(0.7, 0.0)
    assert L.dem_gas_species(None, 1e-4, None, None, None, xin, None, None, None) == -1
    assert L.dem_gas_momentum(None, 1e-4, None, None, None, None, None, None, None, None) == -1
    assert L.dem_react(None, 1e-4, None, None, None, None) == -1
    assert L.dem_set_launch(None, 64, 1, 1024) == -1
    assert L.dem_set_build(None, 512, 2048, 16) == -1


def test_bad_grid_rejected_on_host():
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libdemrx.so not built")
    L = capi.load()
    beds = (capi.DemBed * 1)()
    b = beds[0]
    b.wall_kind = 0
    for i in range(3):
        b.lo[i], b.hi[i], b.origin[i], b.n[i] = 0.0, 0.01, 0.0, 2
    b.h = 0.002  # grid (4 mm) does not contain the walls (10 mm)
    b.refine = 1
    ores = (capi.DemOre * 1)()
    ores[0].xi0, ores[0].d_pore_cm, ores[0].tau = 0.3, 1e-6, 2.0
    P = capi.DemParams()
    P.precision, P.n_beds, P.beds, P.n_ores, P.ores = 0, 1, beds, 1, ores
    P.kn, P.e_p, P.mu_s, P.kt_over_kn, P.eps_min, P.dt, P.max_nbr, P.check_every = 1e3, 0.9, 0.3, 0.28, 0.35, 1e-5, 16, 10
    dummy = C.c_double(0)
    pc = capi.DemParcels(*[C.cast(C.byref(dummy), C.c_void_p)] * 17)
    h = C.c_void_p()
    assert L.dem_init(C.byref(P), C.byref(pc), 1, None, C.byref(h)) == -1
    assert b"does not contain" in L.dem_last_error(None)
