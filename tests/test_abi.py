"""Host-side checks that need no GPU: the C-ABI library exists, loads and
exports every function include/swe.h declares; the binding mirrors the
header; the oracle library builds; the scenario generators are seeded."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1705_00614_amd import scenarios as S
from paper_1705_00614_amd import swe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("swe_create", "swe_step", "swe_run", "swe_mass", "swe_destroy"):
        assert required in names
    assert len(names) >= 15


def test_library_loads_and_exports_every_declared_symbol():
    L = swe.load()
    raw = ctypes.CDLL(swe.LIB_PATH)
    for name in header_functions():
        assert hasattr(raw, name), name
    assert sorted(swe.EXPORTS) == header_functions()
    assert isinstance(L.swe_last_error(), bytes)


def _struct_fields(name):
    txt = open(HEADER).read()
    end = txt.index("} %s;" % name)
    body = txt[txt.rindex("typedef struct {", 0, end):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";")[:-1]:
        decl = decl.replace("typedef struct {", "").strip()
        if not decl:
            continue
        for part in decl.split(","):
            fields.append(part.strip().split()[-1].lstrip("*"))
    return fields


def test_params_struct_matches_header_field_order():
    assert _struct_fields("swe_params") == [f[0] for f in swe.SweParams._fields_]


def test_patch_struct_matches_header_field_order():
    assert _struct_fields("swe_patch") == [f[0] for f in swe.SwePatch._fields_]
    txt = open(HEADER).read()
    assert "#define SWE_NEST_FRAME %d" % swe.NEST_FRAME in txt


def test_library_built_for_gfx950():
    data = open(swe.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_oracle_builds_and_loads():
    from oracle import oracle as orc
    orc.build()
    L = orc.lib()
    assert L.orc_hydrograph_volume(1.0, 1.0, 0.0, 0.0, 0.0, 2.0) == 2.0


def test_scenarios_are_seeded_and_shaped():
    a = S.floodplain(n=64, seed=3)
    b = S.floodplain(n=64, seed=3)
    c = S.floodplain(n=64, seed=4)
    assert np.array_equal(a["b"], b["b"]) and not np.array_equal(a["b"], c["b"])
    assert a["b"].shape == (64, 64) and a["H0"].min() >= 0.0
    i0, j0, ni, nj = a["params"]["inlet"]
    assert 0 <= j0 and j0 + nj <= 64 and ni == 40
    assert 0.0 <= S.fbm(32, 32, 0.8, 1, 15.0).min() and S.fbm(32, 32, 0.8, 1, 15.0).max() <= 15.0 + 1e-12
    w = S.floodplain_wet(n=64, seed=3)
    assert 0.5 < (w["H0"] > 1e-4).mean() < 0.7


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(swe, "_lib", None)
    monkeypatch.setattr(swe, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        swe.load()


def test_create_rejects_more_tiles_than_a_list_entry_holds():
    """A tile-list entry keeps the tile index in 20 bits: a 32768 x 32768
    grid of 32 x 32 tiles (2^20 tiles) is refused before the inputs are read
    or any device memory is touched (the one-element bed is never read)."""
    L = swe.load()
    p = swe.make_params(S.dam_break(nx=16, ny=8)["params"])
    b = np.zeros(1)
    h = L.swe_create(32768, 32768, 1.0, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, ctypes.byref(p))
    assert not h
    assert "too many tiles" in swe.last_error()
