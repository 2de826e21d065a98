"""CPU checks of the C ABI: the library loads, exports every function that
include/frjf.h declares, and its compiled-in coefficient tables equal the
oracle's (independently typed) tables."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frjf.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    from paper_1904_04825_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares signatures for all of them
    assert set(names) <= set(_lib._SIGS), set(names) - set(_lib._SIGS)


def test_binding_struct_sizes_match_header_layout():
    from paper_1904_04825_amd import _lib
    assert ctypes.sizeof(_lib.DiscDesc) == 5 * 4 + 4 + 4 * 8 + 8 + 3 * 4 + 4 + 4 * 8
    assert ctypes.sizeof(_lib.GmresOptsC) == 2 * 4 + 3 * 8 + 8
    assert ctypes.sizeof(_lib.SolverOptsC) == ctypes.sizeof(_lib.GmresOptsC) + 3 * 8 + 4 * 4 + 4 * 8
    assert ctypes.sizeof(_lib.StepStatsC) == 7 * 4 + 4 + 8 + 8
    assert ctypes.sizeof(_lib.MlpC) == 3 * 4 + 4 + 3 * 8
    assert ctypes.sizeof(_lib.StageLogC) == 2 * 8 + 3 * 4 + 4


@pytest.mark.parametrize("scheme", [2, 3, 4])
def test_row_tables_match_oracle(scheme):
    from paper_1904_04825_amd.api import scheme_table
    from oracle.tableaux import ROW
    A, C, m, g = scheme_table(0, scheme)
    t = ROW[f"ROW{scheme}"]
    assert g == pytest.approx(t.gamma, abs=1e-15)
    assert np.allclose(A, t.A, atol=1e-13) and np.allclose(C, t.C, atol=1e-12) and np.allclose(m, t.m, atol=1e-13)


@pytest.mark.parametrize("scheme", [2, 3, 4])
def test_esdirk_tables_match_oracle(scheme):
    from paper_1904_04825_amd.api import scheme_table
    from oracle.tableaux import ESDIRK
    A, _, b, g = scheme_table(1, scheme)
    t = ESDIRK[f"ESDIRK{scheme}"]
    assert np.allclose(A, t.A, atol=1e-15) and np.allclose(b, t.b, atol=1e-15) and g == t.gamma


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1904_04825_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_ctypes_layouts_match_the_c_compiler(tmp_path):
    """Compile the header with gcc and compare every struct the binding declares."""
    import shutil
    import subprocess
    from paper_1904_04825_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "frjf.h"\nint main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(fr_disc_desc),sizeof(fr_ejacobi),sizeof(fr_gmres_opts),sizeof(fr_gmres_stats),'
                   'sizeof(fr_solver_opts),sizeof(fr_step_stats),sizeof(fr_mlp),sizeof(fr_mlp_trainer),'
                   'sizeof(fr_stage_log),sizeof(fr_pmg),sizeof(fr3d_desc),offsetof(fr_disc_desc,q_far));}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(t) for t in (_lib.DiscDesc, _lib.EjacobiC, _lib.GmresOptsC, _lib.GmresStatsC,
                                       _lib.SolverOptsC, _lib.StepStatsC, _lib.MlpC, _lib.MlpTrainerC,
                                       _lib.StageLogC, _lib.PmgC, _lib.Desc3C)] + [_lib.DiscDesc.q_far.offset]
    assert got == want


def test_invalid_arguments_are_rejected_before_any_device_work():
    """Caller errors come back as FR_EINVAL (-1) with a message, from checks that run
    before the library touches a GPU; outputs are left as they were."""
    from paper_1904_04825_amd import _lib
    L = _lib.lib()
    nodes = ctypes.c_double(0.0)
    good = dict(nx=4, ny=4, p=3, physics=0, flux=0, gamma=1.4, rgas=1.0, mu=0.0, prandtl=0.71,
                d_nodes=ctypes.cast(ctypes.pointer(nodes), ctypes.c_void_p))
    cases = [({"p": 7}, "p must be"), ({"p": 1}, "p must be"), ({"p": 5, "physics": 1}, "Navier-Stokes supports"),
             ({"viscous": 2}, "viscous scheme"), ({"bc_south": 3}, "bad boundary"),
             ({"bc_north": 1}, "need the Navier-Stokes physics"),
             ({"physics": 1, "bc_north": 2}, "far-field state"),
             ({"nx": 1}, "nx and ny"), ({"physics": 7}, "physics"),
             ({"flux": 9}, "flux"), ({"d_nodes": None}, "d_nodes"), ({"gamma": 1.0}, "gamma"),
             ({"nx": 1 << 16, "ny": 1 << 15}, "too large")]
    for change, msg in cases:
        kw = dict(good, **change)
        desc = _lib.DiscDesc(**kw)
        out = ctypes.c_void_p(12345)
        st = L.fr_disc_create(ctypes.byref(desc), ctypes.byref(out))
        assert st == -1, (change, st)
        assert msg in L.fr_last_error().decode(), (change, L.fr_last_error())
        assert out.value == 12345
    assert L.fr_disc_create(None, None) == -1


def test_fr3d_invalid_arguments_and_sizes():
    """The 3D descriptor is checked before any device work; the sizes follow the layout."""
    from paper_1904_04825_amd import _lib
    L = _lib.lib()

    def desc(**kw):
        d = dict(nx=3, ny=4, nz=5, p=3, flux=1, lo=(0.0, 0.0, 0.0), len=(1.0, 2.0, 3.0), gamma=1.4, rgas=1.0,
                 mu=0.01, prandtl=0.71)
        d.update(kw)
        return _lib.Desc3C(d["nx"], d["ny"], d["nz"], d["p"], d["flux"], (ctypes.c_double * 3)(*d["lo"]),
                           (ctypes.c_double * 3)(*d["len"]), d["gamma"], d["rgas"], d["mu"], d["prandtl"])
    for change, msg in (({"p": 5}, "p must be"), ({"nz": 1}, "nx, ny and nz"), ({"flux": 7}, "bad flux"),
                        ({"len": (1.0, 0.0, 1.0)}, "lengths"), ({"mu": -1.0}, "mu >= 0")):
        out = ctypes.c_void_p(7)
        assert L.fr3d_create(ctypes.byref(desc(**change)), ctypes.byref(out)) == -1, change
        assert msg in L.fr_last_error().decode(), (change, L.fr_last_error())
        assert out.value == 7
    h = ctypes.c_void_p()
    assert L.fr3d_create(ctypes.byref(desc()), ctypes.byref(h)) == 0
    try:
        assert L.fr3d_ndof(h) == 5 * 60 * 64
        n2, nel = 16, 60
        assert L.fr3d_workspace_bytes(h) >= 2 * nel * 6 * 5 * n2 * 8 + 2 * 5 * nel * 64 * 8
        # implicit steps: 320-row blocks at P3, two block stores in the step workspace
        nb = 5 * 64
        assert L.fr3d_ejacobi_bytes(h) == nel * nb * nb * 8
        assert L.fr3d_step_workspace_bytes(h, 0) == 0 and L.fr3d_step_workspace_bytes(h, 65) == 0
        w20, w30 = L.fr3d_step_workspace_bytes(h, 20), L.fr3d_step_workspace_bytes(h, 30)
        assert w20 >= 2 * nel * nb * nb * 8 + (41 + 16) * 5 * nel * 64 * 8
        assert w30 - w20 >= 20 * 5 * nel * 64 * 8           # ten more V and ten more Z vectors
        null = ctypes.c_void_p()
        assert L.fr3d_ejacobi_factor(h, null, 1.0, null, null, null) == -1
        assert L.fr3d_ejacobi_apply(h, null, null, null, null) == -1
        assert L.fr3d_gmres_solve(h, null, null, null, 1.0, null, null, None, None, null, null) == -1
        assert "null argument" in L.fr_last_error().decode()
        st = _lib.StepStatsC()
        assert L.fr3d_row_step(h, 3, 0.1, null, None, ctypes.byref(st), null, null) == -1
        assert L.fr3d_bdf2_step(h, 0.1, null, null, null, None, ctypes.byref(st), null, null) == -1
    finally:
        L.fr3d_destroy(h)
