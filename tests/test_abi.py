"""The C-ABI library loads and exports every entry point that include/spff.h
declares; host-side validation works without a GPU (no compute calls)."""

import ctypes
import os
import re

import pytest

from paper_2203_16467_amd import spff

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spff.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spff_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for required in ("spff_create_problem", "spff_load_step", "spff_get_fields", "spff_create_batch",
                     "spff_load_step_batch", "spff_workspace_bytes", "spff_destroy_problem"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = spff.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows all of them
    assert set(declared_functions()) <= set(spff._SIGS)


def test_version_and_defaults():
    assert "gfx950" in spff.version()
    cfg = spff.default_config()
    assert (cfg.nx, cfg.ny, cfg.at, cfg.split, cfg.irreversibility, cfg.precision) == (64, 64, 1, 1, 0, 0)
    assert cfg.nu == 0.2 and cfg.ell == 2.0 and cfg.crack_set_threshold == 0.9


def test_workspace_bytes_scales_with_batch():
    cfg = spff.default_config(nx=256, ny=256)
    one = spff.workspace_bytes(cfg, 1)
    four = spff.workspace_bytes(cfg, 4)
    n = 256 * 256
    # 18 real planes per problem (state + scratch + spectrum) at minimum
    assert one >= 18 * 4 * n
    assert four - one >= 3 * 18 * 4 * n
    cfg64 = spff.default_config(nx=256, ny=256, precision=spff.FP64)
    assert spff.workspace_bytes(cfg64, 1) > 1.9 * one


@pytest.mark.parametrize("field,value", [("nx", 100), ("ny", 4), ("nx", 4096), ("nu", 0.5), ("nu", -1.0),
                                         ("ell", 0.0), ("gc", -1.0), ("at", 3), ("split", 3), ("split", -1),
                                         ("contact", 3), ("contact", -2),
                                         ("irreversibility", 5), ("precision", 2), ("max_cg", 0),
                                         ("ticks_per_sync", 0), ("tol_pf", -1.0), ("k_res", -0.1)])
def test_invalid_config_rejected(field, value):
    cfg = spff.default_config()
    setattr(cfg, field, value)
    out = ctypes.c_size_t(0)
    st = spff.lib().spff_workspace_bytes(ctypes.byref(cfg), 1, ctypes.byref(out))
    assert st == spff.E_INVALID
    assert spff.last_error()


@pytest.mark.parametrize("field,value", [("evolution", 3), ("evolution", -1), ("eta", -1.0), ("dt_min", 0.0),
                                         ("dt_max", 1e-4), ("dphi_max", 0.0), ("dphi_min", -1.0)])
def test_invalid_time_discretized_config_rejected(field, value):
    """Algorithm 3's parameters are checked only when it is selected."""
    cfg = spff.default_config(evolution=spff.EVOL_TIME, eta=1.0)
    assert spff.workspace_bytes(cfg, 1) > 0
    setattr(cfg, field, value)
    out = ctypes.c_size_t(0)
    assert spff.lib().spff_workspace_bytes(ctypes.byref(cfg), 1, ctypes.byref(out)) == spff.E_INVALID
    if field not in ("evolution",):
        cfg.evolution = spff.EVOL_AM
        assert spff.workspace_bytes(cfg, 1) > 0


@pytest.mark.parametrize("field,value", [("fphi_max", 0.0), ("fphi_max", float("inf")), ("drive_threshold", -1.0),
                                         ("deps_max", -1e-3), ("dt_max", 0.0), ("eta", -1.0), ("dphi_min", -1.0)])
def test_invalid_near_equilibrium_config_rejected(field, value):
    """Algorithm 4's parameters are checked only when it is selected."""
    cfg = spff.default_config(evolution=spff.EVOL_NEAR_EQ)
    assert spff.workspace_bytes(cfg, 1) > 0
    setattr(cfg, field, value)
    out = ctypes.c_size_t(0)
    assert spff.lib().spff_workspace_bytes(ctypes.byref(cfg), 1, ctypes.byref(out)) == spff.E_INVALID
    if field not in ("dt_max", "eta", "dphi_min"):
        cfg.evolution = spff.EVOL_AM
        assert spff.workspace_bytes(cfg, 1) > 0


def test_time_discretized_defaults():
    cfg = spff.default_config()
    assert cfg.evolution == spff.EVOL_AM and cfg.eta == 0.0
    assert 0.0 < cfg.dt_min <= cfg.dt_max and cfg.dphi_max > 0.0 and cfg.dphi_min >= 0.0


@pytest.mark.parametrize("split,contact", [(0, -1), (1, -1), (2, -1), (1, 0), (1, 2), (0, 1), (2, 2)])
def test_model_matrix_accepted(split, contact):
    """Every driving-force / contact pairing of the three energy models is a
    valid configuration (variational when equal or SPFF_CONTACT_SAME)."""
    cfg = spff.default_config(split=split, contact=contact)
    assert spff.workspace_bytes(cfg, 1) > 0


def test_create_rejects_null_arguments_without_device():
    cfg = spff.default_config()
    h = ctypes.c_void_p()
    L = spff.lib()
    assert L.spff_create_batch(ctypes.byref(cfg), 1, None, None, None, 0, None, ctypes.byref(h)) == spff.E_INVALID
    assert L.spff_create_batch(ctypes.byref(cfg), 0, ctypes.c_void_p(256), None, ctypes.c_void_p(256), 0, None,
                               ctypes.byref(h)) == spff.E_INVALID
    # misaligned workspace
    assert L.spff_create_batch(ctypes.byref(cfg), 1, ctypes.c_void_p(256), None, ctypes.c_void_p(257), 1 << 30,
                               None, ctypes.byref(h)) == spff.E_INVALID
    # too small workspace
    assert L.spff_create_batch(ctypes.byref(cfg), 1, ctypes.c_void_p(256), None, ctypes.c_void_p(512), 16, None,
                               ctypes.byref(h)) == spff.E_NOMEM
    assert L.spff_load_step(None, None, None) == spff.E_INVALID
    assert L.spff_get_fields(None, 0, 1, None) == spff.E_INVALID
    assert L.spff_destroy_problem(None) == spff.OK


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of spff_config, spff_step_stats, spff_profile and
    spff_plan have the header's size and field offsets (compiled with the
    host C compiler against include/spff.h)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"spff_config": spff.Config, "spff_step_stats": spff.StepStats, "spff_profile": spff.Profile,
               "spff_plan": spff.Plan}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "spff.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        parts = line.split()
        if len(parts) == 3:
            got[(parts[0], parts[1])] = int(parts[2])
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_static_step_rejects_before_any_device_work():
    """spff_load_step_static checks its configuration and the size of the
    scratch the grid needs against the static array before it touches a
    device (dummy pointers are never dereferenced)."""
    L = spff.lib()
    eb = (ctypes.c_double * 3)(0.0, 0.01, 0.0)
    dummy = ctypes.c_void_p(256)
    for kw in (dict(nx=2048, ny=2048), dict(nx=1024, ny=1024, precision=spff.FP64),
               dict(nx=64, ny=64, evolution=spff.EVOL_TIME), dict(nx=100, ny=64)):
        cfg = spff.default_config(**kw)
        st = L.spff_load_step_static(ctypes.byref(cfg), dummy, dummy, eb, None, None)
        assert st == spff.E_INVALID, kw
    cfg = spff.default_config(nx=2048, ny=2048)
    L.spff_load_step_static(ctypes.byref(cfg), dummy, dummy, eb, None, None)
    assert "static scratch" in spff.last_error()
    cfg = spff.default_config(nx=64, ny=64)
    assert L.spff_load_step_static(ctypes.byref(cfg), None, dummy, eb, None, None) == spff.E_INVALID
    bad = (ctypes.c_double * 3)(0.0, float("nan"), 0.0)
    assert L.spff_load_step_static(ctypes.byref(cfg), dummy, dummy, bad, None, None) == spff.E_INVALID


@pytest.mark.parametrize("ny", [128, 512, 1024, 2048])
def test_autotuner_column_candidates_cover_both_point_counts(ny):
    """Register column candidates: 8 points per lane (ny/8 lanes per column)
    at every size, and for 1024 and 2048 points also the 16-point form; a
    group never exceeds 256 lanes and holds a whole number of columns."""
    from paper_2203_16467_amd import autotune
    cfg = spff.default_config(nx=256, ny=ny)
    reg = [(W, T) for kind, W, T in autotune.col_candidates(cfg) if kind == spff.FFT_REG]
    assert (max(1, 64 // (ny // 8)), max(1, 64 // (ny // 8)) * (ny // 8)) in reg
    if ny >= 1024:
        assert (1, ny // 16) in reg and (1, ny // 8) in reg
    for W, T in reg:
        assert 64 <= T <= 256 and T % W == 0 and (T // W) in (ny // 8, ny // 16)
    cfg64 = spff.default_config(nx=256, ny=ny, precision=spff.FP64)
    assert not [c for c in autotune.col_candidates(cfg64) if c[0] == spff.FFT_REG]
