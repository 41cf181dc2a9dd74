"""The C interface: every symbol declared in include/sbi.h is exported by
libsbi.so, and the host-only entry points validate their arguments.  Runs
without a GPU (no compute call is made)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(sbi_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2310_19840_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsbi.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_interface():
    names = _declared_functions()
    for n in ("sbi_init", "sbi_vertical_velocity", "sbi_step", "sbi_diagnostics", "sbi_destroy",
              "sbi_workspace_bytes", "sbi_status_string"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2310_19840_amd import _lib
    for n in _declared_functions():
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"


def test_grid_defaults_and_workspace(lib):
    from paper_2310_19840_amd import _lib, make_grid
    g = _lib.sbi_grid()
    lib.sbi_grid_defaults(C.byref(g))
    assert g.order == 7 and abs(g.dealias - 0.5) < 1e-15 and g.max_sweeps == 64 and g.relax == 1
    g = make_grid(1024, 1024, 100.0, 100.0)
    b1 = lib.sbi_workspace_bytes(C.byref(g), 1)
    b2 = lib.sbi_workspace_bytes(C.byref(g), 2)
    assert b1 > 0 and b2 > b1
    g32 = make_grid(1024, 1024, 100.0, 100.0, precision="fp32")
    assert lib.sbi_workspace_bytes(C.byref(g32), 1) < b1


@pytest.mark.parametrize("bad", [dict(nx=100), dict(nx=8), dict(ny=8), dict(ny=3000), dict(order=8),
                                 dict(order=0), dict(dealias=1.0), dict(max_sweeps=0), dict(lx=-1.0)])
def test_invalid_grids_rejected(lib, bad):
    from paper_2310_19840_amd import make_grid
    kw = dict(nx=64, ny=16, lx=10.0, ly=10.0)
    kw.update(bad)
    g = make_grid(**kw)
    assert lib.sbi_workspace_bytes(C.byref(g), 1) == 0
    assert lib.sbi_workspace_bytes(C.byref(make_grid(64, 16, 10.0, 10.0)), 0) == 0


def test_status_strings(lib):
    from paper_2310_19840_amd import _lib
    for code in (0, 1, 2, 3, 4, -1, -2, -3, -4, -5, -6):
        s = _lib.status_string(code)
        assert s.startswith("SBI_")
    assert "unknown" in _lib.status_string(42)


def test_null_arguments_rejected(lib):
    from paper_2310_19840_amd import _lib, make_grid
    g = make_grid(64, 1, 10.0)
    ctx = C.c_void_p()
    # null depth / null out
    assert lib.sbi_init(C.byref(ctx), C.byref(g), 1, None, -1.0, None, 0, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_init(None, C.byref(g), 1, None, -1.0, None, 0, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_destroy(None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_vertical_velocity(None, None, None, None, 1e-8, None, None, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_step(None, None, 0.1, 1, 1e-8, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_step_adaptive(None, None, 1.0, 0.1, 1e-3, 1e-8, 10, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_set_wavemaker(None, None, 0, 0.0, 0.0, 0.0) == _lib.SBI_ERR_INVALID_ARG


def test_adapt_info_layout():
    # the ctypes mirror of sbi_adapt_info: two int32, three doubles, then sbi_step_info
    from paper_2310_19840_amd import _lib
    assert C.sizeof(_lib.sbi_adapt_info) == 8 + 3 * 8 + C.sizeof(_lib.sbi_step_info)
    assert _lib.sbi_adapt_info.solve.offset == 32


def test_product_path_has_no_cpu_fallback():
    # the package must not import the oracle nor offer a CPU path
    pkg = os.path.join(ROOT, "paper_2310_19840_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("the oracle", ""), f


def test_net_interface_host_checks(lib):
    from oracle import warmstart as ws
    from paper_2310_19840_amd import _lib
    assert lib.sbi_net_param_count() == ws.PARAM_COUNT == _lib.SBI_NET_PARAMS
    assert lib.sbi_net_blob_bytes() == C.sizeof(_lib.sbi_net_header) + 4 * ws.PARAM_COUNT
    assert C.sizeof(_lib.sbi_net_header) == 64
    assert lib.sbi_net_trainer_bytes(0, 64, 64) == 0
    assert lib.sbi_net_trainer_bytes(1, 64, 48) == 0      # nx must be a multiple of 64
    assert lib.sbi_net_trainer_bytes(2, 32, 64) > 2 * 32 * 64 * 4 * 9 * 32
    theta = (C.c_float * ws.PARAM_COUNT)()
    tr = C.c_void_p()
    assert lib.sbi_net_trainer_init(None, 1, 64, 64, theta, None, 0, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_net_trainer_init(C.byref(tr), 1, 64, 64, theta, None, 0, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_net_trainer_adam(None, C.c_float(1e-3)) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_net_load(None, None, 0) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_net_features(None, None, None, None, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_net_infer(None, None, None, None, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_last_correction(None, None, None) == _lib.SBI_ERR_INVALID_ARG


def test_batch_interface_host_checks(lib):
    from paper_2310_19840_amd import _lib, make_grid
    g = (_lib.sbi_grid * 3)(make_grid(64, 64, 10.0, 10.0), make_grid(128, 64, 20.0, 10.0),
                            make_grid(64, 64, 10.0, 10.0))
    one = lib.sbi_batch_workspace_bytes(1, g)
    assert lib.sbi_batch_workspace_bytes(3, g) > one > 0
    assert lib.sbi_batch_workspace_bytes(0, g) == 0
    bad = (_lib.sbi_grid * 1)(make_grid(64, 64, 10.0, 10.0))
    bad[0].nx = 100
    assert lib.sbi_batch_workspace_bytes(1, bad) == 0
    b = C.c_void_p()
    assert lib.sbi_batch_init(C.byref(b), 1, g, None, -1.0, None, 0, None, 0) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_batch_step(None, None, 0.1, 1, 1e-8, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_batch_destroy(None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_batch_groups(None, None, None, 0) == 0
    assert lib.sbi_batch_net_load(None, None, 0) == _lib.SBI_ERR_INVALID_ARG


def test_plan_interface_host_checks(lib, tmp_path):
    """The plan cache as a file (host only): entries that parse are merged,
    junk lines are skipped, a save writes back every entry; the plan calls
    reject null contexts."""
    from paper_2310_19840_amd import _lib
    src = tmp_path / "plans_in.txt"
    src.write_text("# sbi launch plans: key row_variant row_rows col_split us\n"
                   "devA/gfx950|1024x1024|b1|fp64|iter|a1|o7|vd1 0 4 0 97.500\n"
                   "this line does not parse\n"
                   "devA/gfx950|512x512|b16|fp32|sa|a0|o7|vd1 2 16 2048 512.250\n"
                   "devA/gfx950|64x64|b1|fp32|sa|a0|o7|vd0 7 1 0 1.0\n")  # variant out of range: skipped
    n = C.c_int32(-1)
    assert lib.sbi_tune_cache_load(str(src).encode(), C.byref(n)) == _lib.SBI_OK
    assert n.value == 2
    out = tmp_path / "plans_out.txt"
    assert lib.sbi_tune_cache_save(str(out).encode(), C.byref(n)) == _lib.SBI_OK
    lines = out.read_text().splitlines()
    assert lines[0].startswith("#") and n.value == len(lines) - 1 >= 2
    body = {ln.split()[0]: ln.split()[1:] for ln in lines[1:]}
    assert body["devA/gfx950|1024x1024|b1|fp64|iter|a1|o7|vd1"] == ["0", "4", "0", "97.500"]
    assert body["devA/gfx950|512x512|b16|fp32|sa|a0|o7|vd1"] == ["2", "16", "2048", "512.250"]
    assert lib.sbi_tune_cache_load(str(tmp_path / "missing.txt").encode(), None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_tune_cache_load(None, None) == _lib.SBI_ERR_INVALID_ARG
    p = _lib.sbi_plan()
    assert lib.sbi_plan_get(None, C.byref(p)) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_plan_set(None, C.byref(p)) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_autotune(None, 0, None) == _lib.SBI_ERR_INVALID_ARG
    assert lib.sbi_plan_variants(None) == 0
    assert lib.sbi_batch_plan(None, 0, C.byref(p)) == _lib.SBI_ERR_INVALID_ARG


def test_full_mode_grids(lib):
    """The fully nonlinear mode takes one-dimensional grids only and sizes its
    FP64 tables and pair slices into the workspace."""
    from paper_2310_19840_amd import _lib, make_grid
    g1 = make_grid(1024, 1, 50.0, mode="full")
    gi = make_grid(1024, 1, 50.0, mode="iter")
    assert lib.sbi_workspace_bytes(C.byref(g1), 1) > lib.sbi_workspace_bytes(C.byref(gi), 1)
    g2 = make_grid(64, 64, 50.0, 50.0, mode="full")
    assert lib.sbi_workspace_bytes(C.byref(g2), 1) == 0
    assert _lib.SBI_MODE_FULL == 2


def test_mixed_precision_grids(lib):
    """SBI_MIXED refines an iteration: its workspace holds the FP64 context and
    the FP32 one of the correction sweeps; SA and fully nonlinear grids refuse it."""
    from paper_2310_19840_amd import _lib, make_grid
    for nx, ny in ((256, 1), (128, 64)):
        gm = make_grid(nx, ny, 50.0, 50.0, precision="mixed")
        g64 = make_grid(nx, ny, 50.0, 50.0, precision="fp64")
        g32 = make_grid(nx, ny, 50.0, 50.0, precision="fp32")
        bm = lib.sbi_workspace_bytes(C.byref(gm), 2)
        assert bm == lib.sbi_workspace_bytes(C.byref(g64), 2) + lib.sbi_workspace_bytes(C.byref(g32), 2)
    for mode in ("sa", "full"):
        g = make_grid(256, 1, 50.0, precision="mixed", mode=mode)
        assert lib.sbi_workspace_bytes(C.byref(g), 1) == 0
    assert _lib.SBI_MIXED == 2
    # the solve info carries the FP32 share after the FP64 fields
    assert _lib.sbi_solve_info.sweeps_fp32.offset == 24
    assert _lib.sbi_step_info.sweeps_fp32_total.offset == 32
