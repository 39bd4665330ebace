"""The C-ABI library loads and exports every function include/abea.h declares
(no compute call: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_2101_05012_amd import abea

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "abea.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(abea_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("abea_create", "abea_align_batch", "abea_destroy", "abea_align_batch_device"):
        assert n in names
    assert set(names) == set(abea.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(abea.LIB_PATH):
        pytest.fail("libabea.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(abea.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_strerror_without_gpu():
    lib = abea.lib()
    assert lib.abea_strerror(0) == b"ok"
    assert lib.abea_strerror(-4) == b"pair capacity too small"
    assert lib.abea_last_error(None) == b""


def test_create_rejects_bad_config_without_touching_the_gpu():
    lib = abea.lib()
    import numpy as np

    lm = np.full(16, 80, np.float32)
    ls = np.full(16, 2, np.float32)
    mdl = abea.abea_model_t(2, lm.ctypes.data, ls.ctypes.data)
    h = ctypes.c_void_p()
    for W in (1, 0, 513):
        cfg = abea.abea_config_t(W, 0, 0, 0)
        assert lib.abea_create(ctypes.byref(cfg), ctypes.byref(mdl), ctypes.byref(h)) == abea.ABEA_E_INVAL
    cfg = abea.abea_config_t(100, 0, 0, 0)
    bad = abea.abea_model_t(13, lm.ctypes.data, ls.ctypes.data)
    assert lib.abea_create(ctypes.byref(cfg), ctypes.byref(bad), ctypes.byref(h)) == abea.ABEA_E_INVAL
    ls0 = ls.copy()
    ls0[3] = 0
    bad2 = abea.abea_model_t(2, lm.ctypes.data, ls0.ctypes.data)
    assert lib.abea_create(ctypes.byref(cfg), ctypes.byref(bad2), ctypes.byref(h)) == abea.ABEA_E_INVAL
    for flags in (8, 16, 1 << 31):  # bits no ABEA_F_* defines
        cfg_f = abea.abea_config_t(100, 0, 0, flags)
        assert lib.abea_create(ctypes.byref(cfg_f), ctypes.byref(mdl), ctypes.byref(h)) == abea.ABEA_E_INVAL


def test_cells_per_lane_rule_for_every_band_width():
    """Host planning without a device: the band fill's slots per lane is the
    smallest power of two whose 64*c slots hold the band plus the slot-refill
    interval (32/c bands per trace group, refilled once or twice per group,
    at least every 2 bands), and 0 outside 2 <= W <= ABEA_MAX_BANDWIDTH."""
    lib = abea.lib()

    def fits(W, c):
        return any((32 // c) // rpg >= 2 and 64 * c - W >= (32 // c) // rpg for rpg in (1, 2))

    for W in range(2, 513):
        c = lib.abea_cells_per_lane(W)
        assert c in (1, 2, 4, 8, 16), (W, c)
        assert fits(W, c), (W, c)
        assert c == 1 or not fits(W, c // 2), (W, c)
    assert [lib.abea_cells_per_lane(W) for W in (100, 200, 250, 512)] == [2, 4, 4, 16]
    for W in (-1, 0, 1, 513, 1 << 20):
        assert lib.abea_cells_per_lane(W) == 0


def test_binding_constants_and_structs_match_the_header():
    """Every integer #define of the header has the binding's value, and the
    binding's launch and plan-info structures have the header's fields in
    order."""
    src = open(os.path.join(ROOT, "include", "abea.h")).read()
    defs = dict(re.findall(r"#define\s+(ABEA_[A-Z0-9_]+)\s+\(?(-?\d+)u?\)?\s", src))
    checked = 0
    for name, val in defs.items():
        if hasattr(abea, name):
            assert int(getattr(abea, name)) == int(val), name
            checked += 1
    for name in ("ABEA_CLEAR_AUTO", "ABEA_CLEAR_WINDOW", "ABEA_CLEAR_EDGES", "ABEA_WORKERS_SPLIT"):
        assert name in defs and hasattr(abea, name), name
    assert checked >= 8
    body = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for cname, cls in (("abea_launch_t", abea.abea_launch_t), ("abea_plan_info_t", abea.abea_plan_info_t),
                       ("abea_detect_params_t", abea.abea_detect_params_t),
                       ("abea_raw_batch_t", abea.abea_raw_batch_t)):
        m = re.search(r"typedef struct \{([^}]*)\}\s*" + cname + ";", body)
        assert m, cname
        fields = re.findall(r"\b([a-z_]+);", m.group(1))
        assert fields == [f for f, _ in cls._fields_], cname


def test_detect_defaults_agree():
    """The header's default detector, the binding's and the oracle's default
    parameters are the same four numbers."""
    src = open(os.path.join(ROOT, "include", "abea.h")).read()
    m = re.search(r"#define ABEA_DETECT_DEFAULT_PARAMS \{([^}]*)\}", src)
    vals = [float(v.strip().rstrip("f")) for v in m.group(1).split(",")]
    assert vals == [float(v) for v in abea.DETECT_DEFAULT]
    from oracle import oracle as orc

    p = orc.ed_params()
    assert vals == [p.w_short, p.w_long, p.t_short, p.t_long]
