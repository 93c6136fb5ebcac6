"""CPU checks of the C-ABI library: it loads, exports every function that
include/sgpdeconv.h declares, reports the paper's defaults and rejects bad
arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


@pytest.fixture(scope="module")
def lib():
    import paper_1210_2258_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1210_2258_amd.build import build
        build()
    return m.load()


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(INCLUDE, h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M))
    return sorted(n for n in names if n not in ("if", "defined"))


def test_exports_every_declared_function(lib):
    from paper_1210_2258_amd import EXPORTS
    names = _declared_functions()
    assert "sgp_deconv" in names and "sgp_boundary_deconv" in names and "sgp_cnn_infer" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(EXPORTS) | {"sgp_strerror", "sgp_last_error"}


def test_params_defaults_are_the_papers(lib):
    from paper_1210_2258_amd import default_params
    p = default_params()
    # Sect. 3.2 of the paper
    assert p["beta"] == 1e-4 and p["theta"] == 0.4
    assert p["alpha0"] == 1.3 and p["tau1"] == 0.5
    assert p["alpha_max"] == 1e5 and p["alpha_min"] == 1e-5 and p["m_alpha"] == 3
    assert p["n_bb2_only"] == 20 and p["auto_bounds"] == 1
    assert p["disc_target"] == 1.0 and p["max_backtracks"] == 40


def _call(lib, fn, ny, nx, prm=None):
    from paper_1210_2258_amd._lib import _Params, _Report
    p = _Params()
    lib.sgp_params_init(ctypes.byref(p))
    for k, v in (prm or {}).items():
        setattr(p, k, v)
    rep = _Report()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    return getattr(lib, fn)(fake, fake, None, ctypes.c_float(1.0), ny, nx, ctypes.byref(p), fake,
                            ctypes.byref(rep), None)


def test_rejects_unsupported_sizes(lib):
    assert _call(lib, "sgp_deconv", 1031, 256) == -2
    assert _call(lib, "sgp_deconv", 256, 96) == -2          # 96 = 3 * 32 has a factor 3
    assert _call(lib, "rl_deconv", 4096, 4096) == -2
    assert b"FFT" in lib.sgp_last_error()


def test_rejects_bad_parameters(lib):
    assert _call(lib, "sgp_deconv", 64, 64, {"beta": 2.0}) == -1
    assert _call(lib, "sgp_deconv", 64, 64, {"m_alpha": 9}) == -1
    assert _call(lib, "sgp_deconv", 64, 64, {"max_backtracks": 41}) == -1
    assert _call(lib, "sgp_deconv", 64, 64, {"auto_bounds": 0, "L1": 5.0, "L2": 1.0}) == -1
    assert _call(lib, "rl_deconv", 64, 64, {"init": 1}) == -1        # RL from zero is a fixed point
    assert _call(lib, "sgp_deconv", 64, 64, {"init": 3}) == -1       # user start without f0


def test_rejects_bad_background_and_window(lib):
    from paper_1210_2258_amd._lib import _Params, _Report
    p = _Params()
    lib.sgp_params_init(ctypes.byref(p))
    rep = _Report()
    fake = ctypes.c_void_p(0x1000)
    b = (ctypes.c_float * 8)(-1.0)
    assert lib.sgp_multi_deconv(fake, fake, None, ctypes.cast(b, ctypes.c_void_p), 1, 64, 64,
                                ctypes.byref(p), fake, ctypes.byref(rep), None) == -4
    b = (ctypes.c_float * 8)(1.0)
    assert lib.sgp_multi_deconv(fake, fake, None, ctypes.cast(b, ctypes.c_void_p), 9, 64, 64,
                                ctypes.byref(p), fake, ctypes.byref(rep), None) == -1
    # S must fit inside Sbar
    assert lib.sgp_boundary_deconv(fake, fake, None, ctypes.cast(b, ctypes.c_void_p), 1, 64, 64, 80, 64,
                                   20, 8, ctypes.byref(p), fake, ctypes.byref(rep), None) == -1


def test_cnn_parameter_count(lib):
    from oracle import cnn as OC
    assert lib.sgp_cnn_num_params() == OC.n_params() == 13649


def test_strerror(lib):
    assert lib.sgp_strerror(-2) == b"unsupported FFT size"
    assert lib.sgp_strerror(0) == b"success"


def test_device_steplength_rule_matches_hand_table(lib):
    """The steplength rule the GPU runs (same source, compiled for the host)
    against the hand-computed table of Sect. 2.1 decisions."""
    import numpy as np
    from paper_1210_2258_amd import steplength_rule
    path = os.path.join(ROOT, "tests", "golden", "steplength_rules.txt")
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split("|"))
    assert len(rows) >= 8
    for r in rows:
        k, alpha, tau = int(r[0]), float(r[1]), float(r[2])
        Q = [float(v) for v in r[3].split()] if r[3].strip() else []
        a, c1, c2, e = (float(v) for v in r[4].split())
        ea1, ea2, enext, etau, ealt = (float(v) for v in r[5].split())
        out = steplength_rule(k, alpha, tau, Q, a, c1, c2, e)
        assert np.isclose(out["a1"], ea1, rtol=1e-15), r
        assert np.isclose(out["a2"], ea2, rtol=1e-15), r
        assert np.isclose(out["alpha_next"], enext, rtol=1e-15), r
        assert np.isclose(out["tau"], etau, rtol=1e-15), r
        assert out["alt"] == int(ealt), r
        assert len(out["Q"]) <= 3 and out["Q"][-1] == out["a2"]
