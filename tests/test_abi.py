"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and its host-side validation rejects bad input
before touching the device."""
from __future__ import annotations

import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2604_09221_amd import inputs as I
from paper_2604_09221_amd import patchwork as pw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("patchwork_scheme_batch", "patchwork_scheme_histogram", "patchwork_scheme_enumerate_range",
                     "pw_tri_create", "pw_hist_create", "pw_hist_read"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = pw.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_multi_config_layout_and_default_lane_groups():
    """The ctypes mirror of pw_multi_config and the Python copy of
    PW_MULTI_DEFAULT_LANE_GROUPS agree with the header; the lane-group
    code round-trips."""
    text = open(os.path.join(ROOT, "include", "patchwork.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} pw_multi_config;", text).group(1)
    fields = re.findall(r"(u?int32_t)\s+([a-z_]+);", body)
    assert [f for _, f in fields] == [f for f, _ in pw.MultiConfig._fields_]
    expr = re.search(r"#define PW_MULTI_DEFAULT_LANE_GROUPS (.*)", text).group(1)
    assert eval(expr.replace("u", "")) == pw.DEFAULT_LANE_GROUPS
    g = {8: 2, 9: 4, 11: 4, 12: 2}
    assert pw.lane_groups_of(pw.lane_groups_code(g)) == g
    assert pw.lane_groups_code({7: 1}) == 0


def test_mask_bytes():
    assert [pw.mask_bytes(d) for d in range(1, 13)] == [4] * 6 + [8] * 3 + [16] * 3
    with pytest.raises(pw.PatchworkError):
        pw.mask_bytes(0)
    with pytest.raises(pw.PatchworkError):
        pw.mask_bytes(13)


def _create(d, edges):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int16).reshape(-1, 4))
    h = ctypes.c_void_p()
    rc = pw.lib().pw_tri_create(d, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)), len(e), ctypes.byref(h))
    if rc == pw.PW_OK:
        pw.lib().pw_tri_destroy(h)
    return rc


def test_tri_validation_on_host():
    E = I.standard_triangulation(5).tolist()
    assert _create(0, E) == pw.PW_ERR_ARG
    assert _create(13, E) == pw.PW_ERR_ARG
    assert _create(5, E[:-1]) == pw.PW_ERR_TRI
    bad = list(E)
    bad[0] = (0, 0, 2, 0)
    assert _create(5, bad) == pw.PW_ERR_TRI
    bad = list(E)
    bad[0] = (0, 0, 6, 0)
    assert _create(5, bad) == pw.PW_ERR_TRI
    bad = list(E)
    bad[1] = bad[0]
    assert _create(5, bad) == pw.PW_ERR_TRI
    Es = [tuple(e) for e in E]
    k = Es.index((1, 0, 0, 1))
    Es[k] = (2, 0, 0, 1)
    assert _create(5, Es) == pw.PW_ERR_TRI
    # valid input passes validation (then needs a device)
    for d in (1, 4, 8, 12):
        assert _create(d, I.standard_triangulation(d)) in (pw.PW_OK, pw.PW_ERR_HIP)
    assert _create(6, I.lift_triangulation(6, 5, noise=1.0)) in (pw.PW_OK, pw.PW_ERR_HIP)


def test_null_arguments_rejected():
    L = pw.lib()
    assert L.pw_tri_create(4, None, 0, None) == pw.PW_ERR_ARG
    assert L.patchwork_scheme_batch(None, None, 0, None, None) == pw.PW_ERR_ARG
    assert L.pw_hist_create(100, ctypes.byref(ctypes.c_void_p())) == pw.PW_ERR_ARG   # not a power of two
    assert L.pw_hist_read(None, None, None, None, 0, None) == pw.PW_ERR_ARG
    assert L.pw_last_error()


def test_specialized_source_compiles_for_gfx950():
    """The generated per-triangulation source compiles with hipRTC (no GPU
    needed) and names the literal program of the triangulation."""
    d = 3
    E = I.standard_triangulation(d)
    src = pw.jit_source(d, E)
    assert "struct JitEval" in src and src.count("E::vertex3e(") == 2 * d * d + 2 * d + 1
    assert src.count("E::pair(") == 2 * d
    assert pw.jit_compile(d, E) > 0
    with pytest.raises(pw.PatchworkError):
        pw.jit_compile(10, I.standard_triangulation(10))       # above the specialised range
