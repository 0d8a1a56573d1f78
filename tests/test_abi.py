"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol the header declares, and its pure host helpers behave."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
L = pytest.importorskip("paper_1810_12357_amd.l2t")


def _header_functions():
    src = open(os.path.join(ROOT, "include", "l2t.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(l2t_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_version_strerror_and_exchange_rate():
    assert L.l2t_version() >= 10000
    assert "range" in L.l2t_strerror(L.L2T_ERANGE) or "T_min" in L.l2t_strerror(L.L2T_ERANGE)
    assert L.l2t_strerror(12345) == "unknown status"
    # Eq. 3 with the paper's Ni constants and the 1.1a lattice sum 12 a^2
    a = W.A_LAT * 1e-10
    K = L.l2t_exchange_rate(91.0, 3.6886e5, 3, 12 * a * a)
    assert K * 1e-15 == pytest.approx(W.K_NI, rel=1e-4)
    import math
    assert math.isnan(L.l2t_exchange_rate(-1.0, 1.0, 3, 1.0))


def test_argument_validation_without_device():
    lib = L.load()
    # NULL output handle and bad sizes are rejected before any device call
    assert lib.l2t_create(None, 1, None, 0, None) == L.L2T_EINVAL
    h = ctypes.c_void_p()
    assert lib.l2t_create(ctypes.byref(h), 0, None, 0, None) == L.L2T_EINVAL
    d = (L.l2t_system_desc * 1)()
    d[0].n_atoms = 0
    assert lib.l2t_create(ctypes.byref(h), 1, d, 0, None) == L.L2T_EINVAL
    d[0].n_atoms = 10
    d[0].box_len[0] = d[0].box_len[1] = d[0].box_len[2] = 10.0
    assert lib.l2t_create(ctypes.byref(h), 1, d, 7, None) == L.L2T_EINVAL
    assert lib.l2t_pair_fp32(None, None, None, -1, None) == L.L2T_EINVAL
    assert lib.l2t_pair_fp32(None, None, None, 5, None) == L.L2T_EINVAL
    assert lib.l2t_sync(None) == L.L2T_EINVAL
    assert lib.l2t_coupling(None, 0, L.L2T_XI_INSTANT, 1.0, None, None, None, L.L2T_HOST) == L.L2T_EINVAL
    assert lib.l2t_damping_step(None, 0, 1.0, None, None, None, None, L.L2T_HOST) == L.L2T_EINVAL
    assert lib.l2t_set_counters(None, 0, 0, 0.0, 0.0, 0.0) == L.L2T_EINVAL
    assert lib.l2t_set_allocator(None, ctypes.cast(None, L.ALLOC_FN),
                                 ctypes.cast(None, L.FREE_FN), None) == L.L2T_EINVAL
    assert lib.l2t_last_error(None) == b""


def test_parameter_struct_layout_matches_header():
    assert ctypes.sizeof(L.l2t_params) == 8 * 5 + 4 * 2 + 8 * 10
    assert ctypes.sizeof(L.l2t_system_desc) == 4 + 4 * 3 + 8 * 3 * 2
    assert ctypes.sizeof(L.l2t_energy_report) == 8 * 9


def test_binding_constants_match_the_header():
    """Every #define L2T_* value of the header (status codes, precisions,
    memory kinds, fields, heat-capacity models, options, coupling modes) has
    the same value under the same name in the Python binding."""
    src = open(os.path.join(ROOT, "include", "l2t.h")).read()
    defs = dict(re.findall(r"^#define\s+(L2T_\w+)\s+(-?\d+)\b", src, re.M))
    assert len(defs) >= 30
    for name, value in defs.items():
        assert hasattr(L, name), name
        assert getattr(L, name) == int(value), name
