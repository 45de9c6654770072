"""The C-ABI library loads and exports every symbol the header declares;
argument checks that need no device return their status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simradar.h")
LIB = os.path.join(ROOT, "paper_2408_11472_amd", "libsimradar.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*\s*|sim_status\s+|int\s+)(sim_\w+)\s*\(",
                                 text, re.M)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    from paper_2408_11472_amd import simradar
    assert sorted(simradar.EXPORTED) == names


def test_version_and_status_strings():
    from paper_2408_11472_amd import simradar
    import re
    with open(HEADER) as f:
        declared = int(re.search(r"#define SIM_ABI_VERSION (\d+)", f.read()).group(1))
    assert simradar.sim_abi_version() == declared
    assert simradar.sim_status_string(0) == "ok"
    assert "workspace" in simradar.sim_status_string(4)


def test_host_side_argument_checks():
    from paper_2408_11472_amd import simradar as s
    lib = s._lib
    ctx = ctypes.c_void_p()
    assert lib.sim_create(ctypes.byref(ctx), 0, 7) == s.SIM_ERR_ARG
    assert lib.sim_create(None, 0, 0) == s.SIM_ERR_ARG
    g = s.sim_grid(64, 64, 1, 0, 1.0, 1.0, 0.0, 0.0, 9.81)
    r = s.sim_radar(815e3, 7e3, 0, 0, 13.575e9, 18e3, 0.43, 815e3 - 30, 0.0227, 0.62, 0.01,
                    64, 64, 64, 0)
    fac = s.sim_facets(*([None] * 9))
    n = ctypes.c_size_t()
    assert lib.sim_workspace_size(None, ctypes.byref(g), ctypes.byref(r), ctypes.byref(n)) == s.SIM_ERR_ARG
    assert lib.sim_surface_update(None, ctypes.byref(g), None, 0.0, 1e-4, ctypes.byref(fac), None) == s.SIM_ERR_ARG
    assert lib.sim_range_doppler_accumulate(None, ctypes.byref(g), ctypes.byref(fac), ctypes.byref(r),
                                            0.0, 0, None, 1, None, None, None) == s.SIM_ERR_ARG
    assert lib.sim_update_and_accumulate(None, ctypes.byref(g), None, ctypes.byref(r), 0.0, 0, None,
                                         1, None, None, None) == s.SIM_ERR_ARG
    assert lib.sim_segments_to_iq(None, ctypes.byref(r), None, 2, None, None) == s.SIM_ERR_ARG
    assert lib.sim_destroy(None) == s.SIM_OK
    assert lib.sim_set_workspace(None, None, 0) == s.SIM_ERR_ARG
