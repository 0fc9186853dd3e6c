"""The C-ABI library loads on the host and exports every function that
include/pdhg.h declares; host-only entry points answer without a GPU."""
import ctypes as C

from paper_2105_12715_amd import _lib


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = _lib.declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name


def test_host_only_entry_points():
    p = _lib.default_params()
    assert p.eta == 0.0 and p.omega == 1.0 and p.check_period == 30 and p.tau0 == 1
    assert abs(p.beta - 0.36787944117144233) < 1e-16
    assert p.restart_mode == _lib.RESTART_ADAPTIVE
    assert _lib.workspace_bytes(50, 100, 500) > 0
    assert _lib.workspace_bytes(-1, 100, 5) == 0
    assert _lib.workspace_bytes(10, 0, 5) == 0
    assert _lib.workspace_bytes(0, 1, 0) > 0
    assert _lib.workspace_bytes(10, 2**31, 5) == 0
    # A' (16 B/entry), column slabs of A and A' (12 B/entry each plus
    # partial sums), the reordered col_idx, 16 m- and n-vectors, the
    # trust-region buffers: about 1 GB for 1M x 2M with 10M entries
    big = _lib.workspace_bytes(1_000_000, 2_000_000, 10_000_000)
    assert 300e6 < big < 1.5e9
    assert "workspace" in _lib.strerror(_lib.E_WORKSPACE)
    assert _lib.load().pdhg_trust_region_workspace_bytes(-1) == 0


def test_create_rejects_bad_arguments_before_touching_the_device():
    L = _lib.load()
    h = C.c_void_p()
    lp = _lib.LP(10, 0, 0, None, None, None, None, None, None, None, None)
    assert L.pdhg_create(C.byref(lp), None, None, 0, None, C.byref(h)) == _lib.E_INVALID
    lp = _lib.LP(10, 20, 30, None, None, None, None, None, None, None, None)
    assert L.pdhg_create(C.byref(lp), None, None, 0, None, C.byref(h)) == _lib.E_INVALID
    bad = _lib.default_params()
    bad.beta = 1.5
    assert L.pdhg_create(C.byref(lp), C.byref(bad), None, 0, None, C.byref(h)) == _lib.E_INVALID
    assert L.pdhg_create(None, None, None, 0, None, C.byref(h)) == _lib.E_INVALID
    assert not h.value
    # null handles are rejected, not dereferenced
    assert L.pdhg_step(None, 1) == _lib.E_INVALID
    assert L.pdhg_solve(None, 1, 1e-8, None) == _lib.E_INVALID
    L.pdhg_destroy(None)
    assert L.pdhg_linear_trust_region(-1, None, None, 1.0, None, 0, None, None, None) == _lib.E_INVALID
    # checkpoint calls
    assert L.pdhg_state_bytes(None) == 0
    assert L.pdhg_get_state(None, None, 0) == _lib.E_INVALID
    assert L.pdhg_set_state(None, None, 0) == _lib.E_INVALID
