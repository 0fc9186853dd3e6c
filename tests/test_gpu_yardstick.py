"""The measurement yardsticks (pdhg_time_copy, pdhg_time_gather) compute
what they claim: the copy leaves dst equal to src (even and odd lengths),
the gather leaves out = val * x[idx] exactly, and bad arguments are
rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12715_amd import _lib
    _lib.load(build_if_missing=False)
    return _lib


@pytest.mark.parametrize("n", [1, 2, 7, 1000, 4_194_305])
def test_copy_yardstick(lib, n):
    src = torch.arange(n, dtype=torch.float64, device="cuda") * 0.5 - 3.0
    dst = torch.full_like(src, np.nan)
    ms = lib.time_copy(src, dst, reps=3)
    assert ms > 0.0
    assert torch.equal(src, dst)


def test_gather_yardstick(lib):
    rng = np.random.default_rng(3)
    n, ln = 300_001, 70_000
    idx = torch.as_tensor(rng.integers(0, ln, n).astype(np.int32), device="cuda")
    val = torch.as_tensor(rng.standard_normal(n), device="cuda")
    x = torch.as_tensor(rng.standard_normal(ln), device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert lib.time_gather(idx, val, x, out, reps=2) > 0.0
    assert torch.equal(out, val * x[idx.long()])


def test_yardsticks_reject_bad_arguments(lib):
    L = lib.load()
    import ctypes as C
    ms = C.c_double()
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    assert L.pdhg_time_copy(None, None, 8, 1, None, C.byref(ms)) == lib.E_INVALID
    assert L.pdhg_time_copy(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr() + 8), 4, 1, None,
                            C.byref(ms)) == lib.E_INVALID
    assert L.pdhg_time_copy(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), 0, 1, None,
                            C.byref(ms)) == lib.E_INVALID
    assert L.pdhg_time_gather(None, None, None, None, 8, 1, None, C.byref(ms)) == lib.E_INVALID
