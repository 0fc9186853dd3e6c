"""The measurement yardsticks (pdhg_time_copy, pdhg_time_gather,
pdhg_time_gather_only) compute what they claim: the copy leaves dst equal
to src (even and odd lengths), the gather leaves out = val * x[idx]
exactly, the gathers alone leave each thread's sum of its four gathered
values (from an index stream or from hashed indices), and bad arguments are
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


def _gather_only_expected(xh, n, idx=None):
    """Thread t of block b sums x at entries b*1024 + t + 256 k, k < 4, that
    are below n; hashed indices are the top lg bits of e * 0x9E3779B97F4A7C15
    modulo 2^64 (Fibonacci hashing)."""
    nblk = -(-n // 1024)
    e = (np.arange(nblk)[:, None, None] * 1024 + np.arange(256)[None, :, None]
         + 256 * np.arange(4)[None, None, :])
    ok = e < n
    if idx is None:
        lg = int(np.log2(xh.size))
        ee = np.minimum(e, n - 1).astype(np.uint64)
        c = ((ee * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(64 - lg)).astype(np.int64)
    else:
        c = idx[np.minimum(e, n - 1)]
    vals = np.where(ok, xh[c], 0.0)
    # the kernel adds k = 0, 1, 2, 3 in order
    s = ((vals[..., 0] + vals[..., 1]) + vals[..., 2]) + vals[..., 3]
    return s.reshape(-1)


@pytest.mark.parametrize("n", [1, 1000, 300_001])
def test_gather_only_yardstick(lib, n):
    rng = np.random.default_rng(4)
    ln = 1 << 16
    xh = rng.standard_normal(ln)
    x = torch.as_tensor(xh, device="cuda")
    idx_h = rng.integers(0, ln, n).astype(np.int32)
    idx = torch.as_tensor(idx_h, device="cuda")
    ms, out = lib.time_gather_only(x, n, idx=idx, reps=2)
    assert ms > 0.0
    assert np.array_equal(out.cpu().numpy(), _gather_only_expected(xh, n, idx_h))
    ms, out = lib.time_gather_only(x, n, reps=2)
    assert ms > 0.0
    assert np.array_equal(out.cpu().numpy(), _gather_only_expected(xh, n))


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
    # hashed indices need a window of a power of two
    y = torch.zeros(6, dtype=torch.float64, device="cuda")
    assert L.pdhg_time_gather_only(None, 8, C.c_void_p(y.data_ptr()), 6, C.c_void_p(x.data_ptr()),
                                   1, None, C.byref(ms)) == lib.E_INVALID
    assert L.pdhg_time_gather_only(None, 0, C.c_void_p(x.data_ptr()), 8, C.c_void_p(x.data_ptr()),
                                   1, None, C.byref(ms)) == lib.E_INVALID
