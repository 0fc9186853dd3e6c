"""pdhg_linear_trust_region_static, the trust region for callers that
cannot allocate device memory (its scratch is a static device array of the
library), against pdhg_linear_trust_region with a caller workspace (the
same kernels, so bitwise the same value and multiplier) and against the
oracle's Algorithm 2 (to the trust-region tolerance of the parity tests),
on two calls in a row, the second with a smaller input, so that the
second call runs on what the first left in the array."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12715_amd import _lib
    _lib.load(build_if_missing=False)
    return _lib


def _case(seed, N, inf_frac, atb=0.1, zero_frac=0.1, dup=False):
    rng = np.random.default_rng(seed)
    a = np.abs(rng.standard_normal(N)) * 10 ** rng.uniform(-3, 3, N)
    d = np.abs(rng.standard_normal(N)) * 10 ** rng.uniform(-3, 3, N)
    a[rng.random(N) < zero_frac] = 0.0
    d[rng.random(N) < inf_frac] = np.inf
    d[rng.random(N) < atb] = 0.0
    if dup:
        d = np.round(d, 1)
        a = np.where(a > 0, 1.0, 0.0)
    return a, d


def _radii(a, d):
    fin = d[np.isfinite(d) & (a > 0)]
    full = np.sqrt(np.sum(fin ** 2)) if fin.size else 1.0
    return [0.0, 1e-6 * full, 0.3 * full, 1.5 * full + 1.0]


@pytest.mark.parametrize("first,second", [
    ((1, 200_000, 0.2, False), (2, 5_000, 0.0, False)),
    ((3, 262_144, 0.05, True), (4, 300, 0.5, False)),
])
def test_static_scratch_matches_workspace_entry_point(lib, first, second):
    for seed, N, inf_frac, dup in (first, second):
        a, d = _case(seed, N, inf_frac, dup=dup)
        ta = torch.as_tensor(a, device="cuda:0")
        td = torch.as_tensor(d, device="cuda:0")
        torch.cuda.synchronize()
        for r in _radii(a, d):
            _say("static trust region", seed, N, r)
            before = torch.cuda.memory_allocated()
            v_s, l_s = lib.linear_trust_region_static(ta, td, r)
            assert torch.cuda.memory_allocated() == before
            v_w, l_w = lib.linear_trust_region(ta, td, r)
            assert v_s == v_w and (l_s == l_w or (np.isinf(l_s) and np.isinf(l_w)))
            v_o, l_o = oracle.trust_region(a, d, r)
            assert v_s == pytest.approx(v_o, rel=1e-11, abs=1e-300)
            if np.isfinite(l_o):
                assert l_s == pytest.approx(l_o, rel=1e-9)
            else:
                assert np.isinf(l_s)


def test_static_scratch_limits(lib):
    assert lib.linear_trust_region_static(np.zeros(0), np.zeros(0), 1.0)[0] == 0.0
    n = lib.TR_STATIC_MAX_N + 1
    with pytest.raises(lib.PdhgError) as e:
        lib.linear_trust_region_static(np.ones(n), np.ones(n), 1.0)
    assert e.value.code == lib.E_INVALID
    with pytest.raises(lib.PdhgError):
        lib.linear_trust_region_static([1.0, np.nan], [1.0, 1.0], 1.0)
    # the array still serves a good call after the rejected ones
    v, lam = lib.linear_trust_region_static([3.0, 4.0], [np.inf, np.inf], 2.0)
    assert v == pytest.approx(10.0) and lam == pytest.approx(0.4)
