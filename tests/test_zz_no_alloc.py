"""gd_force_noalloc (no context, no device allocation: the library's scratch
array) against gd_force with an index list on a context of the same
particles and parameters, through the C ABI, on two calls in a row, the
second with a smaller input."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, dev, host, rel_err_rows
from paper_1702_00440_amd import gravidy as g
from synth_inputs import plummer

pytestmark = pytest.mark.gpu

# (eps, flags, central particle): the FP64 pair, the masked eps = 0 pair, the
# mixed-precision pair, and a central particle with its own softening.
VARIANTS = [(1e-4, 0, False), (0.0, 0, False), (1e-4, g.GD_FLAG_MIXED, False), (1e-4, 0, True)]


def _inputs(n, seed, n_act, central):
    m, x, v = plummer(n, seed)
    if central:
        m = m.copy()
        m[n // 3] = 0.01
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, n_act, replace=False).astype(np.int32)
    idx[-1] = idx[0]  # a repeated index
    return m, x, v, idx


def _via_context(m, x, v, idx, params):
    """gd_force(idx) on a context whose state at t = 0 is (x, v): gd_predict
    to t = 0 leaves the predicted state equal to it."""
    n = len(m)
    ws = torch.empty(g.gd_workspace_bytes(n, params), dtype=torch.uint8, device=DEV)
    ctx = g.gd_init(params, dev(m), dev(x).reshape(n, 3), dev(v).reshape(n, 3), ws)
    g.gd_predict(ctx, 0.0)
    acc = torch.empty(len(idx), 3, dtype=torch.float64, device=DEV)
    jerk = torch.empty_like(acc)
    g.gd_force(ctx, dev(idx, torch.int32), acc, jerk)
    torch.cuda.synchronize()
    g.gd_destroy(ctx)
    return host(acc), host(jerk)


@pytest.mark.parametrize("eps,flags,central", VARIANTS)
def test_noalloc_equals_gd_force_two_calls(eps, flags, central):
    # the second call is smaller (fewer particles and a smaller list)
    for n, seed, n_act in [(20000, 71, 5000), (3001, 72, 300)]:
        m, x, v, idx = _inputs(n, seed, n_act, central)
        bh = n // 3 if central else -1
        params = g.make_params(eps=eps, flags=flags, bh_index=bh, eps_bh=1e-6 if central else None)
        a_ref, j_ref = _via_context(m, x, v, idx, params)
        acc = torch.full((n_act, 3), np.nan, dtype=torch.float64, device=DEV)
        jerk = torch.full_like(acc, np.nan)
        g.gd_force_noalloc(params, dev(m), dev(x).reshape(n, 3), dev(v).reshape(n, 3), dev(idx, torch.int32),
                           acc, jerk)
        torch.cuda.synchronize()
        a, j = host(acc), host(jerk)
        print(f"n={n} n_act={n_act} eps={eps} flags={flags} central={central}", flush=True)
        np.testing.assert_array_equal(a, a_ref)
        np.testing.assert_array_equal(j, j_ref)
        if flags == 0 and n < 5000:
            ra, rj = oracle.force(m, x, v, eps, idx=idx, compensated=True, eps_bh=1e-6 if central else None,
                                  bh=bh)
            assert rel_err_rows(a, ra).max() <= 1e-12
            assert rel_err_rows(j, rj).max() <= 1e-12


def test_noalloc_largest_size_and_limits():
    n = g.GD_NOALLOC_MAX_N
    m, x, v, idx = _inputs(n, 73, 64, False)
    params = g.make_params()
    a_ref, j_ref = _via_context(m, x, v, idx, params)
    acc = torch.empty(64, 3, dtype=torch.float64, device=DEV)
    g.gd_force_noalloc(params, dev(m), dev(x), dev(v), dev(idx, torch.int32), acc, None)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(acc), a_ref)
    m1, x1, v1, idx1 = _inputs(n + 1, 74, 8, False)
    with pytest.raises(g.GdError) as e:
        g.gd_force_noalloc(params, dev(m1), dev(x1), dev(v1), dev(idx1, torch.int32), None, None)
    assert e.value.status == g.GD_EINVAL and "GD_NOALLOC_MAX_N" in str(e.value)


def test_noalloc_out_of_range_index_gives_nan_rows():
    n = 1000
    m, x, v, idx = _inputs(n, 75, 40, False)
    idx[5] = n
    idx[9] = -3
    acc = torch.empty(40, 3, dtype=torch.float64, device=DEV)
    g.gd_force_noalloc(g.make_params(), dev(m), dev(x), dev(v), dev(idx, torch.int32), acc, None)
    torch.cuda.synchronize()
    a = host(acc)
    bad = np.zeros(40, bool)
    bad[[5, 9]] = True
    assert np.isnan(a[bad]).all() and np.isfinite(a[~bad]).all()
