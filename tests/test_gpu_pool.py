"""Pools (continuous batching of independent clusters): every cluster's
result is bitwise the same alone (a plain context) and packed with others,
admission follows the arena footprint, and the request loop completes
staggered arrivals. Clusters are equal-mass Plummer spheres of different N
(eps 1e-4, eta 0.01, dt_max 1/8)."""
import numpy as np
import pytest
import torch

from paper_1702_00440_amd import gravidy as g
from paper_1702_00440_amd import serving
from synth_inputs import plummer
from tests.gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu

PARAMS = dict(eta=0.01, eps=1e-4, dt_max=0.125, dt_min=2.0 ** -22)


def _ics(n, seed):
    m, x, v = plummer(n, seed)
    return dev(m), dev(x), dev(v)


def _alone(n, seed, t_end):
    m, x, v = _ics(n, seed)
    p = g.make_params(**PARAMS)
    ws = torch.empty(g.gd_workspace_bytes(n, p), dtype=torch.uint8, device=DEV)
    ctx = g.gd_init(p, m, x, v, ws)
    st = g.gd_step_to(ctx, t_end)
    xo, vo = torch.empty_like(x), torch.empty_like(v)
    g.gd_get_state(ctx, xo, vo)
    g.gd_destroy(ctx)
    return host(xo), host(vo), st


def _drain(pool):
    done = []
    for _ in range(100000):
        if g.gd_pool_resident(pool) == 0:
            break
        done += g.gd_pool_run(pool)
    return done


def test_pool_results_equal_alone_bitwise():
    sizes = [(256, 11), (700, 12), (1024, 13), (2048, 14), (333, 15)]
    t_end = 0.25
    p = g.make_params(**PARAMS)
    arena = torch.empty(g.gd_pool_arena_bytes(8, [n for n, _ in sizes]), dtype=torch.uint8, device=DEV)
    pool = g.gd_pool_create(p, 8, arena)
    slots = {}
    for n, seed in sizes:
        m, x, v = _ics(n, seed)
        slots[g.gd_pool_admit(pool, m, x, v, t_end)] = (n, seed)
    assert g.gd_pool_resident(pool) == len(sizes)
    finished = _drain(pool)
    assert sorted(finished) == sorted(slots)
    for sl, (n, seed) in slots.items():
        xo = torch.empty(n, 3, dtype=torch.float64, device=DEV)
        vo = torch.empty_like(xo)
        st = g.gd_pool_result(pool, sl, xo, vo)
        xa, va, sa = _alone(n, seed, t_end)
        np.testing.assert_array_equal(host(xo), xa)
        np.testing.assert_array_equal(host(vo), va)
        assert st["block_steps"] == sa["block_steps"] and st["particle_steps"] == sa["particle_steps"]
        assert st["t"] == t_end
        assert st["e"] == sa["e"] and st["e0"] == sa["e0"]
        g.gd_pool_release(pool, sl)
    g.gd_pool_destroy(pool)


def test_admission_by_footprint_and_slot_reuse():
    """An arena with room for two workspaces: the third cluster waits until a
    release frees room, then runs to the same result as alone."""
    p = g.make_params(**PARAMS)
    n = 512
    arena = torch.empty(g.gd_pool_arena_bytes(4, [n, n]), dtype=torch.uint8, device=DEV)
    pool = g.gd_pool_create(p, 4, arena)
    a = g.gd_pool_admit(pool, *_ics(n, 21), 0.125)
    b = g.gd_pool_admit(pool, *_ics(n, 22), 0.125)
    assert a is not None and b is not None
    assert g.gd_pool_admit(pool, *_ics(n, 23), 0.125) is None
    first = []
    while not first:
        first = g.gd_pool_run(pool)
    g.gd_pool_release(pool, first[0])
    c = g.gd_pool_admit(pool, *_ics(n, 23), 0.125)
    assert c is not None
    _drain(pool)
    xo = torch.empty(n, 3, dtype=torch.float64, device=DEV)
    g.gd_pool_result(pool, c, xo)
    np.testing.assert_array_equal(host(xo), _alone(n, 23, 0.125)[0])
    g.gd_pool_destroy(pool)


def test_serving_loop_staggered_arrivals():
    rng = np.random.default_rng(3)
    reqs = []
    for k in range(12):
        n = int(round(np.exp(rng.uniform(np.log(256), np.log(1024)))))
        m, x, v = _ics(n, 100 + k)
        reqs.append(serving.Request(k, 0.002 * k, m, x, v, 0.125))
    p = g.make_params(**PARAMS)
    srv = serving.PoolServer(p, 6, g.gd_pool_arena_bytes(6, [1024] * 6), keep_state=True)
    res = srv.serve(reqs)
    srv.close()
    assert sorted(r.rid for r in res) == list(range(12))
    seq = {r.rid: r for r in serving.serve_sequential(p, reqs, keep_state=True)}
    for r in res:
        assert r.done >= r.admitted >= r.arrival - 1e-6
        np.testing.assert_array_equal(host(r.x), host(seq[r.rid].x))
        assert r.stats["block_steps"] == seq[r.rid].stats["block_steps"]
