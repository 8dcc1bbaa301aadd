"""Mixed-precision pair arithmetic (GD_FLAG_MIXED): FP64 differences and
scalar factors, FP32 acceleration terms with FP32 tile sums folded into
FP64, FP64 jerk terms. Tolerance: max relative error
2e-6 per particle on acceleration and on jerk against the oracle's
compensated FP64 sums (and the mode must differ from FP64, showing it runs).
Energy drift of an integration stays below 1e-6 per time unit. Pools in
mixed mode give bitwise the results of mixed contexts."""
import numpy as np
import pytest
import torch

import oracle
from paper_1702_00440_amd import gravidy as g
from synth_inputs import plummer, plummer_imf, plummer_with_bh
from tests.gpu_util import DEV, dev, host, rel_err_rows

pytestmark = pytest.mark.gpu

MIX_TOL = 2e-6
MIXED = g.GD_FLAG_MIXED


def _initial(m, x, v, flags, **kw):
    cl = g.Cluster(m, x, v, device=DEV, flags=flags, **kw)
    _, _, a, j, _, _, _ = cl.state()
    out = host(a), host(j)
    cl.close()
    return out


def _sample(n, x, k, seed=0):
    idx = np.random.default_rng(seed).choice(n, min(k, n), replace=False)
    r = np.linalg.norm(x, axis=1)
    return np.unique(np.concatenate([idx, np.argsort(r)[:32]]))


@pytest.mark.parametrize("n,seed", [(257, 2), (1000, 3), (4096, 4), (16384, 1)])
def test_mixed_initial_force_plummer(n, seed):
    m, x, v = plummer(n, seed)
    a, j = _initial(m, x, v, MIXED)
    a64, _ = _initial(m, x, v, 0)
    idx = _sample(n, x, 512)
    ra, rj = oracle.force(m, x, v, 1e-4, idx=idx, compensated=True, threads=oracle.max_threads())
    ea, ej = rel_err_rows(a[idx], ra).max(), rel_err_rows(j[idx], rj).max()
    print(f"n={n}: mixed max rel err acc {ea:.2e} jerk {ej:.2e}")
    assert ea <= MIX_TOL and ej <= MIX_TOL
    assert np.abs(a - a64).max() > 0.0


def _kappa(m, x, v, eps, i):
    """Conditioning of particle i's sums: sum over j of |pair term| over
    |sum|, for the acceleration and for the jerk (Euclidean norms)."""
    r = x - x[i]
    w = v - v[i]
    s = (r * r).sum(1) + eps * eps
    q = 1.0 / np.sqrt(s)
    mq3 = m * q ** 3
    mq3[i] = 0.0
    ta = mq3[:, None] * r
    tj = mq3[:, None] * (w - 3.0 * ((r * w).sum(1) * q * q)[:, None] * r)
    ka = np.linalg.norm(ta, axis=1).sum() / np.linalg.norm(ta.sum(0))
    kj = np.linalg.norm(tj, axis=1).sum() / np.linalg.norm(tj.sum(0))
    return ka, kj


def test_mixed_imf_n262144_against_oracle():
    """The mixed-precision workload: N = 262144, power-law IMF (slope -2.35
    on [0.1, 100], total mass 1), eps 1e-4. 4096 random particles, the 32
    innermost, and the 64 rows where the mixed forces differ most from the
    FP64 path's (acceleration and jerk each) against the oracle's
    compensated sums: at most 2e-6 on every row."""
    n = 262144
    m, x, v = plummer_imf(n, 5)
    a, j = _initial(m, x, v, MIXED)
    a64, j64 = _initial(m, x, v, 0)
    worst = np.concatenate([np.argsort(rel_err_rows(a, a64))[-64:], np.argsort(rel_err_rows(j, j64))[-64:]])
    idx = np.unique(np.concatenate([_sample(n, x, 4096, seed=1), worst]))
    ra, rj = oracle.force(m, x, v, 1e-4, idx=idx, compensated=True, threads=oracle.max_threads())
    ea, ej = rel_err_rows(a[idx], ra), rel_err_rows(j[idx], rj)
    print(f"IMF N=262144, {len(idx)} rows: mixed max rel err acc {ea.max():.2e} jerk {ej.max():.2e}")
    for k in np.argsort(np.maximum(ea, ej))[-3:]:
        ka, kj = _kappa(m, x, v, 1e-4, idx[k])
        print(f"  row {idx[k]}: acc {ea[k]:.2e} (kappa {ka:.1e}), jerk {ej[k]:.2e} (kappa {kj:.1e})")
    assert ea.max() <= MIX_TOL and ej.max() <= MIX_TOL


def test_mixed_unsoftened_and_central_particle():
    m, x, v = plummer(300, 6)
    a, j = _initial(m, x, v, MIXED, eps=0.0)
    ra, rj = oracle.force(m, x, v, 0.0, compensated=True)
    assert rel_err_rows(a, ra).max() <= MIX_TOL and rel_err_rows(j, rj).max() <= MIX_TOL
    n_s = 2048
    m, x, v = plummer_with_bh(n_s, 7, m_bh=0.01)
    a, j = _initial(m, x, v, MIXED, eps_bh=1e-6, bh_index=n_s)
    ra, rj = oracle.force(m, x, v, 1e-4, compensated=True, eps_bh=1e-6, bh=n_s)
    assert rel_err_rows(a, ra).max() <= MIX_TOL and rel_err_rows(j, rj).max() <= MIX_TOL


def test_mixed_run_energy_and_steps():
    """Plummer N = 1024 to t = 1 in mixed mode: energy drift below 1e-6 and
    block-step statistics within 1 % of the FP64 run."""
    m, x, v = plummer(1024, 1)
    sts = []
    for flags in (MIXED, 0):
        cl = g.Cluster(m, x, v, device=DEV, flags=flags)
        sts.append(g.gd_step_to(cl.ctx, 1.0))
        cl.close()
    mix, f64 = sts
    assert abs(mix["e"] - mix["e0"]) / abs(mix["e0"]) < 1e-6
    assert abs(mix["block_steps"] - f64["block_steps"]) <= 0.01 * f64["block_steps"]
    assert abs(mix["particle_steps"] - f64["particle_steps"]) <= 0.01 * f64["particle_steps"]


def test_mixed_pool_equals_mixed_context_bitwise():
    p = g.make_params(flags=MIXED)
    sizes = [(300, 21), (900, 22)]
    arena = torch.empty(g.gd_pool_arena_bytes(4, [n for n, _ in sizes]), dtype=torch.uint8, device=DEV)
    pool = g.gd_pool_create(p, 4, arena)
    slots = {}
    for n, seed in sizes:
        m, x, v = plummer(n, seed)
        slots[g.gd_pool_admit(pool, dev(m), dev(x), dev(v), 0.125)] = (n, seed)
    while g.gd_pool_resident(pool):
        g.gd_pool_run(pool)
    for sl, (n, seed) in slots.items():
        xo = torch.empty(n, 3, dtype=torch.float64, device=DEV)
        vo = torch.empty_like(xo)
        st = g.gd_pool_result(pool, sl, xo, vo)
        m, x, v = plummer(n, seed)
        cl = g.Cluster(m, x, v, device=DEV, flags=MIXED)
        sa = g.gd_step_to(cl.ctx, 0.125)
        np.testing.assert_array_equal(host(xo), host(cl.state()[0]))
        assert st["block_steps"] == sa["block_steps"] and st["e"] == sa["e"]
        cl.close()
    g.gd_pool_destroy(pool)


def test_mixed_against_fp64_all_particles():
    """All N = 16384 particles, mixed against the FP64 path on the same state:
    acceleration and jerk within 2e-6 on every particle."""
    n = 16384
    m, x, v = plummer(n, 1)
    idx = torch.arange(n, dtype=torch.int32, device=DEV)
    out = {}
    for flags in (0, MIXED):
        cl = g.Cluster(m, x, v, device=DEV, flags=flags)
        acc = torch.empty(n, 3, dtype=torch.float64, device=DEV)
        jrk = torch.empty_like(acc)
        g.gd_predict(cl.ctx, 0.0)
        g.gd_force(cl.ctx, idx, acc, jrk)
        out[flags] = host(acc), host(jrk)
        cl.close()
    ea = rel_err_rows(out[MIXED][0], out[0][0])
    ej = rel_err_rows(out[MIXED][1], out[0][1])
    print(f"all particles: acc max {ea.max():.2e}; jerk max {ej.max():.2e}")
    assert ea.max() <= MIX_TOL
    assert ej.max() <= MIX_TOL


def test_mixed_replays_fp64_block_steps_imf():
    """The mixed-precision workload (N = 262144, power-law IMF) replayed along
    an FP64 run: before each of the first 256 block steps the mixed context
    takes the FP64 context's state, so both predict the same j stream and
    select the same active block; the mixed force of that block is then
    compared with the FP64 one, row by row: acceleration and jerk within
    2e-6 on every row."""
    n = 262144
    m, x, v = plummer_imf(n, 5)
    ctx = {0: g.Cluster(m, x, v, device=DEV), MIXED: g.Cluster(m, x, v, device=DEV, flags=MIXED)}
    out = {f: (torch.empty(n, 3, dtype=torch.float64, device=DEV),
               torch.empty(n, 3, dtype=torch.float64, device=DEV),
               torch.empty(n, dtype=torch.int32, device=DEV)) for f in ctx}
    ea, ej, sizes = [], [], []
    for step in range(256):
        xs, vs, a, j, t_i, dt_i, t_now = ctx[0].state()
        g.gd_set_state(ctx[MIXED].ctx, xs, vs, a, j, t_i, dt_i, t_now)
        rows = {}
        for f, cl in ctx.items():
            acc, jrk, idx = out[f]
            g.gd_predict(cl.ctx)
            g.gd_force(cl.ctx, None, acc, jrk)
            k = g.gd_active(cl.ctx, idx)
            order = torch.argsort(idx[:k])
            rows[f] = host(idx[:k][order]), host(acc[:k][order]), host(jrk[:k][order])
        np.testing.assert_array_equal(rows[MIXED][0], rows[0][0])
        ea.append(rel_err_rows(rows[MIXED][1], rows[0][1]))
        ej.append(rel_err_rows(rows[MIXED][2], rows[0][2]))
        sizes.append(len(rows[0][0]))
        g.gd_correct(ctx[0].ctx)
    for cl in ctx.values():
        cl.close()
    ea, ej = np.concatenate(ea), np.concatenate(ej)
    print(f"256 replayed steps, {len(ea)} rows (N_act {min(sizes)}..{max(sizes)}): acc max {ea.max():.2e} "
          f"(p99.9 {np.percentile(ea, 99.9):.2e}); jerk max {ej.max():.2e}")
    assert min(sizes) < max(sizes)
    assert ea.max() <= MIX_TOL
    assert ej.max() <= MIX_TOL
