"""Central massive particle (the paper's planned extension, Sec. 6): pairs
that involve it are softened with eps_bh, all others with eps. Parity of the
HIP path with the oracle on a Plummer sphere of 2048 stars plus a particle of
mass 0.01 at rest at the origin (eps 1e-4, eps_bh 1e-6, dt_min 2^-22)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1702_00440_amd import gravidy as g
from synth_inputs import plummer_with_bh
from tests.gpu_util import DEV, host, rel_err_rows

pytestmark = pytest.mark.gpu

EPS, EPS_BH, ETA, DTMAX, DTMIN = 1e-4, 1e-6, 0.01, 0.125, 2.0 ** -22
NS = 2048


@pytest.fixture(scope="module")
def system():
    return plummer_with_bh(NS, 5)


def _cluster(m, x, v):
    return g.Cluster(m, x, v, eta=ETA, eps=EPS, dt_max=DTMAX, dt_min=DTMIN, device=DEV, eps_bh=EPS_BH,
                     bh_index=NS)


def _oracle_state(cl, m):
    xs, vs, a, j, t_i, dt_i, t_now = cl.state()
    return oracle.State.from_arrays(m, host(xs), host(vs), host(a), host(j), host(t_i), host(dt_i), t_now,
                                    EPS, ETA, DTMAX, DTMIN, threads=oracle.max_threads(), eps_bh=EPS_BH, bh=NS)


def test_initial_force_and_energy(system):
    m, x, v = system
    cl = _cluster(m, x, v)
    _, _, a, j, _, _, _ = cl.state()
    ra, rj = oracle.force(m, x, v, EPS, compensated=True, threads=oracle.max_threads(), eps_bh=EPS_BH, bh=NS)
    assert rel_err_rows(host(a), ra).max() <= 1e-12
    assert rel_err_rows(host(j), rj).max() <= 1e-12
    ek, ep = g.gd_energy(cl.ctx)
    rk, rp = oracle.energy(m, x, v, EPS, eps_bh=EPS_BH, bh=NS)
    assert ek == pytest.approx(rk, rel=1e-13) and ep == pytest.approx(rp, rel=1e-13)
    cl.close()


def test_block_steps_from_identical_state(system):
    m, x, v = system
    cl = _cluster(m, x, v)
    saw_bh = False
    for _ in range(60):
        ref = _oracle_state(cl, m)
        act = ref.block_step()
        saw_bh |= NS in act
        g.gd_predict(cl.ctx)
        idx = torch.empty(len(m), dtype=torch.int32, device=DEV)
        n_act = g.gd_active(cl.ctx, idx)
        np.testing.assert_array_equal(np.sort(host(idx[:n_act])), act)
        g.gd_force(cl.ctx)
        g.gd_correct(cl.ctx)
        xs, vs, a, j, t_i, dt_i, t_now = cl.state()
        assert t_now == ref.t_now
        np.testing.assert_array_equal(host(dt_i), ref.dt_i)
        assert rel_err_rows(host(xs), ref.x).max() <= 1e-13
        assert rel_err_rows(host(a)[act], ref.a[act]).max() <= 1e-12
        assert rel_err_rows(host(j)[act], ref.jk[act]).max() <= 1e-12
    assert saw_bh
    cl.close()


def test_run_against_oracle(system):
    m, x, v = system
    cl = _cluster(m, x, v)
    st = g.gd_step_to(cl.ctx, 0.125)
    ref = oracle.State(m, x, v, EPS, ETA, DTMAX, DTMIN, threads=oracle.max_threads(), eps_bh=EPS_BH, bh=NS)
    rows = ref.run(0.125)
    assert st["block_steps"] == ref.stats[0]
    assert st["particle_steps"] == ref.stats[1]
    assert st["dtmin_clamps"] == ref.stats[3]
    assert st["e"] == pytest.approx(rows[-1, 3], rel=1e-10)
    assert np.abs(host(cl.state()[0]) - ref.x).max() < 1e-9
    cl.close()


@pytest.mark.parametrize("flags,tol", [(g.GD_FLAG_MIXED, 2e-6), (0, 1e-12)])
def test_full_size_sampled(flags, tol):
    """The full central-particle workload: 2^20 stars plus the central particle
    (seed 5, dt_min 2^-22), in mixed precision (its configuration) and FP64.
    Initial forces of 1024 random stars, the central particle and its 64
    nearest stars against the oracle's compensated sums (mixed: 2e-6, FP64:
    1e-12 per particle); then 3 block steps from the GPU's state with the
    active set and times identical to the oracle's step, and the new block
    steps too (FP64; in mixed precision a particle whose Aarseth step lies
    within the mixed error of a power of two may take the neighbouring level:
    at most one such tie per step, a factor of exactly 2)."""
    ns = 1 << 20
    m, x, v = plummer_with_bh(ns, 5)
    cl = g.Cluster(m, x, v, eta=ETA, eps=EPS, dt_max=DTMAX, dt_min=DTMIN, device=DEV, eps_bh=EPS_BH,
                   bh_index=ns, flags=flags)
    r = np.linalg.norm(x[:ns], axis=1)
    idx = np.unique(np.concatenate([np.random.default_rng(11).choice(ns, 1024, replace=False),
                                    np.argsort(r)[:64], [ns]]))
    _, _, a, j, _, _, _ = cl.state()
    ra, rj = oracle.force(m, x, v, EPS, idx=idx, compensated=True, threads=oracle.max_threads(),
                          eps_bh=EPS_BH, bh=ns)
    ea, ej = rel_err_rows(host(a)[idx], ra), rel_err_rows(host(j)[idx], rj)
    print(f"flags={flags}: max rel err acc {ea.max():.2e} jerk {ej.max():.2e}; central particle "
          f"acc {ea[-1]:.2e} jerk {ej[-1]:.2e}")
    assert ea.max() <= tol and ej.max() <= tol
    idx_t = torch.empty(ns + 1, dtype=torch.int32, device=DEV)
    for step in range(3):
        xs, vs, a, j, t_i, dt_i, t_now = cl.state()
        ref = oracle.State.from_arrays(m, host(xs), host(vs), host(a), host(j), host(t_i), host(dt_i), t_now,
                                       EPS, ETA, DTMAX, DTMIN, threads=oracle.max_threads(), eps_bh=EPS_BH, bh=ns)
        act_ref = ref.block_step()
        g.gd_predict(cl.ctx)
        n_act = g.gd_active(cl.ctx, idx_t)
        np.testing.assert_array_equal(np.sort(host(idx_t[:n_act])), act_ref)
        g.gd_force(cl.ctx)
        g.gd_correct(cl.ctx)
        _, _, _, _, t_i, dt_i, t_now = cl.state()
        assert t_now == ref.t_now
        np.testing.assert_array_equal(host(t_i), ref.t_i)
        dt_gpu = host(dt_i)
        if flags == 0:
            np.testing.assert_array_equal(dt_gpu, ref.dt_i)
        else:
            diff = np.nonzero(dt_gpu != ref.dt_i)[0]
            assert len(diff) <= 1
            for i in diff:
                assert dt_gpu[i] in (2.0 * ref.dt_i[i], 0.5 * ref.dt_i[i])
    cl.close()


@pytest.mark.parametrize("ns,bh", [(20000, 7777), (16383, 16383), (16383, 0)])
def test_energy_with_central_particle_anywhere(ns, bh):
    """Energy (Eq. (2)) with the central particle at any index, both
    potentials: 20001 particles (four i per lane in the energy kernel, a
    ragged last i tile) and 16384 (the smallest such context), with the
    particle moved to the given index. Against the oracle to 1e-12."""
    m, x, v = plummer_with_bh(ns, 9)
    order = np.concatenate([np.arange(bh), [ns], np.arange(bh, ns)])
    m, x, v = m[order], x[order], v[order]
    cl = g.Cluster(m, x, v, eta=ETA, eps=EPS, dt_max=DTMAX, dt_min=DTMIN, device=DEV, eps_bh=EPS_BH,
                   bh_index=bh)
    ek, ep, eu = g.gd_energy(cl.ctx, unsoftened=True)
    rk, rp, ru = oracle.energy(m, x, v, EPS, unsoftened=True, eps_bh=EPS_BH, bh=bh)
    assert ek == pytest.approx(rk, rel=1e-12)
    assert ep == pytest.approx(rp, rel=1e-12)
    assert eu == pytest.approx(ru, rel=1e-12)
    # the central particle's pairs matter at this tolerance: eps instead of eps_bh fails
    _, rp_plain = oracle.energy(m, x, v, EPS)
    assert abs(rp_plain - rp) > 1e-10 * abs(rp)
    cl.close()
