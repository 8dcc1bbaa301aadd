"""Seeded random shapes against the oracle: particle counts from 2 to 3000
(tile edges included), softening 0 or 1e-4, FP64 or mixed pair arithmetic,
with or without a central particle. For each configuration the initial
acceleration and jerk of every particle are compared with the oracle's
compensated sums (1e-12 per particle in FP64, 2e-6 in mixed precision); the
FP64 configurations of up to 1200 particles are then integrated to t = 1/8
and must take the oracle's block, particle and clamp counts, with positions
within 1e-9."""
import numpy as np
import pytest

import oracle
from paper_1702_00440_amd import gravidy as g
from synth_inputs import plummer, plummer_with_bh
from tests.gpu_util import DEV, host, rel_err_rows

pytestmark = pytest.mark.gpu

ETA, DT_MAX, DT_MIN = 0.01, 0.125, 2.0 ** -22


def _configs():
    rng = np.random.default_rng(20240601)
    edges = [2, 3, 255, 256, 257, 511, 1023, 1025]
    ns = edges + [int(v) for v in rng.integers(4, 3001, 8)]
    out = []
    for k, n in enumerate(ns):
        eps = 0.0 if (k % 3 == 0 and n <= 1100) else 1e-4
        mixed = k % 4 == 1
        central = eps > 0 and n >= 16 and k % 5 == 2
        out.append((n, eps, mixed, central, 700 + k))
    return out


@pytest.mark.parametrize("n,eps,mixed,central,seed", _configs())
def test_random_shape_against_oracle(n, eps, mixed, central, seed):
    if central:
        m, x, v = plummer_with_bh(n - 1, seed, m_bh=0.01)
        bh, eps_bh = n - 1, 1e-6
    else:
        m, x, v = plummer(n, seed)
        bh, eps_bh = -1, eps
    flags = g.GD_FLAG_MIXED if mixed else 0
    kw = dict(eps_bh=eps_bh, bh_index=bh) if central else {}
    cl = g.Cluster(m, x, v, eta=ETA, eps=eps, dt_max=DT_MAX, dt_min=DT_MIN, device=DEV, flags=flags, **kw)
    _, _, a, j, _, _, _ = cl.state()
    ra, rj = oracle.force(m, x, v, eps, compensated=True, threads=oracle.max_threads(), eps_bh=eps_bh, bh=bh)
    ea, ej = rel_err_rows(host(a), ra).max(), rel_err_rows(host(j), rj).max()
    tol = 2e-6 if mixed else 1e-12
    print(f"n={n} eps={eps} mixed={mixed} central={central}: acc {ea:.2e} jerk {ej:.2e}")
    assert ea <= tol and ej <= tol
    if not mixed and n <= 1200:
        st = g.gd_step_to(cl.ctx, 0.125)
        ref = oracle.State(m, x, v, eps, ETA, DT_MAX, DT_MIN, threads=oracle.max_threads(), eps_bh=eps_bh, bh=bh)
        ref.run(0.125)
        assert (st["block_steps"], st["particle_steps"], st["dtmin_clamps"]) == \
            (int(ref.stats[0]), int(ref.stats[1]), int(ref.stats[3]))
        dx = np.abs(host(cl.state()[0]) - ref.x).max()
        assert dx <= 1e-9, dx
    cl.close()
