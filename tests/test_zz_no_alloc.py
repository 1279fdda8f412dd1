"""The allocation-free pool step (hgks_pool_step_static) against hgks_pool_step.

Both run the same kernels; only where the launch tables live differs (a static
per-GPU array of the library against memory the pool allocates), so the results
must agree bitwise.  Two calls in a row, the second on a smaller batch, so the
static array is rewritten with smaller tables between them.
"""
import sys

import numpy as np
import pytest

from paper_2407_00656_amd import hgks
from tests.helpers import advection_case

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(mesh, q0, **kw):
    s = hgks.Solver(hgks.params(**kw))
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    s.init_state(q0)
    return s


def test_static_pool_step_equals_pool_step():
    say("case: allocation-free pool step against the pool step (two calls, the second smaller)")
    cases = [(7, 141, dict()), (6, 142, dict(precision=hgks.FP32_MIXED)), (5, 143, dict(tau_mode=1)),
             (8, 144, dict(precision=hgks.FP32))]
    ref, stat = [], []
    for n, seed, kw in cases:
        mesh, case, q0 = advection_case(n, seed=seed, vel=(0.6, -0.2, 0.4))
        ref.append(_solver(mesh, q0, **kw))
        stat.append(_solver(mesh, q0, **kw))
    pa, pb = hgks.Pool(), hgks.Pool()
    sa = [pa.add(s) for s in ref]
    sb = [pb.add(s) for s in stat]
    # call 1: the whole batch
    pa.step(sa, 2)
    pb.step_static(sb, 2)
    for k in range(len(cases)):
        qa, ta = ref[k].get_state()
        qb, tb = stat[k].get_state()
        assert ta == tb and ta > 0.0, k
        assert np.array_equal(qa, qb), k
    # call 2: a smaller batch (two of the four problems, one the smallest mesh)
    pick = [2, 1]
    pa.step([sa[k] for k in pick], 3)
    pb.step_static([sb[k] for k in pick], 3)
    for k in range(len(cases)):
        qa, ta = ref[k].get_state()
        qb, tb = stat[k].get_state()
        assert ta == tb, k
        assert np.array_equal(qa, qb), k
    for s in ref + stat:
        s.close()            # each leaves its pool first
    assert pa.used() == (0, 0) and pb.used() == (0, 0)
    pa.close()
    pb.close()
