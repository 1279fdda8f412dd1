"""Serve loop on the GPU: every request finishes, each result is bitwise the
result of running that request alone, and admission respects the HBM budget."""
import sys

import numpy as np
import pytest

from paper_2407_00656_amd import hgks, serve
from paper_2407_00656_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_serve_mix_equals_alone_and_respects_budget():
    print("case: serve 8 requests N in [5, 10], 12 steps", flush=True)
    reqs = W.serve_requests(8, seed=77, n_range=(5, 10), steps=12, rate=200.0)
    # a budget that fits about three of the larger requests at once
    budget = 3 * hgks.pool_footprint(hgks.params(), 6 * 10 ** 3)
    res = serve.run(reqs, budget, max_steps_per_tick=5)
    assert res["requests"] == 8
    assert res["p99_s"] >= res["p50_s"] > 0
    for j in res["jobs"]:
        s = hgks.Solver(hgks.params(precision=j.req.precision))
        s.mesh_upload(j.mesh.nodes, j.mesh.cell_nodes, j.mesh.period)
        s.init_state(j.q0)
        s.step(j.req.steps)
        q, t = s.get_state()
        s.close()
        assert np.array_equal(q, j.q), j.req.rid
        assert t == j.t_sim
    errs = serve.exact_errors(res["jobs"])
    print("relative L1 vs exact", max(errs), flush=True)
    assert np.all(np.isfinite(errs)) and max(errs) < 0.2
