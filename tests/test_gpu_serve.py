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


def _scaled_err(q, q_ref, gamma=1.4):
    rho = q_ref[:, 0]
    m = q_ref[:, 1:4]
    p = (gamma - 1) * (q_ref[:, 4] - 0.5 * np.sum(m * m, axis=1) / rho)
    ms = max(np.sqrt(np.sum(m * m, axis=1)).max(), np.max(rho * np.sqrt(gamma * p / rho)))
    s = np.array([np.abs(rho).max(), ms, ms, ms, np.abs(q_ref[:, 4]).max()])
    return np.abs(q - q_ref).max(axis=0) / s


def test_served_requests_match_the_oracle():
    """Served results against the FP64 CPU oracle run on the same request: six small
    requests over their whole run (40 steps) and two larger ones over two steps, all
    served together with mixed precisions.  FP64 requests agree to 1e-11 scaled error
    (the per-step bar of 1e-12 with room for 40 steps of accumulated rounding), FP32-mixed
    ones to 1e-5 relative L1 in every variable (momentum against a momentum scale)."""
    import dataclasses

    from oracle import oracle as O
    from tests.helpers import rel_l1_scaled

    print("case: serve 6 small requests (40 steps) and 2 larger ones (2 steps) against the oracle", flush=True)
    small = W.serve_requests(6, seed=91, n_range=(6, 9), steps=40, rate=100.0)
    large = W.serve_requests(2, seed=92, n_range=(20, 24), steps=2, rate=100.0)
    reqs = small + [dataclasses.replace(r, rid=len(small) + k, arrival=r.arrival + 0.01) for k, r in enumerate(large)]
    assert {r.precision for r in reqs} == {0, 1}
    res = serve.run(reqs, 0, max_steps_per_tick=7)
    assert res["requests"] == len(reqs)
    for j in res["jobs"]:
        om = O.Mesh.from_workload(j.mesh)
        q_orc, _ = om.step(j.q0, j.req.steps)
        vol = W.tet_volumes(j.mesh.cell_vertices)
        if j.req.precision == 0:
            e = _scaled_err(j.q, q_orc)
            print(f"rid {j.req.rid} N={j.req.n} FP64 {j.req.steps} steps: max scaled err {e.max():.2e}", flush=True)
            assert np.all(e <= 1e-11), (j.req.rid, e)
        else:
            e = rel_l1_scaled(j.q, q_orc, vol)
            print(f"rid {j.req.rid} N={j.req.n} FP32-mixed {j.req.steps} steps: rel L1 {e.max():.2e}", flush=True)
            assert np.all(e <= 1e-5), (j.req.rid, e)
