"""Continuous-batching serve loop: many HGKS solves of uneven size on one GPU.

Requests arrive over wall-clock time (Poisson), each carrying its payload: the
mesh (nodes and cells) and the initial state, which the client generated
beforehand (`make_payloads`, outside the timed run).  An arrived request is
prepared on a host worker thread: its mesh is uploaded on a stream of its own
(the host precompute runs there, and the copies overlap the pool's steps on the
device) and its initial state is set.  A
prepared request is admitted into the pool once its device footprint fits the
HBM budget.  Every tick advances all admitted requests together by K steps,
with one launch per phase covering every slot's tiles
(`hgks_pool_step`).  K is the smallest remaining step count, capped.  Finished
requests are read back and released, which frees budget for the next admissions.
Latency is completion minus arrival.

    python -m paper_2407_00656_amd.serve --requests 64 --rate 6 --budget-gb 64
"""
from __future__ import annotations

import argparse
import json
import math
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import hgks
from . import workloads as W


class Job:
    def __init__(self, req: W.Request):
        self.req = req
        self.mesh = None
        self.q0 = None
        self.solver = None
        self.slot = None
        self.done = 0
        self.t_arrive = None
        self.t_ready = None
        self.t_admit = None
        self.t_finish = None
        self.q = None
        self.t_sim = None
        self.error = None


def make_payloads(requests, npts: int = 3, workers: int = 8) -> dict:
    """The client side: each request's mesh and initial cell averages, by request id."""
    def one(r):
        mesh = W.kuhn_box(r.n, seed=r.seed)
        return r.rid, (mesh, r.case.conservative(mesh, npts=npts))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return dict(ex.map(one, requests))


def _prepare(job: Job, payload):
    r = job.req
    mesh, q0 = payload
    # each request uploads on a stream of its own, so its copies overlap the pool's steps
    s = hgks.Solver(hgks.params(precision=r.precision), stream=hgks.OWN_STREAM)
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    s.init_state(q0)
    job.mesh, job.q0, job.solver = mesh, q0, s
    return job


def run(requests, hbm_budget: int, max_steps_per_tick: int = 20, workers: int = 2, npts: int = 3,
        log=None, payloads: dict | None = None) -> dict:
    """Serves `requests` (arrival times in seconds from the start) and returns statistics.
    `payloads` (from make_payloads) is made here, before the clock starts, if not given."""
    if payloads is None:
        payloads = make_payloads(requests, npts)
    jobs = sorted((Job(r) for r in requests), key=lambda j: j.req.arrival)
    pool = hgks.Pool(hbm_budget=hbm_budget, stream=hgks.OWN_STREAM)
    exe = ThreadPoolExecutor(max_workers=workers)
    lock = threading.Lock()
    prepared = []                   # jobs ready for admission (arrival order)
    futures = []
    active = {}                     # slot -> job
    finished = []
    nxt = 0
    t0 = time.perf_counter()
    cell_updates = 0
    ticks = 0
    busy_s = 0.0

    def on_ready(fut):
        job = fut.result()
        job.t_ready = time.perf_counter() - t0
        with lock:
            prepared.append(job)

    try:
        while len(finished) < len(jobs):
            now = time.perf_counter() - t0
            while nxt < len(jobs) and jobs[nxt].req.arrival <= now:
                j = jobs[nxt]
                j.t_arrive = j.req.arrival
                f = exe.submit(_prepare, j, payloads[j.req.rid])
                f.add_done_callback(on_ready)
                futures.append(f)
                nxt += 1
            # admit prepared jobs in arrival order while they fit
            with lock:
                prepared.sort(key=lambda j: j.req.arrival)
                waiting = []
                for j in prepared:
                    used, _ = pool.used()
                    if hbm_budget and used + j.solver.footprint() > hbm_budget:
                        if not active and j.solver.footprint() > hbm_budget:
                            raise ValueError(f"request {j.req.rid} needs {j.solver.footprint()} B, over the budget")
                        waiting.append(j)
                        continue
                    j.slot = pool.add(j.solver)
                    j.t_admit = time.perf_counter() - t0
                    active[j.slot] = j
                prepared[:] = waiting
            if not active:
                for f in futures:
                    if f.done() and f.exception() is not None:
                        raise f.exception()
                time.sleep(0.002)
                continue
            k = min(max_steps_per_tick, min(j.req.steps - j.done for j in active.values()))
            slots = sorted(active)
            tb = time.perf_counter()
            pool.step(slots, k)
            next(iter(active.values())).solver.sync()      # waits for the pool's stream
            busy_s += time.perf_counter() - tb
            ticks += 1
            for s_ in slots:
                j = active[s_]
                j.done += k
                cell_updates += k * j.mesh.n_cells
            for s_ in slots:
                j = active[s_]
                if j.done >= j.req.steps:
                    j.q, j.t_sim = j.solver.get_state()
                    pool.remove(s_)
                    del active[s_]
                    j.t_finish = time.perf_counter() - t0
                    j.solver.close()
                    j.solver = None
                    finished.append(j)
                    if log:
                        log(f"done rid={j.req.rid} n={j.req.n} prec={j.req.precision} "
                            f"latency={j.t_finish - j.t_arrive:.3f}s")
        makespan = time.perf_counter() - t0
    finally:
        # on any exit the pool lets go of its slots before a solver can be freed
        exe.shutdown(wait=True)
        for s_ in list(active):
            pool.remove(s_)
        pool.close()
        for f in futures:
            if f.done() and f.exception() is None:
                j = f.result()
                if j.solver is not None and j not in finished:
                    j.solver.close()
    lat = np.array([j.t_finish - j.t_arrive for j in finished])
    return {
        "requests": len(finished),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "makespan_s": makespan,
        "gpu_busy_s": busy_s,
        "ticks": ticks,
        "cell_updates": int(cell_updates),
        "cell_updates_per_s": cell_updates / makespan,
        "cell_updates_per_busy_s": cell_updates / max(busy_s, 1e-9),
        "jobs": finished,
    }


def exact_errors(jobs, npts: int = 3):
    """Relative L1 density error of each finished job against the translated exact solution."""
    out = []
    for j in jobs:
        vol = W.tet_volumes(j.mesh.cell_vertices)
        ex = j.req.case.density_average(j.mesh, j.t_sim, npts=npts)
        out.append(float(np.sum(np.abs(j.q[:, 0] - ex) * vol) / np.sum(np.abs(ex) * vol)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=6.0, help="Poisson arrivals per second")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--nmin", type=int, default=8)
    ap.add_argument("--nmax", type=int, default=48)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--seed", type=int, default=2407)
    ap.add_argument("--tick", type=int, default=20)
    args = ap.parse_args()
    reqs = W.serve_requests(args.requests, seed=args.seed, n_range=(args.nmin, args.nmax), steps=args.steps,
                            rate=args.rate)
    res = run(reqs, int(args.budget_gb * 1e9), max_steps_per_tick=args.tick)
    errs = exact_errors(res["jobs"])
    res.pop("jobs")
    res["rel_L1_vs_exact_max"] = max(errs)
    res["rel_L1_vs_exact_median"] = float(np.median(errs))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
