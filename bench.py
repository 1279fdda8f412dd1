"""Throughput of the HGKS S2O4 step on one MI355X.

Workload: the smooth-advection accuracy test of Sec. 5.1 at 6*64^3 = 1,572,864
jittered Kuhn tetrahedra (periodic [0,2]^3, rho = 1 + 0.2 sin(pi(x+y+z)),
U = V = W = 1, p = 1, CFL 0.3, tau = 0), inputs already resident in HBM.
A step is one full two-stage S2O4 step (CFL dt, two WENO reconstructions,
two face-flux passes, two stage updates).  Reports cell-updates/s for the FP64
path (the headline value) and for the FP32-mixed and FP32 forms, the roofline position
of the dominant kernel (per-kernel HIP events inside the timed region), and the
CPU oracle timed on this host.

The serve loop (continuous batching of many smaller solves) runs after the
step timings: a seeded stream of 256 requests (Kuhn boxes of 6 N^3 cells,
N ~ U{8..48}, random smooth data, Mach 0.1-2, FP64 or FP32-mixed, 200 steps
each); the first 64 are served all at once to measure the loop's capacity, then
all 256 with Poisson arrivals at 0.8 of that capacity; the line reports p50/p99
latency (arrival to result on the host, host mesh precompute included),
aggregate cell-updates/s, and (with the CPU leg) the oracle's verdict on the
served requests with N = 8 over their whole run and on two steps of eight
sampled larger ones.

    python bench.py [--steps K] [--warmup W] [--n N] [--no-cpu-baseline] [--serve R]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector

# Algorithmic bytes each kernel must move, per unit (cell or face), FP64 form:
#   weno   per cell: 16 stencil ids (64) + own state (40) + big-stencil pseudo-inverse
#          9x16 (1152) + 1/h and second moments (56) + own centroid (24) + slot image
#          codes (16) + reconstruction written (400)                           = 1752
#          (the sub-stencil fits are formed on the device from the centroids;
#          FP32-mixed writes 200)
#   flux   per face: cells (8) + normal, area, Gauss offsets and the centroid difference
#          (128) + flux written (80) = 216 in the first stage and 176 in the second (dF
#          only), plus per cell the reconstruction read once (400)
#   update per cell: face ids (16) + its faces' fluxes (2 faces' worth, 160) + 1/|V|
#          and h (16) + state traffic (stage 1: 3 x 40, stage 2: 2 x 40)       ~ 292
# The FP32 form (fp32=True) stores state, cell and face geometry and face fluxes in
# 4-byte words and streams a 576 B pseudo-inverse; ids, centroids and codes are as above.
def algorithmic_bytes(kernel: str, nc: int, nf: int, mixed: bool, fp32: bool = False) -> float:
    es = 4 if fp32 else 8
    if kernel == "weno":
        return nc * (64 + 5 * es + (576 if fp32 else 1152) + 7 * es + 24 + 16 + (200 if mixed else 400))
    if kernel == "flux":   # first stage F and dF/dt, second stage dF/dt only
        return nf * (8 + 16 * es + 7.5 * es) + nc * ((200 + 5 * es) if mixed else 400)
    if kernel == "update":
        return nc * (16 + 20 * es + 2 * es + 12.5 * es)
    if kernel == "weno_hex":   # 24 stencil ids, own state, 9 x 24 pseudo-inverse, eight 3 x 3 inverses,
        # seven geometry values, the record written (FP64 or FP32-mixed)
        return nc * (96 + 40 + 1728 + 576 + 56 + (200 if mixed else 400))
    return 0.0


# Lower bound on the bytes a cell-update must move whatever the design (FP64, Kuhn
# tets, K = 14, two stages): per stage the state (40), cell geometry (80), stencil
# ids and sub-stencil positions (80), a 9 x 14 big-stencil pseudo-inverse (1008), four
# 3 x 6 sub-stencil pseudo-inverses (576), two faces' geometry (224), L and dL/dt
# written (80) and the update's state traffic (40-120), with the time-step pass:
# about 4.34 KB, the HBM roofline 8 TB/s / 4.34 KB = 1.84e9 cell-updates/s.
TABLE_BOUND_BYTES_PER_CELL_UPDATE = 4340.0


def reduced_weno(r, nc: int, nf: int, fp32: bool):
    """Average WENO launch time of a reduced-precision run, and its algorithmic rate."""
    ms, cnt = r["prof"]["weno"]
    if not cnt:
        return None
    avg_s = ms / 1e3 / cnt
    return {"us": round(1e6 * avg_s, 2),
            "alg_GBps": round(algorithmic_bytes("weno", nc, nf, True, fp32) / avg_s / 1e9, 1)}


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2407_00656_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernels_hip_sha") != kernel_source_hash() or t.get("workload") != workload:
        return None
    v = t.get("bytes_per_launch", {}).get(kernel)
    return float(v) if v is not None else None


def run_gpu(mesh, q0, precision, steps, warmup):
    from paper_2407_00656_amd import hgks
    s = hgks.Solver(hgks.params(precision=precision))
    t0 = time.perf_counter()
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    t_setup = time.perf_counter() - t0
    s.init_state(q0)
    s.step(warmup)
    s.sync()
    s.profile_enable(True)
    s.profile_reset()
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    el = time.perf_counter() - t0
    prof = {k: s.profile_read(k) for k in ("dt", "weno", "flux", "update")}
    s.profile_enable(False)
    info = s.info()
    foot = s.footprint()
    q, t = s.get_state()
    s.close()
    return {"seconds": el, "setup_s": t_setup, "prof": prof, "info": info, "footprint": foot, "t": t, "q": q}


def sphere_bench(n: int, layers: int, run_steps: int, steps: int, warmup: int) -> dict:
    """The viscous sphere (Sec. 5.2) on the cubed-sphere O-grid of hexahedra, FP64 and
    FP32-mixed: `steps` timed steps after `warmup`, then the rest of a `run_steps`
    run from the free stream, and the FP32-mixed state's relative L1 against FP64's
    at its end."""
    from paper_2407_00656_amd import hgks
    from paper_2407_00656_amd import workloads as W
    case = W.SphereCase()
    mesh = W.cubed_sphere(n, layers)
    q0 = case.conservative(mesh)
    kw = dict(tau_mode=2, mu_ref=case.mu_inf(), T_ref=case.t_inf(), mu_exp=0.7, prandtl=case.prandtl,
              farfield=case.freestream())
    nc = mesh.n_cells
    out = {"workload": f"viscous sphere, cubed-sphere O-grid 6*{n}*{n}*{layers} hexahedra, r 0.5 to 20, "
                       f"Ma {case.mach}, Re {case.reynolds}, Pr {case.prandtl}, mu ~ T^0.7, no-slip wall, "
                       f"far field, CFL 0.3", "cells": nc}
    states = {}
    for name, prec in (("fp64", hgks.FP64), ("fp32_mixed", hgks.FP32_MIXED)):
        print(f"bench: sphere {name}", file=sys.stderr, flush=True)
        s = hgks.Solver(hgks.params(precision=prec, **kw))
        t0 = time.perf_counter()
        s.upload(mesh)
        setup = time.perf_counter() - t0
        s.init_state(q0)
        t_run = time.perf_counter()
        s.step(warmup)
        s.sync()
        s.profile_enable(True)
        s.profile_reset()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        el = time.perf_counter() - t0
        prof = {k: s.profile_read(k) for k in ("dt", "weno", "flux", "update")}
        s.profile_enable(False)
        rest = max(0, run_steps - warmup - steps)
        s.step(rest)
        s.sync()
        run_s = time.perf_counter() - t_run
        q, t = s.get_state()
        out["faces"] = s.info()["n_faces"]
        wms, wcnt = prof["weno"]
        wb = algorithmic_bytes("weno_hex", nc, 0, prec != hgks.FP64)
        wgbs = wb / (wms / 1e3 / max(1, wcnt)) / 1e9
        out[name] = {"value": round(nc * steps / el, 1), "ms_per_step": round(1e3 * el / steps, 4),
                     "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items()},
                     "weno_roofline": {"bound": "hbm", "achieved": round(wgbs, 1), "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(wgbs / HBM_PEAK_GBS, 4),
                                       "alg_bytes_per_launch": wb,
                                       "avg_launch_us": round(1e3 * wms / max(1, wcnt), 1)},
                     "run_steps": warmup + steps + rest, "run_s": round(run_s, 2), "t": t,
                     "setup_s": round(setup, 2), "footprint_GB": round(s.footprint() / 1e9, 3)}
        s.close()
        states[name] = q
    out["fp32_mixed"]["speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["fp32_mixed"]["ms_per_step"], 3)
    vol = W.hex_volumes(mesh.cell_vertices)
    a, b = states["fp32_mixed"], states["fp64"]
    rho = b[:, 0]
    p = (case.gamma - 1) * (b[:, 4] - 0.5 * np.sum(b[:, 1:4] ** 2, axis=1) / rho)
    ms = np.maximum(np.linalg.norm(b[:, 1:4], axis=1), rho * np.sqrt(case.gamma * np.abs(p) / rho))
    den = np.array([np.sum(rho * vol), *(3 * [np.sum(ms * vol)]), np.sum(np.abs(b[:, 4]) * vol)])
    out["rel_L1_fp32_mixed_vs_fp64"] = (np.sum(np.abs(a - b) * vol[:, None], axis=0) / den).tolist()
    out["max_mach"] = float(np.max(np.linalg.norm(b[:, 1:4], axis=1) / rho / np.sqrt(case.gamma * p / rho)))
    return out


def cpu_oracle_step(mesh, q0):
    """Seconds of one FP64 oracle S2O4 step on `mesh` (its mesh precompute not timed)."""
    from oracle import oracle as O
    om = O.Mesh.from_workload(mesh)
    t0 = time.perf_counter()
    om.step(q0, 1)
    return time.perf_counter() - t0


def cpu_single_thread(n: int) -> dict:
    """Child-process leg: one oracle step on 6*n^3 tets, one OpenMP thread pinned to one
    core (this process never touches the GPU)."""
    from oracle import oracle as O
    from paper_2407_00656_amd import workloads as W
    core = min(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {core})
    mesh = W.kuhn_box(n, seed=W.SEED_ADVECTION + n)
    q0 = W.AdvectionCase().conservative(mesh)
    el = cpu_oracle_step(mesh, q0)
    return {"value": mesh.n_cells / el, "cells": mesh.n_cells, "seconds": el, "threads": O.threads(), "core": core}


def cpu_baseline(mesh, q0, workload: str, n_single: int = 32):
    """The FP64 oracle on this host: one step of the bench's own mesh on all host threads
    (the reported value), and one step of 6*n_single^3 tets single-threaded, pinned."""
    from oracle import oracle as O
    el = cpu_oracle_step(mesh, q0)
    out = {"value": mesh.n_cells / el, "unit": "cell-updates/s", "cores": O.threads(), "kind": "oracle",
           "sample": f"one S2O4 step of the FP64 oracle on the bench mesh ({workload}, {mesh.n_cells} tets) "
                     f"on {O.threads()} OpenMP threads, {el:.1f} s"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-single", str(n_single)], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode == 0 and r.stdout.strip():
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["single_thread"] = {"value": one["value"], "unit": "cell-updates/s", "cores": one["threads"],
                                "sample": f"one S2O4 step on 6*{n_single}^3 = {one['cells']} tets, one thread "
                                          f"pinned to core {one['core']}, {one['seconds']:.1f} s"}
    else:
        out["single_thread"] = {"error": (r.stderr or "")[-300:]}
    return out


def serve_bench(count: int, steps: int, budget_gb: float, capacity_count: int, two_step_sample: int = 8):
    """Closed-loop capacity on the first `capacity_count` requests, then all `count`
    requests with Poisson arrivals at 0.8 of that capacity (requests/s).  Also runs a
    seeded sample of the larger requests alone for two steps on the GPU (alone and in
    the mix are bitwise the same), for the oracle check of the CPU leg."""
    from paper_2407_00656_amd import hgks
    from paper_2407_00656_amd import serve
    from paper_2407_00656_amd import workloads as W
    reqs = W.serve_requests(count, seed=2407, n_range=(8, 48), steps=steps, rate=1.0)
    budget = int(budget_gb * 1e9)
    print(f"bench: serve payloads for {count} requests", file=sys.stderr, flush=True)
    payloads = serve.make_payloads(reqs)          # the clients' meshes and initial states
    first = reqs[:capacity_count]
    for r in first:
        r.arrival = 0.0
    print(f"bench: serve capacity pass ({capacity_count} requests at once)", file=sys.stderr, flush=True)
    burst = serve.run(first, budget, workers=4, payloads=payloads)
    capacity = burst["requests"] / burst["makespan_s"]
    rate = 0.8 * capacity
    reqs = W.serve_requests(count, seed=2407, n_range=(8, 48), steps=steps, rate=rate)
    print(f"bench: serve Poisson pass ({count} requests at {rate:.2f}/s)", file=sys.stderr, flush=True)
    res = serve.run(reqs, budget, workers=4, payloads=payloads,
                    log=lambda m: print("bench: serve " + m, file=sys.stderr, flush=True)
                    if m.startswith("done") and int(m.split("rid=")[1].split()[0]) % 32 == 0 else None)
    errs = serve.exact_errors(res["jobs"])
    cells = [j.mesh.n_cells for j in res["jobs"]]
    # two-step GPU results of a seeded sample of the requests with N > 8
    big = [j for j in res["jobs"] if j.req.n > 8]
    pick = sorted(big, key=lambda j: (j.req.rid * 2654435761) % 4294967296)[:two_step_sample]
    two = []
    for j in pick:
        s = hgks.Solver(hgks.params(precision=j.req.precision))
        s.mesh_upload(j.mesh.nodes, j.mesh.cell_nodes, j.mesh.period)
        s.init_state(j.q0)
        s.step(2)
        two.append((j, s.get_state()[0]))
        s.close()
    out = {"requests": res["requests"], "steps_each": steps, "n_range": [8, 48],
           "cells_mean": round(float(sum(cells)) / len(cells), 1),
           "precision_mix_fp32": sum(j.req.precision for j in res["jobs"]),
           "rate_req_per_s": round(rate, 4), "capacity_req_per_s": round(capacity, 4),
           "capacity_pass_requests": capacity_count,
           "p50_s": round(res["p50_s"], 4), "p99_s": round(res["p99_s"], 4),
           "cell_updates_per_s": round(res["cell_updates_per_s"], 1),
           "cell_updates_per_gpu_busy_s": round(res["cell_updates_per_busy_s"], 1),
           "ticks": res["ticks"], "hbm_budget_GB": budget_gb,
           "rel_L1_rho_vs_exact_max": max(errs)}
    return out, res["jobs"], two


def serve_oracle_check(jobs, two) -> dict:
    """The CPU oracle on served requests: every served request with N = 8 over its whole
    run, and the two-step results of the sampled larger ones.  FP64 requests report the
    largest scaled error per conserved variable (the norm of the GPU parity tests),
    FP32-mixed ones the relative L1 of density against the FP64 oracle."""
    import numpy as np
    from oracle import oracle as O
    from paper_2407_00656_amd import workloads as W

    def compare(j, q_gpu, nsteps):
        om = O.Mesh.from_workload(j.mesh)
        q_orc, _ = om.step(j.q0, nsteps)
        vol = W.tet_volumes(j.mesh.cell_vertices)
        rho = q_orc[:, 0]
        l1 = float(np.sum(np.abs(q_gpu[:, 0] - rho) * vol) / np.sum(np.abs(rho) * vol))
        m = q_orc[:, 1:4]
        pr = 0.4 * (q_orc[:, 4] - 0.5 * np.sum(m * m, axis=1) / rho)
        ms = max(np.sqrt(np.sum(m * m, axis=1)).max(), np.max(rho * np.sqrt(1.4 * pr / rho)))
        scale = np.array([np.abs(rho).max(), ms, ms, ms, np.abs(q_orc[:, 4]).max()])
        scaled = float((np.abs(q_gpu - q_orc).max(axis=0) / scale).max())
        return {"rid": j.req.rid, "n": j.req.n, "precision": "fp32_mixed" if j.req.precision else "fp64",
                "steps": nsteps, "max_scaled_err": scaled, "rel_L1_rho": l1}

    t0 = time.perf_counter()
    full = [compare(j, j.q, j.req.steps) for j in jobs if j.req.n == 8]
    short = [compare(j, q2, 2) for j, q2 in two]
    rows = full + short

    def worst(prec, key):
        v = [r[key] for r in rows if r["precision"] == prec]
        return max(v) if v else None
    return {"full_runs": len(full), "two_step_runs": len(short), "seconds": round(time.perf_counter() - t0, 1),
            "fp64_max_scaled_err": worst("fp64", "max_scaled_err"),
            "fp32_mixed_max_rel_L1_rho": worst("fp32_mixed", "rel_L1_rho"), "requests": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--serve", type=int, default=256, help="requests in the serve-loop run (0 skips it)")
    ap.add_argument("--serve-capacity", type=int, default=64,
                    help="requests of the closed-loop pass that measures the loop's capacity")
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--sphere", type=int, default=48, help="cells across a patch of the sphere O-grid (0 skips it)")
    ap.add_argument("--sphere-layers", type=int, default=64)
    ap.add_argument("--sphere-run", type=int, default=2000, help="steps of the sphere run (FP64 vs FP32-mixed)")
    ap.add_argument("--cpu-single", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 1 GiB (x5) to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.cpu_single:          # the single-threaded oracle leg, run as a child process
        print(json.dumps(cpu_single_thread(args.cpu_single)), flush=True)
        return
    if args.copy_calibration:
        import torch
        x = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": x.numel() * 8, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU halo "
              "exchange is not part of this build", file=sys.stderr)
        sys.exit(2)

    from paper_2407_00656_amd import hgks
    from paper_2407_00656_amd import workloads as W

    n = args.n
    print(f"bench: building inputs 6*{n}^3", file=sys.stderr, flush=True)
    mesh = W.kuhn_box(n, seed=W.SEED_ADVECTION + (0 if n == 8 else n))
    q0 = W.AdvectionCase().conservative(mesh)
    nc = mesh.n_cells
    workload = f"advection 6*{n}^3 tets"

    print("bench: FP64", file=sys.stderr, flush=True)
    r64 = run_gpu(mesh, q0, hgks.FP64, args.steps, args.warmup)
    nf = r64["info"]["n_faces"]
    value = nc * args.steps / r64["seconds"]
    r32 = r32f = None
    if not args.no_fp32:
        print("bench: FP32-mixed", file=sys.stderr, flush=True)
        r32 = run_gpu(mesh, q0, hgks.FP32_MIXED, args.steps, args.warmup)
        print("bench: FP32", file=sys.stderr, flush=True)
        r32f = run_gpu(mesh, q0, hgks.FP32, args.steps, args.warmup)

    sph = None
    if args.sphere > 0:
        sph = sphere_bench(args.sphere, args.sphere_layers, args.sphere_run, args.steps, args.warmup)

    # dominant kernel of the FP64 step and its roofline position
    prof = r64["prof"]
    dom = max(("weno", "flux", "update"), key=lambda k: prof[k][0])
    ms_total, launches = prof[dom]
    avg_s = ms_total / 1e3 / max(1, launches)
    per_launch = algorithmic_bytes(dom, nc, nf, False)
    achieved = per_launch / avg_s / 1e9
    kernels = {}
    for k in ("dt", "weno", "flux", "update"):
        ms, cnt = prof[k]
        b = algorithmic_bytes(k, nc, nf, False)
        kernels[k] = {"avg_us": 1e3 * ms / max(1, cnt), "launches": cnt,
                      "share": ms / max(1e-12, sum(v[0] for v in prof.values())),
                      "alg_GBps": (b / (ms / 1e3 / max(1, cnt)) / 1e9) if b and cnt else None}
    # the whole step: every kernel's algorithmic bytes over the measured step time
    step_bytes = sum(algorithmic_bytes(k, nc, nf, False) * prof[k][1] for k in ("weno", "flux", "update")) / args.steps
    step_s = r64["seconds"] / args.steps
    path = {"alg_bytes_per_step": step_bytes, "alg_bytes_per_cell_update": round(step_bytes / nc, 1),
            "achieved_GBps": round(step_bytes / step_s / 1e9, 1),
            "frac": round(step_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
            "table_bound_cell_updates_per_s": round(HBM_PEAK_GBS * 1e9 / TABLE_BOUND_BYTES_PER_CELL_UPDATE, 1),
            "frac_of_table_bound": round(value / (HBM_PEAK_GBS * 1e9 / TABLE_BOUND_BYTES_PER_CELL_UPDATE), 4)}
    traffic = measured_traffic(dom, workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": per_launch, "avg_launch_us": round(avg_s * 1e6, 2)}

    srv = jobs = two = None
    if args.serve > 0:
        print("bench: serve loop", file=sys.stderr, flush=True)
        srv, jobs, two = serve_bench(args.serve, args.serve_steps, args.serve_budget_gb,
                                     min(args.serve, args.serve_capacity))

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(mesh, q0, workload, 32 if n >= 32 else n)
        if srv is not None:
            print("bench: CPU oracle on served requests", file=sys.stderr, flush=True)
            srv["vs_oracle"] = serve_oracle_check(jobs, two)

    out = {
        "metric": "cell-updates/s per S2O4 step on 1 MI355X (FP64 vs FP32-mixed); serve p50/p99",
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r64["seconds"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{workload}, periodic [0,2]^3, jitter 0.1h, rho=1+0.2sin(pi(x+y+z)), "
                               f"U=(1,1,1), p=1, CFL 0.3, tau=0", "cells": nc, "faces": nf},
        "roofline": roofline,
        "path_roofline": path,
        "cpu_baseline": cpu,
        "fp32_mixed": None if r32 is None else {
            "value": round(nc * args.steps / r32["seconds"], 1),
            "ms_per_step": round(1e3 * r32["seconds"] / args.steps, 4),
            "speedup_vs_fp64": round(r64["seconds"] / r32["seconds"], 3),
            "weno": reduced_weno(r32, nc, nf, False)},
        "fp32": None if r32f is None else {
            "value": round(nc * args.steps / r32f["seconds"], 1),
            "ms_per_step": round(1e3 * r32f["seconds"] / args.steps, 4),
            "speedup_vs_fp64": round(r64["seconds"] / r32f["seconds"], 3),
            "weno": reduced_weno(r32f, nc, nf, True)},
        "serve": srv,
        "sphere": sph,
        "kernels": kernels,
        "setup_s": round(r64["setup_s"], 2),
        "footprint_GB": round(r64["footprint"] / 1e9, 3),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
