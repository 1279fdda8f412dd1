"""Sod's shock tube on jittered Kuhn tetrahedra, FP64, FP32-mixed and FP32, on one GPU.

The configured case is the tube on [0, 1]^3 with 128^3 cubes (12.6 M cells): the
diaphragm at x = 0.5, transmissive walls at x = 0 and x = 1 (mirror-image
ghosts), y and z periodic, collision time tau_mode 1, CFL 0.3, to t = 0.2.
With --doubled the tube is instead laid out periodically (workloads.sod_box
without walls): on [0, 2) x [0, Ly) x [0, Lz) the high state fills [0.5, 1.5), so
each half of the period holds one tube, equal to the tube with transmissive ends
until t = 0.286 (use --nx 256 --ny 128 --nz 64 for the same spacing).

For each precision it reports the step rate (cell-updates/s over the whole run,
state resident on the GPU), the kernel split, and the volume-weighted L1 error
of density and pressure against the exact solution; the two reduced-precision
forms also report their relative L1 difference from FP64.

    python -m paper_2407_00656_amd.shock_tube [--nx 128 --ny 128 --nz 128] [--t-end 0.2] [--doubled]
"""
from __future__ import annotations

import argparse
import math
import json
import sys
import time

import numpy as np

from . import hgks
from . import workloads as W


def _pressure(q, gamma=1.4):
    return (gamma - 1.0) * (q[:, 4] - 0.5 * np.sum(q[:, 1:4] ** 2, axis=1) / q[:, 0])


def run(mesh, q0, precision, t_end, chunk=20, log=print, profile=True):
    s = hgks.Solver(hgks.params(precision=precision, tau_mode=1))
    t0 = time.perf_counter()
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    setup = time.perf_counter() - t0
    s.init_state(q0)
    s.profile_enable(profile)
    s.profile_reset()
    steps, t = 0, 0.0
    t0 = time.perf_counter()
    dt = s.step(1, want_dt=True)              # the CFL step, read back to plan the run
    steps += 1
    t = s.get_time()
    while t_end - t > 1e-12:
        rest = t_end - t
        if rest > (chunk + 4) * dt:
            s.step(chunk)                     # no host synchronisation inside a chunk
            steps += chunk
        elif rest > dt:
            # the last stretch in equal fixed steps, each at most 0.99 of the last CFL
            # step, so that no step overshoots t_end even if the CFL step would grow
            s.step(1, dt_fixed=rest / math.ceil(rest / (0.99 * dt)))
            steps += 1
        else:
            s.step(1, dt_fixed=rest)          # land on t_end (rest <= the CFL step)
            steps += 1
        t = s.get_time()
        if steps % 100 < chunk:
            log(f"shock_tube: prec={precision} steps={steps} t={t:.5f}")
    s.sync()
    el = time.perf_counter() - t0
    prof = {k: s.profile_read(k) for k in ("dt", "weno", "flux", "update")}
    q, t = s.get_state()
    s.close()
    return {"q": q, "t": t, "steps": steps, "seconds": el, "setup_s": setup, "prof": prof}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--ny", type=int, default=128)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--doubled", action="store_true", help="periodic doubled tube instead of walls")
    ap.add_argument("--t-end", type=float, default=0.2)
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel events")
    ap.add_argument("--fp64-only", action="store_true")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    log(f"shock_tube: building {args.nx}x{args.ny}x{args.nz} cubes")
    mesh, case = W.sod_box(args.nx, args.ny, args.nz, walls=not args.doubled)
    q0 = case.conservative(mesh)
    vol = W.tet_volumes(mesh.cell_vertices)
    x = mesh.cell_vertices[:, :, 0].mean(axis=1)
    layout = "periodic doubled" if args.doubled else "transmissive walls in x, periodic y/z"
    out = {"workload": f"shock tube, {layout}, {args.nx}x{args.ny}x{args.nz} cubes, tau_mode 1, CFL 0.3",
           "cells": mesh.n_cells, "t_end": args.t_end}
    res = {}
    precs = ((hgks.FP64, "fp64"),) if args.fp64_only else \
        ((hgks.FP64, "fp64"), (hgks.FP32_MIXED, "fp32_mixed"), (hgks.FP32, "fp32"))
    for prec, name in precs:
        r = run(mesh, q0, prec, args.t_end, log=log, profile=not args.no_profile)
        ex = case.exact(x, r["t"])
        q = r["q"]
        tot = float(np.sum(vol))
        entry = {"steps": r["steps"], "t": r["t"], "setup_s": round(r["setup_s"], 2),
                 "ms_per_step": round(1e3 * r["seconds"] / r["steps"], 4),
                 "cell_updates_per_s": round(mesh.n_cells * r["steps"] / r["seconds"], 1),
                 "kernel_ms_per_step": {k: round(v[0] / r["steps"], 4) for k, v in r["prof"].items()},
                 "L1_rho_vs_exact": float(np.sum(np.abs(q[:, 0] - ex[:, 0]) * vol) / tot),
                 "L1_p_vs_exact": float(np.sum(np.abs(_pressure(q) - ex[:, 2]) * vol) / tot)}
        res[name] = q
        out[name] = entry
    if args.fp64_only:
        print(json.dumps(out), flush=True)
        return
    d64 = res["fp64"]
    p64 = _pressure(d64)
    for name in ("fp32_mixed", "fp32"):
        d32 = res[name]
        out[name]["rel_L1_rho_vs_fp64"] = float(np.sum(np.abs(d32[:, 0] - d64[:, 0]) * vol) /
                                                np.sum(np.abs(d64[:, 0]) * vol))
        p32 = _pressure(d32)
        out[name]["rel_L1_p_vs_fp64"] = float(np.sum(np.abs(p32 - p64) * vol) / np.sum(np.abs(p64) * vol))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
