"""The viscous flow past a sphere (Sec. 5.2) run to a steady wake on one GPU, with the
closed wake length L and the separation angle theta the paper reports: Re = 118,
Ma = 0.2535 (the default; its table: L = 0.99, theta = 128.4 degrees on 3.1 M
hexahedra) and Re = 300, Ma = 1.5 (--reynolds 300 --mach 1.5; L = 1.18, theta = 136.8).

The run starts from the free stream on the cubed-sphere O-grid (workloads.cubed_sphere,
the +x patch downstream) and steps at CFL 0.3; every `--every` steps it prints the
simulated time and the current L and theta, so that their convergence shows.

  * L: along the downstream axis, the mean streamwise velocity of the four cells of the
    +x patch around the axis in each radial layer; L is the distance from the sphere's
    rear point (x = 0.5) to the first sign change of that profile (linear
    interpolation between layers), in diameters.
  * theta: in the first cell layer, the velocity along the meridian (e_theta, pointing
    from the front stagnation point at -x towards the rear), averaged over azimuth in
    one-degree bins of the polar angle from the front point; theta is the first angle
    beyond 90 degrees where it changes sign (linear interpolation between bins).

    python -m paper_2407_00656_amd.sphere_run [--n 48 --layers 64] [--t-end 150] [--precision fp64]
                                              [--reynolds 300 --mach 1.5]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import hgks
from . import workloads as W


# the paper's values for its two sphere cases (Sec. 5.2 tables, 3,145,728 hexahedra)
PAPER = {(118.0, 0.2535): {"L": 0.99, "theta_deg": 128.4, "cells": 3145728},
         (300.0, 1.5): {"L": 1.18, "theta_deg": 136.8, "cells": 3145728}}


def axis_profile(mesh, q, n: int, layers: int):
    """(x, u_x) per radial layer of the four +x-patch cells around the downstream axis."""
    c = mesh.cell_vertices.mean(axis=1)
    lo = (n - 1) // 2
    ij = [(i, j) for i in (lo, n // 2) for j in (lo, n // 2)]
    ij = sorted(set(ij))
    xs, us = [], []
    for k in range(layers):
        ids = [(i * n + j) * layers + k for i, j in ij]          # patch 0: the +x patch
        xs.append(float(np.mean(c[ids, 0])))
        us.append(float(np.mean(q[ids, 1] / q[ids, 0])))
    return np.array(xs), np.array(us)


def wake_length(mesh, q, n: int, layers: int, r0: float = 0.5) -> float:
    """Distance from the rear point to the first zero of the axial velocity behind it
    (nan if the flow on the axis never reverses)."""
    x, u = axis_profile(mesh, q, n, layers)
    if not u[0] < 0.0:
        return float("nan")
    for k in range(1, layers):
        if u[k] >= 0.0:
            xz = x[k - 1] + (x[k] - x[k - 1]) * (-u[k - 1]) / (u[k] - u[k - 1])
            return float(xz - r0)
    return float("nan")


def meridional_profile(mesh, q, layers: int, bins: int = 180):
    """(theta in degrees, mean u_theta) in the first cell layer, per one-degree bin."""
    first = np.arange(mesh.n_cells) % layers == 0
    c = mesh.cell_vertices[first].mean(axis=1)
    u = q[first, 1:4] / q[first, :1]
    r = np.linalg.norm(c, axis=1)
    ryz = np.maximum(np.hypot(c[:, 1], c[:, 2]), 1e-300)
    th = np.degrees(np.arccos(np.clip(-c[:, 0] / r, -1.0, 1.0)))
    e = np.stack([ryz / r, (-c[:, 0] / r) * c[:, 1] / ryz, (-c[:, 0] / r) * c[:, 2] / ryz], axis=1)
    ut = np.sum(u * e, axis=1)
    b = np.minimum((th / (180.0 / bins)).astype(int), bins - 1)
    cnt = np.bincount(b, minlength=bins)
    ok = cnt > 0
    tm = np.bincount(b, weights=th, minlength=bins)[ok] / cnt[ok]
    um = np.bincount(b, weights=ut, minlength=bins)[ok] / cnt[ok]
    return tm, um


def separation_angle(mesh, q, layers: int) -> float:
    """First polar angle beyond 90 degrees (from the front point) where the meridional
    velocity next to the wall turns negative (nan if it never does)."""
    th, ut = meridional_profile(mesh, q, layers)
    for k in range(1, len(th)):
        if th[k - 1] > 90.0 and ut[k - 1] > 0.0 and ut[k] <= 0.0:
            return float(th[k - 1] + (th[k] - th[k - 1]) * ut[k - 1] / (ut[k - 1] - ut[k]))
    return float("nan")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--layers", type=int, default=64)
    ap.add_argument("--t-end", type=float, default=150.0)
    ap.add_argument("--every", type=int, default=2000)
    ap.add_argument("--precision", choices=("fp64", "fp32_mixed"), default="fp64")
    ap.add_argument("--mach", type=float, default=0.2535)
    ap.add_argument("--reynolds", type=float, default=118.0)
    a = ap.parse_args(argv)
    case = W.SphereCase(mach=a.mach, reynolds=a.reynolds)
    mesh = W.cubed_sphere(a.n, a.layers)
    prec = hgks.FP64 if a.precision == "fp64" else hgks.FP32_MIXED
    s = hgks.Solver(hgks.params(precision=prec, tau_mode=2, mu_ref=case.mu_inf(), T_ref=case.t_inf(), mu_exp=0.7,
                                prandtl=case.prandtl, farfield=case.freestream()))
    s.upload(mesh)
    s.init_state(case.conservative(mesh))
    hist, steps, t0 = [], 0, time.perf_counter()
    t = 0.0
    while t < a.t_end:
        s.step(a.every)
        steps += a.every
        q, t = s.get_state()
        rec = {"steps": steps, "t": round(t, 3), "L": wake_length(mesh, q, a.n, a.layers),
               "theta": separation_angle(mesh, q, a.layers), "wall_s": round(time.perf_counter() - t0, 1)}
        hist.append(rec)
        print(json.dumps(rec), flush=True)
    s.close()
    x, u = axis_profile(mesh, q, a.n, a.layers)
    out = {"case": f"sphere Re {case.reynolds} Ma {case.mach}, cubed-sphere O-grid 6*{a.n}*{a.n}*{a.layers} "
                   f"({mesh.n_cells} hexahedra), {a.precision}",
           "t": t, "steps": steps, "L": hist[-1]["L"], "theta_deg": hist[-1]["theta"],
           "paper": PAPER.get((case.reynolds, case.mach)),
           "history": hist, "axis_x": x[:24].round(4).tolist(), "axis_u": u[:24].round(5).tolist()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
