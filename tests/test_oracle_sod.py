"""Pins of the oracle on Sod's shock tube (the shock-tube workload, tau_mode = 1).

The reference is the exact solution of the Riemann problem, computed here from
the textbook construction (pressure function and its Newton iteration, then the
wave pattern sampled along x/t; Toro, "Riemann Solvers and Numerical Methods
for Fluid Dynamics", ch. 4).  The solver itself is pinned against the star
state that book tabulates for this data (p* = 0.30313, u* = 0.92745).  The
oracle runs the periodic doubled tube, whose two halves equal the tube with
transmissive ends until t = 0.286; at t = 0.2:

  * L1 density error against the exact solution is small and halves with h
    (first order is what any shock-capturing scheme reaches);
  * the shock, the contact and the rarefaction tail sit where the exact
    solution puts them;
  * mass, momentum and energy are conserved to round-off (periodic box);
  * the solution stays physical (the Gauss-point positivity fallback acts).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_00656_amd import workloads as W

GAMMA = 1.4
T_END = 0.2


def _pressure_fn(p, rk, pk, ck):
    """Toro's f_K(p) and its derivative for one side K."""
    g = GAMMA
    if p > pk:                               # shock
        a = 2.0 / ((g + 1.0) * rk)
        b = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(a / (p + b))
        df = math.sqrt(a / (b + p)) * (1.0 - (p - pk) / (2.0 * (b + p)))
    else:                                    # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rk * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr):
    cl, cr = math.sqrt(GAMMA * pl / rl), math.sqrt(GAMMA * pr / rr)
    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = _pressure_fn(p, rl, pl, cl)
        f2, d2 = _pressure_fn(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(1e-14, p - dp)
        if abs(dp) < 1e-15 * p:
            break
    f1, _ = _pressure_fn(p, rl, pl, cl)
    f2, _ = _pressure_fn(p, rr, pr, cr)
    return p, 0.5 * (ul + ur) + 0.5 * (f2 - f1)


def sod_exact(xi):
    """(rho, u, p) of Sod's data (1, 0, 1 | 0.125, 0, 0.1) at xi = (x - x_d)/t.
    Left state: rarefaction; right state: shock (the only pattern this data has)."""
    g = GAMMA
    rl, ul, pl, rr, ur, pr = 1.0, 0.0, 1.0, 0.125, 0.0, 0.1
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(rl, ul, pl, rr, ur, pr)
    rho_sl = rl * (ps / pl) ** (1.0 / g)                                   # behind the rarefaction
    rho_sr = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1.0))
    head, tail = ul - cl, us - cl * (ps / pl) ** ((g - 1) / (2 * g))
    shock = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
    out = np.empty((len(xi), 3))
    for k, s in enumerate(xi):
        if s < head:
            out[k] = (rl, ul, pl)
        elif s < tail:
            u = 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * ul + s)
            c = 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * (ul - s))
            out[k] = (rl * (c / cl) ** (2 / (g - 1)), u, pl * (c / cl) ** (2 * g / (g - 1)))
        elif s < us:
            out[k] = (rho_sl, us, ps)
        elif s < shock:
            out[k] = (rho_sr, us, ps)
        else:
            out[k] = (rr, ur, pr)
    return out, {"head": head, "tail": tail, "contact": us, "shock": shock}


def test_star_state_matches_the_tabulated_values():
    p, u = star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    assert abs(p - 0.30313) < 5e-6 and abs(u - 0.92745) < 5e-6
    # a symmetric collision has u* = 0 and a shock on both sides
    p2, u2 = star_state(1.0, 1.0, 1.0, 1.0, -1.0, 1.0)
    assert abs(u2) < 1e-14 and p2 > 1.0


def _run(nx):
    mesh, case = W.sod_box(nx, 4, 4)
    q = case.conservative(mesh)
    om = O.Mesh.from_workload(mesh)
    prm = O.default_params(tau_mode=1)
    vol = W.tet_volumes(mesh.cell_vertices)
    tot0 = (q * vol[:, None]).sum(axis=0)
    t = 0.0
    while t < T_END - 1e-14:
        dt = min(om.cfl_dt(q, prm), T_END - t)
        q, _ = om.step(q, 1, dt_fixed=dt, params=prm)
        t += dt
    x = mesh.cell_vertices[:, :, 0].mean(axis=1)
    # right half: the standard tube with its diaphragm at 1.5; left half: its mirror about x = 1
    xi = np.where(x >= 1.0, (x - 1.5) / T_END, (0.5 - x) / T_END)
    ex, waves = sod_exact(xi)
    return mesh, q, vol, tot0, x, ex, waves


@pytest.fixture(scope="module")
def runs():
    return {nx: _run(nx) for nx in (32, 64)}


def test_sod_l1_error_is_small_and_first_order(runs):
    err = {}
    for nx, (mesh, q, vol, _, _, ex, _) in runs.items():
        err[nx] = float(np.sum(np.abs(q[:, 0] - ex[:, 0]) * vol) / np.sum(vol))
    assert err[32] < 0.025 and err[64] < 0.013, err
    assert err[32] / err[64] > 1.6, err


def test_sod_waves_are_where_the_exact_solution_puts_them(runs):
    mesh, q, vol, _, x, ex, waves = runs[64]
    h = 2.0 / 64
    right = x >= 1.0
    xr, rho = x[right], q[right, 0]
    order = np.argsort(xr)
    xr, rho = xr[order], rho[order]
    # shock: the last cell above the mid density of the shock jump
    rho_sr = ex[:, 0][(ex[:, 0] > 0.2) & (ex[:, 0] < 0.3)].max()
    x_shock = 1.5 + waves["shock"] * T_END
    x_num = xr[rho > 0.5 * (rho_sr + 0.125)].max()
    assert abs(x_num - x_shock) < 2.5 * h, (x_num, x_shock)
    # rarefaction head: the first cell measurably below the left state
    x_head = 1.5 + waves["head"] * T_END
    x_num = xr[rho < 0.98].min()
    assert abs(x_num - x_head) < 2.5 * h, (x_num, x_head)


def test_sod_conserves_and_stays_physical(runs):
    for nx, (mesh, q, vol, tot0, _, _, _) in runs.items():
        tot = (q * vol[:, None]).sum(axis=0)
        assert np.all(np.abs(tot - tot0) <= 1e-13 * np.maximum(1.0, np.abs(tot0))), (nx, tot - tot0)
        rho = q[:, 0]
        p = (GAMMA - 1.0) * (q[:, 4] - 0.5 * (q[:, 1:4] ** 2).sum(axis=1) / rho)
        assert rho.min() > 0.1 and p.min() > 0.05 and rho.max() < 1.05 and p.max() < 1.05


def test_workload_exact_solution_matches():
    """The vectorised exact solution the shock-tube driver reports against equals
    the construction above on both halves of the periodic tube."""
    case = W.SodCase()
    x = np.linspace(0.0, 2.0, 2001)[:-1] + 1e-4
    got = case.exact(x, T_END)
    xi = np.where(x >= 1.0, (x - 1.5) / T_END, (0.5 - x) / T_END)
    ref, _ = sod_exact(xi)
    ref[:, 1] *= np.where(x >= 1.0, 1.0, -1.0)
    assert np.abs(got - ref).max() < 1e-13
