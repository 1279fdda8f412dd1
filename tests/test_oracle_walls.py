"""Pins of the oracle's transmissive walls (non-periodic axes).

The ghost across a wall face is the mirror image of the wall cell holding the wall
cell's state, and a ghost's neighbours are the mirror images of the wall cell's
neighbours.  So on a wall box the oracle must give the same right-hand side as on
the box doubled by its mirror image (a periodic mesh on which the "ghosts" are real
cells, handled by the interior code path and pinned elsewhere) with the state
copied into the mirror cells.  Beyond that:

  * a uniform moving state is preserved exactly, also with walls on two axes
    (edges, where members are images under two mirrors);
  * in Sod's tube with walls, while the wall cells still hold the initial states the
    only fluxes through the walls are the pressures there: mass and energy stay
    constant and the total x-momentum grows as (p_L - p_R) A t;
  * the density error against the exact Riemann solution is small and first order.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_00656_amd import workloads as W

from helpers import mirror_double, smooth_state

GAMMA = 1.4


@pytest.mark.parametrize("tau_mode,axes", [(0, (0,)), (1, (0,)), (0, (0, 1))])
def test_walls_equal_the_mirror_doubled_box(tau_mode, axes):
    periodic = tuple(a not in axes for a in range(3))
    mesh = W.kuhn_box((5, 4, 4), (1.0, 0.8, 0.8), jitter=0.15, seed=4242, periodic=periodic)
    q = smooth_state(mesh, 7)
    doubled, qd = mesh, q
    for a in axes:
        doubled = mirror_double(doubled, a)
        qd = np.concatenate([qd, qd])
    prm = O.default_params(tau_mode=tau_mode)
    dt = 2e-3
    L, dL = O.Mesh.from_workload(mesh).rhs(q, dt, prm)
    Ld, dLd = O.Mesh.from_workload(doubled).rhs(qd, dt, prm)
    nc = mesh.n_cells
    for a, b in ((L, Ld[:nc]), (dL, dLd[:nc])):
        scale = np.abs(b).max(axis=0)
        assert np.all(np.abs(a - b).max(axis=0) <= 1e-11 * scale), (np.abs(a - b).max(axis=0), scale)
    # the mirror cells of the doubled box see the same values (the symmetry is exact)
    assert np.abs(L).max() > 1e-3


def test_walls_preserve_a_uniform_moving_state():
    mesh = W.kuhn_box((4, 5, 4), (1.0, 1.0, 0.8), jitter=0.15, seed=99, periodic=(False, False, True))
    q0 = np.tile([1.1, 0.66, -0.33, 0.22, 3.1], (mesh.n_cells, 1))
    om = O.Mesh.from_workload(mesh)
    q, _ = om.step(q0, 3, params=O.default_params(tau_mode=1))
    assert np.abs(q - q0).max() <= 1e-13 * np.abs(q0).max()


def _sod(nx, t_end):
    mesh, case = W.sod_box(nx, 4, 4, walls=True)
    q = case.conservative(mesh)
    om = O.Mesh.from_workload(mesh)
    prm = O.default_params(tau_mode=1)
    vol = W.tet_volumes(mesh.cell_vertices)
    t, tot0, hist = 0.0, (q * vol[:, None]).sum(axis=0), []
    while t < t_end - 1e-14:
        dt = min(om.cfl_dt(q, prm), t_end - t)
        q, _ = om.step(q, 1, dt_fixed=dt, params=prm)
        t += dt
        hist.append((t, (q * vol[:, None]).sum(axis=0)))
    return mesh, case, q, vol, tot0, hist


@pytest.fixture(scope="module")
def sod_runs():
    return {nx: _sod(nx, 0.2) for nx in (16, 32)}


def test_wall_fluxes_are_the_wall_pressures(sod_runs):
    mesh, case, q, vol, tot0, hist = sod_runs[32]
    area = 4.0 / 32 * 4.0 / 32                       # the y-z cross-section of the tube
    for t, tot in hist:
        # The scheme's domain of dependence grows by a few cells per step, so tails of
        # the waves (1e-7 in density by t = 0.15) reach the walls long before the
        # waves; until about t = 0.1 the wall cells hold the initial states to rounding.
        if t > 0.08:
            break
        assert abs(tot[0] - tot0[0]) <= 1e-13 * tot0[0]
        assert abs(tot[4] - tot0[4]) <= 1e-13 * tot0[4]
        assert abs(tot[1] - (case.p_l - case.p_r) * area * t) <= 1e-12 * (case.p_l * area * t)
        assert abs(tot[2]) <= 1e-15 and abs(tot[3]) <= 1e-15


def test_sod_with_walls_against_the_exact_solution(sod_runs):
    err = {}
    for nx, (mesh, case, q, vol, _, _) in sod_runs.items():
        x = mesh.cell_vertices[:, :, 0].mean(axis=1)
        ex = case.exact(x, 0.2)
        err[nx] = float(np.sum(np.abs(q[:, 0] - ex[:, 0]) * vol) / np.sum(vol))
        p = (GAMMA - 1.0) * (q[:, 4] - 0.5 * (q[:, 1:4] ** 2).sum(axis=1) / q[:, 0])
        assert q[:, 0].min() > 0.1 and p.min() > 0.05
    assert err[16] < 0.025 and err[32] < 0.013, err
    assert err[16] / err[32] > 1.6, err
