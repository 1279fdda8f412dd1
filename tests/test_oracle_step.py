"""Whole-step pins of the oracle: free-stream preservation, conservation,
symmetry, relabelling invariance and the design order of accuracy."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_00656_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_free_stream_preserved_on_jittered_mesh():
    m = W.kuhn_box(6, jitter=0.1, seed=11)
    om = O.Mesh.from_workload(m)
    q = W.uniform_state(om.nc, rho=1.3, vel=(0.7, -0.4, 1.1), p=0.9)
    for tau_mode in (0, 1):
        q1, dt = om.step(q, 2, params=O.default_params(tau_mode=tau_mode))
        assert np.abs(q1 - q).max() <= 1e-13 * np.abs(q).max()


def test_exact_conservation():
    m = W.kuhn_box(6, seed=12)
    om = O.Mesh.from_workload(m)
    vol = om.cells()[0]
    case = W.AdvectionCase(amp=0.2, k=(1, 2, 1), vel=(1.0, 0.5, 0.2))
    q = case.conservative(m)
    q1, _ = om.step(q, 3)
    tot0 = (vol[:, None] * q).sum(0)
    tot1 = (vol[:, None] * q1).sum(0)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(q).sum(0).max() * 1e-1 + 1e-13 * np.abs(tot0))


def test_cyclic_axis_permutation_symmetry():
    """Permuting the axes of every node, of the velocity and of the data permutes the
    result; the local tangent choice is free (any orthonormal pair)."""
    m = W.kuhn_box(6, seed=13)
    case = W.AdvectionCase(amp=0.2, k=(1, 2, 1), vel=(1.0, 0.5, 0.2))
    q = case.conservative(m)
    perm = [2, 0, 1]                                  # new axis a takes old axis perm[a]
    om1 = O.Mesh.from_workload(m)
    om2 = O.Mesh(m.nodes[:, perm], m.cell_nodes, m.period[perm])
    qp = q.copy()
    qp[:, 1:4] = q[:, 1:4][:, perm]
    r1, dt1 = om1.step(q, 2)
    r2, dt2 = om2.step(qp, 2)
    assert abs(dt1 - dt2) < 1e-15
    r1p = r1.copy()
    r1p[:, 1:4] = r1[:, 1:4][:, perm]
    assert np.abs(r2 - r1p).max() < 1e-13


def test_relabelling_invariance():
    """Renumbering cells and nodes (keeping each cell's node order) changes nothing."""
    m = W.kuhn_box(6, seed=14)
    case = W.AdvectionCase(amp=0.15, k=(2, 1, 1), vel=(0.3, 1.0, -0.5))
    q = case.conservative(m)
    rng = np.random.default_rng(7)
    cp = rng.permutation(m.n_cells)                     # new cell c holds old cell cp[c]
    npm = rng.permutation(m.n_nodes)                    # old node k becomes npm[k]
    nodes2 = np.empty_like(m.nodes)
    nodes2[npm] = m.nodes
    cells2 = npm[m.cell_nodes[cp]]
    r1, _ = O.Mesh.from_workload(m).step(q, 2)
    r2, _ = O.Mesh(nodes2, cells2, m.period).step(q[cp], 2)
    assert np.abs(r2 - r1[cp]).max() < 1e-13


def test_tau_positive_branch_is_conservative_and_close_to_tau0_in_smooth_flow():
    m = W.kuhn_box(6, seed=15)
    om = O.Mesh.from_workload(m)
    vol = om.cells()[0]
    q = W.AdvectionCase(amp=0.05).conservative(m)
    r0, dt = om.step(q, 2)
    r1, _ = om.step(q, 2, params=O.default_params(tau_mode=1, tau_eps=0.01, tau_C=1.0))
    assert np.all(np.abs((vol[:, None] * (r1 - q)).sum(0)) < 1e-13)
    assert np.abs(r1 - r0).max() < 5e-3 * np.abs(r0 - q).max() + 1e-12


def _paper_table():
    rows = []
    for line in open(os.path.join(GOLDEN, "paper_accuracy_tet.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, l1, o1, l2, o2 = line.split()
        rows.append((int(n), float(l1), float(l2)))
    return rows


def test_paper_table_norms_are_consistently_scaled():
    """The paper's L1/L2 ratio is 2.547-2.551 on every row, which is what a sine-shaped
    error gives when L1 and L2 carry the same volume scaling (both un-normalised or
    both divided by |D|); the mean-normalised pair would give 0.90."""
    for n, l1, l2 in _paper_table():
        assert 2.54 < l1 / l2 < 2.56
    assert abs(8 * (2 / math.pi) / 2 - 2.546) < 1e-3


@pytest.mark.slow
def test_design_order_on_regular_kuhn_meshes():
    """The design order 3 (Sec. 5.1, accuracy table for tetrahedral meshes: 2.92-3.00):
    smooth advection on the six-tetrahedra split of N^3 cubes without jitter, N = 16,
    24, 32, at a common final time T = 0.05 with dt = T / (0.75 N) (CFL about 0.23);
    the L1 density error against the exact cell averages gives orders in [2.85, 3.15]
    for both refinements (measured 2.97 and 2.89).  A dropped term in the reconstruction,
    the flux time expansion or the S2O4 update shows up here as order 2 or lower."""
    case = W.AdvectionCase()
    T = 0.05
    res = []
    for n in (16, 24, 32):
        m = W.kuhn_box(n, jitter=0.0)
        om = O.Mesh.from_workload(m)
        vol = om.cells()[0]
        steps = int(round(0.75 * n))
        qT, _ = om.step(case.conservative(m), steps, T / steps)
        e = W.error_norms(vol, qT[:, 0], case.density_average(m, T))
        res.append((n, e["L1"]))
    orders = [math.log(a[1] / b[1]) / math.log(b[0] / a[0]) for a, b in zip(res, res[1:])]
    assert all(2.85 <= o <= 3.15 for o in orders), orders


@pytest.mark.slow
def test_order_of_accuracy_on_jittered_meshes():
    """The same on the jittered meshes of the workload (nodes moved by up to 10% of h),
    at N = 8, 12, 16 and T = 0.1: the errors fall at better than second order and the
    observed order rises (2.74 then 2.87).  On the jittered N = 16/24/32 meshes at
    T = 0.05 it is 2.84 and 2.72 (2.86 and 2.84 with linear weights): random node
    displacements keep the order below 3 at these resolutions, weights or not."""
    case = W.AdvectionCase()
    T = 0.1
    res = []
    for n in (8, 12, 16):
        m = W.kuhn_box(n)
        om = O.Mesh.from_workload(m)
        vol = om.cells()[0]
        q = case.conservative(m)
        steps = int(1.5 * n)
        qT, _ = om.step(q, steps, T / steps)
        e = W.error_norms(vol, qT[:, 0], case.density_average(m, T))
        assert 2.3 < e["L1"] / e["L2"] < 2.7
        res.append((n, e["L1"]))
    orders = [math.log(a[1] / b[1]) / math.log(b[0] / a[0]) for a, b in zip(res, res[1:])]
    assert orders[0] > 2.6 and orders[1] > 2.75 and orders[1] > orders[0]
