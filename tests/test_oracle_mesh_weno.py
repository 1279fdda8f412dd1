"""Pins of the oracle's mesh layer (connectivity, geometry, stencils) and of its
WENO reconstruction (Sec. 2.3) against exact polynomial data."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_00656_amd import workloads as W


@pytest.fixture(scope="module")
def box8():
    m = W.kuhn_box(8)
    return m, O.Mesh.from_workload(m)


def test_faces_and_volumes(box8):
    m, om = box8
    assert om.nf == 2 * om.nc
    vol, cen, hdt = om.cells()
    assert np.allclose(vol, W.tet_volumes(m.cell_vertices), rtol=1e-14)
    assert abs(vol.sum() - 8.0) < 1e-12
    assert np.allclose(cen, m.cell_vertices.mean(axis=1), atol=1e-15)


def test_per_cell_closure(box8):
    """sum over a cell's faces of the outward n*S vanishes (divergence theorem)."""
    m, om = box8
    f = om.faces()
    s = np.zeros((om.nc, 3))
    nS = f["normal"] * f["area"][:, None]
    np.add.at(s, f["lr"][:, 0], nS)
    np.add.at(s, f["lr"][:, 1], -nS)
    assert np.abs(s).max() < 1e-15 * 100


def test_normals_point_left_to_right_and_shifts_are_periods(box8):
    m, om = box8
    vol, cen, _ = om.cells()
    f = om.faces()
    l, r = f["lr"][:, 0], f["lr"][:, 1]
    d = cen[r] + f["shift"] - cen[l]
    assert np.all(np.einsum("fa,fa->f", d, f["normal"]) > 0)
    assert np.allclose(f["shift"] / 2.0, np.rint(f["shift"] / 2.0), atol=1e-14)


def test_face_gauss_rule_exact_for_quadratics(box8):
    """3-point rule on each face vs the exact triangle moment
    int_T x_a x_b = S/12 (sum_v v_a v_b + (sum_v v_a)(sum_v v_b))."""
    m, om = box8
    f = om.faces()
    nodes = f["gauss"]  # [nf, 3, 3]
    # recover the triangle vertices from the rule: V = 2 G_v - (sum G)/... ; use the inverse
    # of the barycentric map (2/3, 1/6, 1/6): G = (1/2) V_v + (1/6) sum V
    G = nodes
    sumV = G.sum(axis=1) * 1.0           # sum G = (1/2 + 3/6) sum V = sum V
    V = 2.0 * (G - sumV[:, None, :] / 6.0)
    area = 0.5 * np.linalg.norm(np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]), axis=1)
    assert np.allclose(area, f["area"], rtol=1e-13)
    for a in range(3):
        for b in range(3):
            rule = f["area"] * np.mean(G[:, :, a] * G[:, :, b], axis=1)
            exact = f["area"] / 12.0 * (np.einsum("fv,fv->f", V[:, :, a], V[:, :, b])
                                        + V[:, :, a].sum(1) * V[:, :, b].sum(1))
            assert np.allclose(rule, exact, rtol=1e-12, atol=1e-15)


def test_stencil_sizes_on_kuhn_mesh(box8):
    """Two-layer stencil of 14 cells besides the cell itself; four 6-cell sub-stencils."""
    m, om = box8
    nb = om.neighbors()
    for i in range(0, om.nc, 37):
        mem, sh, subs = om.stencil(i)
        assert len(mem) == 14
        assert list(mem[:4]) == list(nb[i])
        assert all(len(s) == 6 for s in subs)
        # sub-stencil m holds three first-layer cells and the three other neighbours of i_m
        excl = [3, 2, 0, 1]
        for s in range(4):
            first = [nb[i][p] for p in range(4) if p != excl[s]]
            assert sorted(subs[s][:3]) == sorted(first)
            others = sorted(c for c in nb[nb[i][s]] if c != i)
            assert sorted(subs[s][3:]) == others


def test_monomial_means_match_high_order_quadrature(box8):
    m, om = box8
    vol, cen, _ = om.cells()
    ref, w = W.tet_rule(3)
    exps = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    for i in (0, 17, 1001):
        c, h = cen[i] + np.array([0.1, -0.05, 0.02]), 0.3
        got = om.monomial_means(i, c, h)
        v = m.cell_vertices[i]
        pts = v[0] + ref @ (v[1:] - v[0])
        xi = (pts - c) / h
        for d, e in enumerate(exps):
            ex = 6.0 * np.sum(w * xi[:, 0] ** e[0] * xi[:, 1] ** e[1] * xi[:, 2] ** e[2])
            assert abs(got[d] - ex) < 1e-13


def _interior_cells(n, margin=3):
    out = []
    for i in range(margin, n - margin):
        for j in range(margin, n - margin):
            for k in range(margin, n - margin):
                base = 6 * ((i * n + j) * n + k)
                out.extend(range(base, base + 6))
    return out


def test_weno_constant_field():
    m = W.kuhn_box(8)
    om = O.Mesh.from_workload(m)
    q = W.uniform_state(om.nc)
    for i in (0, 100, 2000):
        w = om.weno_cell(q, i)
        assert np.all(w["beta"] == 0.0)
        assert np.allclose(w["wbar"], [0.9, 0.025, 0.025, 0.025, 0.025], rtol=1e-15)
        val, grad = om.reconstruct(q, i, om.cells()[1][i] + 0.01)
        assert np.allclose(val, q[i], rtol=1e-15) and np.all(np.abs(grad) < 1e-15)


def test_weno_linear_field_is_exact():
    """Cell averages of a linear field: every polynomial is exact, beta_0 = beta_m,
    so the non-linear weights equal the linear ones (Sec. 2.3)."""
    n = 8
    m = W.kuhn_box(n)
    om = O.Mesh.from_workload(m)
    vol, cen, _ = om.cells()
    g = np.array([[0.3, -0.2, 0.5], [1.0, 0.1, 0.0], [0.0, 0.7, -0.4], [0.2, 0.2, 0.2], [-1.0, 0.5, 2.0]])
    c0 = np.array([1.0, 0.5, -0.3, 0.2, 3.0])
    q = c0[None, :] + cen @ g.T           # average of a linear function = value at centroid
    rng = np.random.default_rng(0)
    for i in _interior_cells(n)[::29]:
        w = om.weno_cell(q, i)
        assert np.allclose(w["wbar"], np.array([0.9, 0.025, 0.025, 0.025, 0.025])[None, :], rtol=1e-9)
        x = cen[i] + rng.normal(size=3) * 0.05
        val, grad = om.reconstruct(q, i, x)
        assert np.allclose(val, c0 + g @ x, rtol=1e-12, atol=1e-12)
        assert np.allclose(grad, g, rtol=1e-11, atol=1e-11)


def test_weno_quadratic_field_P0_exact():
    """Cell averages of a quadratic: P0 (the big-stencil quadratic) is exact."""
    n = 8
    m = W.kuhn_box(n)
    om = O.Mesh.from_workload(m)
    vol, cen, _ = om.cells()
    H = np.array([[0.5, 0.1, -0.2], [0.1, -0.3, 0.4], [-0.2, 0.4, 0.2]])
    gvec = np.array([0.3, -0.1, 0.2])
    f = lambda x, y, z: 1.0 + gvec[0] * x + gvec[1] * y + gvec[2] * z + (
        H[0, 0] * x * x + H[1, 1] * y * y + H[2, 2] * z * z + 2 * H[0, 1] * x * y + 2 * H[0, 2] * x * z + 2 * H[1, 2] * y * z)
    avg = W.cell_average(m.cell_vertices, f, 3)
    q = W.uniform_state(om.nc)
    q[:, 0] = avg
    # linear weights (huge epsilon) make the WENO combination equal P0 exactly
    p = O.default_params(weno_eps=1e30)
    rng = np.random.default_rng(1)
    for i in _interior_cells(n)[::31]:
        x = cen[i] + rng.normal(size=3) * 0.05
        val, grad = om.reconstruct(q, i, x, p)
        exact_val = f(*x)
        exact_grad = gvec + 2 * H @ x
        assert abs(val[0] - exact_val) < 1e-12
        assert np.allclose(grad[0], exact_grad, atol=1e-11)


def test_smoothness_indicators_match_their_definition():
    """beta_m = sum_{1<=|l|<=r_m} |Omega|^(2|l|/3-1) int_Omega (d^l P_m)^2 dV, computed here
    by high-order quadrature of the exact polynomial (P0 and P_m are exact for
    quadratic / linear data; mixed second derivatives counted once)."""
    n = 8
    m = W.kuhn_box(n)
    om = O.Mesh.from_workload(m)
    vol, cen, _ = om.cells()
    H = np.array([[0.5, 0.1, -0.2], [0.1, -0.3, 0.4], [-0.2, 0.4, 0.2]])
    gvec = np.array([0.3, -0.1, 0.2])
    f = lambda x, y, z: 1.0 + gvec[0] * x + gvec[1] * y + gvec[2] * z + (
        H[0, 0] * x * x + H[1, 1] * y * y + H[2, 2] * z * z + 2 * H[0, 1] * x * y + 2 * H[0, 2] * x * z + 2 * H[1, 2] * y * z)
    q = W.uniform_state(om.nc)
    q[:, 0] = W.cell_average(m.cell_vertices, f, 3)
    ref, w = W.tet_rule(3)
    for i in _interior_cells(n)[::53]:
        v = m.cell_vertices[i]
        pts = v[0] + ref @ (v[1:] - v[0])
        V = vol[i]
        grad = gvec[None, :] + 2 * pts @ H                       # exact gradient at the points
        b1 = V ** (-1 / 3) * sum(6 * V * np.sum(w * grad[:, j] ** 2) for j in range(3))
        second = [2 * H[0, 0], 2 * H[1, 1], 2 * H[2, 2], 2 * H[0, 1], 2 * H[0, 2], 2 * H[1, 2]]
        b2 = V ** (1 / 3) * V * sum(s * s for s in second)
        wc = om.weno_cell(q, i)
        assert abs(wc["beta"][0, 0] - (b1 + b2)) < 1e-10 * (b1 + b2)


def test_weights_shift_away_from_a_discontinuity():
    """Step data through the big stencil while one sub-stencil stays on one side:
    that sub-stencil (beta = 0) takes almost all the weight and the quadratic's
    weight collapses (WENO-Z weights, Sec. 2.3)."""
    n = 8
    m = W.kuhn_box(n, jitter=0.0)
    om = O.Mesh.from_workload(m)
    vol, cen, _ = om.cells()
    q = W.uniform_state(om.nc)
    q[:, 0] = np.where(cen[:, 0] < 1.0, 1.0, 0.2)
    q[:, 4] = 2.5
    seen = 0
    for i in _interior_cells(n, 2):
        if abs(cen[i, 0] - 1.0) > 0.3:
            continue
        wc = om.weno_cell(q, i)
        wb, beta = wc["wbar"][0], wc["beta"][0]
        if beta[0] > 1e-3 and beta[1:].min() == 0.0:
            seen += 1
            assert wb[0] < 1e-3
            assert wb[1 + np.argmin(beta[1:])] == wb[1:].max()
            assert abs(wb.sum() - 1.0) < 1e-14
    assert seen > 0
