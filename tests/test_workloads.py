"""Seeded input generators: RNG vectors, Kuhn mesh, tetrahedral quadrature."""
import math
import os

import numpy as np

from paper_2407_00656_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vectors():
    for line in open(os.path.join(GOLDEN, "splitmix64.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, *outs = line.split()
        got = W.splitmix64(int(seed), len(outs))
        assert [int(x) for x in got] == [int(o, 16) for o in outs]


def test_uniform01_range_and_counter_form():
    u = W.uniform01(7, 1000)
    assert u.min() >= 0.0 and u.max() < 1.0
    # counter form: draws 500..999 do not depend on the earlier ones
    assert np.array_equal(W.uniform01(7, 500, start=500), u[500:])


def test_kuhn_box_counts_and_volume():
    for n in (4, 8):
        m = W.kuhn_box(n)
        assert m.n_cells == 6 * n ** 3
        assert m.n_nodes == n ** 3
        vol = W.tet_volumes(m.cell_vertices)
        assert abs(vol.sum() - 8.0) < 1e-12
        assert vol.min() > 0


def test_kuhn_box_boundary_nodes_not_jittered():
    n = 6
    m = W.kuhn_box(n, jitter=0.1, seed=3)
    h = 2.0 / n
    idx = np.rint(m.nodes / h).astype(int)
    lattice = idx * h
    on_bnd = np.any(idx % n == 0, axis=1)
    assert np.all(m.nodes[on_bnd] == lattice[on_bnd])
    d = np.abs(m.nodes[~on_bnd] - lattice[~on_bnd])
    assert d.max() <= 0.1 * h and d.max() > 0.05 * h


def test_kuhn_cells_follow_lattice_paths():
    # Tet sigma of cube (0,0,0): v0=(0,0,0), then unit steps along the permutation's axes.
    m = W.kuhn_box(4, jitter=0.0)
    h = 0.5
    for s, perm in enumerate(W.KUHN_PERMS):
        v = m.cell_vertices[s] / h
        assert np.allclose(v[0], 0)
        for k in range(3):
            step = v[k + 1] - v[k]
            e = np.zeros(3)
            e[perm[k]] = 1
            assert np.allclose(step, e)


def test_tet_rule_exactness():
    # Mean of x^a y^b z^c over the reference tetrahedron = 6 a! b! c! / (a+b+c+3)!
    for npts in (2, 3, 5):
        ref, w = W.tet_rule(npts)
        deg = 2 * npts - 1
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                c = deg - a - b
                exact = 6.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                got = 6.0 * np.sum(w * ref[:, 0] ** a * ref[:, 1] ** b * ref[:, 2] ** c)
                assert abs(got - exact) < 1e-14 * max(1.0, exact) * 10


def test_cell_average_converges():
    m = W.kuhn_box(4)
    case = W.AdvectionCase()
    f = case.density_fn(0.0)
    a = W.cell_average(m.cell_vertices, f, 9)
    b = W.cell_average(m.cell_vertices, f, 11)
    assert np.abs(a - b).max() < 1e-12


def test_serve_requests_seeded():
    r1 = W.serve_requests(16, seed=5)
    r2 = W.serve_requests(16, seed=5)
    assert [(r.n, r.precision, r.arrival) for r in r1] == [(r.n, r.precision, r.arrival) for r in r2]
    assert all(8 <= r.n <= 48 for r in r1)
    assert all(r1[i].arrival < r1[i + 1].arrival for i in range(15))
