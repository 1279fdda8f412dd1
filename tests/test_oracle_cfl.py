"""Pin of the CFL length scale: h_i = 6 |Omega_i| / sum_p S_ip is the diameter of
the tetrahedron's inscribed sphere.  Checked here from a different
characterisation: the incentre is the vertex average weighted by the areas of the
opposite faces, and its distance to each of the four face planes is the inradius."""
import numpy as np

from oracle import oracle as O
from paper_2407_00656_amd import workloads as W


def test_cfl_length_is_inscribed_sphere_diameter():
    mesh = W.kuhn_box(5, seed=2407)
    v = mesh.cell_vertices                                    # [nc, 4, 3]
    opp = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]
    area = np.stack([0.5 * np.linalg.norm(np.cross(v[:, b] - v[:, a], v[:, c] - v[:, a]), axis=1)
                     for a, b, c in opp], axis=1)             # area of the face opposite vertex p
    inc = np.einsum("cp,cpd->cd", area, v) / area.sum(axis=1)[:, None]
    dist = []
    for a, b, c in opp:
        nrm = np.cross(v[:, b] - v[:, a], v[:, c] - v[:, a])
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        dist.append(np.abs(np.einsum("cd,cd->c", inc - v[:, a], nrm)))
    dist = np.stack(dist, axis=1)
    assert np.allclose(dist, dist[:, :1], rtol=1e-12)         # equidistant: it is the incentre
    _, _, hdt = O.Mesh.from_workload(mesh).cells()
    assert np.allclose(hdt, 2.0 * dist[:, 0], rtol=1e-12)


def test_cfl_dt_of_a_fluid_at_rest():
    """A uniform state at rest: dt = CFL min_i h_i / c with c = sqrt(gamma p / rho)."""
    mesh = W.kuhn_box(4, seed=7)
    om = O.Mesh.from_workload(mesh)
    _, _, hdt = om.cells()
    q = W.uniform_state(mesh.n_cells, rho=1.3, vel=(0.0, 0.0, 0.0), p=0.7)
    c = np.sqrt(1.4 * 0.7 / 1.3)
    for cfl in (0.3, 0.5):
        assert abs(om.cfl_dt(q, O.default_params(cfl=cfl)) - cfl * hdt.min() / c) <= 1e-15
