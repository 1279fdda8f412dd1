"""The wake-length and separation-angle measures of the sphere run, on synthetic
fields with a known answer (host only)."""
import numpy as np

from paper_2407_00656_amd import sphere_run as S
from paper_2407_00656_amd import workloads as W


def test_wake_length_of_a_linear_axial_profile():
    """u_x = x - (0.5 + L): the axial profile crosses zero at x = 0.5 + L exactly
    (the measure interpolates linearly between layers)."""
    n, layers, L = 8, 12, 0.83
    mesh = W.cubed_sphere(n, layers)
    c = mesh.cell_vertices.mean(axis=1)
    q = np.zeros((mesh.n_cells, 5))
    q[:, 0] = 2.0
    q[:, 1] = 2.0 * (c[:, 0] - (0.5 + L))
    q[:, 4] = 3.0
    assert abs(S.wake_length(mesh, q, n, layers) - L) < 1e-12
    q[:, 1] = 2.0 * (c[:, 0] + 1.0)                  # no reverse flow on the axis
    assert np.isnan(S.wake_length(mesh, q, n, layers))


def test_separation_angle_of_a_linear_meridional_profile():
    """u = (theta_s - theta) e_theta next to the wall: the meridional velocity changes
    sign at theta_s; binning and interpolation recover it to rounding."""
    n, layers, ths = 12, 6, 127.3
    mesh = W.cubed_sphere(n, layers)
    c = mesh.cell_vertices.mean(axis=1)
    r = np.linalg.norm(c, axis=1)
    ryz = np.hypot(c[:, 1], c[:, 2])
    th = np.degrees(np.arccos(-c[:, 0] / r))
    e = np.stack([ryz / r, (-c[:, 0] / r) * c[:, 1] / ryz, (-c[:, 0] / r) * c[:, 2] / ryz], axis=1)
    q = np.zeros((mesh.n_cells, 5))
    q[:, 0] = 1.5
    q[:, 1:4] = 1.5 * (ths - th)[:, None] * e
    q[:, 4] = 3.0
    assert abs(S.separation_angle(mesh, q, layers) - ths) < 1e-9
    q[:, 1:4] = 1.5 * np.abs(ths - th)[:, None] * e   # attached everywhere
    assert np.isnan(S.separation_angle(mesh, q, layers))
