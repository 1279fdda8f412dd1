"""Pins of the oracle's viscous and boundary parts (Sec. 5.2): the collision time
tau = mu(T)/p with mu = mu_inf (T/T_inf)^0.7, the Navier-Stokes stress and heat
flux it produces, the Prandtl-number correction of the heat flux, the far-field
Riemann-invariant state, and the no-slip wall.

Expected values are the Navier-Stokes fluxes of smooth data (the BGK model's
Chapman-Enskog limit, mu = tau p and kappa = c_p mu / Pr), the invariants that
define the characteristic boundary state, and symmetries of the wall's ghost.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_00656_amd import workloads as W

G = 1.4
CP = G / (G - 1.0)          # c_p with T = p / rho (gas constant 1)


def _cons(rho, U, p):
    U = np.asarray(U, dtype=float)
    return np.array([rho, *(rho * U), p / (G - 1) + 0.5 * rho * U @ U])


def _grad_from_prim(rho, U, p, drho, dU, dp):
    """Gradient [5][3] of the conservative variables from primitive gradients
    (each d* is the derivative along x, y, z)."""
    U = np.asarray(U, float)
    drho, dp = np.asarray(drho, float), np.asarray(dp, float)
    dU = np.asarray(dU, float)                     # [3 components][3 directions]
    g = np.zeros((5, 3))
    g[0] = drho
    for a in range(3):
        g[1 + a] = drho * U[a] + rho * dU[a]
    g[4] = dp / (G - 1) + 0.5 * drho * (U @ U) + rho * (U @ dU)
    return g


def _visc(mu_ref=2e-3, T_ref=1 / G, prandtl=1.0, C=0.0):
    return O.default_params(tau_mode=2, mu_ref=mu_ref, T_ref=T_ref, mu_exp=0.7, prandtl=prandtl, tau_C=C)


def test_shear_stress_is_navier_stokes_with_the_power_law_viscosity():
    """Equal smooth states with a shear dV/dx = alpha across a face of normal x: the
    flux of y-momentum is -mu alpha with mu = mu_ref (T/T_ref)^0.7, T = p/rho; the
    normal momentum flux is p, the mass flux 0 (the BGK Navier-Stokes flux, exact for
    equal continuous states)."""
    rho, p, alpha = 0.6, 1.3, 0.8
    T = p / rho
    q = _cons(rho, (0.0, 0.0, 0.0), p)
    g = _grad_from_prim(rho, (0, 0, 0), p, (0, 0, 0), [[0, 0, 0], [alpha, 0, 0], [0, 0, 0]], (0, 0, 0))
    par = _visc()
    F, _ = O.gks_flux(q, g, q, g, (1.0, 0.0, 0.0), 0.01, par)
    mu = 2e-3 * (T * G) ** 0.7
    assert abs(F[2] - (-mu * alpha)) < 1e-12
    assert abs(F[1] - p) < 1e-12 and abs(F[0]) < 1e-14 and abs(F[3]) < 1e-14
    # the same with a different temperature: the viscosity follows T^0.7
    q2 = _cons(rho * 2, (0, 0, 0), p)
    g2 = _grad_from_prim(rho * 2, (0, 0, 0), p, (0, 0, 0), [[0, 0, 0], [alpha, 0, 0], [0, 0, 0]], (0, 0, 0))
    F2, _ = O.gks_flux(q2, g2, q2, g2, (1.0, 0.0, 0.0), 0.01, par)
    assert abs(F2[2] / F[2] - 0.5 ** 0.7) < 1e-10


@pytest.mark.parametrize("prandtl", [1.0, 0.72])
@pytest.mark.parametrize("vel", [(0.0, 0.0, 0.0), (0.0, 0.4, 0.0), (0.3, 0.2, 0.0)])
def test_heat_flux_is_fourier_with_the_prandtl_number(prandtl, vel):
    """At uniform pressure and uniform velocity U with a temperature gradient along the
    normal x (density varying), the Navier-Stokes fluxes are the Euler ones plus the
    heat flux -kappa dT/dx, kappa = c_p mu / Pr (no stress: the velocity is uniform):
    F = (rho U_x, rho U_x U + p e_x, (rho E + p) U_x - kappa dT/dx)."""
    rho, p = 0.9, 1.0
    dTdx = 0.3
    drho = -rho * rho / p * dTdx                   # p uniform: d(p/rho) = -p/rho^2 drho
    U = np.asarray(vel, float)
    q = _cons(rho, U, p)
    g = _grad_from_prim(rho, U, p, (drho, 0, 0), np.zeros((3, 3)), (0, 0, 0))
    par = _visc(prandtl=prandtl)
    F, _ = O.gks_flux(q, g, q, g, (1.0, 0.0, 0.0), 0.01, par)
    mu = 2e-3 * ((p / rho) * G) ** 0.7
    assert abs(F[4] - ((q[4] + p) * U[0] - CP * mu / prandtl * dTdx)) < 1e-12
    assert abs(F[0] - rho * U[0]) < 1e-14
    assert np.allclose(F[1:4], rho * U[0] * U + p * np.array([1.0, 0, 0]), rtol=0, atol=1e-13)


def test_prandtl_correction_acts_only_in_the_viscous_mode():
    rho, p = 0.9, 1.0
    q = _cons(rho, (0.2, 0.1, 0.0), p)
    g = _grad_from_prim(rho, (0.2, 0.1, 0), p, (-0.2, 0.1, 0), np.full((3, 3), 0.05), (0.1, 0, 0))
    qr = _cons(1.1, (0.1, 0.0, 0.1), 1.2)
    a = O.gks_flux(q, g, qr, g, (0.6, 0.8, 0.0), 0.01, O.default_params(tau_mode=1, prandtl=0.72))
    b = O.gks_flux(q, g, qr, g, (0.6, 0.8, 0.0), 0.01, O.default_params(tau_mode=1, prandtl=1.0))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = O.gks_flux(q, g, qr, g, (0.6, 0.8, 0.0), 0.01, _visc(prandtl=0.72))
    d = O.gks_flux(q, g, qr, g, (0.6, 0.8, 0.0), 0.01, _visc(prandtl=1.0))
    assert np.array_equal(c[0][:4], d[0][:4]) and c[0][4] != d[0][4]


def test_viscous_tau_adds_the_pressure_jump_term():
    """tau = mu/p0 + C |pl - pr|/(pl + pr) dt: with mu_ref = 0 the viscous mode is the
    shock mode without its eps*dt part."""
    ql = _cons(1.0, (0.1, 0, 0), 1.0)
    qr = _cons(0.5, (0.0, 0, 0), 0.4)
    g = np.zeros((5, 3))
    a = O.gks_flux(ql, g, qr, g, (1.0, 0, 0), 0.01, O.default_params(tau_mode=2, mu_ref=0.0, tau_C=1.0))
    b = O.gks_flux(ql, g, qr, g, (1.0, 0, 0), 0.01, O.default_params(tau_mode=1, tau_eps=0.0, tau_C=1.0))
    assert np.allclose(a[0], b[0], rtol=1e-14, atol=1e-15) and np.allclose(a[1], b[1], rtol=1e-13, atol=1e-14)


def _farfield_params():
    return O.default_params(farfield=(1.0, 0.2535, 0.0, 0.0, 1 / G))


def test_farfield_state_keeps_the_free_stream():
    p = _farfield_params()
    qf = _cons(1.0, (0.2535, 0, 0), 1 / G)
    for n in ([1, 0, 0], [-1, 0, 0], [0.6, 0.8, 0], [0, 0, -1]):
        assert np.allclose(O.ghost_state(O.BC_FAR, qf, n, p), qf, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("vn", [0.3, -0.3])
def test_farfield_state_by_its_invariants(vn):
    """Subsonic boundary: the outgoing invariant U.n + 2c/(g-1) is the interior's, the
    incoming U.n - 2c/(g-1) the free stream's; entropy p/rho^g and tangential velocity
    come from the interior at an outflow (U.n > 0 on the boundary) and from the free
    stream at an inflow."""
    p = _farfield_params()
    n = np.array([0.6, 0.8, 0.0])
    t = np.array([-0.8, 0.6, 0.0])
    rho_i, p_i = 1.1, 0.8
    Ui = vn * n + 0.15 * t + np.array([0, 0, 0.05])
    q = _cons(rho_i, Ui, p_i)
    b = O.ghost_state(O.BC_FAR, q, n, p)
    rb = b[0]
    Ub = b[1:4] / rb
    pb = (G - 1) * (b[4] - 0.5 * rb * Ub @ Ub)
    cb, ci = math.sqrt(G * pb / rb), math.sqrt(G * p_i / rho_i)
    Uf = np.array([0.2535, 0, 0])
    cf = math.sqrt(G * (1 / G) / 1.0)
    assert abs((Ub @ n + 2 * cb / (G - 1)) - (Ui @ n + 2 * ci / (G - 1))) < 1e-13
    assert abs((Ub @ n - 2 * cb / (G - 1)) - (Uf @ n - 2 * cf / (G - 1))) < 1e-13
    out = Ub @ n > 0
    src_U, src_s = (Ui, p_i / rho_i ** G) if out else (Uf, (1 / G) / 1.0)
    assert np.allclose(Ub - (Ub @ n) * n, src_U - (src_U @ n) * n, atol=1e-14)
    assert abs(pb / rb ** G - src_s) < 1e-13


def test_farfield_state_supersonic():
    p = _farfield_params()
    n = np.array([1.0, 0, 0])
    q = _cons(1.0, (3.0, 0.1, 0), 1.0)            # supersonic outflow: the interior
    assert np.allclose(O.ghost_state(O.BC_FAR, q, n, p), q, rtol=1e-15)
    q = _cons(1.0, (-3.0, 0.1, 0), 1.0)           # supersonic inflow: the free stream
    assert np.allclose(O.ghost_state(O.BC_FAR, q, n, p), _cons(1.0, (0.2535, 0, 0), 1 / G), rtol=1e-15)


def test_wall_ghost_and_wall_flux():
    """The wall ghost holds (rho, -rho U, rho E): zero velocity and the cell's
    temperature on the face.  The collision of a state with its ghost has zero
    velocity, so with no gradients the tau = 0 wall flux is (0, p n, 0) for any
    velocity of the state (pressure of the collided state on the face)."""
    q = _cons(0.9, (0.3, -0.2, 0.4), 1.1)
    gq = O.ghost_state(O.BC_WALL, q, (1, 0, 0))
    assert np.array_equal(gq, [q[0], -q[1], -q[2], -q[3], q[4]])
    n = np.array([0.6, 0.0, 0.8])
    g = np.zeros((5, 3))
    F, _ = O.gks_flux(q, g, gq, g, n, 0.01, O.default_params())
    q0 = O.collision(q, gq)                        # in the frame (n, t1, t2) the velocity is 0 anyway
    assert abs(q0[1]) < 1e-15
    assert abs(F[0]) < 1e-15 and abs(F[4]) < 1e-15
    assert np.allclose(F[1:4], (F[1:4] @ n) * n, rtol=0, atol=1e-14)   # momentum flux along n only


def test_sphere_wall_and_far_field_in_a_step():
    """A few viscous steps of the free stream on a small O-grid: finite, positive; the
    wall faces carry no mass (the collided state at a wall point has zero normal
    velocity only for gradient-free data, so the mass through the wall is small, not
    zero) and the free stream far from the sphere is unchanged after one step."""
    mesh = W.cubed_sphere(3, 6)
    sc = W.SphereCase()
    m = O.Mesh.from_workload(mesh)
    p = O.default_params(tau_mode=2, mu_ref=sc.mu_inf(), T_ref=sc.t_inf(), prandtl=sc.prandtl,
                         farfield=sc.freestream())
    q0 = sc.conservative(mesh)
    q1, dt = m.step(q0, 1, params=p)
    assert np.all(np.isfinite(q1)) and dt > 0
    r = np.linalg.norm(m.cells()[1], axis=1)
    far = r > 10.0
    assert np.abs(q1[far] - q0[far]).max() < 1e-3
