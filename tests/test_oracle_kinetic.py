"""Pins of the oracle's kinetic layer: Maxwellian moments, micro-slopes,
collision, the Gauss-point GKS flux, and the S2O4 combination.

Every expected value here comes from mathematics independent of the oracle's
code path: closed forms, numerical quadrature, the Euler equations, or the
Taylor polynomial.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si

from oracle import oracle as O

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)


def test_full_moments_match_gaussian_central_moments():
    # <u^n> = sum_k C(n,k) U^(n-k) <(u-U)^k>, <(u-U)^(2j)> = (2j-1)!! / (2 lam)^j
    for U, lam in [(0.3, 0.8), (-1.7, 2.5), (0.0, 1.0)]:
        full, _, _ = O.moments_1d(U, lam)
        for n in range(7):
            s = 0.0
            for k in range(0, n + 1, 2):
                dfact = 1.0
                for t in range(k - 1, 0, -2):
                    dfact *= t
                s += math.comb(n, k) * U ** (n - k) * dfact / (2 * lam) ** (k // 2)
            assert abs(full[n] - s) < 1e-13 * max(1.0, abs(s))


def test_half_moments_match_quadrature():
    for U, lam in [(0.3, 0.8), (-1.2, 2.5), (2.0, 0.4)]:
        _, pos, neg = O.moments_1d(U, lam)
        rho = lambda u: math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)
        for n in range(7):
            p, _ = si.quad(lambda u: u ** n * rho(u), 0, np.inf, epsabs=1e-15, epsrel=1e-14)
            q, _ = si.quad(lambda u: u ** n * rho(u), -np.inf, 0, epsabs=1e-15, epsrel=1e-14)
            assert abs(pos[n] - p) < 1e-12 * max(1.0, abs(p))
            assert abs(neg[n] - q) < 1e-12 * max(1.0, abs(q))


def test_half_moments_sum_to_full():
    full, pos, neg = O.moments_1d(0.77, 1.3)
    assert np.allclose(pos + neg, full, rtol=1e-14, atol=1e-15)


def _gauss_moment_quadrature(U, V, W, lam, fun):
    """E[fun(u, v, w, xi2)] for the normalised Maxwellian with K = 2 internal DOF:
    Gauss-Hermite in u, v, w and Gauss-Laguerre in xi^2 ~ Exp(mean 1/lam)."""
    x, wx = np.polynomial.hermite.hermgauss(12)
    s, ws = np.polynomial.laguerre.laggauss(8)
    u = U + x / math.sqrt(lam)
    v = V + x / math.sqrt(lam)
    w = W + x / math.sqrt(lam)
    xi2 = s / lam
    uu, vv, ww, ss = np.meshgrid(u, v, w, xi2, indexing="ij")
    wt = (wx[:, None, None, None] * wx[None, :, None, None] * wx[None, None, :, None]
          * ws[None, None, None, :]) / math.pi ** 1.5
    return np.sum(wt * fun(uu, vv, ww, ss))


def test_slope_solve_recovers_known_slope():
    assert K == pytest.approx(2.0)
    U, V, W, lam = 0.4, -0.3, 0.9, 1.7
    rng = np.random.default_rng(1)
    for _ in range(3):
        a_true = rng.normal(size=5)

        def psi(k, u, v, w, s):
            return [np.ones_like(u), u, v, w, 0.5 * (u * u + v * v + w * w + s)][k]

        b = np.array([_gauss_moment_quadrature(
            U, V, W, lam,
            lambda u, v, w, s: sum(a_true[j] * psi(j, u, v, w, s) for j in range(5)) * psi(k, u, v, w, s))
            for k in range(5)])
        a = O.slope(U, V, W, lam, K, b)
        assert np.allclose(a, a_true, rtol=1e-11, atol=1e-11)


def _prim_to_cons(rho, u, p):
    u = np.asarray(u, float)
    return np.array([rho, *(rho * u), p / (GAMMA - 1) + 0.5 * rho * u @ u])


def test_collision_of_equal_states_is_identity():
    q = _prim_to_cons(1.3, [0.4, -0.2, 0.7], 0.9)
    q0 = O.collision(q, q)
    assert np.allclose(q0, q, rtol=1e-14, atol=1e-14)


def _euler_flux(q, n):
    rho, m, E = q[0], q[1:4], q[4]
    u = m / rho
    p = (GAMMA - 1) * (E - 0.5 * rho * (u @ u))
    un = u @ n
    return np.concatenate([[rho * un], rho * un * u + p * n, [(E + p) * un]])


def _jac(fun, q):
    """Complex-step Jacobian (exact to rounding for analytic functions)."""
    h = 1e-30
    J = np.empty((5, 5))
    for k in range(5):
        e = np.zeros(5, complex)
        e[k] = 1j * h
        J[:, k] = np.imag(fun(q.astype(complex) + e)) / h
    return J


@pytest.mark.parametrize("tau_mode", [0, 1])
def test_uniform_state_gives_euler_flux(tau_mode):
    p = O.default_params(tau_mode=tau_mode)
    q = _prim_to_cons(1.1, [0.3, -0.6, 0.25], 0.8)
    g = np.zeros((5, 3))
    rng = np.random.default_rng(2)
    for _ in range(4):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        F, dF = O.gks_flux(q, g, q, g, n, 0.01, p)
        assert np.allclose(F, _euler_flux(q, n), rtol=1e-13, atol=1e-13)
        assert np.allclose(dF, 0.0, atol=1e-11)


def test_tau0_linear_data_gives_euler_flux_and_its_time_derivative():
    """tau = 0 with identical smooth states: f = g(1 + A t) so F = F_Euler(Q) and
    dF/dt = dF_Euler/dQ . Q_t with Q_t = -sum_j dF_j/dQ dQ/dx_j (Euler equations)."""
    q = _prim_to_cons(1.2, [0.5, 0.2, -0.3], 1.1)
    rng = np.random.default_rng(3)
    grad = rng.normal(size=(5, 3)) * 0.2
    E = np.eye(3)
    Qt = -sum(_jac(lambda z: _euler_flux(z, E[j]), q) @ grad[:, j] for j in range(3))
    for _ in range(3):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        F, dF = O.gks_flux(q, grad, q, grad, n, 0.02)
        assert np.allclose(F, _euler_flux(q, n), rtol=1e-13, atol=1e-13)
        dF_exact = _jac(lambda z: _euler_flux(z, n), q) @ Qt
        assert np.allclose(dF, dF_exact, rtol=1e-11, atol=1e-12)


def _rotation(rng):
    A = rng.normal(size=(3, 3))
    Qm, R = np.linalg.qr(A)
    Qm *= np.sign(np.diag(R))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    return Qm


@pytest.mark.parametrize("tau_mode", [0, 1])
def test_flux_is_frame_invariant(tau_mode):
    """Rotating the whole configuration rotates the flux: the choice of tangents
    in the local frame does not matter."""
    p = O.default_params(tau_mode=tau_mode)
    rng = np.random.default_rng(4)
    ql = _prim_to_cons(1.0, [0.3, 0.1, -0.2], 1.0)
    qr = _prim_to_cons(0.8, [0.1, 0.3, 0.2], 0.7)
    gl = rng.normal(size=(5, 3)) * 0.1
    gr = rng.normal(size=(5, 3)) * 0.1
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    F, dF = O.gks_flux(ql, gl, qr, gr, n, 0.01, p)
    for _ in range(3):
        R = _rotation(rng)

        def rot_q(q):
            return np.concatenate([[q[0]], R @ q[1:4], [q[4]]])

        def rot_g(g):
            g2 = g @ R.T                      # spatial derivatives rotate
            g2[1:4] = R @ g2[1:4]             # momentum components rotate
            return g2

        F2, dF2 = O.gks_flux(rot_q(ql), rot_g(gl), rot_q(qr), rot_g(gr), R @ n, 0.01, p)
        assert np.allclose(F2, rot_q(F), rtol=1e-12, atol=1e-13)
        assert np.allclose(dF2, rot_q(dF), rtol=1e-10, atol=1e-11)


def test_small_tau_limit_matches_tau_zero():
    """The q-coefficients of the time integrals tend to the tau = 0 values."""
    rng = np.random.default_rng(5)
    ql = _prim_to_cons(1.0, [0.3, 0.1, -0.2], 1.0)
    qr = _prim_to_cons(1.0005, [0.3, 0.1, -0.2], 1.0004)
    gl = rng.normal(size=(5, 3)) * 0.1
    gr = gl + 1e-3
    n = np.array([0.6, 0.8, 0.0])
    dt = 0.01
    F0, dF0 = O.gks_flux(ql, gl, qr, gr, n, dt, O.default_params(tau_mode=0))
    prev = None
    for eps in (1e-2, 1e-3, 1e-4):
        F1, dF1 = O.gks_flux(ql, gl, qr, gr, n, dt, O.default_params(tau_mode=1, tau_eps=eps, tau_C=0.0))
        err = np.abs(F1 - F0).max() + dt * np.abs(dF1 - dF0).max()
        if prev is not None:
            assert err < prev * 0.2
        prev = err
    assert prev < 1e-4


def test_time_fit_recovers_linear_flux():
    """For tau = 0 the fitted F^n, dF^n reproduce int_0^dt and int_0^(dt/2) of the
    linear-in-time flux exactly, whatever dt."""
    q = _prim_to_cons(1.2, [0.5, 0.2, -0.3], 1.1)
    grad = np.random.default_rng(6).normal(size=(5, 3)) * 0.2
    n = np.array([0.0, 0.6, 0.8])
    F1, dF1 = O.gks_flux(q, grad, q, grad, n, 0.01)
    F2, dF2 = O.gks_flux(q, grad, q, grad, n, 0.0371)
    assert np.allclose(F1, F2, rtol=1e-13, atol=1e-14)
    assert np.allclose(dF1, dF2, rtol=1e-11, atol=1e-12)


def test_s2o4_reproduces_fourth_order_taylor_polynomial():
    """With L(q) = lam q and dL/dt = lam^2 q, one S2O4 step multiplies q by
    1 + z + z^2/2 + z^3/6 + z^4/24, z = lam dt (Sec. 2.2)."""
    q = np.array([1.0, -2.0, 0.5])
    for lam, dt in [(-1.3, 0.1), (0.7, 0.05), (-3.0, 0.2)]:
        L, dL = lam * q, lam * lam * q
        qs = O.s2o4_stage1(q, L, dL, dt)
        dLs = lam * lam * qs
        qn = O.s2o4_stage2(q, L, dL, dLs, dt)
        z = lam * dt
        assert np.allclose(qn, q * (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24), rtol=1e-15, atol=1e-15)
