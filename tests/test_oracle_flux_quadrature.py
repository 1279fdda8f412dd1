"""Pins of the oracle's gas-kinetic flux against direct quadrature of the
interface distribution of Sec. 2.1, Eq. (flux).

Everything expected here is computed in this file from the paper's formulas,
by numerical quadrature, with none of the oracle's machinery:

* velocity space: Gauss-Hermite nodes in v and w (and in u over the whole line),
  composite Gauss-Legendre nodes on a truncated half line in u for the half-space parts,
  and generalised Gauss-Laguerre nodes for xi^2, which for K internal degrees of
  freedom of a Maxwellian is Gamma(K/2)-distributed with scale 1/lam;
* micro-slopes from the compatibility conditions of Sec. 2.1 (<a^k> = dQ_k/dn_j,
  <a_1 u + a_2 v + a_3 w + A> = 0), with the 5x5 moment matrices built by that
  quadrature and solved by numpy;
* the equilibrium state from the compatibility condition Q0 = int_{u>0} psi g_l
  + int_{u<0} psi g_r, again by quadrature;
* time integrals I(delta) = int_0^delta F(t) dt by Gauss-Legendre in t, and the
  linear fit F dt + dF dt^2/2 = I(dt), F dt/2 + dF dt^2/8 = I(dt/2) of Sec. 2.2.

The tangents of the local frame are chosen differently from the oracle's (the
global-frame flux does not depend on them).
"""
import math

import numpy as np
import pytest
from scipy import special as sp

from oracle import oracle as O

GAMMA = 1.4
K = (5 - 3 * GAMMA) / (GAMMA - 1)


def _prim_to_cons(rho, u, p):
    u = np.asarray(u, float)
    return np.array([rho, *(rho * u), p / (GAMMA - 1) + 0.5 * rho * u @ u])


def _frame(n):
    """n and two tangents: Gram-Schmidt of the coordinate axis with the smallest |n_a|
    taken last (not the oracle's cross-product rule)."""
    a = int(np.argmin(np.abs(n)))
    e = np.zeros(3)
    e[(a + 1) % 3] = 1.0
    t1 = e - (e @ n) * n
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    return np.stack([n, t1, t2])          # rows: the local axes


def _rot(q, R):
    return np.concatenate([[q[0]], R @ q[1:4], [q[4]]])


class Maxwellian:
    """A Maxwellian of density rho, velocity (U, V, W) in the local frame and
    lam = rho / (2 p), with quadrature nodes for full-space and half-space moments."""

    NH, NL = 14, 8
    PANELS, NG = 32, 16               # composite Gauss-Legendre on the half line

    def __init__(self, q_local):
        self.rho = q_local[0]
        self.U = q_local[1:4] / self.rho
        p = (GAMMA - 1) * (q_local[4] - 0.5 * self.rho * self.U @ self.U)
        self.lam = self.rho / (2 * p)

    def _nodes(self, half):
        lam, (U, V, W) = self.lam, self.U
        x, wx = np.polynomial.hermite.hermgauss(self.NH)
        s, ws = sp.roots_genlaguerre(self.NL, K / 2 - 1)
        v, w = V + x / math.sqrt(lam), W + x / math.sqrt(lam)
        wv = wx / math.sqrt(math.pi)
        xi2, wxi = s / lam, ws / math.gamma(K / 2)
        if half == 0:
            u, wu = U + x / math.sqrt(lam), wv
        else:
            # the half line, truncated where the Gaussian has fallen below e^-196
            lo, hi = (0.0, max(0.0, U) + 14 / math.sqrt(lam)) if half > 0 else (min(0.0, U) - 14 / math.sqrt(lam), 0.0)
            t, wt = np.polynomial.legendre.leggauss(self.NG)
            e = np.linspace(lo, hi, self.PANELS + 1)
            a, b = e[:-1, None], e[1:, None]
            u = (0.5 * (b - a) * t + 0.5 * (b + a)).ravel()
            wu = (0.5 * (b - a) * wt).ravel() * math.sqrt(lam / math.pi) * np.exp(-lam * (u - U) ** 2)
        uu, vv, ww, ss = np.meshgrid(u, v, w, xi2, indexing="ij")
        wt4 = wu[:, None, None, None] * wv[None, :, None, None] * wv[None, None, :, None] * wxi[None, None, None, :]
        return (uu, vv, ww, ss), wt4

    def expect(self, fun, half=0):
        """rho * int fun g over all u (half = 0), u > 0 (+1) or u < 0 (-1)."""
        (u, v, w, s), wt = self._nodes(half)
        vals = fun(u, v, w, s)
        if isinstance(vals, (list, tuple)):
            return np.array([self.rho * np.sum(wt * f) for f in vals])
        return self.rho * np.sum(wt * vals)


def _psi(u, v, w, s):
    return [np.ones_like(u), u, v, w, 0.5 * (u * u + v * v + w * w + s)]


def _lin(a, u, v, w, s):
    """a . psi"""
    ps = _psi(u, v, w, s)
    return sum(a[k] * ps[k] for k in range(5))


def _slopes(g: Maxwellian, dQ):
    """Spatial micro-slopes a_j from <a_j . psi> = dQ/dn_j and the time slope A from
    <a_1 u + a_2 v + a_3 w + A> = 0, with <...> = int g (...) psi (Sec. 2.1; g
    carries its density)."""
    M = np.array([[g.expect(lambda u, v, w, s, i=i, j=j: _psi(u, v, w, s)[i] * _psi(u, v, w, s)[j])
                   for j in range(5)] for i in range(5)])
    a = [np.linalg.solve(M, dQ[j]) for j in range(3)]
    rhs = g.expect(lambda u, v, w, s: [(u * _lin(a[0], u, v, w, s) + v * _lin(a[1], u, v, w, s)
                                        + w * _lin(a[2], u, v, w, s)) * p for p in _psi(u, v, w, s)])
    A = np.linalg.solve(M, -rhs)
    return a, A


def quadrature_flux(ql, gl, qr, gr, n, dt, tau, dq0_mean=True):
    """F^n and dF^n/dt (global frame) of Eq. (flux) by direct quadrature."""
    R = _frame(np.asarray(n, float))
    Ql, Qr = _rot(ql, R), _rot(qr, R)
    # derivative along local axis j of each variable, momentum rotated into the frame
    dQl = [_rot(gl @ R[j], R) for j in range(3)]
    dQr = [_rot(gr @ R[j], R) for j in range(3)]
    Gl, Gr = Maxwellian(Ql), Maxwellian(Qr)
    # compatibility condition: the equilibrium collects the left state's particles
    # moving right and the right state's particles moving left
    Q0 = (Gl.expect(lambda u, v, w, s: _psi(u, v, w, s), +1)
          + Gr.expect(lambda u, v, w, s: _psi(u, v, w, s), -1))
    G0 = Maxwellian(Q0)
    dQ0 = [0.5 * (dQl[j] + dQr[j]) for j in range(3)]
    al, Al = _slopes(Gl, dQl)
    ar, Ar = _slopes(Gr, dQr)
    a0, A0 = _slopes(G0, dQ0)

    def moments(G, a, A, half):
        """<u psi>, <u (a_1 u + a_2 v + a_3 w) psi>, <u (A.psi) psi> over the given half space"""
        m0 = G.expect(lambda u, v, w, s: [u * p for p in _psi(u, v, w, s)], half)
        m1 = G.expect(lambda u, v, w, s: [u * (u * _lin(a[0], u, v, w, s) + v * _lin(a[1], u, v, w, s)
                                               + w * _lin(a[2], u, v, w, s)) * p for p in _psi(u, v, w, s)], half)
        m2 = G.expect(lambda u, v, w, s: [u * _lin(A, u, v, w, s) * p for p in _psi(u, v, w, s)], half)
        return m0, m1, m2

    e0, el, er = moments(G0, a0, A0, 0), moments(Gl, al, Al, +1), moments(Gr, ar, Ar, -1)

    def F_of_t(t):
        if tau == 0.0:
            c = [1.0, 0.0, t, 0.0, 0.0, 0.0]
        else:
            E = math.exp(-t / tau)
            c = [1 - E, (t + tau) * E - tau, t - tau + tau * E, E, -(tau + t) * E, -tau * E]
        return (c[0] * e0[0] + c[1] * e0[1] + c[2] * e0[2]
                + c[3] * (el[0] + er[0]) + c[4] * (el[1] + er[1]) + c[5] * (el[2] + er[2]))

    x, w = np.polynomial.legendre.leggauss(40)

    def I(d):
        return sum(0.5 * d * wk * F_of_t(0.5 * d * (xk + 1)) for xk, wk in zip(x, w))

    I1, I2 = I(dt), I(0.5 * dt)
    M = np.array([[dt, 0.5 * dt * dt], [0.5 * dt, dt * dt / 8]])
    sol = np.linalg.solve(M, np.stack([I1, I2]))
    Fl, dFl = sol[0], sol[1]
    # back to the global frame: the local momentum components are along the rows of R
    F = np.concatenate([[Fl[0]], R.T @ Fl[1:4], [Fl[4]]])
    dF = np.concatenate([[dFl[0]], R.T @ dFl[1:4], [dFl[4]]])
    return F, dF, Q0


def _oracle_flux(ql, gl, qr, gr, n, dt, tau):
    p = O.default_params(tau_mode=1, tau_eps=tau / dt, tau_C=0.0) if tau > 0 else O.default_params(tau_mode=0)
    return O.gks_flux(ql, gl, qr, gr, n, dt, p)


def _cases():
    rng = np.random.default_rng(2407)
    out = []
    for k in range(3):
        ql = _prim_to_cons(1.0 + 0.3 * k, [0.4, -0.2, 0.3 - 0.2 * k], 1.0 + 0.1 * k)
        qr = _prim_to_cons(0.55 + 0.1 * k, [-0.1, 0.35, 0.1], 0.45 + 0.2 * k)
        gl = rng.normal(size=(5, 3)) * 0.3
        gr = rng.normal(size=(5, 3)) * 0.3
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        out.append((ql, gl, qr, gr, n))
    return out


def test_quadrature_reproduces_half_space_closed_forms():
    """The quadrature itself: zeroth and first half-space moments of a 1-D Gaussian
    against erfc and the Gaussian closed forms."""
    g = Maxwellian(_prim_to_cons(1.0, [0.7, 0.0, 0.0], 0.6))
    sl = math.sqrt(g.lam)
    for half, sgn in ((+1, 1.0), (-1, -1.0)):
        m0 = g.expect(lambda u, v, w, s: np.ones_like(u), half)
        m1 = g.expect(lambda u, v, w, s: u, half)
        e0 = 0.5 * sp.erfc(-sgn * sl * g.U[0])
        e1 = g.U[0] * e0 + sgn * math.exp(-g.lam * g.U[0] ** 2) / (2 * math.sqrt(math.pi * g.lam))
        assert abs(m0 - e0) < 1e-14 and abs(m1 - e1) < 1e-14


def test_collision_of_unequal_states_matches_quadrature():
    """Q0 = int_{u>0} psi g_l + int_{u<0} psi g_r (the compatibility condition)."""
    for ql, _, qr, _, _ in _cases():
        want = (Maxwellian(ql).expect(lambda u, v, w, s: _psi(u, v, w, s), +1)
                + Maxwellian(qr).expect(lambda u, v, w, s: _psi(u, v, w, s), -1))
        got = O.collision(ql, qr)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-14), (got, want)
        # and not the swapped half spaces
        swapped = (Maxwellian(ql).expect(lambda u, v, w, s: _psi(u, v, w, s), -1)
                   + Maxwellian(qr).expect(lambda u, v, w, s: _psi(u, v, w, s), +1))
        assert np.abs(swapped - want).max() > 1e-2


@pytest.mark.parametrize("tau_frac", [0.0, 0.1, 1.0])
def test_flux_matches_quadrature_of_the_interface_distribution(tau_frac):
    """Unequal states with independent nonzero gradients: the oracle's F^n and
    dF^n/dt equal the direct quadrature of Eq. (flux) for tau = 0, dt/10 and dt."""
    dt = 0.02
    for ql, gl, qr, gr, n in _cases():
        tau = tau_frac * dt
        F, dF = _oracle_flux(ql, gl, qr, gr, n, dt, tau)
        Fq, dFq, _ = quadrature_flux(ql, gl, qr, gr, n, dt, tau)
        scale = np.abs(Fq).max()
        assert np.abs(F - Fq).max() <= 1e-12 * scale, (F, Fq)
        assert dt * np.abs(dF - dFq).max() <= 1e-10 * scale, (dF, dFq)


def test_equal_states_give_the_navier_stokes_distribution():
    """Equal states and equal nonzero gradients on both sides: Eq. (flux) collapses
    to f = g [1 - tau (a.u + A) + t A], the Chapman-Enskog distribution of the BGK
    model (viscosity tau p), so F^n = F_Euler - tau rho <u (a_1 u + a_2 v + a_3 w + A) psi>
    and dF^n/dt = rho <u A psi>, its tau = 0 value, for any tau."""
    rng = np.random.default_rng(11)
    dt = 0.02
    for k in range(3):
        q = _prim_to_cons(1.1 + 0.2 * k, [0.3, -0.5, 0.2 + 0.1 * k], 0.9)
        g = rng.normal(size=(5, 3)) * 0.3
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        R = _frame(n)
        Q = _rot(q, R)
        dQ = [_rot(g @ R[j], R) for j in range(3)]
        G = Maxwellian(Q)
        a, A = _slopes(G, dQ)
        euler = G.expect(lambda u, v, w, s: [u * p for p in _psi(u, v, w, s)])
        visc = G.expect(lambda u, v, w, s: [u * (u * _lin(a[0], u, v, w, s) + v * _lin(a[1], u, v, w, s)
                                                 + w * _lin(a[2], u, v, w, s) + _lin(A, u, v, w, s)) * p
                                            for p in _psi(u, v, w, s)])
        dFl = G.expect(lambda u, v, w, s: [u * _lin(A, u, v, w, s) * p for p in _psi(u, v, w, s)])
        F0, dF0 = O.gks_flux(q, g, q, g, n, dt, O.default_params(tau_mode=0))
        for tau in (0.0, 0.1 * dt, dt, 3 * dt):
            Fl = euler - tau * visc
            want_F = np.concatenate([[Fl[0]], R.T @ Fl[1:4], [Fl[4]]])
            want_dF = np.concatenate([[dFl[0]], R.T @ dFl[1:4], [dFl[4]]])
            F, dF = _oracle_flux(q, g, q, g, n, dt, tau)
            scale = np.abs(want_F).max()
            assert np.abs(F - want_F).max() <= 1e-12 * scale, (tau, F, want_F)
            assert dt * np.abs(dF - want_dF).max() <= 1e-10 * scale, (tau, dF, want_dF)
            assert dt * np.abs(dF - dF0).max() <= 1e-10 * scale
        # the viscous term is really there (otherwise the pin would be vacuous)
        assert np.abs(visc).max() > 1e-2
