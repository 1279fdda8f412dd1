"""The basis of the FP32 forms' warm-point rule (the tau > 0 Gauss points evaluated in
FP64): the micro-slope solve of Sec. 2.1 (<(a.psi) psi> = b, solved in closed form)
replayed in float32 and float64 on the same state (the float32 side also rounds the
state itself, as the FP32 path does).  Its FP32 error grows with kappa = E / (rho e):
below 1e-5 of the slope's size for kappa <= 10, above 1e-4 from kappa = 1e3 (the cold
states where the FP32 flux departed had kappa from 37 to 4e5, and there the half-space
slope moments multiply the error further).

Test infrastructure: a numpy replay of the closed-form inverse of the 5x5 moment
matrix, checked first against the oracle's dense solve in FP64."""
import numpy as np
import pytest

from oracle import oracle as O

G = 1.4
K = (5 - 3 * G) / (G - 1)


def slope_closed_form(q, b_dir, T):
    """Micro-slope a for the state q (conservative) and b = dQ/rho along one direction."""
    q = np.asarray(q, dtype=T)
    rho = q[0]
    U = q[1:4] / rho
    q2 = U @ U
    p = T(G - 1) * (q[4] - T(0.5) * rho * q2)
    i2l = p / rho
    lam = T(0.5) * rho / p
    c4 = T(4) / T(K + 3) * lam * lam
    e2 = q2 + T(K + 3) * i2l
    b = np.asarray(b_dir, dtype=T) / rho
    R = b[1:4] - U * b[0]
    R4 = T(2) * b[4] - e2 * b[0]
    a = np.empty(5, dtype=T)
    a[4] = c4 * (R4 - T(2) * (U @ R))
    a[1:4] = T(2) * lam * R - U * a[4]
    a[0] = b[0] - U @ a[1:4] - T(0.5) * a[4] * e2
    return a, U, lam


def _state(kappa, speed_dir=(0.6, -0.48, 0.64), rho=0.8):
    """A state with E / (rho e) = kappa at pressure 1e-2 scaled speed."""
    p = 0.05
    e = p / ((G - 1) * rho)
    ke = (kappa - 1.0) * e                       # kinetic energy per mass
    u = np.sqrt(2 * ke) * np.asarray(speed_dir) / np.linalg.norm(speed_dir)
    return np.array([rho, *(rho * u), rho * (e + ke)])


def test_closed_form_matches_the_oracle_solve():
    q = _state(3.0)
    b = np.array([0.3, -0.2, 0.5, 0.1, 0.7])
    a, U, lam = slope_closed_form(q, b, np.float64)
    a_orc = O.slope(*U, lam, K, b / q[0])
    assert np.allclose(a, a_orc, rtol=1e-10, atol=1e-12 * np.abs(a_orc).max())


@pytest.mark.parametrize("kappa,ok", [(1.05, True), (2.0, True), (10.0, True), (1e3, False), (1e4, False)])
def test_fp32_slope_error_grows_with_kappa(kappa, ok):
    rng = np.random.default_rng(int(kappa * 100))
    worst = 0.0
    for _ in range(200):
        q = _state(kappa, speed_dir=rng.standard_normal(3), rho=rng.uniform(0.1, 2.0))
        b = rng.standard_normal(5) * 50.0          # steep gradients, as at a shock
        a32, _, _ = slope_closed_form(q.astype(np.float32), b.astype(np.float32), np.float32)
        a64, _, _ = slope_closed_form(q, b, np.float64)
        worst = max(worst, float(np.abs(a32 - a64).max() / np.abs(a64).max()))
    if ok:
        assert worst < 1e-5, worst
    else:
        assert worst > 1e-4, worst
