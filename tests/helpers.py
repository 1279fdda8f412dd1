"""Shared test helpers: parity norms and small case builders."""
import numpy as np

from paper_2407_00656_amd import workloads as W


def scaled_err(q_gpu, q_ref, gamma=1.4):
    """Per-variable error normalised by a physical scale of that variable:
    rho and rho E by their maximum magnitude; each momentum component by
    max(max |rho U|, max rho c), so a component that is zero or tiny is measured
    against a momentum scale of the flow."""
    q_ref = np.asarray(q_ref)
    d = np.abs(np.asarray(q_gpu) - q_ref).max(axis=0)
    rho = q_ref[:, 0]
    m = q_ref[:, 1:4]
    p = (gamma - 1) * (q_ref[:, 4] - 0.5 * np.sum(m * m, axis=1) / rho)
    mom_scale = max(np.sqrt(np.sum(m * m, axis=1)).max(), np.max(rho * np.sqrt(gamma * p / rho)))
    s = np.array([np.abs(rho).max(), mom_scale, mom_scale, mom_scale, np.abs(q_ref[:, 4]).max()])
    return d / s


def rel_l1(q, q_ref, vol):
    """Volume-weighted L1 of the difference relative to the L1 of the reference, per variable."""
    return np.sum(np.abs(q - q_ref) * vol[:, None], axis=0) / np.sum(np.abs(q_ref) * vol[:, None], axis=0)


def advection_case(n, seed=None, **kw):
    mesh = W.kuhn_box(n, seed=W.SEED_ADVECTION if seed is None else seed)
    case = W.AdvectionCase(**kw)
    return mesh, case, case.conservative(mesh)
