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


def rel_l1_scaled(q, q_ref, vol, gamma=1.4):
    """Volume-weighted L1 of the difference per variable, relative to the L1 of the
    reference for rho and rho E, and for each momentum component to the L1 of a
    momentum scale per cell, max(|rho U|, rho c), so that a component that is zero or
    small in the flow is not measured against itself."""
    q_ref = np.asarray(q_ref)
    rho = q_ref[:, 0]
    m = q_ref[:, 1:4]
    p = (gamma - 1) * (q_ref[:, 4] - 0.5 * np.sum(m * m, axis=1) / rho)
    ms = np.maximum(np.sqrt(np.sum(m * m, axis=1)), rho * np.sqrt(gamma * np.abs(p) / rho))
    den = np.array([np.sum(np.abs(rho) * vol), *(3 * [np.sum(ms * vol)]), np.sum(np.abs(q_ref[:, 4]) * vol)])
    return np.sum(np.abs(np.asarray(q) - q_ref) * vol[:, None], axis=0) / den


def advection_case(n, seed=None, **kw):
    mesh = W.kuhn_box(n, seed=W.SEED_ADVECTION if seed is None else seed)
    case = W.AdvectionCase(**kw)
    return mesh, case, case.conservative(mesh)


def mirror_double(mesh, axis):
    """The mesh and its mirror image across its highest wall on `axis`, as one mesh
    periodic on that axis with twice the length.  Cells [0, nc) are the original
    ones, cells [nc, 2 nc) their mirror images in the same order.  On this mesh the
    state (q, q) is mirror-symmetric about both walls of the original box, so the
    original cells see real cells where the wall mesh has ghosts."""
    x = mesh.nodes[:, axis]
    lo, hi = x.min(), x.max()
    assert lo == 0.0 and mesh.period[axis] == 0.0
    inner = (x > lo) & (x < hi)
    n0 = mesh.nodes.shape[0]
    copy_id = np.arange(n0)
    copy_id[inner] = n0 + np.arange(int(inner.sum()))
    extra = mesh.nodes[inner].copy()
    extra[:, axis] = 2.0 * hi - extra[:, axis]
    nodes = np.concatenate([mesh.nodes, extra])
    cells = np.concatenate([mesh.cell_nodes, copy_id[mesh.cell_nodes]])
    verts_m = mesh.cell_vertices.copy()
    verts_m[:, :, axis] = 2.0 * hi - verts_m[:, :, axis]
    period = mesh.period.copy()
    period[axis] = 2.0 * hi
    return W.TetMesh(nodes=nodes, cell_nodes=cells, period=period,
                     cell_vertices=np.concatenate([mesh.cell_vertices, verts_m]))


def smooth_state(mesh, seed, gamma=1.4):
    """A smooth state with every component nonzero (moving in all directions)."""
    rng = np.random.default_rng(seed)
    c = mesh.cell_vertices.mean(axis=1)
    k = rng.uniform(1.0, 3.0, size=(5, 3))
    ph = rng.uniform(0.0, 2 * np.pi, size=5)
    s = np.sin(c @ k.T + ph)
    rho = 1.0 + 0.2 * s[:, 0]
    u = np.stack([0.4 + 0.3 * s[:, 1], -0.3 + 0.2 * s[:, 2], 0.2 + 0.25 * s[:, 3]], axis=1)
    p = 1.0 + 0.15 * s[:, 4]
    q = np.empty((c.shape[0], 5))
    q[:, 0] = rho
    q[:, 1:4] = rho[:, None] * u
    q[:, 4] = p / (gamma - 1.0) + 0.5 * rho * (u * u).sum(axis=1)
    return q
