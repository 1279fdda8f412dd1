"""Accuracy of the HIP path on the smooth advection test (Sec. 5.1): errors against
the exact translated solution, and the convergence order at a common final time.

Config 1 (6*8^3 jittered tets, CFL 0.3, 20 steps): L1 / L2 / Linf of the density
against the exact cell averages of rho = 1 + 0.2 sin(pi(x + y + z - 3t)).
Config 2's order study: 6*N^3 tets for N = 16, 32, 64 at T = 0.12 with fixed steps
dt = T / (25 N / 16) (CFL about 0.3 at every N), in FP64, FP32-mixed and FP32, on
the regular six-tetrahedra split and on the jittered meshes of the workload.  The
reduced-precision forms stay within 1e-5 relative L1 of FP64 in every variable.
"""
import math
import sys

import numpy as np
import pytest

from paper_2407_00656_amd import hgks
from paper_2407_00656_amd import workloads as W
from tests.helpers import rel_l1_scaled

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(mesh, q0, precision, steps, dt_fixed=0.0):
    s = hgks.Solver(hgks.params(precision=precision))
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    s.init_state(q0)
    s.step(steps, dt_fixed=dt_fixed)
    q, t = s.get_state()
    s.close()
    return q, t


def test_config1_errors_against_exact_solution():
    say("case: config 1, 6*8^3 jittered tets, CFL 0.3, 20 steps, errors vs exact")
    mesh, case = W.advection_config(8)
    q0 = case.conservative(mesh)
    vol = W.tet_volumes(mesh.cell_vertices)
    q, t = _run(mesh, q0, hgks.FP64, 20)
    e = W.error_norms(vol, q[:, 0], case.density_average(mesh, t))
    say(f"config 1 FP64 at t = {t:.6f}: L1 {e['L1']:.4e} L2 {e['L2']:.4e} Linf {e['Linf']:.4e} "
        f"(normalised by |D| = 8: L1 {e['L1'] / 8:.4e})")
    assert 0.15 < t < 0.25
    assert 2.3 < e["L1"] / e["L2"] < 2.7          # a sine-shaped error (reading of the norms)
    # N = 8 resolves the wave with under five cells per wavelength along the diagonal:
    # the error is about a tenth of the amplitude 0.2 at its worst (measured Linf 0.022)
    assert e["Linf"] < 0.05 and e["L1"] < 0.15
    # and it is the oracle's error, run over the same 20 steps
    from oracle import oracle as O
    q_orc, _ = O.Mesh.from_workload(mesh).step(q0, 20)
    e_orc = W.error_norms(vol, q_orc[:, 0], case.density_average(mesh, t))
    say(f"config 1 oracle: L1 {e_orc['L1']:.4e} L2 {e_orc['L2']:.4e} Linf {e_orc['Linf']:.4e}")
    for k in ("L1", "L2", "Linf"):
        assert abs(e[k] - e_orc[k]) <= 1e-10 * e_orc[k], k
    for prec in (hgks.FP32_MIXED, hgks.FP32):
        q32, _ = _run(mesh, q0, prec, 20)
        d = rel_l1_scaled(q32, q, vol)
        say(f"config 1 precision {prec} vs FP64: relative L1 {d}")
        assert np.all(d < 1e-5), d


@pytest.mark.parametrize("jitter,eps", [(0.0, 1e-8), (0.1, 1e-8), (0.1, 1.0)])
def test_config2_order_study(jitter, eps):
    """Order study at T = 0.12.  With the WENO-Z weights of the build (weno_eps 1e-8)
    the FP64 L1 order is 2.88-2.93 on both mesh kinds, and the max-norm order drops to
    about 2.2 on the finest pair: near the extrema of the wave the smoothness
    indicators of all stencils are small and alike, so the non-linear weights leave
    the linear ones there.  With weno_eps = 1 the weights are the linear ones and the
    scheme shows its design order, 2.93-3.00 in L1 (and in max norm on regular meshes)."""
    T = 0.12
    precs = (hgks.FP64, hgks.FP32_MIXED, hgks.FP32) if eps < 1e-3 else (hgks.FP64,)
    say(f"case: order study 6*N^3, N = 16/32/64, T = {T}, jitter {jitter}, weno_eps {eps}")
    rows = []
    for n in (16, 32, 64):
        mesh, case = W.advection_config(n, jitter=jitter)
        q0 = case.conservative(mesh)
        vol = W.tet_volumes(mesh.cell_vertices)
        steps = 25 * n // 16
        exact = case.density_average(mesh, T)
        res = {}
        for prec in precs:
            s = hgks.Solver(hgks.params(precision=prec, weno_eps=eps))
            s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
            s.init_state(q0)
            s.step(steps, dt_fixed=T / steps)
            res[prec], t = s.get_state()
            s.close()
            assert abs(t - T) < 1e-12
        e = W.error_norms(vol, res[hgks.FP64][:, 0], exact)
        line = f"N={n} steps={steps} FP64 L1 {e['L1']:.4e} L2 {e['L2']:.4e} Linf {e['Linf']:.4e}"
        for p in precs[1:]:
            d = rel_l1_scaled(res[p], res[hgks.FP64], vol)
            line += f"; precision {p} vs FP64 rel L1 {d.max():.2e}"
            assert np.all(d < 1e-5), (n, p, d)
        say(line)
        rows.append((n, e["L1"], e["Linf"]))
    orders = [math.log(a[1] / b[1]) / math.log(b[0] / a[0]) for a, b in zip(rows, rows[1:])]
    orders_inf = [math.log(a[2] / b[2]) / math.log(b[0] / a[0]) for a, b in zip(rows, rows[1:])]
    say(f"jitter {jitter} weno_eps {eps}: L1 orders {orders}, Linf orders {orders_inf}")
    if eps >= 1.0:
        assert all(2.85 <= o <= 3.15 for o in orders), orders
    else:
        assert all(2.8 <= o <= 3.15 for o in orders), orders


@pytest.mark.parametrize("weno_eps,lo", [(1.0, 2.85), (1e-8, 1.8)])
def test_hex_order_on_the_gpu(weno_eps, lo):
    """Hexahedral boxes N = 16, 24, 32 without jitter, T = 0.05, dt = T / (0.75 N):
    with near-linear weights the L1 density error falls at third order (the oracle
    measures 2.86 and 2.91 at N = 12/16/24); with the default WENO-Z epsilon the
    weights leave the linear ones at the extrema and the observed order on these
    meshes is lower (reported, bounded below by 1.8).  FP32-mixed stays within 1e-5
    relative L1 of FP64."""
    case = W.AdvectionCase()
    T = 0.05
    res = []
    for n in (16, 24, 32):
        mesh = W.hex_box(n, jitter=0.0)
        q0 = case.conservative(mesh)
        steps = int(round(0.75 * n))
        out = {}
        for prec in (hgks.FP64, hgks.FP32_MIXED):
            s = hgks.Solver(hgks.params(precision=prec, weno_eps=weno_eps))
            s.upload(mesh)
            s.init_state(q0)
            s.step(steps, dt_fixed=T / steps)
            out[prec], _ = s.get_state()
            s.close()
        vol = W.hex_volumes(mesh.cell_vertices)
        e = W.error_norms(vol, out[hgks.FP64][:, 0], case.density_average(mesh, T))
        d = rel_l1_scaled(out[hgks.FP32_MIXED], out[hgks.FP64], vol)
        say(f"hex N={n} eps={weno_eps}: L1 {e['L1']:.4e} Linf {e['Linf']:.4e}; FP32-mixed vs FP64 {d.max():.2e}")
        assert np.all(d < 1e-5)
        res.append((n, e["L1"]))
    orders = [math.log(a[1] / b[1]) / math.log(b[0] / a[0]) for a, b in zip(res, res[1:])]
    say("hex orders", orders)
    assert all(lo <= o <= 3.2 for o in orders), orders
