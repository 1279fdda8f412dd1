"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (per conserved variable, normalised as in helpers.scaled_err):
  FP64 path      <= 1e-12 after one step from an identical state;
  FP32-mixed     <= 1e-5 relative L1 after the full run;
  FP32           the same bar (the pseudo-inverse rounded once to FP32 adds a
                 relative 6e-8 to each coefficient, the FP32 contractions about
                 16 roundings of the largest product: the same order as the
                 FP32-mixed form's own rounding of the weights and fluxes).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_00656_amd import hgks
from paper_2407_00656_amd import workloads as W
from tests.helpers import advection_case, rel_l1, rel_l1_scaled, scaled_err, smooth_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_solver(mesh, q, **kw):
    s = hgks.Solver(hgks.params(**kw))
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    s.init_state(q)
    return s


def oracle_params(**kw):
    keep = {k: v for k, v in kw.items() if k in ("tau_mode", "tau_eps", "tau_C", "weno_eps", "gamma_lin", "cfl")}
    return O.default_params(**keep)


def per_step_parity(mesh, q0, nsteps, **kw):
    om = O.Mesh.from_workload(mesh)
    op = oracle_params(**kw)
    s = make_solver(mesh, q0, **kw)
    worst = np.zeros(5)
    q = q0
    for k in range(nsteps):
        dt_gpu = s.step(1, want_dt=True)
        q_gpu, _ = s.get_state()
        q_orc, dt_orc = om.step(q, 1, params=op)
        assert abs(dt_gpu - dt_orc) <= 1e-14 * dt_orc, (k, dt_gpu, dt_orc)
        e = scaled_err(q_gpu, q_orc)
        worst = np.maximum(worst, e)
        assert np.all(e <= TOL64), (k, e)
        q = q_gpu                    # next step starts from the same state on both sides
    s.close()
    return worst


def test_fp64_config1_every_step():
    """The accuracy-test box: 6*8^3 jittered tets, 20 CFL-0.3 steps, each step matched."""
    say("case: fp64 N=8 20 steps")
    mesh, case, q0 = advection_case(8)
    worst = per_step_parity(mesh, q0, 20)
    say("worst scaled error", worst)


@pytest.mark.parametrize("n,seed", [(5, 101), (7, 102), (6, 103)])
def test_fp64_odd_and_ragged_sizes(n, seed):
    """6 n^3 cells with n odd / not a multiple of the tile sizes (ragged last tiles)."""
    say(f"case: fp64 ragged N={n} seed={seed}")
    mesh, case, q0 = advection_case(n, seed=seed, k=(1, 2, 1), vel=(0.8, -0.3, 0.5), amp=0.15)
    assert mesh.n_cells % 64 != 0
    per_step_parity(mesh, q0, 2)


def test_fp64_tau_positive_branch():
    say("case: fp64 tau_mode=1 N=6")
    mesh, case, q0 = advection_case(6, seed=104, amp=0.2, vel=(1.0, 0.2, -0.4))
    per_step_parity(mesh, q0, 2, tau_mode=1, tau_eps=0.05, tau_C=1.0)


def test_fp64_coloured_accumulation():
    say("case: fp64 coloured accumulation N=6, N=8")
    for n in (6, 8):
        mesh, case, q0 = advection_case(n, seed=105 + n)
        per_step_parity(mesh, q0, 2, accumulation=hgks.ACC_COLOURED)


@pytest.mark.parametrize("prec", [hgks.FP32_MIXED, hgks.FP32])
def test_fp32_config1_full_run(prec):
    say(f"case: precision {prec} N=8 20 steps vs oracle")
    mesh, case, q0 = advection_case(8)
    om = O.Mesh.from_workload(mesh)
    vol = om.cells()[0]
    q_orc, _ = om.step(q0, 20)
    s = make_solver(mesh, q0, precision=prec)
    s.step(20)
    q32, _ = s.get_state()
    err = rel_l1(q32, q_orc, vol)
    say("relative L1 (reduced precision vs fp64 oracle)", err)
    assert np.all(err <= TOL32), err


def test_fp32_odd_ragged_tau_positive():
    """The FP32 form on an odd, ragged mesh (tiles with a tail) with tau > 0."""
    say("case: fp32 N=(7,5,4) tau_mode=1 8 steps vs oracle")
    mesh = W.kuhn_box((7, 5, 4), (1.4, 1.0, 0.8), jitter=0.12, seed=4245)
    q0 = smooth_state(mesh, 13)
    om = O.Mesh.from_workload(mesh)
    vol = om.cells()[0]
    q_orc, _ = om.step(q0, 8, params=oracle_params(tau_mode=1))
    s = make_solver(mesh, q0, precision=hgks.FP32, tau_mode=1)
    s.step(8)
    q32, _ = s.get_state()
    s.close()
    err = rel_l1(q32, q_orc, vol)
    say("relative L1 (fp32 vs fp64 oracle)", err)
    assert np.all(err <= TOL32), err


def test_bitwise_determinism_and_restart():
    say("case: determinism + checkpoint/restart N=6")
    mesh, case, q0 = advection_case(6, seed=110, vel=(0.5, 1.0, -0.2))
    for prec in (hgks.FP64, hgks.FP32_MIXED, hgks.FP32):
        a = make_solver(mesh, q0, precision=prec)
        a.step(6)
        qa, ta = a.get_state()
        b = make_solver(mesh, q0, precision=prec)
        b.step(6)
        assert b.get_time() == ta          # time-only read back (no state copy)
        qb, tb = b.get_state()
        assert np.array_equal(qa, qb) and ta == tb
        c = make_solver(mesh, q0, precision=prec)
        c.step(3)
        qm, tm = c.get_state()
        d = make_solver(mesh, qm, precision=prec)
        d.init_state(qm, tm)
        d.step(3)
        qd, td = d.get_state()
        assert np.array_equal(qd, qa) and abs(td - ta) <= 1e-15 * ta
        for x in (a, b, c, d):
            x.close()


def test_free_stream_and_conservation_on_gpu():
    say("case: free stream + conservation N=8")
    mesh = W.kuhn_box(8, seed=111)
    vol = W.tet_volumes(mesh.cell_vertices)
    qu = W.uniform_state(mesh.n_cells, rho=1.2, vel=(0.4, -0.9, 0.3), p=0.8)
    for prec in (hgks.FP64, hgks.FP32_MIXED, hgks.FP32):
        s = make_solver(mesh, qu, precision=prec)
        s.step(5)
        q, _ = s.get_state()
        tol = 1e-13 if prec == hgks.FP64 else 1e-6
        assert np.abs(q - qu).max() <= tol * np.abs(qu).max(), prec
        s.close()
    q0 = W.AdvectionCase(k=(2, 1, 1), vel=(0.3, 0.9, -0.6)).conservative(mesh)
    # conservation: exact up to FP64 rounding wherever the state and the face fluxes are
    # FP64; in the FP32 form each stored value is rounded to FP32
    for prec, tol in ((hgks.FP64, 1e-13), (hgks.FP32_MIXED, 1e-13), (hgks.FP32, 1e-6)):
        s = make_solver(mesh, q0, precision=prec)
        q_start, _ = s.get_state()
        s.step(5)
        q, _ = s.get_state()
        s.close()
        t0, t1 = (vol[:, None] * q_start).sum(0), (vol[:, None] * q).sum(0)
        assert np.all(np.abs(t1 - t0) <= tol * np.abs(vol[:, None] * q_start).sum(0)), (prec, t1 - t0)


def test_error_paths():
    say("case: error paths")
    mesh, case, q0 = advection_case(5, seed=112)
    s = hgks.Solver()
    with pytest.raises(hgks.HGKSError) as e:
        s.init_state(q0)
    assert e.value.status == hgks.E_STATE
    s.mesh_upload(mesh.nodes, mesh.cell_nodes, mesh.period)
    with pytest.raises(hgks.HGKSError) as e:
        s.step(1)
    assert e.value.status == hgks.E_STATE
    bad = q0.copy()
    bad[3, 0] = -1.0
    with pytest.raises(hgks.HGKSError) as e:
        s.init_state(bad)
    assert e.value.status == hgks.E_NONPHYSICAL
    s.init_state(q0)
    s.step(1, dt_fixed=50.0)                 # far past stability: the state blows up
    with pytest.raises(hgks.HGKSError) as e:
        s.get_state()
    assert e.value.status == hgks.E_NONPHYSICAL
    s.init_state(q0)                          # a fresh state clears the flag
    s.step(1)
    s.get_state()
    s.close()


def test_pool_alone_vs_mix_bitwise():
    """Continuous batching: each problem's result is bitwise the same alone and in a
    mixed pooled launch (different sizes, precisions and collision-time modes)."""
    say("case: pool alone vs mix")
    cases = [(6, 120, dict()), (8, 121, dict(precision=hgks.FP32_MIXED)), (5, 122, dict(tau_mode=1)),
             (7, 123, dict()), (6, 125, dict(precision=hgks.FP32)), (5, 126, dict(precision=hgks.FP32, tau_mode=1))]
    alone, solvers = [], []
    for n, seed, kw in cases:
        mesh, case, q0 = advection_case(n, seed=seed, vel=(0.7, 0.1, -0.5))
        s = make_solver(mesh, q0, **kw)
        s.step(3)
        alone.append(s.get_state()[0])
        s.close()
        solvers.append(make_solver(mesh, q0, **kw))
    pool = hgks.Pool()
    slots = [pool.add(s) for s in solvers]
    pool.step(slots, 1)
    pool.step(slots[::-1], 2)
    for k, s in enumerate(solvers):
        q, _ = s.get_state()
        assert np.array_equal(q, alone[k]), k
    used, n = pool.used()
    assert n == len(cases) and used == sum(s.footprint() for s in solvers)
    for sl in slots:
        pool.remove(sl)
    pool.close()
    for s in solvers:
        s.close()


def test_pool_admission_budget():
    say("case: pool budget")
    mesh, case, q0 = advection_case(5, seed=124)
    a = make_solver(mesh, q0)
    b = make_solver(mesh, q0)
    assert a.footprint() == hgks.pool_footprint(hgks.params(), mesh.n_cells)
    pool = hgks.Pool(hbm_budget=a.footprint() + b.footprint() // 2)
    pool.add(a)
    with pytest.raises(hgks.HGKSError) as e:
        pool.add(b)
    assert e.value.status == hgks.E_OOM
    pool.close()


def test_full_size_config2_sampled_parity():
    """6*64^3 = 1,572,864 tets in the launch configuration the benchmark times:
    one GPU step against the oracle's step of 48 sampled cells, plus the CFL dt."""
    say("case: fp64 N=64 sampled parity")
    mesh, case, q0 = advection_case(64, seed=W.SEED_ADVECTION + 64)
    s = make_solver(mesh, q0)
    dt_gpu = s.step(1, want_dt=True)
    q_gpu, _ = s.get_state()
    s.close()
    om = O.Mesh.from_workload(mesh)
    dt_orc = om.cfl_dt(q0)
    assert abs(dt_gpu - dt_orc) <= 1e-14 * dt_orc
    rng = np.random.default_rng(64)
    cells = np.concatenate([[0, mesh.n_cells - 1], rng.choice(mesh.n_cells, 46, replace=False)])
    ref = om.step_sample(q0, dt_orc, cells)
    e = scaled_err(q_gpu[cells], ref)
    say("worst scaled error (sample)", e)
    assert np.all(e <= TOL64), e


def test_full_size_config2_fp32_mixed_vs_fp64():
    """Config 2 in full: 100 steps at 6*64^3; FP32-mixed and FP32 against the FP64
    path, whose every step matches the oracle."""
    say("case: N=64 100 steps fp64 vs fp32-mixed and fp32")
    mesh, case, q0 = advection_case(64, seed=W.SEED_ADVECTION + 64)
    vol = W.tet_volumes(mesh.cell_vertices)
    out = {}
    for prec in (hgks.FP64, hgks.FP32_MIXED, hgks.FP32):
        s = make_solver(mesh, q0, precision=prec)
        s.step(100)
        out[prec] = s.get_state()
        s.close()
    for prec in (hgks.FP32_MIXED, hgks.FP32):
        err = rel_l1(out[prec][0], out[hgks.FP64][0], vol)
        say(f"relative L1 precision {prec} vs fp64 after 100 steps", err)
        assert np.all(err <= TOL32), err
        assert out[prec][1] == pytest.approx(out[hgks.FP64][1], rel=1e-5)


@pytest.mark.timeout(900)
def test_full_size_shock_tube_walls_sampled_parity():
    """The 128^3 shock tube with walls in full (12.6 M tets, tau_mode 1, the shock-tube
    driver's configuration): one GPU step against the oracle's step of 48 sampled
    cells (at both walls, across the diaphragm and at random), plus the CFL dt.  The
    oracle's mesh of this size takes about a minute and 55 GB of host memory."""
    say("case: fp64 shock tube 128^3 with walls, tau_mode=1, sampled parity (12.6 M cells)")
    mesh, case = W.sod_box(128, 128, 128, walls=True)
    q0 = case.conservative(mesh)
    s = make_solver(mesh, q0, tau_mode=1)
    dt_gpu = s.step(1, want_dt=True)
    q_gpu, _ = s.get_state()
    s.close()
    say("gpu step done; building the oracle mesh")
    om = O.Mesh.from_workload(mesh)
    dt_orc = om.cfl_dt(q0)
    assert abs(dt_gpu - dt_orc) <= 1e-14 * dt_orc, (dt_gpu, dt_orc)
    x = mesh.cell_vertices[:, :, 0].mean(axis=1)
    rng = np.random.default_rng(128)

    def pick(sel, k):
        return rng.choice(np.flatnonzero(sel), k, replace=False)

    cells = np.concatenate([pick(np.abs(x - 0.5) < 0.01, 16), pick(x < 0.01, 8), pick(x > 0.99, 8),
                            rng.choice(mesh.n_cells, 16, replace=False)])
    ref = om.step_sample(q0, dt_orc, cells, params=oracle_params(tau_mode=1))
    e = scaled_err(q_gpu[cells], ref)
    say("worst scaled error (sample)", e)
    assert np.all(e <= TOL64), e


# ---------------------------------------------------------------------------
# Shock tube: discontinuous data, the positivity fallback at Gauss points
# ---------------------------------------------------------------------------
def _sod(nx=32, ny=4, nz=4):
    mesh, case = W.sod_box(nx, ny, nz)
    return mesh, case.conservative(mesh)


@pytest.mark.parametrize("tau_mode", [0, 1])
def test_fp64_shock_tube_every_step(tau_mode):
    """Sod's tube from its discontinuous initial state: the first steps put
    non-physical reconstructed states at Gauss points next to the diaphragm, so
    the fallback path of the flux runs (the tau = 0 fix-up pass, the tau > 0
    inline check); each step matches the oracle."""
    say(f"case: fp64 shock tube nx=32 tau_mode={tau_mode} 6 steps")
    mesh, q0 = _sod()
    worst = per_step_parity(mesh, q0, 6, tau_mode=tau_mode)
    say("worst scaled error", worst)


def test_fp64_shock_tube_coloured_accumulation():
    say("case: fp64 shock tube coloured accumulation 3 steps")
    mesh, q0 = _sod(24, 4, 4)
    per_step_parity(mesh, q0, 3, accumulation=hgks.ACC_COLOURED)


def test_fp32_mixed_shock_tube_against_fp64():
    """FP32-mixed against FP64 on the tube to t = 0.1 (tau_mode 1): the rounding
    difference stays small next to the scheme's own error at the shock."""
    say("case: fp32-mixed and fp32 vs fp64 shock tube nx=48 to t=0.1")
    mesh, q0 = _sod(48, 4, 4)
    vol = W.tet_volumes(mesh.cell_vertices)
    out = {}
    for prec in (hgks.FP64, hgks.FP32_MIXED, hgks.FP32):
        s = make_solver(mesh, q0, precision=prec, tau_mode=1)
        t = 0.0
        while t < 0.1 - 1e-14:
            dt = s.step(1, want_dt=True)
            _, t = s.get_state()
        out[prec] = s.get_state()[0]
        s.close()
    for prec in (hgks.FP32_MIXED, hgks.FP32):
        e = rel_l1_scaled(out[prec], out[hgks.FP64], vol)
        say(f"precision {prec} vs fp64 relative L1 (momentum against a momentum scale)", e)
        assert np.all(np.isfinite(out[prec]))
        assert np.all(e < 1e-5), e


# ---------------------------------------------------------------------------
# Transmissive walls (non-periodic axes): mirror-image ghosts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tau_mode", [0, 1])
def test_fp64_walls_smooth_every_step(tau_mode):
    """Walls on x and y (edges, where members are images under two mirrors), a
    smooth state moving in every direction: each step matches the oracle."""
    say(f"case: fp64 walls on x and y, smooth state, tau_mode={tau_mode}, 4 steps")
    mesh = W.kuhn_box((6, 5, 4), (1.0, 0.9, 0.8), jitter=0.15, seed=4243, periodic=(False, False, True))
    per_step_parity(mesh, smooth_state(mesh, 11), 4, tau_mode=tau_mode)


def test_fp64_walls_shock_tube_every_step():
    say("case: fp64 shock tube with walls nx=16 tau_mode=1 6 steps")
    mesh, case = W.sod_box(16, 4, 4, walls=True)
    per_step_parity(mesh, case.conservative(mesh), 6, tau_mode=1)


def test_fp64_walls_coloured_accumulation():
    say("case: fp64 walls coloured accumulation 3 steps")
    mesh = W.kuhn_box((6, 5, 4), (1.0, 0.9, 0.8), jitter=0.15, seed=4244, periodic=(False, True, True))
    per_step_parity(mesh, smooth_state(mesh, 12), 3, accumulation=hgks.ACC_COLOURED)


def test_fp32_mixed_walls_shock_tube_against_fp64():
    say("case: fp32-mixed and fp32 vs fp64 shock tube with walls nx=32 to t=0.1")
    mesh, case = W.sod_box(32, 4, 4, walls=True)
    q0 = case.conservative(mesh)
    vol = W.tet_volumes(mesh.cell_vertices)
    out = {}
    for prec in (hgks.FP64, hgks.FP32_MIXED, hgks.FP32):
        s = make_solver(mesh, q0, precision=prec, tau_mode=1)
        t = 0.0
        while t < 0.1 - 1e-14:
            s.step(1, want_dt=True)
            t = s.get_time()
        out[prec] = s.get_state()[0]
        s.close()
    for prec in (hgks.FP32_MIXED, hgks.FP32):
        e = rel_l1_scaled(out[prec], out[hgks.FP64], vol)
        say(f"precision {prec} vs fp64 relative L1 (momentum against a momentum scale)", e)
        assert np.all(np.isfinite(out[prec]))
        assert np.all(e < 1e-5), e


def test_destroying_a_pooled_context_detaches_it():
    """A context closed while in a pool leaves the pool first: the pool's
    accounting drops it and the remaining slots keep stepping."""
    say("case: destroy a pooled context")
    mesh, case, q0 = advection_case(5, seed=127)
    a = make_solver(mesh, q0)
    b = make_solver(mesh, q0)
    ref = make_solver(mesh, q0)
    pool = hgks.Pool()
    sa = pool.add(a)
    sb = pool.add(b)
    with pytest.raises(hgks.HGKSError) as e:
        hgks.Pool().add(a)                    # one pool at a time
    assert e.value.status == hgks.E_INVALID_ARG
    pool.step([sa, sb], 1)
    a.close()
    assert pool.used() == (b.footprint(), 1)
    with pytest.raises(hgks.HGKSError):
        pool.step([sa, sb], 1)                # the freed slot is gone
    pool.step([sb], 1)
    ref.step(2)
    assert np.array_equal(b.get_state()[0], ref.get_state()[0])
    pool.close()
    b.step(1)                                 # out of the pool, the context steps alone again
    b.close()
    ref.close()
