"""Pressure-driven runs on the GPU (pressure faces with the Zou-He rule, K_app of
Eq. 18-19 at the local pressure) against the oracle's pressure mode.

Element by element after fixed steps (same tolerances as the body-force parity
tests), converged k of a uniform medium with pressure-dependent K (closed form
pinned in the oracle tests), and the paper's Sec. 3.2 layer cases: the GPU
reproduces the oracle's k of each case and its ordering (organic matter near the
outlet above organic matter near the inlet).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import kapp
from helpers import gpu_solver, random_case
from test_gpu_parity import _compare

pytestmark = pytest.mark.gpu


def _kp_table(seed, pin=0.2e6, pout=0.1e6, open_pore=True):
    """Random per-class K(P) coefficients of the size the shale classes have in lattice units."""
    rng = np.random.default_rng(seed)
    pm = 0.5 * (pin + pout)
    A = 10 ** rng.uniform(-3, -1, 256)
    B = A * rng.uniform(0.5, 5, 256) * pm
    C = np.where(rng.random(256) < 0.5, A * rng.uniform(0.1, 2, 256) * pm * 1.04, 0.0)
    b = np.where(C > 0, 0.25e-6, 0.0)
    if open_pore:
        A[0] = math.inf
    return A, B, C, b


@pytest.mark.parametrize("store", ["f64", "f32", "f32loc", "f16loc"])
def test_pressure_faces_constant_k(gpu, store):
    """D2Q9, pressure faces on x, constant K, wall nodes next to the faces, a body force too."""
    cls, eps, k, _ = random_case((36, 70), seed=41, wall_frac=0.06)
    pr = oracle.Pressure(axis=0, rho_in=1.0004, rho_out=0.9996)
    _compare(gpu, 9, cls, eps, k, None, store, 150, G=(0, 5e-6, 0), pressure=pr)


@pytest.mark.parametrize("store", ["f64", "f32", "f32loc", "f16loc"])
def test_pressure_faces_k_of_p_d2q9_y_axis(gpu, store):
    """D2Q9, pressure faces on y, K(P) per class (Eq. 18-19 form), tau != 1."""
    cls, eps, k, _ = random_case((66, 48), seed=42)
    A, B, C, b = _kp_table(42)
    pr = oracle.Pressure(axis=1, rho_in=1.0005, rho_out=0.9995, k_const=A, k_kn=B, k_surf=C, lang_b=b,
                         p_in=0.2e6, p_out=0.1e6)
    _compare(gpu, 9, cls, eps, k, None, store, 150, G=(0, 0, 0), tau=0.85, pressure=pr)


@pytest.mark.parametrize("store", ["f64", "f32", "f16loc"])
def test_pressure_faces_k_of_p_d3q19(gpu, store):
    """D3Q19, pressure faces on z, K(P), wall nodes."""
    cls, eps, k, _ = random_case((24, 12, 20), seed=43, wall_frac=0.04)
    A, B, C, b = _kp_table(43)
    pr = oracle.Pressure(axis=2, rho_in=1.0005, rho_out=0.9995, k_const=A, k_kn=B, k_surf=C, lang_b=b,
                         p_in=0.2e6, p_out=0.1e6)
    _compare(gpu, 19, cls, eps, k, None, store, 60, G=(0, 0, 0), pressure=pr)


def _solve_both(g, store, q, cls, eps, pr, tol, budget):
    prob = oracle.Problem(q=q, cls=cls, eps=eps, k=np.ones(256), f_eps=0.0, tau=1.0, G=(0, 0, 0),
                          precision="ext", pressure=pr)
    ref = oracle.solve(prob, tol=tol, max_steps=budget, check_every=100)
    s = gpu_solver(g, q, cls, eps, np.ones(256), store=store, G=(0, 0, 0), pressure=pr)
    try:
        rc = s.step(budget, tol=tol)
        kg = s.permeability()[0]
        r, st = s.residual()
    finally:
        s.close()
    a = pr.axis
    return ref.k[a], kg[a], ref.steps, st[0], rc, r[0]


@pytest.mark.parametrize("store,tol", [("f64", 1e-10), ("f32loc", 1e-5), ("f32", 1e-5)])
def test_uniform_medium_k_of_p_converged(gpu, store, tol):
    """Uniform medium with K(P): the converged k of the GPU equals the oracle's, which the
    oracle tests pin to the closed form of integral K(P) dP."""
    A, B, C, b = (np.full(256, math.inf), np.zeros(256), np.zeros(256), np.zeros(256))
    pm = 0.15e6
    A[1], B[1], C[1], b[1] = 0.01, 0.02 * pm, 0.015 * pm * (1 + 0.25e-6 * pm), 0.25e-6
    eps = np.ones(256)
    eps[1] = 0.3
    pr = oracle.Pressure(axis=0, rho_in=1 + 5e-5, rho_out=1 - 5e-5, k_const=A, k_kn=B, k_surf=C, lang_b=b,
                         p_in=0.2e6, p_out=0.1e6)
    cls = np.ones((4, 64), np.uint8)
    ko, kg, so, sg, rc, r = _solve_both(gpu, store, 9, cls, eps, pr, 1e-9, 200000)
    rel = abs(kg - ko) / ko
    print("store %s: k oracle %.12e gpu %.12e rel %.2e; steps %d / %d; r %.2e" % (store, ko, kg, rel, so, sg, r))
    assert rel <= tol


def _layered_case(case, nx=128, ny=8):
    """Sec. 3.2 cases 2 / 3: organic matter in the upstream (2) or downstream (3) half,
    Tab. 7 inputs (0.2 -> 0.1 MPa; porosities 0.02 / 0.04; q_sat 4000 mol/m^3; D_s 1e-8;
    b 0.25 1/MPa; tortuosity 2), OM pores 3 times smaller than IOM pores."""
    T, eta, tort, dx, b = 400.0, 18.231e-6, 2.0, 5e-9, 0.25e-6
    cls = np.ones((ny, nx), np.uint8)
    if case == 2:
        cls[:, :nx // 2] = 2
    else:
        cls[:, nx // 2:] = 2
    A, B, C, lb, e = (np.full(256, math.inf), np.zeros(256), np.zeros(256), np.zeros(256), np.ones(256))
    for c, r, ep, qs in ((1, 15e-9, 0.02, 0.0), (2, 5e-9, 0.04, 4000.0)):
        a_, b_, c_ = kapp.pressure_coefficients(r, T, ep, tort, eta, qs, b, 1e-8)
        A[c], B[c], C[c], lb[c], e[c] = a_ / dx ** 2, b_ / dx ** 2, c_ / dx ** 2, b, ep
    pr = oracle.Pressure(axis=0, rho_in=1 + 5e-5, rho_out=1 - 5e-5, k_const=A, k_kn=B, k_surf=C, lang_b=lb,
                         p_in=0.2e6, p_out=0.1e6)
    return cls, e, pr


@pytest.mark.parametrize("store,tol", [("f64", 1e-9), ("f32loc", 1e-5)])
def test_layer_cases_match_oracle_and_order(gpu, store, tol):
    """Both layer cases converge to the oracle's k, and case 3 > case 2 on the GPU as in
    the oracle and the paper (Sec. 3.2)."""
    ks = {}
    for case in (2, 3):
        cls, e, pr = _layered_case(case)
        ko, kg, so, sg, rc, r = _solve_both(gpu, store, 9, cls, e, pr, 1e-9, 400000)
        rel = abs(kg - ko) / ko
        print("case %d store %s: k oracle %.10e gpu %.10e rel %.2e; steps %d / %d; rc %d r %.2e" % (
            case, store, ko, kg, rel, so, sg, rc, r))
        assert rc == gpu.GLBM_OK
        assert rel <= tol
        ks[case] = kg
    print("case 3 / case 2 - 1 = %.3e" % (ks[3] / ks[2] - 1))
    assert ks[3] > ks[2]


@pytest.mark.parametrize("timing", [False, True])
@pytest.mark.parametrize("store", ["f64", "f32"])
@pytest.mark.parametrize("axis,shape,tile,walls", [(0, (36, 70), (64, 4), 0.06), (1, (66, 48), (64, 8), 0.0),
                                                   (0, (40, 130), (128, 4), 0.05), (1, (20, 50), (64, 4), 0.04),
                                                   (0, (9, 40), (64, 8), 0.0)])
def test_pressure_two_step_bitwise(gpu, store, axis, shape, tile, walls, timing):
    """Two time steps per launch under pressure faces (K(P) per class, with and without
    wall nodes, the faces on x or on y, tiles wider than the grid) gives the same bits as
    one step per launch, with graph replay or eager launches, over check intervals that
    are and are not multiples of 4 and runs that start off a check boundary."""
    g = gpu
    cls, eps, k, _ = random_case(shape, seed=77, wall_frac=walls)
    A, B, C, b = _kp_table(77)
    pr = oracle.Pressure(axis=axis, rho_in=1.0005, rho_out=0.9995, k_const=A, k_kn=B, k_surf=C, lang_b=b,
                         p_in=0.2e6, p_out=0.1e6)
    out = []
    for cache, every in ((13, 100), (77, 100), (79, 100), (13, 102), (77, 102), (69, 100), (71, 102), (65, 100)):
        print("case store=%s axis=%d shape=%s tile=%s walls=%.2f timing=%d cache=%d every=%d"
              % (store, axis, shape, tile, walls, timing, cache, every), flush=True)
        s = gpu_solver(g, 9, cls, eps, k, G=(0, 0, 0), store=store, tile=tile, cache=cache, check_every=every,
                       pressure=pr)
        assert g.glbm_sweeps_per_launch(s.ctx) == (2 if cache & 64 else 1)
        if timing:
            s.set_option(g.GLBM_OPT_TIMING, 1)
        s.step(2 * every)
        s.step(6)
        s.step(every)
        p = s.populations()
        r, st = s.residual()
        kk = s.permeability()[0]
        if timing:
            ms, nl = g.glbm_sweep_time(s.ctx)
            assert nl == 3 * every + 6
        s.close()
        out.append((p, r[0], st[0], kk[axis]))
    for a, b2 in ((0, 1), (0, 2), (3, 4), (0, 5), (3, 6), (0, 7)):
        assert np.array_equal(out[a][0], out[b2][0])
        assert out[a][1:] == out[b2][1:]


def test_pressure_argument_errors(gpu):
    """Pressure faces with walls on another axis, equal densities or a one-node axis are
    rejected; glbm_set_pressure_perm needs pressure faces; F_eps > 0 is rejected."""
    g = gpu
    cls = np.ones((8, 16), np.uint8)
    for kw in (dict(pressure_axis=0, rho_in=1.0, rho_out=1.0), dict(pressure_axis=0, wall_faces=0b1100),
               dict(pressure_axis=2)):
        args = dict(rho_in=1.001, rho_out=0.999)
        args.update(kw)
        with pytest.raises(g.GlbmError):
            g.Solver([g.make_desc(cls.shape, **args)], [cls])
    s = g.Solver([g.make_desc(cls.shape)], [cls])
    with pytest.raises(g.GlbmError):
        s.set_pressure_perm(np.ones(2), np.ones(2), np.zeros(2), np.zeros(2), np.zeros(2), 2e5, 1e5)
    s.close()
    s = g.Solver([g.make_desc(cls.shape, pressure_axis=0, rho_in=1.001, rho_out=0.999)], [cls])
    with pytest.raises(g.GlbmError):
        s.set_local_perm(np.ones(2), np.full(2, 0.1), np.full(2, 0.5))
    s.close()
