"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test fixes a part of the oracle against mathematics or the paper:
closed forms of the steady state (uniform Darcy medium, Poiseuille, Brinkman
channel), conservation laws of the lattice Boltzmann step, the moments that
Eq. (30)-(31) must have, and brute-force properties of streaming on tiny
grids.  A plausible slip (a dropped 1/eps, a wrong sign, a transposed index, a
misplaced bounce-back) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def uniform_problem(shape, eps, K, tau=1.0, G=(1e-6, 0, 0), walls=0, q=9, f_eps=0.0, precision="ext"):
    cls = np.ones(shape, np.uint8)
    e = np.ones(256)
    k = np.full(256, math.inf)
    e[1] = eps
    k[1] = K
    fe = np.zeros(256)
    fe[1] = f_eps
    return oracle.Problem(q=q, cls=cls, eps=e, k=k, f_eps=fe, tau=tau, G=G, walls=walls,
                          precision=precision)


# ---------------------------------------------------------------- lattice --
@pytest.mark.parametrize("q", [9, 19])
def test_lattice_isotropy(q):
    """Weights sum to 1; first and third moments vanish; second moment c_s^2 = 1/3;
    fourth moment is the isotropic (1/9)(d_ab d_cd + d_ac d_bd + d_ad d_bc)."""
    e, w, opp = oracle.lattice(q)
    dim = 2 if q == 9 else 3
    e = e[:, :dim].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ e).max() < 1e-15
    m2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(m2, np.eye(dim) / 3, atol=1e-15)
    m3 = np.einsum("i,ia,ib,ic->abc", w, e, e, e)
    assert np.abs(m3).max() < 1e-15
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    I = np.eye(dim)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I) + np.einsum("ad,bc->abcd", I, I)) / 9
    assert np.allclose(m4, iso, atol=1e-15)
    for i in range(q):
        assert np.all(e[opp[i]] == -e[i])


# ------------------------------------------------- equilibrium and forcing --
@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    """Eq. (30): sum feq = rho, sum feq e = rho u, sum feq e e = rho u u / eps + rho/3 I."""
    e, w, _ = oracle.lattice(q)
    rho, u, eps = 1.013, np.array([3e-3, -2e-3, 1e-3 if q == 19 else 0.0]), 0.37
    feq, _ = oracle.feq_force(q, rho, u, np.zeros(3), eps, 1.0)
    ef = e.astype(float)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(feq @ ef - rho * u).max() < 2e-16
    dim = 2 if q == 9 else 3
    m2 = np.einsum("i,ia,ib->ab", feq, ef, ef)[:dim, :dim]
    want = rho * np.outer(u, u)[:dim, :dim] / eps + rho / 3 * np.eye(dim)
    assert np.abs(m2 - want).max() < 2e-15


@pytest.mark.parametrize("q", [9, 19])
def test_forcing_moments(q):
    """Eq. (31) with the 1/eps reading: sum F_i = 0 (no mass source) and
    sum F_i e_i = (1 - 1/(2 tau)) rho F."""
    e, w, _ = oracle.lattice(q)
    rho, eps, tau = 0.998, 0.3, 1.0
    u = np.array([1e-3, 2e-4, -3e-4 if q == 19 else 0.0])
    F = np.array([1e-5, -3e-6, 2e-6 if q == 19 else 0.0])
    _, fi = oracle.feq_force(q, rho, u, F, eps, tau)
    assert abs(fi.sum()) < 5e-21
    assert np.abs(fi @ e.astype(float) - (1 - 0.5 / tau) * rho * F).max() < 5e-21


def test_printed_forcing_term_creates_mass():
    """The forcing term as printed (last term without 1/eps) is not mass
    conserving for eps < 1: sum_i F_i = 3 rho (1 - 1/(2 tau)) (u.F)(1/eps - 1).
    The oracle's reading differs from it by exactly that term, spread as w_i."""
    q, rho, eps, tau = 9, 1.0, 0.3, 1.0
    u = np.array([1e-3, 2e-4, 0.0])
    F = np.array([1e-5, -3e-6, 0.0])
    _, w, _ = oracle.lattice(q)
    _, fi = oracle.feq_force(q, rho, u, F, eps, tau)
    printed = fi + w * rho * (1 - 0.5 / tau) * (3 / eps - 3) * (u @ F)
    assert abs(printed.sum() - 3 * rho * (1 - 0.5 / tau) * (u @ F) * (1 / eps - 1)) < 1e-20
    assert abs(printed.sum()) > 1e-9


@pytest.mark.parametrize("q", [9, 19])
def test_collision_conserves_mass_and_adds_force(q):
    """One collision: sum f* = sum f; sum f* e = sum f e + rho F (Eq. 29 with Eq. 33)."""
    rng = np.random.default_rng(4)
    e, w, _ = oracle.lattice(q)
    f = w * (1 + 1e-3 * rng.standard_normal(q))
    G = np.array([1e-4, 2e-5, 3e-5 if q == 19 else 0.0])
    for eps, kinv, fe in ((1.0, 0.0, 0.0), (0.4, 30.0, 0.0), (0.2, 400.0, 0.9)):
        fo, rho, u, F = oracle.collide_node(q, f, eps, kinv, fe, 0.8, G)
        assert abs(fo.sum() - f.sum()) < 1e-15
        j0 = f @ e.astype(float)
        j1 = fo @ e.astype(float)
        assert np.abs(j1 - j0 - rho * F).max() < 5e-16
        # Eq. (33): rho u = sum f e + rho F / 2, with F evaluated at u
        assert np.abs(rho * u - j0 - 0.5 * rho * F).max() < 5e-16


def test_velocity_root_of_quadratic():
    """Eq. (34)-(37): u solves u = v - (1/2)(eps nu / K) u - (1/2)(eps F_eps / sqrt K)|u| u."""
    q, tau = 9, 1.0
    nu = (tau - 0.5) / 3
    e, w, _ = oracle.lattice(q)
    rng = np.random.default_rng(7)
    f = w * (1 + 1e-2 * rng.standard_normal(q))
    eps, K, fe = 0.35, 0.02, 1.3
    G = np.array([2e-3, -1e-3, 0.0])
    _, rho, u, F = oracle.collide_node(q, f, eps, 1 / K, fe, tau, G)
    v = (f @ e.astype(float)) / rho + 0.5 * eps * G
    resid = u - v + 0.5 * eps * nu / K * u + 0.5 * eps * fe / math.sqrt(K) * np.linalg.norm(u) * u
    assert np.abs(resid).max() < 1e-17


# ------------------------------------------------------------ streaming --
def test_streaming_is_a_permutation_brute_force():
    """With tau = 1, F = 0 and a node state at exact equilibrium replaced by
    labelled values, one step moves value (i, x) to (i, x + e_i) periodically:
    checked node by node against a brute-force shift on a 5x4 grid."""
    q = 9
    e, w, opp = oracle.lattice(q)
    ny, nx = 4, 5
    cls = np.ones((ny, nx), np.uint8)
    p = oracle.Problem(q=q, cls=cls, eps=1.0, k=math.inf, f_eps=0.0, tau=1e9, G=(0, 0, 0),
                       precision="ext")
    # huge tau: collision is (almost) the identity; labels are tiny perturbations on w
    rng = np.random.default_rng(0)
    lab = rng.random((q, ny, nx)) * 1e-6
    f = (w[:, None, None] * (1 + lab)).reshape(-1)
    out = p.step(f).reshape(q, ny, nx)
    fin = f.reshape(q, ny, nx)
    for i in range(q):
        want = np.roll(np.roll(fin[i], e[i, 1], axis=0), e[i, 0], axis=1)
        assert np.abs(out[i] - want).max() < 1e-12 * w[i]


def test_bounce_back_brute_force():
    """Walls at the y faces: a population moving in -y at y = 0 comes back at
    the same node in +y (halfway bounce-back), and likewise at y = ny - 1."""
    q = 9
    e, w, opp = oracle.lattice(q)
    ny, nx = 3, 4
    cls = np.ones((ny, nx), np.uint8)
    p = oracle.Problem(q=q, cls=cls, eps=1.0, k=math.inf, f_eps=0.0, tau=1e9, G=(0, 0, 0),
                       walls=0b1100, precision="ext")
    rng = np.random.default_rng(1)
    f = (w[:, None, None] * (1 + 1e-6 * rng.random((q, ny, nx)))).reshape(-1)
    out = p.step(f).reshape(q, ny, nx)
    fin = f.reshape(q, ny, nx)
    for i in range(q):
        if e[i, 1] == 0:
            continue
        y = 0 if e[i, 1] < 0 else ny - 1
        j = opp[i]
        for x in range(nx):
            assert abs(out[j, y, x] - fin[i, y, x]) < 1e-12


@pytest.mark.parametrize("q,shape,walls", [(9, (24, 30), 0), (9, (20, 26), 0b1100), (19, (6, 8, 10), 0b001111)])
def test_mass_conservation(q, shape, walls):
    """Sum of all populations is invariant (periodic faces, halfway bounce-back,
    wall nodes, eps < 1 classes) — fails with the printed form of Eq. (31)."""
    rng = np.random.default_rng(3)
    cls = rng.integers(0, 5, size=shape).astype(np.uint8)
    cls[rng.random(shape) < 0.1] = 255
    eps = np.concatenate([[1.0], rng.uniform(0.1, 0.9, 255)])
    k = np.concatenate([[math.inf], 10 ** rng.uniform(-3, -1, 255)])
    G = (3e-5, -2e-5, 1e-5) if q == 19 else (3e-5, -2e-5, 0)
    p = oracle.Problem(q=q, cls=cls, eps=eps, k=k, f_eps=0.0, tau=0.9, G=G, walls=walls, precision="ext")
    f = p.rest()
    m0 = f.reshape(q, -1)[:, p.fluid].sum()
    p.run(f, 400)
    m1 = f.reshape(q, -1)[:, p.fluid].sum()
    assert abs(m1 - m0) / m0 < 1e-15


@pytest.mark.parametrize("mode,scale,tol", [(3, 24, 4e-3), (4, 0, 3e-5), (5, 24, 4e-3)])
def test_storage_emulation_modes(mode, scale, tol):
    """The reduced-precision storage emulations (local-density forms: FP16 parts with an
    FP32 density, FP32 parts, FP16 parts with an FP16 density scaled by 2^10) stay within
    their storage tolerance of the plain FP64 oracle and keep the total mass up to the
    rounding of the stored parts.  A dropped w_i rho term or a wrong scale is off by many
    orders of magnitude."""
    rng = np.random.default_rng(12)
    shape = (24, 34)
    cls = rng.integers(0, 6, size=shape).astype(np.uint8)
    eps = np.concatenate([[1.0], rng.uniform(0.1, 0.9, 255)])
    k = np.concatenate([[math.inf], 10 ** rng.uniform(-3, -1, 255)])
    G = (2e-5, 1e-5, 0)
    runs = {}
    for m, sc in ((0, 0), (mode, scale)):
        p = oracle.Problem(q=9, cls=cls, eps=eps, k=k, f_eps=0.0, tau=1.0, G=G, store_mode=m, scale_log2=sc)
        f = p.rest()
        p.run(f, 300)
        runs[m] = f.reshape(9, -1)
    _, w = oracle.lattice(9)[:2]
    dev = np.abs(runs[0] - np.asarray(w)[:, None]).max()
    err = np.abs(runs[mode] - runs[0]).max()
    assert dev > 1e-6
    assert 0 < err <= tol * dev
    assert abs(runs[mode].sum() - runs[0].sum()) <= 1e-3 * tol * dev * runs[0].size


# ------------------------------------------------------ steady closed forms --
@pytest.mark.parametrize("eps,K", [(0.4, 0.01), (0.1, 1e-3), (1.0, 0.5)])
def test_uniform_medium_darcy(eps, K):
    """P1: a uniform porous medium relaxes to F = 0, i.e. u = K G / nu and the
    Darcy read-off returns K exactly."""
    p = uniform_problem((6, 8), eps, K)
    sol = oracle.solve(p, tol=0.0, max_steps=3000, check_every=100, stop_at=3000)
    assert abs(sol.k[0] - K) / K < 1e-12
    nu = p.nu
    assert np.abs(sol.u[0] - K * 1e-6 / nu).max() / (K * 1e-6 / nu) < 1e-12


def test_uniform_medium_forchheimer_root():
    """With F_eps > 0 the uniform steady velocity solves
    (eps nu / K) u + (eps F_eps / sqrt K) u^2 = eps G."""
    eps, K, fe, G = 0.5, 0.05, 1.2, 2e-3
    p = uniform_problem((4, 6), eps, K, G=(G, 0, 0), f_eps=fe)
    sol = oracle.solve(p, tol=0.0, max_steps=4000, check_every=100, stop_at=4000)
    a = eps * fe / math.sqrt(K)
    b = eps * p.nu / K
    u = (-b + math.sqrt(b * b + 4 * a * eps * G)) / (2 * a)
    assert abs(sol.u[0].mean() - u) / u < 1e-12


def _poiseuille(H, tau, walls_axis=1, q=9):
    nx = 4
    if q == 9:
        shape, walls, G = (H, nx), 0b1100, (1e-6, 0, 0)
    else:
        shape, walls, G = (4, H, nx), 0b1100, (1e-6, 0, 0)
    cls = np.zeros(shape, np.uint8)
    p = oracle.Problem(q=q, cls=cls, eps=1.0, k=math.inf, f_eps=0.0, tau=tau, G=G, walls=walls,
                       precision="ext")
    steps = int(6 * H * H / p.nu) + 1000
    sol = oracle.solve(p, tol=1e-13, max_steps=steps, check_every=100)
    u = sol.u[0].reshape(shape)
    prof = u[:, 0] if q == 9 else u[0, :, 0]
    y = np.arange(H) + 0.5
    exact = 1e-6 / (2 * p.nu) * y * (H - y)
    return prof, exact


@pytest.mark.parametrize("q", [9, 19])
def test_poiseuille_exact_at_magic_tau(q):
    """P4: force-driven Poiseuille flow with halfway bounce-back walls is exact
    (parabola with the wall half a link outside the last node) at
    tau = 1/2 + sqrt(3/16)."""
    prof, exact = _poiseuille(16, 0.5 + math.sqrt(3 / 16), q=q)
    assert np.abs(prof - exact).max() / exact.max() < 1e-10


def test_poiseuille_second_order():
    """P4 at tau = 1: the error decays as H^-2."""
    errs = []
    for H in (8, 16, 32):
        prof, exact = _poiseuille(H, 1.0)
        errs.append(np.abs(prof - exact).max() / exact.max())
    order = math.log(errs[0] / errs[2], 4)
    assert 1.8 < order < 2.2, errs


def test_brinkman_channel():
    """P5: uniform porous channel between walls, steady profile of the
    generalized NS equation (Eq. 26 with Eq. 28, nu_e = nu):
    u = (K G / nu) [1 - cosh(s (y - H/2)) / cosh(s H / 2)],  s = sqrt(eps / K)."""
    errs = []
    for H in (16, 32, 64):
        eps = 0.5
        s_H = 6.0
        K = eps * (H / s_H) ** 2
        shape = (H, 4)
        cls = np.ones(shape, np.uint8)
        e = np.ones(256)
        k = np.full(256, math.inf)
        e[1], k[1] = eps, K
        p = oracle.Problem(q=9, cls=cls, eps=e, k=k, f_eps=0.0, tau=1.0, G=(1e-6, 0, 0), walls=0b1100,
                           precision="ext")
        sol = oracle.solve(p, tol=1e-13, max_steps=400000, check_every=100)
        u = sol.u[0].reshape(shape)[:, 0]
        y = np.arange(H) + 0.5
        s = math.sqrt(eps / K)
        exact = K * 1e-6 / p.nu * (1 - np.cosh(s * (y - H / 2)) / np.cosh(s * H / 2))
        errs.append(np.sqrt(np.sum((u - exact) ** 2) / np.sum(exact ** 2)))
    assert errs[1] < 1e-3, errs
    order = math.log(errs[0] / errs[2], 4)
    assert 1.6 < order < 2.4, errs


def test_force_balance_at_steady_state():
    """P3: in a periodic domain the total momentum source sum_x rho F vanishes
    at steady state (drag balances the body force)."""
    rng = np.random.default_rng(9)
    shape = (24, 24)
    cls = rng.integers(0, 4, size=shape).astype(np.uint8)
    eps = np.array([1.0, 0.3, 0.5, 0.2] + [1.0] * 252)
    k = np.array([math.inf, 0.05, 0.2, 0.01] + [math.inf] * 252)
    p = oracle.Problem(q=9, cls=cls, eps=eps, k=k, f_eps=0.0, tau=1.0, G=(1e-6, 0, 0), precision="ext")
    sol = oracle.solve(p, tol=1e-12, max_steps=300000, check_every=100)
    e_n = eps[cls.reshape(-1)]
    kinv = np.where(np.isinf(k), 0.0, 1.0 / k)[cls.reshape(-1)]
    Fx = e_n * (1e-6 - p.nu * kinv * sol.u[0])
    src = np.sum(sol.rho * Fx)
    assert abs(src) / np.sum(sol.rho * e_n * 1e-6) < 1e-8


def test_layered_medium_parallel_flow():
    """P6: layers parallel to the drive, Darcy limit (K << layer width^2):
    k tends to the thickness-weighted mean of K."""
    ny, nx = 40, 4
    cls = np.ones((ny, nx), np.uint8)
    cls[ny // 2:] = 2
    eps = np.ones(256)
    k = np.full(256, math.inf)
    eps[1], k[1] = 0.5, 0.01
    eps[2], k[2] = 0.5, 0.04
    p = oracle.Problem(q=9, cls=cls, eps=eps, k=k, f_eps=0.0, tau=1.0, G=(1e-6, 0, 0), precision="ext")
    sol = oracle.solve(p, tol=1e-12, max_steps=200000, check_every=100)
    kmean = 0.5 * (0.01 + 0.04)
    # Brinkman boundary layers of width sqrt(K/eps) at the two interfaces
    assert abs(sol.k[0] - kmean) / kmean < 2 * math.sqrt(0.04 / 0.5) / (ny / 2)


def test_linearity_in_G():
    """P8: halving G leaves k unchanged to O(Re^2)."""
    rng = np.random.default_rng(2)
    cls = rng.integers(0, 3, size=(16, 16)).astype(np.uint8)
    eps = np.array([1.0, 0.3, 0.5] + [1.0] * 253)
    k = np.array([math.inf, 0.02, 0.1] + [math.inf] * 253)
    ks = []
    for G in (1e-6, 5e-7):
        p = oracle.Problem(q=9, cls=cls, eps=eps, k=k, f_eps=0.0, tau=1.0, G=(G, 0, 0), precision="ext")
        ks.append(oracle.solve(p, tol=1e-12, max_steps=200000, check_every=100).k[0])
    assert abs(ks[0] - ks[1]) / ks[0] < 1e-6


def test_translation_invariance():
    """Cyclic shift of a periodic geometry gives the same k (to rounding)."""
    rng = np.random.default_rng(5)
    cls = rng.integers(0, 3, size=(12, 18)).astype(np.uint8)
    eps = np.array([1.0, 0.3, 0.5] + [1.0] * 253)
    k = np.array([math.inf, 0.02, 0.1] + [math.inf] * 253)
    out = []
    for c in (cls, np.roll(np.roll(cls, 5, 0), 7, 1)):
        p = oracle.Problem(q=9, cls=c, eps=eps, k=k, f_eps=0.0, tau=1.0, G=(1e-6, 0, 0), precision="ext")
        out.append(oracle.solve(p, tol=0, max_steps=3000, check_every=100, stop_at=3000).k[0])
    assert abs(out[0] - out[1]) / out[0] < 1e-13


def test_fp64_and_extended_builds_agree():
    """The FP64 oracle and the extended-precision build of the same source agree
    to the FP64 cancellation floor."""
    rng = np.random.default_rng(6)
    cls = rng.integers(0, 3, size=(16, 20)).astype(np.uint8)
    eps = np.array([1.0, 0.3, 0.5] + [1.0] * 253)
    k = np.array([math.inf, 0.02, 0.1] + [math.inf] * 253)
    ks = []
    for prec in ("f64", "ext"):
        p = oracle.Problem(q=9, cls=cls, eps=eps, k=k, f_eps=0.0, tau=1.0, G=(1e-6, 0, 0), precision=prec)
        ks.append(oracle.solve(p, tol=0, max_steps=2000, check_every=100, stop_at=2000).k[0])
    assert abs(ks[0] - ks[1]) / ks[1] < 1e-9


# ------------------------------------------- residual, rounding, storage --
@pytest.mark.parametrize("q,shape", [(9, (6, 10)), (19, (4, 5, 6))])
def test_residual_open_pore_closed_form(q, shape):
    """R8 residual against a closed form.  In a periodic domain of open pore
    (eps = 1, K = inf) the body force is the only momentum source, so the
    momentum grows by rho G per step and the velocity of Eq. (34) after t steps
    from rest is u(t) = G (t + 1/2).  Then r(t) = ||u(t) - u(t - n_c)|| /
    (n_c ||u(t)||) = 1 / (t + 1/2) exactly, at every check, for both the C
    residual (the solve's history) and Problem.residual."""
    cls = np.zeros(shape, np.uint8)
    G = (3e-6, -2e-6, 1e-6 if q == 19 else 0.0)
    p = oracle.Problem(q=q, cls=cls, eps=1.0, k=math.inf, f_eps=0.0, tau=0.9, G=G, precision="ext")
    nc, n = 100, 1000
    sol = oracle.solve(p, tol=0, max_steps=n, check_every=nc, stop_at=n)
    t = np.arange(nc, n + 1, nc)
    assert len(sol.history) == len(t)
    hist = np.array([h for _, h in sol.history])
    assert np.all(np.abs(hist * (t + 0.5) - 1.0) < 1e-12)
    assert np.allclose(sol.u[:, 0] / (n + 0.5), np.asarray(G), rtol=1e-12, atol=0)
    f = p.rest()
    p.run(f, n - nc)
    _, u0 = p.fields(f)
    p.run(f, nc)
    _, u1 = p.fields(f)
    assert abs(p.residual(u1, u0, nc) * (n + 0.5) - 1.0) < 1e-12


def _half_cases():
    rng = np.random.default_rng(2024)
    # random magnitudes across the whole half range, subnormals and beyond the top
    a = rng.uniform(-1, 1, 60000) * 2.0 ** rng.uniform(-27, 17, 60000)
    # exact ties: odd multiples of half a half-precision quantum in every binade
    e = rng.integers(-14, 16, 20000)
    m = rng.integers(1024, 2048, 20000)
    ties = (2 * m + 1) * 2.0 ** (e - 11.0)
    sub = (2 * rng.integers(0, 1024, 10000) + 1) * 2.0 ** -25          # subnormal ties
    near = 2.0 ** rng.integers(-24, 16, 10000) * (1 + rng.uniform(-1e-3, 1e-3, 10000))
    edge = np.array([65504.0, 65519.0, 65519.999, 65520.0, 65535.0, 65536.0, 1e6, 2.0 ** -24, 2.0 ** -25,
                     2.0 ** -25 * 1.0000001, 2.0 ** -26, 6.0e-8, 0.0, -0.0, 1.0, 2049.0, 2051.0])
    x = np.concatenate([a, ties, -ties, sub, -sub, near, edge, -edge])
    return x


def test_round_half_matches_numpy_float16():
    """The oracle's FP16 rounding (used by the FP16 storage emulations) equals
    IEEE binary16 round-to-nearest-even as NumPy implements it, bit for bit:
    random values over the whole range, exact ties in every binade, subnormals
    (quantum 2^-24) and the overflow edge (65504 stays, 65520 and above go to
    infinity)."""
    x = _half_cases()
    want = x.astype(np.float16).astype(np.float64)
    got = oracle.round_half(x)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert np.all(same), x[~same][:10]
    assert np.array_equal(np.signbit(got), np.signbit(want))


@pytest.mark.parametrize("scale", [0, 20, 24])
def test_store_round_modes_1_and_2(scale):
    """Storage emulation modes 1 and 2 against NumPy's FP32 and FP16 conversions:
    mode 1 keeps w + fp32(f - w), mode 2 keeps w + fp16((f - w) 2^s) 2^-s."""
    rng = np.random.default_rng(7 + scale)
    w = np.array([4 / 9, 1 / 9, 1 / 36])
    for _ in range(3000):
        wi = w[rng.integers(0, 3)]
        f = wi + rng.uniform(-1, 1) * 10.0 ** rng.uniform(-14, -2)
        want1 = float(np.float32(f - wi)) + wi
        want2 = float(np.float16((f - wi) * 2.0 ** scale)) / 2.0 ** scale + wi
        assert oracle.store_round(f, wi, 1) == want1
        assert oracle.store_round(f, wi, 2, scale) == want2


@pytest.mark.parametrize("mode,scale,tol", [(1, 0, 3e-5), (2, 20, 4e-3)])
def test_storage_emulation_modes_deviation_forms(mode, scale, tol):
    """Whole runs in storage modes 1 (FP32 deviations f - w) and 2 (FP16
    deviations (f - w) 2^s) stay within their storage tolerance of the plain
    oracle; a wrong scale or a dropped weight is off by orders of magnitude."""
    rng = np.random.default_rng(12)
    shape = (24, 34)
    cls = rng.integers(0, 6, size=shape).astype(np.uint8)
    eps = np.concatenate([[1.0], rng.uniform(0.1, 0.9, 255)])
    k = np.concatenate([[math.inf], 10 ** rng.uniform(-3, -1, 255)])
    G = (2e-5, 1e-5, 0)
    runs = {}
    for m, sc in ((0, 0), (mode, scale)):
        p = oracle.Problem(q=9, cls=cls, eps=eps, k=k, f_eps=0.0, tau=1.0, G=G, store_mode=m, scale_log2=sc)
        f = p.rest()
        p.run(f, 300)
        runs[m] = f.reshape(9, -1)
    _, w = oracle.lattice(9)[:2]
    dev = np.abs(runs[0] - np.asarray(w)[:, None]).max()
    err = np.abs(runs[mode] - runs[0]).max()
    assert dev > 1e-6
    assert 0 < err <= tol * dev
