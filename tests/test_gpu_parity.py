"""GPU path vs the CPU oracle, element by element on the same seeded inputs.

Every case builds one problem twice: as an oracle.Problem (extended-precision
oracle unless stated) and as a GPU context through the C ABI, runs the same
number of steps from rest, and compares populations and fields.

Tolerances, relative to the largest population deviation max|f - w| of the
oracle state:
  F64 storage    1e-11  (FP64 arithmetic, different summation order)
  F32 storage    3e-5   (FP32 arithmetic: ~6e-8 per operation, a few hundred steps)
  F16DEV / F16LOC storage 4e-3 vs the oracle that rounds every stored value
                 through FP16 the same way (a rounding tie may break
                 differently in FP32 than in FP64, a 2^-11 step that then
                 diffuses)
"""
import numpy as np
import pytest

import oracle
import shale_inputs as si
from helpers import gpu_solver, oracle_order, oracle_problem, random_case

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 3e-5, "f16dev": 4e-3, "f16loc": 4e-3, "f32loc": 3e-5}


def _compare(g, q, cls, eps, k, fe, store, steps, G, walls=0, tau=1.0, tile=None, cache=None, scale=20,
             pressure=None):
    print("case q=%d shape=%s store=%s steps=%d walls=%d tile=%s cache=%s pressure=%s" % (
        q, cls.shape, store, steps, walls, tile, cache, None if pressure is None else pressure.axis), flush=True)
    if store == "f16loc" and scale == 20:
        scale = 24
    emul = {"f64": (0, 0), "f32": (0, 0), "f16dev": (2, scale), "f16loc": (3, scale), "f32loc": (4, 0)}[store]
    prob = oracle_problem(q, cls, eps, k, fe, tau=tau, G=G, walls=walls, store_mode=emul[0],
                          scale_log2=emul[1], pressure=pressure)
    f = prob.rest()
    prob.run(f, steps)
    rho_o, u_o = prob.fields(f)
    s = gpu_solver(g, q, cls, eps, k, fe, tau=tau, G=G, walls=walls, store=store, tile=tile, cache=cache,
                   scale_log2=scale if store in ("f16dev", "f16loc") else None, pressure=pressure)
    try:
        s.step(steps)
        fg = s.populations()
        rho_g, u_g = s.fields()
        _, st = s.residual()
    finally:
        s.close()
    assert st[0] == steps
    perm = oracle_order(q, g)
    fo = f.reshape(q, -1)[perm]
    _, w = g.glbm_velocity_set(q)
    fluid = cls.reshape(-1) != 255
    dev = np.abs(fo[:, fluid] - w[:, None]).max()
    err = np.abs(fg[:, fluid] - fo[:, fluid]).max()
    uerr = np.abs(u_g[:, fluid] - u_o[:, fluid]).max() / np.abs(u_o[:, fluid]).max()
    print("  max dev %.3e  pop err %.3e (rel %.3e)  u rel err %.3e" % (dev, err, err / dev, uerr), flush=True)
    assert dev > 0
    assert err <= TOL[store] * dev
    assert uerr <= 10 * TOL[store]
    if store not in ("f16dev", "f16loc", "f32loc"):
        assert np.abs(rho_g[fluid] - rho_o[fluid]).max() <= TOL[store] * dev * q


@pytest.mark.parametrize("store", ["f64", "f32", "f16dev", "f16loc", "f32loc"])
@pytest.mark.parametrize("shape", [(48, 64), (37, 100)])
def test_d2q9_periodic_fixed_steps(gpu, store, shape):
    cls, eps, k, fe = random_case(shape, seed=11 + shape[1])
    _compare(gpu, 9, cls, eps, k, None, store, 120, G=(2e-5, 7e-6, 0))


@pytest.mark.parametrize("store", ["f64", "f32", "f16loc", "f32loc"])
def test_d2q9_walls_and_wall_nodes(gpu, store):
    cls, eps, k, fe = random_case((40, 70), seed=5, wall_frac=0.12)
    _compare(gpu, 9, cls, eps, k, None, store, 150, G=(3e-5, -1e-5, 0), walls=0b1100)


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_d2q9_tile_shapes_and_cache_policies(gpu, store):
    """Results do not depend on the tile shape or the cache policy (ragged tiles included)."""
    cls, eps, k, fe = random_case((70, 130), seed=8)
    for tile, cache in (((64, 4), 0), ((128, 2), 1), ((256, 1), 2), ((1024, 1), 3), ((256, 16), 13),
                        ((512, 2), 9), ((64, 8), 15)):
        _compare(gpu, 9, cls, eps, k, None, store, 60, G=(2e-5, 0, 0), tile=tile, cache=cache)


@pytest.mark.parametrize("store", ["f64", "f32", "f32loc", "f16loc"])
def test_d2q9_forchheimer(gpu, store):
    """Eq. (27) with F_eps > 0: the velocity is the root of Eq. (34) with c1 > 0 (Eq. 37)."""
    cls, eps, k, fe = random_case((32, 64), seed=21)
    fe = np.full(256, 0.7)
    fe[0] = 0.0
    _compare(gpu, 9, cls, eps, k, fe, store, 100, G=(5e-4, 1e-4, 0))


@pytest.mark.parametrize("store", ["f64", "f32", "f32loc", "f16loc"])
def test_d2q9_tau(gpu, store):
    cls, eps, k, fe = random_case((33, 64), seed=4)
    _compare(gpu, 9, cls, eps, k, None, store, 100, G=(2e-5, 0, 0), tau=0.8)


@pytest.mark.parametrize("store", ["f64", "f32", "f16loc"])
def test_d3q19_forchheimer_walls(gpu, store):
    """D3Q19 with Forchheimer classes, tau != 1, face walls and wall nodes."""
    cls, eps, k, fe = random_case((10, 14, 40), seed=33, wall_frac=0.05)
    fe = np.full(256, 0.5)
    fe[0] = 0.0
    _compare(gpu, 19, cls, eps, k, fe, store, 60, G=(1e-4, 0, 4e-4), walls=0b001111, tau=0.9)


@pytest.mark.parametrize("store", ["f64", "f32", "f16dev", "f16loc", "f32loc"])
def test_d3q19_walls(gpu, store):
    cls, eps, k, fe = random_case((12, 20, 70), seed=31, wall_frac=0.05)
    _compare(gpu, 19, cls, eps, k, None, store, 60, G=(0, 0, 3e-5), walls=0b001111)


def test_d3q19_periodic(gpu):
    cls, eps, k, fe = random_case((16, 9, 64), seed=32)
    _compare(gpu, 19, cls, eps, k, None, "f64", 50, G=(1e-5, 2e-5, 3e-5))


@pytest.fixture(scope="module")
def shale4096_crops():
    """512 x 512 crops of the 4096 x 4096 benchmark map, with its physical class table."""
    from oracle import kapp
    inst = si.shale4096()
    crops = si.shale4096_crops(inst, inst.classes(), 512)
    return crops, kapp.class_table(inst)


@pytest.mark.parametrize("store,crop", [("f64", 0), ("f32", 1), ("f32loc", 2), ("f16loc", 3)])
def test_shale4096_crop_fixed_steps(gpu, shale4096_crops, store, crop):
    """The benchmark's own map and class table (K_app from DGM/GMS at 10 MPa, body force 1e-6):
    200 steps on a 512 x 512 crop, element by element."""
    crops, (eps, k, fe) = shale4096_crops
    _compare(gpu, 9, crops[crop], eps, k, fe, store, 200, G=(1e-6, 0, 0))
