"""Shared test helpers: build the same problem for the oracle and for the GPU library."""
from __future__ import annotations

import numpy as np

import oracle
import shale_inputs as si


def oracle_problem(q, cls, eps, k, f_eps=0.0, tau=1.0, G=(1e-6, 0, 0), walls=0, precision="ext",
                   store_mode=0, scale_log2=0, pressure=None):
    if f_eps is None:
        f_eps = 0.0
    return oracle.Problem(q=q, cls=cls, eps=eps, k=k, f_eps=f_eps, tau=tau, G=G, walls=walls,
                          precision=precision, store_mode=store_mode, scale_log2=scale_log2, pressure=pressure)


def gpu_solver(g, q, cls, eps, k, f_eps=None, tau=1.0, G=(1e-6, 0, 0), walls=0, store="f64",
               check_every=100, scale_log2=None, tile=None, cache=None, pressure=None):
    """A GPU context of the same problem; `pressure` is an oracle.Pressure (the input record
    of the pressure faces and, optionally, the K(P) coefficients)."""
    shape = cls.shape
    pk = {} if pressure is None else dict(pressure_axis=pressure.axis, rho_in=pressure.rho_in,
                                          rho_out=pressure.rho_out)
    d = g.make_desc(shape, lattice=q, store=g.STORE_NAMES[store], tau=tau, g=G, wall_faces=walls,
                    check_every=check_every,
                    dev_scale_log2=g.GLBM_SCALE_AUTO if scale_log2 is None else scale_log2,
                    flags=g.GLBM_FLAG_F16DEV_OPT_IN if store == "f16dev" else 0, **pk)
    s = g.Solver([d], [cls])
    n_cls = 255
    eps = np.broadcast_to(np.asarray(eps, np.float64), (256,))[:n_cls]
    k = np.broadcast_to(np.asarray(k, np.float64), (256,))[:n_cls]
    fe = None if f_eps is None else np.broadcast_to(np.asarray(f_eps, np.float64), (256,))[:n_cls]
    if pressure is not None and pressure.k_const is not None:
        cut = [np.broadcast_to(np.asarray(a, np.float64), (256,))[:n_cls]
               for a in (pressure.k_const, pressure.k_kn, pressure.k_surf, pressure.lang_b)]
        s.set_pressure_perm(eps, *cut, pressure.p_in, pressure.p_out)
    else:
        s.set_local_perm(eps, k, fe)
    if tile is not None:
        s.set_option(g.GLBM_OPT_TILE_WIDTH, tile[0])
        s.set_option(g.GLBM_OPT_TILE_ROWS, tile[1])
    if cache is not None:
        s.set_option(g.GLBM_OPT_CACHE, cache)
    return s


def oracle_order(q, g):
    """Index map: gpu plane j holds oracle direction perm[j]."""
    e_o, _, _ = oracle.lattice(q)
    e_g, _ = g.glbm_velocity_set(q)
    perm = []
    for j in range(q):
        m = [i for i in range(q) if tuple(e_o[i]) == tuple(e_g[j])]
        assert len(m) == 1
        perm.append(m[0])
    return np.array(perm)


def random_case(shape, seed, n_classes=8, wall_frac=0.0, k_range=(2e-3, 5e-1)):
    cls = si.random_classes(shape, seed, n_classes=n_classes, wall_frac=wall_frac)
    eps, k, fe = si.random_table(256, seed, k_range=k_range)
    return cls, eps, k, fe
