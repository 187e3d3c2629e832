"""FP64 CPU oracle of the paper's generalized lattice Boltzmann model.

TEST INFRASTRUCTURE ONLY.  The oracle is what the GPU path is checked
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product (the package and its native library) never
does, and the two share no code.

    glbm_ref.c   the lattice Boltzmann step, moments and initial states (C, FP64)
    kapp.py      the DGM / GMS apparent permeability of a pore class (NumPy, FP64)

This module wraps the C file with ctypes and adds the two observables of a
solve, written out in NumPy:
    residual   r(t) = ||u(t) - u(t - n_c)||_2 / (n_c ||u(t)||_2) over fluid nodes
    k_lattice  nu <u_d> / G_d, <.> the mean over fluid nodes (Darcy's law on the
               volume-averaged velocity of Eq. 26)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBDIR = os.path.join(_HERE, "lib")
_LIBS = {"f64": os.path.join(_LIBDIR, "libglbm_ref.so"),
         "ext": os.path.join(_LIBDIR, "libglbm_ref_ext.so")}
_lib = {}

WALL = 255


def build(force: bool = True):
    """Compile the C oracle with gcc and OpenMP: an FP64 build and an extended-precision build."""
    os.makedirs(_LIBDIR, exist_ok=True)
    for kind, path in _LIBS.items():
        if force or not os.path.exists(path):
            tmp = path + ".tmp%d" % os.getpid()
            extra = ["-DREF_LONG_DOUBLE"] if kind == "ext" else []
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                                   "-fno-fast-math", "-ffp-contract=off"] + extra +
                                  [os.path.join(_HERE, "glbm_ref.c"), "-o", tmp, "-lm"])
            os.replace(tmp, path)
    return list(_LIBS.values())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def lib(kind: str = "f64"):
    if kind not in _lib:
        if not os.path.exists(_LIBS[kind]):
            build(force=False)
        L = ctypes.CDLL(_LIBS[kind])
        vp, i32, i64, f64, u32 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_uint)
        L.ref_lattice.argtypes = [i32, vp, vp, vp]
        L.ref_collide_node.argtypes = [i32, vp, f64, f64, f64, f64, vp, vp, vp]
        L.ref_feq_force.argtypes = [i32, f64, vp, vp, f64, f64, vp, vp]
        L.ref_step.argtypes = [i32, i32, i32, i32, u32, f64, vp, vp, vp, vp, vp, vp, vp, i32, i32, vp]
        L.ref_fields.argtypes = [i32, i32, i32, i32, u32, f64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ref_init_rest.argtypes = [i32, i64, f64, vp]
        L.ref_init_fields.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.ref_solve.argtypes = [i32, i32, i32, i32, u32, f64, vp, vp, vp, vp, vp, vp, i64, i32, f64,
                                i32, i32, vp, vp, vp, i64, vp]
        L.ref_round_half.argtypes = [i64, vp, vp]
        L.ref_store_round.argtypes = [f64, f64, i32, i32, f64]
        L.ref_store_round.restype = f64
        for fn in ("ref_lattice", "ref_collide_node", "ref_feq_force", "ref_step",
                   "ref_fields", "ref_init_rest", "ref_init_fields", "ref_round_half"):
            getattr(L, fn).restype = ctypes.c_int
        L.ref_solve.restype = ctypes.c_int64
        _lib[kind] = L
    return _lib[kind]


def num_threads() -> int:
    """Threads the oracle's OpenMP loops run on."""
    L = lib()
    L.ref_num_threads.restype = ctypes.c_int
    return int(L.ref_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's later parallel regions (both builds)."""
    for kind in _LIBS:
        L = lib(kind)
        L.ref_set_threads.restype = ctypes.c_int
        assert L.ref_set_threads(int(n)) == 0


def round_half(x):
    """The oracle's nearest-float16 rounding (ties to even) of every element, as float64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    assert lib().ref_round_half(x.size, _p(x), _p(out)) == 0
    return out


def store_round(f, w, mode, scale_log2=0, rho_x=1.0):
    """The value a reduced-precision store of emulation mode `mode` keeps of population f
    (w its weight, rho_x the density of the node that writes it)."""
    return float(lib().ref_store_round(float(f), float(w), int(mode), int(scale_log2), float(rho_x)))


def lattice(q: int):
    e = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    opp = np.zeros(q, np.int32)
    assert lib().ref_lattice(q, _p(e), _p(w), _p(opp)) == 0
    return e, w, opp


def collide_node(q, f, eps, kinv, feps, tau, G):
    f = np.ascontiguousarray(f, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = np.zeros(q)
    aux = np.zeros(7)
    assert lib().ref_collide_node(q, _p(f), eps, kinv, feps, tau, _p(G), _p(out), _p(aux)) == 0
    return out, aux[0], aux[1:4].copy(), aux[4:7].copy()


def feq_force(q, rho, u, F, eps, tau):
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    feq = np.zeros(q)
    fi = np.zeros(q)
    assert lib().ref_feq_force(q, rho, _p(u), _p(F), eps, tau, _p(feq), _p(fi)) == 0
    return feq, fi


def _shape3(shape):
    if len(shape) == 2:
        return 1, shape[0], shape[1]
    return tuple(shape)


class _RefPressure(ctypes.Structure):
    """glbm_ref.c ref_pressure: pressure faces and the per-class K(P) coefficients."""
    _fields_ = [("axis", ctypes.c_int), ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("k_const", ctypes.c_void_p), ("k_kn", ctypes.c_void_p), ("k_surf", ctypes.c_void_p),
                ("lang_b", ctypes.c_void_p), ("p_in", ctypes.c_double), ("p_out", ctypes.c_double)]


@dataclass
class Pressure:
    """Pressure-driven run: density rho_in on the face c_a = 0 and rho_out on c_a = n_a - 1
    of axis `axis` (0 = x, 1 = y, 2 = z); optional per-class K(P) = k_const + k_kn / P +
    k_surf / (P (1 + lang_b P)) in lattice units with P mapped affinely from the density
    between (rho_out, p_out) and (rho_in, p_in).  Without k_const the class table's
    constant K is used."""
    axis: int
    rho_in: float
    rho_out: float
    k_const: Optional[np.ndarray] = None
    k_kn: Optional[np.ndarray] = None
    k_surf: Optional[np.ndarray] = None
    lang_b: Optional[np.ndarray] = None
    p_in: float = 0.0
    p_out: float = 0.0

    def struct(self):
        def arr(a):
            return None if a is None else np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (256,)))
        self._keep = [arr(self.k_const), arr(self.k_kn), arr(self.k_surf), arr(self.lang_b)]
        st = _RefPressure(self.axis + 1, self.rho_in, self.rho_out,
                          *[None if a is None else a.ctypes.data for a in self._keep], self.p_in, self.p_out)
        return st


@dataclass
class Problem:
    """One oracle problem: class map plus per-class table, all in lattice units."""
    q: int
    cls: np.ndarray                 # uint8, (ny, nx) or (nz, ny, nx)
    eps: np.ndarray                 # 256 doubles
    k: np.ndarray                   # 256 doubles, K in lattice units (+inf = open pore)
    f_eps: np.ndarray               # 256 doubles
    tau: float = 1.0
    G: Sequence[float] = (1e-6, 0.0, 0.0)
    walls: int = 0
    store_mode: int = 0             # 0 plain; 1-5 emulate reduced-precision storage (glbm_ref.c store_round)
    scale_log2: int = 0
    precision: str = "f64"          # "f64", or "ext" for the x87 extended-precision build
    pressure: Optional[Pressure] = None

    def __post_init__(self):
        if self.f_eps is None:
            self.f_eps = 0.0
        self.cls = np.ascontiguousarray(self.cls, dtype=np.uint8)
        self.eps = np.ascontiguousarray(np.broadcast_to(np.asarray(self.eps, np.float64), (256,)))
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(self.k, np.float64), (256,)))
        self.kinv = np.where(np.isinf(k), 0.0, 1.0 / k)
        self.k = k
        self.f_eps = np.ascontiguousarray(np.broadcast_to(np.asarray(self.f_eps, np.float64), (256,)))
        self.G = np.ascontiguousarray(np.asarray(self.G, np.float64).reshape(3))
        self.nz, self.ny, self.nx = _shape3(self.cls.shape)
        self.N = self.nx * self.ny * self.nz
        self.fluid = self.cls.reshape(-1) != WALL
        for a in range(3):
            if ((self.walls >> (2 * a)) & 1) != ((self.walls >> (2 * a + 1)) & 1):
                raise ValueError("wall faces come in pairs per axis (a one-sided wall with a periodic "
                                 "opposite face is undefined)")
        self._pr = None if self.pressure is None else self.pressure.struct()

    def _prp(self):
        return None if self._pr is None else ctypes.addressof(self._pr)

    @property
    def nu(self):
        return (self.tau - 0.5) / 3.0

    def rest(self, rho0=1.0):
        f = np.zeros(self.q * self.N)
        assert lib().ref_init_rest(self.q, self.N, rho0, _p(f)) == 0
        return f

    def equilibrium(self, rho, u):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        f = np.zeros(self.q * self.N)
        assert lib().ref_init_fields(self.q, self.nx, self.ny, self.nz, _p(self.cls), _p(self.eps),
                                     _p(rho), _p(u), _p(f)) == 0
        return f

    def step(self, f):
        out = np.zeros_like(f)
        assert lib(self.precision).ref_step(self.q, self.nx, self.ny, self.nz, self.walls, self.tau, _p(self.G),
                              _p(self.cls), _p(self.eps), _p(self.kinv), _p(self.f_eps), _p(f),
                              _p(out), self.store_mode, self.scale_log2, self._prp()) == 0
        return out

    def iterate(self, f, nsteps, check_every=0, tol=0.0):
        """Advance f (in place) by up to nsteps; returns (steps, rho, u[3,N], residual history)."""
        assert f.flags.c_contiguous and f.dtype == np.float64 and f.size == self.q * self.N
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        cap = int(nsteps // check_every) + 1 if check_every > 0 else 1
        hist = np.zeros(cap)
        s = lib(self.precision).ref_solve(
            self.q, self.nx, self.ny, self.nz, self.walls, self.tau, _p(self.G), _p(self.cls),
            _p(self.eps), _p(self.kinv), _p(self.f_eps), _p(f), int(nsteps), int(check_every),
            float(tol), self.store_mode, self.scale_log2, _p(rho), _p(u), _p(hist), cap, self._prp())
        assert s >= 0, "ref_solve failed (%d)" % s
        nh = int(s // check_every) if check_every > 0 else 0
        return int(s), rho, u.reshape(3, self.N), hist[:nh].copy()

    def run(self, f, nsteps):
        """Advance f in place by nsteps."""
        self.iterate(f, nsteps)
        return f

    def fields(self, f):
        """(rho[N], u[3, N]) of the state f."""
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        assert lib(self.precision).ref_fields(self.q, self.nx, self.ny, self.nz, self.walls, self.tau,
                                _p(self.G), _p(self.cls), _p(self.eps), _p(self.kinv), _p(self.f_eps),
                                _p(f), _p(rho), _p(u), self._prp()) == 0
        return rho, u.reshape(3, self.N)

    def k_lattice(self, u):
        """Darcy read-off per axis: nu <u_d> / G_d over fluid nodes (nan where G_d = 0).  Along
        the axis of pressure faces: nu <u_a> (n_a - 1) / (c_s^2 (rho_in - rho_out)), Darcy's
        law with the lattice pressure c_s^2 rho over the node distance between the faces."""
        m = u[:, self.fluid].mean(axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            k = np.where(self.G != 0, self.nu * m / np.where(self.G != 0, self.G, 1.0), np.nan)
        if self.pressure is not None:
            a = self.pressure.axis
            na = (self.nx, self.ny, self.nz)[a]
            k[a] = self.nu * m[a] * (na - 1) / ((self.pressure.rho_in - self.pressure.rho_out) / 3.0)
        return k

    def residual(self, u, u_prev, dsteps):
        d = (u - u_prev)[:, self.fluid]
        a = u[:, self.fluid]
        return float(np.sqrt(np.sum(d * d)) / (dsteps * np.sqrt(np.sum(a * a))))


@dataclass
class Solution:
    f: np.ndarray
    steps: int
    residual: float
    k: np.ndarray
    rho: np.ndarray
    u: np.ndarray
    history: list = field(default_factory=list)


def solve(prob: Problem, tol: float, max_steps: int, check_every: int = 100,
          f0: Optional[np.ndarray] = None, stop_at: Optional[int] = None) -> Solution:
    """Iterate from f0 (rest state by default), checking every n_c steps.

    Stops at the first check with r <= tol, or at max_steps; if stop_at is
    given, runs exactly that many steps (still recording the residuals).
    """
    f = prob.rest() if f0 is None else np.array(f0, dtype=np.float64, copy=True)
    n = stop_at if stop_at is not None else max_steps
    steps, rho, u, hist = prob.iterate(f, n, check_every, 0.0 if stop_at is not None else tol)
    r = float(hist[-1]) if len(hist) else np.inf
    history = [((i + 1) * check_every, float(h)) for i, h in enumerate(hist)]
    return Solution(f=f, steps=steps, residual=r, k=prob.k_lattice(u), rho=rho, u=u,
                    history=history)
