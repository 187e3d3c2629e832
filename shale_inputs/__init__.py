"""Seeded synthetic inputs shared by the FP64 CPU oracle and the GPU path.

The paper's own samples (an Eagle Ford pore-size distribution and images of
reconstructed shale, Sec. 3.2-3.3) are not available, so every workload is a
synthetic stand-in: a three-phase map (pore / inorganic matter / organic
matter) grown by seeded QSGS, a per-node radius class drawn from a lognormal
pore-size distribution per matter phase, and the gas / adsorption parameters
of each instance.

This module holds no lattice Boltzmann or permeability arithmetic: it only
produces maps, radius bins and parameter sets.  Radii are tabulated per class
(127 equal-probability lognormal bins per matter phase) so both sides consume
identical classes.

Class codes of the uint8 map (x fastest, then y, then z):
    0            open pore (porosity 1, no drag)
    1 .. 127     inorganic-matter radius bins
    128 .. 254   organic-matter radius bins
    255          solid wall node (no fluid; halfway bounce-back)
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

PORE, IOM, OM = 0, 1, 2
N_BINS = 127
CLS_PORE = 0
CLS_IOM0 = 1
CLS_OM0 = 128
CLS_WALL = 255

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBDIR = os.path.join(_HERE, "lib")
_LIB = os.path.join(_LIBDIR, "libqsgs.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the QSGS helper with gcc (plain C, no GPU)."""
    os.makedirs(_LIBDIR, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               os.path.join(_HERE, "qsgs.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.qsgs_grow.restype = ctypes.c_int64
        lib.qsgs_grow.argtypes = [ctypes.c_int32] * 4 + [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64,
            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


def _neighbourhood(ndim: int, p_axial: float, p_diag: float, p_corner: float):
    offs, probs = [], []
    rng = (-1, 0, 1)
    if ndim == 2:
        for dy in rng:
            for dx in rng:
                k = abs(dx) + abs(dy)
                if k == 0:
                    continue
                offs.append((dx, dy, 0))
                probs.append(p_axial if k == 1 else p_diag)
    else:
        for dz in rng:
            for dy in rng:
                for dx in rng:
                    k = abs(dx) + abs(dy) + abs(dz)
                    if k == 0:
                        continue
                    offs.append((dx, dy, dz))
                    probs.append({1: p_axial, 2: p_diag, 3: p_corner}[k])
    return (np.ascontiguousarray(np.array(offs, dtype=np.int32).reshape(-1)),
            np.ascontiguousarray(np.array(probs, dtype=np.float64)))


def qsgs_grow(shape: Tuple[int, ...], allowed: np.ndarray, target: int, seed: int, stream: int,
              p_seed: float = 0.01, p_axial: float = 0.001, p_diag: float = 0.00025,
              p_corner: float = 0.0000625) -> np.ndarray:
    """Grow exactly `target` nodes inside `allowed` (uint8 mask of `shape`, z,y,x order)."""
    lib = _load()
    nz, ny, nx = (1,) + tuple(shape) if len(shape) == 2 else tuple(shape)
    off, prob = _neighbourhood(len(shape), p_axial, p_diag, p_corner)
    allowed = np.ascontiguousarray(allowed.astype(np.uint8).reshape(-1))
    out = np.zeros(allowed.size, dtype=np.uint8)
    got = lib.qsgs_grow(nx, ny, nz, len(prob), off.ctypes.data, prob.ctypes.data, p_seed,
                        ctypes.c_uint64(seed & (2**64 - 1)), ctypes.c_uint64(stream),
                        allowed.ctypes.data, int(target), out.ctypes.data)
    if got < 0:
        raise MemoryError("qsgs_grow: allocation failed")
    return out.reshape(shape)


def phase_map(shape: Tuple[int, ...], solid_frac: float, toc: float, seed: int) -> np.ndarray:
    """Three-phase map: 0 pore, 1 IOM, 2 OM.

    Solid grows by QSGS to round(solid_frac * N) nodes; organic matter grows
    by the same process restricted to the solid, to round(toc * N_solid).
    """
    n = int(np.prod(shape))
    solid = qsgs_grow(shape, np.ones(shape, np.uint8), int(round(solid_frac * n)), seed, 1)
    n_solid = int(solid.sum())
    om = qsgs_grow(shape, solid, int(round(toc * n_solid)), seed, 2)
    ph = solid.astype(np.uint8)
    ph[om.astype(bool)] = OM
    return ph


def class_map(phase: np.ndarray, seed: int) -> np.ndarray:
    """Per-node radius class: each matter node draws one of 127 bins uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000003 + 7))
    k = rng.integers(0, N_BINS, size=phase.shape, dtype=np.int64)
    cls = np.zeros(phase.shape, dtype=np.uint8)
    cls[phase == IOM] = (CLS_IOM0 + k[phase == IOM]).astype(np.uint8)
    cls[phase == OM] = (CLS_OM0 + k[phase == OM]).astype(np.uint8)
    return cls


def radius_bins(median: float, sigma: float, nbins: int = N_BINS) -> np.ndarray:
    """Radii of `nbins` equal-probability bins of a lognormal distribution.

    Bin k holds the quantile at probability (k + 1/2) / nbins:
    r_k = median * exp(sigma * Phi^-1((k + 1/2) / nbins)).
    """
    from scipy.special import ndtri
    p = (np.arange(nbins, dtype=np.float64) + 0.5) / nbins
    return median * np.exp(sigma * ndtri(p))


@dataclasses.dataclass
class Instance:
    """One GLBM problem: geometry recipe plus the physical inputs of its classes."""
    shape: Tuple[int, ...]            # (ny, nx) or (nz, ny, nx)
    seed: int
    solid_frac: float = 0.60
    toc: float = 0.15
    pressure: float = 5.0e6           # Pa
    temperature: float = 400.0        # K
    eps_iom: float = 0.1
    eps_om: float = 0.3
    r_iom_median: float = 20e-9       # m
    r_om_median: float = 5e-9         # m
    sigma_ln_r: float = 0.5
    langmuir_pl: float = 4.0e6        # Pa, b = 1 / P_L
    q_sat: Optional[float] = 4000.0   # mol/m^3; None -> from langmuir_vl
    langmuir_vl: Optional[float] = None  # m^3/kg
    d_s: float = 1e-8                 # m^2/s
    viscosity: float = 18.231e-6      # Pa s
    tortuosity: float = 2.0
    dx: float = 62.5e-9               # m per lattice spacing
    tau: float = 1.0
    g: float = 1e-6                   # body force, lattice units
    drive_axis: int = 0               # 0 = x, 1 = y, 2 = z
    wall_faces: int = 0               # bit per face: x-, x+, y-, y+, z-, z+

    def classes(self) -> np.ndarray:
        return class_map(phase_map(self.shape, self.solid_frac, self.toc, self.seed), self.seed)

    def radii(self) -> Tuple[np.ndarray, np.ndarray]:
        return (radius_bins(self.r_iom_median, self.sigma_ln_r),
                radius_bins(self.r_om_median, self.sigma_ln_r))

    def gvec(self) -> Tuple[float, float, float]:
        g = [0.0, 0.0, 0.0]
        g[self.drive_axis] = self.g
        return tuple(g)


def shale128() -> Instance:
    """128^2 D2Q9 case: 60% solid, TOC 0.15, methane at 400 K and 5 MPa."""
    return Instance(shape=(128, 128), seed=0)


def shale4096(side: int = 4096) -> Instance:
    """4096^2 D2Q9 case: TOC 0.10 at 10 MPa, otherwise as the 128^2 case."""
    return Instance(shape=(side, side), seed=1, toc=0.10, pressure=10.0e6)


def shale4096_crops(inst: Instance, cls: np.ndarray, size: int = 512):
    """Four periodic crops of the large map at (0,0), (0,W/2), (W/2,0), (W/2,W/2)."""
    h = cls.shape[0] // 2
    out = []
    for (y0, x0) in ((0, 0), (0, h), (h, 0), (h, h)):
        out.append(np.ascontiguousarray(cls[y0:y0 + size, x0:x0 + size]))
    return out


BATCH_SIDES = (256, 384, 512, 768, 1024)


def batch_instance(k: int, side: Optional[int] = None) -> Instance:
    """Instance k of the uneven batch: seed 2000+k, parameters drawn per instance."""
    seed = 2000 + k
    rng = np.random.Generator(np.random.PCG64(seed))
    s = int(rng.choice(BATCH_SIDES))
    toc = float(rng.uniform(0.05, 0.30))
    p = float(math.exp(rng.uniform(math.log(1.0e6), math.log(30.0e6))))
    pl = float(rng.uniform(2.0e6, 8.0e6))
    vl = float(rng.uniform(0.002, 0.008))
    if side is not None:
        s = side
    return Instance(shape=(s, s), seed=seed, toc=toc, pressure=p, langmuir_pl=pl,
                    q_sat=None, langmuir_vl=vl)


def shale3d(side: int = 256) -> Instance:
    """256^3 D3Q19 case: 55% solid, TOC 0.20, 20 MPa, drive along z, walls on x/y faces."""
    return Instance(shape=(side, side, side), seed=3, solid_frac=0.55, toc=0.20,
                    pressure=20.0e6, drive_axis=2, wall_faces=0b001111)


def warmstart_instance(seed: int, side: int = 512) -> Instance:
    """A warm-start problem: the uneven batch's parameter distributions at a fixed side."""
    inst = batch_instance(0)
    rng = np.random.Generator(np.random.PCG64(seed))
    rng.choice(BATCH_SIDES)
    inst.seed = seed
    inst.shape = (side, side)
    inst.toc = float(rng.uniform(0.05, 0.30))
    inst.pressure = float(math.exp(rng.uniform(math.log(1.0e6), math.log(30.0e6))))
    inst.langmuir_pl = float(rng.uniform(2.0e6, 8.0e6))
    inst.langmuir_vl = float(rng.uniform(0.002, 0.008))
    return inst


def _classes_of(inst: "Instance") -> np.ndarray:
    return inst.classes()


def batch_classes(instances: Sequence["Instance"], processes: Optional[int] = None):
    """Class maps of many instances, generated in worker processes (fork).
    Call before the process touches the GPU."""
    import multiprocessing as mp
    n = processes or min(16, os.cpu_count() or 1)
    if n <= 1 or len(instances) < 2:
        return [i.classes() for i in instances]
    ctx = mp.get_context("fork")
    with ctx.Pool(n) as pool:
        return pool.map(_classes_of, list(instances), chunksize=1)


def uneven_batch(n: int = 256):
    """The uneven batch: instances 0 .. n-1, largest first (longest-processing-time order)."""
    insts = [batch_instance(k) for k in range(n)]
    return sorted(insts, key=lambda i: -int(np.prod(i.shape)))


def uniform_classes(shape: Sequence[int], cls: int = 1) -> np.ndarray:
    return np.full(tuple(shape), cls, dtype=np.uint8)


def random_classes(shape: Sequence[int], seed: int, n_classes: int = 8,
                   wall_frac: float = 0.0) -> np.ndarray:
    """Unstructured random class map for small parity cases (classes 0..n_classes-1, walls 255)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cls = rng.integers(0, n_classes, size=tuple(shape), dtype=np.int64).astype(np.uint8)
    if wall_frac > 0:
        cls[rng.random(tuple(shape)) < wall_frac] = CLS_WALL
    return cls


def random_table(n_classes: int, seed: int, k_range=(1e-3, 1e-1), eps_range=(0.1, 1.0),
                 open_pore: bool = True, f_eps: float = 0.0):
    """Random per-class (eps, K_lattice, F_eps) for parity cases; class 0 is open pore."""
    rng = np.random.Generator(np.random.PCG64(seed + 99991))
    eps = rng.uniform(*eps_range, size=n_classes)
    k = np.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1]), size=n_classes))
    fe = np.full(n_classes, f_eps)
    if open_pore:
        eps[0] = 1.0
        k[0] = math.inf
        fe[0] = 0.0
    return eps, k, fe


# ------------------------------------------------------------- pore-size samples
# The paper's validation set of the EM fit (Sec. 2.2, Tab. 3): two Gaussian
# clusters as (mean, standard deviation, fraction).
TAB3_CLUSTERS = ((10.0, 1.0, 0.25), (20.0, 4.0, 0.75))


def mixture_samples(seed: int, m: int, clusters=TAB3_CLUSTERS) -> np.ndarray:
    """m draws from a one-dimensional Gaussian mixture given as (mean, sd, fraction)
    triples: component counts from one multinomial draw, then normal draws, shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    frac = np.array([c[2] for c in clusters], dtype=np.float64)
    counts = rng.multinomial(m, frac / frac.sum())
    x = np.concatenate([rng.normal(c[0], c[1], n) for c, n in zip(clusters, counts)])
    rng.shuffle(x)
    return x


def pore_radius_samples(seed: int, m: int, r_iom_median: float = 20e-9, r_om_median: float = 5e-9,
                        sigma_ln_r: float = 0.5, om_fraction: float = 0.3) -> np.ndarray:
    """A synthetic measured pore-size distribution of a shale matrix: m pore radii (m),
    a lognormal mode per phase (inorganic and organic matter) mixed in the given
    fraction; the paper's Eagle Ford data are not available."""
    clusters = ((math.log(r_om_median), sigma_ln_r, om_fraction),
                (math.log(r_iom_median), sigma_ln_r, 1.0 - om_fraction))
    return np.exp(mixture_samples(seed, m, clusters))


# ---------------------------------------------------- the paper's parameter studies
# Sec. 3.2-3.3 inputs.  Tab. 6 lists the pore-size modes of organic (OM) and
# inorganic (IOM) matter as mu = 0.4 / 1.4 and sigma = 0.18 / 0.44 "nm"; read as
# the mean and standard deviation of ln(r / nm) (medians 1.49 and 4.06 nm, a
# ratio of e: the "roughly 3 times smaller" OM pores of Sec. 3.2).  Tab. 7 gives
# the pressures, Langmuir and diffusion inputs, porosities and the 16 x 8 um
# domain.
TAB6_OM = (0.4, 0.18)     # mean, sd of ln(r / nm)
TAB6_IOM = (1.4, 0.44)
TAB7 = dict(p_in=0.2e6, p_out=0.1e6, q_sat=4000.0, d_s=1e-8, langmuir_b=0.25e-6, tortuosity=2.0,
            eps_iom=0.02, eps_om=0.04, length=16e-6, width=8e-6)


@dataclasses.dataclass
class StudyCase:
    """One pressure-driven study sample: a matter-only map (IOM / OM, no open pore),
    per-node radius classes drawn from each phase's mode, Tab. 7-type inputs.
    Flow along x from p_in (x = 0) to p_out."""
    name: str
    phase: np.ndarray                 # uint8 (ny, nx): IOM = 1, OM = 2
    seed: int
    r_om_median: float = math.exp(TAB6_OM[0]) * 1e-9
    r_iom_median: float = math.exp(TAB6_IOM[0]) * 1e-9
    sigma_om: float = TAB6_OM[1]
    sigma_iom: float = TAB6_IOM[1]
    eps_iom: float = TAB7["eps_iom"]
    eps_om: float = TAB7["eps_om"]
    temperature: float = 400.0
    p_in: float = TAB7["p_in"]
    p_out: float = TAB7["p_out"]
    q_sat: float = TAB7["q_sat"]
    langmuir_b: float = TAB7["langmuir_b"]
    d_s: float = TAB7["d_s"]
    tortuosity: float = TAB7["tortuosity"]
    viscosity: float = 18.231e-6
    dx: float = TAB7["width"] / 128
    labels: dict = dataclasses.field(default_factory=dict)

    def classes(self) -> np.ndarray:
        return class_map(self.phase, self.seed)

    def radii(self) -> Tuple[np.ndarray, np.ndarray]:
        return radius_bins(self.r_iom_median, self.sigma_iom), radius_bins(self.r_om_median, self.sigma_om)


def layout_phase(case: int, shape: Tuple[int, int], seed: int, toc: float = 0.5) -> np.ndarray:
    """Sec. 3.2 layout cases of OM and IOM (flow along x): 1 layers parallel to the flow
    (OM in the lower rows), 2 OM upstream then IOM, 3 IOM upstream then OM (both in
    sequence along the flow), 4 OM grown at random by QSGS inside the matter.  TOC is
    the OM fraction (0.5 for the layered cases, a reading: the paper's figure is
    not available)."""
    ny, nx = shape
    ph = np.full(shape, IOM, np.uint8)
    if case == 1:
        ph[:int(round(toc * ny)), :] = OM
    elif case == 2:
        ph[:, :int(round(toc * nx))] = OM
    elif case == 3:
        ph[:, nx - int(round(toc * nx)):] = OM
    elif case == 4:
        om = qsgs_grow(shape, np.ones(shape, np.uint8), int(round(toc * ny * nx)), seed, 2)
        ph[om.astype(bool)] = OM
    else:
        raise ValueError("layout case must be 1..4")
    return ph


def layout_study(shape=(128, 256), realizations: int = 4, seed0: int = 5000):
    """Cases 1-4 of Sec. 3.2, several radius realizations each (Tab. 6, Tab. 7)."""
    out = []
    for case in (1, 2, 3, 4):
        for r in range(realizations):
            seed = seed0 + 100 * case + r
            out.append(StudyCase("layout%d_r%d" % (case, r), layout_phase(case, shape, seed), seed,
                                 labels={"case": case, "realization": r}))
    return out


def toc_study(shape=(128, 256), tocs=(0.2, 0.4, 0.6, 0.8), d_s=(1e-9, 1e-8, 1e-7, 1e-6, 1e-5), seed0: int = 6000):
    """Sec. 3.3: OM grown by QSGS inside the matter to each TOC (one map per TOC, shared
    by every surface diffusivity), times the surface diffusivities of Fig. 15."""
    out = []
    for i, toc in enumerate(tocs):
        seed = seed0 + i
        ph = layout_phase(4, shape, seed, toc)
        for ds in d_s:
            out.append(StudyCase("toc%.1f_ds%.0e" % (toc, ds), ph, seed, d_s=ds, labels={"toc": toc, "d_s": ds}))
    return out


def single_phase_study(phase: int, shape=(64, 64), r_medians=(2e-9, 5e-9, 11e-9, 20e-9, 50e-9, 100e-9),
                       pressures=((22e6, 20e6),), q_sats=(4000.0,), bs=(0.25e-6,), d_s=5e-7, sigma_ln=0.25,
                       k_lattice=1e-3, seed0: int = 7000):
    """Sec. 3.1 (Figs. 5, 6, 9-11): single-phase samples (IOM with eps 0.04, or OM) whose
    per-node radii follow one lognormal mode (sigma 0.25 in ln r), swept over the mean
    radius, the pressures, q_sat and b (Tab. 4 inputs: 22 -> 20 MPa, tortuosity 2).
    The lattice spacing of each sample is chosen so that its K at the mean pressure is
    about k_lattice in lattice units (Darcy regime; dx only scales the time to converge)."""
    out = []
    k = 0
    for rm in r_medians:
        for (pin, pout) in pressures:
            for qs in q_sats:
                for b in bs:
                    seed = seed0 + k
                    k += 1
                    ph = np.full(shape, phase, np.uint8)
                    eps = 0.04
                    # K_0 + Knudsen of the median radius at the mean pressure sets dx
                    pm = 0.5 * (pin + pout)
                    d = 2 * rm
                    kc = eps / 2.0 * d / 4.0
                    kk = kc * d / 8.0 + 18.231e-6 * (4.0 / 3.0) * kc * math.sqrt(8 * 8.314462618 * 400.0 /
                                                                              (math.pi * 0.016043)) / pm
                    dx = math.sqrt(kk / k_lattice)
                    out.append(StudyCase("phase%d_r%.0e_p%.0f_q%.0f_b%.2e" % (phase, rm, pm / 1e6, qs, b), ph, seed,
                                         r_om_median=rm, r_iom_median=rm, sigma_om=sigma_ln, sigma_iom=sigma_ln,
                                         eps_iom=eps, eps_om=eps, p_in=pin, p_out=pout, q_sat=qs, langmuir_b=b,
                                         d_s=d_s, dx=dx, labels={"phase": phase, "r_median": rm, "p_mean": pm,
                                                                 "q_sat": qs, "b": b}))
    return out
