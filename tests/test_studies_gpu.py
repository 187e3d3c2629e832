"""The paper's parameter studies as batched pressure-driven workloads (Sec. 3.2-3.3).

Small lattices (32 x 64, lattice spacing 20 nm so that a solve takes thousands of
steps, not millions); the studies themselves run at the paper's 16 x 8 um domain
in bench.py --workload studies.  Checked: one sample of the batch against the
oracle's converged k (its K(P) table built independently by oracle/kapp.py), and
the trends the paper states: organic matter near the outlet above organic matter
near the inlet with a small spread over the layout cases (Sec. 3.2), and k falling
with TOC when surface diffusion is negligible but rising with TOC at high surface
diffusivity (Sec. 3.3).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import kapp
import shale_inputs as si

pytestmark = pytest.mark.gpu

DX = 20e-9


def _small(cases):
    for c in cases:
        c.dx = DX
    return cases


def _oracle_k(case, cls, tol=1e-10):
    """Converged k_p of one study sample by the oracle, with its own class coefficients."""
    r_iom, r_om = case.radii()
    A, B, C, b, e = (np.full(256, math.inf), np.zeros(256), np.zeros(256), np.zeros(256), np.ones(256))
    for lo, radii, ep, qs, lb in ((1, r_iom, case.eps_iom, 0.0, 0.0),
                                  (128, r_om, case.eps_om, case.q_sat, case.langmuir_b)):
        a_, b_, c_ = kapp.pressure_coefficients(radii, case.temperature, ep, case.tortuosity, case.viscosity, qs, lb,
                                                case.d_s)
        sl = slice(lo, lo + len(radii))
        A[sl], B[sl], C[sl], b[sl], e[sl] = a_ / case.dx ** 2, b_ / case.dx ** 2, c_ / case.dx ** 2, lb, ep
    pr = oracle.Pressure(axis=0, rho_in=1 + 5e-5, rho_out=1 - 5e-5, k_const=A, k_kn=B, k_surf=C, lang_b=b,
                         p_in=case.p_in, p_out=case.p_out)
    p = oracle.Problem(q=9, cls=cls, eps=e, k=np.ones(256), f_eps=0.0, tau=1.0, G=(0, 0, 0), precision="f64",
                       pressure=pr)
    sol = oracle.solve(p, tol=tol, max_steps=2000000, check_every=100)
    return sol.k[0], sol.steps


def test_layout_study_matches_oracle_and_orders_cases(gpu):
    from paper_1601_00704_amd import studies
    cases = _small(si.layout_study((32, 64), realizations=2))
    maps = [c.classes() for c in cases]
    res, run = studies.solve_study(cases, maps, store="f64", tol=1e-10, max_steps=2000000)
    print("run: %s" % run)
    for r in res:
        print("  %s: k_lattice %.6e steps %d r %.2e" % (r["name"], r["k_lattice"], r["steps"], r["residual"]))
    assert run["rc"] == gpu.GLBM_OK
    i = [r["name"] for r in res].index("layout2_r0")
    ko, so = _oracle_k(cases[i], maps[i])
    rel = abs(res[i]["k_lattice"] - ko) / ko
    print("layout2_r0: gpu %.12e oracle %.12e rel %.2e (steps %d / %d)" % (res[i]["k_lattice"], ko, rel,
                                                                         res[i]["steps"], so))
    assert rel < 1e-9
    mean = {c: np.mean([r["k_lattice"] for r in res if r["case"] == c]) for c in (1, 2, 3, 4)}
    print("case means: %s" % mean)
    assert mean[3] > mean[2]
    assert (max(mean.values()) - min(mean.values())) / np.mean(list(mean.values())) < 0.1


def test_toc_study_trend_depends_on_surface_diffusivity(gpu):
    from paper_1601_00704_amd import studies
    cases = _small(si.toc_study((32, 64), tocs=(0.2, 0.8), d_s=(1e-9, 1e-5)))
    res, run = studies.solve_study(cases, store="f64", tol=1e-8, max_steps=2000000)
    k = {(r["toc"], r["d_s"]): r["k_lattice"] for r in res}
    print("run: %s; k: %s" % (run, k))
    assert run["rc"] == gpu.GLBM_OK
    assert k[(0.8, 1e-9)] < k[(0.2, 1e-9)]
    assert k[(0.8, 1e-5)] > k[(0.2, 1e-5)]
