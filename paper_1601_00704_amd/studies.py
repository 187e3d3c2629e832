"""The paper's parameter studies as batched, pressure-driven GLBM workloads.

Orchestration only: every solve runs in libglbm.  Each study is a list of
samples (shale_inputs.StudyCase: a matter-only map of inorganic and organic
matter with per-node pore radii, Tab. 6 / Tab. 7 inputs); one GLBM context holds
all samples of a study as instances, each with pressure faces along x (inlet at
x = 0) and the apparent permeability of Eq. (18)-(19) evaluated at every node's
local pressure (glbm_class_table_pressure, glbm_set_pressure_perm).  The
context is solved to a residual and each sample's permeability is read off
Darcy's law with the lattice pressure (k_p; a uniform medium of porosity eps
gives K / eps).

  layout  Sec. 3.2 cases 1-4 (OM layers parallel to the flow, OM upstream, OM
          downstream, OM at random), several radius realizations each
  toc     Sec. 3.3 TOC 0.2-0.8 for surface diffusivities 1e-9 .. 1e-5 m^2/s
  iom / om  Sec. 3.1 single-phase samples over mean radius, pressure, q_sat, b

Run: python -m paper_1601_00704_amd.studies layout --out layout.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import glbm as g

N_C = 100
DARCY_M2 = 9.869233e-13
DRHO = 1e-4   # lattice density drop between the faces (low Mach)


def gas_params(case, molar_mass=0.016043):
    """glbm_gas_params of a study sample (plain field copy of its inputs)."""
    p = g.glbm_gas_params()
    p.pressure = 0.5 * (case.p_in + case.p_out)
    p.temperature, p.viscosity, p.molar_mass = case.temperature, case.viscosity, molar_mass
    p.tortuosity, p.dx = case.tortuosity, case.dx
    p.eps_iom, p.eps_om = case.eps_iom, case.eps_om
    p.langmuir_b, p.q_sat, p.langmuir_vl, p.toc, p.d_s = case.langmuir_b, case.q_sat, 0.0, 0.0, case.d_s
    return p


def solve_study(cases, maps=None, store="f64", tol=1e-8, max_steps=3000000, tile=None):
    """Solve every sample of a study in one batched context; returns per-sample records
    and the run's wall time, steps and lattice updates.  tile: (width, rows[, cache
    policy]), default two time steps per launch on 64 x 4 tiles for F64 and F32."""
    maps = maps if maps is not None else [c.classes() for c in cases]
    descs = [g.make_desc(m.shape, store=g.STORE_NAMES[store], tau=1.0, g=(0, 0, 0), check_every=N_C,
                         pressure_axis=0, rho_in=1 + DRHO / 2, rho_out=1 - DRHO / 2) for m in maps]
    s = g.Solver(descs, maps)
    try:
        for i, c in enumerate(cases):
            eps, kc, kk, ks, b = g.glbm_class_table_pressure(gas_params(c), *c.radii())
            s.set_pressure_perm(eps[:255], kc[:255], kk[:255], ks[:255], b[:255], c.p_in, c.p_out, inst=i)
        if tile is None and store in ("f64", "f32"):
            # two time steps per launch on 64 x 4 tiles (cache policy 77), bitwise equal
            # to one step per launch
            tile = (64, 4, 77)
        if tile:
            s.set_option(g.GLBM_OPT_TILE_WIDTH, tile[0])
            s.set_option(g.GLBM_OPT_TILE_ROWS, tile[1])
            if len(tile) > 2:
                s.set_option(g.GLBM_OPT_CACHE, tile[2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = s.step(max_steps, tol=tol)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r, st = s.residual()
        k = s.permeability()[:, 0]
    finally:
        s.close()
    out = []
    for i, c in enumerate(cases):
        kp = float(k[i]) * c.dx ** 2
        out.append({"name": c.name, **c.labels, "percolates_x": g.glbm_pore_percolates(maps[i], 1),
                    "steps": int(st[i]), "residual": float(r[i]),
                    "k_lattice": float(k[i]), "k_m2": kp, "k_mD": kp / DARCY_M2 * 1e3})
    lups = float(sum(int(m.size) * int(st[i]) for i, m in enumerate(maps)))
    return out, {"rc": int(rc), "wall_s": wall, "lattice_updates": lups, "max_steps": int(st.max())}


def main(argv=None):
    import shale_inputs as si
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=("layout", "toc", "iom", "om"))
    ap.add_argument("--store", default="f64")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--realizations", type=int, default=4)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.study == "layout":
        cases = si.layout_study(realizations=args.realizations)
    elif args.study == "toc":
        cases = si.toc_study()
    else:
        cases = si.single_phase_study(si.IOM if args.study == "iom" else si.OM)
    res, run = solve_study(cases, store=args.store, tol=args.tol)
    rep = {"study": args.study, "store": args.store, "tol": args.tol, **run, "samples": res}
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rep, fh, indent=1)


if __name__ == "__main__":
    main()
