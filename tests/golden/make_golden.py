"""Write the stored oracle results the GPU tests compare against.

Calls only the CPU oracle (oracle/) and the seeded input generators
(shale_inputs/); nothing here touches the GPU path.  Run from the repository
root:  python tests/golden/make_golden.py [case ...]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import kapp  # noqa: E402
import shale_inputs as si  # noqa: E402


def map_sha(cls):
    return hashlib.sha256(np.ascontiguousarray(cls).tobytes()).hexdigest()[:16]


def solve_case(name, inst, cls, tol, max_steps, precision="ext"):
    e, k, fe = kapp.class_table(inst)
    prob = oracle.Problem(q=9 if len(cls.shape) == 2 else 19, cls=cls, eps=e, k=k, f_eps=fe, tau=inst.tau,
                          G=inst.gvec(), walls=inst.wall_faces, precision=precision)
    t0 = time.time()
    sol = oracle.solve(prob, tol=tol, max_steps=max_steps, check_every=100)
    dt = time.time() - t0
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(cls.size, size=32, replace=False))
    rec = {
        "case": name, "shape": list(cls.shape), "map_sha": map_sha(cls), "precision": precision,
        "tol": tol, "check_every": 100, "steps": sol.steps, "residual": sol.residual,
        "k_lattice": [None if not np.isfinite(v) else float(v) for v in sol.k],
        "history": sol.history[::10] + [sol.history[-1]],
        "sample_nodes": idx.tolist(),
        "sample_u": sol.u[:, idx].T.tolist(), "sample_rho": sol.rho[idx].tolist(),
        "oracle_seconds": round(dt, 1), "oracle_threads": oracle.num_threads(),
    }
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(name, "steps", sol.steps, "r", sol.residual, "k", sol.k, "%.1fs" % dt, flush=True)


def case_shale128():
    inst = si.shale128()
    solve_case("shale128_oracle", inst, inst.classes(), 1e-8, 400000)


def case_crop():
    """The (0, 0) 512 x 512 crop of the 4096^2 benchmark map, run as a periodic instance."""
    inst = si.shale4096(4096)
    cls = inst.classes()
    crop = si.shale4096_crops(inst, cls, 512)[0]
    solve_case("shale4096_crop512_oracle", inst, crop, 1e-8, 2000000, precision="f64")


def case_crop3d():
    """The 64^3 corner crop of the 256^3 D3Q19 map (walls on the x/y faces, drive along z)."""
    inst = si.shale3d(256)
    cls = inst.classes()
    crop = np.ascontiguousarray(cls[:64, :64, :64])
    solve_case("shale3d_crop64_oracle", inst, crop, 1e-7, 400000, precision="f64")


CASES = {"shale128": case_shale128, "crop": case_crop, "crop3d": case_crop3d}

if __name__ == "__main__":
    for c in (sys.argv[1:] or ["shale128"]):
        CASES[c]()
