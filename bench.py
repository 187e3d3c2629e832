"""Throughput of the GLBM hot path on one MI355X.

One bench "step" is one check interval of the hot path on the whole lattice:
n_c = 100 stream-and-collide sweeps (Eq. 29-37 with per-node eps and K_app)
followed by the FP64 residual and Darcy-flux reductions of that state, all in
the HIP library.  The workload is a 4096 x 4096 D2Q9 shale map (seeded QSGS,
60% solid, TOC 0.10, methane at 400 K and 10 MPa) with FP32 populations.

Reported (one JSON line):
  value        lattice updates per second over the timed steps (MLUPS)
  roofline     the sweep kernel's algorithmic HBM bytes per launch
               (2 x 9 x 4 B populations + 1 B class per node) over its mean
               launch time, measured with HIP events on the library's stream
               around every sweep launch of the timed region
  cpu_baseline the CPU oracle (FP64 C, OpenMP) on a 512 x 512 crop of the
               same map, rank 0 only
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLBM MLUPS + % HBM peak; time-to-converged k_app, plain vs warm-start"
PEAK_HBM_GBS = 8000.0
N_C = 100


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("glbm_kernels.hip", "glbm_internal.h"):
        with open(os.path.join(ROOT, "paper_1601_00704_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(store: str, side: int):
    """HBM bytes per sweep launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "sweep_d2q9_%s_%d_traffic.json" % (store, side))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def calibrate_copy(nbytes=1 << 30, reps=5):
    """A plain elementwise copy of known size, for scaling the HBM counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def _pmc_per_kernel(path):
    import csv
    import glob
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def pmc_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, store, side):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE / WRITE_SIZE of the bench and of
    calibrate_copy) into HBM bytes per sweep launch.  Counters are KiB per
    dispatch; each is scaled by (known copy bytes) / (counter on the copy)."""
    def pick(d, key):
        vals = [v for k, vs in d.items() if key in k for v in vs]
        return sum(vals) / len(vals), len(vals)
    nbytes = 1 << 30
    cf, _ = pick(_pmc_per_kernel(cfetch_dir), "neg")
    cw, _ = pick(_pmc_per_kernel(cwrite_dir), "neg")
    f_scale = nbytes / (cf * 1024.0)
    w_scale = nbytes / (cw * 1024.0)
    sf, nf = pick(_pmc_per_kernel(fetch_dir), "k_sweep")
    sw, nw = pick(_pmc_per_kernel(write_dir), "k_sweep")
    read = sf * 1024.0 * f_scale
    write = sw * 1024.0 * w_scale
    n = side * side
    bpl = {"f32": 73, "f16dev": 37, "f16loc": 45, "f64": 145}[store]
    rec = {"kernel": "k_sweep<9,%s> on %dx%d" % (store, side, side),
           "kernel_source_hash": kernel_source_hash(),
           "fetch_kib_per_launch": sf, "write_kib_per_launch": sw, "launches": [nf, nw],
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_read_bytes_per_launch": read, "hbm_write_bytes_per_launch": write,
           "hbm_bytes_per_launch": read + write,
           "algorithmic_bytes_per_launch": bpl * n,
           "traffic_over_algorithmic": (read + write) / (bpl * n)}
    path = os.path.join(ROOT, "profiles", "sweep_d2q9_%s_%d_traffic.json" % (store, side))
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def cpu_baseline(cls_crop, table, steps):
    import oracle
    eps, k, fe = table
    prob = oracle.Problem(q=9, cls=cls_crop, eps=eps, k=k, f_eps=fe, tau=1.0, G=(1e-6, 0, 0))
    f = prob.rest()
    prob.run(f, 2)
    t0 = time.perf_counter()
    prob.run(f, steps)
    dt = time.perf_counter() - t0
    return cls_crop.size * steps / dt / 1e6, dt, oracle.num_threads()


def _json_line(metric_unit_value, steps, warmup, ms_per_step, dtype, config, roofline, extra=None):
    out = {"metric": METRIC, "value": round(metric_unit_value, 1), "unit": "MLUPS", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded QSGS shale maps, generated in-process)", "config": config,
           "roofline": roofline}
    if extra:
        out.update(extra)
    return out


DTYPE = {"f32": "f32", "f16dev": "f32 math / f16 storage", "f16loc": "f32 math / f16 storage", "f64": "f64"}


def _timed_chunks(s, g, steps, warmup, graph):
    """Warm up, then time `steps` chunks of N_C sweeps + the FP64 check."""
    import torch
    s.set_option(g.GLBM_OPT_GRAPH, 1 if graph else 0)
    s.set_option(g.GLBM_OPT_TIMING, 0 if graph else 1)
    for _ in range(warmup):
        s.step(N_C)
    torch.cuda.synchronize()
    s.set_option(g.GLBM_OPT_TIMING, 0 if graph else 1)  # resets the sweep timer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        s.step(N_C)
        print("step %d/%d done" % (k + 1, steps), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _sweep_mean_ms(s, g, chunks=1):
    """Mean sweep launch time from HIP events on the library stream (eager launches)."""
    s.set_option(g.GLBM_OPT_GRAPH, 0)
    s.set_option(g.GLBM_OPT_TIMING, 1)
    for _ in range(chunks):
        s.step(N_C)
    ms, n = g.glbm_sweep_time(s.ctx)
    s.set_option(g.GLBM_OPT_TIMING, 0)
    return ms / max(n, 1), n


def run_batch(args):
    """Uneven batch: 256 instances, sides from {256..1024}, per-instance gas and
    Langmuir parameters, one HIP graph per n_c-step chunk over all instances."""
    import numpy as np
    import shale_inputs as si
    insts = si.cfg2_batch(args.batch)
    t0 = time.perf_counter()
    maps = si.batch_classes(insts)
    t_geom = time.perf_counter() - t0
    import torch
    import paper_1601_00704_amd.glbm as g
    torch.cuda.set_device(0)
    store = g.STORE_NAMES[args.store]
    descs = [g.make_desc(m.shape, store=store, tau=i.tau, g=i.gvec(), check_every=N_C) for i, m in zip(insts, maps)]
    s = g.Solver(descs, maps)
    for k, inst in enumerate(insts):
        r_iom, r_om = inst.radii()
        eps, kl = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
        s.set_local_perm(eps[:255], kl[:255], inst=k)
    N = int(sum(m.size for m in maps))
    print("setup: %d instances, %d nodes, maps in %.1fs, store %s" % (len(maps), N, t_geom, args.store),
          file=sys.stderr, flush=True)
    wall = _timed_chunks(s, g, args.steps, args.warmup, graph=True)
    per_launch, launches = _sweep_mean_ms(s, g)
    r, st = s.residual()
    s.close()
    bpl = g.bytes_per_update(9, store)
    achieved = bpl * N / (per_launch * 1e-3) / 1e9
    sides = sorted(set(int(m.shape[0]) for m in maps))
    cfg = {"workload": "batched D2Q9 GLBM: %d QSGS instances, sides %s, TOC U(0.05,0.30), P log-U(1,30) MPa, "
                       "P_L U(2,8) MPa, V_L U(0.002,0.008) m3/kg; %s populations; one HIP graph per "
                       "n_c=%d-sweep chunk + FP64 per-instance checks" % (len(maps), sides, args.store.upper(), N_C),
           "instances": len(maps), "nodes": N, "sweeps_per_step": N_C, "graph": True,
           "median_residual": float(np.median(r)), "steps_total": int(st.max())}
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "kernel": "k_sweep<9,%s> over the flat tile list" % args.store, "bytes_per_lu": bpl,
            "mean_launch_ms": round(per_launch, 5), "launches": launches}
    return _json_line(N * N_C * args.steps / wall / 1e6, args.steps, args.warmup, wall / args.steps * 1e3,
                      DTYPE[args.store], cfg, roof)


def run_d3q19(args):
    """256^3 D3Q19: 3-D QSGS (55% solid, TOC 0.20, 20 MPa), drive along z,
    halfway bounce-back on the x and y faces."""
    import shale_inputs as si
    inst = si.cfg3(args.side3)
    t0 = time.perf_counter()
    cls = inst.classes()
    t_geom = time.perf_counter() - t0
    import torch
    import paper_1601_00704_amd.glbm as g
    torch.cuda.set_device(0)
    store = g.STORE_NAMES[args.store]
    r_iom, r_om = inst.radii()
    eps, kl = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
    d = g.make_desc(cls.shape, lattice=g.GLBM_D3Q19, store=store, tau=inst.tau, g=inst.gvec(),
                    wall_faces=inst.wall_faces, check_every=N_C)
    s = g.Solver([d], [cls])
    s.set_local_perm(eps[:255], kl[:255])
    N = cls.size
    print("setup: %s map in %.1fs" % (cls.shape, t_geom), file=sys.stderr, flush=True)
    wall = _timed_chunks(s, g, args.steps, args.warmup, graph=False)
    ms, n = g.glbm_sweep_time(s.ctx)
    per_launch = ms / max(n, 1)
    r, st = s.residual()
    kk = s.permeability()[0]
    s.close()
    bpl = g.bytes_per_update(19, store)
    achieved = bpl * N / (per_launch * 1e-3) / 1e9
    cfg = {"workload": "D3Q19 GLBM %d^3, 3-D QSGS 55%% solid, TOC 0.20, CH4 400 K 20 MPa, drive z, walls on x/y "
                       "faces, %s populations" % (args.side3, args.store.upper()),
           "nodes": N, "sweeps_per_step": N_C, "steps_total": int(st[0]), "residual": float(r[0]),
           "k_lattice_z": float(kk[2])}
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "kernel": "k_sweep<19,%s>" % args.store, "bytes_per_lu": bpl,
            "mean_launch_ms": round(per_launch, 5), "launches": n}
    return _json_line(N * N_C * args.steps / wall / 1e6, args.steps, args.warmup, wall / args.steps * 1e3,
                      DTYPE[args.store], cfg, roof)


def main():

    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side", type=int, default=4096)
    ap.add_argument("--store", default="f32", choices=("f32", "f16dev", "f16loc", "f64"))
    ap.add_argument("--cpu-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="shale4096", choices=("shale4096", "batch", "d3q19"),
                    help="shale4096: the benchmark line; batch / d3q19: supplementary workloads")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--side3", type=int, default=256)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB elementwise copy (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="summarise rocprofv3 --pmc output directories into profiles/")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, store=args.store, side=args.side)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "d3q19":
        print(json.dumps(run_d3q19(args)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the GLBM hot path here is built and timed on a single "
              "MI355X (multi-GPU sharding is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import shale_inputs as si
    import paper_1601_00704_amd.glbm as g

    torch.cuda.set_device(0)
    inst = si.cfg1(args.side)
    t0 = time.perf_counter()
    cls = inst.classes()
    t_geom = time.perf_counter() - t0
    r_iom, r_om = inst.radii()
    eps, kl = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
    store = g.STORE_NAMES[args.store]
    d = g.make_desc(cls.shape, store=store, tau=inst.tau, g=inst.gvec(), check_every=N_C)
    s = g.Solver([d], [cls])
    s.set_local_perm(eps[:255], kl[:255])
    s.set_option(g.GLBM_OPT_GRAPH, 0)
    s.set_option(g.GLBM_OPT_TIMING, 1)
    N = cls.size
    print("setup: %dx%d map in %.1fs, store %s" % (args.side, args.side, t_geom, args.store),
          file=sys.stderr, flush=True)

    for w in range(args.warmup):
        s.step(N_C)
    torch.cuda.synchronize()
    s.set_option(g.GLBM_OPT_TIMING, 1)  # reset the sweep timer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s.step(N_C)
        print("step %d/%d done" % (k + 1, args.steps), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms, launches = g.glbm_sweep_time(s.ctx)
    r, st = s.residual()
    kk = s.permeability()[0]
    s.close()

    lups = N * N_C * args.steps
    mlups = lups / wall / 1e6
    bytes_per_lu = g.bytes_per_update(9, store)
    per_launch = sweep_ms / max(launches, 1)
    achieved = bytes_per_lu * N / (per_launch * 1e-3) / 1e9
    traffic = traffic_from_profile(args.store, args.side)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16dev": "f32 math / f16 storage", "f16loc": "f32 math / f16 storage",
                  "f64": "f64"}[args.store],
        "data": "synthetic (seeded QSGS shale map, generated in-process)",
        "config": {"workload": "D2Q9 GLBM %dx%d, QSGS 60%% solid, TOC 0.10, CH4 400 K 10 MPa, %s "
                               "populations, n_c=%d sweeps + FP64 residual/flux per step"
                               % (args.side, args.side, args.store.upper(), N_C),
                   "nodes": N, "sweeps_per_step": N_C, "steps_total": int(st[0]),
                   "residual": float(r[0]), "k_lattice": float(kk[0])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_sweep<9,%s>" % args.store, "bytes_per_lu": bytes_per_lu,
                     "mean_launch_ms": round(per_launch, 5), "launches": launches},
    }
    if not args.no_cpu:
        y0, x0 = 0, 0
        crop = np.ascontiguousarray(cls[y0:y0 + 512, x0:x0 + 512])
        import oracle
        from oracle import kapp
        e_o, k_o, f_o = kapp.class_table(inst)
        v, dt, cores = cpu_baseline(crop, (e_o, k_o, f_o), args.cpu_steps)
        out["cpu_baseline"] = {"value": round(v, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                               "sample": "%d steps of a 512x512 crop of the same map (FP64 oracle, %.1f s)"
                                         % (args.cpu_steps, dt)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
