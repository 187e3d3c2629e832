"""Throughput of the GLBM hot path on one MI355X.

One bench "step" is one check interval of the hot path on the whole lattice:
n_c = 100 stream-and-collide sweeps (Eq. 29-37 with per-node eps and K_app)
followed by the FP64 residual and Darcy-flux reductions of that state, all in
the HIP library.  The workload is a 4096 x 4096 D2Q9 shale map (seeded QSGS,
60% solid, TOC 0.10, methane at 400 K and 10 MPa) with FP32 populations.

The tile shape and cache policy of the sweep are chosen by the library's
autotuner (glbm_autotune) before the warm-up, or given with --tile.

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
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLBM MLUPS + % HBM peak; time-to-converged k_app, plain vs warm-start"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CUs at 2.4 GHz)
GMM_OPS_PER_SAMPLE_K2 = 25
N_C = 100


def opt_in(store):
    """The literal FP16 deviation store runs only as an explicit study form."""
    import paper_1601_00704_amd.glbm as g
    return g.GLBM_FLAG_F16DEV_OPT_IN if store == g.GLBM_STORE_F16DEV else 0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("glbm_kernels.hip", "glbm_internal.h"):
        with open(os.path.join(ROOT, "paper_1601_00704_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload_key(args):
    """(profile key, lattice Q, nodes) of the workload the arguments select."""
    if args.workload == "batch":
        import shale_inputs as si
        nodes = sum(int(np.prod(i.shape)) for i in si.uneven_batch(args.batch))
        return "sweep_batch%d_d2q9_%s" % (args.batch, args.store), 9, nodes
    if args.workload == "d3q19":
        return "sweep_d3q19_%s_%d" % (args.store, args.side3), 19, args.side3 ** 3
    return "sweep_d2q9_%s_%d" % (args.store, args.side), 9, args.side * args.side


def traffic_from_profile(key):
    """HBM bytes per sweep launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "%s_traffic.json" % key)
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


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """HBM bandwidth (GB/s, read + write) of the library's streaming copy (16-byte
    nontemporal loads and stores) and of torch's copy_, on the current stream."""
    import torch
    import paper_1601_00704_amd.glbm as g
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("stream_copy", lambda: g.glbm_stream_copy(a.data_ptr(), b.data_ptr(), nbytes)),
                     ("torch_copy", lambda: b.copy_(a))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(2.0 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pmc_per_kernel(path):
    import csv
    import glob
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def pmc_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, args):
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
    # the sweep kernel with the most dispatches in the run
    fd = _pmc_per_kernel(fetch_dir)
    main = max((k for k in fd if "k_sweep" in k), key=lambda k: len(fd[k]))
    sf, nf = pick(fd, main)
    sw, nw = pick(_pmc_per_kernel(write_dir), main)
    read = sf * 1024.0 * f_scale
    write = sw * 1024.0 * w_scale
    import paper_1601_00704_amd.glbm as g
    key, q, n = workload_key(args)
    bpl = g.bytes_per_update(q, g.STORE_NAMES[args.store])
    per = 2 if "k_sweep9tb" in main else 1
    bpl = bpl * per  # algorithmic bytes of the sweeps one launch performs, per node
    rec = {"kernel": "%s, %s, %d nodes" % (sweep_kernel(q, args.store, per), args.workload, n),
           "kernel_symbol": main,
           "sweeps_per_launch": per,
           "kernel_source_hash": kernel_source_hash(),
           "fetch_kib_per_launch": sf, "write_kib_per_launch": sw, "launches": [nf, nw],
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_read_bytes_per_launch": read, "hbm_write_bytes_per_launch": write,
           "hbm_bytes_per_launch": read + write,
           "algorithmic_bytes_per_launch": bpl * n,
           "traffic_over_algorithmic": (read + write) / (bpl * n)}
    path = os.path.join(ROOT, "profiles", "%s_traffic.json" % key)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


TWO_STEP_NOTE = ("two time steps per launch with the intermediate state in LDS: the algorithmic bytes of two "
                 "plain sweeps over the launch time can exceed the HBM peak; traffic is what HBM moved")


def sweep_kernel(q, store, per=1):
    """Name of the sweep kernel that runs for a lattice and store, `per` time
    steps per launch (glbm_sweeps_per_launch)."""
    if q == 19:
        return "k_sweep19<%s>" % store
    if per == 2:
        return "k_sweep9tb<%s> (two time steps per launch)" % store
    return ("k_sweep9<%s>" if store in ("f64", "f32", "f32loc") else "k_sweep<9,%s>") % store


def cpu_baseline(cls_crop, table, steps, threads=None):
    """Oracle MLUPS on a crop (all host threads, or `threads`)."""
    import oracle
    eps, k, fe = table
    all_threads = oracle.num_threads()
    if threads:
        oracle.set_threads(threads)
    try:
        prob = oracle.Problem(q=9, cls=cls_crop, eps=eps, k=k, f_eps=fe, tau=1.0, G=(1e-6, 0, 0))
        f = prob.rest()
        prob.run(f, 2)
        t0 = time.perf_counter()
        prob.run(f, steps)
        dt = time.perf_counter() - t0
        used = oracle.num_threads()
    finally:
        if threads:
            oracle.set_threads(all_threads)
    return cls_crop.size * steps / dt / 1e6, dt, used


def time_to_converge(store="f32", n=8, side=512, tol=1e-8, max_steps=2000000):
    """Time to converged k_app, plain (from rest) vs learned warm start, on held-out
    512^2 warm-start problems (seeds 200000 + k): both solves run all problems in one
    batched context to r <= tol; the warm time includes the network's inference and the
    equilibrium write of its prediction.  Network weights: paper_1601_00704_amd/weights."""
    import torch
    import shale_inputs as si
    import paper_1601_00704_amd.glbm as g
    from paper_1601_00704_amd import warmstart as ws
    wpath = os.path.join(ROOT, "paper_1601_00704_amd", "weights", "warmstart_cnn.npy")
    params = np.load(wpath, allow_pickle=False)
    with open(os.path.splitext(wpath)[0] + ".json") as fh:
        manifest = json.load(fh)
    insts = [si.warmstart_instance(200000 + k, side) for k in range(n)]
    maps = si.batch_classes(insts, processes=8)
    s_rho, s_u = ws._scales(insts[0].g)
    cold = ws.Batch(insts, maps, store)
    wc, rcc, rcold, stc = cold.solve(tol, max_steps)
    kc = cold.s.permeability()[:, 0]
    cold.close()
    print("time to converge: cold %.2fs, max steps %d" % (wc, int(stc.max())), file=sys.stderr, flush=True)
    cnn = g.glbm_cnn_create(1, side, side, seed=0)
    g.glbm_cnn_set_params(cnn, params)
    xb = torch.empty((1, side, side, 8), dtype=torch.int16, device="cuda")
    yb = torch.empty((1, side, side, 4), dtype=torch.float32, device="cuda")
    warm = ws.Batch(insts, maps, store)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, inst in enumerate(insts):
        g.glbm_cnn_features(warm.s.ctx, j, math.log10(inst.pressure / 1e6), xb.data_ptr())
        g.glbm_cnn_forward(cnn, xb.data_ptr(), yb.data_ptr(), 1)
        g.glbm_cnn_apply(warm.s.ctx, j, yb.data_ptr(), s_rho, s_u)
    torch.cuda.synchronize()
    ti = time.perf_counter() - t0
    ww, rcw, rwarm, stw = warm.solve(tol, max_steps)
    kw = warm.s.permeability()[:, 0]
    warm.close()
    g.glbm_cnn_destroy(cnn)
    print("time to converge: warm %.2fs + inference %.3fs, max steps %d" % (ww, ti, int(stw.max())),
          file=sys.stderr, flush=True)
    kd = np.abs(kw - kc) / np.abs(kc)
    return {"problems": n, "side": side, "tol": tol, "store": store,
            "cold": {"wall_s": round(wc, 3), "converged": int(rcc) == g.GLBM_OK, "steps": [int(v) for v in stc],
                     "steps_median": float(np.median(stc))},
            "warm": {"wall_s": round(ww + ti, 3), "inference_s": round(ti, 4), "converged": int(rcw) == g.GLBM_OK,
                     "steps": [int(v) for v in stw], "steps_median": float(np.median(stw))},
            "speedup_wall": round(wc / (ww + ti), 4), "steps_ratio_median": round(float(np.median(stc / stw)), 4),
            "k_rel_diff_max": float(kd.max()),
            "percolates_x": [g.glbm_pore_percolates(m, 1) for m in maps],
            "network": {"weights": "paper_1601_00704_amd/weights/warmstart_cnn.npy", "trained_by": manifest["command"],
                        "train_side": manifest["side"], "final_loss": manifest["final_loss"]}}


def _json_line(metric_unit_value, steps, warmup, ms_per_step, dtype, config, roofline, extra=None):
    out = {"metric": METRIC, "value": round(metric_unit_value, 1), "unit": "MLUPS", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded QSGS shale maps, generated in-process)", "config": config,
           "roofline": roofline}
    if extra:
        out.update(extra)
    return out


DTYPE = {"f32": "f32", "f16dev": "f32 math / f16 storage", "f16loc": "f32 math / f16 storage", "f32loc": "f32",
         "f64": "f64"}


def _choose_tile(s, g, args):
    """Tile shape and cache policy: given with --tile, else picked by glbm_autotune
    (unless --no-autotune); returns the config record or None (library defaults)."""
    if args.tile:
        s.set_option(g.GLBM_OPT_TILE_WIDTH, args.tile[0])
        s.set_option(g.GLBM_OPT_TILE_ROWS, args.tile[1])
        s.set_option(g.GLBM_OPT_CACHE, args.tile[2])
        return {"width": args.tile[0], "rows": args.tile[1], "cache_policy": args.tile[2], "by": "--tile"}
    if args.no_autotune:
        return None
    t0 = time.perf_counter()
    ch = g.glbm_autotune(s.ctx, 20)
    print("autotune: width %d rows %d cache %d (%.1fs)" % (ch[0], ch[1], ch[2], time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    return {"width": int(ch[0]), "rows": int(ch[1]), "cache_policy": int(ch[2]), "by": "glbm_autotune"}


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
    insts = si.uneven_batch(args.batch)
    t0 = time.perf_counter()
    maps = si.batch_classes(insts, processes=args.map_procs or None)
    t_geom = time.perf_counter() - t0
    import torch
    import paper_1601_00704_amd.glbm as g
    torch.cuda.set_device(0)
    store = g.STORE_NAMES[args.store]
    descs = [g.make_desc(m.shape, store=store, tau=i.tau, g=i.gvec(), check_every=N_C,
                    flags=opt_in(store)) for i, m in zip(insts, maps)]
    s = g.Solver(descs, maps)
    for k, inst in enumerate(insts):
        r_iom, r_om = inst.radii()
        eps, kl = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
        s.set_local_perm(eps[:255], kl[:255], inst=k)
    N = int(sum(m.size for m in maps))
    print("setup: %d instances, %d nodes, maps in %.1fs, store %s" % (len(maps), N, t_geom, args.store),
          file=sys.stderr, flush=True)
    tile = _choose_tile(s, g, args)
    wall = _timed_chunks(s, g, args.steps, args.warmup, graph=True)
    per_sweep, launches = _sweep_mean_ms(s, g)
    per = g.glbm_sweeps_per_launch(s.ctx)
    r, st = s.residual()
    s.close()
    bpl = g.bytes_per_update(9, store)
    per_launch = per_sweep * per
    achieved = bpl * N * per / (per_launch * 1e-3) / 1e9
    sides = sorted(set(int(m.shape[0]) for m in maps))
    cfg = {"workload": "batched D2Q9 GLBM: %d QSGS instances, sides %s, TOC U(0.05,0.30), P log-U(1,30) MPa, "
                       "P_L U(2,8) MPa, V_L U(0.002,0.008) m3/kg; %s populations; one HIP graph per "
                       "n_c=%d-sweep chunk + FP64 per-instance checks" % (len(maps), sides, args.store.upper(), N_C),
           "instances": len(maps), "nodes": N, "sweeps_per_step": N_C, "graph": True,
           "tile": tile,
           "median_residual": float(np.median(r)), "steps_total": int(st.max()),
           "percolating_instances": int(sum(g.glbm_pore_percolates(m, 1) for m in maps))}
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_from_profile(workload_key(args)[0]),
            "kernel": "%s over the flat tile list" % sweep_kernel(9, args.store, per),
            "bytes_per_lu": bpl, "sweeps_per_launch": per,
            "mean_launch_ms": round(per_launch, 5), "launches": launches // per}
    if per == 2:
        roof["note"] = TWO_STEP_NOTE
    return _json_line(N * N_C * args.steps / wall / 1e6, args.steps, args.warmup, wall / args.steps * 1e3,
                      DTYPE[args.store], cfg, roof)


def run_d3q19(args):
    """256^3 D3Q19: 3-D QSGS (55% solid, TOC 0.20, 20 MPa), drive along z,
    halfway bounce-back on the x and y faces."""
    import shale_inputs as si
    inst = si.shale3d(args.side3)
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
                    wall_faces=inst.wall_faces, check_every=N_C,
                    flags=opt_in(store))
    s = g.Solver([d], [cls])
    s.set_local_perm(eps[:255], kl[:255])
    N = cls.size
    print("setup: %s map in %.1fs" % (cls.shape, t_geom), file=sys.stderr, flush=True)
    tile = _choose_tile(s, g, args)
    wall = _timed_chunks(s, g, args.steps, args.warmup, graph=False)
    ms, n = g.glbm_sweep_time(s.ctx)
    per_launch = ms / max(n, 1)
    conv = None
    if args.converge_tol > 0:
        # time to converge, from rest, with graph replays of the n_c-sweep chunks
        import numpy as np
        s.set_fields(np.ones(N), np.zeros((3, N)))
        s.set_option(g.GLBM_OPT_TIMING, 0)
        s.set_option(g.GLBM_OPT_GRAPH, 1)
        _, st0 = s.residual()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, rc = 0, g.GLBM_ENOTCONVERGED
        while done < args.max_steps and rc != g.GLBM_OK:
            rc = s.step(min(20000, args.max_steps - done), tol=args.converge_tol)
            done += 20000
            rr, stt = s.residual()
            print("converge: %d steps, r %.3e" % (int(stt[0] - st0[0]), rr[0]), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        rr, stt = s.residual()
        conv = {"tol": args.converge_tol, "converged": rc == g.GLBM_OK, "steps": int(stt[0] - st0[0]),
                "residual": float(rr[0]), "wall_s": round(time.perf_counter() - t0, 2),
                "k_lattice": [float(v) for v in s.permeability()[0]]}
    r, st = s.residual()
    kk = s.permeability()[0]
    s.close()
    bpl = g.bytes_per_update(19, store)
    achieved = bpl * N / (per_launch * 1e-3) / 1e9
    cfg = {"workload": "D3Q19 GLBM %d^3, 3-D QSGS 55%% solid, TOC 0.20, CH4 400 K 20 MPa, drive z, walls on x/y "
                       "faces, %s populations" % (args.side3, args.store.upper()),
           "nodes": N, "sweeps_per_step": N_C, "steps_total": int(st[0]), "residual": float(r[0]),
           "k_lattice_z": float(kk[2]), "tile": tile}
    if conv:
        cfg["time_to_converge"] = conv
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_from_profile(workload_key(args)[0]),
            "kernel": sweep_kernel(19, args.store), "bytes_per_lu": bpl,
            "mean_launch_ms": round(per_launch, 5), "launches": n}
    return _json_line(N * N_C * args.steps / wall / 1e6, args.steps, args.warmup, wall / args.steps * 1e3,
                      DTYPE[args.store], cfg, roof)


def run_pressure(args):
    """The 4096^2 map driven by pressure faces along x (10.5 -> 9.5 MPa around the map's
    10 MPa) with K_app of Eq. 18-19 evaluated at every node's local pressure."""
    import torch
    import shale_inputs as si
    import paper_1601_00704_amd.glbm as g
    inst = si.shale4096(args.side)
    cls = inst.classes()
    torch.cuda.set_device(0)
    store = g.STORE_NAMES[args.store]
    prm = g.gas_params(inst)
    eps, kc, kk, ks, b = g.glbm_class_table_pressure(prm, *inst.radii())
    d = g.make_desc(cls.shape, store=store, tau=inst.tau, g=(0, 0, 0), check_every=N_C, flags=opt_in(store),
                    pressure_axis=0, rho_in=1.0 + 5e-5, rho_out=1.0 - 5e-5)
    s = g.Solver([d], [cls])
    s.set_pressure_perm(eps[:255], kc[:255], kk[:255], ks[:255], b[:255], inst.pressure + 0.5e6,
                        inst.pressure - 0.5e6)
    N = cls.size
    tile = _choose_tile(s, g, args)
    wall = _timed_chunks(s, g, args.steps, args.warmup, graph=False)
    ms, n = g.glbm_sweep_time(s.ctx)
    per = g.glbm_sweeps_per_launch(s.ctx)
    per_launch = ms / max(n, 1) * per  # the library counts sweeps
    r, st = s.residual()
    kx = s.permeability()[0, 0]
    s.close()
    bpl = g.bytes_per_update(9, store)
    achieved = bpl * N * per / (per_launch * 1e-3) / 1e9
    cfg = {"workload": "D2Q9 GLBM %dx%d QSGS map (TOC 0.10), pressure faces on x 10.5 -> 9.5 MPa, K_app(P) at every "
                       "node, %s populations" % (args.side, args.side, args.store.upper()),
           "nodes": N, "sweeps_per_step": N_C, "steps_total": int(st[0]), "residual": float(r[0]),
           "k_p_lattice": float(kx), "percolates_x": g.glbm_pore_percolates(cls, 1), "tile": tile}
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "kernel": "%s, pressure faces + K(P)" % sweep_kernel(9, args.store, per), "bytes_per_lu": bpl,
            "sweeps_per_launch": per, "mean_launch_ms": round(per_launch, 5), "launches": n // per}
    if per == 2:
        roof["note"] = TWO_STEP_NOTE
    return _json_line(N * N_C * args.steps / wall / 1e6, args.steps, args.warmup, wall / args.steps * 1e3,
                      DTYPE[args.store], cfg, roof)


def run_gmm(args):
    """Batched EM fit of pore-size mixtures (Sec. 2.2): 64 sets of 2^20 log-radius samples,
    two components, a fixed number of iterations; throughput in samples x iterations / s."""
    import torch
    import shale_inputs as si
    import paper_1601_00704_amd.glbm as g
    torch.cuda.set_device(0)
    n_sets, m, iters = 64, 1 << 20, args.gmm_iters
    xs = np.concatenate([np.log(si.pore_radius_samples(9000 + k, m)) for k in range(n_sets)])
    xd = torch.from_numpy(xs).cuda()
    offs = np.arange(n_sets + 1, dtype=np.int64) * m
    st = (np.full((n_sets, 2), 0.5), np.tile([math.log(3e-9), math.log(30e-9)], (n_sets, 1)),
          np.full((n_sets, 2), 0.5))
    g.glbm_gmm_fit(offs, xd.data_ptr(), *st, 2)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, mu, var, ll, it = g.glbm_gmm_fit(offs, xd.data_ptr(), *st, iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    passes = iters + 1
    # FP64 operations per sample and pass for k = 2, Eq. 20-24 as computed (an exp,
    # log or division counts as one): log-densities 2 x 4, responsibilities 5,
    # shifted sums 2 x 5, log-likelihood 2
    ops = GMM_OPS_PER_SAMPLE_K2 * n_sets * m * passes
    achieved = ops / wall / 1e12
    cfg = {"workload": "batched EM fit, %d sets x %d samples (ln r of a two-phase lognormal PSD), k = 2, %d "
                       "iterations, FP64" % (n_sets, m, iters),
           "sets": n_sets, "samples_per_set": m, "iterations": iters,
           "median_fitted_medians_nm": [float(np.median(np.exp(np.sort(mu, axis=1)[:, j])) * 1e9) for j in (0, 1)]}
    roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
            "kernel": "k_gmm_pass<2> + k_gmm_update (%d FP64 operations per sample and pass, an exp, log or "
                      "division counted as one; 8 B per sample and pass, %.0f GB/s; wall time of the whole fit)"
                      % (GMM_OPS_PER_SAMPLE_K2, 8.0 * n_sets * m * passes / wall / 1e9)}
    return {"metric": "EM pore-size fit throughput", "value": round(n_sets * m * passes / wall / 1e9, 3),
            "unit": "Gsample-iterations/s", "n_gpus": 1, "steps": iters, "warmup": 1,
            "ms_per_step": round(wall / passes * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded lognormal pore radii)", "config": cfg,
            "roofline": roof}


def run_studies(args):
    """The paper's layout (Sec. 3.2) and TOC (Sec. 3.3) studies at its 16 x 8 um domain
    (256 x 128 nodes), pressure-driven 0.2 -> 0.1 MPa, every sample of a study in one
    batched context, solved to r <= 1e-8."""
    import torch
    import shale_inputs as si
    from paper_1601_00704_amd import studies
    torch.cuda.set_device(0)
    out = {}
    total_lu, total_wall = 0.0, 0.0
    for name, cases in (("layout", si.layout_study(realizations=2)), ("toc", si.toc_study())):
        res, run = studies.solve_study(cases, store=args.store, tol=1e-8, max_steps=args.max_steps,
                                       tile=tuple(args.tile) if args.tile else None)
        total_lu += run["lattice_updates"]
        total_wall += run["wall_s"]
        out[name] = {"run": run, "samples": [{k: v for k, v in r.items() if k not in ("name",)} for r in res]}
        print("study %s: %.1fs, max steps %d, rc %d" % (name, run["wall_s"], run["max_steps"], run["rc"]),
              file=sys.stderr, flush=True)
    cfg = {"workload": "paper studies (layout cases 1-4 x 2 realizations; TOC 0.2-0.8 x D_s 1e-9..1e-5), "
                       "256 x 128 nodes each, pressure faces 0.2 -> 0.1 MPa, K_app(P) per node, %s" % args.store.upper(),
           "studies": out}
    return {"metric": "GLBM study throughput (solved to r <= 1e-8)", "value": round(total_lu / total_wall / 1e6, 1),
            "unit": "MLUPS", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(total_wall * 1e3, 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.store],
            "data": "synthetic (seeded layout and QSGS maps, Tab. 6 / Tab. 7 inputs)", "config": cfg,
            "roofline": None}


# (cin, cout, level) of the ten convolutions of the warm-start network; level l runs at H/2^l
CNN_LAYERS = [(8, 32, 0), (32, 32, 0), (32, 64, 1), (64, 64, 1), (64, 128, 2), (128, 128, 2),
              (192, 64, 1), (64, 64, 1), (96, 32, 0), (32, 3, 0)]


def run_cnn(args):
    """Warm-start network on the GPU: whole-network inference and training-step
    throughput at B x side x side, and the dominant convolution on its own
    (BF16 MFMA, FP32 accumulate) against the dense BF16 peak."""
    import numpy as np
    import torch
    import paper_1601_00704_amd.glbm as g
    torch.cuda.set_device(0)
    B, H = args.cnn_batch, args.cnn_side
    W = H
    flops = sum(2.0 * (H >> l) * (W >> l) * co * 9 * ci for ci, co, l in CNN_LAYERS)
    rng = np.random.default_rng(0)
    x = np.zeros((B, H, W, 8), np.float32)
    x[..., :6] = rng.standard_normal((B, H, W, 6))
    xd = torch.from_numpy(g.to_bf16_bits(x).view(np.int16)).cuda()
    yd = torch.zeros(B * H * W * 4, dtype=torch.float32, device="cuda")
    td = torch.from_numpy(rng.standard_normal((B, H, W, 4)).astype(np.float32)).cuda()
    md = torch.ones((B, H, W), dtype=torch.uint8, device="cuda")
    cnn = g.glbm_cnn_create(B, H, W, seed=7)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    fwd_ms = timed(lambda: g.glbm_cnn_forward(cnn, xd.data_ptr(), yd.data_ptr(), B), args.steps)
    print("forward %.3f ms per batch of %d" % (fwd_ms, B), file=sys.stderr, flush=True)
    train_ms = timed(lambda: g.glbm_cnn_train_step(cnn, xd.data_ptr(), td.data_ptr(), md.data_ptr(), B, 1e-4),
                     args.steps)
    print("train step %.3f ms per batch of %d" % (train_ms, B), file=sys.stderr, flush=True)
    g.glbm_cnn_destroy(cnn)
    # the dominant convolution alone: 96 -> 32 channels at full resolution
    ci, co = 96, 32
    kp = -(-(9 * ci) // 32) * 32
    xc = torch.from_numpy(g.to_bf16_bits(rng.standard_normal((B, H, W, ci)).astype(np.float32)).view(np.int16)).cuda()
    wc = torch.from_numpy(g.to_bf16_bits((0.03 * rng.standard_normal((co, kp))).astype(np.float32))
                          .view(np.int16)).cuda()
    bc = torch.zeros(co, dtype=torch.float32, device="cuda")
    yc = torch.empty(B * H * W * co, dtype=torch.int16, device="cuda")
    conv_ms = timed(lambda: g.glbm_conv3x3_forward(xc.data_ptr(), ci, 0, ci, wc.data_ptr(), bc.data_ptr(),
                                                    yc.data_ptr(), co, 0, co, 1, 0, 0, B, H, W), args.steps)
    conv_flops = 2.0 * B * H * W * co * 9 * ci
    achieved = conv_flops / (conv_ms * 1e-3) / 1e12
    cfg = {"workload": "warm-start encoder-decoder (32/64/128 channels, 3x3, BF16 activations and weights, "
                       "FP32 accumulate), batch %d at %dx%d" % (B, H, W),
           "flop_per_sample": flops, "forward_ms_per_batch": round(fwd_ms, 3),
           "train_step_ms_per_batch": round(train_ms, 3),
           "forward_tflops": round(flops * B / (fwd_ms * 1e-3) / 1e12, 1),
           "train_tflops": round(3 * flops * B / (train_ms * 1e-3) / 1e12, 1)}
    roof = {"bound": "mfma", "achieved": round(achieved, 1), "peak": 2500.0, "unit": "TFLOP/s",
            "frac": round(achieved / 2500.0, 4), "traffic": None,
            "kernel": "conv3x3 forward 96->32 channels, %d x %dx%d, bf16 MFMA 16x16x32" % (B, H, W),
            "flop_per_launch": conv_flops, "mean_launch_ms": round(conv_ms, 4)}
    out = {"metric": "warm-start network inference throughput", "value": round(B / (fwd_ms * 1e-3), 1),
           "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(fwd_ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16", "data": "synthetic (random features)", "config": cfg, "roofline": roof}
    return out


def main():

    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 80 for the benchmark line, at least 8000 sweeps and about "
                         "1 s of timed work; 10 for the other workloads)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side", type=int, default=4096)
    ap.add_argument("--store", default=None, choices=("f32", "f16dev", "f16loc", "f32loc", "f64"),
                    help="population store (default: f64 for the studies, which are solved to r <= 1e-8 "
                         "under a pressure drive, f32 otherwise)")
    ap.add_argument("--cpu-steps", type=int, default=4000, help="oracle steps of the CPU baseline (about 10 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="shale4096",
                    choices=("shale4096", "batch", "d3q19", "cnn", "pressure", "gmm", "studies"),
                    help="shale4096: the benchmark line; the others: supplementary workloads")
    ap.add_argument("--gmm-iters", type=int, default=50)
    ap.add_argument("--cnn-batch", type=int, default=8)
    ap.add_argument("--cnn-side", type=int, default=512)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true", help="keep the library's default tile shape")
    ap.add_argument("--tile", type=int, nargs=3, metavar=("WIDTH", "ROWS", "CACHE"),
                    help="use this tile shape and cache policy instead of the autotuner's")
    ap.add_argument("--map-procs", type=int, default=0,
                    help="worker processes for the batch's maps (0: one per core, at most 16)")
    ap.add_argument("--side3", type=int, default=256)
    ap.add_argument("--converge-tol", type=float, default=0.0,
                    help="d3q19: after the timed steps, solve from rest to this residual and report it")
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the time-to-converge leg (plain vs warm start) of the benchmark line")
    ap.add_argument("--converge-problems", type=int, default=8)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB elementwise copy (counter calibration)")
    ap.add_argument("--forchheimer", action="store_true",
                    help="benchmark line with the inertial drag of Eq. 27 on every matrix class (Ergun F_eps)")
    ap.add_argument("--record", default=None, metavar="PATH",
                    help="append a JSON record of the run (workload, seed, steps, r, k, throughput, HBM fraction, "
                         "wall time, oracle rate, host threads) to PATH")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="summarise rocprofv3 --pmc output directories into profiles/")
    args = ap.parse_args()
    if args.store is None:
        args.store = "f64" if args.workload == "studies" else "f32"
    if args.steps is None:
        args.steps = 80 if args.workload == "shale4096" else 10
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the GLBM hot path here is built and timed on a single "
              "MI355X; sharding over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    runs = {"batch": run_batch, "d3q19": run_d3q19, "cnn": run_cnn, "pressure": run_pressure, "gmm": run_gmm,
            "studies": run_studies, "shale4096": run_shale4096}
    line = runs[args.workload](args)
    print(json.dumps(line), flush=True)
    if args.record:
        append_record(args.record, args, line)


def append_record(path, args, line):
    """Append one JSON line per run to `path`: the workload, its seed where it has one,
    the solver's state and k, the throughput and HBM fraction, the wall time, the oracle's
    CPU rate and the host's thread count."""
    cfg = line.get("config", {})
    roof = line.get("roofline") or {}
    cpu = line.get("cpu_baseline") or {}
    rec = {"time": time.strftime("%Y-%m-%dT%H:%M:%S"), "workload": args.workload, "config": cfg.get("workload"),
           "store": args.store, "seed": cfg.get("seed"), "steps_total": cfg.get("steps_total"),
           "residual": cfg.get("residual", cfg.get("median_residual")), "k_lattice": cfg.get("k_lattice"),
           "k_m2": cfg.get("k_m2"), "k_mD": cfg.get("k_mD"), "percolates_x": cfg.get("percolates_x"),
           "metric": line.get("metric"), "value": line.get("value"), "unit": line.get("unit"),
           "hbm_frac": roof.get("frac"), "wall_s": round(line.get("ms_per_step", 0.0) * line.get("steps", 0) / 1e3, 3),
           "oracle_mlups": cpu.get("value"), "host_threads": os.cpu_count()}
    with open(path, "a") as fh:
        fh.write(json.dumps(rec) + "\n")


def run_shale4096(args):
    """The benchmark line: the 4096^2 D2Q9 map, autotuned, timed over args.steps checks of
    n_c sweeps each, then the time-to-converge leg and the oracle's CPU rate."""
    import numpy as np
    import torch
    import shale_inputs as si
    import paper_1601_00704_amd.glbm as g

    torch.cuda.set_device(0)
    inst = si.shale4096(args.side)
    t0 = time.perf_counter()
    cls = inst.classes()
    t_geom = time.perf_counter() - t0
    r_iom, r_om = inst.radii()
    eps, kl = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
    store = g.STORE_NAMES[args.store]
    d = g.make_desc(cls.shape, store=store, tau=inst.tau, g=inst.gvec(), check_every=N_C,
                    flags=opt_in(store))
    s = g.Solver([d], [cls])
    fe = None
    if args.forchheimer:
        # the geometric function of the inertial drag (Eq. 27) in the Ergun form of
        # the generalized LBE's source, F_eps = 1.75 / sqrt(150 eps^3); it acts only
        # where K is finite (the open pores carry no drag)
        fe = np.where(np.isfinite(kl), 1.75 / np.sqrt(150.0 * eps ** 3), 0.0)[:255]
    s.set_local_perm(eps[:255], kl[:255], fe)
    N = cls.size
    print("setup: %dx%d map in %.1fs, store %s" % (args.side, args.side, t_geom, args.store),
          file=sys.stderr, flush=True)
    tile = _choose_tile(s, g, args)
    s.set_option(g.GLBM_OPT_GRAPH, 0)
    s.set_option(g.GLBM_OPT_TIMING, 1)

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
    per = g.glbm_sweeps_per_launch(s.ctx)
    r, st = s.residual()
    kk = s.permeability()[0]
    s.close()

    lups = N * N_C * args.steps
    mlups = lups / wall / 1e6
    bytes_per_lu = g.bytes_per_update(9, store)
    # the library counts sweeps (a two-step launch counts as two); a launch of the
    # chosen kernel performs `per` sweeps
    per_sweep = sweep_ms / max(launches, 1)
    per_launch = per_sweep * per
    achieved = bytes_per_lu * N * per / (per_launch * 1e-3) / 1e9
    traffic = traffic_from_profile(workload_key(args)[0])
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
        "dtype": DTYPE[args.store],
        "data": "synthetic (seeded QSGS shale map, generated in-process)",
        "config": {"workload": "D2Q9 GLBM %dx%d, QSGS 60%% solid, TOC 0.10, CH4 400 K 10 MPa, %s "
                               "populations, n_c=%d sweeps + FP64 residual/flux per step"
                               % (args.side, args.side, args.store.upper(), N_C),
                   "nodes": N, "sweeps_per_step": N_C, "steps_total": int(st[0]),
                   "residual": float(r[0]), "k_lattice": float(kk[0]), "seed": inst.seed,
                   "k_m2": float(kk[0]) * inst.dx ** 2, "k_mD": float(kk[0]) * inst.dx ** 2 / 9.869233e-13 * 1e3,
                   "percolates_x": g.glbm_pore_percolates(cls, 1), "tile": tile,
                   "forchheimer": "F_eps = 1.75 / sqrt(150 eps^3) per class" if args.forchheimer else None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": sweep_kernel(9, args.store, per),
                     "bytes_per_lu": bytes_per_lu, "sweeps_per_launch": per,
                     "mean_launch_ms": round(per_launch, 5), "launches": launches // per,
                     "measured_copy_gbs": copy_bandwidth()},
    }
    if per == 2:
        out["roofline"]["note"] = TWO_STEP_NOTE
    if not args.no_converge:
        out["time_to_converge"] = time_to_converge(args.store if args.store in ("f32", "f32loc", "f64") else "f32",
                                                   n=args.converge_problems)
    if not args.no_cpu:
        y0, x0 = 0, 0
        crop = np.ascontiguousarray(cls[y0:y0 + 512, x0:x0 + 512])
        import oracle
        from oracle import kapp
        e_o, k_o, f_o = kapp.class_table(inst)
        v, dt, cores = cpu_baseline(crop, (e_o, k_o, f_o), args.cpu_steps)
        v1, dt1, _ = cpu_baseline(crop, (e_o, k_o, f_o), max(args.cpu_steps // 16, 20), threads=1)
        out["cpu_baseline"] = {"value": round(v, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                               "sample": "%d steps of a 512x512 crop of the same map (FP64 oracle, %.1f s)"
                                         % (args.cpu_steps, dt),
                               "single_thread_value": round(v1, 2), "single_thread_sample":
                                   "%d steps of the same crop on 1 thread (%.1f s)" % (max(args.cpu_steps // 16, 20),
                                                                                      dt1),
                               "cpu_model": cpu_model(), "host_threads": os.cpu_count()}
    return out


if __name__ == "__main__":
    main()
