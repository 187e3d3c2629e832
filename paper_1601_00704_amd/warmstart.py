"""Learned warm start of batched GLBM solves: data generation, training, evaluation.

Orchestration only: every solve, feature map, target, network pass and
update runs in libglbm (include/glbm.h, include/glbm_cnn.h); PyTorch holds
the device buffers and slices them.

  1. cold-solve many QSGS instances with the batch engine to r <= tol and turn
     each converged state into a training target ((rho - 1)/s_rho, u/s_u);
  2. train the encoder-decoder on (features -> targets);
  3. on held-out instances, solve twice: from rest (cold) and from the
     equilibrium of the network's prediction (warm); report steps, wall time
     and the permeability difference.  The solver decides the answer: the warm
     solve iterates to the same residual as the cold one.

Run: python -m paper_1601_00704_amd.warmstart --train 2000 --test 200 --out report.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import glbm as g

N_C = 100


def _instances(seeds, side):
    import shale_inputs as si
    return [si.warmstart_instance(s, side) for s in seeds]


def _maps(insts):
    import shale_inputs as si
    return si.batch_classes(insts)


def _scales(G):
    """Normalisation of the targets.  The steady Stokes-regime fields are linear
    in G; on these maps pore velocities are of order G (lattice units) and
    density deviations of order 30 G, so both targets come out of order one."""
    return 30.0 * G, G


class Batch:
    """One GLBM context over many instances, with per-instance class tables."""

    def __init__(self, insts, maps, store="f32"):
        self.insts = insts
        self.descs = [g.make_desc(m.shape, store=g.STORE_NAMES[store], tau=i.tau, g=i.gvec(), check_every=N_C)
                      for i, m in zip(insts, maps)]
        self.s = g.Solver(self.descs, maps)
        if store == "f32":
            # two time steps per launch on 64 x 8 tiles (cache policy 71): the fastest
            # measured setting of the FP32 sweep on these maps, bitwise equal to one step
            # per launch
            self.s.set_option(g.GLBM_OPT_TILE_WIDTH, 64)
            self.s.set_option(g.GLBM_OPT_TILE_ROWS, 8)
            self.s.set_option(g.GLBM_OPT_CACHE, 71)
        for k, inst in enumerate(insts):
            r_iom, r_om = inst.radii()
            eps, kl = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
            self.s.set_local_perm(eps[:255], kl[:255], inst=k)

    def solve(self, tol, max_steps, trace_every=0):
        """Solve to r <= tol; with trace_every > 0, in chunks, recording the residuals."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.trace = []
        if trace_every <= 0:
            rc = self.s.step(max_steps, tol=tol)
        else:
            done = 0
            rc = g.GLBM_ENOTCONVERGED
            while done < max_steps and rc != g.GLBM_OK:
                rc = self.s.step(min(trace_every, max_steps - done), tol=tol)
                done += trace_every
                r, st = self.s.residual()
                self.trace.append([int(st.max())] + [float(v) for v in r[:4]])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r, st = self.s.residual()
        return wall, rc, r, st

    def close(self):
        self.s.close()


def generate(insts, maps, tol, max_steps, ctx_size, x, t, m, offset, G, store):
    """Cold-solve insts (ctx_size per context) and write features, targets and masks
    of sample offset + k into the device tensors x, t, m."""
    s_rho, s_u = _scales(G)
    per = []
    for c0 in range(0, len(insts), ctx_size):
        sub, sm = insts[c0:c0 + ctx_size], maps[c0:c0 + ctx_size]
        b = Batch(sub, sm, store)
        wall, rc, r, st = b.solve(tol, max_steps)
        k = b.s.permeability()[:, 0]
        for j, inst in enumerate(sub):
            n = offset + c0 + j
            g.glbm_cnn_features(b.s.ctx, j, math.log10(inst.pressure / 1e6), x[n].data_ptr())
            g.glbm_cnn_targets(b.s.ctx, j, s_rho, s_u, t[n].data_ptr(), m[n].data_ptr())
            per.append({"seed": inst.seed, "steps": int(st[j]), "residual": float(r[j]), "k_lattice": float(k[j])})
        b.close()
        print("generated %d/%d (batch wall %.1fs, max steps %d, rc %d)" % (c0 + len(sub), len(insts), wall,
                                                                          int(st.max()), rc), flush=True)
    return per


def train(cnn, x, t, m, n, epochs, batch, lr, H, W):
    xb = torch.empty((batch, H, W, 8), dtype=torch.int16, device="cuda")
    tb = torch.empty((batch, H, W, 4), dtype=torch.float32, device="cuda")
    mb = torch.empty((batch, H, W), dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cpu")
    gen.manual_seed(1234)
    hist = []
    steps = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen)
        losses = []
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / max(1, epochs)))
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch].to("cuda")
            torch.index_select(x, 0, idx, out=xb)
            torch.index_select(t, 0, idx, out=tb)
            torch.index_select(m, 0, idx, out=mb)
            losses.append(g.glbm_cnn_train_step(cnn, xb.data_ptr(), tb.data_ptr(), mb.data_ptr(), batch, lr_ep))
            steps += 1
        hist.append(float(np.mean(losses)))
        print("epoch %d loss %.5f (%.1fs)" % (ep, hist[-1], time.perf_counter() - t0), flush=True)
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0, steps


def evaluate(cnn, insts, maps, tol, max_steps, ctx_size, G, H, W, store, trace_every=0):
    """Cold and warm solves of the same instances; returns per-instance records and wall times
    (and, with trace_every, the residual histories of the first context)."""
    s_rho, s_u = _scales(G)
    out, cold_wall, warm_wall, infer_wall = [], 0.0, 0.0, 0.0
    traces = {}
    xb = torch.empty((1, H, W, 8), dtype=torch.int16, device="cuda")
    yb = torch.empty((1, H, W, 4), dtype=torch.float32, device="cuda")
    tb = torch.empty((1, H, W, 4), dtype=torch.float32, device="cuda")
    mb = torch.empty((1, H, W), dtype=torch.uint8, device="cuda")
    for c0 in range(0, len(insts), ctx_size):
        sub, sm = insts[c0:c0 + ctx_size], maps[c0:c0 + ctx_size]
        te = trace_every if c0 == 0 else 0
        cold = Batch(sub, sm, store)
        wc, rcc, rc_, stc = cold.solve(tol, max_steps, te)
        print("cold-solved %d/%d (%.1fs, max steps %d)" % (c0 + len(sub), len(insts), wc, int(stc.max())), flush=True)
        if te:
            traces["cold"] = cold.trace
        kc = cold.s.permeability()[:, 0]
        truth = []
        for j in range(len(sub)):
            g.glbm_cnn_targets(cold.s.ctx, j, s_rho, s_u, tb.data_ptr(), mb.data_ptr())
            truth.append((tb.cpu().numpy().reshape(H, W, 4).copy(), mb.cpu().numpy().reshape(H, W).copy()))
        cold.close()
        warm = Batch(sub, sm, store)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        preds = []
        for j, inst in enumerate(sub):
            g.glbm_cnn_features(warm.s.ctx, j, math.log10(inst.pressure / 1e6), xb.data_ptr())
            g.glbm_cnn_forward(cnn, xb.data_ptr(), yb.data_ptr(), 1)
            g.glbm_cnn_apply(warm.s.ctx, j, yb.data_ptr(), s_rho, s_u)
            preds.append(yb.clone())
        torch.cuda.synchronize()
        ti = time.perf_counter() - t0
        errs = [prediction_errors(p.cpu().numpy().reshape(H, W, 4), *truth[j]) for j, p in enumerate(preds)]
        ww, rcw, rw, stw = warm.solve(tol, max_steps, te)
        if te:
            traces["warm"] = warm.trace
        kw = warm.s.permeability()[:, 0]
        warm.close()
        cold_wall += wc
        warm_wall += ww
        infer_wall += ti
        for j, inst in enumerate(sub):
            out.append({"seed": inst.seed, "cold_steps": int(stc[j]), "warm_steps": int(stw[j]),
                        "k_cold": float(kc[j]), "k_warm": float(kw[j]),
                        "k_rel_diff": float(abs(kw[j] - kc[j]) / abs(kc[j])),
                        "cold_residual": float(rc_[j]), "warm_residual": float(rw[j]), **errs[j]})
        print("evaluated %d/%d: cold %.1fs, warm %.1fs + inference %.2fs" % (c0 + len(sub), len(insts), wc, ww, ti),
              flush=True)
    return out, cold_wall, warm_wall, infer_wall, traces


def prediction_errors(y, target, mask, block=16):
    """Relative L2 errors of a prediction against the converged fields (normalised units,
    fluid nodes): density, velocity, and the density averaged over block x block tiles
    (the large-scale part that sets how long the solve still takes)."""
    m = mask.astype(bool)
    d0, t0 = (y[..., 0] - target[..., 0]) * m, target[..., 0] * m
    du, tu = (y[..., 1:3] - target[..., 1:3]) * m[..., None], target[..., 1:3] * m[..., None]
    H, W = m.shape

    def coarse(a):
        return a.reshape(H // block, block, W // block, block).mean(axis=(1, 3))
    return {"rho_rel_err": float(np.linalg.norm(d0) / max(np.linalg.norm(t0), 1e-300)),
            "u_rel_err": float(np.linalg.norm(du) / max(np.linalg.norm(tu), 1e-300)),
            "rho_coarse_rel_err": float(np.linalg.norm(coarse(d0)) / max(np.linalg.norm(coarse(t0)), 1e-300))}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--side", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--ctx", type=int, default=256, help="instances per GLBM context")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--store", default="f32loc", choices=sorted(g.STORE_NAMES))
    ap.add_argument("--eval-store", default=None, choices=sorted(g.STORE_NAMES),
                    help="storage of the evaluation solves (default: --store)")
    ap.add_argument("--trace-every", type=int, default=0)
    ap.add_argument("--out", default="warmstart_report.json")
    ap.add_argument("--params-out", default=None)
    args = ap.parse_args(argv)

    H = W = args.side
    train_seeds = list(range(100000, 100000 + args.train))
    test_seeds = list(range(200000, 200000 + args.test))
    t0 = time.perf_counter()
    tr_insts, te_insts = _instances(train_seeds, args.side), _instances(test_seeds, args.side)
    tr_maps, te_maps = _maps(tr_insts), _maps(te_insts)
    print("maps: %.1fs" % (time.perf_counter() - t0), flush=True)
    G = tr_insts[0].g
    torch.cuda.set_device(0)
    n = len(tr_insts)
    x = torch.zeros((n, H, W, 8), dtype=torch.int16, device="cuda")
    t = torch.zeros((n, H, W, 4), dtype=torch.float32, device="cuda")
    m = torch.zeros((n, H, W), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    gen = generate(tr_insts, tr_maps, args.tol, args.max_steps, args.ctx, x, t, m, 0, G, args.store)
    gen_wall = time.perf_counter() - t0
    cnn = g.glbm_cnn_create(args.batch, H, W, seed=7)
    hist, train_wall, train_steps = train(cnn, x, t, m, n, args.epochs, args.batch, args.lr, H, W)
    del x, t, m
    torch.cuda.empty_cache()
    res, cw, ww, iw, traces = evaluate(cnn, te_insts, te_maps, args.tol, args.max_steps, args.ctx, G, H, W,
                                       args.eval_store or args.store, args.trace_every)
    if args.params_out:
        np.save(args.params_out, g.glbm_cnn_get_params(cnn))
        manifest = {"command": "python -m paper_1601_00704_amd.warmstart " + " ".join(argv if argv is not None
                                                                                    else sys.argv[1:]),
                    "train_seeds": [train_seeds[0], train_seeds[-1]], "test_seeds": [test_seeds[0], test_seeds[-1]],
                    "side": args.side, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
                    "store": args.store, "tol": args.tol, "final_loss": hist[-1] if hist else None,
                    "params": int(g.glbm_cnn_num_params(cnn)), "layout": "glbm_cnn_get_params (float32)"}
        with open(os.path.splitext(args.params_out)[0] + ".json", "w") as fh:
            json.dump(manifest, fh, indent=1)
    g.glbm_cnn_destroy(cnn)
    cs = np.array([r["cold_steps"] for r in res], float)
    ws = np.array([r["warm_steps"] for r in res], float)
    kd = np.array([r["k_rel_diff"] for r in res])
    report = {
        "store": args.store, "train_instances": n, "test_instances": len(res), "side": args.side, "tol": args.tol,
        "generation_wall_s": gen_wall, "train_wall_s": train_wall, "train_steps": train_steps,
        "loss_history": hist, "train_cold_steps_median": float(np.median([r["steps"] for r in gen])),
        "cold_wall_s": cw, "warm_wall_s": ww, "inference_wall_s": iw,
        "wall_speedup": cw / (ww + iw),
        "steps_ratio_median": float(np.median(cs / np.maximum(ws, 1))),
        "steps_cold_median": float(np.median(cs)), "steps_warm_median": float(np.median(ws)),
        "k_rel_diff_max": float(kd.max()), "k_rel_diff_median": float(np.median(kd)),
        "rho_rel_err_median": float(np.median([r["rho_rel_err"] for r in res])),
        "u_rel_err_median": float(np.median([r["u_rel_err"] for r in res])),
        "rho_coarse_rel_err_median": float(np.median([r["rho_coarse_rel_err"] for r in res])),
        "eval_store": args.eval_store or args.store, "traces": traces,
        "per_instance": res,
    }
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k not in ("per_instance", "loss_history", "traces")}),
          flush=True)


if __name__ == "__main__":
    main()
