"""Train the learned warm start on solves the library itself generates, then
measure it on held-out geometries.

    python -m paper_1412_7466_amd.train_warm --out warm_start.npz

1. Training set: geometries inputs.warm_problem(i) (the M=1000 workload's rules
   with M uniform in [M_lo, M_hi], P = 20, (omega, phi) from a 4 x 4 grid over
   omega in [10, 40] and phi in [-pi/3, pi/3], each grid cell sharing one
   factorization of the layers), each solved by FP64 GMRES to 1e-10; the network's
   inputs and exact target (every order |n| <= p_out = P by default) are kept on the
   GPU (grt_nn_add_sample).
2. Adam on the GPU (grt_nn_train), one geometry per step.
3. Held-out geometries (other seeds): FP64 GMRES to 1e-9 from x0 = 0 and from the
   network's guess (prediction time included), iterations and time for both, and
   the normalised error of the guess against the cold solution (with the
   single-scattering guess s alpha0 for reference).

Writes the FP32 weights, the configuration and the measured summary to --out.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=1024)
    ap.add_argument("--n-held", type=int, default=128)
    ap.add_argument("--M-lo", type=int, default=200)
    ap.add_argument("--M-hi", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--width", type=int, default=128)
    ap.add_argument("--layers", type=int, default=3)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--p-out", type=int, default=20)
    ap.add_argument("--restart", type=int, default=800)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="warm_start.npz")
    ap.add_argument("--load", default=None,
                    help="evaluate the network stored in this file (no training)")
    a = ap.parse_args(argv)

    import torch
    from . import inputs
    from .grating import Context, Network

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    loaded = None
    if a.load:
        loaded = np.load(a.load)
        a.width, a.layers, a.k, a.p_out = (int(v) for v in loaded["config"])
    net = Network(a.width, a.layers, a.k, a.p_out)
    net.set_params(inputs.nn_init(a.width, a.layers, a.p_out, seed=a.seed) if loaded is None
                   else loaded["theta"])
    anchors = {}   # one live context per (omega, phi) keeps the shared layer factors

    def build(pb):
        ctx = Context(0)
        ctx.set_problem(pb)
        ctx.build()
        anchors.setdefault((pb.omega, pb.phi), ctx)
        return ctx

    t0 = time.perf_counter()
    ids, train_iters = [], []
    if loaded is not None:
        a.n_train, a.epochs = 0, 0
    for i in range(a.n_train):
        pb = inputs.warm_problem(i, M_range=(a.M_lo, a.M_hi))
        ctx = build(pb)
        beta, st = ctx.solve(tol=1e-10, restart=a.restart, maxit=3000)
        ids.append(net.add_sample(ctx, beta))
        train_iters.append(st.iters)
        if ctx is not anchors[(pb.omega, pb.phi)]:
            ctx.close()
        if (i + 1) % 32 == 0:
            log(f"[train] solved {i + 1}/{a.n_train} geometries ({time.perf_counter() - t0:.1f}s)")
    t_data = time.perf_counter() - t0

    t1 = time.perf_counter()
    losses = []
    chunk = max(1, a.epochs // 10)
    done = 0
    while done < a.epochs:
        e = min(chunk, a.epochs - done)
        lr = a.lr * (0.5 * (1 + math.cos(math.pi * done / a.epochs)))
        losses.append(net.train(ids, epochs=e, lr=lr, seed=a.seed + done))
        done += e
        log(f"[train] epoch {done}/{a.epochs} loss {losses[-1]:.4e} ({time.perf_counter() - t1:.1f}s)")
    t_train = time.perf_counter() - t1
    net.clear_samples()

    rows = []
    for i in range(a.n_held):
        pb = inputs.warm_problem(i, held_out=True, M_range=(a.M_lo, a.M_hi))
        ctx = build(pb)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        bc, sc = ctx.solve(tol=1e-9, restart=a.restart, maxit=3000)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc
        tw = time.perf_counter()
        x0 = net.predict(ctx)
        bw, sw = ctx.solve(tol=1e-9, restart=a.restart, maxit=3000, x0=x0)
        torch.cuda.synchronize()
        tw = time.perf_counter() - tw
        # normalised error of the guesses against the cold solution
        ref = bc.cpu().numpy()
        b0 = ctx.rhs().cpu().numpy()
        g = x0.cpu().numpy()
        from_b = np.linalg.norm(b0 - ref) / np.linalg.norm(ref)
        from_nn = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        agree = np.linalg.norm(bw.cpu().numpy() - ref) / np.linalg.norm(ref)
        rows.append(dict(M=pb.M, omega=pb.omega, phi=pb.phi, iters_cold=sc.iters,
                         iters_warm=sw.iters, t_cold=tc, t_warm=tw, err_single=from_b,
                         err_nn=from_nn, rejected=sw.x0_rejected, warm_vs_cold=agree))
        log(f"[eval] M={pb.M} iters cold {sc.iters} warm {sw.iters} "
            f"err single {from_b:.3e} nn {from_nn:.3e} rejected {sw.x0_rejected}")
        if ctx is not anchors[(pb.omega, pb.phi)]:
            ctx.close()

    ic = np.array([r["iters_cold"] for r in rows], float)
    iw = np.array([r["iters_warm"] for r in rows], float)
    tcs = np.array([r["t_cold"] for r in rows])
    tws = np.array([r["t_warm"] for r in rows])
    summary = dict(
        n_train=a.n_train, n_held=a.n_held, M_range=[a.M_lo, a.M_hi], epochs=a.epochs,
        lr=a.lr, width=a.width, layers=a.layers, k=a.k, p_out=a.p_out,
        data_seconds=t_data, train_seconds=t_train, final_loss=losses[-1] if losses else None,
        loss_curve=losses, train_iters_mean=float(np.mean(train_iters)) if train_iters else None,
        held_iters_cold_mean=float(ic.mean()), held_iters_warm_mean=float(iw.mean()),
        held_seconds_cold=float(tcs.sum()), held_seconds_warm=float(tws.sum()),
        held_err_single_mean=float(np.mean([r["err_single"] for r in rows])),
        held_err_nn_mean=float(np.mean([r["err_nn"] for r in rows])),
        held_rejected=int(sum(r["rejected"] for r in rows)),
        held_warm_vs_cold_max=float(max(r["warm_vs_cold"] for r in rows)),
        rows=rows)
    if loaded is not None:
        # evaluation of a stored network: keep the record of its training
        prev = json.loads(str(loaded["summary"]))
        for k in ("n_train", "M_range", "epochs", "lr", "data_seconds", "train_seconds",
                  "final_loss", "loss_curve", "train_iters_mean"):
            if k in prev:
                summary[k] = prev[k]
        summary["evaluated_from"] = a.load
    log("[summary] " + json.dumps({k: v for k, v in summary.items() if k != "rows"}))
    theta = net.get_params()
    np.savez(a.out, theta=theta,
             config=np.array([a.width, a.layers, a.k, a.p_out], dtype=np.int64),
             summary=json.dumps(summary))
    log(f"[train] wrote {a.out}")


if __name__ == "__main__":
    main()
