"""Train the warm-start network and compare the three ways of solving the local
spectral problems (dense Jacobi, DCT-II start, network start) on a held-out field.

    python -m paper_1807_07220_amd.train_warmstart [--train-seeds 6] [--steps 3000]
        [--out paper_1807_07220_amd/data/warmstart_b16.npy] [--eval-only]

Training fields: 1024 x 1024 channelized permeability (contrast 1e6, the
generator of the 1024 x 1024 workloads) with seeds 10000, 10001, ...; every
interior coarse face of 16 x 16 blocks is one sample (8064 per field), its
targets the eigenvectors of the face's pencil from an exact setup.  The
evaluation field is the 1024 x 1024 workload's own (seed 3), not seen in
training.  Prints one JSON line per mode and writes the weights as .npy.
With --eval-only the stored weights are evaluated without training, and every
mode runs with the FP64 and the FP32 preconditioner: setup + solve time to
relative residual 1e-8 and the solution's difference from the FP64 exact-setup
solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def evaluate(kd, Fd, w, tol, weights=None, reps=3, precision="fp64", ref_u=None):
    import numpy as np
    import torch

    import paper_1807_07220_amd as tg
    out = {}
    for mode in ("exact", "dct", "cnn"):
        ts, tv = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = tg.Solver(kd, w.bx, w.by, tol, warm_start=mode, cnn_weights=weights if mode == "cnn" else None,
                          precision=precision)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = s.solve(Fd, rtol=w.rtol)
            torch.cuda.synchronize()
            ts.append(t1 - t0)
            tv.append(time.perf_counter() - t1)
            if len(ts) < reps:
                s.close()
        inf = s.info()
        u = r["u"].cpu().numpy()
        if ref_u is None and mode == "exact":
            ref_u = u
        rec = {"mode": mode, "precision": precision, "setup_s": float(np.median(ts)), "solve_s": float(np.median(tv)),
               "setup_plus_solve_s": float(np.median(np.add(ts, tv))), "t_eig_ms": inf["t_eig_ms"],
               "t_cnn_ms": inf["t_cnn_ms"], "faces": inf["n_coarse_faces"], "dim": inf["dim"],
               "pcg_iters": r["iters"], "u_rel_diff_vs_fp64_exact": float(np.linalg.norm(u - ref_u) / np.linalg.norm(ref_u)),
               "counts": s.counts()}
        if mode != "exact":
            st = s.warm_status()
            rec.update(accepted=int(np.sum(st >= 0)), mean_iters=float(st[st >= 0].mean()) if np.any(st >= 0) else None,
                       iter_histogram=np.bincount(st + 1).tolist())
        s.close()
        out[mode] = rec
    return out, ref_u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", type=int, default=6)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=os.path.join(HERE, "data", "warmstart_b16.npy"))
    ap.add_argument("--eval-only", action="store_true", help="evaluate the stored weights (FP64 and FP32 preconditioner)")
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_1807_07220_amd import warmstart as ws
    from workloads import configs, fields
    w = configs.get("darcy2d_1024_b16")
    if args.eval_only:
        weights = ws.load_weights(args.out)
        kappa, F = w.make_inputs()
        kd = torch.tensor(kappa, device="cuda:0")
        Fd = torch.tensor(F, device="cuda:0")
        ref = None
        for prec in ("fp64", "mixed"):
            res, ref = evaluate(kd, Fd, w, w.eig_tol, weights, precision=prec, ref_u=ref)
            for m, rec in res.items():
                rec = dict(rec)
                rec["counts_equal_exact"] = bool(np.array_equal(rec.pop("counts"), res["exact"]["counts"]))
                print(json.dumps({"workload": w.name, **rec}), flush=True)
        return
    t0 = time.perf_counter()
    train_fields = [fields.field_channelized(w.nx, w.ny, 10000 + i, contrast=w.contrast) for i in range(args.train_seeds)]
    X, V = ws.collect_samples(train_fields, w.bx, w.eig_tol)
    torch.cuda.synchronize()
    print(json.dumps({"samples": X.shape[0], "window": list(X.shape[1:]), "s": time.perf_counter() - t0}), flush=True)
    t0 = time.perf_counter()
    weights, losses = ws.train(X, V, k=8, steps=args.steps, batch=args.batch, lr=args.lr, seed=0)
    torch.cuda.synchronize()
    print(json.dumps({"train_steps": args.steps, "s": time.perf_counter() - t0, "loss_first": float(np.mean(losses[:20])),
                      "loss_last": float(np.mean(losses[-100:]))}), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    ws.save_weights(args.out, weights)
    kappa, F = w.make_inputs()
    kd = torch.tensor(kappa, device="cuda:0")
    Fd = torch.tensor(F, device="cuda:0")
    res, _ = evaluate(kd, Fd, w, w.eig_tol, weights)
    same = {m: bool(np.array_equal(res[m]["counts"], res["exact"]["counts"])) for m in ("dct", "cnn")}
    for m, rec in res.items():
        rec = dict(rec)
        rec.pop("counts")
        rec["counts_equal_exact"] = same.get(m, True)
        print(json.dumps({"workload": w.name, **rec}), flush=True)


if __name__ == "__main__":
    main()
