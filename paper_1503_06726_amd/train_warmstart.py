"""Train the steady-state surrogate on solver-generated static-tissue samples and measure the
warm start on held-out ones.

  python -m paper_1503_06726_amd.train_warmstart [--samples N] [--epochs E] [--batch B]
                                                 [--eval M] [--out PATH] [--warm-targets PATH]
                                                 [--target-budget SECONDS]

1. N training samples (seed stream of the training set) and M held-out samples are generated
   on the host;
2. every training sample's steady state is solved by the library's batched ADE-only iteration
   (FP64, relative change 1e-8) and scaled to phi * decay / source; with --warm-targets the
   solves start from the prediction of an earlier network (the stopping rule, not the start,
   fixes the target), and --target-budget stops solving after that many seconds and trains on
   the samples solved so far;
3. the network (library kernels) is trained with Adam and a cosine learning-rate decay;
4. the held-out samples are solved to 1e-6 from zero and from the network's prediction, and
   the iteration counts are printed; the parameters and a summary are saved to PATH.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=15)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--target-tol", type=float, default=1e-8)
    ap.add_argument("--out", default=None)
    ap.add_argument("--warm-targets", default=None, help="weights (.npz) whose predictions start the target solves")
    ap.add_argument("--target-budget", type=float, default=None, help="seconds for the target solves")
    args = ap.parse_args(argv)

    import numpy as np
    from . import warmstart as WS

    def log(*a):
        print(*a, flush=True)

    t0 = time.perf_counter()
    train_ws = WS.generate(range(args.samples), held_out=False)
    held_ws = WS.generate(range(args.eval), held_out=True)
    log(f"generated {len(train_ws)} training and {len(held_ws)} held-out samples ({time.perf_counter() - t0:.0f} s)")

    import torch
    from . import lbib
    torch.cuda.set_device(0)

    src, _, feat = WS.prepare(train_ws)
    log(f"masks and features ({time.perf_counter() - t0:.0f} s)")
    net0 = None
    if args.warm_targets:
        p0, _ = WS.load(args.warm_targets)
        net0 = lbib.Net(src.shape[1], src.shape[2], 16)
        net0.set_params(p0)
    targets = np.zeros((len(train_ws),) + src.shape[1:], np.float32)
    its_all = np.zeros(len(train_ws), np.int64)
    chunk = 512
    t_tgt = time.perf_counter()
    n_done = 0
    for k in range(0, len(train_ws), chunk):
        if args.target_budget is not None and time.perf_counter() - t_tgt > args.target_budget:
            log(f"target budget reached after {n_done} samples")
            break
        phi0 = None if net0 is None else WS.predict(net0, feat[k:k + chunk], train_ws[k:k + chunk])
        its, phi = WS.solve(train_ws[k:k + chunk], src[k:k + chunk], phi0=phi0, tol=args.target_tol)
        for j in range(phi.shape[0]):
            targets[k + j] = phi[j] / WS.scale(train_ws[k + j])
        its_all[k:k + chunk] = its
        n_done = k + phi.shape[0]
        log(f"  targets {n_done}/{len(train_ws)} (median {int(np.median(its))} iterations; "
            f"{time.perf_counter() - t0:.0f} s)")
    if net0 is not None:
        net0.close()
    keep = np.flatnonzero(its_all[:n_done] > 0)
    if len(keep) < n_done:
        log(f"warning: {n_done - len(keep)} training targets did not converge and are left out")
    feat, targets, train_ws = feat[keep], targets[keep], [train_ws[i] for i in keep]

    fx = torch.tensor(feat, dtype=torch.float32, device="cuda")
    ty = torch.tensor(targets, dtype=torch.float32, device="cuda")
    del feat
    ny, nx = src.shape[1], src.shape[2]
    net = lbib.Net(ny, nx, args.batch)
    net.set_params(WS.init_params(args.seed, net.n_params))
    hist = WS.train(net, fx, ty, args.epochs, batch=args.batch, lr=args.lr, seed=args.seed, log=log)
    params = net.get_params()
    t_train = time.perf_counter() - t0
    del fx, ty

    hsrc, _, hfeat = WS.prepare(held_ws)
    k0, _ = WS.solve(held_ws, hsrc, tol=1e-6)
    phi_hat = WS.predict(net, hfeat, held_ws)
    kw, _ = WS.solve(held_ws, hsrc, phi0=phi_hat, tol=1e-6)
    net.close()
    summary = {
        "samples": len(train_ws), "warm_targets": bool(args.warm_targets), "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "seed": args.seed,
        "target_tol": args.target_tol, "loss_per_epoch": [float(h) for h in hist],
        "held_out": len(held_ws), "zero_start_median": float(np.median(k0)), "zero_start_mean": float(k0.mean()),
        "warm_start_median": float(np.median(kw)), "warm_start_mean": float(kw.mean()),
        "unconverged_zero": int((k0 == 0).sum()), "unconverged_warm": int((kw == 0).sum()),
        "seconds": round(time.perf_counter() - t0, 1), "seconds_to_trained": round(t_train, 1)}
    log(json.dumps(summary))
    if args.out:
        WS.save(params, summary, args.out)
        log(f"saved {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
