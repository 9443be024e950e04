"""Train and evaluate the learned unrolled solver on the 32 x 32 C-scan shape.

    python -m paper_2012_04534_amd.train_unrolled --transform --train 10000 --train-offset 0 \
        --eval 48 --epochs 4 --out weights.bin --report report.json [--init weights.bin] \
        [--lr 1e-4] [--lr-decay 0.9] [--max-minutes 15]
    python -m paper_2012_04534_amd.train_unrolled --transform --eval-only --eval 1000 \
        --init weights.bin --report eval.json

The operator is fixed for the run (per-position bins of the 32 x 32 C-scan
workload); scenes follow that workload's rule with 5-30 scatterers and
10-20 dB SNR; targets are the plain FP32 FISTA iterate after 200 iterations.
Training scenes are indices --train-offset ... of the set keyed 1005 (so a
run over a slice of the 20,000 training scenes can follow another), evaluation
scenes indices --eval-offset ... of the set keyed 2005 (held out).  Prints one
line per epoch, writes the checkpoint after every epoch and a JSON report at
the end.  --init continues from a checkpoint (parameters and Adam state);
--max-minutes stops after the epoch that crosses the wall-clock budget.
--eval-only evaluates a checkpoint on the held-out scenes in chunks: the
network with the fallback rule, the untrained network (= 16 FISTA iterations)
and plain FISTA given the network's wall time, all against FISTA-200.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def fista_s_per_iter(ufss, plan, y, L, mu, iters=200):
    import torch
    x = torch.zeros((plan.g["ny"], plan.g["nx"], plan.g["nz"]), dtype=torch.complex64, device=y.device)
    ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, 5, x)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, iters, x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / iters


def eval_report(ufss, LN, net, untrained, plan, g, w, L, n, offset, ref_iters, chunk=100, log=None):
    """Held-out evaluation in chunks (the targets of a chunk live on the GPU)."""
    import numpy as np
    acc = {}
    spi = None
    for c0 in range(0, n, chunk):
        data = LN.make_dataset(plan, g, min(chunk, n - c0), LN.EVAL_SEED, ref_iters, L, mu=w["mu"],
                               offset=offset + c0, back_wall=w["back_wall"])
        if spi is None:
            spi = fista_s_per_iter(ufss, plan, data[0][0], L, w["mu"])
        r = LN.evaluate(net, plan, data, L, w["mu"], fista_s_per_iter=spi)
        ru = LN.evaluate(untrained, plan, data, L, w["mu"], factor=float("inf"))
        r["err_untrained"] = ru["err_net"]
        for k, v in r.items():
            acc.setdefault(k, []).append(v)
        del data
        if log:
            log("eval %d / %d scenes, running mean error %.4f" % (
                c0 + chunk, n, float(np.concatenate(acc["err"]).mean())))
    a = {k: np.concatenate(v) for k, v in acc.items()}
    q = lambda v: [float(np.percentile(v, p)) for p in (50, 90, 99)]
    return {
        "eval_scenes": int(a["err"].size), "eval_offset": offset, "reference": "FISTA-%d" % ref_iters,
        "err_mean": float(a["err"].mean()), "err_max": float(a["err"].max()), "err_p50_p90_p99": q(a["err"]),
        "err_net_mean": float(a["err_net"].mean()),
        "scenes_within_1e-2": int((a["err"] <= 1e-2).sum()),
        "fallbacks": int(a["fallback"].sum()),
        "fallback_time_s_total": float(a["t_fallback"].sum()),
        "time_s_mean": float(a["time_s"].mean()), "time_s_max": float(a["time_s"].max()),
        "fista_s_per_iter": spi,
        "untrained_err_mean": float(a["err_untrained"].mean()),
        "fista_same_time_iters_mean": float(a["iters_same_time"].mean()),
        "fista_same_time_err_mean": float(a["err_fista_same_time"].mean()),
        "fista_iters_to_target_time_s": ref_iters * spi,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=96)
    ap.add_argument("--train-offset", type=int, default=0)
    ap.add_argument("--eval", type=int, default=24)
    ap.add_argument("--eval-offset", type=int, default=0)
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--stages", type=int, default=16)
    ap.add_argument("--channels", type=int, default=8)
    ap.add_argument("--ref-iters", type=int, default=200)
    ap.add_argument("--bf16", action="store_true", help="BF16 operator inside the network")
    ap.add_argument("--transform", action="store_true",
                    help="the transform-domain operator (FP32) for the data and the network")
    ap.add_argument("--init", default=None, help="checkpoint to continue from")
    ap.add_argument("--autotune", action="store_true", help="tune the operator's tiling first")
    ap.add_argument("--lr-decay", type=float, default=1.0, help="learning-rate factor per epoch")
    ap.add_argument("--max-minutes", type=float, default=0.0, help="training wall-clock budget (0: none)")
    ap.add_argument("--out", default="unrolled.bin")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()

    import numpy as np
    import torch  # noqa: F401  (before the library: one HIP runtime per process)
    from paper_2012_04534_amd import learned as LN
    from paper_2012_04534_amd import ufss
    from paper_2012_04534_amd import workloads as W

    log = lambda m: print(m, flush=True)
    t_all = time.time()
    w = W.workload("cscan32")
    g = w["geom"]
    bins, _ = ufss.ufss_select_freqs(g, w["m"], True, w["seed"])
    plan = ufss.Plan(g, w["m"], True, bins,
                     algo=ufss.ALGO_FFT if args.transform else ufss.ALGO_GEMM)
    if args.autotune and not args.transform:
        ufss.ufss_autotune(plan, None, False, False)
    L = ufss.ufss_lipschitz(plan, max_iters=200, rtol=1e-6, margin=0.01)
    log("L %.6e" % L)
    net_plan = plan
    if args.bf16:
        net_plan = ufss.Plan(g, w["m"], True, bins, dtype=ufss.BF16, algo=ufss.ALGO_GEMM)
        if args.autotune:
            ufss.ufss_autotune(net_plan, None, False, False)
    net = ufss.Net(net_plan, stages=args.stages, channels=args.channels, L=L, mu=w["mu"], seed=3)
    if args.init:
        ufss.ufss_unrolled_load(net, args.init)
    rep = {"stages": args.stages, "channels": args.channels, "ref_iters": args.ref_iters, "L": L,
           "operator": "bf16" if args.bf16 else ("f32 transform" if args.transform else "f32"),
           "init": os.path.basename(args.init) if args.init else None}

    if args.eval_only:
        untrained = ufss.Net(net_plan, stages=args.stages, channels=args.channels, L=L, mu=w["mu"],
                             seed=3)
        rep.update(eval_report(ufss, LN, net, untrained, plan, g, w, L, args.eval, args.eval_offset,
                               args.ref_iters, log=log))
        rep["eval_s"] = time.time() - t_all
    else:
        train = LN.make_dataset(plan, g, args.train, LN.TRAIN_SEED, args.ref_iters, L, mu=w["mu"],
                                offset=args.train_offset, back_wall=w["back_wall"],
                                log=lambda m: log("train set " + m))
        log("train set ready %.1f s" % (time.time() - t_all))
        ev = LN.make_dataset(plan, g, args.eval, LN.EVAL_SEED, args.ref_iters, L, mu=w["mu"],
                             offset=args.eval_offset, back_wall=w["back_wall"])
        log("validation set ready %.1f s" % (time.time() - t_all))
        r0 = LN.evaluate(net, plan, ev, L, w["mu"])
        log("start validation err %.4f" % r0["err"].mean())
        t0 = time.time()
        hist, val = [], []
        lr = args.lr
        for ep in range(args.epochs):
            h = LN.train(net, train, 1, args.batch, lr, seed=args.train_offset + ep, log=log,
                         log_every=256)
            hist += h
            ufss.ufss_unrolled_save(net, args.out)
            rv = LN.evaluate(net, plan, ev, L, w["mu"])
            val.append(float(rv["err"].mean()))
            log("epoch %d loss %.6f lr %.2e validation err %.4f (%.1f s)" % (
                ep, h[0], lr, val[-1], time.time() - t0))
            lr *= args.lr_decay
            if args.max_minutes > 0 and time.time() - t0 > 60 * args.max_minutes:
                break
        t_train = time.time() - t0
        r1 = LN.evaluate(net, plan, ev, L, w["mu"])
        ufss.ufss_unrolled_save(net, args.out)
        rep.update({
            "train_scenes": args.train, "train_offset": args.train_offset,
            "validation_scenes": args.eval, "epochs_run": len(hist), "batch": args.batch,
            "lr": args.lr, "lr_decay": args.lr_decay, "loss_per_epoch": hist,
            "validation_err_per_epoch": val, "train_s": t_train,
            "start_err_mean": float(r0["err"].mean()),
            "trained_err_mean": float(r1["err"].mean()), "trained_err_max": float(r1["err"].max()),
            "fallbacks": int(r1["fallback"].sum()),
            "net_time_s_mean": float(r1["time_s"].mean()),
        })
    log(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
