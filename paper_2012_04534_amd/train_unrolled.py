"""Train the learned unrolled solver on the 32 x 32 C-scan shape.

    python -m paper_2012_04534_amd.train_unrolled --train 96 --eval 24 --epochs 6 \
        --out weights.bin --report report.json [--init weights.bin] [--autotune] \
        [--lr-decay 0.9] [--max-minutes 15]

The operator is fixed for the run (per-position bins of the 32 x 32 C-scan
workload); scenes follow that workload's rule with 5-30 scatterers and
10-20 dB SNR; targets are the plain FP32 FISTA iterate after 100 iterations.
Training seeds start at 1005, evaluation seeds at 2005.  Prints one line per
epoch, writes the checkpoint after every epoch and a JSON report at the end.
--init continues from a checkpoint (parameters and Adam state); --max-minutes
stops after the epoch that crosses the wall-clock budget.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=96)
    ap.add_argument("--eval", type=int, default=24)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--stages", type=int, default=16)
    ap.add_argument("--channels", type=int, default=8)
    ap.add_argument("--ref-iters", type=int, default=100)
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
    import torch
    from paper_2012_04534_amd import learned as LN
    from paper_2012_04534_amd import ufss
    from paper_2012_04534_amd import workloads as W

    t_all = time.time()
    w = W.workload("cscan32")
    g = w["geom"]
    bins, _ = ufss.ufss_select_freqs(g, w["m"], True, w["seed"])
    plan = ufss.Plan(g, w["m"], True, bins,
                     algo=ufss.ALGO_FFT if args.transform else ufss.ALGO_GEMM)
    if args.autotune and not args.transform:
        ufss.ufss_autotune(plan, None, False, False)
    L = ufss.ufss_lipschitz(plan, max_iters=200, rtol=1e-6, margin=0.01)
    print("L %.6e" % L, flush=True)
    train = LN.make_dataset(plan, g, args.train, 1005, args.ref_iters, L, back_wall=w["back_wall"],
                            log=lambda m: print("train set " + m, flush=True))
    print("train set ready %.1f s" % (time.time() - t_all), flush=True)
    ev = LN.make_dataset(plan, g, args.eval, 2005, args.ref_iters, L, back_wall=w["back_wall"])
    print("eval set ready %.1f s" % (time.time() - t_all), flush=True)
    net_plan = plan
    if args.bf16:
        net_plan = ufss.Plan(g, w["m"], True, bins, dtype=ufss.BF16, algo=ufss.ALGO_GEMM)
        if args.autotune:
            ufss.ufss_autotune(net_plan, None, False, False)
    net = ufss.Net(net_plan, stages=args.stages, channels=args.channels, L=L, mu=w["mu"], seed=3)
    if args.init:
        ufss.ufss_unrolled_load(net, args.init)
    r0 = LN.evaluate(net, plan, ev, L)
    print("start eval err %.4f" % r0["err"].mean(), flush=True)
    t0 = time.time()
    hist = []
    lr = args.lr
    for ep in range(args.epochs):
        h = LN.train(net, train, 1, args.batch, lr, seed=ep,
                     log=lambda m: print(m, flush=True), log_every=64)
        hist += h
        ufss.ufss_unrolled_save(net, args.out)
        print("epoch %d loss %.5f lr %.2e (%.1f s)" % (ep, h[0], lr, time.time() - t0), flush=True)
        lr *= args.lr_decay
        if args.max_minutes > 0 and time.time() - t0 > 60 * args.max_minutes:
            break
    t_train = time.time() - t0
    r1 = LN.evaluate(net, plan, ev, L)
    ufss.ufss_unrolled_save(net, args.out)
    rep = {
        "stages": args.stages, "channels": args.channels, "train_scenes": args.train,
        "eval_scenes": args.eval, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
        "operator": "bf16" if args.bf16 else ("f32 transform" if args.transform else "f32"),
        "ref_iters": args.ref_iters, "L": L,
        "init": os.path.basename(args.init) if args.init else None, "lr_decay": args.lr_decay,
        "epochs_run": len(hist), "start_err_mean": float(r0["err"].mean()),
        "loss_per_epoch": hist, "train_s": t_train,
        "untrained_err_mean": None if args.init else float(r0["err"].mean()),
        "trained_err_mean": float(r1["err"].mean()), "trained_err_max": float(r1["err"].max()),
        "fallbacks": int(r1["fallback"].sum()),
        "net_time_s_mean": float(r1["time_s"].mean()),
    }
    print(json.dumps(rep), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    np.random.default_rng(0)


if __name__ == "__main__":
    main()
