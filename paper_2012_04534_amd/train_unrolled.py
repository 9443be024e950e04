"""Train the learned unrolled solver on the 32 x 32 C-scan shape.

    python -m paper_2012_04534_amd.train_unrolled --train 96 --eval 24 --epochs 6 \
        --out weights.bin --report report.json

The operator is fixed for the run (per-position bins of the 32 x 32 C-scan
workload); scenes follow that workload's rule with 5-30 scatterers and
10-20 dB SNR; targets are the plain FP32 FISTA iterate after 100 iterations.
Training seeds start at 1005, evaluation seeds at 2005.  Prints one line per
epoch and writes the checkpoint and a JSON report.
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
    plan = ufss.Plan(g, w["m"], True, bins, algo=ufss.ALGO_GEMM)
    L = ufss.ufss_lipschitz(plan, max_iters=200, rtol=1e-6, margin=0.01)
    print("L %.6e" % L, flush=True)
    train = LN.make_dataset(plan, g, args.train, 1005, args.ref_iters, L, back_wall=w["back_wall"])
    print("train set ready %.1f s" % (time.time() - t_all), flush=True)
    ev = LN.make_dataset(plan, g, args.eval, 2005, args.ref_iters, L, back_wall=w["back_wall"])
    print("eval set ready %.1f s" % (time.time() - t_all), flush=True)
    net_plan = plan
    if args.bf16:
        net_plan = ufss.Plan(g, w["m"], True, bins, dtype=ufss.BF16, algo=ufss.ALGO_GEMM)
    net = ufss.Net(net_plan, stages=args.stages, channels=args.channels, L=L, mu=w["mu"], seed=3)
    r0 = LN.evaluate(net, plan, ev, L)
    t0 = time.time()
    hist = LN.train(net, train, args.epochs, args.batch, args.lr,
                    log=lambda s: print(s + " (%.1f s)" % (time.time() - t0), flush=True))
    t_train = time.time() - t0
    r1 = LN.evaluate(net, plan, ev, L)
    ufss.ufss_unrolled_save(net, args.out)
    rep = {
        "stages": args.stages, "channels": args.channels, "train_scenes": args.train,
        "eval_scenes": args.eval, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
        "operator": "bf16" if args.bf16 else "f32", "ref_iters": args.ref_iters, "L": L,
        "loss_per_epoch": hist, "train_s": t_train,
        "untrained_err_mean": float(r0["err"].mean()),
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
