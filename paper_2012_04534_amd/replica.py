"""Replica of the simulated-specimen study of Sec. VII on the HIP operator.

The 50 x 50 x 50 specimen of Table III (line and tilted-rectangle defects of
amplitude exp(j pi/4), noise free) is measured with n_f in {1, 2, 5, 10}
coefficients per A-scan under each sampling strategy of Sec. III-A (random
with Sigma = I or with Rademacher mixing, maximal, energy-based; shared or per
position) and recovered
with FISTA (80 iterations, lambda = mu ||A^H y||_inf, L by power iteration).

Reported per run (one JSON line each):
  depth_hit    fraction of the defect's lateral columns whose reconstructed
               depth profile peaks at the true depth (the depth localisation
               the paper reads off its C-scan images)
  depth_err    mean |peak depth - true depth| over those columns, in samples
  corr         |<x_hat, x>| / (||x_hat|| ||x||), scale-free image agreement
  ms_per_iter  FISTA time per iteration (forward + adjoint + update)
  algo         operator algorithm the plan used (GEMM or phasor)

The asymptotic study of Sec. VI is ``--crb``: the Cramer-Rao bound on the
position of one scatterer 33.3 mm below the centre of the same scan grid, for
n_f in {1, 2, 5, 10, 20} under each strategy, the mixed ones included (50
seeded draws for the random ones), relative to the bound with every bin
0..N_t/2 measured.

Usage: python -m paper_2012_04534_amd.replica [--quick] [--algos] [--crb]
  --algos  also times A + A^H under both per-position algorithms for each n_f
  --crb    the Cramer-Rao study only
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import ufss
from . import workloads as W

STRATEGIES = {
    "rnd": ufss.SAMPLE_RND, "max": ufss.SAMPLE_MAX, "nrg": ufss.SAMPLE_NRG,
    "rnd_f": ufss.SAMPLE_RND_F, "nrg_f": ufss.SAMPLE_NRG_F,
}
# random mixing (Rademacher signs before the DFT; uniform subsets of all N_t
# coefficients): one sign row for all positions, one per position, and per
# position signs and subsets (Table I Phi_rnd, Phi_rnd,m, Phi_rnd,m,f)
MIXED = {"rnd_mix": (False, False), "rnd_m": (True, False), "rnd_mf": (True, True)}
# the Re{H} comparison of Sec. VII: the same measurements recovered as a real
# reflectivity (its "mirrored" variant is the same problem for a real unknown)
REAL = {"max_re": "max", "rnd_f_re": "rnd_f"}
ALGO_NAMES = {ufss.ALGO_GEMM: "gemm", ufss.ALGO_PHASOR: "phasor", ufss.ALGO_FFT: "transform"}


def depth_metrics(xhat, xtrue):
    """Depth localisation over the lateral columns that hold the defect."""
    mag_t = np.abs(xtrue)
    cols = np.argwhere(mag_t.max(axis=2) > 0)
    hits, errs = 0, []
    for iy, ix in cols:
        zt = int(np.argmax(mag_t[iy, ix]))
        zh = int(np.argmax(np.abs(xhat[iy, ix])))
        hits += zh == zt
        errs.append(abs(zh - zt))
    return hits / len(cols), float(np.mean(errs))


def run(g, scene_name, xtrue, strategy, nf, mu, iters, seed, dev, algo=ufss.ALGO_AUTO):
    signs = None
    real = strategy in REAL
    base = REAL.get(strategy, strategy)
    if base in MIXED:
        per_sign, per = MIXED[base]
        lead = (g["ny"], g["nx"])
        bins = W.uniform_subsets(g["nt"], nf, lead if per else (), seed)
        signs = W.rademacher(lead + (g["nt"],) if per_sign else (g["nt"],), seed + 1)
        algo = ufss.ALGO_FFT             # the core runs over all N_t bins: the transform path
    else:
        bins, per = ufss.ufss_sample_bins(g, nf, STRATEGIES[base], seed)
    t0 = time.perf_counter()
    plan = ufss.Plan(g, nf, per, bins, algo=algo, signs=signs)
    info = plan.info()
    xt = torch.from_numpy(xtrue.astype(np.complex64)).to(dev)
    y = torch.empty((g["ny"], g["nx"], nf), dtype=torch.complex64, device=dev)
    ufss.ufss_forward(plan, xt, y)
    L = ufss.ufss_lipschitz(plan, margin=0.01)
    build_s = time.perf_counter() - t0
    x = torch.zeros_like(xt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, iters, x, real=real)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t1) * 1e3 / iters
    xh = x.cpu().numpy().astype(np.complex128)
    hit, derr = depth_metrics(xh, xtrue)
    nrm = np.linalg.norm(xh) * np.linalg.norm(xtrue)
    corr = float(abs(np.vdot(xh, xtrue)) / nrm) if nrm > 0 else 0.0
    plan.close()
    return dict(scene=scene_name, strategy=strategy, n_f=nf, mu=mu, iters=iters,
                depth_hit=round(hit, 4), depth_err=round(derr, 3), corr=round(corr, 4),
                ms_per_iter=round(ms, 4), plan_and_L_s=round(build_s, 3), L=L,
                algo=ALGO_NAMES.get(info["algo"], str(info["algo"])),
                union=info["union_size"], final_res=float(st["res"][-1]))


def time_algos(g, nf, seed, dev, reps=20):
    """A + A^H time under each per-position algorithm (same bins)."""
    bins, _ = ufss.ufss_sample_bins(g, nf, ufss.SAMPLE_NRG_F, seed)
    out = {}
    for algo in (ufss.ALGO_GEMM, ufss.ALGO_PHASOR):
        plan = ufss.Plan(g, nf, True, bins, algo=algo)
        x = torch.randn((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
        y = torch.empty((g["ny"], g["nx"], nf), dtype=torch.complex64, device=dev)
        for _ in range(3):
            ufss.ufss_forward(plan, x, y)
            ufss.ufss_adjoint(plan, y, x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ufss.ufss_forward(plan, x, y)
            ufss.ufss_adjoint(plan, y, x)
        e1.record()
        torch.cuda.synchronize()
        out[ALGO_NAMES[algo]] = round(e0.elapsed_time(e1) / reps, 4)
        out["union"] = plan.info()["union_size"]
        plan.close()
    return out


CRB_NF = (1, 2, 5, 10, 20)
CRB_TRIALS = 50


def crb_study(g, seed):
    """Bounds relative to the full band, per strategy and n_f (one JSON line each)."""
    pt = dict(x=(g["nx"] - 1) / 2 * g["dx"], y=(g["ny"] - 1) / 2 * g["dy"], z=33.3e-3,
              amp=1.0, phase=math.pi / 4, sigma2=1.0)
    full = np.arange(0, g["nt"] // 2 + 1, dtype=np.int32)
    c_full, _ = ufss.ufss_crb(g, len(full), False, full, pt)
    # every coefficient of a mixed A-scan carries the whole spectrum: its full
    # selection gives the bound over every signed bin (the mixing is unitary)
    c_all, _ = ufss.ufss_crb(g, g["nt"], False, np.arange(g["nt"], dtype=np.int32), pt,
                             signs=np.ones(g["nt"], np.int8))
    print(json.dumps(dict(kind="crb_full_signed", crb_m2=[float(v) for v in c_all])), flush=True)
    print(json.dumps(dict(kind="crb_full", crb_m2=[float(v) for v in c_full])), flush=True)
    lead = (g["ny"], g["nx"])
    for nf in CRB_NF:
        for strat in list(STRATEGIES) + list(MIXED):
            trials = 1 if strat == "max" else CRB_TRIALS
            sel, sg = [], None
            per = False
            for t in range(trials):
                sd = seed + 1000 * nf + t
                if strat in MIXED:
                    per_sign, per = MIXED[strat]
                    sel.append(W.uniform_subsets(g["nt"], nf, lead if per else (), sd))
                    sg = (sg or []) + [W.rademacher(lead + (g["nt"],) if per_sign else (g["nt"],), sd + 1)]
                else:
                    b, per = ufss.ufss_sample_bins(g, nf, STRATEGIES[strat], sd)
                    sel.append(b)
            t0 = time.perf_counter()
            c, _ = ufss.ufss_crb(g, nf, per, np.stack(sel), pt,
                                 signs=None if sg is None else np.stack(sg))
            ms = (time.perf_counter() - t0) * 1e3
            ratio = c / c_full[None, :]
            print(json.dumps(dict(kind="crb", strategy=strat, n_f=nf, trials=trials,
                                  mean=[round(float(v), 4) for v in ratio.mean(axis=0)],
                                  best=[round(float(v), 4) for v in ratio.min(axis=0)],
                                  worst=[round(float(v), 4) for v in ratio.max(axis=0)],
                                  call_ms=round(ms, 3))), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--quick", action="store_true", help="n_f in {1, 10}, mu = 0.1 only")
    ap.add_argument("--algos", action="store_true", help="time both per-position algorithms")
    ap.add_argument("--time-only", action="store_true",
                    help="with --algos: the timings only, no reconstructions")
    ap.add_argument("--crb", action="store_true", help="the Cramer-Rao study only")
    ap.add_argument("--seed", type=int, default=5001)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("replica: needs a GPU (the operator runs only in the HIP library)")
    dev = torch.device("cuda:0")
    g = W.sim_geometry()
    if args.crb:
        crb_study(g, args.seed)
        return
    scenes = {"line": W.sim_line(g), "rectangle": W.sim_rectangle(g)}
    nfs = (1, 10) if args.quick else W.SIM_NF
    mus = (0.1,) if args.quick else W.SIM_MU
    if args.algos:
        for nf in W.SIM_NF:
            print(json.dumps(dict(kind="algo_time", n_f=nf, **time_algos(g, nf, args.seed, dev))),
                  flush=True)
        if args.time_only:
            return
    for sname, xtrue in scenes.items():
        for mu in mus:
            for nf in nfs:
                for strat in list(STRATEGIES) + list(MIXED) + list(REAL):
                    r = run(g, sname, xtrue, strat, nf, mu, W.SIM_ITERS, args.seed, dev)
                    print(json.dumps(dict(kind="recon", **r)), flush=True)


if __name__ == "__main__":
    main()
