"""Training and evaluation driver of the learned unrolled solver.

Host-side orchestration only: every arithmetic step (operator, FISTA targets,
network forward / backward, Adam) runs in libufss through the binding.

Data: scenes drawn like the 32 x 32 C-scan workload (seeded point scatterers
plus the back wall), measurements y = A x + n at a drawn SNR, and as target
the plain FP32 FISTA iterate after ``ref_iters`` iterations on the same y --
the network learns to reach FISTA's answer in fewer stages.

Evaluation follows the fallback rule: if the network's residual
||A x_net - y|| exceeds 1.1 times the residual of the FISTA reference, plain
FISTA is run warm-started from x_net and its time is counted.
"""
import time

import numpy as np

from . import ufss
from . import workloads as W


def make_dataset(plan, geom, n, seed0, ref_iters, L, mu=0.1, n_scat=(5, 30), snr=(10.0, 20.0),
                 back_wall=None, dev=None, log=None):
    """List of (y, target, x_true) device tensors for n seeded scenes; `log`
    (optional) receives a progress line every 64 scenes."""
    import torch
    dev = dev or torch.device("cuda:0")
    rng = np.random.default_rng(seed0)
    shape_x = (geom["ny"], geom["nx"], geom["nz"])
    shape_y = (geom["ny"], geom["nx"], plan.m)
    out = []
    for i in range(n):
        k = int(rng.integers(n_scat[0], n_scat[1] + 1))
        snr_db = float(rng.uniform(snr[0], snr[1]))
        x = W.scene(geom, k, amp=(0.5, 1.0), seed=seed0 * 100003 + i, back_wall=back_wall)
        xt = torch.from_numpy(x.astype(np.complex64)).to(dev)
        y0 = torch.empty(shape_y, dtype=torch.complex64, device=dev)
        ufss.ufss_forward(plan, xt, y0)
        torch.cuda.synchronize()
        sig = W.noise_sigma(float((y0.abs() ** 2).sum().item()), y0.numel(), snr_db)
        y = (y0 + sig * torch.from_numpy(W.cn(shape_y, seed0 * 7919 + i).astype(np.complex64)).to(dev))
        y = y.contiguous()
        tgt = torch.zeros(shape_x, dtype=torch.complex64, device=dev)
        ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, ref_iters, tgt)
        out.append((y, tgt, xt))
        if log and (i + 1) % 64 == 0:
            log("%d / %d scenes" % (i + 1, n))
    return out


def train(net, data, epochs, batch, lr, seed=0, log=None, log_every=0):
    """Adam over shuffled mini-batches; returns the mean loss per epoch.
    ``log_every`` > 0 also logs the running loss every that many batches."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(data))
        losses = []
        for s in range(0, len(order), batch):
            idx = order[s:s + batch]
            l = ufss.ufss_unrolled_train_step(net, [data[i][0] for i in idx],
                                              [data[i][1] for i in idx], lr)
            losses.append(l)
            if log and log_every > 0 and len(losses) % log_every == 0:
                log("epoch %d batch %d running loss %.5f" % (ep, len(losses), float(np.mean(losses))))
        hist.append(float(np.mean(losses)))
        if log:
            log("epoch %d loss %.5f" % (ep, hist[-1]))
    return hist


def relerr(a, b):
    import torch
    return float((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item())


def evaluate(net, plan, data, L, mu=0.1, fallback_iters=100):
    """Per-sample error of the network against the FISTA reference, with the
    residual fallback rule; returns a dict of arrays and timings."""
    import torch
    errs, res_net, res_ref, used_fb, t_net = [], [], [], [], []
    for y, tgt, _ in data:
        x = torch.zeros_like(tgt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ufss.ufss_unrolled_forward(net, y, x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = torch.empty_like(y)
        ufss.ufss_forward(plan, x, r)
        rn = float(torch.linalg.norm(r - y).item())
        ufss.ufss_forward(plan, tgt, r)
        rr = float(torch.linalg.norm(r - y).item())
        fb = rn > 1.1 * rr
        if fb:
            t0 = time.perf_counter()
            ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, fallback_iters, x)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
        errs.append(relerr(x, tgt))
        res_net.append(rn)
        res_ref.append(rr)
        used_fb.append(fb)
        t_net.append(dt)
    return {"err": np.array(errs), "res_net": np.array(res_net), "res_ref": np.array(res_ref),
            "fallback": np.array(used_fb), "time_s": np.array(t_net)}
