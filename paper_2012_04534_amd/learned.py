"""Training, inference and evaluation driver of the learned unrolled solver.

Host-side orchestration only: every arithmetic step (operator, FISTA targets,
network forward / backward, Adam, the residual norms of the fallback rule)
runs in libufss through the binding or in torch device reductions.

Data: scenes drawn like the 32 x 32 C-scan workload (seeded point scatterers
plus the back wall), measurements y = A x + n at a drawn SNR, both generated
on the device, and as target the plain FP32 FISTA iterate after ``ref_iters``
(200) iterations on the same y -- the network learns to reach FISTA's answer
in fewer stages.  Scene i of a set keyed by ``seed0`` draws its scatterer
count and SNR from the generator keyed (seed0, i), its scene from the device
stream seed0 * 100003 + i and its noise from seed0 * 7919 + i, so any slice of
a set can be rebuilt on its own.

Inference follows the fallback rule: if the network's residual ||A x_net - y||
exceeds ``factor`` (1.1) times the residual of the FISTA answer, plain FISTA is
run warm-started from x_net and its time is counted.
"""
import time

import numpy as np

from . import ufss

TRAIN_SEED = 1005
EVAL_SEED = 2005


def scene_draw(seed0, i, n_scat=(5, 30), snr=(10.0, 20.0)):
    """(scatterer count, SNR in dB) of scene i of the set keyed seed0."""
    rng = np.random.default_rng((seed0, i))
    return int(rng.integers(n_scat[0], n_scat[1] + 1)), float(rng.uniform(snr[0], snr[1]))


def measurements(plan, geom, seed0, i, back_wall=None, dev=None, n_scat=(5, 30), snr=(10.0, 20.0)):
    """(y, x_true) device tensors of scene i of the set keyed seed0, generated
    on the device (ufss_synth_scene, ufss_synth_measure: no host round trip);
    scatterers lie above the back wall's depth minus 8."""
    import torch
    dev = dev or torch.device("cuda:0")
    k, snr_db = scene_draw(seed0, i, n_scat, snr)
    shape_x = (geom["ny"], geom["nx"], geom["nz"])
    shape_y = (geom["ny"], geom["nx"], plan.m)
    max_depth = geom["nz"] if back_wall is None else back_wall - 8
    xt = torch.empty(shape_x, dtype=torch.complex64, device=dev)
    ufss.ufss_synth_scene(geom, k, (0.5, 1.0), max_depth, back_wall, seed0 * 100003 + i, xt)
    y = torch.empty(shape_y, dtype=torch.complex64, device=dev)
    ufss.ufss_synth_measure(plan, xt, snr_db, seed0 * 7919 + i, y)
    return y, xt


def make_dataset(plan, geom, n, seed0, ref_iters, L, mu=0.1, offset=0, back_wall=None, dev=None,
                 log=None, keep_truth=False):
    """List of (y, target, x_true or None) device tensors for scenes
    offset .. offset + n - 1 of the set keyed seed0; `log` (optional) receives
    a progress line every 256 scenes."""
    import torch
    dev = dev or torch.device("cuda:0")
    shape_x = (geom["ny"], geom["nx"], geom["nz"])
    out = []
    for j in range(n):
        i = offset + j
        y, xt = measurements(plan, geom, seed0, i, back_wall=back_wall, dev=dev)
        tgt = torch.zeros(shape_x, dtype=torch.complex64, device=dev)
        ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, ref_iters, tgt)
        out.append((y, tgt, xt if keep_truth else None))
        if log and (j + 1) % 256 == 0:
            log("%d / %d scenes" % (j + 1, n))
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


def residual(plan, x, y):
    """||A x - y|| (device operator, norm by a torch reduction)."""
    import torch
    r = torch.empty_like(y)
    ufss.ufss_forward(plan, x, r)
    return float(torch.linalg.norm(r - y).item())


def solve(net, plan, y, L, mu, ref_res, factor=1.1, fallback_iters=200, x=None):
    """Inference with the fallback rule.  Runs the network; if
    ||A x_net - y|| > factor * ref_res (the residual of the FISTA answer), runs
    ``fallback_iters`` plain FISTA iterations warm-started from x_net.  Returns
    (x, info) with the wall times of both parts (GPU synchronised)."""
    import torch
    shape_x = (plan.g["ny"], plan.g["nx"], plan.g["nz"])
    if x is None:
        x = torch.zeros(shape_x, dtype=torch.complex64, device=y.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ufss.ufss_unrolled_forward(net, y, x)
    rn = residual(plan, x, y)
    t_net = time.perf_counter() - t0
    fb = rn > factor * ref_res
    t_fb = 0.0
    if fb:
        t0 = time.perf_counter()
        ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, fallback_iters, x)
        torch.cuda.synchronize()
        t_fb = time.perf_counter() - t0
    return x, {"res_net": rn, "fallback": bool(fb), "t_net": t_net, "t_fallback": t_fb}


def evaluate(net, plan, data, L, mu=0.1, factor=1.1, fallback_iters=200, fista_s_per_iter=None):
    """Per-sample error of the network (with the fallback rule) against the
    FISTA reference; with ``fista_s_per_iter``, also the error of plain FISTA
    from zero given the same wall time (at least one iteration).  Returns a
    dict of arrays."""
    import torch
    keys = ("err", "err_net", "res_net", "res_ref", "fallback", "time_s", "t_fallback",
            "err_fista_same_time", "iters_same_time")
    out = {k: [] for k in keys}
    for y, tgt, _ in data:
        rr = residual(plan, tgt, y)
        x, info = solve(net, plan, y, L, mu, rr, factor, fallback_iters)
        out["err"].append(relerr(x, tgt))
        out["res_net"].append(info["res_net"])
        out["res_ref"].append(rr)
        out["fallback"].append(info["fallback"])
        out["time_s"].append(info["t_net"] + info["t_fallback"])
        out["t_fallback"].append(info["t_fallback"])
        if info["fallback"]:
            # the network's own output, for the record
            xn = torch.zeros_like(tgt)
            ufss.ufss_unrolled_forward(net, y, xn)
            out["err_net"].append(relerr(xn, tgt))
        else:
            out["err_net"].append(out["err"][-1])
        if fista_s_per_iter:
            k = max(1, int(info["t_net"] / fista_s_per_iter))
            xf = torch.zeros_like(tgt)
            ufss.ufss_fista(plan, y, ufss.lambda_from_mu(mu), L, k, xf)
            out["err_fista_same_time"].append(relerr(xf, tgt))
            out["iters_same_time"].append(k)
    return {k: np.array(v) for k, v in out.items()}
