"""GPU tests of the learned unrolled solver against the FP64 oracle: the
untrained network equals FISTA, the forward pass matches the oracle network,
gradients match central finite differences of the oracle loss, and training
with checkpoint / resume behaves."""
import numpy as np
import pytest

from oracle import learned as N
from oracle import operator as O
from oracle import solver as V
from paper_2012_04534_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def ufss():
    from paper_2012_04534_amd import ufss as u
    return u


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def tiny(u, dev, seed=2):
    g = W.geometry(6, 5, 12, 64, win_x=2, win_y=2)
    bins, _ = u.ufss_select_freqs(g, 5, True, 3)
    Amat = O.dense_A(g, bins)
    x_true = W.scene(g, 4, amp=(0.5, 1.0), seed=seed)
    y = (Amat @ x_true.reshape(-1) + 0.05 * W.cn(Amat.shape[0], seed + 1)).astype(np.complex64)
    yd = y.astype(np.complex128)
    L = V.lipschitz_dense(Amat) * 1.01
    plan = u.Plan(g, 5, True, bins, algo=u.ALGO_GEMM)
    yt = torch.from_numpy(y.reshape(5, 6, 5)).to(dev)
    A = lambda v: Amat @ v
    AH = lambda v: Amat.conj().T @ v
    return g, plan, A, AH, yd, yt, L


def random_params(stages, ch, seed):
    rng = np.random.default_rng(seed)
    p = 0.05 * rng.standard_normal(stages * N.stage_size(ch))
    return p.astype(np.float32)


def test_untrained_network_is_fista(dev):
    u = ufss()
    g, plan, A, AH, yd, yt, L = tiny(u, dev)
    net = u.Net(plan, stages=6, channels=3, L=L, mu=0.1, seed=5)
    x = torch.zeros((5, 6, 12), dtype=torch.complex64, device=dev)
    u.ufss_unrolled_forward(net, yt, x)
    xf = torch.zeros_like(x)
    u.ufss_fista(plan, yt, u.lambda_from_mu(0.1), L, 6, xf)
    e = (torch.linalg.norm(x - xf) / torch.linalg.norm(xf)).item()
    assert e < 1e-5, e
    p = u.ufss_unrolled_params(net)
    xo = N.forward(A, AH, yd, p.astype(np.float64), 6, 3, L, 0.1, (5, 6, 12))
    lam = V.lambda_rule(AH, yd, 0.1)
    a, _ = V.fista(A, AH, yd, lam, L, 6)
    assert np.abs(xo.reshape(-1) - a).max() < 1e-12 * np.abs(a).max()
    e2 = np.linalg.norm(x.cpu().numpy().reshape(-1) - a) / np.linalg.norm(a)
    assert e2 < 1e-5, e2
    net.close()
    plan.close()


def test_forward_matches_oracle_network(dev):
    u = ufss()
    g, plan, A, AH, yd, yt, L = tiny(u, dev)
    S, ch = 4, 3
    net = u.Net(plan, stages=S, channels=ch, L=L, mu=0.1)
    p = random_params(S, ch, 11)
    u.ufss_unrolled_params(net, set_to=p)
    x = torch.zeros((5, 6, 12), dtype=torch.complex64, device=dev)
    u.ufss_unrolled_forward(net, yt, x)
    xo = N.forward(A, AH, yd, p.astype(np.float64), S, ch, L, 0.1, (5, 6, 12))
    e = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
    assert e < 1e-5, e
    net.close()
    plan.close()


def test_gradients_match_oracle_finite_differences(dev):
    """P13: FP32 GPU gradients vs FP64 central differences (h = 1e-6) of the
    oracle loss, for the step / threshold parameters of every stage and a
    sample of convolution weights and biases."""
    u = ufss()
    g, plan, A, AH, yd, yt, L = tiny(u, dev, seed=6)
    S, ch = 3, 2
    shape = (5, 6, 12)
    net = u.Net(plan, stages=S, channels=ch, L=L, mu=0.1)
    p = random_params(S, ch, 12)
    u.ufss_unrolled_params(net, set_to=p)
    a_ref = (0.5 * W.cn(shape, 13)).astype(np.complex64)
    loss, grad = u.ufss_unrolled_grad(net, yt, torch.from_numpy(a_ref).to(dev))
    pd = p.astype(np.float64)
    ref_loss = N.loss(A, AH, yd, pd, S, ch, L, 0.1, shape, a_ref.astype(np.complex128))
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    n = N.stage_size(ch)
    rng = np.random.default_rng(0)
    idx = []
    for i in range(S):
        base = i * n
        idx += [base, base + 1]                                      # rho, kappa
        idx += list(base + 2 + rng.choice(ch * 54, 4, replace=False))  # W1
        idx += [base + 2 + ch * 54 + int(rng.integers(ch))]             # b1
        idx += list(base + 2 + ch * 54 + ch + rng.choice(2 * ch * 27, 4, replace=False))  # W2
        idx += [base + n - 2, base + n - 1]                               # b2
    fd = N.fd_grad(A, AH, yd, pd, S, ch, L, 0.1, shape, a_ref.astype(np.complex128), idx)
    got = grad[idx].astype(np.float64)
    err = np.linalg.norm(got - fd) / np.linalg.norm(fd)
    assert err < 1e-3, (err, np.c_[got, fd])
    net.close()
    plan.close()


def test_training_reduces_loss_and_checkpoint_roundtrip(dev, tmp_path):
    u = ufss()
    g, plan, A, AH, yd, yt, L = tiny(u, dev)
    S, ch = 4, 2
    lam = V.lambda_rule(AH, yd, 0.1)
    ys, refs = [], []
    for s in range(3):
        xs = W.scene(g, 4, amp=(0.5, 1.0), seed=40 + s)
        yv = (A(xs.reshape(-1))).astype(np.complex64)
        lam_s = V.lambda_rule(AH, yv.astype(np.complex128), 0.1)
        aref, _ = V.fista(A, AH, yv.astype(np.complex128), lam_s, L, 60)
        ys.append(torch.from_numpy(yv.reshape(5, 6, 5)).to(dev))
        refs.append(torch.from_numpy(aref.reshape(5, 6, 12).astype(np.complex64)).to(dev))
    assert lam > 0
    net = u.Net(plan, stages=S, channels=ch, L=L, mu=0.1, seed=1)
    losses = [u.ufss_unrolled_train_step(net, ys, refs, 3e-3) for _ in range(25)]
    assert losses[-1] < 0.8 * losses[0], losses
    path = tmp_path / "net.bin"
    u.ufss_unrolled_save(net, path)
    net2 = u.Net(plan, stages=S, channels=ch, L=L, mu=0.1, seed=99)
    u.ufss_unrolled_load(net2, path)
    assert np.array_equal(u.ufss_unrolled_params(net), u.ufss_unrolled_params(net2))
    l1 = u.ufss_unrolled_train_step(net, ys, refs, 3e-3)
    l2 = u.ufss_unrolled_train_step(net2, ys, refs, 3e-3)
    assert l1 == l2
    assert np.array_equal(u.ufss_unrolled_params(net), u.ufss_unrolled_params(net2))
    net.close()
    net2.close()
    plan.close()


def test_network_on_transform_operator_matches_oracle(dev):
    """The unrolled network with the transform-domain operator as its fixed
    layers: forward against the oracle network, and gradients equal to those
    on the GEMM plan (same parameters)."""
    u = ufss()
    g, plan, A, AH, yd, yt, L = tiny(u, dev)
    bins, _ = u.ufss_select_freqs(g, 5, True, 3)        # the bins of tiny()
    pf = u.Plan(g, 5, True, bins, algo=u.ALGO_FFT)
    S, ch = 4, 3
    p = random_params(S, ch, 21)
    out = []
    for pl in (pf, plan):
        net = u.Net(pl, stages=S, channels=ch, L=L, mu=0.1)
        u.ufss_unrolled_params(net, set_to=p)
        x = torch.zeros((5, 6, 12), dtype=torch.complex64, device=dev)
        u.ufss_unrolled_forward(net, yt, x)
        a_ref = torch.from_numpy((0.5 * W.cn((5, 6, 12), 23)).astype(np.complex64)).to(dev)
        loss, grad = u.ufss_unrolled_grad(net, yt, a_ref)
        out.append((x.cpu().numpy(), loss, np.asarray(grad)))
        net.close()
    xo = N.forward(A, AH, yd, p.astype(np.float64), S, ch, L, 0.1, (5, 6, 12))
    assert np.linalg.norm(out[0][0] - xo) / np.linalg.norm(xo) < 1e-5
    assert out[0][1] == pytest.approx(out[1][1], rel=1e-5)
    ga, gb = out[0][2], out[1][2]
    assert np.abs(ga - gb).max() <= 1e-4 * np.abs(gb).max()
    pf.close()
    plan.close()


def test_fallback_forced_runs_warm_started_fista_vs_oracle(dev):
    """The inference fallback rule (learned.solve): with factor 0 every
    network answer falls back, and the result is plain FISTA warm-started from
    the network's output -- against the oracle network followed by the oracle
    FISTA from that start.  With factor = inf nothing falls back and the result
    is the network's output."""
    from paper_2012_04534_amd import learned as LN
    u = ufss()
    g, plan, A, AH, yd, yt, L = tiny(u, dev, seed=8)
    S, ch, K = 4, 3, 30
    shape = (5, 6, 12)
    net = u.Net(plan, stages=S, channels=ch, L=L, mu=0.1)
    p = random_params(S, ch, 31)
    u.ufss_unrolled_params(net, set_to=p)
    xo_net = N.forward(A, AH, yd, p.astype(np.float64), S, ch, L, 0.1, shape)
    lam = V.lambda_rule(AH, yd, 0.1)
    a_fb, _ = V.fista(A, AH, yd, lam, L, K, a0=xo_net.reshape(-1))
    x, info = LN.solve(net, plan, yt, L, 0.1, ref_res=1.0, factor=0.0, fallback_iters=K)
    assert info["fallback"] and info["t_fallback"] > 0
    xg = x.cpu().numpy().reshape(-1)
    e = np.linalg.norm(xg - a_fb) / np.linalg.norm(a_fb)
    assert e < 1e-5, e
    # the warm start matters: FISTA from zero ends elsewhere
    a0, _ = V.fista(A, AH, yd, lam, L, K)
    assert np.linalg.norm(a0 - a_fb) / np.linalg.norm(a_fb) > 1e-3
    x2, info2 = LN.solve(net, plan, yt, L, 0.1, ref_res=1.0, factor=float("inf"), fallback_iters=K)
    assert not info2["fallback"] and info2["t_fallback"] == 0.0
    e2 = np.linalg.norm(x2.cpu().numpy() - xo_net) / np.linalg.norm(xo_net)
    assert e2 < 1e-5, e2
    # the residual the rule compares is ||A x_net - y|| of the oracle's x_net
    r_or = np.linalg.norm(A(xo_net.reshape(-1)) - yd)
    assert info2["res_net"] == pytest.approx(r_or, rel=1e-5)
    net.close()
    plan.close()


def test_shipped_checkpoint_beats_untrained_and_equal_time_fista(dev):
    """The shipped checkpoint on held-out scenes of the 32 x 32 C-scan rule
    (evaluation set, never trained on), against the FISTA-200 answer: its
    error is far below the untrained network's (16 plain FISTA iterations) and
    below plain FISTA given the network's wall time, with the fallback rule."""
    import os
    from paper_2012_04534_amd import learned as LN
    u = ufss()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = os.path.join(root, "paper_2012_04534_amd", "weights", "unrolled_cscan32_s16c8.bin")
    w = W.workload("cscan32")
    g = w["geom"]
    bins, _ = u.ufss_select_freqs(g, w["m"], True, w["seed"])
    plan = u.Plan(g, w["m"], True, bins, algo=u.ALGO_FFT)
    L = u.ufss_lipschitz(plan, max_iters=200, rtol=1e-6, margin=0.01)
    data = LN.make_dataset(plan, g, 6, LN.EVAL_SEED, 200, L, mu=w["mu"], offset=0,
                           back_wall=w["back_wall"])
    net = u.Net(plan, stages=16, channels=8, L=L, mu=w["mu"])
    u.ufss_unrolled_load(net, path)
    untrained = u.Net(plan, stages=16, channels=8, L=L, mu=w["mu"])
    # plain FISTA's time per iteration on this plan
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    u.ufss_fista(plan, data[0][0], u.lambda_from_mu(w["mu"]), L, 5, x)
    x.zero_()
    torch.cuda.synchronize()
    import time
    t0 = time.perf_counter()
    u.ufss_fista(plan, data[0][0], u.lambda_from_mu(w["mu"]), L, 100, x)
    torch.cuda.synchronize()
    spi = (time.perf_counter() - t0) / 100
    r = LN.evaluate(net, plan, data, L, w["mu"], fista_s_per_iter=spi)
    ru = LN.evaluate(untrained, plan, data, L, w["mu"], factor=float("inf"))
    assert r["iters_same_time"].min() >= 16
    err, err_u, err_f = r["err"].mean(), ru["err_net"].mean(), r["err_fista_same_time"].mean()
    assert err < 0.25 * err_u, (err, err_u)
    assert err < 0.25 * err_f, (err, err_f)
    assert err_u > 0.5
    assert err < 0.1, err
    net.close()
    untrained.close()
    plan.close()
