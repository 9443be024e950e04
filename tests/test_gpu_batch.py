"""GPU tests of batched FISTA (one grouped launch per phase, graph-captured),
of the persistent batch (captured once, replayed), of the 64-scan uneven batch
at its own shapes, and of the split-K autotuner."""
import json
import os

import numpy as np
import pytest

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


def make_scan(u, spec, dtype, dev, band_cap=True):
    g = spec["geom"]
    _, band = u.ufss_select_freqs(g, 1, False, 0)
    m = min(spec["m"], band)
    bins, _ = u.ufss_select_freqs(g, m, spec["per_position"], spec["seed"])
    plan = u.Plan(g, m, spec["per_position"], bins, dtype=dtype, algo=u.ALGO_GEMM)
    x_true = W.scene(g, spec["n_scat"], amp=spec["amp"], seed=spec["seed"])
    xt = torch.from_numpy(x_true.astype(np.complex64)).to(dev)
    y = torch.empty((g["ny"], g["nx"], m), dtype=torch.complex64, device=dev)
    u.ufss_forward(plan, xt, y)
    torch.cuda.synchronize()
    sig = W.noise_sigma(float((y.abs() ** 2).sum().item()), y.numel(), spec["snr_db"])
    y = (y + sig * torch.from_numpy(W.cn(y.shape, spec["seed"] + 1).astype(np.complex64)).to(dev)).contiguous()
    return plan, bins, m, y


def small_batch():
    specs = W.batch_workload(seed=77, n=6, max_lateral=20, max_depth=128)
    # force a mix of dtypes: every third scan BF16
    return specs, [1 if i % 3 == 2 else 0 for i in range(len(specs))]


def test_batched_matches_single_scan_fista(dev):
    u = ufss()
    specs, dts = small_batch()
    assert {s["geom"]["ny"] == 1 for s in specs} == {True, False}       # B- and C-scans
    assert {s["per_position"] for s in specs} == {True, False}           # both bin modes
    scans = [make_scan(u, s, dt, dev) for s, dt in zip(specs, dts)]
    Ls = [u.ufss_lipschitz(p, max_iters=100, rtol=1e-5) for p, _, _, _ in scans]
    lams = []
    singles = []
    for (p, _, _, y), L in zip(scans, Ls):
        x = torch.zeros(p.nvox, dtype=torch.complex64, device=dev)
        st = u.ufss_fista(p, y, u.lambda_from_mu(0.1), L, 20, x)
        lams.append(st["lambda"])
        singles.append(x.clone())
    xs = [torch.zeros(p.nvox, dtype=torch.complex64, device=dev) for p, _, _, _ in scans]
    res = u.ufss_fista_batched([s[0] for s in scans], [s[3] for s in scans], xs, lams, Ls, 20)
    assert np.all(np.isfinite(res))
    for i, (xb, xs1) in enumerate(zip(xs, singles)):
        e = (torch.linalg.norm(xb - xs1) / torch.linalg.norm(xs1)).item()
        assert e < (1e-4 if dts[i] else 1e-5), (i, e)
    # the mu rule inside the batched call gives the same lambdas
    xs2 = [torch.zeros_like(x) for x in xs]
    u.ufss_fista_batched([s[0] for s in scans], [s[3] for s in scans], xs2, [-0.1] * len(scans), Ls, 20)
    for xb, x2 in zip(xs, xs2):
        assert (torch.linalg.norm(xb - x2) / torch.linalg.norm(xb)).item() < 1e-5
    # repeated call: identical result (graph built and replayed fresh)
    xs3 = [torch.zeros_like(x) for x in xs]
    u.ufss_fista_batched([s[0] for s in scans], [s[3] for s in scans], xs3, lams, Ls, 20)
    for xb, x3 in zip(xs, xs3):
        assert torch.equal(xb, x3)
    for p, _, _, _ in scans:
        p.close()


def test_batched_scan_against_oracle(dev):
    """One FP32 scan of a batch against the FP64 oracle's FISTA iterate."""
    u = ufss()
    g = W.geometry(12, 10, 40, 128, win_x=4, win_y=4)
    bins, _ = u.ufss_select_freqs(g, 10, True, 3)
    A = O.dense_A(g, bins)
    x_true = W.scene(g, 5, amp=(0.5, 1.0), seed=4)
    y = (A @ x_true.reshape(-1)).astype(np.complex64)
    yd = y.astype(np.complex128)
    L = V.lipschitz_dense(A) * 1.01
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, 0.1)
    a_ref, _ = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, yd, lam, L, 30)
    g2 = W.geometry(40, 1, 64, 128)
    bins2, _ = u.ufss_select_freqs(g2, 12, False, 5)
    p1 = u.Plan(g, 10, True, bins, algo=u.ALGO_GEMM)
    p2 = u.Plan(g2, 12, False, bins2)
    y1 = torch.from_numpy(y.reshape(10, 12, 10)).to(dev)
    y2 = torch.from_numpy(W.cn((1, 40, 12), 9).astype(np.complex64)).to(dev)
    x1 = torch.zeros((10, 12, 40), dtype=torch.complex64, device=dev)
    x2 = torch.zeros((1, 40, 64), dtype=torch.complex64, device=dev)
    L2 = u.ufss_lipschitz(p2)
    u.ufss_fista_batched([p1, p2], [y1, y2], [x1, x2], [lam, -0.1], [L, L2], 30)
    e = np.linalg.norm(x1.cpu().numpy().reshape(-1) - a_ref) / np.linalg.norm(a_ref)
    assert e < 1e-5, e
    p1.close()
    p2.close()


def test_batched_divergence_and_errors(dev):
    u = ufss()
    g = W.geometry(10, 1, 32, 128)
    bins, _ = u.ufss_select_freqs(g, 8, False, 1)
    p = u.Plan(g, 8, False, bins)
    L = u.ufss_lipschitz(p)
    y = torch.from_numpy(W.cn((1, 10, 8), 1).astype(np.complex64)).to(dev)
    x = torch.zeros((1, 10, 32), dtype=torch.complex64, device=dev)
    with pytest.raises(u.UfssError) as e:
        u.ufss_fista_batched([p], [y], [x], [1e-3], [L / 4], 300)
    assert e.value.name == "DIVERGED"
    with pytest.raises(u.UfssError) as e:
        u.ufss_fista_batched([p, p], [y, y], [x, x], [1.0, 1.0], [L, L], 3)
    assert e.value.name == "INVALID_ARG"
    pp = u.Plan(W.geometry(6, 6, 16, 64), 4, True,
                u.ufss_select_freqs(W.geometry(6, 6, 16, 64), 4, True, 1)[0], algo=u.ALGO_PHASOR)
    y6 = torch.zeros((6, 6, 4), dtype=torch.complex64, device=dev)
    x6 = torch.zeros((6, 6, 16), dtype=torch.complex64, device=dev)
    with pytest.raises(u.UfssError) as e:
        u.ufss_fista_batched([pp], [y6], [x6], [1.0], [1.0], 2)
    assert e.value.name == "UNSUPPORTED"
    p.close()
    pp.close()


def test_autotune_cache_and_correctness(dev, tmp_path):
    u = ufss()
    g = W.geometry(24, 20, 96, 256, win_x=6, win_y=6)
    bins, _ = u.ufss_select_freqs(g, 20, False, 8)
    cache = str(tmp_path / "tune.json")
    for dt in (u.F32, u.BF16):
        p = u.Plan(g, 20, False, bins, dtype=dt)
        fs, asp = u.ufss_autotune(p, cache, use_cache=True, write_cache=True)
        info = p.info()
        assert (info["fwd_split"], info["adj_split"]) == (fs, asp)
        # candidates 1, 2, 3, 4, 6, 8, 12, ... up to the d_y rows (2 W_y + 1 = 13)
        assert fs in (1, 2, 3, 4, 6, 8, 12) and asp in (1, 2, 3, 4, 6, 8, 12)
        data = json.load(open(cache))
        key = [k for k in data if ("bf16" if dt else "f32") in k][0]
        assert data[key][:2] == [fs, asp]
        p2 = u.Plan(g, 20, False, bins, dtype=dt)
        assert u.ufss_autotune(p2, cache, use_cache=True, write_cache=False) == (fs, asp)
        # the operator is unchanged by the re-split
        x = W.cn((20, 24, 96), 2)
        y_ref = np.stack([O.apply_A_at(g, bins, x, py, px) for (py, px) in [(0, 0), (10, 12)]])
        yt = torch.empty((20, 24, 20), dtype=torch.complex64, device=dev)
        u.ufss_forward(p2, torch.from_numpy(x.astype(np.complex64)).to(dev), yt)
        yg = yt.cpu().numpy()
        got = np.stack([yg[0, 0], yg[10, 12]])
        e = np.linalg.norm(got - y_ref) / np.linalg.norm(y_ref)
        assert e < (1e-2 if dt else 1e-5), e
        p.close()
        p2.close()
    assert os.path.exists(cache)


def test_persistent_batch_replays_new_data_and_holds_plans(dev):
    """ufss_batch_*: the captured iterations replayed; every replay starts from
    the x buffers' contents and reads the y buffers' contents, so replays equal
    single-scan FISTA on whatever the buffers hold; plans are held meanwhile."""
    u = ufss()
    specs, dts = small_batch()
    scans = [make_scan(u, s, dt, dev) for s, dt in zip(specs, dts)]
    plans = [sc[0] for sc in scans]
    ys = [sc[3] for sc in scans]
    Ls = [u.ufss_lipschitz(p, max_iters=100, rtol=1e-5) for p in plans]
    xs = [torch.zeros(p.nvox, dtype=torch.complex64, device=dev) for p in plans]
    K = 15
    b = u.Batch(plans, ys, xs, [-0.1] * len(plans), Ls, K)
    _, lam1 = b.run()
    first = [x.clone() for x in xs]
    for x in xs:
        x.zero_()
    _, lam2 = b.run()
    assert np.array_equal(lam1, lam2)
    for a, c in zip(first, xs):
        assert torch.equal(a, c)                      # replay is bitwise repeatable
    tol = lambda i: 1e-4 if dts[i] else 1e-5
    for i, (p, y) in enumerate(zip(plans, ys)):
        x1 = torch.zeros(p.nvox, dtype=torch.complex64, device=dev)
        st = u.ufss_fista(p, y, u.lambda_from_mu(0.1), Ls[i], K, x1)
        assert st["lambda"] == pytest.approx(lam1[i], rel=1e-6)
        e = (torch.linalg.norm(xs[i] - x1) / torch.linalg.norm(x1)).item()
        assert e < tol(i), (i, e)
    # warm start: a replay continues from the current x (momentum restarted)
    start = [x.clone() for x in xs]
    b.run()
    for i, (p, y) in enumerate(zip(plans, ys)):
        x1 = start[i].clone()
        u.ufss_fista(p, y, lam1[i], Ls[i], K, x1)
        e = (torch.linalg.norm(xs[i] - x1) / torch.linalg.norm(x1)).item()
        assert e < tol(i), (i, e)
    # new measurements in the same buffers, lambdas re-resolved by the mu rule
    for i, y in enumerate(ys):
        y.copy_(torch.from_numpy(W.cn(tuple(y.shape), 500 + i).astype(np.complex64)).to(dev))
    b.set_lambdas([-0.1] * len(plans))
    for x in xs:
        x.zero_()
    _, lam3 = b.run()
    assert not np.allclose(lam3, lam1)
    for i, (p, y) in enumerate(zip(plans, ys)):
        x1 = torch.zeros(p.nvox, dtype=torch.complex64, device=dev)
        st = u.ufss_fista(p, y, u.lambda_from_mu(0.1), Ls[i], K, x1)
        assert st["lambda"] == pytest.approx(lam3[i], rel=1e-6)
        e = (torch.linalg.norm(xs[i] - x1) / torch.linalg.norm(x1)).item()
        assert e < tol(i), (i, e)
    # held plans: no destroy, retile or second batch while the batch lives
    with pytest.raises(u.UfssError) as e:
        u.ufss_plan_set_tiling(plans[0], fwd_split=1)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(u.UfssError) as e:
        u.ufss_autotune(plans[0], None, False, False)
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(u.UfssError) as e:
        plans[0].close()
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(u.UfssError) as e:
        u.Batch(plans[:1], ys[:1], xs[:1], [1.0], Ls[:1], 2)
    assert e.value.name == "INVALID_ARG"
    b.close()
    u.ufss_plan_set_tiling(plans[0], fwd_split=1)
    for p in plans:
        p.close()


def test_config4_batch_at_full_shapes(dev):
    """The 64 uneven scans of the batched workload at their own shapes (lateral
    16-58, depth 128-512, 32-128 shared or per-position bins, B- and C-scans),
    with the tilings the autotuner picks (quick search, as in the benchmark):
    three batched iterations equal single-scan FISTA on every scan, and the
    operator of the two largest scans matches the oracle on sampled positions
    and voxel columns."""
    u = ufss()
    specs = W.batch_workload()
    plans, ys, bins_l = [], [], []
    for s in specs:
        p, bins, m, y = make_scan(u, s, u.F32, dev)
        u.ufss_autotune(p, None, use_cache=False, write_cache=False, quick=True)
        plans.append(p)
        ys.append(y)
        bins_l.append(bins)
    # any L above ||A||^2 keeps FISTA stable; the Frobenius norm is one
    Ls = [u.ufss_sigma_estimate(s["geom"], p.m, s["per_position"], b)["fro_sq"]
          for s, p, b in zip(specs, plans, bins_l)]
    K = 3
    xs = [torch.zeros(p.nvox, dtype=torch.complex64, device=dev) for p in plans]
    b = u.Batch(plans, ys, xs, [-0.1] * len(plans), Ls, K)
    res, lam = b.run()
    assert np.all(np.isfinite(res)) and np.all(lam > 0)
    b.close()
    worst = 0.0
    for i, (p, y) in enumerate(zip(plans, ys)):
        x1 = torch.zeros(p.nvox, dtype=torch.complex64, device=dev)
        u.ufss_fista(p, y, lam[i], Ls[i], K, x1)
        e = (torch.linalg.norm(xs[i] - x1) / torch.linalg.norm(x1)).item()
        worst = max(worst, e)
        assert e < 1e-5, (i, e)
    # the operator of the two largest scans against the oracle, sampled
    big = sorted(range(len(specs)), key=lambda i: -plans[i].nvox)[:2]
    for i in big:
        g = specs[i]["geom"]
        p = plans[i]
        x = W.cn((g["ny"], g["nx"], g["nz"]), 70 + i)
        yv = W.cn((g["ny"], g["nx"], p.m), 80 + i)
        yo = torch.empty((g["ny"], g["nx"], p.m), dtype=torch.complex64, device=dev)
        xo = torch.empty((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
        u.ufss_forward(p, torch.from_numpy(x.astype(np.complex64)).to(dev), yo)
        u.ufss_adjoint(p, torch.from_numpy(yv.astype(np.complex64)).to(dev), xo)
        yg, xg = yo.cpu().numpy(), xo.cpu().numpy()
        for py, px in ((0, 0), (g["ny"] // 2, g["nx"] - 1), (g["ny"] - 1, g["nx"] // 3)):
            want = O.apply_A_at(g, bins_l[i], x, py, px)
            assert np.abs(yg[py, px] - want).max() <= 1e-5 * np.abs(want).max(), (i, py, px)
        for vy, vx in ((g["ny"] - 1, 0), (g["ny"] // 2, g["nx"] // 2)):
            want = O.apply_AH_at(g, bins_l[i], yv, vy, vx)
            assert np.abs(xg[vy, vx] - want).max() <= 1e-5 * np.abs(want).max(), (i, vy, vx)
    for p in plans:
        p.close()
