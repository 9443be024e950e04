"""GPU parity of the solver calls (C ABI) against the FP64 oracle: fused
update, absmax / lambda rule, Lipschitz power iteration, FISTA / ISTA
trajectories, resume, divergence detection."""
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


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def test_shrink_update_matches_oracle(dev):
    u = ufss()
    n = 100003
    gam = W.cn(n, 1).astype(np.complex64)
    g = W.cn(n, 2).astype(np.complex64)
    a = W.cn(n, 3).astype(np.complex64)
    aref = W.cn(n, 4).astype(np.complex64)
    gam[:10] = 0
    g[:10] = 0
    step, thr, beta = 0.3, 0.45, 0.6
    gt, gg, at, rt = to_dev(gam, dev), to_dev(g, dev), to_dev(a, dev), to_dev(aref, dev)
    norms = u.ufss_shrink_update(gt, gg, at, step, thr, beta, a_ref=rt)
    G = gam.astype(np.complex128)
    a_new = V.soft(G - step * g.astype(np.complex128), thr)
    g_new = a_new + beta * (a_new - a.astype(np.complex128))
    ag, gn = at.cpu().numpy(), gt.cpu().numpy()
    assert np.abs(ag - a_new).max() < 1e-6 * np.abs(a_new).max()
    assert np.abs(gn - g_new).max() < 1e-6 * np.abs(g_new).max()
    assert np.all(ag[:10] == 0)
    want = [np.abs(a_new).sum(), np.abs(g_new).sum(), np.sum(np.abs(a_new - a) ** 2),
            np.sum(np.abs(a_new) ** 2), np.sum(np.abs(a_new - aref) ** 2)]
    np.testing.assert_allclose(norms, want, rtol=1e-6)
    # bitwise reproducible reductions
    gt2, at2 = to_dev(gam, dev), to_dev(a, dev)
    norms2 = u.ufss_shrink_update(gt2, gg, at2, step, thr, beta, a_ref=rt)
    assert np.array_equal(norms, norms2)


def test_shrink_update_empty_and_absmax(dev):
    u = ufss()
    e = torch.zeros(0, dtype=torch.complex64, device=dev)
    norms = u.ufss_shrink_update(e, e, e, 1.0, 1.0, 0.0)
    assert np.all(norms == 0)
    v = W.cn(5000, 9).astype(np.complex64)
    assert u.ufss_absmax(to_dev(v, dev)) == pytest.approx(np.abs(v.astype(np.complex128)).max(), rel=1e-7)


def bscan_problem():
    w = W.workload("bscan32")
    g = w["geom"]
    u = ufss()
    bins, _ = u.ufss_select_freqs(g, w["m"], False, w["seed"])
    A = O.dense_A(g, bins)
    x_true = W.scene(g, w["n_scat"], amp=w["amp"], seed=11)
    y0 = A @ x_true.reshape(-1)
    sig = W.noise_sigma(float(np.vdot(y0, y0).real), y0.size, w["snr_db"])
    y = (y0 + sig * W.cn(y0.size, 12)).astype(np.complex64)
    return w, g, bins, A, x_true, y


def test_lipschitz_power_iteration(dev):
    u = ufss()
    w, g, bins, A, _, _ = bscan_problem()
    L_exact = V.lipschitz_dense(A)
    plan = u.Plan(g, w["m"], False, bins)
    L = u.ufss_lipschitz(plan, max_iters=500, rtol=1e-9, margin=0.0, seed=3)
    assert L <= L_exact * (1 + 2e-5)
    assert L >= L_exact * (1 - 1e-4)
    Lm = u.ufss_lipschitz(plan, max_iters=500, rtol=1e-9, margin=0.01, seed=3)
    assert Lm == pytest.approx(1.01 * L, rel=1e-5)
    assert plan.info()["lipschitz"] == Lm
    plan.close()


@pytest.mark.parametrize("accel", [True, False])
def test_fista_trajectory_matches_oracle_bscan(accel, dev):
    """200 iterations of the B-scan workload: GPU iterate vs oracle iterate
    with the same L and lambda, relative image error <= 1e-5 (FP32)."""
    u = ufss()
    w, g, bins, A, x_true, y = bscan_problem()
    yd = y.reshape(-1).astype(np.complex128)
    L = V.lipschitz_dense(A) * 1.01
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, w["mu"])
    a_ref, st = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, yd, lam, L, w["iters"], accel=accel)
    plan = u.Plan(g, w["m"], False, bins)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    stats = u.ufss_fista(plan, yt, lam, L, w["iters"], x, accel=accel)
    a = x.cpu().numpy().reshape(-1).astype(np.complex128)
    err = np.linalg.norm(a - a_ref) / np.linalg.norm(a_ref)
    assert err < 1e-5, err
    assert stats["iters_done"] == w["iters"]
    np.testing.assert_allclose(stats["res"], st["res"], rtol=1e-5)
    np.testing.assert_allclose(stats["obj"], st["obj"], rtol=1e-5)
    if not accel:
        assert np.all(np.diff(stats["obj"]) <= 1e-6 * stats["obj"][0])
    # lambda rule on the GPU: lambda = mu * max |A^H y|
    x2 = torch.zeros_like(x)
    st2 = u.ufss_fista(plan, yt, u.lambda_from_mu(w["mu"]), L, 3, x2, accel=accel)
    assert st2["lambda"] == pytest.approx(lam, rel=1e-6)
    plan.close()


def test_fista_support_recovery_and_ref_error(dev):
    """Check (d) on the GPU: the B-scan scene's support is recovered; err_ref
    stats agree with the host-side error."""
    u = ufss()
    w, g, bins, A, x_true, y = bscan_problem()
    plan = u.Plan(g, w["m"], False, bins)
    L = u.ufss_lipschitz(plan, margin=0.01)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    aref = to_dev(x_true, dev)
    stats = u.ufss_fista(plan, yt, u.lambda_from_mu(w["mu"]), L, w["iters"], x, a_ref=aref)
    a = x.cpu().numpy().reshape(-1)
    top = set(np.argsort(np.abs(a))[-w["n_scat"]:])
    assert top == set(np.flatnonzero(x_true.reshape(-1)))
    e = np.linalg.norm(a - x_true.reshape(-1)) / np.linalg.norm(x_true)
    assert stats["err_ref"][-1] == pytest.approx(e, rel=1e-5)
    plan.close()


def test_fista_resume_bitwise(dev):
    u = ufss()
    w, g, bins, A, _, y = bscan_problem()
    plan = u.Plan(g, w["m"], False, bins)
    L = float(V.lipschitz_dense(A) * 1.01)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    shape = (g["ny"], g["nx"], g["nz"])
    x100 = torch.zeros(shape, dtype=torch.complex64, device=dev)
    u.ufss_fista(plan, yt, 50.0, L, 100, x100)
    x = torch.zeros(shape, dtype=torch.complex64, device=dev)
    state = {"gamma": torch.zeros(shape, dtype=torch.complex64, device=dev), "k_done": 0}
    u.ufss_fista(plan, yt, 50.0, L, 50, x, state=state)
    assert state["k_done"] == 50
    u.ufss_fista(plan, yt, 50.0, L, 50, x, state=state)
    assert state["k_done"] == 100
    assert torch.equal(x, x100)
    plan.close()


def test_fista_divergence_detected(dev):
    """An under-estimated L (L/4) makes FISTA blow up; the library reports
    UFSS_ERR_DIVERGED instead of returning garbage silently."""
    u = ufss()
    w, g, bins, A, _, y = bscan_problem()
    plan = u.Plan(g, w["m"], False, bins)
    L = float(V.lipschitz_dense(A))
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    with pytest.raises(u.UfssError) as e:
        u.ufss_fista(plan, yt, 1.0, L / 4, 300, x)
    assert e.value.name == "DIVERGED"
    plan.close()


@pytest.mark.parametrize("algo_name", ["ALGO_GEMM", "ALGO_PHASOR"])
def test_fista_per_position_small(algo_name, dev):
    """Per-position bins, both algorithms: 30 FISTA iterations vs the oracle."""
    u = ufss()
    g = W.geometry(10, 8, 32, 128, win_x=3, win_y=3)
    bins, _ = u.ufss_select_freqs(g, 8, True, 77)
    A = O.dense_A(g, bins)
    x_true = W.scene(g, 4, amp=(0.5, 1.0), seed=2)
    y = (A @ x_true.reshape(-1)).astype(np.complex64)
    yd = y.astype(np.complex128)
    L = V.lipschitz_dense(A) * 1.01
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, 0.1)
    a_ref, _ = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, yd, lam, L, 30)
    plan = u.Plan(g, 8, True, bins, algo=getattr(u, algo_name))
    x = torch.zeros((8, 10, 32), dtype=torch.complex64, device=dev)
    u.ufss_fista(plan, to_dev(y.reshape(8, 10, 8), dev), lam, L, 30, x)
    err = np.linalg.norm(x.cpu().numpy().reshape(-1) - a_ref) / np.linalg.norm(a_ref)
    assert err < 1e-5, err
    plan.close()


@pytest.mark.parametrize("mu", [1.0, 2.5])
def test_mu_at_least_one_keeps_zero_iterate(mu, dev):
    """lambda = mu max|A^H y| with mu >= 1: the soft threshold removes every
    entry of the first step from a = 0, so all iterates stay exactly zero."""
    u = ufss()
    w, g, bins, A, _, y = bscan_problem()
    plan = u.Plan(g, w["m"], False, bins)
    L = float(V.lipschitz_dense(A))
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    st = u.ufss_fista(plan, yt, u.lambda_from_mu(mu), L, 5, x)
    torch.cuda.synchronize()
    assert torch.count_nonzero(x).item() == 0
    assert st["lambda"] > 0
    plan.close()


def test_kernel_timing_mode_counts_core_launches(dev):
    """Timing mode brackets each core kernel launch: K FISTA iterations give K
    forward and K adjoint records; enabling again clears them; off records none."""
    u = ufss()
    w, g, bins, A, _, y = bscan_problem()
    plan = u.Plan(g, w["m"], False, bins)
    L = float(V.lipschitz_dense(A))
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    u.ufss_plan_kernel_timing(plan, True)
    u.ufss_fista(plan, yt, u.lambda_from_mu(0.1), L, 7, x)
    u.ufss_plan_kernel_timing(plan, False)
    f, a, nf, na = u.ufss_plan_kernel_times(plan)
    # the lambda rule adds one adjoint (A^H y) before the iterations
    assert nf == 7 and na == 8 and f > 0 and a > 0
    u.ufss_fista(plan, yt, u.lambda_from_mu(0.1), L, 3, x)
    assert u.ufss_plan_kernel_times(plan)[2:] == (7, 8)
    u.ufss_plan_kernel_timing(plan, True)
    assert u.ufss_plan_kernel_times(plan)[2:] == (0, 0)
    u.ufss_plan_kernel_timing(plan, False)
    plan.close()


def _bt_oracle(A, y, lam, L0, eta, iters, a_ref=None, eps=1e-6):
    yd = y.reshape(-1).astype(np.complex128)
    slack = eps * 0.5 * float(np.vdot(yd, yd).real)
    return V.fista_backtracking(lambda v: A @ v, lambda v: A.conj().T @ v, yd, lam, L0, eta,
                                iters, a_ref=a_ref, slack=slack)


def test_backtracking_matches_oracle_bscan(dev):
    """Backtracking FISTA on the B-scan workload from L0 = L/1000, eta = 2:
    the accepted constants and trial counts equal the oracle's, and the
    iterates agree to FP32 tolerance."""
    u = ufss()
    w, g, bins, A, x_true, y = bscan_problem()
    L = V.lipschitz_dense(A)
    yd = y.reshape(-1).astype(np.complex128)
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, w["mu"])
    a_o, st_o = _bt_oracle(A, y, lam, L / 1000.0, 2.0, 120, a_ref=x_true.reshape(-1))
    plan = u.Plan(g, w["m"], False, bins)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    st = u.ufss_fista_backtracking(plan, yt, lam, L / 1000.0, 2.0, 120, x,
                                   a_ref=to_dev(x_true, dev))
    assert st["iters_done"] == 120
    assert list(st["trials"]) == st_o["trials"]
    np.testing.assert_allclose(st["L"], st_o["L"], rtol=1e-12)
    assert st["L"][-1] <= 2.0 * L
    a = x.cpu().numpy().reshape(-1).astype(np.complex128)
    assert np.linalg.norm(a - a_o) / np.linalg.norm(a_o) < 1e-5
    np.testing.assert_allclose(st["obj"], st_o["obj"], rtol=1e-5)
    np.testing.assert_allclose(st["res"], st_o["res"], rtol=1e-5)
    np.testing.assert_allclose(st["err_ref"], st_o["err_ref"], rtol=1e-5)
    plan.close()


def test_backtracking_from_upper_bound_is_fista(dev):
    """L0 above sigma_max^2: one trial per iteration and the plain FISTA
    iterate (same L), up to FP32 rounding."""
    u = ufss()
    w, g, bins, A, _, y = bscan_problem()
    L0 = 1.5 * V.lipschitz_dense(A)
    plan = u.Plan(g, w["m"], False, bins)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    shape = (g["ny"], g["nx"], g["nz"])
    x1 = torch.zeros(shape, dtype=torch.complex64, device=dev)
    x2 = torch.zeros(shape, dtype=torch.complex64, device=dev)
    st = u.ufss_fista_backtracking(plan, yt, u.lambda_from_mu(0.1), L0, 3.0, 60, x1)
    u.ufss_fista(plan, yt, u.lambda_from_mu(0.1), L0, 60, x2)
    assert np.all(st["trials"] == 1) and np.all(st["L"] == L0)
    d = (x1 - x2).abs().max().item() / x2.abs().max().item()
    assert d < 1e-5, d
    plan.close()


@pytest.mark.parametrize("algo_name", ["ALGO_GEMM", "ALGO_PHASOR"])
def test_backtracking_per_position_small(algo_name, dev):
    u = ufss()
    g = W.geometry(10, 8, 32, 128, win_x=3, win_y=3)
    bins, _ = u.ufss_select_freqs(g, 8, True, 77)
    A = O.dense_A(g, bins)
    x_true = W.scene(g, 4, amp=(0.5, 1.0), seed=2)
    y = (A @ x_true.reshape(-1)).astype(np.complex64)
    L = V.lipschitz_dense(A)
    lam = V.lambda_rule(lambda v: A.conj().T @ v, y.astype(np.complex128), 0.1)
    a_o, st_o = _bt_oracle(A, y, lam, L / 50.0, 1.5, 40)
    plan = u.Plan(g, 8, True, bins, algo=getattr(u, algo_name))
    x = torch.zeros((8, 10, 32), dtype=torch.complex64, device=dev)
    st = u.ufss_fista_backtracking(plan, to_dev(y.reshape(8, 10, 8), dev), lam, L / 50.0, 1.5,
                                   40, x)
    assert list(st["trials"]) == st_o["trials"]
    err = np.linalg.norm(x.cpu().numpy().reshape(-1) - a_o) / np.linalg.norm(a_o)
    assert err < 1e-5, err
    plan.close()


def test_backtracking_bf16_and_errors(dev):
    """BF16 operator: the run converges to the FP64 oracle's solution within
    the BF16 tolerance; bad arguments are rejected."""
    u = ufss()
    w, g, bins, A, x_true, y = bscan_problem()
    L = V.lipschitz_dense(A)
    yd = y.reshape(-1).astype(np.complex128)
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, w["mu"])
    a_o, _ = _bt_oracle(A, y, lam, L / 100.0, 2.0, 150, eps=2.0 ** -8)
    plan = u.Plan(g, w["m"], False, bins, dtype=u.BF16)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    st = u.ufss_fista_backtracking(plan, yt, lam, L / 100.0, 2.0, 150, x)
    err = np.linalg.norm(x.cpu().numpy().reshape(-1) - a_o) / np.linalg.norm(a_o)
    assert err < 1e-2, err
    assert st["L"][-1] <= 2.0 * L * 1.02
    for L0, eta in ((0.0, 2.0), (1.0, 1.0), (-1.0, 2.0), (1.0, float("nan"))):
        with pytest.raises(u.UfssError) as e:
            u.ufss_fista_backtracking(plan, yt, lam, L0, eta, 3, x)
        assert e.value.name == "INVALID_ARG"
    plan.close()


def test_sigma_hat_as_lipschitz_bscan(dev):
    """The Sec. IV-C estimate sigma_hat^2 over-estimates L on the B-scan
    workload (1.37x): FISTA with it matches the oracle run with the same
    constant (100 iterations, 1e-5) and after 200 iterations reaches nearly
    the objective of the exact-L run (the oracle's gap is 7.9e-4)."""
    u = ufss()
    w, g, bins, A, _, y = bscan_problem()
    L = V.lipschitz_dense(A)
    est = u.ufss_sigma_estimate(g, w["m"], False, bins)
    Lh = est["sigma_hat"] ** 2
    assert L < Lh < 2 * L
    yd = y.reshape(-1).astype(np.complex128)
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, 0.1)
    a_o, _ = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, yd, lam, Lh, 100)
    plan = u.Plan(g, w["m"], False, bins)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    shape = (g["ny"], g["nx"], g["nz"])
    xa = torch.zeros(shape, dtype=torch.complex64, device=dev)
    xb = torch.zeros(shape, dtype=torch.complex64, device=dev)
    u.ufss_fista(plan, yt, lam, Lh, 100, xa)
    a = xa.cpu().numpy().reshape(-1)
    assert np.linalg.norm(a - a_o) / np.linalg.norm(a_o) < 1e-5
    xa.zero_()
    sa = u.ufss_fista(plan, yt, lam, Lh, 200, xa)
    sb = u.ufss_fista(plan, yt, lam, 1.01 * L, 200, xb)
    gap = (sa["obj"][-1] - sb["obj"][-1]) / sb["obj"][-1]
    assert abs(gap) < 2e-3, gap
    plan.close()


def test_fista_real_iterates_match_oracle(dev):
    """Real-reflectivity FISTA (accel bit 1, the Re{H} comparison) on the
    B-scan workload: iterates real and equal to the oracle's; unknown flag
    bits are refused."""
    u = ufss()
    w, g, bins, A, x_true, y = bscan_problem()
    yd = y.reshape(-1).astype(np.complex128)
    L = V.lipschitz_dense(A) * 1.01
    lam = V.lambda_rule(lambda v: A.conj().T @ v, yd, w["mu"])
    a_ref, _ = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, yd, lam, L, 100, real=True)
    plan = u.Plan(g, w["m"], False, bins)
    x = torch.zeros((g["ny"], g["nx"], g["nz"]), dtype=torch.complex64, device=dev)
    yt = to_dev(y.reshape(g["ny"], g["nx"], w["m"]), dev)
    u.ufss_fista(plan, yt, lam, L, 100, x, real=True)
    a = x.cpu().numpy().reshape(-1)
    assert np.all(a.imag == 0)
    assert np.linalg.norm(a - a_ref) / np.linalg.norm(a_ref) < 1e-5
    with pytest.raises(u.UfssError) as e:
        u._check(u.lib().ufss_fista(plan.handle, u._ptr(yt, "y"), lam, L, 2, 0.0, 4,
                                    u._ptr(x, "x"), None, None, None, u._stream(None)))
    assert e.value.name == "INVALID_ARG"
    plan.close()
