"""GPU parity of the BF16 operator (BF16 phasors and operands, FP32
accumulation) against the FP64 oracle: relative error <= 1e-2, norm-wise and
element-wise against the largest output.  Also the precision study on the
64 x 64 C-scan workload restricted to a 16 x 16 x 128 sub-volume (same bins
and window start), where FP32 and BF16 errors are both measured."""
import numpy as np
import pytest

from oracle import geometry as G
from oracle import operator as O
from oracle import solver as V
from paper_2012_04534_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL16 = 1e-2


def ufss():
    from paper_2012_04534_amd import ufss as u
    return u


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def errs(got, ref):
    d = np.asarray(got).astype(np.complex128) - ref
    return (np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


def apply_both(u, plan, x, y, dev):
    xt = torch.from_numpy(x.astype(np.complex64)).to(dev)
    yt = torch.from_numpy(y.astype(np.complex64)).to(dev)
    yo = torch.empty_like(yt)
    xo = torch.empty_like(xt)
    u.ufss_forward(plan, xt, yo)
    u.ufss_adjoint(plan, yt, xo)
    torch.cuda.synchronize()
    return yo.cpu().numpy(), xo.cpu().numpy()


CASES = [
    (dict(nx=6, ny=5, nz=24, nt=64, win=-1), 6, False),
    (dict(nx=6, ny=5, nz=24, nt=64, win=2), 6, True),
    (dict(nx=13, ny=7, nz=45, nt=128, win=3), 11, False),
    (dict(nx=40, ny=1, nz=70, nt=128, win=-1), 11, True),
    (dict(nx=5, ny=3, nz=9, nt=64, win=1), 1, False),
    (dict(nx=19, ny=17, nz=100, nt=256, win=5), 30, False),
    # union of 66 bins: a second forward bin tile with one active 16-bin sub-tile
    (dict(nx=20, ny=3, nz=20, nt=512, win=4), 40, True),
    # grid wide enough for 64-position tiles, ragged in x
    (dict(nx=50, ny=2, nz=16, nt=128, win=-1), 10, False),
]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_bf16_small(ci, dev):
    u = ufss()
    gs, m, per_pos = CASES[ci]
    g = W.geometry(gs["nx"], gs["ny"], gs["nz"], gs["nt"], win_x=gs["win"], win_y=gs["win"])
    bins, _ = u.ufss_select_freqs(g, m, per_pos, 50 + ci)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 300 + ci)
    y = W.cn((g["ny"], g["nx"], m), 400 + ci)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1)).reshape(x.shape)
    plan = u.Plan(g, m, per_pos, bins, dtype=u.BF16)
    yo, xo = apply_both(u, plan, x, y, dev)
    ey, ex = errs(yo, y_ref), errs(xo, x_ref)
    assert max(ey) < TOL16, ey
    assert max(ex) < TOL16, ex
    # BF16 rounding is visible: not accidentally the FP32 path
    assert ey[0] > 1e-5
    plan.close()


def test_precision_study_subvolume(dev, record_property):
    """64 x 64 C-scan physics (same 128 bins and window start) on sub-volumes:
    the operator on 16 x 16 x 128 (outputs sampled one position / voxel column
    at a time by the oracle) and 50 FISTA iterations on 8 x 8 x 64 with 15 dB
    noise (dense oracle).  FP32 within 1e-5 and BF16 within 1e-2."""
    u = ufss()
    w = W.workload("cscan64")
    full = w["geom"]
    bins, _ = u.ufss_select_freqs(full, w["m"], False, w["seed"])
    t0 = G.t0(full)
    g = W.subvolume(full, 16, 16, 128)
    g["t0"] = t0
    xr = W.cn((16, 16, 128), 23)
    yr = W.cn((16, 16, w["m"]), 24)
    pos = [(0, 0), (15, 15), (8, 7), (2, 13)]
    cols = [(0, 15), (9, 6)]
    y_ref = np.stack([O.apply_A_at(g, bins, xr, py, px) for (py, px) in pos])
    x_ref = np.stack([O.apply_AH_at(g, bins, yr, vy, vx) for (vy, vx) in cols])
    gs = W.subvolume(full, 8, 8, 64)
    gs["t0"] = t0
    A = O.dense_A(gs, bins)
    x_true = W.scene(gs, 5, amp=(0.5, 1.0), seed=21)
    y0 = A @ x_true.reshape(-1)
    sig = W.noise_sigma(float(np.vdot(y0, y0).real), y0.size, w["snr_db"])
    y = (y0 + sig * W.cn(y0.size, 22)).astype(np.complex64).astype(np.complex128)
    L = V.lipschitz_dense(A) * 1.01
    lam = V.lambda_rule(lambda v: A.conj().T @ v, y, w["mu"])
    a_ref, _ = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, y, lam, L, 50)
    out = {}
    for dt, tol in ((u.F32, 1e-5), (u.BF16, TOL16)):
        plan = u.Plan(g, w["m"], False, bins, dtype=dt)
        yo, xo = apply_both(u, plan, xr, yr, dev)
        e_op = max(errs(np.stack([yo[py, px] for (py, px) in pos]), y_ref)[0],
                   errs(np.stack([xo[vy, vx] for (vy, vx) in cols]), x_ref)[0])
        plan.close()
        plan = u.Plan(gs, w["m"], False, bins, dtype=dt)
        x = torch.zeros((8, 8, 64), dtype=torch.complex64, device=dev)
        yt = torch.from_numpy(y.reshape(8, 8, w["m"]).astype(np.complex64)).to(dev)
        u.ufss_fista(plan, yt, lam, L, 50, x)
        e_img = np.linalg.norm(x.cpu().numpy().reshape(-1) - a_ref) / np.linalg.norm(a_ref)
        plan.close()
        out[dt] = (e_op, e_img)
        assert e_op < tol and e_img < tol, (dt, e_op, e_img)
    record_property("fp32_operator_err", out[u.F32][0])
    record_property("fp32_image_err", out[u.F32][1])
    record_property("bf16_operator_err", out[u.BF16][0])
    record_property("bf16_image_err", out[u.BF16][1])
    print("precision study: FP32 op %.2e img %.2e | BF16 op %.2e img %.2e" % (
        out[u.F32][0], out[u.F32][1], out[u.BF16][0], out[u.BF16][1]))


def test_bf16_fista_bscan(dev):
    """BF16 operator inside FISTA on the B-scan workload: image within 1e-2
    of the FP64 oracle's FISTA iterate (same L and lambda)."""
    u = ufss()
    w = W.workload("bscan32")
    g = w["geom"]
    bins, _ = u.ufss_select_freqs(g, w["m"], False, w["seed"])
    A = O.dense_A(g, bins)
    x_true = W.scene(g, w["n_scat"], seed=11)
    y0 = A @ x_true.reshape(-1)
    sig = W.noise_sigma(float(np.vdot(y0, y0).real), y0.size, w["snr_db"])
    y = (y0 + sig * W.cn(y0.size, 12)).astype(np.complex64).astype(np.complex128)
    L = V.lipschitz_dense(A) * 1.01
    lam = V.lambda_rule(lambda v: A.conj().T @ v, y, w["mu"])
    a_ref, _ = V.fista(lambda v: A @ v, lambda v: A.conj().T @ v, y, lam, L, w["iters"])
    plan = u.Plan(g, w["m"], False, bins, dtype=u.BF16)
    x = torch.zeros((1, 32, 128), dtype=torch.complex64, device=dev)
    u.ufss_fista(plan, torch.from_numpy(y.reshape(1, 32, w["m"]).astype(np.complex64)).to(dev),
                 lam, L, w["iters"], x)
    e = np.linalg.norm(x.cpu().numpy().reshape(-1) - a_ref) / np.linalg.norm(a_ref)
    assert e < TOL16, e
    plan.close()


@pytest.mark.parametrize("m", [33, 36, 37, 68, 100])
def test_bf16_adjoint_short_last_chunk(m, dev):
    """Bin counts whose last 32-bin chunk holds 1, 4, 5, 4 and 4 bins: with the
    phasor tables, up to 4 such bins are folded into the previous chunk's
    offset steps (4 x 4 x 4 products), 5 take a chunk of their own; both match
    the oracle, with the tables and with in-kernel phasor generation."""
    u = ufss()
    g = W.geometry(9, 5, 40, 1024, win_x=3, win_y=3)
    bins, _ = u.ufss_select_freqs(g, m, False, 7 + m)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 500 + m)
    y = W.cn((g["ny"], g["nx"], m), 600 + m)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1)).reshape(x.shape)
    plan = u.Plan(g, m, False, bins, dtype=u.BF16)
    for enable in (True, False):
        assert u.ufss_plan_set_phasor_tables(plan, enable) == enable
        yo, xo = apply_both(u, plan, x, y, dev)
        ey, ex = errs(yo, y_ref), errs(xo, x_ref)
        assert max(ey) < TOL16 and max(ex) < TOL16, (enable, ey, ex)
        assert ex[0] > 1e-5
    plan.close()


@pytest.mark.parametrize("ci", [2, 5, 6, 7])
def test_bf16_tables_and_generation_agree(ci, dev):
    """The precomputed phasor tables (default) and in-kernel generation give
    the oracle's operator to BF16 accuracy, and agree closely with each other."""
    u = ufss()
    gs, m, per_pos = CASES[ci]
    g = W.geometry(gs["nx"], gs["ny"], gs["nz"], gs["nt"], win_x=gs["win"], win_y=gs["win"])
    bins, _ = u.ufss_select_freqs(g, m, per_pos, 50 + ci)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 300 + ci)
    y = W.cn((g["ny"], g["nx"], m), 400 + ci)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1)).reshape(x.shape)
    plan = u.Plan(g, m, per_pos, bins, dtype=u.BF16)
    out = {}
    for enable in (True, False, True):
        assert u.ufss_plan_set_phasor_tables(plan, enable) == enable
        yo, xo = apply_both(u, plan, x, y, dev)
        ey, ex = errs(yo, y_ref), errs(xo, x_ref)
        assert max(ey) < TOL16 and max(ex) < TOL16, (enable, ey, ex)
        out.setdefault(enable, []).append((yo, xo))
    # tables rebuilt after freeing: identical results
    (y1, x1), (y2, x2) = out[True]
    assert np.array_equal(y1, y2) and np.array_equal(x1, x2)
    plan.close()
    fplan = u.Plan(g, m, per_pos, bins, dtype=u.F32)
    with pytest.raises(u.UfssError):
        u.ufss_plan_set_phasor_tables(fplan, True)
    fplan.close()
