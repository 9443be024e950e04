"""GPU parity of the operator A / A^H (C ABI) against the FP64 oracle.

Tolerance: FP32 operator, relative error <= 1e-5 measured both norm-wise and
element by element against the largest output (max |gpu - ref| / max |ref|).
Cases: tiny grids for every mode, ragged sizes spanning several tiles, edge
cases, the full B-scan workload (dense oracle), and the full C-scan workloads
on outputs the oracle computes one position / one voxel column at a time.
"""
import json
import os

import numpy as np
import pytest

from oracle import operator as O
from oracle import select as S
from paper_2012_04534_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def ufss():
    from paper_2012_04534_amd import ufss as u
    return u


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def errs(got, ref):
    got = np.asarray(got).astype(np.complex128)
    d = got - ref
    return (np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


def run_op(plan, x, y_shape, dev):
    u = ufss()
    xt = torch.from_numpy(x.astype(np.complex64)).to(dev)
    yt = torch.empty(y_shape, dtype=torch.complex64, device=dev)
    u.ufss_forward(plan, xt, yt)
    return yt


def case_list():
    cases = []
    for win in (-1, 2):
        for per_pos in (False, True):
            cases.append(("tiny", dict(nx=6, ny=5, nz=24, nt=64, win=win), 6, per_pos))
    cases.append(("bscan", dict(nx=9, ny=1, nz=20, nt=64, win=3), 5, True))
    cases.append(("bscan-shared", dict(nx=40, ny=1, nz=37, nt=128, win=-1), 11, False))
    cases.append(("ragged", dict(nx=13, ny=7, nz=45, nt=128, win=3), 11, False))
    cases.append(("ragged-pp", dict(nx=13, ny=7, nz=45, nt=128, win=3), 11, True))
    cases.append(("one-bin", dict(nx=5, ny=3, nz=9, nt=64, win=1), 1, False))
    cases.append(("one-depth", dict(nx=6, ny=6, nz=1, nt=64, win=-1), 4, True))
    cases.append(("one-pos", dict(nx=1, ny=1, nz=30, nt=64, win=-1), 7, False))
    cases.append(("win0", dict(nx=7, ny=4, nz=17, nt=64, win=0), 8, False))
    cases.append(("tall", dict(nx=3, ny=21, nz=16, nt=64, win=5), 6, True))
    return cases


CASES = case_list()


def algos(per_pos):
    u = ufss()
    return [u.ALGO_GEMM, u.ALGO_PHASOR] if per_pos else [u.ALGO_GEMM]


@pytest.mark.parametrize("ci", range(len(CASES)), ids=[c[0] + str(i) for i, c in enumerate(CASES)])
def test_forward_adjoint_small(ci, dev):
    u = ufss()
    name, gs, m, per_pos = CASES[ci]
    g = W.geometry(gs["nx"], gs["ny"], gs["nz"], gs["nt"], win_x=gs["win"], win_y=gs["win"])
    bins, _ = u.ufss_select_freqs(g, m, per_pos, 31 + ci)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 100 + ci).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], m), 200 + ci).astype(np.complex64)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1).astype(np.complex128)).reshape(g["ny"], g["nx"], m)
    x_ref = (A.conj().T @ y.reshape(-1).astype(np.complex128)).reshape(x.shape)
    for algo in algos(per_pos):
        plan = u.Plan(g, m, per_pos, bins, algo=algo)
        yt = run_op(plan, x, y.shape, dev)
        xt = torch.empty(x.shape, dtype=torch.complex64, device=dev)
        u.ufss_adjoint(plan, torch.from_numpy(y).to(dev), xt)
        torch.cuda.synchronize()
        ey = errs(yt.cpu().numpy(), y_ref)
        ex = errs(xt.cpu().numpy(), x_ref)
        assert max(ey) < TOL32, (name, algo, "forward", ey)
        assert max(ex) < TOL32, (name, algo, "adjoint", ex)
        plan.close()


@pytest.mark.parametrize("per_pos", [False, True])
def test_gpu_adjointness_and_determinism(per_pos, dev):
    u = ufss()
    g = W.geometry(20, 12, 64, 256, win_x=6, win_y=6)
    bins, _ = u.ufss_select_freqs(g, 24, per_pos, 5)
    for algo in algos(per_pos):
        plan = u.Plan(g, 24, per_pos, bins, algo=algo)
        x = torch.from_numpy(W.cn((12, 20, 64), 1).astype(np.complex64)).to(dev)
        y = torch.from_numpy(W.cn((12, 20, 24), 2).astype(np.complex64)).to(dev)
        Ax = torch.empty_like(y)
        AHy = torch.empty_like(x)
        u.ufss_forward(plan, x, Ax)
        u.ufss_adjoint(plan, y, AHy)
        Ax2 = torch.empty_like(y)
        AHy2 = torch.empty_like(x)
        u.ufss_forward(plan, x, Ax2)
        u.ufss_adjoint(plan, y, AHy2)
        torch.cuda.synchronize()
        assert torch.equal(Ax, Ax2) and torch.equal(AHy, AHy2)
        lhs = np.vdot(y.cpu().numpy().astype(np.complex128), Ax.cpu().numpy().astype(np.complex128))
        rhs = np.vdot(AHy.cpu().numpy().astype(np.complex128), x.cpu().numpy().astype(np.complex128))
        scale = np.linalg.norm(Ax.cpu().numpy()) * np.linalg.norm(y.cpu().numpy())
        assert abs(lhs - rhs) < 1e-6 * scale
        plan.close()


def test_bscan_workload_full(dev):
    """Full 32-position B-scan workload against the dense FP64 oracle."""
    u = ufss()
    w = W.workload("bscan32")
    g = w["geom"]
    bins, _ = u.ufss_select_freqs(g, w["m"], False, w["seed"])
    A = O.dense_A(g, bins)
    plan = u.Plan(g, w["m"], False, bins)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 3).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], w["m"]), 4).astype(np.complex64)
    yt = run_op(plan, x, y.shape, dev)
    xt = torch.empty(x.shape, dtype=torch.complex64, device=dev)
    u.ufss_adjoint(plan, torch.from_numpy(y).to(dev), xt)
    torch.cuda.synchronize()
    assert max(errs(yt.cpu().numpy().reshape(-1), A @ x.reshape(-1).astype(np.complex128))) < TOL32
    assert max(errs(xt.cpu().numpy().reshape(-1), A.conj().T @ y.reshape(-1).astype(np.complex128))) < TOL32
    plan.close()


# The bench runs the tilings of the shipped autotuner cache; each full-size
# workload is checked at the plan's default tiling and at that one.
SHIPPED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2012_04534_amd", "tuning_gfx950.json")
WORKLOADS = [("cscan32", "f32"), ("cscan32", "bf16"), ("cscan64", "f32"), ("cscan64", "bf16")]


def shipped_tiling(plan, g, dtype):
    """ufss_tiling values of the shipped cache entry for this plan's shape, or None."""
    info = plan.info()
    key = "gfx950/nx%d/ny%d/nz%d/mu%d/m%d/wx%d/wy%d/%s" % (
        g["nx"], g["ny"], g["nz"], info["union_size"], info["m"], info["win_x"], info["win_y"], dtype)
    e = json.load(open(SHIPPED)).get(key)
    if e is None or len(e) < 12:
        return None
    vals = [int(v) for v in e]
    fs, as_, _, _, nw, zs, npf, npa, rf, ra, zc, kc = vals[:12]
    if dtype == "bf16":          # BF16: adj_tile carries the adjoint's depth sub-tiles
        npa = vals[12] if len(vals) > 12 else 4
    aw = vals[13] if len(vals) > 13 else 4
    return dict(fwd_split=fs, adj_split=as_, fwd_waves=nw, fwd_zsplit=zs, fwd_tile=npf, adj_tile=npa,
                fwd_rows=rf, adj_rows=ra, fwd_chunk=zc, adj_chunk=kc, adj_waves=aw)


@pytest.mark.parametrize("name,dtype", WORKLOADS)
def test_cscan_workloads_full_sampled(name, dtype, dev):
    """Full-size C-scan workloads, in the bench's launch configurations, checked
    on positions / voxel columns the oracle evaluates one at a time (corners,
    edges and the centre)."""
    u = ufss()
    w = W.workload(name)
    g = w["geom"]
    m = w["m"]
    bins, _ = u.ufss_select_freqs(g, m, w["per_position"], w["seed"])
    x = W.cn((g["ny"], g["nx"], g["nz"]), 5).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], m), 6).astype(np.complex64)
    nx, ny = g["nx"], g["ny"]
    pos = [(0, 0), (ny - 1, nx - 1), (ny // 2, nx // 2), (3, nx - 5)]
    cols = [(0, nx - 1), (ny // 2 + 1, nx // 2 - 2)]
    y_ref = np.stack([O.apply_A_at(g, bins, x, py, px) for (py, px) in pos])
    x_ref = np.stack([O.apply_AH_at(g, bins, y, vy, vx) for (vy, vx) in cols])
    tol = TOL32 if dtype == "f32" else 1e-2
    runs = [(u.ALGO_GEMM, None), (u.ALGO_GEMM, "shipped")]
    if dtype == "f32" and w["per_position"]:
        runs.append((u.ALGO_PHASOR, None))
    if dtype == "f32":
        runs.append((u.ALGO_FFT, None))
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    for algo, tiling in runs:
        plan = u.Plan(g, m, w["per_position"], bins, algo=algo, dtype=u.F32 if dtype == "f32" else u.BF16)
        if tiling == "shipped":
            tiling = shipped_tiling(plan, g, dtype)
            assert tiling is not None, "no shipped tiling for %s %s" % (name, dtype)
            u.ufss_plan_set_tiling(plan, **tiling)
        yt = torch.empty(y.shape, dtype=torch.complex64, device=dev)
        xt = torch.empty(x.shape, dtype=torch.complex64, device=dev)
        u.ufss_forward(plan, xd, yt)
        u.ufss_adjoint(plan, yd, xt)
        torch.cuda.synchronize()
        yg = yt.cpu().numpy()
        xg = xt.cpu().numpy()
        ey = errs(np.stack([yg[py, px] for (py, px) in pos]), y_ref)
        ex = errs(np.stack([xg[vy, vx] for (vy, vx) in cols]), x_ref)
        assert max(ey) < tol, (name, dtype, algo, tiling, ey)
        assert max(ex) < tol, (name, dtype, algo, tiling, ex)
        plan.close()


def test_plan_info_and_errors(dev):
    u = ufss()
    g = W.workload("cscan32")["geom"]
    bins, _ = u.ufss_select_freqs(g, 64, True, 1002)
    plan = u.Plan(g, 64, True, bins)
    info = plan.info()
    assert info["band_size"] == 66 and info["union_size"] <= 66 and info["per_position"] == 1
    assert abs(info["t0"] - 7.6234185e-6) < 1e-12
    x = torch.zeros(10, dtype=torch.complex64, device=dev)
    y = torch.zeros(32 * 32 * 64, dtype=torch.complex64, device=dev)
    with pytest.raises(ValueError):
        u.ufss_forward(plan, x, y)
    plan.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_manual_tiling_same_operator(dtype, dev):
    """Every tiling of the GEMM path computes the same operator: d_y and depth
    splits (including parts left without rows), waves per workgroup."""
    u = ufss()
    g = W.geometry(11, 9, 40, 256, win_x=4, win_y=4)
    bins, _ = u.ufss_select_freqs(g, 20, True, 77)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 5).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], 20), 6).astype(np.complex64)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1).astype(np.complex128)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1).astype(np.complex128)).reshape(x.shape)
    tol = TOL32 if dtype == "f32" else 1e-2
    plan = u.Plan(g, 20, True, bins, dtype=u.F32 if dtype == "f32" else u.BF16)
    # (fwd_split, adj_split, fwd_waves, fwd_zsplit, fwd_tile, adj_tile, fwd_rows,
    #  adj_rows, fwd_chunk, adj_chunk, adj_waves)
    tilings = [(1, 1, 1, 1, 2, 2, 0, 0, 16, 16, 8), (3, 2, 2, 3, 4, 4, 0, 0, 8, 8, 8),
               (9, 9, 8, 10, 4, 2, 0, 0, 16, 8, 4), (64, 64, 3, 64, 2, 4, 0, 0, 8, 16, 4),
               (2, 5, 4, 1, 2, 2, 0, 0, 16, 8, 8)]
    if dtype == "bf16":
        rows = [(1, 1), (2, 2), (1, 2), (2, 1)]
        zsplits = [1, 2, 3, 64]          # depth parts (64: most of them empty)
        nzs = [4, 2, 2, 4]               # adjoint depth sub-tiles per wave
        tilings = [(t[0], t[1], 0, zsplits[n], 0, nzs[n]) + rows[n] + (0, 0, 0)
                   for n, t in enumerate(tilings[:4])]
    xt = torch.from_numpy(x).to(dev)
    yt = torch.from_numpy(y).to(dev)
    for t in tilings:
        u.ufss_plan_set_tiling(plan, *t)
        info = plan.info()
        assert info["fwd_split"] == t[0] and info["adj_split"] == t[1]
        if dtype == "f32":
            assert (info["fwd_tile"], info["adj_tile"], info["fwd_zsplit"]) == (t[4], t[5], t[3])
            assert (info["fwd_chunk"], info["adj_chunk"]) == (t[8], t[9])
            # 8 waves per adjoint workgroup with 2 sub-tiles per wave only
            assert info["adj_waves"] == (t[10] if t[5] == 2 else 4)
        else:
            assert (info["fwd_rows"], info["adj_rows"], info["fwd_zsplit"], info["adj_tile"]) == \
                (t[6], t[7], t[3], t[5])
        yo = torch.empty_like(yt)
        xo = torch.empty_like(xt)
        u.ufss_forward(plan, xt, yo)
        u.ufss_adjoint(plan, yt, xo)
        torch.cuda.synchronize()
        ey, ex = errs(yo.cpu().numpy(), y_ref), errs(xo.cpu().numpy(), x_ref)
        assert max(ey) < tol and max(ex) < tol, (t, ey, ex)
    for bad in [(-1, 0, 0, 0, 0, 0), (65, 0, 0, 0, 0, 0), (0, 0, 9, 0, 0, 0), (0, 0, 0, 65, 0, 0),
                (0, 0, 0, 0, 3, 0), (0, 0, 0, 0, 0, 8), (0, 0, 0, 0, 0, 0, 3, 0), (0, 0, 0, 0, 0, 0, 0, -1),
                (0, 0, 0, 0, 0, 0, 0, 0, 4, 0), (0, 0, 0, 0, 0, 0, 0, 0, 0, 12),
                (0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 6)]:
        with pytest.raises(u.UfssError):
            u.ufss_plan_set_tiling(plan, *bad)
    plan.close()


@pytest.mark.parametrize("name,dtype", WORKLOADS)
def test_full_size_frobenius_hutchinson(name, dtype, dev):
    """Whole operator at full size, bench tiling: for x ~ CN(0, I), E||A x||^2 =
    ||A||_F^2 and likewise E||A^H y||^2 (Hutchinson), with ||A||_F^2 counted
    in closed form by the oracle.  The tolerance is four standard errors of
    the sample mean (at least 0.5%): a wrong scale, a missing block of terms
    or a dropped factor moves the mean by far more."""
    u = ufss()
    w = W.workload(name)
    g = w["geom"]
    m = w["m"]
    bins, _ = u.ufss_select_freqs(g, m, w["per_position"], w["seed"])
    fro = O.frobenius_sq(g, bins)
    plan = u.Plan(g, m, w["per_position"], bins, dtype=u.F32 if dtype == "f32" else u.BF16)
    u.ufss_plan_set_tiling(plan, **shipped_tiling(plan, g, dtype))
    gen = torch.Generator(device=dev).manual_seed(11)
    shx, shy = (g["ny"], g["nx"], g["nz"]), (g["ny"], g["nx"], m)
    ax, ahy = [], []
    yo = torch.empty(shy, dtype=torch.complex64, device=dev)
    xo = torch.empty(shx, dtype=torch.complex64, device=dev)
    n = 32
    for _ in range(n):
        x = torch.randn(shx, dtype=torch.complex64, device=dev, generator=gen)
        y = torch.randn(shy, dtype=torch.complex64, device=dev, generator=gen)
        u.ufss_forward(plan, x, yo)
        u.ufss_adjoint(plan, y, xo)
        ax.append(float((yo.abs() ** 2).sum().item()))
        ahy.append(float((xo.abs() ** 2).sum().item()))
    plan.close()
    for v in (np.array(ax), np.array(ahy)):
        tol = max(0.005, 4 * v.std(ddof=1) / np.sqrt(n) / fro)
        assert abs(v.mean() / fro - 1) < tol, (v.mean(), fro, tol)


def random_case(rng):
    """Seeded random small problem: shape, window, bins, precision and a valid tiling."""
    ny = int(rng.choice([1, 1, 2, 3, 5, 8]))
    nx = int(rng.integers(1, 33 if ny == 1 else 13))
    nz = int(rng.integers(1, 49))
    nt = int(rng.choice([64, 128, 256]))
    win = int(rng.choice([-1, 0, 1, 2, 5]))
    g = W.geometry(nx, ny, nz, nt, win_x=win, win_y=win)
    band = {64: 8, 128: 17, 256: 33}[nt]
    m = int(rng.integers(1, min(16, band) + 1))
    per_pos = bool(rng.integers(0, 2))
    dtype = "bf16" if rng.random() < 0.35 else "f32"
    t = dict(fwd_split=int(rng.integers(1, 9)), adj_split=int(rng.integers(1, 9)))
    if dtype == "f32":
        t.update(fwd_waves=int(rng.integers(1, 9)), fwd_zsplit=int(rng.integers(1, 5)),
                 fwd_tile=int(rng.choice([2, 4])), adj_tile=int(rng.choice([2, 4])),
                 fwd_chunk=int(rng.choice([8, 16])), adj_chunk=int(rng.choice([8, 16])),
                 adj_waves=int(rng.choice([4, 8])))
    else:
        t.update(fwd_zsplit=int(rng.integers(1, 5)), adj_tile=int(rng.choice([2, 4])))
        if ny > 1:
            t.update(fwd_rows=int(rng.integers(1, 3)), adj_rows=int(rng.integers(1, 3)))
    return g, m, per_pos, dtype, t


@pytest.mark.parametrize("seed", range(24))
def test_random_small_problems_against_dense_oracle(seed, dev):
    """Randomised parity sweep: every draw is checked element-wise against the
    dense FP64 oracle (FP32 1e-5, BF16 1e-2)."""
    u = ufss()
    rng = np.random.default_rng(9000 + seed)
    g, m, per_pos, dtype, t = random_case(rng)
    bins, _ = u.ufss_select_freqs(g, m, per_pos, 700 + seed)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 800 + seed).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], m), 900 + seed).astype(np.complex64)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1).astype(np.complex128)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1).astype(np.complex128)).reshape(x.shape)
    plan = u.Plan(g, m, per_pos, bins, dtype=u.F32 if dtype == "f32" else u.BF16, algo=u.ALGO_GEMM)
    try:
        u.ufss_plan_set_tiling(plan, **t)
    except u.UfssError:
        pass                     # a shape the option does not fit: default tiling
    yo = torch.empty(y.shape, dtype=torch.complex64, device=dev)
    xo = torch.empty(x.shape, dtype=torch.complex64, device=dev)
    u.ufss_forward(plan, torch.from_numpy(x).to(dev), yo)
    u.ufss_adjoint(plan, torch.from_numpy(y).to(dev), xo)
    torch.cuda.synchronize()
    tol = TOL32 if dtype == "f32" else 1e-2
    ey, ex = errs(yo.cpu().numpy(), y_ref), errs(xo.cpu().numpy(), x_ref)
    assert max(ey) < tol and max(ex) < tol, (g["nx"], g["ny"], g["nz"], g["nt"], m, per_pos, dtype, t, ey, ex)
    plan.close()


@pytest.mark.parametrize("m,waves,tile,beam", [(65, 4, 2, False), (66, 4, 2, False), (68, 4, 4, False),
                                               (66, 4, 2, True), (69, 4, 2, False), (66, 5, 2, False),
                                               (130, 4, 4, False), (132, 4, 2, True)])
def test_forward_folded_tail_bins(m, waves, tile, beam, dev):
    """FP32 forward with 1-4 bins past the last full 64-bin tile: with four
    waves those bins are folded into that tile (each wave takes the offsets
    d_x = wave mod 4, the partial sums meet in LDS); 5 bins past it (69) take
    a tile of their own, five waves (66) a tail wave.  Against the dense FP64
    oracle, with and without the beam, over several depth and d_y splits."""
    u = ufss()
    g = W.geometry(9, 5, 40, 1024, win_x=3, win_y=2)
    if beam:
        g["theta"] = float(np.radians(30.0))
    bins, _ = u.ufss_select_freqs(g, m, False, 41 + m)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 51 + m).astype(np.complex64)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1).astype(np.complex128)).reshape(g["ny"], g["nx"], m)
    plan = u.Plan(g, m, False, bins, algo=u.ALGO_GEMM)
    for fs, zs in ((1, 1), (3, 2), (2, 3)):
        u.ufss_plan_set_tiling(plan, fwd_split=fs, fwd_zsplit=zs, fwd_waves=waves, fwd_tile=tile, fwd_chunk=16)
        assert plan.info()["fwd_waves"] == waves
        yt = run_op(plan, x, (g["ny"], g["nx"], m), dev)
        torch.cuda.synchronize()
        ey = errs(yt.cpu().numpy(), y_ref)
        assert max(ey) < TOL32, (m, waves, tile, beam, fs, zs, ey)
    plan.close()


@pytest.mark.parametrize("nz,m,beam,gaps", [(200, 20, False, False), (130, 18, True, False), (16, 34, False, False),
                                            (129, 64, False, False), (129, 64, False, True), (200, 36, True, True)])
def test_adjoint_eight_waves_per_workgroup(nz, m, beam, gaps, dev):
    """FP32 adjoint with 8 waves per workgroup (one staged halo for 128
    depths): two depth workgroups with a ragged last one (200, 130, 129),
    fewer depths than one wave group covers (16), a short last bin chunk (20,
    36), the paired last 2 bins (18, 34) and whole chunks only (64), with and
    without the beam, over two d_y splits; bins in one band without gaps (the
    8-wave kernel then rotates each lane's phasor from one bin step to the
    next) or every other bin of the band (cos/sin at every step).  Against the
    dense FP64 oracle, and against 4 waves per workgroup (the same products:
    bit for bit with gaps, within the rotations' rounding without)."""
    u = ufss()
    g = W.geometry(6, 5, nz, 1024, win_x=3, win_y=2)
    if beam:
        g["theta"] = float(np.radians(30.0))
    drawn, _ = u.ufss_select_freqs(g, m, False, 61 + m)
    probe = u.Plan(g, m, False, drawn, algo=u.ALGO_GEMM)
    lo, hi = probe.info()["band_lo"], probe.info()["band_hi"]
    probe.close()
    assert hi - lo + 1 >= 2 * m
    if gaps:                                   # every other bin of the band
        bins = (lo + 2 * np.arange(m)).astype(drawn.dtype)
    else:                                      # m consecutive bins mid-band
        bins = (lo + (hi - lo + 1 - m) // 2 + np.arange(m)).astype(drawn.dtype)
    y = W.cn((g["ny"], g["nx"], m), 71 + nz).astype(np.complex64)
    A = O.dense_A(g, bins)
    x_ref = (A.conj().T @ y.reshape(-1).astype(np.complex128)).reshape(g["ny"], g["nx"], nz)
    plan = u.Plan(g, m, False, bins, algo=u.ALGO_GEMM)
    yt = torch.from_numpy(y).to(dev)
    for split in (1, 3):
        out = {}
        for aw in (4, 8):
            u.ufss_plan_set_tiling(plan, adj_split=split, adj_tile=2, adj_chunk=16, adj_waves=aw)
            assert plan.info()["adj_waves"] == aw
            xo = torch.empty((g["ny"], g["nx"], nz), dtype=torch.complex64, device=dev)
            u.ufss_adjoint(plan, yt, xo)
            torch.cuda.synchronize()
            out[aw] = xo.cpu().numpy()
            ex = errs(out[aw], x_ref)
            assert max(ex) < TOL32, (nz, m, beam, gaps, split, aw, ex)
        if gaps:
            assert np.array_equal(out[4].view(np.int32), out[8].view(np.int32)), (nz, m, beam, split)
        else:
            d = np.abs(out[8] - out[4]).max() / np.abs(out[4]).max()
            assert d < 2e-6, (nz, m, beam, split, d)
    plan.close()


@pytest.mark.parametrize("seed", range(16))
def test_random_beam_problems_against_dense_oracle(seed, dev):
    """Gaussian beam (Sec. VI directivity): random small problems with a beam
    half-angle of 5-60 degrees, every path (FP32 GEMM with a random tiling,
    phasor path for per-position bins, BF16 with phasor tables) against the
    dense FP64 oracle."""
    u = ufss()
    rng = np.random.default_rng(12000 + seed)
    g, m, per_pos, dtype, t = random_case(rng)
    g["theta"] = float(np.radians(rng.choice([5.0, 15.0, 30.0, 60.0])))
    algo = u.ALGO_PHASOR if (per_pos and dtype == "f32" and rng.random() < 0.5) else u.ALGO_AUTO
    bins, _ = u.ufss_select_freqs(g, m, per_pos, 1700 + seed)
    x = W.cn((g["ny"], g["nx"], g["nz"]), 1800 + seed).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], m), 1900 + seed).astype(np.complex64)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1).astype(np.complex128)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1).astype(np.complex128)).reshape(x.shape)
    plan = u.Plan(g, m, per_pos, bins, dtype=u.F32 if dtype == "f32" else u.BF16, algo=algo)
    if algo == u.ALGO_AUTO:
        try:
            u.ufss_plan_set_tiling(plan, **t)
        except u.UfssError:
            pass
    yo = torch.empty(y.shape, dtype=torch.complex64, device=dev)
    xo = torch.empty(x.shape, dtype=torch.complex64, device=dev)
    u.ufss_forward(plan, torch.from_numpy(x).to(dev), yo)
    u.ufss_adjoint(plan, torch.from_numpy(y).to(dev), xo)
    torch.cuda.synchronize()
    tol = TOL32 if dtype == "f32" else 1e-2
    ey, ex = errs(yo.cpu().numpy(), y_ref), errs(xo.cpu().numpy(), x_ref)
    assert max(ey) < tol and max(ex) < tol, (g, m, per_pos, dtype, algo, t, ey, ex)
    plan.close()


def test_beam_limits(dev):
    """A BF16 plan with a beam keeps its phasor tables (the in-kernel generation
    has no amplitude); batched FISTA refuses beam plans; theta outside
    [0, pi/2) is an argument error."""
    u = ufss()
    g = W.geometry(8, 6, 24, 128, win_x=3, win_y=3)
    g["theta"] = float(np.radians(20.0))
    bins, _ = u.ufss_select_freqs(g, 8, False, 3)
    pb = u.Plan(g, 8, False, bins, dtype=u.BF16)
    assert pb.info()["phasor_tables"] == 1
    with pytest.raises(u.UfssError) as e:
        u.ufss_plan_set_phasor_tables(pb, 0)
    assert e.value.name == "UNSUPPORTED"
    assert u.ufss_plan_set_phasor_tables(pb, 1) == 1
    pf = u.Plan(g, 8, False, bins)
    y = torch.zeros((6, 8, 8), dtype=torch.complex64, device=dev)
    x = torch.zeros((6, 8, 24), dtype=torch.complex64, device=dev)
    with pytest.raises(u.UfssError) as e:
        u.ufss_fista_batched([pf], [y], [x], [1.0], [1.0], 2)
    assert e.value.name == "UNSUPPORTED"
    for bad in (-0.1, float(np.pi / 2), float("nan")):
        gb = dict(g, theta=bad)
        with pytest.raises(u.UfssError) as e:
            u.Plan(gb, 8, False, bins)
        assert e.value.name == "INVALID_ARG"
    pb.close()
    pf.close()


def test_auto_picks_phasor_for_sparse_per_position_subsets(dev):
    """UFSS_ALGO_AUTO: FP32 per-position subsets whose union holds at least 5x
    one position's bins run on the phasor path (one selected bin per A-scan of
    the 50 x 50 x 50 replica), denser ones (64 of a 66-bin union) on the
    union-GEMM; the AUTO plan computes the same operator as the explicit one."""
    u = ufss()
    g = W.sim_geometry()
    g.update(nx=12, ny=10, nz=30)
    bins, per = u.ufss_sample_bins(g, 1, u.SAMPLE_RND_F, 5001)
    assert per
    auto = u.Plan(g, 1, True, bins)
    assert auto.info()["algo"] == u.ALGO_PHASOR
    gemm = u.Plan(g, 1, True, bins, algo=u.ALGO_GEMM)
    x = torch.from_numpy(W.cn((g["ny"], g["nx"], g["nz"]), 3).astype(np.complex64)).to(dev)
    ya = torch.empty((g["ny"], g["nx"], 1), dtype=torch.complex64, device=dev)
    yg = torch.empty_like(ya)
    u.ufss_forward(auto, x, ya)
    u.ufss_forward(gemm, x, yg)
    assert (torch.linalg.norm(ya - yg) / torch.linalg.norm(yg)).item() < 1e-5
    A = O.dense_A(g, bins)
    y_ref = (A @ x.cpu().numpy().reshape(-1).astype(np.complex128)).reshape(ya.shape)
    assert max(errs(ya.cpu().numpy(), y_ref)) < TOL32
    auto.close()
    gemm.close()
    w = W.workload("cscan32")
    b32, _ = u.ufss_select_freqs(w["geom"], w["m"], True, w["seed"])
    p32 = u.Plan(w["geom"], w["m"], True, b32)
    assert p32.info()["algo"] == u.ALGO_GEMM
    p32.close()


@pytest.mark.parametrize("nz,m", [(1, 1), (63, 2), (64, 3), (65, 5), (100, 17), (128, 8),
                                  (129, 33), (300, 4)])
def test_phasor_bin_groups_and_adjoint_lanes(nz, m, dev):
    """The phasor path sizes its forward bin group to the selection (1, 2, 4,
    ..., 32 bins, several groups above 32) and gives each adjoint voxel column
    64, 128 or 256 lanes (several columns per workgroup, or several depth
    chunks per column): depth counts around each boundary and bin counts
    around each group size, against the dense FP64 oracle."""
    u = ufss()
    nt = 512 if nz > 128 else 256
    g = W.geometry(5, 4, nz, nt, win_x=2, win_y=3)
    bins, _ = u.ufss_select_freqs(g, m, True, 31 + nz + m)
    x = W.cn((g["ny"], g["nx"], nz), 41 + m).astype(np.complex64)
    y = W.cn((g["ny"], g["nx"], m), 51 + nz).astype(np.complex64)
    A = O.dense_A(g, bins)
    y_ref = (A @ x.reshape(-1).astype(np.complex128)).reshape(y.shape)
    x_ref = (A.conj().T @ y.reshape(-1).astype(np.complex128)).reshape(x.shape)
    plan = u.Plan(g, m, True, bins, algo=u.ALGO_PHASOR)
    assert plan.info()["algo"] == u.ALGO_PHASOR
    yo = torch.empty(y.shape, dtype=torch.complex64, device=dev)
    xo = torch.empty(x.shape, dtype=torch.complex64, device=dev)
    u.ufss_forward(plan, torch.from_numpy(x).to(dev), yo)
    u.ufss_adjoint(plan, torch.from_numpy(y).to(dev), xo)
    torch.cuda.synchronize()
    assert max(errs(yo.cpu().numpy(), y_ref)) < TOL32
    assert max(errs(xo.cpu().numpy(), x_ref)) < TOL32
    plan.close()
