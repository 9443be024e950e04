"""GPU checks on the simulated specimen of Sec. VII (50 x 50 x 50, Table III):
operator parity with the oracle on sampled outputs under each sampling
strategy, and the depth-localisation contrast between shared and per-position
subsets at one coefficient per A-scan."""
import numpy as np
import pytest

from oracle import operator as O
from paper_2012_04534_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("strategy,nf,algo", [("max", 10, "ALGO_AUTO"), ("nrg", 5, "ALGO_AUTO"),
                                              ("nrg_f", 1, "ALGO_AUTO"), ("nrg_f", 1, "ALGO_PHASOR"),
                                              ("rnd_f", 10, "ALGO_AUTO")])
def test_sim50_operator_sampled_parity(strategy, nf, algo, dev):
    from paper_2012_04534_amd import ufss as u
    from paper_2012_04534_amd import replica as R
    g = W.sim_geometry()
    bins, per = u.ufss_sample_bins(g, nf, R.STRATEGIES[strategy], 5001)
    plan = u.Plan(g, nf, per, bins, algo=getattr(u, algo))
    x = W.sim_rectangle(g) + 0.3 * W.cn((g["ny"], g["nx"], g["nz"]), 4)
    y = W.cn((g["ny"], g["nx"], nf), 5)
    xt = torch.from_numpy(x.astype(np.complex64)).to(dev)
    yt = torch.from_numpy(y.astype(np.complex64)).to(dev)
    yo = torch.empty_like(yt)
    xo = torch.empty_like(xt)
    u.ufss_forward(plan, xt, yo)
    u.ufss_adjoint(plan, yt, xo)
    yo, xo = yo.cpu().numpy(), xo.cpu().numpy()
    xq = x.astype(np.complex64).astype(np.complex128)
    yq = y.astype(np.complex64).astype(np.complex128)
    pts = [(0, 0), (0, 49), (49, 0), (25, 25), (49, 49), (13, 37)]
    ref = np.array([O.apply_A_at(g, bins, xq, py, px) for py, px in pts])
    got = np.array([yo[py, px] for py, px in pts])
    assert np.abs(got - ref).max() <= TOL32 * np.abs(ref).max()
    refc = np.array([O.apply_AH_at(g, bins, yq, vy, vx) for vy, vx in pts])
    gotc = np.array([xo[vy, vx] for vy, vx in pts])
    assert np.abs(gotc - refc).max() <= TOL32 * np.abs(refc).max()
    plan.close()


def test_sim50_per_position_subsets_restore_depth(dev):
    """One coefficient per A-scan, line defect, mu = 0.1, 80 iterations: a
    shared subset localises the depth in few columns, distinct subsets per
    position in nearly all (Sec. VII, first scenario)."""
    from paper_2012_04534_amd import replica as R
    g = W.sim_geometry()
    xt = W.sim_line(g)
    shared = R.run(g, "line", xt, "max", 1, 0.1, W.SIM_ITERS, 5001, dev)
    per = R.run(g, "line", xt, "rnd_f", 1, 0.1, W.SIM_ITERS, 5001, dev)
    assert shared["depth_hit"] <= 0.5
    assert per["depth_hit"] >= 0.9
    assert per["corr"] > shared["corr"]
