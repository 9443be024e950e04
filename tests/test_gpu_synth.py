"""GPU checks of the device-side synthetic data (ufss_synth_scene,
ufss_synth_measure) against the host mirror of the same counter-based
generator: scenes equal bit for bit, measurements equal A x (the library's own
forward) plus the mirror's noise at the SNR scale, to FP32 rounding."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("case", [(32, 32, 256, 20, 232, 240, 1), (9, 7, 40, 25, 30, 35, 2),
                                  (2, 2, 3, 12, 3, None, 3), (16, 1, 64, 0, 64, None, 4),
                                  (5, 4, 20, 1, 1, 10, 5)])
def test_scene_equals_host_mirror(case, dev):
    nx, ny, nz, n, max_depth, wall, seed = case
    u = ufss()
    g = W.geometry(nx, ny, nz, 128)
    x = torch.full((ny, nx, nz), complex(7.0, 7.0), dtype=torch.complex64, device=dev)
    u.ufss_synth_scene(g, n, (0.5, 1.0), max_depth, wall, seed, x)
    want = W.synth_scene(g, n, (0.5, 1.0), max_depth, wall, seed).astype(np.complex64)
    assert np.array_equal(x.cpu().numpy(), want)


@pytest.mark.parametrize("snr", [10.0, 20.0])
def test_measurements_equal_forward_plus_mirror_noise(snr, dev):
    u = ufss()
    w = W.workload("cscan32")
    g = dict(w["geom"])
    g.update(nx=12, ny=10, nz=64, nt=128)
    bins, _ = u.ufss_select_freqs(g, 9, True, 4)
    plan = u.Plan(g, 9, True, bins, algo=u.ALGO_GEMM)
    x = torch.empty((10, 12, 64), dtype=torch.complex64, device=dev)
    u.ufss_synth_scene(g, 7, (0.5, 1.0), 56, 60, 21, x)
    y = torch.empty((10, 12, 9), dtype=torch.complex64, device=dev)
    u.ufss_synth_measure(plan, x, snr, 99, y)
    y0 = torch.empty_like(y)
    u.ufss_forward(plan, x, y0)
    a = y0.cpu().numpy().astype(np.complex128)
    e2 = float(np.sum(np.abs(a) ** 2))
    s = np.sqrt(e2 / (a.size * 10.0 ** (snr / 10.0)))
    want = a + s * W.synth_noise(a.size, 99).reshape(a.shape)
    got = y.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()
    # the realised SNR is the requested one (to the sampling spread of 1080 values)
    n = got - a
    snr_real = 10 * np.log10(e2 / np.sum(np.abs(n) ** 2))
    assert abs(snr_real - snr) < 0.5
    # noise free
    u.ufss_synth_measure(plan, x, float("inf"), 99, y)
    assert torch.equal(y, y0)
    plan.close()


def test_synth_argument_errors(dev):
    u = ufss()
    g = W.geometry(4, 3, 10, 64)
    x = torch.empty((3, 4, 10), dtype=torch.complex64, device=dev)
    for args in [(5, (0.5, 1.0), 11, None), (5, (0.5, 1.0), 0, None), (5, (1.0, 0.5), 5, None),
                 (121, (0.5, 1.0), 10, None), (5, (0.5, 1.0), 5, 10), (-1, (0.5, 1.0), 5, None)]:
        with pytest.raises(u.UfssError) as e:
            u.ufss_synth_scene(g, args[0], args[1], args[2], args[3], 1, x)
        assert e.value.name == "INVALID_ARG"
