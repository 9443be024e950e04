"""GPU check of ufss_shrink_update_noalloc (the fused update of Alg. 1 without
device allocation) against ufss_shrink_update: identical iterates and FP64
norms, bit for bit, on two calls in a row -- the second with a smaller input,
so stale partials of the first call in the shared scratch array would show."""
import numpy as np
import pytest

from oracle import solver as V
from paper_2012_04534_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _inputs(n, seed):
    gam = W.cn(n, seed).astype(np.complex64)
    g = W.cn(n, seed + 1).astype(np.complex64)
    a = W.cn(n, seed + 2).astype(np.complex64)
    aref = W.cn(n, seed + 3).astype(np.complex64)
    gam[:7] = 0
    g[:7] = 0
    return gam, g, a, aref


@pytest.mark.parametrize("sizes", [(1 << 20, 4099), (300001, 1)])
def test_noalloc_update_equals_allocating_update(dev, sizes):
    from paper_2012_04534_amd import ufss
    step, thr, beta = 0.3, 0.45, 0.6
    for call, n in enumerate(sizes):
        gam, g, a, aref = _inputs(n, 11 + 10 * call)
        use_ref = call == 0
        # allocating entry point
        g1, gg1, a1 = to_dev(gam, dev), to_dev(g, dev), to_dev(a, dev)
        r1 = to_dev(aref, dev) if use_ref else None
        want = ufss.ufss_shrink_update(g1, gg1, a1, step, thr, beta, a_ref=r1)
        # allocation-free entry point on copies of the same inputs
        g2, gg2, a2 = to_dev(gam, dev), to_dev(g, dev), to_dev(a, dev)
        r2 = to_dev(aref, dev) if use_ref else None
        got = ufss.ufss_shrink_update_noalloc(g2, gg2, a2, step, thr, beta, a_ref=r2)
        torch.cuda.synchronize()
        assert np.array_equal(got, want), (call, n, got, want)
        assert torch.equal(a2, a1) and torch.equal(g2, g1), (call, n)
        # and both against the oracle's soft threshold (FP32 bar)
        a_new = V.soft(gam.astype(np.complex128) - step * g.astype(np.complex128), thr)
        an = a2.cpu().numpy()
        assert np.abs(an - a_new).max() <= 1e-6 * max(np.abs(a_new).max(), 1e-30)
        np.testing.assert_allclose(got[3], np.sum(np.abs(a_new) ** 2), rtol=1e-6)
        if not use_ref:
            assert got[4] == 0.0


def test_noalloc_without_norms_then_with(dev):
    from paper_2012_04534_amd import ufss
    n = 70000
    gam, g, a, _ = _inputs(n, 41)
    g1, gg1, a1 = to_dev(gam, dev), to_dev(g, dev), to_dev(a, dev)
    assert ufss.ufss_shrink_update_noalloc(g1, gg1, a1, 0.5, 0.2, 0.0, want_norms=False) is None
    torch.cuda.synchronize()
    g2, gg2, a2 = to_dev(gam, dev), to_dev(g, dev), to_dev(a, dev)
    want = ufss.ufss_shrink_update(g2, gg2, a2, 0.5, 0.2, 0.0)
    assert torch.equal(a1, a2) and torch.equal(g1, g2)
    # a second call on the updated state still reduces only its own partials
    got = ufss.ufss_shrink_update_noalloc(g1, gg1, a1, 0.5, 0.2, 0.0)
    want2 = ufss.ufss_shrink_update(g2, gg2, a2, 0.5, 0.2, 0.0)
    assert np.array_equal(got, want2)
    assert not np.array_equal(want, want2)


def test_noalloc_argument_errors(dev):
    from paper_2012_04534_amd import ufss
    import ctypes
    lib = ufss.lib()
    code = lib.ufss_shrink_update_noalloc(-1, None, None, None, 1.0, 0.0, 0.0, None, None, None)
    assert code == -1
    code = lib.ufss_shrink_update_noalloc(5, None, None, None, 1.0, 0.0, 0.0, None, None, None)
    assert code == -1
    assert b"NULL" in lib.ufss_last_error()
    # n = 0 is accepted and leaves every norm at zero
    z = torch.zeros(1, dtype=torch.complex64, device=dev)
    out = np.ones(5)
    code = lib.ufss_shrink_update_noalloc(0, ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                          ctypes.c_void_p(z.data_ptr()), 1.0, 0.0, 0.0, None,
                                          out.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == 0 and np.all(out == 0.0)
