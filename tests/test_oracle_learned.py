"""Pins of the oracle's unrolled network (CPU only)."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import learned as N
from oracle import operator as O
from oracle import select as S
from oracle import solver as V
from paper_2012_04534_amd import workloads as W


def tiny_problem():
    g = W.geometry(6, 5, 12, 64, win_x=2, win_y=2)
    bins = S.select_freqs(g, 5, True, 3)
    Amat = O.dense_A(g, bins)
    x_true = W.scene(g, 4, amp=(0.5, 1.0), seed=2)
    y = Amat @ x_true.reshape(-1) + 0.05 * W.cn(Amat.shape[0], 3)
    A = lambda v: Amat @ v
    AH = lambda v: Amat.conj().T @ v
    L = V.lipschitz_dense(Amat) * 1.01
    return g, Amat, A, AH, y, L


def init_params(stages, ch, seed=0):
    rng = np.random.default_rng(seed)
    ps = []
    for _ in range(stages):
        p = np.zeros(N.stage_size(ch))
        p[2:2 + ch * 54] = 0.1 * rng.standard_normal(ch * 54)     # W1
        ps.append(p)
    return np.concatenate(ps)


def test_zero_correction_is_fista():
    """P14: rho = kappa = 0 and W2 = b2 = 0 -> S plain FISTA iterations."""
    g, Amat, A, AH, y, L = tiny_problem()
    shape = (g["ny"], g["nx"], g["nz"])
    p = init_params(5, 3)
    x = N.forward(A, AH, y, p, 5, 3, L, 0.1, shape)
    lam = V.lambda_rule(AH, y, 0.1)
    a, _ = V.fista(A, AH, y, lam, L, 5)
    np.testing.assert_allclose(x.reshape(-1), a, rtol=0, atol=1e-13 * np.abs(a).max())


def test_conv_matches_scipy_correlate():
    """The 3x3x3 convolution is scipy.ndimage.correlate with zero padding."""
    rng = np.random.default_rng(1)
    v = rng.standard_normal((2, 4, 5, 6))
    W1 = rng.standard_normal((3, 2, 27))
    b = rng.standard_normal(3)
    out = N.conv3(W1, b, v)
    for o in range(3):
        ref = np.full(v.shape[1:], b[o])
        for c in range(2):
            ref += ndimage.correlate(v[c], W1[o, c].reshape(3, 3, 3), mode="constant", cval=0.0)
        np.testing.assert_allclose(out[o], ref, rtol=1e-12, atol=1e-12)


def test_fd_matches_closed_form_bias_derivative():
    """For one stage, d loss / d b2 = 2 c sum (x - a_ref) / ||a_ref||^2 over each
    real channel, c = lam / L (x_1 depends on b2 as the shift c b2)."""
    g, Amat, A, AH, y, L = tiny_problem()
    shape = (g["ny"], g["nx"], g["nz"])
    ch = 2
    p = init_params(1, ch, 4)
    a_ref = W.cn(shape, 9)
    x = N.forward(A, AH, y, p, 1, ch, L, 0.1, shape)
    r2 = float(np.vdot(a_ref, a_ref).real)
    c = V.lambda_rule(AH, y, 0.1) / L
    want = [2 * c * float((x - a_ref).real.sum()) / r2, 2 * c * float((x - a_ref).imag.sum()) / r2]
    n = N.stage_size(ch)
    got = N.fd_grad(A, AH, y, p, 1, ch, L, 0.1, shape, a_ref, [n - 2, n - 1], h=1e-2)
    np.testing.assert_allclose(got, want, rtol=1e-6)


def test_fd_kappa_matches_soft_threshold_derivative():
    """d loss / d kappa for one stage with no correction equals
    sum <2(x - a_ref), -theta z/|z|> / ||a_ref||^2 over |z| > theta."""
    g, Amat, A, AH, y, L = tiny_problem()
    shape = (g["ny"], g["nx"], g["nz"])
    ch = 1
    p = np.zeros(N.stage_size(ch))
    a_ref = W.cn(shape, 5)
    lam = V.lambda_rule(AH, y, 0.1)
    z = -(1.0 / L) * AH(-y).reshape(shape)
    theta = lam / L
    x = V.soft(z, theta)
    on = np.abs(z) > theta
    d = (x - a_ref)[on]
    want = float(np.sum(2 * (d.real * (-theta * z[on].real / np.abs(z[on]))
                             + d.imag * (-theta * z[on].imag / np.abs(z[on])))))
    want /= float(np.vdot(a_ref, a_ref).real)
    got = N.fd_grad(A, AH, y, p, 1, ch, L, 0.1, shape, a_ref, [1])[0]
    assert got == pytest.approx(want, rel=1e-5)


def test_network_is_homogeneous_in_y():
    """With the correction scaled by c = lam / L the network commutes with a
    positive scaling of the measurements (all parameters non-zero)."""
    g, Amat, A, AH, y, L = tiny_problem()
    shape = (g["ny"], g["nx"], g["nz"])
    rng = np.random.default_rng(3)
    p = 0.1 * rng.standard_normal(3 * N.stage_size(2))
    x1 = N.forward(A, AH, y, p, 3, 2, L, 0.1, shape)
    x2 = N.forward(A, AH, 7.5 * y, p, 3, 2, L, 0.1, shape)
    np.testing.assert_allclose(x2, 7.5 * x1, rtol=0, atol=1e-12 * np.abs(x2).max())
