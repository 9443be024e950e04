"""Oracle for the learned unrolled shrinkage network (test infrastructure only).

The network unrolls the FISTA iteration of the paper (Alg. 1, Sec. IV-A) into
S stages with learned step sizes and thresholds and a small 3-D convolutional
correction; it is not in the paper, so its definition is written here:

  x_0 = x_{-1} = 0,  t_1 = 1,  t_{i+1} = (1 + sqrt(1 + 4 t_i^2)) / 2,
  beta_0 = 0, beta_i = (t_i - 1) / t_{i+1} for i >= 1  (FISTA momentum, fixed;
  stage i is FISTA iteration i + 1, so beta_0 = beta_1 = 0)
  gamma_i = x_i + beta_i (x_i - x_{i-1})
  z_i     = gamma_i - s_i A^H (A gamma_i - y),       s_i     = exp(rho_i) / L
  u_i     = soft(z_i, theta_i),                       theta_i = exp(kappa_i) lam / L
  x_{i+1} = u_i + C_i(u_i)
  C_i(u)  = c conv(W2_i, b2_i, relu(conv(W1_i, b1_i, [Re u, Im u] / c)))   (as Re + j Im)
  c       = lam / L  (the base threshold: makes the network homogeneous in y)

conv(W, b, v)[o](p) = b[o] + sum_c sum_{e in {-1,0,1}^3} W[o, c, e] v[c](p + e),
zero outside the grid, with p = (y, x, z) over the [ny][nx][nz] voxel grid
and e ordered (e_y, e_x, e_z) lexicographically (index 9 (e_y+1) + 3 (e_x+1) + e_z+1).
lam = mu max|A^H y| is computed from y and treated as a constant.  Loss:
||x_S - a_ref||^2 / ||a_ref||^2.  With rho = kappa = 0 and W2 = b2 = 0 the
network is exactly S FISTA iterations.

Parameters of one stage, flattened in this order:
  rho, kappa, W1 [ch, 2, 27], b1 [ch], W2 [2, ch, 27], b2 [2].
"""
import math

import numpy as np

from . import solver


def stage_size(ch):
    return 2 + ch * 2 * 27 + ch + 2 * ch * 27 + 2


def unpack(params, stages, ch):
    """List of per-stage dicts from the flat parameter vector."""
    params = np.asarray(params, dtype=np.float64)
    n = stage_size(ch)
    assert params.size == stages * n
    out = []
    for i in range(stages):
        p = params[i * n:(i + 1) * n]
        k = 0
        rho, kappa = p[0], p[1]
        k = 2
        W1 = p[k:k + ch * 54].reshape(ch, 2, 27)
        k += ch * 54
        b1 = p[k:k + ch]
        k += ch
        W2 = p[k:k + 2 * ch * 27].reshape(2, ch, 27)
        k += 2 * ch * 27
        b2 = p[k:k + 2]
        out.append(dict(rho=rho, kappa=kappa, W1=W1, b1=b1, W2=W2, b2=b2))
    return out


def conv3(W, b, v):
    """3x3x3 convolution with zero padding. v: [cin, ny, nx, nz] -> [cout, ...]."""
    cout = W.shape[0]
    ny, nx, nz = v.shape[1:]
    pad = np.zeros((v.shape[0], ny + 2, nx + 2, nz + 2))
    pad[:, 1:-1, 1:-1, 1:-1] = v
    out = np.zeros((cout, ny, nx, nz)) + np.asarray(b)[:, None, None, None]
    for ey in (-1, 0, 1):
        for ex in (-1, 0, 1):
            for ez in (-1, 0, 1):
                e = 9 * (ey + 1) + 3 * (ex + 1) + (ez + 1)
                sh = pad[:, 1 + ey:1 + ey + ny, 1 + ex:1 + ex + nx, 1 + ez:1 + ez + nz]
                out += np.tensordot(W[:, :, e], sh, axes=([1], [0]))
    return out


def correction(st, u, c):
    """C_i(u) for complex u of shape [ny, nx, nz] and scale c."""
    v = np.stack([u.real, u.imag]) / c
    h = np.maximum(conv3(st["W1"], st["b1"], v), 0.0)
    o = c * conv3(st["W2"], st["b2"], h)
    return o[0] + 1j * o[1]


def forward(A, AH, y, params, stages, ch, L, mu, shape, return_all=False):
    """x_S of the unrolled network (complex128, shape [ny, nx, nz])."""
    sts = unpack(params, stages, ch)
    lam = solver.lambda_rule(AH, y, mu)
    x = np.zeros(shape, dtype=np.complex128)
    x_prev = x.copy()
    t = 1.0
    trace = []
    for i, st in enumerate(sts):
        beta = 0.0
        if i > 0:
            t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
            beta = (t - 1.0) / t_new
            t = t_new
        gam = x + beta * (x - x_prev)
        g = AH(A(gam.reshape(-1)) - y).reshape(shape)
        z = gam - (math.exp(st["rho"]) / L) * g
        u = solver.soft(z, math.exp(st["kappa"]) * lam / L)
        x_prev, x = x, u + correction(st, u, lam / L)
        trace.append(x)
    return (x, trace) if return_all else x


def loss(A, AH, y, params, stages, ch, L, mu, shape, a_ref):
    x = forward(A, AH, y, params, stages, ch, L, mu, shape)
    d = x - a_ref
    return float(np.vdot(d, d).real / np.vdot(a_ref, a_ref).real)


def fd_grad(A, AH, y, params, stages, ch, L, mu, shape, a_ref, idx, h=1e-6):
    """Central finite differences of the loss for the parameter indices idx."""
    params = np.asarray(params, dtype=np.float64)
    out = []
    for i in idx:
        p1 = params.copy()
        p2 = params.copy()
        p1[i] += h
        p2[i] -= h
        out.append((loss(A, AH, y, p1, stages, ch, L, mu, shape, a_ref)
                    - loss(A, AH, y, p2, stages, ch, L, mu, shape, a_ref)) / (2 * h))
    return np.array(out)
