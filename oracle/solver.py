"""Oracle sparse-recovery solvers (test infrastructure only).

Problem (Sec. IV-A, l1 relaxation, taken in its penalised LASSO form):

    F(a) = 1/2 ||A a - y||_2^2 + lam ||a||_1,   lam = mu ||A^H y||_inf  (Sec. VII).

FISTA follows Algorithm 1 (Sec. IV-A) with these readings of its garbles:
  * step: the printed "2 s beta(.)" with s = 1/sigma_max^2 is the step for
    ||.||^2; on the 1/2 ||.||^2 objective the step is 1/L, L = sigma_max^2;
  * threshold lam / L;
  * momentum is applied to the newest iterate (Beck & Teboulle 2009):
    gamma_{k+1} = a_k + ((t_k - 1) / t_{k+1}) (a_k - a_{k-1});
  * the complex soft threshold is z max(0, 1 - alpha/|z|) (sgn z = z/|z|, 0 at 0).
ISTA is the same iteration with gamma_{k+1} = a_k.

With this reading a = 0 is optimal exactly when mu >= 1, matching the lambda rule.

The Lipschitz constant L = sigma_max(A)^2 (Sec. IV-C) is computed exactly with
``numpy.linalg.eigvalsh`` on a dense A, or by power iteration on A^H A (the
paper uses ARPACK; it warns that under-estimates make FISTA diverge).
"""
import math

import numpy as np


def soft(z, alpha):
    """Complex soft threshold z * max(0, 1 - alpha/|z|), with soft(0) = 0."""
    z = np.asarray(z, dtype=np.complex128)
    mag = np.abs(z)
    scale = np.where(mag > alpha, 1.0 - alpha / np.where(mag > 0, mag, 1.0), 0.0)
    return z * scale


def objective(A, y, a, lam):
    r = A(a) - y
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.abs(a).sum())


def lambda_rule(AH, y, mu):
    """lam = mu * ||A^H y||_inf (Sec. VII)."""
    return mu * float(np.abs(AH(y)).max())


def momentum_weights(iters, t1=1.0):
    """t_k and beta_k = (t_k - 1)/t_{k+1} for k = 1..iters (t_1 = 1)."""
    t = [t1]
    for _ in range(iters):
        t.append((1.0 + math.sqrt(1.0 + 4.0 * t[-1] * t[-1])) / 2.0)
    beta = [(t[i] - 1.0) / t[i + 1] for i in range(iters)]
    return t, beta


def fista(A, AH, y, lam, L, iters, a0=None, accel=True, a_ref=None, state=None, real=False):
    """Run ``iters`` FISTA (or ISTA) iterations in complex128.

    A, AH    callables for x -> A x and y -> A^H y
    a0       start value (zeros if None)
    state    optional dict {"a", "gamma", "t", "k"} to resume; updated on return
    real     reconstruct a real reflectivity (the Re{H} comparison of Sec. VII):
             the gradient with respect to a real a is Re(A^H r), so the step
             keeps the real part before the threshold and every iterate is real
    Returns (a_K, stats) where stats holds, per iteration k, the objective at
    gamma_k, ||A gamma_k - y||, ||a_k - a_{k-1}|| / ||a_k|| and, if a_ref is
    given, ||a_k - a_ref|| / ||a_ref||.
    """
    y = np.asarray(y, dtype=np.complex128)
    if state is not None and state.get("k", 0) > 0:
        a = np.array(state["a"], dtype=np.complex128)
        gamma = np.array(state["gamma"], dtype=np.complex128)
        t = float(state["t"])
        k0 = int(state["k"])
    else:
        shape = AH(y).shape if a0 is None else np.shape(a0)
        a = np.zeros(shape, np.complex128) if a0 is None else np.array(a0, np.complex128)
        gamma = a.copy()
        t, k0 = 1.0, 0
    ref_norm = None if a_ref is None else float(np.linalg.norm(a_ref))
    stats = {"obj": [], "res": [], "rel_change": [], "err_ref": []}
    for _ in range(iters):
        r = A(gamma) - y
        res = float(np.linalg.norm(r))
        stats["obj"].append(0.5 * res * res + lam * float(np.abs(gamma).sum()))
        grad = AH(r)
        z = gamma - grad / L
        a_new = soft(z.real if real else z, lam / L).astype(np.complex128)
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        if accel:
            gamma = a_new + ((t - 1.0) / t_new) * (a_new - a)
        else:
            gamma = a_new
        stats["res"].append(res)
        nrm = float(np.linalg.norm(a_new))
        stats["rel_change"].append(float(np.linalg.norm(a_new - a)) / nrm if nrm > 0 else 0.0)
        if a_ref is not None:
            stats["err_ref"].append(float(np.linalg.norm(a_new - a_ref)) / ref_norm)
        a, t = a_new, t_new
    if state is not None:
        state.update({"a": a.copy(), "gamma": gamma.copy(), "t": t, "k": k0 + iters})
    return a, stats


def lipschitz_dense(Amat):
    """L = lambda_max(A^H A) by a dense Hermitian eigensolver.

    A^H A and A A^H share their non-zero eigenvalues, so the smaller Gram
    matrix is decomposed.
    """
    G = Amat.conj().T @ Amat if Amat.shape[1] <= Amat.shape[0] else Amat @ Amat.conj().T
    return float(np.linalg.eigvalsh(G)[-1])


def power_iteration(A, AH, v0, max_iters=200, rtol=1e-6):
    """Rayleigh quotient rho = ||A v||^2/||v||^2 of A^H A by power iteration.

    Returns (rho, iterations used).  rho never exceeds lambda_max(A^H A).
    """
    v = np.array(v0, dtype=np.complex128)
    v /= np.linalg.norm(v)
    rho_old = 0.0
    for it in range(1, max_iters + 1):
        Av = A(v)
        rho = float(np.vdot(Av, Av).real)
        w = AH(Av)
        v = w / np.linalg.norm(w)
        if rho_old > 0 and abs(rho - rho_old) <= rtol * rho:
            return rho, it
        rho_old = rho
    return rho, max_iters


def fista_backtracking(A, AH, y, lam, L0, eta, iters, a0=None, a_ref=None, slack=0.0,
                       max_trials=200):
    """FISTA with backtracking (Sec. IV-C, backtracking; Beck & Teboulle 2009).

    Needs only a lower start value L0 and a growth factor eta > 1.  At the
    extrapolated point gamma_k, trial constants L = L_{k-1} eta^i (i = 0, 1,
    ...) are tried in turn: p = soft(gamma - grad f(gamma) / L, lam / L) is
    accepted as soon as

        f(p) <= f(gamma) + Re<p - gamma, grad f(gamma)> + L/2 ||p - gamma||^2 (+ slack),

    with f = 1/2 ||A . - y||^2 (the l1 terms of F and of its quadratic model
    cancel).  ``slack`` (default 0) is an absolute margin for rounding.  The
    momentum is that of plain FISTA.
    Returns (a_K, stats): per iteration the objective F(a_k), ||A a_k - y||,
    ||a_k - a_{k-1}|| / ||a_k||, the accepted L_k, the trial count and, if
    a_ref is given, ||a_k - a_ref|| / ||a_ref||.
    """
    if not (eta > 1.0) or not (L0 > 0.0):
        raise ValueError("need L0 > 0 and eta > 1")
    y = np.asarray(y, dtype=np.complex128)
    shape = AH(y).shape if a0 is None else np.shape(a0)
    a = np.zeros(shape, np.complex128) if a0 is None else np.array(a0, np.complex128)
    gamma = a.copy()
    t, L = 1.0, float(L0)
    ref_norm = None if a_ref is None else float(np.linalg.norm(a_ref))
    stats = {"obj": [], "res": [], "rel_change": [], "L": [], "trials": [], "err_ref": []}
    for _ in range(iters):
        r = A(gamma) - y
        f_gamma = 0.5 * float(np.vdot(r, r).real)
        grad = AH(r)
        trials = 0
        while True:
            trials += 1
            if trials > max_trials:
                raise RuntimeError("backtracking did not terminate")
            p = soft(gamma - grad / L, lam / L)
            rp = A(p) - y
            f_p = 0.5 * float(np.vdot(rp, rp).real)
            d = p - gamma
            model = f_gamma + float(np.vdot(d, grad).real) + 0.5 * L * float(np.vdot(d, d).real)
            if f_p <= model + slack:
                break
            L *= eta
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        gamma = p + ((t - 1.0) / t_new) * (p - a)
        nrm = float(np.linalg.norm(p))
        stats["obj"].append(f_p + lam * float(np.abs(p).sum()))
        stats["res"].append(math.sqrt(2.0 * f_p))
        stats["rel_change"].append(float(np.linalg.norm(p - a)) / nrm if nrm > 0 else 0.0)
        stats["L"].append(L)
        stats["trials"].append(trials)
        if a_ref is not None:
            stats["err_ref"].append(float(np.linalg.norm(p - a_ref)) / ref_norm)
        a, t = p, t_new
    return a, stats
