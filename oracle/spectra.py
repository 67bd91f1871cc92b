"""Eigen-solvers of the oracle (test infrastructure, FP64).

* ``dense_lowest``: LAPACK ``eigh`` of the dense sector matrix (the paper uses
  LAPACK for small sectors, Sec. 6 "Diagonalization").
* ``lanczos_full_reorth``: Lanczos (Sec. 6 "Diagonalization") with full
  re-orthogonalisation against the stored basis, so that it converges to the
  exact lowest eigenvalue with no ghost copies; returns the eigenvector too.
* ``arpack_lowest``: SciPy ``eigsh`` (ARPACK), an independent cross-check.
* ``plain_lanczos``: the plain three-term recurrence without
  re-orthogonalisation, as the paper runs it, returning the recurrence
  coefficients (used for the Krylov Green's function).
* ``tridiag_eigh``: eigenpairs of the symmetric tridiagonal matrix.

Breakdown rule (the paper is silent): the recurrence stops when
beta_{j+1} <= 1e-12 * max_i(|alpha_i| + beta_i + beta_{i+1}) so far.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

BREAKDOWN_REL = 1e-12


def dense_lowest(H, k=1):
    A = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    w, V = np.linalg.eigh(A)
    return w[:k], V[:, :k]


def tridiag_eigh(alpha, beta):
    """alpha[0..m-1] diagonal, beta[0..m-2] off-diagonal."""
    alpha = np.asarray(alpha, float)
    beta = np.asarray(beta, float)
    if alpha.size == 1:
        return alpha.copy(), np.ones((1, 1))
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    return np.linalg.eigh(T)


def lanczos_full_reorth(matvec, v0, maxiter=300, tol=1e-13):
    """Lowest eigenpair by Lanczos with two passes of full Gram-Schmidt per step.
    Converged when the residual bound beta_{m} |y_m| <= tol * max(1, |E|)."""
    v = np.asarray(v0, float)
    v = v / np.linalg.norm(v)
    Q = [v]
    alpha, beta = [], []
    E = None
    y = None
    for j in range(maxiter):
        w = matvec(Q[j])
        a = float(Q[j] @ w)
        alpha.append(a)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[-1] * Q[j - 1]
        Qm = np.array(Q)
        for _ in range(2):
            w = w - Qm.T @ (Qm @ w)
        b = float(np.linalg.norm(w))
        th, U = tridiag_eigh(alpha, beta)
        E, y = th[0], U[:, 0]
        tnorm = max(abs(x) for x in alpha) + (max(beta) if beta else 0.0) + b
        if b * abs(y[-1]) <= tol * max(1.0, abs(E)) or b <= BREAKDOWN_REL * tnorm:
            break
        beta.append(b)
        Q.append(w / b)
    psi = np.array(Q[: len(alpha)]).T @ y
    psi /= np.linalg.norm(psi)
    return E, psi, len(alpha)


def arpack_lowest(H, tol=1e-14):
    w, V = spla.eigsh(H, k=1, which="SA", tol=tol)
    return float(w[0]), V[:, 0]


def plain_lanczos(matvec, v0, nsteps):
    """Plain Lanczos from v0/|v0| (no re-orthogonalisation).

    Returns (alpha[m], beta[m-1]) with m <= nsteps; stops early on breakdown."""
    v = np.asarray(v0, float)
    v = v / np.linalg.norm(v)
    vprev = np.zeros_like(v)
    alpha, beta = [], []
    bprev = 0.0
    tnorm = 0.0
    for j in range(nsteps):
        w = matvec(v)
        a = float(v @ w)
        alpha.append(a)
        w = w - a * v - bprev * vprev
        b = float(np.linalg.norm(w))
        tnorm = max(tnorm, abs(a) + bprev + b)
        if j == nsteps - 1 or b <= BREAKDOWN_REL * tnorm:
            break
        beta.append(b)
        vprev, v = v, w / b
        bprev = b
    return np.array(alpha), np.array(beta)


def lanczos_ground_energy_plain(matvec, v0, niter, tol):
    """Plain Lanczos ground energy with the stop rule |E_j - E_{j-1}| <=
    tol * max(1, |E_j|), breakdown, or niter steps.  Returns (E, steps)."""
    v = np.asarray(v0, float)
    v = v / np.linalg.norm(v)
    vprev = np.zeros_like(v)
    alpha, beta = [], []
    bprev, tnorm, Eold = 0.0, 0.0, None
    for j in range(niter):
        w = matvec(v)
        a = float(v @ w)
        alpha.append(a)
        w = w - a * v - bprev * vprev
        b = float(np.linalg.norm(w))
        tnorm = max(tnorm, abs(a) + bprev + b)
        E = tridiag_eigh(alpha, beta)[0][0]
        if Eold is not None and abs(E - Eold) <= tol * max(1.0, abs(E)):
            return E, j + 1
        if b <= BREAKDOWN_REL * tnorm:
            return E, j + 1
        Eold = E
        beta.append(b)
        vprev, v = v, w / b
        bprev = b
    return E, niter
