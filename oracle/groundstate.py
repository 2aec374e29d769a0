"""Ground state (E_G, |G>) of the Hubbard Hamiltonian (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper obtains the ground state with an Arnoldi solver (Sec. III, text after
Eq. ``Hubbard``).  For a real symmetric H the lowest eigenpair is what is
needed; the oracle computes it

* exactly, by dense symmetric diagonalisation (``numpy.linalg.eigh``), for
  small sectors; or
* by Lanczos with full reorthogonalisation from a caller-supplied start
  vector, with the tridiagonal eigenproblem solved by ``numpy.linalg.eigh``.

Pinned by: the U = 0 closed form, the two-site closed form, agreement of the
two routes, and the eigen-residual ||H G - E_G G||.
"""
from __future__ import annotations

import numpy as np


def dense_ground_state(H):
    """Lowest eigenpair of a (small) real symmetric matrix by dense eigh."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    w, V = np.linalg.eigh(Hd)
    return float(w[0]), V[:, 0].copy(), w


def lanczos_ground_state(H, v0: np.ndarray, tol: float = 1e-13, maxit: int = 500):
    """Lowest eigenpair by Lanczos with full reorthogonalisation.

    Builds an orthonormal Krylov basis q_0 = v0/|v0|, q_{k+1} ~ H q_k minus its
    projections on all previous q (Gram-Schmidt applied twice), forms the
    tridiagonal T_k = Q^T H Q and stops when the lowest Ritz pair's residual
    estimate |b_{k+1} y_k| falls below tol * |theta|.  Returns (E_G, G, iters).
    """
    D = v0.shape[0]
    Q = np.zeros((min(maxit + 1, D) + 1, D))
    q = v0 / np.linalg.norm(v0)
    Q[0] = q
    a, b = [], []
    theta, y = None, None
    k = 0
    for k in range(min(maxit, D)):
        w = H @ Q[k]
        a.append(float(Q[k] @ w))
        for _ in range(2):
            w -= Q[: k + 1].T @ (Q[: k + 1] @ w)
        beta = float(np.linalg.norm(w))
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        evals, evecs = np.linalg.eigh(T)
        theta, y = evals[0], evecs[:, 0]
        if abs(beta * y[-1]) <= tol * abs(theta) or beta < 1e-300:
            break
        b.append(beta)
        Q[k + 1] = w / beta
    G = Q[: len(a)].T @ y
    G /= np.linalg.norm(G)
    return float(theta), G, k + 1


def ground_state(H, v0=None, tol: float = 1e-13, maxit: int = 500, dense_max: int = 5000):
    """(E_G, G): dense eigh when dim <= dense_max, else Lanczos from v0."""
    D = H.shape[0]
    if D <= dense_max:
        E, G, _ = dense_ground_state(H)
        return E, G
    if v0 is None:
        raise ValueError("Lanczos route needs a start vector")
    E, G, _ = lanczos_ground_state(H, v0, tol, maxit)
    return E, G
