"""Kramers-Heisenberg intensity I(w_in, w) (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definition (paper Eq. ``kramers1`` with phi = O_1 Psi_int):

    I(w_in, w) = (1/pi) Im <phi| (H - E_G - w - i eta)^{-1} |phi>,

with the infinitesimal 0+ of the paper replaced by a finite broadening eta
(reading: the proportionality constant is taken as 1/pi so that I >= 0 and the
integral over w of I equals |phi|^2).

Three routes:

* ``lehmann`` -- the definition through the eigendecomposition of H:
  (1/pi) sum_n |<n|phi>|^2 eta / ((E_n - E_G - w)^2 + eta^2).
* ``continued_fraction`` -- Lanczos tridiagonalisation of H started from phi
  and the continued-fraction Green function (paper Sec. I, the route for
  linear spectra that the method reuses after all Psi_int are solved, Sec. III).
* ``correction_vector`` -- one sparse linear solve per (w_in, w) point.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def lehmann(evals: np.ndarray, evecs: np.ndarray, phi: np.ndarray, E_G: float,
            w_loss, eta: float) -> np.ndarray:
    """I[k, j] for phi[k] (rows) and losses w_loss[j] from the full spectrum of H."""
    phi = np.atleast_2d(phi)
    weights = np.abs(phi.conj() @ evecs) ** 2            # |<n|phi_k>|^2 ; evecs real
    x = evals[None, :] - E_G - np.asarray(w_loss)[:, None]   # [n_w, n_states]
    lor = eta / (x ** 2 + eta ** 2) / np.pi
    return weights @ lor.T


def lanczos_tridiag(H, phi: np.ndarray, kmax: int, b_stop: float = 0.0):
    """Hermitian Lanczos on H from phi (no reorthogonalisation).

    Returns (a, b, norm) with a_k = <q_k|H|q_k>, b_k = |w_k| for k >= 1 and
    norm = |phi| (b_0 in the moment sense).
    """
    norm = float(np.linalg.norm(phi))
    q_prev = np.zeros_like(phi)
    q = phi / norm
    a, b = [], []
    bk = 0.0
    for k in range(kmax):
        w = H @ q
        ak = float(np.real(np.vdot(q, w)))
        w = w - ak * q - bk * q_prev
        a.append(ak)
        bk = float(np.linalg.norm(w))
        if bk <= b_stop:
            break
        b.append(bk)
        q_prev, q = q, w / bk
    return np.array(a), np.array(b), norm


def cf_green(a, b, norm, z):
    """G(z) = norm^2 / (z - a_0 - b_1^2/(z - a_1 - ...)), evaluated bottom-up."""
    z = np.asarray(z, dtype=np.complex128)
    g = np.zeros_like(z)
    n = len(a)
    for k in range(n - 1, -1, -1):
        bk2 = b[k] ** 2 if k < len(b) else 0.0
        g = 1.0 / (z - a[k] - bk2 * g)
    return norm ** 2 * g


def continued_fraction(H, phi: np.ndarray, E_G: float, w_loss, eta: float,
                       tol: float = 1e-13, kmax: int = 2000, check_every: int = 10):
    """I(w) for one phi by Lanczos + continued fraction, deepened until stable.

    Stops when max_w |I_k - I_{k-check}| / max_w I_k < tol or the Lanczos
    vector vanishes.  Returns (I, depth).
    """
    z = E_G + np.asarray(w_loss) + 1j * eta
    kmax = min(kmax, H.shape[0])
    a, b, norm = lanczos_tridiag(H, phi, kmax, b_stop=1e-14 * np.linalg.norm(phi))
    prev = None
    depth = len(a)
    for k in range(check_every, len(a) + check_every, check_every):
        kk = min(k, len(a))
        I = -cf_green(a[:kk], b[:kk], norm, z).imag / np.pi
        if prev is not None and np.max(np.abs(I - prev)) <= tol * np.max(np.abs(I)):
            depth = kk
            return I, depth
        prev = I
        if kk == len(a):
            break
    return -cf_green(a, b, norm, z).imag / np.pi, depth


def correction_vector(H, phi: np.ndarray, E_G: float, w: float, eta: float) -> float:
    """I(w) = (1/pi) Im phi^H (H - E_G - w - i eta)^{-1} phi by one sparse LU solve."""
    D = H.shape[0]
    M = sp.csc_matrix(H, dtype=np.complex128) - (E_G + w + 1j * eta) * sp.identity(D, format="csc")
    x = spla.splu(M).solve(phi.astype(np.complex128))
    return float(np.imag(np.vdot(phi, x)) / np.pi)
