"""Intermediate states Psi_int(w_in) (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Problem (paper Eq. ``intermediateState`` and its shifted form, Appendix A,
Eq. ``shifted_linear_eq``):

    (A - w_in I) Psi(w_in) = E,   A = H' - E_G - i Gamma,   E = O_2 |G>.

Two independent routes:

* ``direct_solve`` -- the definition: one linear solve per shift (dense LU,
  eigendecomposition, or sparse LU).
* ``msbicg_reference`` -- the multi-shift complex-symmetric BiCG recurrence of
  Appendix D (Algorithm 1) with the readings stated below, written step by
  step in the paper's order and notation, vectorised over shifts only.

Readings of the printed algorithm (each verified against ``direct_solve`` by
``tests/test_oracle_solve.py``):

1. zeta recurrence sign.  Appendix C derives zeta_m(w) = P_m(w) from the
   residual polynomial (Eq. ``zeta``) and the three-term recurrence
   Eq. ``poly_recurrsion``; evaluating that recurrence at A = w gives the factor
   (1 - alpha_m w).  The printed (1 + alpha_m w) solves the mirrored shifts.
2. beta index.  The derivation (Eqs. ``recast1`` / ``seed_res_rec``) couples
   p_m to p_{m-1}, i.e. uses the previous iteration's beta.  At iteration m
   the zeta and beta^(w) formulas therefore use beta_{m-1} = rho_m/rho_{m-1},
   with beta_{-1} = 0 and alpha_{-1} = 1.
3. Inner products.  The shadow residual is r* (Appendix A), so <r~_j|r_i> is
   the unconjugated bilinear form r_j^T r_i (complex-symmetric COCG).
4. Step order.  v = A p, alpha, r_{m+1}, rho_{m+1}, beta_m, shift loop,
   p_{m+1}: the listing uses r_{m+1} before forming it.
5. Seed shift.  The seed system is A - sigma_s I; shift w is then solved with
   w' = w - sigma_s in the recurrences.  The default sigma_s = 0 is the
   paper's choice of the edge as seed (Sec. III).
6. Convergence.  Shift w is frozen once |r_{m+1}| / |zeta_{m+1}(w)| <=
   tol * |E| (ordinary 2-norms); the seed keeps iterating until every shift is
   frozen or the iteration cap is reached.
7. Breakdown.  The method is silent on it; the oracle stops when
   |r^T A p| <= 1e-14 |r| |A p| or, with shifts still open, when
   |r^T r| <= 1e-14 |r|^2 (convergence is tested first).
8. Seed exhaustion.  Also silent: a seed far from the resonances converges
   much faster than the shifts it carries, and once |r_{m+1}| falls below
   1e-150 |E| its bilinear products (about |r|^2) leave the normal float64
   range and beta = rho_{m+1}/rho_m soon turns inf or NaN.  The seed then
   stops and the open shifts are reported unconverged (``exhausted``);
   Appendix E's reseeding is the remedy.
9. Reseeding (Appendix E).  The collinearity deviation of shift w is
   dr(w) = |r_t(w) - r(w)| with the true residual r_t = E - (A - w)Psi(w) and
   the recurrence residual r(w) = r_M / zeta_M(w) at the shift's last
   iteration M.  A shift is restarted when dr(w) > reseed_tol |E| or when it
   was never frozen; the failing shift with the largest dr becomes the next
   seed, and the failing shifts are solved again from r_0 = E with it.
10. Dual space.  For a non-symmetric A (the general case of Appendix A that
   the method's BiCG form covers) the shadow residual is no longer r*: r~ and
   p~ run their own recurrence with A^T (bilinear form, so no conjugates),
   r~_0 = r_0 = E, sigma = r~^T A p, rho = r~^T r -- two products with the
   matrix per iteration.  With A symmetric, r~ = r at every step and the
   iteration is the complex-symmetric one above.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def direct_solve(Hp, E: np.ndarray, E_G: float, Gamma: float, w_in, method: str = "auto"):
    """Psi[k] = (H' - E_G - w_k - i Gamma)^{-1} E for every shift w_k.

    method: "eig" (dense eigendecomposition of H'), "lu" (dense LU per shift),
    "splu" (sparse LU per shift) or "auto" (eig below dim 5000, else splu).
    """
    w_in = np.asarray(w_in, dtype=np.float64)
    D = Hp.shape[0]
    if method == "auto":
        method = "eig" if D <= 5000 else "splu"
    out = np.zeros((len(w_in), D), dtype=np.complex128)
    if method == "eig":
        Hd = Hp.toarray() if hasattr(Hp, "toarray") else np.asarray(Hp)
        lam, V = np.linalg.eigh(Hd)
        c = V.T @ E
        for k, w in enumerate(w_in):
            out[k] = V @ (c / (lam - E_G - w - 1j * Gamma))
    elif method == "lu":
        Hd = Hp.toarray() if hasattr(Hp, "toarray") else np.asarray(Hp)
        for k, w in enumerate(w_in):
            M = Hd - (E_G + w + 1j * Gamma) * np.eye(D)
            out[k] = np.linalg.solve(M, E)
    elif method == "splu":
        I = sp.identity(D, format="csc", dtype=np.complex128)
        Hc = sp.csc_matrix(Hp, dtype=np.complex128)
        for k, w in enumerate(w_in):
            lu = spla.splu(Hc - (E_G + w + 1j * Gamma) * I)
            out[k] = lu.solve(E.astype(np.complex128))
    else:
        raise ValueError(method)
    return out


class MSBiCGResult:
    def __init__(self):
        self.psi = None           # [n_shift, D]
        self.iters = 0            # seed iterations (= matrix-vector products)
        self.alpha = []           # seed alpha_m
        self.beta = []            # seed beta_m
        self.rnorm = []           # |r_m|, m = 0..iters
        self.conv_iter = None     # per-shift iteration count at freeze
        self.zeta = None          # zeta history [iters+1, n_shift] (if requested)
        self.breakdown = False
        self.converged = False
        self.exhausted = False
        self.r_shift = None       # [n_shift, D] r_M / zeta_M at each shift's last iteration (if requested)


SEED_FLOOR = 1e-150      # reading 8


def msbicg_reference(A_apply, E: np.ndarray, w_in, tol: float, maxit: int,
                     seed_shift: float = 0.0, keep_zeta: bool = False,
                     breakdown_tol: float = 1e-14, keep_r: bool = False,
                     AT_apply=None) -> MSBiCGResult:
    """Multi-shift COCG for (A - w I) Psi = E, all shifts from one seed.

    ``A_apply(x)`` returns A x with A = H' - E_G - i Gamma.  The seed system is
    A_s = A - seed_shift I.  Follows Appendix D with readings 1-6 of the
    module docstring.  Returns an ``MSBiCGResult``.  ``AT_apply`` (x -> A^T x)
    selects the dual-space form of reading 10 for a non-symmetric A.
    """
    E = np.asarray(E, dtype=np.complex128)
    w = np.asarray(w_in, dtype=np.float64) - seed_shift       # w' = w - sigma_s
    n = len(w)
    D = E.shape[0]
    res = MSBiCGResult()

    # Initialisation (Algorithm 1, first two lines).
    dual = AT_apply is not None
    r = E.copy()
    p = E.copy()
    rt = E.copy() if dual else None      # shadow residual and direction (reading 10)
    pt = E.copy() if dual else None
    rho = r @ r                          # bilinear, reading 3
    normE = np.linalg.norm(E)
    psi = np.zeros((n, D), dtype=np.complex128)
    p_w = np.zeros((n, D), dtype=np.complex128)    # p_{-1}^(w) = 0
    zeta_prev = np.ones(n, dtype=np.complex128)    # zeta_{-1}
    zeta = np.ones(n, dtype=np.complex128)         # zeta_0
    alpha_prev = 1.0 + 0j                          # alpha_{-1}
    beta_prev = 0.0 + 0j                           # beta_{-1}
    active = np.ones(n, dtype=bool)
    conv_iter = np.full(n, -1, dtype=np.int64)
    res.rnorm.append(np.linalg.norm(r))
    zhist = [zeta.copy()] if keep_zeta else None
    r_shift = np.repeat(E[None, :], n, axis=0) if keep_r else None    # r_0 / zeta_0 = E

    if not (abs(rho) > breakdown_tol * normE * normE):
        # E = 0 is solved by Psi = 0; E^T E = 0 with E != 0 cannot start COCG
        res.psi = psi
        res.breakdown = normE > 0
        res.converged = normE == 0
        res.conv_iter = np.zeros(n, dtype=np.int64) if normE == 0 else conv_iter
        if keep_zeta:
            res.zeta = np.array(zhist)
        return res

    m = 0
    for m in range(maxit):
        v = A_apply(p) - seed_shift * p                 # matrix-vector product
        lhs = rt if dual else r
        sigma = lhs @ v
        if abs(sigma) <= breakdown_tol * np.linalg.norm(lhs) * np.linalg.norm(v):
            res.breakdown = True
            break
        alpha = rho / sigma
        r_new = r - alpha * v
        if dual:
            vt = AT_apply(pt) - seed_shift * pt         # the dual product
            rt_new = rt - alpha * vt
            rho_new = rt_new @ r_new
        else:
            rho_new = r_new @ r_new
        beta = rho_new / rho
        rn = np.linalg.norm(r_new)

        # Shift loop (reading 1 and 2).
        zeta_next = ((1.0 - alpha * w) * zeta
                     + (alpha * beta_prev / alpha_prev) * (zeta - zeta_prev))
        a = active
        alpha_w = (zeta[a] / zeta_next[a]) * alpha
        beta_w = (zeta_prev[a] / zeta[a]) ** 2 * beta_prev
        p_w[a] = r[None, :] / zeta[a, None] + beta_w[:, None] * p_w[a]
        psi[a] += alpha_w[:, None] * p_w[a]
        newly = a & (rn / np.abs(zeta_next) <= tol * normE)
        conv_iter[newly] = m + 1
        if keep_r:
            r_shift[a] = r_new[None, :] / zeta_next[a, None]
        zeta_prev = np.where(a, zeta, zeta_prev)
        zeta = np.where(a, zeta_next, zeta)
        active = a & ~newly

        # Seed update.
        p = r_new + beta * p
        r = r_new
        if dual:
            pt = rt_new + beta * pt
            rt = rt_new
        rho = rho_new
        alpha_prev, beta_prev = alpha, beta
        res.alpha.append(alpha)
        res.beta.append(beta)
        res.rnorm.append(rn)
        if keep_zeta:
            zhist.append(zeta.copy())
        if not np.any(active):
            m += 1
            break
        if not (rn > SEED_FLOOR * normE and np.isfinite(beta)):
            res.exhausted = True    # reading 8: stop before the products underflow
            break
        rtn = np.linalg.norm(rt) if dual else rn
        if not (abs(rho) > breakdown_tol * rn * rtn):
            res.breakdown = True        # rho_{m+1} = 0 while shifts are still open
            break
    else:
        m = maxit

    res.psi = psi
    res.iters = len(res.alpha)
    res.conv_iter = conv_iter
    res.converged = not np.any(active)
    res.r_shift = r_shift
    if keep_zeta:
        res.zeta = np.array(zhist)
    return res


def residual_polynomial(alpha, beta, x):
    """P_m(x), m = 0..len(alpha), from the seed scalars alone (Eq. ``poly_recurrsion``).

    P_0 = 1, P_{-1} = 1, and
    P_{m+1}(x) = (1 - alpha_m x) P_m + (alpha_m beta_{m-1}/alpha_{m-1}) (P_m - P_{m-1}),
    the residual polynomial of the seed evaluated at scalar x; by Eq. ``zeta``
    this equals zeta_m(x).  Independent of the vector recurrence.

    Pinned by ``tests/test_oracle_solve.py``: r_m = P_m(A_s) r_0 with the
    polynomial applied in the eigenbasis of A_s (App. C's definition of the
    residual polynomial), P_m(0) = 1, P_1(x) = 1 - alpha_0 x, and the two
    misreadings ((1 + alpha_m x), beta_m for beta_{m-1}) break that identity.
    """
    x = np.asarray(x, dtype=np.complex128)
    P_prev = np.ones_like(x)
    P = np.ones_like(x)
    out = [P.copy()]
    a_prev, b_prev = 1.0 + 0j, 0.0 + 0j
    for a, b in zip(alpha, beta):
        P_next = (1 - a * x) * P + (a * b_prev / a_prev) * (P - P_prev)
        P_prev, P = P, P_next
        out.append(P.copy())
        a_prev, b_prev = a, b
    return np.array(out)


class ReseedResult:
    def __init__(self):
        self.psi = None           # [n_shift, D]
        self.seed_of = None       # [n_shift] seed whose solve gave the final Psi of each shift
        self.dr = None            # [n_shift] final collinearity deviation dr(w) / |E|
        self.frozen = None        # [n_shift] bool: the final solve froze the shift
        self.seeds = []           # seeds in the order used
        self.iters = []           # seed iterations of every round


def reseed_solve(A_apply, E: np.ndarray, w_in, tol: float, maxit: int, seed_shift: float,
                 reseed_tol: float, max_rounds: int = 8) -> ReseedResult:
    """Appendix E: MSBiCG with adaptive reseeding (readings 8 and 9).

    Round 0 solves every shift from ``seed_shift``.  After each round, every
    shift of that round gets dr(w) = |r_t(w) - r(w)| (true residual against
    the recurrence residual r_M / zeta_M); shifts with dr > reseed_tol |E| or
    never frozen fail, the failing shift with the largest dr is the next seed,
    and only the failing shifts are solved again, from r_0 = E.  Stops when no
    shift fails or after ``max_rounds`` rounds.
    """
    E = np.asarray(E, dtype=np.complex128)
    w = np.asarray(w_in, dtype=np.float64)
    n = len(w)
    normE = np.linalg.norm(E)
    out = ReseedResult()
    out.psi = np.zeros((n, E.shape[0]), dtype=np.complex128)
    out.seed_of = np.full(n, np.nan)
    out.dr = np.full(n, np.inf)
    out.frozen = np.zeros(n, dtype=bool)
    todo = np.arange(n)
    seed = float(seed_shift)
    for _ in range(max_rounds):
        res = msbicg_reference(A_apply, E, w[todo], tol, maxit, seed_shift=seed, keep_r=True)
        out.seeds.append(seed)
        out.iters.append(res.iters)
        for j, k in enumerate(todo):
            rt = E - (A_apply(res.psi[j]) - w[k] * res.psi[j])
            out.psi[k] = res.psi[j]
            out.seed_of[k] = seed
            out.dr[k] = np.linalg.norm(rt - res.r_shift[j]) / normE
            out.frozen[k] = res.conv_iter[j] >= 0
        fail = todo[(out.dr[todo] > reseed_tol) | ~out.frozen[todo]]
        if len(fail) == 0:
            break
        seed = float(w[fail[np.argmax(out.dr[fail])]])
        todo = fail
    return out
