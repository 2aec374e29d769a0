"""Pins of the oracle's intermediate-state solvers.

* ``direct_solve`` is checked against the U_c = 0 closed form, the
  complex-symmetric resolvent identity and the a-posteriori bound.
* ``msbicg_reference`` (Appendix D in the corrected reading) is checked against
  ``direct_solve``, against the collinearity of the shifted true residuals
  with the seed residual (Eqs. shiftCoeff / collinearity), against the m = 0
  closed form, and against exact termination for a diagonal H.
"""
import numpy as np
import pytest

import workloads as W
from oracle import groundstate as gs
from oracle import hubbard as hb
from oracle import solve as so


@pytest.fixture(scope="module")
def ring():
    B = hb.Basis(6, 3, 3)
    bonds = W.chain_bonds(6, 1.0)
    H = hb.hamiltonian(B, bonds, 8.0)
    Hp = hb.hamiltonian(B, bonds, 8.0, core_site=0, Uc=-4.0)
    E_G, G, _ = gs.dense_ground_state(H)
    return B, H, Hp, E_G, G


def test_direct_methods_agree(ring):
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 3)
    w = np.linspace(-5, 5, 7)
    a = so.direct_solve(Hp, E, E_G, 1.0, w, "eig")
    b = so.direct_solve(Hp, E, E_G, 1.0, w, "lu")
    c = so.direct_solve(Hp, E, E_G, 1.0, w, "splu")
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    assert np.max(np.abs(a - c)) <= 1e-12 * np.max(np.abs(a))


def test_uc_zero_closed_form(ring):
    """U_c = 0: E = G is an eigenvector of A, Psi = -G / (w + i Gamma)."""
    B, H, Hp, E_G, G = ring
    w = np.array([-3.0, 0.0, 0.7, 5.0])
    psi = so.direct_solve(H, G.astype(complex), E_G, 0.5, w, "lu")
    for k, wk in enumerate(w):
        assert np.allclose(psi[k], -G / (wk + 0.5j), rtol=0, atol=1e-12)


def test_resolvent_identity(ring):
    """E^T (Psi_1 - Psi_2) = (w_1 - w_2) Psi_1^T Psi_2 for complex-symmetric A."""
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 4)
    w = np.array([-2.0, 1.3])
    p = so.direct_solve(Hp, E, E_G, 1.0, w, "lu")
    lhs = E @ (p[0] - p[1])
    rhs = (w[0] - w[1]) * (p[0] @ p[1])
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_reference_recurrence_matches_direct_solve(ring):
    B, H, Hp, E_G, G = ring
    E = G.astype(complex)
    w = np.linspace(-10, 10, 41)
    ref = so.direct_solve(Hp, E, E_G, 1.0, w, "eig")
    A = lambda x: Hp @ x - (E_G + 1j) * x
    res = so.msbicg_reference(A, E, w, 1e-13, 2000)
    assert res.converged and not res.breakdown
    err = np.linalg.norm(res.psi - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-10


def test_reference_with_seed_shift_and_complex_rhs(ring):
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 8)
    w = np.linspace(-6, 6, 13)
    ref = so.direct_solve(Hp, E, E_G, 0.7, w, "eig")
    A = lambda x: Hp @ x - (E_G + 0.7j) * x
    res = so.msbicg_reference(A, E, w, 1e-12, 3000, seed_shift=2.5)
    err = np.linalg.norm(res.psi - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-9


def test_printed_plus_sign_solves_mirrored_shifts(ring):
    """The zeta recurrence with (1 + alpha w) (as printed) reproduces the solve at -w,
    so the oracle's (1 - alpha w) reading is the one that solves (A - w) Psi = E."""
    B, H, Hp, E_G, G = ring
    E = G.astype(complex)
    w = np.array([-4.0, 3.0])
    A = lambda x: Hp @ x - (E_G + 1j) * x
    res_minus = so.msbicg_reference(A, E, -w, 1e-12, 2000)    # run with -w == "+" sign at w
    ref_plus = so.direct_solve(Hp, E, E_G, 1.0, w, "eig")
    ref_mirror = so.direct_solve(Hp, E, E_G, 1.0, -w, "eig")
    assert np.max(np.abs(res_minus.psi - ref_mirror)) <= 1e-9 * np.max(np.abs(ref_mirror))
    assert np.max(np.abs(res_minus.psi - ref_plus)) > 1e-3 * np.max(np.abs(ref_plus))


@pytest.mark.parametrize("m", [1, 4, 15, 40])
def test_shifted_residuals_are_collinear_with_seed(ring, m):
    """True residual of every shifted iterate = r_m / zeta_m (Eq. collinearity).

    The seed itself is one of the shifts (w = seed shift -> zeta = 1), so its true
    residual is the seed residual r_m; every other shift's true residual must equal
    it divided by the recurrence's zeta_m(w)."""
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 6)
    seed = 0.0
    w = np.array([seed, -7.0, -1.0, 2.5, 9.0])
    A = lambda x: Hp @ x - (E_G + 1j) * x
    res = so.msbicg_reference(A, E, w, 1e-30, m, seed_shift=seed, keep_zeta=True)
    assert res.iters == m
    zeta = res.zeta[-1]
    assert np.all(res.zeta[:, 0] == 1.0)           # the seed's zeta stays exactly 1
    r_true = np.stack([E - (A(res.psi[k]) - w[k] * res.psi[k]) for k in range(len(w))])
    r_seed = r_true[0]
    for k in range(1, len(w)):
        pred = r_seed / zeta[k]
        assert np.linalg.norm(r_true[k] - pred) <= 1e-8 * np.linalg.norm(E) + 1e-8 * np.linalg.norm(pred)


def test_first_iterate_closed_form(ring):
    """After one iteration Psi_1(w) = alpha_0(w) E with alpha_0(w) = rho_0 / (E^T A E - w rho_0)."""
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 7)
    w = np.array([-2.0, 0.0, 3.0])
    A = lambda x: Hp @ x - (E_G + 1j) * x
    res = so.msbicg_reference(A, E, w, 1e-30, 1)
    rho0 = E @ E
    for k, wk in enumerate(w):
        a0 = rho0 / (E @ A(E) - wk * rho0)
        assert np.allclose(res.psi[k], a0 * E, rtol=1e-12, atol=0)


def test_diagonal_hamiltonian_terminates_exactly():
    """t = 0: A is diagonal with few distinct values; the Krylov space is exhausted
    after (#distinct eigenvalues) iterations and the solve is exact."""
    B = hb.Basis(6, 3, 3)
    Hp = hb.hamiltonian(B, [(i, (i + 1) % 6, 0.0) for i in range(6)], 4.0, core_site=0, Uc=-3.0)
    n_distinct = len(np.unique(Hp.diagonal()))
    E = W.random_vector(B.dim, 2).astype(complex)
    w = np.linspace(-3, 3, 5)
    A = lambda x: Hp @ x - (0.5 + 1j) * x
    res = so.msbicg_reference(A, E, w, 1e-12, 50)
    assert res.iters <= n_distinct
    ref = so.direct_solve(Hp, E, 0.5, 1.0, w, "eig")
    assert np.max(np.abs(res.psi - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_a_posteriori_bound(ring):
    """A - w is normal with |(A - w)^{-1}| <= 1/Gamma, so |Psi - Psi*| <= |r_true| / Gamma."""
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 9)
    w = np.linspace(-5, 5, 6)
    A = lambda x: Hp @ x - (E_G + 0.8j) * x
    res = so.msbicg_reference(A, E, w, 1e-5, 2000)
    ref = so.direct_solve(Hp, E, E_G, 0.8, w, "eig")
    for k in range(len(w)):
        r = E - (A(res.psi[k]) - w[k] * res.psi[k])
        assert np.linalg.norm(res.psi[k] - ref[k]) <= np.linalg.norm(r) / 0.8 * (1 + 1e-10)


def test_rho_breakdown_detected():
    """E = e_0 + i e_1 has E^T E = 0 (COCG cannot start)."""
    B = hb.Basis(4, 2, 2)
    Hp = hb.hamiltonian(B, W.chain_bonds(4, 1.0), 4.0, core_site=0, Uc=-2.0)
    E = np.zeros(B.dim, complex)
    E[0], E[1] = 1.0, 1.0j
    res = so.msbicg_reference(lambda x: Hp @ x - (1 + 1j) * x, E, [0.0, 1.0], 1e-10, 10)
    assert res.breakdown and res.iters == 0


@pytest.fixture(scope="module")
def sharp():
    """The L=8 ring with a narrow core-hole broadening (Gamma = 0.3): an edge
    seed (w_in = -12) converges far faster than the resonant shifts it carries."""
    bonds = W.chain_bonds(8, 1.0)
    B = hb.Basis(8, 4, 4)
    E_G, G, _ = gs.dense_ground_state(hb.hamiltonian(B, bonds, 8.0))
    Hp = hb.hamiltonian(B, bonds, 8.0, core_site=0, Uc=-4.0)
    Gamma = 0.3
    w = np.linspace(-12.0, 12.0, 64)
    E = G.astype(np.complex128)

    def A(x):
        return Hp @ x - (E_G + 1j * Gamma) * x
    ref = so.direct_solve(Hp, E, E_G, Gamma, w, method="eig")
    return A, E, w, ref


def test_edge_seed_exhausts_without_nan(sharp):
    """Reading 8: the seed stops at the float64 floor instead of producing
    NaN; the shifts frozen before that are the direct solution."""
    A, E, w, ref = sharp
    res = so.msbicg_reference(A, E, w, 1e-10, 3000, seed_shift=-12.0, keep_r=True)
    assert res.exhausted and not res.converged and not res.breakdown
    assert res.rnorm[-1] <= so.SEED_FLOOR * np.linalg.norm(E) * 1e3
    assert np.all(np.isfinite(res.psi))
    frozen = res.conv_iter >= 0
    assert 0 < frozen.sum() < len(w)
    err = np.linalg.norm(res.psi[frozen] - ref[frozen], axis=1) / np.linalg.norm(ref[frozen], axis=1)
    assert err.max() <= 1e-8
    # the open shifts have not met tol, some by orders of magnitude
    rt = np.array([np.linalg.norm(E - (A(res.psi[k]) - w[k] * res.psi[k])) for k in np.nonzero(~frozen)[0]])
    assert rt.min() > 1e-10 * np.linalg.norm(E) and rt.max() > 1e-6 * np.linalg.norm(E)


def test_collinearity_deviation_vanishes_for_a_good_seed(sharp):
    """dr(w) of Appendix E is rounding-small when collinearity holds (seed 0),
    which pins the stored recurrence residuals r_M / zeta_M."""
    A, E, w, ref = sharp
    out = so.reseed_solve(A, E, w, 1e-10, 3000, 0.0, 1e-9)
    assert out.seeds == [0.0] and out.frozen.all()
    assert out.dr.max() <= 1e-12
    res = so.msbicg_reference(A, E, w, 1e-10, 3000, seed_shift=0.0)
    assert np.array_equal(out.psi, res.psi)


def test_reseeding_recovers_from_an_edge_seed(sharp):
    """Appendix E: the failing shifts restart from the worst one and every
    shift ends at the direct solution."""
    A, E, w, ref = sharp
    out = so.reseed_solve(A, E, w, 1e-10, 3000, -12.0, 1e-9)
    assert len(out.seeds) >= 2 and out.seeds[0] == -12.0
    assert out.frozen.all() and out.dr.max() <= 1e-9
    assert set(out.seed_of) <= set(out.seeds)
    assert np.all(np.isin(out.seeds[1:], w))       # later seeds are shifts of the list
    err = np.linalg.norm(out.psi - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-8
    # the shifts kept from round 0 are exactly those the edge seed froze
    r0 = so.msbicg_reference(A, E, w, 1e-10, 3000, seed_shift=-12.0)
    assert np.array_equal(out.seed_of == -12.0, r0.conv_iter >= 0)


def _directed_ring(g, open_chain=False):
    """L=6 ring (or open chain), N=3+3, hopping e^{+g} to the right and e^{-g}
    to the left (non-reciprocal), core hole on site 0."""
    L = 6
    bonds = [(i, i + 1, np.exp(g), np.exp(-g)) for i in range(L - 1)]
    if not open_chain:
        bonds.append((L - 1, 0, np.exp(g), np.exp(-g)))
    return hb.Basis(L, 3, 3), bonds


def test_directed_transpose_swaps_directions():
    B, bonds = _directed_ring(0.3)
    H = hb.hamiltonian(B, bonds, 8.0, core_site=0, Uc=-4.0)
    swapped = [(i, j, tr, t) for (i, j, t, tr) in bonds]
    HT = hb.hamiltonian(B, swapped, 8.0, core_site=0, Uc=-4.0)
    assert abs(H - H.T).max() > 0.1                       # really non-symmetric
    assert abs(HT - H.T).max() == 0.0


def test_directed_open_chain_is_an_imaginary_gauge_transform():
    """Open chain: H_g = S H_0 S^-1 with S = diag(e^{g * sum of electron
    positions}) -- fixes which direction carries e^{+g}."""
    g = 0.4
    B, bonds = _directed_ring(g, open_chain=True)
    B0, bonds0 = _directed_ring(0.0, open_chain=True)
    Hg = hb.hamiltonian(B, bonds, 8.0).toarray()
    H0 = hb.hamiltonian(B0, bonds0, 8.0).toarray()
    S = B.states()
    L = B.L
    pos = np.zeros(B.dim)
    for k in range(2 * L):
        pos += ((S >> k) & 1) * (k % L)
    sc = np.exp(g * pos)
    assert np.allclose(Hg, sc[:, None] * H0 / sc[None, :], atol=1e-12, rtol=0)


def test_dual_space_form_solves_nonsymmetric_systems():
    B, bonds = _directed_ring(0.3)
    H = hb.hamiltonian(B, bonds, 8.0, core_site=0, Uc=-4.0)
    HT = H.T.tocsr()
    E_G, Gamma = -3.0, 1.0
    E = W.random_complex(B.dim, 5)
    w = np.linspace(-6, 6, 12)
    ref = so.direct_solve(H, E, E_G, Gamma, w, method="lu")

    def A(x):
        return H @ x - (E_G + 1j * Gamma) * x

    def AT(x):
        return HT @ x - (E_G + 1j * Gamma) * x
    res = so.msbicg_reference(A, E, w, 1e-13, 2000, AT_apply=AT)
    assert res.converged
    err = np.max(np.linalg.norm(res.psi - ref, axis=1) / np.linalg.norm(ref, axis=1))
    assert err <= 1e-10
    # the complex-symmetric form (no dual) does not solve them
    bad = so.msbicg_reference(A, E, w, 1e-13, 2000)
    errb = np.max(np.linalg.norm(bad.psi - ref, axis=1) / np.linalg.norm(ref, axis=1))
    assert errb > 1e-3


def test_dual_space_form_reduces_to_the_symmetric_one(ring):
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 8)
    w = np.linspace(-5, 5, 9)

    def A(x):
        return Hp @ x - (E_G + 1j) * x
    a = so.msbicg_reference(A, E, w, 1e-12, 500)
    b = so.msbicg_reference(A, E, w, 1e-12, 500, AT_apply=A)
    assert a.iters == b.iters
    assert np.array_equal(a.psi, b.psi)


# ---- residual polynomial (App. C, Eqs. zeta and poly_recurrsion) ------------

def _seed_scalars(Hp, E_G, Gamma, E, seed, m):
    """alpha_j, beta_j of the oracle's seed recurrence for m iterations, and its
    seed iterate x_m (the shift equal to the seed has zeta = 1, so its Psi is x_m)."""
    A = lambda x: Hp @ x - (E_G + 1j * Gamma) * x
    res = so.msbicg_reference(A, E, np.array([seed, seed + 0.9, seed - 2.3]), 0.0, m,
                              seed_shift=seed, keep_zeta=True)
    assert res.iters == m and not res.breakdown
    return res


def _poly_of_matrix(P_at, lam, V, E):
    """P(A_s) E for the diagonalisable A_s = V diag(lam) V^{-1}: the polynomial's
    values at the eigenvalues applied in the eigenbasis."""
    return V @ (P_at * np.linalg.solve(V, E))


@pytest.mark.parametrize("seed", [0.0, 1.7])
def test_residual_polynomial_gives_the_seed_residuals(ring, seed):
    """r_m = P_m(A_s) r_0 (the residual-polynomial definition of App. C), with
    P_m from the seed scalars alone: the polynomial evaluated at the eigenvalues
    of A_s and applied in its eigenbasis reproduces the seed residual
    E - A_s x_m of the vector recurrence, at every m checked."""
    B, H, Hp, E_G, G = ring
    Gamma = 0.8
    E = W.random_complex(B.dim, 11)
    As = Hp.toarray() - (E_G + seed + 1j * Gamma) * np.eye(B.dim)
    lam, V = np.linalg.eig(As)
    for m in (1, 2, 5, 17, 40):
        res = _seed_scalars(Hp, E_G, Gamma, E, seed, m)
        x_m = res.psi[0]
        r_m = E - As @ x_m
        P = so.residual_polynomial(res.alpha, res.beta, lam)[m]
        r_poly = _poly_of_matrix(P, lam, V, E)
        assert np.linalg.norm(r_poly - r_m) <= 1e-9 * np.linalg.norm(E), m
        assert abs(np.linalg.norm(r_poly) - res.rnorm[m]) <= 1e-9 * np.linalg.norm(E), m


def test_residual_polynomial_normalisation_and_first_degree(ring):
    """P_m(0) = 1 for every m (r_m = E - A x_m with x_m in the Krylov space),
    and P_1(x) = 1 - alpha_0 x."""
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 12)
    res = _seed_scalars(Hp, E_G, 1.0, E, 0.0, 25)
    x = np.array([0.0, 0.3 - 0.2j, -4.0 + 1j, 7.5])
    P = so.residual_polynomial(res.alpha, res.beta, x)
    assert np.allclose(P[:, 0], 1.0, rtol=0, atol=1e-12)
    assert np.allclose(P[1], 1.0 - res.alpha[0] * x, rtol=1e-15, atol=1e-15)
    assert P.shape == (26, 4)


def test_residual_polynomial_equals_zeta(ring):
    """Eq. zeta: the shift coefficient zeta_m(w') of the recurrence is P_m(w')
    evaluated from the seed scalars, for shifts on both sides of the seed."""
    B, H, Hp, E_G, G = ring
    E = W.random_complex(B.dim, 13)
    seed = 1.7
    res = _seed_scalars(Hp, E_G, 0.8, E, seed, 30)
    w_prime = np.array([0.0, 0.9, -2.3])                   # the three shifts minus the seed
    P = so.residual_polynomial(res.alpha, res.beta, w_prime)
    assert np.max(np.abs(P - res.zeta) / np.abs(res.zeta)) <= 1e-12


def test_residual_polynomial_pin_rejects_misprints(ring):
    """The two plausible misreadings of Eq. poly_recurrsion, the printed
    (1 + alpha_m x) sign and beta_m in place of beta_{m-1}, break the identity
    r_m = P_m(A_s) E that the correct recurrence satisfies."""
    B, H, Hp, E_G, G = ring
    Gamma = 0.8
    E = W.random_complex(B.dim, 14)
    As = Hp.toarray() - (E_G + 1j * Gamma) * np.eye(B.dim)
    lam, V = np.linalg.eig(As)
    m = 12
    res = _seed_scalars(Hp, E_G, Gamma, E, 0.0, m)
    r_m = E - As @ res.psi[0]

    def variant(x, sign, shift_beta):
        P_prev = np.ones_like(x)
        P = np.ones_like(x)
        a_prev, b_prev = 1.0 + 0j, 0.0 + 0j
        for j in range(m):
            a, b = res.alpha[j], res.beta[j]
            bb = b if shift_beta else b_prev
            P_next = (1 + sign * a * x) * P + (a * bb / a_prev) * (P - P_prev)
            P_prev, P = P, P_next
            a_prev, b_prev = a, b
        return P

    good = so.residual_polynomial(res.alpha, res.beta, lam)[m]
    assert np.allclose(variant(lam, -1, False), good, rtol=1e-13, atol=1e-13)
    for sign, shift_beta in ((+1, False), (-1, True)):
        r_bad = _poly_of_matrix(variant(lam, sign, shift_beta), lam, V, E)
        assert np.linalg.norm(r_bad - r_m) >= 1e-3 * np.linalg.norm(E), (sign, shift_beta)
