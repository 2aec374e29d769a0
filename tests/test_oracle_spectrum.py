"""Pins of the oracle's ground state and Kramers-Heisenberg intensity.

* Lanczos ground state vs dense diagonalisation and its eigen-residual.
* Lehmann sum vs continued fraction vs correction vector (three routes).
* Moments (norm and a_0), the sum rule and positivity of I.
* The U_c = 0 pipeline closed form I = eta / (pi (w^2 + eta^2)(w_in^2 + Gamma^2)).
"""
import numpy as np
import pytest

import workloads as W
from oracle import groundstate as gs
from oracle import hubbard as hb
from oracle import solve as so
from oracle import spectrum as sp


@pytest.fixture(scope="module")
def small():
    B = hb.Basis(6, 3, 3)
    bonds = W.chain_bonds(6, 1.0)
    H = hb.hamiltonian(B, bonds, 8.0)
    ev, V = np.linalg.eigh(H.toarray())
    return B, bonds, H, ev, V


def test_lanczos_ground_state_matches_dense():
    B = hb.Basis(8, 3, 3)
    H = hb.hamiltonian(B, W.chain_bonds(8, 1.0, -0.3), 6.0)
    E0, G0, _ = gs.dense_ground_state(H)
    E, G, it = gs.lanczos_ground_state(H, W.random_vector(B.dim, 12345), 1e-12, 400)
    assert abs(E - E0) <= 1e-12 * abs(E0)
    assert abs(G @ G0) >= 1 - 1e-12
    assert np.linalg.norm(H @ G - E * G) <= 1e-9


def test_three_spectrum_routes_agree(small):
    B, bonds, H, ev, V = small
    E_G = ev[0]
    phi = W.random_complex(B.dim, 5)
    w = np.linspace(0.0, 10.0, 41)
    eta = 0.1
    I_l = sp.lehmann(ev, V, phi, E_G, w, eta)[0]
    I_cf, depth = sp.continued_fraction(H, phi, E_G, w, eta, tol=1e-13)
    assert np.max(np.abs(I_cf - I_l)) <= 1e-10 * np.max(I_l)
    for j in (0, 7, 23, 40):
        I_cv = sp.correction_vector(H, phi, E_G, w[j], eta)
        assert I_cv == pytest.approx(I_l[j], rel=1e-11)


def test_moments_sum_rule_and_positivity(small):
    B, bonds, H, ev, V = small
    phi = W.random_complex(B.dim, 6)
    a, b, norm = sp.lanczos_tridiag(H, phi, 5)
    assert norm ** 2 == pytest.approx(np.vdot(phi, phi).real, rel=1e-14)
    assert a[0] == pytest.approx(np.vdot(phi, H @ phi).real / np.vdot(phi, phi).real, rel=1e-13)
    E_G = ev[0]
    w = np.linspace(-60.0, 80.0, 140001)
    I = sp.lehmann(ev, V, phi, E_G, w, 0.1)[0]
    assert np.all(I >= 0)
    total = np.trapezoid(I, w)
    assert total == pytest.approx(np.vdot(phi, phi).real, rel=2e-3)   # Lorentzian tails outside the grid


def test_uc_zero_pipeline_closed_form(small):
    """U_c = 0, O_1 = O_2 = 1: Psi = -G/(w_in + i Gamma), so
    I(w_in, w) = eta / (pi (w^2 + eta^2) (w_in^2 + Gamma^2))."""
    B, bonds, H, ev, V = small
    E_G, G = ev[0], V[:, 0]
    Gamma, eta = 1.0, 0.1
    w_in = np.array([-3.0, 0.0, 2.0])
    w = np.linspace(0.0, 5.0, 11)
    psi = so.direct_solve(H, G.astype(complex), E_G, Gamma, w_in, "eig")
    I = sp.lehmann(ev, V, psi, E_G, w, eta)
    expect = eta / (np.pi * (w[None, :] ** 2 + eta ** 2) * (w_in[:, None] ** 2 + Gamma ** 2))
    assert np.max(np.abs(I - expect)) <= 1e-12 * np.max(expect)


def test_cf_green_simple_pole():
    """A one-level continued fraction is a single Lorentzian."""
    z = np.array([0.5 + 0.1j, 2.0 + 0.1j])
    g = sp.cf_green(np.array([1.0]), np.array([]), 2.0, z)
    assert np.allclose(g, 4.0 / (z - 1.0))
