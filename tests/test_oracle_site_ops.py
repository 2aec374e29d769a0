"""Pins of the oracle's electron-number-changing site operators
(``hubbard.site_op`` / ``dipole_op``): canonical anticommutation, the number
operator, and free-fermion plane waves, which fix every Jordan-Wigner sign
(within a spin, across spins and across the periodic boundary)."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import groundstate as gs
from oracle import hubbard as hb

L = 5


def _B(nu, nd):
    return hb.Basis(L, nu, nd)


@pytest.mark.parametrize("spin", [0, 1])
def test_number_operator(spin):
    B = _B(2, 3)
    lower = _B(1, 3) if spin == 0 else _B(2, 2)
    for j in range(L):
        c = hb.site_op(B, lower, j, spin, create=False)
        cd = hb.site_op(lower, B, j, spin, create=True)
        n = hb.number_op(B, j, 1.0 if spin == 0 else 0.0, 1.0 if spin == 1 else 0.0)
        assert np.array_equal((cd @ c).toarray(), np.diag(n))
        assert np.array_equal(cd.toarray(), c.toarray().T)      # c+ is the adjoint of c (real)


def _shift(nu, nd, spin, d):
    return (nu + d, nd) if spin == 0 else (nu, nd + d)


@pytest.mark.parametrize("s1,s2", list(itertools.product([0, 1], repeat=2)))
def test_canonical_anticommutation(s1, s2):
    """{c_{i s1}, c+_{j s2}} = delta_ij delta_{s1 s2} and {c_i, c_j} = 0 on the (2, 2) sector."""
    nu, nd = 2, 2
    B = _B(nu, nd)
    for i, j in itertools.product(range(L), repeat=2):
        # c_i c+_j : B -> B+j -> B+j-i ;  c+_j c_i : B -> B-i -> B-i+j
        up_j = _B(*_shift(nu, nd, s2, +1))
        dn_i = _B(*_shift(nu, nd, s1, -1))
        tgt = _shift(*_shift(nu, nd, s2, +1), s1, -1)
        T = _B(*tgt)
        a = hb.site_op(up_j, T, i, s1, False) @ hb.site_op(B, up_j, j, s2, True)
        b = hb.site_op(dn_i, T, j, s2, True) @ hb.site_op(B, dn_i, i, s1, False)
        anti = (a + b).toarray()
        expect = np.eye(B.dim) if (i == j and s1 == s2) else np.zeros_like(anti)
        assert np.array_equal(anti, expect), (i, j, s1, s2)
        # two annihilators anticommute as well
        if (i, s1) != (j, s2):
            m1 = _B(*_shift(nu, nd, s1, -1))
            m2 = _B(*_shift(nu, nd, s2, -1))
            tt = _B(*_shift(*_shift(nu, nd, s1, -1), s2, -1))
            x = hb.site_op(m1, tt, j, s2, False) @ hb.site_op(B, m1, i, s1, False)
            y = hb.site_op(m2, tt, i, s1, False) @ hb.site_op(B, m2, j, s2, False)
            assert np.array_equal((x + y).toarray(), np.zeros((tt.dim, B.dim)))


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("m", [2, 3])
def test_free_fermion_plane_wave(spin, m):
    """U = 0 ring with t' : c+_k |G> is an eigenvector of H in the N + 1
    sector with energy E_G + eps_k for an empty momentum k (the periodic
    bond's fermion sign and the inter-spin order both enter)."""
    Lr, nu, nd = 6, 3, 3
    bonds = W.chain_bonds(Lr, 1.0, -0.3)
    B = hb.Basis(Lr, nu, nd)
    E_G, G, ev = gs.dense_ground_state(hb.hamiltonian(B, bonds, 0.0))
    assert ev[1] - ev[0] > 1e-8
    k = 2 * np.pi * m / Lr
    eps = -2.0 * np.cos(k) - 2.0 * (-0.3) * np.cos(2 * k)
    B1 = hb.Basis(Lr, nu + (spin == 0), nd + (spin == 1))
    coef = np.exp(1j * k * np.arange(Lr)) / np.sqrt(Lr)
    psi = hb.dipole_op(B, B1, coef, spin, create=True) @ G.astype(np.complex128)
    assert np.linalg.norm(psi) == pytest.approx(1.0, abs=1e-12)      # k is empty in G
    H1 = hb.hamiltonian(B1, bonds, 0.0)
    assert np.linalg.norm(H1 @ psi - (E_G + eps) * psi) <= 1e-12


def test_sector_mismatch_rejected():
    with pytest.raises(ValueError):
        hb.site_op(_B(2, 2), _B(2, 2), 0, 0, True)
