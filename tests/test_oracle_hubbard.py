"""Pins of the oracle's Hubbard Hamiltonian against closed forms and invariants.

A wrong Jordan-Wigner sign, a dropped wrap-around bond, a wrong diagonal or a
transposed index changes at least one of: the U = 0 free-fermion energy, the
two-site energy, the symmetry of H or the sampled-row apply.
"""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import workloads as W
from oracle import groundstate as gs
from oracle import hubbard as hb

GOLD = json.loads((Path(__file__).parent / "golden" / "closed_forms.json").read_text())


def lowest(H):
    """Lowest eigenvalue: dense eigh for small sectors, ARPACK (eigsh) above."""
    if H.shape[0] <= 3000:
        return gs.dense_ground_state(H)[0]
    import scipy.sparse.linalg as spla
    return float(spla.eigsh(H, k=1, which="SA", tol=1e-13)[0][0])


@pytest.mark.parametrize("L,nu,nd", [(4, 2, 2), (6, 3, 3), (8, 4, 4), (8, 3, 4), (10, 5, 5), (16, 5, 5)])
def test_sector_dimension(L, nu, nd):
    B = hb.Basis(L, nu, nd)
    assert B.dim == math.comb(L, nu) * math.comb(L, nd)
    assert np.all(np.diff(B.up) > 0) and np.all(np.bitwise_count(B.up) == nu)


def test_workload_dimensions():
    assert W.get("tiny").dim == 4900
    assert W.get("scale").dim == 853776
    assert W.get("precision").dim == 11778624          # C(14,7)^2
    assert W.get("batched").dim == 19079424            # C(16,5)^2
    assert W.get("learned").dim == 63504


@pytest.mark.parametrize("case", GOLD["dimer_ground_state"]["cases"])
def test_dimer_closed_form(case):
    B = hb.Basis(2, 1, 1)
    H = hb.hamiltonian(B, [(0, 1, case["t"])], case["U"])
    assert lowest(H) == pytest.approx(case["E_G"], abs=1e-13)


@pytest.mark.parametrize("case", GOLD["free_fermion_ring"]["cases"])
def test_free_fermion_ring_golden(case):
    L = case["L"]
    B = hb.Basis(L, case["N_up"], case["N_dn"])
    H = hb.hamiltonian(B, W.chain_bonds(L, case["t"]), 0.0)
    assert lowest(H) == pytest.approx(case["E_G"], abs=1e-12)


def _free_energy(eps, nu, nd):
    e = np.sort(eps)
    return e[:nu].sum() + e[:nd].sum()


@pytest.mark.parametrize("L,nu,nd,t,tp", [(6, 3, 3, 1.0, 0.0), (7, 3, 2, 1.0, -0.3), (8, 3, 4, 0.7, 0.25),
                                          (10, 3, 2, 1.0, -0.2)])
def test_u0_chain_matches_single_particle_spectrum(L, nu, nd, t, tp):
    """U = 0: many-body ground energy = filled single-particle levels (pins wrap-around signs)."""
    k = 2 * np.pi * np.arange(L) / L
    eps = -2 * t * np.cos(k) - 2 * tp * np.cos(2 * k)
    B = hb.Basis(L, nu, nd)
    H = hb.hamiltonian(B, W.chain_bonds(L, t, tp), 0.0)
    assert lowest(H) == pytest.approx(_free_energy(eps, nu, nd), abs=1e-11)


@pytest.mark.parametrize("Lx,Ly,nu,nd,tp", [(4, 4, 2, 1, -0.25), (4, 4, 2, 2, -0.25), (3, 3, 3, 2, 0.3)])
def test_u0_square_matches_single_particle_spectrum(Lx, Ly, nu, nd, tp):
    """U = 0 on periodic square clusters with diagonal hops (the batched workload's geometry)."""
    kx = 2 * np.pi * np.arange(Lx) / Lx
    ky = 2 * np.pi * np.arange(Ly) / Ly
    KX, KY = np.meshgrid(kx, ky, indexing="ij")
    eps = (-2 * (np.cos(KX) + np.cos(KY)) - 4 * tp * np.cos(KX) * np.cos(KY)).ravel()
    B = hb.Basis(Lx * Ly, nu, nd)
    H = hb.hamiltonian(B, W.square_bonds(Lx, Ly, 1.0, tp), 0.0)
    assert lowest(H) == pytest.approx(_free_energy(eps, nu, nd), abs=1e-11)


def test_hamiltonian_is_real_symmetric():
    B = hb.Basis(8, 3, 4)
    H = hb.hamiltonian(B, W.chain_bonds(8, 1.0, -0.3), 6.0, core_site=2, Uc=-4.0)
    assert H.dtype == np.float64
    assert abs(H - H.T).max() == 0.0


def test_zero_hopping_is_diagonal_with_interaction_and_core_terms():
    B = hb.Basis(6, 3, 2)
    H = hb.hamiltonian(B, [(i, (i + 1) % 6, 0.0) for i in range(6)], 5.0, core_site=1, Uc=-2.0)
    off = H - np.diag(H.diagonal())
    assert abs(off).max() == 0.0
    S = B.states()
    u, d = S & 63, S >> 6
    expect = 5.0 * np.bitwise_count(u & d) - 2.0 * (((u >> 1) & 1) + ((d >> 1) & 1))
    assert np.array_equal(H.diagonal(), expect.astype(float))


def test_half_filled_ring_has_unique_ground_state():
    """Lieb: the half-filled bipartite ring (t' = 0) has a non-degenerate ground state."""
    B = hb.Basis(8, 4, 4)
    w = gs.dense_ground_state(hb.hamiltonian(B, W.chain_bonds(8, 1.0), 8.0))[2]
    assert w[1] - w[0] > 1e-3


def test_apply_rows_matches_matrix_rows():
    B = hb.Basis(8, 3, 4)
    bonds = W.chain_bonds(8, 1.0, -0.3)
    H = hb.hamiltonian(B, bonds, 6.0, core_site=3, Uc=-4.0)
    x = W.random_complex(B.dim, 1)
    rows = np.array([0, 5, 17, B.dim // 2, B.dim - 1])
    shift = 1.5 + 0.5j
    ref = (H @ x - shift * x)[rows]
    got = hb.apply_rows(B, bonds, 6.0, x, rows, core_site=3, Uc=-4.0, shift=shift)
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_number_operator_counts_electrons():
    B = hb.Basis(6, 3, 2)
    tot = sum(hb.number_op(B, j, 1.0, 1.0) for j in range(6))
    assert np.all(tot == 5.0)
