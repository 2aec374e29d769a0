"""Parity of the auxiliary entry points with the oracle.

* msb_number_op: O = w_up n_{j up} + w_dn n_{j dn} applied to real and complex
  vectors, identity when site < 0 (the right-hand sides E = O_2 G);
* msb_combine: phi = sum_s e^{i q s} O_1,s Psi_s with and without O_1;
* msb_sector_info: per-spin sector sizes C(L, N_sigma) and bond types.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hubbard as hb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring(gpu):
    msb = gpu
    L, nu, nd = 8, 3, 4
    bonds = W.chain_bonds(L, 1.0, -0.3)
    ctx = msb.msb_create(L, nu, nd, bonds, 6.0)
    yield msb, ctx, hb.Basis(L, nu, nd), L, nu, nd
    msb.msb_destroy(ctx)


def test_sector_info(ring):
    msb, ctx, B, L, nu, nd = ring
    n_up, n_dn, n_types = msb.msb_sector_info(ctx)
    assert (n_up, n_dn, n_types) == (math.comb(L, nu), math.comb(L, nd), 2)
    assert msb.msb_dim(ctx) == B.dim


@pytest.mark.parametrize("site,wu,wd", [(0, 1.0, 1.0), (5, 1.0, -1.0), (7, 0.25, 2.0), (-1, 1.0, 1.0)])
def test_number_op_matches_oracle(ring, site, wu, wd):
    import torch
    msb, ctx, B, L, nu, nd = ring
    D = B.dim
    diag = np.ones(D) if site < 0 else hb.number_op(B, site, wu, wd)
    xr = W.random_vector(D, 3)
    xc = W.random_complex(D, 4)
    out = torch.empty(D, dtype=torch.complex128, device="cuda")
    msb.msb_number_op(ctx, site, wu, wd, torch.from_numpy(xr).cuda(), out)
    assert np.array_equal(out.cpu().numpy(), diag * xr)
    msb.msb_number_op(ctx, site, wu, wd, torch.from_numpy(xc).cuda(), out)
    assert np.array_equal(out.cpu().numpy(), diag * xc)


@pytest.mark.parametrize("with_o1", [False, True])
def test_combine_matches_oracle(ring, with_o1):
    import torch
    msb, ctx, B, L, nu, nd = ring
    D = B.dim
    nsys, n_shift = 5, 7
    q = math.pi / 2
    phases = [complex(math.cos(q * s), math.sin(q * s)) for s in range(nsys)]
    psi = np.stack([np.stack([W.random_complex(D, 100 * s + k) for k in range(n_shift)]) for s in range(nsys)])
    o1 = [(s, 1.0, 0.5 + 0.1 * s) for s in range(nsys)] if with_o1 else None
    phi = torch.empty(n_shift, D, dtype=torch.complex128, device="cuda")
    msb.msb_combine(ctx, torch.from_numpy(psi).cuda(), nsys, n_shift, msb.MSB_C128, phases, phi, o1=o1)
    expect = np.zeros((n_shift, D), dtype=np.complex128)
    for s in range(nsys):
        d = hb.number_op(B, *o1[s]) if with_o1 else np.ones(D)
        expect += phases[s] * d[None, :] * psi[s]
    err = np.max(np.abs(phi.cpu().numpy() - expect)) / np.max(np.abs(expect))
    assert err <= 1e-14
    # complex64 input: the same sum of the rounded values
    psi32 = psi.astype(np.complex64)
    msb.msb_combine(ctx, torch.from_numpy(psi32).cuda(), nsys, n_shift, msb.MSB_C64, phases, phi, o1=o1)
    expect32 = np.zeros((n_shift, D), dtype=np.complex128)
    for s in range(nsys):
        d = hb.number_op(B, *o1[s]) if with_o1 else np.ones(D)
        expect32 += phases[s] * d[None, :] * psi32[s].astype(np.complex128)
    assert np.max(np.abs(phi.cpu().numpy() - expect32)) / np.max(np.abs(expect32)) <= 1e-14


@pytest.mark.parametrize("spin,create", [(0, True), (1, True), (0, False), (1, False)])
def test_dipole_matches_oracle(ring, spin, create):
    """sum_j coef_j c+_{j s} (or c_{j s}) between the (3, 4) sector and its
    neighbour, two vectors at once, against the oracle's sparse operator."""
    import torch
    msb, ctx, B, L, nu, nd = ring
    d = 1 if create else -1
    nu2, nd2 = (nu + d, nd) if spin == 0 else (nu, nd + d)
    bonds = W.chain_bonds(L, 1.0, -0.3)
    ctx2 = msb.msb_create(L, nu2, nd2, bonds, 6.0)
    try:
        B2 = hb.Basis(L, nu2, nd2)
        rng = np.random.default_rng(11 + 2 * spin + int(create))
        coef = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        x = np.stack([W.random_complex(B.dim, 90 + k) for k in range(2)])
        y = torch.full((2, B2.dim), float("nan"), dtype=torch.complex128, device="cuda")
        msb.msb_dipole(ctx, ctx2, spin, create, coef, torch.from_numpy(x).cuda(), y)
        Op = hb.dipole_op(B, B2, coef, spin, create)
        ref = np.stack([Op @ x[k] for k in range(2)])
        got = y.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
        msb.msb_dipole(ctx, ctx2, spin, create, coef, torch.from_numpy(x).cuda(), y, accumulate=True)
        assert np.max(np.abs(y.cpu().numpy() - 2 * ref)) <= 2e-14 * np.max(np.abs(ref))
        with pytest.raises(msb.MsbError):           # wrong direction for this pair of sectors
            msb.msb_dipole(ctx, ctx2, spin, not create, coef, torch.from_numpy(x).cuda(), y)
    finally:
        msb.msb_destroy(ctx2)


def test_direct_edge_pipeline_matches_lehmann(gpu):
    """A direct edge with a valence electron added at the core-hole site:
    E = c+_{0 up} G in the (N+1, N) sector, the multi-shift solve there with
    the core hole on site 0, phi = c_{0 up} Psi back in the (N, N) sector,
    and the continued-fraction spectrum -- against the oracle's direct
    solves and Lehmann sum over exact eigenstates."""
    import torch
    from oracle import groundstate as ogs
    from oracle import solve as osolve
    from oracle import spectrum as ospec
    msb = gpu
    L, N, U, Uc, Gamma, eta = 8, 4, 8.0, -4.0, 1.0, 0.1
    bonds = W.chain_bonds(L, 1.0)
    w_in = np.linspace(-8.0, 8.0, 24)
    w = np.linspace(0.0, 10.0, 128)
    B0, B1 = hb.Basis(L, N, N), hb.Basis(L, N + 1, N)
    H0 = hb.hamiltonian(B0, bonds, U)
    E_G, G, _ = ogs.dense_ground_state(H0)
    H1c = hb.hamiltonian(B1, bonds, U, core_site=0, Uc=Uc)
    cd = hb.site_op(B0, B1, 0, 0, True)
    c = hb.site_op(B1, B0, 0, 0, False)
    E = cd @ G.astype(np.complex128)
    psi_ref = osolve.direct_solve(H1c, E, E_G, Gamma, w_in, "eig")
    phi_ref = np.stack([c @ psi_ref[k] for k in range(len(w_in))])
    ev, V = np.linalg.eigh(H0.toarray())
    I_ref = ospec.lehmann(ev, V, phi_ref, E_G, w, eta)

    c0 = msb.msb_create(L, N, N, bonds, U)
    c1 = msb.msb_create(L, N + 1, N, bonds, U)
    try:
        coef = np.zeros(L, dtype=np.complex128)
        coef[0] = 1.0
        Gt = torch.from_numpy(G.astype(np.complex128)).reshape(1, -1).cuda()
        Et = torch.empty(1, B1.dim, dtype=torch.complex128, device="cuda")
        msb.msb_dipole(c0, c1, 0, True, coef, Gt, Et)
        psi = torch.empty(1, len(w_in), B1.dim, dtype=torch.complex128, device="cuda")
        sysd = msb.make_system(core_site=0, Uc=Uc, E_G=E_G, Gamma=Gamma)
        msb.msb_solve(c1, [sysd], Et, w_in, 0.0, 1e-12, 3000, msb.MSB_C128, psi)
        phi = torch.empty(len(w_in), B0.dim, dtype=torch.complex128, device="cuda")
        msb.msb_dipole(c1, c0, 0, False, coef, psi[0].contiguous(), phi)
        I, _ = msb.msb_spectrum(c0, msb.make_system(E_G=E_G), phi, w, eta, 2000, 1e-13)
        p = psi[0].cpu().numpy()
        assert np.max(np.linalg.norm(p - psi_ref, axis=1) / np.linalg.norm(psi_ref, axis=1)) <= 1e-9
        assert np.max(np.abs(np.asarray(I) - I_ref)) <= 1e-8 * np.max(I_ref)
    finally:
        msb.msb_destroy(c0)
        msb.msb_destroy(c1)
