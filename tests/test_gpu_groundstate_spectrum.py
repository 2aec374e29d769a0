"""Parity of the ground-state Lanczos and the continued-fraction spectrum (HIP)
with the oracle's dense diagonalisation and Lehmann sum."""
import numpy as np
import pytest

import workloads as W
from oracle import groundstate as ogs
from oracle import spectrum as ospec
from tests._cases import oracle_H, small_models

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["chain6", "chain8", "chain8_doped", "square3x3"])
def test_ground_state_matches_dense(gpu, name):
    import torch
    msb = gpu
    m = small_models()[name]
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        x0 = W.random_vector(D, 12345)
        H = oracle_H(m)
        E_ref, G_ref, ev = ogs.dense_ground_state(H)
        if ev[1] - ev[0] < 1e-8:
            # degenerate: only the energy and the eigenspace are unique; a
            # Krylov space from x0 meets that space in the direction P x0
            ew, V = np.linalg.eigh(H.toarray())
            Vg = V[:, ew - ew[0] < 1e-8]
            G_ref = Vg @ (Vg.T @ x0)
            G_ref /= np.linalg.norm(G_ref)
        x0t = torch.from_numpy(x0).cuda()
        G = torch.empty(D, dtype=torch.float64, device="cuda")
        E_G, iters = msb.msb_ground_state(ctx, msb.make_system(), x0t, 1e-11, 600, G)
        g = G.cpu().numpy()
        assert abs(E_G - E_ref) <= 1e-12 * abs(E_ref), (E_G, E_ref)
        assert abs(np.dot(g, G_ref)) >= 1 - 1e-12
        assert np.dot(x0, g) >= 0
        assert abs(np.linalg.norm(g) - 1) < 1e-13
    finally:
        msb.msb_destroy(ctx)


def test_spectrum_matches_lehmann(gpu):
    import torch
    msb = gpu
    wl = W.get("tiny")
    m = dict(L=wl.n_sites, nu=wl.n_up, nd=wl.n_dn, bonds=wl.bonds, U=wl.U)
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        H = oracle_H(m).toarray()
        evals, evecs = np.linalg.eigh(H)
        E_G = evals[0]
        phi = np.stack([W.random_complex(D, 70 + k) for k in range(6)])
        phi[1] *= 1e-3                      # different norms
        ref = ospec.lehmann(evals, evecs, phi, E_G, wl.w_loss, wl.eta)
        phit = torch.from_numpy(phi).cuda()
        I, depth = msb.msb_spectrum(ctx, msb.make_system(E_G=E_G), phit, wl.w_loss, wl.eta, 2000,
                                    1e-13)
        err = np.max(np.abs(I - ref)) / np.max(np.abs(ref))
        assert err <= 1e-10, f"spectrum rel err {err:.3e}, depth {depth}"
        assert np.all(I > -1e-12 * np.max(ref))
    finally:
        msb.msb_destroy(ctx)


def test_tiny_pipeline_end_to_end_at_1e10(gpu):
    """The tiny workload whole, on its own inputs: GPU Lanczos ground state
    from the seeded start, E = G, all 64 incident energies at tol 1e-13, the
    continued fraction on all 256 losses -- against dense eigh, the exact
    solves and the Lehmann sum of the oracle (its own ground state, aligned in
    sign), to 1e-10 relative."""
    import torch
    from oracle import solve as osolve
    msb = gpu
    wl = W.get("tiny")
    m = dict(L=wl.n_sites, nu=wl.n_up, nd=wl.n_dn, bonds=wl.bonds, U=wl.U)
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        x0 = torch.from_numpy(W.random_vector(D, wl.gs_seed)).cuda()
        G = torch.empty(D, dtype=torch.float64, device="cuda")
        E_G, _ = msb.msb_ground_state(ctx, msb.make_system(), x0, 1e-13, 1000, G)
        E = G.to(torch.complex128).reshape(1, D).contiguous()
        sysd = msb.make_system(core_site=wl.core_sites[0], Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
        psi = torch.empty(1, len(wl.w_in), D, dtype=torch.complex128, device="cuda")
        _, info = msb.msb_solve(ctx, [sysd], E, wl.w_in, 0.0, 1e-13, 3000, msb.MSB_C128, psi, want_true=True)
        phi = torch.empty(len(wl.w_in), D, dtype=torch.complex128, device="cuda")
        msb.msb_combine(ctx, psi, 1, len(wl.w_in), msb.MSB_C128, [1.0], phi)
        I, _ = msb.msb_spectrum(ctx, msb.make_system(E_G=E_G), phi, wl.w_loss, wl.eta, 3000, 1e-13)

        H = oracle_H(m).toarray()
        ev, V = np.linalg.eigh(H)
        # the oracle's own ground state, signed as the library signs G: <x0|G> >= 0
        G_ref = V[:, 0] * np.sign(np.dot(W.random_vector(D, wl.gs_seed), V[:, 0]))
        assert abs(E_G - ev[0]) <= 1e-12 * abs(ev[0])
        Hp = oracle_H(m, core_site=wl.core_sites[0], Uc=wl.Uc)
        ref_psi = osolve.direct_solve(Hp, G_ref.astype(complex), ev[0], wl.Gamma, wl.w_in, method="eig")
        p = psi[0].cpu().numpy()
        err_psi = np.linalg.norm(p - ref_psi, axis=1) / np.linalg.norm(ref_psi, axis=1)
        assert err_psi.max() <= 1e-10, err_psi.max()
        assert np.max(info["resid_true"]) <= 1e-12
        ref_I = ospec.lehmann(ev, V, ref_psi, ev[0], wl.w_loss, wl.eta)
        err_I = np.max(np.abs(I - ref_I)) / np.max(np.abs(ref_I))
        assert err_I <= 1e-10, err_I
    finally:
        msb.msb_destroy(ctx)
