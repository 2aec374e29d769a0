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
