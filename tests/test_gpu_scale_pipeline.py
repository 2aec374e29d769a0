"""The scale workload end to end (L = 12 ring, N = 6 + 6, D = 853,776, the 12
core-hole sites x 200 incident energies) at its stated stopping residual 1e-10,
and the continued-fraction spectrum at that size.

Pins at a size the oracle cannot solve whole:

* the solve: the library's FP64 true residuals and the oracle's row-by-row
  operator on sampled rows of sampled (site, shift) pairs, both <= 1e-10 |E|;
* the spectrum's continued fraction: its first Lanczos coefficients (a_0 and
  b_0^2, b_1^2 are the spectral moments) against the oracle's Lanczos on the
  oracle's sparse H, from seeded random vectors;
* the spectrum against its definition (Eq. kramers1): correction vectors
  x(w) = (H - E_G - w - i eta)^{-1} phi from the multi-shift solve, whose
  residuals the oracle checks on sampled rows, give I(w) = Im phi^H x / pi to
  within |phi| |r| / (pi eta) (the resolvent of a real symmetric H has norm
  <= 1/eta);
* chain reflection j -> -j maps the core-hole sum with phases e^{iqj} onto
  the one with e^{-iqj}, so I(q) = I(-q).
"""
import numpy as np
import pytest

import workloads as W
from oracle import hubbard as hb
from oracle import spectrum as ospec
from tests._cases import basis

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def scale(gpu):
    import torch
    msb = gpu
    wl = W.get("scale")
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    D = msb.msb_dim(ctx)
    x0 = torch.from_numpy(W.random_vector(D, wl.gs_seed)).cuda()
    G = torch.empty(D, dtype=torch.float64, device="cuda")
    E_G, _ = msb.msb_ground_state(ctx, msb.make_system(), x0, 1e-11, 600, G)
    E = G.to(torch.complex128).reshape(1, D).repeat(wl.nrhs, 1).contiguous()   # O2 = identity
    systems = [msb.make_system(core_site=c, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for c in wl.core_sites]
    psi = torch.empty(wl.nrhs, len(wl.w_in), D, dtype=torch.complex128, device="cuda")
    st, info = msb.msb_solve(ctx, systems, E, wl.w_in, wl.seed_shift, TOL, wl.maxit, msb.MSB_C128, psi,
                             want_true=True, raise_on_fail=False)
    yield msb, ctx, wl, E_G, E, systems, psi, st, info
    del psi
    msb.msb_destroy(ctx)


def test_scale_solve_meets_1e10(scale):
    msb, ctx, wl, E_G, E, systems, psi, st, info = scale
    assert st == msb.MSB_OK
    assert np.all(info["shift_iters"] > 0)
    assert np.max(info["resid_true"]) <= 1.01 * TOL
    B = basis(wl.n_sites, wl.n_up, wl.n_dn)
    D = B.dim
    rng = np.random.default_rng(23)
    rows = np.unique(np.concatenate([rng.integers(0, D, 200), [0, D - 1]]))
    n = len(wl.w_in)
    for s in (0, 5, 11):
        Es = E[s].cpu().numpy()
        nE = np.linalg.norm(Es)
        for k in (0, n // 4, n // 2, 3 * n // 4, n - 1):
            ps = psi[s, k].cpu().numpy()
            Ax = hb.apply_rows(B, wl.bonds, wl.U, ps, rows, core_site=systems[s].core_site, Uc=wl.Uc,
                               shift=E_G + wl.w_in[k] + 1j * wl.Gamma)
            assert np.max(np.abs(Es[rows] - Ax)) <= 1.01 * TOL * nE, (s, k)


def _phi(msb, ctx, wl, psi, sub, phases):
    import torch
    D = msb.msb_dim(ctx)
    ps = psi[:, torch.as_tensor(sub, device=psi.device)].contiguous()
    phi = torch.empty(len(sub), D, dtype=torch.complex128, device=psi.device)
    msb.msb_combine(ctx, ps, wl.nrhs, len(sub), msb.MSB_C128, phases, phi)
    return phi


def test_scale_spectrum_reflection_symmetry(scale):
    """I(q) = I(-q) on every loss of four incident energies."""
    msb, ctx, wl, E_G, E, systems, psi, st, info = scale
    n = len(wl.w_in)
    sub = [n // 8, 3 * n // 8, n // 2, 7 * n // 8]
    gs = msb.make_system(E_G=E_G)
    I_p, _ = msb.msb_spectrum(ctx, gs, _phi(msb, ctx, wl, psi, sub, wl.phases), wl.w_loss, wl.eta, 3000, 1e-12)
    I_m, _ = msb.msb_spectrum(ctx, gs, _phi(msb, ctx, wl, psi, sub, [np.conj(p) for p in wl.phases]),
                              wl.w_loss, wl.eta, 3000, 1e-12)
    peak = np.max(I_p, axis=1)
    assert np.all(peak > 0)
    assert np.max(np.abs(I_p - I_m) / peak[:, None]) <= 1e-8
    assert np.all(I_p >= -1e-10 * peak[:, None])


def test_scale_spectrum_matches_correction_vectors(scale):
    """The continued fraction of one phi = sum_j e^{iqj} Psi_j against the
    correction vectors of the same phi on all 256 losses."""
    import torch
    msb, ctx, wl, E_G, E, systems, psi, st, info = scale
    D = msb.msb_dim(ctx)
    n = len(wl.w_in)
    phi = _phi(msb, ctx, wl, psi, [n // 2], wl.phases)
    gs = msb.make_system(E_G=E_G)
    I_cf, _ = msb.msb_spectrum(ctx, gs, phi, wl.w_loss, wl.eta, 3000, 1e-12)
    # x(w) = (H - E_G - w - i eta)^{-1} phi: the losses as shifts, and phi's
    # real and imaginary parts as two right-hand sides (the complex-symmetric
    # iteration starts from rho = E^T E, which a complex phi can make tiny)
    cv_sys = msb.make_system(core_site=-1, E_G=E_G, Gamma=wl.eta)
    parts = torch.stack([phi[0].real, phi[0].imag]).to(torch.complex128).contiguous()
    x = torch.empty(2, len(wl.w_loss), D, dtype=torch.complex128, device="cuda")
    st_cv, info_cv = msb.msb_solve(ctx, [cv_sys, cv_sys], parts, wl.w_loss, 5.0, TOL, 6000, msb.MSB_C128, x,
                                   want_true=True)
    r_max = float(np.max(info_cv["resid_true"]))
    assert r_max <= 1.01 * TOL
    # the residual of the correction vectors, checked by the oracle on sampled rows
    B = basis(wl.n_sites, wl.n_up, wl.n_dn)
    rows = np.unique(np.random.default_rng(29).integers(0, D, 150))
    for part in range(2):
        rhs = parts[part].cpu().numpy()
        for k in (0, 60, 128, 255):
            xk = x[part, k].cpu().numpy()
            Ax = hb.apply_rows(B, wl.bonds, wl.U, xk, rows, shift=E_G + wl.w_loss[k] + 1j * wl.eta)
            assert np.max(np.abs(rhs[rows] - Ax)) <= 1.01 * TOL * np.linalg.norm(rhs), (part, k)
    xphi = (x[0] + 1j * x[1]).contiguous()
    I_cv = (torch.mv(xphi, phi[0].conj().resolve_conj()).imag / np.pi).cpu().numpy()
    nphi = float(torch.linalg.vector_norm(phi[0]).item())
    nre = float(torch.linalg.vector_norm(parts[0]).item())
    nim = float(torch.linalg.vector_norm(parts[1]).item())
    # |x - x*| <= |r| / eta for each part (the resolvent of a real symmetric H
    # has norm <= 1/eta), and |I - I*| <= |phi| |x - x*| / pi
    bound = nphi * r_max * (nre + nim) / (np.pi * wl.eta)
    peak = np.max(I_cf)
    assert np.max(np.abs(I_cf[0] - I_cv)) <= bound + 1e-10 * peak, (np.max(np.abs(I_cf[0] - I_cv)), bound, peak)


def test_scale_cf_coefficients_match_oracle_lanczos(scale):
    """First 40 continued-fraction coefficients from seeded random vectors:
    b_0 = |phi|, a_0 = <phi|H|phi> / |phi|^2 and the rest against the oracle's
    Lanczos on its sparse H."""
    import torch
    msb, ctx, wl, E_G, E, systems, psi, st, info = scale
    D = msb.msb_dim(ctx)
    phis = np.stack([W.random_complex(D, 400 + j) * (1.0 + j) for j in range(2)])
    ld = 40
    _, depth, a, b = msb.msb_spectrum_cf(ctx, msb.make_system(E_G=E_G), torch.from_numpy(phis).cuda(),
                                         wl.w_loss, wl.eta, 3000, 1e-10, ld)
    assert np.all(depth >= ld)
    B = basis(wl.n_sites, wl.n_up, wl.n_dn)
    H = hb.hamiltonian(B, wl.bonds, wl.U).astype(np.complex128).tocsr()
    for j in range(2):
        ao, bo, norm = ospec.lanczos_tridiag(H, phis[j], ld)
        assert abs(b[j, 0] - norm) <= 1e-13 * norm
        assert abs(a[j, 0] - np.real(np.vdot(phis[j], H @ phis[j])) / norm ** 2) <= 1e-12 * np.max(np.abs(ao))
        assert np.max(np.abs(a[j] - ao[:ld])) <= 1e-10 * np.max(np.abs(ao))
        assert np.max(np.abs(b[j, 1:] - bo[:ld - 1])) <= 1e-10 * np.max(bo)
