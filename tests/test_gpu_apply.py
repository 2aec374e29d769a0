"""Parity of the matrix-free Hamiltonian apply (HIP) with the oracle's explicit sparse H.

The oracle builds H' from fermion operators on bit strings (no Kronecker
form); the GPU applies H_up (x) I + I (x) H_dn + diagonal.  Element-wise
agreement on random complex vectors pins the basis order, the Jordan-Wigner
signs, the bond amplitudes, the diagonal and the -E_G - i Gamma - shift terms.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hubbard as hb
from tests._cases import basis, oracle_H, small_models

pytestmark = pytest.mark.gpu

CASES = list(small_models().items())


@pytest.mark.parametrize("name,m", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_apply_matches_sparse_oracle(gpu, name, m, prec):
    import torch
    msb = gpu
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        systems = [
            msb.make_system(core_site=0, Uc=-4.0, E_G=-3.0, Gamma=1.0),
            msb.make_system(core_site=m["L"] - 1, Uc=-2.5, E_G=0.5, Gamma=0.25),
            msb.make_system(core_site=-1, E_G=0.0, Gamma=0.0),
        ]
        shift = 0.75
        x = np.stack([W.random_complex(D, seed=100 + s) for s in range(len(systems))])
        expect = []
        for s, sysd in enumerate(systems):
            H = oracle_H(m, core_site=sysd.core_site if sysd.core_site >= 0 else None, Uc=sysd.Uc)
            expect.append(H @ x[s] - (sysd.E_G + shift + 1j * sysd.Gamma) * x[s])
        expect = np.stack(expect)
        dt = torch.complex128 if prec == "c128" else torch.complex64
        xt = torch.from_numpy(x).to(dt).cuda().contiguous()
        yt = torch.empty_like(xt)
        msb.msb_apply(ctx, systems, shift, msb.MSB_C128 if prec == "c128" else msb.MSB_C64, xt, yt)
        torch.cuda.synchronize()
        y = yt.cpu().numpy().astype(np.complex128)
        if prec == "c64":
            # the c64 input is itself rounded: compare with the oracle applied to the rounded input
            xr = x.astype(np.complex64).astype(np.complex128)
            expect = np.stack([
                oracle_H(m, core_site=systems[s].core_site if systems[s].core_site >= 0 else None,
                         Uc=systems[s].Uc) @ xr[s]
                - (systems[s].E_G + shift + 1j * systems[s].Gamma) * xr[s] for s in range(len(systems))])
        err = np.max(np.abs(y - expect)) / np.max(np.abs(expect))
        tol = 1e-14 if prec == "c128" else 2e-6
        assert err <= tol, f"{name} {prec}: rel err {err:.3e}"
    finally:
        msb.msb_destroy(ctx)


@pytest.mark.parametrize("wl_name", ["scale", "precision", "batched"])
def test_apply_full_size_sampled_rows(gpu, wl_name):
    """At the workloads' full sizes: sampled rows against the oracle's row-by-row apply."""
    import torch
    msb = gpu
    wl = W.get(wl_name)
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        assert D == wl.dim
        B = basis(wl.n_sites, wl.n_up, wl.n_dn)
        rng = np.random.default_rng(7)
        rows = np.unique(np.concatenate([rng.integers(0, D, 400), [0, 1, D - 2, D - 1]]))
        sysd = msb.make_system(core_site=wl.core_sites[-1], Uc=wl.Uc, E_G=-4.0, Gamma=wl.Gamma)
        prec = msb.MSB_C128 if wl.dtype == "c128" else msb.MSB_C64
        dt = torch.complex128 if prec == msb.MSB_C128 else torch.complex64
        g = torch.Generator(device="cuda").manual_seed(11)
        xt = torch.randn(D, dtype=dt, device="cuda", generator=g)
        yt = torch.empty_like(xt)
        msb.msb_apply(ctx, [sysd], 0.0, prec, xt, yt)
        torch.cuda.synchronize()
        x = xt.cpu().numpy().astype(np.complex128)
        y = yt.cpu().numpy().astype(np.complex128)
        ref = hb.apply_rows(B, wl.bonds, wl.U, x, rows, core_site=sysd.core_site, Uc=sysd.Uc,
                            shift=sysd.E_G + 1j * sysd.Gamma)
        err = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
        tol = 1e-14 if prec == msb.MSB_C128 else 2e-6
        assert err <= tol, f"{wl_name}: sampled rel err {err:.3e}"
    finally:
        msb.msb_destroy(ctx)
