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


WIDE = {
    # long down-spin rows (n_dn = 924, 3432, 4368) with few up-spin rows,
    # so the 1024-thread shapes are exercised at sizes the oracle builds quickly
    "chain12_2_6": dict(L=12, nu=2, nd=6, bonds=W.chain_bonds(12, 1.0), U=8.0),
    "chain14_1_7_tp": dict(L=14, nu=1, nd=7, bonds=W.chain_bonds(14, 1.0, -0.2), U=8.0),
    "square4x4_1_5": dict(L=16, nu=1, nd=5, bonds=W.square_bonds(4, 4, 1.0, -0.25), U=8.0),
    "chain8": dict(L=8, nu=4, nd=4, bonds=W.chain_bonds(8, 1.0), U=8.0),
}


@pytest.mark.parametrize("name", list(WIDE))
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_every_apply_shape_matches_oracle(gpu, name, prec):
    """Every launch shape the autotuner may pick gives the oracle's H x (1, 3
    and 4 systems per call: full and ragged system groups)."""
    import torch
    msb = gpu
    m = WIDE[name]
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    p = msb.MSB_C128 if prec == "c128" else msb.MSB_C64
    dt = torch.complex128 if prec == "c128" else torch.complex64
    try:
        D = msb.msb_dim(ctx)
        all_sys = [msb.make_system(core_site=j % m["L"], Uc=-4.0 + 0.5 * j, E_G=-3.0 + j, Gamma=1.0 + 0.1 * j)
                   for j in range(4)]
        shift = 0.25
        x = np.stack([W.random_complex(D, seed=300 + s) for s in range(4)])
        xr = x.astype(np.complex64).astype(np.complex128) if prec == "c64" else x
        expect = np.stack([oracle_H(m, core_site=s.core_site, Uc=s.Uc) @ xr[j]
                           - (s.E_G + shift + 1j * s.Gamma) * xr[j] for j, s in enumerate(all_sys)])
        tol = 1e-14 if prec == "c128" else 2e-6
        seen = set()
        for nsys in (1, 3, 4):
            table = msb.msb_autotune(ctx, nsys, p)
            assert table and all(t[5] > 0 for t in table)
            assert {t[3] for t in table} == {1, 2, 3}       # single-pass, L2- and LDS-panel two-pass forms
            assert {t[4] for t in table} == {0, 1}          # both row orders
            for shape in table:
                msb.msb_set_shape(ctx, nsys, p, shape)
                xt = torch.from_numpy(x[:nsys]).to(dt).cuda().contiguous()
                yt = torch.full_like(xt, float("nan"))
                msb.msb_apply(ctx, all_sys[:nsys], shift, p, xt, yt)
                torch.cuda.synchronize()
                y = yt.cpu().numpy().astype(np.complex128)
                err = np.max(np.abs(y - expect[:nsys])) / np.max(np.abs(expect[:nsys]))
                assert err <= tol, f"{name} {prec} nsys={nsys} shape={shape[:5] + shape[6:]}: {err:.3e}"
                seen.add(shape[:5] + shape[6:])
            msb.msb_set_shape(ctx, nsys, p, None)
        assert len(seen) >= 2
        with pytest.raises(msb.MsbError):
            msb.msb_set_shape(ctx, 1, p, (512, 3, 1))      # not a compiled shape
    finally:
        msb.msb_destroy(ctx)


def test_longest_row_and_the_lds_limit(gpu):
    """The longest down-spin row one workgroup can stage: L = 16, N_dn = 8
    (12,870 states, 103 KB in complex64) applies correctly in complex64 and is
    refused in complex128 (206 KB would exceed the 160 KB of LDS)."""
    import torch
    msb = gpu
    m = dict(L=16, nu=1, nd=8, bonds=W.square_bonds(4, 4, 1.0, -0.25), U=8.0)
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        assert D == 16 * 12870
        s = msb.make_system(core_site=3, Uc=-4.0, E_G=-2.0, Gamma=1.0)
        x = W.random_complex(D, 77)
        xt = torch.from_numpy(x).to(torch.complex64).cuda()
        yt = torch.empty_like(xt)
        msb.msb_apply(ctx, [s], 0.0, msb.MSB_C64, xt, yt)
        torch.cuda.synchronize()
        xr = x.astype(np.complex64).astype(np.complex128)
        ref = oracle_H(m, core_site=3, Uc=-4.0) @ xr - (-2.0 + 1j) * xr
        got = yt.cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))
        x2 = torch.from_numpy(x).cuda()
        with pytest.raises(msb.MsbError):
            msb.msb_apply(ctx, [s], 0.0, msb.MSB_C128, x2, torch.empty_like(x2))
    finally:
        msb.msb_destroy(ctx)


def test_one_state_spin_sector(gpu):
    """N_up = 0: a single up-spin configuration (no up hops, one row)."""
    import torch
    msb = gpu
    m = dict(L=6, nu=0, nd=3, bonds=W.chain_bonds(6, 1.0, -0.3), U=8.0)
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        assert D == 20
        s = msb.make_system(core_site=1, Uc=-4.0, E_G=-1.0, Gamma=0.5)
        x = W.random_complex(D, 78)
        xt = torch.from_numpy(x).cuda()
        yt = torch.empty_like(xt)
        msb.msb_apply(ctx, [s], 0.25, msb.MSB_C128, xt, yt)
        torch.cuda.synchronize()
        ref = oracle_H(m, core_site=1, Uc=-4.0) @ x - (-1.0 + 0.25 + 0.5j) * x
        assert np.max(np.abs(yt.cpu().numpy() - ref)) <= 1e-14 * np.max(np.abs(ref))
    finally:
        msb.msb_destroy(ctx)


@pytest.mark.parametrize("name,m", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("group,nsys", [(2, 3), (4, 5), (4, 4)])
def test_block_apply_matches_sparse_oracle(gpu, name, m, prec, group, nsys):
    """The interleaved block apply (msb_apply_block) against the oracle's
    explicit H' on every system of ragged and whole groups; per-system core
    holes, broadenings and one system with its own U and bond amplitudes."""
    import torch
    msb = gpu
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        n_types = msb.msb_sector_info(ctx)[2]
        systems = []
        for s in range(nsys):
            if s == 1:
                amps = [0.7 + 0.1 * t for t in range(n_types)]
                systems.append(msb.make_system(core_site=s % m["L"], Uc=-3.0, E_G=-1.0, Gamma=0.6, U=5.5,
                                               t_amp=amps))
            else:
                systems.append(msb.make_system(core_site=(s * 3) % m["L"], Uc=-4.0 + 0.5 * s, E_G=-2.0 + s,
                                               Gamma=1.0 / (s + 1)))
        shift = -0.3
        x = np.stack([W.random_complex(D, seed=300 + s) for s in range(nsys)])
        if prec == "c64":
            x = x.astype(np.complex64).astype(np.complex128)      # the rounded input is the input
        expect = []
        bond_types = []
        for b in m["bonds"]:
            if b[2] not in bond_types:
                bond_types.append(b[2])
        for s, sysd in enumerate(systems):
            bonds = m["bonds"]
            U = m["U"]
            if s == 1:
                amp = {t: 0.7 + 0.1 * k for k, t in enumerate(bond_types)}
                bonds = [(i, j, amp[t]) for (i, j, t) in m["bonds"]]
                U = 5.5
            B = basis(m["L"], m["nu"], m["nd"])
            H = hb.hamiltonian(B, bonds, U, core_site=sysd.core_site, Uc=sysd.Uc)
            expect.append(H @ x[s] - (sysd.E_G + shift + 1j * sysd.Gamma) * x[s])
        expect = np.stack(expect)
        ng = (nsys + group - 1) // group
        xi = np.zeros((ng * group, D), dtype=np.complex128)
        xi[:nsys] = x
        xi = xi.reshape(ng, group, D).transpose(0, 2, 1).copy()          # [group][D][g]
        dt = torch.complex128 if prec == "c128" else torch.complex64
        xt = torch.from_numpy(xi).to(dt).cuda().contiguous()
        yt = torch.full_like(xt, float("nan"))
        p = msb.MSB_C128 if prec == "c128" else msb.MSB_C64
        msb.msb_apply_block(ctx, systems, shift, p, group, xt, yt)
        torch.cuda.synchronize()
        y = yt.cpu().numpy().astype(np.complex128).transpose(0, 2, 1).reshape(ng * group, D)[:nsys]
        err = np.max(np.abs(y - expect)) / np.max(np.abs(expect))
        tol = 1e-14 if prec == "c128" else 2e-6
        assert err <= tol, f"{name} {prec} group {group}: rel err {err:.3e}"
    finally:
        msb.msb_destroy(ctx)


PANEL = {
    # large up-spin sectors (the whole column panel, n_up rows, staged in one
    # workgroup's LDS) and an odd row length (no whole 16-byte units in
    # complex64: the element-wise staging path)
    "square4x4_5_1": dict(L=16, nu=5, nd=1, bonds=W.square_bonds(4, 4, 1.0, -0.25), U=8.0),
    "chain14_7_1": dict(L=14, nu=7, nd=1, bonds=W.chain_bonds(14, 1.0, -0.2), U=8.0),
    "chain7_3_3": dict(L=7, nu=3, nd=3, bonds=W.chain_bonds(7, 1.0), U=8.0),
    # odd rows (91 states) under a large up-spin sector: complex64 panels
    # take the element-wise staging path
    "chain14_7_2": dict(L=14, nu=7, nd=2, bonds=W.chain_bonds(14, 1.0), U=8.0),
    # three bond types (third neighbours added): the per-type panel table,
    # not the hop-count-ordered one (built for at most two types)
    "chain12_6_1_t3": dict(L=12, nu=6, nd=1, U=8.0,
                           bonds=W.chain_bonds(12, 1.0, -0.2) + [(i, (i + 3) % 12, 0.07) for i in range(12)]),
}


@pytest.mark.parametrize("name", list(PANEL))
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_lds_panel_pass_matches_oracle(gpu, name, prec):
    """Every LDS column-panel shape (passes = 3) gives the oracle's H x, for 1
    and 3 systems, at up-spin sectors of 4,368 and 3,432 rows and on rows of
    odd length."""
    import torch
    msb = gpu
    m = PANEL[name]
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    p = msb.MSB_C128 if prec == "c128" else msb.MSB_C64
    dt = torch.complex128 if prec == "c128" else torch.complex64
    try:
        D = msb.msb_dim(ctx)
        all_sys = [msb.make_system(core_site=(3 * j) % m["L"], Uc=-4.0 + 0.5 * j, E_G=-2.0 + j, Gamma=1.0 + 0.1 * j)
                   for j in range(3)]
        shift = -0.5
        x = np.stack([W.random_complex(D, seed=700 + s) for s in range(3)])
        xr = x.astype(np.complex64).astype(np.complex128) if prec == "c64" else x
        expect = np.stack([oracle_H(m, core_site=s.core_site, Uc=s.Uc) @ xr[j]
                           - (s.E_G + shift + 1j * s.Gamma) * xr[j] for j, s in enumerate(all_sys)])
        tol = 1e-14 if prec == "c128" else 2e-6
        n_panel = 0
        for nsys in (1, 3):
            table = [t for t in msb.msb_autotune(ctx, nsys, p) if t[3] == 3]
            assert table, "no LDS panel shape offered"
            assert all(t[6] > 0 for t in table)
            for shape in table:
                msb.msb_set_shape(ctx, nsys, p, shape)
                xt = torch.from_numpy(x[:nsys]).to(dt).cuda().contiguous()
                yt = torch.full_like(xt, float("nan"))
                msb.msb_apply(ctx, all_sys[:nsys], shift, p, xt, yt)
                torch.cuda.synchronize()
                y = yt.cpu().numpy().astype(np.complex128)
                err = np.max(np.abs(y - expect[:nsys])) / np.max(np.abs(expect[:nsys]))
                assert err <= tol, f"{name} {prec} nsys={nsys} shape={shape[:5] + shape[6:]}: {err:.3e}"
                n_panel += 1
            msb.msb_set_shape(ctx, nsys, p, None)
        assert n_panel >= 2
    finally:
        msb.msb_destroy(ctx)


@pytest.mark.parametrize("wl_name", ["precision", "batched"])
def test_lds_panel_pass_full_size_sampled_rows(gpu, wl_name):
    """The fastest LDS column-panel shape at the full L = 14 and 4x4 sizes:
    sampled rows against the oracle's row-by-row apply (the 4x4 block of four
    systems, complex64)."""
    import torch
    msb = gpu
    wl = W.get(wl_name)
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        nsys = 4 if wl_name == "batched" else 1
        prec = msb.MSB_C64
        table = [t for t in msb.msb_autotune(ctx, nsys, prec) if t[3] == 3]
        assert table
        best = min(table, key=lambda t: t[5])
        msb.msb_set_shape(ctx, nsys, prec, best)
        B = basis(wl.n_sites, wl.n_up, wl.n_dn)
        rng = np.random.default_rng(17)
        rows = np.unique(np.concatenate([rng.integers(0, D, 300), [0, 1, D - 2, D - 1]]))
        systems = [msb.make_system(core_site=wl.core_sites[j % len(wl.core_sites)], Uc=wl.Uc, E_G=-4.0 + 0.1 * j,
                                   Gamma=wl.Gamma) for j in range(nsys)]
        g = torch.Generator(device="cuda").manual_seed(23)
        xt = torch.randn(nsys, D, dtype=torch.complex64, device="cuda", generator=g)
        yt = torch.empty_like(xt)
        msb.msb_apply(ctx, systems, 0.0, prec, xt, yt)
        torch.cuda.synchronize()
        for j in (0, nsys - 1):
            x = xt[j].cpu().numpy().astype(np.complex128)
            y = yt[j].cpu().numpy().astype(np.complex128)
            s = systems[j]
            ref = hb.apply_rows(B, wl.bonds, wl.U, x, rows, core_site=s.core_site, Uc=s.Uc,
                                shift=s.E_G + 1j * s.Gamma)
            err = np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))
            assert err <= 2e-6, f"{wl_name} system {j} shape {best[:5] + best[6:]}: sampled rel err {err:.3e}"
        msb.msb_set_shape(ctx, nsys, prec, None)
    finally:
        msb.msb_destroy(ctx)
