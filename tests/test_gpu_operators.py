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
