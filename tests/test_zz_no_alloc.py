"""The allocation-free apply (msb_apply_noalloc) against msb_apply.

Two calls in a row through the C ABI, the second with fewer systems (the
staging array keeps the first call's contents beyond the second's range),
each compared with msb_apply on the same inputs; sizes beyond the staging
array's limit are refused before any device work.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _systems(msb, wl, n, E_G):
    return [msb.make_system(core_site=j % wl.n_sites, Uc=wl.Uc - 0.5 * (j // wl.n_sites), E_G=E_G,
                            Gamma=wl.Gamma + 0.1 * j) for j in range(n)]


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_apply_matches_apply(gpu, prec):
    import torch
    msb = gpu
    wl = W.get("tiny")
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        p = msb.MSB_C128 if prec == "c128" else msb.MSB_C64
        dt = torch.complex128 if prec == "c128" else torch.complex64
        tol = 1e-14 if prec == "c128" else 2e-6
        for n, seed in ((11, 300), (3, 301)):             # second call: a smaller input
            systems = _systems(msb, wl, n, -2.66 + 0.01 * seed)
            x = torch.from_numpy(np.stack([W.random_complex(D, seed + j) for j in range(n)])).to(dt).cuda()
            y_ref = torch.empty_like(x)
            y = torch.full_like(x, float("nan"))
            msb.msb_apply_noalloc(ctx, systems, 0.25, p, x, y)
            msb.msb_apply(ctx, systems, 0.25, p, x, y_ref)
            torch.cuda.synchronize()
            a, b = y.cpu().numpy(), y_ref.cpu().numpy()
            assert np.all(np.isfinite(a))
            err = np.max(np.abs(a - b)) / np.max(np.abs(b))
            assert err <= tol, (n, err)
    finally:
        msb.msb_destroy(ctx)


def test_noalloc_apply_rejects_too_many_systems(gpu):
    import torch
    msb = gpu
    wl = W.get("tiny")
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        n = 1025                                          # MSB_NOALLOC_MAX_SYS + 1
        systems = [msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.0, Gamma=1.0)] * n
        x = torch.zeros(n, D, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        with pytest.raises(msb.MsbError) as e:
            msb.msb_apply_noalloc(ctx, systems, 0.0, msb.MSB_C64, x, y)
        assert e.value.status == msb.MSB_EINVAL
        assert "1024" in e.value.message
    finally:
        msb.msb_destroy(ctx)
