"""The stream argument of the C ABI (header: a stream of the library's own HIP
runtime or NULL; every call is ordered after the stream's queued work and
returns when its own work has completed).

The binding passes a ``LibStream`` handle through and turns a torch stream
into NULL after synchronising it (torch bundles a separate HIP runtime).
These tests call the ABI with a stream made by ``msb_stream_create`` and
check that the results are those of the NULL-stream calls, bit for bit, and
that they are complete when the call returns.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring(gpu):
    msb = gpu
    wl = W.get("tiny")
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    yield msb, ctx, wl
    msb.msb_destroy(ctx)


def test_library_stream_apply_matches_null_stream(ring):
    import torch
    msb, ctx, wl = ring
    D = msb.msb_dim(ctx)
    systems = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=-2.5, Gamma=wl.Gamma) for j in (0, 3)]
    x = torch.from_numpy(np.stack([W.random_complex(D, 200 + j) for j in range(2)])).cuda()
    y0 = torch.empty_like(x)
    msb.msb_apply(ctx, systems, 0.4, msb.MSB_C128, x, y0)
    torch.cuda.synchronize()
    with msb.LibStream() as s:
        for _ in range(3):
            y1 = torch.full_like(x, float("nan"))
            torch.cuda.synchronize()
            msb.msb_apply(ctx, systems, 0.4, msb.MSB_C128, x, y1, stream=s)
            # complete on return: read back with no further synchronisation
            assert torch.equal(y1, y0)


def test_library_stream_solve_and_spectrum_match_null_stream(ring):
    import torch
    msb, ctx, wl = ring
    D = msb.msb_dim(ctx)
    E = torch.from_numpy(W.random_complex(D, 210).reshape(1, D)).cuda()
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.6661474201323485, Gamma=wl.Gamma)
    w = wl.w_in[::8]
    psi0 = torch.empty(1, len(w), D, dtype=torch.complex128, device="cuda")
    _, info0 = msb.msb_solve(ctx, [sysd], E, w, 0.0, 1e-10, 3000, msb.MSB_C128, psi0, want_true=True)
    gs = msb.make_system(E_G=-2.6661474201323485)
    I0, d0 = msb.msb_spectrum(ctx, gs, psi0[0].contiguous(), wl.w_loss[::16], wl.eta, 400, 1e-10)
    with msb.LibStream() as s:
        psi1 = torch.full_like(psi0, float("nan"))
        torch.cuda.synchronize()
        _, info1 = msb.msb_solve(ctx, [sysd], E, w, 0.0, 1e-10, 3000, msb.MSB_C128, psi1, want_true=True,
                                 stream=s)
        assert torch.equal(psi1, psi0)
        assert np.array_equal(info1["resid_true"], info0["resid_true"])
        I1, d1 = msb.msb_spectrum(ctx, gs, psi1[0].contiguous(), wl.w_loss[::16], wl.eta, 400, 1e-10, stream=s)
        assert np.array_equal(I1, I0) and np.array_equal(d1, d0)


def test_stream_create_rejects_null(gpu):
    import ctypes
    msb = gpu
    assert msb.lib().msb_stream_create(None) == msb.MSB_EINVAL
    assert msb.lib().msb_stream_destroy(ctypes.c_void_p(0)) == msb.MSB_EINVAL
