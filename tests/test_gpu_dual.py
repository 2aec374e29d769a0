"""Non-symmetric H' (directed, non-reciprocal bonds) and the dual-space form
of the multi-shift solve, against the oracle's explicit matrices and direct
solves."""
import numpy as np
import pytest

import workloads as W
from oracle import hubbard as hb
from oracle import solve as osolve

pytestmark = pytest.mark.gpu

L, N, G_ = 8, 4, 0.3


def _bonds(g):
    return [(i, (i + 1) % L, np.exp(g), np.exp(-g)) for i in range(L)]


@pytest.fixture(scope="module")
def directed(gpu):
    """Context of the ring with one directed bond class (types 0: i -> i+1,
    1: back); the model itself is symmetric (g = 0), systems make it not."""
    msb = gpu
    ctx = msb.msb_create(L, N, N, _bonds(0.0), 8.0)
    yield msb, ctx, hb.Basis(L, N, N)
    msb.msb_destroy(ctx)


def _sys(msb, g, **kw):
    return msb.make_system(t_amp=[np.exp(g), np.exp(-g)], **kw)


def test_directed_apply_matches_oracle(directed):
    import torch
    msb, ctx, B = directed
    H = hb.hamiltonian(B, _bonds(G_), 8.0, core_site=2, Uc=-4.0)
    x = np.stack([W.random_complex(B.dim, 40 + k) for k in range(3)])
    systems = [_sys(msb, G_, core_site=2, Uc=-4.0, E_G=-3.0, Gamma=1.0),
               _sys(msb, -G_, core_site=2, Uc=-4.0, E_G=-3.0, Gamma=1.0),     # = the transpose
               _sys(msb, G_, core_site=2, Uc=-4.0, E_G=-3.0, Gamma=1.0)]
    xt = torch.from_numpy(x).cuda()
    yt = torch.empty_like(xt)
    msb.msb_apply(ctx, systems, 0.5, msb.MSB_C128, xt, yt)
    y = yt.cpu().numpy()
    c = -3.0 + 0.5 + 1j
    HT = H.T.tocsr()
    for k, M in enumerate([H, HT, H]):
        ref = M @ x[k] - c * x[k]
        assert np.max(np.abs(y[k] - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_dual_space_solve_matches_direct(directed):
    msb, ctx, B = directed
    from tests.test_gpu_solve import _run
    H = hb.hamiltonian(B, _bonds(G_), 8.0, core_site=0, Uc=-4.0)
    E = W.random_complex(B.dim, 3)
    w = np.linspace(-6.0, 6.0, 16)
    ref = osolve.direct_solve(H, E, -3.0, 1.0, w, method="lu")
    sysd = _sys(msb, G_, core_site=0, Uc=-4.0, E_G=-3.0, Gamma=1.0)
    st, info, psi = _run(msb, ctx, [sysd], E, w, 1e-13, 3000, msb.MSB_C128)
    err = np.max(np.linalg.norm(psi[0] - ref, axis=1) / np.linalg.norm(ref, axis=1))
    assert err <= 1e-10, err
    assert np.max(info["resid_true"]) <= 1e-11
    assert info["mvms"] == 2 * info["iters"]                 # A and A^T per iteration
    # the oracle's dual-space recurrence needs about as many iterations
    A = lambda v: H @ v - (-3.0 + 1j) * v                     # noqa: E731
    AT = lambda v: H.T @ v - (-3.0 + 1j) * v                  # noqa: E731
    res = osolve.msbicg_reference(A, E, w, 1e-13, 3000, AT_apply=AT)
    assert abs(res.iters - info["iters"]) <= max(3, 0.03 * res.iters)


def test_dual_space_form_on_symmetric_system_is_identical(directed):
    msb, ctx, B = directed
    from tests.test_gpu_solve import _run
    E = W.random_complex(B.dim, 6)
    w = np.linspace(-6.0, 6.0, 16)
    sysd = _sys(msb, 0.0, core_site=0, Uc=-4.0, E_G=-3.0, Gamma=1.0)
    # the dual form applies A to p_m itself, as the direct COCG form does
    _, i1, p1 = _run(msb, ctx, [sysd], E, w, 1e-12, 3000, msb.MSB_C128, opts={"direct_ap": 1})
    _, i2, p2 = _run(msb, ctx, [sysd], E, w, 1e-12, 3000, msb.MSB_C128, opts={"dual": 1})
    assert i1["iters"] == i2["iters"] and i2["mvms"] == 2 * i1["mvms"]
    assert np.array_equal(p1, p2)


def test_dual_space_form_limits(directed):
    import torch
    msb, ctx, B = directed
    from tests.test_gpu_solve import _run
    E = W.random_complex(B.dim, 7)
    sysd = _sys(msb, G_, core_site=0, Uc=-4.0, E_G=-3.0, Gamma=1.0)
    with pytest.raises(msb.MsbError):                        # complex128 only
        _run(msb, ctx, [sysd], E, [0.0, 1.0], 1e-8, 100, msb.MSB_C64)
    x0 = torch.from_numpy(W.random_vector(B.dim, 1)).cuda()
    G = torch.empty(B.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(msb.MsbError):                        # Lanczos needs a symmetric H
        msb.msb_ground_state(ctx, _sys(msb, G_), x0, 1e-10, 300, G)
    E_G, _ = msb.msb_ground_state(ctx, _sys(msb, 0.0), x0, 1e-10, 300, G)
    assert np.isfinite(E_G)
