"""Parity of the surrogate network's HIP kernels with the oracle (learned form).

The oracle runs the same network in float64 with the GPU's bfloat16
roundings applied at the same points (``oracle.mlp`` with ``bf16_ops``), so
the remaining differences are float32 accumulation order and the rare
bfloat16 rounding of a value that lies within float32 noise of a tie.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = W.SURROGATE_LO + rng.uniform(0, 1, (n, 6)) * (W.SURROGATE_HI - W.SURROGATE_LO)
    T = 0.5 + np.sin(X[:, 4] * 0.4) * np.exp(-0.1 * (X[:, 5] - 4.0) ** 2) + 0.05 * X[:, 0]
    return X.astype(np.float32), T.astype(np.float32)


def _make(msb, members, out_scale=2.0):
    shift, scale = W.surrogate_normalisation()
    return msb.msb_mlp_create(members, shift, scale, out_scale)


def _oracle_grad(p, X, T, out_scale):
    shift, scale = W.surrogate_normalisation()
    Xn = omlp.normalize(X.astype(np.float64), shift.astype(np.float32), scale.astype(np.float32))
    t = out_scale * T.astype(np.float64)
    y, c = omlp.forward(p.astype(np.float64), Xn, bf16_ops=True)
    return omlp.loss(y, t), omlp.backward(p.astype(np.float64), c, y, t, bf16_ops=True), y


@pytest.mark.parametrize("n", [128, 300, 1024])
def test_loss_and_gradient_match_oracle(gpu, n):
    """Full network, one member of two, n points (300: a ragged last tile)."""
    import torch
    msb = gpu
    mlp = _make(msb, 2)
    try:
        p = W.mlp_init(21)
        msb.msb_mlp_set_params(mlp, 1, p)
        X, T = _inputs(n, 5)
        loss, g = msb.msb_mlp_grad(mlp, 1, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
        lo, go, _ = _oracle_grad(p, X, T, 2.0)
        assert loss == pytest.approx(lo, rel=2e-3)
        P = omlp.unflatten(go)
        G = omlp.unflatten(g.astype(np.float64))
        for name in P:
            err = np.linalg.norm(G[name] - P[name]) / np.linalg.norm(P[name])
            assert err <= 1e-2, f"{name}: rel err {err:.2e}"
        assert np.linalg.norm(g - go) <= 5e-3 * np.linalg.norm(go)
    finally:
        msb.msb_mlp_destroy(mlp)


def test_predict_matches_oracle_ensemble(gpu):
    import torch
    msb = gpu
    members = 3
    mlp = _make(msb, members, out_scale=0.5)
    try:
        ps = [W.mlp_init(40 + m) for m in range(members)]
        for m, p in enumerate(ps):
            msb.msb_mlp_set_params(mlp, m, p)
        n = 33000                                  # two chunks, the second ragged
        X, _ = _inputs(n, 9)
        mean = torch.empty(n, dtype=torch.float32, device="cuda")
        sd = torch.empty_like(mean)
        msb.msb_mlp_predict(mlp, torch.from_numpy(X).cuda(), mean, sd)
        shift, scale = W.surrogate_normalisation()
        Xn = omlp.normalize(X.astype(np.float64), shift.astype(np.float32), scale.astype(np.float32))
        ys = np.stack([omlp.forward(p.astype(np.float64), Xn, bf16_ops=True)[0] / 0.5 for p in ps])
        mu, sdo = ys.mean(axis=0), ys.std(axis=0)
        m_gpu, s_gpu = mean.cpu().numpy(), sd.cpu().numpy()
        scale_y = np.max(np.abs(mu))
        assert np.max(np.abs(m_gpu - mu)) <= 2e-3 * scale_y
        assert np.max(np.abs(s_gpu - sdo)) <= 2e-3 * scale_y
    finally:
        msb.msb_mlp_destroy(mlp)


def test_adam_steps_match_oracle(gpu):
    """Two Adam steps of two members on their own permutations."""
    import torch
    msb = gpu
    members, batch, steps, lr = 2, 256, 2, 1e-3
    mlp = _make(msb, members)
    try:
        ps = [W.mlp_init(60 + m) for m in range(members)]
        for m, p in enumerate(ps):
            msb.msb_mlp_set_params(mlp, m, p)
        n = 700
        X, T = _inputs(n, 13)
        perm = W.permutations(members, steps, batch, n, seed=3)
        hist = msb.msb_mlp_train(mlp, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(),
                                 torch.from_numpy(perm).cuda(), batch, steps, lr, members)
        for m in range(members):
            p = ps[m].astype(np.float64)
            mm = np.zeros_like(p)
            vv = np.zeros_like(p)
            for k in range(steps):
                idx = perm[m, k * batch:(k + 1) * batch]
                lo, go, _ = _oracle_grad(p.astype(np.float32), X[idx], T[idx], 2.0)
                assert hist[m, k] == pytest.approx(lo, rel=5e-3)
                p, mm, vv = omlp.adam_step(p, go, mm, vv, k + 1, lr)
                p = p.astype(np.float32).astype(np.float64)
            got = msb.msb_mlp_get_params(mlp, m).astype(np.float64)
            d_gpu = got - ps[m]
            d_ora = p - ps[m]
            # every parameter moves by about lr per step; where the gradient
            # is clearly non-zero both sides move the same way
            big = np.abs(d_ora) > 0.5 * lr
            assert np.mean(np.sign(d_gpu[big]) == np.sign(d_ora[big])) >= 0.99
            assert np.max(np.abs(d_gpu)) <= steps * lr * 1.01
            assert np.linalg.norm(d_gpu - d_ora) <= 0.1 * np.linalg.norm(d_ora)
    finally:
        msb.msb_mlp_destroy(mlp)


def test_training_fits_smooth_target(gpu):
    import torch
    msb = gpu
    members, batch, steps = 2, 512, 300
    mlp = _make(msb, members)
    try:
        for m in range(members):
            msb.msb_mlp_set_params(mlp, m, W.mlp_init(80 + m))
        n = 8192
        X, T = _inputs(n, 17)
        perm = W.permutations(members, steps, batch, n, seed=5)
        hist = msb.msb_mlp_train(mlp, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(),
                                 torch.from_numpy(perm).cuda(), batch, steps, 1e-3, members)
        assert np.all(np.isfinite(hist))
        assert np.all(hist[:, -20:].mean(axis=1) <= 0.05 * hist[:, :5].mean(axis=1))
        mean = torch.empty(n, dtype=torch.float32, device="cuda")
        sd = torch.empty_like(mean)
        msb.msb_mlp_predict(mlp, torch.from_numpy(X).cuda(), mean, sd)
        err = np.sqrt(np.mean((mean.cpu().numpy() - T) ** 2))
        assert err <= 0.1 * np.sqrt(np.mean(T ** 2))
    finally:
        msb.msb_mlp_destroy(mlp)


def test_adam_update_on_a_known_gradient(gpu):
    """Adam (float32 on the GPU) against the oracle's update computed from the
    gradient the GPU itself reports for the same points (msb_mlp_grad), over
    two steps, so bias correction, beta_1, beta_2 and eps all enter: equal to
    float32 rounding of the parameters plus 2e-5 lr (the float32 constants
    0.9f, 0.999f move 1 - beta_2^k by 1.3e-5 relative)."""
    import torch
    msb = gpu
    lr = 1e-3
    mlp = _make(msb, 1)
    try:
        p0 = W.mlp_init(71)
        msb.msb_mlp_set_params(mlp, 0, p0)
        n = 256
        perm = torch.arange(n, dtype=torch.int32, device="cuda").reshape(1, n)
        p_prev = p0.astype(np.float64)
        m = np.zeros_like(p_prev)
        v = np.zeros_like(p_prev)
        for k, seed in ((1, 31), (2, 32)):
            X, T = _inputs(n, seed)
            Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
            _, g = msb.msb_mlp_grad(mlp, 0, Xt, Tt)          # gradient at the current parameters
            msb.msb_mlp_train(mlp, Xt, Tt, perm, n, 1, lr, 1)  # one Adam step on the same points
            got = msb.msb_mlp_get_params(mlp, 0).astype(np.float64)
            want, m, v = omlp.adam_step(p_prev, g.astype(np.float64), m, v, k, lr)
            tol = 2.0 * np.spacing(np.abs(want).astype(np.float32)).astype(np.float64) + 2e-5 * lr
            bad = np.abs(got - want) > tol
            assert not np.any(bad), (k, int(bad.sum()), float(np.max(np.abs(got - want))))
            assert np.max(np.abs(got - p_prev)) > 0.5 * lr        # the step moved the parameters
            p_prev = got
    finally:
        msb.msb_mlp_destroy(mlp)
