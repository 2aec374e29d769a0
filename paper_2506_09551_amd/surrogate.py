"""Learned form: solver-generated spectra, the network ensemble, and the
prediction with solver fallback.

Host orchestration of C-ABI calls only; every numerical step runs in the HIP
library (ground state, multi-shift solve, continued fraction, network
kernels).  A parameter set is (U, t', U_c, Gamma) of a ring with nearest and
next-nearest hopping; its spectrum is I(w_in, w) on a fixed grid
(Eq. kramers1 through the intermediate states of Eq. intermediateState, one
core-hole site, O_1 = O_2 = identity).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import _capi as C


@dataclass
class SpectrumJob:
    """Grid and solver settings shared by every parameter set."""
    w_in: np.ndarray
    w: np.ndarray
    eta: float = 0.1
    core_site: int = 0
    tol: float = 1e-8
    maxit: int = 3000
    gs_tol: float = 1e-10
    gs_maxit: int = 600
    lanczos_max: int = 1500
    cf_tol: float = 1e-5
    batch: int = 16                    # parameter sets per multi-system solve
    timings: dict = field(default_factory=lambda: {"gs": 0.0, "solve": 0.0, "spectrum": 0.0})


def _system(C_, p, E_G=0.0, core=-1, with_core=False):
    U, tp, Uc, Gamma = (float(v) for v in p)
    return C_.make_system(core_site=core if with_core else -1, Uc=Uc if with_core else 0.0, E_G=E_G,
                          Gamma=Gamma, U=U, t_amp=[1.0, tp])


def solver_spectra(ctx, params, job: SpectrumJob, x0, rows=None):
    """I[p][i][j] (float64 host) for parameter sets params[p] = (U, t', U_c, Gamma)
    on the grid (w_in[rows], w); rows = None: every w_in.

    The context must hold the ring with two bond types, nearest (amplitude
    1) first and next-nearest second; x0 is the seeded Lanczos start."""
    import torch
    params = np.asarray(params, dtype=np.float64)
    D = C.msb_dim(ctx)
    w_in = job.w_in if rows is None else job.w_in[np.asarray(rows)]
    n_sh = len(w_in)
    out = np.empty((len(params), n_sh, len(job.w)))
    dev = x0.device
    for b0 in range(0, len(params), job.batch):
        ps = params[b0:b0 + job.batch]
        nb = len(ps)
        E = torch.empty(nb, D, dtype=torch.complex128, device=dev)
        G = torch.empty(D, dtype=torch.float64, device=dev)
        EG = []
        t0 = time.perf_counter()
        for j, p in enumerate(ps):
            e_g, _ = C.msb_ground_state(ctx, _system(C, p), x0, job.gs_tol, job.gs_maxit, G)
            EG.append(e_g)
            E[j].copy_(G.to(torch.complex128))     # O_2 = identity
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        systems = [_system(C, p, E_G=EG[j], core=job.core_site, with_core=True) for j, p in enumerate(ps)]
        psi = torch.empty(nb, n_sh, D, dtype=torch.complex128, device=dev)
        C.msb_solve(ctx, systems, E, w_in, 0.0, job.tol, job.maxit, C.MSB_C128, psi)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for j, p in enumerate(ps):
            I, _ = C.msb_spectrum(ctx, _system(C, p, E_G=EG[j]), psi[j].contiguous(), job.w, job.eta,
                                  job.lanczos_max, job.cf_tol)
            out[b0 + j] = I
        t3 = time.perf_counter()
        job.timings["gs"] += t1 - t0
        job.timings["solve"] += t2 - t1
        job.timings["spectrum"] += t3 - t2
        del psi, E
    return out


def features(params, w_in, w):
    """[P * n_win * n_w][6] float32 rows (U, t', U_c, Gamma, w_in, w), grid-major per set."""
    params = np.asarray(params, dtype=np.float64)
    P, a, b = len(params), len(w_in), len(w)
    X = np.empty((P, a, b, 6), dtype=np.float32)
    X[..., :4] = params[:, None, None, :]
    X[..., 4] = np.asarray(w_in)[None, :, None]
    X[..., 5] = np.asarray(w)[None, None, :]
    return X.reshape(-1, 6)


class Ensemble:
    """The network ensemble on the device (msb_mlp_* calls)."""

    def __init__(self, members, in_shift, in_scale, out_scale, init_params):
        self.members = members
        self.h = C.msb_mlp_create(members, in_shift, in_scale, out_scale)
        for m in range(members):
            C.msb_mlp_set_params(self.h, m, init_params[m])

    def close(self):
        if self.h is not None:
            C.msb_mlp_destroy(self.h)
            self.h = None

    def train(self, X, T, perm, batch, steps, lr):
        return C.msb_mlp_train(self.h, X, T, perm, batch, steps, lr, self.members)

    def predict(self, X):
        import torch
        n = X.shape[0]
        mean = torch.empty(n, dtype=torch.float32, device=X.device)
        sd = torch.empty_like(mean)
        C.msb_mlp_predict(self.h, X.contiguous(), mean, sd)
        return mean, sd


def calibrate_fallback(mean, sd, I_ref, eps):
    """Smallest spread threshold that sends every row with error above eps to the solver.

    mean, sd, I_ref: [P][n_win][n_w] ensemble mean and spread and the solver's
    spectra of a validation set.  A row's error is max_w |mean - I_ref| over
    the spectrum's peak; a row falls back when sd exceeds frac * max(mean of
    its spectrum) somewhere in it (the msb_mlp_fallback rule).  Returns the
    largest frac that still flags every row with error > eps (just below the
    smallest spread ratio among those rows), or the largest spread ratio seen
    when no row exceeds eps."""
    mean, sd, I_ref = (np.asarray(a, dtype=np.float64) for a in (mean, sd, I_ref))
    peak_ref = I_ref.reshape(len(I_ref), -1).max(axis=1)
    peak_pred = mean.reshape(len(mean), -1).max(axis=1)
    err = np.abs(mean - I_ref).max(axis=2) / peak_ref[:, None]
    ratio = sd.max(axis=2) / peak_pred[:, None]
    bad = err > eps
    if not np.any(bad):
        return float(ratio.max()) * (1 + 1e-6)
    return float(ratio[bad].min()) * (1 - 1e-6)


def predict_with_fallback(ens: Ensemble, ctx, params, job: SpectrumJob, x0, frac=0.05):
    """Spectra of params from the ensemble; every w_in row whose ensemble
    spread exceeds frac * peak is recomputed by the solver.  Returns
    (I [P][n_win][n_w], fallback mask [P][n_win], seconds in the network,
    seconds in the solver)."""
    import torch
    params = np.asarray(params, dtype=np.float64)
    a, b = len(job.w_in), len(job.w)
    X = torch.from_numpy(features(params, job.w_in, job.w)).to(x0.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, sd = ens.predict(X)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    mu = mean.cpu().numpy().reshape(len(params), a, b)
    s = sd.cpu().numpy().reshape(len(params), a, b)
    I = mu.astype(np.float64)
    mask = np.zeros((len(params), a), dtype=bool)
    t_solver = 0.0
    for p in range(len(params)):
        mask[p] = C.msb_mlp_fallback(mu[p], s[p], frac)
        rows = np.nonzero(mask[p])[0]
        if len(rows):
            t1 = time.perf_counter()
            I[p, rows] = solver_spectra(ctx, params[p:p + 1], job, x0, rows=rows)[0]
            t_solver += time.perf_counter() - t1
    return I, mask, t_net, t_solver
