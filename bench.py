"""Benchmark of the multi-shift BiCG hot path on one MI355X.

Workload (default): the 12-site periodic Hubbard ring, N_up = N_dn = 6
(D = 853,776), t = 1, U = 8, a core hole U_c = -4 on each of the 12 sites
(12 systems), Gamma = 1, 200 incident energies in [-12, 12], complex128.
One step = the multi-shift solve of all 12 x 200 shifted systems to a
relative recurrence residual of 1e-8, confirmed by the FP64 true residual of
every shift.  The ground state (precondition) and the continued-fraction
spectrum that follows are timed once and reported beside the metric.

Prints one JSON line.  Inputs are synthetic and resident in device memory
before the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6

# The complex64 workloads (precision, batched) run the library's complex64
# form as it is (the direct seed form with residual replacement).
C64_OPTS = None

# HBM counters of the assembly kernel on the scale step (one launch), from
# profiles/solve_scale_L12_hbm_counters.md: raw FETCH_SIZE / WRITE_SIZE in KiB
# and the copy-calibrated factors; valid while the kernel source is unchanged.
FLUSH_COUNTERS = {
    "source": "paper_2506_09551_amd/csrc/k_shift.hip", "sha256_16": "1ae052f0b875109a",
    "fetch_kib": 64184085.1, "write_kib": 32016600.0, "fetch_factor": 2.0, "write_factor": 1.0,
    "workload": "scale_L12_N6",
}


def flush_traffic_gb(wl_name):
    """Counter-measured HBM bytes (GB) of one assembly launch, or None."""
    import hashlib
    c = FLUSH_COUNTERS
    if wl_name != c["workload"]:
        return None
    try:
        h = hashlib.sha256(open(os.path.join(ROOT, c["source"]), "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if h != c["sha256_16"]:
        return None
    return 1024.0 * (c["fetch_factor"] * c["fetch_kib"] + c["write_factor"] * c["write_kib"]) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, iters_gpu: int, n_iter: int = 6, threads: int = 1):
    """Oracle recurrence (one system, all shifts) for a few iterations, extrapolated;
    BLAS / OpenMP pools limited to `threads` (NumPy's elementwise work and
    SciPy's sparse product run on one core whatever the limit)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import hubbard as hb
    from oracle import solve as osolve
    import workloads as W

    B = hb.Basis(wl.n_sites, wl.n_up, wl.n_dn)
    Hp = hb.hamiltonian(B, wl.bonds, wl.U, core_site=wl.core_sites[0], Uc=wl.Uc)
    E = W.random_vector(B.dim, 5).astype(np.complex128)
    shift = -4.0 + 1j * wl.Gamma
    A = lambda x: Hp @ x - shift * x
    with threadpool_limits(limits=threads):
        osolve.msbicg_reference(A, E, wl.w_in, 1e-30, 1)          # warm-up
        t0 = time.perf_counter()
        osolve.msbicg_reference(A, E, wl.w_in, 1e-30, n_iter)
        dt = time.perf_counter() - t0
    per_iter = dt / n_iter
    per_system = per_iter * iters_gpu
    return {
        "value": len(wl.w_in) / per_system,
        "unit": "shift-solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"one of {wl.nrhs} core-hole systems with all {len(wl.w_in)} shifts: "
                   f"{n_iter} iterations of the oracle's multi-shift recurrence (NumPy/SciPy "
                   f"CSR, thread pools limited to {threads}) took {dt:.2f} s, scaled to the "
                   f"{iters_gpu} iterations the GPU run needs"),
        "host": {"cpu": cpu_model(), "os_cpu_count": os.cpu_count()},
    }


def precision_extras(msb, ctx, wl, systems, E, E_G, box, info64, ms64, tol, n_sub=16):
    """complex64 form against complex128: final FP64 true residual per shift,
    the speedup of the whole solve, and the continued-fraction spectrum error
    on `n_sub` incident energies spread over the shift list."""
    import numpy as np
    import torch

    psi64 = box.pop()
    dev = psi64.device
    D = msb.msb_dim(ctx)
    n_shift = len(wl.w_in)
    sub = np.unique(np.linspace(0, n_shift - 1, n_sub).round().astype(int))
    rt = info64["resid_true"]
    res = {
        "c64_true_residual": {"max": float(rt.max()), "median": float(np.median(rt)),
                              "min": float(rt.min())},
        "c64_replacements": int(info64["replacements"]),
        "c64_iters": int(info64["iters"]),
        "c64_ms": round(ms64, 3),
    }

    def spectrum(psi_all):
        ps = psi_all[:, torch.as_tensor(sub, device=dev)].contiguous()
        phi = torch.empty(len(sub), D, dtype=torch.complex128, device=dev)
        msb.msb_combine(ctx, ps, wl.nrhs, len(sub), msb.MSB_C64 if ps.dtype == torch.complex64
                        else msb.MSB_C128, wl.phases, phi)
        I, _ = msb.msb_spectrum(ctx, msb.make_system(E_G=E_G), phi, wl.w_loss, wl.eta, 1500, 1e-12)
        return np.asarray(I)

    I64 = spectrum(psi64)
    del psi64
    torch.cuda.empty_cache()
    psi128 = torch.empty(wl.nrhs, n_shift, D, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    msb.msb_solve(ctx, systems, E, wl.w_in, wl.seed_shift, tol, wl.maxit, msb.MSB_C128, psi128,
                  want_true=True)   # warm-up: sizes the workspace the timed call reuses
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info128 = msb.msb_solve(ctx, systems, E, wl.w_in, wl.seed_shift, tol, wl.maxit, msb.MSB_C128,
                               psi128, want_true=True)
    torch.cuda.synchronize()
    ms128 = (time.perf_counter() - t0) * 1e3
    I128 = spectrum(psi128)
    del psi128
    torch.cuda.empty_cache()
    peak = np.max(np.abs(I128), axis=1)
    err = np.max(np.abs(I64 - I128), axis=1) / peak
    res.update({
        "c128_ms": round(ms128, 3),
        "c128_iters": int(info128["iters"]),
        "c128_split_ms": {"seed": round(info128["t_iter_ms"], 2), "assembly": round(info128["t_flush_ms"], 2),
                          "true_residual": round(info128["t_true_ms"], 2), "flushes": int(info128["flushes"])},
        "c64_split_ms": {"seed": round(info64["t_iter_ms"], 2), "assembly": round(info64["t_flush_ms"], 2),
                         "true_residual": round(info64["t_true_ms"], 2), "flushes": int(info64["flushes"])},
        "c128_true_residual_max": float(np.max(info128["resid_true"])),
        "speedup_c64_vs_c128": round(ms128 / ms64, 3),
        "spectrum_rel_err_vs_c128": {"max": float(err.max()), "median": float(np.median(err)),
                                     "shifts": [float(wl.w_in[k]) for k in sub],
                                     "norm": "max_w |I64 - I128| / max_w I128 per w_in"},
    })
    log(f"precision {res}")
    return res


def batched_extras(msb, ctx, wl, systems, E, psi, ms_batched, tol, prec, E_G, n_sub=4):
    """Batched form against the same right-hand sides solved one at a time (in
    its own precision, and in the plain complex128 form), the continued-fraction
    spectrum error of the batched solution against the complex128 one on
    `n_sub` incident energies per right-hand side, and the block apply's rate
    for the whole batch and for one vector."""
    import numpy as np
    import torch

    D = msb.msb_dim(ctx)
    n = wl.nrhs
    # the batched solution's rows for the spectrum check (psi is reused below)
    n_shift = len(wl.w_in)
    sub_k = np.unique(np.linspace(0, n_shift - 1, n_sub).round().astype(int))
    kk = torch.as_tensor(sub_k, device=psi.device)
    phi_b = psi[:, kk].to(torch.complex128).reshape(n * len(sub_k), D)

    sep_split = {}

    def separate():
        sep_split.clear()
        for j in range(n):
            st, inf = msb.msb_solve(ctx, [systems[j]], E[j:j + 1], wl.w_in, wl.seed_shift, tol, wl.maxit,
                                    prec, psi[j:j + 1], want_true=True, raise_on_fail=False, opts=C64_OPTS)
            if st not in (msb.MSB_OK, msb.MSB_FLOOR):
                raise msb.MsbError(st, msb.lib().msb_last_error().decode())
            for key, name in (("t_iter_ms", "seed_iterations_ms"), ("t_flush_ms", "assembly_ms"),
                              ("t_true_ms", "true_residual_ms")):
                sep_split[name] = sep_split.get(name, 0.0) + inf[key]

    separate()                     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    separate()
    torch.cuda.synchronize()
    ms_sep = (time.perf_counter() - t0) * 1e3
    # plain complex128 multi-shift solves, one right-hand side at a time (the
    # complex64 solves' workspace is released first: it holds most of the HBM)
    msb.msb_release_workspace(ctx)
    phi_p = torch.empty_like(phi_b)
    psi128 = torch.empty(1, n_shift, D, dtype=torch.complex128, device=psi.device)
    msb.msb_solve(ctx, [systems[0]], E[0:1], wl.w_in, wl.seed_shift, tol, wl.maxit, msb.MSB_C128, psi128,
                  want_true=True)   # warm-up: sizes the workspace
    ms128 = 0.0
    for j in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        msb.msb_solve(ctx, [systems[j]], E[j:j + 1], wl.w_in, wl.seed_shift, tol, wl.maxit, msb.MSB_C128,
                      psi128, want_true=True)
        torch.cuda.synchronize()
        ms128 += (time.perf_counter() - t0) * 1e3
        phi_p[j * len(sub_k):(j + 1) * len(sub_k)] = psi128[0, kk]
    del psi128
    torch.cuda.empty_cache()
    gs = msb.make_system(E_G=E_G)
    I_b, _ = msb.msb_spectrum(ctx, gs, phi_b, wl.w_loss, wl.eta, 1500, 1e-10)
    I_p, _ = msb.msb_spectrum(ctx, gs, phi_p, wl.w_loss, wl.eta, 1500, 1e-10)
    del phi_b, phi_p
    torch.cuda.empty_cache()
    peak = np.max(np.abs(I_p), axis=1)
    err = np.max(np.abs(np.asarray(I_b) - np.asarray(I_p)), axis=1) / peak
    dt = psi.dtype
    x = torch.randn(n, D, dtype=dt, device=psi.device)
    y = torch.empty_like(x)
    ms_blk = msb.msb_apply_timed(ctx, systems, 0.0, prec, x, y, 20)
    ms_one = msb.msb_apply_timed(ctx, systems[0], 0.0, prec, x[0], y[0], 20)
    # the same block interleaved (groups of four): the apply the batched solve runs
    ms_il = msb.msb_apply_block(ctx, systems, 0.0, prec, 4, x, y, reps=20) if n % 4 == 0 else None
    el = x.element_size()
    res = {
        "separate_ms": round(ms_sep, 3), "batched_ms": round(ms_batched, 3),
        "separate_split_ms": {k: round(v, 3) for k, v in sep_split.items()},
        "speedup_batched_vs_separate": round(ms_sep / ms_batched, 3),
        "plain_c128_separate_ms": round(ms128, 3),
        "speedup_batched_vs_plain_c128": round(ms128 / ms_batched, 3),
        "spectrum_rel_err_vs_c128": {"max": float(err.max()), "median": float(np.median(err)),
                                     "shifts": [float(wl.w_in[k]) for k in sub_k],
                                     "norm": "max_w |I_batched - I_c128| / max_w I_c128 per (RHS, w_in)"},
        "apply_block_ms": round(ms_blk, 4), "apply_one_ms": round(ms_one, 4),
        "apply_block_GBs": round(2 * n * D * el / (ms_blk * 1e-3) / 1e9, 1),
        "apply_block_interleaved_ms": None if ms_il is None else round(ms_il, 4),
        "apply_block_interleaved_GBs": None if ms_il is None else round(2 * n * D * el / (ms_il * 1e-3) / 1e9, 1),
        "apply_one_GBs": round(2 * D * el / (ms_one * 1e-3) / 1e9, 1),
    }
    log(f"batched {res}")
    return res


def mlp_train_main(args):
    """Training throughput of the surrogate alone: 5 members, batch 8192,
    `--mlp-train-steps` Adam steps on 2^20 seeded random points (targets
    uniform), after one warm-up call; reports the matrix-core rate of the
    six 8192 x 512 x 512 products per member and step."""
    import numpy as np
    import torch

    from paper_2506_09551_amd import surrogate as S
    import workloads as W

    dev = torch.device("cuda:0")
    members, batch, steps = 5, 8192, args.mlp_train_steps
    shift, scale = W.surrogate_normalisation()
    ens = S.Ensemble(members, shift, scale, 1.0, [W.mlp_init(100 + m) for m in range(members)])
    n = 1 << 20
    rng = np.random.default_rng(0)
    X = torch.from_numpy((W.SURROGATE_LO + rng.uniform(0, 1, (n, 6)) * (W.SURROGATE_HI - W.SURROGATE_LO))
                         .astype(np.float32)).to(dev)
    T = torch.from_numpy(rng.uniform(0, 1, n).astype(np.float32)).to(dev)
    perm = W.permutations_device(members, steps, batch, n, seed=1, device=dev)
    ens.train(X, T, perm, batch, steps, 1e-3)            # warm-up (graph capture, buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ens.train(X, T, perm, batch, steps, 1e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ens.close()
    flops = members * steps * batch * 6 * 2 * 512 * 512
    out = {"metric": "surrogate training step", "value": round(dt / steps * 1e3, 4), "unit": "ms/step",
           "higher_is_better": False, "n_gpus": 1, "steps": steps, "members": members, "batch": batch,
           "matrix_core_TFLOPs": round(flops / dt / 1e12, 2), "peak_TFLOPs": 2500.0,
           "loss_first_last": [float(hist[:, 0].mean()), float(hist[:, -1].mean())], "data": "synthetic"}
    print(json.dumps(out), flush=True)


def learned_main(args):
    """Learned form: the ensemble surrogate against the plain solver.

    Training spectra and held-out spectra come from the solver (ground state,
    128-shift multi-shift solve, continued fraction) at scrambled-Sobol
    parameter sets; the surrogate is trained on the training set, and a step
    is the prediction of every held-out spectrum with solver fallback for the
    rows where the ensemble spread exceeds 5% of the predicted peak."""
    import numpy as np
    import torch

    import paper_2506_09551_amd as msb
    from paper_2506_09551_amd import surrogate as S
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.get("learned")
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    D = msb.msb_dim(ctx)
    x0 = torch.from_numpy(W.random_vector(D, wl.gs_seed)).to(dev)
    n_tr, n_ho = args.train_spectra, args.heldout_spectra
    p_tr = W.sobol_params(n_tr, seed=7)
    p_ho = W.sobol_params(n_ho, seed=7, skip=n_tr)
    job = S.SpectrumJob(w_in=wl.w_in, w=wl.w_loss, eta=wl.eta, gs_tol=1e-7, cf_tol=1e-4, batch=32)
    log(f"learned: D={D}, {n_tr} training + {n_ho} held-out spectra of {len(wl.w_in)}x{len(wl.w_loss)}")

    t0 = time.perf_counter()
    I_tr = np.empty((n_tr, len(wl.w_in), len(wl.w_loss)), dtype=np.float32)
    for c0 in range(0, n_tr, 256):
        I_tr[c0:c0 + 256] = S.solver_spectra(ctx, p_tr[c0:c0 + 256], job, x0)
        log(f"  solver spectra {min(c0 + 256, n_tr)}/{n_tr} ({time.perf_counter() - t0:.1f} s)")
    t_gen = time.perf_counter() - t0
    solver_ms = t_gen / n_tr * 1e3
    # the held-out spectra judge the network: solved with tight tolerances, so
    # that their own error (ground state 1e-10, continued fraction converged
    # to 1e-9 of the peak) is far below the errors being measured
    t0 = time.perf_counter()
    job_ho = S.SpectrumJob(w_in=wl.w_in, w=wl.w_loss, eta=wl.eta, gs_tol=1e-10, cf_tol=1e-9, batch=32)
    I_ho = S.solver_spectra(ctx, p_ho, job_ho, x0)
    solver_ho_ms = (time.perf_counter() - t0) / n_ho * 1e3
    log(f"solver: {solver_ms:.1f} ms per training spectrum, {solver_ho_ms:.1f} ms per held-out spectrum; "
        f"split {job.timings}")

    X = torch.from_numpy(S.features(p_tr, wl.w_in, wl.w_loss)).to(dev)
    T = torch.from_numpy(I_tr.ravel()).to(dev)
    n_pts = T.numel()
    out_scale = 1.0 / float(np.mean(I_tr.reshape(n_tr, -1).max(axis=1)))
    del I_tr
    members, batch = 5, 8192
    shift, scale = W.surrogate_normalisation()
    ens = S.Ensemble(members, shift, scale, out_scale, [W.mlp_init(1000 + m) for m in range(members)])
    steps_total = max(1, int(args.epochs * n_pts / batch))
    t0 = time.perf_counter()
    hist_all = []
    chunk = 4096
    done = 0
    while done < steps_total:
        st = min(chunk, steps_total - done)
        lr = 1e-3 if done < 0.6 * steps_total else 2e-4
        perm = W.permutations_device(members, st, batch, n_pts, seed=77 + done, device=dev)
        hist_all.append(ens.train(X, T, perm, batch, st, lr))
        del perm
        done += st
        log(f"  train {done}/{steps_total} steps, loss {hist_all[-1][:, -50:].mean():.3e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hist = np.concatenate(hist_all, axis=1)
    gemm_flops = members * steps_total * batch * 6 * 2 * 512 * 512
    del X, T

    # evaluation: network alone, then with fallback (the timed step: the 5%
    # spread rule on all held-out spectra)
    def run(params, frac):
        return S.predict_with_fallback(ens, ctx, params, job_ho, x0, frac=frac)
    run(p_ho, 0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    I_pred, mask, t_net, t_fb = run(p_ho, 0.05)
    t_step = time.perf_counter() - t0
    Xh = torch.from_numpy(S.features(p_ho, wl.w_in, wl.w_loss)).to(dev)
    mean, sd = ens.predict(Xh)
    mu = mean.cpu().numpy().reshape(I_ho.shape)
    sdv = sd.cpu().numpy().reshape(I_ho.shape)
    peak = I_ho.reshape(n_ho, -1).max(axis=1)
    err_net = np.abs(mu - I_ho).reshape(n_ho, -1).max(axis=1) / peak
    err_fb = np.abs(I_pred - I_ho).reshape(n_ho, -1).max(axis=1) / peak
    # error-bounded fallback: the held-out sets split into a validation half,
    # on which the spread threshold is calibrated for each error bound eps
    # (every validation row above eps falls back), and a test half, on which
    # the rule is timed and its max error measured
    nv = n_ho // 2
    val, tst = slice(0, nv), slice(nv, n_ho)
    peak_t = peak[tst]
    sweep = []
    for eps in (0.1, 0.05, 0.02, 0.01, 0.005):
        frac = S.calibrate_fallback(mu[val], sdv[val], I_ho[val], eps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        I_r, m_r, tn, tf = run(p_ho[tst], frac)
        t_r = time.perf_counter() - t0
        e_r = np.abs(I_r - I_ho[tst]).reshape(n_ho - nv, -1).max(axis=1) / peak_t
        sweep.append({"eps": eps, "spread_frac": frac, "test_max_err": float(e_r.max()),
                      "test_p95_err": float(np.quantile(e_r, 0.95)), "bound_held": bool(e_r.max() <= eps),
                      "fallback_row_rate": float(m_r.mean()),
                      "fallback_spectrum_rate": float(np.any(m_r, axis=1).mean()),
                      "ms_per_spectrum": round(t_r / (n_ho - nv) * 1e3, 3),
                      "speedup_vs_solver": round(solver_ho_ms / (t_r / (n_ho - nv) * 1e3), 2)})
        log(f"  fallback eps={eps}: {sweep[-1]}")
    ens.close()
    surrogate_ms = t_step / n_ho * 1e3
    value = n_ho * len(wl.w_in) / t_step
    out = {
        "metric": "\u03a8_int shift-solves/sec at rel. residual 1e-8; H-apply HBM GB/s vs peak",
        "value": round(value, 2),
        "unit": "shift-solves/s (surrogate with solver fallback; 128 incident energies per spectrum)",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (network), c128 (solver)",
        "data": "synthetic", "config": {"workload": wl.note, "name": wl.name, "D": D,
                                        "train_spectra": n_tr, "heldout_spectra": n_ho,
                                        "grid": [len(wl.w_in), len(wl.w_loss)], "members": members},
        "learned": {
            "solver_ms_per_spectrum": round(solver_ho_ms, 2),
            "solver_ms_per_spectrum_training_settings": round(solver_ms, 2),
            "surrogate_ms_per_spectrum": round(surrogate_ms, 3),
            "network_only_ms_per_spectrum": round(t_net / n_ho * 1e3, 3),
            "speedup_vs_solver": round(solver_ho_ms / surrogate_ms, 2),
            "fallback_row_rate": float(mask.mean()),
            "fallback_spectrum_rate": float(np.any(mask, axis=1).mean()),
            "err_vs_solver_network": {"median": float(np.median(err_net)), "p95": float(np.quantile(err_net, 0.95)),
                                      "max": float(err_net.max()), "norm": "max |I - I_solver| / peak per spectrum"},
            "err_vs_solver_with_fallback": {"median": float(np.median(err_fb)), "p95": float(np.quantile(err_fb, 0.95)),
                                            "max": float(err_fb.max()), "rule": "spread > 5% of the predicted peak"},
            "error_bounded_fallback": {"calibration": f"first {nv} held-out spectra", "test": f"last {n_ho - nv}",
                                       "sweep": sweep},
            "reference": "held-out spectra solved with ground-state tol 1e-10 and cf_tol 1e-9",
            "train": {"points": int(n_pts), "steps": steps_total, "batch": batch, "seconds": round(t_train, 2),
                      "loss_first": float(hist[:, :20].mean()), "loss_last": float(hist[:, -200:].mean()),
                      "matrix_core_TFLOPs": round(gemm_flops / t_train / 1e12, 2),
                      "solver_generation_s": round(t_gen, 1)},
        },
    }
    msb.msb_destroy(ctx)
    print(json.dumps(out), flush=True)


def reseed_main(args):
    """Adaptive reseeding (Appendix E): a step is one reseeded solve of all
    shifts from the edge seed; beside it, the plain solve from the same edge
    seed (which leaves shifts unsolved) and from the default seed 0."""
    import numpy as np
    import torch

    import paper_2506_09551_amd as msb
    import workloads as W

    assert torch.cuda.is_available(), "bench needs the GPU"
    dev = torch.device("cuda:0")
    wl = W.get("reseed")
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    D = msb.msb_dim(ctx)
    x0 = torch.from_numpy(W.random_vector(D, wl.gs_seed)).to(dev)
    G = torch.empty(D, dtype=torch.float64, device=dev)
    E_G, _ = msb.msb_ground_state(ctx, msb.make_system(), x0, 1e-10, 600, G)
    E = G.to(torch.complex128).reshape(1, D).contiguous()
    system = msb.make_system(core_site=wl.core_sites[0], Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    n_shift = len(wl.w_in)
    psi = torch.empty(1, n_shift, D, dtype=torch.complex128, device=dev)
    reseed_tol = 10 * wl.tol

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    def plain(seed):
        return msb.msb_solve(ctx, [system], E, wl.w_in, seed, wl.tol, wl.maxit, msb.MSB_C128, psi,
                             want_true=True, raise_on_fail=False)

    def reseeded():
        return msb.msb_solve_reseed(ctx, [system], E, wl.w_in, wl.seed_shift, wl.tol, wl.maxit, msb.MSB_C128,
                                    psi, reseed_tol, 8)

    plain(0.0)                                        # tunes the apply and sizes the workspace
    (st_e, info_e), ms_edge = timed(lambda: plain(wl.seed_shift))
    fail_e = int(np.sum((info_e["shift_iters"][0] < 0) | ~(info_e["resid_true"][0] <= reseed_tol)))
    (st_0, info_0), ms_zero = timed(lambda: plain(0.0))
    for _ in range(args.warmup):
        reseeded()
    times = []
    for _ in range(args.steps):
        (st_r, info_r), ms = timed(reseeded)
        times.append(ms)
    ms_step = float(np.mean(times))
    seeds = sorted(set(float(s) for s in info_r["seed_of"][0]))
    res = {
        "initial_seed": wl.seed_shift, "reseed_tol": reseed_tol, "rounds": int(info_r["rounds"][0]),
        "seeds": seeds,
        "shifts_per_seed": {f"{s:g}": int(np.sum(info_r["seed_of"][0] == s)) for s in seeds},
        "max_true_residual": float(np.max(info_r["resid_true"])),
        "plain_edge_seed": {"ms": round(ms_edge, 3), "status": msb.STATUS.get(st_e, st_e),
                            "iters": int(info_e["iters"]), "shifts_failing": fail_e,
                            "max_true_residual": float(np.nanmax(info_e["resid_true"]))},
        "plain_seed_0": {"ms": round(ms_zero, 3), "status": msb.STATUS.get(st_0, st_0),
                         "iters": int(info_0["iters"]),
                         "max_true_residual": float(np.max(info_0["resid_true"]))},
    }
    log(f"reseed {res}")
    out = {
        "metric": "\u03a8_int shift-solves/sec at rel. residual 1e-8; H-apply HBM GB/s vs peak",
        "value": round(n_shift / (ms_step * 1e-3), 2),
        "unit": "shift-solves/s (adaptive reseeding from an edge seed, tol 1e-10)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wl.note, "name": wl.name, "D": D, "systems": 1, "shifts": n_shift,
                   "tol": wl.tol, "Gamma": wl.Gamma},
        "reseed": res,
    }
    msb.msb_destroy(ctx)
    print(json.dumps(out), flush=True)


def dipole_main(args):
    """Direct edge that adds a valence electron: E_j = c+_{j up} G moves the
    ground state of (N, N) into (N+1, N), the 12 x 200 multi-shift solve runs
    there (the step), and phi = sum_j e^{iqj} c_{j up} Psi_j brings the
    intermediate states back for the continued-fraction spectrum."""
    import numpy as np
    import torch

    import paper_2506_09551_amd as msb
    import workloads as W

    assert torch.cuda.is_available(), "bench needs the GPU"
    dev = torch.device("cuda:0")
    wl = W.get("dipole")
    L, s = wl.n_sites, wl.dipole_spin
    c0 = msb.msb_create(L, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    c1 = msb.msb_create(L, wl.n_up + (s == 0), wl.n_dn + (s == 1), wl.bonds, wl.U)
    D0, D1 = msb.msb_dim(c0), msb.msb_dim(c1)
    x0 = torch.from_numpy(W.random_vector(D0, wl.gs_seed)).to(dev)
    G = torch.empty(D0, dtype=torch.float64, device=dev)
    E_G, gs_iters = msb.msb_ground_state(c0, msb.make_system(), x0, 1e-10, 600, G)
    Gc = G.to(torch.complex128).reshape(1, D0).contiguous()
    n_sys, n_shift = wl.nrhs, len(wl.w_in)
    E = torch.empty(n_sys, D1, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, site in enumerate(wl.core_sites):
        coef = np.zeros(L, dtype=np.complex128)
        coef[site] = 1.0
        msb.msb_dipole(c0, c1, s, True, coef, Gc, E[j:j + 1])
    torch.cuda.synchronize()
    op2_ms = (time.perf_counter() - t0) * 1e3
    systems = [msb.make_system(core_site=c, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for c in wl.core_sites]
    msb.msb_autotune(c1, n_sys, msb.MSB_C128)
    psi = torch.empty(n_sys, n_shift, D1, dtype=torch.complex128, device=dev)

    def step():
        st, info = msb.msb_solve(c1, systems, E, wl.w_in, wl.seed_shift, args.tol, wl.maxit, msb.MSB_C128,
                                 psi, want_true=True)
        return info
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    last = infos[-1]
    phi = torch.empty(n_shift, D0, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, site in enumerate(wl.core_sites):
        coef = np.zeros(L, dtype=np.complex128)
        coef[site] = wl.phases[j]
        msb.msb_dipole(c1, c0, s, False, coef, psi[j], phi, accumulate=j > 0)
    torch.cuda.synchronize()
    op1_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    I, depth = msb.msb_spectrum(c0, msb.make_system(E_G=E_G), phi, wl.w_loss, wl.eta, 1500, 1e-8)
    torch.cuda.synchronize()
    cf_ms = (time.perf_counter() - t0) * 1e3
    out = {
        "metric": "\u03a8_int shift-solves/sec at rel. residual 1e-8; H-apply HBM GB/s vs peak",
        "value": round(n_sys * n_shift / (ms_step * 1e-3), 2),
        "unit": "shift-solves/s (intermediate sector N+1 reached by c+_{j up})",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": wl.note, "name": wl.name, "D_ground": D0, "D_intermediate": D1,
                   "systems": n_sys, "shifts": n_shift, "tol": args.tol},
        "iters": int(last["iters"]), "max_true_residual": float(np.max(last["resid_true"])),
        "split_ms": {"seed_iterations_ms": round(last["t_iter_ms"], 3),
                     "assembly_ms": round(last["t_flush_ms"], 3),
                     "true_residual_ms": round(last["t_true_ms"], 3)},
        "operators_ms": {"O2 (12 x c+ G)": round(op2_ms, 3), "O1 (site sum of c Psi)": round(op1_ms, 3)},
        "ground_state": {"E_G": E_G, "lanczos_steps": int(gs_iters)},
        "spectrum": {"ms": round(cf_ms, 1), "lanczos_depth_max": int(depth.max()),
                     "lanczos_depth_mean": float(depth.mean()), "I_max": float(np.max(I))},
    }
    msb.msb_destroy(c0)
    msb.msb_destroy(c1)
    print(json.dumps(out), flush=True)


def h_apply_rates(msb, ctx, wl, systems, prec, reps=50):
    """H-apply rates: algorithmic bytes 2 D s R over the mean of `reps` applies,
    against the 8 TB/s spec and a 1 GiB device copy measured here, for the
    given context's block and one vector, and the HBM-resident L = 14 and 4x4
    workloads."""
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    cdt = torch.complex128 if prec == msb.MSB_C128 else torch.complex64
    D = msb.msb_dim(ctx)
    # H-apply bandwidth: algorithmic bytes 2 D s per vector
    # H-apply rate: algorithmic bytes 2 D s R over the mean of 50 applies,
    # against the 8 TB/s spec and a device copy measured here
    happly = {}
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)   # 1 GiB
    dstc = torch.empty_like(src)
    for _ in range(3):
        dstc.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        dstc.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dstc
    happly["copy_1GiB_GB/s"] = round(copy_gbs, 1)

    def rate(c, syss, pr, dt, Dn, label, note=None):
        n = len(syss)
        x = torch.randn(n, Dn, dtype=dt, device=dev)
        y = torch.empty_like(x)
        ms = msb.msb_apply_timed(c, syss, 0.0, pr, x, y, reps)
        gbs = 2 * n * Dn * x.element_size() / (ms * 1e-3) / 1e9
        happly[label] = {"ms": round(ms, 5), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "frac_of_copy": round(gbs / copy_gbs, 4)}
        if note:
            happly[label]["note"] = note
        del x, y
    rate(ctx, systems, prec, cdt, D, f"{wl.name}_x{len(systems)}",
         f"the solve's block of {len(systems)} vectors ({len(systems) * D * (16 if prec == msb.MSB_C128 else 8) / 1e6:.0f} MB)")
    rate(ctx, systems[:1], prec, cdt, D, wl.name, "one 13.7 MB vector: served from the 256 MB Infinity Cache")
    for other in ("precision", "batched"):
        wo = W.get(other)
        c2 = msb.msb_create(wo.n_sites, wo.n_up, wo.n_dn, wo.bonds, wo.U)
        D2 = msb.msb_dim(c2)
        s2 = [msb.make_system(core_site=c, Uc=wo.Uc, E_G=-4.0, Gamma=wo.Gamma) for c in wo.core_sites]
        if other == "precision":
            for dname, dt, pr in (("c128", torch.complex128, msb.MSB_C128), ("c64", torch.complex64, msb.MSB_C64)):
                rate(c2, s2, pr, dt, D2, f"{wo.name}_{dname}", "HBM-resident")
        else:
            rate(c2, s2, msb.MSB_C64, torch.complex64, D2, f"{wo.name}_c64_x{len(s2)}", "HBM-resident block")
        msb.msb_destroy(c2)
    return happly


def form_summary(name, out):
    """The figures of one form (precision or batched) for the default line."""
    s = {"workload": out["config"]["workload"], "dtype": out["dtype"], "tol": out["config"]["tol"],
         "ms_per_step": out["ms_per_step"], "shift_solves_per_s": out["value"], "iters": out["iters"],
         "solve_status": out["solve_status"], "max_true_residual": out["max_true_residual"],
         "split_ms": out["split_ms"], "assembly_tflops": out["roofline"]["achieved"]}
    if name == "precision":
        p = out["precision"]
        s.update({"c128_ms": p["c128_ms"], "speedup_vs_c128": p["speedup_c64_vs_c128"],
                  "c128_max_true_residual": p["c128_true_residual_max"],
                  "spectrum_rel_err_vs_c128": p["spectrum_rel_err_vs_c128"]["max"],
                  "replacements": p["c64_replacements"]})
    else:
        b = out["batched"]
        s.update({"separate_same_precision_ms": b["separate_ms"],
                  "speedup_vs_separate_same_precision": b["speedup_batched_vs_separate"],
                  "separate_split_ms": b["separate_split_ms"], "group": out["group"],
                  "separate_c128_ms": b["plain_c128_separate_ms"],
                  "speedup_vs_c128": b["speedup_batched_vs_plain_c128"],
                  "spectrum_rel_err_vs_c128": b["spectrum_rel_err_vs_c128"]["max"],
                  "apply_block_GBs": b["apply_block_GBs"], "apply_one_GBs": b["apply_one_GBs"],
                  "apply_block_interleaved_GBs": b["apply_block_interleaved_GBs"]})
    return s


def run_solver_workload(wl_name, args, extras=True, cpu=True):
    """One solver workload: ground state, timed solve steps and, optionally,
    its extras and the CPU baseline; returns the JSON object."""
    import numpy as np
    import torch

    import paper_2506_09551_amd as msb
    import workloads as W

    assert torch.cuda.is_available(), "bench needs the GPU"
    dev = torch.device("cuda:0")
    wl = W.get(wl_name)
    prec = msb.MSB_C128 if wl.dtype == "c128" else msb.MSB_C64
    cdt = torch.complex128 if prec == msb.MSB_C128 else torch.complex64
    log(f"workload {wl.name}: D={wl.dim} systems={wl.nrhs} shifts={len(wl.w_in)}")

    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    D = msb.msb_dim(ctx)

    # ---- precondition: ground state (timed once, outside the metric) -------
    x0 = torch.from_numpy(W.random_vector(D, wl.gs_seed)).to(dev)
    G = torch.empty(D, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E_G, gs_iters = msb.msb_ground_state(ctx, msb.make_system(), x0, 1e-10, 600, G)
    torch.cuda.synchronize()
    gs_ms = (time.perf_counter() - t0) * 1e3
    log(f"ground state E_G={E_G:.12f} ({gs_iters} Lanczos steps, {gs_ms:.1f} ms)")

    # right-hand sides E_j = O2_j G
    E = torch.empty(wl.nrhs, D, dtype=torch.complex128, device=dev)
    for j, w2 in enumerate(wl.o2_weights):
        site, wu, wd = (-1, 1.0, 1.0) if w2 is None else (wl.core_sites[j], w2[0], w2[1])
        msb.msb_number_op(ctx, site, wu, wd, G, E[j])
    systems = [msb.make_system(core_site=c, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma, t_amp=wl.t_amp_sys)
               for c in wl.core_sites]
    n_shift = len(wl.w_in)
    # apply launch shape: the autotuner's table for this batch (the solve reuses the winner)
    tune_table = msb.msb_autotune(ctx, wl.nrhs, prec)
    log("autotune " + " ".join(f"{t[0]}x{t[1]}/nv{t[2]}/p{t[3]}/o{t[4]}/w{t[6]}:{t[5]:.4f}ms" for t in tune_table))
    psi = torch.empty(wl.nrhs, n_shift, D, dtype=cdt, device=dev)
    torch.cuda.synchronize()

    ok = (msb.MSB_OK, msb.MSB_FLOOR) if prec == msb.MSB_C64 else (msb.MSB_OK,)
    step_opts = dict(C64_OPTS or {}) if prec == msb.MSB_C64 else {}
    if getattr(args, "assembly_engine", None) is not None:
        step_opts["assembly_engine"] = args.assembly_engine
    step_opts = step_opts or None

    def step():
        st, info = msb.msb_solve(ctx, systems, E, wl.w_in, wl.seed_shift, args.tol, wl.maxit, prec, psi,
                                 want_true=True, raise_on_fail=False, opts=step_opts)
        if st not in ok:
            raise msb.MsbError(st, msb.lib().msb_last_error().decode())
        info["status_name"] = msb.STATUS[st]
        return st, info

    for i in range(args.warmup):
        _, info = step()
        log(f"warmup {i}: iters={info['iters']} t_iter={info['t_iter_ms']:.1f} ms "
            f"t_flush={info['t_flush_ms']:.1f} ms t_true={info['t_true_ms']:.1f} ms "
            f"setup={info['t_setup_ms']:.1f} alloc={info['t_alloc_ms']:.1f} wall={info['t_wall_ms']:.1f} ms "
            f"flushes={info['flushes']}")
    torch.cuda.synchronize()
    infos = []
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record()
    for i in range(args.steps):
        _, info = step()
        infos.append(info)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = max(start.elapsed_time(stop), wall * 1e3)
    ms_per_step = ms_total / args.steps
    value = wl.nrhs * n_shift / (ms_per_step / 1e3)
    last = infos[-1]
    max_true = float(np.max(last["resid_true"]))
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, max true residual {max_true:.2e}; last: "
        f"setup={last['t_setup_ms']:.1f} alloc={last['t_alloc_ms']:.1f} wall={last['t_wall_ms']:.1f} ms "
        f"flushes={last['flushes']}")

    # ---- dominant kernel roofline: the dense multi-shift assembly ----------
    gemm_ms = sum(i["t_gemm_ms"] for i in infos) / max(1, sum(i["n_gemm"] for i in infos))
    gemm_flops = last["gemm_flops"] / max(1, last["n_gemm"])
    gemm_tflops = gemm_flops / (gemm_ms * 1e-3) / 1e12
    split = {
        "seed_iterations_ms": sum(i["t_iter_ms"] for i in infos) / args.steps,
        "assembly_ms": sum(i["t_flush_ms"] for i in infos) / args.steps,
        "true_residual_ms": sum(i["t_true_ms"] for i in infos) / args.steps,
    }
    roofline = {
        "bound": "alu",
        "kernel": "k_flush_gauss (dense multi-shift assembly, three-product FP64 VALU)",
        "achieved": round(gemm_tflops, 3),
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(gemm_tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
        "traffic": (None if flush_traffic_gb(wl.name) is None else round(flush_traffic_gb(wl.name), 2)),
        "traffic_unit": "GB per launch (HBM, rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
        "per_launch": {"flops": gemm_flops, "avg_ms": gemm_ms,
                       "alg_bytes": last["gemm_bytes"] / max(1, last["n_gemm"])},
    }

    out = {
        "metric": "Ψ_int shift-solves/sec at rel. residual 1e-8; H-apply HBM GB/s vs peak",
        "value": round(value, 2),
        "unit": "shift-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if prec == msb.MSB_C128 else "c64",
        "data": "synthetic",
        "config": {
            "workload": wl.note, "name": wl.name, "D": D, "systems": wl.nrhs, "shifts": n_shift,
            "tol": args.tol, "Gamma": wl.Gamma, "U": wl.U, "Uc": wl.Uc,
        },
        "iters": last["iters"],
        "solve_status": last["status_name"],
        "group": int(last["group"]), "bank_slots": int(last["bank_slots"]),
        "apply_shape": {"threads": last["apply_shape"][0], "elems_per_thread": last["apply_shape"][1],
                        "systems_per_workgroup": last["apply_shape"][2], "passes": last["apply_shape"][3],
                        "row_order": last["apply_shape"][4], "panel_width": last["apply_shape"][5]},
        "autotune_ms": {f"{t[0]}x{t[1]}/nv{t[2]}/passes{t[3]}/order{t[4]}" + (f"/w{t[6]}" if t[3] == 3 else ""):
                        round(t[5], 5)
                        for t in sorted(tune_table, key=lambda t: t[5])[:6]},   # the six fastest
        "mvms_per_step": last["mvms"],
        "max_true_residual": max_true,
        "split_ms": {k: round(v, 3) for k, v in split.items()},
        "roofline": roofline,
        "ground_state": {"E_G": E_G, "lanczos_steps": gs_iters, "ms": round(gs_ms, 2)},
    }

    if extras and wl.nrhs > 1 and prec == msb.MSB_C64:
        out["batched"] = batched_extras(msb, ctx, wl, systems, E, psi, ms_per_step, args.tol, prec, E_G)
    elif extras and prec == msb.MSB_C64:
        box = [psi]       # hand the only reference over so the c64 result can be freed
        del psi
        out["precision"] = precision_extras(msb, ctx, wl, systems, E, E_G, box, last, ms_per_step, args.tol)
    elif extras:
        happly = h_apply_rates(msb, ctx, wl, systems, prec)
        out["h_apply"] = happly
        log(f"h_apply {happly}")

        # continued-fraction spectrum of the coherent site sum (stage 2)
        phases = wl.phases
        phi = torch.empty(n_shift, D, dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        msb.msb_combine(ctx, psi, wl.nrhs, n_shift, prec, phases, phi)
        # continued fraction converged to 1e-8 of the peak (10 more levels change I by less)
        I, depth = msb.msb_spectrum(ctx, msb.make_system(E_G=E_G), phi, wl.w_loss, wl.eta, 1500, 1e-8)
        torch.cuda.synchronize()
        cf_ms = (time.perf_counter() - t0) * 1e3
        out["spectrum"] = {"ms": round(cf_ms, 1), "lanczos_depth_max": int(depth.max()),
                           "lanczos_depth_mean": float(depth.mean()), "I_max": float(I.max())}
        log(f"spectrum {out['spectrum']}")
        del phi

        # the multi-shift assembly engines on this step (one solve each; the
        # default is the one the timed steps used)
        engines = {}
        for eng in range(7):
            _, inf = msb.msb_solve(ctx, systems, E, wl.w_in, wl.seed_shift, args.tol, wl.maxit, prec, psi,
                                   want_true=False, raise_on_fail=False, opts={"assembly_engine": eng})
            ms = inf["t_gemm_ms"] / max(1, inf["n_gemm"])
            engines[str(eng)] = {"ms": round(ms, 3),
                                 "TFLOPs": round(inf["gemm_flops"] / max(1, inf["n_gemm"]) / (ms * 1e-3) / 1e12, 2)}
        out["assembly_engines"] = {"note": "0: three real products per complex product (default); 1: FP64 "
                                           "matrix cores; 2: four real products; 3, 4: variants of 0; 5: int8 "
                                           "matrix cores on 8-bit digit planes; 6: FP64 matrix cores, three "
                                           "products, bank staged in LDS (TFLOPs counts the contraction's "
                                           "algorithmic flops)",
                                   **engines}
        log(f"assembly engines {out['assembly_engines']}")

    if cpu and prec == msb.MSB_C128:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(wl, last["iters"])
        log(f"cpu baseline {out['cpu_baseline']['value']:.3f} shift-solves/s")
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        out["cpu_baseline_all_cores"] = cpu_baseline(wl, last["iters"], threads=ncpu)
        log(f"cpu baseline, {ncpu} threads: {out['cpu_baseline_all_cores']['value']:.3f} shift-solves/s")

    if args.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 8
        del src, dst

    msb.msb_destroy(ctx)
    psi = None                      # (the precision extras already dropped their reference)
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--apply-only", action="store_true",
                    help="only the H-apply rates (--steps applies per shape)")
    ap.add_argument("--assembly-engine", type=int, default=None,
                    help="multi-shift assembly engine of the timed steps (msb_opts.assembly_engine)")
    ap.add_argument("--no-forms", action="store_true",
                    help="scale workload: skip the precision and batched forms")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--train-spectra", type=int, default=4096, help="learned form: training spectra")
    ap.add_argument("--heldout-spectra", type=int, default=256, help="learned form: held-out spectra")
    ap.add_argument("--epochs", type=float, default=2.0, help="learned form: passes over the training set")
    ap.add_argument("--mlp-train-steps", type=int, default=0,
                    help="learned form: only time this many training steps on seeded random points")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the solver has no multi-GPU path; run with --gpus 1"}))
        sys.exit(2)
    if args.workload == "learned" and args.mlp_train_steps > 0:
        mlp_train_main(args)
        return
    if args.workload == "learned":
        learned_main(args)
        return
    if args.workload == "reseed":
        reseed_main(args)
        return
    if args.workload == "dipole":
        dipole_main(args)
        return
    if args.apply_only:
        # the H-apply rates alone (for profiling the apply kernels)
        import paper_2506_09551_amd as msb
        import workloads as W
        wl = W.get("scale")
        ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
        systems = [msb.make_system(core_site=c, Uc=wl.Uc, E_G=-4.0, Gamma=wl.Gamma) for c in wl.core_sites]
        out = {"metric": "H-apply HBM GB/s", "h_apply": h_apply_rates(msb, ctx, wl, systems, msb.MSB_C128,
                                                                     reps=args.steps)}
        msb.msb_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    out = run_solver_workload(args.workload, args, extras=not args.no_extras, cpu=not args.no_cpu)
    if args.workload == "scale" and not args.no_forms:
        # the precision and batched forms beside the plain solver, each on its
        # own workload, against complex128 (and separate solves)
        import torch
        fargs = argparse.Namespace(**dict(vars(args), steps=2, warmup=1))
        out["forms"] = {}
        for name in ("precision", "batched"):
            log(f"form {name} ...")
            sub = run_solver_workload(name, fargs, extras=True, cpu=False)
            out["forms"][name] = form_summary(name, sub)
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
