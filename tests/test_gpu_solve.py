"""Parity of the multi-shift solve (HIP) with the oracle's direct solves.

The oracle solves (H' - E_G - w - i Gamma) Psi = E for every shift by a
dense eigendecomposition / LU; the GPU runs the multi-shift COCG with the
residual bank and the dense multi-shift assembly.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hubbard as hb
from oracle import solve as osolve
from tests._cases import oracle_H, small_models

pytestmark = pytest.mark.gpu


def _run(msb, ctx, systems, E, w, tol, maxit, prec, seed_shift=0.0, opts=None, want_true=True,
         raise_on_fail=True, hist_len=0):
    import torch
    D = msb.msb_dim(ctx)
    n = len(systems)
    Et = torch.from_numpy(np.ascontiguousarray(E.reshape(n, D))).to(torch.complex128).cuda()
    dt = torch.complex128 if prec == msb.MSB_C128 else torch.complex64
    psi = torch.empty(n, len(w), D, dtype=dt, device="cuda")
    st, info = msb.msb_solve(ctx, systems, Et, w, seed_shift, tol, maxit, prec, psi,
                             want_true=want_true, opts=opts, raise_on_fail=raise_on_fail,
                             hist_len=hist_len)
    torch.cuda.synchronize()
    return st, info, psi.cpu().numpy().astype(np.complex128)


def _rel(a, b):
    return np.max(np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1))


@pytest.fixture(scope="module")
def tiny(gpu):
    msb = gpu
    wl = W.get("tiny")
    m = dict(L=wl.n_sites, nu=wl.n_up, nd=wl.n_dn, bonds=wl.bonds, U=wl.U)
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    yield msb, ctx, wl, m
    msb.msb_destroy(ctx)


def test_tiny_all_shifts_match_direct_solve(tiny):
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 3).astype(np.complex128)
    E_G = -2.6661474201323485
    Hp = oracle_H(m, core_site=0, Uc=wl.Uc)
    ref = osolve.direct_solve(Hp, E, E_G, wl.Gamma, wl.w_in, method="eig")
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in, 1e-13, 3000, msb.MSB_C128)
    err = _rel(psi[0], ref)
    assert err <= 1e-10, f"max rel err {err:.3e}"
    assert info["mvms"] == info["iters"]
    assert np.all(info["shift_iters"] > 0)
    assert np.max(info["resid_true"]) <= 1e-11


def test_release_workspace_then_solve_again(tiny):
    """Freeing the workspace between two identical solves changes nothing:
    the second call allocates it again and gives the same bits."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 4).astype(np.complex128)
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.6661474201323485, Gamma=wl.Gamma)
    _, info1, psi1 = _run(msb, ctx, [sysd], E, wl.w_in, 1e-10, 3000, msb.MSB_C128)
    msb.msb_release_workspace(ctx)
    msb.msb_release_workspace(ctx)          # a second release is a no-op
    _, info2, psi2 = _run(msb, ctx, [sysd], E, wl.w_in, 1e-10, 3000, msb.MSB_C128)
    assert info2["t_alloc_ms"] > 0.0
    assert info1["iters"] == info2["iters"]
    assert np.array_equal(psi1, psi2)


def test_seed_shift_and_batched_systems(tiny):
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    systems = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for j in (0, 3, 5)]
    E = np.stack([W.random_complex(D, 20 + j) for j in range(3)])
    w = np.linspace(-6.0, 9.0, 37)
    st, info, psi = _run(msb, ctx, systems, E, w, 1e-12, 3000, msb.MSB_C128, seed_shift=1.5)
    for j, s in enumerate(systems):
        ref = osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=wl.Uc), E[j], E_G,
                                  wl.Gamma, w, method="eig")
        err = _rel(psi[j], ref)
        assert err <= 1e-9, f"system {j}: {err:.3e}"


@pytest.mark.parametrize("direct_ap", [0, 1])
def test_seed_forms_agree(tiny, direct_ap):
    """The recurred seed form (A p_m = A r_m + beta_{m-1} A p_{m-1}, the default)
    and the direct one (A p_m applied, as Algorithm 1 writes it) both match the
    direct solves, and their seed residual histories agree while rounding has
    not yet separated them."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    systems = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for j in (0, 2, 4)]
    E = np.stack([W.random_complex(D, 40 + j) for j in range(3)])
    w = np.linspace(-5.0, 8.0, 29)
    st, info, psi = _run(msb, ctx, systems, E, w, 1e-12, 3000, msb.MSB_C128, seed_shift=0.5,
                         opts={"direct_ap": direct_ap}, hist_len=3001)
    for j, s in enumerate(systems):
        ref = osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=wl.Uc), E[j], E_G,
                                  wl.Gamma, w, method="eig")
        assert _rel(psi[j], ref) <= 1e-9
    assert info["mvms"] == int(np.sum(info["sys_iters"]))   # one product per iteration
    assert np.max(info["resid_true"]) <= 1e-11
    _, info_o, psi_o = _run(msb, ctx, systems, E, w, 1e-12, 3000, msb.MSB_C128, seed_shift=0.5,
                            opts={"direct_ap": 1 - direct_ap}, hist_len=3001)
    for j in range(3):
        n = min(info["sys_iters"][j], info_o["sys_iters"][j])
        assert abs(int(info["sys_iters"][j]) - int(info_o["sys_iters"][j])) <= max(2, n // 30)
        k = min(40, int(n))
        h, ho = info["seed_hist"][j][:k], info_o["seed_hist"][j][:k]
        assert np.max(np.abs(h - ho) / ho) <= 1e-9
    assert _rel(psi.reshape(-1, D), psi_o.reshape(-1, D)) <= 1e-9


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_solve_with_lds_panel_apply(tiny, prec):
    """The solve with its seed applies pinned to each LDS column-panel shape
    (the recurred sigma-fused apply in complex128, the direct one in complex64;
    the residual check keeps a single pass) matches the direct solves."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    p = msb.MSB_C128 if prec == "c128" else msb.MSB_C64
    systems = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for j in (0, 3, 5)]
    E = np.stack([W.random_complex(D, 60 + j) for j in range(3)])
    w = np.linspace(-6.0, 9.0, 23)
    refs = [osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=wl.Uc), E[j], E_G, wl.Gamma, w, method="eig")
            for j, s in enumerate(systems)]
    table = [t for t in msb.msb_autotune(ctx, 3, p) if t[3] == 3]
    assert table
    try:
        for shape in table:
            msb.msb_set_shape(ctx, 3, p, shape)
            tol, bar = (1e-12, 1e-9) if prec == "c128" else (1e-6, 5e-5)
            st, info, psi = _run(msb, ctx, systems, E, w, tol, 3000, p)
            assert info["apply_shape"][3] == 3 and info["apply_shape"][5] == shape[6]
            for j in range(3):
                err = _rel(psi[j], refs[j])
                assert err <= bar, f"{prec} shape {shape[:5] + shape[6:]} system {j}: {err:.3e}"
    finally:
        msb.msb_set_shape(ctx, 3, p, None)


@pytest.mark.parametrize("case", ["plain", "small_bank", "c64_replace"])
def test_large_batch_runs_in_two_parts(tiny, case):
    """Nine systems (the recurred seed then runs as two parts of 4 and 5 on two
    streams): every shift of every system against its direct solve, and the
    same iterations per system as the direct form, which runs unsplit; also
    with bank restarts and in complex64 with residual replacement, in the
    direct seed form (complex64 always runs that form)."""
    msb, ctx, wl, m = tiny
    opts = {"small_bank": {"bank_slots": 40}, "c64_replace": {"replace_every": 20}}.get(case, {})
    c64 = case.startswith("c64")
    prec = msb.MSB_C64 if c64 else msb.MSB_C128
    tol, bar = (1e-6, 5e-5) if c64 else (1e-12, 1e-9)
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    L = m["L"]
    systems = [msb.make_system(core_site=j % L, Uc=wl.Uc - 0.25 * (j // L), E_G=E_G, Gamma=wl.Gamma)
               for j in range(9)]
    E = np.stack([W.random_complex(D, 80 + j) for j in range(9)])
    w = np.linspace(-6.0, 8.0, 23)
    st, info, psi = _run(msb, ctx, systems, E, w, tol, 3000, prec, opts=opts, hist_len=3001)
    for j, s in enumerate(systems):
        ref = osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=s.Uc), E[j], E_G,
                                  wl.Gamma, w, method="eig")
        assert _rel(psi[j], ref) <= bar, f"system {j}"
    if case == "small_bank":
        assert info["flushes"] > 1
    if c64:
        assert st == msb.MSB_OK
        assert info["replacements"] > 0
        assert np.max(info["resid_true"]) <= 20 * tol
        return
    assert np.max(info["resid_true"]) <= 1e-11
    _, info_d, _ = _run(msb, ctx, systems, E, w, tol, 3000, prec, opts=dict(opts, direct_ap=1),
                        hist_len=3001)
    for j in range(9):
        n = int(min(info["sys_iters"][j], info_d["sys_iters"][j]))
        assert abs(int(info["sys_iters"][j]) - int(info_d["sys_iters"][j])) <= max(2, n // 30)
        k = min(40, n)
        assert np.max(np.abs(info["seed_hist"][j][:k] - info_d["seed_hist"][j][:k])
                      / info_d["seed_hist"][j][:k]) <= 1e-9


def test_memory_bound_batch_runs_in_groups(tiny):
    """A batch whose residual banks do not fit in the allowed memory runs in
    groups of systems whose banks hold at least 512 slots each, so that no
    flush before the last iteration (which also assembles the search
    directions) is needed; only when no group reaches 512 slots does the
    whole batch run with a short bank and carried directions.  Both plans
    give every system's solution to the direct solve's and the unlimited
    solve's accuracy.  (Budgets of about 100 MB and 34 MB for four systems of
    D = 4,900: the first holds 2 x ~600 slots but not 3 x 512, the second
    4 x 64 but not 1 x 512.)"""
    import torch
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    systems = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for j in range(4)]
    E = np.stack([W.random_complex(D, 140 + j) for j in range(4)])
    w = np.linspace(-6.0, 8.0, 16)
    tol = 1e-12
    _, info_u, psi_u = _run(msb, ctx, systems, E, w, tol, 3000, msb.MSB_C128)
    assert info_u["group"] == 4 and info_u["bank_slots"] == 1024 and info_u["flushes"] == 1
    ctx2 = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        for budget, want_group in ((100e6, 2), (34e6, 4)):
            msb.msb_release_workspace(ctx2)
            free = torch.cuda.mem_get_info()[0]
            st, info, psi = _run(msb, ctx2, systems, E, w, tol, 3000, msb.MSB_C128,
                                 opts={"mem_fraction": budget / free})
            assert st == msb.MSB_OK
            assert info["group"] == want_group, (budget, info["group"], info["bank_slots"])
            if want_group == 2:
                assert info["bank_slots"] >= 512
                assert info["iters"] < info["bank_slots"]
                assert info["flushes"] == 2                  # one per group, none carried
            else:
                assert info["bank_slots"] < 512
                assert info["flushes"] > 1
            for j, s in enumerate(systems):
                ref = osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=s.Uc), E[j], E_G,
                                          wl.Gamma, w, method="eig")
                assert _rel(psi[j], ref) <= 1e-9, f"system {j}"
                assert _rel(psi[j], psi_u[j]) <= 1e-10, f"system {j}"
            assert np.max(info["resid_true"]) <= 1e-11
    finally:
        msb.msb_destroy(ctx2)


def test_c64_batch_of_four_unsplit(tiny):
    """Four systems with real right-hand sides (as E = O_2 G of the workloads)
    in one batch: complex64 with residual replacement against the direct
    solves, at the precision workload's default schedule (replacement every
    50 iterations)."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    systems = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for j in (0, 2, 5, 7)]
    E = np.stack([W.random_vector(D, 120 + j) for j in range(4)]).astype(np.complex128)
    w = np.linspace(-10.0, 10.0, 31)
    st, info, psi = _run(msb, ctx, systems, E, w, 1e-6, 3000, msb.MSB_C64)
    assert st == msb.MSB_OK and info["replacements"] > 0
    for j, s in enumerate(systems):
        ref = osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=wl.Uc), E[j], E_G, wl.Gamma, w,
                                  method="eig")
        assert _rel(psi[j], ref) <= 5e-5, f"system {j}"
    assert np.max(info["resid_true"]) <= 20 * 1e-6


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_interleaved_block_apply_matches_per_system_vectors(tiny, prec):
    """The direct seed form on five systems (groups of four and two
    interleaved systems would leave a ragged group) with the interleaved
    block apply and with one vector per system: both against the direct
    solves, the same iterations, and seed residual histories that agree while
    rounding has not separated them."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E_G = -2.6661474201323485
    c64 = prec == "c64"
    systems = [msb.make_system(core_site=j, Uc=wl.Uc - 0.3 * (j % 2), E_G=E_G, Gamma=wl.Gamma) for j in range(5)]
    E = np.stack([W.random_vector(D, 140 + j) for j in range(5)]).astype(np.complex128)
    w = np.linspace(-8.0, 8.0, 21)
    tol, bar = (1e-6, 5e-5) if c64 else (1e-12, 1e-9)
    p = msb.MSB_C64 if c64 else msb.MSB_C128
    runs = {}
    for il in (1, 0):
        runs[il] = _run(msb, ctx, systems, E, w, tol, 3000, p, opts={"direct_ap": 1, "interleave": il},
                        hist_len=3001)
        st, info, psi = runs[il]
        assert st == msb.MSB_OK
        for j, s in enumerate(systems):
            ref = osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=s.Uc), E[j], E_G, wl.Gamma, w,
                                      method="eig")
            assert _rel(psi[j], ref) <= bar, (il, j)
    assert runs[1][1]["apply_shape"][2] in (2, 4) and runs[1][1]["apply_shape"][3] == 2   # interleaved, two passes
    for j in range(5):
        n = int(min(runs[1][1]["sys_iters"][j], runs[0][1]["sys_iters"][j]))
        assert abs(int(runs[1][1]["sys_iters"][j]) - int(runs[0][1]["sys_iters"][j])) <= max(2, n // 30)
        k = min(30, n)
        h0, h1 = runs[1][1]["seed_hist"][j][:k], runs[0][1]["seed_hist"][j][:k]
        assert np.max(np.abs(h0 - h1) / h1) <= (1e-4 if c64 else 1e-9)


def test_two_part_batch_is_deterministic(tiny):
    """The two parts of a split batch share no mutable state, so two solves give
    the same bits whatever the interleaving of their streams."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    systems = [msb.make_system(core_site=j % m["L"], Uc=wl.Uc, E_G=-2.6661474201323485, Gamma=wl.Gamma)
               for j in range(8)]
    E = np.stack([W.random_complex(D, 90 + j) for j in range(8)])
    w = np.linspace(-4.0, 6.0, 17)
    _, i1, p1 = _run(msb, ctx, systems, E, w, 1e-11, 3000, msb.MSB_C128)
    _, i2, p2 = _run(msb, ctx, systems, E, w, 1e-11, 3000, msb.MSB_C128)
    assert np.array_equal(i1["sys_iters"], i2["sys_iters"])
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("direct_ap", [0, 1])
@pytest.mark.parametrize("slots", [5, 37, 120])
def test_small_bank_forces_carry_flushes(tiny, slots, direct_ap):
    """A bank smaller than the iteration count: blocked assembly with carried p^w
    (in the recurred seed form A p_{m-1} simply carries over the bank restart)."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 5).astype(np.complex128)
    E_G = -2.6661474201323485
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    w = wl.w_in[::3]
    ref = osolve.direct_solve(oracle_H(m, core_site=0, Uc=wl.Uc), E, E_G, wl.Gamma, w, method="eig")
    st, info, psi = _run(msb, ctx, [sysd], E, w, 1e-12, 3000, msb.MSB_C128,
                         opts={"bank_slots": slots, "direct_ap": direct_ap})
    assert info["flushes"] > 1
    err = _rel(psi[0], ref)
    assert err <= 1e-9, f"slots={slots}: {err:.3e}"


def test_matches_reference_recurrence_iteration_count(tiny):
    """Same freeze iteration per shift as the oracle's Algorithm-1 recurrence (up to +-1)."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 9).astype(np.complex128)
    E_G = -2.6661474201323485
    Hp = oracle_H(m, core_site=0, Uc=wl.Uc)
    A = lambda x: Hp @ x - (E_G + 1j * wl.Gamma) * x
    ref = osolve.msbicg_reference(A, E, wl.w_in, 1e-10, 3000)
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in, 1e-10, 3000, msb.MSB_C128)
    # the freeze test compares a residual that flattens near the threshold, so
    # rounding can move the crossing by a few iterations
    slack = max(2, int(0.03 * ref.iters))
    assert abs(info["iters"] - ref.iters) <= slack
    assert np.max(np.abs(info["shift_iters"][0] - ref.conv_iter)) <= slack
    err = _rel(psi[0], ref.psi)
    assert err <= 1e-8


def test_c64_form_accuracy(tiny):
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 4).astype(np.complex128)
    E_G = -2.6661474201323485
    ref = osolve.direct_solve(oracle_H(m, core_site=0, Uc=wl.Uc), E, E_G, wl.Gamma, wl.w_in,
                              method="eig")
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in, 1e-6, 3000, msb.MSB_C64)
    err = _rel(psi[0], ref)
    assert err <= 5e-5, f"c64 rel err {err:.3e}"


@pytest.mark.parametrize("opts", [None, {"replace_every": 7, "chunk": 3},
                                  {"replace_every": 20, "bank_slots": 33}])
def test_c64_residual_replacement(tiny, opts):
    """complex64 vectors with residual replacement r_m <- E - A_s x_m (complex128,
    x_m rebuilt from the bank slots at each replacement): same accuracy as the
    plain form, replacements counted, and with a small bank the replacement
    survives the flush / bank restart."""
    msb, ctx, wl, m = tiny
    opts = dict(opts or {})
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 4).astype(np.complex128)
    E_G = -2.6661474201323485
    ref = osolve.direct_solve(oracle_H(m, core_site=0, Uc=wl.Uc), E, E_G, wl.Gamma, wl.w_in,
                              method="eig")
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in, 1e-6, 3000, msb.MSB_C64, opts=opts,
                         hist_len=3001)
    # replacement happens at the first chunk boundary at least `period`
    # iterations after the previous one (at most period + chunk apart), while
    # the seed residual is above tol |E|
    period = (opts or {}).get("replace_every", 50)
    chunk = (opts or {}).get("chunk", min(period, 64))
    hist = info["seed_hist"][0]
    m_seed = int(np.argmax(hist <= 1e-6))
    assert 0 < m_seed < info["iters"]
    assert info["replacements"] >= max(m_seed // (period + chunk) - 1, 1)
    assert info["replacements"] <= m_seed // period + 1
    err = _rel(psi[0], ref)
    assert err <= 5e-5, f"c64 rel err {err:.3e}"
    # after a replacement the recurrence residual tracks the true one
    assert np.max(info["resid_true"]) <= 20 * 1e-6
    st0, info0, psi0 = _run(msb, ctx, [sysd], E, wl.w_in, 1e-6, 3000, msb.MSB_C64,
                            opts={"replace_every": -1})
    assert info0["replacements"] == 0
    assert _rel(psi0[0], ref) <= 5e-5


def test_recurred_form_is_complex128_only(tiny):
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 4).astype(np.complex128)
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.66, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in[:4], 1e-6, 100, msb.MSB_C64,
                         opts={"direct_ap": -1}, raise_on_fail=False, want_true=False)
    assert st == msb.MSB_EINVAL


def test_c64_replacement_tight_tol(tiny):
    """tol far below complex64 resolution: replacements pull the seed down to
    FP64 accuracy (the replaced residual is the FP64 true one), then stop, and
    the shifted systems converge on the unperturbed recurrence as in the plain
    form; Psi keeps complex64 accuracy."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 4).astype(np.complex128)
    E_G = -2.6661474201323485
    ref = osolve.direct_solve(oracle_H(m, core_site=0, Uc=wl.Uc), E, E_G, wl.Gamma, wl.w_in,
                              method="eig")
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in, 1e-13, 3000, msb.MSB_C64)
    st0, info0, _ = _run(msb, ctx, [sysd], E, wl.w_in, 1e-13, 3000, msb.MSB_C64,
                         opts={"replace_every": -1})
    assert st == msb.MSB_OK and info["replacements"] >= 4
    assert info["iters"] <= 1.3 * info0["iters"]
    assert _rel(psi[0], ref) <= 5e-5
    assert np.max(info["resid_true"]) <= 2e-5


def test_breakdown_reported(tiny):
    """E = e_0 + i e_1 has E^T E = 0: COCG cannot start (rho_0 = 0)."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = np.zeros(D, dtype=np.complex128)
    E[0] = 1.0
    E[1] = 1.0j
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.0, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in[:4], 1e-10, 100, msb.MSB_C128,
                         raise_on_fail=False, want_true=False)
    assert st == msb.MSB_BREAKDOWN
    assert info["breakdown_iter"] == 0


def test_not_converged_reported(tiny):
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_vector(D, 2).astype(np.complex128)
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.66, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in[:8], 1e-12, 3, msb.MSB_C128,
                         raise_on_fail=False)
    assert st == msb.MSB_NOT_CONVERGED
    assert info["iters"] == 3
    assert np.all(np.isfinite(psi))


def test_zero_rhs_gives_zero(tiny):
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = np.zeros(D, dtype=np.complex128)
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=-2.0, Gamma=wl.Gamma)
    st, info, psi = _run(msb, ctx, [sysd], E, wl.w_in[:5], 1e-10, 100, msb.MSB_C128,
                         want_true=False)
    assert st == msb.MSB_OK
    assert np.all(psi == 0)


@pytest.mark.parametrize("name", ["chain8_doped", "square3x3_doped"])
def test_other_models(gpu, name):
    msb = gpu
    m = small_models()[name]
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        E = W.random_vector(D, 31).astype(np.complex128)
        E_G = -1.0
        w = np.linspace(-8, 8, 7)
        sysd = msb.make_system(core_site=1, Uc=-3.0, E_G=E_G, Gamma=0.8)
        st, info, psi = _run(msb, ctx, [sysd], E, w, 1e-12, 4000, msb.MSB_C128)
        Hp = oracle_H(m, core_site=1, Uc=-3.0)
        ref = osolve.direct_solve(Hp, E, E_G, 0.8, w, method="eig")
        err = _rel(psi[0], ref)
        assert err <= 1e-9, f"{name}: {err:.3e}"
    finally:
        msb.msb_destroy(ctx)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("engine", [0, 1, 2, 3, 4, 5, 6, 7])
def test_assembly_engines_match_direct_solve(tiny, engine, prec):
    """Every multi-shift assembly engine (three-product vector ALU and its two
    variants, FP64 matrix cores with four products, four-product vector ALU,
    int8 matrix cores on digit planes (six planes for complex128 banks, five
    for complex64), FP64 matrix cores with three products (complex64 banks
    take the vector engine), and 7, the vector engine in every case), with
    and without carry
    (a 41-slot bank), in both storage precisions; 70 shifts span more than one
    shift tile with a ragged last one, and D = 4900 ends in a ragged element
    tile."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    c64 = prec == "c64"
    E = W.random_vector(D, 41).astype(np.complex128) if c64 else W.random_complex(D, 41)
    tol, bar = (1e-6, 5e-5) if c64 else (1e-12, 1e-9)
    E_G = -2.6661474201323485
    sysd = [msb.make_system(core_site=j, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for j in (0, 2)]
    w = np.linspace(-9.0, 9.0, 70)                 # more than one shift tile, ragged
    refs = [osolve.direct_solve(oracle_H(m, core_site=s.core_site, Uc=wl.Uc), E, E_G, wl.Gamma, w,
                                method="eig") for s in sysd]
    for slots in (0, 41):
        st, info, psi = _run(msb, ctx, sysd, np.stack([E, E]), w, tol, 3000,
                             msb.MSB_C64 if c64 else msb.MSB_C128,
                             opts={"assembly_engine": engine, "bank_slots": slots})
        for j in range(2):
            err = _rel(psi[j], refs[j])
            assert err <= bar, f"engine {engine} slots {slots} system {j}: {err:.3e}"


@pytest.mark.parametrize("engine", [5, 6])
def test_matrix_core_engines_many_shifts_match_direct_solve(tiny, engine):
    """The matrix-core assemblies over 300 shifts (19 tiles of 16): the int8
    engine (5) in two groups of 256 shift slots, the second ragged; the FP64
    engine (6) in two groups of 10 and 9 tiles, four of each shared by two
    wavefronts.  With and without carry (a 37-slot bank, so several flushes
    add into the output and carry p).  Against the oracle's direct solves at
    1e-9 (tol 1e-12), and against the FP64 three-product vector engine on the
    same bank to 1e-10 relative (engine 5 keeps 46 bits of every operand per
    64-slot chunk; engine 6 differs by rounding only)."""
    msb, ctx, wl, m = tiny
    D = msb.msb_dim(ctx)
    E = W.random_complex(D, 45)
    E_G = -2.6661474201323485
    sysd = [msb.make_system(core_site=1, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma)]
    w = np.linspace(-11.0, 11.0, 300)
    ref = osolve.direct_solve(oracle_H(m, core_site=1, Uc=wl.Uc), E, E_G, wl.Gamma, w, method="eig")
    for slots in (0, 37):
        _, _, psi5 = _run(msb, ctx, sysd, E, w, 1e-12, 3000, msb.MSB_C128,
                          opts={"assembly_engine": engine, "bank_slots": slots})
        _, _, psi0 = _run(msb, ctx, sysd, E, w, 1e-12, 3000, msb.MSB_C128,
                          opts={"assembly_engine": 0, "bank_slots": slots})
        assert _rel(psi5[0], ref) <= 1e-9, f"slots {slots}"
        assert _rel(psi5[0], psi0[0]) <= 1e-10, f"slots {slots}: {_rel(psi5[0], psi0[0]):.3e}"


@pytest.mark.parametrize("engine", [0, 5])
def test_c64_odd_dimension(gpu, engine):
    """An odd D (L = 7 ring, N = 3 + 3, D = 1225): complex64 slots are not
    16-byte aligned, so the assembly (the default, and the int8 engine when
    asked for) falls back to the four-product vector engine."""
    msb = gpu
    m = dict(L=7, nu=3, nd=3, bonds=W.chain_bonds(7, 1.0), U=6.0)
    ctx = msb.msb_create(m["L"], m["nu"], m["nd"], m["bonds"], m["U"])
    try:
        D = msb.msb_dim(ctx)
        assert D % 2 == 1
        E = W.random_vector(D, 43).astype(np.complex128)
        w = np.linspace(-6.0, 6.0, 19)
        sysd = msb.make_system(core_site=2, Uc=-3.0, E_G=-1.5, Gamma=0.9)
        for slots in (0, 17):
            st, info, psi = _run(msb, ctx, [sysd], E, w, 1e-6, 2000, msb.MSB_C64,
                                 opts={"bank_slots": slots, "assembly_engine": engine})
            ref = osolve.direct_solve(oracle_H(m, core_site=2, Uc=-3.0), E, -1.5, 0.9, w, method="eig")
            assert _rel(psi[0], ref) <= 5e-5
    finally:
        msb.msb_destroy(ctx)


@pytest.mark.parametrize("wl_name", ["scale", "precision", "batched"])
def test_full_size_solve_sampled_rows(gpu, wl_name):
    """The workloads at full size in the bench's configuration (all systems and
    shifts of one msb_solve call): the equation (A - w)Psi = E checked by the
    oracle's row-by-row operator on sampled rows of sampled (system, shift)
    pairs, and the library's own FP64 true residuals."""
    import torch
    msb = gpu
    from tests._cases import basis
    wl = W.get(wl_name)
    ctx = msb.msb_create(wl.n_sites, wl.n_up, wl.n_dn, wl.bonds, wl.U)
    try:
        D = msb.msb_dim(ctx)
        x0 = torch.from_numpy(W.random_vector(D, wl.gs_seed)).cuda()
        G = torch.empty(D, dtype=torch.float64, device="cuda")
        E_G, _ = msb.msb_ground_state(ctx, msb.make_system(), x0, 1e-10, 600, G)
        E = torch.empty(wl.nrhs, D, dtype=torch.complex128, device="cuda")
        for j, w2 in enumerate(wl.o2_weights):
            site, wu, wd = (-1, 1.0, 1.0) if w2 is None else (wl.core_sites[j], w2[0], w2[1])
            msb.msb_number_op(ctx, site, wu, wd, G, E[j])
        systems = [msb.make_system(core_site=c, Uc=wl.Uc, E_G=E_G, Gamma=wl.Gamma) for c in wl.core_sites]
        prec = msb.MSB_C128 if wl.dtype == "c128" else msb.MSB_C64
        dt = torch.complex128 if prec == msb.MSB_C128 else torch.complex64
        n = len(wl.w_in)
        psi = torch.empty(wl.nrhs, n, D, dtype=dt, device="cuda")
        tol = 1e-8
        st, info = msb.msb_solve(ctx, systems, E, wl.w_in, wl.seed_shift, tol, wl.maxit, prec, psi,
                                 want_true=True, raise_on_fail=False)
        assert st in ((msb.MSB_OK,) if prec == msb.MSB_C128 else (msb.MSB_OK, msb.MSB_FLOOR))
        floor = tol if prec == msb.MSB_C128 else 2e-5          # complex64 storage of Psi
        assert np.max(info["resid_true"]) <= 1.01 * floor
        B = basis(wl.n_sites, wl.n_up, wl.n_dn)
        rng = np.random.default_rng(17)
        rows = np.unique(np.concatenate([rng.integers(0, D, 150), [0, D - 1]]))
        for s in sorted({0, wl.nrhs - 1}):
            Es = E[s].cpu().numpy()
            nE = np.linalg.norm(Es)
            for k in sorted({0, n // 3, n // 2, n - 1}):
                ps = psi[s, k].cpu().numpy().astype(np.complex128)
                sysd = systems[s]
                Ax = hb.apply_rows(B, wl.bonds, wl.U, ps, rows, core_site=sysd.core_site, Uc=sysd.Uc,
                                   shift=E_G + wl.w_in[k] + 1j * wl.Gamma)
                r = Es[rows] - Ax
                assert np.max(np.abs(r)) <= 1.01 * floor * nE, (s, k, np.max(np.abs(r)) / nE)
    finally:
        msb.msb_destroy(ctx)


@pytest.fixture(scope="module")
def sharp(tiny):
    """The L=8 ring with Gamma = 0.3 and the 64 shifts of the tiny workload
    widened to [-12, 12]: an edge seed exhausts before the resonant shifts."""
    msb, ctx, wl, m = tiny
    Hp = oracle_H(m, core_site=0, Uc=wl.Uc)
    H = oracle_H(m)
    from oracle import groundstate as ogs
    E_G, G, _ = ogs.dense_ground_state(H)
    w = np.linspace(-12.0, 12.0, 64)
    Gamma = 0.3
    E = G.astype(np.complex128)
    ref = osolve.direct_solve(Hp, E, E_G, Gamma, w, method="eig")
    sysd = msb.make_system(core_site=0, Uc=wl.Uc, E_G=E_G, Gamma=Gamma)
    return msb, ctx, sysd, E, w, ref


def test_edge_seed_exhaustion_reported(sharp):
    msb, ctx, sysd, E, w, ref = sharp
    st, info, psi = _run(msb, ctx, [sysd], E, w, 1e-10, 3000, msb.MSB_C128, seed_shift=-12.0,
                         raise_on_fail=False)
    assert st == msb.MSB_NOT_CONVERGED
    assert np.all(np.isfinite(psi))
    frozen = info["shift_iters"][0] >= 0
    assert 0 < frozen.sum() < len(w)
    err = np.linalg.norm(psi[0][frozen] - ref[frozen], axis=1) / np.linalg.norm(ref[frozen], axis=1)
    assert err.max() <= 1e-8
    assert np.all(info["resid_true"][0][~frozen] > 1e-10)


def test_reseeding_recovers_from_edge_seed(sharp):
    """Appendix E on the GPU: every shift ends at the direct solution; the
    final seeds are the edge seed (shifts it froze) and shifts of the list."""
    import torch
    msb, ctx, sysd, E, w, ref = sharp
    D = msb.msb_dim(ctx)
    Et = torch.from_numpy(E.reshape(1, D)).cuda()
    psi = torch.empty(1, len(w), D, dtype=torch.complex128, device="cuda")
    st, info = msb.msb_solve_reseed(ctx, [sysd], Et, w, -12.0, 1e-10, 3000, msb.MSB_C128, psi, 1e-9, 6)
    assert st == msb.MSB_OK
    assert info["rounds"][0] >= 2
    assert np.all(info["resid_true"][0] <= 1e-9)
    seeds = set(info["seed_of"][0])
    assert -12.0 in seeds and (seeds - {-12.0}) <= set(w)
    got = psi[0].cpu().numpy()
    err = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-8
    # round 0 keeps exactly the shifts the edge seed froze
    st0, info0, _ = _run(msb, ctx, [sysd], E, w, 1e-10, 3000, msb.MSB_C128, seed_shift=-12.0,
                         raise_on_fail=False)
    kept = info["seed_of"][0] == -12.0
    assert np.array_equal(kept, (info0["shift_iters"][0] >= 0) & (info0["resid_true"][0] <= 1e-9))


def test_reseeding_without_failures_is_the_plain_solve(sharp):
    import torch
    msb, ctx, sysd, E, w, ref = sharp
    D = msb.msb_dim(ctx)
    Et = torch.from_numpy(E.reshape(1, D)).cuda()
    psi = torch.empty(1, len(w), D, dtype=torch.complex128, device="cuda")
    st, info = msb.msb_solve_reseed(ctx, [sysd], Et, w, 0.0, 1e-10, 3000, msb.MSB_C128, psi, 1e-9, 6)
    assert st == msb.MSB_OK and info["rounds"][0] == 1 and np.all(info["seed_of"] == 0.0)
    _, _, psi0 = _run(msb, ctx, [sysd], E, w, 1e-10, 3000, msb.MSB_C128, seed_shift=0.0)
    assert np.array_equal(psi[0].cpu().numpy(), psi0[0])
    with pytest.raises(msb.MsbError):
        msb.msb_solve_reseed(ctx, [sysd], Et, w, 0.0, 1e-10, 3000, msb.MSB_C128, psi, 0.0, 6)
