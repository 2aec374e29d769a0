"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench.

This module holds only the *description* of each workload: lattice geometry
(the list of hopping bonds), model parameters, incident-energy and energy-loss
grids, and seeded random numbers.  It contains none of the method's
arithmetic: no basis, no Hamiltonian, no solver and no spectrum code.  Both
the CPU oracle (``oracle/``) and the HIP library receive these values as plain
arguments, so neither side imports the other.

Models follow the single-band Hubbard Hamiltonian with nearest-neighbour
hopping t and next-nearest-neighbour hopping t' (paper Sec. III, Eq.
``Hubbard``); the core hole adds U_c on one site of the intermediate-state
Hamiltonian (Eq. ``intermediate_H``).  Energies are in units of t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "chain_bonds", "square_bonds", "Workload", "WORKLOADS", "get",
    "random_vector", "random_complex", "sobol_params", "sector_dim",
]


def chain_bonds(L: int, t: float = 1.0, tp: float = 0.0, periodic: bool = True):
    """Bonds (i, j, t_ij) of an L-site chain.

    Nearest-neighbour bonds carry ``t``; if ``tp`` is non-zero, next-nearest
    bonds (i, i+2) carry ``tp``.  With ``periodic`` the wrap-around bonds are
    included as ordinary bonds.  Each unordered pair appears once.
    """
    bonds = []
    seen = set()

    def add(i, j, amp):
        key = (min(i, j), max(i, j))
        if i == j or key in seen:
            return
        seen.add(key)
        bonds.append((i, j, float(amp)))

    for i in range(L):
        j = i + 1
        if j < L:
            add(i, j, t)
        elif periodic:
            add(i, j % L, t)
    if tp != 0.0:
        for i in range(L):
            j = i + 2
            if j < L:
                add(i, j, tp)
            elif periodic:
                add(i, j % L, tp)
    return bonds


def square_bonds(Lx: int, Ly: int, t: float = 1.0, tp: float = 0.0):
    """Bonds of an Lx x Ly periodic square cluster; site index = x + Lx*y.

    Nearest neighbours (x+1, y), (x, y+1) carry ``t``; diagonal neighbours
    (x+1, y+1), (x+1, y-1) carry ``tp``.  Each unordered pair appears once.
    """
    bonds = []
    seen = set()

    def site(x, y):
        return (x % Lx) + Lx * (y % Ly)

    def add(a, b, amp):
        key = (min(a, b), max(a, b))
        if a == b or key in seen:
            return
        seen.add(key)
        bonds.append((a, b, float(amp)))

    for y in range(Ly):
        for x in range(Lx):
            s = site(x, y)
            add(s, site(x + 1, y), t)
            add(s, site(x, y + 1), t)
    if tp != 0.0:
        for y in range(Ly):
            for x in range(Lx):
                s = site(x, y)
                add(s, site(x + 1, y + 1), tp)
                add(s, site(x + 1, y - 1), tp)
    return bonds


def sector_dim(L: int, n_up: int, n_dn: int) -> int:
    """Dimension of the fixed-(N_up, N_dn) sector: C(L, N_up) * C(L, N_dn)."""
    return math.comb(L, n_up) * math.comb(L, n_dn)


@dataclass
class Workload:
    """One synthetic workload: model, right-hand sides and grids."""
    name: str
    n_sites: int
    n_up: int
    n_dn: int
    bonds: list
    U: float
    Uc: float
    Gamma: float
    w_in: np.ndarray            # incident energies (measured from the edge)
    tol: float
    dtype: str                  # "c128" or "c64"
    core_sites: list            # core-hole site of each right-hand side
    o2_weights: list            # (w_up, w_dn) of O2 = w_up n_up(j) + w_dn n_dn(j); None = identity
    phases: list                # complex phase of each right-hand side in the coherent sum
    w_loss: np.ndarray = field(default_factory=lambda: np.zeros(0))
    eta: float = 0.1
    gs_seed: int = 12345
    seed_shift: float = 0.0
    maxit: int = 2000
    dipole_spin: int = -1       # >= 0: O2_j = c+_{j spin}, O1_j = c_{j spin} (intermediate sector N_spin + 1)
    t_amp_sys: list = None      # per-system bond-type amplitudes of H' (None: the model's)
    note: str = ""

    @property
    def dim(self) -> int:
        return sector_dim(self.n_sites, self.n_up, self.n_dn)

    @property
    def nrhs(self) -> int:
        return len(self.core_sites)


def _tiny():
    L = 8
    return Workload(
        name="tiny_L8_N4", n_sites=L, n_up=4, n_dn=4,
        bonds=chain_bonds(L, 1.0), U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-10.0, 10.0, 64), tol=1e-13, dtype="c128",
        core_sites=[0], o2_weights=[None], phases=[1.0 + 0j],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1,
        note="L=8 ring, N=4+4, D=4900, 64 shifts in [-10,10], 256 losses in [0,10]")


def _scale():
    L = 12
    q = math.pi / 2
    return Workload(
        name="scale_L12_N6", n_sites=L, n_up=6, n_dn=6,
        bonds=chain_bonds(L, 1.0, 0.0), U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-12.0, 12.0, 200), tol=1e-10, dtype="c128",
        core_sites=list(range(L)), o2_weights=[None] * L,
        phases=[complex(math.cos(q * j), math.sin(q * j)) for j in range(L)],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1,
        note="L=12 ring, N=6+6, D=853776, 12 core-hole sites x 200 shifts in [-12,12], q=pi/2")


def _precision():
    L = 14
    return Workload(
        name="precision_L14_N7", n_sites=L, n_up=7, n_dn=7,
        bonds=chain_bonds(L, 1.0), U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-12.0, 12.0, 256), tol=1e-8, dtype="c64",
        core_sites=[0], o2_weights=[None], phases=[1.0 + 0j],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1,
        note="L=14 ring, N=7+7, D=11778624, 256 shifts in [-12,12]")


def _batched():
    # Two core-hole sites x two diagonal O2 patterns (charge-like n_up+n_dn,
    # spin-like n_up-n_dn) -> four real right-hand sides.
    return Workload(
        name="batched_4x4_N5", n_sites=16, n_up=5, n_dn=5,
        bonds=square_bonds(4, 4, 1.0, -0.25), U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-10.0, 10.0, 64), tol=1e-8, dtype="c64",
        core_sites=[0, 0, 5, 5], o2_weights=[(1.0, 1.0), (1.0, -1.0), (1.0, 1.0), (1.0, -1.0)],
        phases=[1.0 + 0j] * 4,
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1,
        note="4x4 periodic, t'=-0.25, N=5+5, D=19079424, 4 RHS x 64 shifts in [-10,10]")


def _learned():
    L = 10
    return Workload(
        name="learned_L10_N5", n_sites=L, n_up=5, n_dn=5,
        bonds=chain_bonds(L, 1.0, -0.2), U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-10.0, 10.0, 128), tol=1e-8, dtype="c128",
        core_sites=[0], o2_weights=[None], phases=[1.0 + 0j],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1,
        note="L=10 ring, N=5+5, D=63504; per-sample (U, t', Uc, Gamma) vary")


def _reseed():
    # a narrow core-hole broadening and an edge seed: the seed converges far
    # faster than the resonant shifts it carries (Appendix E's setting)
    L = 10
    return Workload(
        name="reseed_L10_N5", n_sites=L, n_up=5, n_dn=5,
        bonds=chain_bonds(L, 1.0), U=8.0, Uc=-4.0, Gamma=0.3,
        w_in=np.linspace(-12.0, 12.0, 128), tol=1e-10, dtype="c128",
        core_sites=[0], o2_weights=[None], phases=[1.0 + 0j],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1, seed_shift=-12.0, maxit=4000,
        note="L=10 ring, N=5+5, D=63504, Gamma=0.3, 128 shifts in [-12,12], initial seed w_in=-12")


def _dipole():
    # direct edge with a valence electron added at the core-hole site: the
    # ground state in (6, 6), the intermediate states in (7, 6)
    L = 12
    q = math.pi / 2
    return Workload(
        name="dipole_L12_N6", n_sites=L, n_up=6, n_dn=6,
        bonds=chain_bonds(L, 1.0, 0.0), U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-12.0, 12.0, 200), tol=1e-8, dtype="c128",
        core_sites=list(range(L)), o2_weights=[None] * L,
        phases=[complex(math.cos(q * j), math.sin(q * j)) for j in range(L)],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1, dipole_spin=0,
        note="L=12 ring, ground state N=6+6, intermediate N=7+6 (D=731808) with O2_j = c+_{j up}, "
             "O1_j = c_{j up}; 12 core-hole sites x 200 shifts in [-12,12], q=pi/2")


def _dual():
    # the scale workload with non-reciprocal hopping in H' (e^{+g} to the right,
    # e^{-g} back, g = 0.2): the ground state is the symmetric ring's, the
    # intermediate Hamiltonians are not symmetric
    L = 12
    q = math.pi / 2
    g = 0.2
    return Workload(
        name="dual_L12_N6", n_sites=L, n_up=6, n_dn=6,
        bonds=[(i, (i + 1) % L, 1.0, 1.0) for i in range(L)], U=8.0, Uc=-4.0, Gamma=1.0,
        w_in=np.linspace(-12.0, 12.0, 200), tol=1e-8, dtype="c128",
        core_sites=list(range(L)), o2_weights=[None] * L,
        phases=[complex(math.cos(q * j), math.sin(q * j)) for j in range(L)],
        w_loss=np.linspace(0.0, 10.0, 256), eta=0.1, t_amp_sys=[math.exp(g), math.exp(-g)],
        note="L=12 ring, N=6+6, D=853776; H' with hopping e^{0.2} right / e^{-0.2} left; "
             "12 core-hole sites x 200 shifts in [-12,12]")


WORKLOADS = {
    "tiny": _tiny,
    "scale": _scale,
    "precision": _precision,
    "batched": _batched,
    "learned": _learned,
    "reseed": _reseed,
    "dipole": _dipole,
    "dual": _dual,
}


def get(name: str) -> Workload:
    return WORKLOADS[name]()


def random_vector(dim: int, seed: int) -> np.ndarray:
    """Seeded standard-normal real vector (float64)."""
    return np.random.default_rng(seed).standard_normal(dim)


def random_complex(dim: int, seed: int) -> np.ndarray:
    """Seeded complex vector with standard-normal real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(dim) + 1j * rng.standard_normal(dim)


def sobol_params(n: int, seed: int = 7, skip: int = 0) -> np.ndarray:
    """Scrambled-Sobol samples of (U, t', U_c, Gamma) in the learned-form box.

    Ranges: U in [4, 12], t' in [-0.4, 0], U_c in [-6, -2], Gamma in [0.5, 2].
    """
    from scipy.stats import qmc
    eng = qmc.Sobol(d=4, scramble=True, seed=seed)
    if skip:
        eng.fast_forward(skip)
    u = eng.random(n)
    lo = np.array([4.0, -0.4, -6.0, 0.5])
    hi = np.array([12.0, 0.0, -2.0, 2.0])
    return lo + u * (hi - lo)


# ---- learned form: inputs of the surrogate network -------------------------
# Feature order (U, t', U_c, Gamma, w_in, w) and the box each feature spans.
SURROGATE_LO = np.array([4.0, -0.4, -6.0, 0.5, -10.0, 0.0])
SURROGATE_HI = np.array([12.0, 0.0, -2.0, 2.0, 10.0, 10.0])


def surrogate_normalisation():
    """(shift, scale) mapping every feature's box onto [-1, 1]."""
    shift = 0.5 * (SURROGATE_LO + SURROGATE_HI)
    scale = 2.0 / (SURROGATE_HI - SURROGATE_LO)
    return shift, scale


def mlp_init(seed: int, widths=(6, 512, 512, 512, 1)) -> np.ndarray:
    """Seeded initial parameters (flat float32, layout W1 b1 W2 b2 ...): weights
    uniform in +-sqrt(6 / fan_in) (He), the output layer scaled by 0.1, biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(widths) - 1
    for i in range(L):
        lim = np.sqrt(6.0 / widths[i]) * (0.1 if i == L - 1 else 1.0)
        parts.append(rng.uniform(-lim, lim, widths[i] * widths[i + 1]))
        parts.append(np.zeros(widths[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def permutations(members: int, steps: int, batch: int, n_points: int, seed: int) -> np.ndarray:
    """[members][steps * batch] int32 point indices: each member walks its own
    shuffled passes over the n_points training points."""
    rng = np.random.default_rng(seed)
    need = steps * batch
    out = np.empty((members, need), dtype=np.int32)
    for m in range(members):
        idx = []
        have = 0
        while have < need:
            p = rng.permutation(n_points)
            idx.append(p)
            have += n_points
        out[m] = np.concatenate(idx)[:need]
    return out


def permutations_device(members: int, steps: int, batch: int, n_points: int, seed: int, device):
    """As ``permutations`` but drawn on the device with torch's seeded
    generator (for training sets of 10^8 points): [members][steps * batch] int32."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    need = steps * batch
    out = torch.empty((members, need), dtype=torch.int32, device=device)
    for m in range(members):
        have = 0
        while have < need:
            p = torch.randperm(n_points, generator=g, device=device, dtype=torch.int64)
            k = min(n_points, need - have)
            out[m, have:have + k] = p[:k].to(torch.int32)
            have += k
    return out
