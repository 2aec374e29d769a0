"""Hubbard and core-hole Hamiltonians in a fixed-(N_up, N_dn) sector (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definitions followed:

* H = -sum_{<ij>,sigma} t_ij (c+_{j sigma} c_{i sigma} + h.c.) + U sum_i n_{i up} n_{i dn}
  -- paper Sec. III, Eq. ``Hubbard``.
* H' = H + U_c (n_{j up} + n_{j dn}) for a core hole on site j -- the valence
  part of Eq. ``intermediate_H`` with the core-hole energy absorbed into
  omega_in; U_c < 0 is an attraction.

Fock-space convention (a plain choice, fixed here and nowhere else in the
oracle): a state is a 2L-bit integer s whose bit o is the occupation of
spin-orbital o, with o = site for spin up and o = L + site for spin down.
Basis kets are ordered products  c+_{o_1} c+_{o_2} ... |0>  with
o_1 < o_2 < ... .  Fermion operators act on s generically:
c_o |s> = (-1)^{#occupied orbitals below o} |s without o>, and likewise for
c+_o.  No Kronecker decomposition is used to build matrix elements.

Basis order (the vector layout shared with the GPU path through the
input description): index = rank_up(u) * n_dn + rank_dn(d), where u, d are the
up / down occupation bit strings and rank is the position in the ascending list
of L-bit integers with the given number of set bits.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def sector_configs(L: int, N: int) -> np.ndarray:
    """Ascending array of L-bit integers with exactly N set bits (int64)."""
    s = np.arange(1 << L, dtype=np.int64)
    return s[np.bitwise_count(s) == N]


class Basis:
    """Fixed-(N_up, N_dn) basis with the layout index = rank_up * n_dn + rank_dn."""

    def __init__(self, L: int, n_up: int, n_dn: int):
        if not (0 <= n_up <= L and 0 <= n_dn <= L):
            raise ValueError("electron numbers must lie in [0, L]")
        self.L, self.n_up, self.n_dn = L, n_up, n_dn
        self.up = sector_configs(L, n_up)
        self.dn = sector_configs(L, n_dn)
        self.nu, self.nd = len(self.up), len(self.dn)
        self.dim = self.nu * self.nd
        assert self.nu == math.comb(L, n_up) and self.nd == math.comb(L, n_dn)

    def states(self, idx=None) -> np.ndarray:
        """2L-bit Fock codes of basis states (all, or the given indices)."""
        if idx is None:
            idx = np.arange(self.dim, dtype=np.int64)
        idx = np.asarray(idx, dtype=np.int64)
        u = self.up[idx // self.nd]
        d = self.dn[idx % self.nd]
        return u | (d << self.L)

    def index(self, codes: np.ndarray) -> np.ndarray:
        """Basis index of 2L-bit Fock codes (must lie in the sector)."""
        codes = np.asarray(codes, dtype=np.int64)
        mask = (1 << self.L) - 1
        u = codes & mask
        d = codes >> self.L
        iu = np.searchsorted(self.up, u)
        idn = np.searchsorted(self.dn, d)
        ok = (iu < self.nu) & (idn < self.nd)
        ok &= self.up[np.minimum(iu, self.nu - 1)] == u
        ok &= self.dn[np.minimum(idn, self.nd - 1)] == d
        if not np.all(ok):
            raise ValueError("state outside the sector")
        return iu * self.nd + idn


def _parity_below(s: np.ndarray, o: int) -> np.ndarray:
    """(-1)^{number of occupied orbitals with index < o} for each code in s."""
    below = s & ((np.int64(1) << o) - 1)
    return 1 - 2 * (np.bitwise_count(below) & 1).astype(np.int64)


def hop_terms(basis: Basis, bonds, src_idx: np.ndarray, t_scale=None):
    """Matrix elements <dst| H_kin |src> for the given source states.

    For every bond (i, j, t), spin sigma and direction, applies
    -t * c+_{a} c_{b} (a, b the two spin-orbitals of the bond) to each source
    state with Jordan-Wigner signs from the generic operator action.  A bond
    (i, j, t, t_rev) is directed: -t c+_j c_i - t_rev c+_i c_j (an electron
    hops from i to j with t and back with t_rev; non-symmetric when they
    differ, as in non-reciprocal, dissipative models).
    Returns (dst_index, src_index, value) arrays.  ``t_scale`` optionally maps
    a bond's t to a replacement amplitude (used for per-parameter models).
    """
    L = basis.L
    src_idx = np.asarray(src_idx, dtype=np.int64)
    S = basis.states(src_idx)
    dst_all, src_all, val_all = [], [], []
    for bond in bonds:
        i, j, t = bond[0], bond[1], bond[2]
        t_rev = bond[3] if len(bond) > 3 else t
        amp = t if t_scale is None else t_scale(t)
        amp_rev = t_rev if t_scale is None else t_scale(t_rev)
        for sigma in (0, 1):
            oi, oj = i + sigma * L, j + sigma * L
            for a, b, am in ((oj, oi, amp), (oi, oj, amp_rev)):       # c+_j c_i, c+_i c_j
                occ_b = (S >> b) & 1
                occ_a = (S >> a) & 1
                m = (occ_b == 1) & (occ_a == 0)
                if not np.any(m):
                    continue
                s0 = S[m]
                sign1 = _parity_below(s0, b)          # c_b
                s1 = s0 ^ (np.int64(1) << b)
                sign2 = _parity_below(s1, a)          # c+_a
                s2 = s1 | (np.int64(1) << a)
                dst_all.append(basis.index(s2))
                src_all.append(src_idx[m])
                val_all.append(-am * (sign1 * sign2).astype(np.float64))
    if not dst_all:
        z = np.zeros(0, dtype=np.int64)
        return z, z, np.zeros(0)
    return np.concatenate(dst_all), np.concatenate(src_all), np.concatenate(val_all)


def diagonal(basis: Basis, U: float, core_site=None, Uc: float = 0.0, idx=None) -> np.ndarray:
    """Diagonal of H or H': U * #doubly-occupied + U_c * (n_{j up} + n_{j dn})."""
    S = basis.states(idx)
    L = basis.L
    mask = (np.int64(1) << L) - 1
    u = S & mask
    d = S >> L
    diag = U * np.bitwise_count(u & d).astype(np.float64)
    if core_site is not None and core_site >= 0:
        nj = ((u >> core_site) & 1) + ((d >> core_site) & 1)
        diag = diag + Uc * nj.astype(np.float64)
    return diag


def hamiltonian(basis: Basis, bonds, U: float, core_site=None, Uc: float = 0.0,
                t_scale=None) -> sp.csr_matrix:
    """Sparse real matrix of H (core_site None) or H' (core hole on core_site);
    symmetric unless some bond is directed (see ``hop_terms``)."""
    D = basis.dim
    dst, src, val = hop_terms(basis, bonds, np.arange(D, dtype=np.int64), t_scale)
    diag = diagonal(basis, U, core_site, Uc)
    rows = np.concatenate([dst, np.arange(D)])
    cols = np.concatenate([src, np.arange(D)])
    vals = np.concatenate([val, diag])
    return sp.csr_matrix((vals, (rows, cols)), shape=(D, D))


def apply_rows(basis: Basis, bonds, U: float, x: np.ndarray, rows, core_site=None,
               Uc: float = 0.0, shift: complex = 0.0) -> np.ndarray:
    """((H' - shift) x)[rows] evaluated row by row, without building the matrix.

    Uses that H' is real symmetric: the elements of row r are the hop terms
    generated from source state r.  Intended for sampled checks at dimensions
    where the full sparse matrix is too large to build.
    """
    if any(len(b) > 3 and b[3] != b[2] for b in bonds):
        raise ValueError("apply_rows needs a symmetric Hamiltonian")
    rows = np.asarray(rows, dtype=np.int64)
    dst, src, val = hop_terms(basis, bonds, rows)
    out = (diagonal(basis, U, core_site, Uc, idx=rows) - shift) * x[rows]
    pos = np.searchsorted(rows, src) if np.all(np.diff(rows) > 0) else None
    if pos is None:
        order = {int(r): k for k, r in enumerate(rows)}
        pos = np.array([order[int(s)] for s in src], dtype=np.int64)
    contrib = val * x[dst]
    out = out.astype(np.result_type(out, contrib))
    np.add.at(out, pos, contrib)
    return out


def number_op(basis: Basis, site: int, w_up: float, w_dn: float) -> np.ndarray:
    """Diagonal of O = w_up n_{site up} + w_dn n_{site dn} (a sector-preserving operator)."""
    S = basis.states()
    L = basis.L
    mask = (np.int64(1) << L) - 1
    u = S & mask
    d = S >> L
    return w_up * ((u >> site) & 1).astype(np.float64) + w_dn * ((d >> site) & 1).astype(np.float64)


def site_op(src: Basis, dst: Basis, site: int, spin: int, create: bool) -> sp.csr_matrix:
    """Matrix of c+_{site spin} (``create``) or c_{site spin} from the sector of
    ``src`` to the sector of ``dst`` (the dipole-type operators of Sec. III that
    change the electron number).

    Spin-orbital a = site + spin * L (all up orbitals first, then all down
    ones, the order the Hamiltonian's Jordan-Wigner signs assume); the
    operator acting on a Fock code picks up (-1)^{number of occupied orbitals
    with index < a}, as in ``hop_terms``.
    """
    L = src.L
    if dst.L != L:
        raise ValueError("sectors of different lattices")
    dn_up = (1 if create else -1) if spin == 0 else 0
    dn_dn = (1 if create else -1) if spin == 1 else 0
    if (dst.n_up, dst.n_dn) != (src.n_up + dn_up, src.n_dn + dn_dn):
        raise ValueError("destination sector does not match the operator")
    a = site + spin * L
    S = src.states()
    occ = (S >> a) & 1
    m = (occ == 0) if create else (occ == 1)
    s0 = S[m]
    sign = _parity_below(s0, a).astype(np.float64)
    s1 = (s0 | (np.int64(1) << a)) if create else (s0 ^ (np.int64(1) << a))
    rows = dst.index(s1)
    cols = np.nonzero(m)[0]
    return sp.csr_matrix((sign, (rows, cols)), shape=(dst.dim, src.dim))


def dipole_op(src: Basis, dst: Basis, coef, spin: int, create: bool) -> sp.csr_matrix:
    """sum_j coef[j] c+_{j spin} (or c_{j spin}): one spin species, complex coefficients per site."""
    out = sp.csr_matrix((dst.dim, src.dim), dtype=np.complex128)
    for j, c in enumerate(coef):
        if c != 0:
            out = out + complex(c) * site_op(src, dst, j, spin, create)
    return out
