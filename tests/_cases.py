"""Shared builders for the tests: oracle objects and GPU contexts for a workload.

Inputs come from ``workloads`` only; expected values come from ``oracle`` only.
"""
from __future__ import annotations

import functools

import numpy as np

import workloads as W
from oracle import hubbard as hb


@functools.lru_cache(maxsize=None)
def basis(L, nu, nd):
    return hb.Basis(L, nu, nd)


def small_models():
    """Small models spanning chains, next-nearest hops and a 2D cluster."""
    return {
        "chain6": dict(L=6, nu=3, nd=3, bonds=W.chain_bonds(6, 1.0), U=8.0),
        "chain8": dict(L=8, nu=4, nd=4, bonds=W.chain_bonds(8, 1.0), U=8.0),
        "chain8_doped": dict(L=8, nu=3, nd=4, bonds=W.chain_bonds(8, 1.0, -0.3), U=6.0),
        "chain10_tp": dict(L=10, nu=5, nd=5, bonds=W.chain_bonds(10, 1.0, -0.2), U=8.0),
        "square4x4_n2": dict(L=16, nu=2, nd=2, bonds=W.square_bonds(4, 4, 1.0, -0.25), U=8.0),
        "square3x3": dict(L=9, nu=3, nd=3, bonds=W.square_bonds(3, 3, 1.0, -0.25), U=4.0),
        "square3x3_doped": dict(L=9, nu=2, nd=3, bonds=W.square_bonds(3, 3, 1.0, -0.25), U=6.0),
    }


def oracle_H(m, core_site=None, Uc=0.0):
    B = basis(m["L"], m["nu"], m["nd"])
    return hb.hamiltonian(B, m["bonds"], m["U"], core_site=core_site, Uc=Uc)
