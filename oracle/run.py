"""Drivers that feed synthetic problems to the oracle (test infrastructure)."""
import numpy as np

from . import integrals
from .classes import ClassOracle
from .space import ActiveSpace
from .literal import lowest_state, reference_hamiltonian, reference_energy


def space_of(pb):
    return ActiveSpace(pb.n_c, pb.sub_sizes, pb.n_elec, pb.base, pb.max_hops, pb.n_v)


def correlated_inputs(h, Bs, ws, n_fc):
    """numpy h^FC and factor sets over the correlated spinors."""
    h = np.asarray(h)
    Bs = [np.asarray(B) for B in Bs]
    return integrals.fold_frozen_core(h, Bs, ws, n_fc)


def full_eri_callable(Bs, ws):
    n = Bs[0].shape[1]
    idx = np.arange(n)
    g = integrals.eri_block(Bs, ws, idx, idx, idx, idx)
    return g, (lambda p, q, r, s: g[p, q, r, s])


def ground_state(space, h, g_callable):
    H = reference_hamiltonian(space, h, g_callable)
    e, c = lowest_state(H)
    return H, e, c


def class_oracle(pb, h, Bs, ws):
    hfc, Bc = correlated_inputs(h, Bs, ws, pb.n_fc)
    return ClassOracle(space_of(pb), hfc, Bc, ws)


__all__ = ["space_of", "correlated_inputs", "full_eri_callable", "ground_state",
           "class_oracle", "reference_energy"]
