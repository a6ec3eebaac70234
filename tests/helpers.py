"""Shared test helpers: synthetic problems, oracle references and the
mapping between the oracle's and the library's reference-space order."""
import functools
import math

import numpy as np

import synth.problems as SP
from oracle import run
from oracle.classes import ClassOracle

CLASSES = [(2, 2), (1, 2), (0, 2), (2, 1), (1, 1), (0, 1), (2, 0), (1, 0), (0, 0)]


def host_tensors(pb):
    """torch CPU tensors (h, [B_t]) of a problem."""
    return SP.one_body(pb), SP.factors(pb)


@functools.lru_cache(maxsize=8)
def oracle_reference(name, q_mode=0):
    """Oracle E2 parts, E0 and the oracle's ground-state C for a named small
    problem (see SMALL) or a config."""
    pb = problem(name)
    h, Bs = host_tensors(pb)
    ws = SP.weights(pb)
    co = run.class_oracle(pb, h.numpy(), [B.numpy() for B in Bs], ws)
    H, E0 = co.reference(np.ones(len(co.P), dtype=np.complex128))
    w, v = np.linalg.eigh(H)
    c = v[:, 0]
    k = int(np.argmax(np.abs(c)))
    c = c * (abs(c[k]) / c[k])
    parts, E0 = co.e2(c, q_mode)
    return parts, E0, c, co.P


SMALL = {
    # name: (seed, n_fc, n_c, subs, n_elec, n_v, sets, max_hops, base)
    "s_cas": (101, 0, 3, [4], 2, 9, [(14, 1.0), (6, -0.03)], SP.CAS, None),
    "s_das": (102, 0, 4, [3, 3], 3, 10, [(16, 1.0)], 1, [2, 1]),
    "s_fc": (103, 2, 3, [2, 3], 3, 8, [(12, 1.0), (5, -0.02), (5, 0.01)], 1, [1, 2]),
    "s_hop0": (104, 1, 2, [2, 2, 2], 3, 7, [(10, 1.0)], 0, [1, 1, 1]),
    "s_tiles": (105, 0, 3, [3], 2, 70, [(20, 1.0)], SP.CAS, None),   # > one 64-wide virtual tile
    "s_single": (106, 0, 4, [], 0, 9, [(12, 1.0)], SP.CAS, None),     # single determinant
    "s_nocore": (107, 0, 0, [4], 2, 6, [(10, 1.0)], SP.CAS, None),    # no core spinors
    "s_full": (108, 0, 2, [3], 3, 5, [(8, 1.0)], SP.CAS, None),       # active space full
    # wide active spaces: class (1,2) couples through 20, 24 and 32 active
    # spinors, which selects the dense-coefficient kernels sized for up to
    # 24 and 32 couplings (and the adjoint's 20-, 24- and 32-wide forms);
    # s_j20 has 190 strings in that class (three 64-string chunks, the last
    # one partial)
    "s_j20": (109, 0, 2, [20], 3, 10, [(16, 1.0), (6, -0.02)], SP.CAS, None),
    "s_j24": (110, 1, 3, [12, 12], 2, 9, [(14, 1.0)], 1, [1, 1]),
    "s_j32": (111, 0, 2, [32], 2, 8, [(12, 1.0), (4, 0.01)], SP.CAS, None),
}


def problem(name):
    if name in SMALL:
        seed, nfc, nc, subs, ne, nv, sets, hops, base = SMALL[name]
        return SP.small(name, seed, nfc, nc, subs, ne, nv, sets, max_hops=hops, base=base)
    return SP.config(name)


def to_plan_order(c_oracle, oracle_P, plan_bits, n_c):
    """Reorder the oracle's C (over its sorted P list of correlated-space
    determinants) into the plan's order (active bit strings)."""
    pos = {d: i for i, d in enumerate(oracle_P)}
    idx = [pos[int(b) << n_c] for b in plan_bits]
    return np.asarray(c_oracle)[idx]


def e2_total(parts):
    return math.fsum(parts.values())
