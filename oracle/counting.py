"""Closed-form size of the external space (test infrastructure, oracle).

With the STP-DAS class rule (oracle.space.ActiveSpace.class_strings) the
number of external determinants with h core holes and v virtual electrons is
    C(n_c, h) * C(n_v, v) * sum over admissible active categories m of
    prod_k C(s_k, m_k).
For a complete active space (one subspace) the rule reduces to: at most two
core holes and at most two virtual electrons (the excitation restriction
stated with the MRCISD comparison in Sec. 3.3), and (h, v) != (0, 0).
"""
from math import comb


def class_count(space, h, v, q_mode=0):
    n_el = space.n_elec + h - v
    if n_el < 0 or n_el > space.n_a:
        return 0
    pcats = set(space.p_categories())
    tot = 0
    for m in space.categories(n_el):
        if space.level(m, v) > 2:
            continue
        if h == 0 and v == 0 and (m in pcats or q_mode == 1):
            continue
        w = 1
        for s, mk in zip(space.sub_sizes, m):
            w *= comb(s, mk)
        tot += w
    return comb(space.n_c, h) * comb(space.n_v, v) * tot


def external_count(space, q_mode=0):
    return {(h, v): class_count(space, h, v, q_mode) for h in range(3) for v in range(3)}


def cas_external_count(n_core, n_act, n_elec, n_virt):
    """N_Q for a CAS(n_elec, n_act) reference with n_core core and n_virt
    virtual spinors: sum over h, v <= 2, (h, v) != (0, 0)."""
    tot = 0
    for h in range(3):
        for v in range(3):
            if h == 0 and v == 0:
                continue
            tot += comb(n_core, h) * comb(n_virt, v) * comb(n_act, n_elec + h - v)
    return tot
