"""Pins of the CPU oracle against facts fixed outside it: Jordan-Wigner
brute force, the paper's printed determinant counts, closed forms and exact
invariances.  CPU only."""
import json
import math
import os
from itertools import combinations

import numpy as np
import pytest

import synth.problems as SP
from oracle import counting, integrals, literal, run
from oracle.classes import ClassOracle
from oracle.space import ActiveSpace

from jw_bruteforce import e2_bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tensors(spec):
    h = SP.one_body(spec).numpy()
    Bs = [B.numpy() for B in SP.factors(spec)]
    return h, Bs, SP.weights(spec)


def ground(space, h, Bs, ws):
    g, gc = run.full_eri_callable(Bs, ws)
    H, e, c = run.ground_state(space, h, gc)
    return g, gc, H, c


def class_e2(space, h, Bs, ws, C, q_mode=0, b=0.0):
    parts, E0 = ClassOracle(space, h, Bs, ws).e2(C, q_mode, b=b)
    return math.fsum(parts.values()), parts, E0


# ---------------------------------------------------------------- brute force

JW_CASES = [
    # name, seed, n_fc, n_c, subs, n_elec, n_v, sets, max_hops, base
    ("jw_cas", 11, 0, 2, [4], 2, 6, [(8, 1.0), (4, -0.05)], SP.CAS, None),
    ("jw_das", 12, 0, 1, [2, 3], 3, 5, [(9, 1.0)], 1, [1, 2]),
    ("jw_fc", 13, 1, 2, [2, 2], 2, 5, [(8, 1.0), (3, 0.02)], 0, [1, 1]),
]


@pytest.mark.parametrize("case", JW_CASES, ids=[c[0] for c in JW_CASES])
def test_jordan_wigner_bruteforce(case):
    name, seed, n_fc, n_c, subs, ne, nv, sets, hops, base = case
    spec = SP.small(name, seed, n_fc, n_c, subs, ne, nv, sets, max_hops=hops, base=base)
    h, Bs, ws = tensors(spec)
    n = h.shape[0]
    # brute force on the unfolded problem: frozen spinors stay occupied
    idx = np.arange(n)
    g_full = integrals.eri_block(Bs, ws, idx, idx, idx, idx)
    sp = run.space_of(spec)
    fc_mask = (1 << n_fc) - 1
    p_dets = [fc_mask | (d << n_fc) for d in sp.p_dets()]
    P = set(p_dets)
    N = bin(p_dets[0]).count("1")
    Q = []
    for K in range(1 << n):
        if bin(K).count("1") != N or K in P or (K & fc_mask) != fc_mask:
            continue
        if min(bin(K ^ L).count("1") for L in p_dets) <= 4:
            Q.append(K)
    e2_bf, e0_bf, c_bf, _ = e2_bruteforce(h, g_full, p_dets, Q)
    # oracle on the folded problem
    hfc, Bc = run.correlated_inputs(h, Bs, ws, n_fc)
    g, gc, H, c = ground(sp, hfc, Bc, ws)
    e2_lit, e0_lit, parts, nq = literal.e2_literal(sp, hfc, gc, c_bf, 0)
    assert nq == len(Q)
    assert abs(e2_lit - e2_bf) < 1e-12 * max(1.0, abs(e2_bf))
    e2_cls, _, _ = class_e2(sp, hfc, Bc, ws, c_bf)
    assert abs(e2_cls - e2_bf) < 1e-12 * max(1.0, abs(e2_bf))


@pytest.mark.parametrize("case", JW_CASES[:2], ids=[c[0] for c in JW_CASES[:2]])
@pytest.mark.parametrize("q_mode", [0, 1])
def test_denominator_stats_bruteforce(case, q_mode):
    """Smallest |E0 - H_KK| per excitation class and the count below a
    threshold (Sec. 2.6) against a brute-force pass over every N-electron
    determinant within two replacements of P, its diagonal taken from the
    Slater-Condon rule (not from the pair energies the oracle uses)."""
    name, seed, n_fc, n_c, subs, ne, nv, sets, hops, base = case
    spec = SP.small(name, seed, n_fc, n_c, subs, ne, nv, sets, max_hops=hops, base=base)
    h, Bs, ws = tensors(spec)
    n = h.shape[0]
    sp = run.space_of(spec)
    g, gc, H, c = ground(sp, h, Bs, ws)
    E0 = literal.reference_energy(H, c)
    P = sp.p_dets()
    N = bin(P[0]).count("1")
    deltas = {}
    for K in range(1 << n):
        if bin(K).count("1") != N or K in set(P):
            continue
        if min(bin(K ^ L).count("1") for L in P) > 4:
            continue
        holes = sp.n_c - bin(K & sp.core_mask).count("1")
        virt = bin(K & sp.virt_mask).count("1")
        if q_mode == 1 and holes == 0 and virt == 0:
            continue
        d = abs(E0 - literal.matrix_element(K, K, h, gc).real)
        deltas.setdefault((holes, virt), []).append(d)
    allv = np.sort(np.concatenate([np.array(v) for v in deltas.values()]))
    k = len(allv) // 3
    thresh = 0.5 * (allv[k] + allv[k + 1])     # between two values: no tie at the threshold
    got = literal.denominator_stats(sp, h, gc, c, thresh, q_mode)
    assert set(got) == set(deltas)
    for cls, v in deltas.items():
        m, cnt = got[cls]
        assert abs(m - min(v)) <= 1e-12 * max(1.0, min(v)), (cls, m, min(v))
        assert cnt == sum(1 for x in v if x < thresh), cls


# ------------------------------------------------------------ level shift
# Sec. 2.6: 1/Delta -> Re 1/(Delta + i eps) with eps = b/Delta.  The oracle
# writes the shifted inverse as complex arithmetic; the pins below reach it
# by a linear solve over Q (Jordan-Wigner), by the real closed form
# Delta^3/(Delta^4 + b^2) (single determinant), and by its limits.

def jw_problem(case):
    name, seed, n_fc, n_c, subs, ne, nv, sets, hops, base = case
    spec = SP.small(name, seed, n_fc, n_c, subs, ne, nv, sets, max_hops=hops, base=base)
    h, Bs, ws = tensors(spec)
    n = h.shape[0]
    idx = np.arange(n)
    g_full = integrals.eri_block(Bs, ws, idx, idx, idx, idx)
    sp = run.space_of(spec)
    fc_mask = (1 << n_fc) - 1
    p_dets = [fc_mask | (d << n_fc) for d in sp.p_dets()]
    P = set(p_dets)
    N = bin(p_dets[0]).count("1")
    Q = [K for K in range(1 << n)
         if bin(K).count("1") == N and K not in P and (K & fc_mask) == fc_mask
         and min(bin(K ^ L).count("1") for L in p_dets) <= 4]
    return spec, h, Bs, ws, g_full, sp, p_dets, Q


@pytest.mark.parametrize("b", [0.05, 2.0])
@pytest.mark.parametrize("case", JW_CASES[:2], ids=[c[0] for c in JW_CASES[:2]])
def test_level_shift_jordan_wigner_bruteforce(case, b):
    spec, h, Bs, ws, g_full, sp, p_dets, Q = jw_problem(case)
    e2_bf, e0_bf, c_bf, _ = e2_bruteforce(h, g_full, p_dets, Q, b=b)
    e2_0, _, _, _ = e2_bruteforce(h, g_full, p_dets, Q)
    assert abs(e2_bf - e2_0) > 1e-9 * abs(e2_0)          # the shift is visible
    hfc, Bc = run.correlated_inputs(h, Bs, ws, spec.n_fc)
    g, gc, H, c = ground(sp, hfc, Bc, ws)
    e2_lit, _, _, _ = literal.e2_literal(sp, hfc, gc, c_bf, 0, b=b)
    assert abs(e2_lit - e2_bf) < 1e-12 * max(1.0, abs(e2_bf))
    e2_cls, _, _ = class_e2(sp, hfc, Bc, ws, c_bf, b=b)
    assert abs(e2_cls - e2_bf) < 1e-12 * max(1.0, abs(e2_bf))


@pytest.mark.parametrize("root", [1, 2])
def test_excited_reference_state_jordan_wigner(root):
    """State-specific E2_m (the index m of eq. pt2): with the m-th eigenvector
    of H_PP as reference, E0_m and the first-order vector are those of that
    state; the oracle (which takes E0 from C) reproduces the brute force."""
    spec, h, Bs, ws, g_full, sp, p_dets, Q = jw_problem(JW_CASES[1])
    e2_bf, e0_bf, c_bf, _ = e2_bruteforce(h, g_full, p_dets, Q, root=root)
    e2_g, e0_g, _, _ = e2_bruteforce(h, g_full, p_dets, Q)
    assert e0_bf > e0_g + 1e-6
    hfc, Bc = run.correlated_inputs(h, Bs, ws, spec.n_fc)
    g, gc, H, c = ground(sp, hfc, Bc, ws)
    e2_lit, e0_lit, _, _ = literal.e2_literal(sp, hfc, gc, c_bf, 0)
    assert abs(e2_lit - e2_bf) < 1e-12 * max(1.0, abs(e2_bf))
    e2_cls, _, E0c = class_e2(sp, hfc, Bc, ws, c_bf)
    assert abs(e2_cls - e2_bf) < 1e-12 * max(1.0, abs(e2_bf))


def test_level_shift_limits():
    """b -> 0 recovers eq. pt2en; for large b the shifted weight tends to
    Delta^3 / b^2, so b^2 E2 -> sum_K |sigma_K|^2 Delta_K^3; the shift
    shrinks every term, so |E2| decreases with b."""
    spec, h, Bs, ws, g_full, sp, p_dets, Q = jw_problem(JW_CASES[0])
    _, _, c_bf, _, (v, dq) = e2_bruteforce(h, g_full, p_dets, Q, vectors=True)
    hfc, Bc = run.correlated_inputs(h, Bs, ws, spec.n_fc)
    e0, _, _ = class_e2(sp, hfc, Bc, ws, c_bf)
    tiny, _, _ = class_e2(sp, hfc, Bc, ws, c_bf, b=1e-9)
    assert abs(tiny - e0) <= 1e-14 * abs(e0)
    big = 1e8                       # next term: relative max Delta^4 / b^2 ~ 1e-9 here
    eb, _, _ = class_e2(sp, hfc, Bc, ws, c_bf, b=big)
    lim = float(np.sum(np.abs(v) ** 2 * dq ** 3))
    assert abs(eb * big ** 2 - lim) <= 1e-8 * abs(lim)
    vals = [abs(class_e2(sp, hfc, Bc, ws, c_bf, b=x)[0]) for x in (0.0, 0.1, 1.0, 10.0)]
    assert all(a > b_ for a, b_ in zip(vals, vals[1:]))


def test_hermiticity_of_matrix_elements():
    spec = SP.small("herm", 21, 0, 2, [3], 2, 3, [(6, 1.0), (3, -0.1)])
    h, Bs, ws = tensors(spec)
    sp = run.space_of(spec)
    _, gc = run.full_eri_callable(Bs, ws)
    dets = [d for d in range(1 << sp.n) if bin(d).count("1") == sp.n_c + sp.n_elec]
    rng = np.random.default_rng(0)
    for _ in range(400):
        K, L = rng.choice(dets, 2)
        a = literal.matrix_element(int(K), int(L), h, gc)
        b = literal.matrix_element(int(L), int(K), h, gc)
        assert abs(a - np.conj(b)) < 1e-13
    for K in dets[:50]:
        assert abs(np.imag(literal.matrix_element(K, K, h, gc))) < 1e-13


# ---------------------------------------------------------- external space

def test_table3_and_hbr_counts():
    """Sec. 3.3 Table 3 (nDets of 4C-MRPT2) and Sec. 3.1 (HBr external
    space): the class rule with a CAS reference reproduces the printed
    counts; HBr's printed exponent differs by one (see fixture)."""
    with open(os.path.join(GOLDEN, "table3_counts.json")) as f:
        fx = json.load(f)
    for row in fx["systems"]:
        nq = counting.cas_external_count(row["n_core"], row["n_act"], row["n_elec_act"], row["n_virt"])
        assert nq == row["exact"]
        mant, ex = row["printed"]
        digits = len(str(mant).replace(".", "")) - 1
        scale = 10 ** (ex - digits)
        if row.get("exponent_differs"):
            scale //= 10
        printed = int(str(mant).replace(".", ""))
        # the paper rounds (Table 3) or truncates (HBr) to the printed digits
        assert printed in (round(nq / scale), nq // scale), row["system"]


DAS_CASES = [
    (2, [4], 2, 5, SP.CAS, None),
    (2, [2, 3], 3, 4, 1, [1, 2]),
    (1, [2, 2, 2], 3, 3, 1, [1, 1, 1]),
    (2, [3, 2], 2, 3, 0, [1, 1]),
]


@pytest.mark.parametrize("case", DAS_CASES)
@pytest.mark.parametrize("q_mode", [0, 1])
def test_external_space_rule_matches_enumeration(case, q_mode):
    n_c, subs, ne, nv, hops, base = case
    base = base or SP.default_base(subs, ne)
    sp = ActiveSpace(n_c, subs, ne, base, hops, nv)
    Q = sp.q_dets_literal(q_mode)
    by = {}
    for K in Q:
        cl = literal.external_class(sp, K)
        by[cl] = by.get(cl, 0) + 1
    cnt = counting.external_count(sp, q_mode)
    for cl, v in cnt.items():
        assert by.get(cl, 0) == v, (cl, by.get(cl, 0), v)
    # class strings agree with the enumeration too
    for (h, v), c in cnt.items():
        assert len(sp.class_strings(h, v, q_mode)) * math.comb(n_c, h) * math.comb(nv, v) == c


def test_das_reduces_to_cas():
    """One subspace, or a hop limit >= the electron count, gives the CAS."""
    a = ActiveSpace(2, [6], 3, [3], SP.CAS, 4)
    b = ActiveSpace(2, [2, 2, 2], 3, [1, 1, 1], 3, 4)
    assert sorted(a.p_strings()) == sorted(b.p_strings())
    assert len(a.p_strings()) == math.comb(6, 3)
    assert counting.external_count(a) == counting.external_count(b)


# ------------------------------------------------------------- closed forms

def single_det_problem(seed, n_c, n_v, rank, lam=1.0, zero_g=False):
    spec = SP.small("sd", seed, 0, n_c, [], 0, n_v, [(rank, 1.0)])
    h = SP.one_body(spec).numpy()
    B = SP.factors(spec)[0].numpy() * math.sqrt(lam)
    if zero_g:
        B = B * 0.0
    return spec, h, [B], [1.0]


def test_single_determinant_closed_form():
    """n_a = 0: P = {core}; EN-PT2 from Fock-matrix singles and
    antisymmetrised doubles with explicit Epstein-Nesbet diagonals."""
    spec, h, Bs, ws = single_det_problem(31, 4, 7, 12)
    n_c, n = 4, h.shape[0]
    idx = np.arange(n)
    g = integrals.eri_block(Bs, ws, idx, idx, idx, idx)
    occ, vir = list(range(n_c)), list(range(n_c, n))
    W = np.array([[(g[p, p, q, q] - g[p, q, q, p]).real if p != q else 0.0
                   for q in range(n)] for p in range(n)])
    hd = np.diag(h).real
    E0 = hd[occ].sum() + sum(W[i, j] for i, j in combinations(occ, 2))
    f = h + sum(g[:, :, j, j] - g[:, j, j, :] for j in occ)
    e2 = 0.0
    for i in occ:
        for a in vir:
            rest = [j for j in occ if j != i]
            Hkk = hd[rest].sum() + hd[a] + sum(W[p, q] for p, q in combinations(rest + [a], 2))
            e2 += abs(f[a, i]) ** 2 / (E0 - Hkk)
    for i, j in combinations(occ, 2):
        for a, b in combinations(vir, 2):
            rest = [k for k in occ if k not in (i, j)]
            Hkk = hd[rest].sum() + hd[a] + hd[b] + sum(W[p, q] for p, q in combinations(rest + [a, b], 2))
            amp = (g[a, i, b, j] - g[a, j, b, i])
            e2 += abs(amp) ** 2 / (E0 - Hkk)
    sp = run.space_of(spec)
    got, parts, E0o = class_e2(sp, h, Bs, ws, np.array([1.0 + 0j]))
    assert abs(E0o - E0) < 1e-10
    assert abs(got - e2) < 1e-12 * abs(e2)
    assert set(k for k, v in parts.items() if v != 0.0) <= {(1, 1), (2, 2)}


def test_level_shift_single_determinant_closed_form():
    """n_a = 0 with the level shift: every Epstein-Nesbet term takes the real
    weight Delta^3 / (Delta^4 + b^2)."""
    spec, h, Bs, ws = single_det_problem(31, 4, 7, 12)
    b = 3.0
    n_c, n = 4, h.shape[0]
    idx = np.arange(n)
    g = integrals.eri_block(Bs, ws, idx, idx, idx, idx)
    occ, vir = list(range(n_c)), list(range(n_c, n))
    W = np.array([[(g[p, p, q, q] - g[p, q, q, p]).real if p != q else 0.0
                   for q in range(n)] for p in range(n)])
    hd = np.diag(h).real
    E0 = hd[occ].sum() + sum(W[i, j] for i, j in combinations(occ, 2))
    f = h + sum(g[:, :, j, j] - g[:, j, j, :] for j in occ)

    def wt(dl):
        return dl ** 3 / (dl ** 4 + b * b)

    e2 = 0.0
    for i in occ:
        for a in vir:
            rest = [j for j in occ if j != i]
            Hkk = hd[rest].sum() + hd[a] + sum(W[p, q] for p, q in combinations(rest + [a], 2))
            e2 += abs(f[a, i]) ** 2 * wt(E0 - Hkk)
    for i, j in combinations(occ, 2):
        for a, bb in combinations(vir, 2):
            rest = [k for k in occ if k not in (i, j)]
            Hkk = hd[rest].sum() + hd[a] + hd[bb] + sum(W[p, q] for p, q in combinations(rest + [a, bb], 2))
            e2 += abs(g[a, i, bb, j] - g[a, j, bb, i]) ** 2 * wt(E0 - Hkk)
    got, _, _ = class_e2(run.space_of(spec), h, Bs, ws, np.array([1.0 + 0j]), b=b)
    unshifted, _, _ = class_e2(run.space_of(spec), h, Bs, ws, np.array([1.0 + 0j]))
    assert abs(got - unshifted) > 1e-6 * abs(unshifted)
    assert abs(got - e2) < 1e-12 * abs(e2)


def test_one_body_only():
    """g = 0: E2 = sum_{i,a} |h_ai|^2 / (h_ii - h_aa)."""
    spec, h, Bs, ws = single_det_problem(32, 3, 6, 4, zero_g=True)
    n_c = 3
    e2 = sum(abs(h[a, i]) ** 2 / (h[i, i].real - h[a, a].real)
             for i in range(n_c) for a in range(n_c, h.shape[0]))
    got, _, _ = class_e2(run.space_of(spec), h, Bs, ws, np.array([1.0 + 0j]))
    assert abs(got - e2) < 1e-13 * abs(e2)


def mp2_ratio(lam):
    spec, h0, Bs, ws = single_det_problem(33, 4, 8, 10, lam=lam)
    n_c, n = 4, h0.shape[0]
    idx = np.arange(n)
    g = integrals.eri_block(Bs, ws, idx, idx, idx, idx)
    eps = np.sort(np.diag(h0).real)
    occ = range(n_c)
    # canonical construction: f = h + sum_j <pj||qj> = diag(eps)
    h = np.diag(eps).astype(np.complex128) - sum(g[:, :, j, j] - g[:, j, j, :] for j in occ)
    mp2 = 0.0
    for i, j in combinations(range(n_c), 2):
        for a, b in combinations(range(n_c, n), 2):
            mp2 += abs(g[a, i, b, j] - g[a, j, b, i]) ** 2 / (eps[i] + eps[j] - eps[a] - eps[b])
    got, parts, _ = class_e2(run.space_of(spec), h, Bs, ws, np.array([1.0 + 0j]))
    assert abs(parts[(1, 1)]) < 1e-20 * max(1.0, abs(got))   # Brillouin: no singles
    return got / mp2


def test_mp2_limit():
    """Canonical single determinant, integrals scaled by lam: E2/E2_MP2 -> 1
    with a deviation linear in lam."""
    d1 = mp2_ratio(1e-3) - 1.0
    d2 = mp2_ratio(5e-4) - 1.0
    assert abs(d1) < 5e-2
    assert abs(d1 / d2 - 2.0) < 0.05


# -------------------------------------------------------------- invariances

def inv_problem():
    spec = SP.small("inv", 41, 0, 3, [2, 3], 3, 6, [(10, 1.0), (5, -0.02)], max_hops=1, base=[1, 2])
    h, Bs, ws = tensors(spec)
    sp = run.space_of(spec)
    _, _, _, c = ground(sp, h, Bs, ws)
    return spec, sp, h, Bs, ws, c


def transform(h, Bs, U):
    return U.conj().T @ h @ U, [np.einsum("pi,lpq,qj->lij", U.conj(), B, U) for B in Bs]


def test_phase_gauge_invariance():
    spec, sp, h, Bs, ws, c = inv_problem()
    ref, _, _ = class_e2(sp, h, Bs, ws, c)
    rng = np.random.default_rng(1)
    phi = rng.uniform(0, 2 * np.pi, sp.n)
    act = slice(sp.n_c, sp.n_c + sp.n_a)
    phi[act] = 0.0
    U = np.diag(np.exp(1j * phi))
    h2, B2 = transform(h, Bs, U)
    got, _, _ = class_e2(sp, h2, B2, ws, c)
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_permutation_invariance():
    spec, sp, h, Bs, ws, c = inv_problem()
    ref, _, _ = class_e2(sp, h, Bs, ws, c)
    perm = np.arange(sp.n)
    rng = np.random.default_rng(2)
    perm[:sp.n_c] = rng.permutation(sp.n_c)
    v0 = sp.n_c + sp.n_a
    perm[v0:] = v0 + rng.permutation(sp.n_v)
    U = np.eye(sp.n)[:, perm]
    h2, B2 = transform(h, Bs, U)
    got, _, _ = class_e2(sp, h2, B2, ws, c)
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_diagonal_shift_invariance():
    spec, sp, h, Bs, ws, c = inv_problem()
    ref, _, _ = class_e2(sp, h, Bs, ws, c)
    got, _, _ = class_e2(sp, h + 3.7 * np.eye(sp.n), Bs, ws, c)
    assert abs(got - ref) < 1e-11 * abs(ref)


def test_cholesky_rotation_and_split_invariance():
    spec, sp, h, Bs, ws, c = inv_problem()
    ref, _, _ = class_e2(sp, h, Bs, ws, c)
    rng = np.random.default_rng(3)
    R, _ = np.linalg.qr(rng.standard_normal((Bs[0].shape[0],) * 2))
    B0 = np.einsum("kl,lpq->kpq", R, Bs[0])
    half = Bs[0].shape[0] // 2
    sets = [B0[:half], B0[half:], Bs[1]]
    got, _, _ = class_e2(sp, h, sets, [ws[0], ws[0], ws[1]], c)
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_scaling():
    """E2(lam h, lam g) = lam E2 at fixed C."""
    spec, sp, h, Bs, ws, c = inv_problem()
    ref, _, _ = class_e2(sp, h, Bs, ws, c)
    lam = 1.7
    got, _, _ = class_e2(sp, lam * h, [B * math.sqrt(lam) for B in Bs], ws, c)
    assert abs(got - lam * ref) < 1e-12 * abs(ref)


def test_degenerate_virtual_rotation_invariance():
    """Two virtuals a1, a2 made exactly degenerate (equal diagonals, no
    coupling, and Cholesky vectors paired so that <a j||a' j> is diagonal in
    (a, a') for every j): any U(2) rotation of (a1, a2) leaves E2 unchanged."""
    spec, sp, h, Bs, ws, c = inv_problem()
    n = sp.n
    a1, a2 = n - 2, n - 1
    h = h.copy()
    h[a2, a2] = h[a1, a1]
    h[a1, a2] = h[a2, a1] = 0.0
    new = []
    for B in Bs:
        nl = B.shape[0] - (B.shape[0] % 2)
        B = B[:nl].copy()
        for l in range(0, nl, 2):
            B0, B1 = B[l], B[l + 1]
            for Bx in (B0, B1):
                Bx[a1, a2] = Bx[a2, a1] = 0.0
                Bx[a2, a2] = Bx[a1, a1]
            others = [j for j in range(n) if j not in (a1, a2)]
            B0[a2, others] = -np.conj(B1[a1, others])
            B1[a2, others] = np.conj(B0[a1, others])
            for Bx in (B0, B1):
                Bx[others, a2] = np.conj(Bx[a2, others])
        new.append(B)
    Bs = new
    _, _, _, c = ground(sp, h, Bs, ws)
    ref, _, _ = class_e2(sp, h, Bs, ws, c)
    th, ph = 0.7, 1.3
    U = np.eye(n, dtype=np.complex128)
    U[np.ix_([a1, a2], [a1, a2])] = [[np.cos(th), -np.exp(-1j * ph) * np.sin(th)],
                                      [np.exp(1j * ph) * np.sin(th), np.cos(th)]]
    h2, B2 = transform(h, Bs, U)
    got, _, _ = class_e2(sp, h2, B2, ws, c)
    assert abs(got - ref) < 1e-12 * abs(ref)
    # a generic (non-degenerate) pair is not invariant: the pin has teeth
    spec, sp, h, Bs, ws, c = inv_problem()
    ref2, _, _ = class_e2(sp, h, Bs, ws, c)
    h3, B3 = transform(h, Bs, U)
    got2, _, _ = class_e2(sp, h3, B3, ws, c)
    assert abs(got2 - ref2) > 1e-8 * abs(ref2)


# ------------------------------------------------------------ literal vs class

def test_literal_equals_class_oracle_c0():
    pb = SP.config("c0")
    h, Bs, ws = tensors(pb)
    hfc, Bc = run.correlated_inputs(h, Bs, ws, pb.n_fc)
    sp = run.space_of(pb)
    g, gc, H, c = ground(sp, hfc, Bc, ws)
    e2_lit, e0, parts_l, nq = literal.e2_literal(sp, hfc, gc, c, 0, H)
    assert nq == 118116
    got, parts_c, e0c = class_e2(sp, hfc, Bc, ws, c)
    assert abs(e0 - e0c) < 1e-11
    for k in parts_l:
        assert abs(parts_l[k] - parts_c[k]) < 1e-12 * max(1.0, abs(e2_lit)), k
    assert abs(e2_lit - got) < 1e-12 * abs(e2_lit)
