"""Determinant-by-determinant MRPT2 energy (test infrastructure, oracle).

Every quantity is taken straight from its definition:
  * <K|H|L> by the Slater-Condon rules for spin-orbital (spinor)
    determinants, with the sign found by applying the excitation operators to
    the ascending creation string of L;
  * H_PP, E0 = Re(C^H H_PP C) / C^H C  (eq. pt2: E0 is the reference energy
    of the normalised reference Psi0 = C / ||C||);
  * sigma_K = sum_{L in P} <K|H|L> C_L  (eq. sumsigma, for K in Q);
  * H_KK = sum_{p in K} h_pp + sum_{p<q in K} [(pp|qq) - (pq|qp)]  (eq. zeroh);
  * E2 = sum_{K in Q} |sigma_K|^2 / (||C||^2 (E0 - H_KK))  (eq. pt2en);
  * with the imaginary level shift of Sec. 2.6 (b != 0) the inverse
    denominator 1/(E0 - H_KK) becomes the real part of 1/(E0 - H_KK + i eps)
    with eps = b/(E0 - H_KK) (the paper does not say to take the real part:
    E2 is kept real, as for the unshifted sum).
Sums are compensated (math.fsum).

Integrals are passed as a callable g(p, q, r, s) = (pq|rs) and a matrix h.
"""
import math
from itertools import combinations

import numpy as np

from .space import apply_ops, bits


def matrix_element(K, L, h, g):
    """<K|H|L> for determinants K, L (bit masks) with H = sum h_pq a+_p a_q
    + 1/2 sum (pq|rs) a+_p a+_r a_s a_q."""
    cre = bits(K & ~L)
    ann = bits(L & ~K)
    if len(cre) != len(ann) or len(cre) > 2:
        return 0.0
    if len(cre) == 0:
        occ = bits(K)
        e = sum(h[p, p] for p in occ)
        for i, p in enumerate(occ):
            for q in occ[i + 1:]:
                e += g(p, p, q, q) - g(p, q, q, p)
        return e
    if len(cre) == 1:
        p, q = cre[0], ann[0]
        sgn, D = apply_ops(L, [("a", q), ("c", p)])
        assert D == K
        v = h[p, q]
        for j in bits(L):
            v += g(p, q, j, j) - g(p, j, j, q)
        return sgn * v
    p, r = cre
    q, s = ann
    sgn, D = apply_ops(L, [("a", q), ("a", s), ("c", r), ("c", p)])
    assert D == K
    return sgn * (g(p, q, r, s) - g(p, s, r, q))


def diagonal(K, hd, W):
    """H_KK from the diagonal one-body energies hd and pair energies W."""
    occ = np.array(bits(K), dtype=np.int64)
    return float(hd[occ].sum() + 0.5 * W[np.ix_(occ, occ)].sum())


def active_connections(space, L):
    """All determinants reached from L by single and double excitations that
    stay inside the active orbitals (used for H_PP)."""
    occ = [p for p in bits(L & space.act_mask)]
    vir = [p for p in bits(space.act_mask & ~L)]
    out = []
    for q in occ:
        for p in vir:
            out.append(L ^ (1 << q) ^ (1 << p))
    for q, s in combinations(occ, 2):
        for p, r in combinations(vir, 2):
            out.append(L ^ (1 << q) ^ (1 << s) ^ (1 << p) ^ (1 << r))
    return out


def reference_hamiltonian(space, h, g):
    """Dense H_PP over space.p_dets() order."""
    P = space.p_dets()
    idx = {d: i for i, d in enumerate(P)}
    H = np.zeros((len(P), len(P)), dtype=np.complex128)
    for j, L in enumerate(P):
        H[j, j] = matrix_element(L, L, h, g)
        for K in active_connections(space, L):
            i = idx.get(K)
            if i is not None:
                H[i, j] = matrix_element(K, L, h, g)
    return H


def reference_energy(H, C):
    """E0 = Re(C^H H C) / (C^H C)."""
    return float((np.vdot(C, H @ C)).real / np.vdot(C, C).real)


def lowest_state(H):
    """Lowest eigenvector of H_PP, normalised, with its largest component
    real and positive."""
    w, v = np.linalg.eigh(H)
    c = v[:, 0]
    k = int(np.argmax(np.abs(c)))
    c = c * (abs(c[k]) / c[k])
    return float(w[0]), c


def en_weight(d, b=0.0):
    """Inverse Epstein-Nesbet denominator 1/d, or with the imaginary level
    shift of Sec. 2.6 the real part of 1/(d + i b/d), as complex arithmetic."""
    if b == 0.0:
        return 1.0 / d
    return (1.0 / complex(d, b / d)).real


def external_class(space, K):
    """(core holes, virtual electrons) of determinant K."""
    h = space.n_c - bin(K & space.core_mask).count("1")
    v = bin(K & space.virt_mask).count("1")
    return h, v


def e2_literal(space, h, g, C, q_mode=0, H_PP=None, b=0.0):
    """Returns (E2, E0, {class: E2 part}, N_Q) by explicit enumeration; b is
    the level-shift constant (0: eq. pt2en exactly)."""
    P = space.p_dets()
    if H_PP is None:
        H_PP = reference_hamiltonian(space, h, g)
    E0 = reference_energy(H_PP, C)
    norm = float(np.vdot(C, C).real)
    Pset = set(P)
    sigma = {}
    n = space.n
    for j, L in enumerate(P):
        occ = bits(L)
        vir = [p for p in range(n) if not L >> p & 1]
        targets = []
        for q in occ:
            for p in vir:
                targets.append(L ^ (1 << q) ^ (1 << p))
        for q, s in combinations(occ, 2):
            for p, r in combinations(vir, 2):
                targets.append(L ^ (1 << q) ^ (1 << s) ^ (1 << p) ^ (1 << r))
        for K in targets:
            if K in Pset:
                continue
            if q_mode == 1 and (K & space.core_mask) == space.core_mask and not (K & space.virt_mask):
                continue
            sigma[K] = sigma.get(K, 0.0) + matrix_element(K, L, h, g) * C[j]
    hd = np.real(np.diag(h)).astype(np.float64)
    W = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            if p != q:
                W[p, q] = (g(p, p, q, q) - g(p, q, q, p)).real
    terms = {}
    for K, s in sigma.items():
        d = E0 - diagonal(K, hd, W)
        terms.setdefault(external_class(space, K), []).append(abs(s) ** 2 * en_weight(d, b) / norm)
    parts = {k: math.fsum(v) for k, v in terms.items()}
    return math.fsum(parts.values()), E0, parts, len(sigma)


def denominator_stats(space, h, g, C, thresh, q_mode=0, H_PP=None):
    """Per excitation class (core holes, virtual electrons): the smallest
    |E0 - H_KK| over the external determinants K of Q and the number of them
    with |E0 - H_KK| < thresh (Sec. 2.6: intruder states are the K whose
    denominator of eq. pt2en comes close to zero).  Q is every determinant one
    or two replacements away from a reference determinant that is not itself
    one (Sec. 2.3; q_mode 1 keeps those with a core hole or a virtual
    electron).  Returns {class: (min |Delta|, count)}."""
    P = space.p_dets()
    if H_PP is None:
        H_PP = reference_hamiltonian(space, h, g)
    E0 = reference_energy(H_PP, C)
    Pset = set(P)
    n = space.n
    Q = set()
    for L in P:
        occ = bits(L)
        vir = [p for p in range(n) if not L >> p & 1]
        for q in occ:
            for p in vir:
                Q.add(L ^ (1 << q) ^ (1 << p))
        for q, s in combinations(occ, 2):
            for p, r in combinations(vir, 2):
                Q.add(L ^ (1 << q) ^ (1 << s) ^ (1 << p) ^ (1 << r))
    Q -= Pset
    if q_mode == 1:
        Q = {K for K in Q if (K & space.core_mask) != space.core_mask or (K & space.virt_mask)}
    hd = np.real(np.diag(h)).astype(np.float64)
    W = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            if p != q:
                W[p, q] = (g(p, p, q, q) - g(p, q, q, p)).real
    out = {}
    for K in Q:
        a = abs(E0 - diagonal(K, hd, W))
        cls = external_class(space, K)
        m, c = out.get(cls, (math.inf, 0))
        out[cls] = (min(m, a), c + (1 if a < thresh else 0))
    return out
