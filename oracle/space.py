"""Determinant spaces of STP-DAS MRPT2 (test infrastructure, oracle).

Orbital order over the correlated spinors: core [0, n_c), active
[n_c, n_c + n_a) split into DAS subspaces in order, virtual [n_c + n_a, n).
A determinant is a Python int whose bit p is set when spinor p is occupied;
its phase convention is |D> = a+_{p1} a+_{p2} ... a+_{pN} |0> with
p1 < p2 < ... < pN.

Sec. 2.4 (STP-DAS): a configuration category is the electron count in each
DAS subspace; every subspace is a local complete active space.  The primary
space P holds the core-full, virtual-empty determinants whose active
occupation lies in an allowed category.  A category m is allowed when
sum_k m_k = n and its hop count sum_k max(0, m_k - base_k) does not exceed the
hop limit (the paper's calculations use complete active spaces: one
subspace, no limit).

Sec. 2.3: the external space Q holds every single and double excitation of a
P determinant that is not in P.
"""
from itertools import combinations, product


class ActiveSpace:
    def __init__(self, n_c, sub_sizes, n_elec, base, max_hops, n_v):
        self.n_c = n_c
        self.sub_sizes = list(sub_sizes)
        self.n_a = sum(self.sub_sizes)
        self.n_elec = n_elec
        self.base = list(base)
        self.max_hops = max_hops
        self.n_v = n_v
        self.n = n_c + self.n_a + n_v
        self.offsets = []
        o = n_c
        for s in self.sub_sizes:
            self.offsets.append(o)
            o += s
        self.core_mask = (1 << n_c) - 1
        self.act_mask = ((1 << self.n_a) - 1) << n_c
        self.virt_mask = ((1 << n_v) - 1) << (n_c + self.n_a)

    # -- categories --------------------------------------------------------
    def category(self, det):
        return tuple(bin((det >> o) & ((1 << s) - 1)).count("1")
                     for o, s in zip(self.offsets, self.sub_sizes))

    def hops(self, m):
        return sum(max(0, mk - bk) for mk, bk in zip(m, self.base))

    def categories(self, n_el):
        ranges = [range(0, s + 1) for s in self.sub_sizes]
        return [m for m in product(*ranges) if sum(m) == n_el]

    def p_categories(self):
        return [m for m in self.categories(self.n_elec) if self.hops(m) <= self.max_hops]

    def strings_of_category(self, m):
        """Active-orbital bit masks (global bit positions) of category m."""
        per_sub = []
        for o, s, mk in zip(self.offsets, self.sub_sizes, m):
            per_sub.append([sum(1 << (o + i) for i in c) for c in combinations(range(s), mk)])
        out = []
        for parts in product(*per_sub):
            out.append(sum(parts))
        return out

    def p_strings(self):
        """Active parts of the P determinants, sorted by their bit pattern."""
        out = []
        for m in self.p_categories():
            out.extend(self.strings_of_category(m))
        return sorted(out)

    def p_dets(self):
        return [self.core_mask | a for a in self.p_strings()]

    # -- external space by its definition ---------------------------------
    def q_dets_literal(self, q_mode=0):
        """Every single and double excitation of every P determinant, minus P.
        q_mode 1 keeps only determinants with a core hole or a virtual
        electron."""
        P = set(self.p_dets())
        Q = set()
        n = self.n
        for L in P:
            occ = [p for p in range(n) if L >> p & 1]
            vir = [p for p in range(n) if not L >> p & 1]
            for q in occ:
                for p in vir:
                    Q.add(L ^ (1 << q) ^ (1 << p))
            for q, s in combinations(occ, 2):
                for p, r in combinations(vir, 2):
                    Q.add(L ^ (1 << q) ^ (1 << s) ^ (1 << p) ^ (1 << r))
        Q -= P
        if q_mode == 1:
            Q = {K for K in Q if (K & self.core_mask) != self.core_mask or (K & self.virt_mask)}
        return sorted(Q)

    # -- external space by excitation class --------------------------------
    def level(self, m, v):
        """Excitations needed to reach an occupation with v virtual electrons
        and active category m from the nearest P determinant: each virtual
        electron and each surplus electron in a subspace needs one creation
        (a subspace is a local complete space, so the rest can be matched)."""
        return v + min(sum(max(0, a - b) for a, b in zip(m, mp)) for mp in self.p_categories())

    def class_strings(self, h, v, q_mode=0):
        """Active strings of the external determinants with h core holes and
        v virtual electrons."""
        n_el = self.n_elec + h - v
        if n_el < 0 or n_el > self.n_a:
            return []
        pcats = set(self.p_categories())
        out = []
        for m in self.categories(n_el):
            if self.level(m, v) > 2:
                continue
            if h == 0 and v == 0 and (m in pcats or q_mode == 1):
                continue
            out.extend(self.strings_of_category(m))
        return sorted(out)


def bits(x):
    out = []
    p = 0
    while x:
        if x & 1:
            out.append(p)
        x >>= 1
        p += 1
    return out


def apply_ops(det, ops):
    """Apply operators right to left as listed: ops = [('a', q), ('c', p)...]
    with the first entry acting first.  Returns (sign, det) or (0, None) when
    the result vanishes.  a_p and a+_p each take the sign (-1)^(number of
    occupied spinors below p) in the ascending-creation-string convention."""
    sign = 1
    for kind, p in ops:
        below = bin(det & ((1 << p) - 1)).count("1")
        if kind == "a":
            if not det >> p & 1:
                return 0, None
            det ^= 1 << p
        else:
            if det >> p & 1:
                return 0, None
            det |= 1 << p
        if below & 1:
            sign = -sign
    return sign, det
