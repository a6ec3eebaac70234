"""MRPT2 energy organised by excitation class (test infrastructure, oracle).

Same quantity as oracle.literal, for spaces too large to enumerate one
determinant at a time.  External determinants are grouped as in the STP-DAS
organisation (Sec. 2.4): by the number h of core holes, the number v of
virtual electrons and the active string.  A determinant with h core holes, v
virtual electrons and active category m is in Q when its excitation level
v + min_{m' in P} sum_k max(0, m_k - m'_k) is at most 2 and it is not in P
(oracle.space.ActiveSpace.class_strings).

For each class the oracle loops in Python over core holes, active strings and
the reference determinants connected to them, and works on whole arrays over
the virtual spinors (which carry no sign: all virtuals lie above every
occupied spinor of a P determinant, so creating them gives a sign that
depends only on electron counts).  Matrix elements are the Slater-Condon
rules of oracle.literal:
    single  K = a+_p a_q L     : G [ h_pq + sum_{j in L} ((pq|jj) - (pj|jq)) ]
    double  K = a+_p a+_r a_s a_q L : G [ (pq|rs) - (ps|rq) ]
with G the sign of the operator string on L, found with oracle.space.apply_ops
using the lowest virtual spinors as representatives.  Denominators are
E0 - H_KK with H_KK = sum_{p in K} h_pp + sum_{p<q in K} W_pq (eq. zeroh),
W_pq = (pp|qq) - (pq|qp); with the level shift b of Sec. 2.6 each inverse
denominator is the real part of 1/(Delta + i b/Delta) (oracle.literal).

Optional restrictions (used to check sampled parts of a large sum): a set of
core-hole tuples, and index ranges for the first and second virtual spinor.
"""
import math
from itertools import combinations

import numpy as np

from . import integrals
from .literal import matrix_element, reference_hamiltonian, reference_energy
from .space import apply_ops, bits

CLASSES = [(2, 2), (1, 2), (0, 2), (2, 1), (1, 1), (0, 1), (2, 0), (1, 0), (0, 0)]


class ClassOracle:
    def __init__(self, space, h, Bs, ws):
        """space: oracle.space.ActiveSpace over the correlated spinors;
        h: h^FC (complex, n x n); Bs: factor sets restricted to the correlated
        spinors; ws: their weights."""
        self.sp = space
        self.h = np.asarray(h)
        self.Bs = [np.asarray(B) for B in Bs]
        self.ws = list(ws)
        n_c, n_a, n = space.n_c, space.n_a, space.n
        self.O = np.arange(0, n_c + n_a)
        self.V = np.arange(n_c + n_a, n)
        self.hd = np.real(np.diag(self.h)).astype(np.float64)
        self.W = integrals.pair_energies(self.Bs, self.ws)
        self._goooo = None
        self._gvooo = None
        self._gvv = {}
        self.P = space.p_strings()
        self.pidx = {a: i for i, a in enumerate(self.P)}
        self.core = space.core_mask

    # -- integrals ----------------------------------------------------------
    @property
    def gOOOO(self):
        """(pq|rs) over core and active spinors (computed on first use)."""
        if self._goooo is None:
            self._goooo = integrals.eri_block(self.Bs, self.ws, self.O, self.O, self.O, self.O)
        return self._goooo

    @property
    def gVOOO(self):
        """(a x|y z), a virtual, x, y, z core or active (computed on first use)."""
        if self._gvooo is None:
            self._gvooo = integrals.eri_block(self.Bs, self.ws, self.V, self.O, self.O, self.O)
        return self._gvooo

    def g_occ(self, p, q, r, s):
        return self.gOOOO[p, q, r, s]

    def g_vv(self, x, y):
        """(a x | b y) over all virtual a, b."""
        key = (x, y)
        if key not in self._gvv:
            out = np.zeros((len(self.V), len(self.V)), dtype=np.complex128)
            for B, w in zip(self.Bs, self.ws):
                out += w * (B[:, self.V, x].T @ B[:, self.V, y])
            self._gvv[key] = out
        return self._gvv[key]

    def g_vo(self, x, y, z):
        """(a x | y z) over all virtual a."""
        return self.gVOOO[:, x, y, z]

    # -- reference -----------------------------------------------------------
    def reference(self, C):
        H = reference_hamiltonian(self.sp, self.h, self.g_occ)
        return H, reference_energy(H, C)

    def energy_of(self, det):
        occ = np.array(bits(det), dtype=np.int64)
        if len(occ) == 0:
            return 0.0
        return float(self.hd[occ].sum() + 0.5 * self.W[np.ix_(occ, occ)].sum())

    # -- main ------------------------------------------------------------------
    def e2(self, C, q_mode=0, E0=None, core_sets=None, va=None, vb=None, classes=None, strings=None, b=0.0):
        """Per-class E2 parts (dict) and E0.  b: level-shift constant (Sec.
        2.6; 0 gives eq. pt2en exactly).  core_sets: allowed core-hole
        tuples (sorted, correlated core indices); va / vb: (lo, hi) ranges of
        virtual positions (0-based within the virtual block) for the lowest
        and the second virtual spinor of K; strings: allowed active strings
        of K (bit masks in this space's positions)."""
        self.strings_filter = None if strings is None else set(int(x) for x in strings)
        C = np.asarray(C, dtype=np.complex128)
        if E0 is None:
            _, E0 = self.reference(C)
        self.E0 = E0
        self.b = float(b)
        self.norm = float(np.vdot(C, C).real)
        self.C = C
        self.core_sets = None if core_sets is None else set(tuple(s) for s in core_sets)
        nv = len(self.V)
        self.mask_a = np.zeros(nv, bool)
        self.mask_b = np.zeros(nv, bool)
        lo, hi = va if va is not None else (0, nv)
        self.mask_a[lo:hi] = True
        lo, hi = vb if vb is not None else (0, nv)
        self.mask_b[lo:hi] = True
        iu = np.triu(np.ones((nv, nv), bool), 1)
        self.pair_mask = iu & self.mask_a[:, None] & self.mask_b[None, :]
        out = {}
        for cl in (classes or CLASSES):
            if cl == (0, 0) and q_mode == 1:
                out[cl] = 0.0
                continue
            out[cl] = getattr(self, "_c%d%d" % cl)(q_mode)
        return out, E0

    def _holes(self, h):
        for Hc in combinations(range(self.sp.n_c), h):
            if self.core_sets is None or tuple(Hc) in self.core_sets:
                yield Hc

    def _cls_strings(self, h, v, q_mode):
        out = self.sp.class_strings(h, v, q_mode)
        if self.strings_filter is not None:
            out = [a for a in out if a in self.strings_filter]
        return out

    def _rep(self, v):
        return [int(x) for x in self.V[:v]]

    def _weight(self, d):
        """1/d, or Re 1/(d + i b/d) under the level shift (arrays or scalars)."""
        if self.b == 0.0:
            return 1.0 / d
        return np.real(1.0 / (d + 1j * (self.b / d)))

    def _sum_vv(self, sig, D0, terms):
        """Add sum over a<b of |sig|^2 / (N (E0 - H_KK)) for K = D0 + {a, b}."""
        e0 = self.energy_of(D0)
        occ = np.array(bits(D0), dtype=np.int64)
        va = self.hd[self.V] + self.W[np.ix_(self.V, occ)].sum(axis=1)
        Hkk = e0 + va[:, None] + va[None, :] + self.W[np.ix_(self.V, self.V)]
        t = np.abs(sig) ** 2 * self._weight(self.E0 - Hkk) / self.norm
        terms.append(math.fsum(t[self.pair_mask].tolist()))

    def _sum_v(self, sig, D0, terms):
        e0 = self.energy_of(D0)
        occ = np.array(bits(D0), dtype=np.int64)
        va = self.hd[self.V] + self.W[np.ix_(self.V, occ)].sum(axis=1)
        t = np.abs(sig) ** 2 * self._weight(self.E0 - (e0 + va)) / self.norm
        terms.append(math.fsum(t[self.mask_a].tolist()))

    def _sign(self, L, ops, K):
        s, D = apply_ops(L, ops)
        assert D == K, "operator string does not connect L to K"
        return s

    # (2,2): K = core - {c,c'} + alpha + {a,b}; only L = core + alpha
    def _c22(self, q_mode):
        terms = []
        a0, b0 = self._rep(2)
        for c, c2 in self._holes(2):
            X = self.g_vv(c, c2) - self.g_vv(c2, c)            # (ac|bc') - (ac'|bc)
            for i, al in enumerate(self.P):
                if self.strings_filter is not None and al not in self.strings_filter:
                    continue
                L = self.core | al
                D0 = L & ~(1 << c) & ~(1 << c2)
                K = D0 | (1 << a0) | (1 << b0)
                G = self._sign(L, [("a", c), ("a", c2), ("c", b0), ("c", a0)], K)
                self._sum_vv(G * X * self.C[i], D0, terms)
        return math.fsum(terms)

    # (1,2): K = core - {c} + alpha' + {a,b}; L = core + alpha' + {t}
    def _c12(self, q_mode):
        terms = []
        a0, b0 = self._rep(2)
        acts = bits(self.sp.act_mask)
        for (c,) in self._holes(1):
            for al in self._cls_strings(1, 2, q_mode):
                D0 = (self.core & ~(1 << c)) | al
                K = D0 | (1 << a0) | (1 << b0)
                sig = 0.0
                for t in acts:
                    if al >> t & 1:
                        continue
                    j = self.pidx.get(al | (1 << t))
                    if j is None:
                        continue
                    L = self.core | al | (1 << t)
                    G = self._sign(L, [("a", c), ("a", t), ("c", b0), ("c", a0)], K)
                    sig = sig + G * (self.g_vv(c, t) - self.g_vv(t, c)) * self.C[j]
                if not isinstance(sig, float):
                    self._sum_vv(sig, D0, terms)
        return math.fsum(terms)

    # (0,2): K = core + alpha'' + {a,b}; L = core + alpha'' + {t,w}
    def _c02(self, q_mode):
        terms = []
        a0, b0 = self._rep(2)
        acts = bits(self.sp.act_mask)
        for al in self._cls_strings(0, 2, q_mode):
            D0 = self.core | al
            K = D0 | (1 << a0) | (1 << b0)
            sig = 0.0
            free = [t for t in acts if not al >> t & 1]
            for t, w in combinations(free, 2):
                j = self.pidx.get(al | (1 << t) | (1 << w))
                if j is None:
                    continue
                L = self.core | al | (1 << t) | (1 << w)
                G = self._sign(L, [("a", t), ("a", w), ("c", b0), ("c", a0)], K)
                sig = sig + G * (self.g_vv(t, w) - self.g_vv(w, t)) * self.C[j]
            if not isinstance(sig, float):
                self._sum_vv(sig, D0, terms)
        return math.fsum(terms)

    # (2,1): K = core - {c,c'} + alpha+ + {a}; L = core + alpha+ - {u}
    def _c21(self, q_mode):
        terms = []
        (a0,) = self._rep(1)
        for c, c2 in self._holes(2):
            for al in self._cls_strings(2, 1, q_mode):
                D0 = (self.core & ~(1 << c) & ~(1 << c2)) | al
                K = D0 | (1 << a0)
                sig = 0.0
                for u in bits(al):
                    j = self.pidx.get(al & ~(1 << u))
                    if j is None:
                        continue
                    L = self.core | (al & ~(1 << u))
                    G = self._sign(L, [("a", c), ("a", c2), ("c", u), ("c", a0)], K)
                    sig = sig + G * (self.g_vo(c, u, c2) - self.g_vo(c2, u, c)) * self.C[j]
                if not isinstance(sig, float):
                    self._sum_v(sig, D0, terms)
        return math.fsum(terms)

    # (1,1): K = core - {c} + alpha + {a}; L = core + alpha (single c->a) or
    # L = core + alpha - {u} + {t} (double c,t -> a,u)
    def _c11(self, q_mode):
        terms = []
        (a0,) = self._rep(1)
        acts = bits(self.sp.act_mask)
        for (c,) in self._holes(1):
            for al in self._cls_strings(1, 1, q_mode):
                D0 = (self.core & ~(1 << c)) | al
                K = D0 | (1 << a0)
                sig = 0.0
                j = self.pidx.get(al)
                if j is not None:
                    L = self.core | al
                    G = self._sign(L, [("a", c), ("c", a0)], K)
                    f = self.h[self.V, c].copy()
                    for q in bits(L):
                        f = f + self.g_vo(c, q, q) - self.g_vo(q, q, c)
                    sig = sig + G * f * self.C[j]
                for u in bits(al):
                    for t in acts:
                        if al >> t & 1:
                            continue
                        j = self.pidx.get((al & ~(1 << u)) | (1 << t))
                        if j is None:
                            continue
                        L = self.core | (al & ~(1 << u)) | (1 << t)
                        G = self._sign(L, [("a", c), ("a", t), ("c", u), ("c", a0)], K)
                        sig = sig + G * (self.g_vo(c, u, t) - self.g_vo(t, u, c)) * self.C[j]
                if not isinstance(sig, float):
                    self._sum_v(sig, D0, terms)
        return math.fsum(terms)

    # (0,1): K = core + alpha' + {a}; L = core + alpha' + {t} (single t->a)
    # or L = core + alpha' - {u} + {t,w} (double t,w -> a,u)
    def _c01(self, q_mode):
        terms = []
        (a0,) = self._rep(1)
        acts = bits(self.sp.act_mask)
        for al in self._cls_strings(0, 1, q_mode):
            D0 = self.core | al
            K = D0 | (1 << a0)
            sig = 0.0
            free = [t for t in acts if not al >> t & 1]
            for t in free:
                j = self.pidx.get(al | (1 << t))
                if j is None:
                    continue
                L = self.core | al | (1 << t)
                G = self._sign(L, [("a", t), ("c", a0)], K)
                f = self.h[self.V, t].copy()
                for q in bits(L):
                    f = f + self.g_vo(t, q, q) - self.g_vo(q, q, t)
                sig = sig + G * f * self.C[j]
            for u in bits(al):
                for t, w in combinations(free, 2):
                    j = self.pidx.get((al & ~(1 << u)) | (1 << t) | (1 << w))
                    if j is None:
                        continue
                    L = self.core | (al & ~(1 << u)) | (1 << t) | (1 << w)
                    G = self._sign(L, [("a", t), ("a", w), ("c", u), ("c", a0)], K)
                    sig = sig + G * (self.g_vo(t, u, w) - self.g_vo(w, u, t)) * self.C[j]
            if not isinstance(sig, float):
                self._sum_v(sig, D0, terms)
        return math.fsum(terms)

    # classes without virtual electrons: literal Slater-Condon on whole
    # determinants, connected reference determinants found by removing r
    # active electrons and adding r - h active electrons (r <= 2)
    def _novirt(self, h, q_mode):
        terms = []
        acts = bits(self.sp.act_mask)
        for Hc in self._holes(h):
            core_k = self.core
            for c in Hc:
                core_k &= ~(1 << c)
            for al in self._cls_strings(h, 0, q_mode):
                K = core_k | al
                occ_a = bits(al)
                free = [t for t in acts if not al >> t & 1]
                sig = 0.0
                for r in range(h, 3):
                    for R in combinations(occ_a, r):
                        for A in combinations(free, r - h):
                            beta = al
                            for u in R:
                                beta &= ~(1 << u)
                            for t in A:
                                beta |= 1 << t
                            j = self.pidx.get(beta)
                            if j is None:
                                continue
                            sig += matrix_element(K, self.core | beta, self.h, self.g_occ) * self.C[j]
                d = self.E0 - self.energy_of(K)
                terms.append(abs(sig) ** 2 * float(self._weight(d)) / self.norm)
        return math.fsum(terms)

    def _c20(self, q_mode):
        return self._novirt(2, q_mode)

    def _c10(self, q_mode):
        return self._novirt(1, q_mode)

    def _c00(self, q_mode):
        return self._novirt(0, q_mode)
