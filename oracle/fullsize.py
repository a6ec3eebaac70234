"""Full-size runs of the class oracle (test infrastructure, oracle).

The class oracle (oracle.classes) needs the whole factor array B, which at
the largest workloads does not fit in host memory (69 GB), and its two-virtual
classes cost a Python-level vector operation per (core holes, string).  This
module keeps the same definitions and changes only how the numbers are
gathered:

  * streamed_inputs: one pass over every Cholesky vector, in chunks, gives
    h^FC (frozen-core fold of the notation list of Sec. 2, the same formula
    as oracle.integrals.fold_frozen_core, summed over chunks), the pair
    energies W_pq = (pp|qq) - (pq|qp) of the Epstein-Nesbet diagonal
    (eq. zeroh; oracle.integrals.pair_energies, summed over chunks) and the
    factor columns B[L][p][x] of the occupied spinors x for every correlated
    p, which is all that the integrals (px|qy), (ax|by) of the external space
    need;
  * SlabOracle: oracle.classes.ClassOracle on those columns (every per-class
    sum of the class oracle unchanged);
  * vv_class: the classes with two virtual electrons, (2,2), (1,2) and (0,2),
    with the same coupling bookkeeping as the class oracle (the reference
    determinants L connected to each external string, the sign of the
    operator string a_x a_y -> a+_b a+_a found with oracle.space.apply_ops on
    the two lowest virtuals) and the arithmetic over the virtual pairs
    (a < b) written as plain C loops (oracle/vvsum.c):
        sigma_K = sum_L G <ab||xy> C_L,   <ab||xy> = (ax|by) - (ay|bx),
        H_KK = E(core - holes + alpha) + v_a + v_b + W_ab,
        v_a = h_aa + sum_{p in core - holes + alpha} W_ap,
        E2 part = sum |sigma_K|^2 / (||C||^2 (E0 - H_KK))   (eq. pt2en).
"""
import ctypes
import math
import os
import subprocess
from itertools import combinations

import numpy as np

from . import integrals
from .classes import ClassOracle
from .space import apply_ops, bits

HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(HERE, "vvsum.c")
_LIB = os.path.join(HERE, "_vvsum.so")
_lib = None


def build_c():
    """Compile oracle/vvsum.c (gcc, OpenMP) into oracle/_vvsum.so."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"],
                   check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _vv_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_c()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        lib.oracle_vv_block.restype = ctypes.c_double
        lib.oracle_vv_block.argtypes = [ctypes.c_int64, ctypes.c_int64, p, p, p, p, p, p, p, p, p,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double]
        _lib = lib
    return _lib


def streamed_inputs(pb, chunk=32):
    """(h^FC, slabs, W) of a synthetic problem from one pass over its factors.
    slabs[t]: complex128 [rank_t][n_corr][n_o], B[t][L][p][x] over correlated
    p and occupied correlated x (core then active)."""
    import synth.problems as SP
    n_fc, n = pb.n_fc, pb.n
    n_o = pb.n_c + pb.n_a
    keep = slice(n_fc, n)
    h = SP.one_body(pb).numpy()
    hfc = h[keep, keep].astype(np.complex128).copy()
    n_corr = n - n_fc
    W = np.zeros((n_corr, n_corr))
    zero = np.zeros_like(h)
    slabs = []
    for t, (r, w) in enumerate(pb.sets):
        slab = np.empty((r, n_corr, n_o), dtype=np.complex128)
        for l0 in range(0, r, chunk):
            l1 = min(r, l0 + chunk)
            B = SP.factor_slice(pb, t, l0, l1).numpy()
            if n_fc > 0:
                hfc += integrals.fold_frozen_core(zero, [B], [w], n_fc)[0]
            Bc = B[:, keep, keep]
            W += integrals.pair_energies([Bc], [w])
            slab[l0:l1] = Bc[:, :, :n_o]
            del B, Bc
        slabs.append(slab)
    return hfc, slabs, W


class SlabOracle(ClassOracle):
    """The class oracle on the occupied factor columns only, with the pair
    energies given (streamed_inputs)."""

    def __init__(self, space, h, slabs, ws, W):
        self.sp = space
        self.h = np.asarray(h)
        self.Bs = [np.asarray(B) for B in slabs]
        self.ws = list(ws)
        n_c, n_a, n = space.n_c, space.n_a, space.n
        assert self.Bs[0].shape[1:] == (n, n_c + n_a)
        self.O = np.arange(0, n_c + n_a)
        self.V = np.arange(n_c + n_a, n)
        self.hd = np.real(np.diag(self.h)).astype(np.float64)
        self.W = np.asarray(W)
        self._goooo = None
        self._gvooo = None
        self._gvv = {}
        self.P = space.p_strings()
        self.pidx = {a: i for i, a in enumerate(self.P)}
        self.core = space.core_mask

    def g_vv(self, x, y):
        """(a x | b y) over all virtual a, b (not cached: at full size the
        matrices of every occupied pair would not fit in memory)."""
        out = np.zeros((len(self.V), len(self.V)), dtype=np.complex128)
        for B, w in zip(self.Bs, self.ws):
            out += w * (B[:, self.V, x].T @ B[:, self.V, y])
        return out


def _couplings(co, cl, al, hole, acts):
    """(x, y, beta) of the double excitations a_x a_y -> a+_b a+_a that lead
    from L = core + beta to an external determinant of class cl with active
    string al and core holes hole."""
    h_ = cl[0]
    if h_ == 2:
        return [(hole[0], hole[1], al)]
    if h_ == 1:
        return [(hole[0], t, al | (1 << t)) for t in acts if not al >> t & 1]
    free = [t for t in acts if not al >> t & 1]
    return [(t, w, al | (1 << t) | (1 << w)) for t, w in combinations(free, 2)]


def vv_class(co, cl, C, E0, q_mode=0, core_sets=None, va=None, vb=None, strings=None, b=0.0):
    """E2 part of class cl in {(2,2), (1,2), (0,2)}; arguments as in
    ClassOracle.e2 (restrictions to core-hole tuples, virtual position ranges
    of the lower and the upper virtual spinor, and active strings)."""
    h_, v_ = cl
    assert v_ == 2
    sp = co.sp
    C = np.asarray(C, dtype=np.complex128)
    norm = float(np.vdot(C, C).real)
    V, O = co.V, co.O
    nv = len(V)
    amask = np.zeros(nv, np.uint8)
    bmask = np.zeros(nv, np.uint8)
    lo, hi = va if va is not None else (0, nv)
    amask[lo:hi] = 1
    lo, hi = vb if vb is not None else (0, nv)
    bmask[lo:hi] = 1
    if nv < 2:
        return 0.0
    a0, b0 = int(V[0]), int(V[1])
    if h_ == 2:
        strs = list(co.P)
    else:
        strs = sp.class_strings(h_, 2, q_mode)
    if strings is not None:
        keep = set(int(x) for x in strings)
        strs = [a for a in strs if a in keep]
    acts = bits(sp.act_mask)
    hd_o, hd_v = co.hd[O], co.hd[V]
    WOO = np.ascontiguousarray(co.W[np.ix_(O, O)])
    WOV = np.ascontiguousarray(co.W[np.ix_(O, V)])
    Wvv = np.ascontiguousarray(co.W[np.ix_(V, V)])
    lib = _vv_lib()
    cs = None if core_sets is None else set(tuple(s) for s in core_sets)
    terms = []
    for hole in combinations(range(sp.n_c), h_):
        if cs is not None and tuple(hole) not in cs:
            continue
        core_k = co.core
        for c in hole:
            core_k &= ~(1 << c)
        keys, ptr, kidx, cval, d0s = {}, [0], [], [], []
        for al in strs:
            D0 = core_k | al
            K = D0 | (1 << a0) | (1 << b0)
            n0 = len(kidx)
            for x, y, beta in _couplings(co, cl, al, hole, acts):
                j = co.pidx.get(beta)
                if j is None:
                    continue
                L = co.core | beta
                G, D = apply_ops(L, [("a", x), ("a", y), ("c", b0), ("c", a0)])
                assert D == K, "operator string does not connect L to K"
                kidx.append(keys.setdefault((x, y), len(keys)))
                cval.append(G * C[j])
            if len(kidx) > n0:
                ptr.append(len(kidx))
                d0s.append(D0)
        if not d0s:
            continue
        X = np.empty((len(keys), nv, nv), dtype=np.complex128)
        for (x, y), k in keys.items():
            X[k] = co.g_vv(x, y) - co.g_vv(y, x)
        occ = np.array([[(D >> int(p)) & 1 for p in O] for D in d0s], dtype=np.float64)
        e0 = occ @ hd_o + 0.5 * np.einsum("si,ij,sj->s", occ, WOO, occ)
        vva = np.ascontiguousarray(hd_v[None, :] + occ @ WOV)
        ptr_a = np.asarray(ptr, dtype=np.int64)
        kidx_a = np.asarray(kidx, dtype=np.int64)
        cval_a = np.asarray(cval, dtype=np.complex128)
        e0 = np.ascontiguousarray(e0)
        r = lib.oracle_vv_block(len(d0s), nv, ptr_a.ctypes.data, kidx_a.ctypes.data, cval_a.ctypes.data,
                                X.ctypes.data, e0.ctypes.data, vva.ctypes.data, Wvv.ctypes.data,
                                amask.ctypes.data, bmask.ctypes.data, float(E0), norm, float(b))
        terms.append(r)
    return math.fsum(terms)


def sub_oracle(co, vpos):
    """SlabOracle on the occupied spinors and the virtual spinors at the
    given positions (0-based within the virtual block).  Every term of an
    external determinant whose virtual spinors are all among them is the same
    as in the whole space, so restricted sums can be taken on it."""
    O, V = co.O, co.V
    idx = np.concatenate([O, V[np.asarray(vpos, dtype=np.int64)]])
    sp = co.sp
    from .space import ActiveSpace
    sub = ActiveSpace(sp.n_c, sp.sub_sizes, sp.n_elec, sp.base, sp.max_hops, len(vpos))
    h = co.h[np.ix_(idx, idx)]
    slabs = [np.ascontiguousarray(B[:, idx, :]) for B in co.Bs]
    return SlabOracle(sub, h, slabs, co.ws, co.W[np.ix_(idx, idx)])
