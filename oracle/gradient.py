"""Gradient of the MRPT2 energy by reverse-mode differentiation of its
definition (test infrastructure, oracle; CPU, torch complex128 autograd).

The energy is written out in plain tensor operations of the inputs, so that
torch's autograd differentiates every step:
  * (pq|rs) = sum_t w_t sum_L B[t][L,p,q] B[t][L,r,s], frozen core folded into
    h as in oracle.integrals (Sec. 2, notation list);
  * <K|H|L> by the Slater-Condon rules (the same rules as oracle.literal):
      single K = a+_p a_q L      : G [ h_pq + sum_{j in L} ((pq|jj) - (pj|jq)) ]
      double K = a+_p a+_r a_s a_q L : G [ (pq|rs) - (ps|rq) ]
    with the sign G from oracle.space.apply_ops;
  * H_PP, E0 = Re(C^H H_PP C) / C^H C (eq. pt2 with Psi0 = C / ||C||);
  * sigma_K = sum_L <K|H|L> C_L for K in Q (Sec. 2.3);
  * H_KK = sum_{p in K} Re h_pp + sum_{p<q in K} Re[(pp|qq) - (pq|qp)] (eq. zeroh);
  * E2 = sum_K |sigma_K|^2 / (||C||^2 (E0 - H_KK)) (eq. pt2en), or with the
    level shift b of Sec. 2.6 the inverse denominator replaced by the real
    part of 1/(E0 - H_KK + i b/(E0 - H_KK)).
The determinant lists and signs are plain integer bookkeeping computed once
per space.  Only small spaces are meant (the full (pq|rs) array is built).

Gradient convention: for a real E2 of a complex input z the gradient is
dE2/dRe z + i dE2/dIm z (what torch returns).  h and every B[t][L] are
Hermitian parameters, so their gradients are projected, (G + G^H) / 2; C is
an unconstrained complex vector.
"""
from itertools import combinations

import numpy as np
import torch

from .space import apply_ops, bits


class CouplingLists:
    """Every <K|H|L> of one space as index lists: singles (K, L, p, q, sign)
    and doubles (K, L, p, q, r, s, sign) with K running over Q (q_mode rule of
    oracle.space) and, separately, over P (the reference Hamiltonian)."""

    def __init__(self, space, q_mode=0):
        P = space.p_dets()
        self.P = P
        pidx = {d: i for i, d in enumerate(P)}
        n = space.n
        qidx = {}
        sq = {"K": [], "L": [], "p": [], "q": [], "g": []}
        dq = {"K": [], "L": [], "p": [], "q": [], "r": [], "s": [], "g": []}
        sp = {"K": [], "L": [], "p": [], "q": [], "g": []}
        dp = {"K": [], "L": [], "p": [], "q": [], "r": [], "s": [], "g": []}
        for j, L in enumerate(P):
            occ = bits(L)
            vir = [p for p in range(n) if not L >> p & 1]
            for q in occ:
                for p in vir:
                    K = L ^ (1 << q) ^ (1 << p)
                    g, D = apply_ops(L, [("a", q), ("c", p)])
                    assert D == K
                    tgt = self._target(space, K, pidx, qidx, q_mode)
                    if tgt is None:
                        continue
                    lst, k = tgt
                    t = sp if lst == "P" else sq
                    for key, val in (("K", k), ("L", j), ("p", p), ("q", q), ("g", g)):
                        t[key].append(val)
            for q, s in combinations(occ, 2):
                for p, r in combinations(vir, 2):
                    K = L ^ (1 << q) ^ (1 << s) ^ (1 << p) ^ (1 << r)
                    g, D = apply_ops(L, [("a", q), ("a", s), ("c", r), ("c", p)])
                    assert D == K
                    tgt = self._target(space, K, pidx, qidx, q_mode)
                    if tgt is None:
                        continue
                    lst, k = tgt
                    t = dp if lst == "P" else dq
                    for key, val in (("K", k), ("L", j), ("p", p), ("q", q), ("r", r), ("s", s),
                                     ("g", g)):
                        t[key].append(val)
        self.Q = sorted(qidx, key=lambda d: qidx[d])
        self.single_q = {k: np.asarray(v, dtype=np.int64) for k, v in sq.items()}
        self.double_q = {k: np.asarray(v, dtype=np.int64) for k, v in dq.items()}
        self.single_p = {k: np.asarray(v, dtype=np.int64) for k, v in sp.items()}
        self.double_p = {k: np.asarray(v, dtype=np.int64) for k, v in dp.items()}
        occ_q = np.zeros((len(self.Q), n))
        for i, K in enumerate(self.Q):
            occ_q[i, bits(K)] = 1.0
        occ_p = np.zeros((len(P), n))
        for i, L in enumerate(P):
            occ_p[i, bits(L)] = 1.0
        self.occ_q = occ_q
        self.occ_p = occ_p

    @staticmethod
    def _target(space, K, pidx, qidx, q_mode):
        if K in pidx:
            return "P", pidx[K]
        if q_mode == 1 and (K & space.core_mask) == space.core_mask and not (K & space.virt_mask):
            return None
        if K not in qidx:
            qidx[K] = len(qidx)
        return "Q", qidx[K]


def _t(x):
    return torch.from_numpy(np.asarray(x))


def eri(Bs, ws):
    """(pq|rs) over all spinors from the factor sets."""
    out = 0
    for B, w in zip(Bs, ws):
        out = out + w * torch.einsum("lpq,lrs->pqrs", B, B)
    return out


def fold_frozen_core(h, g, n_fc):
    """h^FC and (pq|rs) restricted to the correlated spinors."""
    if n_fc > 0:
        fc = torch.arange(n_fc)
        h = h + g[:, :, fc, fc].sum(-1) - g[:, fc, fc, :].sum(1)
    return h[n_fc:, n_fc:], g[n_fc:, n_fc:, n_fc:, n_fc:]


def energy(space, cl, h_full, Bs, ws, n_fc, c, b=0.0):
    """E2 and E0 (E0 within the correlated space, frozen-core constant
    dropped) as torch scalars differentiable in h_full, every B and c.
    cl: CouplingLists of space."""
    g_full = eri(Bs, ws)
    h, g = fold_frozen_core(h_full, g_full, n_fc)
    n = space.n
    occ_p = _t(cl.occ_p).to(torch.complex128)
    # one-body operator in the field of each reference determinant:
    # F_L[p,q] = h_pq + sum_{j in L} ((pq|jj) - (pj|jq))
    gJ = torch.diagonal(g, dim1=2, dim2=3)             # [p,q,j] = (pq|jj)
    gK = torch.diagonal(g, dim1=1, dim2=2)             # [p,q,j] = (pj|jq)
    FL = h.unsqueeze(0) + torch.einsum("pqj,lj->lpq", gJ - gK, occ_p)

    def sigma(single, double, n_k):
        out = torch.zeros(n_k, dtype=torch.complex128)
        if len(single["K"]):
            v = FL[_t(single["L"]), _t(single["p"]), _t(single["q"])] * _t(single["g"]).to(torch.float64)
            out = out.index_add(0, _t(single["K"]), v * c[_t(single["L"])])
        if len(double["K"]):
            p, q, r, s = (_t(double[k]) for k in "pqrs")
            v = (g[p, q, r, s] - g[p, s, r, q]) * _t(double["g"]).to(torch.float64)
            out = out.index_add(0, _t(double["K"]), v * c[_t(double["L"])])
        return out

    # diagonal energies: sum_{p in D} Re h_pp + sum_{p<q in D} W_pq
    hd = torch.real(torch.diagonal(h))
    W = torch.real(torch.einsum("ppqq->pq", g) - torch.einsum("pqqp->pq", g))
    W = W - torch.diag(torch.diagonal(W))

    def diag(occ):
        occ = _t(occ)
        return occ @ hd + 0.5 * ((occ @ W) * occ).sum(-1)

    sig_pp = sigma(cl.single_p, cl.double_p, len(cl.P))
    Hc = sig_pp + diag(cl.occ_p).to(torch.complex128) * c
    norm = torch.real(torch.vdot(c, c))
    E0 = torch.real(torch.vdot(c, Hc)) / norm
    sig_q = sigma(cl.single_q, cl.double_q, len(cl.Q))
    den = E0 - diag(cl.occ_q)
    if b == 0.0:
        wgt = 1.0 / den
    else:
        wgt = torch.real(1.0 / torch.complex(den, b / den))
    E2 = (torch.abs(sig_q) ** 2 * wgt).sum() / norm
    return E2, E0


def hermitian_part(G):
    """(G + G^H) / 2 over the last two dimensions."""
    return 0.5 * (G + G.conj().transpose(-1, -2))


def energy_and_gradient(space, h_full, Bs, ws, n_fc, c, q_mode=0, cl=None, b=0.0):
    """E2 and its gradients (dh, [dB_t], dc) as numpy arrays; dh and dB are
    Hermitian-projected.  b: level-shift constant (Sec. 2.6)."""
    if cl is None:
        cl = CouplingLists(space, q_mode)
    h = torch.tensor(np.asarray(h_full), dtype=torch.complex128, requires_grad=True)
    B = [torch.tensor(np.asarray(x), dtype=torch.complex128, requires_grad=True) for x in Bs]
    cc = torch.tensor(np.asarray(c), dtype=torch.complex128, requires_grad=True)
    E2, E0 = energy(space, cl, h, B, ws, n_fc, cc, b)
    grads = torch.autograd.grad(E2, [h] + B + [cc])
    dh = hermitian_part(grads[0]).numpy()
    dB = [hermitian_part(x).numpy() for x in grads[1:-1]]
    dc = grads[-1].numpy()
    return E2.item(), E0.item(), dh, dB, dc, cl
