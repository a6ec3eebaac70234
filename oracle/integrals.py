"""Integrals for the oracle (test infrastructure).

Two-electron integrals come in Cholesky form, one factor set per operator
(Dirac-Coulomb, Gaunt, gauge) with a real weight:
    (pq|rs) = sum_t w_t sum_L B[t][L,p,q] B[t][L,r,s]   (chemists' notation).
The Hamiltonian is H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q.

Frozen core (Sec. 2, notation list): with frozen spinors i' always occupied,
    h^FC_pq = h_pq + sum_i' [ (pq|i'i') - (pi'|i'q) ]
and the frozen spinors leave the correlated space; their constant energy is
the same for every determinant and cancels in every denominator, so it is
dropped.
"""
import numpy as np


def eri_block(Bs, ws, P, Q, R, S):
    """(pq|rs) for p in P, q in Q, r in R, s in S (index arrays)."""
    P, Q, R, S = (np.asarray(x) for x in (P, Q, R, S))
    out = np.zeros((len(P), len(Q), len(R), len(S)), dtype=np.complex128)
    for B, w in zip(Bs, ws):
        left = B[:, P][:, :, Q].reshape(B.shape[0], -1)
        right = B[:, R][:, :, S].reshape(B.shape[0], -1)
        out += w * (left.T @ right).reshape(out.shape)
    return out


def fold_frozen_core(h, Bs, ws, n_fc):
    """Returns (h^FC, B) restricted to the correlated spinors."""
    n = h.shape[0]
    hfc = h.astype(np.complex128).copy()
    if n_fc > 0:
        fc = np.arange(n_fc)
        for B, w in zip(Bs, ws):
            d = np.einsum("lii->l", B[:, fc][:, :, fc])          # sum_i' B[L,i',i']
            hfc += w * np.einsum("lpq,l->pq", B, d)               # (pq|i'i')
            hfc -= w * np.einsum("lpi,liq->pq", B[:, :, fc], B[:, fc, :])   # (pi'|i'q)
    keep = slice(n_fc, n)
    return hfc[keep, keep], [B[:, keep, keep] for B in Bs]


def pair_energies(Bs, ws):
    """W_pq = (pp|qq) - (pq|qp), real for Hermitian factors with real weights;
    W_pp = 0."""
    n = Bs[0].shape[1]
    W = np.zeros((n, n))
    for B, w in zip(Bs, ws):
        d = np.einsum("lpp->lp", B)
        coul = np.einsum("lp,lq->pq", d, d)
        exch = np.einsum("lpq,lqp->pq", B, B)
        W += w * (coul - exch).real
    np.fill_diagonal(W, 0.0)
    return W
