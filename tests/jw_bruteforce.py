"""Brute-force second quantisation by the Jordan-Wigner construction.

Independent of the Slater-Condon rules used by the oracle: creation operators
are Kronecker products of 2x2 matrices,
    a+_p = Z x ... x Z (p factors) x s+ x 1 x ... x 1,   Z = diag(1, -1),
acting on the occupation-number basis, and the Hamiltonian
    H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q
is assembled as a sparse matrix through E_pq = a+_p a_q and
a+_p a+_r a_s a_q = E_pq E_rs - delta_qr E_ps.  Kronecker index i of a basis
state holds spinor p in bit (n - 1 - p); determinant bit masks are mapped to
it by reversing the bits.  Feasible for n <= 12 spinors.
"""
import numpy as np
import scipy.sparse as sps


def creation_ops(n):
    Z = sps.csr_matrix(np.diag([1.0, -1.0]))
    I2 = sps.identity(2, format="csr")
    sp = sps.csr_matrix(np.array([[0.0, 0.0], [1.0, 0.0]]))   # |0> -> |1>
    ops = []
    for p in range(n):
        m = sps.identity(1, format="csr")
        for q in range(n):
            m = sps.kron(m, Z if q < p else (sp if q == p else I2), format="csr")
        ops.append(m.astype(np.complex128))
    return ops


def hamiltonian(h, g):
    """Sparse H over all 2^n occupation states; g[p,q,r,s] = (pq|rs)."""
    n = h.shape[0]
    cr = creation_ops(n)
    an = [c.T.conj().tocsr() for c in cr]
    E = [[(cr[p] @ an[q]).tocsr() for q in range(n)] for p in range(n)]
    dim = 2 ** n
    H = sps.csr_matrix((dim, dim), dtype=np.complex128)
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0:
                H = H + h[p, q] * E[p][q]
    for p in range(n):
        for q in range(n):
            M = sps.csr_matrix((dim, dim), dtype=np.complex128)
            for r in range(n):
                for s in range(n):
                    M = M + g[p, q, r, s] * E[r][s]
            H = H + 0.5 * (E[p][q] @ M)
    for p in range(n):
        for s in range(n):
            c = sum(g[p, q, q, s] for q in range(n))
            H = H - 0.5 * c * E[p][s]
    return H.tocsr()


def kron_index(det, n):
    i = 0
    for p in range(n):
        if det >> p & 1:
            i |= 1 << (n - 1 - p)
    return i


def shifted_resolvent_sum(v, dq, b):
    """Re v^H R^-1 v with R = diag(dq) + i b diag(dq)^-1: the second-order sum
    with the imaginary level shift of Sec. 2.6, by a linear solve over Q."""
    R = np.diag(dq + 1j * b / dq)
    return float(np.real(np.vdot(v, np.linalg.solve(R, v))))


def e2_bruteforce(h, g, p_dets, q_dets, b=0.0, vectors=False, root=0):
    """State `root` (0: lowest) of H restricted to P, its energy E0, and
    E2 = sum_{K in Q} |(H Psi0)_K|^2 / (E0 - H_KK) (b = 0) or its level-shifted
    form (shifted_resolvent_sum); returns (E2, E0, C, H), and with vectors=True
    also ((H Psi0)_Q, E0 - H_QQ)."""
    n = h.shape[0]
    H = hamiltonian(h, g)
    pi = [kron_index(d, n) for d in p_dets]
    qi = [kron_index(d, n) for d in q_dets]
    Hpp = H[pi][:, pi].toarray()
    w, v = np.linalg.eigh(Hpp)
    c = v[:, root]
    k = int(np.argmax(np.abs(c)))
    c = c * (abs(c[k]) / c[k])
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[pi] = c
    s = H @ psi
    diag = H.diagonal()
    e0 = w[root]
    v, dq = s[qi], e0 - diag[qi].real
    if b == 0.0:
        e2 = float(np.sum(np.abs(v) ** 2 / dq))
    else:
        e2 = shifted_resolvent_sum(v, dq, b)
    if vectors:
        return e2, float(e0), c, H, (v, dq)
    return e2, float(e0), c, H
