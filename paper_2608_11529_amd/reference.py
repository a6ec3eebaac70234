"""Reference states for a problem: the lowest eigenvectors of the
reference-space Hamiltonian H_PP (eq. zeroh: H^(0) is the full H inside P);
Psi0 is the lowest, and several states serve the state-specific E2_m.

H_PP is assembled on the GPU by the library (mrpt2_reference_hamiltonian);
its lowest eigenpair is found on the host with LAPACK (dense, small N_P) or
ARPACK Lanczos (large N_P).  This prepares an input of the energy; it is not
part of the E2 evaluation.
"""
import numpy as np


def lowest_eigenvector(H):
    """Lowest eigenpair of a Hermitian host matrix, phase fixed so that the
    largest component is real and positive."""
    n = H.shape[0]
    if n <= 3000:
        w, v = np.linalg.eigh(H)
        e, c = float(w[0]), v[:, 0]
    else:
        import scipy.sparse.linalg as sla
        w, v = sla.eigsh(H, k=1, which="SA", tol=1e-13, maxiter=20000)
        e, c = float(w[0]), v[:, 0]
    k = int(np.argmax(np.abs(c)))
    c = c * (abs(c[k]) / c[k])
    return e, c / np.linalg.norm(c)


def ground_state(engine, h, Bs, inst=0):
    """Psi0 in the plan's reference order as a complex128 device tensor, and
    its energy relative to the core energy."""
    torch = engine.torch
    H = engine.reference_hamiltonian(h, Bs, inst).cpu().numpy()
    e, c = lowest_eigenvector(H)
    return torch.from_numpy(np.ascontiguousarray(c)).to(engine.device), e


def lowest_states(H, k):
    """The k lowest eigenpairs of a Hermitian host matrix (ascending), each
    vector normalised with its largest component real and positive."""
    n = H.shape[0]
    if n <= 3000:
        w, v = np.linalg.eigh(H)
        w, v = w[:k], v[:, :k]
    else:
        import scipy.sparse.linalg as sla
        w, v = sla.eigsh(H, k=k, which="SA", tol=1e-13, maxiter=20000)
        o = np.argsort(w)
        w, v = w[o], v[:, o]
    out = np.empty((k, n), dtype=np.complex128)
    for j in range(k):
        c = v[:, j]
        i = int(np.argmax(np.abs(c)))
        out[j] = c * (abs(c[i]) / c[i]) / np.linalg.norm(c)
    return np.asarray(w, dtype=np.float64), out


def states(engine, h, Bs, k, inst=0):
    """The k lowest reference states as a complex128 device tensor
    [k, N_P] in the plan's order, and their energies relative to the core."""
    torch = engine.torch
    H = engine.reference_hamiltonian(h, Bs, inst).cpu().numpy()
    e, C = lowest_states(H, k)
    return torch.from_numpy(np.ascontiguousarray(C)).to(engine.device), e
