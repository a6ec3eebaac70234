"""Reference states for a problem: the lowest eigenvectors of the
reference-space Hamiltonian H_PP (eq. zeroh: H^(0) is the full H inside P);
Psi0 is the lowest, and several states serve the state-specific E2_m.

ground_state and states use the library's device solver
(mrpt2_reference_states: H_PP assembled on the GPU, block Davidson).
host_ground_state copies the library's H_PP to the host and diagonalises it
with LAPACK (dense, small N_P) or ARPACK Lanczos (large N_P); it is kept as a
second route to the same state.  Both prepare an input of the energy; neither
is part of the E2 evaluation.
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


def ground_state(engine, h, Bs, inst=0, tol=1e-10):
    """Psi0 in the plan's reference order as a complex128 device tensor, and
    its energy relative to the core energy (device Davidson solver)."""
    C, e, _ = engine.reference_states(h, Bs, 1, tol=tol, inst=inst)
    return C[0].contiguous(), float(e[0])


def host_ground_state(engine, h, Bs, inst=0):
    """ground_state through the host: the library's H_PP copied to the host
    and diagonalised with LAPACK or ARPACK."""
    torch = engine.torch
    H = engine.reference_hamiltonian(h, Bs, inst).cpu().numpy()
    e, c = lowest_eigenvector(H)
    return torch.from_numpy(np.ascontiguousarray(c)).to(engine.device), e


def states(engine, h, Bs, k, inst=0, tol=1e-10):
    """The k lowest reference states as a complex128 device tensor
    [k, N_P] in the plan's order, and their energies relative to the core
    (device Davidson solver)."""
    C, e, _ = engine.reference_states(h, Bs, k, tol=tol, inst=inst)
    return C, e
