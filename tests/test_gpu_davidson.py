"""Reference states by the library's block Davidson solver on the device
(mrpt2_reference_states): eigenpairs against dense LAPACK diagonalisation of
the same H_PP, and E2 with the Davidson state against the oracle (whose
reference state comes from its own CPU H_PP)."""
import math

import numpy as np
import pytest

import synth.problems as SP

from helpers import e2_total, oracle_reference, problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,k", [("s_das", 3), ("s_fc", 2), ("s_single", 1), ("s_tiles", 3), ("c0", 4),
                                    ("c0", 12), ("c0", 20), ("c1", 3)])
def test_davidson_matches_dense_eigh(name, k):
    import paper_2608_11529_amd as M
    pb = problem(name)
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    k = min(k, plan.info().n_ref)
    dev = eng.device
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)]
    print(f"[gpu] davidson {name} k={k} N_P={plan.info().n_ref}", flush=True)
    C, e, its = eng.reference_states(h, Bs, k, tol=1e-10)
    H = eng.reference_hamiltonian(h, Bs).cpu().numpy()
    w, v = np.linalg.eigh(H)
    scale = max(1.0, float(np.abs(w).max()))
    assert np.abs(e - w[:k]).max() <= 1e-12 * scale, (e, w[:k])
    Cn = C.cpu().numpy()
    assert np.abs(np.linalg.norm(Cn, axis=1) - 1.0).max() <= 1e-13
    for j in range(k):
        gap = min([abs(w[j] - w[i]) for i in range(len(w)) if i != j] or [1.0])
        ov = abs(np.vdot(v[:, j], Cn[j]))
        assert ov >= 1.0 - max(1e-12, (1e-10 / gap) ** 2), (name, j, ov, gap)
        assert np.linalg.norm(H @ Cn[j] - e[j] * Cn[j]) <= 2e-10
    assert its >= 1


@pytest.mark.parametrize("name", ["s_das", "s_fc", "c0"])
def test_energy_with_davidson_state_matches_oracle(name):
    import paper_2608_11529_amd as M
    pb = problem(name)
    parts_o, _, _, _ = oracle_reference(name)
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    dev = eng.device
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)]
    C, e, _ = eng.reference_states(h, Bs, 1, tol=1e-11)
    print(f"[gpu] E2 with the Davidson state {name}", flush=True)
    e2, parts = eng.energy([(h, Bs, C[0].contiguous())])
    assert abs(float(e2[0]) - e2_total(parts_o)) <= 1e-9
    assert abs(float(parts[0, 10]) - e[0]) <= 1e-10


def test_davidson_iteration_limit_is_reported():
    import paper_2608_11529_amd as M
    pb = problem("c1")
    eng = M.Engine(M.Plan(M.desc_of_problem(pb)))
    dev = eng.device
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)]
    with pytest.raises(M.Mrpt2Error) as ei:
        eng.reference_states(h, Bs, 2, tol=1e-14, max_iter=2)
    assert ei.value.code == 6
