"""GPU parity: the HIP path through the C interface against the CPU oracle,
class by class, on small problems covering the edge cases (frozen core, DAS
hop limits, several virtual tiles, single-determinant reference, no core,
full active space) and on config c0.  Tolerance 1e-9 Eh on E2 and every
class part (FP64 path)."""
import sys

import numpy as np
import pytest

import synth.problems as SP

from helpers import CLASSES, SMALL, e2_total, oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu

TOL = 1e-9


def gpu_energy(name, q_mode=0):
    import torch
    import paper_2608_11529_amd as M
    pb = problem(name)
    parts_o, E0_o, c_o, P_o = oracle_reference(name, q_mode)
    plan = M.Plan(M.desc_of_problem(pb, q_mode=q_mode))
    eng = M.Engine(plan)
    h, Bs = SP.one_body(pb), SP.factors(pb)
    c = to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c)
    dev = eng.device
    hd = h.to(dev)
    Bd = [B.to(dev) for B in Bs]
    cd = torch.from_numpy(np.ascontiguousarray(c)).to(dev)
    print(f"[gpu] {name} q_mode={q_mode} N_P={plan.info().n_ref} N_Q={plan.info().n_ext}", flush=True)
    e2, parts = eng.energy([(hd, Bd, cd)])
    torch.cuda.synchronize()
    return float(e2[0].item()), parts[0].cpu().numpy(), parts_o, E0_o


@pytest.mark.parametrize("name", list(SMALL) + ["c0"])
def test_energy_matches_oracle(name):
    e2, parts, parts_o, E0_o = gpu_energy(name)
    ref = e2_total(parts_o)
    for k, cl in enumerate(CLASSES):
        assert abs(parts[k] - parts_o.get(cl, 0.0)) <= TOL, (name, cl, parts[k], parts_o.get(cl))
    assert abs(e2 - ref) <= TOL, (name, e2, ref)
    assert abs(parts[9] - e2) <= 1e-15 * max(1.0, abs(e2))


@pytest.mark.parametrize("name", ["s_das", "s_hop0"])
def test_q_mode_core_virtual_only(name):
    e2, parts, parts_o, _ = gpu_energy(name, q_mode=1)
    assert parts[8] == 0.0
    assert abs(e2 - e2_total(parts_o)) <= TOL


def test_reference_energy_relative_to_core():
    """parts[10] = E0 - E_core: check against the oracle's E0 minus the
    core energy computed from its own pair energies."""
    import oracle.run as R
    name = "s_fc"
    e2, parts, parts_o, E0_o = gpu_energy(name)
    pb = problem(name)
    h, Bs = SP.one_body(pb), SP.factors(pb)
    co = R.class_oracle(pb, h.numpy(), [B.numpy() for B in Bs], SP.weights(pb))
    ecore = co.energy_of(co.core)
    assert abs(parts[10] - (E0_o - ecore)) < 1e-10


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-v"]))
