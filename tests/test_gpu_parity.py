"""GPU parity: the HIP path through the C interface against the CPU oracle,
class by class, on small problems covering the edge cases (frozen core, DAS
hop limits, several virtual tiles, single-determinant reference, no core,
full active space, wide active spaces that select every width of the
class (1,2) kernel) and on config c0.  Tolerance 1e-9 Eh on E2 and every
class part (FP64 path), and each part also within 1e-9 of its own size (the
parts of the wide problems are as small as 1e-11 Eh)."""
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
        want = parts_o.get(cl, 0.0)
        assert abs(parts[k] - want) <= TOL, (name, cl, parts[k], want)
        assert abs(parts[k] - want) <= 1e-9 * abs(want) + 1e-15, (name, cl, parts[k], want)
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


def golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "%s_oracle.json" % name)
    with open(path) as f:
        return json.load(f)


def test_c1_matches_oracle_golden():
    """Config c1 in full (1.25e9 external determinants, DAS with one hop,
    Dirac-Coulomb + Gaunt) against the oracle's stored per-class values."""
    import torch
    import paper_2608_11529_amd as M
    g = golden("c1")
    pb = SP.config("c1")
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    c_o = np.array(g["c_re"]) + 1j * np.array(g["c_im"])
    c = to_plan_order(c_o, g["p_strings"], plan.ref_strings(), pb.n_c)
    dev = eng.device
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)]
    print("[gpu] c1", flush=True)
    e2, parts = eng.energy([(h, Bs, torch.from_numpy(np.ascontiguousarray(c)).to(dev))])
    parts = parts[0].cpu().numpy()
    for k, cl in enumerate(CLASSES):
        ref = g["parts"]["%d%d" % cl]
        assert abs(parts[k] - ref) <= TOL, (cl, parts[k], ref)
    assert abs(float(e2[0]) - g["E2"]) <= TOL


def test_c1_mixed_precision_within_tolerance():
    """FP32-MFMA pair integrals with FP64 denominators and sums: within
    1e-6 Eh of the oracle on c1, class by class."""
    import torch
    import paper_2608_11529_amd as M
    g = golden("c1")
    pb = SP.config("c1")
    plan = M.Plan(M.desc_of_problem(pb, precision=1))
    eng = M.Engine(plan)
    c_o = np.array(g["c_re"]) + 1j * np.array(g["c_im"])
    c = to_plan_order(c_o, g["p_strings"], plan.ref_strings(), pb.n_c)
    dev = eng.device
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)]
    print("[gpu] c1 mixed", flush=True)
    e2, parts = eng.energy([(h, Bs, torch.from_numpy(np.ascontiguousarray(c)).to(dev))])
    parts = parts[0].cpu().numpy()
    for k, cl in enumerate(CLASSES):
        ref = g["parts"]["%d%d" % cl]
        assert abs(parts[k] - ref) <= 1e-6, (cl, parts[k], ref)
    assert abs(float(e2[0]) - g["E2"]) <= 1e-6


@pytest.mark.parametrize("name", ["s_tiles", "s_fc"])
def test_mixed_precision_small(name):
    e2_64, parts_64, parts_o, _ = gpu_energy(name)
    import torch
    import paper_2608_11529_amd as M
    pb = problem(name)
    parts_o, E0_o, c_o, P_o = oracle_reference(name)
    plan = M.Plan(M.desc_of_problem(pb, precision=1))
    eng = M.Engine(plan)
    dev = eng.device
    c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c))).to(dev)
    e2, parts = eng.energy([(SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)], c)])
    assert abs(float(e2[0]) - e2_total(parts_o)) <= 1e-6


def test_bitwise_repeatable():
    """Fixed-order reductions: two evaluations agree bit for bit."""
    import torch
    import paper_2608_11529_amd as M
    pb = problem("s_tiles")
    parts_o, E0_o, c_o, P_o = oracle_reference("s_tiles")
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    dev = eng.device
    c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c))).to(dev)
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)]
    a = eng.energy([(h, Bs, c)])[1].clone()
    b = eng.energy([(h, Bs, c)])[1].clone()
    assert torch.equal(a, b)


def test_nonfinite_input_is_reported():
    import torch
    import paper_2608_11529_amd as M
    pb = problem("s_cas")
    parts_o, E0_o, c_o, P_o = oracle_reference("s_cas")
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    dev = eng.device
    c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c))).to(dev)
    h, Bs = SP.one_body(pb).to(dev), [B.to(dev).clone() for B in SP.factors(pb)]
    Bs[0][3, 2, 5] = complex(float("nan"), 0.0)
    with pytest.raises(M.Mrpt2Error) as ei:
        eng.energy([(h, Bs, c)])
    assert ei.value.code == 6


def test_workspace_too_small_is_reported():
    import ctypes
    import paper_2608_11529_amd as M
    pb = problem("s_cas")
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    L = M.capi.lib()
    arr = (M.capi.Inputs * 1)()
    code = L.mrpt2_energy(plan.handle, arr, eng.persistent.data_ptr(), eng.workspace.data_ptr(),
                          plan.workspace_bytes - 1, eng._sptr(), eng.e2.data_ptr(), None)
    assert code == 4


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-v"]))


def test_zero_denominator_is_reported():
    """A degenerate instance: a single-determinant reference, no
    two-electron integrals and one virtual orbital energy equal to a core
    orbital energy, so that the single excitation between them has
    E0 - H_KK = 0 exactly (eq. pt2en is undefined there).  Without a level
    shift the energy and the adjoint call report MRPT2_ERR_NUMERIC; with the
    imaginary level shift of Sec. 2.6 (whose weight Delta^3/(Delta^4 + b^2)
    vanishes at Delta = 0) the same instance gives a finite energy, and the
    adjoint call the same E2."""
    import torch
    import paper_2608_11529_amd as M
    pb = problem("s_single")
    dev = torch.device("cuda:0")
    h = SP.one_body(pb).to(dev)
    c_, a_ = 1, pb.n_fc + pb.n_c + 2
    h[a_, a_] = h[c_, c_]
    assert float(h[a_, c_].abs()) > 0.0
    Bs = [torch.zeros_like(B).to(dev) for B in SP.factors(pb)]
    c = torch.ones(1, dtype=torch.complex128, device=dev)
    eng = M.Engine(M.Plan(M.desc_of_problem(pb)))
    with pytest.raises(M.Mrpt2Error) as ei:
        eng.energy([(h, Bs, c)])
    assert ei.value.code == 6
    # the adjoint call (which forms E2 in its own passes) reports it as well
    with pytest.raises(M.Mrpt2Error) as ei:
        eng.backward([(h, Bs, c)])
    assert ei.value.code == 6
    eng_ls = M.Engine(M.Plan(M.desc_of_problem(pb, level_shift_b=0.5)))
    e2, parts = eng_ls.energy([(h, Bs, c)])
    assert np.isfinite(float(e2[0]))
    outs, e2b = eng_ls.backward([(h, Bs, c)])
    assert abs(float(e2b[0]) - float(e2[0])) <= 1e-13 * max(1.0, abs(float(e2[0])))
