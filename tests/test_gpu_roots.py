"""State-specific E2 of several reference states in one call
(mrpt2_energy_roots): every root equals a single-state call bit for bit and
the oracle with that state as reference (E0_m from the state itself) within
1e-9 Eh; several instances and several roots together; both forms."""
import math

import numpy as np
import pytest

import synth.problems as SP
from oracle import run

from helpers import CLASSES, problem, to_plan_order

pytestmark = pytest.mark.gpu


def oracle_states(name, k):
    pb = problem(name)
    h, Bs = SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)]
    co = run.class_oracle(pb, h, Bs, SP.weights(pb))
    H, _ = co.reference(np.ones(len(co.P), dtype=np.complex128))
    w, v = np.linalg.eigh(H)
    cs, e2 = [], []
    for j in range(k):
        c = v[:, j]
        i = int(np.argmax(np.abs(c)))
        c = c * (abs(c[i]) / c[i])
        parts, _ = co.e2(c)
        cs.append(c)
        e2.append(parts)
    return pb, cs, e2, co.P


def device_inputs(M, pb, plan, cs, P_o, dev, inst=0):
    import torch
    C = np.stack([to_plan_order(c, P_o, plan.ref_strings(inst), pb.n_c) for c in cs])
    h = SP.one_body(pb).to(dev)
    Bs = [B.to(dev) for B in SP.factors(pb)]
    return h, Bs, torch.from_numpy(np.ascontiguousarray(C)).to(dev)


@pytest.mark.parametrize("name,k,precision", [("s_das", 3, 0), ("s_fc", 3, 0), ("s_tiles", 2, 0),
                                              ("c0", 4, 0), ("c0", 3, 1)])
def test_roots_match_single_state_calls_and_oracle(name, k, precision):
    import paper_2608_11529_amd as M
    pb, cs, parts_o, P_o = oracle_states(name, k)
    plan = M.Plan(M.desc_of_problem(pb, precision=precision))
    eng = M.Engine(plan)
    h, Bs, C = device_inputs(M, pb, plan, cs, P_o, eng.device)
    print(f"[gpu] {k} roots of {name} precision={precision}", flush=True)
    e2, parts = eng.energy_roots([(h, Bs, C)])
    e2, parts = e2.cpu().numpy(), parts.cpu().numpy()
    tol = 1e-9 if precision == 0 else 1e-6
    for r in range(k):
        one, q1 = eng.energy([(h, Bs, C[r].contiguous())])
        assert float(one[0]) == e2[r, 0], (name, r, float(one[0]), e2[r, 0])
        assert np.array_equal(q1[0].cpu().numpy(), parts[r, 0])
        for j, cl in enumerate(CLASSES):
            assert abs(parts[r, 0, j] - parts_o[r].get(cl, 0.0)) <= tol, (name, r, cl)
        assert abs(e2[r, 0] - math.fsum(parts_o[r].values())) <= tol, (name, r)
    assert len(set(np.round(parts[:, 0, 10], 9))) == k          # distinct E0_m


def test_roots_of_several_instances():
    import paper_2608_11529_amd as M
    names = ["s_das", "s_fc"]
    got = [oracle_states(nm, 2) for nm in names]
    plan = M.Plan([M.desc_of_problem(g[0]) for g in got])
    eng = M.Engine(plan)
    insts = [device_inputs(M, g[0], plan, g[1], g[3], eng.device, inst=i) for i, g in enumerate(got)]
    print("[gpu] 2 roots x 2 instances", flush=True)
    e2, _ = eng.energy_roots(insts)
    e2 = e2.cpu().numpy()
    for r in range(2):
        one = eng.energy([(h, Bs, C[r].contiguous()) for h, Bs, C in insts], parts=False).cpu().numpy()
        assert np.array_equal(one, e2[r])
        for i, g in enumerate(got):
            assert abs(e2[r, i] - math.fsum(g[2][r].values())) <= 1e-9
