"""GPU parity of the imaginary level shift (Sec. 2.6): every inverse
denominator 1/Delta becomes Re 1/(Delta + i b/Delta).  E2 class by class
(FP64 1e-9 Eh, mixed form 1e-6 Eh) and the adjoint element by element
against the oracle, which is pinned to a Jordan-Wigner resolvent solve, the
single-determinant closed form and finite differences."""
import math

import numpy as np
import pytest

import synth.problems as SP
from oracle import gradient, run

from helpers import CLASSES, oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu

CASES = [("s_tiles", 2.0), ("s_fc", 2.0), ("s_das", 0.5), ("s_single", 2.0), ("c0", 0.05), ("c0", 2.0),
         ("s_j20", 0.5), ("s_j32", 2.0)]


def shifted_oracle(name, b):
    pb = problem(name)
    _, _, c_o, P_o = oracle_reference(name)
    h, Bs = SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)]
    co = run.class_oracle(pb, h, Bs, SP.weights(pb))
    parts, _ = co.e2(c_o, b=b)
    return pb, parts, c_o, P_o


def gpu_setup(pb, b, c_o, P_o, precision=0):
    import torch
    import paper_2608_11529_amd as M
    plan = M.Plan(M.desc_of_problem(pb, precision=precision, level_shift_b=b))
    eng = M.Engine(plan)
    dev = eng.device
    c = to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c)
    h = SP.one_body(pb).to(dev)
    Bs = [B.to(dev) for B in SP.factors(pb)]
    return plan, eng, h, Bs, torch.from_numpy(np.ascontiguousarray(c)).to(dev)


@pytest.mark.parametrize("name,b", CASES)
def test_level_shift_energy_matches_oracle(name, b):
    pb, parts_o, c_o, P_o = shifted_oracle(name, b)
    plan, eng, h, Bs, c = gpu_setup(pb, b, c_o, P_o)
    print(f"[gpu] level shift {name} b={b} N_Q={plan.info().n_ext}", flush=True)
    e2, parts = eng.energy([(h, Bs, c)])
    parts = parts[0].cpu().numpy()
    for k, cl in enumerate(CLASSES):
        assert abs(parts[k] - parts_o.get(cl, 0.0)) <= 1e-9, (name, cl, parts[k], parts_o.get(cl))
    assert abs(float(e2[0]) - math.fsum(parts_o.values())) <= 1e-9


@pytest.mark.parametrize("name,b", [("s_tiles", 2.0), ("c0", 0.05)])
def test_level_shift_mixed_precision(name, b):
    pb, parts_o, c_o, P_o = shifted_oracle(name, b)
    plan, eng, h, Bs, c = gpu_setup(pb, b, c_o, P_o, precision=1)
    print(f"[gpu] level shift mixed {name} b={b}", flush=True)
    e2, _ = eng.energy([(h, Bs, c)])
    assert abs(float(e2[0]) - math.fsum(parts_o.values())) <= 1e-6


def close(a, b, rel=1e-9, floor=1e-3):
    """Element by element: |a - b| <= rel |b| + floor rel max|b| + 1e-14
    (floor 1e-3 against the oracle, 1 between two GPU results)."""
    scale = max(float(np.abs(b).max()), 1e-300)
    d = np.abs(a - b)
    err = float(d.max())
    worst = float((d / (rel * np.abs(b) + floor * rel * scale + 1e-14)).max())
    return worst <= 1.0, err, scale


@pytest.mark.parametrize("name,b", [("s_das", 2.0), ("s_fc", 0.5), ("s_tiles", 2.0), ("c0", 2.0)])
def test_level_shift_gradient_matches_oracle(name, b):
    pb, parts_o, c_o, P_o = shifted_oracle(name, b)
    plan, eng, h, Bs, c = gpu_setup(pb, b, c_o, P_o)
    print(f"[gpu] level shift backward {name} b={b}", flush=True)
    (dh, dBs, dc), = eng.backward([(h, Bs, c)])[0]
    E2, _, dh_o, dB_o, dc_o, _ = gradient.energy_and_gradient(
        run.space_of(pb), SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)],
        SP.weights(pb), pb.n_fc, c_o, b=b)
    assert abs(float(eng.e2[0].item()) - E2) <= 1e-9
    ok, err, sc = close(dh.cpu().numpy(), dh_o)
    assert ok, (name, "dh", err, sc)
    for t, (g, go) in enumerate(zip(dBs, dB_o)):
        ok, err, sc = close(g.cpu().numpy(), go)
        assert ok, (name, "dB", t, err, sc)
    ok, err, sc = close(dc.cpu().numpy(), to_plan_order(dc_o, P_o, plan.ref_strings(), pb.n_c))
    assert ok, (name, "dc", err, sc)


def test_level_shift_mixed_with_unshifted_instances_in_one_plan():
    """One batched plan holding an unshifted and a shifted instance (each
    instance takes its own kernel variants and adjoint passes): energies and
    gradients equal the single-instance calls, energies match the oracle."""
    import paper_2608_11529_amd as M
    cases = [("s_das", 0.0), ("s_fc", 2.0), ("s_tiles", 0.5)]
    got = [shifted_oracle(nm, b) for nm, b in cases]
    plan = M.Plan([M.desc_of_problem(g[0], level_shift_b=b) for g, (_, b) in zip(got, cases)])
    eng = M.Engine(plan)
    insts = []
    for i, (g, (nm, b)) in enumerate(zip(got, cases)):
        pb, _, c_o, P_o = g
        import torch
        c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, plan.ref_strings(i), pb.n_c)))
        insts.append((SP.one_body(pb).to(eng.device), [B.to(eng.device) for B in SP.factors(pb)],
                      c.to(eng.device)))
    print("[gpu] level shift: mixed batch", flush=True)
    e2 = eng.energy(insts, parts=False).cpu().numpy().copy()
    outs = eng.backward(insts)[0]
    for i, (g, (nm, b)) in enumerate(zip(got, cases)):
        pb, parts_o, _, _ = g
        assert abs(e2[i] - math.fsum(parts_o.values())) <= 1e-9, (nm, b)
        p1, e1, h, Bs, c = gpu_setup(pb, b, g[2], g[3])
        assert float(e1.energy([(h, Bs, c)], parts=False)[0].item()) == e2[i]
        (dh1, dB1, dc1), = e1.backward([(h, Bs, c)])[0]
        dh, dB, dc = outs[i]
        ok, err, sc = close(dh.cpu().numpy(), dh1.cpu().numpy(), rel=1e-12, floor=1.0)
        assert ok, (nm, "dh", err, sc)
        ok, err, sc = close(dc.cpu().numpy(), dc1.cpu().numpy(), rel=1e-12, floor=1.0)
        assert ok, (nm, "dc", err, sc)


def test_level_shift_with_several_states():
    """E2_m of two reference states under the shift in one call equals the
    oracle with each state as reference."""
    import torch
    import paper_2608_11529_amd as M
    b = 2.0
    pb = problem("s_das")
    h, Bs = SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)]
    co = run.class_oracle(pb, h, Bs, SP.weights(pb))
    H, _ = co.reference(np.ones(len(co.P), dtype=np.complex128))
    w, v = np.linalg.eigh(H)
    plan = M.Plan(M.desc_of_problem(pb, level_shift_b=b))
    eng = M.Engine(plan)
    cs = []
    for j in range(2):
        c = v[:, j] * (abs(v[np.argmax(np.abs(v[:, j])), j]) / v[np.argmax(np.abs(v[:, j])), j])
        cs.append(c)
    C = np.stack([to_plan_order(c, co.P, plan.ref_strings(), pb.n_c) for c in cs])
    print("[gpu] level shift: two states", flush=True)
    e2, _ = eng.energy_roots([(torch.from_numpy(h).to(eng.device), [torch.from_numpy(x).to(eng.device) for x in Bs],
                               torch.from_numpy(np.ascontiguousarray(C)).to(eng.device))])
    for j in range(2):
        parts, _ = co.e2(cs[j], b=b)
        assert abs(float(e2[j, 0]) - math.fsum(parts.values())) <= 1e-9, j
