"""Extreme launch shapes give the same E2 and gradients as the built-in
rules (only the summation order changes)."""
import numpy as np
import pytest

import synth.problems as SP
from paper_2608_11529_amd import capi

from helpers import oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu


def uniform(v):
    t = capi.Tuning()
    for knob in ("sigma_blocks", "bwd_blocks", "bwd_row_blocks"):
        for k in range(capi.N_CLASS):
            getattr(t, knob)[k] = v
    return t


@pytest.mark.parametrize("name", ["s_das", "s_fc", "c0"])
def test_tuned_plans_match_builtin(name):
    import torch
    import paper_2608_11529_amd as M
    pb = problem(name)
    _, _, c_o, P_o = oracle_reference(name)
    desc = M.desc_of_problem(pb)
    res = []
    for tu in (None, uniform(1), uniform(1 << 20)):
        plan = M.Plan(desc, tuning=tu)
        eng = M.Engine(plan)
        dev = eng.device
        c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c))).to(dev)
        ins = [(SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)], c)]
        print(f"[gpu] tuned plan {name}", flush=True)
        e2 = float(eng.energy(ins, parts=False)[0].item())
        (dh, dB, dc), = eng.backward(ins)[0]
        res.append((e2, dh.cpu().numpy(), [x.cpu().numpy() for x in dB], dc.cpu().numpy()))
    check_same(res)


def check_same(res):
    e0, h0, B0, c0 = res[0]
    for e, h, B, c in res[1:]:
        assert abs(e - e0) <= 1e-12 * max(1.0, abs(e0))
        assert np.abs(h - h0).max() <= 1e-11 * np.abs(h0).max()
        assert np.abs(c - c0).max() <= 1e-11 * np.abs(c0).max()
        for x, y in zip(B, B0):
            assert np.abs(x - y).max() <= 1e-11 * np.abs(y).max()


@pytest.mark.parametrize("name", ["s_tiles", "c0"])
def test_pair_tile_shapes_match_rule(name):
    """Both block edges of the FP64 pair-integral build, forced through the
    tuning, give the built-in rule's E2 and gradients."""
    import torch
    import paper_2608_11529_amd as M
    pb = problem(name)
    _, _, c_o, P_o = oracle_reference(name)
    desc = M.desc_of_problem(pb)
    res = []
    for pt in (0, 64, 128):
        t = capi.Tuning()
        t.pair_tile = pt
        plan = M.Plan(desc, tuning=t)
        eng = M.Engine(plan)
        dev = eng.device
        c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c))).to(dev)
        ins = [(SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)], c)]
        print(f"[gpu] pair_tile {pt} {name}", flush=True)
        e2 = float(eng.energy(ins, parts=False)[0].item())
        (dh, dB, dc), = eng.backward(ins)[0]
        res.append((e2, dh.cpu().numpy(), [x.cpu().numpy() for x in dB], dc.cpu().numpy()))
    check_same(res)
