"""Frozen-core / frozen-virtual sweep in one batched call on the GPU: every
grid point equals its own single-instance call bit for bit and the oracle
run on the same frozen problem (frozen core folded, top virtuals dropped)
within 1e-9 Eh."""
import math

import numpy as np
import pytest

import synth.problems as SP
from oracle import run
from oracle.classes import ClassOracle
from oracle.space import ActiveSpace

from helpers import oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu


def oracle_point(pb, h, Bs, ws, k, m, c_o):
    n = h.shape[0] - m
    hc, Bc = run.correlated_inputs(h[:n, :n], [B[:, :n, :n] for B in Bs], ws, pb.n_fc + k)
    sp = ActiveSpace(pb.n_c - k, pb.sub_sizes, pb.n_elec, pb.base, pb.max_hops, pb.n_v - m)
    parts, _ = ClassOracle(sp, hc, Bc, ws).e2(c_o)
    return math.fsum(parts.values())


@pytest.mark.parametrize("name,core,virt", [("s_tiles", [0, 1, 2], [0, 10, 40]), ("s_fc", [0, 2], [0, 3])])
def test_sweep_matches_single_calls_and_oracle(name, core, virt):
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd.sweep import FrozenSweep
    pb = problem(name)
    _, _, c_o, P_o = oracle_reference(name)
    sw = FrozenSweep(M.desc_of_problem(pb), core, virt)
    dev = sw.engine.device
    h, Bs = SP.one_body(pb), SP.factors(pb)
    c = torch.from_numpy(np.ascontiguousarray(to_plan_order(c_o, P_o, sw.plan.ref_strings(), pb.n_c))).to(dev)
    print(f"[gpu] frozen sweep {name} {core} x {virt}", flush=True)
    insts = sw.inputs(h.to(dev), [B.to(dev) for B in Bs], c)
    grid, _ = sw.energy(None, None, None, insts)
    grid = grid.cpu().numpy()
    hn, Bn, ws = h.numpy(), [B.numpy() for B in Bs], SP.weights(pb)
    for i, k in enumerate(core):
        for j, m in enumerate(virt):
            d = sw.descs[i * len(virt) + j]
            one = float(M.Engine(M.Plan(d)).energy([insts[i * len(virt) + j]], parts=False)[0].item())
            assert one == float(grid[i, j]), (name, k, m, one, grid[i, j])
            ref = oracle_point(pb, hn, Bn, ws, k, m, c_o)
            assert abs(grid[i, j] - ref) <= 1e-9, (name, k, m, grid[i, j], ref)
