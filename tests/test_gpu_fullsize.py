"""Whole-workload parity: the GPU path in the launch configuration the
benchmark times (launch shapes from the package's autotuned table) against
oracle values computed beforehand by committed oracle-only scripts
(tests/golden/make_fullsize_golden.py, make_c3_golden.py).

  * c2 and c4: E0 - E_core and E2 of every excitation class of the whole
    external space (eq. pt2en, Sec. 2.4) with the oracle's ground state,
    FP64 within 1e-9 Eh and the mixed form within 1e-6 Eh, and the partial
    sums of individual work blocks of the two-virtual classes (first and last
    core holes, first tile, the last and partial 64-wide virtual tile,
    diagonal tile pairs) against the oracle's restricted sums;
  * c3: the 64 uneven instances in one batched plan; the fourteen instances
    with oracle values (the eight with the fewest external determinants and
    six covering the other shapes) compared class by class.
"""
import json
import math
import os

import numpy as np
import pytest

import synth.problems as SP

from helpers import CLASSES, to_plan_order

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-9, 1: 1e-6}


def golden(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.skip("oracle values %s not yet written (tests/golden/make_fullsize_golden.py)" % name)
    with open(path) as f:
        g = json.load(f)
    if "instances" not in g and "blocks" not in g:
        pytest.skip("oracle values %s incomplete (run still in progress)" % name)
    return g


def c_of(g):
    return np.array(g["c_re"]) + 1j * np.array(g["c_im"])


def block_index(plan, k, blk, n_tp):
    """Partial-sum indices of the GPU work blocks that make up an oracle
    block (class k, hole tuple, a range, b range): one block for (2,2) and
    (1,2), the blocks of every string tile for (0,2).  Each index is checked
    against the plan's own description of the block."""
    holes = tuple(blk["holes"])
    a_lo, a_hi = blk["a"]
    b_lo, b_hi = blk["b"]
    I, J = a_lo // 64, b_lo // 64
    tps = {}
    for tp in range(n_tp):                    # class (2,2): block tp is core pair 0, tile pair tp
        d = plan.class_block(0, tp)
        tps[(d.a_lo // 64, d.b_lo // 64)] = tp
    tp = tps[(I, J)]
    nb = plan.class_blocks(k)
    if k == 0:
        n_hp = nb // n_tp
        hp = next(i for i in range(n_hp) if tuple(plan.class_block(k, i * n_tp).hole[:2]) == holes)
        idx = [hp * n_tp + tp]
    elif k == 1:
        # 16 x 16 sub-tile (sa, sb) of the tile pair; ranges clamped at the
        # end of the virtual block may be empty, so match the described ranges
        base = holes[0] * n_tp * 16 + tp * 16
        subs = [base + q for q in range(16)
                if (lambda d: (d.a_lo, d.a_hi, d.b_lo, d.b_hi))(plan.class_block(k, base + q)) == (a_lo, a_hi, b_lo, b_hi)]
        assert subs, (k, blk)
        idx = subs[:1]
    else:
        n_tiles = nb // (n_tp * 64)
        la = a_lo - I * 64
        idx = [(tp * 64 + la) * n_tiles + t for t in range(n_tiles)]
    for b in (idx[0], idx[-1]):
        d = plan.class_block(k, b)
        assert tuple(d.hole[:d.n_holes]) == holes, (k, blk, b)
        assert (d.a_lo, d.a_hi, d.b_lo, d.b_hi) == (a_lo, a_hi, b_lo, b_hi), (k, blk, b, d.a_lo, d.a_hi)
    return idx


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_whole_config_matches_oracle(name):
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd import autotune
    g = golden("%s_full_oracle.json" % name)
    pb = SP.config(name)
    dev = torch.device("cuda:0")
    print("[gpu] %s whole: generating inputs" % name, flush=True)
    h = SP.one_body(pb, dev)
    Bs = SP.factors(pb, dev)
    for prec in (0, 1):
        desc = M.desc_of_problem(pb, precision=prec)
        plan = M.Plan(desc, tuning=autotune.tuning_for(desc))
        eng = M.Engine(plan, dev)
        c = to_plan_order(c_of(g), g["p_strings"], plan.ref_strings(), pb.n_c)
        cd = torch.from_numpy(np.ascontiguousarray(c)).to(dev)
        print("[gpu] %s whole, precision %d" % (name, prec), flush=True)
        e2, parts = eng.energy([(h, Bs, cd)])
        parts = parts[0].cpu().numpy().copy()
        assert abs(parts[10] - g["E0_minus_Ecore"]) <= 1e-9, (parts[10], g["E0_minus_Ecore"])
        for k, cl in enumerate(CLASSES):
            want = g["parts"]["%d%d" % cl]
            assert abs(parts[k] - want) <= TOL[prec], (name, prec, cl, parts[k], want)
        assert abs(float(e2[0]) - g["E2"]) <= TOL[prec], (name, prec, float(e2[0]), g["E2"])
        # work blocks of the two-virtual classes
        info = plan.info()
        n_tp = plan.class_blocks(0) // math.comb(pb.n_c, 2)
        norm = parts[11]
        for k in range(3):
            assert info.kernel_class[k] in (1, 2, 3), (name, k)
        partials = {k: eng.class_partials(k) for k in range(3)}
        for blk in g["blocks"]:
            k = ["22", "12", "02"].index(blk["class"])
            idx = block_index(plan, k, blk, n_tp)
            got = math.fsum(partials[k][idx].tolist()) / norm
            want = blk["value"]
            # the synthetic integrals decay as exp(-|p - q|/8), so blocks far
            # from the occupied spinors hold values down to 1e-120: FP64 is
            # checked relative to each block's own size, the mixed form (whose
            # FP32 integrals underflow there) within 1e-6 relative plus 1e-9 Eh
            tol = 1e-30 + 1e-9 * abs(want) if prec == 0 else 1e-9 + 1e-6 * abs(want)
            assert abs(got - want) <= tol, (name, prec, blk, got, want)
        del eng, plan
        torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [0, 1])
def test_c3_instances_in_batched_plan(precision):
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd import autotune
    g = golden("c3_oracle.json")["instances"]
    dev = torch.device("cuda:0")
    pbs = [SP.batched_instance(s) for s in range(64)]
    descs = [M.desc_of_problem(pb, precision=precision) for pb in pbs]
    plan = M.Plan(descs, tuning=autotune.tuning_for(descs))
    eng = M.Engine(plan, dev)
    print("[gpu] c3 batched plan of 64 instances, precision %d: generating inputs" % precision, flush=True)
    ins = []
    for s, pb in enumerate(pbs):
        if str(s) in g:
            c = to_plan_order(c_of(g[str(s)]), g[str(s)]["p_strings"], plan.ref_strings(s), pb.n_c)
        else:
            # any reference vector serves the instances without oracle values
            c = 0.05 * SP.complex_normal(s, 900, (plan.info(s).n_ref,)).numpy()
            c[0] += 1.0
        ins.append((SP.one_body(pb, dev), SP.factors(pb, dev),
                    torch.from_numpy(np.ascontiguousarray(c)).to(dev)))
    print("[gpu] c3 batched call", flush=True)
    e2, parts = eng.energy(ins)
    e2 = e2.cpu().numpy().copy()
    parts = parts.cpu().numpy().copy()
    assert np.all(np.isfinite(e2))
    for key, gi in g.items():
        s = int(key)
        for k, cl in enumerate(CLASSES):
            want = gi["parts"]["%d%d" % cl]
            assert abs(parts[s][k] - want) <= TOL[precision], (s, cl, parts[s][k], want)
        assert abs(e2[s] - gi["E2"]) <= TOL[precision], (s, e2[s], gi["E2"])
