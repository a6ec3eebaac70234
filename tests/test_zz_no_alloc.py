"""The energy entry point without caller-provided workspace
(mrpt2_energy_static), called through the C interface: two calls in a row,
the second on a smaller problem, each equal bit for bit to mrpt2_energy on
the same plan and inputs and within 1e-9 Eh of the oracle; plans whose
workspace exceeds the library's array are refused before any work."""
import ctypes

import numpy as np
import pytest

import synth.problems as SP

from helpers import CLASSES, oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu


def static_call(M, eng, ins):
    import torch
    arr, keep = eng._inputs(ins)
    e2 = torch.full((eng.plan.n_inst,), float("nan"), dtype=torch.float64, device=eng.device)
    parts = torch.full((eng.plan.n_inst, 12), float("nan"), dtype=torch.float64, device=eng.device)
    code = M.capi.lib().mrpt2_energy_static(eng.plan.handle, arr, eng.persistent.data_ptr(), eng._sptr(),
                                            e2.data_ptr(), parts.data_ptr())
    del keep
    return code, e2, parts


def test_static_workspace_energy_matches_energy_and_oracle():
    import torch
    import paper_2608_11529_amd as M
    size = ctypes.c_size_t()
    assert M.capi.lib().mrpt2_static_workspace_bytes(ctypes.byref(size)) == 0
    assert size.value == 64 << 20
    for name in ("s_j20", "c0"):          # the second problem needs less workspace
        pb = problem(name)
        parts_o, _, c_o, P_o = oracle_reference(name)
        plan = M.Plan(M.desc_of_problem(pb))
        assert plan.workspace_bytes <= size.value
        eng = M.Engine(plan)
        dev = eng.device
        c = to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c)
        ins = [(SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)],
                torch.from_numpy(np.ascontiguousarray(c)).to(dev))]
        print("[gpu] static workspace: %s (workspace %d bytes)" % (name, plan.workspace_bytes), flush=True)
        code, e2s, parts_s = static_call(M, eng, ins)
        assert code == 0, M.capi.lib().mrpt2_status_string(code)
        e2r, parts_r = eng.energy(ins)
        assert torch.equal(e2s, e2r), (name, float(e2s[0]), float(e2r[0]))
        assert torch.equal(parts_s, parts_r), name
        got = parts_s[0].cpu().numpy()
        for k, cl in enumerate(CLASSES):
            assert abs(got[k] - parts_o.get(cl, 0.0)) <= 1e-9, (name, cl, got[k], parts_o.get(cl))
        # a repeated call on the shared array gives the same result
        code, e2b, _ = static_call(M, eng, ins)
        assert code == 0 and torch.equal(e2b, e2s), name


def test_static_workspace_refuses_large_plans():
    import torch
    import paper_2608_11529_amd as M
    plan = M.Plan(M.desc_of_problem(problem("c1")))
    assert plan.workspace_bytes > 64 << 20
    pers = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    arr = (M.capi.Inputs * 1)()
    code = M.capi.lib().mrpt2_energy_static(plan.handle, arr, pers.data_ptr(), None, out.data_ptr(), None)
    assert code == 4      # MRPT2_ERR_WORKSPACE, before any device work
