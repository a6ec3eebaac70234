"""Batched form: several independent instances of uneven size in one call
(one launch per stage covering all of them), against one-instance calls and
the oracle; and the asynchronous call captured in a HIP graph and replayed."""
import numpy as np
import pytest

import synth.problems as SP

from helpers import e2_total, oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu

NAMES = ["s_cas", "s_das", "s_fc", "s_tiles", "s_single", "s_nocore", "c0"]


def inputs_for(M, plan, names, dev):
    import torch
    out = []
    for i, nm in enumerate(names):
        pb = problem(nm)
        parts_o, E0_o, c_o, P_o = oracle_reference(nm)
        c = to_plan_order(c_o, P_o, plan.ref_strings(i), pb.n_c)
        out.append((SP.one_body(pb).to(dev), [B.to(dev) for B in SP.factors(pb)],
                    torch.from_numpy(np.ascontiguousarray(c)).to(dev)))
    return out


def test_batched_matches_single_and_oracle():
    import torch
    import paper_2608_11529_amd as M
    descs = [M.desc_of_problem(problem(nm)) for nm in NAMES]
    plan = M.Plan(descs)
    eng = M.Engine(plan)
    ins = inputs_for(M, plan, NAMES, eng.device)
    print("[gpu] batched %d instances" % len(NAMES), flush=True)
    e2, parts = eng.energy(ins)
    e2 = e2.cpu().numpy().copy()
    parts = parts.cpu().numpy().copy()
    for i, nm in enumerate(NAMES):
        p1 = M.Plan(descs[i])
        e1 = M.Engine(p1)
        r1, q1 = e1.energy([ins[i]])
        assert float(r1[0]) == e2[i], (nm, float(r1[0]), e2[i])
        assert np.array_equal(q1[0].cpu().numpy(), parts[i])
        ref = e2_total(oracle_reference(nm)[0])
        assert abs(e2[i] - ref) <= 1e-9, (nm, e2[i], ref)


def test_graph_capture_and_replay():
    import torch
    import paper_2608_11529_amd as M
    names = ["s_fc", "s_tiles", "c0"]
    plan = M.Plan([M.desc_of_problem(problem(nm)) for nm in names])
    eng = M.Engine(plan)
    ins = inputs_for(M, plan, names, eng.device)
    eager = eng.energy(ins)[1].clone()
    # a second engine provides unrelated eager work between replays
    other = M.Engine(M.Plan([M.desc_of_problem(problem("s_das"))]))
    ins2 = inputs_for(M, other.plan, ["s_das"], other.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        eng.energy_async(ins, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    eng.parts.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        eng.energy_async(ins, stream=torch.cuda.current_stream())
    for rep in range(3):
        eng.parts.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eng.check()
        assert torch.equal(eng.parts, eager), rep
        other.energy(ins2)
        torch.cuda.synchronize()


def test_graph_capture_of_forward_and_adjoint():
    """One HIP graph holding the batched adjoint (with its forward
    recomputation) of three instances, replayed three times with unrelated
    eager work in between: E2 and every gradient match an eager call (the
    adjoint sums some partials with atomics, hence a relative bound)."""
    import torch
    import paper_2608_11529_amd as M
    names = ["s_fc", "s_tiles", "c0"]
    plan = M.Plan([M.desc_of_problem(problem(nm)) for nm in names])
    eng = M.Engine(plan)
    ins = inputs_for(M, plan, names, eng.device)
    outs0, e20 = eng.backward(ins)
    ref = [(dh.clone(), [x.clone() for x in dB], dc.clone()) for dh, dB, dc in outs0]
    ref_e2 = e20.clone()
    other = M.Engine(M.Plan([M.desc_of_problem(problem("s_das"))]))
    ins2 = inputs_for(M, other.plan, ["s_das"], other.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        eng.backward(ins, asynchronous=True, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eng.check()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs, e2 = eng.backward(ins, asynchronous=True, stream=torch.cuda.current_stream())
    print("[gpu] captured batched adjoint", flush=True)

    def close(a, b, rel=1e-11):
        return float((a - b).abs().max()) <= rel * float(b.abs().max()) + 1e-15

    for rep in range(3):
        for dh, dB, dc in outs:
            dh.zero_()
            dc.zero_()
            for x in dB:
                x.zero_()
        e2.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eng.check()
        assert close(e2, ref_e2, 1e-13), rep
        for i, ((dh, dB, dc), (rh, rB, rc)) in enumerate(zip(outs, ref)):
            assert close(dh, rh), (rep, i, "dh")
            assert close(dc, rc), (rep, i, "dc")
            for t, (x, rx) in enumerate(zip(dB, rB)):
                assert close(x, rx), (rep, i, "dB", t)
        other.energy(ins2)
        torch.cuda.synchronize()


def test_asynchronous_call_then_synchronous_call_on_one_plan():
    """An asynchronous evaluation followed at once by a synchronous one on
    the same plan, workspace and stream, with different reference vectors and
    output buffers: each returns its own energy (the second call must not
    rewrite the descriptors the first call's queued copy still reads)."""
    import torch
    import paper_2608_11529_amd as M
    name = "s_tiles"
    pb = problem(name)
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    dev = eng.device
    (h, Bs, c), = inputs_for(M, plan, [name], dev)
    c2 = c.clone()
    c2[0] += 0.3
    ref1 = float(eng.energy([(h, Bs, c)], parts=False)[0].item())
    ref2 = float(eng.energy([(h, Bs, c2)], parts=False)[0].item())
    assert ref1 != ref2
    L = M.capi.lib()
    out1 = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    out2 = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    for _ in range(3):
        a1, k1 = eng._inputs([(h, Bs, c)])
        a2, k2 = eng._inputs([(h, Bs, c2)])
        # a long queue ahead of the first call keeps its descriptor copy pending
        big = torch.randn(4096, 4096, dtype=torch.float64, device=dev)
        for _ in range(4):
            big = big @ big * 1e-3
        assert L.mrpt2_energy_async(plan.handle, a1, eng.persistent.data_ptr(), eng.workspace.data_ptr(),
                                    plan.workspace_bytes, eng._sptr(), out1.data_ptr(), None) == 0
        assert L.mrpt2_energy(plan.handle, a2, eng.persistent.data_ptr(), eng.workspace.data_ptr(),
                              plan.workspace_bytes, eng._sptr(), out2.data_ptr(), None) == 0
        torch.cuda.synchronize()
        assert float(out1[0]) == ref1 and float(out2[0]) == ref2
        del k1, k2
