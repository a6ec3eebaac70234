"""GPU adjoint (mrpt2_energy_backward) against the oracle gradient
(oracle.gradient, itself pinned to finite differences of the per-class
oracle), element by element, on the small problems and config c0; the torch
autograd Function; and central finite differences of the GPU forward energy
along random directions at config c1."""
import numpy as np
import pytest

import synth.problems as SP
from oracle import gradient, run

from helpers import SMALL, oracle_reference, problem, to_plan_order

pytestmark = pytest.mark.gpu

REL = 1e-9


def gpu_inputs(name, precision=0):
    import torch
    import paper_2608_11529_amd as M
    pb = problem(name)
    _, _, c_o, P_o = oracle_reference(name)
    plan = M.Plan(M.desc_of_problem(pb, precision=precision))
    eng = M.Engine(plan)
    c = to_plan_order(c_o, P_o, plan.ref_strings(), pb.n_c)
    dev = eng.device
    h = SP.one_body(pb).to(dev)
    Bs = [B.to(dev) for B in SP.factors(pb)]
    cd = torch.from_numpy(np.ascontiguousarray(c)).to(dev)
    return pb, plan, eng, h, Bs, cd, c_o, P_o


def close(a, b, rel=REL):
    scale = max(float(np.abs(b).max()), 1e-300)
    err = float(np.abs(a - b).max())
    return err <= rel * scale + 1e-14, err, scale


@pytest.mark.parametrize("name", list(SMALL) + ["c0"])
def test_gradient_matches_oracle(name):
    pb, plan, eng, h, Bs, c, c_o, P_o = gpu_inputs(name)
    print(f"[gpu] backward {name} N_P={plan.info().n_ref} N_Q={plan.info().n_ext}", flush=True)
    (dh, dBs, dc), = eng.backward([(h, Bs, c)])[0]
    e2_bwd = float(eng.e2[0].item())
    e2_fwd = float(eng.energy([(h, Bs, c)], parts=False)[0].item())
    assert abs(e2_bwd - e2_fwd) <= 1e-13 * max(1.0, abs(e2_fwd))
    E2, _, dh_o, dB_o, dc_o, _ = gradient.energy_and_gradient(
        run.space_of(pb), SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)],
        SP.weights(pb), pb.n_fc, c_o)
    assert abs(E2 - e2_fwd) <= 1e-9
    ok, err, sc = close(dh.cpu().numpy(), dh_o)
    assert ok, (name, "dh", err, sc)
    for t, (g, go) in enumerate(zip(dBs, dB_o)):
        ok, err, sc = close(g.cpu().numpy(), go)
        assert ok, (name, "dB", t, err, sc)
    dc_plan = to_plan_order(dc_o, P_o, plan.ref_strings(), pb.n_c)
    ok, err, sc = close(dc.cpu().numpy(), dc_plan)
    assert ok, (name, "dc", err, sc)


def test_upstream_gradient_scales_and_autograd_function():
    import torch
    import paper_2608_11529_amd as M
    pb, plan, eng, h, Bs, c, _, _ = gpu_inputs("s_fc")
    (dh1, dB1, dc1), = eng.backward([(h, Bs, c)])[0]
    dh1, dB1, dc1 = dh1.clone(), [x.clone() for x in dB1], dc1.clone()
    g = torch.tensor([-2.5], dtype=torch.float64, device=eng.device)
    (dh2, dB2, dc2), = eng.backward([(h, Bs, c)], g)[0]
    assert torch.allclose(dh2, -2.5 * dh1, rtol=1e-12, atol=0)
    assert torch.allclose(dc2, -2.5 * dc1, rtol=1e-12, atol=0)
    hh = h.clone().requires_grad_(True)
    BB = [B.clone().requires_grad_(True) for B in Bs]
    cc = c.clone().requires_grad_(True)
    e2 = M.energy(eng, hh, BB, cc)
    (3.0 * e2).backward()
    assert torch.allclose(hh.grad, 3.0 * dh1, rtol=1e-11, atol=1e-15)
    assert torch.allclose(cc.grad, 3.0 * dc1, rtol=1e-11, atol=1e-15)
    for x, y in zip(BB, dB1):
        assert torch.allclose(x.grad, 3.0 * y, rtol=1e-11, atol=1e-15)


def test_batched_backward_matches_single():
    import torch
    import paper_2608_11529_amd as M
    names = ["s_fc", "s_tiles", "c0"]
    descs = [M.desc_of_problem(problem(nm)) for nm in names]
    plan = M.Plan(descs)
    eng = M.Engine(plan)
    ins = []
    for i, nm in enumerate(names):
        pb = problem(nm)
        _, _, c_o, P_o = oracle_reference(nm)
        c = to_plan_order(c_o, P_o, plan.ref_strings(i), pb.n_c)
        ins.append((SP.one_body(pb).to(eng.device), [B.to(eng.device) for B in SP.factors(pb)],
                    torch.from_numpy(np.ascontiguousarray(c)).to(eng.device)))
    print("[gpu] batched backward", flush=True)
    outs, _ = eng.backward(ins)
    outs = [(a.clone(), [x.clone() for x in b], c.clone()) for a, b, c in outs]
    for i, nm in enumerate(names):
        e1 = M.Engine(M.Plan(descs[i]))
        (dh, dB, dc), = e1.backward([ins[i]])[0]
        assert close(outs[i][0].cpu().numpy(), dh.cpu().numpy(), 1e-12)[0], nm
        assert close(outs[i][2].cpu().numpy(), dc.cpu().numpy(), 1e-12)[0], nm
        for x, y in zip(outs[i][1], dB):
            assert close(x.cpu().numpy(), y.cpu().numpy(), 1e-12)[0], nm


def herm(gen, shape, dev):
    import torch
    z = torch.randn(shape, dtype=torch.complex128, generator=gen).to(dev)
    return 0.5 * (z + z.conj().transpose(-1, -2))


def test_finite_differences_c1():
    """20 random directions in (h, B, c) jointly; central differences at two
    steps with Richardson extrapolation against Re <G, direction>."""
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd.reference import ground_state
    pb = problem("c1")
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine(plan)
    dev = eng.device
    h = SP.one_body(pb, dev)
    Bs = SP.factors(pb, dev)
    c, _ = ground_state(eng, h, Bs)
    print("[gpu] c1 backward", flush=True)
    (dh, dBs, dc), = eng.backward([(h, Bs, c)])[0]
    dh, dBs, dc = dh.clone(), [x.clone() for x in dBs], dc.clone()
    gen = torch.Generator().manual_seed(11)

    def E(x):
        hh, BB, cc = x
        return float(eng.energy([(hh, BB, cc)], parts=False)[0].item())

    for k in range(20):
        Dh = herm(gen, h.shape, dev)
        DB = [herm(gen, B.shape, dev) * 0.05 for B in Bs]
        Dc = torch.randn(c.shape, dtype=torch.complex128, generator=gen).to(dev)
        nrm = (Dh.norm() ** 2 + sum(x.norm() ** 2 for x in DB) + Dc.norm() ** 2).sqrt()
        Dh, DB, Dc = Dh / nrm, [x / nrm for x in DB], Dc / nrm
        ana = float((torch.vdot(dh.flatten(), Dh.flatten()).real
                     + sum(torch.vdot(g.flatten(), d.flatten()).real for g, d in zip(dBs, DB))
                     + torch.vdot(dc, Dc).real).item())

        def shifted(s):
            return (h + s * Dh, [B + s * d for B, d in zip(Bs, DB)], c + s * Dc)

        v = []
        for st in (1e-4, 5e-5):
            v.append((E(shifted(st)) - E(shifted(-st))) / (2 * st))
        num = (4 * v[1] - v[0]) / 3
        print(f"[gpu] c1 direction {k}: analytic {ana:.12e} fd {num:.12e}", flush=True)
        assert abs(num - ana) <= 1e-6 * max(abs(ana), 1e-3), (k, num, ana)


@pytest.mark.parametrize("name", ["s_tiles", "c0"])
def test_mixed_precision_gradient_close_to_fp64(name):
    """The mixed form recomputes its FP32-MFMA pair integrals in the adjoint's
    forward pass; its gradient stays within 1e-6 (relative to the largest
    entry) of the FP64 one."""
    pb, plan, eng, h, Bs, c, _, _ = gpu_inputs(name, precision=0)
    (dh, dB, dc), = eng.backward([(h, Bs, c)])[0]
    dh, dB, dc = dh.cpu().numpy(), [x.cpu().numpy() for x in dB], dc.cpu().numpy()
    _, _, eng32, _, _, _, _, _ = gpu_inputs(name, precision=1)
    (mh, mB, mc), = eng32.backward([(h, Bs, c)])[0]
    assert close(mh.cpu().numpy(), dh, 1e-6)[0]
    assert close(mc.cpu().numpy(), dc, 1e-6)[0]
    for x, y in zip(mB, dB):
        assert close(x.cpu().numpy(), y, 1e-6)[0]
