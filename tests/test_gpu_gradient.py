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


def close(a, b, rel=REL, floor=1e-3):
    """Element by element: |a - b| <= rel |b| + floor rel max|b| + 1e-14 at
    every entry (the last term for entries that vanish in exact arithmetic).  Against the oracle floor = 1e-3, so that small entries (the
    factor gradients of the weak Gaunt and gauge sets, the couplings of the
    wide classes) are checked on their own scale and not only against the
    largest entry; between two GPU results (batched and single, mixed and
    FP64) floor = 1."""
    scale = max(float(np.abs(b).max()), 1e-300)
    d = np.abs(a - b)
    err = float(d.max())
    worst = float((d / (rel * np.abs(b) + floor * rel * scale + 1e-14)).max())
    return worst <= 1.0, err, scale


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
        assert close(outs[i][0].cpu().numpy(), dh.cpu().numpy(), 1e-12, 1.0)[0], nm
        assert close(outs[i][2].cpu().numpy(), dc.cpu().numpy(), 1e-12, 1.0)[0], nm
        for x, y in zip(outs[i][1], dB):
            assert close(x.cpu().numpy(), y.cpu().numpy(), 1e-12, 1.0)[0], nm


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
    assert close(mh.cpu().numpy(), dh, 1e-6, 1.0)[0]
    assert close(mc.cpu().numpy(), dc, 1e-6, 1.0)[0]
    for x, y in zip(mB, dB):
        assert close(x.cpu().numpy(), y, 1e-6, 1.0)[0]


def _rdot(a, b):
    import torch
    return float(torch.vdot(a.flatten(), b.flatten()).real.item())


def _nrm2(xs):
    return sum(float(x.norm().item()) ** 2 for x in xs)


def _aligned(gs, rs):
    """Unit direction (G/|G| + R/|R|) / norm over the components gs (gradient)
    and rs (random, same shapes).  Along a random direction alone the
    derivative of a sum over ~1e12 determinants is ~1e-3 of E2 and the
    rounding of E2 itself (~1e-12 relative) swamps a 1e-6 check; the gradient
    part makes the derivative of order |G| while the random part keeps every
    component of G under test."""
    import torch
    ng, nr = _nrm2(gs) ** 0.5, _nrm2(rs) ** 0.5
    d = [torch.add(g, r, alpha=ng / nr) for g, r in zip(gs, rs)]   # ng (G/|G| + R/|R|), one new tensor each
    nd = _nrm2(d) ** 0.5
    for x in d:
        x.div_(nd)
    return d


def _adaptive(E, h0=1e-3, levels=12):
    """Central differences at h0, h0/2, ..., Richardson-extrapolated over
    consecutive pairs; returns the extrapolation where two consecutive ones
    agree best, and that disagreement.  Near-singular denominators make E2
    strongly curved along some directions, so no single step serves all."""
    cs, rs = [], []
    best, best_err = None, float("inf")
    h = h0
    for _ in range(levels):
        cs.append((E(h) - E(-h)) / (2 * h))
        if len(cs) >= 2:
            rs.append((4 * cs[-1] - cs[-2]) / 3)
        if len(rs) >= 2 and abs(rs[-1] - rs[-2]) < best_err:
            best, best_err = rs[-1], abs(rs[-1] - rs[-2])
        h /= 2
    return best, best_err


def _entry_directions(G, k):
    """The k entries of largest magnitude of a gradient tensor G (flat
    indices, off-diagonal entries of a Hermitian component counted once)."""
    import torch
    a = G.abs().flatten()
    return torch.topk(a, k).indices.tolist()


def _coord_check(E, target, idx, g, hermitian, label, h0=1e-3, levels=4, units=(1.0, 1j)):
    """Central differences of E along one coordinate of tensor `target`
    (flat index idx; a Hermitian matrix moves its (p,q) and (q,p) entries
    together), for the real and the imaginary direction, against the
    gradient entry g = G[idx]: dE along the real unit is Re g (twice that for
    an off-diagonal Hermitian pair), along the imaginary unit Im g."""
    import torch
    flat = target.view(-1)
    n = target.shape[-1]
    save = flat[idx].item()
    partner = None
    if hermitian:
        q, p = idx % n, (idx // n) % n
        if p != q:
            partner = idx - (p * n + q) + (q * n + p)
    psave = flat[partner].item() if partner is not None else None
    out = []
    for unit in units:
        if hermitian and partner is None and unit == 1j:
            continue                                   # a diagonal entry of a Hermitian matrix is real

        def shifted(s, unit=unit):
            flat[idx] = save + s * unit
            if partner is not None:
                flat[partner] = psave + s * complex(unit).conjugate()
            try:
                return E()
            finally:
                flat[idx] = save
                if partner is not None:
                    flat[partner] = psave

        num, err = _adaptive(shifted, h0=h0, levels=levels)
        mult = 2.0 if partner is not None else 1.0
        ana = mult * (g.real if unit == 1.0 else g.imag)
        print(f"[gpu] {label} entry {idx} {'re' if unit == 1.0 else 'im'}: analytic {ana:.12e} fd {num:.12e} "
              f"(fd spread {err:.2e})", flush=True)
        out.append((num, ana, err))
    return out


def test_finite_differences_c2():
    """c2 (28 core, 16 active in four DAS subspaces, 600 virtual, three factor
    sets), FP64.  Element by element: the two largest entries of dE2/dh, of
    the gradient of each factor set and of dE2/dC, each by central
    differences along that coordinate alone (real and imaginary parts), within
    1e-6 of the entry's own size.  One direction mixing the normalised gradient
    with a random direction remains as a smoke check of the whole gradient;
    it sees an error e orthogonal to G only as |e|^2/|G| and is no
    element-wise test."""
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd.reference import ground_state
    pb = problem("c2")
    eng = M.Engine(M.Plan(M.desc_of_problem(pb)))
    dev = eng.device
    h, Bs = SP.one_body(pb, dev), SP.factors(pb, dev)
    c, _ = ground_state(eng, h, Bs)
    (gh, gB, gc), = eng.backward([(h, Bs, c)])[0]
    G = [gh] + list(gB) + [gc]

    def E():
        return float(eng.energy([(h, Bs, c)], parts=False)[0].item())

    print("[gpu] c2 finite differences", flush=True)
    comps = [("dh", h, gh, True, 2)] + [("dB%d" % t, B, g, True, 1) for t, (B, g) in enumerate(zip(Bs, gB))] + \
            [("dC", c, gc, False, 2)]
    for label, target, g, herm_, n_entries in comps:
        for idx in _entry_directions(g, n_entries):
            gv = complex(g.view(-1)[idx].item())
            for num, ana, err in _coord_check(E, target, idx, gv, herm_, "c2 " + label):
                assert abs(num - ana) <= 1e-6 * abs(gv) * (2.0 if herm_ else 1.0) + 1e-12, (label, idx, num, ana)
    gen = torch.Generator().manual_seed(12)
    R = [herm(gen, h.shape, dev)] + [herm(gen, B.shape, dev) for B in Bs] + \
        [torch.randn(c.shape, dtype=torch.complex128, generator=gen).to(dev)]
    D = _aligned(G, R)
    del R
    ana = sum(_rdot(x, d) for x, d in zip(G, D))
    nb = len(Bs)
    num, err = _adaptive(lambda s: float(eng.energy([(h + s * D[0], [B + s * d for B, d in zip(Bs, D[1:1 + nb])],
                                                        c + s * D[-1])], parts=False)[0].item()))
    print(f"[gpu] c2 aligned direction: analytic {ana:.12e} fd {num:.12e} (fd spread {err:.2e})", flush=True)
    assert abs(num - ana) <= 1e-6 * abs(ana), (num, ana)


def test_finite_differences_c4():
    """c4 at full size, FP64, element by element: the largest entries of
    dE2/dh and dE2/dC (real parts; the imaginary part too for C), of the
    gradient of the Gaunt set and of the first Dirac-Coulomb Cholesky vector,
    each by central differences along that coordinate alone, within 1e-6 of
    the entry's own size.  Only the gradient pieces these checks need are kept
    after the adjoint call (the Dirac-Coulomb gradient alone is 43 GB)."""
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd.reference import ground_state
    pb = problem("c4")
    eng = M.Engine(M.Plan(M.desc_of_problem(pb)))
    dev = eng.device
    h, Bs = SP.one_body(pb, dev), SP.factors(pb, dev)
    c, _ = ground_state(eng, h, Bs)
    print("[gpu] c4 inputs ready", flush=True)
    outs, _ = eng.backward([(h, Bs, c)])
    gh, gB, gc = outs[0]
    keep = [("dh", h, gh.clone(), (1.0,)), ("dC", c, gc.clone(), (1.0, 1j)), ("dB1", Bs[1], gB[1].clone(), (1.0,)),
            ("dB0[0]", Bs[0][0], gB[0][0].clone(), (1.0,))]
    del outs, gB, gh, gc
    eng.grad_workspace = None
    torch.cuda.empty_cache()
    print("[gpu] c4 adjoint done", flush=True)

    def E():
        return float(eng.energy([(h, Bs, c)], parts=False)[0].item())

    for label, target, g, units in keep:
        herm_ = label != "dC"
        idx = _entry_directions(g, 1)[0]
        gv = complex(g.view(-1)[idx].item())
        for num, ana, err in _coord_check(E, target, idx, gv, herm_, "c4 " + label, h0=5e-4, levels=3,
                                          units=units):
            assert abs(num - ana) <= 1e-6 * abs(gv) * (2.0 if herm_ else 1.0) + 1e-12, (label, idx, num, ana)


def test_finite_differences_batched_c3_instances():
    """Two instances of the batched workload in one plan: the batched adjoint
    against central differences of the batched energy of each instance."""
    import torch
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd.reference import ground_state
    pbs = [SP.batched_instance(s) for s in (7, 35)]
    dev = torch.device("cuda:0")
    ins = []
    for pb in pbs:
        h, Bs = SP.one_body(pb, dev), SP.factors(pb, dev)
        c, _ = ground_state(M.Engine(M.Plan(M.desc_of_problem(pb))), h, Bs)
        ins.append((h, Bs, c))
    eng = M.Engine(M.Plan([M.desc_of_problem(pb) for pb in pbs]))
    outs, _ = eng.backward(ins)
    outs = [(a.clone(), [x.clone() for x in b], z.clone()) for a, b, z in outs]
    gen = torch.Generator().manual_seed(14)
    for i, (h, Bs, c) in enumerate(ins):
        for k in range(3):
            g = outs[i]
            G = [g[0]] + list(g[1]) + [g[2]]
            R = [herm(gen, h.shape, dev)] + [herm(gen, B.shape, dev) for B in Bs] + \
                [torch.randn(c.shape, dtype=torch.complex128, generator=gen).to(dev)]
            D = _aligned(G, R)
            ana = sum(_rdot(x, d) for x, d in zip(G, D))

            def E(s, i=i, h=h, Bs=Bs, c=c, D=D):
                cur = list(ins)
                cur[i] = (h + s * D[0], [B + s * d for B, d in zip(Bs, D[1:-1])], c + s * D[-1])
                return float(eng.energy(cur, parts=False)[i].item())

            num, err = _adaptive(E)
            print(f"[gpu] c3 instance {i} direction {k}: analytic {ana:.12e} fd {num:.12e} (fd spread {err:.2e})",
                  flush=True)
            assert abs(num - ana) <= 1e-6 * abs(ana), (i, k, num, ana)


def test_mixed_precision_gradient_c1():
    """The mixed form at c1 (FP32-MFMA pair integrals with a per-stage FP64
    carry, FP64 elsewhere): its adjoint against the FP64 adjoint element by
    element (1e-5 of each entry plus 1e-8 of the largest), and against central
    differences of the mixed energy itself along the largest entries of dh
    and dC (1e-5 of the entry)."""
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd.reference import ground_state
    pb = problem("c1")
    e64 = M.Engine(M.Plan(M.desc_of_problem(pb, precision=0)))
    dev = e64.device
    h, Bs = SP.one_body(pb, dev), SP.factors(pb, dev)
    c, _ = ground_state(e64, h, Bs)
    (gh, gB, gc), = e64.backward([(h, Bs, c)])[0]
    gh, gB, gc = gh.cpu().numpy(), [x.cpu().numpy() for x in gB], gc.cpu().numpy()
    e32 = M.Engine(M.Plan(M.desc_of_problem(pb, precision=1)))
    print("[gpu] c1 mixed backward", flush=True)
    (mh, mB, mc), = e32.backward([(h, Bs, c)])[0]
    mh_d, mc_d = mh.clone(), mc.clone()
    assert close(mh.cpu().numpy(), gh, 1e-5, 1e-3)[0]
    assert close(mc.cpu().numpy(), gc, 1e-5, 1e-3)[0]
    for x, y in zip(mB, gB):
        assert close(x.cpu().numpy(), y, 1e-5, 1e-3)[0]

    def E():
        return float(e32.energy([(h, Bs, c)], parts=False)[0].item())

    for label, target, g, herm_ in (("dh", h, mh_d, True), ("dC", c, mc_d, False)):
        idx = _entry_directions(g, 1)[0]
        gv = complex(g.view(-1)[idx].item())
        for num, ana, err in _coord_check(E, target, idx, gv, herm_, "c1 mixed " + label, h0=1e-3, levels=4):
            assert abs(num - ana) <= 1e-5 * abs(gv) * (2.0 if herm_ else 1.0) + 1e-10, (label, idx, num, ana)
