"""Host-side checks of the C library (no GPU): it loads, exports every
symbol the header declares, and its plan (reference strings, external-space
counts per class, argument validation) agrees with the oracle's own
enumeration."""
import ctypes
import os
import re

import pytest

import synth.problems as SP
from oracle import counting, run

from helpers import CLASSES, SMALL, problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib_module():
    import paper_2608_11529_amd as M
    return M


def test_library_exports_header_symbols():
    M = lib_module()
    L = M.capi.lib()
    with open(os.path.join(ROOT, "include", "mrpt2.h")) as f:
        hdr = f.read()
    names = set(re.findall(r"^\s*(?:mrpt2_status|void|const char\*)\s+(mrpt2_\w+)\s*\(", hdr, re.M))
    assert names == set(M.capi.EXPORTED), names
    for nm in names:
        assert hasattr(L, nm), nm


@pytest.mark.parametrize("name", list(SMALL) + ["c0", "c1", "c2"])
def test_plan_matches_oracle_enumeration(name):
    M = lib_module()
    pb = problem(name)
    plan = M.Plan(M.desc_of_problem(pb))
    inf = plan.info()
    sp = run.space_of(pb)
    cnt = counting.external_count(sp, 0)
    for k, cl in enumerate(CLASSES):
        assert inf.n_ext_class[k] == cnt[cl], (cl, inf.n_ext_class[k], cnt[cl])
    assert inf.n_ext == sum(cnt.values())
    if len(sp.p_strings()) < 20000:
        bits = plan.ref_strings()
        assert sorted(int(b) << pb.n_c for b in bits) == sp.p_strings()
    for k, cl in enumerate(CLASSES):
        assert inf.n_strings_class[k] == len(sp.class_strings(*cl, 0)) or inf.n_ext_class[k] == 0


def test_plan_q_mode_1():
    M = lib_module()
    pb = problem("s_das")
    plan = M.Plan(M.desc_of_problem(pb, q_mode=1))
    cnt = counting.external_count(run.space_of(pb), 1)
    assert plan.info().n_ext == sum(cnt.values())
    assert plan.info().n_ext_class[8] == 0


def test_reference_order_is_category_blocked():
    """STP-DAS addressing (Sec. 2.4): reference strings are grouped by
    category, each category a tensor product of per-subspace strings."""
    M = lib_module()
    pb = SP.config("c1")
    bits = M.Plan(M.desc_of_problem(pb)).ref_strings()
    sp = run.space_of(pb)
    cats = [sp.category(int(b) << pb.n_c) for b in bits]
    seen = []
    for c in cats:
        if not seen or seen[-1] != c:
            assert c not in seen, "category appears in two blocks"
            seen.append(c)
    assert set(seen) == set(sp.p_categories())


def test_table3_counts_through_the_plan():
    """The plan's class rule reproduces the paper's printed nDets for Ne
    (Table 3): 4 core, CAS(6e,8o), 108 virtual spinors."""
    M = lib_module()
    d = M.make_desc(0, 4, 108, [8], [6], 6, 6, [(1, 1.0)])
    assert M.Plan(d).info().n_ext == 2692802


@pytest.mark.parametrize("field,value,code", [
    ("n_sub", 17, 1), ("n_sets", 0, 1), ("q_mode", 2, 1), ("precision", 7, 3),
    ("level_shift_b", float("nan"), 1), ("level_shift_b", float("inf"), 1), ("n_act_elec", 9, 2),
    ("layout", 2, 3),
])
def test_plan_rejects_bad_descriptors(field, value, code):
    M = lib_module()
    d = M.desc_of_problem(problem("s_cas"))
    setattr(d, field, value)
    with pytest.raises(M.Mrpt2Error) as ei:
        M.Plan(d)
    assert ei.value.code == code


def test_packed_layout_offsets_and_shapes():
    """The packed factor layout: the plan is the same as the full layout's,
    hermitian_pack puts entry (p, q), p <= q, at the offset the header states
    (p n - p (p - 1) / 2 + (q - p)), and the binding takes [rank, n (n + 1) / 2]
    tensors for a packed plan and refuses full ones."""
    import torch
    M = lib_module()
    pb = problem("s_fc")
    full = M.Plan(M.desc_of_problem(pb)).info()
    plan = M.Plan(M.desc_of_problem(pb, layout=1))
    info = plan.info()
    assert info.n_ext == full.n_ext and list(info.n_ext_class) == list(full.n_ext_class)
    n = info.n_orb
    z = SP.complex_normal(5, 77, (3, n, n))
    B = 0.5 * (z + z.transpose(-1, -2).conj())
    P = M.hermitian_pack(B)
    assert tuple(P.shape) == (3, n * (n + 1) // 2)
    for p in range(n):
        for q in range(p, n):
            assert torch.equal(P[:, p * n - p * (p - 1) // 2 + (q - p)], B[:, p, q])
    eng = M.Engine.__new__(M.Engine)
    eng.torch, eng.plan = torch, plan
    h = torch.zeros((n, n), dtype=torch.complex128)
    c = torch.zeros(info.n_ref, dtype=torch.complex128)
    packed = [torch.zeros((r, n * (n + 1) // 2), dtype=torch.complex128) for r, _ in pb.sets]
    eng._check_shapes(0, h, packed, c)
    with pytest.raises(ValueError, match="packed"):
        eng._check_shapes(0, h, [torch.zeros((r, n, n), dtype=torch.complex128) for r, _ in pb.sets], c)


def test_level_shift_keeps_the_external_space():
    """A nonzero level shift is accepted and changes neither the external
    space nor its counts (the shift acts on the denominators only)."""
    M = lib_module()
    d = M.desc_of_problem(problem("s_cas"))
    ref = M.Plan(d).info()
    d.level_shift_b = 0.05
    got = M.Plan(d).info()
    assert got.n_ext == ref.n_ext
    assert list(got.n_ext_class) == list(ref.n_ext_class)


def test_null_arguments_return_status():
    M = lib_module()
    L = M.capi.lib()
    assert L.mrpt2_plan(None, 1, ctypes.byref(ctypes.c_void_p())) == 1
    assert L.mrpt2_plan_sizes(None, None, None) == 1
    assert L.mrpt2_energy(None, None, None, None, 0, None, None, None) == 1
    assert L.mrpt2_status_string(6) == b"non-finite input or zero denominator"


def test_binding_refuses_inputs_of_the_wrong_shape():
    """The Python binding checks every tensor against the plan's sizes before
    a call (the C interface takes plain pointers and reads the plan's sizes)."""
    import torch
    M = lib_module()
    pb = problem("s_das")
    plan = M.Plan(M.desc_of_problem(pb))
    eng = M.Engine.__new__(M.Engine)        # shape checks need no device
    eng.torch, eng.plan = torch, plan
    info = plan.info()
    n, n_p = info.n_orb, info.n_ref
    h = torch.zeros((n, n), dtype=torch.complex128)
    Bs = [torch.zeros((r, n, n), dtype=torch.complex128) for r, _ in pb.sets]
    c = torch.zeros(n_p, dtype=torch.complex128)
    eng._check_shapes(0, h, Bs, c)
    eng._check_shapes(0, h, Bs, torch.zeros((3, n_p), dtype=torch.complex128))
    bad = [
        (torch.zeros((n, n + 1), dtype=torch.complex128), Bs, c),
        (h.to(torch.complex64), Bs, c),
        (h, Bs[:-1] if len(Bs) > 1 else [], c),
        (h, [torch.zeros((Bs[0].shape[0] + 1, n, n), dtype=torch.complex128)] + Bs[1:], c),
        (h, Bs, torch.zeros(n_p - 1, dtype=torch.complex128)),
        (h, Bs, torch.zeros((2, n_p + 1), dtype=torch.complex128)),
    ]
    for args in bad:
        with pytest.raises(ValueError):
            eng._check_shapes(0, *args)
    with pytest.raises(ValueError):
        eng._inputs([(h, Bs, c), (h, Bs, c)])


def test_wide_active_spaces_select_every_dense_kernel_width():
    """Class (1,2) runs the dense-coefficient kernel sized for its pattern
    count: the small problems with 20, 24 and 32 active spinors select the
    24- and 32-wide forms (forward) and the 20-, 24- and 32-wide adjoint
    forms, which the element-wise GPU parity tests then cover; c4 (18
    active spinors) runs the 24-wide form."""
    import paper_2608_11529_amd as M
    from helpers import problem
    want = {"s_j20": 20, "s_j24": 24, "s_j32": 32, "c4": 18, "c0": 6, "s_das": 6}
    for name, J in want.items():
        info = M.Plan(M.desc_of_problem(problem(name))).info()
        assert info.n_patterns_class[1] == J, (name, info.n_patterns_class[1])
        assert info.kernel_class[1] == 2, name
        assert info.kernel_class[0] == 1 and info.kernel_class[2] in (0, 3), name
        assert info.kernel_class[3] == (4 if info.n_patterns_class[3] <= 32 else 0), name
    assert M.Plan(M.desc_of_problem(problem("s_j20"))).info().n_strings_class[1] == 190


def test_reference_excitation_lists_count():
    """The plan's excitation lists of P hold exactly the ordered pairs of
    reference determinants one or two active replacements apart (bit strings
    differing in two or four positions), by brute force over P."""
    import numpy as np
    import paper_2608_11529_amd as M
    from helpers import problem
    for name in ("s_das", "s_fc", "s_hop0", "s_j24", "c0", "c1"):
        plan = M.Plan(M.desc_of_problem(problem(name)))
        b = [int(x) for x in plan.ref_strings()]
        n = 0
        for i in range(len(b)):
            for j in range(len(b)):
                if i != j and bin(b[i] ^ b[j]).count("1") in (2, 4):
                    n += 1
        assert plan.info().n_ref_couplings == n, (name, plan.info().n_ref_couplings, n)


def test_batched_adjoint_workspace_is_shared_over_instances():
    """One launch of the adjoint's generic row pass covers every instance of a
    plan, so a batch divides the pass's block target among its instances in
    proportion to their work instead of giving each the whole target: the
    64-instance batch's gradient workspace (private coupling-adjoint slices
    per string chunk among it) stays below 50 GB (124.6 GB when every
    instance split its strings for the whole device), and a one-instance
    plan is unchanged by the rule."""
    import paper_2608_11529_amd as M
    ds = [M.desc_of_problem(SP.batched_instance(s), precision=1, layout=1) for s in range(64)]
    plan = M.Plan(ds)
    assert plan.grad_bytes < 50e9, plan.grad_bytes
    one = M.Plan(ds[:1])
    assert one.grad_bytes <= plan.grad_bytes
    # the forward recomputation and adjoint of all 64 instances on one GPU
    # (288 GB): packed factors and their gradients, both workspaces
    fac = sum(16 * pb.n_l * pb.n * (pb.n + 1) // 2 for pb in map(SP.batched_instance, range(64)))
    total = 2 * fac + plan.workspace_bytes + plan.grad_bytes
    assert total < 240e9, total / 1e9
