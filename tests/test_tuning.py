"""Launch-shape tuning (mrpt2_plan_tuned) on the host: the targets reach the
work decomposition, bad values are rejected, and the autotuner's table maps
onto the classes of an instance by size bucket."""
import pytest

import paper_2608_11529_amd as M
from paper_2608_11529_amd import autotune, capi

from helpers import CLASSES, problem


def uniform(**kv):
    t = capi.Tuning()
    for knob, v in kv.items():
        for k in range(capi.N_CLASS):
            getattr(t, knob)[k] = v
    return t


def generic_classes(plan):
    """Classes of the generic sigma kernel: partial blocks = row blocks x string chunks."""
    kc = plan.info().kernel_class
    return [k for k, (h, v) in enumerate(CLASSES) if kc[k] == 0 and plan.class_blocks(k) > 0]


def test_sigma_target_sets_string_chunks():
    desc = M.desc_of_problem(problem("s_das"))
    base = M.Plan(desc)
    one = M.Plan(desc, tuning=uniform(sigma_blocks=1))
    big = M.Plan(desc, tuning=uniform(sigma_blocks=1 << 20))
    ks = generic_classes(base)
    assert ks
    for k in ks:
        info = base.info()
        S = info.n_strings_class[k]
        nb1, nbd, nbb = one.class_blocks(k), base.class_blocks(k), big.class_blocks(k)
        # one chunk per row block at the smallest target, every string its own
        # chunk at the largest
        assert nb1 <= nbd <= nbb
        assert nbb % S == 0 and nb1 == nbb // S


def test_backward_targets_change_partial_buffers():
    desc = M.desc_of_problem(problem("c0"))
    g = [M.Plan(desc, tuning=uniform(bwd_blocks=v, bwd_row_blocks=v)).grad_bytes for v in (1, 2048, 1 << 20)]
    assert g[0] <= g[1] <= g[2] and g[0] < g[2]
    assert M.Plan(desc).grad_bytes == g[1]


def test_zero_targets_equal_builtin_rules():
    desc = M.desc_of_problem(problem("s_fc"))
    a, b = M.Plan(desc), M.Plan(desc, tuning=capi.Tuning())
    assert (a.workspace_bytes, a.grad_bytes) == (b.workspace_bytes, b.grad_bytes)
    for k in range(capi.N_CLASS):
        assert a.class_blocks(k) == b.class_blocks(k)


def test_negative_target_rejected():
    desc = M.desc_of_problem(problem("s_fc"))
    t = capi.Tuning()
    t.bwd_row_blocks[3] = -1
    with pytest.raises(capi.Mrpt2Error) as e:
        M.Plan(desc, tuning=t)
    assert e.value.code == 1
    with pytest.raises(ValueError):
        M.Plan([desc, desc], tuning=[capi.Tuning()])
    t = capi.Tuning()
    t.pair_tile = 32                                 # only 0, 64 and 128 are block edges
    with pytest.raises(capi.Mrpt2Error) as e:
        M.Plan(desc, tuning=t)
    assert e.value.code == 1


def test_pair_tile_bucket_lookup():
    descs = [M.desc_of_problem(problem(n)) for n in ("s_tiles", "c0")]
    plan = M.Plan(descs)
    b = autotune.pair_bucket(descs[0], plan.info(0))
    assert b == "pair/vt2/l%d" % (int(plan.info(0).n_chol).bit_length() - 1)
    tu = autotune.tuning_for(descs, {b: {"pair_tile": 128}})
    assert tu[0].pair_tile == 128
    if autotune.pair_bucket(descs[1], plan.info(1)) != b:
        assert tu[1].pair_tile == 0
    M.Plan(descs, tuning=tu)


def test_table_lookup_by_bucket():
    descs = [M.desc_of_problem(problem(n)) for n in ("s_das", "c0")]
    plan = M.Plan(descs)
    info = plan.info(1)
    k = 4                                            # class (1,1)
    b = autotune.bucket(info, k)
    assert b.startswith("11/q")
    h, v = CLASSES[k]
    assert b == "%d%d/q%d/s%d" % (h, v, int(info.n_ext_class[k]).bit_length() - 1,
                                  int(info.n_strings_class[k]).bit_length() - 1)
    table = {b: {"sigma_blocks": 1234, "bwd_row_blocks": 99}}
    tu = autotune.tuning_for(descs, table)
    assert tu[1].sigma_blocks[k] == 1234 and tu[1].bwd_row_blocks[k] == 99 and tu[1].bwd_blocks[k] == 0
    for kk in range(capi.N_CLASS):
        if kk != k:
            assert tu[1].sigma_blocks[kk] == 0
    # the other instance's class (1,1) falls in another bucket
    if autotune.bucket(plan.info(0), k) != b:
        assert tu[0].sigma_blocks[k] == 0
    M.Plan(descs, tuning=tu)                         # a tuned batched plan builds
