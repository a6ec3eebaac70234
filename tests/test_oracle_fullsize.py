"""Pins of the full-size oracle driver (oracle.fullsize) to the class
oracle, itself pinned to Jordan-Wigner brute force and the closed forms
(test_oracle_pins): streamed frozen-core fold, pair energies and factor
columns give the same per-class E2 as the class oracle on the whole factor
array; the C loops of the two-virtual classes give the class oracle's sums,
also under every restriction (core holes, virtual ranges, strings) and with
the level shift of Sec. 2.6."""
import numpy as np
import pytest

import synth.problems as SP
from oracle import fullsize, run

from helpers import CLASSES, oracle_reference, problem

VV = [(2, 2), (1, 2), (0, 2)]


def slab_oracle(pb, chunk=3):
    hfc, slabs, W = fullsize.streamed_inputs(pb, chunk=chunk)
    return fullsize.SlabOracle(run.space_of(pb), hfc, slabs, SP.weights(pb), W)


@pytest.mark.parametrize("name", ["s_fc", "s_das", "s_hop0", "c0"])
def test_slab_oracle_equals_class_oracle(name):
    pb = problem(name)
    parts, E0, c, _ = oracle_reference(name)
    so = slab_oracle(pb)
    p2, e2 = so.e2(c, 0)
    assert abs(e2 - E0) <= 1e-12 * max(1.0, abs(E0))
    for cl in CLASSES:
        assert abs(p2[cl] - parts[cl]) <= 1e-14 + 1e-12 * abs(parts[cl]), (name, cl, p2[cl], parts[cl])


@pytest.mark.parametrize("name", ["s_fc", "s_das", "s_tiles", "s_nocore", "c0"])
def test_vv_classes_equal_class_oracle(name):
    pb = problem(name)
    parts, E0, c, _ = oracle_reference(name)
    so = slab_oracle(pb)
    for cl in VV:
        got = fullsize.vv_class(so, cl, c, E0)
        assert abs(got - parts[cl]) <= 1e-15 + 1e-12 * abs(parts[cl]), (name, cl, got, parts[cl])


def test_vv_restrictions_and_level_shift():
    name = "s_tiles"
    pb = problem(name)
    _, E0, c, _ = oracle_reference(name)
    h, Bs = SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)]
    co = run.class_oracle(pb, h, Bs, SP.weights(pb))
    so = slab_oracle(pb, chunk=7)
    strs = so.sp.class_strings(1, 2, 0)[::2]
    # hole tuples per class: (2,2) pairs, (1,2) single cores, (0,2) the empty tuple
    holes = {(2, 2): [[(0, 2)], [(0, 1), (1, 2)]], (1, 2): [[(1,)], [(0,), (2,)]], (0, 2): [[()], [()]]}
    for cl in VV:
        cases = [
            dict(core_sets=holes[cl][0]),
            dict(core_sets=holes[cl][1], va=(3, 40), vb=(20, 70)),
            dict(va=(64, 70)),
            dict(strings=strs),
            dict(b=0.7),
            dict(core_sets=holes[cl][1], va=(0, 64), vb=(64, 70), b=2.0),
        ]
        for kw in cases:
            ref, _ = co.e2(c, 0, E0=E0, classes=[cl], **kw)
            got = fullsize.vv_class(so, cl, c, E0, **kw)
            assert abs(got - ref[cl]) <= 1e-15 + 1e-12 * abs(ref[cl]), (kw, cl, got, ref[cl])
    # q_mode = 1 leaves the two-virtual classes unchanged
    for cl in VV:
        assert fullsize.vv_class(so, cl, c, E0, q_mode=1) == fullsize.vv_class(so, cl, c, E0)


def test_streamed_inputs_chunking_invariant():
    pb = problem("s_fc")
    a = fullsize.streamed_inputs(pb, chunk=1)
    b = fullsize.streamed_inputs(pb, chunk=100)
    assert np.allclose(a[0], b[0], rtol=0, atol=1e-13)
    assert np.allclose(a[2], b[2], rtol=0, atol=1e-13)
    for x, y in zip(a[1], b[1]):
        assert np.array_equal(x, y)


def test_sub_oracle_restricted_sums():
    """A restricted sum on the sub-problem of the occupied spinors and the
    restriction's virtual spinors equals the same restricted sum on the whole
    space (every term of those determinants involves no other virtual)."""
    name = "s_tiles"
    pb = problem(name)
    _, E0, c, _ = oracle_reference(name)
    so = slab_oracle(pb)
    for cl, hole, ar, br in [((2, 2), (0, 2), (64, 70), (64, 70)), ((1, 2), (1,), (16, 32), (64, 70)),
                             ((0, 2), (), (5, 6), (0, 64)), ((0, 2), (), (66, 67), (64, 70)),
                             ((2, 2), (0, 1), (0, 64), (64, 70))]:
        vs = sorted(set(range(*ar)) | set(range(*br)))
        sub = fullsize.sub_oracle(so, vs)
        pos = {v: i for i, v in enumerate(vs)}
        got = fullsize.vv_class(sub, cl, c, E0, core_sets=[hole], va=(pos[ar[0]], pos[ar[1] - 1] + 1),
                                vb=(pos[br[0]], pos[br[1] - 1] + 1))
        want = fullsize.vv_class(so, cl, c, E0, core_sets=[hole], va=ar, vb=br)
        assert want != 0.0
        assert abs(got - want) <= 1e-15 + 1e-12 * abs(want), (cl, hole, ar, br, got, want)
