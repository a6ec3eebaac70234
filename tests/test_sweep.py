"""Frozen-core / frozen-virtual sweep descriptors (host only): each grid
point freezes core spinors from the bottom and virtual spinors from the top,
keeps the reference space, and its external space shrinks."""
import pytest

from helpers import problem


def lib():
    import paper_2608_11529_amd as M
    return M


def test_point_descriptors_and_counts():
    M = lib()
    from paper_2608_11529_amd.sweep import point_desc
    pb = problem("s_tiles")
    d = M.desc_of_problem(pb)
    pts = {(k, m): point_desc(d, k, m) for k in (0, 1, 2) for m in (0, 10, 40)}
    for (k, m), p in pts.items():
        assert p.n_frozen_core == d.n_frozen_core + k
        assert p.n_core == d.n_core - k
        assert p.n_virt == d.n_virt - m
    plan = M.Plan(list(pts.values()))
    keys = list(pts)
    info = {key: plan.info(i) for i, key in enumerate(keys)}
    assert len({info[key].n_ref for key in keys}) == 1
    ref = list(plan.ref_strings(0))
    assert all(list(plan.ref_strings(i)) == ref for i in range(len(keys)))
    for k in (0, 1, 2):
        assert info[(k, 0)].n_ext > info[(k, 10)].n_ext > info[(k, 40)].n_ext
    for m in (0, 10, 40):
        assert info[(0, m)].n_ext > info[(1, m)].n_ext > info[(2, m)].n_ext
    assert info[(0, 0)].n_ext == M.Plan(d).info().n_ext


def test_point_descriptor_limits():
    M = lib()
    from paper_2608_11529_amd.sweep import point_desc
    d = M.desc_of_problem(problem("s_tiles"))
    with pytest.raises(ValueError):
        point_desc(d, d.n_core + 1, 0)
    with pytest.raises(ValueError):
        point_desc(d, 0, d.n_virt + 1)
