"""Frozen-core / frozen-virtual sweep as one batched call.

The frozen-core and frozen-virtual approximations (Secs. 2.5 and 3.4) drop
spinors from the excitation space.  The paper maps the recovered correlation
energy over a grid of (frozen core, frozen virtual) counts; here every grid
point is one instance of a single plan, so the whole grid is evaluated by
one launch per stage.

  * Freezing k more core spinors moves the k lowest correlated core spinors
    into the frozen core.  The library folds the frozen core into h, so the
    inputs are unchanged; only the descriptor changes.
  * Freezing m virtual spinors drops the m highest.  The spinor order keeps
    the virtuals ascending in energy, so h and every B are cut to their first
    n - m spinors (contiguous device copies, one per distinct m).
  * Neither changes the reference space P or Psi0: every P determinant holds
    the whole core and no virtual, so one C serves every point.

    python -m paper_2608_11529_amd.sweep --config c2 --core 0,4,8,12 --virt 0,120,240
"""
import argparse
import ctypes
import json
import os
import sys
import time

from . import capi


def point_desc(desc, k, m):
    """Descriptor with k more frozen core and m fewer kept virtual spinors."""
    if k < 0 or m < 0 or k > desc.n_core or m > desc.n_virt:
        raise ValueError("cannot freeze %d core / %d virtual spinors of %d / %d"
                         % (k, m, desc.n_core, desc.n_virt))
    d = capi.Desc.from_buffer_copy(desc)
    d.n_frozen_core = desc.n_frozen_core + k
    d.n_core = desc.n_core - k
    d.n_virt = desc.n_virt - m
    return d


class FrozenSweep:
    """E2 over the grid core_counts x virt_counts (extra frozen core, frozen
    virtual spinors) of one problem, evaluated as one batched call."""

    def __init__(self, desc, core_counts, virt_counts, tuning=None, device="cuda:0"):
        from . import Engine, Plan
        self.core_counts = [int(k) for k in core_counts]
        self.virt_counts = [int(m) for m in virt_counts]
        self.n = desc.n_frozen_core + desc.n_core + sum(desc.sub_size[:desc.n_sub]) + desc.n_virt
        self.descs = [point_desc(desc, k, m) for k in self.core_counts for m in self.virt_counts]
        if tuning is not None and not isinstance(tuning, list):
            tuning = tuning(self.descs)
        self.plan = Plan(self.descs, tuning=tuning)
        ref = self.plan.ref_strings(0)
        for i in range(1, len(self.descs)):
            if list(self.plan.ref_strings(i)) != list(ref):
                raise RuntimeError("sweep point %d has a different reference space" % i)
        self.engine = Engine(self.plan, device)

    def inputs(self, h, Bs, c):
        """Instance inputs of every grid point (row-major over core x virt)."""
        cut = {}
        for m in self.virt_counts:
            if m not in cut:
                k = self.n - m
                cut[m] = (h, Bs) if m == 0 else (h[:k, :k].contiguous(), [B[:, :k, :k].contiguous() for B in Bs])
        return [(cut[m][0], cut[m][1], c) for _ in self.core_counts for m in self.virt_counts]

    def energy(self, h, Bs, c, insts=None):
        """E2 grid [len(core_counts)][len(virt_counts)] (device tensor) and
        the per-instance class parts."""
        insts = self.inputs(h, Bs, c) if insts is None else insts
        e2, parts = self.engine.energy(insts)
        return e2.reshape(len(self.core_counts), len(self.virt_counts)), parts


def _ints(s):
    return [int(x) for x in s.split(",") if x != ""]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", default="c2")
    ap.add_argument("--core", default="0,4,8,12", help="extra frozen core spinors per grid row")
    ap.add_argument("--virt", default="", help="frozen virtual spinors per grid column "
                                               "(default: 0, 20%% and 40%% of the kept virtuals)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import synth.problems as SP
    from . import Engine, Plan, desc_of_problem
    from .reference import ground_state
    pb = SP.config(args.config)
    dev = torch.device("cuda:0")
    h, Bs = SP.one_body(pb, dev), SP.factors(pb, dev)
    desc = desc_of_problem(pb, precision={"fp64": 0, "mixed": 1}[args.precision])
    c, _ = ground_state(Engine(Plan(desc_of_problem(pb)), dev), h, Bs)
    virt = _ints(args.virt) or [0, pb.n_v // 5, 2 * pb.n_v // 5]
    sw = FrozenSweep(desc, _ints(args.core), virt, device=dev)
    insts = sw.inputs(h, Bs, c)
    sw.energy(h, Bs, c, insts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        grid, _ = sw.energy(h, Bs, c, insts)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / args.reps
    print("[sweep] batched grid of %d points: %.1f ms" % (len(insts), ms_b), flush=True)
    # the same points one plan and one call at a time
    singles = [Engine(Plan(d), dev) for d in sw.descs]
    for e, x in zip(singles, insts):
        e.energy([x], parts=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        seq = [float(e.energy([x], parts=False)[0].item()) for e, x in zip(singles, insts)]
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3 / args.reps
    g = grid.cpu().numpy()
    same = all(float(g.flat[i]) == seq[i] for i in range(len(seq)))
    n_ext = [sw.plan.info(i).n_ext for i in range(len(insts))]
    out = {"config": args.config, "precision": args.precision, "core_frozen_extra": sw.core_counts,
           "virt_frozen": sw.virt_counts, "n_virt": pb.n_v, "e2": g.tolist(),
           "e2_fraction_of_full": (g / g[0, 0]).tolist(), "n_ext": n_ext,
           "batched_ms": ms_b, "sequential_ms": ms_s, "batched_equals_sequential": same,
           "dets_per_s_batched": sum(n_ext) / (ms_b * 1e-3)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
