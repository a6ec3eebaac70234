"""Autotuner of the launch shapes (mrpt2_tuning).

The work decomposition of a plan has three block-count targets per
excitation class (see mrpt2_tuning in include/mrpt2.h): the string chunks of
the generic sigma kernel, the row parts of the string-owned adjoint pass and
the string chunks of the generic row-owned adjoint pass; and one tile shape
per instance, the edge (64 or 128) of the FP64 pair-integral blocks.  tune()
times the candidates of each target on the GPU (every class's stage is timed
separately by the library, so one run per candidate serves all classes) and
keeps, per class, the fastest candidate when it beats the built-in rule by
more than MIN_GAIN.  Results are stored in a JSON table keyed by size bucket

    "<h><v>/q<floor log2 N_Q>/s<floor log2 strings>"

(class, external determinants and external strings of the class), or for the
pair-integral blocks

    "pair/vt<64-wide virtual tiles>/l<floor log2 Cholesky vectors>",

and tuning_for() turns a table into the per-instance capi.Tuning that
Plan(descs, tuning=...) takes.  Classes and instances whose bucket is not in
the table keep the built-in rule.

    python -m paper_2608_11529_amd.autotune c1 c2 c4 c3:0 c3:9 ... --out paper_2608_11529_amd/tuning.json
"""
import argparse
import json
import math
import os
import sys
import time

from . import capi

KNOBS = ("sigma_blocks", "bwd_blocks", "bwd_row_blocks")
CANDIDATES = {
    "sigma_blocks": (1024, 4096, 16384, 32768, 65536, 131072, 262144, 524288),
    "bwd_blocks": (512, 1024, 4096, 8192, 16384, 32768, 65536),
    "bwd_row_blocks": (512, 1024, 4096, 8192, 16384, 32768, 65536),   # swept together with bwd_blocks
}
DEFAULTS = {"sigma_blocks": 8192, "bwd_blocks": 2048, "bwd_row_blocks": 2048}
PAIR_TILES = (64, 128)
MIN_GAIN = 0.03
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def bucket(info, k):
    """Size bucket of class k of an instance (None for an empty class)."""
    nq, ns = int(info.n_ext_class[k]), int(info.n_strings_class[k])
    if nq <= 0 or ns <= 0:
        return None
    h, v = capi.CLASSES[k]
    return "%d%d/q%d/s%d" % (h, v, int(math.log2(nq)), int(math.log2(ns)))


def pair_bucket(desc, info):
    """Size bucket of an instance's FP64 pair-integral build (None without
    virtual pairs)."""
    if desc.n_virt < 2:
        return None
    return "pair/vt%d/l%d" % ((desc.n_virt + 63) // 64, int(math.log2(max(info.n_chol, 1))))


def load_table(table=None):
    """The table as a dict: table itself, a JSON path, or the package's
    tuning.json (empty when absent)."""
    if isinstance(table, dict):
        return table
    path = TABLE if table is None else table
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f).get("buckets", {})


def tuning_for(descs, table=None):
    """One capi.Tuning per descriptor: each class takes the entries of its
    size bucket, every other target stays 0 (built-in rule)."""
    from . import Plan
    if isinstance(descs, capi.Desc):
        descs = [descs]
    tab = load_table(table)
    plan = Plan(list(descs))
    out = []
    for i in range(len(descs)):
        info = plan.info(i)
        t = capi.Tuning()
        for k in range(capi.N_CLASS):
            ent = tab.get(bucket(info, k) or "", {})
            for knob in KNOBS:
                getattr(t, knob)[k] = int(ent.get(knob, 0))
        t.pair_tile = int(tab.get(pair_bucket(descs[i], info) or "", {}).get("pair_tile", 0))
        out.append(t)
    return out


def _uniform(knobs, value):
    t = capi.Tuning()
    for knob in knobs:
        for k in range(capi.N_CLASS):
            getattr(t, knob)[k] = value
    return t


def _stage_times(desc, inst, tuning, backward, reps):
    """Per-stage milliseconds (mean over reps after one warm-up) of one plan."""
    import torch
    from . import Engine, Plan
    eng = Engine(Plan(desc, tuning=tuning))
    acc = {}
    for r in range(reps + 1):
        if backward:
            outs, _, ms = eng.backward([inst], timed=True)
            del outs
        else:
            _, _, ms = eng.energy_timed([inst])
        if r:
            for key, v in ms.items():
                acc[key] = acc.get(key, 0.0) + v / reps
    del eng
    torch.cuda.empty_cache()
    return acc


def tune(desc, inst, backward=True, reps=2, log=print, classes=True):
    """Sweep every target of one instance (classes=False: only the
    pair-integral block edge); returns {bucket: {knob: value}} for the
    classes and instances where a candidate beat the built-in rule."""
    from . import Plan
    info = Plan(desc).info()
    found = {}
    # (knob -> (its class stage, shared stages that sum its partials), adjoint?);
    # the two adjoint targets act on different passes, so one sweep times
    # both.  A sweep sets every class at once, so the shared stages carry the
    # effect of all classes: charging it to each class errs on the side of the
    # built-in rule.
    sweeps = [({"sigma_blocks": ("sigma_%d%d", ("reduce",))}, False)] if classes else []
    if backward and classes:
        sweeps.append(({"bwd_blocks": ("bwd_str_%d%d", ("bwd_string_fin",)),
                        "bwd_row_blocks": ("bwd_row_%d%d", ())}, True))
    for knobs, bwd in sweeps:
        cands = CANDIDATES[next(iter(knobs))]
        base = _stage_times(desc, inst, None, bwd, reps)
        times = {}
        for v in cands:
            t0 = time.time()
            times[v] = _stage_times(desc, inst, [_uniform(knobs, v)], bwd, reps)
            log("[autotune] %s = %d (%.1f s)" % ("/".join(knobs), v, time.time() - t0))
        for knob, (stage, shared) in knobs.items():
            for k, cl in enumerate(capi.CLASSES):
                b = bucket(info, k)
                if b is None:
                    continue
                keys = [stage % cl] + list(shared)
                t_def = sum(base.get(x, 0.0) for x in keys)
                best, t_best = None, t_def
                for v, ms in times.items():
                    tv = sum(ms.get(x, 0.0) for x in keys)
                    if tv < t_best:
                        best, t_best = v, tv
                if best is not None and t_best < (1.0 - MIN_GAIN) * t_def:
                    found.setdefault(b, {})[knob] = best
                    log("[autotune] class %s bucket %s: %s %d -> %d, %.2f -> %.2f ms"
                        % (cl, b, knob, DEFAULTS[knob], best, t_def, t_best))
    # block edge of the FP64 pair-integral build (the mixed form has one shape)
    pb_key = pair_bucket(desc, info)
    if pb_key is not None:
        d64 = capi.Desc.from_buffer_copy(desc)
        d64.precision = 0
        t_rule = _stage_times(d64, inst, None, False, reps).get("pair_integrals", 0.0)
        best, t_best = None, t_rule
        for v in PAIR_TILES:
            tu = capi.Tuning()
            tu.pair_tile = v
            tv = _stage_times(d64, inst, [tu], False, reps).get("pair_integrals", 0.0)
            log("[autotune] pair_tile = %d: %.2f ms (rule %.2f ms)" % (v, tv, t_rule))
            if tv < t_best:
                best, t_best = v, tv
        if best is not None and t_best < (1.0 - MIN_GAIN) * t_rule:
            found.setdefault(pb_key, {})["pair_tile"] = best
            log("[autotune] bucket %s: pair_tile %d, %.2f -> %.2f ms" % (pb_key, best, t_rule, t_best))
    return found


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("configs", nargs="+",
                    help="synthetic workloads: synth.problems.config names, or c3:<seed> for one instance "
                         "of the batched workload")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--pair-only", action="store_true", help="sweep only the pair-integral block edge")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch
    import synth.problems as SP
    from . import Engine, Plan, desc_of_problem
    from .reference import ground_state
    table = load_table(args.out)
    runs = []
    for name in args.configs:
        pb = SP.batched_instance(int(name[3:])) if name.startswith("c3:") else SP.config(name)
        dev = torch.device("cuda:0")
        h, Bs = SP.one_body(pb, dev), SP.factors(pb, dev)
        desc = desc_of_problem(pb, precision=1)
        c, _ = ground_state(Engine(Plan(desc_of_problem(pb))), h, Bs)
        print("[autotune] %s: inputs ready" % name, flush=True)
        found = tune(desc, (h, Bs, c), backward=not args.no_backward, reps=args.reps,
                     log=lambda m: print(m, flush=True), classes=not args.pair_only)
        for b, ent in found.items():
            table.setdefault(b, {}).update(ent)
        runs.append(name)
        del h, Bs, c
        torch.cuda.empty_cache()
    made_by, workloads = [], []
    if os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        made_by, workloads = old.get("made_by", []), old.get("workloads", [])
    made_by.append("python -m paper_2608_11529_amd.autotune " + " ".join(sys.argv[1:] if argv is None else argv))
    with open(args.out, "w") as f:
        json.dump({"made_by": made_by, "workloads": workloads + runs,
                   "candidates": dict(CANDIDATES, pair_tile=PAIR_TILES),
                   "defaults": DEFAULTS, "buckets": table}, f, indent=1, sort_keys=True)
    print("[autotune] wrote %s (%d buckets)" % (args.out, len(table)), flush=True)


if __name__ == "__main__":
    main()
