#!/usr/bin/env python3
"""Benchmark of the MI355X Epstein-Nesbet MRPT2 energy on one GPU.

One step = one full E2 evaluation (every step of the hot path: factor tables,
reference energy, integral builds, sigma contractions with the denominator
epilogue, reduction) over the synthetic Xe-like workload c4 (18 frozen + 28
core spinors, 18 active spinors with 8 electrons in six 3-spinor DAS
subspaces with one hop, virtuals up to 50 Eh kept, Dirac-Coulomb rank 2000 +
Gaunt 600 + gauge 600), inputs resident in HBM when the timed region starts.

Prints one JSON line: external determinants per second (value), E2
evaluations per second, the roofline of the dominant kernel (timed with HIP
events on the library's stream) and the CPU oracle timed on a bounded sample;
beside them the adjoint, the level-shifted form (Sec. 2.6), the state-specific
energies of the lowest reference states in one call, and the device
eigensolver for those states (each skipped with a 0 option).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK = 78.6e12       # FLOP/s, dense FP64 matrix
FP64_VALU_PEAK = 78.6e12       # FLOP/s, FP64 vector (256 CU x 64 lanes x 2 x 2.4 GHz)
FP32_MFMA_PEAK = 157.3e12      # FLOP/s, dense FP32 matrix
HBM_PEAK = 8.0e12              # B/s


def cpu_baseline(pb, seconds=15.0):
    """The oracle (as it stands, single thread) on a bounded sample of the
    same workload, extrapolated to its class mix: classes (2,2) and (1,2) for
    the first core pairs (cores), the first 64 virtual spinors and every
    string, on the sub-problem of frozen core + core + active + those
    virtuals, with a one-hot reference vector on the lowest-diagonal
    reference determinant (the oracle's cost per external determinant does
    not depend on the vector's values)."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits
    import synth.problems as SP
    from synth import rng as _rng  # noqa: F401
    from oracle import run
    from oracle.classes import ClassOracle
    from oracle.space import ActiveSpace

    n_keep_v = min(64, pb.n_v)
    n_occ = pb.n_fc + pb.n_c + pb.n_a
    idx = list(range(n_occ)) + list(range(n_occ, n_occ + n_keep_v))
    torch.set_num_threads(8)
    h = SP.one_body(pb)[idx][:, idx].numpy()
    Bs = []
    for t, (r, _) in enumerate(pb.sets):
        Bs.append(SP.factor_rows(pb, t, 0, r, idx).numpy())
    ws = SP.weights(pb)
    with threadpool_limits(limits=1):
        torch.set_num_threads(1)
        hfc, Bc = run.correlated_inputs(h, Bs, ws, pb.n_fc)
        sp = ActiveSpace(pb.n_c, pb.sub_sizes, pb.n_elec, pb.base, pb.max_hops, n_keep_v)
        co = ClassOracle(sp, hfc, Bc, ws)
        # reference: the lowest-diagonal reference determinant (oracle-computed)
        diag = [co.energy_of(co.core | a) for a in co.P]
        c = np.zeros(len(co.P), dtype=np.complex128)
        c[int(np.argmin(diag))] = 1.0
        e0 = min(diag)
        from itertools import combinations
        samples = {}
        n12 = len(sp.class_strings(1, 2, 0))
        for cl, holes, per in (((2, 2), list(combinations(range(pb.n_c), 2)), math.comb(n_keep_v, 2) * len(co.P)),
                               ((1, 2), [(x,) for x in range(pb.n_c)], math.comb(n_keep_v, 2) * n12)):
            done, t0 = 0, time.perf_counter()
            for hh in holes:
                co.e2(c, 0, E0=e0, core_sets=[hh], classes=[cl])
                done += 1
                if time.perf_counter() - t0 > seconds / 2:
                    break
            samples[cl] = (done, done * per, time.perf_counter() - t0)
    # combine the two class rates with the workload's class mix
    import paper_2608_11529_amd as M
    info = M.Plan(M.desc_of_problem(pb)).info()
    nq = {cl: info.n_ext_class[M.CLASSES.index(cl)] for cl in samples}
    rate = {cl: d / t for cl, (_, d, t) in samples.items()}
    value = sum(nq.values()) / sum(nq[cl] / rate[cl] for cl in samples)
    return {
        "value": value, "unit": "dets/s", "cores": 1, "kind": "oracle",
        "sample": "classes (2,2) and (1,2) (%.0f%% of N_Q): %d core pairs and %d cores, each x C(%d,2) virtual "
                  "pairs x all strings (%d and %d external determinants in %.1f s and %.1f s), one-hot reference "
                  "vector; rates extrapolated to the whole workload with its class mix; single-threaded "
                  "numpy oracle"
                  % (100.0 * sum(nq.values()) / info.n_ext, samples[(2, 2)][0], samples[(1, 2)][0], n_keep_v,
                     samples[(2, 2)][1], samples[(1, 2)][1], samples[(2, 2)][2], samples[(1, 2)][2]),
    }


def roofline(dom, ms, cases, precision):
    """Roofline of stage dom (milliseconds ms per launch) over the instances
    cases = [(problem, plan info)]: algorithmic work summed over instances."""
    import paper_2608_11529_amd as M
    mixed = precision == "mixed"
    if dom == "pair_integrals":
        flop = sum(8.0 * ((pb.n_c + pb.n_a) * (pb.n_c + pb.n_a - 1) // 2) * pb.n_v * (pb.n_v - 1) * pb.n_l
                   for pb, _ in cases)
        peak = FP32_MFMA_PEAK if mixed else FP64_MFMA_PEAK
        ach = flop / (ms * 1e-3)
        return {"kernel": ("k_b_abuild_f32 (virtual-pair integrals <ab||xy>, complex FP32 MFMA)" if mixed else
                           "k_b_abuild128 / k_b_abuild (virtual-pair integrals <ab||xy>, complex FP64 MFMA; "
                           "128 x 128 blocks where they fill, else 64 x 64)"),
                "bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": None}
    if dom == "sigma_22":
        # six FP64 vector instructions per determinant (two adds, the share
        # of the merged reciprocal, merge and accumulate)
        ops = 6.0 * sum(info.n_ext_class[0] for _, info in cases)
        ach = ops / (ms * 1e-3)
        peak = FP64_VALU_PEAK / 2.0
        return {"kernel": "k_e22 (class (2,2) denominators and sums, FP64 vector)", "bound": "alu",
                "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "Top/s", "frac": ach / peak, "traffic": None}
    if dom.startswith("sigma_"):
        k = M.CLASSES.index(tuple(int(x) for x in dom.split("_")[1]))
        h, v = M.CLASSES[k]
        flop = sum(8.0 * info.n_conn_class[k] * math.comb(pb.n_c, h) * math.comb(pb.n_v, v) for pb, info in cases)
        ach = flop / (ms * 1e-3)
        return {"kernel": "sigma contraction of class %s (complex FP64, nonzero couplings)" % dom[-2:],
                "bound": "alu", "achieved": ach / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK, "traffic": None}
    return {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None}


def whole_pass_roofline(pb, info, ms, precision, adjoint=False):
    """Bound of one whole evaluation by the algorithmic work of the path:
    MFMA F = complex multiply-adds x 8 of the integral builds and of the sigma
    contractions (nonzero couplings), at the FP64 or FP32 matrix peak; FP64
    vector work of the Epstein-Nesbet epilogue, 6 instructions per external
    determinant, at 39.3e12 instructions/s.  The adjoint doubles both counts
    (every product has two operand adjoints; every determinant's epilogue is
    recomputed and differentiated).  The bound is the larger time (the two
    units could overlap), the fraction bound / measured."""
    mixed = precision == "mixed"
    k = 2.0 if adjoint else 1.0
    flop = k * (info.flop_integral + info.flop_sigma)
    slots = k * 6.0 * info.n_ext
    t_mfma = flop / (FP32_MFMA_PEAK if mixed else FP64_MFMA_PEAK)
    t_valu = slots / (FP64_VALU_PEAK / 2.0)
    t = max(t_mfma, t_valu)
    return {"bound_s": t, "bound": "mfma" if t_mfma >= t_valu else "alu", "t_mfma_s": t_mfma, "t_valu_s": t_valu,
            "measured_s": ms * 1e-3, "frac": t / (ms * 1e-3)}


def roofline_backward(dom, ms, pb, info, precision):
    """Roofline of the dominant adjoint stage: the pair-integral adjoint GEMM
    (two operand adjoints of the forward build: 2 x its flops, on FP32 or FP64
    MFMA), or a per-class pass on the FP64 vector units counted as twice the
    forward epilogue plus two complex multiply-adds (8 instructions) per
    coupling and determinant (the recomputed sigma and its adjoint)."""
    import paper_2608_11529_amd as M
    mixed = precision == "mixed"
    if dom == "bwd_pair_integrals":
        flop = 2.0 * 8.0 * ((pb.n_c + pb.n_a) * (pb.n_c + pb.n_a - 1) // 2) * pb.n_v * (pb.n_v - 1) * pb.n_l
        peak = FP32_MFMA_PEAK if mixed else FP64_MFMA_PEAK
        ach = flop / (ms * 1e-3)
        return {"kernel": "pair-integral adjoint GEMM", "bound": "mfma", "achieved": ach / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s", "frac": ach / peak, "traffic": None, "ms_per_launch": ms}
    if dom.startswith("bwd_row_") or dom.startswith("bwd_str_"):
        k = M.CLASSES.index(tuple(int(x) for x in dom[-2:]))
        n_q = info.n_ext_class[k]
        per_det = 12.0 + (8.0 * info.n_conn_class[k] / max(1, info.n_strings_class[k]) if k != 0 else 0.0)
        ops = n_q * per_det
        ach = ops / (ms * 1e-3)
        peak = FP64_VALU_PEAK / 2.0
        return {"kernel": "adjoint pass %s (FP64 vector, %.1f instructions per determinant)" % (dom, per_det),
                "bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "Top/s", "frac": ach / peak,
                "traffic": None, "ms_per_launch": ms}
    return {"kernel": dom, "bound": None, "frac": None, "ms_per_launch": ms}


def tuning_note(autotune):
    n = len(autotune.load_table())
    return "autotuned table (%d size buckets)" % n if n else "built-in rules"


def bench_batched(args):
    """c3: 64 independent instances of uneven size (core 4-20, active 6-12 at
    half filling in 2-3 subspaces with one hop, virtual 50-400, DC rank
    3 n_orb + Gaunt and gauge n_orb) in one batched call, compared with 64
    one-instance calls in sequence."""
    import torch
    import synth.problems as SP
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd import autotune
    from paper_2608_11529_amd.reference import ground_state

    n_inst = 64
    pbs = [SP.batched_instance(s) for s in range(n_inst)]
    prec = 1 if args.precision == "mixed" else 0
    dev = torch.device("cuda:0")
    t = time.time()
    ins = []
    singles = []
    for pb in pbs:
        h = SP.one_body(pb, dev)
        Bs = SP.factors(pb, dev)
        d1 = M.desc_of_problem(pb, precision=prec)
        e1 = M.Engine(M.Plan(d1, tuning=autotune.tuning_for(d1)), dev)
        c, _ = ground_state(e1, h, Bs)
        ins.append((h, Bs, c))
        singles.append(e1)
        if len(singles) % 8 == 0:
            print("[bench] c3: %d instances ready (%.1f s)" % (len(singles), time.time() - t),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print("[bench] c3: %d instances generated and solved in %.1f s" % (n_inst, time.time() - t),
          file=sys.stderr, flush=True)
    bdescs = [M.desc_of_problem(pb, precision=prec) for pb in pbs]
    plan = M.Plan(bdescs, tuning=autotune.tuning_for(bdescs))
    eng = M.Engine(plan, dev)
    n_ext = sum(plan.info(i).n_ext for i in range(n_inst))
    for _ in range(args.warmup):
        eng.energy(ins)
        for i, e1 in enumerate(singles):
            e1.energy([ins[i]])
    torch.cuda.synchronize()
    stage_sum = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e2, parts, ms = eng.energy_timed(ins)
        for k, v in ms.items():
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    ms_batched = (time.perf_counter() - t0) * 1000.0 / args.steps
    e2_b = e2.cpu().numpy().copy()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e2_s = [float(e1.energy([ins[i]])[0][0]) for i, e1 in enumerate(singles)]
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1000.0 / args.steps
    stage = {k: v / args.steps for k, v in stage_sum.items()}
    dmax = max(abs(a - b) for a, b in zip(e2_b, e2_s))
    print("[bench] c3 batched %.1f ms, sequential %.1f ms, max |dE2| batched vs sequential %.3g"
          % (ms_batched, ms_seq, dmax), file=sys.stderr, flush=True)
    dom = max(stage, key=lambda k: stage[k])
    bwd = None
    if args.backward_steps > 0:
        # adjoint of all 64 instances with the factors in the Hermitian-packed
        # layout (inputs and factor gradients at half the bytes of the full
        # matrices, which together would not fit one GPU)
        del singles, eng
        torch.cuda.empty_cache()
        nb = n_inst
        for i in range(n_inst):
            h_, Bs_, c_ = ins[i]
            ins[i] = (h_, [M.hermitian_pack(B) for B in Bs_], c_)
            del Bs_
        torch.cuda.empty_cache()
        sub = ins
        bdescs = [M.desc_of_problem(pb, precision=prec, layout=1) for pb in pbs]
        bplan = M.Plan(bdescs[:nb], tuning=autotune.tuning_for(bdescs[:nb]))
        beng = M.Engine(bplan, dev)
        n_ext_b = sum(bplan.info(i).n_ext for i in range(nb))
        beng.backward(sub)
        torch.cuda.synchronize()
        outs_b = None
        t0 = time.perf_counter()
        for _ in range(args.backward_steps):
            outs_b = None                      # one set of factor gradients alive at a time
            outs_b, _ = beng.backward(sub)
        torch.cuda.synchronize()
        ms_bb = (time.perf_counter() - t0) * 1000.0 / args.backward_steps
        ref = [(x[0].clone(), x[2].clone()) for x in outs_b]
        del outs_b
        # the same batched forward + adjoint captured once in a HIP graph and
        # replayed (the plan is then reserved for the graph)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            beng.backward(sub, asynchronous=True, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            outs_g, _ = beng.backward(sub, asynchronous=True, stream=torch.cuda.current_stream())
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.backward_steps):
            graph.replay()
        torch.cuda.synchronize()
        ms_bg = (time.perf_counter() - t0) * 1000.0 / args.backward_steps
        beng.check()
        dgraph = max(max(float((x[0] - r[0]).abs().max().item()), float((x[2] - r[1]).abs().max().item()))
                     for x, r in zip(outs_g, ref))
        print("[bench] c3 backward (%d instances, packed factors) as one replayed HIP graph: %.1f ms" % (nb, ms_bg),
              file=sys.stderr, flush=True)
        del outs_g, graph, beng
        torch.cuda.empty_cache()
        seng = [M.Engine(M.Plan(d, tuning=autotune.tuning_for(d)), dev) for d in bdescs[:nb]]
        for i, e1 in enumerate(seng):
            e1.backward([sub[i]])
            e1.grad_workspace = None
        torch.cuda.synchronize()
        dgrad = 0.0
        t0 = time.perf_counter()
        for _ in range(args.backward_steps):
            for i, e1 in enumerate(seng):
                (dh, _, dc), = e1.backward([sub[i]])[0]
                e1.grad_workspace = None
                dgrad = max(dgrad, float((dh - ref[i][0]).abs().max().item()), float((dc - ref[i][1]).abs().max().item()))
        torch.cuda.synchronize()
        ms_bs = (time.perf_counter() - t0) * 1000.0 / args.backward_steps
        print("[bench] c3 backward (%d instances, packed factors): batched %.1f ms, sequential %.1f ms" % (nb, ms_bb, ms_bs),
              file=sys.stderr, flush=True)
        bwd = {"instances": nb, "factor_layout": "hermitian-packed", "n_ext": n_ext_b, "batched_ms": ms_bb, "graph_replay_ms": ms_bg,
               "sequential_ms": ms_bs,
               "grad_evals_per_s": nb * 1000.0 / ms_bb, "max_abs_dgrad_batched_vs_sequential": dgrad,
               "max_abs_dgrad_graph_vs_batched": dgraph,
               "note": "sequential timing includes the per-call gradient workspace allocation"}
    return {
        "metric": "external dets/sec + E2 evals/sec (mixed vs FP64, |dE2| Eh), 1 MI355X",
        "value": n_ext / (ms_batched * 1e-3), "unit": "dets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batched,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-mfma+f64" if prec else "f64", "data": "synthetic",
        "config": {"workload": "c3: 64 uneven instances (seeds 0-63), sum N_Q=%d, one batched call" % n_ext,
                   "precision": args.precision, "n_ext": n_ext, "launch_shapes": tuning_note(autotune)},
        "e2_evals_per_s": n_inst * 1000.0 / ms_batched,
        "compare": {"mode": "64 one-instance calls in sequence", "ms_per_step": ms_seq,
                    "value": n_ext / (ms_seq * 1e-3), "max_abs_dE2": dmax},
        "stages_ms": {k: round(v, 3) for k, v in stage.items() if v > 0},
        "roofline": dict(roofline(dom, stage[dom], [(pb, plan.info(i)) for i, pb in enumerate(pbs)], args.precision),
                         ms_per_launch=stage[dom]),
        "backward": bwd,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--precision", default="fp64", choices=["mixed", "fp64"],
                    help="precision of the headline value (the other form is measured beside it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--backward-steps", type=int, default=1,
                    help="timed adjoint calls after the forward measurement (0: none)")
    ap.add_argument("--level-shift", type=float, default=0.05, metavar="B",
                    help="also time one forward call with the imaginary level shift b = B (Sec. 2.6); 0: skip")
    ap.add_argument("--roots", type=int, default=3, metavar="K",
                    help="also time the state-specific E2 of the K lowest reference states in one call "
                         "against K single-state calls; 0: skip")
    ap.add_argument("--davidson", type=int, default=3, metavar="K",
                    help="also time the device Davidson solver for the 1 and K lowest reference states against "
                         "the host eigensolver path; 0: skip")
    ap.add_argument("--c3-steps", type=int, default=2, metavar="K",
                    help="after the c4 measurement also time the 64-instance batch c3 (one batched call "
                         "against 64 one-instance calls, K steps each); 0: skip")
    ap.add_argument("--no-packed-layout", action="store_true",
                    help="skip the forward call with the factors in the Hermitian-packed layout")
    ap.add_argument("--no-delta-stats", action="store_true",
                    help="skip the denominator statistics (smallest |E0 - H_KK| per class)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers three times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = args.copy_calibration // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "copies": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (N=%d requested); the multi-GPU "
              "decomposition is a design note, not an implementation" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np  # noqa: F401
    import torch
    import synth.problems as SP
    import paper_2608_11529_amd as M
    from paper_2608_11529_amd import autotune
    from paper_2608_11529_amd.reference import ground_state

    if args.config == "c3":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    pb = SP.config(args.config)
    dev = torch.device("cuda:0")
    t = time.time()
    h = SP.one_body(pb, dev)
    Bs = SP.factors(pb, dev)
    torch.cuda.synchronize()
    print("[bench] inputs %s generated on GPU in %.1f s" % (args.config, time.time() - t), file=sys.stderr, flush=True)
    prec = {"mixed": 1, "fp64": 0}
    descs = {p: M.desc_of_problem(pb, precision=prec[p]) for p in ("fp64", "mixed")}
    plans = {p: M.Plan(descs[p], tuning=autotune.tuning_for(descs[p])) for p in descs}
    info = plans["fp64"].info()
    engs = {p: M.Engine(plans[p], dev) for p in plans}
    c, e0 = ground_state(engs["fp64"], h, Bs)
    print("[bench] plan ready, N_P=%d N_Q=%d, reference state E0-Ecore=%.6f" % (info.n_ref, info.n_ext, e0),
          file=sys.stderr, flush=True)
    insts = [(h, Bs, c)]
    res = {}
    for p in (args.precision, "fp64" if args.precision == "mixed" else "mixed"):
        eng = engs[p]
        for _ in range(args.warmup):
            eng.energy(insts)
        torch.cuda.synchronize()
        stage_sum = {}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e2, parts, ms = eng.energy_timed(insts)
            for k, v in ms.items():
                stage_sum[k] = stage_sum.get(k, 0.0) + v
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res[p] = {"ms": (t1 - t0) * 1000.0 / args.steps,
                  "stage": {k: v / args.steps for k, v in stage_sum.items()},
                  "e2": float(e2[0].item()), "parts": parts[0].cpu().tolist()}
        print("[bench] %s: %d steps, %.1f ms/step, E2=%.12f" % (p, args.steps, res[p]["ms"], res[p]["e2"]),
              file=sys.stderr, flush=True)
        print("[bench] %s stages (ms): " % p + json.dumps({k: round(v, 3) for k, v in res[p]["stage"].items() if v > 0}),
              file=sys.stderr, flush=True)
    head = res[args.precision]
    stage = head["stage"]
    ms_per_step = head["ms"]

    # roofline of the dominant kernel of the headline path
    dom = max(stage, key=lambda k: stage[k])
    roof = roofline(dom, stage[dom], [(pb, info)], args.precision)
    n_v, n_l = pb.n_v, pb.n_l
    roof["ms_per_launch"] = stage[dom]
    # HBM bytes need the profiler's counters (FETCH_SIZE, WRITE_SIZE), which a
    # timed run does not collect: traffic stays null here and the counter
    # figures of the kernels are kept with their commands under profiles/
    other = "fp64" if args.precision == "mixed" else "mixed"
    out = {
        "metric": "external dets/sec + E2 evals/sec (mixed vs FP64, |dE2| Eh), 1 MI355X",
        "value": info.n_ext / (ms_per_step * 1e-3),
        "unit": "dets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-mfma+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: n_fc=%d n_core=%d n_act=%d (%s, %d e, base %s, hops<=%d) n_virt=%d "
                               "n_chol=%d (sets %s); N_P=%d N_Q=%d"
                               % (args.config, pb.n_fc, pb.n_c, pb.n_a, "x".join(map(str, pb.sub_sizes)),
                                  pb.n_elec, pb.base, min(pb.max_hops, 99), n_v, n_l, pb.sets,
                                  info.n_ref, info.n_ext),
                   "precision": args.precision, "n_ext": info.n_ext, "n_ref": info.n_ref,
                   "launch_shapes": tuning_note(autotune)},
        "e2_evals_per_s": 1000.0 / ms_per_step,
        "e2": head["e2"],
        "compare": {"precision": other, "value": info.n_ext / (res[other]["ms"] * 1e-3),
                    "ms_per_step": res[other]["ms"], "e2": res[other]["e2"],
                    "e2_evals_per_s": 1000.0 / res[other]["ms"],
                    "stages_ms": {k: round(v, 3) for k, v in res[other]["stage"].items() if v > 0},
                    "roofline": whole_pass_roofline(pb, info, res[other]["ms"], other),
                    "abs_dE2_mixed_vs_fp64": abs(res["mixed"]["e2"] - res["fp64"]["e2"]),
                    "abs_dE2_per_class": [abs(x - y) for x, y in zip(res["mixed"]["parts"][:9], res["fp64"]["parts"][:9])]},
        "stages_ms": {k: round(v, 3) for k, v in stage.items() if v > 0},
        "roofline": roof,
        "roofline_whole_pass": whole_pass_roofline(pb, info, ms_per_step, args.precision),
    }

    def guarded(key, fn):
        # an optional measurement that fails records its error in the JSON
        # line instead of suppressing the headline result
        try:
            fn()
        except Exception as exc:  # noqa: BLE001
            out[key] = {"error": "%s: %s" % (type(exc).__name__, exc)}
            print("[bench] %s failed: %s" % (key, exc), file=sys.stderr, flush=True)
            torch.cuda.synchronize()

    def measure_level_shift():
        # the shifted denominators of Sec. 2.6 on the same inputs: one untimed
        # and one timed call (the shifted form is not the headline path)
        dls = M.desc_of_problem(pb, precision=prec[args.precision], level_shift_b=args.level_shift)
        els = M.Engine(M.Plan(dls, tuning=autotune.tuning_for(dls)), dev)
        els.energy(insts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e2s, _, lms = els.energy_timed(insts)
        torch.cuda.synchronize()
        ls_ms = (time.perf_counter() - t0) * 1000.0
        out["level_shift"] = {
            "b": args.level_shift, "precision": args.precision, "ms_per_step": ls_ms,
            "dets_per_s": info.n_ext / (ls_ms * 1e-3), "e2": float(e2s[0].item()),
            "e2_unshifted": head["e2"], "ratio_to_unshifted": ls_ms / ms_per_step,
            "stages_ms": {k: round(v, 2) for k, v in lms.items() if v > 0.05},
        }
        print("[bench] level shift b=%g (%s): %.1f ms, E2=%.12f" % (args.level_shift, args.precision, ls_ms,
                                                                    out["level_shift"]["e2"]),
              file=sys.stderr, flush=True)
        del els
        torch.cuda.empty_cache()

    if args.level_shift != 0.0:
        guarded("level_shift", measure_level_shift)

    def measure_packed():
        # the same evaluation with the factors in the Hermitian-packed layout
        # (upper triangles, half the memory and half the factor pass)
        dpk = M.desc_of_problem(pb, precision=prec[args.precision], layout=1)
        epk = M.Engine(M.Plan(dpk, tuning=autotune.tuning_for(dpk)), dev)
        Bp = [M.hermitian_pack(B) for B in Bs]
        epk.energy([(h, Bp, c)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e2p, _, pms = epk.energy_timed([(h, Bp, c)])
        torch.cuda.synchronize()
        pk_ms = (time.perf_counter() - t0) * 1000.0
        out["packed_layout"] = {
            "precision": args.precision, "ms_per_step": pk_ms, "dets_per_s": info.n_ext / (pk_ms * 1e-3),
            "factor_bytes": sum(int(x.numel()) * 16 for x in Bp), "e2": float(e2p[0].item()),
            "abs_dE2_vs_full_layout": abs(float(e2p[0].item()) - head["e2"]),
            "factor_tables_ms": round(pms.get("factor_tables", 0.0), 2),
            "factor_tables_ms_full_layout": round(stage.get("factor_tables", 0.0), 2),
        }
        print("[bench] packed layout: %.1f ms, E2=%.12f" % (pk_ms, out["packed_layout"]["e2"]),
              file=sys.stderr, flush=True)
        del epk, Bp
        torch.cuda.empty_cache()

    if not args.no_packed_layout:
        guarded("packed_layout", measure_packed)

    def measure_delta_stats():
        # smallest |E0 - H_KK| per class (intruder measure of Sec. 2.6) and the
        # determinants within 1 Eh of zero
        eng = engs[args.precision]
        t0 = time.perf_counter()
        mn, cnt = eng.delta_stats(insts, 1.0)
        ds_ms = (time.perf_counter() - t0) * 1000.0
        out["delta_stats"] = {"ms": ds_ms, "thresh": 1.0,
                              "min_abs_delta": {"%d%d" % cl: float(mn[0][k]) for k, cl in enumerate(M.CLASSES)},
                              "n_below": {"%d%d" % cl: int(cnt[0][k]) for k, cl in enumerate(M.CLASSES)}}
        print("[bench] delta stats: " + json.dumps(out["delta_stats"]), file=sys.stderr, flush=True)

    if not args.no_delta_stats:
        guarded("delta_stats", measure_delta_stats)

    def measure_davidson():
        # reference states: device block Davidson (H_PP assembled and applied
        # on the GPU) against H_PP copied to the host and ARPACK/LAPACK
        from paper_2608_11529_amd.reference import host_ground_state
        e64 = engs["fp64"]
        dv = {}
        for kk in sorted({1, args.davidson}):
            e64.reference_states(h, Bs, kk)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Cd, ed, its = e64.reference_states(h, Bs, kk)
            torch.cuda.synchronize()
            dv[kk] = {"ms": (time.perf_counter() - t0) * 1000.0, "iterations": its, "e_minus_ecore": ed.tolist()}
        t0 = time.perf_counter()
        c_h, e_h = host_ground_state(e64, h, Bs)
        torch.cuda.synchronize()
        host_ms = (time.perf_counter() - t0) * 1000.0
        e2d = float(engs[args.precision].energy([(h, Bs, Cd[0].contiguous())], parts=False)[0].item())
        out["davidson"] = {"n_ref": info.n_ref, "states": dv, "host_path_ms": host_ms, "host_e0_minus_ecore": e_h,
                           "e2_with_davidson_state": e2d, "e2_with_host_state": head["e2"]}
        print("[bench] davidson: " + json.dumps(out["davidson"]), file=sys.stderr, flush=True)

    if args.davidson > 0:
        guarded("davidson", measure_davidson)

    def measure_roots():
        # state-specific E2_m of the K lowest states: one call (shared integral
        # build) against K single-state calls, same engine and inputs
        from paper_2608_11529_amd.reference import states
        eng = engs[args.precision]
        C, e0s = states(engs["fp64"], h, Bs, args.roots)
        eng.energy_roots([(h, Bs, C)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e2r, _ = eng.energy_roots([(h, Bs, C)])
        torch.cuda.synchronize()
        ms_roots = (time.perf_counter() - t0) * 1000.0
        t0 = time.perf_counter()
        singles = [float(eng.energy([(h, Bs, C[r].contiguous())], parts=False)[0].item()) for r in range(args.roots)]
        torch.cuda.synchronize()
        ms_single = (time.perf_counter() - t0) * 1000.0
        e2r = e2r[:, 0].cpu().tolist()
        out["roots"] = {"k": args.roots, "precision": args.precision, "ms": ms_roots, "sequential_ms": ms_single,
                        "dets_per_s": args.roots * info.n_ext / (ms_roots * 1e-3), "e2": e2r,
                        "e0_minus_ecore": [float(x) for x in e0s], "equal_to_single_calls": e2r == singles}
        print("[bench] %d roots (%s): %.1f ms in one call, %.1f ms as single calls" % (args.roots, args.precision,
                                                                                   ms_roots, ms_single),
              file=sys.stderr, flush=True)

    if args.roots > 0:
        guarded("roots", measure_roots)
    if args.backward_steps > 0:
        # adjoint of the headline form: one call recomputes the forward pass and
        # returns dE2/dh, dE2/dB (every set) and dE2/dC
        for p in list(engs):
            if p != args.precision:
                del engs[p]
        eng = engs[args.precision]
        del res
        torch.cuda.empty_cache()
        bsum, t0 = {}, time.perf_counter()
        for _ in range(args.backward_steps):
            outs, _, bms = eng.backward(insts, timed=True)
            for k, v in bms.items():
                bsum[k] = bsum.get(k, 0.0) + v
        torch.cuda.synchronize()
        bwd_ms = (time.perf_counter() - t0) * 1000.0 / args.backward_steps
        (dh, dBs, dc), = outs
        bst = {k: v / args.backward_steps for k, v in bsum.items()}
        bdom = max((k for k in bst if k.startswith("bwd_")), key=lambda k: bst[k])
        out["backward"] = {
            "roofline": roofline_backward(bdom, bst[bdom], pb, info, args.precision),
            "roofline_whole_pass": whole_pass_roofline(pb, info, bwd_ms, args.precision, adjoint=True),
            "precision": args.precision, "steps": args.backward_steps, "ms_per_step": bwd_ms,
            "grad_evals_per_s": 1000.0 / bwd_ms, "dets_per_s": info.n_ext / (bwd_ms * 1e-3),
            "ratio_to_forward": bwd_ms / ms_per_step,
            "max_abs_grad": {"dh": float(dh.abs().max().item()), "dc": float(dc.abs().max().item()),
                             "dB": [float(x.abs().max().item()) for x in dBs]},
            "stages_ms": {k: round(v, 2) for k, v in bst.items() if v > 0.05},
        }
        print("[bench] backward (%s): %.1f ms/step (%.2f x forward)" % (args.precision, bwd_ms, bwd_ms / ms_per_step),
              file=sys.stderr, flush=True)
        del outs, dh, dBs, dc
        eng.grad_workspace = None
    if not args.no_cpu_baseline or args.c3_steps > 0:
        del Bs, h, engs
        eng = None
        torch.cuda.empty_cache()
    if args.c3_steps > 0 and args.config == "c4":
        # the batched form on its own workload, beside the headline
        def measure_c3():
            c3 = bench_batched(argparse.Namespace(steps=args.c3_steps, warmup=1, precision=args.precision,
                                                  backward_steps=0))
            out["batched_c3"] = {k: c3[k] for k in ("value", "unit", "ms_per_step", "e2_evals_per_s", "dtype",
                                                     "config", "compare", "roofline", "stages_ms")}
            torch.cuda.empty_cache()
        guarded("batched_c3", measure_c3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
