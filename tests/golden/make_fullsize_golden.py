"""Oracle values of a whole large workload (c2 or c4), class by class.

Runs the CPU oracle only (packages `oracle` and `synth`), never the HIP
library: oracle.fullsize streams the factors once (frozen-core fold, pair
energies, occupied factor columns), the class oracle gives the reference
Hamiltonian H_PP and the classes with at most one virtual electron (in
parallel over core-hole tuples or strings), and the C loops of
oracle.fullsize the classes with two virtual electrons.  C is the lowest
eigenvector of the oracle's H_PP (largest component real and positive), in
the oracle's order (sorted active strings).

Results are written after every class, and classes already present in the
output file are not recomputed, so an interrupted run resumes.

Usage: python tests/golden/make_fullsize_golden.py c2 [--jobs 8]
Output: tests/golden/<name>_full_oracle.json
"""
import argparse
import json
import math
import os
import sys
import time
from itertools import combinations
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth.problems as SP  # noqa: E402
from oracle import fullsize, run  # noqa: E402
from oracle.classes import CLASSES  # noqa: E402

_CO = None      # the oracle, shared with forked workers
_C = None
_E0 = None


def _small_task(task):
    cl, core_sets, strings = task
    import threadpoolctl
    with threadpoolctl.threadpool_limits(1):
        parts, _ = _CO.e2(_C, 0, E0=_E0, core_sets=core_sets, classes=[cl], strings=strings)
    return parts[cl]


def small_class(cl, jobs):
    h_, _ = cl
    n_c = _CO.sp.n_c
    tasks = []
    if h_ > 0:
        holes = list(combinations(range(n_c), h_))
        step = max(1, len(holes) // (4 * jobs))
        for i in range(0, len(holes), step):
            tasks.append((cl, holes[i:i + step], None))
    else:
        strs = _CO.sp.class_strings(0, cl[1], 0)
        step = max(1, len(strs) // (4 * jobs))
        for i in range(0, len(strs), step):
            tasks.append((cl, [()], strs[i:i + step]))
    with get_context("fork").Pool(jobs) as pool:
        vals = pool.map(_small_task, tasks, chunksize=1)
    return math.fsum(vals)


def block_list(n_c, nv, seed=5):
    """Work blocks of the two-virtual classes to check one by one: the edges
    of the virtual range (first tile, the last and possibly partial 64-wide
    tile, diagonal tile pairs), the first and last core holes, and a fixed
    pseudo-random choice.  Entries: (class, hole tuple, a range, b range)
    with virtual positions; a < b is implied."""
    T = (nv + 63) // 64
    rng = np.random.default_rng(seed)
    tile = lambda i: (i * 64, min(nv, i * 64 + 64))  # noqa: E731
    sub = lambda i, k: (min(nv, i * 64 + 16 * k), min(nv, i * 64 + 16 * k + 16))  # noqa: E731
    last = T - 1
    pairs = list(combinations(range(n_c), 2))
    out = []
    for hp, I, J in [((n_c - 2, n_c - 1), last, last), ((0, 1), 0, 0), ((0, n_c - 1), 0, last),
                     ((n_c - 2, n_c - 1), max(0, last - 1), last), ((0, 1), last, last)]:
        out.append(("22", hp, tile(I), tile(J)))
    while len(out) < 16:
        I, J = sorted(rng.integers(0, T, 2))
        out.append(("22", pairs[int(rng.integers(len(pairs)))], tile(int(I)), tile(int(J))))
    n12 = len(out)
    for c, I, J, sa, sb in [(n_c - 1, last, last, 1, 2), (n_c - 1, last, last, 0, 2), (0, 0, 0, 0, 0),
                            (0, 0, last, 3, 2), (n_c - 1, max(0, last - 1), last, 3, 0), (1, 0, 0, 2, 1),
                            (2, 0, last, 0, 3)]:
        out.append(("12", (c,), sub(I, sa), sub(J, sb)))
    while len(out) < n12 + 16:
        I, J = sorted(rng.integers(0, T, 2))
        out.append(("12", (int(rng.integers(n_c)),), sub(int(I), int(rng.integers(4))),
                    sub(int(J), int(rng.integers(4)))))
    n02 = len(out)
    lastw = nv - last * 64
    for I, J, la in [(last, last, 0), (last, last, lastw - 2), (last, last, lastw - 1),
                     (max(0, last - 1), last, 63), (0, 0, 0), (0, last, 5), (0, 0, 62)]:
        a = I * 64 + la
        out.append(("02", (), (a, a + 1), tile(J)))
    while len(out) < n02 + 16:
        I, J = sorted(rng.integers(0, T, 2))
        a = min(nv - 1, int(I) * 64 + int(rng.integers(64)))
        out.append(("02", (), (a, a + 1), tile(int(J))))
    return out


def blocks(co, c, E0):
    res = []
    for key, hole, ar, br in block_list(co.sp.n_c, len(co.V)):
        cl = (int(key[0]), int(key[1]))
        vs = sorted(set(range(*ar)) | set(range(*br)))
        if not vs or ar[0] >= ar[1] or br[0] >= br[1]:
            val = 0.0
        else:
            so = fullsize.sub_oracle(co, vs)
            pos = {v: i for i, v in enumerate(vs)}
            va = (pos[ar[0]], pos[ar[1] - 1] + 1)
            vb = (pos[br[0]], pos[br[1] - 1] + 1)
            val = fullsize.vv_class(so, cl, c, E0, core_sets=[hole], va=va, vb=vb)
        res.append({"class": key, "holes": list(hole), "a": list(ar), "b": list(br), "value": val})
        print("block %s %s a %s b %s: %.15e" % (key, hole, ar, br, val), flush=True)
    return res


def main():
    global _CO, _C, _E0
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--out", default=None, help="output path (default tests/golden/<name>_full_oracle.json)")
    args = ap.parse_args()
    pb = SP.config(args.name)
    path = args.out or os.path.join(HERE, "%s_full_oracle.json" % args.name)
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    t0 = time.time()
    hfc, slabs, W = fullsize.streamed_inputs(pb, chunk=args.chunk)
    _CO = fullsize.SlabOracle(run.space_of(pb), hfc, slabs, SP.weights(pb), W)
    del hfc, W
    print("%s: inputs streamed in %.0f s" % (args.name, time.time() - t0), flush=True)
    if "c_re" in out:
        # reference strings as active bit masks (correlated positions); a file
        # written with whole determinants is converted
        out["p_strings"] = [int(d) & _CO.sp.act_mask for d in out["p_strings"]]
        assert out["p_strings"] == [int(x) for x in _CO.P]
        c = np.array(out["c_re"]) + 1j * np.array(out["c_im"])
        _, E0 = _CO.reference(c)
        assert E0 == out["E0"]
    else:
        t1 = time.time()
        H, _ = _CO.reference(np.ones(len(_CO.P), dtype=np.complex128))
        w, v = np.linalg.eigh(H)
        c = v[:, 0]
        k = int(np.argmax(np.abs(c)))
        c = c * (abs(c[k]) / c[k])
        _, E0 = _CO.reference(c)
        out.update({
            "config": args.name,
            "generator": "synth.problems.config(%r), seed %d" % (args.name, pb.seed),
            "note": "oracle-only values (CPU FP64 oracle: class oracle on streamed factor columns, C loops for "
                    "the two-virtual classes); C is the lowest eigenvector of the oracle's H_PP in the oracle's "
                    "order (sorted active strings, bit masks over the correlated spinors)",
            "p_strings": [int(x) for x in _CO.P],
            "c_re": c.real.tolist(),
            "c_im": c.imag.tolist(),
            "gap": float(w[1] - w[0]),
            "E0": E0,
            "E0_minus_Ecore": E0 - _CO.energy_of(_CO.core),
            "parts": {},
            "seconds": {},
        })
        print("%s: reference state in %.0f s, E0 - E_core = %.12f" % (args.name, time.time() - t1,
                                                                     out["E0_minus_Ecore"]), flush=True)
    _C, _E0 = c, E0
    _CO.gOOOO
    _CO.gVOOO
    for cl in CLASSES[3:] + CLASSES[:3]:
        key = "%d%d" % cl
        if key in out["parts"]:
            continue
        t1 = time.time()
        if cl[1] == 2:
            val = fullsize.vv_class(_CO, cl, c, E0)
        else:
            val = small_class(cl, args.jobs)
        out["parts"][key] = val
        out["seconds"][key] = time.time() - t1
        out["E2"] = math.fsum(out["parts"].values()) if len(out["parts"]) == len(CLASSES) else None
        with open(path, "w") as f:
            json.dump(out, f)
        print("%s class %s: %.15e (%.0f s)" % (args.name, key, val, time.time() - t1), flush=True)
    print("%s E2 = %.15f" % (args.name, out["E2"]))
    if "blocks" not in out:
        t1 = time.time()
        out["blocks"] = blocks(_CO, c, E0)
        out["seconds"]["blocks"] = time.time() - t1
        with open(path, "w") as f:
            json.dump(out, f)
        print("%s: %d blocks in %.0f s" % (args.name, len(out["blocks"]), time.time() - t1), flush=True)


if __name__ == "__main__":
    main()
