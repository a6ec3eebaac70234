"""Oracle values for instances of the 64-instance uneven batch (c3).

Runs the CPU oracle only (packages `oracle` and `synth`), never the HIP
library.  For each selected instance s (synth.problems.batched_instance):
the lowest eigenvector C of the oracle's H_PP (phase fixed so that its
largest component is real and positive, stored in the oracle's order of
sorted determinant bit masks), E0, and E2 per excitation class (eq. pt2en,
Sec. 2.4, with the zeroth-order Hamiltonian of eq. zeroh).

The selection is the eight instances with the fewest external determinants
plus six of moderate size that cover the remaining shapes of the batch: two
and three DAS subspaces with 3, 4, 5 and 6 active electrons, several
64-wide virtual tiles with a ragged last tile.

Usage: python tests/golden/make_c3_golden.py [--jobs N]
Output: tests/golden/c3_oracle.json
"""
import argparse
import json
import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth.problems as SP  # noqa: E402
from oracle import run  # noqa: E402
from oracle.classes import CLASSES  # noqa: E402

SMALLEST = [7, 32, 35, 58, 27, 56, 11, 31]
SHAPES = [43, 63, 48, 4, 14, 0]


def one(s):
    import torch
    torch.set_num_threads(1)
    pb = SP.batched_instance(s)
    t0 = time.time()
    h, Bs = SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)]
    co = run.class_oracle(pb, h, Bs, SP.weights(pb))
    H, _ = co.reference(np.ones(len(co.P), dtype=np.complex128))
    w, v = np.linalg.eigh(H)
    c = v[:, 0]
    k = int(np.argmax(np.abs(c)))
    c = c * (abs(c[k]) / c[k])
    parts, E0 = co.e2(c, 0)
    out = {
        "seed": s,
        "shape": {"n_c": pb.n_c, "subs": pb.sub_sizes, "n_elec": pb.n_elec, "n_v": pb.n_v, "sets": pb.sets},
        "p_strings": [int(x) for x in co.P],
        "c_re": c.real.tolist(),
        "c_im": c.imag.tolist(),
        "gap": float(w[1] - w[0]) if len(w) > 1 else None,
        "E0": E0,
        "parts": {"%d%d" % cl: parts[cl] for cl in CLASSES},
        "E2": math.fsum(parts.values()),
        "oracle_seconds": time.time() - t0,
    }
    print("c3.%d E2 %.12f (%.1f s)" % (s, out["E2"], out["oracle_seconds"]), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    args = ap.parse_args()
    sel = SMALLEST + SHAPES
    with Pool(args.jobs) as pool:
        res = pool.map(one, sel, chunksize=1)
    out = {
        "generator": "synth.problems.batched_instance(s)",
        "note": "oracle-only values (class-resolved CPU FP64 oracle); C is the lowest eigenvector of the "
                "oracle's H_PP in the oracle's order (sorted determinant bit masks)",
        "instances": {str(r["seed"]): r for r in res},
    }
    with open(os.path.join(HERE, "c3_oracle.json"), "w") as f:
        json.dump(out, f)
    print("wrote", len(res), "instances")


if __name__ == "__main__":
    main()
