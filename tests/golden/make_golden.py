"""Write oracle reference values for the GPU parity tests.

Runs the CPU oracle only (packages `oracle` and `synth`), never the HIP
library.  Usage: python tests/golden/make_golden.py c1
Output: tests/golden/<name>_oracle.json with the reference coefficients
(oracle order, lowest eigenvector of the oracle's H_PP), E0, and E2 per
excitation class.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth.problems as SP  # noqa: E402
from oracle import run  # noqa: E402
from oracle.classes import CLASSES  # noqa: E402


def main(name):
    pb = SP.config(name)
    h, Bs = SP.one_body(pb).numpy(), [B.numpy() for B in SP.factors(pb)]
    co = run.class_oracle(pb, h, Bs, SP.weights(pb))
    H, _ = co.reference(np.ones(len(co.P), dtype=np.complex128))
    w, v = np.linalg.eigh(H)
    c = v[:, 0]
    k = int(np.argmax(np.abs(c)))
    c = c * (abs(c[k]) / c[k])
    t0 = time.time()
    parts, E0 = co.e2(c, 0)
    out = {
        "config": name,
        "generator": "synth.problems.config(%r), seed %d" % (name, pb.seed),
        "note": "oracle-only values (class-resolved CPU FP64 oracle); C is the lowest eigenvector "
                "of the oracle's H_PP in the oracle's order (sorted determinant bit masks)",
        "p_strings": [int(x) for x in co.P],
        "c_re": c.real.tolist(),
        "c_im": c.imag.tolist(),
        "E0": E0,
        "parts": {"%d%d" % cl: parts[cl] for cl in CLASSES},
        "E2": math.fsum(parts.values()),
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "%s_oracle.json" % name), "w") as f:
        json.dump(out, f, indent=0)
    print(name, out["E2"], out["oracle_seconds"])


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c1"]:
        main(nm)
