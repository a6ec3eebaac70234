"""Reference state and E0 for the sampled full-size parity checks (c2, c4).

Oracle only.  The reference vector is C = e_beta + 0.05 z, with beta the
reference determinant of lowest diagonal energy and z a CN(0,1) vector from
the synthetic generator (seed 7, stream 900); both sides regenerate it.  E0
(relative to the core energy) comes from the oracle's dense H_PP on the
sub-problem of frozen core + core + active spinors (E0 depends on nothing
else).  Usage: python tests/golden/make_sampled_reference.py c2 c4
Output: tests/golden/<name>_sampled_ref.json
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth.problems as SP  # noqa: E402
from oracle import run  # noqa: E402
from oracle.classes import ClassOracle  # noqa: E402
from oracle.space import ActiveSpace  # noqa: E402

NOISE_SEED, NOISE_STREAM, NOISE_SCALE = 7, 900, 0.05


def occupied_subproblem(pb):
    """Oracle on frozen core + core + active spinors only."""
    n_occ = pb.n_fc + pb.n_c + pb.n_a
    idx = list(range(n_occ))
    h = SP.one_body(pb)[idx][:, idx].numpy()
    Bs = [SP.factor_rows(pb, t, 0, r, idx).numpy() for t, (r, _) in enumerate(pb.sets)]
    ws = SP.weights(pb)
    hfc, Bc = run.correlated_inputs(h, Bs, ws, pb.n_fc)
    sp = ActiveSpace(pb.n_c, pb.sub_sizes, pb.n_elec, pb.base, pb.max_hops, 0)
    return ClassOracle(sp, hfc, Bc, ws)


def reference_vector(P_sorted, beta):
    """C over the oracle's sorted reference list."""
    z = SP.complex_normal(NOISE_SEED, NOISE_STREAM, (len(P_sorted),)).numpy()
    c = NOISE_SCALE * z
    c[P_sorted.index(beta)] += 1.0
    return c


def main(name):
    pb = SP.config(name)
    t0 = time.time()
    co = occupied_subproblem(pb)
    diag = [co.energy_of(co.core | a) for a in co.P]
    beta = co.P[int(np.argmin(diag))]
    c = reference_vector(co.P, beta)
    H, E0 = co.reference(c)
    out = {"config": name, "beta": int(beta), "noise": [NOISE_SEED, NOISE_STREAM, NOISE_SCALE],
           "E0_minus_Ecore": E0 - co.energy_of(co.core), "n_ref": len(co.P),
           "note": "oracle-only; C = e_beta + 0.05 z over the oracle's sorted reference list",
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "%s_sampled_ref.json" % name), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c2", "c4"]:
        main(nm)
