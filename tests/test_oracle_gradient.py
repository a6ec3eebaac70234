"""Pins of the oracle gradient (oracle.gradient) against facts fixed outside
it: central finite differences of the independent per-class oracle along
random directions, and exact identities of E2 (phase and scale invariance of
C, the diagonal shift of h, degree-1 homogeneity in (h, g), the orbital phase
gauge of core and virtual spinors).  CPU only."""
import math

import numpy as np
import pytest

import synth.problems as SP
from oracle import gradient, run

from helpers import oracle_reference, problem

CASES = ["s_fc", "s_das", "s_cas"]


def inputs(name):
    pb = problem(name)
    h = SP.one_body(pb).numpy()
    Bs = [B.numpy() for B in SP.factors(pb)]
    _, _, c, _ = oracle_reference(name)
    return pb, h, Bs, SP.weights(pb), np.asarray(c)


def class_oracle_e2(pb, h, Bs, ws, c, b=0.0):
    """E2 from the per-class oracle (oracle.classes), which shares no code
    with oracle.gradient's energy expression."""
    co = run.class_oracle(pb, h, Bs, ws)
    parts, _ = co.e2(c, b=b)
    return math.fsum(parts.values())


def herm_dir(rng, n):
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    z = 0.5 * (z + z.conj().T)
    return z / np.linalg.norm(z)


def fd(f, x, d, steps=(1e-4, 5e-5)):
    """Central differences at two steps with Richardson extrapolation."""
    v = [(f(x + s * d) - f(x - s * d)) / (2 * s) for s in steps]
    return (4 * v[1] - v[0]) / 3


@pytest.fixture(scope="module", params=CASES)
def case(request):
    name = request.param
    pb, h, Bs, ws, c = inputs(name)
    E2, E0, dh, dB, dc, _ = gradient.energy_and_gradient(run.space_of(pb), h, Bs, ws, pb.n_fc, c)
    return name, pb, h, Bs, ws, c, E2, dh, dB, dc


def test_value_matches_class_oracle(case):
    name, pb, h, Bs, ws, c, E2, *_ = case
    assert abs(E2 - class_oracle_e2(pb, h, Bs, ws, c)) <= 1e-12


def test_directional_derivatives_match_class_oracle_fd(case):
    name, pb, h, Bs, ws, c, E2, dh, dB, dc = case
    rng = np.random.default_rng(7)
    # h along Hermitian directions
    for _ in range(2):
        D = herm_dir(rng, h.shape[0])
        num = fd(lambda x: class_oracle_e2(pb, x, Bs, ws, c), h, D)
        ana = float(np.real(np.vdot(dh, D)))
        assert abs(num - ana) <= 1e-7 * max(1.0, abs(ana)), (name, "h", num, ana)
    # one Cholesky vector of every set along Hermitian directions
    for t in range(len(Bs)):
        L = int(rng.integers(Bs[t].shape[0]))
        D = np.zeros_like(Bs[t])
        D[L] = herm_dir(rng, h.shape[0])

        def f(x, t=t):
            bs = list(Bs)
            bs[t] = x
            return class_oracle_e2(pb, h, bs, ws, c)

        num = fd(f, Bs[t], D)
        ana = float(np.real(np.vdot(dB[t], D)))
        assert abs(num - ana) <= 1e-7 * max(1.0, abs(ana)), (name, "B", t, num, ana)
    # c along arbitrary complex directions
    for _ in range(2):
        D = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
        D /= np.linalg.norm(D)
        num = fd(lambda x: class_oracle_e2(pb, h, Bs, ws, x), c, D)
        ana = float(np.real(np.vdot(dc, D)))
        assert abs(num - ana) <= 1e-7 * max(1.0, abs(ana)), (name, "c", num, ana)


def test_identities(case):
    name, pb, h, Bs, ws, c, E2, dh, dB, dc = case
    scale = max(1.0, float(np.abs(dc).max()), float(np.abs(dh).max()))
    # E2 depends on C only through the ray: scale and phase directions vanish
    assert abs(np.real(np.vdot(dc, c))) <= 1e-12 * scale * np.linalg.norm(c)
    assert abs(np.real(np.vdot(dc, 1j * c))) <= 1e-12 * scale * np.linalg.norm(c)
    # h -> h + x I shifts E0 and every H_KK by x N_e
    assert abs(np.trace(dh).real) <= 1e-12 * scale * h.shape[0]
    # E2(l h, l g) = l E2 at fixed C, g quadratic in B
    euler = np.real(np.vdot(dh, h)) + 0.5 * sum(np.real(np.vdot(g, B)) for g, B in zip(dB, Bs))
    assert abs(euler - E2) <= 1e-11 * max(1.0, abs(E2))
    # orbital phase of a frozen-core, core or virtual spinor p (C unchanged):
    # d/dphi of U h U^H and U B U^H with U = exp(i phi E_pp) must vanish
    n = h.shape[0]
    n_act_lo = pb.n_fc + pb.n_c
    n_act_hi = n_act_lo + sum(pb.sub_sizes)
    for p in list(range(n_act_lo)) + list(range(n_act_hi, n)):
        E = np.zeros((n, n))
        E[p, p] = 1.0
        val = np.real(np.vdot(dh, 1j * (E @ h - h @ E)))
        for g, B in zip(dB, Bs):
            val += np.real(np.vdot(g, 1j * (E @ B - B @ E)))
        assert abs(val) <= 1e-11 * scale, (name, p, val)


@pytest.mark.parametrize("name", ["s_das"])
def test_level_shift_gradient_matches_class_oracle_fd(name):
    """Sec. 2.6 level shift (b = 2): value and directional derivatives of
    oracle.gradient against central differences of the per-class oracle."""
    b = 2.0
    pb, h, Bs, ws, c = inputs(name)
    E2, _, dh, dB, dc, _ = gradient.energy_and_gradient(run.space_of(pb), h, Bs, ws, pb.n_fc, c, b=b)
    assert abs(E2 - class_oracle_e2(pb, h, Bs, ws, c, b=b)) <= 1e-12
    assert abs(E2 - class_oracle_e2(pb, h, Bs, ws, c)) > 1e-8 * abs(E2)
    rng = np.random.default_rng(11)
    D = herm_dir(rng, h.shape[0])
    num = fd(lambda x: class_oracle_e2(pb, x, Bs, ws, c, b=b), h, D)
    ana = float(np.real(np.vdot(dh, D)))
    assert abs(num - ana) <= 1e-7 * max(1.0, abs(ana)), ("h", num, ana)
    L = int(rng.integers(Bs[0].shape[0]))
    DB = np.zeros_like(Bs[0])
    DB[L] = herm_dir(rng, h.shape[0])
    num = fd(lambda x: class_oracle_e2(pb, h, [x] + list(Bs[1:]), ws, c, b=b), Bs[0], DB)
    ana = float(np.real(np.vdot(dB[0], DB)))
    assert abs(num - ana) <= 1e-7 * max(1.0, abs(ana)), ("B", num, ana)
    Dc = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
    Dc /= np.linalg.norm(Dc)
    num = fd(lambda x: class_oracle_e2(pb, h, Bs, ws, x, b=b), c, Dc)
    ana = float(np.real(np.vdot(dc, Dc)))
    assert abs(num - ana) <= 1e-7 * max(1.0, abs(ana)), ("c", num, ana)
