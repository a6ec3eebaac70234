"""Seeded synthetic inputs with the structure of the paper's workloads.

The paper's calculations use molecular spinor integrals (Dyall basis sets,
Dirac-Coulomb(-Breit) Hamiltonians) that are not available here.  These
generators produce inputs with the same structure: an ordered spinor space
(frozen core | core | active DAS subspaces | kept virtuals), complex Hermitian
one-electron integrals with orbital energies on the diagonal, and two-electron
integrals in Cholesky form, one factor set per operator (Dirac-Coulomb,
Gaunt, gauge) with a real signed weight:

    (pq|rs) = sum_t w_t sum_L B[t][L,p,q] B[t][L,r,s],   B[t][L] Hermitian.

Recipe (every draw is counter based, see synth.rng):
  * core energies (frozen core included) U[-50,-1], sorted, frozen = lowest;
    active U[-0.5,0.1] sorted; virtual log-uniform on [v_lo, v_hi] sorted,
    keeping those <= v_cut (frozen virtuals are never generated);
  * h_pp = eps_p; h_pq (p<q) = x (1+i)/sqrt(2), x ~ N(0, 0.05^2); h_qp = conj;
  * B[t][L]_pq (p<q) ~ CN(0, 0.1^2) times exp(-|p-q|/8), diagonal real
    N(0, 0.1^2); B_qp = conj(B_pq);
  * weights: Dirac-Coulomb +1, Gaunt -scale, gauge +scale.

No part of the perturbation-theory arithmetic lives here.
"""
from dataclasses import dataclass, field
from typing import List, Tuple
import math

import torch

from . import rng

STRIDE = 1 << 16          # element index of (p, q) is p * STRIDE + q (p <= q)


@dataclass
class Problem:
    name: str
    seed: int
    n_fc: int                      # frozen core spinors (folded into h)
    n_c: int                       # correlated core spinors
    sub_sizes: List[int]           # active DAS subspace sizes, in order
    n_elec: int                    # active electrons
    base: List[int]                # base occupation per subspace
    max_hops: int                  # hop limit of the reference space
    n_v_gen: int                   # virtual spinors drawn
    v_lo: float = 0.2
    v_hi: float = 20.0
    v_cut: float = math.inf        # virtuals above this energy are frozen
    sets: List[Tuple[int, float]] = field(default_factory=list)  # (rank, weight)
    q_mode: int = 0

    @property
    def n_a(self) -> int:
        return sum(self.sub_sizes)

    def virtual_energies(self) -> torch.Tensor:
        key = rng.stream_key(self.seed, 0, 2)
        u = rng.uniform(key, torch.arange(self.n_v_gen, dtype=torch.int64))
        e = torch.exp(math.log(self.v_lo) + u * (math.log(self.v_hi) - math.log(self.v_lo)))
        e, _ = torch.sort(e)
        return e[e <= self.v_cut]

    @property
    def n_v(self) -> int:
        return int(self.virtual_energies().numel())

    @property
    def n(self) -> int:
        return self.n_fc + self.n_c + self.n_a + self.n_v

    @property
    def n_l(self) -> int:
        return sum(r for r, _ in self.sets)


def default_base(sub_sizes, n_elec):
    """Half filling per subspace; remaining electrons go one at a time to
    odd-sized subspaces first (in order), then to the others."""
    base = [s // 2 for s in sub_sizes]
    rem = n_elec - sum(base)
    order = [k for k, s in enumerate(sub_sizes) if s % 2 == 1] + \
            [k for k, s in enumerate(sub_sizes) if s % 2 == 0]
    while rem > 0:
        moved = False
        for k in order:
            if rem > 0 and base[k] < sub_sizes[k]:
                base[k] += 1
                rem -= 1
                moved = True
        if not moved:
            raise ValueError("too many electrons for the active space")
    while rem < 0:
        for k in reversed(order):
            if rem < 0 and base[k] > 0:
                base[k] -= 1
                rem += 1
    return base


def _split(total, parts):
    q, r = divmod(total, parts)
    return [q + (1 if k < r else 0) for k in range(parts)]


CAS = 1 << 20   # hop limit meaning "no limit"


def config(name: str) -> Problem:
    """The named workloads: c0 (tiny CAS), c1 (Ar-like), c2 (Kr-like),
    c4 (Xe-like, frozen core and frozen virtuals)."""
    if name == "c0":
        return Problem("c0", 0, 0, 6, [6], 3, [3], CAS, 24, sets=[(60, 1.0)])
    if name == "c1":
        return Problem("c1", 0, 0, 12, [4, 4, 4], 6, [2, 2, 2], 1, 200,
                       sets=[(600, 1.0), (200, -1e-2)])
    if name == "c2":
        return Problem("c2", 0, 0, 28, [4, 4, 4, 4], 8, [2, 2, 2, 2], 1, 600,
                       sets=[(1500, 1.0), (500, -1e-2), (500, 3e-3)])
    if name == "c4":
        subs = [3] * 6
        return Problem("c4", 0, 18, 28, subs, 8, default_base(subs, 8), 1, 1500,
                       v_hi=372.5, v_cut=50.0,
                       sets=[(2000, 1.0), (600, -1e-2), (600, 3e-3)])
    raise KeyError(name)


def batched_instance(s: int) -> Problem:
    """Instance s of the 64-instance uneven batch (core 4-20, active 6-12 at
    half filling in 2-3 subspaces with at most one hop, virtual 50-400,
    Dirac-Coulomb rank 3*n_orb plus Gaunt and gauge sets of rank n_orb)."""
    n_c = rng.randint(s, 900, 4, 21)[0]
    n_a = 2 * rng.randint(s, 901, 3, 7)[0]
    n_sub = rng.randint(s, 902, 2, 4)[0]
    n_v = rng.randint(s, 903, 50, 401)[0]
    subs = _split(n_a, n_sub)
    n_el = n_a // 2
    n_orb = n_c + n_a + n_v
    return Problem(f"c3.{s}", s, 0, n_c, subs, n_el, default_base(subs, n_el), 1, n_v,
                   sets=[(3 * n_orb, 1.0), (n_orb, -1e-2), (n_orb, 3e-3)])


def small(name, seed, n_fc, n_c, subs, n_elec, n_v, sets, max_hops=CAS, base=None):
    """A small problem for tests (CAS unless a hop limit is given)."""
    return Problem(name, seed, n_fc, n_c, list(subs), n_elec,
                   list(base) if base is not None else default_base(subs, n_elec),
                   max_hops, n_v, sets=list(sets))


# ----------------------------------------------------------------------------
# tensors

def orbital_energies(pb: Problem, device="cpu") -> torch.Tensor:
    n_core = pb.n_fc + pb.n_c
    kc = rng.stream_key(pb.seed, 0, 0)
    ec = -50.0 + 49.0 * rng.uniform(kc, torch.arange(n_core, dtype=torch.int64))
    ka = rng.stream_key(pb.seed, 0, 1)
    ea = -0.5 + 0.6 * rng.uniform(ka, torch.arange(pb.n_a, dtype=torch.int64))
    ec, _ = torch.sort(ec)
    ea, _ = torch.sort(ea)
    return torch.cat([ec, ea, pb.virtual_energies()]).to(device)


def _pair_index(n, device):
    p = torch.arange(n, dtype=torch.int64, device=device)
    lo = torch.minimum(p[:, None], p[None, :])
    hi = torch.maximum(p[:, None], p[None, :])
    return p, lo * STRIDE + hi


def one_body(pb: Problem, device="cpu") -> torch.Tensor:
    """h: complex128 [n, n], Hermitian, diagonal = orbital energies."""
    n = pb.n
    p, idx = _pair_index(n, device)
    z0, _ = rng.normal_pair(rng.stream_key(pb.seed, 1, 0), idx)
    x = 0.05 * z0 / math.sqrt(2.0)
    h = torch.complex(x, torch.where(p[:, None] < p[None, :], x, -x))
    eps = orbital_energies(pb, device)
    h = h * (1 - torch.eye(n, dtype=torch.float64, device=device)) + torch.diag(eps).to(h.dtype)
    return h


def factor_slice(pb: Problem, t: int, l0: int, l1: int, device="cpu") -> torch.Tensor:
    """Cholesky vectors L in [l0, l1) of factor set t: complex128 [l1-l0, n, n]."""
    n = pb.n
    p, idx = _pair_index(n, device)
    upper = (p[:, None] < p[None, :])
    diag = (p[:, None] == p[None, :])
    decay = torch.exp(-(p[:, None] - p[None, :]).abs().to(torch.float64) / 8.0)
    out = torch.empty((l1 - l0, n, n), dtype=torch.complex128, device=device)
    s_off = 0.1 / math.sqrt(2.0)
    for L in range(l0, l1):
        z0, z1 = rng.normal_pair(rng.stream_key(pb.seed, 100 + t, L), idx)
        re = torch.where(diag, 0.1 * z0, s_off * z0) * decay
        im = torch.where(diag, torch.zeros_like(z1), torch.where(upper, s_off * z1, -s_off * z1)) * decay
        out[L - l0] = torch.complex(re, im)
    return out


def factor_rows(pb: Problem, t: int, l0: int, l1: int, idx, device="cpu") -> torch.Tensor:
    """B[t][L][idx][:, idx] for L in [l0, l1): the same entries as
    factor_slice, generated only on the spinor subset idx (global indices)."""
    g = torch.as_tensor(list(idx), dtype=torch.int64, device=device)
    lo = torch.minimum(g[:, None], g[None, :])
    hi = torch.maximum(g[:, None], g[None, :])
    pidx = lo * STRIDE + hi
    upper = (g[:, None] < g[None, :])
    diag = (g[:, None] == g[None, :])
    decay = torch.exp(-(g[:, None] - g[None, :]).abs().to(torch.float64) / 8.0)
    m = len(idx)
    out = torch.empty((l1 - l0, m, m), dtype=torch.complex128, device=device)
    s_off = 0.1 / math.sqrt(2.0)
    for L in range(l0, l1):
        z0, z1 = rng.normal_pair(rng.stream_key(pb.seed, 100 + t, L), pidx)
        re = torch.where(diag, 0.1 * z0, s_off * z0) * decay
        im = torch.where(diag, torch.zeros_like(z1), torch.where(upper, s_off * z1, -s_off * z1)) * decay
        out[L - l0] = torch.complex(re, im)
    return out


def factors(pb: Problem, device="cpu"):
    """All factor sets: list of complex128 [rank_t, n, n]."""
    return [factor_slice(pb, t, 0, r, device) for t, (r, _) in enumerate(pb.sets)]


def weights(pb: Problem):
    return [w for _, w in pb.sets]


def complex_normal(seed: int, stream: int, shape, device="cpu") -> torch.Tensor:
    """CN(0,1) entries (real and imaginary parts N(0, 1/2))."""
    cnt = 1
    for s in shape:
        cnt *= s
    z0, z1 = rng.normal_pair(rng.stream_key(seed, stream, 0),
                             torch.arange(cnt, dtype=torch.int64, device=device))
    return torch.complex(z0, z1).reshape(shape) / math.sqrt(2.0)


def hermitian_direction(seed: int, stream: int, n: int, device="cpu") -> torch.Tensor:
    """A random Hermitian n x n direction with CN(0,1) off-diagonal and real
    N(0,1) diagonal entries, scaled to unit Frobenius norm."""
    z = complex_normal(seed, stream, (n, n), device)
    hz = 0.5 * (z + z.conj().T)
    return hz / torch.linalg.norm(hz)
