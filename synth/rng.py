"""Counter-based random numbers that give the same stream on any torch device.

Each value is a pure function of (seed, stream, slice, element index), so any
slice of a large tensor (one Cholesky vector, one block of rows) can be
regenerated on its own, on the CPU or on the GPU, without generating the rest.

The mixing function is SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014; finaliser constants
as published by S. Vigna).  All arithmetic is done on int64 tensors with
wrap-around multiplication; logical right shifts are emulated with a mask.
Uniforms take the top 53 bits; normals use the Box-Muller transform
(G. Box, M. Muller, 1958).  The integer part is bit-exact across devices; the
float transforms (log, cos, sin) may differ in the last bit between CPU and
GPU libraries, far below any tolerance used with these inputs.

This module holds no part of the perturbation-theory arithmetic.
"""
import math

import torch

_TWO64 = 1 << 64


def _signed(x: int) -> int:
    x &= _TWO64 - 1
    return x - _TWO64 if x >= (1 << 63) else x


_GOLDEN = _signed(0x9E3779B97F4A7C15)
_MIX1 = _signed(0xBF58476D1CE4E5B9)
_MIX2 = _signed(0x94D049BB133111EB)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix64(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function applied to state z (int64 tensor)."""
    z = z + _GOLDEN
    z = (z ^ _srl(z, 30)) * _MIX1
    z = (z ^ _srl(z, 27)) * _MIX2
    return z ^ _srl(z, 31)


def splitmix64_int(z: int) -> int:
    """Pure-Python SplitMix64 on unsigned 64-bit integers (reference form)."""
    m = _TWO64 - 1
    z = (z + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int, sub: int = 0) -> int:
    """Key of the stream (seed, stream, sub) as a signed 64-bit Python int."""
    k = splitmix64_int(seed & (_TWO64 - 1))
    k = splitmix64_int(k ^ (stream & (_TWO64 - 1)))
    k = splitmix64_int(k ^ (sub & (_TWO64 - 1)))
    return _signed(k)


def raw_bits(key: int, index: torch.Tensor) -> torch.Tensor:
    """64 random bits (as int64) for each element index of stream `key`."""
    return splitmix64(index * _GOLDEN + key)


def uniform(key: int, index: torch.Tensor) -> torch.Tensor:
    """U[0,1) doubles from the top 53 bits."""
    return _srl(raw_bits(key, index), 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def normal_pair(key: int, index: torch.Tensor):
    """Two independent N(0,1) doubles per element index (Box-Muller)."""
    u1 = uniform(key, 2 * index)
    u2 = uniform(key, 2 * index + 1)
    r = torch.sqrt(-2.0 * torch.log1p(-u1))
    th = (2.0 * math.pi) * u2
    return r * torch.cos(th), r * torch.sin(th)


def randint(seed: int, stream: int, lo: int, hi: int, count: int = 1):
    """`count` integers uniform in [lo, hi) for stream (seed, stream)."""
    key = stream_key(seed, stream)
    u = uniform(key, torch.arange(count, dtype=torch.int64))
    return [lo + min(int(x * (hi - lo)), hi - lo - 1) for x in u.tolist()]
