"""Counter-based Philox4x32-10 generator and the complex Gaussians drawn from it.

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 128-bit counter is
mixed with a 64-bit key by ten rounds of two 32x32->64-bit multiplies, with the
key bumped by the Weyl constants between rounds.  Every output depends only on
(counter, key), so any element of any synthetic array can be regenerated on its
own, on the CPU or on a GPU, without generating the rest.

All arithmetic is done on int64 torch tensors holding unsigned 32-bit values,
so the integer stream is bit-identical on every device.  Only the final
Box-Muller step uses floating-point transcendental functions (log, cos, sin);
those may differ by an ulp between devices.

This module holds no arithmetic of the solver; it only makes inputs.
"""
from __future__ import annotations

import torch

M32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def _mulhilo(a: int, b: torch.Tensor):
    """(hi, lo) 32-bit halves of the 64-bit product a*b, a a 32-bit constant.

    b is split into 16-bit halves so that no partial product exceeds 2^48 and
    int64 never overflows.
    """
    b_lo = b & 0xFFFF
    b_hi = b >> 16
    t0 = b_lo * a                       # < 2^48
    t1 = b_hi * a                       # < 2^48
    mid = t0 + ((t1 & 0xFFFF) << 16)    # < 2^49
    lo = mid & M32
    hi = (t1 >> 16) + (mid >> 32)
    return hi & M32, lo


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Apply Philox4x32-10 to counters (c0..c3) (int64 tensors of uint32 values).

    Returns four int64 tensors of uint32 outputs.
    """
    k0 = int(k0) & M32
    k1 = int(k1) & M32
    for r in range(10):
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if r < 9:
            k0 = (k0 + PHILOX_W0) & M32
            k1 = (k1 + PHILOX_W1) & M32
    return c0, c1, c2, c3


def complex_normal(index: torch.Tensor, stream: int, seed: int,
                   sub: int = 0) -> torch.Tensor:
    """One standard complex Gaussian per entry of `index` (E|z|^2 = 1).

    Counter = (index low 32 bits, index high 32 bits, stream, sub), key = seed.
    The two 53-bit uniforms u1, u2 (each from two output words) feed the
    Box-Muller transform z = sqrt(-2 ln u1) exp(2 pi i u2) / sqrt(2).
    The result is complex128 on index's device.
    """
    index = index.to(torch.int64)
    c0 = index & M32
    c1 = (index >> 32) & M32
    c2 = torch.full_like(index, int(stream) & M32)
    c3 = torch.full_like(index, int(sub) & M32)
    seed = int(seed)
    o0, o1, o2, o3 = philox4x32_10(c0, c1, c2, c3, seed & M32, (seed >> 32) & M32)
    two53 = float(2 ** 53)
    u1 = ((o0 >> 5) * (1 << 26) + (o1 >> 6)).to(torch.float64)
    u2 = ((o2 >> 5) * (1 << 26) + (o3 >> 6)).to(torch.float64)
    u1 = (u1 + 0.5) / two53            # in (0, 1): log is finite
    u2 = (u2 + 0.5) / two53
    r = torch.sqrt(-2.0 * torch.log(u1)) * (0.5 ** 0.5)
    ang = (2.0 * torch.pi) * u2
    return torch.complex(r * torch.cos(ang), r * torch.sin(ang))
