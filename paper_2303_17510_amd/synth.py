"""Seeded synthetic inputs for hybrid-dealiased convolutions.

This module generates data only: it holds none of the convolution's
arithmetic, so both the GPU path's tests and the CPU oracle can be fed from
it.  All draws are FP64 from numpy's PCG64; complex64 runs use the rounded
values (and the oracle is then fed those rounded values upcast to FP64).

Workload shapes follow the paper's benchmarks (Sec. 7): equal-length complex
inputs, A = 2 (or 3) inputs, B = 1 output, padding ratio 1/2 (M = 2L per
dimension) unless stated.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 17510000


def seed_for(config: int, a: int) -> int:
    """Seed of input ``a`` of workload ``config``: 17510000 + 100*config + a."""
    return SEED_BASE + 100 * int(config) + int(a)


def unit_disk(shape, seed: int) -> np.ndarray:
    """Complex128 entries uniform in the unit disk: r = sqrt(U1), theta = 2 pi U2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(np.prod(shape))
    u1 = rng.random(n)
    u2 = rng.random(n)
    z = np.sqrt(u1) * np.exp(2j * np.pi * u2)
    return z.reshape(shape)


def gaussian(shape, seed: int) -> np.ndarray:
    """Complex128 entries with independent N(0, 1) real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(np.prod(shape))
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return (re + 1j * im).reshape(shape)


def inputs(config: int, A: int, shape, dist: str = "disk", dtype=np.complex128):
    """The ``A`` seeded inputs of a workload, each of ``shape``.

    ``dtype`` complex64 rounds the FP64 draws; the returned arrays are of that
    dtype.  Use :func:`as_oracle` to get the values the oracle must see.
    """
    gen = unit_disk if dist == "disk" else gaussian
    return [gen(shape, seed_for(config, a)).astype(dtype) for a in range(A)]


def as_oracle(x) -> np.ndarray:
    """The exact values of ``x`` (complex64 or complex128) as complex128."""
    return np.asarray(x).astype(np.complex128)


def batched_lengths(count: int = 4096, lo_log2: float = 6.0, span_log2: float = 10.0,
                    seed: int = SEED_BASE + 300) -> np.ndarray:
    """Lengths L = round(2**(lo + span*U)), log-uniform in [2**lo, 2**(lo+span)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(int(count))
    return np.rint(2.0 ** (lo_log2 + span_log2 * u)).astype(np.int64)


def batched_inputs(Ls, A: int = 2, config_id: int = 2, dtype=np.complex128):
    """The A inputs of a batch of 1D convolutions of lengths ``Ls``, each
    drawn as one unit-disk array of sum(Ls) entries (seed of input ``a``:
    ``seed_for(config_id, a)``); convolution i uses the slice at offset
    sum(Ls[:i]).  ``dtype`` complex64 rounds the FP64 draws."""
    tot = int(np.sum(np.asarray(Ls, dtype=np.int64)))
    return [unit_disk((tot,), seed_for(config_id, a)).astype(dtype) for a in range(A)]
