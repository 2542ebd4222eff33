"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws random numbers and builds gate netlists; it holds
none of the scheme's arithmetic.  Random numbers the scheme consumes (key
bits, uniform masks, rounded Gaussian noise) are drawn here and handed to
whichever side needs them, so both sides see identical inputs.

All generators use numpy's PCG64 seeded explicitly.
"""
import numpy as np

from .params import Params


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_u32(g: np.random.Generator, shape) -> np.ndarray:
    return g.integers(0, 1 << 32, size=shape, dtype=np.uint64).astype(np.uint32)


def aligned_u32(g: np.random.Generator, shape, shift: int) -> np.ndarray:
    """Uniform multiples of 2^shift (torus values with zero low bits)."""
    hi = g.integers(0, 1 << (32 - shift), size=shape, dtype=np.uint64)
    return (hi << np.uint64(shift)).astype(np.uint32)


def gaussian_i32(g: np.random.Generator, shape, noise_log2) -> np.ndarray:
    """Rounded Gaussian torus noise: round(2^(32 - x) * z), z ~ N(0, 1).
    ``noise_log2=None`` gives zeros (noiseless test keys)."""
    if noise_log2 is None:
        return np.zeros(shape, dtype=np.int32)
    z = g.standard_normal(size=shape)
    return np.rint(z * float(2 ** (32 - noise_log2))).astype(np.int64) \
        .astype(np.int32)


def binary(g: np.random.Generator, shape) -> np.ndarray:
    return g.integers(0, 2, size=shape, dtype=np.uint8)


def key_draws(p: Params, seed: int, bk_noise=True, ks_noise=True,
              aligned_bsk=False):
    """Random draws for key generation: LWE key s, TRLWE key K, the uniform
    masks and noises of every bootstrapping-key row and key-switching-key
    row.  ``aligned_bsk`` draws bsk masks as multiples of 2^(32 - l*beta)
    (noiseless closed-form tests)."""
    g = rng(seed)
    s = binary(g, (p.n,))
    K = binary(g, (p.N,))
    bshape = (p.n, 2 * p.l, p.N)
    if aligned_bsk:
        bsk_a = aligned_u32(g, bshape, 32 - p.l * p.bg_bit)
    else:
        bsk_a = uniform_u32(g, bshape)
    bsk_e = gaussian_i32(g, bshape, p.bk_noise_log2 if bk_noise else None)
    kshape = (p.N, p.ks_t, p.ks_base)
    ksk_a = uniform_u32(g, kshape + (p.n,))
    ksk_e = gaussian_i32(g, kshape, p.lwe_noise_log2 if ks_noise else None)
    return dict(s=s, K=K, bsk_a=bsk_a, bsk_e=bsk_e, ksk_a=ksk_a, ksk_e=ksk_e)


def encryption_draws(p: Params, seed: int, count: int, noise=True):
    """Masks and noises for ``count`` fresh LWE encryptions, plus random
    plaintext bits."""
    g = rng(seed)
    a = uniform_u32(g, (count, p.n))
    e = gaussian_i32(g, (count,), p.lwe_noise_log2 if noise else None)
    bits = binary(g, (count,))
    return dict(a=a, e=e, bits=bits)


def uniform_keys(p: Params, seed: int):
    """Uniform bsk and ksk of the right shapes.  Under the LWE assumption
    real keys are indistinguishable from these, and every kernel's work is
    independent of key values, so they serve throughput runs where no
    decryption is checked."""
    g = rng(seed)
    bsk = uniform_u32(g, p.bsk_shape)
    ksk = uniform_u32(g, p.ksk_shape)
    return bsk, ksk


def uniform_lwe(p: Params, seed: int, count: int, dim=None) -> np.ndarray:
    """``count`` uniform LWE ciphertexts of dimension ``dim`` (default n);
    real ciphertexts are indistinguishable from these."""
    dim = p.n if dim is None else dim
    return uniform_u32(rng(seed), (count, dim + 1))


# ---------------------------------------------------------------------------
# Gate netlists (structure only)
# ---------------------------------------------------------------------------

OPCODES = {"NAND": 0, "AND": 1, "OR": 2, "XOR": 3, "MUX": 4, "NOT": 5,
           "COPY": 6, "CONST0": 7, "CONST1": 8, "NOR": 9, "XNOR": 10}
BOOTSTRAPS = {0: 1, 1: 1, 2: 1, 3: 1, 4: 2, 5: 0, 6: 0, 7: 0, 8: 0, 9: 1,
              10: 1}


def random_gate_batch(seed: int, count: int, ops=("NAND", "AND", "OR", "XOR",
                                                   "MUX")):
    """``count`` independent gates with opcodes uniform over ``ops``; gate g
    reads wires 3g, 3g+1, 3g+2 and writes wire 3*count + g."""
    g = rng(seed)
    codes = np.array([OPCODES[o] for o in ops], dtype=np.int32)
    op = codes[g.integers(0, len(codes), size=count)]
    idx = np.arange(count, dtype=np.int32)
    gates = np.stack([op, 3 * idx, 3 * idx + 1, 3 * idx + 2,
                      3 * count + idx], axis=1).astype(np.int32)
    return gates
