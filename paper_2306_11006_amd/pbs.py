"""Programmable bootstrapping: lookup tables over small messages.

The blind rotation turns an LWE ciphertext of phase phi into one of
coefficient 0 of X^(-phi~) * v, phi~ = round(2N * phi / 2^32) (Section 2.2,
Fig. 1): v[phi~] for phi~ in [0, N), -v[phi~ - N] above.  Gate bootstrapping
uses v = 1/8 everywhere; choosing v per coefficient evaluates any function
f: Z_p -> Z_p on an encrypted multi-bit message.  Section 2.2 notes that
CGGI supports such programmable bootstrapping of multi-bit encodings, which
the paper leaves out (it works with encrypted bits) while stating that its
method extends to it; the batched kernels here run it unchanged, with the
test polynomial as an argument.

Encoding (message m in [0, p), one padding bit): phase m * delta with
delta = 2^32 / (2p), so valid phases stay below 1/2 and phi~ = m N / p (+
noise) stays in [0, N).  The test polynomial holds delta * f(m) on the box of
N/p coefficients centred on m N / p; the lower half-box of m = 0 sits at the
top of [N, 2N) and is reached through the negacyclic wrap, so the top N/(2p)
coefficients of v hold -delta * f(0).
"""
import numpy as np


def delta(p_msg: int) -> int:
    """Torus step of one message unit (one padding bit)."""
    if p_msg < 2 or p_msg & (p_msg - 1):
        raise ValueError("message modulus must be a power of two >= 2")
    return (1 << 32) // (2 * p_msg)


def encode(m: int, p_msg: int) -> int:
    """Plaintext phase (uint32) of message m in [0, p_msg)."""
    return (int(m) % p_msg) * delta(p_msg)


def decode(phase: int, p_msg: int, padding: bool = False) -> int:
    """Message nearest to a uint32 phase: in [0, p) ignoring the padding
    bit, or in [0, 2p) with it (a valid ciphertext has it clear)."""
    q = int(round((int(phase) % (1 << 32)) / delta(p_msg)))
    return q % (2 * p_msg) if padding else q % p_msg


def lut_test_vector(f, p_msg: int, N: int) -> np.ndarray:
    """uint32 [N] test polynomial evaluating f: Z_p -> Z_p (a callable or a
    length-p sequence) under one programmable bootstrap."""
    table = [int(f(m)) if callable(f) else int(f[m]) for m in range(p_msg)]
    box = N // p_msg
    if box < 2:
        raise ValueError("N must hold at least two coefficients per message")
    d = delta(p_msg)
    v = np.empty(N, dtype=np.uint64)
    for j in range(N):
        m = (j + box // 2) // box            # box centred on m * N / p
        if m < p_msg:
            v[j] = (table[m] % p_msg) * d
        else:                                 # wrap: -v[j] seen at j + N
            v[j] = ((1 << 32) - (table[0] % p_msg) * d) % (1 << 32)
    return v.astype(np.uint32)
