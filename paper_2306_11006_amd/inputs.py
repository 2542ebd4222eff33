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


class Netlist:
    """A gate netlist under construction: wires are integers, gates append
    in a valid sequential order (every input wire exists before the gate).
    Gate tuples are (opcode, in0, in1, in2, out) as in cggi_gate_t."""

    def __init__(self):
        self.gates = []
        self.n_wires = 0
        self.input_wires = []

    def inputs(self, k):
        ids = list(range(self.n_wires, self.n_wires + k))
        self.n_wires += k
        self.input_wires += ids
        return ids

    def gate(self, op, a=0, b=0, c=0):
        out = self.n_wires
        self.n_wires += 1
        self.gates.append((OPCODES[op], a, b, c, out))
        return out

    def array(self):
        return np.array(self.gates, dtype=np.int32).reshape(-1, 5)


def ripple_adder(nl, a, b):
    """Ripple-carry adder of two little-endian bit lists: half adder on bit
    0, then per bit p = a^b, s = p^c, carry = MUX(p, c, a).  Returns the sum
    bits and the carry out."""
    s = [nl.gate("XOR", a[0], b[0])]
    c = nl.gate("AND", a[0], b[0])
    for i in range(1, len(a)):
        p = nl.gate("XOR", a[i], b[i])
        s.append(nl.gate("XOR", p, c))
        c = nl.gate("MUX", p, c, a[i])
    return s, c


def _full_adder_nand(nl, x, y, z):
    """sum = x ^ y ^ z, carry = NAND(NAND(x, y), NAND(x ^ y, z))."""
    p = nl.gate("XOR", x, y)
    s = nl.gate("XOR", p, z)
    c = nl.gate("NAND", nl.gate("NAND", x, y), nl.gate("NAND", p, z))
    return s, c


def array_multiplier(nl, a, b):
    """Array multiplier of two n-bit little-endian operands: AND partial
    products, then one ripple row of full adders (XOR/NAND, half adders
    AND/XOR at the row ends) per partial-product row.  Returns 2n bits."""
    n = len(a)
    pp = [[nl.gate("AND", a[j], b[i]) for j in range(n)] for i in range(n)]
    out = [pp[0][0]]
    acc = pp[0][1:]                       # n-1 bits of weight 1..n-1
    carry_top = None
    for i in range(1, n):
        row = pp[i]
        new = []
        c = None
        for j in range(n):
            x = acc[j] if j < len(acc) else carry_top
            y = row[j]
            if x is None:
                s_, c_ = (y, None) if c is None else (
                    nl.gate("XOR", y, c), nl.gate("AND", y, c))
            elif c is None:
                s_, c_ = nl.gate("XOR", x, y), nl.gate("AND", x, y)
            else:
                s_, c_ = _full_adder_nand(nl, x, y, c)
            new.append(s_)
            c = c_
        out.append(new[0])
        acc = new[1:]
        carry_top = c
    out += acc
    out.append(nl.gate("CONST0") if carry_top is None else carry_top)
    return out


def adder_multiplier_circuit(bits=16):
    """The uneven-level workload: a bits-wide ripple-carry adder and a
    bits x bits array multiplier side by side (independent operands).
    Returns (netlist, dict of input/output wire lists)."""
    nl = Netlist()
    a, b = nl.inputs(bits), nl.inputs(bits)
    x, y = nl.inputs(bits), nl.inputs(bits)
    s, c = ripple_adder(nl, a, b)
    p = array_multiplier(nl, x, y)
    return nl, dict(a=a, b=b, x=x, y=y, sum=s + [c], prod=p)


def random_dag(seed, n_gates, max_width=65536, n_inputs=64,
               ops=("NAND", "AND", "OR", "XOR", "MUX")):
    """Random levelled DAG: level widths log-uniform in [1, max_width] until
    n_gates gates exist (the last level is cut to fit); every gate reads one
    wire of the previous level and the rest uniformly from all earlier
    wires; opcodes uniform over `ops`."""
    g = rng(seed)
    nl = Netlist()
    prev = nl.inputs(n_inputs)
    earlier = list(prev)
    codes = list(ops)
    while len(nl.gates) < n_gates:
        w = int(np.exp(g.uniform(0.0, np.log(max_width))))
        w = max(1, min(w, n_gates - len(nl.gates)))
        ops_l = g.integers(0, len(codes), size=w)
        first = g.integers(0, len(prev), size=w)
        rest = g.integers(0, len(earlier), size=(w, 2))
        cur = []
        for k in range(w):
            cur.append(nl.gate(codes[ops_l[k]], prev[first[k]],
                               earlier[rest[k, 0]], earlier[rest[k, 1]]))
        earlier += cur
        prev = cur
    return nl


def eval_plain(gates, values):
    """Evaluate a netlist on plaintext bits (dict or array indexed by wire),
    gates in the given (sequential) order.  Boolean logic only."""
    v = dict(values) if isinstance(values, dict) else {
        i: int(x) for i, x in enumerate(values)}
    for op, a, b, c, o in np.asarray(gates).tolist():
        if op == 0:
            r = 1 - (v[a] & v[b])
        elif op == 1:
            r = v[a] & v[b]
        elif op == 2:
            r = v[a] | v[b]
        elif op == 3:
            r = v[a] ^ v[b]
        elif op == 4:
            r = v[b] if v[a] else v[c]
        elif op == 5:
            r = 1 - v[a]
        elif op == 6:
            r = v[a]
        elif op == 7:
            r = 0
        elif op == 8:
            r = 1
        elif op == 9:
            r = 1 - (v[a] | v[b])
        elif op == 10:
            r = 1 - (v[a] ^ v[b])
        else:
            raise ValueError(op)
        v[o] = r
    return v
