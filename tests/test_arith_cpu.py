"""Integer-arithmetic netlists on plaintext bits: every adder and multiplier
design returns a + b and a * b for boundary and random operands at several
widths (1-bit full-adder truth table exhaustively), the circuits levelise
into the depths their designs promise, and the latency CLI refuses to run
without a GPU."""
import numpy as np
import pytest

from paper_2306_11006_amd import arith, cggi, inputs
from paper_2306_11006_amd.inputs import Netlist


def run(nl, io, A, B, out_key):
    bits = len(io["a"])
    vals = {}
    for i in range(bits):
        vals[io["a"][i]] = (A >> i) & 1
        vals[io["b"][i]] = (B >> i) & 1
    v = inputs.eval_plain(nl.array(), vals)
    return sum(v[w] << i for i, w in enumerate(io[out_key]))


def operands(bits, seed, count=40):
    top = (1 << bits) - 1
    fixed = [(0, 0), (top, top), (top, 1), (1, top), (top, 0),
             (1 << (bits - 1), 1 << (bits - 1))]
    g = np.random.default_rng(seed)
    rand = [tuple(int(x) for x in g.integers(0, top + 1, size=2, dtype=np.uint64))
            for _ in range(count)]
    return fixed + rand


@pytest.mark.parametrize("style", sorted(arith.ADDERS))
@pytest.mark.parametrize("bits", [1, 2, 3, 7, 16, 32])
def test_adders(style, bits):
    nl, io = arith.adder(bits, style)
    assert len(io["sum"]) == bits + 1
    for A, B in operands(bits, 100 + bits):
        assert run(nl, io, A, B, "sum") == A + B, (A, B)


@pytest.mark.parametrize("style", sorted(arith.MULTIPLIERS))
@pytest.mark.parametrize("bits", [1, 2, 3, 5, 8, 32])
def test_multipliers(style, bits):
    nl, io = arith.multiplier(bits, style)
    assert len(io["prod"]) == 2 * bits
    for A, B in operands(bits, 200 + bits, count=20 if bits == 32 else 40):
        assert run(nl, io, A, B, "prod") == A * B, (A, B)


def test_full_adder_truth_table():
    """The MUX carry of the full adder on all eight inputs."""
    nl = Netlist()
    x, y, z = nl.inputs(3)
    tb = arith._Timed(nl)
    s, c = arith._full_adder(tb, x, y, z)
    for v in range(8):
        bx, by, bz = v & 1, (v >> 1) & 1, v >> 2
        out = inputs.eval_plain(nl.array(), {x: bx, y: by, z: bz})
        assert out[s] == (bx + by + bz) & 1
        assert out[c] == (bx + by + bz) >> 1


def test_small_multipliers_exhaustive():
    for style in arith.MULTIPLIERS:
        nl, io = arith.multiplier(4, style)
        for A in range(16):
            for B in range(16):
                assert run(nl, io, A, B, "prod") == A * B, (style, A, B)


def depth(nl):
    order, start = cggi.levelize(nl.array(), nl.n_wires)
    return len(start) - 1


@pytest.mark.parametrize("bits", [4, 8, 16, 32, 64])
def test_prefix_adder_depth(bits):
    """Sklansky: one level of (g, p), log2(bits) prefix levels, one XOR."""
    nl, _ = arith.adder(bits, "prefix")
    assert depth(nl) == 2 + int(np.log2(bits))
    nl, _ = arith.adder(bits, "ripple")
    assert depth(nl) == bits


def test_multiplier_depths_32():
    """The 32-bit designs measured on the GPU: array 184 levels (5,888
    gates), Dadda 23 levels (4,277 gates); the Dadda tree takes 8 reduction
    stages of two levels each (heights 28, 19, 13, 9, 6, 4, 3, 2)."""
    nl, _ = arith.multiplier(32, "array")
    assert (depth(nl), len(nl.gates)) == (184, 5888)
    nl, _ = arith.multiplier(32, "tree")
    assert depth(nl) <= 1 + 2 * 8 + 2 + 6
    assert (depth(nl), len(nl.gates)) == (23, 4277)


def test_widths_must_match():
    nl = Netlist()
    a, b = nl.inputs(3), nl.inputs(4)
    with pytest.raises(ValueError):
        arith.sklansky_adder(nl, a, b)
    with pytest.raises(ValueError):
        arith.tree_multiplier(nl, a, b)


def test_latency_cli_needs_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2306_11006_amd import latency
    with pytest.raises(SystemExit, match="no GPU"):
        latency.main(["--op", "add"])


def test_uneven_level_circuit_for_the_latency_cli():
    """The latency CLI's uneven-level workload: a 16-bit ripple adder beside
    a 16 x 16 array multiplier, 1455 gates in 88 levels; its input and
    output wire lists compute a + b and x * y on plaintext bits."""
    from paper_2306_11006_amd import latency
    nl, ins, outs = latency.build("uneven", 16, "ripple+array")
    g = nl.array()
    order, starts = cggi.levelize(g, nl.n_wires)
    assert (len(g), len(ins), len(outs), len(starts) - 1) == \
        (1455, 64, 49, 88)
    for A, B, X, Y in [(0, 0, 0, 0), (65535, 65535, 65535, 65535),
                       (12345, 54321, 40000, 333)]:
        vals = {}
        for i in range(16):
            vals[ins[i]] = (A >> i) & 1
            vals[ins[16 + i]] = (B >> i) & 1
            vals[ins[32 + i]] = (X >> i) & 1
            vals[ins[48 + i]] = (Y >> i) & 1
        v = inputs.eval_plain(g, vals)
        s = sum(v[w] << i for i, w in enumerate(outs[:17]))
        p = sum(v[w] << i for i, w in enumerate(outs[17:]))
        assert (s, p) == (A + B, X * Y)
