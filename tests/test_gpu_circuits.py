"""Levelled gate DAGs on the GPU: the uneven-level workload (a 16-bit
ripple-carry adder and a 16x16 array multiplier, levels of width 1 to 273),
HIP-graph replay of a whole circuit, and the 16,384-gate mixed batch."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from conftest import encode, real_keys
from paper_2306_11006_amd import inputs, params

pytestmark = pytest.mark.gpu

FORMS = ("ntt", "int8")
THREADS = min(16, os.cpu_count() or 4)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def encrypt_wires(O, p, keys, bits, seed):
    d = inputs.encryption_draws(p, seed, len(bits))
    return np.stack([O.lwe_encrypt(keys["s"], d["a"][i], d["e"][i],
                                   encode(b)) for i, b in enumerate(bits)])


def circuit_inputs(p, keys, O, seed):
    nl, io = inputs.adder_multiplier_circuit(16)
    g = inputs.rng(seed)
    A, B, X, Y = (int(v) for v in g.integers(0, 1 << 16, size=4))
    bits = {}
    for name, val in zip("abxy", (A, B, X, Y)):
        for i, w in enumerate(io[name]):
            bits[w] = (val >> i) & 1
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    ins = sorted(bits)
    wires[ins] = encrypt_wires(O, p, keys, [bits[w] for w in ins], seed + 1)
    return nl, io, wires, (A, B, X, Y)


def decode(O, keys, wires, ws):
    return sum(O.lwe_decrypt(keys["s"], wires[w]) << i for i, w in
               enumerate(ws))


def oracle_circuit(O, p, keys, circ, wires):
    w = wires.copy()

    def one(gt):
        op, a, b, c, out = (int(v) for v in gt)
        return out, O.gate(p, op, keys["bsk"], keys["ksk"], w[a], w[b], w[c])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        for lv in circ.levels:
            for out, val in ex.map(one, lv):
                w[out] = val
    return w


def test_adder_multiplier_toy_bit_exact(O):
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p = params.TOY
    keys = real_keys(p, 5)
    nl, io, wires, (A, B, X, Y) = circuit_inputs(p, keys, O, 600)
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    assert circ.n_levels == 88
    want = oracle_circuit(O, p, keys, circ, wires)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    for form in FORMS:
        say(f"toy adder+multiplier, {circ.n_levels} levels, form={form}")
        w = cggi.to_device(wires)
        circ.run(ctx, form, w)
        torch.cuda.synchronize()
        got = cggi.to_host(w)
        assert np.array_equal(got, want), form
        assert decode(O, keys, got, io["sum"]) == A + B
        assert decode(O, keys, got, io["prod"]) == X * Y
    ctx.close()


def test_circuit_graph_replay_toy(O):
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p = params.TOY
    keys = real_keys(p, 5)
    nl, io, wires, (A, B, X, Y) = circuit_inputs(p, keys, O, 610)
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    for form in FORMS:
        say(f"toy circuit graph capture form={form}")
        w0 = cggi.to_device(wires)
        eager = w0.clone()
        circ.run(ctx, form, eager)
        torch.cuda.synchronize()
        want = cggi.to_host(eager)
        w = w0.clone()
        graph = circ.capture(ctx, form, w)
        for rep in range(2):
            w.copy_(w0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert np.array_equal(cggi.to_host(w), want), (form, rep)
        del graph
        assert decode(O, keys, want, io["prod"]) == X * Y
    ctx.close()


def test_adder_multiplier_default_decrypts(O):
    """Default sizes, real keys: both forms agree on every wire of the
    88-level circuit and the outputs decrypt to a+b and x*y."""
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p = params.DEFAULT
    keys = real_keys(p, 1)
    nl, io, wires, (A, B, X, Y) = circuit_inputs(p, keys, O, 620)
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    outs = {}
    for form in FORMS:
        say(f"default adder+multiplier form={form}")
        w = cggi.to_device(wires)
        graph = circ.capture(ctx, form, w)
        graph.replay()
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(w)
        del graph
    assert np.array_equal(outs["ntt"], outs["int8"])
    got = outs["int8"]
    assert decode(O, keys, got, io["sum"]) == A + B
    assert decode(O, keys, got, io["prod"]) == X * Y
    ctx.close()


def test_mixed_batch_16384_default(O):
    """16,384 independent gates, opcodes uniform over NAND/AND/OR/XOR/MUX
    (about 19.7k bootstraps) in one level: the forms agree on every output
    and sampled gates (one per opcode, plus first and last) equal the
    oracle."""
    import torch
    from paper_2306_11006_amd import cggi
    p = params.DEFAULT
    bsk, ksk = inputs.uniform_keys(p, 77)
    G = 16384
    gates = inputs.random_gate_batch(78, G)
    wires = np.zeros((4 * G, p.n + 1), dtype=np.uint32)
    wires[: 3 * G] = inputs.uniform_lwe(p, 79, 3 * G)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    d_gates = cggi.to_device(gates)
    outs = {}
    for form in FORMS:
        say(f"default 16384 mixed gates form={form}")
        w = cggi.to_device(wires)
        ctx.eval_level(form, d_gates, w)
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(w[3 * G:])
    assert np.array_equal(outs["ntt"], outs["int8"])
    pick = {0, G - 1}
    for op in range(5):
        pick.add(int(np.nonzero(gates[:, 0] == op)[0][0]))
    pick = sorted(pick)
    say(f"oracle on gates {pick}")

    def one(i):
        op, a, b, c, _ = (int(v) for v in gates[i])
        return O.gate(p, op, bsk, ksk, wires[a], wires[b], wires[c])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(one, pick))
    for i, wv in zip(pick, want):
        assert np.array_equal(outs["int8"][i], wv), i
    ctx.close()
