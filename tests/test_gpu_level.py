"""cggi_eval_level on the GPU: every gate of the paper's gate set against the
oracle (bit-exact), invalid gates skipped, and HIP-graph replay identical to
eager execution."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from conftest import encrypt_bits, real_keys
from paper_2306_11006_amd import inputs, params

pytestmark = pytest.mark.gpu

FORMS = ("ntt", "int8")
OPS = ["NAND", "AND", "OR", "XOR", "NOR", "XNOR", "MUX", "NOT", "COPY",
       "CONST0", "CONST1"]
CODE = {k: i for i, k in enumerate(["NAND", "AND", "OR", "XOR", "MUX", "NOT",
                                    "COPY", "CONST0", "CONST1", "NOR",
                                    "XNOR"])}
THREADS = min(16, os.cpu_count() or 4)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def build_level(p, keys, seed, reps=2):
    """Input wires encrypting random bits, and one gate of every opcode per
    repetition reading them; returns (wires [W][n+1], gates [G][5], bits)."""
    g = inputs.rng(seed)
    n_in = 3 * len(OPS) * reps
    bits = g.integers(0, 2, size=n_in).tolist()
    cts = encrypt_bits(p, keys, bits, seed=seed + 1)
    gates = []
    for r in range(reps):
        for k, op in enumerate(OPS):
            base = 3 * (r * len(OPS) + k)
            gates.append([CODE[op], base, base + 1, base + 2,
                          n_in + len(gates)])
    W = n_in + len(gates)
    wires = np.zeros((W, p.n + 1), dtype=np.uint32)
    wires[:n_in] = cts
    return wires, np.array(gates, dtype=np.int32), bits


def oracle_level(O, p, keys, wires, gates):
    def one(gt):
        op, a, b, c, _ = (int(v) for v in gt)
        return O.gate(p, op, keys["bsk"], keys["ksk"], wires[a], wires[b],
                      wires[c])
    with cf.ThreadPoolExecutor(THREADS) as ex:
        return np.stack(list(ex.map(one, gates)))


def truth(op, a, b, c):
    return {"NAND": 1 - (a & b), "AND": a & b, "OR": a | b, "XOR": a ^ b,
            "NOR": 1 - (a | b), "XNOR": 1 - (a ^ b), "MUX": b if a else c,
            "NOT": 1 - a, "COPY": a, "CONST0": 0, "CONST1": 1}[op]


@pytest.fixture(scope="module")
def toy(O):
    import torch
    from paper_2306_11006_amd import cggi
    assert torch.cuda.is_available()
    p = params.TOY
    keys = real_keys(p, 3)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    yield p, keys, ctx
    ctx.close()


def run_level(ctx, form, wires, gates):
    import torch
    from paper_2306_11006_amd import cggi
    w = cggi.to_device(wires)
    ctx.eval_level(form, cggi.to_device(gates), w)
    torch.cuda.synchronize()
    return cggi.to_host(w)


def test_level_every_gate_bit_exact_toy(O, toy):
    p, keys, ctx = toy
    wires, gates, bits = build_level(p, keys, seed=500)
    want = oracle_level(O, p, keys, wires, gates)
    for form in FORMS:
        say(f"toy eval_level form={form} G={len(gates)}")
        got = run_level(ctx, form, wires, gates)
        assert np.array_equal(got[gates[:, 4]], want), form
        assert np.array_equal(got[: gates[0, 4]], wires[: gates[0, 4]])
        for gt in gates:
            op = [k for k, v in CODE.items() if v == gt[0]][0]
            a, b, c = bits[gt[1]], bits[gt[2]], bits[gt[3]]
            assert O.lwe_decrypt(keys["s"], got[gt[4]]) == truth(op, a, b, c)


def test_level_invalid_gates_are_skipped(O, toy):
    p, keys, ctx = toy
    wires, gates, _ = build_level(p, keys, seed=510, reps=1)
    W = wires.shape[0]
    bad = gates.copy()
    bad[0, 1] = W + 5            # input out of range
    bad[1, 4] = -1               # output out of range
    bad[2, 0] = 99               # unknown opcode
    marker = np.full(p.n + 1, 0xDEADBEEF, dtype=np.uint32)
    wires = wires.copy()
    wires[bad[0, 4]] = marker
    wires[bad[2, 4]] = marker
    want = oracle_level(O, p, keys, wires, gates[3:])
    for form in FORMS:
        say(f"toy eval_level invalid gates form={form}")
        got = run_level(ctx, form, wires, bad)
        assert np.array_equal(got[bad[0, 4]], marker)
        assert np.array_equal(got[bad[2, 4]], marker)
        assert np.array_equal(got[gates[3:, 4]], want)


def test_level_graph_replay_matches_eager(O, toy):
    import torch
    from paper_2306_11006_amd import cggi
    p, keys, ctx = toy
    wires, gates, _ = build_level(p, keys, seed=520)
    ctx.reserve(len(gates))
    d_gates = cggi.to_device(gates)
    for form in FORMS:
        say(f"toy eval_level graph capture form={form}")
        eager = run_level(ctx, form, wires, gates)
        w0 = cggi.to_device(wires)
        w = w0.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.eval_level(form, d_gates, w)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            ctx.eval_level(form, d_gates, w)
        for rep in range(3):
            w.copy_(w0)                       # eager work between replays
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert np.array_equal(cggi.to_host(w), eager), (form, rep)
        del graph


def test_level_default_sizes_mixed_gates(O):
    """Default parameters with real keys: one gate of every opcode, both
    forms bit-exact against the oracle and decrypting correctly."""
    import torch
    from paper_2306_11006_amd import cggi
    p = params.DEFAULT
    keys = real_keys(p, 1)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    wires, gates, bits = build_level(p, keys, seed=530, reps=1)
    want = oracle_level(O, p, keys, wires, gates)
    for form in FORMS:
        say(f"default eval_level form={form} G={len(gates)}")
        got = run_level(ctx, form, wires, gates)
        assert np.array_equal(got[gates[:, 4]], want), form
    ctx.close()
