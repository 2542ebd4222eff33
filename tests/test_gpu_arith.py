"""32-bit encrypted addition and multiplication on the GPU (the workloads of
ArctyrEX's Table 1, built from paper_2306_11006_amd.arith): real keys at
the default sizes, both forms agree on every wire of every circuit, the
output wires decrypt to a + b and a * b, and sampled gates equal the oracle
gate applied to the GPU's own input wires."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from conftest import encrypt_bits, real_keys
from paper_2306_11006_amd import arith, inputs, params

pytestmark = pytest.mark.gpu

FORMS = ("int8", "ntt")
THREADS = min(16, os.cpu_count() or 4)
BITS = 32


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    from paper_2306_11006_amd import cggi
    p = params.DEFAULT
    keys = real_keys(p, 5)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    yield p, keys, ctx
    ctx.close()


CASES = [("add", "prefix"), ("add", "ripple"), ("mul", "tree"),
         ("mul", "array")]


@pytest.mark.parametrize("op,style", CASES)
def test_arith_32(O, setup, op, style):
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p, keys, ctx = setup
    if op == "add":
        nl, io = arith.adder(BITS, style)
        out_wires = io["sum"]
    else:
        nl, io = arith.multiplier(BITS, style)
        out_wires = io["prod"]
    g = inputs.rng(5100 + len(nl.gates))
    A, B = (int(v) for v in g.integers(0, 1 << BITS, size=2, dtype=np.uint64))
    ins = list(io["a"]) + list(io["b"])
    bits = [(A >> i) & 1 for i in range(BITS)] + \
        [(B >> i) & 1 for i in range(BITS)]
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    wires[ins] = encrypt_bits(p, keys, bits, seed=5200 + len(nl.gates))
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    outs = {}
    for form in FORMS:
        say(f"{op}{BITS}-{style} form={form} levels={circ.n_levels} "
            f"gates={len(circ.gates)}")
        w = cggi.to_device(wires)
        circ.run(ctx, form, w)
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(w)
    assert np.array_equal(outs["int8"], outs["ntt"])
    got = outs["int8"]
    value = sum(O.lwe_decrypt(keys["s"], got[w]) << i
                for i, w in enumerate(out_wires))
    assert value == (A + B if op == "add" else A * B), (A, B, value)
    # sampled gates: first, last, and spread over the levels and opcodes
    gates = circ.gates
    pick = sorted({0, len(gates) - 1, len(gates) // 2,
                   int(np.flatnonzero(gates[:, 0] == 4)[0])
                   if (gates[:, 0] == 4).any() else 0,
                   *(int(x) for x in g.integers(0, len(gates), size=4))})

    def one(k):
        op_, a, b, c, _ = (int(v) for v in gates[k])
        return O.gate(p, op_, keys["bsk"], keys["ksk"], got[a], got[b],
                      got[c])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(one, pick))
    for k, wv in zip(pick, want):
        assert np.array_equal(got[int(gates[k, 4])], wv), k
