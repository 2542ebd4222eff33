"""Edge cases of the GPU path: a level of bootstrap-free gates only (the
bootstrap launch sees a device count of zero), an empty level, the largest
LWE dimension the int8 form's LDS layout admits at N=1024 (n=1023), and the
widest level of the large random-DAG recipe (65,536 gates) at the default
sizes."""
import concurrent.futures as cf
import dataclasses
import os
import sys

import numpy as np
import pytest

from conftest import encrypt_bits, real_keys
from paper_2306_11006_amd import inputs, params

pytestmark = pytest.mark.gpu

FORMS = ("ntt", "int8")
THREADS = min(16, os.cpu_count() or 4)
NOT, COPY, CONST0, CONST1, NAND = 5, 6, 7, 8, 0


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_level(ctx, form, wires, gates):
    import torch
    from paper_2306_11006_amd import cggi
    w = cggi.to_device(wires)
    ctx.eval_level(form, cggi.to_device(gates), w)
    torch.cuda.synchronize()
    return cggi.to_host(w)


def test_bootstrap_free_level_and_empty_level(O):
    from paper_2306_11006_amd import cggi
    p = params.TOY
    keys = real_keys(p, 3)
    bits = [0, 1, 1, 0, 1, 0]
    cts = encrypt_bits(p, keys, bits, seed=3300)
    gates = []
    for k in range(len(bits)):
        for op in (NOT, COPY, CONST0, CONST1):
            gates.append([op, k, 0, 0, len(bits) + len(gates)])
    gates = np.array(gates, dtype=np.int32)
    wires = np.zeros((len(bits) + len(gates), p.n + 1), dtype=np.uint32)
    wires[:len(bits)] = cts
    want = np.stack([O.gate(p, int(g[0]), keys["bsk"], keys["ksk"],
                            wires[g[1]]) for g in gates])
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    for form in FORMS:
        say(f"bootstrap-free level form={form} G={len(gates)}")
        got = run_level(ctx, form, wires, gates)
        assert np.array_equal(got[:len(bits)], cts), form
        assert np.array_equal(got[len(bits):], want), form
        for g, row in zip(gates, got[len(bits):]):
            b = bits[g[1]]
            expect = {NOT: 1 - b, COPY: b, CONST0: 0, CONST1: 1}[int(g[0])]
            assert O.lwe_decrypt(keys["s"], row) == expect
        say(f"empty level form={form}")
        got = run_level(ctx, form, wires, np.zeros((0, 5), np.int32))
        assert np.array_equal(got, wires), form
    ctx.close()


def test_largest_lwe_dimension(O):
    """n = 1023 (the largest accepted), N = 1024: the int8 workgroup's LDS
    then holds 158,720 of its 163,840 bytes."""
    import torch
    from paper_2306_11006_amd import cggi
    p = dataclasses.replace(params.DEFAULT, name="n1023", n=1023)
    cggi.params_check(p)
    bsk, ksk = inputs.uniform_keys(p, 3310)
    B = 6
    cts = inputs.uniform_lwe(p, 3311, B)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    outs = {}
    for form in FORMS:
        say(f"n=1023 bootstrap form={form} B={B}")
        o = ctx.bootstrap(form, cggi.to_device(cts))
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(o)
    assert np.array_equal(outs["ntt"], outs["int8"])
    pick = (0, B - 1)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(lambda i: O.bootstrap(p, bsk, cts[i]), pick))
    for i, wv in zip(pick, want):
        assert np.array_equal(outs["int8"][i], wv), i
    ctx.close()


def test_widest_level_default(O):
    """65,536 independent NAND gates in one level (the widest level of the
    large random-DAG recipe) at the default sizes: the forms agree on every
    output, and sampled gates equal the oracle."""
    import torch
    from paper_2306_11006_amd import cggi
    p = params.DEFAULT
    bsk, ksk = inputs.uniform_keys(p, 3320)
    G = 65536
    gates = np.stack([np.zeros(G, np.int32), np.arange(G, dtype=np.int32),
                      np.arange(G, 2 * G, dtype=np.int32),
                      np.zeros(G, np.int32),
                      np.arange(2 * G, 3 * G, dtype=np.int32)], axis=1)
    wires = np.zeros((3 * G, p.n + 1), dtype=np.uint32)
    wires[: 2 * G] = inputs.uniform_lwe(p, 3321, 2 * G)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    d_gates = cggi.to_device(gates)
    outs = {}
    for form in FORMS:
        say(f"default widest level form={form} G={G}")
        w = cggi.to_device(wires)
        ctx.eval_level(form, d_gates, w)
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(w[2 * G:])
        del w
    assert np.array_equal(outs["ntt"], outs["int8"])
    pick = [0, 1, G // 3, G // 2, G - 2, G - 1]

    def one(i):
        return O.gate(p, NAND, bsk, ksk, wires[i], wires[G + i])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(one, pick))
    for i, wv in zip(pick, want):
        assert np.array_equal(outs["int8"][i], wv), i
    ctx.close()
