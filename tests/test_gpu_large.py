"""The large parameter set (n=742, N=2048, Bg=2^10 l=2, KS 2^3 x 5): the
int8 form's two-tile bootstraps and 7-bit sub-digit split against the
oracle and the NTT form, real-key gates, and a random levelled DAG with
log-uniform level widths."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from conftest import encode, encrypt_bits, real_keys
from paper_2306_11006_amd import inputs, params

pytestmark = pytest.mark.gpu

FORMS = ("ntt", "int8")
THREADS = min(16, os.cpu_count() or 4)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def large_uniform():
    from paper_2306_11006_amd import cggi
    p = params.LARGE
    bsk, ksk = inputs.uniform_keys(p, 2048)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    yield p, bsk, ksk, ctx
    ctx.close()


def gpu_bs(ctx, form, cts):
    import torch
    from paper_2306_11006_amd import cggi
    out = ctx.bootstrap(form, cggi.to_device(cts))
    torch.cuda.synchronize()
    return cggi.to_host(out)


def test_large_bootstrap_bit_exact(O, large_uniform):
    p, bsk, ksk, ctx = large_uniform
    cts = inputs.uniform_lwe(p, 2049, 5)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = np.stack(list(ex.map(lambda x: O.bootstrap(p, bsk, x), cts)))
    for form in FORMS:
        say(f"large bootstrap form={form} B=5")
        assert np.array_equal(gpu_bs(ctx, form, cts), want), form


def test_large_forms_agree_batch(large_uniform):
    p, bsk, ksk, ctx = large_uniform
    cts = inputs.uniform_lwe(p, 2050, 300)
    outs = [gpu_bs(ctx, f, cts) for f in FORMS]
    assert np.array_equal(outs[0], outs[1])


def test_large_real_key_gates(O):
    import torch
    from paper_2306_11006_amd import cggi
    p = params.LARGE
    keys = real_keys(p, 2)
    ctx = cggi.Context(p, cggi.to_device(keys["bsk"]),
                       cggi.to_device(keys["ksk"]))
    trip = [(s, x, y) for s in (0, 1) for x in (0, 1) for y in (0, 1)]
    bits = [v for t in trip for v in t]
    cts = encrypt_bits(p, keys, bits, seed=2051)
    ops = ["NAND", "AND", "OR", "XOR", "MUX"]
    code = {"NAND": 0, "AND": 1, "OR": 2, "XOR": 3, "MUX": 4}
    gates = []
    for k, (s, x, y) in enumerate(trip):
        for op in ops:
            gates.append([code[op], 3 * k, 3 * k + 1, 3 * k + 2,
                          len(bits) + len(gates)])
    gates = np.array(gates, dtype=np.int32)
    wires = np.zeros((len(bits) + len(gates), p.n + 1), dtype=np.uint32)
    wires[: len(bits)] = cts
    truth = {0: lambda s, x, y: 1 - (s & x), 1: lambda s, x, y: s & x,
             2: lambda s, x, y: s | x, 3: lambda s, x, y: s ^ x,
             4: lambda s, x, y: x if s else y}
    outs = {}
    for form in FORMS:
        say(f"large real-key gates form={form} G={len(gates)}")
        w = cggi.to_device(wires)
        ctx.eval_level(form, cggi.to_device(gates), w)
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(w)
        for gt in gates:
            s, x, y = (bits[gt[1]], bits[gt[2]], bits[gt[3]])
            assert O.lwe_decrypt(keys["s"], outs[form][gt[4]]) == \
                truth[int(gt[0])](s, x, y), (form, gt)
    assert np.array_equal(outs["ntt"], outs["int8"])
    ctx.close()


def test_large_random_dag(O, large_uniform):
    """A seeded random DAG with log-uniform level widths (reduced to 3000
    gates and widths up to 1024 so the test stays short): both forms agree
    on every wire after every level, and sampled gates of the widest level
    equal the oracle run on the GPU's own inputs of that level."""
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p, bsk, ksk, ctx = large_uniform
    nl = inputs.random_dag(2052, 3000, max_width=1024)
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    wires[nl.input_wires] = inputs.uniform_lwe(p, 2053, len(nl.input_wires))
    widest = int(np.argmax(circ.widths))
    outs, before = {}, {}
    for form in FORMS:
        say(f"large random DAG ({circ.n_levels} levels) form={form}")
        w = cggi.to_device(wires)
        ctx.reserve(max(circ.widths))
        for L, lv in enumerate(circ.d_levels):
            if L == widest:
                torch.cuda.synchronize()
                before[form] = cggi.to_host(w)
            ctx.eval_level(form, lv, w)
        torch.cuda.synchronize()
        outs[form] = cggi.to_host(w)
    assert np.array_equal(outs["ntt"], outs["int8"])
    assert np.array_equal(before["ntt"], before["int8"])
    lv = circ.levels[widest]
    pick = sorted({0, len(lv) - 1, len(lv) // 2, len(lv) // 3})
    w0 = before["int8"]

    def one(k):
        op, a, b, c, _ = (int(v) for v in lv[k])
        return O.gate(p, op, bsk, ksk, w0[a], w0[b], w0[c])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(one, pick))
    for k, wv in zip(pick, want):
        assert np.array_equal(outs["int8"][int(lv[k][4])], wv), k


def test_large_random_dag_wide(O, large_uniform):
    """A 20,000-gate random DAG with log-uniform level widths up to 8192
    (levels that span thousands of workgroups of the N=2048 kernels): the
    two forms agree on every wire, and gates of the widest level (first,
    last and six spread between) equal the oracle on that level's inputs."""
    import time
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p, bsk, ksk, ctx = large_uniform
    nl = inputs.random_dag(2060, 20000, max_width=8192)
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    wires[nl.input_wires] = inputs.uniform_lwe(p, 2061, len(nl.input_wires))
    widest = int(np.argmax(circ.widths))
    outs, before = {}, {}
    ctx.reserve(max(circ.widths))
    for form in FORMS:
        say(f"large wide DAG ({circ.n_levels} levels, widest "
            f"{max(circ.widths)}, {circ.bootstraps()} bootstraps) form={form}")
        w = cggi.to_device(wires)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for L, lv in enumerate(circ.d_levels):
            if L == widest:
                torch.cuda.synchronize()
                before[form] = cggi.to_host(w)
            ctx.eval_level(form, lv, w)
        torch.cuda.synchronize()
        say(f"  {time.perf_counter() - t0:.2f} s")
        outs[form] = cggi.to_host(w)
    assert np.array_equal(outs["ntt"], outs["int8"])
    assert np.array_equal(before["ntt"], before["int8"])
    lv = circ.levels[widest]
    pick = sorted({0, len(lv) - 1} |
                  {int(k) for k in np.linspace(1, len(lv) - 2, 6)})
    w0 = before["int8"]

    def one(k):
        op, a, b, c, _ = (int(v) for v in lv[k])
        return O.gate(p, op, bsk, ksk, w0[a], w0[b], w0[c])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(one, pick))
    for k, wv in zip(pick, want):
        assert np.array_equal(outs["int8"][int(lv[k][4])], wv), k
