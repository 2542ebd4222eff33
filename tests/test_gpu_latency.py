"""Latency mode of the int8 form: a narrow batch runs each column tile's
blind rotation on eight, four or (for up to twice as many tiles) two
workgroups that exchange partial products after every CMux step.  Bit-exact against
the oracle and the NTT form, identical to the one-workgroup kernel, at every
N <= 1024 and digit shape (specialised and generic builds), over partial
tiles, repeated launches (launch epochs), and HIP-graph replays of a whole
circuit whose levels pick every kernel from their device-side counts."""
import concurrent.futures as cf
import dataclasses
import os
import sys

import numpy as np
import pytest

from paper_2306_11006_amd import arith, inputs, params

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 4)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_bs(ctx, form, cts):
    import torch
    from paper_2306_11006_amd import cggi
    out = ctx.bootstrap(form, cggi.to_device(cts))
    torch.cuda.synchronize()
    return cggi.to_host(out)


def make_ctx(p, seed):
    from paper_2306_11006_amd import cggi
    bsk, ksk = inputs.uniform_keys(p, seed)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    return bsk, ksk, ctx


CASES = [
    # (parameter set, batch sizes): N = 1024 (l=3, S=1 build), N = 256 with
    # Bg = 2^8 (two sub-digits, the l=2 S=2 build, four bootstraps per tile);
    # the smallest batches take eight workgroups per tile, the largest two
    (params.DEFAULT, (1, 3, 64, 100, 128)),
    (params.TOY, (1, 5, 255, 300)),
    (dataclasses.replace(params.DEFAULT, name="n512_N512", n=512, N=512),
     (2, 9)),
    # generic build (digit loops with run-time bounds): l = 2 levels of 2^7
    (dataclasses.replace(params.DEFAULT, name="bg7_l2", l=2), (1, 7)),
]


@pytest.mark.parametrize("p,batches", CASES, ids=[c[0].name for c in CASES])
def test_latency_mode_bit_exact(O, p, batches):
    from paper_2306_11006_amd import cggi
    bsk, ksk, ctx = make_ctx(p, 7100 + p.N)
    groups = ctx.latency_groups()
    assert groups >= 1, p.name
    for B in batches:
        tiles = -(-B // (1024 // p.N))
        assert tiles <= groups, (B, groups)
        cts = inputs.uniform_lwe(p, 7200 + B, B)
        say(f"latency mode {p.name} B={B} tiles={tiles} (limit {groups})")
        got = run_bs(ctx, "int8", cts)
        ctx.check()
        ntt = run_bs(ctx, "ntt", cts)
        assert np.array_equal(got, ntt), (p.name, B)
        ctx.latency_mode(False)
        one = run_bs(ctx, "int8", cts)
        ctx.latency_mode(True)
        assert np.array_equal(got, one), (p.name, B)
        pick = sorted({0, B - 1, B // 2})
        with cf.ThreadPoolExecutor(THREADS) as ex:
            want = list(ex.map(lambda i: O.bootstrap(p, bsk, cts[i]), pick))
        for i, wv in zip(pick, want):
            assert np.array_equal(got[i], wv), (p.name, B, i)
    ctx.close()


def test_latency_mode_limits():
    """Off -> no groups; N = 2048 has no latency mode; a batch one tile
    beyond the limit takes the one-workgroup kernel (same result)."""
    from paper_2306_11006_amd import cggi
    p = params.DEFAULT
    bsk, ksk, ctx = make_ctx(p, 7300)
    groups = ctx.latency_groups()
    ctx.latency_mode(False)
    assert ctx.latency_groups() == 0
    ctx.latency_mode(True)
    assert ctx.latency_groups() == groups
    cts = inputs.uniform_lwe(p, 7301, groups + 1)
    a = run_bs(ctx, "int8", cts)
    b = run_bs(ctx, "ntt", cts)
    assert np.array_equal(a, b)
    ctx.check()
    ctx.close()
    bl, kl = inputs.uniform_keys(params.LARGE, 7302)
    cl = cggi.Context(params.LARGE, cggi.to_device(bl), cggi.to_device(kl),
                      forms=("int8",))
    assert cl.latency_groups() == 0
    cl.close()


def test_latency_mode_repeated_launches_and_graph():
    """Back-to-back launches of varying width advance the per-group epochs;
    a 32-bit Dadda multiplier (levels of 14 to 1,024 gates, so its levels
    take latency mode with four and two workgroups per tile and one
    workgroup per 1, 2 or 4 tiles, chosen on the device from each level's
    bootstrap count) captured as one HIP graph and replayed three times,
    with eager work between the replays, equals the eager run every time."""
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p = params.DEFAULT
    bsk, ksk, ctx = make_ctx(p, 7400)
    groups = ctx.latency_groups()
    base = inputs.uniform_lwe(p, 7401, groups)
    ref = run_bs(ctx, "ntt", base)
    for B in (groups, 1, groups // 2, 2, groups):
        say(f"repeated launch B={B}")
        got = run_bs(ctx, "int8", base[:B])
        assert np.array_equal(got, ref[:B]), B
    ctx.check()

    nl, io = arith.multiplier(32, "tree")
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    assert min(circ.widths) * 2 <= groups // 2 and max(circ.widths) > 512
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    ins = list(io["a"]) + list(io["b"])
    wires[ins] = inputs.uniform_lwe(p, 7402, len(ins))
    eager = cggi.to_device(wires)
    say("narrow circuit eager")
    circ.run(ctx, "int8", eager)
    torch.cuda.synchronize()
    want = cggi.to_host(eager)
    ntt = cggi.to_device(wires)
    circ.run(ctx, "ntt", ntt)
    torch.cuda.synchronize()
    assert np.array_equal(cggi.to_host(ntt), want)
    gw = cggi.to_device(wires)
    graph = circ.capture(ctx, "int8", gw)
    for rep in range(3):
        say(f"narrow circuit graph replay {rep}")
        gw.copy_(cggi.to_device(wires))
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cggi.to_host(gw), want), rep
        # eager latency-mode work between replays
        got = run_bs(ctx, "int8", base[:3])
        assert np.array_equal(got, ref[:3])
    ctx.check()
    del graph
    ctx.close()


def test_latency_mode_abort_and_recovery():
    """The error word forced from the host (cggi_ctx_latency_abort, no GPU
    wait involved): a latency-mode launch then writes nothing, other kernels
    still work, cggi_ctx_check reports CGGI_E_TIMEOUT and clears the state,
    and the next latency-mode launch is exact again."""
    import torch
    from paper_2306_11006_amd import cggi
    p = params.DEFAULT
    bsk, ksk, ctx = make_ctx(p, 7500)
    cts = inputs.uniform_lwe(p, 7501, 5)
    ref = run_bs(ctx, "ntt", cts)
    ctx.latency_abort()
    out = torch.full((5, p.N + 1), 0x5A5A5A5A, dtype=torch.int32,
                     device="cuda")
    ctx.bootstrap("int8", cggi.to_device(cts), out)         # latency mode
    torch.cuda.synchronize()
    assert bool((out == 0x5A5A5A5A).all()), "aborted launch wrote output"
    ctx.int8_plan([("tiles1", 2**31 - 1)])                 # not latency mode
    assert np.array_equal(run_bs(ctx, "int8", cts), ref)
    ctx.int8_plan(None)
    with pytest.raises(cggi.CggiError) as e:
        ctx.check()
    assert e.value.code == cggi.E_TIMEOUT
    ctx.check()                                            # cleared
    for _ in range(2):
        assert np.array_equal(run_bs(ctx, "int8", cts), ref)
    ctx.check()
    ctx.close()


def test_latency_mode_contexts_of_different_sizes():
    """Two contexts sharing a latency-mode kernel build with different LDS
    needs (n = 1023 and n = 630 at N = 1024), the larger created first and
    used after the smaller: both stay exact."""
    import dataclasses
    p_big = dataclasses.replace(params.DEFAULT, name="n1023", n=1023)
    p = params.DEFAULT
    bb, kb, cb = make_ctx(p_big, 7600)
    bs, ks, cs = make_ctx(p, 7601)
    xb = inputs.uniform_lwe(p_big, 7602, 3)
    xs = inputs.uniform_lwe(p, 7603, 3)
    for ctx, x in ((cs, xs), (cb, xb), (cs, xs)):
        want = run_bs(ctx, "ntt", x)
        assert np.array_equal(run_bs(ctx, "int8", x), want)
        ctx.check()
    cb.close()
    cs.close()
