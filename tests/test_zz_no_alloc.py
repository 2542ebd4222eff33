"""cggi_eval_level_noalloc (the level on the library's fixed device
workspace) against cggi_eval_level on the same inputs, bit for bit.

Two calls in a row on one context, the second with a smaller level, both
forms; a level beyond the workspace's limit is refused on the host with
nothing written; and the allocation-free call captured into a HIP graph and
replayed, every replay checked against the eager result.  The oracle pins
the first call's outputs through the stored per-row digests of the
benchmark level (tests/golden/digests.py)."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import digests as D  # noqa: E402

pytestmark = pytest.mark.gpu

FORMS = ("ntt", "int8")


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def mixed_level(seed, G, n_in, n_wires):
    """G gates of every opcode reading wires [0, n_in) and writing wires
    n_in .. n_in + G - 1 (a valid single level)."""
    from paper_2306_11006_amd import inputs
    g = inputs.rng(seed)
    ops = g.integers(0, 11, size=G)
    ins = g.integers(0, n_in, size=(G, 3))
    out = n_in + np.arange(G)
    assert n_in + G <= n_wires
    return np.stack([ops, ins[:, 0], ins[:, 1], ins[:, 2], out],
                    axis=1).astype(np.int32)


def run(ctx, form, gates_np, wires_np, noalloc):
    import torch
    from paper_2306_11006_amd import cggi
    g = cggi.to_device(gates_np)
    w = cggi.to_device(wires_np)
    if noalloc:
        ctx.eval_level_noalloc(form, g, w)
    else:
        ctx.reserve(len(gates_np))
        ctx.eval_level(form, g, w)
    ctx.check()
    torch.cuda.synchronize()
    return cggi.to_host(w)


def test_noalloc_matches_eval_level_two_calls():
    """Call 1: the benchmark's 1024-NAND level (every row also equals the
    oracle's stored digest); call 2, on the same context right after: a
    smaller level of 200 gates over every opcode.  Both forms."""
    import oracle as O
    from paper_2306_11006_amd import cggi, inputs
    O.lib()
    case = D.build("level1024_nand_uniform", O)
    p = case["p"]
    ctx = cggi.Context(p, cggi.to_device(case["bsk"]),
                       cggi.to_device(case["ksk"]))
    small_w = inputs.uniform_lwe(p, 4242, 600)
    small_g = mixed_level(4243, 200, 400, 600)
    for form in FORMS:
        say(f"noalloc call 1: 1024 NAND, form={form}")
        want1 = run(ctx, form, case["gates"], case["wires"], False)
        got1 = run(ctx, form, case["gates"], case["wires"], True)
        assert np.array_equal(got1, want1), form
        if os.path.exists(D.path("level1024_nand_uniform")):
            assert not D.compare("level1024_nand_uniform",
                                 got1[case["rows"]]), form
        say(f"noalloc call 2: 200 mixed gates, form={form}")
        want2 = run(ctx, form, small_g, small_w, False)
        got2 = run(ctx, form, small_g, small_w, True)
        assert np.array_equal(got2, want2), form
        # the second call's smaller level wrote only its own output wires
        assert np.array_equal(got2[:400], small_w[:400])
    ctx.close()


def test_noalloc_limit_refused_on_host():
    """A level larger than the fixed workspace is refused before any launch
    (CGGI_E_SHAPE, message naming the limit) and leaves the wires as they
    were."""
    import torch
    from paper_2306_11006_amd import cggi, inputs, params
    p = params.TOY
    bsk, ksk = inputs.uniform_keys(p, 5)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    per = 4 + 8 * (p.n + 1) + 8 * (p.N + 1)
    G = (64 << 20) // per + 1
    W = 2 * G + 2
    wires_np = inputs.uniform_lwe(p, 6, W)
    idx = np.arange(G, dtype=np.int32)
    z = np.zeros(G, np.int32)
    gates = cggi.to_device(np.stack([z, z, z + 1, z, 2 + idx],
                                    axis=1).astype(np.int32))
    w = cggi.to_device(wires_np)
    with pytest.raises(cggi.CggiError) as ei:
        ctx.eval_level_noalloc("int8", gates, w)
    assert ei.value.code == cggi.E_SHAPE
    assert "64 MiB" in str(ei.value)
    torch.cuda.synchronize()
    assert np.array_equal(cggi.to_host(w), wires_np)
    ctx.close()


def test_noalloc_graph_replays():
    """The allocation-free level captured into a HIP graph without any
    cggi_ctx_reserve; three replays with eager work and synchronisation in
    between, each equal to the eager result."""
    import torch
    from paper_2306_11006_amd import cggi, inputs, params
    p = params.DEFAULT
    bsk, ksk = inputs.uniform_keys(p, 31)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    wires_np = inputs.uniform_lwe(p, 32, 300)
    gates_np = mixed_level(33, 96, 200, 300)
    for form in FORMS:
        say(f"noalloc graph: form={form}")
        want = run(ctx, form, gates_np, wires_np, False)
        g = cggi.to_device(gates_np)
        w = cggi.to_device(wires_np)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            ctx.eval_level_noalloc(form, g, w)
        for k in range(3):
            w.copy_(cggi.to_device(wires_np))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            ctx.check()
            assert np.array_equal(cggi.to_host(w), want), (form, k)
        del graph
    ctx.close()
