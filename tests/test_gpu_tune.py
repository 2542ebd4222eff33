"""The int8 kernel plan and its autotuner on the GPU: every kernel kind gives
the same bits at every batch width it can take (equal to the NTT form and,
on samples, the oracle); invalid plans are rejected with nothing changed; a
level evaluated under several plans (device-side choice) gives the same
wires; the tuner's table is valid, survives its JSON cache and, installed,
leaves results unchanged."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from paper_2306_11006_amd import arith, cggi, inputs, params, tune

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 4)
BIG = 2**31 - 1


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_bs(ctx, form, cts):
    import torch
    out = ctx.bootstrap(form, cggi.to_device(cts))
    torch.cuda.synchronize()
    return cggi.to_host(out)


def force(ctx, kind, limits):
    if kind.startswith("split"):
        ctx.int8_plan([(kind, limits[kind]), ("tiles4", BIG)])
    else:
        ctx.int8_plan([(kind, BIG)])


@pytest.mark.parametrize("p", [params.DEFAULT, params.TOY],
                         ids=["default", "toy"])
def test_every_kind_same_bits(O, p):
    bsk, ksk = inputs.uniform_keys(p, 8100)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    limits = ctx.int8_limits()
    assert all(limits[k] > 0 for k in cggi.KINDS), limits
    widths = (1, 7, limits["split8"], limits["split4"], 300,
              limits["split2"])
    cts = inputs.uniform_lwe(p, 8101, max(widths))
    for w in widths:
        x = cts[:w]
        ref = run_bs(ctx, "ntt", x)
        for kind in cggi.KINDS:
            if limits[kind] < w:
                continue
            say(f"{p.name} width={w} kind={kind}")
            force(ctx, kind, limits)
            assert np.array_equal(run_bs(ctx, "int8", x), ref), (w, kind)
        ctx.int8_plan(None)
    ctx.check()
    pick = (0, widths[-1] - 1)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = list(ex.map(lambda i: O.bootstrap(p, bsk, cts[i]), pick))
    for i, wv in zip(pick, want):       # ref holds the widest batch
        assert np.array_equal(ref[i], wv), i
    ctx.close()


def test_invalid_plans_rejected():
    p = params.DEFAULT
    bsk, ksk = inputs.uniform_keys(p, 8200)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    limits = ctx.int8_limits()
    before = ctx.int8_plan_get()
    bad = [
        [("tiles1", 100)],                                  # last cap < 2^24
        [("tiles2", 100), ("tiles1", 50), ("tiles4", BIG)],  # not increasing
        [("split4", limits["split4"] + 1), ("tiles4", BIG)],  # over the limit
        [("split4", BIG)],                                  # latency mode last
        [(7, BIG)],                                         # unknown kind
    ]
    for plan in bad:
        with pytest.raises(cggi.CggiError) as e:
            ctx.int8_plan(plan)
        assert e.value.code == cggi.E_PARAM, plan
        assert ctx.int8_plan_get() == before
    ctx.int8_plan([("tiles2", 5), ("tiles4", BIG)])
    assert ctx.int8_plan_get() == [("tiles2", 5), ("tiles4", BIG)]
    ctx.latency_mode(False)
    assert [k for k, _ in before if k.startswith("split")]
    ctx.int8_plan(None)
    assert not [k for k, _ in ctx.int8_plan_get() if k.startswith("split")]
    ctx.latency_mode(True)
    assert ctx.int8_plan_get() == before
    ctx.close()
    bl, kl = inputs.uniform_keys(params.LARGE, 8201)
    cl = cggi.Context(params.LARGE, cggi.to_device(bl), cggi.to_device(kl),
                      forms=("int8",))
    lim = cl.int8_limits()
    assert lim["tiles4"] > 0 and all(lim[k] == 0 for k in cggi.KINDS
                                     if k != "tiles4")
    assert cl.int8_plan_get() == [("tiles4", BIG)]
    with pytest.raises(cggi.CggiError):
        cl.int8_plan([("tiles1", BIG)])
    cl.close()


def test_levels_under_several_plans():
    """A 16-bit Dadda multiplier (levels of 7 to 256 gates) evaluated with
    the built-in plan, one kind for everything, and a mixed plan: every
    plan's levels pick their kernel on the device; all wires agree."""
    import torch
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p = params.DEFAULT
    bsk, ksk = inputs.uniform_keys(p, 8300)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    nl, io = arith.multiplier(16, "tree")
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    ins = list(io["a"]) + list(io["b"])
    wires[ins] = inputs.uniform_lwe(p, 8301, len(ins))
    plans = [None, [("tiles4", BIG)], [("tiles1", BIG)],
             [("split2", 40), ("tiles1", 100), ("tiles4", BIG)]]
    outs = []
    for plan in plans:
        say(f"16-bit Dadda multiplier, plan {plan}")
        ctx.int8_plan(plan)
        w = cggi.to_device(wires)
        circ.run(ctx, "int8", w)
        torch.cuda.synchronize()
        outs.append(cggi.to_host(w))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ctx.check()
    ctx.close()


def test_autotune_table(tmp_path):
    """Tuner at toy sizes on a small grid: a valid plan that the library
    accepts, the JSON cache written and read back, and unchanged results
    under the tuned plan, per-level form choice included."""
    import torch
    from paper_2306_11006_amd.circuit import LevelledCircuit
    p = params.TOY
    bsk, ksk = inputs.uniform_keys(p, 8400)
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    path = str(tmp_path / "toy.json")
    say("autotune toy")
    table = tune.load_or_tune(ctx, p, path=path, reps=1,
                              widths=[1, 16, 256, 257, 1024])
    assert os.path.exists(path)
    again = tune.load_or_tune(ctx, p, path=path)
    assert again["key"] == table["key"] and again["plan"] == \
        [list(e) for e in table["plan"]]
    plan = table["plan"]
    caps = [c for _, c in plan]
    assert caps == sorted(set(caps)) and caps[-1] == BIG
    for w in table["widths"]:
        t = table["times"][str(w)]
        assert t and all(v > 0 for v in t.values())
        assert set(table["forms"][str(w)]) == {"int8", "ntt"}
    cts = inputs.uniform_lwe(p, 8401, 300)
    base = run_bs(ctx, "int8", cts)
    tune.apply(ctx, table)
    assert ctx.int8_plan_get() == [tuple(e) for e in plan]
    assert np.array_equal(run_bs(ctx, "int8", cts), base)
    nl, io = arith.adder(16, "prefix")
    circ = LevelledCircuit(nl.array(), nl.n_wires)
    wires = np.zeros((nl.n_wires, p.n + 1), dtype=np.uint32)
    ins = list(io["a"]) + list(io["b"])
    wires[ins] = inputs.uniform_lwe(p, 8402, len(ins))
    a, b = cggi.to_device(wires), cggi.to_device(wires)
    circ.run(ctx, "ntt", a)
    circ.run(ctx, "auto", b, table=table)
    torch.cuda.synchronize()
    assert np.array_equal(cggi.to_host(a), cggi.to_host(b))
    ctx.check()
    ctx.close()
