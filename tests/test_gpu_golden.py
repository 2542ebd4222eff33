"""Full-size parity against the oracle through stored per-row digests.

Each case of tests/golden/digests.py is a seeded workload at the default
parameter set whose every output row the CPU oracle computed once (the
digest files are written by that script from the oracle alone).  Here the
HIP library runs the same inputs, in the launch configuration the benchmark
times, and every output row is hashed and compared with the stored digest:
every coefficient of every output ciphertext is checked, for both forms,
including the shared level kernels (slot map, pre-op, MUX combine, key
switch) that a comparison of the two forms with each other cannot see.
Failures name the rows that differ."""
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


def need(name):
    if not os.path.exists(D.path(name)):
        pytest.fail(f"{D.path(name)} is missing: run tests/golden/digests.py")


def check_rows(name, form, rows):
    bad = D.compare(name, rows)
    assert not bad, (f"{name} {form}: {len(bad)} of {len(rows)} rows differ "
                     f"from the oracle, first {bad[:16]}")


def run_level(ctx, form, case, noalloc=False):
    import torch
    from paper_2306_11006_amd import cggi
    w = cggi.to_device(case["wires"])
    g = cggi.to_device(case["gates"])
    if noalloc:
        ctx.eval_level_noalloc(form, g, w)
    else:
        ctx.reserve(len(case["gates"]))
        ctx.eval_level(form, g, w)
    ctx.check()
    torch.cuda.synchronize()
    return cggi.to_host(w)


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.lib()
    return oracle


def make_ctx(case):
    from paper_2306_11006_amd import cggi
    return cggi.Context(case["p"], cggi.to_device(case["bsk"]),
                        cggi.to_device(case["ksk"]))


def test_bench_level_1024_nand_every_row(O):
    """The benchmark's own level (1024 NANDs, uniform keys and inputs, one
    cggi_eval_level): all 1024 output ciphertexts equal the oracle's."""
    name = "level1024_nand_uniform"
    need(name)
    case = D.build(name, O)
    ctx = make_ctx(case)
    for form in FORMS:
        say(f"{name} form={form}")
        got = run_level(ctx, form, case)
        check_rows(name, form, got[case["rows"]])
    ctx.close()


def test_level_1024_nand_keygen_every_row(O):
    """1024 NANDs with oracle-generated keys on fresh encryptions: every
    output equals the oracle and decrypts to the NAND of its inputs."""
    name = "level1024_nand_keygen"
    need(name)
    case = D.build(name, O)
    ctx = make_ctx(case)
    for form in FORMS:
        say(f"{name} form={form}")
        got = run_level(ctx, form, case)
        check_rows(name, form, got[case["rows"]])
        dec = np.array([O.lwe_decrypt(case["s"], got[r])
                        for r in case["rows"]])
        assert np.array_equal(dec, case["plain"]), form
    ctx.close()


def test_adder_multiplier_default_every_wire(O):
    """The uneven-level workload at the default sizes (16-bit ripple adder
    beside a 16x16 array multiplier, 88 levels of width 1 to 273, real
    keys): every wire equals the oracle, eagerly in both forms and as one
    captured HIP graph in the int8 form; outputs decrypt to a+b and x*y."""
    import torch
    from paper_2306_11006_amd import cggi
    from paper_2306_11006_amd.circuit import LevelledCircuit
    name = "adder_mult16_keygen"
    need(name)
    case = D.build(name, O)
    circ = LevelledCircuit(case["gates"], len(case["wires"]))
    assert circ.n_levels == 88
    ctx = make_ctx(case)
    for form, graph in (("ntt", False), ("int8", False), ("int8", True)):
        say(f"{name} form={form} graph={graph}")
        w = cggi.to_device(case["wires"])
        if graph:
            g = circ.capture(ctx, form, w)
            g.replay()
        else:
            circ.run(ctx, form, w)
        ctx.check()
        torch.cuda.synchronize()
        got = cggi.to_host(w)
        if graph:
            del g
        check_rows(name, form, got[case["rows"]])
    A, B, X, Y = case["operands"]
    io = case["io"]

    def decode(ws):
        return sum(O.lwe_decrypt(case["s"], got[w]) << i
                   for i, w in enumerate(ws))
    assert decode(io["sum"]) == A + B
    assert decode(io["prod"]) == X * Y
    ctx.close()


def test_mixed_level_16384_every_row(O):
    """16,384 independent gates uniform over NAND/AND/OR/XOR/MUX (19,727
    bootstraps) in one level, both forms: all 16,384 outputs equal the
    oracle's (256 key-switch row tiles, MUX combine included)."""
    name = "mixed16384_uniform"
    need(name)
    case = D.build(name, O)
    ctx = make_ctx(case)
    for form in FORMS:
        say(f"{name} form={form}")
        got = run_level(ctx, form, case)
        check_rows(name, form, got[case["rows"]])
    ctx.close()
