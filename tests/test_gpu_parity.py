"""Parity of the HIP library against the CPU oracle (bit-exact: integer
arithmetic, tolerance 0), through the C ABI.

Both forms of the blind rotation (NTT mod Q, int8-limb MFMA) must give
every output coefficient exactly as the oracle does; at the default sizes
the oracle is run on sampled outputs of the full-size launch and the two
forms are compared on all of them.
"""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from conftest import MU, encode, encrypt_bits, real_keys, signed
from paper_2306_11006_amd import inputs, params

pytestmark = pytest.mark.gpu

FORMS = ("ntt", "int8")
THREADS = min(16, os.cpu_count() or 4)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    torch.cuda.init()
    return torch


def make_ctx(p, bsk, ksk, forms=FORMS):
    from paper_2306_11006_amd import cggi
    return cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk),
                        forms=forms)


def oracle_map(fn, items):
    with cf.ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(fn, items))


@pytest.fixture(scope="module")
def toy_real(torch_cuda):
    p = params.TOY
    keys = real_keys(p, 1)
    ctx = make_ctx(p, keys["bsk"], keys["ksk"])
    yield p, keys, ctx
    ctx.close()


@pytest.fixture(scope="module")
def default_uniform(torch_cuda):
    p = params.DEFAULT
    bsk, ksk = inputs.uniform_keys(p, 2024)
    ctx = make_ctx(p, bsk, ksk)
    yield p, bsk, ksk, ctx
    ctx.close()


def gpu_bootstrap(ctx, form, cts, testv=None):
    from paper_2306_11006_amd import cggi
    import torch
    tv = None if testv is None else cggi.to_device(testv)
    out = ctx.bootstrap(form, cggi.to_device(cts), testv=tv)
    torch.cuda.synchronize()
    return cggi.to_host(out)


def gpu_keyswitch(ctx, cts):
    from paper_2306_11006_amd import cggi
    import torch
    out = ctx.keyswitch(cggi.to_device(cts))
    torch.cuda.synchronize()
    return cggi.to_host(out)


# ---------------------------------------------------------------------------

def test_toy_nand_gates_bit_exact_and_decrypt(O, toy_real):
    """Four NAND gates over all input pairs (toy sizes): bootstrap outputs of
    both forms equal the oracle's bit for bit, the key switch equals the
    oracle's, and the result decrypts to the NAND truth table."""
    p, keys, ctx = toy_real
    pairs = [(a, b) for a in (0, 1) for b in (0, 1)]
    cts = encrypt_bits(p, keys, [v for ab in pairs for v in ab], seed=11)
    pre = np.stack([O.gate_preop(p.n, "NAND", cts[2 * i], cts[2 * i + 1])
                    for i in range(4)])
    want_bs = np.stack([O.bootstrap(p, keys["bsk"], x) for x in pre])
    want_ks = np.stack([O.keyswitch(p, keys["ksk"], x) for x in want_bs])
    for form in FORMS:
        say(f"toy NAND bootstrap form={form} B=4")
        got = gpu_bootstrap(ctx, form, pre)
        assert np.array_equal(got, want_bs), form
    say("toy keyswitch B=4")
    got_ks = gpu_keyswitch(ctx, want_bs)
    assert np.array_equal(got_ks, want_ks)
    for i, (a, b) in enumerate(pairs):
        assert O.lwe_decrypt(keys["s"], got_ks[i]) == 1 - (a & b)


@pytest.mark.parametrize("B", [1, 15, 16, 17, 37])
def test_toy_ragged_batches_bit_exact(O, torch_cuda, B):
    """Uniform keys and inputs, batch sizes around the int8 workgroup width
    (16 bootstraps at N=256): every output coefficient equals the oracle."""
    p = params.TOY
    bsk, ksk = inputs.uniform_keys(p, 300 + B)
    ctx = make_ctx(p, bsk, ksk)
    cts = inputs.uniform_lwe(p, 400 + B, B)
    want = np.stack(oracle_map(lambda x: O.bootstrap(p, bsk, x), cts))
    for form in FORMS:
        say(f"toy uniform bootstrap form={form} B={B}")
        assert np.array_equal(gpu_bootstrap(ctx, form, cts), want), form
    ctx.close()


def test_toy_custom_test_vector(O, toy_real):
    p, keys, ctx = toy_real
    g = inputs.rng(77)
    tv = inputs.uniform_u32(g, (p.N,))
    cts = inputs.uniform_lwe(p, 78, 9)
    want = np.stack([O.bootstrap(p, keys["bsk"], x, tv) for x in cts])
    for form in FORMS:
        say(f"toy test-vector bootstrap form={form} B=9")
        assert np.array_equal(gpu_bootstrap(ctx, form, cts, tv), want)


def test_toy_noiseless_closed_form(O, torch_cuda):
    """Zero-noise keys with aligned masks: the extracted phase of every GPU
    output is exactly +-2^29 by the rule of the blind rotation (pins the
    GPU path to the mathematics, not only to the oracle)."""
    p = params.TOY
    d = inputs.key_draws(p, 91, bk_noise=False, ks_noise=False,
                         aligned_bsk=True)
    bsk = O.make_bsk(p, d["s"], d["K"], d["bsk_a"], d["bsk_e"])
    ksk = O.make_ksk(p, d["s"], d["K"], d["ksk_a"], d["ksk_e"])
    ctx = make_ctx(p, bsk, ksk)
    cts = inputs.uniform_lwe(p, 92, 20)
    K = d["K"].astype(np.int64)
    for form in FORMS:
        say(f"toy noiseless bootstrap form={form} B=20")
        out = gpu_bootstrap(ctx, form, cts)
        for x, y in zip(cts, out):
            at = [((int(u) * 2 * p.N + (1 << 31)) >> 32) % (2 * p.N)
                  for u in x]
            phi = (at[p.n] - sum(a for a, s in zip(at[:p.n], d["s"]) if s)) \
                % (2 * p.N)
            ph = (int(y[p.N]) - int((y[:p.N].astype(np.int64) * K).sum())) \
                % (1 << 32)
            assert ph == (MU if phi < p.N else (1 << 32) - MU)
    ctx.close()


def test_default_full_batch_forms_agree_and_match_oracle(O, default_uniform):
    """Default sizes, the benchmark's launch (B = 1024): the two forms agree
    on all 1024 x 1025 output coefficients, and sampled outputs (first,
    last, seeded random) equal the oracle's."""
    p, bsk, ksk, ctx = default_uniform
    B = 1024
    cts = inputs.uniform_lwe(p, 5150, B)
    outs = {}
    for form in FORMS:
        say(f"default bootstrap form={form} B={B}")
        outs[form] = gpu_bootstrap(ctx, form, cts)
    assert np.array_equal(outs["ntt"], outs["int8"])
    g = inputs.rng(5151)
    idx = sorted({0, B - 1, *g.integers(0, B, size=4).tolist()})
    say(f"default oracle on samples {idx}")
    want = oracle_map(lambda i: O.bootstrap(p, bsk, cts[i]), idx)
    for i, w in zip(idx, want):
        assert np.array_equal(outs["int8"][i], w), i


def test_default_ragged_small_batch(O, default_uniform):
    p, bsk, ksk, ctx = default_uniform
    B = 6
    cts = inputs.uniform_lwe(p, 5160, B)
    want = np.stack(oracle_map(lambda x: O.bootstrap(p, bsk, x), cts))
    for form in FORMS:
        say(f"default bootstrap form={form} B={B}")
        assert np.array_equal(gpu_bootstrap(ctx, form, cts), want), form


@pytest.mark.parametrize("B", [200, 400, 700])
def test_default_batch_widths_pick_tiles(O, default_uniform, B):
    """Batch widths that give the int8 form 1, 2 and 4 column tiles per
    workgroup (at most one wave of workgroups over the CUs): the forms agree
    on every output and the first and last bootstraps equal the oracle."""
    p, bsk, ksk, ctx = default_uniform
    cts = inputs.uniform_lwe(p, 3400 + B, B)
    outs = {}
    for form in FORMS:
        say(f"default bootstrap form={form} B={B}")
        outs[form] = gpu_bootstrap(ctx, form, cts)
    assert np.array_equal(outs["ntt"], outs["int8"])
    idx = [0, B - 1]
    want = oracle_map(lambda i: O.bootstrap(p, bsk, cts[i]), idx)
    for i, w in zip(idx, want):
        assert np.array_equal(outs["int8"][i], w), i


def test_default_keyswitch_bit_exact(O, default_uniform):
    p, bsk, ksk, ctx = default_uniform
    cts = inputs.uniform_lwe(p, 5170, 67, dim=p.N)
    say("default keyswitch B=67")
    got = gpu_keyswitch(ctx, cts)
    want = np.stack(oracle_map(lambda x: O.keyswitch(p, ksk, x), cts))
    assert np.array_equal(got, want)


def test_zero_batch_is_noop(default_uniform):
    from paper_2306_11006_amd import cggi
    import torch
    p, bsk, ksk, ctx = default_uniform
    inp = torch.zeros((0, p.n + 1), dtype=torch.int32, device="cuda")
    out = torch.zeros((0, p.N + 1), dtype=torch.int32, device="cuda")
    for form in FORMS:
        ctx.bootstrap(form, inp, out)
    ctx.keyswitch(torch.zeros((0, p.N + 1), dtype=torch.int32,
                              device="cuda"))
    torch.cuda.synchronize()


def test_alias_rejected(default_uniform):
    from paper_2306_11006_amd import cggi
    import torch
    p, bsk, ksk, ctx = default_uniform
    buf = torch.zeros((4, p.N + 1), dtype=torch.int32, device="cuda")
    view = buf.view(-1)[: 4 * (p.n + 1)].view(4, p.n + 1)
    for form in FORMS:
        with pytest.raises(cggi.CggiError) as e:
            ctx.bootstrap(form, view, buf)
        assert e.value.code == cggi.E_ALIAS
    # a correctly shaped output that overlaps the input reaches the library
    with pytest.raises(cggi.CggiError) as e:
        ctx.keyswitch(buf, view)
    assert e.value.code == cggi.E_ALIAS


def crafted_modswitch_inputs(p, seed):
    """Eight LWE ciphertexts whose coefficients sit on and next to the
    modulus switch's rounding ties (u = k 2^(32-s) + 2^(31-s), 2N = 2^s,
    rounded up) and on the values that switch to 0 (so the CMux steps with
    a~_i = 0 are skipped): exact ties, ties - 1, ties + 1, all-zero masks,
    masks 90% of which round to 0, masks at the wrap 2^32 - 2^(31-s) (-> 0)
    and one below it (-> 2N - 1), the pair 2^(31-s) - 1 / 2^(31-s) (-> 0 / 1),
    and one uniform row."""
    log2_2n = (2 * p.N).bit_length() - 1
    drop = 32 - log2_2n
    half = 1 << (drop - 1)
    g = inputs.rng(seed)
    m = p.n + 1
    k = g.integers(0, 2 * p.N, size=(8, m), dtype=np.int64)
    tie = (k << drop) + half
    rows = np.empty((8, m), dtype=np.int64)
    rows[0] = tie[0]
    rows[1] = tie[1] - 1
    rows[2] = tie[2] + 1
    rows[3] = 0
    rows[3, -1] = tie[3, -1]
    small = g.integers(-half, half, size=m)
    rows[4] = np.where(g.random(m) < 0.9, small, tie[4])
    wrap = (1 << 32) - half
    rows[5] = np.where(np.arange(m) % 2 == 0, wrap, wrap - 1)
    rows[6] = np.where(np.arange(m) % 2 == 0, half - 1, half)
    rows[6, -1] = (1 << 32) - 1
    rows[7] = g.integers(0, 1 << 32, size=m)
    return (rows % (1 << 32)).astype(np.uint32)


@pytest.mark.parametrize("pname", ["toy", "default"])
def test_modswitch_ties_and_zero_rotations(O, torch_cuda, pname):
    """Crafted inputs on the modulus switch's ties and on rotations that
    switch to 0: the NTT form and every int8 kernel kind (forced through the
    kernel plan) equal the oracle on every output coefficient."""
    from paper_2306_11006_amd import cggi
    p = params.ALL[pname]
    bsk, ksk = inputs.uniform_keys(p, 6100)
    ctx = make_ctx(p, bsk, ksk)
    cts = crafted_modswitch_inputs(p, 6101)
    want = np.stack(oracle_map(lambda x: O.bootstrap(p, bsk, x), cts))
    say(f"{pname} modswitch ties form=ntt")
    assert np.array_equal(gpu_bootstrap(ctx, "ntt", cts), want)
    limits = ctx.int8_limits()
    for kind in cggi.KINDS:
        if limits[kind] < len(cts):
            continue
        if kind.startswith("split"):
            ctx.int8_plan([(kind, limits[kind]), ("tiles4", cggi.INT32_MAX)])
        else:
            ctx.int8_plan([(kind, cggi.INT32_MAX)])
        say(f"{pname} modswitch ties form=int8 kind={kind}")
        got = gpu_bootstrap(ctx, "int8", cts)
        ctx.check()
        bad = np.nonzero((got != want).any(axis=1))[0].tolist()
        assert not bad, (kind, bad)
    ctx.int8_plan(None)
    ctx.close()
