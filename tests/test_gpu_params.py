"""Parameter sets beyond the three named ones: ring degree 512, digit widths
that take the int8 form's generic (run-time l, S) kernel and its 7-bit
sub-digit split, the default 7-bit digits at rings 256 and 512, and
key-switch bases from 2^1 to 2^4 (int8 GEMM key
switch) and 2^5 (row-gather key switch).  Both forms (the int8 form under
its built-in plan and with each throughput kernel forced) and the key
switch are compared with the oracle coefficient by coefficient on uniform
keys, for one full four-tile workgroup of bootstraps plus a ragged tail."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

from paper_2306_11006_amd import inputs, params

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 4)

SETS = [
    # N=512, Bg=2^6 l=4: one 7-bit sub-digit, generic kernel (l=4 run time)
    params.Params("n512_bg6_l4", n=100, N=512, k=1, bg_bit=6, l=4,
                  ks_base_bit=4, ks_t=4, lwe_noise_log2=15,
                  bk_noise_log2=25),
    # N=512, Bg=2^12 l=2: two sub-digits (specialised l=2, S=2 kernel)
    params.Params("n512_bg12_l2", n=64, N=512, k=1, bg_bit=12, l=2,
                  ks_base_bit=1, ks_t=12, lwe_noise_log2=15,
                  bk_noise_log2=25),
    # N=1024, Bg=2^13 l=1: widest digits the int8 form accepts (two
    # sub-digits), generic kernel (l=1 run time)
    params.Params("n1024_bg13_l1", n=40, N=1024, k=1, bg_bit=13, l=1,
                  ks_base_bit=3, ks_t=6, lwe_noise_log2=15,
                  bk_noise_log2=25),
    # N=256, Bg=2^5 l=5: ten digit rows per CMux step, generic kernel
    params.Params("n256_bg5_l5", n=48, N=256, k=1, bg_bit=5, l=5,
                  ks_base_bit=2, ks_t=7, lwe_noise_log2=15,
                  bk_noise_log2=25),
    # N=512 and N=256 with the default digits (Bg=2^7 l=3): the kernels that
    # fix the 7-bit digit width at compile time, at the two smaller rings
    params.Params("n512_bg7_l3", n=56, N=512, k=1, bg_bit=7, l=3,
                  ks_base_bit=2, ks_t=8, lwe_noise_log2=15,
                  bk_noise_log2=25),
    params.Params("n256_bg7_l3", n=40, N=256, k=1, bg_bit=7, l=3,
                  ks_base_bit=2, ks_t=8, lwe_noise_log2=15,
                  bk_noise_log2=25),
    # key-switch base 2^5: past the int8 GEMM's one-hot width, so the key
    # switch gathers key rows instead
    params.Params("n256_ks32", n=64, N=256, k=1, bg_bit=8, l=2,
                  ks_base_bit=5, ks_t=6, lwe_noise_log2=15,
                  bk_noise_log2=25),
]


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def per_workgroup(p):
    # bootstraps one int8 workgroup holds
    return 1 if p.N > 1024 else 4 * (1024 // p.N)


@pytest.mark.parametrize("p", SETS, ids=[s.name for s in SETS])
def test_params_bootstrap_and_keyswitch_bit_exact(O, p):
    import torch
    from paper_2306_11006_amd import cggi
    cggi.params_check(p)
    seed = 3100 + SETS.index(p)
    bsk, ksk = inputs.uniform_keys(p, seed)
    B = per_workgroup(p) + 3
    cts = inputs.uniform_lwe(p, seed + 1, B)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        want = np.stack(list(ex.map(lambda x: O.bootstrap(p, bsk, x), cts)))
    ctx = cggi.Context(p, cggi.to_device(bsk), cggi.to_device(ksk))
    x = cggi.to_device(cts)
    for form in ("ntt", "int8"):
        say(f"params {p.name} form={form} B={B}")
        out = ctx.bootstrap(form, x)
        torch.cuda.synchronize()
        assert np.array_equal(cggi.to_host(out), want), (p.name, form)
    # the built-in plan sends this batch to latency mode; every throughput
    # kernel (one, two and four tiles per workgroup; the four-tile one with
    # offset digit operands; the Karatsuba kernel where its workgroup fits
    # the LDS) on the same full workgroup + ragged tail
    limits = ctx.int8_limits()
    for kind in ("tiles1", "tiles2", "tiles4", "kara2"):
        if limits[kind] < B:
            continue
        say(f"params {p.name} int8 kernel {kind} B={B}")
        ctx.int8_plan([(kind, 2**31 - 1)])
        out = ctx.bootstrap("int8", x)
        torch.cuda.synchronize()
        assert np.array_equal(cggi.to_host(out), want), (p.name, kind)
    ctx.int8_plan(None)
    say(f"params {p.name} key switch B={B}")
    ks = ctx.keyswitch(cggi.to_device(want))
    torch.cuda.synchronize()
    want_ks = np.stack([O.keyswitch(p, ksk, w) for w in want])
    assert np.array_equal(cggi.to_host(ks), want_ks), p.name
    ctx.close()
