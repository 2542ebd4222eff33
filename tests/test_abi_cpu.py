"""Host-side checks of the C ABI: the library loads, exports every function
include/cggi.h declares, and rejects bad parameters on the host (no GPU
call is made by any of these tests)."""
import os
import re

import pytest

from paper_2306_11006_amd import params
from paper_2306_11006_amd import cggi

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include",
                      "cggi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cggi_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "cggi_bootstrap_batch" in names and len(names) >= 8
    L = cggi.lib()
    for name in names:
        assert hasattr(L, name), name
    assert sorted(cggi.EXPORTS) == names, (sorted(cggi.EXPORTS), names)


@pytest.mark.parametrize("p", [params.TOY, params.DEFAULT, params.LARGE])
def test_params_accepted(p):
    assert cggi.params_check(p) == (0, "")


BAD = [
    (dict(k=2), "k must be 1"),
    (dict(N=300), "N must be"),
    (dict(N=4096), "N must be"),
    (dict(n=0), "n must be"),
    (dict(n=2000), "n must be"),
    (dict(bg_bit=0), "bg_bit"),
    (dict(bg_bit=11, l=3), "bg_bit * l"),
    (dict(ks_base_bit=0), "ks_base_bit"),
    (dict(ks_base_bit=4, ks_t=8), "ks_base_bit * ks_t"),
    (dict(bg_bit=30, l=1, N=2048), "Q/2"),
]


@pytest.mark.parametrize("change,msg", BAD)
def test_params_rejected(change, msg):
    import dataclasses
    p = dataclasses.replace(params.DEFAULT, **change)
    rc, text = cggi.params_check(p)
    assert rc == cggi.E_PARAM
    assert msg in text


def test_null_params_rejected():
    L = cggi.lib()
    assert L.cggi_params_check(None) == cggi.E_PARAM
    assert b"NULL" in L.cggi_last_error()


def test_create_rejects_bad_arguments_before_any_gpu_work():
    import ctypes
    L = cggi.lib()
    ps = cggi.params_struct(params.TOY)
    h = ctypes.c_void_p()
    # null output handle
    assert L.cggi_ctx_create(ctypes.byref(ps), None, None, 1, None,
                             None) == cggi.E_SHAPE
    # empty / unknown form mask
    assert L.cggi_ctx_create(ctypes.byref(ps), None, None, 0, None,
                             ctypes.byref(h)) == cggi.E_PARAM
    assert L.cggi_ctx_create(ctypes.byref(ps), None, None, 4, None,
                             ctypes.byref(h)) == cggi.E_PARAM
    # null keys
    assert L.cggi_ctx_create(ctypes.byref(ps), None, None, 1, None,
                             ctypes.byref(h)) == cggi.E_SHAPE
    # misaligned keys
    assert L.cggi_ctx_create(ctypes.byref(ps), ctypes.c_void_p(2),
                             ctypes.c_void_p(8), 1, None,
                             ctypes.byref(h)) == cggi.E_SHAPE
    # int8 form splits digits into at most two 7-bit parts (Bg <= 2^13)
    import dataclasses
    pl = cggi.params_struct(dataclasses.replace(params.LARGE, bg_bit=14,
                                                l=1))
    assert L.cggi_ctx_create(ctypes.byref(pl), ctypes.c_void_p(16),
                             ctypes.c_void_p(16), 2, None,
                             ctypes.byref(h)) == cggi.E_PARAM
    assert b"bg_bit" in L.cggi_last_error()
    assert h.value is None
    # int8 form at N=1024 with sixteen digit rows (Bg=2^3, l=8): the
    # workgroup's digit operands no longer fit the 160 KB of LDS
    pw = cggi.params_struct(dataclasses.replace(params.DEFAULT, bg_bit=3,
                                                l=8))
    assert L.cggi_params_check(ctypes.byref(pw)) == cggi.OK
    assert L.cggi_ctx_create(ctypes.byref(pw), ctypes.c_void_p(16),
                             ctypes.c_void_p(16), 2, None,
                             ctypes.byref(h)) == cggi.E_PARAM
    assert b"LDS" in L.cggi_last_error()
    assert h.value is None


def test_mfma_ceiling_rejects_bad_arguments():
    import ctypes
    L = cggi.lib()
    out = ctypes.c_double()
    assert L.cggi_measure_int8_mfma(0, 1, ctypes.byref(out)) == cggi.E_PARAM
    assert L.cggi_measure_int8_mfma(10, 1, None) == cggi.E_PARAM


def test_batch_calls_reject_null_context():
    L = cggi.lib()
    assert L.cggi_bootstrap_batch(None, 1, None, None, None, 4,
                                  None) == cggi.E_PARAM
    assert L.cggi_keyswitch_batch(None, None, None, 4, None) == cggi.E_PARAM
    assert L.cggi_eval_level(None, 1, None, 1, None, 1, None) == cggi.E_PARAM
    assert L.cggi_ctx_reserve(None, 4) == cggi.E_PARAM
    assert L.cggi_ctx_latency_mode(None, 1) == cggi.E_PARAM
    assert L.cggi_ctx_latency_groups(None, None) == cggi.E_PARAM
    assert L.cggi_ctx_check(None) == cggi.E_PARAM
    assert L.cggi_ctx_int8_plan(None, None, None, 0) == cggi.E_PARAM
    assert L.cggi_ctx_int8_plan_get(None, None, None, 0, None) == \
        cggi.E_PARAM
    assert L.cggi_ctx_int8_limits(None, None) == cggi.E_PARAM
    assert L.cggi_ctx_latency_abort(None) == cggi.E_PARAM
    assert L.cggi_ctx_destroy(None) == cggi.OK


def test_int8_form_rejects_more_than_eight_gadget_levels():
    """The INT8 form's generic digit loops cover at most 8 gadget levels;
    a context with more is refused on the host (N=2048, l=9, Bg=2^3 would
    otherwise fit the LDS)."""
    import ctypes
    import dataclasses
    L = cggi.lib()
    h = ctypes.c_void_p()
    p9 = dataclasses.replace(params.LARGE, bg_bit=3, l=9)
    ps = cggi.params_struct(p9)
    assert L.cggi_params_check(ctypes.byref(ps)) == cggi.OK
    assert L.cggi_ctx_create(ctypes.byref(ps), ctypes.c_void_p(16),
                             ctypes.c_void_p(16), 2, None,
                             ctypes.byref(h)) == cggi.E_PARAM
    assert b"l must be <= 8" in L.cggi_last_error()
    assert h.value is None
    # l = 8 passes the host checks of the INT8 form (it fails later only
    # for want of a GPU, past every parameter check)
    p8 = cggi.params_struct(dataclasses.replace(params.LARGE, bg_bit=3, l=8))
    rc = L.cggi_ctx_create(ctypes.byref(p8), ctypes.c_void_p(16),
                           ctypes.c_void_p(16), 2, None, ctypes.byref(h))
    assert rc != cggi.E_PARAM or b"l must be" not in L.cggi_last_error()


def _fake_context(p):
    """A Context object that never reached the C ABI (no GPU needed): the
    wrapper's own argument checks run before any pointer is passed."""
    ctx = cggi.Context.__new__(cggi.Context)
    ctx.params = p
    ctx.forms = ("ntt", "int8")
    ctx._h = None
    return ctx


def test_wrapper_rejects_bad_shapes_before_the_c_call():
    import torch
    p = params.TOY
    ctx = _fake_context(p)
    n1, N1 = p.n + 1, p.N + 1
    i32 = torch.int32
    bad = [
        lambda: ctx.bootstrap("int8", torch.zeros(n1, dtype=i32)),  # 1-D
        lambda: ctx.bootstrap("int8", torch.zeros((4, N1), dtype=i32)),
        lambda: ctx.bootstrap("int8", torch.zeros((4, n1), dtype=i32),
                              out=torch.zeros((3, N1), dtype=i32)),
        lambda: ctx.bootstrap("int8", torch.zeros((4, n1), dtype=i32),
                              out=torch.zeros((4, N1), dtype=i32),
                              testv=torch.zeros(p.N - 1, dtype=i32)),
        lambda: ctx.keyswitch(torch.zeros((4, n1), dtype=i32)),
        lambda: ctx.keyswitch(torch.zeros((4, N1), dtype=i32),
                              out=torch.zeros((4, N1), dtype=i32)),
        lambda: ctx.eval_level("int8", torch.zeros((3, 4), dtype=i32),
                               torch.zeros((8, n1), dtype=i32)),
        lambda: ctx.eval_level("int8", torch.zeros(15, dtype=i32),
                               torch.zeros((8, n1), dtype=i32)),
        lambda: ctx.eval_level("int8", torch.zeros((3, 5), dtype=i32),
                               torch.zeros((8, n1 - 1), dtype=i32)),
    ]
    for k, f in enumerate(bad):
        with pytest.raises(ValueError):
            f()
            raise AssertionError(f"case {k} passed")


def test_context_rejects_wrong_key_sizes_before_the_c_call():
    import torch
    p = params.TOY
    bsk = torch.zeros(p.bsk_shape, dtype=torch.int32)
    ksk = torch.zeros(p.ksk_shape, dtype=torch.int32)
    with pytest.raises(ValueError, match="bsk"):
        cggi.Context(p, bsk[:-1], ksk)
    with pytest.raises(ValueError, match="ksk"):
        cggi.Context(p, bsk, ksk[:, :-1])


def test_mulmod_ceiling_rejects_bad_arguments():
    import ctypes
    L = cggi.lib()
    out = ctypes.c_double()
    assert L.cggi_measure_mulmod(0, ctypes.byref(out)) == cggi.E_PARAM
    assert L.cggi_measure_mulmod(10, None) == cggi.E_PARAM
