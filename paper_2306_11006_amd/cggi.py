"""ctypes binding of libcggi.so (the C ABI declared in include/cggi.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Device buffers are torch tensors (int32 or uint32
dtype, contiguous, on the context's GPU); streams default to torch's current
stream.  If the library has not been built, importing this module raises.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcggi.so")

FORM_NTT = 1
FORM_INT8 = 2
FORMS = {"ntt": FORM_NTT, "int8": FORM_INT8}

OK = 0
E_PARAM, E_SHAPE, E_ALIAS, E_HIP, E_NOMEM, E_UNSUPPORTED, E_TIMEOUT = \
    -1, -2, -3, -4, -5, -6, -7

OPCODES = {"NAND": 0, "AND": 1, "OR": 2, "XOR": 3, "MUX": 4, "NOT": 5,
           "COPY": 6, "CONST0": 7, "CONST1": 8, "NOR": 9, "XNOR": 10}

EXPORTS = ["cggi_params_check", "cggi_ctx_create", "cggi_ctx_destroy",
           "cggi_ctx_reserve", "cggi_bootstrap_batch", "cggi_keyswitch_batch",
           "cggi_eval_level", "cggi_levelize", "cggi_ctx_profile",
           "cggi_ctx_profile_read", "cggi_measure_int8_mfma",
           "cggi_measure_mulmod",
           "cggi_ctx_latency_mode", "cggi_ctx_latency_groups",
           "cggi_ctx_check", "cggi_ctx_int8_plan", "cggi_ctx_int8_plan_get",
           "cggi_ctx_int8_limits", "cggi_ctx_latency_abort",
           "cggi_eval_level_noalloc", "cggi_last_error"]

# INT8 kernel kinds of a plan (cggi_ctx_int8_plan), in the header's order
KINDS = ("split4", "split2", "tiles1", "tiles2", "tiles4", "split8",
         "kara2")
INT32_MAX = 2**31 - 1


class CggiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cggi error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in
                ("n", "N", "k", "bg_bit", "l", "ks_base_bit", "ks_t")]


_lib = None


def lib():
    """Load libcggi.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing; build it with "
                "paper_2306_11006_amd/build.py (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.cggi_params_check.argtypes = [ctypes.POINTER(Params)]
        L.cggi_ctx_create.argtypes = [ctypes.POINTER(Params), vp, vp,
                                      ctypes.c_uint32, vp,
                                      ctypes.POINTER(vp)]
        L.cggi_ctx_destroy.argtypes = [vp]
        L.cggi_ctx_reserve.argtypes = [vp, i32]
        L.cggi_bootstrap_batch.argtypes = [vp, ctypes.c_int, vp, vp, vp, i32,
                                           vp]
        L.cggi_keyswitch_batch.argtypes = [vp, vp, vp, i32, vp]
        L.cggi_eval_level.argtypes = [vp, ctypes.c_int, vp, i32, vp, i32, vp]
        L.cggi_eval_level_noalloc.argtypes = [vp, ctypes.c_int, vp, i32, vp,
                                              i32, vp]
        L.cggi_levelize.argtypes = [vp, i32, i32, vp, vp,
                                    ctypes.POINTER(i32), vp]
        L.cggi_ctx_profile.argtypes = [vp, ctypes.c_int]
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)
        L.cggi_ctx_profile_read.argtypes = [vp, dp, ip, dp, ip]
        L.cggi_measure_mulmod.argtypes = [i32, dp]
        L.cggi_ctx_latency_mode.argtypes = [vp, i32]
        L.cggi_ctx_latency_groups.argtypes = [vp, ip]
        L.cggi_ctx_check.argtypes = [vp]
        L.cggi_ctx_int8_plan.argtypes = [vp, ip, ip, i32]
        L.cggi_ctx_int8_plan_get.argtypes = [vp, ip, ip, i32, ip]
        L.cggi_ctx_int8_limits.argtypes = [vp, ip]
        L.cggi_ctx_latency_abort.argtypes = [vp]
        L.cggi_last_error.restype = ctypes.c_char_p
        for name in EXPORTS[:-1]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise CggiError(rc, lib().cggi_last_error().decode())


def params_struct(p):
    """Params from a paper_2306_11006_amd.params.Params or a tuple."""
    vals = p.as_tuple() if hasattr(p, "as_tuple") else tuple(p)
    return Params(*vals)


def params_check(p):
    """Return (code, message) of cggi_params_check (host only)."""
    L = lib()
    ps = params_struct(p)
    rc = L.cggi_params_check(ctypes.byref(ps))
    return rc, (L.cggi_last_error().decode() if rc else "")


def measure_int8_mfma(iters=40000, random_operands=True):
    """Tera int8 operations per second a bare v_mfma_i32_32x32x32_i8 loop
    sustains on the current device (random or all-zero operands)."""
    out = ctypes.c_double()
    _check(lib().cggi_measure_int8_mfma(int(iters), int(bool(random_operands)),
                                        ctypes.byref(out)))
    return out.value


def measure_mulmod(iters=20000):
    """Tera Goldilocks multiply-mods per second a bare loop of the NTT
    form's multiply-mod sustains on the current device."""
    out = ctypes.c_double()
    _check(lib().cggi_measure_mulmod(int(iters), ctypes.byref(out)))
    return out.value


def levelize(gates, n_wires):
    """Host levelisation (cggi_levelize): returns (order, level_start) as
    numpy int32 arrays; level L is gates[order[level_start[L]:
    level_start[L+1]]]."""
    import numpy as np
    g = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
    G = g.shape[0]
    order = np.empty(G, dtype=np.int32)
    start = np.empty(G + 1, dtype=np.int32)
    nl = ctypes.c_int32()
    _check(lib().cggi_levelize(g.ctypes.data_as(ctypes.c_void_p), G,
                               int(n_wires),
                               order.ctypes.data_as(ctypes.c_void_p),
                               start.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(nl), None))
    return order, start[: nl.value + 1].copy()


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    if t.dtype not in (torch.int32, torch.uint32):
        raise ValueError("expected an int32/uint32 tensor")
    return ctypes.c_void_p(t.data_ptr())


def _shape(t, name, *dims):
    """Raise ValueError unless tensor t has the given shape (None matches
    any extent).  Checked before any pointer reaches the C ABI, which takes
    sizes on trust from its arguments."""
    if t is None:
        return
    if t.dim() != len(dims) or any(d is not None and t.shape[i] != d
                                   for i, d in enumerate(dims)):
        want = "[" + ", ".join("*" if d is None else str(d)
                               for d in dims) + "]"
        raise ValueError(f"{name}: expected shape {want}, got "
                         f"{list(t.shape)}")


def _numel(t, name, shape):
    n = 1
    for d in shape:
        n *= d
    if t is None or t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements ({list(shape)}), "
                         f"got {None if t is None else t.numel()}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _form(form):
    return FORMS[form] if isinstance(form, str) else int(form)


class Context:
    """A cggi_ctx: derived key forms for one parameter set on one GPU."""

    def __init__(self, params, bsk, ksk, forms=("ntt", "int8"), stream=None):
        self.params = params
        self.forms = tuple(forms)
        self._ksk = ksk          # the library keeps a pointer to it
        mask = 0
        for f in forms:
            mask |= _form(f)
        _numel(bsk, "bsk", params.bsk_shape)
        _numel(ksk, "ksk", params.ksk_shape)
        self._ps = params_struct(params)
        h = ctypes.c_void_p()
        _check(lib().cggi_ctx_create(ctypes.byref(self._ps), _ptr(bsk),
                                     _ptr(ksk), mask, _stream(stream),
                                     ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().cggi_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def profile(self, enable=True):
        _check(lib().cggi_ctx_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """(bootstrap ms, bootstrap launches, key-switch ms, key-switch
        launches) summed since the last read."""
        bm, km = ctypes.c_double(), ctypes.c_double()
        bn, kn = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().cggi_ctx_profile_read(self._h, ctypes.byref(bm),
                                           ctypes.byref(bn), ctypes.byref(km),
                                           ctypes.byref(kn)))
        return bm.value, bn.value, km.value, kn.value

    def latency_mode(self, enable=True):
        """Turn the INT8 form's latency mode (narrow batches over four CUs
        per column tile) on or off."""
        _check(lib().cggi_ctx_latency_mode(self._h, int(bool(enable))))

    def latency_groups(self):
        """Most column tiles a latency-mode launch takes (0: off)."""
        g = ctypes.c_int32()
        _check(lib().cggi_ctx_latency_groups(self._h, ctypes.byref(g)))
        return g.value

    def int8_plan(self, plan=None):
        """Set the INT8 kernel plan: a list of (kind, cap) with kind a name
        of KINDS (or its index) and strictly increasing caps, the last at
        least 2^24; None or [] restores the built-in plan."""
        plan = list(plan or [])
        n = len(plan)
        kinds = (ctypes.c_int32 * max(n, 1))(
            *[KINDS.index(k) if isinstance(k, str) else int(k)
              for k, _ in plan])
        caps = (ctypes.c_int32 * max(n, 1))(*[int(c) for _, c in plan])
        _check(lib().cggi_ctx_int8_plan(self._h, kinds, caps, n))

    def int8_plan_get(self):
        """The INT8 kernel plan in force, as [(kind name, cap)]."""
        kinds = (ctypes.c_int32 * 8)()
        caps = (ctypes.c_int32 * 8)()
        n = ctypes.c_int32()
        _check(lib().cggi_ctx_int8_plan_get(self._h, kinds, caps, 8,
                                            ctypes.byref(n)))
        return [(KINDS[kinds[k]], caps[k]) for k in range(n.value)]

    def int8_limits(self):
        """{kind name: most bootstraps one launch of it may take} (0 when
        the kind is unavailable)."""
        lim = (ctypes.c_int32 * len(KINDS))()
        _check(lib().cggi_ctx_int8_limits(self._h, lim))
        return {KINDS[k]: lim[k] for k in range(len(KINDS))}

    def latency_abort(self):
        """Stop latency-mode kernels now and refuse new ones until check()."""
        _check(lib().cggi_ctx_latency_abort(self._h))

    def check(self):
        """Wait for the device; raise CggiError(E_TIMEOUT) if a
        latency-mode launch timed out since the last check."""
        _check(lib().cggi_ctx_check(self._h))

    def reserve(self, max_gates):
        _check(lib().cggi_ctx_reserve(self._h, int(max_gates)))

    def bootstrap(self, form, inp, out=None, testv=None, stream=None):
        p = self.params
        _shape(inp, "inp", None, p.n + 1)
        B = inp.shape[0]
        _shape(out, "out", B, p.N + 1)
        if testv is not None:
            _numel(testv, "testv", (p.N,))
        if out is None:
            out = torch.empty((B, p.N + 1), dtype=torch.int32,
                              device=inp.device)
        _check(lib().cggi_bootstrap_batch(self._h, _form(form), _ptr(inp),
                                          _ptr(testv), _ptr(out), B,
                                          _stream(stream)))
        return out

    def keyswitch(self, inp, out=None, stream=None):
        p = self.params
        _shape(inp, "inp", None, p.N + 1)
        B = inp.shape[0]
        _shape(out, "out", B, p.n + 1)
        if out is None:
            out = torch.empty((B, p.n + 1), dtype=torch.int32,
                              device=inp.device)
        _check(lib().cggi_keyswitch_batch(self._h, _ptr(inp), _ptr(out), B,
                                          _stream(stream)))
        return out

    def eval_level(self, form, gates, wires, stream=None):
        """gates: int32 tensor [G, 5] (op, in0, in1, in2, out); wires:
        int32 tensor [W, n+1], updated in place."""
        _shape(gates, "gates", None, 5)
        _shape(wires, "wires", None, self.params.n + 1)
        G = gates.shape[0]
        W = wires.shape[0]
        _check(lib().cggi_eval_level(self._h, _form(form), _ptr(gates), G,
                                     _ptr(wires), W, _stream(stream)))
        return wires

    def eval_level_noalloc(self, form, gates, wires, stream=None):
        """eval_level on the library's fixed device workspace
        (cggi_eval_level_noalloc): allocates nothing, no reserve needed;
        calls that overlap on one GPU race."""
        _shape(gates, "gates", None, 5)
        _shape(wires, "wires", None, self.params.n + 1)
        G = gates.shape[0]
        W = wires.shape[0]
        _check(lib().cggi_eval_level_noalloc(self._h, _form(form),
                                             _ptr(gates), G, _ptr(wires), W,
                                             _stream(stream)))
        return wires



def to_device(a, device="cuda"):
    """numpy uint32 array -> int32 CUDA tensor with the same bits."""
    import numpy as np
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(device)


def to_host(t):
    """int32 tensor -> numpy uint32 array with the same bits."""
    import numpy as np
    return t.cpu().numpy().view(np.uint32)
