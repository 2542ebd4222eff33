"""numpy front end of the C oracle (test infrastructure only).

Every function takes and returns numpy arrays of uint32 torus values (int32
digits where noted) in the row-major layouts of the GPU library:
  LWE  [.., n+1]      TRLWE [.., 2, N]      bsk [n, 2l, 2, N]
  ksk  [N, t, 2^gamma, n+1]
The arithmetic lives in cggi_oracle.c; see the comments there for the
passage of the paper each routine follows.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

__all__ = [
    "lib", "poly_mul", "mono_mul", "modswitch", "decomp", "ks_digits",
    "lwe_encrypt", "lwe_phase", "lwe_decrypt", "make_bsk", "make_ksk",
    "external_product", "cmux_rotate", "blind_rotate", "sample_extract",
    "bootstrap", "bootstrap_batch", "keyswitch", "keyswitch_batch", "gate",
    "gate_preop", "OPS",
]

OPS = {"NAND": 0, "AND": 1, "OR": 2, "XOR": 3, "MUX": 4, "NOT": 5,
       "COPY": 6, "CONST0": 7, "CONST1": 8, "NOR": 9, "XNOR": 10}

_lib = None
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_I = ctypes.c_int
_L = ctypes.c_long


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        sigs = {
            "orc_mono_mul": [_I, _I, _u32p, _u32p],
            "orc_poly_mul": [_I, _u32p, _u32p, _u32p],
            "orc_modswitch_array": [_u32p, _u32p, _L, _I],
            "orc_decomp_array": [_u32p, _i32p, _L, _I, _I],
            "orc_ks_digits_array": [_u32p, _u32p, _L, _I, _I],
            "orc_lwe_encrypt": [_I, _u8p, _u32p, ctypes.c_int32,
                                ctypes.c_uint32, _u32p],
            "orc_lwe_phase": [_I, _u8p, _u32p],
            "orc_lwe_decrypt": [_I, _u8p, _u32p],
            "orc_make_bsk": [_I, _I, _I, _I, _u8p, _u8p, _u32p, _i32p, _u32p],
            "orc_make_ksk": [_I, _I, _I, _I, _u8p, _u8p, _u32p, _i32p, _u32p],
            "orc_external_product": [_I, _I, _I, _u32p, _u32p, _u32p],
            "orc_cmux_rotate": [_I, _I, _I, _u32p, _I, _u32p],
            "orc_blind_rotate": [_I, _I, _I, _I, _u32p, _u32p, _u32p, _u32p],
            "orc_sample_extract": [_I, _u32p, _u32p],
            "orc_bootstrap": [_I, _I, _I, _I, _u32p, _u32p, _u32p, _u32p],
            "orc_bootstrap_batch": [_I, _I, _I, _I, _u32p, _u32p, _u32p,
                                    _u32p, _I],
            "orc_keyswitch": [_I, _I, _I, _I, _u32p, _u32p, _u32p],
            "orc_keyswitch_batch": [_I, _I, _I, _I, _u32p, _u32p, _u32p, _I],
            "orc_gate": [_I, _I, _I, _I, _I, _I, _I, _u32p, _u32p, _u32p,
                         _u32p, _u32p, _u32p],
            "orc_gate_preop": [_I, _I, _I, _u32p, _u32p, _u32p, _u32p],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None
        L.orc_lwe_phase.restype = ctypes.c_uint32
        L.orc_lwe_decrypt.restype = ctypes.c_int
        _lib = L
    return _lib


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _p(a, typ):
    if a is None:
        return ctypes.cast(None, typ)
    return a.ctypes.data_as(typ)


def poly_mul(x, y):
    """Negacyclic product x*y mod (X^N+1, 2^32); 1-D arrays of length N."""
    x, y = _u32(x), _u32(y)
    out = np.empty_like(x)
    lib().orc_poly_mul(x.size, _p(x, _u32p), _p(y, _u32p), _p(out, _u32p))
    return out


def mono_mul(e, p):
    """X^e * p, e in [0, 2N)."""
    p = _u32(p)
    out = np.empty_like(p)
    lib().orc_mono_mul(p.size, int(e), _p(p, _u32p), _p(out, _u32p))
    return out


def modswitch(u, N):
    u = _u32(u).ravel()
    out = np.empty_like(u)
    lib().orc_modswitch_array(_p(u, _u32p), _p(out, _u32p), u.size, N)
    return out


def decomp(u, beta, l):
    """[count] -> [count, l] int32 digits."""
    u = _u32(u).ravel()
    d = np.empty((u.size, l), dtype=np.int32)
    lib().orc_decomp_array(_p(u, _u32p), _p(d, _i32p), u.size, beta, l)
    return d


def ks_digits(u, gamma, t):
    u = _u32(u).ravel()
    d = np.empty((u.size, t), dtype=np.uint32)
    lib().orc_ks_digits_array(_p(u, _u32p), _p(d, _u32p), u.size, gamma, t)
    return d


def lwe_encrypt(s, a, e, mu):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    a = _u32(a)
    ct = np.empty(a.size + 1, dtype=np.uint32)
    lib().orc_lwe_encrypt(s.size, _p(s, _u8p), _p(a, _u32p), int(e),
                          int(mu) & 0xFFFFFFFF, _p(ct, _u32p))
    return ct


def lwe_phase(s, ct):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    ct = _u32(ct)
    return int(lib().orc_lwe_phase(s.size, _p(s, _u8p), _p(ct, _u32p)))


def lwe_decrypt(s, ct):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    ct = _u32(ct)
    return int(lib().orc_lwe_decrypt(s.size, _p(s, _u8p), _p(ct, _u32p)))


def make_bsk(p, s, K, a, e):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    K = np.ascontiguousarray(K, dtype=np.uint8)
    a = _u32(a)
    e = np.ascontiguousarray(e, dtype=np.int32)
    bsk = np.empty((p.n, 2 * p.l, 2, p.N), dtype=np.uint32)
    lib().orc_make_bsk(p.n, p.N, p.bg_bit, p.l, _p(s, _u8p), _p(K, _u8p),
                       _p(a, _u32p), _p(e, _i32p), _p(bsk, _u32p))
    return bsk


def make_ksk(p, s, K, a, e):
    s = np.ascontiguousarray(s, dtype=np.uint8)
    K = np.ascontiguousarray(K, dtype=np.uint8)
    a = _u32(a)
    e = np.ascontiguousarray(e, dtype=np.int32)
    base = 1 << p.ks_base_bit
    ksk = np.empty((p.N, p.ks_t, base, p.n + 1), dtype=np.uint32)
    lib().orc_make_ksk(p.n, p.N, p.ks_base_bit, p.ks_t, _p(s, _u8p),
                       _p(K, _u8p), _p(a, _u32p), _p(e, _i32p), _p(ksk, _u32p))
    return ksk


def external_product(N, beta, l, C, d):
    C, d = _u32(C), _u32(d)
    out = np.empty((2, N), dtype=np.uint32)
    lib().orc_external_product(N, beta, l, _p(C, _u32p), _p(d, _u32p),
                               _p(out, _u32p))
    return out


def cmux_rotate(N, beta, l, C, e, acc):
    acc = _u32(acc).copy()
    C = _u32(C)
    lib().orc_cmux_rotate(N, beta, l, _p(C, _u32p), int(e), _p(acc, _u32p))
    return acc


def blind_rotate(p, bsk, ct, testv=None):
    bsk, ct = _u32(bsk), _u32(ct)
    tv = None if testv is None else _u32(testv)
    acc = np.empty((2, p.N), dtype=np.uint32)
    lib().orc_blind_rotate(p.n, p.N, p.bg_bit, p.l, _p(bsk, _u32p),
                           _p(tv, _u32p), _p(ct, _u32p), _p(acc, _u32p))
    return acc


def sample_extract(acc):
    acc = _u32(acc)
    N = acc.shape[-1]
    out = np.empty(N + 1, dtype=np.uint32)
    lib().orc_sample_extract(N, _p(acc, _u32p), _p(out, _u32p))
    return out


def bootstrap(p, bsk, ct, testv=None):
    bsk, ct = _u32(bsk), _u32(ct)
    tv = None if testv is None else _u32(testv)
    out = np.empty(p.N + 1, dtype=np.uint32)
    lib().orc_bootstrap(p.n, p.N, p.bg_bit, p.l, _p(bsk, _u32p),
                        _p(tv, _u32p), _p(ct, _u32p), _p(out, _u32p))
    return out


def bootstrap_batch(p, bsk, cts, testv=None):
    bsk, cts = _u32(bsk), _u32(cts)
    tv = None if testv is None else _u32(testv)
    B = cts.shape[0]
    out = np.empty((B, p.N + 1), dtype=np.uint32)
    lib().orc_bootstrap_batch(p.n, p.N, p.bg_bit, p.l, _p(bsk, _u32p),
                              _p(tv, _u32p), _p(cts, _u32p), _p(out, _u32p), B)
    return out


def keyswitch(p, ksk, ct):
    ksk, ct = _u32(ksk), _u32(ct)
    out = np.empty(p.n + 1, dtype=np.uint32)
    lib().orc_keyswitch(p.n, p.N, p.ks_base_bit, p.ks_t, _p(ksk, _u32p),
                        _p(ct, _u32p), _p(out, _u32p))
    return out


def keyswitch_batch(p, ksk, cts):
    ksk, cts = _u32(ksk), _u32(cts)
    B = cts.shape[0]
    out = np.empty((B, p.n + 1), dtype=np.uint32)
    lib().orc_keyswitch_batch(p.n, p.N, p.ks_base_bit, p.ks_t, _p(ksk, _u32p),
                              _p(cts, _u32p), _p(out, _u32p), B)
    return out


def gate(p, op, bsk, ksk, x, y=None, z=None):
    """One gate of the paper's gate set; op is a name or an opcode."""
    op = OPS[op] if isinstance(op, str) else int(op)
    bsk, ksk, x = _u32(bsk), _u32(ksk), _u32(x)
    y = x if y is None else _u32(y)
    z = x if z is None else _u32(z)
    out = np.empty(p.n + 1, dtype=np.uint32)
    lib().orc_gate(op, p.n, p.N, p.bg_bit, p.l, p.ks_base_bit, p.ks_t,
                   _p(bsk, _u32p), _p(ksk, _u32p), _p(x, _u32p), _p(y, _u32p),
                   _p(z, _u32p), _p(out, _u32p))
    return out


def gate_preop(n, op, x, y=None, z=None, which=0):
    op = OPS[op] if isinstance(op, str) else int(op)
    x = _u32(x)
    y = x if y is None else _u32(y)
    z = x if z is None else _u32(z)
    out = np.empty(n + 1, dtype=np.uint32)
    lib().orc_gate_preop(op, which, n, _p(x, _u32p), _p(y, _u32p),
                         _p(z, _u32p), _p(out, _u32p))
    return out
