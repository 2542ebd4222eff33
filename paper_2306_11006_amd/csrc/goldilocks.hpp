// goldilocks.hpp -- arithmetic modulo Q = 2^64 - 2^32 + 1 on gfx950.
//
// The modulus of the paper's exact NTT (Section 5.4): 2^64 = 2^32 - 1 and
// 2^96 = -1 (mod Q), so a 128-bit product reduces with a few 64-bit adds.
// All functions take and return canonical residues in [0, Q).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cggi {
namespace gl {

constexpr uint64_t Q = 0xFFFFFFFF00000001ull;
constexpr uint64_t EPS = 0xFFFFFFFFull; // 2^64 mod Q

__host__ __device__ __forceinline__ uint64_t add(uint64_t a, uint64_t b)
{
    uint64_t r = a + b;
    if (r < a)          // carry out of 2^64: add 2^64 mod Q
        r += EPS;
    if (r >= Q)
        r -= Q;
    return r;
}

// a + b for any a < 2^64 and a canonical b < Q, left in [0, 2^64) rather
// than reduced to [0, Q): after a carry out of 2^64 the sum is below
// 2^64 + Q, so adding 2^64 mod Q = 2^32 - 1 cannot carry again.  The
// Cooley-Tukey butterflies use it (their V is always a fresh product); a
// product, or sub with a canonical subtrahend, takes such a value as is.
__host__ __device__ __forceinline__ uint64_t add_lazy(uint64_t a, uint64_t b)
{
    uint64_t r = a + b;
    if (r < a)
        r += EPS;
    return r;
}

// a - b for a canonical b (a anything below 2^64): on a borrow the result
// a - b + Q lies in (0, Q), otherwise a - b < 2^64.
__host__ __device__ __forceinline__ uint64_t sub(uint64_t a, uint64_t b)
{
    uint64_t r = a - b;
    if (a < b)          // borrow of 2^64: subtract 2^64 mod Q
        r -= EPS;
    return r;
}

// (hi * 2^64 + lo) mod Q
__host__ __device__ __forceinline__ uint64_t reduce128(uint64_t hi,
                                                       uint64_t lo)
{
    uint64_t hh = hi >> 32;             // * 2^96 = -1
    uint64_t hl = hi & 0xFFFFFFFFull;   // * 2^64 = 2^32 - 1
    uint64_t t0 = lo - hh;
    if (lo < hh)
        t0 -= EPS;
    uint64_t t1 = (hl << 32) - hl;
    uint64_t r = t0 + t1;
    if (r < t1)
        r += EPS;
    if (r >= Q)
        r -= Q;
    return r;
}

// 64 x 64 -> 128-bit product from four 32 x 32 + 64 multiply-adds
// (a*b and __umul64hi separately would repeat the partial products).
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t &hi,
                                       uint64_t &lo)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t m1 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t m2 = (uint64_t)a1 * b0 + (uint32_t)m1;
    lo = (m2 << 32) | (uint32_t)p00;
    hi = (uint64_t)a1 * b1 + (m1 >> 32) + (m2 >> 32);
}

__device__ __forceinline__ uint64_t mul(uint64_t a, uint64_t b)
{
    uint64_t hi, lo;
    mul128(a, b, hi, lo);
    return reduce128(hi, lo);
}

// A sum of products x * y (each below 2^128) kept as the 160-bit integer
// top * 2^128 + hi * 2^64 + lo and reduced once at the end, where
// 2^128 = 2^96 * 2^32 = -2^32 (mod Q).  Exact for fewer than 2^32 terms.
struct MacAcc {
    uint64_t lo, hi;
    uint32_t top;
};

__device__ __forceinline__ void mac(MacAcc &m, uint64_t x, uint64_t y)
{
    uint64_t h, l;
    mul128(x, y, h, l);
    unsigned long long c0, c1;
    m.lo = __builtin_addcll(m.lo, l, 0ull, &c0);
    m.hi = __builtin_addcll(m.hi, h, c0, &c1);
    m.top += (uint32_t)c1;
}

__device__ __forceinline__ uint64_t mac_reduce(const MacAcc &m)
{
    return sub(reduce128(m.hi, m.lo), (uint64_t)m.top << 32);
}

inline uint64_t mul_host(uint64_t a, uint64_t b)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    return reduce128((uint64_t)(p >> 64), (uint64_t)p);
}

inline uint64_t pow_host(uint64_t b, uint64_t e)
{
    uint64_t r = 1;
    while (e) {
        if (e & 1)
            r = mul_host(r, b);
        b = mul_host(b, b);
        e >>= 1;
    }
    return r;
}

// Signed integer -> residue.
__host__ __device__ __forceinline__ uint64_t from_i32(int32_t v)
{
    return v >= 0 ? (uint64_t)v : Q - (uint64_t)(-(int64_t)v);
}

// Residue of an integer Y with |Y| < Q/2 -> Y mod 2^32 (centred lift; the
// low word of Q is 1, so a negative Y = y - Q has low word y_lo - 1).
__host__ __device__ __forceinline__ uint32_t lift32(uint64_t y)
{
    uint32_t lo = (uint32_t)y;
    return y > (Q >> 1) ? lo - 1u : lo;
}

} // namespace gl
} // namespace cggi
