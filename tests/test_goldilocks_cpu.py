"""Host checks of the NTT form's arithmetic modulo Q = 2^64 - 2^32 + 1
(csrc/goldilocks.hpp, the modulus of the paper's exact NTT, Section 5.4):
add, the unreduced add_lazy of the Cooley-Tukey butterflies, sub and the
128-bit reduction, against 128-bit integer arithmetic on edge values (0,
1, Q - 1, the unreduced range [Q, 2^64), 2^64 - 1, values next to 2^32 and
2^63) and seeded random words.  add_lazy must stay below 2^64 for every
a < 2^64 and canonical b and agree with a + b mod Q; sub must do the same
for any a and canonical b.  The reduction is also driven through its wrap
corrections: low words just below, at and above the high word's top half
(the subtraction borrows) and high words with every half-word edge.  Compiled with hipcc; the checks run on the
host (the header's host/device functions), no GPU needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2306_11006_amd", "csrc", "goldilocks.hpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r"""
#include "goldilocks.hpp"
#include <cstdio>
#include <cstdint>
#include <vector>
using namespace cggi::gl;
typedef unsigned __int128 u128;
static uint64_t s = 0x2306110062306110ull;
static uint64_t rnd() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
int main() {
    std::vector<uint64_t> A = {0, 1, 2, Q - 2, Q - 1, Q, Q + 1, ~0ull, ~0ull - 1,
        0xFFFFFFFF00000000ull, 0xFFFFFFFFull, 0x100000000ull, 1ull << 63,
        (1ull << 63) - 1, 0xFFFFFFFEFFFFFFFFull};
    std::vector<uint64_t> B = {0, 1, 2, Q - 1, Q - 2, 0xFFFFFFFFull,
        0x100000000ull, 1ull << 63, 0xFFFFFFFE00000000ull};
    for (int k = 0; k < 200000; ++k) { A.push_back(rnd()); B.push_back(rnd() % Q); }
    long bad = 0, n = 0;
    for (size_t i = 0; i < A.size(); ++i) {
        for (size_t j = 0; j < (i < 64 ? B.size() : 4); ++j) {
            uint64_t a = A[i], b = B[(j + i) % B.size()];
            if (i >= 64) b = B[(i * 7 + j * 13) % B.size()];
            u128 want = ((u128)(a % Q) + b) % Q;
            uint64_t l = add_lazy(a, b);
            if ((u128)l % Q != want) ++bad;
            if (a < Q && add(a, b) != (uint64_t)want) ++bad;
            if (a < Q && add(a, b) >= Q) ++bad;
            u128 wsub = ((u128)(a % Q) + Q - b) % Q;
            if ((u128)sub(a, b) % Q != wsub) ++bad;
            if (a < Q && sub(a, b) >= Q) ++bad;
            uint64_t hi = a, lo = rnd();
            u128 x = ((u128)hi << 64) | lo;
            uint64_t r = reduce128(hi, lo);
            if (r >= Q || (u128)r != x % Q) ++bad;
            n += 1;
        }
    }
    // reduce128's wrap corrections: low words below the high word's top
    // half (borrow), high words whose low half shifted up carries, both.
    std::vector<uint64_t> L = {0, 1, 2, 0xFFFFFFFEull, 0xFFFFFFFFull,
        0x100000000ull, Q - 1, Q, ~0ull, ~0ull - 0xFFFFFFFFull};
    for (size_t i = 0; i < A.size(); ++i) {
        const uint64_t hi = A[i], h1 = hi >> 32;
        uint64_t los[16] = {h1 - 1, h1, h1 + 1, rnd() >> 40, rnd() % (h1 + 1)};
        int nl = 5;
        if (i < 64)
            for (uint64_t v : L) los[nl++ % 16] = v;
        for (int k = 0; k < nl && k < 16; ++k) {
            const uint64_t lo = los[k];
            u128 x = ((u128)hi << 64) | lo;
            uint64_t r = reduce128(hi, lo);
            if (r >= Q || (u128)r != x % Q) ++bad;
            n += 1;
        }
    }
    printf("%ld %ld\n", n, bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC),
                    reason="hipcc not found")
def test_goldilocks_host_arithmetic(tmp_path):
    src = tmp_path / "gl_check.cpp"
    exe = tmp_path / "gl_check"
    src.write_text(SRC)
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip",
                        "--offload-arch=gfx950", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops",
                        f"-I{os.path.dirname(HDR)}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    n, bad = (int(v) for v in out.stdout.split())
    assert n > 200000 and bad == 0, out.stdout
