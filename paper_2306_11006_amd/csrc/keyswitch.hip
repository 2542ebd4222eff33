// keyswitch.hip -- LWE key switching N -> n on gfx950 (ArctyrEX Fig. 1,
// final step), plus the fused post-step of a gate level.
//
//   out = (0, .., 0, b') - sum_{j < N} sum_{p < t} ksk[j][p][d_{j,p}]
//   d_{j,p} = ((a'_j + 2^(31 - t*gamma)) >> (32 - (p+1)*gamma)) & (2^gamma-1)
//
// Work split: a workgroup owns KS_GATES ciphertexts and runs KS_JSPLIT
// wavefronts on each, every one summing the rows of a contiguous range of
// j; the partial sums meet in LDS.  The 64 lanes of a wavefront own the n+1
// output columns (NCH chunks of 64), so every gathered key row is read as
// coalesced 256-byte segments.  The digits are wave-uniform: each lane
// loads one a'_j of a 64-wide chunk, the wave broadcasts them one by one
// with readlane, and the digit, row address and loop control stay in scalar
// registers.  Rows of up to KS_PCH levels are fetched before any of them is
// used, so many loads are in flight per wave.  The key-switching key (tens
// of MB) is shared by every wave and stays in L2 / Infinity Cache; the
// ciphertexts of one workgroup walk j in step, so their gathers of the same
// (j, p) rows also share the L1.
#include "internal.hpp"

namespace cggi {

namespace {

constexpr int KS_GATES = 4;    // ciphertexts per workgroup
constexpr int KS_JSPLIT = 2;   // wavefronts per ciphertext (j ranges)
constexpr int KS_PCH = 4;      // key-switch levels fetched together
constexpr int KS_THREADS = 64 * KS_GATES * KS_JSPLIT;

// Source of the big ciphertext of item `it`:
//   plain batch: src = in + it*(N+1)
//   gate level : gate `it` reads ws_big[slot] (+ ws_big[slot+1] and +1/8
//                on the body for MUX), writes wires[out]
struct KsLevel {
    const cggi_gate_t *gates;
    const int32_t *slot;      // first bootstrap slot of each gate, -1 if none
    const uint32_t *big;      // [2G][N+1]
    uint32_t *wires;          // [W][n+1]
    int W;
};

template <int NCH, bool LEVEL>
__global__ __launch_bounds__(KS_THREADS) void k_keyswitch(
    const uint32_t *__restrict__ ksk, const uint32_t *__restrict__ in,
    uint32_t *__restrict__ out, int B, KsLevel lv, int n, int N, int gamma,
    int t)
{
    __shared__ uint32_t part[KS_GATES][KS_JSPLIT - 1][64 * NCH];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int gsub = wave / KS_JSPLIT, jpart = wave % KS_JSPLIT;
    const int it = blockIdx.x * KS_GATES + gsub;
    const uint32_t *src0 = nullptr, *src1 = nullptr;
    uint32_t *dst = nullptr;
    bool live = it < B;
    if (live) {
        if (LEVEL) {
            cggi_gate_t gt = lv.gates[it];
            int s = lv.slot[it];
            if (s < 0 || gt.out < 0 || gt.out >= lv.W) {
                live = false;
            } else {
                src0 = lv.big + (size_t)s * (N + 1);
                if (gt.op == CGGI_MUX)
                    src1 = lv.big + (size_t)(s + 1) * (N + 1);
                dst = lv.wires + (size_t)gt.out * (n + 1);
            }
        } else {
            src0 = in + (size_t)it * (N + 1);
            dst = out + (size_t)it * (n + 1);
        }
    }
    const int base = 1 << gamma;
    const uint32_t round_off = (t * gamma < 32) ? 1u << (31 - t * gamma) : 0u;
    const size_t rowlen = (size_t)n + 1;

    uint32_t acc[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k)
        acc[k] = 0u;
    if (live) {
        if (jpart == 0) {
            uint32_t body = src0[N];
            if (src1)
                body += src1[N] + (1u << 29);
#pragma unroll
            for (int k = 0; k < NCH; ++k)
                if (lane + 64 * k == n)
                    acc[k] = body;
        }
        const int jlen = N / KS_JSPLIT;
        for (int j0 = jpart * jlen; j0 < (jpart + 1) * jlen; j0 += 64) {
            uint32_t a = src0[j0 + lane];
            if (src1)
                a += src1[j0 + lane];
            a += round_off;
            for (int jj = 0; jj < 64; ++jj) {
                const uint32_t u = __builtin_amdgcn_readlane(a, jj);
                const uint32_t *rows =
                    ksk + (size_t)(j0 + jj) * t * base * rowlen;
                for (int p0 = 0; p0 < t; p0 += KS_PCH) {
                    uint32_t v[KS_PCH][NCH];
#pragma unroll
                    for (int pp = 0; pp < KS_PCH; ++pp) {
                        const int p = p0 + pp;
                        if (p < t) {
                            uint32_t d = (u >> (32 - (p + 1) * gamma)) &
                                         (base - 1);
                            const uint32_t *row =
                                rows + ((size_t)p * base + d) * rowlen;
#pragma unroll
                            for (int k = 0; k < NCH; ++k) {
                                int col = lane + 64 * k;
                                v[pp][k] = col <= n ? row[col] : 0u;
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < NCH; ++k)
                                v[pp][k] = 0u;
                        }
                    }
#pragma unroll
                    for (int pp = 0; pp < KS_PCH; ++pp)
#pragma unroll
                        for (int k = 0; k < NCH; ++k)
                            acc[k] -= v[pp][k];
                }
            }
        }
    }
    if (jpart > 0) {
#pragma unroll
        for (int k = 0; k < NCH; ++k)
            part[gsub][jpart - 1][lane + 64 * k] = acc[k];
    }
    __syncthreads();
    if (jpart == 0 && live) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            int col = lane + 64 * k;
            uint32_t x = acc[k];
            for (int q = 0; q < KS_JSPLIT - 1; ++q)
                x += part[gsub][q][col];
            if (col <= n)
                dst[col] = x;
        }
    }
}

template <bool LEVEL>
int ks_dispatch(const Ctx *c, const uint32_t *in, uint32_t *out, int B,
                KsLevel lv, hipStream_t s)
{
    const Shape &sh = c->sh;
    int nch = (sh.n + 1 + 63) / 64;
    dim3 grid((B + KS_GATES - 1) / KS_GATES), block(KS_THREADS);
#define KS_CASE(K)                                                           \
    case K:                                                                  \
        hipLaunchKernelGGL((k_keyswitch<K, LEVEL>), grid, block, 0, s,       \
                           c->ksk, in, out, B, lv, sh.n, sh.N, sh.gamma,     \
                           sh.t);                                            \
        break;
    switch (nch) {
        KS_CASE(1) KS_CASE(2) KS_CASE(3) KS_CASE(4) KS_CASE(5) KS_CASE(6)
        KS_CASE(7) KS_CASE(8) KS_CASE(9) KS_CASE(10) KS_CASE(11) KS_CASE(12)
        KS_CASE(13) KS_CASE(14) KS_CASE(15) KS_CASE(16)
    default:
        return set_error(CGGI_E_PARAM, "key switch: n + 1 > 1024");
    }
#undef KS_CASE
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

} // namespace

int keyswitch_launch(const Ctx *c, const uint32_t *in, uint32_t *out, int B,
                     hipStream_t s)
{
    KsLevel lv{};
    return ks_dispatch<false>(c, in, out, B, lv, s);
}

int keyswitch_level(const Ctx *c, const cggi_gate_t *gates,
                    const int32_t *slot, const uint32_t *big,
                    uint32_t *wires, int G, int W, hipStream_t s)
{
    KsLevel lv{gates, slot, big, wires, W};
    return ks_dispatch<true>(c, nullptr, nullptr, G, lv, s);
}

} // namespace cggi
