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
//
// For key-switch bases up to 2^4 the sum is computed instead as an int8
// GEMM on v_mfma_i32_32x32x32_i8 (k_ks_mfma): with the one-hot digit matrix
// A[g][(j, p, h)] = (d_{g,j,p} == h) and the key as four signed int8 limbs,
// sum_{j,p} ksk[j][p][d_{g,j,p}][c] = sum_k A[g][k] * ksk[k][c].  The key
// (tens of MB) is then streamed once per 64 ciphertexts instead of being
// gathered row by row for every ciphertext.
#include "internal.hpp"

#include <algorithm>

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

// Source(s) and destination of item `it`; false if it produces nothing.
template <bool LEVEL>
__device__ __forceinline__ bool ks_item(int it, int B, const uint32_t *in,
                                        uint32_t *out, const KsLevel &lv,
                                        int n, int N, const uint32_t *&src0,
                                        const uint32_t *&src1, uint32_t *&dst)
{
    src0 = src1 = nullptr;
    dst = nullptr;
    if (it >= B)
        return false;
    if (LEVEL) {
        const cggi_gate_t gt = lv.gates[it];
        const int s = lv.slot[it];
        if (s < 0 || gt.out < 0 || gt.out >= lv.W)
            return false;
        src0 = lv.big + (size_t)s * (N + 1);
        if (gt.op == CGGI_MUX)
            src1 = lv.big + (size_t)(s + 1) * (N + 1);
        dst = lv.wires + (size_t)gt.out * (n + 1);
    } else {
        src0 = in + (size_t)it * (N + 1);
        dst = out + (size_t)it * (n + 1);
    }
    return true;
}

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
    const uint32_t *src0, *src1;
    uint32_t *dst;
    const bool live = ks_item<LEVEL>(it, B, in, out, lv, n, N, src0, src1, dst);
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

// ---- key switching as an int8 GEMM ----------------------------------------
// K runs over (j, slot), slot = p * 2^gamma + h padded to KSJ * 32 per j, so
// one MFMA K-step of 32 covers one slot block of one j.  Operand layouts of
// v_mfma_i32_32x32x32_i8: lane l holds 16 consecutive k (k = 16 (l >> 5) +
// byte) of row l & 31 (A: ciphertext) or column l & 31 (B: key column).
typedef int ks_v4i __attribute__((ext_vector_type(4)));
typedef int ks_v16i __attribute__((ext_vector_type(16)));

constexpr int KSM_ITEMS = 64;   // ciphertexts per workgroup (2 row tiles)
constexpr int KSM_WAVES = 8;    // most column tiles per workgroup (1 / wave)
constexpr int KSM_JMAX = 256;   // most j per workgroup (LDS: 64 KB of a')

// ksk [N][t][2^gamma][n+1] -> limb blocks [NT][N][KSJ][4][64 lanes][16 B]:
// byte e of lane l in block (nt, j, sj, q) is limb q of
// ksk[j][p][h][32 nt + (l & 31)] for slot 32 sj + 16 (l >> 5) + e = p 2^gamma
// + h, zero where p >= t or the column is past n.  Limbs are signed:
// v = sum_q 2^(8q) v_q with v_q in [-128, 127].
__global__ __launch_bounds__(256) void k_ksk_to_i8(
    const uint32_t *__restrict__ ksk, uint32_t *__restrict__ out, int n,
    int N, int t, int gamma, int ksj, int nt_tiles)
{
    const size_t total = (size_t)nt_tiles * N * ksj * 4 * 256;   // dwords
    const int base = 1 << gamma;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
         idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int dw = (int)(idx & 255);
        size_t b = idx >> 8;
        const int q = (int)(b & 3);
        b >>= 2;
        const int sj = (int)(b % ksj);
        b /= ksj;
        const int j = (int)(b % N);
        const int nt = (int)(b / N);
        const int lane = dw >> 2, e4 = dw & 3;
        const int col = 32 * nt + (lane & 31), kh = lane >> 5;
        uint32_t word = 0;
        for (int e = 0; e < 4; ++e) {
            const int slot = 32 * sj + 16 * kh + 4 * e4 + e;
            const int p = slot >> gamma, h = slot & (base - 1);
            uint32_t v = 0;
            if (p < t && col <= n)
                v = ksk[(((size_t)j * t + p) * base + h) * (n + 1) + col];
            int8_t limb = 0;
            for (int k = 0; k <= q; ++k) {
                limb = (int8_t)(v & 0xFFu);
                v = (v - (uint32_t)(int32_t)limb) >> 8;
            }
            word |= (uint32_t)(uint8_t)limb << (8 * e);
        }
        out[idx] = word;
    }
}

// out rows = (0, .., 0, b'): the GEMM then subtracts into them.
template <bool LEVEL>
__global__ __launch_bounds__(256) void k_ks_init(const uint32_t *__restrict__ in,
                                                 uint32_t *__restrict__ out,
                                                 int B, KsLevel lv, int n, int N)
{
    const size_t total = (size_t)B * (n + 1);
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
         idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int it = (int)(idx / (n + 1)), col = (int)(idx % (n + 1));
        const uint32_t *src0, *src1;
        uint32_t *dst;
        if (!ks_item<LEVEL>(it, B, in, out, lv, n, N, src0, src1, dst))
            continue;
        uint32_t v = 0;
        if (col == n) {
            v = src0[N];
            if (src1)
                v += src1[N] + (1u << 29);
        }
        dst[col] = v;
    }
}

// One workgroup: KSM_ITEMS ciphertexts x (one 32-column tile per wave) x
// one range of j; each wave holds 2 row tiles x 4 limbs accumulators, reads
// its key blocks two K-steps ahead, builds the one-hot digits from a' in
// LDS, and subtracts its recombined partial sums from the output rows with
// device atomics (mod 2^32, so the order of the j ranges does not matter).
template <bool LEVEL>
__global__ __launch_bounds__(64 * KSM_WAVES) void k_ks_mfma(
    const int8_t *__restrict__ kski8, const uint32_t *__restrict__ in,
    uint32_t *__restrict__ out, int B, KsLevel lv, int n, int N, int gamma,
    int t, int ksj, int nt_tiles, int jchunk)
{
    __shared__ uint32_t a_l[KSM_ITEMS * KSM_JMAX];
    __shared__ uint32_t *dst_l[KSM_ITEMS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int it0 = blockIdx.x * KSM_ITEMS;
    const int nt = blockIdx.y * (blockDim.x >> 6) + wave;
    const int j0 = blockIdx.z * jchunk;
    const int JC = min(N, j0 + jchunk) - j0;
    const uint32_t round_off = (t * gamma < 32) ? 1u << (31 - t * gamma) : 0u;
    for (int m = threadIdx.x; m < KSM_ITEMS; m += blockDim.x) {
        const uint32_t *src0, *src1;
        uint32_t *dst;
        ks_item<LEVEL>(it0 + m, B, in, out, lv, n, N, src0, src1, dst);
        dst_l[m] = dst;
    }
    for (int idx = threadIdx.x; idx < KSM_ITEMS * JC; idx += blockDim.x) {
        const int m = idx / JC, jj = idx - m * JC;
        const uint32_t *src0, *src1;
        uint32_t *dst;
        uint32_t a = 0;
        if (ks_item<LEVEL>(it0 + m, B, in, out, lv, n, N, src0, src1, dst)) {
            a = src0[j0 + jj];
            if (src1)
                a += src1[j0 + jj];
        }
        a_l[m * KSM_JMAX + jj] = a + round_off;
    }
    __syncthreads();
    if (nt >= nt_tiles || JC <= 0)
        return;

    const int base = 1 << gamma, kh = lane >> 5, r = lane & 31;
    const int S = JC * ksj;              // K-steps of this workgroup
    const int8_t *bp = kski8 + ((size_t)nt * N + j0) * ksj * 4096 + lane * 16;
    auto loadb = [&](int s, ks_v4i (&dst)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            dst[q] = *reinterpret_cast<const ks_v4i *>(bp + (size_t)s * 4096 +
                                                       q * 1024);
    };
    // the lane's 16 one-hot bytes of K-step slot block sj for a' + offset u
    auto onehot = [&](uint32_t u, int sj) {
        ks_v4i a;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int slot0 = 32 * sj + 16 * kh + 4 * w;
            uint32_t word = 0;
            if (base >= 4) {
                const int p = slot0 >> gamma;
                if (p < t) {
                    const uint32_t d = (u >> (32 - (p + 1) * gamma)) &
                                       (uint32_t)(base - 1);
                    const uint32_t rel = d - (uint32_t)(slot0 & (base - 1));
                    word = rel < 4u ? 1u << (8 * rel) : 0u;
                }
            } else {                       // base 2: two levels per dword
#pragma unroll
                for (int hp = 0; hp < 2; ++hp) {
                    const int p = (slot0 >> 1) + hp;
                    if (p < t) {
                        const uint32_t d = (u >> (31 - p)) & 1u;
                        word |= 1u << (8 * (2 * hp + (int)d));
                    }
                }
            }
            a[w] = (int)word;
        }
        return a;
    };
    ks_v16i acc[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc[mt][q] = ks_v16i{};
    ks_v4i bq[3][4];
    auto step = [&](int s, int b) {
        if (s + 2 < S)
            loadb(s + 2, bq[(b + 2) % 3]);
        const int jj = s / ksj, sj = s - jj * ksj;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const ks_v4i A = onehot(a_l[(32 * mt + r) * KSM_JMAX + jj], sj);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[mt][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                    A, bq[b][q], acc[mt][q], 0, 0, 0);
        }
    };
    loadb(0, bq[0]);
    if (S > 1)
        loadb(1, bq[1]);
    int s = 0;
    for (; s + 3 <= S; s += 3) {
        step(s, 0);
        step(s + 1, 1);
        step(s + 2, 2);
    }
    if (s < S)
        step(s, 0);
    if (s + 1 < S)
        step(s + 1, 1);

    const int col = 32 * nt + r;
    if (col > n)
        return;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int m = 32 * mt + 8 * (v >> 2) + 4 * kh + (v & 3);
            uint32_t *dst = dst_l[m];
            if (!dst)
                continue;
            const uint32_t x = (uint32_t)acc[mt][0][v] +
                               ((uint32_t)acc[mt][1][v] << 8) +
                               ((uint32_t)acc[mt][2][v] << 16) +
                               ((uint32_t)acc[mt][3][v] << 24);
            atomicSub(dst + col, x);
        }
}

template <bool LEVEL>
int ks_mfma_dispatch(const Ctx *c, const uint32_t *in, uint32_t *out, int B,
                     KsLevel lv, hipStream_t s)
{
    const Shape &sh = c->sh;
    const int nt_tiles = (sh.n + 1 + 31) / 32;
    const int ng = (nt_tiles + KSM_WAVES - 1) / KSM_WAVES;
    const int waves = (nt_tiles + ng - 1) / ng;
    const int mg = (B + KSM_ITEMS - 1) / KSM_ITEMS;
    // Split j into kc ranges (at most KSM_JMAX j each, at least 16).  The
    // workgroups run in rounds of (CUs x resident workgroups per CU; one at
    // 212 VGPRs), and a workgroup costs about its j range plus 10 j (the
    // load of its a' and its atomic fold: fitted to launches of 4 to 64
    // ranges of 1024 default ciphertexts on the MI355X), so take the split
    // with the least rounds x (j range + 10), the fewest ranges among
    // equals.  Filling the GPU twice over instead (528 workgroups, three
    // rounds) was 25% slower at 1024 default ciphertexts.
    const long slots = (long)c->cus * c->ks_wg_per_cu;
    const int kc_lo = (sh.N + KSM_JMAX - 1) / KSM_JMAX;
    const int kc_hi = std::max(kc_lo, std::max(1, sh.N / 16));
    int jchunk = (sh.N + kc_lo - 1) / kc_lo;
    long best = -1;
    for (int k = kc_lo; k <= kc_hi; ++k) {
        const int jc = (sh.N + k - 1) / k;
        const int kk = (sh.N + jc - 1) / jc;
        const long rounds = ((long)mg * ng * kk + slots - 1) / slots;
        const long cost = rounds * (jc + 10);
        if (best < 0 || cost < best) {
            best = cost;
            jchunk = jc;
        }
    }
    const int kc = (sh.N + jchunk - 1) / jchunk;
    const size_t total = (size_t)B * (sh.n + 1);
    const int init_blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_ks_init<LEVEL>, dim3(init_blocks), dim3(256), 0, s,
                       in, out, B, lv, sh.n, sh.N);
    CGGI_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_ks_mfma<LEVEL>, dim3(mg, ng, kc), dim3(64 * waves), 0,
                       s, c->ksk_i8, in, out, B, lv, sh.n, sh.N, sh.gamma,
                       sh.t, c->ks_ksj, nt_tiles, jchunk);
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

template <bool LEVEL>
int ks_dispatch(const Ctx *c, const uint32_t *in, uint32_t *out, int B,
                KsLevel lv, hipStream_t s)
{
    if (c->ksk_i8)
        return ks_mfma_dispatch<LEVEL>(c, in, out, B, lv, s);
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

int keyswitch_make_key(Ctx *c, hipStream_t s)
{
    const Shape &sh = c->sh;
    if (sh.gamma > 4)
        return CGGI_OK;             // large bases keep the row gather
    const int nt_tiles = (sh.n + 1 + 31) / 32;
    const int ksj = (sh.t * (1 << sh.gamma) + 31) / 32;
    const size_t bytes = (size_t)nt_tiles * sh.N * ksj * 4 * 1024;
    if (hipMalloc(&c->ksk_i8, bytes) != hipSuccess) {
        c->ksk_i8 = nullptr;
        return set_error(CGGI_E_NOMEM, "hipMalloc of the int8 key-switching "
                                       "key failed");
    }
    c->ks_ksj = ksj;
    // resident workgroups per CU of the GEMM at its launch shape (the
    // split of j over workgroups is sized from it)
    {
        const int ng = (nt_tiles + KSM_WAVES - 1) / KSM_WAVES;
        const int waves = (nt_tiles + ng - 1) / ng;
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(&k_ks_mfma<true>),
                64 * waves, 0) == hipSuccess) {
            if (nb > 0)
                c->ks_wg_per_cu = nb;
        } else {
            (void)hipGetLastError();   // keep one per CU; clear the error
        }
    }
    hipLaunchKernelGGL(k_ksk_to_i8, dim3(4096), dim3(256), 0, s, c->ksk,
                       reinterpret_cast<uint32_t *>(c->ksk_i8), sh.n, sh.N,
                       sh.t, sh.gamma, ksj, nt_tiles);
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

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
