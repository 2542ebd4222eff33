// int8_kara.hip -- the int8-MFMA blind rotation with one Karatsuba level.
//
// A CMux step (ArctyrEX Fig. 1 loop body) adds sum_r D_r * a_{r,c'} to
// each accumulator component c' in Z_{2^32}[X]/(X^N+1).  Split every
// polynomial by coefficient parity, p(X) = p_e(X^2) + X p_o(X^2), and write
// Z = X^2 (so Z^(N/2) = X^N = -1).  Then
//   (a d)_even = a_e d_e + Z a_o d_o
//   (a d)_odd  = a_e d_o + a_o d_e
//              = a_e d_e + a_o d_o - (a_e - a_o)(d_e - d_o)
// with every product negacyclic of length H = N/2: three half-length
// products P1 = a_e d_e, P2 = a_o d_o, P3 = (a_e - a_o)(d_e - d_o) replace
// one full-length product, 3/4 of the multiply-adds.  The digit
// differences d_e - d_o of two sub-digits in [-64, 64) lie in [-127, 127],
// so they and their negations still fit int8; the key differences are
// formed mod 2^32 before the limb split.  Each half-length product is the
// block-Toeplitz GEMM of int8_form.hip at length H:
//   P[32J + rho] = sum_Delta sum_kappa A_Delta[rho][kappa] s(J,Delta)
//                  D_{(J - Delta) mod H/32}[kappa],
//   A_Delta[rho][kappa] = a_ext[32 Delta + rho - kappa],
// on v_mfma_i32_32x32x32_i8 with the key's four int8 limbs recombined mod
// 2^32.  Everything is exact mod 2^32, so the result is bit-identical to
// the other forms.
//
// Launch layout (N <= 1024): 768 threads = 12 waves (three per SIMD), one
// workgroup per CU (LDS-limited).  A column tile holds 32/(H/32)
// bootstraps side by side (two at N = 1024); a workgroup owns two tiles.
// Wave w computes product P = w >> 2 for output component c' = w & 1 and
// key limbs 2((w >> 1) & 1), 2((w >> 1) & 1) + 1, both tiles, over all
// block offsets (2 limbs x 2 tiles = 4 accumulators); the waves of one
// output component add their recombined sums into the LDS accumulator
// (mod 2^32, so the order does not matter):
//   P1 -> even[m] and odd[m];  P2 -> even[m+1] (-even[0] for the top m)
//   and odd[m];  P3 -> minus odd[m].
// The accumulator is stored de-interleaved (even and odd halves, each row
// padded by one dword per 32 so the fold's lanes fall in distinct banks).
// Digit operands live in LDS in both signs (for the wrapped blocks); the E
// and O operands are stored offset (delta + 64 and 63 - delta, both in
// [0, 127]: non-negative operands cost the matrix cores less energy) and
// the P1 and P2 accumulators of limb 0 start from minus the offsets'
// contribution, a function of the key only (k_kara_corr); E - O stays
// signed.  Key windows are wave-private: each wave reads the windows of its
// own (c', P, limb pair) from global memory a stage ahead and writes them to
// LDS as four byte-shifted copies, so a lane reads its 16-byte Toeplitz row
// as four aligned dwords.
#include "internal.hpp"

#include <type_traits>

namespace cggi {

namespace {

typedef int kv4i __attribute__((ext_vector_type(4)));
typedef int kv16i __attribute__((ext_vector_type(16)));

template <int N> struct KCfg {
    static constexpr int H = N / 2;          // half length
    static constexpr int NBH = H / 32;       // blocks per half polynomial
    static constexpr int BPT = 32 / NBH;     // bootstraps per column tile
    static constexpr int TILES = 2;          // column tiles per workgroup
    static constexpr int GPW = TILES * BPT;  // bootstraps per workgroup
    static constexpr int THREADS = 768;      // 3 products x 2 comps x 2 limb pairs
    static constexpr int ELEN = H + 64;      // bytes per key window
    static constexpr int EW = ELEN / 4;      // dwords per key window
    static constexpr int WIN_DW = 2 * 3 * 4 * EW;  // one stage: c', P, limb
    // one byte-shifted copy of a limb window in LDS: the A reads of a stage
    // touch dwords up to 8 NBH + 6.  Copies are laid out [sigma][limb]
    // [CLEN] with CLEN = 12 (mod 16): the two limbs of one copy are CLEN
    // dwords apart (one ds_read2 reaches both), and the copy stride 2 CLEN =
    // 24 (mod 32) puts the four copies one read touches in distinct banks
    static constexpr int CLEN = (8 * NBH + 7 - 12 + 15) / 16 * 16 + 12;
    static constexpr int AH = H + H / 32;    // padded accumulator half
    // dwords per bootstrap's accumulators (2 components x 2 halves), = NBH
    // mod 32 so that the bootstraps of a tile land on distinct banks
    static constexpr int GST = (4 * AH + 31) / 32 * 32 + NBH;
};

template <int N> struct KSmem {
    using C = KCfg<N>;
    // per wave: 2 limbs x 4 byte-shifted copies, single-buffered
    static constexpr size_t win = (size_t)12 * 2 * 4 * C::CLEN * 4;
    static constexpr size_t acc = (size_t)C::GPW * C::GST * 4;
    // digit operands
    __host__ __device__ static size_t dig(int R)
    {
        return (size_t)C::GPW * R * 3 * 2 * C::H;
    }
    static size_t total(int R, int n) { (void)n; return win + acc + dig(R); }
};

__device__ __forceinline__ void kara_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t kara_modswitch(uint32_t u, int log2_2n)
{
    return (u + (1u << (31 - log2_2n))) >> (32 - log2_2n);
}

// bsk [n][2l][2][N] -> half-length key windows [n][R][2][3][4][ELEN]:
// window y of (i, r*S+s, c', P) holds limb q of h_ext[y - 31] * 2^(7s),
// where h = a_e (P = 0), a_o (P = 1) or a_e - a_o (P = 2) of a = bsk[i][r]
// [c'], h_ext[x] = h[x] (0 <= x < H), -h[x+H] (x < 0), 0 beyond H.
template <int N>
__global__ void k_kara_key(const uint32_t *__restrict__ bsk,
                           int8_t *__restrict__ out, int n, int l, int S)
{
    using C = KCfg<N>;
    constexpr int H = C::H;
    const int R = 2 * l * S;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)n * R * 2 * 3 * C::ELEN;
    if (idx >= total)
        return;
    int y = (int)(idx % C::ELEN);
    size_t t = idx / C::ELEN;
    int P = (int)(t % 3);
    t /= 3;
    int cp = (int)(t % 2);
    t /= 2;
    int kb = (int)(t % R);
    int i = (int)(t / R);
    int r = kb / S, s = kb % S;
    const uint32_t *a = bsk + (((size_t)i * 2 * l + r) * 2 + cp) * N;
    auto half = [&](int x) -> uint32_t {
        uint32_t e = a[2 * x], o = a[2 * x + 1];
        return P == 0 ? e : (P == 1 ? o : e - o);
    };
    int x = y - 31;
    uint32_t v = 0;
    if (x >= 0 && x < H)
        v = half(x);
    else if (x < 0)
        v = 0u - half(x + H);
    v <<= 7 * s;
    int8_t *o = out + ((((size_t)i * R + kb) * 2 + cp) * 3 + P) * 4 * C::ELEN + y;
    for (int q = 0; q < 4; ++q) {
        int8_t limb = (int8_t)(v & 0xFFu);
        o[(size_t)q * C::ELEN] = limb;
        v = (v - (uint32_t)(int32_t)limb) >> 8;
    }
}

// Offset correction of the E and O operands.  With the positive copy
// holding delta + 64 and the negated copy 63 - delta, the half-length GEMM
// of product P (0: a_e with E, 1: a_o with O) exceeds the product at
// coefficient m = 32J + rho by
//   sum over digit rows of (63 * total[rho] + head_J[rho]),
// W_Delta[rho] = sum_kappa h_ext[32 Delta + rho - kappa] * 2^(7s) the row
// sum of Toeplitz block Delta of that row's half key h, total = the sum over
// every Delta, head_J = the sum over Delta <= J (blocks read from the
// positive copy).  corr [n][2][2][H] (step, c', P, m) holds minus that
// excess mod 2^32, the start value of the limb-0 accumulators as is (so the
// bootstrap kernel uses the loaded words only at its first MFMA and the read
// latency hides behind the decomposition).  One workgroup per (i, c', P).
template <int N>
__global__ __launch_bounds__(256) void k_kara_corr(
    const uint32_t *__restrict__ bsk, uint32_t *__restrict__ corr, int n,
    int l, int S)
{
    constexpr int H = N / 2, NBH = H / 32, PT = (H + 255) / 256;
    __shared__ uint32_t ext[H + 32];   // ext[x + 31] = h_ext[x], -31 <= x < H
    __shared__ uint32_t W[H];          // W_Delta[rho] at 32 Delta + rho
    const int i = blockIdx.x >> 2, cp = (blockIdx.x >> 1) & 1;
    const int P = blockIdx.x & 1;
    if (i >= n)
        return;
    const int tid = threadIdx.x;
    const int R = 2 * l * S;
    uint32_t accv[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k)
        accv[k] = 0u;
    for (int kb = 0; kb < R; ++kb) {
        const int r = kb / S, s = kb - r * S;
        const uint32_t *a = bsk + (((size_t)i * 2 * l + r) * 2 + cp) * N;
        for (int x = tid - 31; x < H; x += 256)
            ext[x + 31] = x >= 0 ? a[2 * x + P] : 0u - a[2 * (x + H) + P];
        __syncthreads();
        for (int t = tid; t < H; t += 256) {
            uint32_t w = 0;
            for (int kap = 0; kap < 32; ++kap)
                w += ext[t - kap + 31];
            W[t] = w;
        }
        __syncthreads();
        if (tid < 32) {                // prefix over Delta, per rho
            uint32_t run = 0;
            for (int D = 0; D < NBH; ++D) {
                run += W[32 * D + tid];
                W[32 * D + tid] = run;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const int j = tid + 256 * k;
            if (j < H) {
                const int J = j >> 5, rho = j & 31;
                const uint32_t total = W[32 * (NBH - 1) + rho];
                accv[k] += (63u * total + W[32 * J + rho]) << (7 * s);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PT; ++k) {
        const int j = tid + 256 * k;
        if (j < H)
            corr[(((size_t)i * 2 + cp) * 2 + P) * H + j] = 0u - accv[k];
    }
}

// L (gadget levels) and S (sub-digits per digit) are compile-time so the
// digit loops unroll; L = 0 selects a generic build reading l and S at run
// time (at most 8 levels, 2 sub-digits).
template <int N, int L, int S, int BB>
__global__ __launch_bounds__(KCfg<N>::THREADS, 1) void k_bootstrap_int8_kara(
    const int8_t *__restrict__ key, const uint32_t *__restrict__ corr,
    const uint32_t *__restrict__ in, const uint32_t *__restrict__ testv,
    uint32_t *__restrict__ out, int B, const int32_t *__restrict__ d_count,
    int lo, int hi, int n, int beta, int l_rt, int S_rt)
{
    using C = KCfg<N>;
    constexpr int H = C::H, NBH = C::NBH, BPT = C::BPT, GPW = C::GPW;
    constexpr int THREADS = C::THREADS, EW = C::EW, WIN_DW = C::WIN_DW;
    constexpr int AH = C::AH, GST = C::GST;
    constexpr int LOG2_2N = __builtin_ctz(2 * N);
    const int l = L ? L : l_rt;
    const int SS = L ? S : S_rt;
    const int R = 2 * l * SS;

    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int CLEN = C::CLEN;
    uint32_t *win = reinterpret_cast<uint32_t *>(smem);  // [12][2][4][CLEN]
    uint32_t *acc = win + 12 * 2 * 4 * CLEN;              // [GPW][GST]
    // digit operands [GPW][R][3][kappa half][sign: -, +][NBH][16]
    int8_t *dig = reinterpret_cast<int8_t *>(acc + GPW * GST);

    // a launch issued next to others for a count read on the device runs
    // only when lo < count <= hi
    const int dc = d_count ? *d_count : B;
    if (dc <= lo || dc > hi)
        return;
    const int count = min(B, dc);
    const int g0 = blockIdx.x * GPW;
    if (g0 >= count)
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wave index as a scalar: everything derived from it is wave-uniform
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // accumulator word of coefficient j (0 <= j < N) of component c
    auto aidx = [](int gl, int c, int j) {
        const int h = j >> 1;
        return gl * GST + c * 2 * AH + (j & 1) * AH + h + (h >> 5);
    };

    // modulus-switched input coefficient i of bootstrap gl (read from
    // global memory where needed; 0 past the batch)
    auto msw = [&](int gl, int i) -> int {
        const int g = g0 + gl;
        const uint32_t u = g < count ? in[(size_t)g * (n + 1) + i] : 0u;
        return (int)kara_modswitch(u, LOG2_2N);
    };
    // ---- ACC = (0, X^(2N - b~) v) ---------------------------------------
    for (int idx = tid; idx < GPW * N; idx += THREADS) {
        int gl = idx / N, m = idx - gl * N;
        int e = (2 * N - msw(gl, n)) & (2 * N - 1);
        uint32_t v = testv ? testv[m] : (1u << 29);
        int t = m + e;
        if (t >= 2 * N) {
            t -= 2 * N;
        } else if (t >= N) {
            t -= N;
            v = 0u - v;
        }
        acc[aidx(gl, 0, t)] = 0u;
        acc[aidx(gl, 1, t)] = v;
    }

    // ---- per-lane constants ----------------------------------------------
    const int P = wave >> 2;                  // product: 0 e*e, 1 o*o, 2 diff
    const int cp = wave & 1;                  // output component
    const int q0 = 2 * ((wave >> 1) & 1);     // first key limb
    const int rho = lane & 31, hh = lane >> 5;
    const int colJ = rho % NBH, colb = rho / NBH;   // column -> block, bootstrap
    // A operand: first dword and byte shift of this lane's Toeplitz row
    const int a_w0 = (rho & 3) * 2 * CLEN + 4 * hh + (rho >> 2);
    // the wave that starts the offset correction of its product (P1, P2)
    const bool corr_wave = P < 2 && q0 == 0;

    // ---- key-window staging ------------------------------------------------
    // Each wave reads only the windows of its own (c', P, limb pair) and
    // stages them itself: the two limb windows of the next stage are read
    // from global memory a stage ahead, and between two stages the wave
    // writes them to its own LDS buffer as four byte-shifted copies (copy
    // sigma, dword w = window bytes 4w + sigma .. 4w + sigma + 3), so each
    // lane reads its 16-byte Toeplitz row as four aligned dwords.  LDS
    // operations of one wave complete in order, so no barrier is needed.
    constexpr int CI = 2 * CLEN;                      // copy dwords per slice
    constexpr int PER_W = (CI + 63) / 64;
    uint32_t pre_lo[PER_W], pre_hi[PER_W];
    uint32_t *winw = win + wave * (2 * 4 * CLEN);     // [sigma][limb][CLEN]
    const uint32_t *key32 = reinterpret_cast<const uint32_t *>(key) +
                            ((cp * 3 + P) * 4 + q0) * EW;
    auto fetch = [&](int st) {
        const uint32_t *src = key32 + (size_t)st * WIN_DW;
#pragma unroll
        for (int k = 0; k < PER_W; ++k) {
            // every lane loads (a clamped item re-reads a valid word it
            // does not store)
            const int item = min(lane + 64 * k, CI - 1);
            const int q = item / CLEN, w = item - q * CLEN;
            pre_lo[k] = src[q * EW + w];
            pre_hi[k] = src[q * EW + w + 1];
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < PER_W; ++k) {
            const int item = lane + 64 * k;
            if (item < CI) {
                const int q = item / CLEN, w = item - q * CLEN;
                uint32_t *d = winw + q * CLEN + w;
                d[0] = pre_lo[k];
                d[2 * CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 1);
                d[4 * CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 2);
                d[6 * CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 3);
            }
        }
    };
    fetch(0);
    stash();
    if (n * R > 1)
        fetch(1);
    __syncthreads();

    // digit width log2(Bg): a constant where the launch fixes it
    const int bt = BB ? BB : beta;
    const uint32_t round_off = (bt * l < 32) ? (1u << (31 - bt * l)) : 0u;
    uint32_t dig_off = round_off;
    for (int p = 1; p <= l; ++p)
        dig_off += (1u << (bt - 1)) << (32 - p * bt);
    const uint32_t bmask = (1u << bt) - 1u;
    const int32_t bhalf = 1 << (bt - 1);

    // The decomposition works in 64-item chunks (item: 8 consecutive
    // coefficients of one component of one bootstrap); a chunk lies in one
    // bootstrap, so the step's rotation is wave-uniform.  Each wave reads
    // the rotations of the next step during the current one.
    constexpr int ROWI = N / 8, GLI = 2 * ROWI, NCH = GPW * GLI / 64;
    constexpr int CPW = (NCH + THREADS / 64 - 1) / (THREADS / 64);
    // chunk it of this wave, or -1
    auto chunk_of = [&](int it) -> int {
        const int ch = wave + (THREADS / 64) * it;
        return ch < NCH ? ch : -1;
    };
    // The raw input words, modulus-switched where used.  They are read with
    // vector loads (an opaque zero lane offset keeps the compiler from a
    // scalar load, whose counter LDS waits share: an outstanding one turns
    // every LDS wait into a full one) and moved to scalar registers at use.
    uint32_t e_cur[CPW], e_nxt[CPW];
    auto load_e = [&](int ii, uint32_t (&dst)[CPW]) {
        int z = 0;
        asm volatile("" : "+v"(z));
#pragma unroll
        for (int it = 0; it < CPW; ++it) {
            const int ch = chunk_of(it);
            const int g = g0 + ch * 64 / GLI;
            dst[it] = ch >= 0 && g < count
                          ? in[(size_t)g * (n + 1) + ii + z] : 0u;
        }
    };
    load_e(0, e_cur);

    kv16i Cacc[2][2];   // [tile][limb]

    for (int i = 0; i < n; ++i) {
        kara_barrier();   // ACC of the previous step complete
        // limb-0 accumulators of P1 / P2 start from minus the step's offset
        // correction (the same for both tiles: it depends on the key only;
        // the table holds it negated)
        kv16i cinit = {};
        if (corr_wave) {
            const uint32_t *cr = corr + (((size_t)i * 2 + cp) * 2 + P) * H +
                                 32 * colJ + 4 * hh;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const kv4i c4 = *reinterpret_cast<const kv4i *>(cr + 8 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    cinit[4 * g + e] = c4[e];
            }
        }
        // ---- rotate, subtract, decompose into E, O and E - O operands -----
#pragma unroll
        for (int it = 0; it < CPW; ++it) {
            const int ch = chunk_of(it);
            if (ch < 0)
                break;
            const int gl = ch * 64 / GLI;
            const int rem = ch * 64 - gl * GLI + lane;
            const int c = rem / ROWI;
            const int m0 = 8 * (rem - c * ROWI);
            // (X^e ACC)[m] = ACC[m - e].  In halves (even E, odd O; h = m >> 1)
            // with e = 2 f + pe, that reads E[h - f] and O[h - f] (pe = 0) or
            // O[h - f - 1] and E[h - f] (pe = 1) for the even and odd
            // coefficients; a half index u < 0 wraps to u + H with the sign
            // flipped per wrap (Z^H = -1): bit log2(H) of u.
            const int e = (int)kara_modswitch(
                __builtin_amdgcn_readfirstlane(e_cur[it]), LOG2_2N);
            const int f = e >> 1, pe = e & 1;
            const int h0 = m0 >> 1;
            const uint32_t *Ec = acc + gl * GST + c * 2 * AH;
            const uint32_t *Oc = Ec + AH;
            const uint32_t *srcE = pe ? Oc : Ec;
            const uint32_t *srcO = pe ? Ec : Oc;
            const int uE = h0 - f - pe, uO = h0 - f;
            const uint32_t *sE = Ec + h0 + (h0 >> 5);   // 4 unrotated entries
            // all sixteen reads first (the LDS latency is paid once per
            // chunk, not once per coefficient), then the arithmetic
            uint32_t rv[8], sv[8];
            int uu[8];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                uu[2 * kk] = uE + kk;
                uu[2 * kk + 1] = uO + kk;
                const int xe = uu[2 * kk] & (H - 1);
                const int xo = uu[2 * kk + 1] & (H - 1);
                rv[2 * kk] = srcE[xe + (xe >> 5)];
                rv[2 * kk + 1] = srcO[xo + (xo >> 5)];
                sv[2 * kk] = sE[kk];
                sv[2 * kk + 1] = sE[AH + kk];
            }
            __builtin_amdgcn_sched_barrier(0);
            uint32_t w8[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // all ones when bit log2(H) of u is set: the wrapped sign
                const uint32_t mk = (uint32_t)__builtin_amdgcn_sbfe(
                    uu[k], __builtin_ctz(H), 1);
                w8[k] = ((rv[k] ^ mk) - mk) - sv[k] + dig_off;
            }
            // half-length coefficients mh0 .. mh0+3; byte b of a dword holds
            // coefficient mh0 + 3 - b (reversed kappa)
            const int mh0 = m0 >> 1;
            const int kp = 28 - (mh0 & 31), M = mh0 >> 5;
            const int off = (kp >> 4) * (2 * NBH * 16) + M * 16 + (kp & 15);
            int8_t *gbase = dig + (size_t)gl * R * 6 * H + off;
            // four offset sub-digits v = delta + 64 in [0, 128) -> one dword
            auto pack4 = [](uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
                return (a << 24) | (b << 16) | (c << 8) | d;
            };
            // one digit row: E and O offset (delta + 64 and, negated,
            // 63 - delta = 127 - (delta + 64)); E - O signed, formed per
            // byte without borrows: (E' | 0x80) - O' = E - O + 128 in
            // [1, 255], then the top bit flipped
            auto emit = [&](int kb, const uint32_t (&v)[8]) {
                const uint32_t pe = pack4(v[0], v[2], v[4], v[6]);
                const uint32_t po = pack4(v[1], v[3], v[5], v[7]);
                const uint32_t pw[3] = {
                    pe, po, ((pe | 0x80808080u) - po) ^ 0x80808080u};
                const uint32_t nw[3] = {
                    pe ^ 0x7F7F7F7Fu, po ^ 0x7F7F7F7Fu,
                    ((po | 0x80808080u) - pe) ^ 0x80808080u};
#pragma unroll
                for (int pp = 0; pp < 3; ++pp) {
                    int8_t *base = gbase + ((size_t)kb * 3 + pp) * 2 * H;
                    *reinterpret_cast<uint32_t *>(base + NBH * 16) = pw[pp];
                    *reinterpret_cast<uint32_t *>(base) = nw[pp];
                }
            };
#pragma unroll
            for (int p = 1; p <= (L ? L : 8); ++p) {
                if (!L && p > l)
                    break;
                const int sh = 32 - p * bt;
                if (SS == 1) {
                    // one sub-digit: delta + 64 = ((w >> sh) & (Bg-1)) - Bg/2 + 64
                    uint32_t v[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        v[k] = ((w8[k] >> sh) & bmask) + (uint32_t)(64 - bhalf);
                    emit(c * l + (p - 1), v);
                    continue;
                }
                int32_t d[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    d[k] = (int32_t)((w8[k] >> sh) & bmask) - bhalf;
#pragma unroll
                for (int s = 0; s < (L ? S : 2); ++s) {
                    if (!L && s >= SS)
                        break;
                    uint32_t v[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        if (s == SS - 1) {
                            v[k] = (uint32_t)(d[k] + 64);
                        } else {
                            // low 7-bit sub-digit delta = v - 64 in [-64, 64)
                            v[k] = (uint32_t)(d[k] + 64) & 127u;
                            d[k] = (d[k] + 64 - (int32_t)v[k]) >> 7;
                        }
                    }
                    emit((c * l + (p - 1)) * SS + s, v);
                }
            }
        }
        kara_barrier();

        // ---- K loop: digit polynomials x block offsets ----------------------
        auto stage = [&](const int kb, auto first_c) {
            constexpr bool FIRST = decltype(first_c)::value;
            const int st = i * R + kb;
            const bool more = st + 1 < n * R;
            const uint32_t *wb = winw + a_w0;
            // B: this lane's 16 bytes of digit block (J - Delta) mod NBH of
            // tile 0 (tile 1 lies TS bytes further), from the negated copy
            // when the block index wrapped (J < Delta).  Each kappa half of a
            // digit row holds the negated blocks followed by the blocks, so
            // both cases are block NBH + J - Delta of that row: one base per
            // lane and an immediate offset per block offset and tile.
            const int TS = BPT * R * 6 * H;
            // (an opaque lane offset, so that the digit area's own offset is
            // folded into the base rather than into every read's immediate)
            int boff = ((colb * R + kb) * 3 + P) * 2 * H +
                       hh * (2 * NBH * 16) + 16 * colJ + 16;
            asm volatile("" : "+v"(boff));
            const int8_t *bb = dig + boff;
            auto load_a = [&](int dl, kv4i (&af)[2]) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint32_t *ap = wb + q * CLEN + 8 * dl;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        af[q][k] = (int)ap[k];
                }
            };
            auto load_b = [&](int dl, kv4i (&bf)[2]) {
                const int8_t *pb = bb + 16 * (NBH - 1 - dl);
                bf[0] = *reinterpret_cast<const kv4i *>(pb);
                bf[1] = *reinterpret_cast<const kv4i *>(pb + TS);
            };
            kv4i af[2][2], bf[2][2];
            // block offset dl: its four MFMAs on register buffer b, with the
            // operands of dl + 1 read into the other buffer in their issue
            // shadows
            auto group = [&](int dl, int b, bool zero_start) {
                if (dl + 1 < NBH) {
                    load_a(dl + 1, af[b ^ 1]);
                    load_b(dl + 1, bf[b ^ 1]);
                }
                const kv16i zero = {};
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        Cacc[t][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                            af[b][q], bf[b][t],
                            zero_start ? (q == 0 ? cinit : zero) : Cacc[t][q],
                            0, 0, 0);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0); // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0); // DS read
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_barrier(0);
            };
            load_a(0, af[0]);
            load_b(0, bf[0]);
            group(0, 0, FIRST);   // the first stage starts the accumulators
            // the next stage's windows, read once this stage's first MFMAs
            // are issued (before them, the wait of the step's first MFMA
            // for the correction start values would cover these reads too)
            if (more && st >= 1)
                fetch(st + 1);
            if (FIRST && i + 1 < n)
                load_e(i + 1, e_nxt);   // next step's rotations
#pragma unroll 1
            for (int dl = 1; dl + 1 < NBH; dl += 2) {
                group(dl, 1, false);
                group(dl + 1, 0, false);
            }
            group(NBH - 1, 1, false);
            // the next stage's windows replace this one's (every read of
            // this stage was issued before these writes)
            if (more)
                stash();
        };
        stage(0, std::true_type{});
        for (int kb = 1; kb < R; ++kb)
            stage(kb, std::false_type{});

        // ---- fold: each wave adds its sums straight into the accumulator ----
        // The wave's two limbs recombined, C_q0 + C_q0+1 * 2^8, times 2^(8 q0)
        // (limbs 2, 3 only matter mod 2^16), go into the accumulator with
        // LDS atomic adds as soon as the wave's K loop ends:
        //   P1[m] -> even[m] and odd[m]
        //   P2[m] -> even[m+1] (minus even[0] for m = H-1, Z^(N/2) = -1) and
        //            odd[m]
        //   P3[m] -> minus odd[m]
        // Nothing reads the accumulator until the next step's decomposition,
        // after its barrier, and the adds commute mod 2^32, so the waves of
        // the products that finish first fold while the others still run.
        // Lane (colJ, colb, hh) holds m = 32 colJ + 8 g + 4 hh + k of
        // bootstrap t BPT + colb (value v = 4 g + k of tile t), at padded
        // index 33 colJ + 8 g + 4 hh + k: a lane base plus an immediate.
        {
            uint32_t *ab = acc + colb * GST + cp * 2 * AH + 33 * colJ + 4 * hh;
            auto add = [](uint32_t *x, uint32_t v) {
                __hip_atomic_fetch_add(x, v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            // P2's even[m + 1] for the lane's last row (m = 32 colJ + 31 on
            // hh = 1): the next block's first entry, or minus even[0] of
            // the same bootstrap after the last block
            const bool top = hh == 1 && colJ == NBH - 1;
            const int last_off = hh == 0 ? 1 : (top ? -(33 * colJ + 31) : 2);
            const int sh = 8 * q0;
            // one straight-line body per product (the product is
            // wave-uniform; a test per value would cost scalar branches)
            auto fold = [&](auto prod) {
                constexpr int PR = decltype(prod)::value;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    uint32_t *at = ab + t * BPT * GST;
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const uint32_t x =
                            ((uint32_t)Cacc[t][0][v] +
                             ((uint32_t)Cacc[t][1][v] << 8)) << sh;
                        uint32_t *e = at + 8 * (v >> 2) + (v & 3);
                        if (PR == 0) {
                            add(e, x);
                            add(e + AH, x);
                        } else if (PR == 1) {
                            add(e + AH, x);
                            if (v == 15)
                                add(e + last_off, top ? 0u - x : x);
                            else
                                add(e + 1, x);
                        } else {
                            add(e + AH, 0u - x);
                        }
                    }
                }
            };
            if (P == 0)
                fold(std::integral_constant<int, 0>{});
            else if (P == 1)
                fold(std::integral_constant<int, 1>{});
            else
                fold(std::integral_constant<int, 2>{});
        }
#pragma unroll
        for (int it = 0; it < CPW; ++it)
            e_cur[it] = e_nxt[it];
    }
    __syncthreads();

    // ---- sample extraction ---------------------------------------------------
    for (int idx = tid; idx < GPW * (N + 1); idx += THREADS) {
        int gl = idx / (N + 1), j = idx - gl * (N + 1);
        int g = g0 + gl;
        if (g >= count)
            continue;
        uint32_t v;
        if (j == 0)
            v = acc[aidx(gl, 0, 0)];
        else if (j < N)
            v = 0u - acc[aidx(gl, 0, N - j)];
        else
            v = acc[aidx(gl, 1, 0)];
        out[(size_t)g * (N + 1) + j] = v;
    }
}

template <int N, int L, int S, int BB>
int kara_launch_t(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                  uint32_t *out, int B, const int32_t *d_count, int lo, int hi,
                  hipStream_t s)
{
    using C = KCfg<N>;
    const Shape &sh = c->sh;
    const size_t smem = KSmem<N>::total(sh.R, sh.n);
    const int grid = (B + C::GPW - 1) / C::GPW;
    hipLaunchKernelGGL((k_bootstrap_int8_kara<N, L, S, BB>), dim3(grid),
                       dim3(C::THREADS), smem, s, c->bsk_k8, c->corr_k8, in,
                       testv, out, B, d_count, lo, hi, sh.n, sh.beta, sh.l,
                       sh.S);
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

template <int N>
int kara_launch_n(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                  uint32_t *out, int B, const int32_t *d_count, int lo, int hi,
                  hipStream_t s)
{
    const Shape &sh = c->sh;
    if (sh.l == 3 && sh.S == 1 && sh.beta == 7)
        return kara_launch_t<N, 3, 1, 7>(c, in, testv, out, B, d_count, lo, hi,
                                         s);
    if (sh.l == 2 && sh.S == 2)
        return kara_launch_t<N, 2, 2, 0>(c, in, testv, out, B, d_count, lo, hi,
                                         s);
    return kara_launch_t<N, 0, 0, 0>(c, in, testv, out, B, d_count, lo, hi, s);
}

template <int N, int L, int S, int BB>
int kara_attr_t()
{
    CGGI_HIP_TRY(hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_bootstrap_int8_kara<N, L, S, BB>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    return CGGI_OK;
}

template <int N>
int kara_make_key_n(Ctx *c, const uint32_t *bsk, hipStream_t s)
{
    using C = KCfg<N>;
    const Shape &sh = c->sh;
    if (KSmem<N>::total(sh.R, sh.n) > 160 * 1024)
        return CGGI_OK;                  // this kernel kind is unavailable
    const size_t total = (size_t)sh.n * sh.R * 2 * 3 * C::ELEN;
    if (hipMalloc(&c->bsk_k8, total * 4) != hipSuccess) {
        c->bsk_k8 = nullptr;
        return set_error(CGGI_E_NOMEM, "hipMalloc of the Karatsuba int8 key "
                                       "failed");
    }
    hipLaunchKernelGGL(k_kara_key<N>, dim3((unsigned)((total + 255) / 256)),
                       dim3(256), 0, s, bsk, c->bsk_k8, sh.n, sh.l, sh.S);
    CGGI_HIP_TRY(hipGetLastError());
    const size_t cbytes = (size_t)sh.n * 2 * 2 * C::H * sizeof(uint32_t);
    if (hipMalloc(&c->corr_k8, cbytes) != hipSuccess) {
        c->corr_k8 = nullptr;
        return set_error(CGGI_E_NOMEM, "hipMalloc of the Karatsuba offset "
                                       "correction failed");
    }
    hipLaunchKernelGGL(k_kara_corr<N>, dim3(4 * sh.n), dim3(256), 0, s, bsk,
                       c->corr_k8, sh.n, sh.l, sh.S);
    CGGI_HIP_TRY(hipGetLastError());
    int rc;
    if (sh.l == 3 && sh.S == 1 && sh.beta == 7)
        rc = kara_attr_t<N, 3, 1, 7>();
    else if (sh.l == 2 && sh.S == 2)
        rc = kara_attr_t<N, 2, 2, 0>();
    else
        rc = kara_attr_t<N, 0, 0, 0>();
    return rc;
}

} // namespace

size_t kara_smem_bytes(int N, int R, int n)
{
    switch (N) {
    case 256: return KSmem<256>::total(R, n);
    case 512: return KSmem<512>::total(R, n);
    case 1024: return KSmem<1024>::total(R, n);
    default: return (size_t)-1;
    }
}

int kara_bootstraps_per_workgroup(int N)
{
    switch (N) {
    case 256: return KCfg<256>::GPW;
    case 512: return KCfg<512>::GPW;
    case 1024: return KCfg<1024>::GPW;
    default: return 0;
    }
}

int kara_make_key(Ctx *c, const uint32_t *bsk, hipStream_t s)
{
    switch (c->sh.N) {
    case 256: return kara_make_key_n<256>(c, bsk, s);
    case 512: return kara_make_key_n<512>(c, bsk, s);
    case 1024: return kara_make_key_n<1024>(c, bsk, s);
    default: return CGGI_OK;             // N = 2048: not available
    }
}

int kara_launch(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                uint32_t *out, int B, const int32_t *d_count, int lo, int hi,
                hipStream_t s)
{
    switch (c->sh.N) {
    case 256: return kara_launch_n<256>(c, in, testv, out, B, d_count, lo, hi, s);
    case 512: return kara_launch_n<512>(c, in, testv, out, B, d_count, lo, hi, s);
    case 1024: return kara_launch_n<1024>(c, in, testv, out, B, d_count, lo, hi, s);
    default: return set_error(CGGI_E_PARAM, "Karatsuba kernel: N > 1024");
    }
}

} // namespace cggi
