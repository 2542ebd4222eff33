// int8_form.hip -- the int8-MFMA form of the blind rotation on gfx950.
//
// A CMux step (ArctyrEX Fig. 1 loop body) adds to each accumulator
// component c' the sum over digit polynomials r of D_r * a_{r,c'} in
// Z_{2^32}[X]/(X^N+1).  This file computes those products exactly as an
// integer GEMM on v_mfma_i32_32x32x32_i8:
//
//  * Block-Toeplitz form.  With coefficients cut into blocks of 32
//    (j = 32J + rho, m = 32M + kappa), (a * D)[j] =
//    sum_Delta sum_kappa A_Delta[rho][kappa] * s(J,Delta) * D_{(J-Delta)
//    mod N/32}[kappa], where A_Delta[rho][kappa] = a_ext[32 Delta + rho -
//    kappa], a_ext[x] = a[x] for x >= 0 and -a[x+N] for x < 0, and
//    s = -1 exactly when the block index wrapped (J < Delta).  For one
//    Delta, A_Delta is a 32x32 matrix shared by every bootstrap, and the
//    sign-rotated digit blocks of one bootstrap form a 32x32 (N = 1024)
//    operand whose columns are the output blocks J.  So one bootstrap fills
//    the MFMA column dimension by itself and the K loop runs over
//    (r, Delta).
//  * Limbs.  Each key value (negated in uint32 first where a_ext needs it,
//    scaled by 2^(7s) for sub-digit s) is split into four signed int8
//    limbs v = sum_q 2^(8q) v_q; the four limb GEMMs accumulate in int32
//    and are recombined mod 2^32.
//  * Digits.  Gadget digits in [-Bg/2, Bg/2) are split into 7-bit
//    sub-digits delta in [-64, 64) (one for Bg <= 2^7); delta and its
//    negation (for wrapped blocks) both fit int8.  The two- and four-tile
//    kernels store delta + 64 and 63 - delta instead (both in [0, 127]:
//    non-negative operands take the matrix cores less energy) and start one
//    accumulator per output coefficient from minus the offsets'
//    contribution, which depends on the key only and is tabulated once per
//    context.
//  * Exactness: |sum| <= R*N*128*128 < 2^31 for every parameter set the
//    context accepts, and int32 MFMA accumulation wraps mod 2^32 in any
//    case, so the recombination mod 2^32 is exact.
//
// Launch layout (N <= 1024): 512 threads (8 waves, two per SIMD) per
// workgroup, one workgroup per CU (LDS-limited); a workgroup owns 4 column
// tiles = 4*1024/N bootstraps.  Wave w computes output component c' = w & 1
// and key limbs 2((w>>1) & 1), 2((w>>1) & 1) + 1 for all four tiles (8 x 16
// int32 accumulators), over half w >> 2 of the block offsets Delta; the
// four waves of one component add their partial sums into the LDS
// accumulator (mod 2^32, so the order does not matter).  The A operand (key
// window rows) is read from LDS once per Delta and reused by four MFMAs, the
// B operand (digit blocks of a tile) by two; the operands of Delta + 1 are
// read in the issue shadows of Delta's MFMAs.
// LDS holds the accumulators, the digit operands (both signs), the step's
// key windows in four byte-shifted copies (so every lane reads its 16-byte
// Toeplitz row as four aligned dwords), double-buffered per digit
// polynomial, and the modulus-switched inputs.  N = 2048 runs 8 waves per
// bootstrap (all four limbs per wave, a quarter of the block offsets each)
// with single-buffered windows.
#include "internal.hpp"

#include <type_traits>

namespace cggi {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// N <= 1024: a workgroup owns 4 column tiles (4 * 1024 / N bootstraps) and
// runs 8 waves (two per SIMD) with double-buffered key windows; a wave
// computes one output component and two of the four key limbs for all four
// tiles over half of the block offsets (4 x 2 accumulators).
// N = 2048: a bootstrap spans 2 column tiles; a workgroup owns one
// bootstrap, runs 8 waves (two per SIMD; 4% faster than one per SIMD with
// twice the block offsets each) and single-buffers the (twice as long)
// windows; a wave computes one output component and all four limbs for both
// tiles over a quarter of the block offsets (2 x 4 accumulators).
// T (N <= 1024) is the number of column tiles per workgroup: 4 for wide
// batches; 2 or 1 for narrow ones, so that a batch of few bootstraps spreads
// over more CUs and each workgroup's step does less work.  With one tile a
// workgroup runs 16 waves (four per SIMD), each over a quarter of the block
// offsets, to cover the latency of its short MFMA groups.
template <int N, int T = 4> struct I8Cfg {
    static constexpr bool BIG = N > 1024;
    static constexpr int NB = N / 32;          // blocks per polynomial
    static constexpr int TPG = BIG ? N / 1024 : 1;  // column tiles per bootstrap
    static constexpr int GPT = BIG ? 1 : 1024 / N;  // bootstraps per column tile
    static constexpr int TILES = BIG ? 2 : T;       // column tiles per workgroup
    static constexpr int GPW = BIG ? TILES / TPG : TILES * GPT; // bootstraps
    // one tile per workgroup: 16 waves, each over a quarter of the block
    // offsets (17% faster per level than 8 waves; two tiles would spill)
    static constexpr int THREADS = (!BIG && T == 1) ? 1024 : 512;
    static constexpr int LPW = BIG ? 4 : 2;    // key limbs per wave
    static constexpr int WT = TILES;           // column tiles per wave
    static constexpr int EBUF = BIG ? 1 : 2;   // key-window buffers
    // stages between a key window's global read and its use: with one or
    // two tiles a stage's MFMA work is too short to cover the read latency
    // of the next window, so the read is issued two stages ahead
    static constexpr int PD = (!BIG && T <= 2) ? 2 : 1;
    static constexpr int ELEN = N + 64;        // bytes per limb window
    static constexpr int EW = ELEN / 4;        // dwords per limb window
    static constexpr int CW = N / 4 + 8;       // dwords of a shifted copy used
    // stride of a shifted copy: = 8 (mod 32) dwords, so the 48 distinct
    // dwords one Toeplitz-row read touches fall in distinct LDS banks
    static constexpr int CLEN = N / 4 + 8;
    // accumulator rows are padded by one dword per 32 coefficients (stride
    // 33 between the blocks the fold writes from 32 lanes at once)
    static constexpr int AST = N + N / 32;
    static constexpr int ECOP_DW = EBUF * 2 * 4 * 4 * CLEN; // buf, c', q, sigma
};

// Workgroup barrier ordering LDS only.  Inside the CMux loops the threads
// of a workgroup share nothing through global memory, and a full
// __syncthreads would also wait for the key reads issued ahead of use.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t modswitch(uint32_t u, int log2_2n)
{
    return (u + (1u << (31 - log2_2n))) >> (32 - log2_2n);
}

// bsk [n][2l][2][N] -> limb windows [n][R][2][4][ELEN]
//   window y of (i, r*S+s, c') holds a_ext[y - 31] * 2^(7s),
//   a_ext[x] = a[x] (0 <= x < N), -a[x+N] (x < 0), 0 beyond N.
template <int N>
__global__ void k_int8_key(const uint32_t *__restrict__ bsk,
                           int8_t *__restrict__ out, int n, int l, int S)
{
    using C = I8Cfg<N>;
    const int R = 2 * l * S;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)n * R * 2 * C::ELEN;
    if (idx >= total)
        return;
    int y = (int)(idx % C::ELEN);
    size_t t = idx / C::ELEN;
    int cp = (int)(t % 2);
    t /= 2;
    int kb = (int)(t % R);
    int i = (int)(t / R);
    int r = kb / S, s = kb % S;
    int x = y - 31;
    const uint32_t *a = bsk + (((size_t)i * 2 * l + r) * 2 + cp) * N;
    uint32_t v = 0;
    if (x >= 0 && x < N)
        v = a[x];
    else if (x < 0)
        v = 0u - a[x + N];
    v <<= 7 * s;
    int8_t *o = out + (((size_t)i * R + kb) * 2 + cp) * 4 * C::ELEN + y;
    for (int q = 0; q < 4; ++q) {
        int8_t limb = (int8_t)(v & 0xFFu);
        o[(size_t)q * C::ELEN] = limb;
        v = (v - (uint32_t)(int32_t)limb) >> 8;
    }
}

// Offset correction of the digit operands (decompose_acc with OFF).  With
// the positive copy holding delta + 64 and the negated copy 63 - delta, the
// GEMM output for coefficient j = 32J + rho of component c' at step i
// exceeds the product by
//   sum over digit rows of (64 * sum_{Delta <= J} W_Delta[rho]
//                           + 63 * sum_{Delta > J} W_Delta[rho])
//   = sum over digit rows of (63 * total[rho] + head_J[rho]),
// where W_Delta[rho] = sum_{kappa < 32} a_ext[32 Delta + rho - kappa] *
// 2^(7s) is the row sum of the Toeplitz block A_Delta of that row's key
// polynomial, total[rho] the sum over every Delta and head_J[rho] the sum
// over Delta <= J (block offsets up to J use the positive copy).  corr
// [n][2][N] holds that excess mod 2^32; the bootstrap kernel starts one
// accumulator per output coefficient from its negation.  One workgroup per
// (i, c').
template <int N>
__global__ __launch_bounds__(256) void k_int8_corr(
    const uint32_t *__restrict__ bsk, uint32_t *__restrict__ corr, int n,
    int l, int S)
{
    constexpr int NB = N / 32, PT = N / 256;
    __shared__ uint32_t ext[N + 32];   // ext[x + 31] = a_ext[x], -31 <= x < N
    __shared__ uint32_t W[N];          // W_Delta[rho] at 32 Delta + rho
    const int i = blockIdx.x >> 1, cp = blockIdx.x & 1;
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
        for (int x = tid - 31; x < N; x += 256)
            ext[x + 31] = x >= 0 ? a[x] : 0u - a[x + N];
        __syncthreads();
        for (int t = tid; t < N; t += 256) {
            uint32_t w = 0;
            for (int kap = 0; kap < 32; ++kap)
                w += ext[t - kap + 31];
            W[t] = w;
        }
        __syncthreads();
        if (tid < 32) {                // prefix over Delta, per rho
            uint32_t run = 0;
            for (int D = 0; D < NB; ++D) {
                run += W[32 * D + tid];
                W[32 * D + tid] = run;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const int j = tid + 256 * k, J = j >> 5, rho = j & 31;
            const uint32_t total = W[32 * (NB - 1) + rho];
            accv[k] += (63u * total + W[32 * J + rho]) << (7 * s);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PT; ++k)
        corr[((size_t)i * 2 + cp) * N + tid + 256 * k] = accv[k];
}

template <int N, int T = 4>
struct I8Smem {
    using C = I8Cfg<N, T>;
    static constexpr size_t ecop = (size_t)C::ECOP_DW * 4;
    static constexpr size_t acc = (size_t)C::GPW * 2 * C::AST * 4;
    static size_t dig(int R) { return (size_t)C::GPW * R * 2 * N; }
    static size_t ms(int n) { return ((size_t)C::GPW * (n + 1) * 2 + 15) & ~(size_t)15; }
    static size_t total(int R, int n) { return ecop + acc + dig(R) + ms(n); }
};

// Rotate the accumulator of every bootstrap of the workgroup by
// a~_i = ms[i] (X^(a~_i) ACC - ACC), add the digit offset and split each
// coefficient into R signed int8 digit operands, in both signs (ArctyrEX
// Fig. 1, the decomposition of the CMux step; Section 2.2).
// Layout of dig: [GPW][R][kappa half][sign: -, +][NB][16] bytes (the 16
// bytes of a lane's B operand hold one 32-block's kappa half in reverse).
// Each kappa half holds the negated blocks followed by the blocks, so the
// sign-rotated block (J - Delta) mod NB the K loops read is block
// NB + J - Delta of that half: linear in the block offset Delta.
// NC = 1 decomposes component c_sel only, into rows 0 .. l*SS - 1 (R then
// counts the rows per bootstrap of that layout).
// OFF stores each sub-digit delta as delta + 64 and its negation as
// 63 - delta, both in [0, 127]: non-negative operands cost the matrix cores
// less energy (4-5% faster at the power limit).  The offsets' contribution,
// a function of the key alone, is removed with a precomputed table (see
// k_int8_corr).
template <int N, int L, int S, int GPW, int THREADS, int NC = 2,
          bool OFF = false>
__device__ __forceinline__ void decompose_acc(
    const uint32_t *acc, int8_t *dig, const uint16_t *ms, int i, int n, int l,
    int SS, int R, int beta, uint32_t dig_off, uint32_t bmask, int32_t bhalf,
    int tid, int c_sel = 0)
{
    constexpr int NB = N / 32, AST = N + N / 32;
    auto ap = [](int j) { return j + (j >> 5); };
    for (int item = tid; item < GPW * NC * (N / 4); item += THREADS) {
        int gl = item / (NC * (N / 4));
        int rem = item - gl * (NC * (N / 4));
        int c = NC == 2 ? rem / (N / 4) : c_sel;
        int m0 = 4 * (NC == 2 ? rem - c * (N / 4) : rem);
        int e = ms[gl * (n + 1) + i];
        const uint32_t *a = acc + (gl * 2 + c) * AST;
        const int pm0 = ap(m0);           // the quad stays in one block
        uint32_t w4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int t = (m0 + k - e) & (2 * N - 1);
            uint32_t rv = a[ap(t & (N - 1))];
            rv = t >= N ? 0u - rv : rv;
            w4[k] = rv - a[pm0 + k] + dig_off;
        }
        // byte b of the dword holds coefficient m0 + 3 - b (reversed kappa)
        int kap0 = m0 & 31, M = m0 >> 5;
        int kp = 28 - kap0;                 // kappa' of byte 0
        int off = (kp >> 4) * (2 * NB * 16) + M * 16 + (kp & 15);
        int8_t *gbase = dig + (size_t)gl * R * 2 * N + off;
#pragma unroll
        for (int p = 1; p <= (L ? L : 8); ++p) {
            if (!L && p > l)
                break;
            int32_t d[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                d[k] = (int32_t)((w4[k] >> (32 - p * beta)) & bmask) - bhalf;
#pragma unroll
            for (int s = 0; s < (L ? S : 2); ++s) {
                if (!L && s >= SS)
                    break;
                uint32_t pos = 0, neg = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int32_t sd;
                    if (s == SS - 1) {
                        sd = d[k];
                    } else {
                        sd = ((d[k] + 64) & 127) - 64;
                        d[k] = (d[k] - sd) >> 7;
                    }
                    if (OFF) {
                        pos |= (uint32_t)(sd + 64) << (8 * (3 - k));
                        neg |= (uint32_t)(63 - sd) << (8 * (3 - k));
                    } else {
                        pos |= ((uint32_t)sd & 0xFFu) << (8 * (3 - k));
                    }
                }
                if (!OFF) {
                    // negate the four bytes at once: ~b + 1 per byte, the
                    // +1 kept inside each byte's low 7 bits
                    const uint32_t npos = ~pos;
                    neg = ((npos & 0x7F7F7F7Fu) + 0x01010101u) ^
                          (npos & 0x80808080u);
                }
                int kb = ((NC == 2 ? c * l : 0) + (p - 1)) * SS + s;
                int8_t *base = gbase + (size_t)kb * 2 * N;
                *reinterpret_cast<uint32_t *>(base + NB * 16) = pos;
                *reinterpret_cast<uint32_t *>(base) = neg;
            }
        }
    }
}

// L (gadget levels) and S (sub-digits per digit) are compile-time so the
// digit loops unroll; L = 0 selects a generic build that reads l and S at
// run time.
template <int N, int L, int S, int T>
__global__ __launch_bounds__((I8Cfg<N, T>::THREADS), 1) void k_bootstrap_int8(
    const int8_t *__restrict__ key, const uint32_t *__restrict__ corr,
    const uint32_t *__restrict__ in, const uint32_t *__restrict__ testv,
    uint32_t *__restrict__ out, int B, const int32_t *__restrict__ d_count,
    int lo, int hi, int n, int beta, int l_rt, int S_rt)
{
    using C = I8Cfg<N, T>;
    constexpr int NB = C::NB, GPT = C::GPT, GPW = C::GPW, TPG = C::TPG;
    constexpr int EBUF = C::EBUF;
    constexpr bool BIG = C::BIG;
    // offset digits (non-negative operands, which the matrix cores run
    // faster on when the CUs are all busy) with the key-only correction; the
    // latency-bound one-tile kernel gains nothing from it and the N = 2048
    // layout has no registers to spare, so they keep signed digits
    constexpr bool OFF = !BIG && T >= 2;
    constexpr int I8_THREADS = C::THREADS;
    constexpr int CLEN = C::CLEN, CW = C::CW, EW = C::EW, AST = C::AST;
    constexpr int LOG2_2N = __builtin_ctz(2 * N);
    const int l = L ? L : l_rt;
    const int SS = L ? S : S_rt;
    const int R = 2 * l * SS;

    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *ecop = reinterpret_cast<uint32_t *>(smem);
    uint32_t *acc = ecop + C::ECOP_DW;                       // [GPW][2][AST]
    int8_t *dig = reinterpret_cast<int8_t *>(acc + GPW * 2 * AST);
    uint16_t *ms = reinterpret_cast<uint16_t *>(dig + (size_t)GPW * R * 2 * N);
    auto ap = [](int j) { return j + (j >> 5); };            // padded index

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
    const int wave = tid >> 6;

    // ---- modulus switch of the inputs --------------------------------
    for (int idx = tid; idx < GPW * (n + 1); idx += I8_THREADS) {
        int gl = idx / (n + 1), i = idx - gl * (n + 1);
        int g = g0 + gl;
        uint32_t u = g < count ? in[(size_t)g * (n + 1) + i] : 0u;
        ms[idx] = (uint16_t)modswitch(u, LOG2_2N);
    }
    __syncthreads();
    // ---- ACC = (0, X^(2N - b~) v) ---------------------------------------
    for (int idx = tid; idx < GPW * N; idx += I8_THREADS) {
        int gl = idx / N, m = idx - gl * N;
        int e = (2 * N - ms[gl * (n + 1) + n]) & (2 * N - 1);
        uint32_t v = testv ? testv[m] : (1u << 29);
        int t = m + e;
        if (t >= 2 * N) {
            t -= 2 * N;
        } else if (t >= N) {
            t -= N;
            v = 0u - v;
        }
        acc[(gl * 2 + 0) * AST + ap(t)] = 0u;
        acc[(gl * 2 + 1) * AST + ap(t)] = v;
    }

    // ---- key-window staging ----------------------------------------------
    // stage st = i*R + kb uses buffer st & 1; item = (array c'*4+q, word w).
    // The global reads of stage st + PD are issued when stage st starts (for
    // PD = 2 into far_*, whose previous contents, stage st + 1, are first
    // moved into pre_*); the four byte-shifted LDS copies of stage st + 1
    // are written from pre_* between stage st's MFMA groups.
    constexpr int ITEMS = 8 * CW;
    constexpr int PER_T = (ITEMS + I8_THREADS - 1) / I8_THREADS;
    constexpr int PD = C::PD;
    uint32_t pre_lo[PER_T], pre_hi[PER_T];
    uint32_t far_lo[PD > 1 ? PER_T : 1], far_hi[PD > 1 ? PER_T : 1];
    auto fetch = [&](int st, auto &lo, auto &hi) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(key) +
                              (size_t)st * 8 * EW;
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            int item = tid + k * I8_THREADS;
            if (PD > 1) {
                // every lane loads (the surplus ones a valid word they never
                // store), so the registers in flight need no merge and are
                // not waited for until they are used
                item = min(item, ITEMS - 1);
            } else if (item >= ITEMS) {
                continue;
            }
            int arr = item / CW, w = item - arr * CW;
            lo[k] = src[arr * EW + w];
            hi[k] = src[arr * EW + w + 1];
        }
    };
    auto stash_one = [&](int buf, int k) {
        int item = tid + k * I8_THREADS;
        if (item < ITEMS) {
            int arr = item / CW, w = item - arr * CW;
            uint32_t *d = ecop + (EBUF == 2 ? buf : 0) * (2 * 4 * 4 * CLEN) +
                          arr * 4 * CLEN + w;
            d[0] = pre_lo[k];
            d[CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 1);
            d[2 * CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 2);
            d[3 * CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 3);
        }
    };
    auto stash_dyn = [&](int buf, int k) {
#pragma unroll
        for (int kk = 0; kk < PER_T; ++kk)
            if (kk == k)
                stash_one(buf, kk);
    };
    fetch(0, pre_lo, pre_hi);
#pragma unroll
    for (int k = 0; k < PER_T; ++k)
        stash_one(0, k);
    if (PD > 1 && n * R > 1)
        fetch(1, far_lo, far_hi);
    __syncthreads();

    // ---- per-lane constants ----------------------------------------------
    // waves that differ only in `half` split the block offsets; the
    // partial sums of all waves of one output component meet in the fold
    constexpr int WT = C::WT, LPW = C::LPW;
    const int cp = wave & 1;                              // output component
    const int q0 = BIG ? 0 : LPW * ((wave >> 1) & 1);     // first key limb
    // block-offset part: half, or quarter at N = 2048 and with 16 waves
    const int half = BIG ? wave >> 1 : wave >> 2;
    // the wave that adds the offset correction of its output component
    const bool corr_wave = half == 0 && q0 == 0;
    const int rho = lane & 31, hh = lane >> 5;
    // A operand: dword offset of this lane inside one (buf, c', q) group
    const int a_lane = (rho & 3) * CLEN + (rho >> 2) + 4 * hh;
    // B operand: column c of tile t -> bootstrap in the workgroup and
    // output block J of that bootstrap
    int glt[WT], Jt[WT];
#pragma unroll
    for (int tt = 0; tt < WT; ++tt) {
        glt[tt] = BIG ? tt / TPG : tt * GPT + rho / NB;
        Jt[tt] = BIG ? 32 * (tt % TPG) + rho : rho % NB;
    }

    const uint32_t round_off = (beta * l < 32) ? (1u << (31 - beta * l)) : 0u;
    uint32_t dig_off = round_off;
    for (int p = 1; p <= l; ++p)
        dig_off += (1u << (beta - 1)) << (32 - p * beta);
    const uint32_t bmask = (1u << beta) - 1u;
    const int32_t bhalf = 1 << (beta - 1);

    v16i Cacc[WT][LPW];

    for (int i = 0; i < n; ++i) {
        lds_barrier();   // ACC of the previous step complete
        // ---- rotate, subtract, decompose into digit operands --------------
        // one wave per output component starts its limb-0 accumulators
        // from minus the step's offset correction (the same for every tile:
        // output block Jt[t] depends on the lane only)
        v16i cinit = {};
        if (OFF && corr_wave) {
            const uint32_t *cr =
                corr + ((size_t)i * 2 + cp) * N + 32 * Jt[0] + 4 * hh;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const v4i c4 = *reinterpret_cast<const v4i *>(cr + 8 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    cinit[4 * g + e] = -c4[e];
            }
        }
        decompose_acc<N, L, S, GPW, I8_THREADS, 2, OFF>(
            acc, dig, ms, i, n, l, SS, R, beta, dig_off, bmask, bhalf, tid);
        lds_barrier();

        // ---- K loop: digit polynomials x block offsets --------------------
        // one stage per digit polynomial; the first is a separate
        // instantiation so that the correction start values (cinit) are
        // dead in the others
        auto stage = [&](const int kb, auto first_c) {
            constexpr bool FIRST = decltype(first_c)::value;
            const int st = i * R + kb;
            const bool more = st + 1 < n * R;
            if constexpr (PD == 1) {
                if (more)
                    fetch(st + 1, pre_lo, pre_hi);
            } else {
#pragma unroll
                for (int k = 0; k < PER_T; ++k) {
                    pre_lo[k] = far_lo[k];
                    pre_hi[k] = far_hi[k];
                }
                // unconditional (the last stages re-read the final window)
                // for the same reason as the clamped items
                fetch(min(st + 2, n * R - 1), far_lo, far_hi);
            }
            const uint32_t *eb = ecop + (EBUF == 2 ? (st & 1) : 0) *
                                            (2 * 4 * 4 * CLEN) +
                                 cp * (4 * 4 * CLEN) + a_lane;
            // block NB + J of this lane's kappa half (see decompose_acc)
            const int8_t *db[WT];
#pragma unroll
            for (int t = 0; t < WT; ++t)
                db[t] = dig + ((size_t)(glt[t] * R + kb) * 2) * N +
                        hh * (2 * NB * 16) + 16 * (NB + Jt[t]);
            // A operand of block offset dl: this wave's limb rows of the
            // Toeplitz window
            auto load_a = [&](int dl, v4i (&af)[LPW]) {
#pragma unroll
                for (int q = 0; q < LPW; ++q) {
                    const uint32_t *apq = eb + (q0 + q) * (4 * CLEN) + 8 * dl;
                    af[q][0] = (int)apq[0];
                    af[q][1] = (int)apq[1];
                    af[q][2] = (int)apq[2];
                    af[q][3] = (int)apq[3];
                }
            };
            // B operand of block offset dl: the sign-rotated digit blocks of
            // the tiles, block NB + J - dl of the lane's kappa half
            auto load_b = [&](int dl, v4i (&bf)[WT]) {
#pragma unroll
                for (int t = 0; t < WT; ++t)
                    bf[t] = *reinterpret_cast<const v4i *>(db[t] - 16 * dl);
            };
            // block offsets per wave: NB over the waves that share a
            // (component, limb set)
            constexpr int ND = BIG ? NB / 4 : NB / (I8_THREADS / 256);
            constexpr int STASH0 = ND >= PER_T + 4 ? 4 : 0;
            // this wave's block offsets: dl0 .. dl0 + ND - 1.  Group d0
            // reads the operands of d0 + 1 into the other register buffer
            // in the issue shadows of its own MFMAs (one LDS read and a few
            // address ops after each MFMA).
            const int dl0 = half * ND;
            v4i af[2][LPW], bf[2][WT];
            auto group = [&](int d0, int b, bool zero_start) {
                if (d0 + 1 < ND) {
                    load_a(dl0 + d0 + 1, af[b ^ 1]);
                    load_b(dl0 + d0 + 1, bf[b ^ 1]);
                }
                const v16i zero = {};
                auto mfma = [&](int t, int q) {
                    Cacc[t][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        af[b][q], bf[b][t],
                        zero_start ? (q == 0 ? cinit : zero) : Cacc[t][q],
                        0, 0, 0);
                };
                // tile-outer order for four tiles, limb-outer for two (each
                // 1-2% faster than the other order on the MI355X; the sums
                // do not depend on it)
                if constexpr (T == 4) {
#pragma unroll
                    for (int t = 0; t < WT; ++t)
#pragma unroll
                        for (int q = 0; q < LPW; ++q)
                            mfma(t, q);
                } else {
#pragma unroll
                    for (int q = 0; q < LPW; ++q)
#pragma unroll
                        for (int t = 0; t < WT; ++t)
                            mfma(t, q);
                }
#pragma unroll
                for (int k = 0; k < WT * LPW; ++k) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0); // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0); // DS read
                    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0); // VALU
                }
                __builtin_amdgcn_sched_barrier(0);
                // spread the next stage's LDS copies between MFMA groups
                if (EBUF == 2 && more && d0 >= STASH0 && d0 - STASH0 < PER_T)
                    stash_dyn((st + 1) & 1, d0 - STASH0);
                __builtin_amdgcn_sched_barrier(0);
            };
            load_a(dl0, af[0]);
            load_b(dl0, bf[0]);
            group(0, 0, FIRST);   // the first stage starts the accumulators
#pragma unroll 1
            for (int d0 = 1; d0 + 1 < ND; d0 += 2) {
                group(d0, 1, false);
                group(d0 + 1, 0, false);
            }
            group(ND - 1, 1, false);
            if (EBUF == 2 && ND < PER_T + 4 && more) {
                // small N: fewer MFMA groups than copy items
                for (int k = ND - STASH0; k < PER_T; ++k)
                    stash_dyn((st + 1) & 1, k);
            }
            lds_barrier();
            if (EBUF == 1 && more) {
                // single window buffer: refill it once every wave is done
#pragma unroll
                for (int k = 0; k < PER_T; ++k)
                    stash_one(0, k);
                lds_barrier();
            }
        };
        stage(0, std::true_type{});
        for (int kb = 1; kb < R; ++kb)
            stage(kb, std::false_type{});

        // ---- fold limbs, add into ACC ---------------------------------------
#pragma unroll
        for (int t = 0; t < WT; ++t) {
            uint32_t *a = acc + (glt[t] * 2 + cp) * AST + 33 * Jt[t];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                int row = 8 * (v >> 2) + 4 * hh + (v & 3);
                uint32_t x = 0;
#pragma unroll
                for (int q = 0; q < LPW; ++q)
                    x += (uint32_t)Cacc[t][q][v] << (8 * q);
                // every wave of this component adds its limbs' part over its
                // block offsets (mod 2^32, order-free)
                atomicAdd(&a[row], x << (8 * q0));
            }
        }
    }
    __syncthreads();

    // ---- sample extraction ---------------------------------------------------
    for (int idx = tid; idx < GPW * (N + 1); idx += I8_THREADS) {
        int gl = idx / (N + 1), j = idx - gl * (N + 1);
        int g = g0 + gl;
        if (g >= count)
            continue;
        const uint32_t *a = acc + gl * 2 * AST;
        uint32_t v;
        if (j == 0)
            v = a[0];
        else if (j < N)
            v = 0u - a[ap(N - j)];
        else
            v = a[AST];
        out[(size_t)g * (N + 1) + j] = v;
    }
}

// ---- latency mode: one tile's blind rotation over four workgroups --------
//
// A narrow batch leaves most CUs idle and each bootstrap's n CMux steps run
// one after another on a single CU.  Here the step's GEMM of one column
// tile (GPT = 1024/N bootstraps) is split over SPLIT_G = 4 workgroups on
// four CUs along the 2 x 2 block structure of the external product: member
// m adds the digits of accumulator component c = m >> 1 times the key rows
// of that component into output component c' = m & 1, for all four key
// limbs (its 8 waves split the block offsets), so it decomposes only its
// own input component.  Every member keeps a full copy of the
// accumulators; after each step the members exchange their partial sums
// through global memory (64-bit words holding a 32-bit tag and the
// 32-bit value, so a word is either the step's or stale as a whole) and
// each adds all four into its copy.  The tag is the step plus a per-group
// launch epoch (device-resident, advanced by member 0 when its group has
// finished), so words left by an earlier launch never match.  Waits are
// bounded: a member that waits longer than SPLIT_WAIT_TICKS of the 100 MHz
// wall clock, or sees the context's error word set, sets that word and
// stops; later launches on the context do nothing until cggi_ctx_check
// clears it.  The members of a group are placed on one XCD (blocks of one
// group are congruent mod 8), which keeps the exchange in one L2.
constexpr int SPLIT_THREADS = 512;
constexpr int SPLIT_STATIC_LDS = 64;     // bound on the kernel's static LDS
constexpr int SPLIT_RMAX = 8;            // digit polynomials per step
constexpr unsigned long long SPLIT_WAIT_TICKS = 100000000ull;   // 1 s

template <int N> struct SplitCfg {
    static constexpr int NB = N / 32;
    static constexpr int GPT = 1024 / N;    // bootstraps per column tile
    static constexpr int ND = NB / 8;       // block offsets per wave
    static constexpr int EW = (N + 64) / 4; // dwords per limb window
    static constexpr int CW = N / 4 + 8;    // dwords of a shifted copy used
    static constexpr int CLEN = N / 4 + 8;  // stride of a shifted copy
    static constexpr int AST = N + N / 32;  // padded accumulator row
    static constexpr int WORDS = GPT * N;   // partial words per member
};

// G = 4 members per tile as above; G = 8 (for batches of at most half as
// many tiles) splits each member's four key limbs into two pairs; G = 2 (for
// batches up to twice as wide) gives member m = c' both input components.
template <int G> struct SplitRole {
    static constexpr int LPM = G == 8 ? 2 : 4;       // key limbs per member
    static constexpr bool ONE_C = G != 2;            // one input component
};

template <int N, int G>
static size_t split_smem_bytes(int R, int n)
{
    using C = SplitCfg<N>;
    using Ro = SplitRole<G>;
    const int RM = Ro::ONE_C ? R / 2 : R;            // digit rows per member
    size_t b = (size_t)RM * 4 * Ro::LPM * C::CLEN * 4 // key windows of a step
               + (size_t)C::GPT * 3 * C::AST * 4     // accumulators + partial
               + (size_t)C::GPT * RM * 2 * N;        // digit operands
    return b + (((size_t)C::GPT * (n + 1) * 2 + 15) & ~(size_t)15);
}

// Launches that read their bootstrap count from the device may be issued
// for several kernels at once; each runs only when lo < count <= hi.
template <int N, int L, int S, int G>
__global__ __launch_bounds__(SPLIT_THREADS, 1) void k_bootstrap_int8_split(
    const int8_t *__restrict__ key, const uint32_t *__restrict__ in,
    const uint32_t *__restrict__ testv, uint32_t *__restrict__ out, int B,
    const int32_t *__restrict__ d_count, int lo, int hi,
    unsigned long long *xb, uint32_t *epoch, uint32_t *err, int n, int beta,
    int l_rt, int S_rt)
{
    static_assert(G == 8 || G == 4 || G == 2, "8, 4 or 2 members per tile");
    constexpr int LPM = SplitRole<G>::LPM;
    constexpr bool ONE_C = SplitRole<G>::ONE_C;
    using C = SplitCfg<N>;
    constexpr int NB = C::NB, GPT = C::GPT, ND = C::ND, EW = C::EW;
    constexpr int CW = C::CW, CLEN = C::CLEN, AST = C::AST;
    constexpr int WORDS = C::WORDS, T = SPLIT_THREADS;
    constexpr int LOG2_2N = __builtin_ctz(2 * N);
    const int l = L ? L : l_rt;
    const int SS = L ? S : S_rt;
    const int R = 2 * l * SS;
    const int RH = l * SS;                 // digit rows of one component
    const int RM = ONE_C ? RH : R;         // digit rows of this member

    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *ecop = reinterpret_cast<uint32_t *>(smem); // [RM][LPM][4][CLEN]
    uint32_t *acc = ecop + RM * LPM * 4 * CLEN;             // [GPT][2][AST]
    uint32_t *part = acc + GPT * 2 * AST;                   // [GPT][AST]
    int8_t *dig = reinterpret_cast<int8_t *>(part + GPT * AST);
    uint16_t *ms =
        reinterpret_cast<uint16_t *>(dig + (size_t)GPT * RM * 2 * N);
    __shared__ int s_stop;
    __shared__ uint32_t s_ep;
    auto ap = [](int j) { return j + (j >> 5); };

    // block -> (group, member): the members of a group share b mod 8
    const int x8 = blockIdx.x & 7, q8 = blockIdx.x >> 3;
    const int member = q8 % G;
    const int grp = (q8 / G) * 8 + x8;
    const int dc = d_count ? *d_count : B;
    if (dc <= lo || dc > hi)
        return;
    const int count = min(B, dc);
    const int g0 = grp * GPT;
    if (g0 >= count)
        return;
    const int cp = G == 2 ? member : member & 1;          // output component
    const int ch = G == 2 ? 0 : (member >> 1) & 1;        // input component
    const int q0 = G == 8 ? 2 * (member >> 2) : 0;        // first key limb
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    if (tid == 0) {
        s_stop = __hip_atomic_load(err, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) != 0;
        s_ep = __hip_atomic_load(&epoch[grp], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    }
    // ---- modulus switch, ACC = (0, X^(2N - b~) v), partial = 0 -----------
    for (int idx = tid; idx < GPT * (n + 1); idx += T) {
        int gl = idx / (n + 1), i = idx - gl * (n + 1);
        int g = g0 + gl;
        uint32_t u = g < count ? in[(size_t)g * (n + 1) + i] : 0u;
        ms[idx] = (uint16_t)modswitch(u, LOG2_2N);
    }
    for (int idx = tid; idx < GPT * AST; idx += T)
        part[idx] = 0u;
    __syncthreads();
    if (s_stop)
        return;
    const uint32_t ep = s_ep;
    for (int idx = tid; idx < GPT * N; idx += T) {
        int gl = idx / N, m = idx - gl * N;
        int e = (2 * N - ms[gl * (n + 1) + n]) & (2 * N - 1);
        uint32_t v = testv ? testv[m] : (1u << 29);
        int t = m + e;
        if (t >= 2 * N) {
            t -= 2 * N;
        } else if (t >= N) {
            t -= N;
            v = 0u - v;
        }
        acc[(gl * 2 + 0) * AST + ap(t)] = 0u;
        acc[(gl * 2 + 1) * AST + ap(t)] = v;
    }

    // ---- key windows of this member's rows (digit rows of component ch,
    // output component c', four limbs), one step at a time:
    // step i + 1's are read while step i's partials are exchanged (the two
    // latencies overlap) and then written to LDS in four byte-shifted
    // copies; no read stays in flight from one step into the next
    constexpr int RMAX = (L ? 2 * L * S : SPLIT_RMAX) / (ONE_C ? 2 : 1);
    constexpr int PER_T = (RMAX * LPM * CW + T - 1) / T;
    const int items = RM * LPM * CW;
    uint32_t pre_lo[PER_T], pre_hi[PER_T];
    auto fetch = [&](int i) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(key) +
                              ((size_t)i * R + ch * RH) * 8 * EW;
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            // surplus lanes re-read the last word (never stored)
            int item = min(tid + k * T, items - 1);
            int kb = item / (LPM * CW), rem = item - kb * (LPM * CW);
            int q = rem / CW, w = rem - q * CW;
            const uint32_t *sp =
                src + ((size_t)kb * 8 + cp * 4 + q0 + q) * EW + w;
            pre_lo[k] = sp[0];
            pre_hi[k] = sp[1];
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < PER_T; ++k) {
            int item = tid + k * T;
            if (item < items) {
                int kb = item / (LPM * CW), rem = item - kb * (LPM * CW);
                int q = rem / CW, w = rem - q * CW;
                uint32_t *d = ecop + (kb * LPM + q) * 4 * CLEN + w;
                d[0] = pre_lo[k];
                d[CLEN] = __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 1);
                d[2 * CLEN] =
                    __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 2);
                d[3 * CLEN] =
                    __builtin_amdgcn_alignbyte(pre_hi[k], pre_lo[k], 3);
            }
        }
    };
    fetch(0);
    stash();

    // ---- per-lane constants ----------------------------------------------
    const int rho = lane & 31, hh = lane >> 5;
    const int a_lane = (rho & 3) * CLEN + (rho >> 2) + 4 * hh;
    const int glc = rho / NB, Jc = rho % NB;   // column -> bootstrap, block
    const int dl0 = wave * ND;
    const uint32_t round_off = (beta * l < 32) ? (1u << (31 - beta * l)) : 0u;
    uint32_t dig_off = round_off;
    for (int p = 1; p <= l; ++p)
        dig_off += (1u << (beta - 1)) << (32 - p * beta);
    const uint32_t bmask = (1u << beta) - 1u;
    const int32_t bhalf = 1 << (beta - 1);
    unsigned long long *xg = xb + (size_t)grp * 2 * G * WORDS;
    // block NB + Jc of this lane's kappa half (see decompose_acc)
    const int8_t *dbase = dig + (size_t)glc * RM * 2 * N +
                          hh * (2 * NB * 16) + 16 * (NB + Jc);
    constexpr int PW = WORDS / T;                 // words per thread

    for (int i = 0; i < n; ++i) {
        lds_barrier();   // ACC and this step's key windows complete
        if (s_stop)
            break;
        if constexpr (ONE_C)
            decompose_acc<N, L, S, GPT, T, 1>(acc, dig, ms, i, n, l, SS, RH,
                                              beta, dig_off, bmask, bhalf,
                                              tid, ch);
        else
            decompose_acc<N, L, S, GPT, T, 2>(acc, dig, ms, i, n, l, SS, R,
                                              beta, dig_off, bmask, bhalf,
                                              tid);
        lds_barrier();

        // ---- K loop over (digit row of the member, block offset) --------
        auto load = [&](int idx, v4i (&af)[LPM], v4i &bf) {
            const int kb = idx / ND, dl = dl0 + idx % ND;
            const uint32_t *eb = ecop + kb * LPM * 4 * CLEN + a_lane + 8 * dl;
#pragma unroll
            for (int q = 0; q < LPM; ++q) {
                const uint32_t *apq = eb + q * 4 * CLEN;
                af[q][0] = (int)apq[0];
                af[q][1] = (int)apq[1];
                af[q][2] = (int)apq[2];
                af[q][3] = (int)apq[3];
            }
            bf = *reinterpret_cast<const v4i *>(dbase + (size_t)kb * 2 * N -
                                                16 * dl);
        };
        const int K = RM * ND;
        v16i Cq[LPM] = {};
        v4i af0[LPM], af1[LPM], bf0, bf1;
        auto mfma4 = [&](const v4i (&af)[LPM], const v4i &bf) {
#pragma unroll
            for (int q = 0; q < LPM; ++q)
                Cq[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[q], bf, Cq[q],
                                                              0, 0, 0);
        };
        load(0, af0, bf0);
#pragma unroll 1
        for (int idx = 0; idx < K; idx += 2) {
            if (idx + 1 < K)
                load(idx + 1, af1, bf1);
            mfma4(af0, bf0);
            if (idx + 1 >= K)
                break;
            if (idx + 2 < K)
                load(idx + 2, af0, bf0);
            mfma4(af1, bf1);
        }
        // ---- fold the member's limbs, add this wave's block offsets ------
        {
            uint32_t *pp = part + glc * AST + 33 * Jc;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                int row = 8 * (v >> 2) + 4 * hh + (v & 3);
                uint32_t xv = 0;
#pragma unroll
                for (int q = 0; q < LPM; ++q)
                    xv += (uint32_t)Cq[q][v] << (8 * q);
                atomicAdd(&pp[row], xv << (8 * q0));
            }
        }
        lds_barrier();   // partial complete; key windows free

        // ---- publish the partial (tag = epoch * 1024 + step + 1) --------
        const unsigned long long tag =
            (unsigned long long)(ep * 1024u + (uint32_t)i + 1u) << 32;
        unsigned long long *xw =
            xg + ((size_t)(i & 1) * G + member) * WORDS;
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const int m = tid + k * T;
            const int gl = m / N, j = m - gl * N;
            uint32_t *pp = &part[gl * AST + ap(j)];
            __hip_atomic_store(&xw[m], tag | *pp, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            *pp = 0u;
        }
        // ---- gather the partials of every member ------------------------
        const unsigned long long *xr = xg + (size_t)(i & 1) * G * WORDS;
        unsigned long long wv[G][PW];
#pragma unroll
        for (int mb = 0; mb < G; ++mb)
#pragma unroll
            for (int k = 0; k < PW; ++k)
                wv[mb][k] = __hip_atomic_load(&xr[mb * WORDS + tid + k * T],
                                              __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        // the key windows of step i + 1: read while the partials arrive
        // (unconditionally, so the waits below count exactly; the last step
        // re-reads its own windows and stores nothing)
        fetch(min(i + 1, n - 1));
        // every word is tested (no short cut), so no read is left in flight
        auto all_tagged = [&]() {
            unsigned long long diff = 0;
#pragma unroll
            for (int mb = 0; mb < G; ++mb)
#pragma unroll
                for (int k = 0; k < PW; ++k)
                    diff |= (wv[mb][k] & 0xFFFFFFFF00000000ull) ^ tag;
            return diff == 0;
        };
        bool failed = false;
        // the first test sits outside any loop, so it waits for the gather
        // reads only (the key reads issued after them stay in flight)
        if (!all_tagged()) {
            const unsigned long long t_start = wall_clock64();
            for (int it = 1;; ++it) {
                if ((it & 15) == 0 &&
                    (__hip_atomic_load(err, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                     wall_clock64() - t_start > SPLIT_WAIT_TICKS)) {
                    __hip_atomic_store(err, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    failed = true;
                    break;
                }
#pragma unroll
                for (int mb = 0; mb < G; ++mb)
#pragma unroll
                    for (int k = 0; k < PW; ++k)
                        wv[mb][k] = __hip_atomic_load(
                            &xr[mb * WORDS + tid + k * T], __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
                if (all_tagged())
                    break;
            }
        }
        if (failed) {
            s_stop = 1;
        } else {
#pragma unroll
            for (int k = 0; k < PW; ++k) {
                const int m = tid + k * T;
                const int gl = m / N, j = m - gl * N;
#pragma unroll
                for (int c2 = 0; c2 < 2; ++c2) {
                    // the members with output component c2: m & 1 == c2
                    uint32_t add = 0;
#pragma unroll
                    for (int mb = c2; mb < G; mb += 2)
                        add += (uint32_t)wv[mb][k];
                    acc[(gl * 2 + c2) * AST + ap(j)] += add;
                }
            }
        }
        if (i + 1 < n)
            stash();
    }
    __syncthreads();
    if (s_stop || member != 0)
        return;
    if (tid == 0)
        __hip_atomic_fetch_add(&epoch[grp], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);

    // ---- sample extraction (member 0) ----------------------------------------
    for (int idx = tid; idx < GPT * (N + 1); idx += T) {
        int gl = idx / (N + 1), j = idx - gl * (N + 1);
        int g = g0 + gl;
        if (g >= count)
            continue;
        const uint32_t *a = acc + gl * 2 * AST;
        uint32_t v;
        if (j == 0)
            v = a[0];
        else if (j < N)
            v = 0u - a[ap(N - j)];
        else
            v = a[AST];
        out[(size_t)g * (N + 1) + j] = v;
    }
}

} // namespace

size_t int8_smem_bytes(int N, int R, int n)
{
    switch (N) {
    case 256: return I8Smem<256>::total(R, n);
    case 512: return I8Smem<512>::total(R, n);
    case 1024: return I8Smem<1024>::total(R, n);
    case 2048: return I8Smem<2048>::total(R, n);
    default: return (size_t)-1;
    }
}

// Latency mode set-up for one kernel instantiation: the largest number of
// tile groups whose workgroups are all resident at once (so the members'
// waits on each other always end), and the exchange buffers for them.
// Variant v = 0 has four members per tile, v = 1 two; each has its own
// buffers and epochs (their word layouts differ).
template <int N, int L, int S, int G>
static int split_setup_g(Ctx *c, int v, hipStream_t s)
{
    const Shape &sh = c->sh;
    const size_t smem = split_smem_bytes<N, G>(sh.R, sh.n);
    // (the kernel also holds 8 bytes of static LDS)
    if (sh.R > SPLIT_RMAX || smem + SPLIT_STATIC_LDS > 160 * 1024)
        return CGGI_OK;                       // this variant unavailable
    const void *fn =
        reinterpret_cast<const void *>(&k_bootstrap_int8_split<N, L, S, G>);
    // the attribute belongs to the kernel, not the context: set it to the
    // most any context may launch with, so that contexts of different n
    // can share the instantiation
    CGGI_HIP_TRY(hipFuncSetAttribute(
        fn, hipFuncAttributeMaxDynamicSharedMemorySize,
        160 * 1024 - SPLIT_STATIC_LDS));
    int occ = 0;
    CGGI_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, fn, SPLIT_THREADS, smem));
    const int groups = c->cus * occ / G;
    if (groups < 1)
        return CGGI_OK;
    const size_t xwords = (size_t)groups * 2 * G * SplitCfg<N>::WORDS;
    if (hipMalloc(&c->x_buf[v], xwords * 8) != hipSuccess ||
        hipMalloc(&c->x_epoch[v], (size_t)groups * 4) != hipSuccess)
        return set_error(CGGI_E_NOMEM, "hipMalloc of the latency-mode "
                                       "exchange buffers failed");
    CGGI_HIP_TRY(hipMemsetAsync(c->x_buf[v], 0, xwords * 8, s));
    CGGI_HIP_TRY(hipMemsetAsync(c->x_epoch[v], 0, (size_t)groups * 4, s));
    c->x_words[v] = xwords;
    c->split_groups[v] = groups;
    return CGGI_OK;
}

template <int N, int L, int S>
static int split_setup_t(Ctx *c, hipStream_t s)
{
    int rc = split_setup_g<N, L, S, 4>(c, 0, s);
    if (!rc)
        rc = split_setup_g<N, L, S, 2>(c, 1, s);
    if (!rc)
        rc = split_setup_g<N, L, S, 8>(c, 2, s);
    if (rc || (!c->split_groups[0] && !c->split_groups[1] &&
               !c->split_groups[2]))
        return rc;
    if (hipMalloc(&c->x_err, 4) != hipSuccess)
        return set_error(CGGI_E_NOMEM, "hipMalloc of the latency-mode "
                                       "error word failed");
    CGGI_HIP_TRY(hipMemsetAsync(c->x_err, 0, 4, s));
    return CGGI_OK;
}

template <int N>
static int split_setup(Ctx *c, hipStream_t s)
{
    if constexpr (N > 1024) {
        return CGGI_OK;
    } else {
        const Shape &sh = c->sh;
        if (sh.l == 3 && sh.S == 1)
            return split_setup_t<N, 3, 1>(c, s);
        if (sh.l == 2 && sh.S == 2)
            return split_setup_t<N, 2, 2>(c, s);
        return split_setup_t<N, 0, 0>(c, s);
    }
}

int int8_split_reset(Ctx *c)
{
    if (!c->x_err)
        return CGGI_OK;
    for (int v = 0; v < 3; ++v) {
        if (!c->x_buf[v])
            continue;
        CGGI_HIP_TRY(hipMemset(c->x_buf[v], 0, c->x_words[v] * 8));
        CGGI_HIP_TRY(
            hipMemset(c->x_epoch[v], 0, (size_t)c->split_groups[v] * 4));
    }
    CGGI_HIP_TRY(hipMemset(c->x_err, 0, 4));
    CGGI_HIP_TRY(hipDeviceSynchronize());
    return CGGI_OK;
}

// The dynamic-LDS limit of the throughput kernels is raised when a context
// is made (on its device), not at launch: the attribute belongs to the
// kernel on a device, so launches, also under graph capture, need nothing.
template <int N, int L, int S>
static int int8_attrs_ls()
{
    const void *fns[3] = {
        reinterpret_cast<const void *>(&k_bootstrap_int8<N, L, S, 4>),
        nullptr, nullptr};
    if constexpr (N <= 1024) {
        fns[1] = reinterpret_cast<const void *>(&k_bootstrap_int8<N, L, S, 2>);
        fns[2] = reinterpret_cast<const void *>(&k_bootstrap_int8<N, L, S, 1>);
    }
    for (const void *fn : fns)
        if (fn)
            CGGI_HIP_TRY(hipFuncSetAttribute(
                fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    return CGGI_OK;
}

template <int N>
static int int8_attrs(const Shape &sh)
{
    // the same specialisations launch_bs_int8 picks
    if (sh.l == 3 && sh.S == 1)
        return int8_attrs_ls<N, 3, 1>();
    if (sh.l == 2 && sh.S == 2)
        return int8_attrs_ls<N, 2, 2>();
    return int8_attrs_ls<N, 0, 0>();
}

template <int N>
static int make_key_n(Ctx *c, const uint32_t *bsk, hipStream_t s)
{
    using C = I8Cfg<N>;
    const Shape &sh = c->sh;
    size_t kbytes = (size_t)sh.n * sh.R * 2 * 4 * C::ELEN;
    if (hipMalloc(&c->bsk_i8, kbytes) != hipSuccess) {
        c->bsk_i8 = nullptr;
        return set_error(CGGI_E_NOMEM, "hipMalloc of the int8 key failed");
    }
    size_t total = (size_t)sh.n * sh.R * 2 * C::ELEN;
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_int8_key<N>, dim3(blocks), dim3(256), 0, s, bsk,
                       c->bsk_i8, sh.n, sh.l, sh.S);
    CGGI_HIP_TRY(hipGetLastError());
    if (N <= 1024) {
        // offset correction of the throughput kernels' digit operands
        size_t cbytes = (size_t)sh.n * 2 * N * sizeof(uint32_t);
        if (hipMalloc(&c->corr_i8, cbytes) != hipSuccess) {
            c->corr_i8 = nullptr;
            return set_error(CGGI_E_NOMEM,
                             "hipMalloc of the int8 offset correction failed");
        }
        hipLaunchKernelGGL(k_int8_corr<N>, dim3(2 * sh.n), dim3(256), 0, s,
                           bsk, c->corr_i8, sh.n, sh.l, sh.S);
        CGGI_HIP_TRY(hipGetLastError());
    }
    int rc = int8_attrs<N>(sh);
    if (rc)
        return rc;
    if ((rc = kara_make_key(c, bsk, s)))
        return rc;
    rc = split_setup<N>(c, s);
    if (rc)
        return rc;
    constexpr int64_t ANY = (int64_t)1 << 40;
    constexpr int64_t gpt = N <= 1024 ? 1024 / N : 1;
    c->kind_limit[0] = (int64_t)c->split_groups[0] * gpt;
    c->kind_limit[1] = (int64_t)c->split_groups[1] * gpt;
    c->kind_limit[2] = N <= 1024 ? ANY : 0;
    c->kind_limit[3] = N <= 1024 ? ANY : 0;
    c->kind_limit[4] = ANY;
    c->kind_limit[5] = (int64_t)c->split_groups[2] * gpt;
    c->kind_limit[6] = c->bsk_k8 ? ANY : 0;
    return CGGI_OK;
}

int int8_active_plan(const Ctx *c, int32_t *kind, int32_t *cap)
{
    int32_t k0[8], c0[8];
    int n0 = 0;
    if (c->plan_n > 0) {
        for (int k = 0; k < c->plan_n; ++k) {
            k0[k] = c->plan_kind[k];
            c0[k] = c->plan_cap[k];
        }
        n0 = c->plan_n;
    } else {
        // built-in: latency mode with eight workgroups per tile up to half
        // their limit (beyond that their longer exchange outweighs the
        // shorter K loop: 2.87 vs 3.05 ms at 1 bootstrap, 3.48 vs 3.25 ms
        // at 32, N = 1024), four, then two while the tiles fit; then the
        // fewest tiles per workgroup that still fit the batch into one wave
        // of workgroups over the CUs
        const int64_t gpt = c->sh.N <= 1024 ? 1024 / c->sh.N : 1;
        if (c->kind_limit[5] > 1) {
            k0[n0] = 5;
            c0[n0++] = (int32_t)(c->kind_limit[5] / 2);
        }
        if (c->kind_limit[0] > c->kind_limit[5] / 2) {
            k0[n0] = 0;
            c0[n0++] = (int32_t)c->kind_limit[0];
        }
        if (c->kind_limit[1] > c->kind_limit[0]) {
            k0[n0] = 1;
            c0[n0++] = (int32_t)c->kind_limit[1];
        }
        if (c->kind_limit[2] > 0) {
            k0[n0] = 2;
            c0[n0++] = (int32_t)(c->cus * gpt);
            k0[n0] = 3;
            c0[n0++] = (int32_t)(2 * c->cus * gpt);
        }
        // the widest batches: the Karatsuba kernel where it is available
        // (3/4 of the MFMA work; 9% faster at 1024 default bootstraps)
        k0[n0] = c->kind_limit[6] > 0 ? 6 : 4;
        c0[n0++] = INT32_MAX;
    }
    int n = 0;
    for (int k = 0; k < n0; ++k) {
        if (!c->split_on && (k0[k] <= 1 || k0[k] == 5))
            continue;          // its batches go to the next entry
        kind[n] = k0[k];
        cap[n++] = c0[k];
    }
    return n;
}

int int8_make_key(Ctx *c, const uint32_t *bsk, hipStream_t s)
{
    switch (c->sh.N) {
    case 256: return make_key_n<256>(c, bsk, s);
    case 512: return make_key_n<512>(c, bsk, s);
    case 1024: return make_key_n<1024>(c, bsk, s);
    case 2048: return make_key_n<2048>(c, bsk, s);
    default: return set_error(CGGI_E_PARAM, "INT8 form: unsupported N");
    }
}

template <int N, int L, int S, int T>
static int launch_bs_int8_t(const Ctx *c, const uint32_t *in,
                            const uint32_t *testv, uint32_t *out, int B,
                            const int32_t *d_count, int lo, int hi,
                            hipStream_t s)
{
    using C = I8Cfg<N, T>;
    const Shape &sh = c->sh;
    size_t smem = I8Smem<N, T>::total(sh.R, sh.n);
    int grid = (B + C::GPW - 1) / C::GPW;
    hipLaunchKernelGGL((k_bootstrap_int8<N, L, S, T>), dim3(grid),
                       dim3(C::THREADS), smem, s, c->bsk_i8, c->corr_i8, in,
                       testv, out, B, d_count, lo, hi, sh.n, sh.beta, sh.l,
                       sh.S);
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

template <int N, int L, int S, int G>
static int launch_split(const Ctx *c, const uint32_t *in,
                        const uint32_t *testv, uint32_t *out, int B,
                        const int32_t *d_count, int lo, int hi, hipStream_t s)
{
    const Shape &sh = c->sh;
    const int v = G == 4 ? 0 : (G == 2 ? 1 : 2);
    const int groups = (B + SplitCfg<N>::GPT - 1) / SplitCfg<N>::GPT;
    const int grid = (groups + 7) / 8 * 8 * G;
    hipLaunchKernelGGL((k_bootstrap_int8_split<N, L, S, G>), dim3(grid),
                       dim3(SPLIT_THREADS),
                       (split_smem_bytes<N, G>(sh.R, sh.n)), s, c->bsk_i8, in,
                       testv, out, B, d_count, lo, hi, c->x_buf[v],
                       c->x_epoch[v], c->x_err, sh.n, sh.beta, sh.l, sh.S);
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

// Kernel choice by batch size from the context's plan (entries of
// increasing capacity; see int8_active_plan).  A count known on the host
// takes the first entry that holds it.  A count read on the device (a
// level's bootstraps) is bounded by B only, so every entry up to the first
// that holds B is launched, each for the counts in its own range (lo, hi];
// the others exit at once.
template <int N, int L, int S>
static int launch_bs_int8_w(const Ctx *c, const uint32_t *in,
                            const uint32_t *testv, uint32_t *out, int B,
                            const int32_t *d_count, hipStream_t s)
{
    int32_t kind[8], cap[8];
    const int no = int8_active_plan(c, kind, cap);
    long lo = 0;
    for (int k = 0; k < no; ++k) {
        const long hi = cap[k];
        const bool last = B <= hi || k == no - 1;
        if (!d_count && !last) {
            lo = hi;
            continue;
        }
        const int Bk = (int)(B < hi ? B : hi);
        const int a = d_count ? (int)lo : 0;
        const int b = d_count && !last ? (int)hi : INT32_MAX;
        int rc = CGGI_OK;
        if constexpr (N <= 1024) {
            switch (kind[k]) {
            case 0:
                rc = launch_split<N, L, S, 4>(c, in, testv, out, Bk, d_count,
                                              a, b, s);
                break;
            case 1:
                rc = launch_split<N, L, S, 2>(c, in, testv, out, Bk, d_count,
                                              a, b, s);
                break;
            case 5:
                rc = launch_split<N, L, S, 8>(c, in, testv, out, Bk, d_count,
                                              a, b, s);
                break;
            case 2:
                rc = launch_bs_int8_t<N, L, S, 1>(c, in, testv, out, Bk,
                                                  d_count, a, b, s);
                break;
            case 3:
                rc = launch_bs_int8_t<N, L, S, 2>(c, in, testv, out, Bk,
                                                  d_count, a, b, s);
                break;
            case 6:
                rc = kara_launch(c, in, testv, out, Bk, d_count, a, b, s);
                break;
            default:
                rc = launch_bs_int8_t<N, L, S, 4>(c, in, testv, out, Bk,
                                                  d_count, a, b, s);
            }
        } else {
            rc = launch_bs_int8_t<N, L, S, 4>(c, in, testv, out, Bk, d_count,
                                              a, b, s);
        }
        if (rc || last)
            return rc;
        lo = hi;
    }
    return CGGI_OK;
}

template <int N>
static int launch_bs_int8(const Ctx *c, const uint32_t *in,
                          const uint32_t *testv, uint32_t *out, int B,
                          const int32_t *d_count, hipStream_t s)
{
    const Shape &sh = c->sh;
    // specialised digit loops for the parameter sets in use, generic else
    if (sh.l == 3 && sh.S == 1)
        return launch_bs_int8_w<N, 3, 1>(c, in, testv, out, B, d_count, s);
    if (sh.l == 2 && sh.S == 2)
        return launch_bs_int8_w<N, 2, 2>(c, in, testv, out, B, d_count, s);
    return launch_bs_int8_w<N, 0, 0>(c, in, testv, out, B, d_count, s);
}

int int8_bootstrap(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                   uint32_t *out, int B, const int32_t *d_count,
                   hipStream_t s)
{
    switch (c->sh.N) {
    case 256: return launch_bs_int8<256>(c, in, testv, out, B, d_count, s);
    case 512: return launch_bs_int8<512>(c, in, testv, out, B, d_count, s);
    case 1024: return launch_bs_int8<1024>(c, in, testv, out, B, d_count, s);
    case 2048: return launch_bs_int8<2048>(c, in, testv, out, B, d_count, s);
    default: return set_error(CGGI_E_PARAM, "INT8 form: unsupported N");
    }
}

} // namespace cggi
