// ntt_form.hip -- the NTT form of the blind rotation on gfx950.
//
// Every negacyclic product of a CMux step (ArctyrEX Fig. 1: forward
// transforms of the decomposed digit polynomials, pointwise product with
// the transformed TRGSW row, inverse transforms, add into the accumulator)
// is computed exactly modulo Q = 2^64 - 2^32 + 1 with psi = g^(2^32 / 2N)
// for the paper's generator g (Section 5.4).  Since every exact sum is
// below Q/2 in magnitude (checked on the host), the centred lift of the
// result equals the integer product, and its low 32 bits are the product
// mod 2^32.
//
// Layout: one workgroup (256 or 512 threads by N) owns one bootstrap.
// LDS holds the accumulator (2 x N u32), the 2l digit transforms (2l x N
// u64) and the two product transforms (2 x N u64), which at N = 2048
// overwrite the first two digit transforms (80 KB at l = 2: two workgroups
// per CU).  The transformed key row of step i
// ([2l][2][N] u64) streams from L2 / Infinity Cache; it is shared by every
// workgroup.
#include "goldilocks.hpp"
#include "internal.hpp"

#include <vector>

namespace cggi {

namespace {

constexpr int NTT_THREADS = 256;   // table kernels

// Threads of a bootstrap workgroup.  The butterflies are VALU-bound with an
// LDS round trip every three stages, so more waves per SIMD hide more of
// the LDS latency and barrier skew: four per SIMD, from two workgroups of 8
// waves per CU at N = 1024 (1.1x faster than 4 waves each) and at N = 2048
// (its 80 KB of LDS leaves room for two; with the product transforms in
// their own LDS, 113 KB, one workgroup of 16 waves per CU took 76.4 ms per
// 1024 large bootstraps).  Every loop below strides by the thread count, so
// any count is exact.
constexpr int bs_threads(int N) { return N >= 1024 ? 512 : 256; }
// whether the product transforms overwrite the first two digit transforms
constexpr bool ntt_products_alias(int N) { return N >= 2048; }
constexpr uint64_t G_PAPER = 12037493425763644479ull; // order 2^32 mod Q

unsigned bitrev(unsigned x, int bits)
{
    unsigned r = 0;
    for (int i = 0; i < bits; ++i)
        r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

// In-place negacyclic forward NTT of P polynomials of length N in LDS
// (Cooley-Tukey with the psi-twisted twiddles tw[m + i] = psi^bitrev(m + i),
// output in bit-reversed order).  Stages are taken NS = 3 at a time: a thread
// loads the 2^NS elements one radix-2^NS block touches, runs the NS stages
// in registers and stores them back, so each LDS round trip (and barrier)
// covers three stages.
// NS Cooley-Tukey stages on the 2^NS elements of one block held in
// registers: the block starts in group i of stage s0 (m0 = 2^s0 groups).
// U0 > 0 starts at that stage (the earlier ones done by the caller).
template <int NS, int U0 = 0>
__device__ __forceinline__ void fwd_block(uint64_t (&v)[1 << NS], int m0, int i,
                                          const uint64_t *__restrict__ tw)
{
    constexpr int K = 1 << NS;
#pragma unroll
    for (int u = U0; u < NS; ++u) {
        const int d = 1 << (NS - 1 - u);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k & d)
                continue;
            const uint64_t S = tw[(m0 << u) + (i << u) + (k >> (NS - u))];
            // V is a canonical product, so U may stay unreduced
            const uint64_t U = v[k], V = gl::mul(v[k + d], S);
            v[k] = gl::add_lazy(U, V);
            v[k + d] = gl::sub(U, V);
        }
    }
}

template <int N, int NS, int TH = NTT_THREADS>
__device__ __forceinline__ void fwd_pass(uint64_t *a, int P, int s0,
                                         const uint64_t *__restrict__ tw)
{
    constexpr int K = 1 << NS;
    const int m0 = 1 << s0;                 // groups at the first stage
    const int t0 = N >> (s0 + 1);           // half-span at the first stage
    const int stride = (2 * t0) >> NS;      // distance between block elements
    const int per_poly = N / K;
    for (int idx = threadIdx.x; idx < P * per_poly; idx += TH) {
        const int poly = idx / per_poly, r = idx - poly * per_poly;
        const int i = r / stride, off = r - i * stride;
        uint64_t *x = a + poly * N + 2 * t0 * i + off;
        uint64_t v[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            v[k] = x[k * stride];
        fwd_block<NS>(v, m0, i, tw);
#pragma unroll
        for (int k = 0; k < K; ++k)
            x[k * stride] = v[k];
    }
    __syncthreads();
}

template <int N>
__device__ __forceinline__ void ntt_fwd(uint64_t *a, int P,
                                        const uint64_t *__restrict__ tw)
{
    constexpr int LOGN = __builtin_ctz(N);
    int s = 0;
    for (; s + 3 <= LOGN; s += 3)
        fwd_pass<N, 3>(a, P, s, tw);
    if (LOGN - s == 2)
        fwd_pass<N, 2>(a, P, s, tw);
    else if (LOGN - s == 1)
        fwd_pass<N, 1>(a, P, s, tw);
}

// Forward stages 3 .. log2 N - 2 of P polynomials (stages 0..2 are fused
// with the decomposition, the last one with the pointwise product).
template <int N, int TH>
__device__ __forceinline__ void ntt_fwd_middle(uint64_t *a, int P,
                                               const uint64_t *__restrict__ tw)
{
    constexpr int LOGN = __builtin_ctz(N);
    constexpr int END = LOGN - 1;
    int s = 3;
    for (; s + 3 <= END; s += 3)
        fwd_pass<N, 3, TH>(a, P, s, tw);
    if (END - s == 2)
        fwd_pass<N, 2, TH>(a, P, s, tw);
    else if (END - s == 1)
        fwd_pass<N, 1, TH>(a, P, s, tw);
}

// NS inverse (Gentleman-Sande) stages from stage u0 on the two product
// polynomials (bit-reversed input, natural output, twiddles
// twi[h + i] = psi^-bitrev(h + i)), in place, or, for the last pass, added
// into the torus accumulator as the centred lift (the 1/N scaling is folded
// into the transformed key).
template <int N, int NS, bool TO_ACC, int TH>
__device__ __forceinline__ void inv_pass(uint64_t *a, int u0,
                                         const uint64_t *__restrict__ twi,
                                         uint32_t *acc)
{
    constexpr int K = 1 << NS;
    const int t0 = 1 << u0;                 // half-span at the first stage
    const int span = t0 * K;                // block of the pass
    constexpr int per_poly = N / K;
    for (int idx = threadIdx.x; idx < 2 * per_poly; idx += TH) {
        const int poly = idx / per_poly, r = idx - poly * per_poly;
        const int blk = r / t0, off = r - blk * t0;
        const int base = poly * N + blk * span + off;
        uint64_t v[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            v[k] = a[base + k * t0];
#pragma unroll
        for (int w = 0; w < NS; ++w) {
            const int d = 1 << w;
            const int h = N >> (u0 + w + 1);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k & d)
                    continue;
                const uint64_t S = twi[h + (blk << (NS - w - 1)) + (k >> (w + 1))];
                const uint64_t U = v[k], V = v[k + d];
                v[k] = gl::add(U, V);
                v[k + d] = gl::mul(gl::sub(U, V), S);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (TO_ACC)
                acc[base + k * t0] += gl::lift32(v[k]);
            else
                a[base + k * t0] = v[k];
        }
    }
    __syncthreads();
}

// Inverse stages 1 .. log2 N - 1 (stage 0 is fused with the pointwise
// product); the last pass adds the result into the accumulator.
template <int N, int TH>
__device__ __forceinline__ void ntt_inv_to_acc(uint64_t *a,
                                               const uint64_t *__restrict__ twi,
                                               uint32_t *acc)
{
    constexpr int LOGN = __builtin_ctz(N);
    constexpr int NSTG = LOGN - 1;          // stages 1 .. LOGN - 1
    // radix-4 passes when the two polynomials have fewer radix-8 blocks than
    // the workgroup has threads (one more LDS round trip, no idle threads:
    // 1-2% faster at N = 1024 and 2048)
    constexpr int NSI = 2 * (N / 8) < TH ? 2 : 3;
    constexpr int REM = NSTG % NSI;
    constexpr int FULL = NSTG / NSI;
    int u = 1;
    for (int f = 0; f < FULL; ++f, u += NSI) {
        if (REM == 0 && f == FULL - 1)
            inv_pass<N, NSI, true, TH>(a, u, twi, acc);
        else
            inv_pass<N, NSI, false, TH>(a, u, twi, acc);
    }
    if (REM == 2)
        inv_pass<N, 2, true, TH>(a, u, twi, acc);
    else if (REM == 1)
        inv_pass<N, 1, true, TH>(a, u, twi, acc);
}

// bsk -> NTT form, times 1/N (the inverse transform then needs no scaling)
template <int N>
__global__ __launch_bounds__(NTT_THREADS) void k_bsk_to_ntt(
    const uint32_t *__restrict__ bsk, uint64_t *__restrict__ out,
    const uint64_t *__restrict__ tw, uint64_t ninv, int npoly)
{
    __shared__ uint64_t a[N];
    int poly = blockIdx.x;
    if (poly >= npoly)
        return;
    for (int j = threadIdx.x; j < N; j += NTT_THREADS)
        a[j] = bsk[(size_t)poly * N + j];   // torus value as a residue
    __syncthreads();
    ntt_fwd<N>(a, 1, tw);
    for (int j = threadIdx.x; j < N; j += NTT_THREADS)
        out[(size_t)poly * N + j] = gl::mul(a[j], ninv);
}

__device__ __forceinline__ uint32_t modswitch(uint32_t u, int log2_2n)
{
    return (u + (1u << (31 - log2_2n))) >> (32 - log2_2n);
}

// One bootstrap per workgroup.
// at most 128 VGPRs: four waves per SIMD
template <int N, int TH = bs_threads(N)>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(4)))
void k_bootstrap_ntt(
    const uint64_t *__restrict__ bsk_ntt, const uint64_t *__restrict__ tw,
    const uint64_t *__restrict__ twi,
    const uint32_t *__restrict__ in, const uint32_t *__restrict__ testv,
    uint32_t *__restrict__ out, int B, const int32_t *__restrict__ d_count,
    int n, int beta, int l)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int L2 = 2 * l;
    uint64_t *dig = reinterpret_cast<uint64_t *>(smem);          // [2l][N]
    // product transforms [2][N]: at N = 2048 they overwrite digit
    // transforms 0 and 1 (the pointwise pass reads positions 2j, 2j + 1 of
    // every digit row before it writes the same two positions of the
    // products, in the same thread, and no other thread touches them), so
    // that two workgroups fit a CU; below, they have their own LDS (the
    // overlap measured 0.2% slower at N = 1024, where it gains no workgroup)
    uint64_t *res = ntt_products_alias(N) ? dig : dig + (size_t)L2 * N;
    uint32_t *acc = reinterpret_cast<uint32_t *>(
        dig + (size_t)(L2 + (ntt_products_alias(N) ? 0 : 2)) * N); // [2][N]

    int count = B;
    if (d_count)
        count = min(count, *d_count);
    const int g = blockIdx.x;
    if (g >= count)
        return;
    constexpr int LOG2_2N = __builtin_ctz(2 * N);
    // the input ciphertext
    const uint32_t *ct = in + (size_t)g * (n + 1);

    // ACC = (0, X^(2N - b~) * v)
    {
        int e = (2 * N - (int)modswitch(ct[n], LOG2_2N)) & (2 * N - 1);
        for (int m = threadIdx.x; m < N; m += TH) {
            uint32_t v = testv ? testv[m] : (1u << 29);
            int t = m + e;
            if (t >= 2 * N) {
                t -= 2 * N;
            } else if (t >= N) {
                t -= N;
                v = 0u - v;
            }
            acc[t] = 0u;
            acc[N + t] = v;
        }
    }
    __syncthreads();

    const uint32_t round_off = (beta * l < 32) ? (1u << (31 - beta * l)) : 0u;
    uint32_t dig_off = round_off;
    for (int p = 1; p <= l; ++p)
        dig_off += (1u << (beta - 1)) << (32 - p * beta);
    const uint32_t bmask = (1u << beta) - 1u;
    const int32_t bhalf = 1 << (beta - 1);
    // psi^(N/2) is a primitive 4th root of unity: 2^48 or Q - 2^48 (checked
    // when the tables are made)
    const bool w4_neg = tw[1] != (uint64_t(1) << 48);
    const bool small_digits = beta <= 14;

    // each step's rotation is read a step ahead with a vector load (an
    // opaque zero offset keeps it off the scalar unit, whose outstanding
    // loads every LDS wait would also wait for) and made uniform at use
    int z = 0;
    asm volatile("" : "+v"(z));
    uint32_t e_nxt = ct[z];
    for (int i = 0; i < n; ++i) {
        const int e = (int)modswitch(__builtin_amdgcn_readfirstlane(e_nxt),
                                     LOG2_2N);
        e_nxt = ct[i + 1 + z];     // i + 1 <= n: in the ciphertext
        if (e == 0)      // X^0 * ACC - ACC = 0 decomposes to all-zero digits
            continue;
        // (1) rotate, subtract, decompose, and forward stages 0..2: a thread
        // takes the 8 coefficients m = off + k N/8 of one component, forms
        // X^e ACC - ACC there, and runs each digit polynomial's radix-8
        // block in registers
        for (int idx = threadIdx.x; idx < 2 * (N / 8); idx += TH) {
            const int c = idx / (N / 8), off = idx - c * (N / 8);
            const uint32_t *ac = acc + c * N;
            uint32_t w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int m = off + k * (N / 8);
                const int t = (m - e) & (2 * N - 1);
                const uint32_t rot = t < N ? ac[t] : 0u - ac[t - N];
                w[k] = rot - ac[m] + dig_off;
            }
            for (int p = 1; p <= l; ++p) {
                uint64_t v[8];
                int32_t dg[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    dg[k] = (int32_t)((w[k] >> (32 - p * beta)) & bmask) -
                            bhalf;
                if (small_digits) {
                    // stage 0 in signed integers: its twiddle psi^(N/2) is
                    // +-2^48 and |digit| <= 2^13, so U +- 2^48 V stays
                    // below 2^62 and needs no reduction
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        int64_t V = (int64_t)dg[k + 4] * (int64_t(1) << 48);
                        V = w4_neg ? -V : V;
                        const int64_t a0 = (int64_t)dg[k] + V;
                        const int64_t a1 = (int64_t)dg[k] - V;
                        v[k] = a0 >= 0 ? (uint64_t)a0 : (uint64_t)a0 + gl::Q;
                        v[k + 4] = a1 >= 0 ? (uint64_t)a1
                                           : (uint64_t)a1 + gl::Q;
                    }
                    fwd_block<3, 1>(v, 1, 0, tw);
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        v[k] = gl::from_i32(dg[k]);
                    fwd_block<3>(v, 1, 0, tw);
                }
                uint64_t *x = dig + (size_t)(c * l + p - 1) * N + off;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    x[k * (N / 8)] = v[k];
            }
        }
        __syncthreads();
        // (2) forward stages 3 .. log2 N - 2
        ntt_fwd_middle<N, TH>(dig, L2, tw);
        // (3) last forward stage (pairs 2j, 2j+1), pointwise product with
        // the key row summed over the 2l digit polynomials (the 128-bit
        // products summed exactly and reduced once per sum: 6% faster than
        // a reduction per product), and the first inverse stage (the same
        // pairs)
        const uint64_t *row = bsk_ntt + (size_t)i * L2 * 2 * N;
        for (int j = threadIdx.x; j < N / 2; j += TH) {
            const uint64_t S = tw[N / 2 + j];
            gl::MacAcc m0[2] = {{0, 0, 0}, {0, 0, 0}};
            gl::MacAcc m1[2] = {{0, 0, 0}, {0, 0, 0}};
            for (int r = 0; r < L2; ++r) {
                const uint64_t U = dig[(size_t)r * N + 2 * j];
                const uint64_t V = gl::mul(dig[(size_t)r * N + 2 * j + 1], S);
                const uint64_t x0 = gl::add_lazy(U, V), x1 = gl::sub(U, V);
#pragma unroll
                for (int cp = 0; cp < 2; ++cp) {
                    const ulonglong2 kk = *reinterpret_cast<const ulonglong2 *>(
                        row + ((size_t)r * 2 + cp) * N + 2 * j);
                    gl::mac(m0[cp], x0, kk.x);
                    gl::mac(m1[cp], x1, kk.y);
                }
            }
            const uint64_t Si = twi[N / 2 + j];
            uint64_t s0[2], s1[2];
#pragma unroll
            for (int cp = 0; cp < 2; ++cp) {
                s0[cp] = gl::mac_reduce(m0[cp]);
                s1[cp] = gl::mac_reduce(m1[cp]);
            }
#pragma unroll
            for (int cp = 0; cp < 2; ++cp) {
                res[cp * N + 2 * j] = gl::add(s0[cp], s1[cp]);
                res[cp * N + 2 * j + 1] = gl::mul(gl::sub(s0[cp], s1[cp]), Si);
            }
        }
        __syncthreads();
        // (4) inverse stages 1 .. log2 N - 1, the last pass adding into ACC
        ntt_inv_to_acc<N, TH>(res, twi, acc);
    }

    // sample extraction of coefficient 0
    uint32_t *o = out + (size_t)g * (N + 1);
    for (int j = threadIdx.x; j <= N; j += TH) {
        uint32_t v;
        if (j == 0)
            v = acc[0];
        else if (j < N)
            v = 0u - acc[N - j];
        else
            v = acc[N];
        o[j] = v;
    }
}

template <int N>
size_t ntt_smem(int n, int l)
{
    (void)n;
    return (size_t)(2 * l + (ntt_products_alias(N) ? 0 : 2)) * N * 8 +
           2 * N * 4;
}

} // namespace

int ntt_make_tables(Ctx *c, hipStream_t s)
{
    const int N = c->sh.N, logN = c->sh.log2N;
    uint64_t psi = gl::pow_host(G_PAPER, (1ull << 32) / (2ull * N));
    uint64_t psi_inv = gl::pow_host(psi, 2ull * N - 1);
    std::vector<uint64_t> f(N), iv(N);
    for (int i = 0; i < N; ++i) {
        unsigned r = bitrev((unsigned)i, logN);
        f[i] = gl::pow_host(psi, r);
        iv[i] = gl::pow_host(psi_inv, r);
    }
    // the bootstrap kernel does the first forward stage as a shift by 48
    if (f[1] != (1ull << 48) && f[1] != gl::Q - (1ull << 48))
        return set_error(CGGI_E_PARAM, "NTT form: psi^(N/2) is not +-2^48");
    CGGI_HIP_TRY(hipMalloc(&c->tw_fwd, N * sizeof(uint64_t)));
    CGGI_HIP_TRY(hipMalloc(&c->tw_inv, N * sizeof(uint64_t)));
    CGGI_HIP_TRY(hipMemcpyAsync(c->tw_fwd, f.data(), N * sizeof(uint64_t),
                                hipMemcpyHostToDevice, s));
    CGGI_HIP_TRY(hipMemcpyAsync(c->tw_inv, iv.data(), N * sizeof(uint64_t),
                                hipMemcpyHostToDevice, s));
    CGGI_HIP_TRY(hipStreamSynchronize(s));
    return CGGI_OK;
}

int ntt_transform_bsk(Ctx *c, const uint32_t *bsk, hipStream_t s)
{
    const Shape &sh = c->sh;
    int npoly = sh.n * 2 * sh.l * 2;
    size_t bytes = (size_t)npoly * sh.N * sizeof(uint64_t);
    if (hipMalloc(&c->bsk_ntt, bytes) != hipSuccess) {
        c->bsk_ntt = nullptr;
        return set_error(CGGI_E_NOMEM, "hipMalloc of the NTT key failed");
    }
    const uint64_t ninv = gl::pow_host((uint64_t)sh.N, gl::Q - 2);
    switch (sh.N) {
    case 256:
        hipLaunchKernelGGL(k_bsk_to_ntt<256>, dim3(npoly), dim3(NTT_THREADS),
                           0, s, bsk, c->bsk_ntt, c->tw_fwd, ninv, npoly);
        break;
    case 512:
        hipLaunchKernelGGL(k_bsk_to_ntt<512>, dim3(npoly), dim3(NTT_THREADS),
                           0, s, bsk, c->bsk_ntt, c->tw_fwd, ninv, npoly);
        break;
    case 1024:
        hipLaunchKernelGGL(k_bsk_to_ntt<1024>, dim3(npoly), dim3(NTT_THREADS),
                           0, s, bsk, c->bsk_ntt, c->tw_fwd, ninv, npoly);
        break;
    case 2048:
        hipLaunchKernelGGL(k_bsk_to_ntt<2048>, dim3(npoly), dim3(NTT_THREADS),
                           0, s, bsk, c->bsk_ntt, c->tw_fwd, ninv, npoly);
        break;
    default:
        return set_error(CGGI_E_PARAM, "NTT form: unsupported N");
    }
    CGGI_HIP_TRY(hipGetLastError());
    // the bootstrap kernel's dynamic-LDS limit, set when a context is made
    // (on its device) so that launches, also under graph capture, need
    // nothing
    const void *fn = nullptr;
    switch (sh.N) {
    case 256: fn = reinterpret_cast<const void *>(&k_bootstrap_ntt<256>); break;
    case 512: fn = reinterpret_cast<const void *>(&k_bootstrap_ntt<512>); break;
    case 1024: fn = reinterpret_cast<const void *>(&k_bootstrap_ntt<1024>); break;
    default: fn = reinterpret_cast<const void *>(&k_bootstrap_ntt<2048>); break;
    }
    CGGI_HIP_TRY(hipFuncSetAttribute(
        fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    return CGGI_OK;
}

template <int N>
static int launch_bs_ntt(const Ctx *c, const uint32_t *in,
                         const uint32_t *testv, uint32_t *out, int B,
                         const int32_t *d_count, hipStream_t s)
{
    const Shape &sh = c->sh;
    size_t smem = ntt_smem<N>(sh.n, sh.l);
    hipLaunchKernelGGL(k_bootstrap_ntt<N>, dim3(B), dim3(bs_threads(N)), smem,
                       s, c->bsk_ntt, c->tw_fwd, c->tw_inv, in, testv,
                       out, B, d_count, sh.n, sh.beta, sh.l);
    CGGI_HIP_TRY(hipGetLastError());
    return CGGI_OK;
}

int ntt_bootstrap(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                  uint32_t *out, int B, const int32_t *d_count, hipStream_t s)
{
    switch (c->sh.N) {
    case 256: return launch_bs_ntt<256>(c, in, testv, out, B, d_count, s);
    case 512: return launch_bs_ntt<512>(c, in, testv, out, B, d_count, s);
    case 1024: return launch_bs_ntt<1024>(c, in, testv, out, B, d_count, s);
    case 2048: return launch_bs_ntt<2048>(c, in, testv, out, B, d_count, s);
    default: return set_error(CGGI_E_PARAM, "NTT form: unsupported N");
    }
}

size_t ntt_smem_bytes(int N, int n, int l)
{
    (void)n;
    return (size_t)(2 * l + (ntt_products_alias(N) ? 0 : 2)) * N * 8 +
           2 * N * 4;
}

} // namespace cggi
