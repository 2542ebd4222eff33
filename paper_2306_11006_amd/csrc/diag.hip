// diag.hip -- measured ceilings for the rooflines of the two forms.
//
// The int8 blind rotation is bound by v_mfma_i32_32x32x32_i8.  The published
// dense int8 rate assumes the top engine clock; with random operands the GPU
// lowers its clock to stay within its power limit, so this routine times a
// bare loop of that MFMA on the same launch shape the int8 form uses (one
// workgroup of 8 waves per CU, 8 independent accumulators per wave) and
// reports the rate, with random or all-zero operands.
//
// The NTT form is bound by integer VALU work, most of it the Goldilocks
// multiply-mod (a 64 x 64 -> 128-bit product from four 32 x 32 + 64
// multiply-adds and the reduction modulo Q).  A second routine times a bare
// loop of that same multiply-mod (gl::mul, the routine the NTT kernel
// calls) on independent chains, on the NTT form's launch shape (two
// workgroups of 512 threads per CU), which bounds the multiply-mods per
// second the NTT form could reach if it did nothing else.
#include "goldilocks.hpp"
#include "internal.hpp"

#include <vector>

namespace cggi {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int DIAG_THREADS = 512;
constexpr int DIAG_TABLE = 4096;        // v4i operand entries (64 KB)

__global__ __launch_bounds__(DIAG_THREADS, 1) void k_mfma_loop(
    const v4i *__restrict__ ops, int iters, int *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    v4i a[4], b[4];
    for (int j = 0; j < 4; ++j) {
        a[j] = ops[(j * 64 + lane) & (DIAG_TABLE - 1)];
        b[j] = ops[((j + 4) * 64 + lane) & (DIAG_TABLE - 1)];
    }
    v16i c[8];
    for (int j = 0; j < 8; ++j)
        c[j] = v16i{};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            c[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                a[j & 3], b[(j + (it & 1)) & 3], c[j], 0, 0, 0);
    }
    int s = 0;
    for (int j = 0; j < 8; ++j)
        s += c[j][0] ^ c[j][15];
    out[blockIdx.x * DIAG_THREADS + threadIdx.x] = s;
}

constexpr int MM_THREADS = 512;
constexpr int MM_CHAINS = 8;             // independent chains per thread

__global__ __launch_bounds__(MM_THREADS) void k_mulmod_loop(
    const uint64_t *__restrict__ seeds, int iters, uint64_t *__restrict__ out)
{
    const int t = threadIdx.x;
    uint64_t x[MM_CHAINS], y[MM_CHAINS];
#pragma unroll
    for (int j = 0; j < MM_CHAINS; ++j) {
        x[j] = seeds[(t * MM_CHAINS + j) & (DIAG_TABLE - 1)] % gl::Q;
        y[j] = seeds[(t * MM_CHAINS + j + 7) & (DIAG_TABLE - 1)] % gl::Q;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < MM_CHAINS; ++j)
            x[j] = gl::mul(x[j], y[j]);
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < MM_CHAINS; ++j)
        s ^= x[j];
    out[(size_t)blockIdx.x * MM_THREADS + t] = s;
}

} // namespace
} // namespace cggi

extern "C" int cggi_measure_mulmod(int32_t iters, double *tmulmods)
{
    using namespace cggi;
    if (iters < 1 || !tmulmods)
        return set_error(CGGI_E_PARAM,
                         "iters must be >= 1 and tmulmods non-NULL");
    int dev = 0, cus = 0;
    CGGI_HIP_TRY(hipGetDevice(&dev));
    CGGI_HIP_TRY(hipDeviceGetAttribute(
        &cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = 2 * cus;
    std::vector<uint64_t> h(DIAG_TABLE);
    uint64_t x = 0x2306ull;
    for (auto &v : h) {
        x = x * 6364136223846793005ull + 1442695040888963407ull; // MMIX LCG
        v = x;
    }
    void *seeds = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CGGI_OK;
    float ms = 0.f;
    auto fail = [&](hipError_t e) {
        if (rc == CGGI_OK && e != hipSuccess)
            rc = set_error(CGGI_E_HIP, hipGetErrorString(e));
    };
    fail(hipMalloc(&seeds, h.size() * sizeof(uint64_t)));
    if (rc == CGGI_OK)
        fail(hipMalloc(&out, (size_t)blocks * MM_THREADS * sizeof(uint64_t)));
    if (rc == CGGI_OK)
        fail(hipMemcpy(seeds, h.data(), h.size() * sizeof(uint64_t),
                       hipMemcpyHostToDevice));
    if (rc == CGGI_OK)
        fail(hipEventCreate(&e0));
    if (rc == CGGI_OK)
        fail(hipEventCreate(&e1));
    if (rc == CGGI_OK) {
        hipLaunchKernelGGL(k_mulmod_loop, dim3(blocks), dim3(MM_THREADS), 0,
                           0, static_cast<const uint64_t *>(seeds), 64,
                           static_cast<uint64_t *>(out));
        fail(hipGetLastError());
    }
    if (rc == CGGI_OK)
        fail(hipEventRecord(e0, 0));
    if (rc == CGGI_OK) {
        hipLaunchKernelGGL(k_mulmod_loop, dim3(blocks), dim3(MM_THREADS), 0,
                           0, static_cast<const uint64_t *>(seeds), iters,
                           static_cast<uint64_t *>(out));
        fail(hipGetLastError());
    }
    if (rc == CGGI_OK)
        fail(hipEventRecord(e1, 0));
    if (rc == CGGI_OK)
        fail(hipEventSynchronize(e1));
    if (rc == CGGI_OK)
        fail(hipEventElapsedTime(&ms, e0, e1));
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(seeds);
    (void)hipFree(out);
    if (rc != CGGI_OK)
        return rc;
    const double total = (double)blocks * MM_THREADS * MM_CHAINS * iters;
    *tmulmods = total / (ms * 1e-3) / 1e12;
    return CGGI_OK;
}

extern "C" int cggi_measure_int8_mfma(int32_t iters, int32_t random_operands,
                                      double *tops)
{
    using namespace cggi;
    if (iters < 1 || !tops)
        return set_error(CGGI_E_PARAM, "iters must be >= 1 and tops non-NULL");
    int dev = 0, cus = 0;
    CGGI_HIP_TRY(hipGetDevice(&dev));
    CGGI_HIP_TRY(hipDeviceGetAttribute(
        &cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<uint32_t> h((size_t)DIAG_TABLE * 4, 0u);
    if (random_operands) {
        uint32_t x = 0x2306u;
        for (auto &v : h) {
            x = x * 1664525u + 1013904223u;     // LCG (Numerical Recipes)
            v = x;
        }
    }
    void *ops = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CGGI_OK;
    float ms = 0.f;
    auto fail = [&](hipError_t e) {
        if (rc == CGGI_OK && e != hipSuccess)
            rc = set_error(CGGI_E_HIP, hipGetErrorString(e));
    };
    fail(hipMalloc(&ops, h.size() * sizeof(uint32_t)));
    if (rc == CGGI_OK)
        fail(hipMalloc(&out, (size_t)cus * DIAG_THREADS * sizeof(int)));
    if (rc == CGGI_OK)
        fail(hipMemcpy(ops, h.data(), h.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice));
    if (rc == CGGI_OK)
        fail(hipEventCreate(&e0));
    if (rc == CGGI_OK)
        fail(hipEventCreate(&e1));
    if (rc == CGGI_OK) {
        // warm-up launch, then the timed one
        hipLaunchKernelGGL(k_mfma_loop, dim3(cus), dim3(DIAG_THREADS), 0, 0,
                           static_cast<const v4i *>(ops), 64,
                           static_cast<int *>(out));
        fail(hipGetLastError());
    }
    if (rc == CGGI_OK)
        fail(hipEventRecord(e0, 0));
    if (rc == CGGI_OK) {
        hipLaunchKernelGGL(k_mfma_loop, dim3(cus), dim3(DIAG_THREADS), 0, 0,
                           static_cast<const v4i *>(ops), iters,
                           static_cast<int *>(out));
        fail(hipGetLastError());
    }
    if (rc == CGGI_OK)
        fail(hipEventRecord(e1, 0));
    if (rc == CGGI_OK)
        fail(hipEventSynchronize(e1));
    if (rc == CGGI_OK)
        fail(hipEventElapsedTime(&ms, e0, e1));
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(ops);
    (void)hipFree(out);
    if (rc != CGGI_OK)
        return rc;
    // 8 MFMAs x 32*32*32 multiply-adds x 2 ops per wave and iteration
    const double total = (double)cus * (DIAG_THREADS / 64) * 8.0 * iters *
                         (32.0 * 32 * 32 * 2);
    *tops = total / (ms * 1e-3) / 1e12;
    return CGGI_OK;
}
