// diag.hip -- a measured ceiling for the int8 MFMA roofline.
//
// The int8 blind rotation is bound by v_mfma_i32_32x32x32_i8.  The published
// dense int8 rate assumes the top engine clock; with random operands the GPU
// lowers its clock to stay within its power limit, so this routine times a
// bare loop of that MFMA on the same launch shape the int8 form uses (one
// workgroup of 8 waves per CU, 8 independent accumulators per wave) and
// reports the rate, with random or all-zero operands.
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

} // namespace
} // namespace cggi

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
