// internal.hpp -- shared host-side declarations of libcggi (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cggi.h"

namespace cggi {

// Derived parameter values used by the launchers.
struct Shape {
    int n, N, beta, l, gamma, t;
    int log2N;
    int R;        // digit polynomials per CMux step in the INT8 form: 2l*S
    int S;        // 7-bit sub-digits per gadget digit (INT8 form)
    int nblk;     // N / 32 blocks of the block-Toeplitz product
    int elen;     // bytes per limb window of the INT8 key form
};

} // namespace cggi

// The context behind the opaque handle of cggi.h.
struct cggi_ctx {
    cggi_params_t p;
    cggi::Shape sh;
    int device;
    int cus = 256;                // compute units of the device
    uint32_t forms;
    const uint32_t *ksk;          // caller-owned [N][t][2^gamma][n+1]
    // NTT form
    uint64_t *bsk_ntt = nullptr;  // [n][2l][2][N] mod Q, bit-reversed order
    uint64_t *tw_fwd = nullptr;   // [N] psi^bitrev(i)
    uint64_t *tw_inv = nullptr;   // [N] psi^-bitrev(i)
    // INT8 form
    int8_t *bsk_i8 = nullptr;     // [n][R][2][4][elen] limb windows
    uint32_t *corr_i8 = nullptr;  // [n][2][N] digit-offset correction (N <= 1024)
    // Karatsuba kernel: half-length key windows [n][R][2][3][4][N/2+64]
    // (N <= 1024 and LDS permitting; null otherwise)
    int8_t *bsk_k8 = nullptr;
    uint32_t *corr_k8 = nullptr;  // [n][2][2][N/2] its digit-offset correction
    // INT8 latency mode (one tile over G = 8, 4 or 2 workgroups, N <= 1024);
    // index 0: G = 4, index 1: G = 2, index 2: G = 8
    bool split_on = true;         // cggi_ctx_latency_mode
    int split_groups[3] = {0, 0, 0}; // most tile groups per launch (0: none)
    unsigned long long *x_buf[3] = {}; // [groups][2][G][1024]
    size_t x_words[3] = {0, 0, 0};
    uint32_t *x_epoch[3] = {};    // [groups] launch epochs
    uint32_t *x_err = nullptr;    // [1] set when a member's wait timed out
    hipStream_t abort_stream = nullptr; // non-blocking, for latency_abort
    // INT8 kernel plan (cggi_ctx_int8_plan): entry k runs the batches of
    // (cap[k-1], cap[k]] bootstraps with kernel kind[k]; plan_n = 0 selects
    // the built-in plan.  kind_limit: most bootstraps one launch of each
    // kind may take (0: kind unavailable for this context).
    int plan_n = 0;
    int32_t plan_kind[8] = {};
    int32_t plan_cap[8] = {};
    int64_t kind_limit[7] = {0, 0, 0, 0, 0, 0, 0};
    // key switch as an int8 GEMM (bases up to 2^4)
    int8_t *ksk_i8 = nullptr;     // [NT][N][ksj][4][64][16] limb blocks
    int ks_ksj = 0;               // 32-slot K-steps per j
    int ks_wg_per_cu = 1;         // resident k_ks_mfma workgroups per CU
    // eval_level workspace
    int32_t ws_gates = 0;
    uint32_t *ws_small = nullptr; // [2G][n+1] bootstrap inputs
    uint32_t *ws_big = nullptr;   // [2G][N+1] bootstrap outputs
    int32_t *ws_slot = nullptr;   // [G] first slot of each gate (-1: none)
    int32_t *ws_count = nullptr;  // [1] number of bootstrap slots
    // this device's address of the fixed level workspace of
    // cggi_eval_level_noalloc (taken at context creation)
    unsigned char *scratch = nullptr;
    // kernel timing (cggi_ctx_profile)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks; // (kind, first event)
};

namespace cggi {

using Ctx = ::cggi_ctx;

// Error plumbing (thread-local message).
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);

#define CGGI_HIP_TRY(expr)                                                   \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            return ::cggi::hip_error(e_, #expr);                             \
    } while (0)

int shape_of(const cggi_params_t *p, Shape *sh);

// Kernel launchers (each returns CGGI_OK or an error code).
int ntt_make_tables(Ctx *c, hipStream_t s);
int ntt_transform_bsk(Ctx *c, const uint32_t *bsk, hipStream_t s);
int ntt_bootstrap(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                  uint32_t *out, int B, const int32_t *d_count,
                  hipStream_t s);

int int8_make_key(Ctx *c, const uint32_t *bsk, hipStream_t s);
int int8_bootstrap(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                   uint32_t *out, int B, const int32_t *d_count,
                   hipStream_t s);
// Karatsuba kernel (int8_kara.hip): key windows at context creation (a
// no-op where the kernel is unavailable), and a launch over B bootstraps
// (device count in (lo, hi] when d_count is given).
int kara_make_key(Ctx *c, const uint32_t *bsk, hipStream_t s);
int kara_launch(const Ctx *c, const uint32_t *in, const uint32_t *testv,
                uint32_t *out, int B, const int32_t *d_count, int lo, int hi,
                hipStream_t s);
// Re-zeroes the latency-mode exchange buffers, epochs and error word
// (synchronous).
int int8_split_reset(Ctx *c);
// The INT8 kernel plan in force (the caller's, or the built-in one), with
// latency-mode entries dropped while latency mode is off.  Returns the
// number of entries (at most 8).
int int8_active_plan(const Ctx *c, int32_t *kind, int32_t *cap);

// Key switch.  in_a/in_b: optional second input added before switching
// (MUX combine); the plain batch call passes null maps.
int keyswitch_make_key(Ctx *c, hipStream_t s);
int keyswitch_launch(const Ctx *c, const uint32_t *in, uint32_t *out, int B,
                     hipStream_t s);

// Brackets one kernel launch with profiling events when enabled and the
// stream is not capturing.  kind: 0 = bootstrap, 1 = key switch.  A null
// context records nothing.
class ProfScope {
  public:
    ProfScope(Ctx *c, int kind, hipStream_t s);
    ~ProfScope();

  private:
    Ctx *c_;
    hipStream_t s_;
    long idx_ = -1;
};

// Device buffers of one level: bootstrap inputs [2G][n+1], bootstrap
// outputs [2G][N+1], first slot of each gate [G], bootstrap count [1].
struct LevelWs {
    uint32_t *small;
    uint32_t *big;
    int32_t *slot;
    int32_t *count;
};

// Launch one level on `ws`; `prof` brackets its kernels with the
// context's profiling events (when profiling is enabled).
int level_launch(Ctx *c, cggi_form_t form, const cggi_gate_t *gates, int G,
                 uint32_t *wires, int W, const LevelWs &ws, bool prof,
                 hipStream_t s);

// Host-side checks shared by the level entry points (before any launch).
int level_args_check(Ctx *c, cggi_form_t form, const cggi_gate_t *gates,
                     int32_t G, uint32_t *wires, int32_t W);

} // namespace cggi
