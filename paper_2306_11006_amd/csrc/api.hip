// api.hip -- the C ABI of libcggi: validation, contexts, dispatch.
//
// Every shape and parameter error is detected here, on the host, before
// anything is launched.
#include "internal.hpp"

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

namespace cggi {

size_t ntt_smem_bytes(int N, int n, int l);
size_t int8_smem_bytes(int N, int R, int n);

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    g_last_error = m;
    return e == hipErrorOutOfMemory ? CGGI_E_NOMEM : CGGI_E_HIP;
}

constexpr size_t LDS_BYTES = 160 * 1024;

int shape_of(const cggi_params_t *p, Shape *sh)
{
    if (!p)
        return set_error(CGGI_E_PARAM, "params is NULL");
    if (p->k != 1)
        return set_error(CGGI_E_PARAM, "k must be 1");
    if (p->N != 256 && p->N != 512 && p->N != 1024 && p->N != 2048)
        return set_error(CGGI_E_PARAM, "N must be 256, 512, 1024 or 2048");
    if (p->n < 1 || p->n > 1023)
        return set_error(CGGI_E_PARAM, "n must be in [1, 1023]");
    if (p->bg_bit < 1 || p->l < 1 || p->bg_bit * p->l > 31)
        return set_error(CGGI_E_PARAM,
                         "need bg_bit >= 1, l >= 1 and bg_bit * l <= 31");
    if (p->ks_base_bit < 1 || p->ks_base_bit > 8 || p->ks_t < 1 ||
        p->ks_base_bit * p->ks_t > 31)
        return set_error(CGGI_E_PARAM, "need 1 <= ks_base_bit <= 8, "
                                        "ks_t >= 1 and ks_base_bit * ks_t <= 31");
    // Exactness of the NTT form: |sum of 2l*N products| < Q/2.
    long double bound = (long double)(2 * p->l) * p->N *
                        (long double)(1ull << (p->bg_bit - 1)) * 4294967295.0L;
    if (bound >= 9.2e18L)
        return set_error(CGGI_E_PARAM,
                         "2l * N * 2^(bg_bit-1) * 2^32 must stay below Q/2");
    Shape s{};
    s.n = p->n;
    s.N = p->N;
    s.beta = p->bg_bit;
    s.l = p->l;
    s.gamma = p->ks_base_bit;
    s.t = p->ks_t;
    s.log2N = __builtin_ctz((unsigned)p->N);
    s.S = p->bg_bit <= 7 ? 1 : (p->bg_bit <= 13 ? 2 : 0);
    s.R = 2 * p->l * s.S;
    s.nblk = p->N / 32;
    s.elen = p->N + 64;
    if (sh)
        *sh = s;
    return CGGI_OK;
}

static int check_form(const Shape &s, uint32_t form)
{
    if (form & CGGI_FORM_NTT) {
        if (ntt_smem_bytes(s.N, s.n, s.l) > LDS_BYTES)
            return set_error(CGGI_E_PARAM,
                             "NTT form: (2l+3)*N*8 + 2(n+1) bytes exceed LDS");
    }
    if (form & CGGI_FORM_INT8) {
        if (s.S == 0)
            return set_error(CGGI_E_PARAM, "INT8 form: bg_bit must be <= 13");
        // the generic build's digit loops run over at most 8 gadget levels
        if (s.l > 8)
            return set_error(CGGI_E_PARAM, "INT8 form: l must be <= 8");
        if (int8_smem_bytes(s.N, s.R, s.n) > LDS_BYTES)
            return set_error(CGGI_E_PARAM, "INT8 form: workgroup exceeds LDS");
    }
    return CGGI_OK;
}

static bool aligned4(const void *p)
{
    return ((uintptr_t)p & 3u) == 0;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

static int check_device(const Ctx *c)
{
    int dev = -1;
    CGGI_HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device)
        return set_error(CGGI_E_PARAM,
                         "current device differs from the context's device");
    return CGGI_OK;
}

static void free_ctx(Ctx *c)
{
    if (!c)
        return;
    (void)hipFree(c->bsk_ntt);
    (void)hipFree(c->tw_fwd);
    (void)hipFree(c->tw_inv);
    (void)hipFree(c->bsk_i8);
    (void)hipFree(c->corr_i8);
    (void)hipFree(c->bsk_k8);
    (void)hipFree(c->corr_k8);
    for (int v = 0; v < 3; ++v) {
        (void)hipFree(c->x_buf[v]);
        (void)hipFree(c->x_epoch[v]);
    }
    (void)hipFree(c->x_err);
    if (c->abort_stream)
        (void)hipStreamDestroy(c->abort_stream);
    (void)hipFree(c->ksk_i8);
    (void)hipFree(c->ws_small);
    (void)hipFree(c->ws_big);
    (void)hipFree(c->ws_slot);
    (void)hipFree(c->ws_count);
    for (hipEvent_t e : c->ev_pool)
        (void)hipEventDestroy(e);
    delete c;
}

static int reserve(Ctx *c, int32_t G, hipStream_t s)
{
    if (G <= c->ws_gates)
        return CGGI_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    CGGI_HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return set_error(CGGI_E_UNSUPPORTED,
                         "eval_level workspace too small under capture: call "
                         "cggi_ctx_reserve first");
    CGGI_HIP_TRY(hipDeviceSynchronize());
    (void)hipFree(c->ws_small);
    (void)hipFree(c->ws_big);
    (void)hipFree(c->ws_slot);
    (void)hipFree(c->ws_count);
    c->ws_small = c->ws_big = nullptr;
    c->ws_slot = c->ws_count = nullptr;
    c->ws_gates = 0;
    const size_t n1 = (size_t)c->sh.n + 1, N1 = (size_t)c->sh.N + 1;
    if (hipMalloc(&c->ws_small, 2 * (size_t)G * n1 * 4) != hipSuccess ||
        hipMalloc(&c->ws_big, 2 * (size_t)G * N1 * 4) != hipSuccess ||
        hipMalloc(&c->ws_slot, (size_t)G * 4) != hipSuccess ||
        hipMalloc(&c->ws_count, 16) != hipSuccess)
        return set_error(CGGI_E_NOMEM, "hipMalloc of the level workspace");
    c->ws_gates = G;
    return CGGI_OK;
}

ProfScope::ProfScope(Ctx *c, int kind, hipStream_t s) : c_(c), s_(s)
{
    if (!c_ || !c_->prof)
        return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return;
    while (c_->ev_pool.size() < c_->ev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return;
        c_->ev_pool.push_back(e);
    }
    idx_ = (long)c_->ev_used;
    c_->ev_used += 2;
    c_->ev_marks.push_back({kind, (size_t)idx_});
    (void)hipEventRecord(c_->ev_pool[idx_], s_);
}

ProfScope::~ProfScope()
{
    if (idx_ >= 0)
        (void)hipEventRecord(c_->ev_pool[idx_ + 1], s_);
}

// ---- fixed level workspace of cggi_eval_level_noalloc ---------------------
// A file-scope device array: every GPU the library runs on holds its own
// copy, at its own address, from the code object's load until the process
// ends.  On the host the name `scratch` is only a stand-in symbol, never a
// device address: host code uses the address hipGetSymbolAddress returns
// for the current device, taken once per device (at the first context
// created there) and kept in g_scratch_addr.
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_addr[SCRATCH_MAX_DEVICES];

// This device's address of `scratch` (the device must be current).
static int scratch_address(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return set_error(CGGI_E_PARAM, "device index beyond the scratch "
                                       "table (64 devices)");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return set_error(CGGI_E_HIP, "hipGetSymbolAddress(scratch) gave "
                                         "a null address");
        g_scratch_addr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_addr[dev];
    return CGGI_OK;
}

static size_t align256(size_t x)
{
    return (x + 255) & ~size_t(255);
}

// Carve a level's workspace out of `base` (count, slots, bootstrap inputs,
// bootstrap outputs, each 256-byte aligned); returns the bytes it needs.
static size_t scratch_layout(const Shape &sh, int64_t G, unsigned char *base,
                             LevelWs *ws)
{
    const size_t slot_off = 256;
    const size_t small_off = align256(slot_off + (size_t)G * 4);
    const size_t big_off = align256(small_off + 2 * (size_t)G * (sh.n + 1) * 4);
    const size_t total = big_off + 2 * (size_t)G * (sh.N + 1) * 4;
    if (ws && base) {
        ws->count = reinterpret_cast<int32_t *>(base);
        ws->slot = reinterpret_cast<int32_t *>(base + slot_off);
        ws->small = reinterpret_cast<uint32_t *>(base + small_off);
        ws->big = reinterpret_cast<uint32_t *>(base + big_off);
    }
    return total;
}

// Most gates of one level that fit the fixed workspace.
static int64_t scratch_max_gates(const Shape &sh)
{
    const size_t per = 4 + 2 * (size_t)(sh.n + 1) * 4 + 2 * (size_t)(sh.N + 1) * 4;
    int64_t g = (int64_t)(SCRATCH_BYTES / per);
    while (g > 0 && scratch_layout(sh, g, nullptr, nullptr) > SCRATCH_BYTES)
        --g;
    return g;
}

static void prof_clear(Ctx *c)
{
    c->ev_used = 0;
    c->ev_marks.clear();
}

int level_args_check(Ctx *c, cggi_form_t form, const cggi_gate_t *gates,
                     int32_t G, uint32_t *wires, int32_t W)
{
    if (!c)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    if (form != CGGI_FORM_NTT && form != CGGI_FORM_INT8)
        return set_error(CGGI_E_PARAM, "unknown form");
    if (!(c->forms & (uint32_t)form))
        return set_error(CGGI_E_UNSUPPORTED, "form not built into the context");
    if (G < 0 || G > (1 << 22) || W < 1 || W > (1 << 26))
        return set_error(CGGI_E_SHAPE, "need 0 <= G <= 2^22, 1 <= W <= 2^26");
    if (G == 0)
        return CGGI_OK;
    if (!gates || !wires || !aligned4(gates) || !aligned4(wires))
        return set_error(CGGI_E_SHAPE, "gates/wires must be non-NULL and "
                                       "4-byte aligned");
    if (overlap(gates, (size_t)G * sizeof(cggi_gate_t), wires,
                (size_t)W * (c->sh.n + 1) * 4))
        return set_error(CGGI_E_ALIAS, "gates overlap wires");
    return check_device(c);
}

} // namespace cggi

using namespace cggi;

extern "C" {

int cggi_params_check(const cggi_params_t *params)
{
    return shape_of(params, nullptr);
}

int cggi_ctx_create(const cggi_params_t *params, const uint32_t *d_bsk,
                    const uint32_t *d_ksk, uint32_t forms, void *stream,
                    cggi_ctx **out)
{
    if (!out)
        return set_error(CGGI_E_SHAPE, "out is NULL");
    *out = nullptr;
    Shape sh;
    int rc = shape_of(params, &sh);
    if (rc)
        return rc;
    if (forms == 0 || (forms & ~(uint32_t)(CGGI_FORM_NTT | CGGI_FORM_INT8)))
        return set_error(CGGI_E_PARAM, "forms must be a non-empty mask of "
                                       "CGGI_FORM_NTT | CGGI_FORM_INT8");
    if ((rc = check_form(sh, forms)))
        return rc;
    if (!d_bsk || !d_ksk || !aligned4(d_bsk) || !aligned4(d_ksk))
        return set_error(CGGI_E_SHAPE, "bsk and ksk must be non-NULL and "
                                       "4-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    cggi_ctx *c = new cggi_ctx();
    c->p = *params;
    c->sh = sh;
    c->forms = forms;
    c->ksk = d_ksk;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount,
                              c->device) != hipSuccess || c->cus < 1) {
        free_ctx(c);
        return set_error(CGGI_E_HIP, "hipGetDevice / CU count failed");
    }
    if ((rc = scratch_address(c->device, &c->scratch))) {
        free_ctx(c);
        return rc;
    }
    if (forms & CGGI_FORM_NTT) {
        if ((rc = ntt_make_tables(c, s)) || (rc = ntt_transform_bsk(c, d_bsk, s))) {
            free_ctx(c);
            return rc;
        }
    }
    if (forms & CGGI_FORM_INT8) {
        if ((rc = int8_make_key(c, d_bsk, s))) {
            free_ctx(c);
            return rc;
        }
    }
    if ((rc = keyswitch_make_key(c, s))) {
        free_ctx(c);
        return rc;
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_ctx(c);
        return hip_error(e, "hipStreamSynchronize after key derivation");
    }
    *out = c;
    return CGGI_OK;
}

int cggi_ctx_destroy(cggi_ctx *ctx)
{
    if (!ctx)
        return CGGI_OK;
    (void)hipDeviceSynchronize();
    free_ctx(ctx);
    return CGGI_OK;
}

int cggi_ctx_reserve(cggi_ctx *ctx, int32_t max_gates)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    if (max_gates < 0 || max_gates > (1 << 22))
        return set_error(CGGI_E_SHAPE, "max_gates must be in [0, 2^22]");
    int rc = check_device(ctx);
    if (rc)
        return rc;
    return reserve(ctx, max_gates, nullptr);
}

int cggi_bootstrap_batch(cggi_ctx *ctx, cggi_form_t form,
                         const uint32_t *d_in, const uint32_t *d_testv,
                         uint32_t *d_out, int32_t B, void *stream)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    if (form != CGGI_FORM_NTT && form != CGGI_FORM_INT8)
        return set_error(CGGI_E_PARAM, "unknown form");
    if (!(ctx->forms & (uint32_t)form))
        return set_error(CGGI_E_UNSUPPORTED, "form not built into the context");
    if (B < 0 || B > (1 << 24))
        return set_error(CGGI_E_SHAPE, "B must be in [0, 2^24]");
    if (B == 0)
        return CGGI_OK;
    if (!d_in || !d_out || !aligned4(d_in) || !aligned4(d_out) ||
        (d_testv && !aligned4(d_testv)))
        return set_error(CGGI_E_SHAPE, "in/out must be non-NULL and 4-byte "
                                       "aligned");
    const size_t nin = (size_t)B * (ctx->sh.n + 1) * 4;
    const size_t nout = (size_t)B * (ctx->sh.N + 1) * 4;
    if (overlap(d_out, nout, d_in, nin) ||
        (d_testv && overlap(d_out, nout, d_testv, (size_t)ctx->sh.N * 4)))
        return set_error(CGGI_E_ALIAS, "out overlaps an input");
    int rc = check_device(ctx);
    if (rc)
        return rc;
    hipStream_t s = (hipStream_t)stream;
    ProfScope ps(ctx, 0, s);
    return form == CGGI_FORM_INT8
               ? int8_bootstrap(ctx, d_in, d_testv, d_out, B, nullptr, s)
               : ntt_bootstrap(ctx, d_in, d_testv, d_out, B, nullptr, s);
}

int cggi_keyswitch_batch(cggi_ctx *ctx, const uint32_t *d_in,
                         uint32_t *d_out, int32_t B, void *stream)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    if (B < 0 || B > (1 << 24))
        return set_error(CGGI_E_SHAPE, "B must be in [0, 2^24]");
    if (B == 0)
        return CGGI_OK;
    if (!d_in || !d_out || !aligned4(d_in) || !aligned4(d_out))
        return set_error(CGGI_E_SHAPE, "in/out must be non-NULL and 4-byte "
                                       "aligned");
    const size_t nin = (size_t)B * (ctx->sh.N + 1) * 4;
    const size_t nout = (size_t)B * (ctx->sh.n + 1) * 4;
    if (overlap(d_out, nout, d_in, nin))
        return set_error(CGGI_E_ALIAS, "out overlaps in");
    int rc = check_device(ctx);
    if (rc)
        return rc;
    ProfScope ps(ctx, 1, (hipStream_t)stream);
    return keyswitch_launch(ctx, d_in, d_out, B, (hipStream_t)stream);
}

int cggi_eval_level(cggi_ctx *ctx, cggi_form_t form,
                    const cggi_gate_t *d_gates, int32_t G, uint32_t *d_wires,
                    int32_t W, void *stream)
{
    int rc = level_args_check(ctx, form, d_gates, G, d_wires, W);
    if (rc || G == 0)
        return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = reserve(ctx, G, s)))
        return rc;
    LevelWs ws{ctx->ws_small, ctx->ws_big, ctx->ws_slot, ctx->ws_count};
    return level_launch(ctx, form, d_gates, G, d_wires, W, ws, true, s);
}

int cggi_eval_level_noalloc(cggi_ctx *ctx, cggi_form_t form,
                            const cggi_gate_t *d_gates, int32_t G,
                            uint32_t *d_wires, int32_t W, void *stream)
{
    int rc = level_args_check(ctx, form, d_gates, G, d_wires, W);
    if (rc || G == 0)
        return rc;
    if (!ctx->scratch)
        return set_error(CGGI_E_HIP, "the context has no scratch address");
    const int64_t gmax = scratch_max_gates(ctx->sh);
    if (G > gmax)
        return set_error(CGGI_E_SHAPE,
                         "level of " + std::to_string(G) + " gates exceeds "
                         "the fixed 64 MiB workspace (at most " +
                         std::to_string(gmax) + " gates at these parameters)");
    LevelWs ws{};
    scratch_layout(ctx->sh, G, ctx->scratch, &ws);
    // no profiling events here: their creation would allocate
    return level_launch(ctx, form, d_gates, G, d_wires, W, ws, false,
                        (hipStream_t)stream);
}

int cggi_ctx_profile(cggi_ctx *ctx, int enable)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    ctx->prof = enable != 0;
    prof_clear(ctx);
    return CGGI_OK;
}

int cggi_ctx_profile_read(cggi_ctx *ctx, double *bs_ms, int32_t *bs_launches,
                          double *ks_ms, int32_t *ks_launches)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    double ms[2] = {0.0, 0.0};
    int32_t cnt[2] = {0, 0};
    for (const auto &m : ctx->ev_marks) {
        hipEvent_t a = ctx->ev_pool[m.second], b = ctx->ev_pool[m.second + 1];
        CGGI_HIP_TRY(hipEventSynchronize(b));
        float t = 0.f;
        CGGI_HIP_TRY(hipEventElapsedTime(&t, a, b));
        ms[m.first] += t;
        cnt[m.first] += 1;
    }
    prof_clear(ctx);
    if (bs_ms)
        *bs_ms = ms[0];
    if (bs_launches)
        *bs_launches = cnt[0];
    if (ks_ms)
        *ks_ms = ms[1];
    if (ks_launches)
        *ks_launches = cnt[1];
    return CGGI_OK;
}

int cggi_ctx_latency_mode(cggi_ctx *ctx, int32_t enable)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    ctx->split_on = enable != 0;
    return CGGI_OK;
}

int cggi_ctx_latency_groups(const cggi_ctx *ctx, int32_t *groups)
{
    if (!ctx || !groups)
        return set_error(CGGI_E_PARAM, "ctx or groups is NULL");
    int g = 0;
    for (int v = 0; v < 3; ++v)
        g = ctx->split_groups[v] > g ? ctx->split_groups[v] : g;
    *groups = ctx->split_on ? g : 0;
    return CGGI_OK;
}

int cggi_ctx_int8_plan(cggi_ctx *ctx, const int32_t *kinds,
                       const int32_t *caps, int32_t count)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    if (!(ctx->forms & CGGI_FORM_INT8))
        return set_error(CGGI_E_UNSUPPORTED, "INT8 form not built into the "
                                             "context");
    if (count == 0) {
        ctx->plan_n = 0;
        return CGGI_OK;
    }
    if (count < 0 || count > 8 || !kinds || !caps)
        return set_error(CGGI_E_PARAM, "count must be in [0, 8] and kinds, "
                                       "caps non-NULL");
    for (int k = 0; k < count; ++k) {
        if (kinds[k] < 0 || kinds[k] > 6 || ctx->kind_limit[kinds[k]] <= 0)
            return set_error(CGGI_E_PARAM, "plan entry " + std::to_string(k) +
                                               ": kernel kind unavailable");
        if (caps[k] < 1 || (k > 0 && caps[k] <= caps[k - 1]))
            return set_error(CGGI_E_PARAM, "plan caps must be positive and "
                                           "strictly increasing");
        if ((int64_t)caps[k] > ctx->kind_limit[kinds[k]])
            return set_error(CGGI_E_PARAM,
                             "plan entry " + std::to_string(k) +
                                 ": cap exceeds the kind's limit (" +
                                 std::to_string(ctx->kind_limit[kinds[k]]) +
                                 " bootstraps)");
    }
    if (caps[count - 1] < (1 << 24))
        return set_error(CGGI_E_PARAM, "the last plan entry must hold every "
                                       "batch (cap >= 2^24)");
    for (int k = 0; k < count; ++k) {
        ctx->plan_kind[k] = kinds[k];
        ctx->plan_cap[k] = caps[k];
    }
    ctx->plan_n = count;
    return CGGI_OK;
}

int cggi_ctx_int8_plan_get(const cggi_ctx *ctx, int32_t *kinds,
                           int32_t *caps, int32_t max, int32_t *count)
{
    if (!ctx || !count || max < 0 || (max > 0 && (!kinds || !caps)))
        return set_error(CGGI_E_PARAM, "ctx or count NULL, or arrays NULL");
    if (!(ctx->forms & CGGI_FORM_INT8))
        return set_error(CGGI_E_UNSUPPORTED, "INT8 form not built into the "
                                             "context");
    int32_t k0[8], c0[8];
    const int n = int8_active_plan(ctx, k0, c0);
    if (n > max)
        return set_error(CGGI_E_SHAPE, "max is smaller than the plan (" +
                                           std::to_string(n) + " entries)");
    for (int k = 0; k < n; ++k) {
        kinds[k] = k0[k];
        caps[k] = c0[k];
    }
    *count = n;
    return CGGI_OK;
}

int cggi_ctx_int8_limits(const cggi_ctx *ctx, int32_t *limits)
{
    if (!ctx || !limits)
        return set_error(CGGI_E_PARAM, "ctx or limits is NULL");
    for (int k = 0; k < 7; ++k)
        limits[k] = ctx->kind_limit[k] > INT32_MAX
                        ? INT32_MAX
                        : (int32_t)ctx->kind_limit[k];
    return CGGI_OK;
}

int cggi_ctx_latency_abort(cggi_ctx *ctx)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    int rc = check_device(ctx);
    if (rc)
        return rc;
    if (!ctx->x_err)
        return CGGI_OK;
    // a stream that does not wait for the legacy default stream, so the
    // write lands while latency-mode kernels on any stream still run
    if (!ctx->abort_stream)
        CGGI_HIP_TRY(hipStreamCreateWithFlags(&ctx->abort_stream,
                                              hipStreamNonBlocking));
    const uint32_t one = 1;
    CGGI_HIP_TRY(hipMemcpyAsync(ctx->x_err, &one, 4, hipMemcpyHostToDevice,
                                ctx->abort_stream));
    CGGI_HIP_TRY(hipStreamSynchronize(ctx->abort_stream));
    return CGGI_OK;
}

int cggi_ctx_check(cggi_ctx *ctx)
{
    if (!ctx)
        return set_error(CGGI_E_PARAM, "ctx is NULL");
    int rc = check_device(ctx);
    if (rc)
        return rc;
    CGGI_HIP_TRY(hipDeviceSynchronize());
    if (!ctx->x_err)
        return CGGI_OK;
    uint32_t flag = 0;
    CGGI_HIP_TRY(hipMemcpy(&flag, ctx->x_err, 4, hipMemcpyDeviceToHost));
    if (!flag)
        return CGGI_OK;
    if ((rc = int8_split_reset(ctx)))
        return rc;
    return set_error(CGGI_E_TIMEOUT,
                     "a latency-mode bootstrap timed out waiting for its "
                     "workgroups; its outputs and those of later latency-mode "
                     "calls since the last check are invalid");
}

const char *cggi_last_error(void)
{
    return g_last_error.c_str();
}

} // extern "C"
