/*
 * cggi.h -- C ABI of the MI355X (gfx950) batched CGGI gate-bootstrapping
 * library libcggi.so.
 *
 * The method: ArctyrEX (arXiv 2306.11006), Section 2.2 "The CGGI
 * Cryptosystem" and Fig. 1 "Encrypted Logic Gate Evaluation" -- a
 * bootstrapped gate is a linear pre-op on LWE ciphertexts, a modulus switch
 * of the result to Z_2N, an accumulator initialised to X^(-b~) * v, n CMux
 * steps (rotate, subtract, gadget-decompose, multiply by a TRGSW row of the
 * bootstrapping key, add), sample extraction, and a key switch back to the
 * LWE key.  Section 4.2 ("waves") levelises a gate DAG so that every gate of
 * a level is independent; Section 5.3 runs one batched launch per set of
 * gates.
 *
 * Torus values are uint32_t (Z/2^32; the value u stands for u / 2^32) and
 * every addition wraps mod 2^32.  All array arguments are DEVICE pointers
 * (for example torch tensor data pointers) unless stated otherwise, are
 * row-major and contiguous, and stay owned by the caller.  Layouts:
 *   LWE ciphertext of dimension d : uint32_t[d + 1] = (a_0..a_{d-1}, b)
 *   bootstrapping key (bsk)       : uint32_t[n][2l][2][N]; row r = c*l+(p-1)
 *       (c = 0 mask / 1 body component being decomposed, p = 1..l gadget
 *       level), then output component (0 = mask, 1 = body), then coefficient
 *   key-switching key (ksk)       : uint32_t[N][t][2^gamma][n + 1]; entry
 *       [j][p][h] is an LWE encryption of h * K_j * 2^(32 - (p+1)*gamma)
 *
 * Every entry point returns CGGI_OK (0) or a negative error code and, on
 * error, leaves a message for cggi_last_error().  Shape and parameter errors
 * are found on the host before anything is launched and leave every output
 * untouched.  Batch calls are asynchronous on the given stream, allocate
 * nothing while the workspace suffices (see cggi_ctx_reserve), never read
 * device data on the host, and may be captured into a HIP graph.
 * Calls on one context must not run concurrently from several host threads.
 */
#ifndef CGGI_H
#define CGGI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Scheme parameters.  k must be 1 (one TRLWE mask polynomial).
 * N in {256, 512, 1024, 2048}; gadget base Bg = 2^bg_bit with l levels;
 * key switch base 2^ks_base_bit with ks_t levels. */
typedef struct {
    int32_t n, N, k, bg_bit, l, ks_base_bit, ks_t;
} cggi_params_t;

/* Forms of the negacyclic products inside the blind rotation.  Both give
 * bit-identical results.
 *  NTT : exact NTT modulo Q = 2^64 - 2^32 + 1 with the paper's generator
 *        (Section 5.4), centred lift, low 32 bits.
 *  INT8: exact split-limb block-Toeplitz GEMM on int8 MFMA with int32
 *        accumulation; each key coefficient is split into four signed
 *        8-bit limbs and the limbs are recombined mod 2^32. */
typedef enum { CGGI_FORM_NTT = 1, CGGI_FORM_INT8 = 2 } cggi_form_t;

enum {
    CGGI_OK = 0,
    CGGI_E_PARAM = -1,       /* unsupported or inconsistent parameters     */
    CGGI_E_SHAPE = -2,       /* bad size, null or misaligned pointer        */
    CGGI_E_ALIAS = -3,       /* output overlaps an input                    */
    CGGI_E_HIP = -4,         /* a HIP runtime call failed                   */
    CGGI_E_NOMEM = -5,       /* device allocation failed                    */
    CGGI_E_UNSUPPORTED = -6, /* form not built into the context, or an
                                allocation would be needed during capture   */
    CGGI_E_TIMEOUT = -7      /* a latency-mode bootstrap's workgroups did
                                not meet (see cggi_ctx_check)               */
};

/* Gate opcodes of cggi_eval_level.  MUX(in0 = select, in1 = value if 1,
 * in2 = value if 0) takes two bootstraps and one key switch; NOT, COPY and
 * the constants take none; every other opcode takes one of each. */
enum {
    CGGI_NAND = 0, CGGI_AND = 1, CGGI_OR = 2, CGGI_XOR = 3, CGGI_MUX = 4,
    CGGI_NOT = 5, CGGI_COPY = 6, CGGI_CONST0 = 7, CGGI_CONST1 = 8,
    CGGI_NOR = 9, CGGI_XNOR = 10
};

typedef struct {
    int32_t op, in0, in1, in2, out; /* wire indices; unused inputs ignored */
} cggi_gate_t;

typedef struct cggi_ctx cggi_ctx; /* opaque */

/* Check a parameter set without touching the GPU.  Returns CGGI_OK or
 * CGGI_E_PARAM (with a message).  Pure host code. */
int cggi_params_check(const cggi_params_t *params);

/* Create a context on the current HIP device.  Reads d_bsk
 * ([n][2l][2][N]) once to derive the key forms selected by `forms` (a
 * bitmask of cggi_form_t): the NTT form stores the bootstrapping key
 * transformed mod Q (8 * n*2l*2*N bytes), the INT8 form stores its int8
 * limb windows (n*R*2*4*(N+64) bytes, R = 2l digit rows for Bg <= 2^7,
 * 4l for Bg <= 2^13) and, for N <= 1024, the key-only correction of its
 * offset digit operands (4 * n*2*N bytes).  For key-switch bases up to 2^4
 * the context also stores d_ksk as int8 limb blocks for the GEMM key switch
 * (ceil((n+1)/32) * N * ceil(t*2^gamma/32) * 4 KB).  d_bsk may be freed
 * once this call returns (it synchronises `stream`).  d_ksk
 * ([N][t][2^gamma][n+1]) must stay valid and unchanged for the context's
 * life (larger bases gather its rows directly).
 * `stream` is a hipStream_t (NULL = default stream).  On success *out
 * receives the context.  The INT8 form takes Bg <= 2^13 and l <= 8 (and a
 * workgroup that fits the LDS); otherwise CGGI_E_PARAM. */
int cggi_ctx_create(const cggi_params_t *params, const uint32_t *d_bsk,
                    const uint32_t *d_ksk, uint32_t forms, void *stream,
                    cggi_ctx **out);

/* Free a context and everything it allocated (waits for the device).
 * NULL is accepted. */
int cggi_ctx_destroy(cggi_ctx *ctx);

/* Pre-allocate the workspace of cggi_eval_level for levels of up to
 * max_gates gates, so that later calls allocate nothing (required before
 * graph capture).  cggi_bootstrap_batch and cggi_keyswitch_batch need no
 * workspace. */
int cggi_ctx_reserve(cggi_ctx *ctx, int32_t max_gates);

/* Bootstrap a batch (Fig. 1, the looped steps plus sample extraction):
 * for each of the B LWE ciphertexts d_in[B][n+1] (key s), modulus switch,
 * initialise ACC = (0, X^(-b~) * v), run n CMux steps with the
 * bootstrapping key, and extract coefficient 0 into d_out[B][N+1], an LWE
 * ciphertext of dimension N under the TRLWE key.  d_testv is the test
 * polynomial v ([N] torus values) or NULL for v = 2^29 * sum_j X^j (gate
 * bootstrapping).  B == 0 is a no-op.  d_out must not overlap d_in or
 * d_testv.  Bit-identical for both forms. */
int cggi_bootstrap_batch(cggi_ctx *ctx, cggi_form_t form,
                         const uint32_t *d_in, const uint32_t *d_testv,
                         uint32_t *d_out, int32_t B, void *stream);

/* Key switch a batch (Fig. 1, last step): d_in[B][N+1] (key K) ->
 * d_out[B][n+1] (key s), out = (0,..,0, b') - sum_{j<N, p<t}
 * ksk[j][p][digit_p(a'_j)], with unsigned base-2^gamma digits of a'_j
 * rounded to t*gamma bits.  Bases up to 2^4 run as an int8 GEMM of the
 * one-hot digit matrix with the key, split over j and summed into d_out
 * with device atomics (exact mod 2^32, so the result does not depend on
 * their order); larger bases gather key rows.  B == 0 is a no-op.  d_out
 * must not overlap d_in. */
int cggi_keyswitch_batch(cggi_ctx *ctx, const uint32_t *d_in,
                         uint32_t *d_out, int32_t B, void *stream);

/* Evaluate one level (Section 4.2 "wave") of a gate DAG in place on the
 * wire array d_wires[W][n+1]: every gate reads its input wires and writes
 * its output wire.  d_gates[G] is a device array of cggi_gate_t.  Contract
 * (the levelizer guarantees it): no gate's out equals any input of a gate
 * of the same level, and no two gates share an out.  A gate with an
 * unknown opcode or a wire index outside [0, W) is skipped on the device
 * (its output wire is not written); nothing is ever accessed out of
 * bounds.  Gate pre-ops (Fig. 1 first
 * box; bit 1 = +1/8, bit 0 = -1/8):
 *   NAND (0,1/8)-x-y  AND (0,-1/8)+x+y  OR (0,1/8)+x+y  XOR (0,1/4)+2(x+y)
 *   NOR (0,-1/8)-x-y  XNOR (0,-1/4)-2(x+y)  NOT -x  COPY x  CONST (0,+-1/8)
 *   MUX u1 = BS((0,-1/8)+c+x), u2 = BS((0,-1/8)-c+y), out = KS((0,1/8)+u1+u2)
 * G == 0 is a no-op.  Needs cggi_ctx_reserve(ctx, >= G) when called
 * under graph capture. */
int cggi_eval_level(cggi_ctx *ctx, cggi_form_t form,
                    const cggi_gate_t *d_gates, int32_t G, uint32_t *d_wires,
                    int32_t W, void *stream);

/* cggi_eval_level for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same level, the same kernels and bit-identical wires,
 * but the level's workspace (bootstrap slots, bootstrap inputs [2G][n+1]
 * and outputs [2G][N+1]) lives in a fixed 64 MiB device array of the
 * library instead of the context's reserved workspace, so no
 * cggi_ctx_reserve is needed and nothing is allocated or freed: no
 * hipMalloc, hipFree or allocating library call, and no profiling events.
 * Every GPU the library runs on holds its own copy of that array from the
 * first context created on it until the process ends.  Limit: G may be at
 * most floor(~64 MiB / (4 + 8(n+1) + 8(N+1))) gates (5,063 at n=630,
 * N=1024; 3,003 at n=742, N=2048); a larger G returns CGGI_E_SHAPE with
 * the limit in the message and launches nothing.  All calls on one GPU
 * share the one array: calls that may overlap on a GPU (several streams,
 * several contexts, several host threads) race and must be serialised by
 * the caller.  Arguments, contract and other errors as cggi_eval_level. */
int cggi_eval_level_noalloc(cggi_ctx *ctx, cggi_form_t form,
                            const cggi_gate_t *d_gates, int32_t G,
                            uint32_t *d_wires, int32_t W, void *stream);

/* Levelise a gate DAG on the host (Section 4.2, "waves"): every gate gets
 * level 1 + max(level of the gates producing its inputs), 0 when all its
 * inputs are circuit inputs (wires no gate writes); gates are visited in
 * first-in-first-out order of readiness, so the work is linear in gates
 * plus wires and disconnected circuits are fine.  Within a level, gates are
 * ordered by opcode (stable), the paper's per-opcode batching.
 *   gates       HOST array [G] (only op, the used inputs and out are read)
 *   W           number of wires; every used index must be in [0, W)
 *   order       HOST out [G]: gate indices, level by level
 *   level_start HOST out [G+1]: level L is order[level_start[L] ..
 *               level_start[L+1]); *n_levels receives the level count
 *   level       HOST out [G] or NULL: level of each gate
 * Errors (nothing useful is written): CGGI_E_SHAPE for a bad size, NULL
 * pointer, unknown opcode or wire out of range; CGGI_E_PARAM when two gates
 * write the same wire, a gate writes a wire it reads, or the gates form a
 * cycle.  Pure host code. */
int cggi_levelize(const cggi_gate_t *gates, int32_t G, int32_t W,
                  int32_t *order, int32_t *level_start, int32_t *n_levels,
                  int32_t *level);

/* Kernel timing (tracing for benchmarks).  While enabled, every bootstrap
 * and key-switch kernel launched eagerly (not under graph capture) through
 * this context is bracketed by HIP events recorded on the stream it is
 * launched on.  cggi_ctx_profile_read waits for those events, returns the
 * summed milliseconds and launch counts of each kind (any output pointer
 * may be NULL) and clears them.  Enabling or disabling also clears. */
int cggi_ctx_profile(cggi_ctx *ctx, int enable);
int cggi_ctx_profile_read(cggi_ctx *ctx, double *bs_ms, int32_t *bs_launches,
                          double *ks_ms, int32_t *ks_launches);

/* Diagnostic: the int8 MFMA rate this GPU sustains.  Times a bare loop of
 * v_mfma_i32_32x32x32_i8 (`iters` iterations of 8 independent MFMAs per
 * wave, one workgroup of 8 waves per CU, the int8 form's launch shape) on
 * random (random_operands != 0) or all-zero operand bits, and writes the
 * rate in tera-operations per second (2 per multiply-add) to *tops.  With
 * random operands the GPU lowers its clock to stay within its power limit,
 * so this is the ceiling the int8 blind rotation can approach; the
 * published dense int8 rate assumes the top clock.  Not a batch call: it
 * allocates and frees 64 KB of device memory, runs on the default stream
 * of the current device and waits for completion.  CGGI_E_PARAM for
 * iters < 1 or tops NULL, CGGI_E_HIP on a runtime error. */
int cggi_measure_int8_mfma(int32_t iters, int32_t random_operands,
                           double *tops);

/* Diagnostic: the Goldilocks multiply-mod rate this GPU sustains.  Times a
 * bare loop of the NTT form's own multiply-mod modulo Q = 2^64 - 2^32 + 1
 * (Section 5.4's modulus: a 64 x 64 -> 128-bit product from four 32 x 32 +
 * 64 multiply-adds, then the reduction) on 8 independent chains per
 * thread, two workgroups of 512 threads per CU (the NTT form's launch
 * shape), `iters` iterations, random residues; writes tera multiply-mods
 * per second to *tmulmods.  An upper bound for the NTT form, whose
 * butterflies also add, subtract and address.  Not a batch call: it
 * allocates and frees 32 KB plus one word per thread of device memory,
 * runs on the default stream of the current device and waits for
 * completion.  CGGI_E_PARAM for iters < 1 or tmulmods NULL, CGGI_E_HIP on
 * a runtime error. */
int cggi_measure_mulmod(int32_t iters, double *tmulmods);

/* Latency mode of the INT8 form (N <= 1024).  ArctyrEX's closing section
 * names splitting one gate over several SMs as the way to speed up narrow
 * circuit levels; here a narrow batch runs each column tile's blind
 * rotation (1024/N bootstraps) on four workgroups on four CUs, one per
 * block (input component, output component) of the external product, or,
 * for at most half as many tiles, on eight (each block's four key limbs in
 * two pairs), or, for up to twice as many tiles, on two (one per output
 * component), which exchange their partial products after every CMux step
 * through device memory.  Results are bit-identical to the one-workgroup
 * kernel.  Every INT8 call picks its kernel from the batch size: latency
 * mode with eight, four, then two workgroups per tile while the tiles fit,
 * then one workgroup per 1, 2 or 4 tiles (or as cggi_ctx_int8_plan sets).
 * cggi_bootstrap_batch decides on the host from B;
 * cggi_eval_level, whose bootstrap count is known only on the device,
 * launches every candidate up to the one that holds 2G bootstraps, and each
 * runs only if the device count falls in its range.  cggi_ctx_latency_groups
 * reports the most tiles a latency-mode launch takes (every workgroup of
 * such a launch is resident at once; 0 when latency mode is off or
 * unavailable: N = 2048, more than 8 digit polynomials, or LDS).  It is on
 * by default; cggi_ctx_latency_mode(ctx, 0) turns it off, e.g. when other
 * streams keep the GPU's CUs busy, since the workgroups of a tile wait for
 * each other.  Each wait is bounded (1 s): on a time-out the kernel sets an
 * error word in the context and stops, and every later latency-mode launch
 * on the context does nothing until cggi_ctx_check, which waits for the
 * device, returns CGGI_E_TIMEOUT if the word was set (clearing it and the
 * exchange buffers), else CGGI_OK.  Latency-mode launches on one context
 * must not run concurrently (they share its exchange buffers). */
int cggi_ctx_latency_mode(cggi_ctx *ctx, int32_t enable);
int cggi_ctx_latency_groups(const cggi_ctx *ctx, int32_t *groups);
int cggi_ctx_check(cggi_ctx *ctx);
/* Sets the context's latency-mode error word from the host at once (not
 * stream-ordered: the write goes through a non-blocking stream of the
 * context, so it does not queue behind kernels on the default stream or
 * any other), as a time-out would: latency-mode kernels still running
 * stop at their next poll, later ones do nothing (their outputs are left
 * untouched) until cggi_ctx_check, which then returns CGGI_E_TIMEOUT and
 * clears the state.  Other INT8 kernels and the NTT form are unaffected.
 * CGGI_OK also when the context has no latency mode. */
int cggi_ctx_latency_abort(cggi_ctx *ctx);

/* INT8 kernel plan (autotuning).  The INT8 form has seven kernels for a
 * batch: CGGI_K_SPLIT8, CGGI_K_SPLIT4 and CGGI_K_SPLIT2 (latency mode,
 * eight, four or two workgroups per column tile; N <= 1024),
 * CGGI_K_TILES1, CGGI_K_TILES2
 * (one workgroup per one or two column tiles; N <= 1024), CGGI_K_TILES4
 * (four tiles, or one bootstrap per workgroup at N = 2048) and
 * CGGI_K_KARA2 (one Karatsuba level: each negacyclic product of length N
 * as three of length N/2 over the even and odd coefficients, 3/4 of the
 * multiply-adds, two column tiles of N/2-length products per workgroup;
 * N <= 1024 where its workgroup fits the LDS, which costs the context a
 * second int8 key form of n*R*2*3*4*(N/2+64) bytes).  A plan is a
 * list of entries (kinds[k], caps[k]) with strictly increasing caps: entry
 * k takes the batches of caps[k-1] + 1 .. caps[k] bootstraps (caps[-1] = 0);
 * the last cap must be at least 2^24 (every batch); a latency-mode entry's
 * cap may not exceed that kind's limit (cggi_ctx_int8_limits: the most
 * bootstraps one launch of each kind may take, 0 if the kind is
 * unavailable; latency-mode limits keep every workgroup resident).  All
 * kinds give bit-identical results; the plan only changes speed.  count = 0
 * restores the built-in plan (latency mode with eight, four, then two
 * workgroups while the tiles fit, then 1, 2 or 4 tiles per workgroup by
 * batch width;
 * see cggi_ctx_latency_mode).  While latency mode is off its entries are
 * skipped and their batches go to the next entry.  cggi_ctx_int8_plan_get
 * writes the plan in force (at most max entries; count = entries).  Host
 * state only: affects calls made afterwards.  Errors: CGGI_E_PARAM for a NULL
 * ctx or an invalid plan (nothing changes), CGGI_E_UNSUPPORTED without the
 * INT8 form, CGGI_E_SHAPE when max is too small. */
enum {
    CGGI_K_SPLIT4 = 0,
    CGGI_K_SPLIT2 = 1,
    CGGI_K_TILES1 = 2,
    CGGI_K_TILES2 = 3,
    CGGI_K_TILES4 = 4,
    CGGI_K_SPLIT8 = 5,
    CGGI_K_KARA2 = 6
};
int cggi_ctx_int8_plan(cggi_ctx *ctx, const int32_t *kinds,
                       const int32_t *caps, int32_t count);
int cggi_ctx_int8_plan_get(const cggi_ctx *ctx, int32_t *kinds,
                           int32_t *caps, int32_t max, int32_t *count);
int cggi_ctx_int8_limits(const cggi_ctx *ctx, int32_t *limits /* [7] */);

/* Message of the last error on the calling thread ("" if none). */
const char *cggi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CGGI_H */
