/*
 * cggi_oracle.c -- plain CPU oracle for batched CGGI gate bootstrapping over
 * the 32-bit discretised torus (ArctyrEX, arXiv 2306.11006, Section 2.2
 * "The CGGI Cryptosystem" and Fig. 1 "Encrypted Logic Gate Evaluation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and
 * the CPU-baseline leg of the benchmark may load this library.  The GPU
 * library shares no code, header, table or helper with this file; the two
 * meet only through the seeded input arrays the tests hand to both.
 *
 * Everything is written the slow, obvious way: every negacyclic product is
 * the schoolbook sum over monomials X^m * X^k with X^N = -1, every torus
 * value is a uint32_t whose wrap-around IS the reduction mod 2^32, and the
 * steps of a gate run in the order of Fig. 1 (linear pre-op, accumulator
 * init, n CMux steps, key switch), with sample extraction between the loop
 * and the key switch.
 *
 * Conventions the paper leaves open (each is listed with its reading in the
 * design notes of the repository; the one-line summary is repeated at the
 * function that uses it):
 *   - bit encoding: 1 -> +2^29 (+1/8), 0 -> -2^29 (-1/8);
 *   - modulus switch rounds half up;
 *   - gadget digits are signed, in [-Bg/2, Bg/2), rounded to the nearest
 *     multiple of 2^(32 - l*beta);
 *   - TRGSW row r = c*l + (p-1), c = 0 for the mask component, 1 for body;
 *   - key-switch digits are unsigned in [0, 2^gamma), rounded;
 *   - sample extraction takes coefficient 0.
 *
 * Parity status (see the tests): every function here is pinned by a closed
 * form, an exhaustive or brute-force check, or a decryption truth table.
 * The key and noise generation helpers take their random draws as inputs;
 * the rounded-Gaussian draws themselves come from the shared input
 * generator and are pinned there by statistical tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Polynomials in T32[X]/(X^N + 1)                                     */
/* ------------------------------------------------------------------ */

/* out = X^e * p, e in [0, 2N).  Monomial rule: X^(m+e) with m+e >= N
 * wraps to -X^(m+e-N); a second wrap (m+e >= 2N) restores the sign. */
void orc_mono_mul(int N, int e, const uint32_t *p, uint32_t *out)
{
    for (int m = 0; m < N; ++m) {
        int t = m + e;
        uint32_t v = p[m];
        if (t >= 2 * N) {
            t -= 2 * N;
        } else if (t >= N) {
            t -= N;
            v = 0u - v;
        }
        out[t] = v;
    }
}

/* out = x * y in Z_{2^32}[X]/(X^N + 1), schoolbook.  Each product
 * x_m * y_k lands on X^(m+k); if m+k >= N it lands on X^(m+k-N) with a
 * minus sign (X^N = -1).  Section 2.2 names these products as the
 * dominant cost of bootstrapping. */
void orc_poly_mul(int N, const uint32_t *x, const uint32_t *y, uint32_t *out)
{
    uint32_t *acc = (uint32_t *)calloc((size_t)N, sizeof(uint32_t));
    for (int m = 0; m < N; ++m) {
        uint32_t xm = x[m];
        for (int k = 0; k < N - m; ++k)
            acc[m + k] += xm * y[k];
        for (int k = N - m; k < N; ++k)
            acc[m + k - N] -= xm * y[k];
    }
    memcpy(out, acc, (size_t)N * sizeof(uint32_t));
    free(acc);
}

/* ------------------------------------------------------------------ */
/* Scalar maps: modulus switch, gadget decomposition, KS digits        */
/* ------------------------------------------------------------------ */

/* Modulus switch of one torus value to Z_{2N} (the exponents of X in
 * Fig. 1): round(u * 2N / 2^32) mod 2N, ties rounded up. */
uint32_t orc_modswitch(uint32_t u, int N)
{
    int log2_2n = 0;
    while ((1 << log2_2n) < 2 * N)
        ++log2_2n;
    uint32_t half = 1u << (31 - log2_2n);
    return (uint32_t)((uint32_t)(u + half) >> (32 - log2_2n));
}

/* Signed gadget decomposition of u in base Bg = 2^beta with l levels:
 * digits d_1..d_l in [-Bg/2, Bg/2) with sum_p d_p * 2^(32 - p*beta) equal
 * to u rounded to the nearest multiple of 2^(32 - l*beta) (ties up), mod
 * 2^32.  Adding Bg/2 at every level and subtracting it from each digit
 * turns the unsigned base-Bg expansion into the centred one. */
void orc_decomp(uint32_t u, int beta, int l, int32_t *d)
{
    uint32_t w = u;
    if (32 - l * beta >= 1)
        w += 1u << (31 - l * beta);          /* rounding offset */
    for (int p = 1; p <= l; ++p)
        w += (1u << (beta - 1)) << (32 - p * beta);
    for (int p = 1; p <= l; ++p) {
        uint32_t digit = (w >> (32 - p * beta)) & ((1u << beta) - 1u);
        d[p - 1] = (int32_t)digit - (int32_t)(1u << (beta - 1));
    }
}

/* Key-switch digits of u in base 2^gamma, t levels, unsigned, u rounded
 * to the nearest multiple of 2^(32 - t*gamma) (ties up). */
void orc_ks_digits(uint32_t u, int gamma, int t, uint32_t *d)
{
    uint32_t w = u;
    if (32 - t * gamma >= 1)
        w += 1u << (31 - t * gamma);
    for (int p = 1; p <= t; ++p)
        d[p - 1] = (w >> (32 - p * gamma)) & ((1u << gamma) - 1u);
}

/* ------------------------------------------------------------------ */
/* LWE                                                                  */
/* ------------------------------------------------------------------ */

/* ct = (a, <a,s> + e + mu); a is supplied (uniform), e is supplied
 * (rounded Gaussian), s is binary. */
void orc_lwe_encrypt(int n, const uint8_t *s, const uint32_t *a, int32_t e,
                     uint32_t mu, uint32_t *ct)
{
    uint32_t dot = 0;
    for (int i = 0; i < n; ++i) {
        ct[i] = a[i];
        if (s[i])
            dot += a[i];
    }
    ct[n] = dot + (uint32_t)e + mu;
}

/* phase = b - <a,s> mod 2^32 */
uint32_t orc_lwe_phase(int n, const uint8_t *s, const uint32_t *ct)
{
    uint32_t dot = 0;
    for (int i = 0; i < n; ++i)
        if (s[i])
            dot += ct[i];
    return ct[n] - dot;
}

/* bit = 1 iff the phase, read as a signed value, is positive. */
int orc_lwe_decrypt(int n, const uint8_t *s, const uint32_t *ct)
{
    return (int32_t)orc_lwe_phase(n, s, ct) > 0 ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* Key generation (random draws are inputs)                             */
/* ------------------------------------------------------------------ */

/* Bootstrapping key: for every LWE key bit s_i, a TRGSW encryption of s_i
 * under the binary TRLWE key K (Section 2.2: a TGSW ciphertext is a stack
 * of TLWE ciphertexts, and the bootstrapping key encrypts the LWE secret
 * with them).  Row r = c*l + (p-1) is the TRLWE encryption of zero
 * (a_r, a_r * K + e_r), plus s_i * 2^(32 - p*beta) on coefficient 0 of
 * component c.
 *   a: [n][2l][N] uniform, e: [n][2l][N] noise, bsk: [n][2l][2][N]. */
void orc_make_bsk(int n, int N, int beta, int l, const uint8_t *s,
                  const uint8_t *K, const uint32_t *a, const int32_t *e,
                  uint32_t *bsk)
{
    uint32_t *Kp = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    uint32_t *prod = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    for (int j = 0; j < N; ++j)
        Kp[j] = K[j];
    for (int i = 0; i < n; ++i) {
        for (int r = 0; r < 2 * l; ++r) {
            const uint32_t *ar = a + ((size_t)i * 2 * l + r) * N;
            const int32_t *er = e + ((size_t)i * 2 * l + r) * N;
            uint32_t *mask = bsk + (((size_t)i * 2 * l + r) * 2 + 0) * N;
            uint32_t *body = bsk + (((size_t)i * 2 * l + r) * 2 + 1) * N;
            orc_poly_mul(N, ar, Kp, prod);
            for (int j = 0; j < N; ++j) {
                mask[j] = ar[j];
                body[j] = prod[j] + (uint32_t)er[j];
            }
            int c = r / l, p = r % l + 1;
            if (s[i]) {
                uint32_t g = 1u << (32 - p * beta);
                if (c == 0)
                    mask[0] += g;
                else
                    body[0] += g;
            }
        }
    }
    free(Kp);
    free(prod);
}

/* Key-switching key: ksk[j][p][h] encrypts h * K_j * 2^(32 - p*gamma)
 * under s, for h in [1, 2^gamma); the h = 0 slot is all zeros, so
 * gathering it is the same as skipping it.
 *   a: [N][t][2^gamma][n] uniform, e: [N][t][2^gamma] noise,
 *   ksk: [N][t][2^gamma][n+1]. */
void orc_make_ksk(int n, int N, int gamma, int t, const uint8_t *s,
                  const uint8_t *K, const uint32_t *a, const int32_t *e,
                  uint32_t *ksk)
{
    int base = 1 << gamma;
    for (int j = 0; j < N; ++j)
        for (int p = 1; p <= t; ++p)
            for (int h = 0; h < base; ++h) {
                size_t row = ((size_t)j * t + (p - 1)) * base + h;
                uint32_t *ct = ksk + row * (size_t)(n + 1);
                if (h == 0) {
                    memset(ct, 0, (size_t)(n + 1) * sizeof(uint32_t));
                    continue;
                }
                uint32_t mu = (uint32_t)h * (uint32_t)K[j] *
                              (1u << (32 - p * gamma));
                orc_lwe_encrypt(n, s, a + row * (size_t)n, e[row], mu, ct);
            }
}

/* ------------------------------------------------------------------ */
/* TRLWE x TRGSW external product, CMux, blind rotation, extraction      */
/* ------------------------------------------------------------------ */

/* out = C (ext) d:  decompose both components of the TRLWE d and sum the
 * digit polynomials times the TRGSW rows:
 *   out[c'] = sum_{c, p} D[c][p] * C[c*l + p - 1][c'].
 * C: [2l][2][N], d: [2][N], out: [2][N] (may alias d). */
void orc_external_product(int N, int beta, int l, const uint32_t *C,
                          const uint32_t *d, uint32_t *out)
{
    uint32_t *dig = (uint32_t *)malloc((size_t)2 * l * N * sizeof(uint32_t));
    uint32_t *prod = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    uint32_t *res = (uint32_t *)calloc((size_t)2 * N, sizeof(uint32_t));
    int32_t digits[32];
    for (int c = 0; c < 2; ++c)
        for (int j = 0; j < N; ++j) {
            orc_decomp(d[c * N + j], beta, l, digits);
            for (int p = 0; p < l; ++p)
                dig[(size_t)(c * l + p) * N + j] = (uint32_t)digits[p];
        }
    for (int r = 0; r < 2 * l; ++r)
        for (int cp = 0; cp < 2; ++cp) {
            orc_poly_mul(N, dig + (size_t)r * N, C + ((size_t)r * 2 + cp) * N,
                         prod);
            for (int j = 0; j < N; ++j)
                res[cp * N + j] += prod[j];
        }
    memcpy(out, res, (size_t)2 * N * sizeof(uint32_t));
    free(dig);
    free(prod);
    free(res);
}

/* One CMux step of the blind rotation (Fig. 1, loop body):
 *   acc <- acc + C (ext) (X^e * acc - acc). */
void orc_cmux_rotate(int N, int beta, int l, const uint32_t *C, int e,
                     uint32_t *acc)
{
    uint32_t *tmp = (uint32_t *)malloc((size_t)2 * N * sizeof(uint32_t));
    for (int c = 0; c < 2; ++c) {
        orc_mono_mul(N, e, acc + c * N, tmp + c * N);
        for (int j = 0; j < N; ++j)
            tmp[c * N + j] -= acc[c * N + j];
    }
    orc_external_product(N, beta, l, C, tmp, tmp);
    for (int j = 0; j < 2 * N; ++j)
        acc[j] += tmp[j];
    free(tmp);
}

/* Blind rotation of an LWE ciphertext (a, b) of dimension n:
 *   acc = (0, X^(-b~) * v);  for i < n: CMux step with exponent a~_i.
 * bsk: [n][2l][2][N], testv: [N] (NULL means every coefficient 2^29),
 * acc: [2][N] output. */
void orc_blind_rotate(int n, int N, int beta, int l, const uint32_t *bsk,
                      const uint32_t *testv, const uint32_t *in, uint32_t *acc)
{
    uint32_t *v = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    for (int j = 0; j < N; ++j)
        v[j] = testv ? testv[j] : (1u << 29);
    uint32_t bt = orc_modswitch(in[n], N);
    memset(acc, 0, (size_t)N * sizeof(uint32_t));
    orc_mono_mul(N, (int)((2u * N - bt) % (2u * N)), v, acc + N);
    for (int i = 0; i < n; ++i) {
        uint32_t ai = orc_modswitch(in[i], N);
        orc_cmux_rotate(N, beta, l, bsk + (size_t)i * 2 * l * 2 * N, (int)ai,
                        acc);
    }
    free(v);
}

/* Sample extraction of coefficient 0: an LWE ciphertext of dimension N
 * under the coefficients of K, with a'_0 = A_0, a'_j = -A_{N-j},
 * b' = B_0.  acc: [2][N], out: [N+1]. */
void orc_sample_extract(int N, const uint32_t *acc, uint32_t *out)
{
    out[0] = acc[0];
    for (int j = 1; j < N; ++j)
        out[j] = 0u - acc[N - j];
    out[N] = acc[N];
}

/* Bootstrap: blind rotation followed by sample extraction.
 * in: [n+1] (LWE under s), out: [N+1] (LWE under K). */
void orc_bootstrap(int n, int N, int beta, int l, const uint32_t *bsk,
                   const uint32_t *testv, const uint32_t *in, uint32_t *out)
{
    uint32_t *acc = (uint32_t *)malloc((size_t)2 * N * sizeof(uint32_t));
    orc_blind_rotate(n, N, beta, l, bsk, testv, in, acc);
    orc_sample_extract(N, acc, out);
    free(acc);
}

/* Key switch from dimension N (key K) back to n (key s), Fig. 1 last
 * step: out = (0, b') - sum_{j<N, p<t} ksk[j][p][d_{j,p}].
 * ksk: [N][t][2^gamma][n+1], in: [N+1], out: [n+1]. */
void orc_keyswitch(int n, int N, int gamma, int t, const uint32_t *ksk,
                   const uint32_t *in, uint32_t *out)
{
    int base = 1 << gamma;
    uint32_t dig[32];
    memset(out, 0, (size_t)(n + 1) * sizeof(uint32_t));
    out[n] = in[N];
    for (int j = 0; j < N; ++j) {
        orc_ks_digits(in[j], gamma, t, dig);
        for (int p = 0; p < t; ++p) {
            const uint32_t *row =
                ksk + (((size_t)j * t + p) * base + dig[p]) * (size_t)(n + 1);
            for (int x = 0; x <= n; ++x)
                out[x] -= row[x];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Gates                                                                */
/* ------------------------------------------------------------------ */

enum {
    ORC_NAND = 0, ORC_AND = 1, ORC_OR = 2, ORC_XOR = 3, ORC_MUX = 4,
    ORC_NOT = 5, ORC_COPY = 6, ORC_CONST0 = 7, ORC_CONST1 = 8,
    ORC_NOR = 9, ORC_XNOR = 10
};

#define ORC_MU (1u << 29) /* +1/8 */

/* Linear pre-op of a two-input bootstrapped gate (Fig. 1, first box; all
 * bootstrapped gates differ only here).  out = (0, c) + sx*x + sy*y with
 * the constant and signs of the gate; dimension n. */
static void orc_linear(int n, uint32_t c, int sx, const uint32_t *x, int sy,
                       const uint32_t *y, uint32_t *out)
{
    for (int i = 0; i <= n; ++i) {
        uint32_t v = (i == n) ? c : 0u;
        v += (uint32_t)sx * x[i];
        v += (uint32_t)sy * y[i];
        out[i] = v;
    }
}

/* Bootstrapped gate per Fig. 1: linear pre-op, bootstrap (dimension N),
 * key switch back to dimension n.  MUX(sel, a, b) = sel ? a : b takes two
 * bootstraps (AND(sel, a) and AND(!sel, b) without key switch), adds them
 * to (0, +1/8) and key-switches once.  NOT, COPY and the constants are
 * linear and take no bootstrap.  All ciphertexts are [n+1]. */
void orc_gate(int op, int n, int N, int beta, int l, int gamma, int t,
              const uint32_t *bsk, const uint32_t *ksk, const uint32_t *x,
              const uint32_t *y, const uint32_t *z, uint32_t *out)
{
    uint32_t *lin = (uint32_t *)calloc((size_t)(n + 1), sizeof(uint32_t));
    uint32_t *big = (uint32_t *)malloc((size_t)(N + 1) * sizeof(uint32_t));
    uint32_t *big2 = (uint32_t *)malloc((size_t)(N + 1) * sizeof(uint32_t));
    switch (op) {
    case ORC_NOT:
        for (int i = 0; i <= n; ++i)
            out[i] = 0u - x[i];
        goto done;
    case ORC_COPY:
        memcpy(out, x, (size_t)(n + 1) * sizeof(uint32_t));
        goto done;
    case ORC_CONST0:
    case ORC_CONST1:
        memset(out, 0, (size_t)n * sizeof(uint32_t));
        out[n] = op == ORC_CONST1 ? ORC_MU : 0u - ORC_MU;
        goto done;
    case ORC_MUX:
        orc_linear(n, 0u - ORC_MU, 1, x, 1, y, lin);      /* AND(sel, a)  */
        orc_bootstrap(n, N, beta, l, bsk, NULL, lin, big);
        orc_linear(n, 0u - ORC_MU, -1, x, 1, z, lin);     /* AND(!sel, b) */
        orc_bootstrap(n, N, beta, l, bsk, NULL, lin, big2);
        for (int j = 0; j <= N; ++j)
            big[j] += big2[j];
        big[N] += ORC_MU;
        orc_keyswitch(n, N, gamma, t, ksk, big, out);
        goto done;
    case ORC_NAND: orc_linear(n, ORC_MU, -1, x, -1, y, lin); break;
    case ORC_AND:  orc_linear(n, 0u - ORC_MU, 1, x, 1, y, lin); break;
    case ORC_OR:   orc_linear(n, ORC_MU, 1, x, 1, y, lin); break;
    case ORC_XOR:  orc_linear(n, 2u * ORC_MU, 2, x, 2, y, lin); break;
    case ORC_NOR:  orc_linear(n, 0u - ORC_MU, -1, x, -1, y, lin); break;
    case ORC_XNOR: orc_linear(n, 0u - 2u * ORC_MU, -2, x, -2, y, lin); break;
    default:
        memset(out, 0, (size_t)(n + 1) * sizeof(uint32_t));
        goto done;
    }
    orc_bootstrap(n, N, beta, l, bsk, NULL, lin, big);
    orc_keyswitch(n, N, gamma, t, ksk, big, out);
done:
    free(lin);
    free(big);
    free(big2);
}

/* Linear pre-op only (for tests that feed the GPU bootstrap the same
 * input the oracle gate bootstraps).  For MUX, `which` selects the first
 * (0) or second (1) bootstrap input. */
void orc_gate_preop(int op, int which, int n, const uint32_t *x,
                    const uint32_t *y, const uint32_t *z, uint32_t *out)
{
    switch (op) {
    case ORC_NAND: orc_linear(n, ORC_MU, -1, x, -1, y, out); break;
    case ORC_AND:  orc_linear(n, 0u - ORC_MU, 1, x, 1, y, out); break;
    case ORC_OR:   orc_linear(n, ORC_MU, 1, x, 1, y, out); break;
    case ORC_XOR:  orc_linear(n, 2u * ORC_MU, 2, x, 2, y, out); break;
    case ORC_NOR:  orc_linear(n, 0u - ORC_MU, -1, x, -1, y, out); break;
    case ORC_XNOR: orc_linear(n, 0u - 2u * ORC_MU, -2, x, -2, y, out); break;
    case ORC_MUX:
        if (which == 0)
            orc_linear(n, 0u - ORC_MU, 1, x, 1, y, out);
        else
            orc_linear(n, 0u - ORC_MU, -1, x, 1, z, out);
        break;
    default:
        memset(out, 0, (size_t)(n + 1) * sizeof(uint32_t));
    }
}

/* Batch drivers: plain loops over independent items. */
void orc_bootstrap_batch(int n, int N, int beta, int l, const uint32_t *bsk,
                         const uint32_t *testv, const uint32_t *in,
                         uint32_t *out, int B)
{
    for (int g = 0; g < B; ++g)
        orc_bootstrap(n, N, beta, l, bsk, testv, in + (size_t)g * (n + 1),
                      out + (size_t)g * (N + 1));
}

void orc_keyswitch_batch(int n, int N, int gamma, int t, const uint32_t *ksk,
                         const uint32_t *in, uint32_t *out, int B)
{
    for (int g = 0; g < B; ++g)
        orc_keyswitch(n, N, gamma, t, ksk, in + (size_t)g * (N + 1),
                      out + (size_t)g * (n + 1));
}

/* Elementwise maps over arrays (for exhaustive tests). */
void orc_modswitch_array(const uint32_t *u, uint32_t *out, long count, int N)
{
    for (long i = 0; i < count; ++i)
        out[i] = orc_modswitch(u[i], N);
}

void orc_decomp_array(const uint32_t *u, int32_t *d, long count, int beta,
                      int l)
{
    for (long i = 0; i < count; ++i)
        orc_decomp(u[i], beta, l, d + i * l);
}

void orc_ks_digits_array(const uint32_t *u, uint32_t *d, long count,
                         int gamma, int t)
{
    for (long i = 0; i < count; ++i)
        orc_ks_digits(u[i], gamma, t, d + i * t);
}
