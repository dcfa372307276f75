/*
 * Reference (oracle) GEMM: plain, slow, obviously correct CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper
 * with the GPU path.
 *
 * What it computes (paper section 3.1, "The baseline algorithm": the matrix
 * multiplication C = C + A B with A m x k, B k x n, C m x n), generalised to
 * the BLAS form C = alpha * op(A) * op(B) + beta * C0 with row-major storage:
 *   op(A)(i,p) = A[i*lda + p]  if transA is 'N',  A[p*lda + i]  if 'T'
 *   op(B)(p,j) = B[p*ldb + j]  if transB is 'N',  B[j*ldb + p]  if 'T'
 * Each C(i,j) is the sum over p = 0..k-1, taken in increasing p, of
 * op(A)(i,p) * op(B)(p,j): the paper's basic triple loop (section 5.1,
 * "Basic GEMM with TVM") in the i -> p -> j nesting, with no blocking.
 * Floating point is FP64; INT8 accumulates exactly in int64 and wraps the
 * final value to int32 (two's complement); INT16 and INT32 keep the exact
 * value modulo 2^32 (int32 C).
 *
 * BLAS conventions (the paper defines only C += AB):
 *   alpha == 0 or k == 0 : the product is not formed and A, B are not read;
 *   beta  == 0           : C0 is not read (NaN/Inf in C0 do not propagate).
 *
 * Also here, each written from its format definition:
 *   - bfloat16 round-to-nearest-even and the hi/mid/lo split of an FP32 value
 *     into bf16 pieces (inputs of the split-product FP32-accurate path);
 *   - exact decoders for bfloat16, IEEE binary16 and OCP FP8 E4M3FN codes;
 *   - the power-of-two scaled quantisation of the scaled low-precision path
 *     (per-row exponents, round-to-nearest-even encoders of each format).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHUNK 256

static int is_t(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* FP64 GEMM.  C = alpha * op(A) op(B) + beta * C0.  C must not alias C0.   */
/* Columns are visited in chunks of CHUNK so the row accumulator lives on   */
/* the stack; each entry still sums p = 0..k-1 in order.                    */
/* ---------------------------------------------------------------------- */
void oracle_gemm_f64(char ta, char tb, int64_t m, int64_t n, int64_t k,
                     double alpha, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double beta,
                     const double *C0, int64_t ldc0, double *C, int64_t ldc)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0.0) && (k > 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        double acc[CHUNK];
        for (int64_t j0 = 0; j0 < n; j0 += CHUNK) {
            const int64_t jn = (n - j0 < CHUNK) ? n - j0 : CHUNK;
            for (int64_t j = 0; j < jn; ++j) acc[j] = 0.0;
            if (form) {
                for (int64_t p = 0; p < k; ++p) {
                    const double a = at ? A[p * lda + i] : A[i * lda + p];
                    for (int64_t j = 0; j < jn; ++j) {
                        const double b = bt ? B[(j0 + j) * ldb + p] : B[p * ldb + (j0 + j)];
                        acc[j] += a * b;
                    }
                }
            }
            for (int64_t j = 0; j < jn; ++j) {
                double v = form ? alpha * acc[j] : 0.0;
                if (beta != 0.0) v += beta * C0[i * ldc0 + (j0 + j)];
                C[i * ldc + (j0 + j)] = v;
            }
        }
    }
}

/* Selected entries of the same product: out[t] = C(rows[t], cols[t]). */
void oracle_gemm_entries_f64(char ta, char tb, int64_t k, double alpha,
                             const double *A, int64_t lda,
                             const double *B, int64_t ldb, double beta,
                             const double *C0, int64_t ldc0,
                             int64_t count, const int64_t *rows,
                             const int64_t *cols, double *out)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0.0) && (k > 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = rows[t], j = cols[t];
        double s = 0.0;
        if (form)
            for (int64_t p = 0; p < k; ++p)
                s += (at ? A[p * lda + i] : A[i * lda + p]) *
                     (bt ? B[j * ldb + p] : B[p * ldb + j]);
        double v = form ? alpha * s : 0.0;
        if (beta != 0.0) v += beta * C0[i * ldc0 + j];
        out[t] = v;
    }
}

/* ---------------------------------------------------------------------- */
/* Split-product form: op(A) = sum_u PA[u], op(B) = sum_v PB[v] (pieces     */
/* stored with the same lda/ldb), and only the listed (u,v) piece products */
/* are formed:  C = alpha * sum_p sum_t PA[u_t](i,p) PB[v_t](p,j) + beta*C0 */
/* The inner sum over the listed pairs is taken for each p in list order.   */
/* ---------------------------------------------------------------------- */
void oracle_gemm_pieces_f64(char ta, char tb, int64_t m, int64_t n, int64_t k,
                            double alpha, int npa, const double *const *PA, int64_t lda,
                            int npb, const double *const *PB, int64_t ldb,
                            int nterms, const int *tu, const int *tv,
                            double beta, const double *C0, int64_t ldc0,
                            double *C, int64_t ldc)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0.0) && (k > 0);
    (void)npa; (void)npb;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        double acc[CHUNK];
        for (int64_t j0 = 0; j0 < n; j0 += CHUNK) {
            const int64_t jn = (n - j0 < CHUNK) ? n - j0 : CHUNK;
            for (int64_t j = 0; j < jn; ++j) acc[j] = 0.0;
            if (form) {
                for (int64_t p = 0; p < k; ++p) {
                    for (int t = 0; t < nterms; ++t) {
                        const double *Ap = PA[tu[t]], *Bp = PB[tv[t]];
                        const double a = at ? Ap[p * lda + i] : Ap[i * lda + p];
                        for (int64_t j = 0; j < jn; ++j) {
                            const double b = bt ? Bp[(j0 + j) * ldb + p] : Bp[p * ldb + (j0 + j)];
                            acc[j] += a * b;
                        }
                    }
                }
            }
            for (int64_t j = 0; j < jn; ++j) {
                double v = form ? alpha * acc[j] : 0.0;
                if (beta != 0.0) v += beta * C0[i * ldc0 + (j0 + j)];
                C[i * ldc + (j0 + j)] = v;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* INT8 GEMM: exact int64 sums, then alpha*acc + beta*C0 in int64, wrapped  */
/* to int32 by keeping the low 32 bits (two's complement).                  */
/* ---------------------------------------------------------------------- */
static int32_t wrap32(int64_t v)
{
    uint32_t u = (uint32_t)((uint64_t)v & 0xFFFFFFFFull);
    int32_t r;
    memcpy(&r, &u, sizeof r);
    return r;
}

void oracle_gemm_i8(char ta, char tb, int64_t m, int64_t n, int64_t k,
                    int64_t alpha, const int8_t *A, int64_t lda,
                    const int8_t *B, int64_t ldb, int64_t beta,
                    const int32_t *C0, int64_t ldc0, int32_t *C, int64_t ldc)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0) && (k > 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        int64_t acc[CHUNK];
        for (int64_t j0 = 0; j0 < n; j0 += CHUNK) {
            const int64_t jn = (n - j0 < CHUNK) ? n - j0 : CHUNK;
            for (int64_t j = 0; j < jn; ++j) acc[j] = 0;
            if (form) {
                for (int64_t p = 0; p < k; ++p) {
                    const int64_t a = at ? A[p * lda + i] : A[i * lda + p];
                    for (int64_t j = 0; j < jn; ++j) {
                        const int64_t b = bt ? B[(j0 + j) * ldb + p] : B[p * ldb + (j0 + j)];
                        acc[j] += a * b;
                    }
                }
            }
            for (int64_t j = 0; j < jn; ++j) {
                /* unsigned arithmetic: the low 32 bits of the exact value */
                uint64_t v = form ? (uint64_t)alpha * (uint64_t)acc[j] : 0u;
                if (beta != 0) v += (uint64_t)beta * (uint64_t)(int64_t)C0[i * ldc0 + (j0 + j)];
                C[i * ldc + (j0 + j)] = wrap32((int64_t)v);
            }
        }
    }
}

void oracle_gemm_entries_i8(char ta, char tb, int64_t k, int64_t alpha,
                            const int8_t *A, int64_t lda,
                            const int8_t *B, int64_t ldb, int64_t beta,
                            const int32_t *C0, int64_t ldc0,
                            int64_t count, const int64_t *rows,
                            const int64_t *cols, int32_t *out)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0) && (k > 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = rows[t], j = cols[t];
        int64_t s = 0;
        if (form)
            for (int64_t p = 0; p < k; ++p)
                s += (int64_t)(at ? A[p * lda + i] : A[i * lda + p]) *
                     (int64_t)(bt ? B[j * ldb + p] : B[p * ldb + j]);
        uint64_t v = form ? (uint64_t)alpha * (uint64_t)s : 0u;
        if (beta != 0) v += (uint64_t)beta * (uint64_t)(int64_t)C0[i * ldc0 + j];
        out[t] = wrap32((int64_t)v);
    }
}

/* ---------------------------------------------------------------------- */
/* INT16 and INT32 GEMM (the paper's 16- and 32-bit integer routines of its */
/* data-type study, section 8.5).  A and B hold int16 (ebytes 2) or int32   */
/* (ebytes 4) values; C0 and C are int32.  The result is the exact integer  */
/* alpha * sum_p op(A)(i,p) op(B)(p,j) + beta * C0(i,j) reduced modulo 2^32 */
/* (two's complement).  It is computed in unsigned 64-bit arithmetic, which */
/* wraps modulo 2^64 and so keeps the low 32 bits of every product and sum  */
/* exact.  alpha and beta are int32 values.                                  */
/* ---------------------------------------------------------------------- */
static int64_t int_at(const void *X, int ebytes, int64_t idx)
{
    if (ebytes == 2) return ((const int16_t *)X)[idx];
    return ((const int32_t *)X)[idx];
}

static int32_t low32(uint64_t v)
{
    uint32_t u = (uint32_t)(v & 0xFFFFFFFFull);
    int32_t r;
    memcpy(&r, &u, sizeof r);
    return r;
}

void oracle_gemm_int(int ebytes, char ta, char tb, int64_t m, int64_t n, int64_t k,
                     int64_t alpha, const void *A, int64_t lda,
                     const void *B, int64_t ldb, int64_t beta,
                     const int32_t *C0, int64_t ldc0, int32_t *C, int64_t ldc)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0) && (k > 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; ++i) {
        uint64_t acc[CHUNK];
        for (int64_t j0 = 0; j0 < n; j0 += CHUNK) {
            const int64_t jn = (n - j0 < CHUNK) ? n - j0 : CHUNK;
            for (int64_t j = 0; j < jn; ++j) acc[j] = 0u;
            if (form) {
                for (int64_t p = 0; p < k; ++p) {
                    const uint64_t a = (uint64_t)int_at(A, ebytes, at ? p * lda + i : i * lda + p);
                    for (int64_t j = 0; j < jn; ++j) {
                        const uint64_t b =
                            (uint64_t)int_at(B, ebytes, bt ? (j0 + j) * ldb + p : p * ldb + (j0 + j));
                        acc[j] += a * b;
                    }
                }
            }
            for (int64_t j = 0; j < jn; ++j) {
                uint64_t v = form ? (uint64_t)alpha * acc[j] : 0u;
                if (beta != 0) v += (uint64_t)beta * (uint64_t)(int64_t)C0[i * ldc0 + (j0 + j)];
                C[i * ldc + (j0 + j)] = low32(v);
            }
        }
    }
}

/* Selected entries of the same definition: out[t] = C(rows[t], cols[t]). */
void oracle_gemm_entries_int(int ebytes, char ta, char tb, int64_t k, int64_t alpha,
                             const void *A, int64_t lda, const void *B, int64_t ldb,
                             int64_t beta, const int32_t *C0, int64_t ldc0,
                             int64_t count, const int64_t *rows, const int64_t *cols,
                             int32_t *out)
{
    const int at = is_t(ta), bt = is_t(tb);
    const int form = (alpha != 0) && (k > 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = rows[t], j = cols[t];
        uint64_t s = 0u;
        if (form)
            for (int64_t p = 0; p < k; ++p)
                s += (uint64_t)int_at(A, ebytes, at ? p * lda + i : i * lda + p) *
                     (uint64_t)int_at(B, ebytes, bt ? j * ldb + p : p * ldb + j);
        uint64_t v = form ? (uint64_t)alpha * s : 0u;
        if (beta != 0) v += (uint64_t)beta * (uint64_t)(int64_t)C0[i * ldc0 + j];
        out[t] = low32(v);
    }
}


/* ---------------------------------------------------------------------- */
/* Number formats.                                                          */
/* ---------------------------------------------------------------------- */

/* bfloat16 is the upper half of an IEEE binary32: decode by placing the 16 */
/* bits in the high half of a 32-bit pattern.                               */
void oracle_decode_bf16(const uint16_t *x, int64_t n, double *out)
{
    for (int64_t t = 0; t < n; ++t) {
        uint32_t u = (uint32_t)x[t] << 16;
        float f;
        memcpy(&f, &u, sizeof f);
        out[t] = (double)f;
    }
}

/* IEEE binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits. */
void oracle_decode_f16(const uint16_t *x, int64_t n, double *out)
{
    for (int64_t t = 0; t < n; ++t) {
        const uint16_t h = x[t];
        const int s = h >> 15, e = (h >> 10) & 0x1F, f = h & 0x3FF;
        double v;
        if (e == 0)
            v = ldexp((double)f, -24);             /* subnormal: f * 2^-14 * 2^-10 */
        else if (e == 31)
            v = f ? NAN : INFINITY;
        else
            v = ldexp(1.0 + (double)f / 1024.0, e - 15);
        out[t] = s ? -v : v;
    }
}

/* OCP 8-bit E4M3FN: 1 sign bit, 4 exponent bits (bias 7), 3 fraction bits.  */
/* No infinities; exponent 15 with fraction 7 is NaN, so the largest finite */
/* magnitude is 1.75 * 2^8 = 448.  Exponent 0 is subnormal: f * 2^-9.       */
void oracle_decode_e4m3(const uint8_t *x, int64_t n, double *out)
{
    for (int64_t t = 0; t < n; ++t) {
        const uint8_t b = x[t];
        const int s = b >> 7, e = (b >> 3) & 0xF, f = b & 0x7;
        double v;
        if (e == 15 && f == 7)
            v = NAN;
        else if (e == 0)
            v = ldexp((double)f, -9);
        else
            v = ldexp(1.0 + (double)f / 8.0, e - 7);
        out[t] = s ? -v : v;
    }
}

/* Round an FP32 value to bfloat16, round-to-nearest, ties to even, on the  */
/* bit pattern: add 0x7FFF plus the lowest kept bit, then drop 16 bits.     */
/* NaN stays a (quiet) NaN.  Overflow rounds to infinity as IEEE requires.   */
static uint16_t rne_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
        return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

static float bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

/* Split x into `pieces` bf16 values:  hi = RNE(x),  mid = RNE(x - hi),     */
/* lo = RNE(x - hi - mid).  Each residual is formed in FP32, which is exact */
/* here because it is a difference of nearby FP32 values.                   */
void oracle_split_bf16(const float *x, int64_t n, int pieces, uint16_t *hi,
                       uint16_t *mid, uint16_t *lo)
{
    for (int64_t t = 0; t < n; ++t) {
        float r = x[t];
        const uint16_t h = rne_bf16(r);
        hi[t] = h;
        if (pieces < 2) continue;
        r = r - bf16_to_f32(h);
        const uint16_t md = rne_bf16(r);
        mid[t] = md;
        if (pieces < 3) continue;
        r = r - bf16_to_f32(md);
        lo[t] = rne_bf16(r);
    }
}

/* ------------------------------------------------------------------------ */
/* Power-of-two scaled quantisation (the scaled low-precision GEMM).         */
/* A row r of x (rows x cols, row-major) gets the exponent                   */
/*     e_r = floor(log2(M_r)) - T,   M_r = max_p |x[r][p]|,                   */
/* so that M_r * 2^-e_r lies in [2^T, 2^(T+1)); e_r = 0 when M_r is zero or  */
/* not finite.  Each value is then scaled by 2^-e_r in FP32 and rounded to   */
/* the narrow format, to nearest, ties to even.                              */
/* ------------------------------------------------------------------------ */
void oracle_scale_exponents(const float *x, int64_t rows, int64_t cols, int T, int32_t *e)
{
    for (int64_t r = 0; r < rows; ++r) {
        float mx = 0.0f;
        int finite = 1;
        for (int64_t p = 0; p < cols; ++p) {
            const float a = fabsf(x[r * cols + p]);
            if (!isfinite(a)) finite = 0;
            else if (a > mx) mx = a;
        }
        if (!finite || mx == 0.0f) {
            e[r] = 0;
            continue;
        }
        int ex;
        frexpf(mx, &ex);          /* mx = f * 2^ex, f in [0.5, 1) */
        e[r] = (ex - 1) - T;
    }
}

/* binary16, round to nearest even: subnormals are multiples of 2^-24,     */
/* normals 1.f * 2^E with E in [-14, 15] and 10 fraction bits.             */
static uint16_t rne_f16(float y)
{
    const uint16_t s = signbit(y) ? 0x8000u : 0u;
    const float a = fabsf(y);
    if (isnan(a)) return (uint16_t)(s | 0x7E00u);
    if (a == 0.0f) return s;
    if (a < 0x1p-14f) return (uint16_t)(s | (uint16_t)nearbyintf(a * 0x1p24f));
    int ex;
    frexpf(a, &ex);
    int E = ex - 1;
    const float mant = ldexpf(a, -E) - 1.0f;            /* in [0, 1), exact */
    int q = (int)nearbyintf(mant * 1024.0f);
    if (q == 1024) {
        q = 0;
        ++E;
    }
    if (E > 15) return (uint16_t)(s | 0x7C00u);         /* overflow: infinity */
    return (uint16_t)(s | ((E + 15) << 10) | q);
}

/* OCP E4M3FN, round to nearest even, saturating at 448 (no infinities):   */
/* subnormals are multiples of 2^-9, normals 1.f * 2^E, E in [-6, 8],      */
/* 3 fraction bits.                                                          */
static uint8_t rne_e4m3(float y)
{
    const uint8_t s = signbit(y) ? 0x80u : 0u;
    const float a = fabsf(y);
    if (isnan(a)) return (uint8_t)(s | 0x7Fu);
    if (a == 0.0f) return s;
    if (a < 0x1p-6f) return (uint8_t)(s | (uint8_t)nearbyintf(a * 0x1p9f));
    int ex;
    frexpf(a, &ex);
    int E = ex - 1;
    const float mant = ldexpf(a, -E) - 1.0f;
    int q = (int)nearbyintf(mant * 8.0f);
    if (q == 8) {
        q = 0;
        ++E;
    }
    int code = ((E + 7) << 3) | q;
    if (E > 8 || code > 0x7E) code = 0x7E;               /* saturate to 448 */
    return (uint8_t)(s | code);
}

/* Codes of x (rows x cols) scaled by 2^-e[r] per row.  fmt: 0 bfloat16,   */
/* 1 binary16, 2 E4M3FN (one byte per code, stored in the low byte).       */
void oracle_scaled_codes(const float *x, int64_t rows, int64_t cols, const int32_t *e, int fmt,
                         uint16_t *out)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t p = 0; p < cols; ++p) {
            const float y = ldexpf(x[r * cols + p], -e[r]);
            out[r * cols + p] = fmt == 0 ? rne_bf16(y) : (fmt == 1 ? rne_f16(y) : rne_e4m3(y));
        }
}
