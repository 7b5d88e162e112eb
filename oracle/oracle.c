/*
 * oracle.c -- plain CPU reference ("oracle") for the out-of-core compressed
 * stencil path of Shen, Wu, Okita, Ino, "Accelerating GPU-Based Out-of-Core
 * Stencil Computation with On-the-Fly Compression" (arXiv 2109.05410).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU library shares
 * no source, header, table or helper with it.
 *
 * What it computes, each written as the plain definition:
 *   - heat7:   the 3D seven-point analogue of the Laplace/heat stencil of
 *              Sec. III (Fig. 1a describes the five-point 2D case).
 *              u' = u + a*((xm+xp)+(ym+yp)+(zm+zp) - 6u), zero Dirichlet
 *              ghosts outside the grid.
 *   - wave25:  the 25-point acoustic propagator of Sec. VI (radius HALO=4,
 *              Table I): 8th-order central second derivative on each axis,
 *              two time levels (leapfrog), one read-only coefficient field
 *              w = (v dt/dx)^2, zero ghosts of width 4.
 *   - codec:   fixed-rate compression with a user-chosen number of bits per
 *              value (Sec. IV), the 4x4x4 block transform coder of
 *              P. Lindstrom, "Fixed-Rate Compressed Floating-Point Arrays",
 *              IEEE TVCG 20(12), 2014, in the exact format stated in the
 *              header comment of the codec section below.
 *   - replay:  the compressed out-of-core schedule of Sec. V-A reaches the
 *              same state as "k plain steps, then decode(encode(.)) of every
 *              compressed field", repeated per residency (see replay_*).
 *
 * Every floating-point path has an FP64 version (the accuracy reference) and
 * an FP32 version with a fixed operation order and no fused multiply-add, so
 * that an FP32 computation in that same order can be compared bit for bit.
 * Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, l, nx, ny) ((size_t)(i) + (size_t)(nx) * ((size_t)(j) + (size_t)(ny) * (size_t)(l)))

int orc_version(void) { return 1; }

/* ------------------------------------------------------------------------ */
/* Heat, seven-point Jacobi, zero Dirichlet ghosts (Sec. III, Fig. 1a).     */
/* ------------------------------------------------------------------------ */

static double at_f64(const double* u, long i, long j, long l, long nx, long ny, long nz)
{
    if (i < 0 || j < 0 || l < 0 || i >= nx || j >= ny || l >= nz) return 0.0;
    return u[IDX(i, j, l, nx, ny)];
}

static float at_f32(const float* u, long i, long j, long l, long nx, long ny, long nz)
{
    if (i < 0 || j < 0 || l < 0 || i >= nx || j >= ny || l >= nz) return 0.0f;
    return u[IDX(i, j, l, nx, ny)];
}

/* One or more steps, in place (a temporary holds the new level). */
int orc_heat7_f64(double* u, long nx, long ny, long nz, double alpha, long steps)
{
    size_t n = (size_t)nx * ny * nz;
    double* t = (double*)malloc(n * sizeof(double));
    if (!t) return -1;
    for (long s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(static)
        for (long l = 0; l < nz; ++l)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) {
                    double c = u[IDX(i, j, l, nx, ny)];
                    double sum = (at_f64(u, i - 1, j, l, nx, ny, nz) + at_f64(u, i + 1, j, l, nx, ny, nz))
                               + (at_f64(u, i, j - 1, l, nx, ny, nz) + at_f64(u, i, j + 1, l, nx, ny, nz));
                    sum = sum + (at_f64(u, i, j, l - 1, nx, ny, nz) + at_f64(u, i, j, l + 1, nx, ny, nz));
                    sum = sum - 6.0 * c;
                    t[IDX(i, j, l, nx, ny)] = c + alpha * sum;
                }
        memcpy(u, t, n * sizeof(double));
    }
    free(t);
    return 0;
}

/* FP32 with the operation order fixed as:
 *   s = (xm + xp) + (ym + yp);  s = s + (zm + zp);  s = s - 6*c;  u' = c + alpha*s */
int orc_heat7_f32(float* u, long nx, long ny, long nz, float alpha, long steps)
{
    size_t n = (size_t)nx * ny * nz;
    float* t = (float*)malloc(n * sizeof(float));
    if (!t) return -1;
    for (long s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(static)
        for (long l = 0; l < nz; ++l)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) {
                    float c = u[IDX(i, j, l, nx, ny)];
                    float sum = (at_f32(u, i - 1, j, l, nx, ny, nz) + at_f32(u, i + 1, j, l, nx, ny, nz))
                              + (at_f32(u, i, j - 1, l, nx, ny, nz) + at_f32(u, i, j + 1, l, nx, ny, nz));
                    sum = sum + (at_f32(u, i, j, l - 1, nx, ny, nz) + at_f32(u, i, j, l + 1, nx, ny, nz));
                    sum = sum - 6.0f * c;
                    t[IDX(i, j, l, nx, ny)] = c + alpha * sum;
                }
        memcpy(u, t, n * sizeof(float));
    }
    free(t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Acoustic wave, 25 points (Sec. VI; HALO = 4 in Table I).                 */
/*   p(n+1) = 2 p(n) - p(n-1) + w * L p(n) + s(n) * delta(src)              */
/*   L p = 3*c0*p + sum_{m=1..4} c_m * S_m,  S_m = sum over the 3 axes of   */
/*         (p[+m] + p[-m]).                                                 */
/* Coefficients: 8th-order central second difference (Fornberg 1988):       */
/*   c0 = -205/72, c1 = 8/5, c2 = -1/5, c3 = 8/315, c4 = -1/560.            */
/* ------------------------------------------------------------------------ */

static const double W_C0X3 = -205.0 / 24.0; /* 3*c0 */
static const double W_C[5] = {0.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

/* Laplacian in grid-index units (dx absorbed into w), FP64. */
int orc_lap25_f64(const double* p, double* out, long nx, long ny, long nz)
{
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nz; ++l)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                double acc = W_C0X3 * p[IDX(i, j, l, nx, ny)];
                for (int m = 1; m <= 4; ++m) {
                    double sm = (at_f64(p, i + m, j, l, nx, ny, nz) + at_f64(p, i - m, j, l, nx, ny, nz))
                              + (at_f64(p, i, j + m, l, nx, ny, nz) + at_f64(p, i, j - m, l, nx, ny, nz));
                    sm = sm + (at_f64(p, i, j, l + m, nx, ny, nz) + at_f64(p, i, j, l - m, nx, ny, nz));
                    acc = acc + W_C[m] * sm;
                }
                out[IDX(i, j, l, nx, ny)] = acc;
            }
    return 0;
}

/* steps of the leapfrog. On entry (pm, p) = (p(n-1), p(n)); on exit
 * (pm, p) = (p(n+steps-1), p(n+steps)). src[s] is the source amplitude added
 * at cell src_index when p(n+s+1) is formed; src may be NULL (no source). */
int orc_wave25_f64(double* p, double* pm, const double* w, long nx, long ny, long nz, long steps,
                   const double* src, long src_index)
{
    size_t n = (size_t)nx * ny * nz;
    double* lp = (double*)malloc(n * sizeof(double));
    if (!lp) return -1;
    for (long s = 0; s < steps; ++s) {
        orc_lap25_f64(p, lp, nx, ny, nz);
#pragma omp parallel for schedule(static)
        for (long c = 0; c < (long)n; ++c) {
            double pn = (2.0 * p[c] - pm[c]) + w[c] * lp[c];
            pm[c] = p[c];
            p[c] = pn;
        }
        if (src && src_index >= 0) p[src_index] = p[src_index] + src[s];
    }
    free(lp);
    return 0;
}

/* FP32, operation order fixed as:
 *   acc = C0X3*p;  for m = 1..4: S = ((x+m + x-m) + (y+m + y-m)) + (z+m + z-m); acc = acc + C_m*S
 *   p'  = (2*p - pm) + w*acc;   at the source cell: p' = p' + s
 * with the coefficients rounded once from the exact fractions to FP32. */
int orc_wave25_f32(float* p, float* pm, const float* w, long nx, long ny, long nz, long steps,
                   const float* src, long src_index)
{
    const float c0x3 = (float)(-205.0 / 24.0);
    const float cm[5] = {0.0f, (float)(8.0 / 5.0), (float)(-1.0 / 5.0), (float)(8.0 / 315.0), (float)(-1.0 / 560.0)};
    size_t n = (size_t)nx * ny * nz;
    float* pn = (float*)malloc(n * sizeof(float));
    if (!pn) return -1;
    for (long s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(static)
        for (long l = 0; l < nz; ++l)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) {
                    size_t c = IDX(i, j, l, nx, ny);
                    float acc = c0x3 * p[c];
                    for (int m = 1; m <= 4; ++m) {
                        float sm = (at_f32(p, i + m, j, l, nx, ny, nz) + at_f32(p, i - m, j, l, nx, ny, nz))
                                 + (at_f32(p, i, j + m, l, nx, ny, nz) + at_f32(p, i, j - m, l, nx, ny, nz));
                        sm = sm + (at_f32(p, i, j, l + m, nx, ny, nz) + at_f32(p, i, j, l - m, nx, ny, nz));
                        acc = acc + cm[m] * sm;
                    }
                    float v = (2.0f * p[c] - pm[c]) + w[c] * acc;
                    if (src && (long)c == src_index) v = v + src[s];
                    pn[c] = v;
                }
        memcpy(pm, p, n * sizeof(float));
        memcpy(p, pn, n * sizeof(float));
    }
    free(pn);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fixed-rate 4^3 block transform codec (Sec. IV; Lindstrom 2014).          */
/*                                                                          */
/* Format (one block of 64 FP32 values, `rate` bits per value, so exactly   */
/* 64*rate bits per block, stored at 64-bit word offset b*rate):            */
/*  1. values ordered i + 4j + 16l inside the block; blocks of a field are  */
/*     ordered x fastest, then y, then z.                                   */
/*  2. e(x) = exponent of frexp (x = f 2^e, f in [1/2,1)), clamped below at */
/*     -126; e(0) = -inf. emax = max e over the block. If every value is    */
/*     zero the block is one 0 bit followed by zero padding. Otherwise the  */
/*     header is a 1 bit and the 8-bit field emax+127, least significant    */
/*     bit first.                                                           */
/*  3. q = trunc(x * 2^(30-emax)) as int32 (exact power-of-two scaling).    */
/*  4. forward lifting on every 4-vector (a,b,c,d) along x, then y, then z  */
/*     (>> is the arithmetic, flooring shift):                              */
/*        a=(a+d)>>1; d-=a;  c=(c+b)>>1; b-=c;  a=(a+c)>>1; c-=a;           */
/*        d=(d+b)>>1; b-=d;  d+=b>>1; b-=d>>1;                              */
/*     whose exact-arithmetic action is M/16, M = [[4,4,4,4],[5,1,-1,-5],   */
/*     [-4,4,4,-4],[-2,6,-6,2]] (Lindstrom 2014, Sec. 3).                   */
/*  5. reorder by total sequency i+j+l; ties by i^2+j^2+l^2, then by        */
/*     (l, j, i) lexicographically.                                         */
/*  6. negabinary: u = (q + 0xAAAAAAAA) ^ 0xAAAAAAAA (uint32 arithmetic).   */
/*  7. bit planes 31..0 with group testing, budget 64*rate-9 bits; n =      */
/*     number of coefficients already significant:                          */
/*       - emit bits 0..n-1 of the plane word X verbatim;                   */
/*       - while n < 64: emit g = [X has a 1 at a position >= n]; stop the  */
/*         plane if g = 0; otherwise emit X bits at n, n+1, ... (n grows    */
/*         with each) up to and including the first 1; when the scan       */
/*         reaches position 63 that bit is known to be 1: it is not emitted */
/*         and n becomes 64.                                                */
/*     Every emitted bit costs one unit of budget; coding stops the moment  */
/*     the budget is zero. Bits are written least significant first into   */
/*     little-endian 64-bit words; the rest of the block is zero.           */
/*  8. decoding reads the same sequence with the same budget; bits never    */
/*     read are zero (or, with mid-point reconstruction, see below). Then   */
/*     inverse negabinary, inverse reorder, the inverse                     */
/*     lifting along z, then y, then x:                                     */
/*        b+=d>>1; d-=b>>1;  b+=d; d=2d-b;  c+=a; a=2a-c;                    */
/*        b+=c; c=2c-b;  d+=a; a=2a-d;                                      */
/*     and x = (float)q * 2^(emax-30) (round to nearest even, then exact    */
/*     power-of-two scaling).                                               */
/*  9. mid-point reconstruction (a decoding option; the stream is the same): */
/*     when the budget ends inside the stream, the digits a coefficient did */
/*     not receive are its L lowest planes: L = P for the coefficients     */
/*     whose plane-P digit was read (or implied by a negative group test)  */
/*     and L = P + 1 for the others, P being the plane in which the budget */
/*     ran out with the plane incomplete (a plane that the last bit        */
/*     completes makes the next plane P with none read). A coefficient     */
/*     with a nonzero decoded digit then takes, instead of zero digits,    */
/*     the middle of the values those L digits can add: they add           */
/*     sum d_j (-2)^j, between the all-odd and all-even sums, whose middle */
/*     is half of the all-ones sum (1 - (-2)^L) / 3; it is added rounded  */
/*     down, in 32-bit wrap-around arithmetic, to the integer coefficient  */
/*     before the inverse transform. Coefficients decoded as zero stay     */
/*     zero. Nothing changes when the whole stream fits the budget.        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t emax;        /* block exponent; INT32_MIN for an all-zero block */
    int32_t q[64];       /* block-floating-point integers, natural order */
    int32_t t[64];       /* after the forward transform, natural order */
    uint32_t u[64];      /* reordered (sequency order) and negabinary */
    uint64_t plane[32];  /* plane[p] = word X of bit plane p (bit i = bit p of u[i]) */
    int32_t bits_used;   /* bits written before padding, header included */
    int32_t stop_plane;  /* decode: plane P in which the budget ran out (-1: stream complete) */
    int32_t stop_known;  /* decode: coefficients (sequency order) whose plane-P digit is known */
} orc_stages;

static int g_perm_ready = 0;
static int g_perm[64]; /* g_perm[k] = natural index i+4j+16l of the k-th coefficient */

static void build_perm(void)
{
    if (g_perm_ready) return;
    /* simple selection: repeatedly take the smallest remaining key */
    int used[64] = {0};
    for (int k = 0; k < 64; ++k) {
        int best = -1;
        long bestkey = 0;
        for (int idx = 0; idx < 64; ++idx) {
            if (used[idx]) continue;
            int i = idx & 3, j = (idx >> 2) & 3, l = idx >> 4;
            long key = ((long)(i + j + l) << 24) | ((long)(i * i + j * j + l * l) << 12) | ((long)l << 8) | ((long)j << 4) | (long)i;
            if (best < 0 || key < bestkey) { best = idx; bestkey = key; }
        }
        used[best] = 1;
        g_perm[k] = best;
    }
    g_perm_ready = 1;
}

int orc_codec_perm(int32_t* out64)
{
    build_perm();
    for (int k = 0; k < 64; ++k) out64[k] = g_perm[k];
    return 0;
}

/* 64-bit signed arithmetic with range checks: the format is defined on
 * int32, and every intermediate of both lifting passes stays inside int32
 * for |q| < 2^30; a violation is reported instead of silently wrapping. */
static _Thread_local int g_range_violation = 0;
static int64_t chk(int64_t v)
{
    if (v > INT32_MAX || v < INT32_MIN) g_range_violation = 1;
    return v;
}
static int64_t asr1(int64_t v) { return v >> 1; } /* arithmetic shift (floor) on int64 */

static void fwd4(int64_t* a, int64_t* b, int64_t* c, int64_t* d)
{
    int64_t A = *a, B = *b, C = *c, D = *d;
    A = chk(asr1(chk(A + D))); D = chk(D - A);
    C = chk(asr1(chk(C + B))); B = chk(B - C);
    A = chk(asr1(chk(A + C))); C = chk(C - A);
    D = chk(asr1(chk(D + B))); B = chk(B - D);
    D = chk(D + asr1(B));      B = chk(B - asr1(D));
    *a = A; *b = B; *c = C; *d = D;
}

static void inv4(int64_t* a, int64_t* b, int64_t* c, int64_t* d)
{
    int64_t A = *a, B = *b, C = *c, D = *d;
    B = chk(B + asr1(D)); D = chk(D - asr1(B));
    B = chk(B + D);       D = chk(2 * D - B);
    C = chk(C + A);       A = chk(2 * A - C);
    B = chk(B + C);       C = chk(2 * C - B);
    D = chk(D + A);       A = chk(2 * A - D);
    *a = A; *b = B; *c = C; *d = D;
}

/* Apply a 4-point lifting to every line of the block along `axis` (0=x,1=y,2=z). */
static void lift_axis(int64_t* v, int axis, int inverse)
{
    int stride = axis == 0 ? 1 : (axis == 1 ? 4 : 16);
    for (int o1 = 0; o1 < 4; ++o1)
        for (int o2 = 0; o2 < 4; ++o2) {
            int base;
            if (axis == 0) base = 4 * o1 + 16 * o2;
            else if (axis == 1) base = o1 + 16 * o2;
            else base = o1 + 4 * o2;
            int64_t* a = &v[base];
            int64_t* b = &v[base + stride];
            int64_t* c = &v[base + 2 * stride];
            int64_t* d = &v[base + 3 * stride];
            if (inverse) inv4(a, b, c, d); else fwd4(a, b, c, d);
        }
}

int orc_fwd_xform(const int32_t* in64, int32_t* out64)
{
    int64_t v[64];
    g_range_violation = 0;
    for (int i = 0; i < 64; ++i) v[i] = in64[i];
    lift_axis(v, 0, 0); lift_axis(v, 1, 0); lift_axis(v, 2, 0);
    for (int i = 0; i < 64; ++i) out64[i] = (int32_t)v[i];
    return g_range_violation ? -2 : 0;
}

int orc_inv_xform(const int32_t* in64, int32_t* out64)
{
    int64_t v[64];
    g_range_violation = 0;
    for (int i = 0; i < 64; ++i) v[i] = in64[i];
    lift_axis(v, 2, 1); lift_axis(v, 1, 1); lift_axis(v, 0, 1);
    for (int i = 0; i < 64; ++i) out64[i] = (int32_t)v[i];
    return g_range_violation ? -2 : 0;
}

static int exponent_of(float x)
{
    int e;
    (void)frexpf(x, &e);
    return e < -126 ? -126 : e;
}

/* bit writer / reader over a zero-initialised block of words */
typedef struct { uint64_t* w; long pos; } bitw;
typedef struct { const uint64_t* w; long pos; } bitr;
static void put1(bitw* s, int b) { if (b) s->w[s->pos >> 6] |= (uint64_t)1 << (s->pos & 63); s->pos++; }
static int get1(bitr* s) { int b = (int)((s->w[s->pos >> 6] >> (s->pos & 63)) & 1u); s->pos++; return b; }

/* Encode the 64 sequency-ordered negabinary coefficients; returns bits used. */
static long code_planes(const uint32_t* u, long budget, bitw* s, uint64_t* planes_out)
{
    long used = 0;
    int n = 0;
    for (int p = 31; p >= 0; --p) {
        uint64_t X = 0;
        for (int i = 0; i < 64; ++i) X |= (uint64_t)((u[i] >> p) & 1u) << i;
        if (planes_out) planes_out[p] = X;
        if (budget <= 0) continue;
        /* verbatim part */
        for (int i = 0; i < n && budget > 0; ++i) { put1(s, (int)((X >> i) & 1u)); budget--; used++; }
        /* group tests */
        while (n < 64 && budget > 0) {
            int g = (X >> n) != 0;
            put1(s, g); budget--; used++;
            if (!g) break;
            for (;;) {
                if (n == 63) { n = 64; break; }
                if (budget <= 0) break;
                int b = (int)((X >> n) & 1u);
                put1(s, b); budget--; used++;
                n++;
                if (b) break;
            }
        }
    }
    return used;
}

/* Decodes the planes; *stop_plane / *stop_known say where the budget ran
 * out (format step 9): `known` counts the coefficients (a prefix in
 * sequency order) whose digit of the current plane has been read or
 * implied, 64 once the plane is complete. */
static void decode_planes(uint32_t* u, long budget, bitr* s, uint64_t* planes_out, int* stop_plane, int* stop_known)
{
    int n = 0;
    *stop_plane = -1;
    *stop_known = 0;
    for (int i = 0; i < 64; ++i) u[i] = 0;
    for (int p = 31; p >= 0; --p) {
        uint64_t X = 0;
        if (budget > 0) {
            int known = 0;
            for (int i = 0; i < n && budget > 0; ++i) { X |= (uint64_t)get1(s) << i; budget--; known = i + 1; }
            while (n < 64 && budget > 0) {
                int g = get1(s); budget--;
                if (!g) { known = 64; break; }   /* every digit left in the plane is 0 */
                for (;;) {
                    if (n == 63) { X |= (uint64_t)1 << 63; n = 64; known = 64; break; }
                    if (budget <= 0) break;
                    int b = get1(s); budget--;
                    known = n + 1;
                    if (b) { X |= (uint64_t)1 << n; n++; break; }
                    n++;
                }
            }
            if (budget <= 0 && *stop_plane < 0) {
                if (known < 64) { *stop_plane = p; *stop_known = known; }
                else if (p > 0) { *stop_plane = p - 1; *stop_known = 0; }
            }
        }
        if (planes_out) planes_out[p] = X;
        for (int i = 0; i < 64; ++i) u[i] |= (uint32_t)((X >> i) & 1u) << p;
    }
}

/* Half of the all-ones sum of L negabinary digits, (1 - (-2)^L) / 3,
 * rounded down (format step 9). */
static int64_t midpoint_offset(int L)
{
    int64_t m = 1;
    for (int j = 0; j < L; ++j) m *= -2;
    const int64_t all_ones = (1 - m) / 3;
    return all_ones >= 0 ? all_ones / 2 : -((-all_ones + 1) / 2);
}

/* One block: in64 natural order -> rate words. st may be NULL. */
int orc_encode_block(const float* in64, int rate, uint64_t* out, orc_stages* st)
{
    if (rate < 1 || rate > 64) return -1;
    build_perm();
    memset(out, 0, (size_t)rate * sizeof(uint64_t));
    orc_stages local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    int nonzero = 0, emax = -100000;
    for (int i = 0; i < 64; ++i)
        if (in64[i] != 0.0f) {
            nonzero = 1;
            int e = exponent_of(in64[i]);
            if (e > emax) emax = e;
        }
    bitw s = {out, 0};
    if (!nonzero) {
        st->emax = INT32_MIN;
        put1(&s, 0);
        st->bits_used = 1;
        return 0;
    }
    st->emax = emax;
    put1(&s, 1);
    int biased = emax + 127;
    for (int b = 0; b < 8; ++b) put1(&s, (biased >> b) & 1);
    for (int i = 0; i < 64; ++i) st->q[i] = (int32_t)ldexpf(in64[i], 30 - emax); /* C conversion truncates */
    int rc = orc_fwd_xform(st->q, st->t);
    for (int k = 0; k < 64; ++k) {
        uint32_t v = (uint32_t)st->t[g_perm[k]];
        st->u[k] = (v + 0xAAAAAAAAu) ^ 0xAAAAAAAAu;
    }
    long used = code_planes(st->u, 64L * rate - 9, &s, st->plane);
    st->bits_used = (int32_t)(9 + used);
    return rc;
}

/* One block: rate words -> 64 floats, natural order; mid = 1 for mid-point
 * reconstruction (format step 9). st may be NULL (st->q then holds the
 * integers after the inverse transform). */
int orc_decode_block_mode(const uint64_t* in, int rate, int mid, float* out64, orc_stages* st)
{
    if (rate < 1 || rate > 64) return -1;
    build_perm();
    orc_stages local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    bitr s = {in, 0};
    if (!get1(&s)) {
        st->emax = INT32_MIN;
        for (int i = 0; i < 64; ++i) out64[i] = 0.0f;
        return 0;
    }
    int biased = 0;
    for (int b = 0; b < 8; ++b) biased |= get1(&s) << b;
    int emax = biased - 127;
    st->emax = emax;
    decode_planes(st->u, 64L * rate - 9, &s, st->plane, &st->stop_plane, &st->stop_known);
    for (int k = 0; k < 64; ++k) {
        uint32_t v = (st->u[k] ^ 0xAAAAAAAAu) - 0xAAAAAAAAu;
        if (mid && st->stop_plane >= 0 && st->u[k] != 0) {
            const int L = k < st->stop_known ? st->stop_plane : st->stop_plane + 1;
            v += (uint32_t)midpoint_offset(L);  /* wraps like int32 */
        }
        st->t[g_perm[k]] = (int32_t)v;
    }
    int rc = orc_inv_xform(st->t, st->q);
    for (int i = 0; i < 64; ++i) out64[i] = ldexpf((float)st->q[i], emax - 30);
    return rc;
}

int orc_decode_block(const uint64_t* in, int rate, float* out64, orc_stages* st)
{
    return orc_decode_block_mode(in, rate, 0, out64, st);
}

size_t orc_codec_words(long nx, long ny, long nz, int rate)
{
    return (size_t)(nx / 4) * (size_t)(ny / 4) * (size_t)(nz / 4) * (size_t)rate;
}

static void gather_block(const float* f, long nx, long ny, long bx, long by, long bz, float* blk)
{
    for (int l = 0; l < 4; ++l)
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i)
                blk[i + 4 * j + 16 * l] = f[IDX(4 * bx + i, 4 * by + j, 4 * bz + l, nx, ny)];
}

static void scatter_block(float* f, long nx, long ny, long bx, long by, long bz, const float* blk)
{
    for (int l = 0; l < 4; ++l)
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i)
                f[IDX(4 * bx + i, 4 * by + j, 4 * bz + l, nx, ny)] = blk[i + 4 * j + 16 * l];
}

/* Whole field (x fastest), dims multiples of 4. Returns 0, or -1 on bad args,
 * -2 if an integer intermediate left int32 (never expected). */
int orc_codec_encode(const float* f, long nx, long ny, long nz, int rate, uint64_t* out)
{
    if (nx % 4 || ny % 4 || nz % 4 || rate < 1 || rate > 64) return -1;
    long bxn = nx / 4, byn = ny / 4, bzn = nz / 4;
    int bad = 0;
    build_perm();
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long bz = 0; bz < bzn; ++bz)
        for (long by = 0; by < byn; ++by)
            for (long bx = 0; bx < bxn; ++bx) {
                float blk[64];
                gather_block(f, nx, ny, bx, by, bz, blk);
                size_t b = (size_t)bx + (size_t)bxn * ((size_t)by + (size_t)byn * (size_t)bz);
                orc_stages st;
                if (orc_encode_block(blk, rate, out + b * (size_t)rate, &st) != 0) bad = 1;
            }
    return bad ? -2 : 0;
}

int orc_codec_decode_mode(const uint64_t* in, long nx, long ny, long nz, int rate, int mid, float* f)
{
    if (nx % 4 || ny % 4 || nz % 4 || rate < 1 || rate > 64) return -1;
    long bxn = nx / 4, byn = ny / 4, bzn = nz / 4;
    int bad = 0;
    build_perm();
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long bz = 0; bz < bzn; ++bz)
        for (long by = 0; by < byn; ++by)
            for (long bx = 0; bx < bxn; ++bx) {
                float blk[64];
                size_t b = (size_t)bx + (size_t)bxn * ((size_t)by + (size_t)byn * (size_t)bz);
                orc_stages st;
                if (orc_decode_block_mode(in + b * (size_t)rate, rate, mid, blk, &st) != 0) bad = 1;
                scatter_block(f, nx, ny, bx, by, bz, blk);
            }
    return bad ? -2 : 0;
}

int orc_codec_decode(const uint64_t* in, long nx, long ny, long nz, int rate, float* f)
{
    return orc_codec_decode_mode(in, nx, ny, nz, rate, 0, f);
}

/* Q = decode(encode(.)) in place on an FP32 field (mid: format step 9). */
int orc_codec_roundtrip_mode(float* f, long nx, long ny, long nz, int rate, int mid)
{
    size_t nw = orc_codec_words(nx, ny, nz, rate);
    uint64_t* w = (uint64_t*)calloc(nw ? nw : 1, sizeof(uint64_t));
    if (!w) return -1;
    int rc = orc_codec_encode(f, nx, ny, nz, rate, w);
    if (rc == 0) rc = orc_codec_decode_mode(w, nx, ny, nz, rate, mid, f);
    free(w);
    return rc;
}

int orc_codec_roundtrip(float* f, long nx, long ny, long nz, int rate)
{
    return orc_codec_roundtrip_mode(f, nx, ny, nz, rate, 0);
}

/* FP64 field through the FP32 codec: round to FP32, Q, widen back. */
int orc_codec_roundtrip_f64_mode(double* f, long nx, long ny, long nz, int rate, int mid)
{
    size_t n = (size_t)nx * ny * nz;
    float* t = (float*)malloc(n * sizeof(float));
    if (!t) return -1;
    for (size_t i = 0; i < n; ++i) t[i] = (float)f[i];
    int rc = orc_codec_roundtrip_mode(t, nx, ny, nz, rate, mid);
    for (size_t i = 0; i < n; ++i) f[i] = (double)t[i];
    free(t);
    return rc;
}

int orc_codec_roundtrip_f64(double* f, long nx, long ny, long nz, int rate)
{
    return orc_codec_roundtrip_f64_mode(f, nx, ny, nz, rate, 0);
}

/* ------------------------------------------------------------------------ */
/* Replay of the compressed out-of-core schedule (Sec. V-A).                */
/*                                                                          */
/* Out-of-core decomposition with halos, region sharing and temporal        */
/* blocking computes every output cell from exactly the inputs the plain    */
/* stencil would use, so it is exact. What changes the numbers is where the */
/* data passes through the codec: each residency starts from the decoded    */
/* host store and ends by encoding the result back. So after `steps` steps  */
/* with k steps per residency the state is                                  */
/*     Q( F_k'( Q( F_k( ... Q( F_k( Q(u0) ) ) ... ) ) ) )                   */
/* where F_k is k plain steps, k' = the remainder for the last residency,   */
/* and Q = decode o encode applied to every compressed read-write field.    */
/* A read-only field is compressed once when the host store is built, so it */
/* enters every step as Q(w). rate 0 means "not compressed".                */
/* ------------------------------------------------------------------------ */

int orc_replay_heat_f32_mode(float* u, long nx, long ny, long nz, float alpha, long steps, long k, int rate, int mid)
{
    if (k < 1) return -1;
    int rc = 0;
    if (rate > 0 && (rc = orc_codec_roundtrip_mode(u, nx, ny, nz, rate, mid))) return rc;
    for (long done = 0; done < steps;) {
        long kk = steps - done < k ? steps - done : k;
        if ((rc = orc_heat7_f32(u, nx, ny, nz, alpha, kk))) return rc;
        if (rate > 0 && (rc = orc_codec_roundtrip_mode(u, nx, ny, nz, rate, mid))) return rc;
        done += kk;
    }
    return 0;
}

int orc_replay_heat_f32(float* u, long nx, long ny, long nz, float alpha, long steps, long k, int rate)
{
    return orc_replay_heat_f32_mode(u, nx, ny, nz, alpha, steps, k, rate, 0);
}

int orc_replay_heat_f64_mode(double* u, long nx, long ny, long nz, double alpha, long steps, long k, int rate, int mid)
{
    if (k < 1) return -1;
    int rc = 0;
    if (rate > 0 && (rc = orc_codec_roundtrip_f64_mode(u, nx, ny, nz, rate, mid))) return rc;
    for (long done = 0; done < steps;) {
        long kk = steps - done < k ? steps - done : k;
        if ((rc = orc_heat7_f64(u, nx, ny, nz, alpha, kk))) return rc;
        if (rate > 0 && (rc = orc_codec_roundtrip_f64_mode(u, nx, ny, nz, rate, mid))) return rc;
        done += kk;
    }
    return 0;
}

int orc_replay_heat_f64(double* u, long nx, long ny, long nz, double alpha, long steps, long k, int rate)
{
    return orc_replay_heat_f64_mode(u, nx, ny, nz, alpha, steps, k, rate, 0);
}

/* Wave: fields (pm, p) read-write at rates rate_pm / rate_p, w read-only at
 * rate_w (0 = raw). src holds one amplitude per step (may be NULL). */
int orc_replay_wave_f32_mode(float* p, float* pm, float* w, long nx, long ny, long nz, long steps, long k,
                        const float* src, long src_index, int rate_p, int rate_pm, int rate_w, int mid)
{
    if (k < 1) return -1;
    int rc = 0;
    if (rate_w > 0 && (rc = orc_codec_roundtrip_mode(w, nx, ny, nz, rate_w, mid))) return rc;
    if (rate_p > 0 && (rc = orc_codec_roundtrip_mode(p, nx, ny, nz, rate_p, mid))) return rc;
    if (rate_pm > 0 && (rc = orc_codec_roundtrip_mode(pm, nx, ny, nz, rate_pm, mid))) return rc;
    for (long done = 0; done < steps;) {
        long kk = steps - done < k ? steps - done : k;
        if ((rc = orc_wave25_f32(p, pm, w, nx, ny, nz, kk, src ? src + done : NULL, src_index))) return rc;
        if (rate_p > 0 && (rc = orc_codec_roundtrip_mode(p, nx, ny, nz, rate_p, mid))) return rc;
        if (rate_pm > 0 && (rc = orc_codec_roundtrip_mode(pm, nx, ny, nz, rate_pm, mid))) return rc;
        done += kk;
    }
    return 0;
}

int orc_replay_wave_f32(float* p, float* pm, float* w, long nx, long ny, long nz, long steps, long k,
                        const float* src, long src_index, int rate_p, int rate_pm, int rate_w)
{
    return orc_replay_wave_f32_mode(p, pm, w, nx, ny, nz, steps, k, src, src_index, rate_p, rate_pm, rate_w, 0);
}

int orc_replay_wave_f64_mode(double* p, double* pm, double* w, long nx, long ny, long nz, long steps, long k,
                        const double* src, long src_index, int rate_p, int rate_pm, int rate_w, int mid)
{
    if (k < 1) return -1;
    int rc = 0;
    if (rate_w > 0 && (rc = orc_codec_roundtrip_f64_mode(w, nx, ny, nz, rate_w, mid))) return rc;
    if (rate_p > 0 && (rc = orc_codec_roundtrip_f64_mode(p, nx, ny, nz, rate_p, mid))) return rc;
    if (rate_pm > 0 && (rc = orc_codec_roundtrip_f64_mode(pm, nx, ny, nz, rate_pm, mid))) return rc;
    for (long done = 0; done < steps;) {
        long kk = steps - done < k ? steps - done : k;
        if ((rc = orc_wave25_f64(p, pm, w, nx, ny, nz, kk, src ? src + done : NULL, src_index))) return rc;
        if (rate_p > 0 && (rc = orc_codec_roundtrip_f64_mode(p, nx, ny, nz, rate_p, mid))) return rc;
        if (rate_pm > 0 && (rc = orc_codec_roundtrip_f64_mode(pm, nx, ny, nz, rate_pm, mid))) return rc;
        done += kk;
    }
    return 0;
}

int orc_replay_wave_f64(double* p, double* pm, double* w, long nx, long ny, long nz, long steps, long k,
                        const double* src, long src_index, int rate_p, int rate_pm, int rate_w)
{
    return orc_replay_wave_f64_mode(p, pm, w, nx, ny, nz, steps, k, src, src_index, rate_p, rate_pm, rate_w, 0);
}

/* The bit-plane coder alone (step 7/8 above) on 64 sequency-ordered
 * negabinary words with an arbitrary budget in bits, writing from bit 0 of
 * out[] (which must hold ceil(budget/64) zeroed words). Exposed so that the
 * coder can be checked on integer inputs. Returns bits used. */
long orc_code_ints(const uint32_t* u64, long budget, uint64_t* out)
{
    bitw s = {out, 0};
    return code_planes(u64, budget, &s, NULL);
}

int orc_decode_ints(const uint64_t* in, long budget, uint32_t* u64)
{
    bitr s = {in, 0};
    int stop_plane, stop_known;
    decode_planes(u64, budget, &s, NULL, &stop_plane, &stop_known);
    return 0;
}

/* The same, also returning where the budget ran out (format step 9):
 * stop[0] = plane (-1 if the stream was complete), stop[1] = coefficients
 * whose digit of that plane is known. */
int orc_decode_ints_stop(const uint64_t* in, long budget, uint32_t* u64, int32_t* stop)
{
    bitr s = {in, 0};
    int stop_plane, stop_known;
    decode_planes(u64, budget, &s, NULL, &stop_plane, &stop_known);
    stop[0] = stop_plane;
    stop[1] = stop_known;
    return 0;
}


/* ------------------------------------------------------------------------ */
/* The fixed-rate method for FP64 values (the precision of the paper's      */
/* experiments, Sec. VI). Same blocks, lifting steps, sequency order, group */
/* testing and layout as the FP32 format above, with 64-bit integers:       */
/*  - e(x) from frexp, clamped below at -1022; header: a 1 bit and the      */
/*    11-bit field emax + 1023, least significant bit first (12 bits); an   */
/*    all-zero block is one 0 bit;                                          */
/*  - q = trunc(x * 2^(62 - emax)) as int64 (so |q| < 2^62, the same two    */
/*    bits of headroom as 2^30 in int32), the lifting on int64;             */
/*  - negabinary u = (q + 0xAAAA...AA) ^ 0xAAAA...AA on uint64;             */
/*  - bit planes 63..0 with budget 64*rate - 12 bits; rates 1..68 bits per */
/*    value (the worst case, 12 + 64*64 + 64 + 64 bits, fits rate 67);    */
/*  - decoding: x = (double)q * 2^(emax - 62).                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t emax;        /* INT32_MIN for an all-zero block */
    int64_t q[64];       /* natural order */
    int64_t t[64];       /* after the forward transform, natural order */
    uint64_t u[64];      /* sequency order, negabinary */
    uint64_t plane[64];  /* plane[p]: bit i = bit p of u[i] */
    int32_t bits_used;
} orc_stages64;

/* Lifting on int64 values, checked with 128-bit intermediates: every
 * intermediate must stay inside int64 (reported, never wrapped). */
static _Thread_local int g_range64 = 0;
static __int128 chk64(__int128 v)
{
    if (v > (__int128)INT64_MAX || v < (__int128)INT64_MIN) g_range64 = 1;
    return v;
}
static __int128 asr1_128(__int128 v) { return v >> 1; }

static void fwd4_64(__int128* a, __int128* b, __int128* c, __int128* d)
{
    __int128 A = *a, B = *b, C = *c, D = *d;
    A = chk64(asr1_128(chk64(A + D))); D = chk64(D - A);
    C = chk64(asr1_128(chk64(C + B))); B = chk64(B - C);
    A = chk64(asr1_128(chk64(A + C))); C = chk64(C - A);
    D = chk64(asr1_128(chk64(D + B))); B = chk64(B - D);
    D = chk64(D + asr1_128(B));        B = chk64(B - asr1_128(D));
    *a = A; *b = B; *c = C; *d = D;
}

static void inv4_64(__int128* a, __int128* b, __int128* c, __int128* d)
{
    __int128 A = *a, B = *b, C = *c, D = *d;
    B = chk64(B + asr1_128(D)); D = chk64(D - asr1_128(B));
    B = chk64(B + D);           D = chk64(2 * D - B);
    C = chk64(C + A);           A = chk64(2 * A - C);
    B = chk64(B + C);           C = chk64(2 * C - B);
    D = chk64(D + A);           A = chk64(2 * A - D);
    *a = A; *b = B; *c = C; *d = D;
}

static void lift_axis64(__int128* v, int axis, int inverse)
{
    int stride = axis == 0 ? 1 : (axis == 1 ? 4 : 16);
    for (int o1 = 0; o1 < 4; ++o1)
        for (int o2 = 0; o2 < 4; ++o2) {
            int base;
            if (axis == 0) base = 4 * o1 + 16 * o2;
            else if (axis == 1) base = o1 + 16 * o2;
            else base = o1 + 4 * o2;
            __int128* a = &v[base];
            __int128* b = &v[base + stride];
            __int128* c = &v[base + 2 * stride];
            __int128* d = &v[base + 3 * stride];
            if (inverse) inv4_64(a, b, c, d); else fwd4_64(a, b, c, d);
        }
}

int orc64_fwd_xform(const int64_t* in64, int64_t* out64)
{
    __int128 v[64];
    g_range64 = 0;
    for (int i = 0; i < 64; ++i) v[i] = in64[i];
    lift_axis64(v, 0, 0); lift_axis64(v, 1, 0); lift_axis64(v, 2, 0);
    for (int i = 0; i < 64; ++i) out64[i] = (int64_t)v[i];
    return g_range64 ? -2 : 0;
}

int orc64_inv_xform(const int64_t* in64, int64_t* out64)
{
    __int128 v[64];
    g_range64 = 0;
    for (int i = 0; i < 64; ++i) v[i] = in64[i];
    lift_axis64(v, 2, 1); lift_axis64(v, 1, 1); lift_axis64(v, 0, 1);
    for (int i = 0; i < 64; ++i) out64[i] = (int64_t)v[i];
    return g_range64 ? -2 : 0;
}

static int exponent64_of(double x)
{
    int e;
    (void)frexp(x, &e);
    return e < -1022 ? -1022 : e;
}

/* Group-testing bit-plane coder on 64 sequency-ordered 64-bit negabinary
 * words: the FP32 coder's rules with planes 63..0. */
static long code_planes64(const uint64_t* u, long budget, bitw* s, uint64_t* planes_out)
{
    long used = 0;
    int n = 0;
    for (int p = 63; p >= 0; --p) {
        uint64_t X = 0;
        for (int i = 0; i < 64; ++i) X |= ((u[i] >> p) & 1u) << i;
        if (planes_out) planes_out[p] = X;
        if (budget <= 0) continue;
        for (int i = 0; i < n && budget > 0; ++i) { put1(s, (int)((X >> i) & 1u)); budget--; used++; }
        while (n < 64 && budget > 0) {
            int g = (X >> n) != 0;
            put1(s, g); budget--; used++;
            if (!g) break;
            for (;;) {
                if (n == 63) { n = 64; break; }
                if (budget <= 0) break;
                int b = (int)((X >> n) & 1u);
                put1(s, b); budget--; used++;
                n++;
                if (b) break;
            }
        }
    }
    return used;
}

static void decode_planes64(uint64_t* u, long budget, bitr* s, uint64_t* planes_out)
{
    int n = 0;
    for (int i = 0; i < 64; ++i) u[i] = 0;
    for (int p = 63; p >= 0; --p) {
        uint64_t X = 0;
        if (budget > 0) {
            for (int i = 0; i < n && budget > 0; ++i) { X |= (uint64_t)get1(s) << i; budget--; }
            while (n < 64 && budget > 0) {
                int g = get1(s); budget--;
                if (!g) break;
                for (;;) {
                    if (n == 63) { X |= (uint64_t)1 << 63; n = 64; break; }
                    if (budget <= 0) break;
                    int b = get1(s); budget--;
                    if (b) { X |= (uint64_t)1 << n; n++; break; }
                    n++;
                }
            }
        }
        if (planes_out) planes_out[p] = X;
        for (int i = 0; i < 64; ++i) u[i] |= ((X >> i) & 1u) << p;
    }
}

#define NB64 0xAAAAAAAAAAAAAAAAull

int orc64_encode_block(const double* in64, int rate, uint64_t* out, orc_stages64* st)
{
    if (rate < 1 || rate > 68) return -1;
    build_perm();
    memset(out, 0, (size_t)rate * sizeof(uint64_t));
    orc_stages64 local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    int nonzero = 0, emax = -100000;
    for (int i = 0; i < 64; ++i)
        if (in64[i] != 0.0) {
            nonzero = 1;
            int e = exponent64_of(in64[i]);
            if (e > emax) emax = e;
        }
    bitw s = {out, 0};
    if (!nonzero) {
        st->emax = INT32_MIN;
        put1(&s, 0);
        st->bits_used = 1;
        return 0;
    }
    st->emax = emax;
    put1(&s, 1);
    int biased = emax + 1023;
    for (int b = 0; b < 11; ++b) put1(&s, (biased >> b) & 1);
    for (int i = 0; i < 64; ++i) st->q[i] = (int64_t)ldexp(in64[i], 62 - emax); /* C conversion truncates */
    int rc = orc64_fwd_xform(st->q, st->t);
    for (int k = 0; k < 64; ++k) st->u[k] = ((uint64_t)st->t[g_perm[k]] + NB64) ^ NB64;
    long used = code_planes64(st->u, 64L * rate - 12, &s, st->plane);
    st->bits_used = (int32_t)(12 + used);
    return rc;
}

int orc64_decode_block(const uint64_t* in, int rate, double* out64, orc_stages64* st)
{
    if (rate < 1 || rate > 68) return -1;
    build_perm();
    orc_stages64 local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    bitr s = {in, 0};
    if (!get1(&s)) {
        st->emax = INT32_MIN;
        for (int i = 0; i < 64; ++i) out64[i] = 0.0;
        return 0;
    }
    int biased = 0;
    for (int b = 0; b < 11; ++b) biased |= get1(&s) << b;
    int emax = biased - 1023;
    st->emax = emax;
    decode_planes64(st->u, 64L * rate - 12, &s, st->plane);
    for (int k = 0; k < 64; ++k) st->t[g_perm[k]] = (int64_t)((st->u[k] ^ NB64) - NB64);
    int rc = orc64_inv_xform(st->t, st->q);
    for (int i = 0; i < 64; ++i) out64[i] = ldexp((double)st->q[i], emax - 62);
    return rc;
}

long orc64_code_ints(const uint64_t* u64, long budget, uint64_t* out)
{
    bitw s = {out, 0};
    return code_planes64(u64, budget, &s, NULL);
}

int orc64_decode_ints(const uint64_t* in, long budget, uint64_t* u64)
{
    bitr s = {in, 0};
    decode_planes64(u64, budget, &s, NULL);
    return 0;
}

static void gather_block64(const double* f, long nx, long ny, long bx, long by, long bz, double* blk)
{
    for (int l = 0; l < 4; ++l)
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i)
                blk[i + 4 * j + 16 * l] = f[IDX(4 * bx + i, 4 * by + j, 4 * bz + l, nx, ny)];
}

static void scatter_block64(double* f, long nx, long ny, long bx, long by, long bz, const double* blk)
{
    for (int l = 0; l < 4; ++l)
        for (int j = 0; j < 4; ++j)
            for (int i = 0; i < 4; ++i)
                f[IDX(4 * bx + i, 4 * by + j, 4 * bz + l, nx, ny)] = blk[i + 4 * j + 16 * l];
}

int orc64_codec_encode(const double* f, long nx, long ny, long nz, int rate, uint64_t* out)
{
    if (nx % 4 || ny % 4 || nz % 4 || rate < 1 || rate > 68) return -1;
    long bxn = nx / 4, byn = ny / 4, bzn = nz / 4;
    int bad = 0;
    build_perm();
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long bz = 0; bz < bzn; ++bz)
        for (long by = 0; by < byn; ++by)
            for (long bx = 0; bx < bxn; ++bx) {
                double blk[64];
                gather_block64(f, nx, ny, bx, by, bz, blk);
                size_t b = (size_t)bx + (size_t)bxn * ((size_t)by + (size_t)byn * (size_t)bz);
                orc_stages64 st;
                if (orc64_encode_block(blk, rate, out + b * (size_t)rate, &st) != 0) bad = 1;
            }
    return bad ? -2 : 0;
}

int orc64_codec_decode(const uint64_t* in, long nx, long ny, long nz, int rate, double* f)
{
    if (nx % 4 || ny % 4 || nz % 4 || rate < 1 || rate > 68) return -1;
    long bxn = nx / 4, byn = ny / 4, bzn = nz / 4;
    int bad = 0;
    build_perm();
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long bz = 0; bz < bzn; ++bz)
        for (long by = 0; by < byn; ++by)
            for (long bx = 0; bx < bxn; ++bx) {
                double blk[64];
                size_t b = (size_t)bx + (size_t)bxn * ((size_t)by + (size_t)byn * (size_t)bz);
                orc_stages64 st;
                if (orc64_decode_block(in + b * (size_t)rate, rate, blk, &st) != 0) bad = 1;
                scatter_block64(f, nx, ny, bx, by, bz, blk);
            }
    return bad ? -2 : 0;
}

/* Q = decode(encode(.)) in place on an FP64 field with the FP64 format. */
int orc64_codec_roundtrip(double* f, long nx, long ny, long nz, int rate)
{
    size_t nw = orc_codec_words(nx, ny, nz, rate);
    uint64_t* w = (uint64_t*)calloc(nw ? nw : 1, sizeof(uint64_t));
    if (!w) return -1;
    int rc = orc64_codec_encode(f, nx, ny, nz, rate, w);
    if (rc == 0) rc = orc64_codec_decode(w, nx, ny, nz, rate, f);
    free(w);
    return rc;
}

/* The compressed schedule's state in FP64 with the FP64 format (the
 * paper's setting): as orc_replay_wave_f64, Q being the FP64 codec. */
int orc64_replay_wave(double* p, double* pm, double* w, long nx, long ny, long nz, long steps, long k,
                      const double* src, long src_index, int rate_p, int rate_pm, int rate_w)
{
    if (k < 1) return -1;
    int rc = 0;
    if (rate_w > 0 && (rc = orc64_codec_roundtrip(w, nx, ny, nz, rate_w))) return rc;
    if (rate_p > 0 && (rc = orc64_codec_roundtrip(p, nx, ny, nz, rate_p))) return rc;
    if (rate_pm > 0 && (rc = orc64_codec_roundtrip(pm, nx, ny, nz, rate_pm))) return rc;
    for (long done = 0; done < steps;) {
        long kk = steps - done < k ? steps - done : k;
        if ((rc = orc_wave25_f64(p, pm, w, nx, ny, nz, kk, src ? src + done : NULL, src_index))) return rc;
        if (rate_p > 0 && (rc = orc64_codec_roundtrip(p, nx, ny, nz, rate_p))) return rc;
        if (rate_pm > 0 && (rc = orc64_codec_roundtrip(pm, nx, ny, nz, rate_pm))) return rc;
        done += kk;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Misfit gradient of the wave propagator by the discrete adjoint.          */
/*                                                                          */
/* Forward (p_0 = p_-1 = 0):  p_{t+1} = 2 p_t - p_{t-1} + w . L p_t + s_t   */
/* at the source cell, t = 0..T-1. Receivers record r_t = p_t at nr cells,  */
/* t = 1..T; J = 1/2 sum_t |r_t - d_t|^2.                                   */
/* Stationarity of the Lagrangian with one multiplier per step gives, with  */
/* lam_{T+1} = lam_{T+2} = 0 and L symmetric under zero ghosts:             */
/*   lam_t = 2 lam_{t+1} - lam_{t+2} + L (w . lam_{t+1}) + res_t at rcvs    */
/*   dJ/dw = sum_{t=1..T} lam_t . L p_{t-1},   res_t = r_t - d_t.           */
/* Every forward state is kept (small grids only).                          */
/* ------------------------------------------------------------------------ */

static double lap_at_f64(const double* p, long i, long j, long l, long nx, long ny, long nz)
{
    double acc = W_C0X3 * at_f64(p, i, j, l, nx, ny, nz);
    for (int m = 1; m <= 4; ++m) {
        double sm = (at_f64(p, i + m, j, l, nx, ny, nz) + at_f64(p, i - m, j, l, nx, ny, nz))
                  + (at_f64(p, i, j + m, l, nx, ny, nz) + at_f64(p, i, j - m, l, nx, ny, nz));
        sm = sm + (at_f64(p, i, j, l + m, nx, ny, nz) + at_f64(p, i, j, l - m, nx, ny, nz));
        acc = acc + W_C[m] * sm;
    }
    return acc;
}

/* L (w . lam) at one cell, FP64 */
static double lapw_at_f64(const double* lam, const double* w, long i, long j, long l, long nx, long ny, long nz)
{
#define WL(a, b, c) (at_f64(w, a, b, c, nx, ny, nz) * at_f64(lam, a, b, c, nx, ny, nz))
    double acc = W_C0X3 * WL(i, j, l);
    for (int m = 1; m <= 4; ++m) {
        double sm = (WL(i + m, j, l) + WL(i - m, j, l)) + (WL(i, j + m, l) + WL(i, j - m, l));
        sm = sm + (WL(i, j, l + m) + WL(i, j, l - m));
        acc = acc + W_C[m] * sm;
    }
    return acc;
#undef WL
}

/* Forward run keeping every state: states[(t)*n + c] = p_t, t = 0..T.
 * records[(t-1)*nr + i] = p_t at rcv[i], t = 1..T. */
int orc_wave_forward_states_f64(const double* w, long nx, long ny, long nz, long T, const double* src, long src_index,
                                const long* rcv, long nr, double* records, double* states)
{
    size_t n = (size_t)nx * ny * nz;
    double* pm = (double*)calloc(n, sizeof(double));
    double* p = (double*)calloc(n, sizeof(double));
    if (!pm || !p) { free(pm); free(p); return -1; }
    memcpy(states, p, n * sizeof(double));
    for (long t = 0; t < T; ++t) {
        int rc = orc_wave25_f64(p, pm, w, nx, ny, nz, 1, src ? src + t : NULL, src_index);
        if (rc) { free(pm); free(p); return rc; }
        memcpy(states + (size_t)(t + 1) * n, p, n * sizeof(double));
        for (long i = 0; i < nr; ++i) records[t * nr + i] = p[rcv[i]];
    }
    free(pm);
    free(p);
    return 0;
}

/* Adjoint run driven by the receiver residual series res (T x nr, row t-1
 * for time t). If states != NULL, accumulates grad (n values, overwritten)
 * = sum_t lam_t . L p_{t-1}. If src_adj != NULL, src_adj[t] = lam_{t+1} at
 * src_index for t = 0..T-1 (the transpose of source -> receivers). */
int orc_wave_adjoint_f64(const double* w, long nx, long ny, long nz, long T, const long* rcv, long nr,
                         const double* res, const double* states, double* grad, long src_index, double* src_adj)
{
    size_t n = (size_t)nx * ny * nz;
    double* l1 = (double*)calloc(n, sizeof(double)); /* lam_{t+1} */
    double* l2 = (double*)calloc(n, sizeof(double)); /* lam_{t+2} */
    double* l0 = (double*)calloc(n, sizeof(double)); /* lam_t */
    if (!l1 || !l2 || !l0) { free(l1); free(l2); free(l0); return -1; }
    if (grad) memset(grad, 0, n * sizeof(double));
    for (long t = T; t >= 1; --t) {
#pragma omp parallel for schedule(static)
        for (long l = 0; l < nz; ++l)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) {
                    size_t c = IDX(i, j, l, nx, ny);
                    l0[c] = (2.0 * l1[c] - l2[c]) + lapw_at_f64(l1, w, i, j, l, nx, ny, nz);
                }
        for (long i = 0; i < nr; ++i) l0[rcv[i]] = l0[rcv[i]] + res[(t - 1) * nr + i];
        if (grad && states) {
            const double* pt = states + (size_t)(t - 1) * n;
#pragma omp parallel for schedule(static)
            for (long l = 0; l < nz; ++l)
                for (long j = 0; j < ny; ++j)
                    for (long i = 0; i < nx; ++i) {
                        size_t c = IDX(i, j, l, nx, ny);
                        grad[c] += l0[c] * lap_at_f64(pt, i, j, l, nx, ny, nz);
                    }
        }
        if (src_adj) src_adj[t - 1] = l0[src_index];
        double* tmp = l2; l2 = l1; l1 = l0; l0 = tmp;
    }
    free(l1);
    free(l2);
    free(l0);
    return 0;
}

/* J and dJ/dw for observed records d (T x nr). */
int orc_wave_misfit_grad_f64(const double* w, long nx, long ny, long nz, long T, const double* src, long src_index,
                             const long* rcv, long nr, const double* d, double* J, double* grad)
{
    size_t n = (size_t)nx * ny * nz;
    double* states = (double*)malloc((size_t)(T + 1) * n * sizeof(double));
    double* rec = (double*)malloc((size_t)T * nr * sizeof(double));
    if (!states || !rec) { free(states); free(rec); return -1; }
    int rc = orc_wave_forward_states_f64(w, nx, ny, nz, T, src, src_index, rcv, nr, rec, states);
    double j = 0.0;
    for (long q = 0; q < T * nr; ++q) {
        rec[q] -= d[q];
        j += rec[q] * rec[q];
    }
    *J = 0.5 * j;
    if (rc == 0 && grad) rc = orc_wave_adjoint_f64(w, nx, ny, nz, T, rcv, nr, rec, states, grad, 0, NULL);
    free(states);
    free(rec);
    return rc;
}

/* FP32 adjoint in a fixed operation order. Iteration t = T..1:
 *   lam_t = (2*lam1 - lam2) + accw,  accw = C0X3*(w*lam1) + sum_m C_m*(((wl[x+m] + wl[x-m]) +
 *           (wl[y+m] + wl[y-m])) + (wl[z+m] + wl[z-m])), wl[q] = w[q]*lam1[q]
 *   grad  = grad + lam1 * Lp_t (lam1 = lam_{t+1} after its receiver injection,
 *           Lp_t in the forward order)
 *   then lam_t = lam_t + res_t at each receiver, in receiver order.
 * Forward states come from the FP32 forward (orc_wave25_f32 order). res is
 * given (T x nr, FP32). src_adj optional as in the FP64 version. */
static float at32(const float* u, long i, long j, long l, long nx, long ny, long nz) { return at_f32(u, i, j, l, nx, ny, nz); }

int orc_wave_adjoint_f32(const float* w, long nx, long ny, long nz, long T, const long* rcv, long nr,
                         const float* res, const float* states, float* grad, long src_index, float* src_adj)
{
    const float c0x3 = (float)(-205.0 / 24.0);
    const float cm[5] = {0.0f, (float)(8.0 / 5.0), (float)(-1.0 / 5.0), (float)(8.0 / 315.0), (float)(-1.0 / 560.0)};
    size_t n = (size_t)nx * ny * nz;
    float* l1 = (float*)calloc(n, sizeof(float));
    float* l2 = (float*)calloc(n, sizeof(float));
    float* l0 = (float*)calloc(n, sizeof(float));
    if (!l1 || !l2 || !l0) { free(l1); free(l2); free(l0); return -1; }
    if (grad) memset(grad, 0, n * sizeof(float));
    for (long t = T; t >= 1; --t) {
        const float* pt = states ? states + (size_t)t * n : NULL;
#pragma omp parallel for schedule(static)
        for (long l = 0; l < nz; ++l)
            for (long j = 0; j < ny; ++j)
                for (long i = 0; i < nx; ++i) {
                    size_t c = IDX(i, j, l, nx, ny);
#define WL(a, b, e) (at32(w, a, b, e, nx, ny, nz) * at32(l1, a, b, e, nx, ny, nz))
                    float acc = c0x3 * WL(i, j, l);
                    for (int m = 1; m <= 4; ++m) {
                        float sm = (WL(i + m, j, l) + WL(i - m, j, l)) + (WL(i, j + m, l) + WL(i, j - m, l));
                        sm = sm + (WL(i, j, l + m) + WL(i, j, l - m));
                        acc = acc + cm[m] * sm;
                    }
#undef WL
                    l0[c] = (2.0f * l1[c] - l2[c]) + acc;
                    if (grad && pt) {
                        float lp = c0x3 * pt[c];
                        for (int m = 1; m <= 4; ++m) {
                            float sm = (at32(pt, i + m, j, l, nx, ny, nz) + at32(pt, i - m, j, l, nx, ny, nz))
                                     + (at32(pt, i, j + m, l, nx, ny, nz) + at32(pt, i, j - m, l, nx, ny, nz));
                            sm = sm + (at32(pt, i, j, l + m, nx, ny, nz) + at32(pt, i, j, l - m, nx, ny, nz));
                            lp = lp + cm[m] * sm;
                        }
                        grad[c] = grad[c] + l1[c] * lp;
                    }
                }
        for (long i = 0; i < nr; ++i) l0[rcv[i]] = l0[rcv[i]] + res[(t - 1) * nr + i];
        if (src_adj) src_adj[t - 1] = l0[src_index];
        float* tmp = l2; l2 = l1; l1 = l0; l0 = tmp;
    }
    free(l1);
    free(l2);
    free(l0);
    return 0;
}

/* FP32 forward keeping every state (states[t*n], t = 0..T) and records. */
int orc_wave_forward_states_f32(const float* w, long nx, long ny, long nz, long T, const float* src, long src_index,
                                const long* rcv, long nr, float* records, float* states)
{
    size_t n = (size_t)nx * ny * nz;
    float* pm = (float*)calloc(n, sizeof(float));
    float* p = (float*)calloc(n, sizeof(float));
    if (!pm || !p) { free(pm); free(p); return -1; }
    memcpy(states, p, n * sizeof(float));
    for (long t = 0; t < T; ++t) {
        int rc = orc_wave25_f32(p, pm, w, nx, ny, nz, 1, src ? src + t : NULL, src_index);
        if (rc) { free(pm); free(p); return rc; }
        memcpy(states + (size_t)(t + 1) * n, p, n * sizeof(float));
        for (long i = 0; i < nr; ++i) records[t * nr + i] = p[rcv[i]];
    }
    free(pm);
    free(p);
    return 0;
}
