// codec_dev.hpp -- gfx950 device code of the fixed-rate 4^3 block codec
// (Sec. IV: fixed rate, the user chooses the bits kept per value; transform
// of Lindstrom, IEEE TVCG 20(12), 2014).
//
// Mapping: one lane codes one whole block. A wavefront takes 64 blocks that
// are consecutive in x, so every row load or store of the field is one
// 1 KiB contiguous access per wave instruction, and the 64 blocks' words
// are one contiguous run of the compressed stream. All 64 values of a block
// stay in registers: the separable lifting, the sequency reorder (compile
// time register renaming) and the negabinary map need no data exchange,
// and the 64 x 32 bit matrix of coefficients is turned into 32 bit-plane
// words by two in-register 32 x 32 bit transposes. The variable-length
// group-test code is then written (or parsed) by each lane on its own,
// through a per-wave LDS buffer that holds the block words transposed
// (word w of lane L at w*64 + L), which the wave moves to or from global
// memory with coalesced accesses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace oocs {
namespace codec {

// ---- total-sequency order ---------------------------------------------------
// Coefficients are ordered by i+j+l, then i^2+j^2+l^2, then (l, j, i)
// lexicographically. kFwd<k> = in-block index of the k-th coefficient.
constexpr int seq_key(int idx)
{
    const int i = idx & 3, j = (idx >> 2) & 3, l = idx >> 4;
    return ((((i + j + l) * 32 + (i * i + j * j + l * l)) * 4 + l) * 4 + j) * 4 + i;
}

constexpr int seq_rank(int idx)
{
    int rank = 0;
    for (int o = 0; o < 64; ++o) rank += seq_key(o) < seq_key(idx);
    return rank;
}

constexpr int seq_fwd(int k)
{
    for (int idx = 0; idx < 64; ++idx)
        if (seq_rank(idx) == k) return idx;
    return -1;
}

template <int K> constexpr int kFwd = seq_fwd(K);
template <int I> constexpr int kRank = seq_rank(I);

constexpr uint32_t kNB = 0xAAAAAAAAu;  // negabinary mask

// ---- lifting (uint32 arithmetic wraps; >> is arithmetic) ---------------------
__device__ inline int add_(int a, int b) { return (int)((uint32_t)a + (uint32_t)b); }
__device__ inline int sub_(int a, int b) { return (int)((uint32_t)a - (uint32_t)b); }

__device__ inline void fwd_lift(int& a, int& b, int& c, int& d)
{
    a = add_(a, d) >> 1; d = sub_(d, a);
    c = add_(c, b) >> 1; b = sub_(b, c);
    a = add_(a, c) >> 1; c = sub_(c, a);
    d = add_(d, b) >> 1; b = sub_(b, d);
    d = add_(d, b >> 1); b = sub_(b, d >> 1);
}

__device__ inline void inv_lift(int& a, int& b, int& c, int& d)
{
    b = add_(b, d >> 1); d = sub_(d, b >> 1);
    b = add_(b, d);      d = sub_(add_(d, d), b);
    c = add_(c, a);      a = sub_(add_(a, a), c);
    b = add_(b, c);      c = sub_(add_(c, c), b);
    d = add_(d, a);      a = sub_(add_(a, a), d);
}

// Forward transform along x, then y, then z (in-block index i + 4j + 16l).
__device__ inline void fwd_xform(int (&v)[64])
{
#pragma unroll
    for (int o = 0; o < 16; ++o) fwd_lift(v[4 * o], v[4 * o + 1], v[4 * o + 2], v[4 * o + 3]);
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int i = 0; i < 4; ++i) fwd_lift(v[16 * l + i], v[16 * l + i + 4], v[16 * l + i + 8], v[16 * l + i + 12]);
#pragma unroll
    for (int o = 0; o < 16; ++o) fwd_lift(v[o], v[o + 16], v[o + 32], v[o + 48]);
}

// Inverse transform along z, then y, then x.
__device__ inline void inv_xform(int (&v)[64])
{
#pragma unroll
    for (int o = 0; o < 16; ++o) inv_lift(v[o], v[o + 16], v[o + 32], v[o + 48]);
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int i = 0; i < 4; ++i) inv_lift(v[16 * l + i], v[16 * l + i + 4], v[16 * l + i + 8], v[16 * l + i + 12]);
#pragma unroll
    for (int o = 0; o < 16; ++o) inv_lift(v[4 * o], v[4 * o + 1], v[4 * o + 2], v[4 * o + 3]);
}

// u[k] = negabinary of coefficient kFwd<k> (sequency order).
template <int... K>
__device__ inline void to_sequency(const int (&t)[64], uint32_t (&u)[64], std::integer_sequence<int, K...>)
{
    ((u[K] = ((uint32_t)t[kFwd<K>] + kNB) ^ kNB), ...);
}

// t[idx] = integer of the coefficient at sequency position kRank<idx>.
template <int... I>
__device__ inline void from_sequency(const uint32_t (&u)[64], int (&t)[64], std::integer_sequence<int, I...>)
{
    ((t[I] = (int)((u[kRank<I>] ^ kNB) - kNB)), ...);
}

// The same with mid-point reconstruction: a nonzero coefficient at sequency
// position k gets off_a added if k < known (its digit of the stop plane was
// read), else off_b (32-bit wrap-around).
template <int... I>
__device__ inline void from_sequency_mid(const uint32_t (&u)[64], int (&t)[64], int known, uint32_t off_a,
                                         uint32_t off_b, std::integer_sequence<int, I...>)
{
    ((t[I] = (int)(((u[kRank<I>] ^ kNB) - kNB) + (u[kRank<I>] ? (kRank<I> < known ? off_a : off_b) : 0u))), ...);
}

// Middle of the values L cut-off negabinary digits can add: half of the
// all-ones sum (1 - (-2)^L) / 3, rounded down.
__device__ inline uint32_t midpoint_offset(int L)
{
    const int64_t pw = (L & 1) ? -((int64_t)1 << L) : ((int64_t)1 << L);
    const int64_t all_ones = (1 - pw) / 3;
    return (uint32_t)(all_ones >> 1);
}

// One stage of the in-place 32 x 32 bit transpose: swap the off-diagonal
// S x S sub-blocks of every 2S x 2S block.
template <int S, uint32_t M>
__device__ inline void transpose_stage(uint32_t (&a)[32])
{
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        if (r & S) continue;
        const uint32_t t = ((a[r] >> S) ^ a[r + S]) & M;
        a[r + S] ^= t;
        a[r] ^= t << S;
    }
}

// In-place transpose of a 32 x 32 bit matrix held as 32 rows: afterwards
// bit c of a[r] is what bit r of a[c] was.
__device__ inline void transpose32(uint32_t (&a)[32])
{
    transpose_stage<16, 0x0000FFFFu>(a);
    transpose_stage<8, 0x00FF00FFu>(a);
    transpose_stage<4, 0x0F0F0F0Fu>(a);
    transpose_stage<2, 0x33333333u>(a);
    transpose_stage<1, 0x55555555u>(a);
}

// Bit planes of the 64 sequency-ordered coefficients: bit k of plane p is
// bit p of u[k]. lo[p] holds coefficients 0..31, hi[p] 32..63.
__device__ inline void planes_of(const uint32_t (&u)[64], uint32_t (&lo)[32], uint32_t (&hi)[32])
{
#pragma unroll
    for (int i = 0; i < 32; ++i) { lo[i] = u[i]; hi[i] = u[32 + i]; }
    transpose32(lo);
    transpose32(hi);
}

__device__ inline void coefficients_of(uint32_t (&lo)[32], uint32_t (&hi)[32], uint32_t (&u)[64])
{
    transpose32(lo);
    transpose32(hi);
#pragma unroll
    for (int i = 0; i < 32; ++i) { u[i] = lo[i]; u[32 + i] = hi[i]; }
}

__device__ inline uint64_t plane_word(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

__device__ inline int exponent_of(float x)
{
    const int e = __builtin_amdgcn_frexp_expf(x);
    return e < -126 ? -126 : e;
}

// ---- per-lane bit writer over the wave's LDS words --------------------------
// Branch-free: every put writes the lane's current word to LDS (the last
// write of a word wins), so no lane takes a divergent path to flush.
struct LaneWriter {
    uint64_t* lds;  // this wave's buffer; word w of this lane at lds[w * 64]
    uint64_t acc;   // bits of word wi written so far
    int off, wi, budget;

    __device__ void put(uint64_t v, int m)  // m in [0, 64]
    {
        m = max(0, min(m, budget));
        const uint64_t mask = m >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << m) - 1);
        v &= mask;
        const uint64_t lo = acc | (v << off);
        const uint64_t hi = off == 0 ? 0 : (v >> (64 - off));  // bits that spill into word wi+1
        const int end = off + m;
        if (m > 0) lds[wi * 64] = lo;
        const bool cross = end >= 64;
        acc = cross ? hi : lo;
        off = cross ? end - 64 : end;
        wi += cross ? 1 : 0;
        budget -= m;
    }
};

struct EncStageOut {
    int32_t* emax; int32_t* q; int32_t* t; uint32_t* u; uint64_t* planes; int32_t* bits;
};

// Encode this lane's block x[64] (natural order) into words w*64 of `lds`
// (rate words, zero padded). With STAGES the intermediate stages of block b
// are written out.
template <bool STAGES>
__device__ inline void encode_lane(const float (&x)[64], int rate, uint64_t* lds, EncStageOut st = {}, int64_t b = 0)
{
    int emax = -1000;
#pragma unroll
    for (int i = 0; i < 64; ++i)
        if (x[i] != 0.0f) emax = max(emax, exponent_of(x[i]));
    LaneWriter w{lds, 0, 0, 0, 64 * rate};
    if (emax == -1000) {  // all-zero block: a single 0 bit
        w.put(0, 1);
        if (STAGES) {
            if (st.emax) st.emax[b] = INT32_MIN;
            if (st.bits) st.bits[b] = 1;
#pragma unroll
            for (int i = 0; i < 64; ++i) {
                if (st.q) st.q[64 * b + i] = 0;
                if (st.t) st.t[64 * b + i] = 0;
                if (st.u) st.u[64 * b + i] = 0;
            }
#pragma unroll
            for (int p = 0; p < 32; ++p)
                if (st.planes) st.planes[32 * b + p] = 0;
        }
    } else {
        int t[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) t[i] = (int)ldexpf(x[i], 30 - emax);  // exact scaling, truncation
        if (STAGES) {
            if (st.emax) st.emax[b] = emax;
#pragma unroll
            for (int i = 0; i < 64; ++i)
                if (st.q) st.q[64 * b + i] = t[i];
        }
        fwd_xform(t);
        uint32_t u[64];
        to_sequency(t, u, std::make_integer_sequence<int, 64>{});
        if (STAGES) {
#pragma unroll
            for (int i = 0; i < 64; ++i) {
                if (st.t) st.t[64 * b + i] = t[i];
                if (st.u) st.u[64 * b + i] = u[i];
            }
        }
        uint32_t lo[32], hi[32];
        planes_of(u, lo, hi);
        if (STAGES) {
#pragma unroll
            for (int p = 0; p < 32; ++p)
                if (st.planes) st.planes[32 * b + p] = plane_word(lo[p], hi[p]);
        }
        w.put(1u | ((uint64_t)(uint32_t)(emax + 127) << 1), 9);
        int n = 0;  // coefficients already significant
        for (int p = 31; p >= 0; --p) {
            if (w.budget > 0) {
                const int pu = __builtin_amdgcn_readfirstlane(p);  // uniform: plain register indexing
                const uint64_t X = plane_word(lo[pu], hi[pu]);
                w.put(X, n);  // verbatim bits of the significant coefficients
                if (n < 64 && w.budget > 0) {
                    // The plane's group tests as one string of at most 127 bits
                    // (c0: bits 0..63, c1: 64..127), written with two puts: for
                    // each 1 of X at or above n, a positive test and the bits up
                    // to and including that 1 (the last coefficient's 1 is
                    // implied); then a negative test if coefficients remain.
                    // Truncation at the budget happens in put, as bit by bit.
                    uint64_t c0 = 0, c1 = 0;
                    int len = 0;
                    auto append = [&](uint64_t v, int l) {  // l in [1, 64], len + l <= 127
                        c0 |= len < 64 ? v << len : 0;
                        c1 |= len == 0 ? 0 : (len < 64 ? v >> (64 - len) : v << (len - 64));
                        len += l;
                    };
                    uint64_t Y = X >> n;
                    while (Y != 0) {
                        const int m = __builtin_ctzll(Y);  // zeros before the next 1
                        if (n + m == 63) {                 // the last coefficient
                            append(1, 1 + m);
                            n = 64;
                            break;
                        }
                        append(1u | ((uint64_t)1 << (m + 1)), m + 2);  // test 1, m zeros, the 1
                        n += m + 1;
                        Y >>= m + 1;
                    }
                    if (n < 64) append(0, 1);
                    w.put(c0, min(len, 64));
                    if (len > 64) w.put(c1, len - 64);
                }
            }
        }
    }
    if (STAGES && st.bits && emax != -1000) st.bits[b] = 64 * rate - w.budget;
    if (w.off > 0) { lds[w.wi * 64] = w.acc; ++w.wi; }
    for (int k = w.wi; k < rate; ++k) lds[k * 64] = 0;
}

// ---- per-lane bit reader over the wave's LDS words --------------------------
// Keeps the current word and the next two, plus the word three ahead, which
// every skip loads unconditionally and the next skip takes if it crosses a
// word boundary: the reader has no branches, and the LDS latency of each
// load is hidden behind the bits decoded before its first use.
struct LaneReader {
    const uint64_t* lds;  // word w of this lane at lds[w * 64]
    int rate;
    uint64_t cur, nxt, nx2, pend;  // words wi, wi+1, wi+2, wi+3 (0 past the block)
    int wi, off;

    __device__ uint64_t word(int w) const
    {
        const uint64_t v = lds[min(w, rate - 1) * 64];  // an address inside the block either way
        return w < rate ? v : 0;
    }
    __device__ void init()
    {
        wi = 0; off = 0;
        cur = word(0);
        nxt = word(1);
        nx2 = word(2);
        pend = word(3);
    }
    // the next 64 bits of the stream (bits past the block read as zero)
    __device__ uint64_t window() const { return (cur >> off) | ((nxt << 1) << (63 - off)); }
    __device__ void skip(int m)  // m in [0, 64]
    {
        off += m;
        const bool cross = off >= 64;
        off -= cross ? 64 : 0;
        wi += cross ? 1 : 0;
        cur = cross ? nxt : cur;
        nxt = cross ? nx2 : nxt;
        nx2 = cross ? pend : nx2;
        pend = word(wi + 3);
    }
    __device__ uint64_t get(int m)  // m in [0, 64]
    {
        uint64_t v = window();
        if (m < 64) v &= ((uint64_t)1 << m) - 1;
        skip(m);
        return v;
    }
};

struct DecStageOut {
    int32_t* emax; uint64_t* planes; uint32_t* u; int32_t* q;
};

// Decode this lane's block from words w*64 of `lds` into x[64] (natural order).
// MID: mid-point reconstruction. Where the budget runs out the decoder
// notes the plane and how many coefficients (a prefix in sequency order)
// know their digit of it; a plane that the last bit completes makes the
// next plane the stop plane with none known.
template <bool STAGES, bool MID = false>
__device__ inline void decode_lane(const uint64_t* lds, int rate, float (&x)[64], DecStageOut st = {}, int64_t b = 0)
{
    LaneReader r{lds, rate, 0, 0, 0, 0, 0, 0};
    r.init();
    if (r.get(1) == 0) {
#pragma unroll
        for (int i = 0; i < 64; ++i) x[i] = 0.0f;
        if (STAGES) {
            if (st.emax) st.emax[b] = INT32_MIN;
#pragma unroll
            for (int i = 0; i < 64; ++i) {
                if (st.u) st.u[64 * b + i] = 0;
                if (st.q) st.q[64 * b + i] = 0;
            }
#pragma unroll
            for (int p = 0; p < 32; ++p)
                if (st.planes) st.planes[32 * b + p] = 0;
        }
        return;
    }
    const int emax = (int)r.get(8) - 127;
    int budget = 64 * rate - 9;
    int n = 0;
    int stop_p = -1, stop_m = 0;  // MID: where the budget ran out
    uint32_t lo[32], hi[32];
    for (int p = 31; p >= 0; --p) {
        uint64_t X = 0;
        if (budget > 0) {
            const int m = n < budget ? n : budget;
            X = r.get(m);
            budget -= m;
            int known = m;  // MID: digits of this plane read or implied (a prefix)
            // One window per group test: the test bit, the run of zeros and
            // the 1 that ends it are read together (the run is at most 62
            // bits unless it reaches the last coefficient or the budget).
            // The body has no branches: a negative test, a run that reaches
            // the last coefficient (its 1 implied) or the end of the budget,
            // and an ordinary run only select different updates.
            bool more = n < 64 && budget > 0;
            while (more) {
                const uint64_t win = r.window();
                const int b1 = budget - 1;                   // the test bit
                const bool neg = !(win & 1);                 // no more ones in this plane
                const uint64_t rest = win >> 1;
                int z = rest ? __builtin_ctzll(rest) : 63;  // zeros before the next 1
                z = min(z, 63 - n);
                z = min(z, b1);
                const int n1 = n + z, b2 = b1 - z;
                const bool last = n1 == 63;
                const bool stop = last || b2 == 0;
                X |= (!neg && !stop) ? (uint64_t)1 << n1 : 0;
                X |= (!neg && last) ? (uint64_t)1 << 63 : 0;
                r.skip(neg ? 1 : (stop ? 1 + z : 2 + z));
                if (MID) known = (neg || last) ? 64 : (stop ? n1 : n1 + 1);
                n = neg ? n : (last ? 64 : (stop ? n1 : n1 + 1));
                budget = neg ? b1 : (stop ? b2 : b2 - 1);
                more = !neg && !stop && budget > 0;
            }
            if (MID && budget == 0 && stop_p < 0) {
                stop_p = known < 64 ? p : p - 1;
                stop_m = known < 64 ? known : 0;
            }
        }
        const int pu = __builtin_amdgcn_readfirstlane(p);  // uniform: plain register indexing
        lo[pu] = (uint32_t)X;
        hi[pu] = (uint32_t)(X >> 32);
        if (STAGES && st.planes) st.planes[32 * b + p] = X;
    }
    uint32_t u[64];
    coefficients_of(lo, hi, u);
    int t[64];
    if (MID) {
        const uint32_t off_a = stop_p >= 0 ? midpoint_offset(stop_p) : 0u;
        const uint32_t off_b = stop_p >= 0 ? midpoint_offset(stop_p + 1) : 0u;
        from_sequency_mid(u, t, stop_m, off_a, off_b, std::make_integer_sequence<int, 64>{});
    } else {
        from_sequency(u, t, std::make_integer_sequence<int, 64>{});
    }
    inv_xform(t);
    if (STAGES) {
        if (st.emax) st.emax[b] = emax;
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            if (st.u) st.u[64 * b + i] = u[i];
            if (st.q) st.q[64 * b + i] = t[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = ldexpf((float)t[i], emax - 30);
}

// ---- wave-level movement of block words between global memory and LDS ------
// The 64 blocks of a wave own words [0, 64*rate) of `g` (block-major:
// block k's word w at k*rate + w). LDS holds them transposed (w*64 + k).
__device__ inline void words_to_lds(const uint64_t* g, uint64_t* lds, int rate, int nblocks, int lane)
{
    const int total = 64 * rate;
    for (int f = lane; f < total; f += 64) {
        const int k = f / rate, w = f - k * rate;
        lds[w * 64 + k] = k < nblocks ? g[f] : 0;
    }
}

__device__ inline void lds_to_words(const uint64_t* lds, uint64_t* g, int rate, int nblocks, int lane)
{
    const int total = nblocks * rate;
    for (int f = lane; f < total; f += 64) {
        const int k = f / rate, w = f - k * rate;
        g[f] = lds[w * 64 + k];
    }
}

}  // namespace codec
}  // namespace oocs
