// codec_dev.hpp -- gfx950 device code of the fixed-rate 4^3 block codec
// (Sec. IV: fixed rate, the user chooses the bits kept per value; transform
// of Lindstrom, IEEE TVCG 20(12), 2014).
//
// Mapping: one 64-lane wavefront codes one block; lane i holds value i of
// the block (i = x + 4y + 16z inside the block). The three separable
// lifting passes exchange the four values of each line with lane shuffles,
// the 32 bit planes come out of 32 ballots (bit k of plane p = bit p of
// coefficient k), and the variable-length group-test code is produced (or
// parsed) by code that is uniform across the wave, so it runs once per
// block rather than once per lane. Every lane keeps one 64-bit output word
// (lane w owns word w of the block) and stores it with an ordinary vector
// store.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oocs {
namespace codec {

// Total-sequency order of the 64 coefficients: by i+j+l, then i^2+j^2+l^2,
// then (l, j, i) lexicographically. fwd[k] = in-block index of the k-th
// coefficient; inv[idx] = its position k.
struct SeqOrder {
    int8_t fwd[64];
    int8_t inv[64];
};

constexpr int seq_key(int idx)
{
    // (s, e, l, j, i) packed so that integer order = lexicographic order
    return (((((idx & 3) + ((idx >> 2) & 3) + (idx >> 4)) * 32 +
              ((idx & 3) * (idx & 3) + ((idx >> 2) & 3) * ((idx >> 2) & 3) + (idx >> 4) * (idx >> 4))) * 4 +
             (idx >> 4)) * 4 + ((idx >> 2) & 3)) * 4 + (idx & 3);
}

constexpr SeqOrder make_seq_order()
{
    SeqOrder o{};
    // rank of each index = number of indices with a smaller key
    for (int idx = 0; idx < 64; ++idx) {
        int rank = 0;
        for (int other = 0; other < 64; ++other) rank += seq_key(other) < seq_key(idx);
        o.inv[idx] = (int8_t)rank;
        o.fwd[rank] = (int8_t)idx;
    }
    return o;
}

__constant__ const SeqOrder kSeq = make_seq_order();

// ---- lifting ----------------------------------------------------------------
// Arithmetic in uint32 (wrap-around is defined); >> is an arithmetic shift.
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

// One pass along the axis whose in-block stride is S (1 = x, 4 = y, 16 = z).
template <bool INVERSE>
__device__ inline int lift_pass(int v, int lane, int S)
{
    const int pos = (lane / S) & 3;
    const int base = lane - pos * S;
    int a = __shfl(v, base);
    int b = __shfl(v, base + S);
    int c = __shfl(v, base + 2 * S);
    int d = __shfl(v, base + 3 * S);
    if (INVERSE) inv_lift(a, b, c, d); else fwd_lift(a, b, c, d);
    return pos == 0 ? a : (pos == 1 ? b : (pos == 2 ? c : d));
}

constexpr uint32_t kNB = 0xAAAAAAAAu;  // negabinary mask

__device__ inline int exponent_of(float x)
{
    int e = __builtin_amdgcn_frexp_expf(x);
    return e < -126 ? -126 : e;
}

__device__ inline uint64_t readlane64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Appends bits to a block stream held one word per lane (uniform control).
struct BitSink {
    uint64_t acc;   // partially filled word
    int off;        // bits already in acc
    int wi;         // index of the word being filled
    int budget;     // bits still allowed
    uint64_t mine;  // this lane's finished word
    int lane;

    __device__ void put(uint64_t v, int m)
    {
        if (m > budget) m = budget;
        if (m <= 0) return;
        if (m < 64) v &= ((uint64_t)1 << m) - 1;
        acc |= v << off;
        int end = off + m;
        if (end >= 64) {
            if (lane == wi) mine = acc;
            ++wi;
            acc = off == 0 ? 0 : (v >> (64 - off));
            end -= 64;
        }
        off = end;
        budget -= m;
    }
    __device__ void finish()
    {
        if (off > 0 && lane == wi) mine = acc;
    }
};

struct EncStageOut {
    int32_t* emax; int32_t* q; int32_t* t; uint32_t* u; uint64_t* planes; int32_t* bits;
};

// Encode one block. `v` is this lane's value (natural order). Returns the
// lane's output word (valid for lanes < rate).
template <bool STAGES>
__device__ inline uint64_t encode_block(float v, int lane, int rate, EncStageOut st = {}, int64_t b = 0)
{
    // 1. common exponent
    int e = v != 0.0f ? exponent_of(v) : -1000;
    for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o));
    const int emax = __builtin_amdgcn_readfirstlane(e);
    BitSink s{0, 0, 0, 64 * rate, 0, lane};
    if (emax == -1000) {  // all-zero block: a single 0 bit
        if (STAGES) {
            if (lane == 0) { if (st.emax) st.emax[b] = INT32_MIN; if (st.bits) st.bits[b] = 1; }
            if (st.q) st.q[64 * b + lane] = 0;
            if (st.t) st.t[64 * b + lane] = 0;
            if (st.u) st.u[64 * b + lane] = 0;
            if (st.planes && lane < 32) st.planes[32 * b + lane] = 0;
        }
        return 0;
    }
    // 2. block floating point: exact scaling, then truncation toward zero
    const int q = (int)ldexpf(v, 30 - emax);
    // 3. forward transform along x, y, z
    int t = lift_pass<false>(q, lane, 1);
    t = lift_pass<false>(t, lane, 4);
    t = lift_pass<false>(t, lane, 16);
    // 4. sequency order and negabinary
    const int tk = __shfl(t, (int)kSeq.fwd[lane]);
    const uint32_t u = ((uint32_t)tk + kNB) ^ kNB;
    if (STAGES) {
        if (lane == 0 && st.emax) st.emax[b] = emax;
        if (st.q) st.q[64 * b + lane] = q;
        if (st.t) st.t[64 * b + lane] = t;
        if (st.u) st.u[64 * b + lane] = u;
    }
    // 5. header: 1, then emax + 127 (8 bits, least significant first)
    s.put(1u | ((uint64_t)(uint32_t)(emax + 127) << 1), 9);
    // 6. bit planes with group testing
    int n = 0;  // coefficients already significant (uniform)
    for (int p = 31; p >= 0; --p) {
        const uint64_t X = __ballot((u >> p) & 1u);
        if (STAGES && st.planes && lane == 0) st.planes[32 * b + p] = X;
        if (s.budget <= 0) {
            if (STAGES) continue;
            break;
        }
        s.put(X, n);  // verbatim bits of the significant coefficients
        while (n < 64 && s.budget > 0) {
            const uint64_t Y = X >> n;
            if (Y == 0) { s.put(0, 1); break; }
            const int m = __builtin_ctzll(Y);  // zeros before the next 1
            if (n + m == 63) {                 // that 1 is the last coefficient: implied
                s.put(1, 1 + m);
                n = 64;
                break;
            }
            s.put(1u | ((uint64_t)1 << (m + 1)), m + 2);  // test 1, m zeros, the 1
            n += m + 1;
        }
    }
    if (STAGES && st.bits && lane == 0) st.bits[b] = 64 * rate - s.budget;
    s.finish();
    return s.mine;
}

struct DecStageOut {
    int32_t* emax; uint64_t* planes; uint32_t* u; int32_t* q;
};

// Reads a block stream held one word per lane (uniform control).
struct BitSource {
    uint64_t mine;  // this lane's word (0 beyond the block)
    int pos;

    __device__ uint64_t window() const  // 64 bits starting at pos
    {
        const int wi = pos >> 6, off = pos & 63;
        const uint64_t w0 = readlane64(mine, wi);
        if (off == 0) return w0;
        const uint64_t w1 = wi + 1 < 64 ? readlane64(mine, wi + 1) : 0;
        return (w0 >> off) | (w1 << (64 - off));
    }
    __device__ uint64_t get(int m)  // m in [0, 64]
    {
        if (m <= 0) return 0;
        uint64_t v = window();
        if (m < 64) v &= ((uint64_t)1 << m) - 1;
        pos += m;
        return v;
    }
};

// Decode one block; `word` is this lane's word of the block (0 for lanes >=
// rate). Returns this lane's value (natural order).
template <bool STAGES>
__device__ inline float decode_block(uint64_t word, int lane, int rate, DecStageOut st = {}, int64_t b = 0)
{
    BitSource s{word, 0};
    if (s.get(1) == 0) {
        if (STAGES) {
            if (lane == 0 && st.emax) st.emax[b] = INT32_MIN;
            if (st.planes && lane < 32) st.planes[32 * b + lane] = 0;
            if (st.u) st.u[64 * b + lane] = 0;
            if (st.q) st.q[64 * b + lane] = 0;
        }
        return 0.0f;
    }
    const int emax = (int)s.get(8) - 127;
    int budget = 64 * rate - 9;
    int n = 0;
    uint32_t u = 0;
    for (int p = 31; p >= 0; --p) {
        uint64_t X = 0;
        if (budget > 0) {
            const int m = n < budget ? n : budget;
            X = s.get(m);
            budget -= m;
            while (n < 64 && budget > 0) {
                const uint64_t g = s.get(1);
                --budget;
                if (!g) break;
                const uint64_t win = s.window();
                int z = win ? __builtin_ctzll(win) : 64;  // zeros before the next 1
                const int maxscan = 63 - n;
                if (z > maxscan) z = maxscan;
                if (z > budget) z = budget;
                s.pos += z; budget -= z; n += z;
                if (n == 63) { X |= (uint64_t)1 << 63; n = 64; break; }
                if (budget == 0) break;
                s.pos += 1; --budget;  // the 1 that ends the run
                X |= (uint64_t)1 << n;
                ++n;
            }
        }
        if (STAGES && st.planes && lane == 0) st.planes[32 * b + p] = X;
        u = (u << 1) | (uint32_t)((X >> lane) & 1u);
    }
    // inverse negabinary (lane k = sequency position k), back to natural order
    const int qk = (int)((u ^ kNB) - kNB);
    int q = __shfl(qk, (int)kSeq.inv[lane]);
    q = lift_pass<true>(q, lane, 16);
    q = lift_pass<true>(q, lane, 4);
    q = lift_pass<true>(q, lane, 1);
    if (STAGES) {
        if (lane == 0 && st.emax) st.emax[b] = emax;
        if (st.u) st.u[64 * b + lane] = u;
        if (st.q) st.q[64 * b + lane] = q;
    }
    return ldexpf((float)q, emax - 30);
}

}  // namespace codec
}  // namespace oocs
