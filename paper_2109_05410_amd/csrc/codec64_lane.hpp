// codec64_lane.hpp -- one lane per 4^3 block for the FP64 format (the
// method of the FP32 codec, Sec. IV; Lindstrom, IEEE TVCG 20(12), 2014, with
// 64-bit integers, an 11-bit exponent field and 64 bit planes).
//
// Mapping as in the FP32 lane codec: a lane holds its block's 64 values in
// registers; the lifting, the sequency reorder and the negabinary map need no
// data exchange; the 64 x 64 bit matrix of coefficients becomes 64 plane
// words through four in-register 32 x 32 bit transposes (low and high
// halves of the coefficients, coefficients 0..31 and 32..63); the group-test
// code is written or parsed by each lane on its own through the wave's LDS
// words (word w of lane L at w*64 + L). Every lane runs its own block's
// serial coding in vector registers, so a wave codes 64 blocks at once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "codec_dev.hpp"

namespace oocs {
namespace codec64 {

constexpr uint64_t kNB64 = 0xAAAAAAAAAAAAAAAAull;

__device__ inline int64_t ladd(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
__device__ inline int64_t lsub(int64_t a, int64_t b) { return (int64_t)((uint64_t)a - (uint64_t)b); }

__device__ inline void lane_fwd_lift(int64_t& a, int64_t& b, int64_t& c, int64_t& d)
{
    a = ladd(a, d) >> 1; d = lsub(d, a);
    c = ladd(c, b) >> 1; b = lsub(b, c);
    a = ladd(a, c) >> 1; c = lsub(c, a);
    d = ladd(d, b) >> 1; b = lsub(b, d);
    d = ladd(d, b >> 1); b = lsub(b, d >> 1);
}

__device__ inline void lane_inv_lift(int64_t& a, int64_t& b, int64_t& c, int64_t& d)
{
    b = ladd(b, d >> 1); d = lsub(d, b >> 1);
    b = ladd(b, d);      d = lsub(ladd(d, d), b);
    c = ladd(c, a);      a = lsub(ladd(a, a), c);
    b = ladd(b, c);      c = lsub(ladd(c, c), b);
    d = ladd(d, a);      a = lsub(ladd(a, a), d);
}

// Along x, then y, then z (in-block index i + 4j + 16l).
__device__ inline void lane_fwd_xform(int64_t (&v)[64])
{
#pragma unroll
    for (int o = 0; o < 16; ++o) lane_fwd_lift(v[4 * o], v[4 * o + 1], v[4 * o + 2], v[4 * o + 3]);
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            lane_fwd_lift(v[16 * l + i], v[16 * l + i + 4], v[16 * l + i + 8], v[16 * l + i + 12]);
#pragma unroll
    for (int o = 0; o < 16; ++o) lane_fwd_lift(v[o], v[o + 16], v[o + 32], v[o + 48]);
}

// Along z, then y, then x.
__device__ inline void lane_inv_xform(int64_t (&v)[64])
{
#pragma unroll
    for (int o = 0; o < 16; ++o) lane_inv_lift(v[o], v[o + 16], v[o + 32], v[o + 48]);
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            lane_inv_lift(v[16 * l + i], v[16 * l + i + 4], v[16 * l + i + 8], v[16 * l + i + 12]);
#pragma unroll
    for (int o = 0; o < 16; ++o) lane_inv_lift(v[4 * o], v[4 * o + 1], v[4 * o + 2], v[4 * o + 3]);
}

// Negabinary coefficients in sequency order, split into low and high words.
template <int... K>
__device__ inline void lane_to_sequency(const int64_t (&t)[64], uint32_t (&lo)[64], uint32_t (&hi)[64],
                                        std::integer_sequence<int, K...>)
{
    ((lo[K] = (uint32_t)(((uint64_t)t[codec::kFwd<K>] + kNB64) ^ kNB64),
      hi[K] = (uint32_t)((((uint64_t)t[codec::kFwd<K>] + kNB64) ^ kNB64) >> 32)), ...);
}

template <int... I>
__device__ inline void lane_from_sequency(const uint32_t (&lo)[64], const uint32_t (&hi)[64], int64_t (&t)[64],
                                          std::integer_sequence<int, I...>)
{
    ((t[I] = (int64_t)(((((uint64_t)hi[codec::kRank<I>] << 32) | lo[codec::kRank<I>]) ^ kNB64) - kNB64)), ...);
}

__device__ inline int lane_exponent(double x)
{
    const int e = __builtin_amdgcn_frexp_exp(x);
    return e < -1022 ? -1022 : e;
}

struct LaneEncOut {
    int32_t* emax; int64_t* q; int64_t* t; uint64_t* u; uint64_t* planes; int32_t* bits;
};
struct LaneDecOut {
    int32_t* emax; uint64_t* planes; uint64_t* u; int64_t* q;
};

// The group tests of one plane after its verbatim bits (the FP32 coder's
// rule, 64 coefficients): for each 1 of X at or above n, a positive test and
// the bits up to and including that 1 (the last coefficient's 1 implied);
// then a negative test if coefficients remain. Written as one string of at
// most 127 bits with two puts; truncation at the budget happens in put.
__device__ inline void lane_code_plane(uint64_t X, int& n, codec::LaneWriter& w)
{
    w.put(X, n);
    if (n >= 64 || w.budget <= 0) return;
    uint64_t c0 = 0, c1 = 0;
    int len = 0;
    auto append = [&](uint64_t v, int l) {  // l in [1, 64], len + l <= 127
        c0 |= len < 64 ? v << len : 0;
        c1 |= len == 0 ? 0 : (len < 64 ? v >> (64 - len) : v << (len - 64));
        len += l;
    };
    uint64_t Y = X >> n;
    while (Y != 0) {
        const int m = __builtin_ctzll(Y);
        if (n + m == 63) {
            append(1, 1 + m);
            n = 64;
            break;
        }
        append(1u | ((uint64_t)1 << (m + 1)), m + 2);
        n += m + 1;
        Y >>= m + 1;
    }
    if (n < 64) append(0, 1);
    w.put(c0, min(len, 64));
    if (len > 64) w.put(c1, len - 64);
}

// Encode this lane's block x[64] (natural order) into words w*64 of `lds`
// (rate words, zero padded).
template <bool STAGES>
__device__ inline void encode_lane64(const double (&x)[64], int rate, uint64_t* lds, LaneEncOut st = {}, int64_t b = 0)
{
    int emax = -100000;
#pragma unroll
    for (int i = 0; i < 64; ++i)
        if (x[i] != 0.0) emax = max(emax, lane_exponent(x[i]));
    codec::LaneWriter w{lds, 0, 0, 0, 64 * rate};
    if (emax == -100000) {  // all-zero block: a single 0 bit
        w.put(0, 1);
        if (STAGES) {
            if (st.emax) st.emax[b] = INT32_MIN;
            if (st.bits) st.bits[b] = 1;
            for (int i = 0; i < 64; ++i) {
                if (st.q) st.q[64 * b + i] = 0;
                if (st.t) st.t[64 * b + i] = 0;
                if (st.u) st.u[64 * b + i] = 0;
                if (st.planes) st.planes[64 * b + i] = 0;
            }
        }
    } else {
        int64_t t[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) t[i] = (int64_t)ldexp(x[i], 62 - emax);  // exact scaling, truncation
        if (STAGES) {
            if (st.emax) st.emax[b] = emax;
            for (int i = 0; i < 64; ++i)
                if (st.q) st.q[64 * b + i] = t[i];
        }
        lane_fwd_xform(t);
        if (STAGES)
            for (int i = 0; i < 64; ++i)
                if (st.t) st.t[64 * b + i] = t[i];
        uint32_t ulo[64], uhi[64];
        lane_to_sequency(t, ulo, uhi, std::make_integer_sequence<int, 64>{});
        if (STAGES)
            for (int i = 0; i < 64; ++i)
                if (st.u) st.u[64 * b + i] = ((uint64_t)uhi[i] << 32) | ulo[i];
        // planes 0..31 from the low words, 32..63 from the high words
        uint32_t alo[32], ahi[32], clo[32], chi[32];
        codec::planes_of(ulo, alo, ahi);
        codec::planes_of(uhi, clo, chi);
        if (STAGES && st.planes) {
            for (int p = 0; p < 32; ++p) {
                st.planes[64 * b + p] = codec::plane_word(alo[p], ahi[p]);
                st.planes[64 * b + 32 + p] = codec::plane_word(clo[p], chi[p]);
            }
        }
        w.put(1u | ((uint64_t)(uint32_t)(emax + 1023) << 1), 12);
        int n = 0;  // coefficients already significant
        for (int p = 31; p >= 0; --p) {
            if (w.budget <= 0) break;
            const int pu = __builtin_amdgcn_readfirstlane(p);  // uniform: plain register indexing
            lane_code_plane(codec::plane_word(clo[pu], chi[pu]), n, w);
        }
        for (int p = 31; p >= 0; --p) {
            if (w.budget <= 0) break;
            const int pu = __builtin_amdgcn_readfirstlane(p);
            lane_code_plane(codec::plane_word(alo[pu], ahi[pu]), n, w);
        }
    }
    if (STAGES && st.bits && emax != -100000) st.bits[b] = 64 * rate - w.budget;
    if (w.off > 0) { lds[w.wi * 64] = w.acc; ++w.wi; }
    for (int k = w.wi; k < rate; ++k) lds[k * 64] = 0;
}

// One plane of the decoder: verbatim bits of the n significant
// coefficients, then the group tests (the FP32 decoder's body).
__device__ inline uint64_t lane_decode_plane(int& n, int& budget, codec::LaneReader& r)
{
    uint64_t X = 0;
    if (budget <= 0) return 0;
    const int m = n < budget ? n : budget;
    X = r.get(m);
    budget -= m;
    bool more = n < 64 && budget > 0;
    while (more) {
        const uint64_t win = r.window();
        const int b1 = budget - 1;                  // the test bit
        const bool neg = !(win & 1);                // no more ones in this plane
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
        n = neg ? n : (last ? 64 : (stop ? n1 : n1 + 1));
        budget = neg ? b1 : (stop ? b2 : b2 - 1);
        more = !neg && !stop && budget > 0;
    }
    return X;
}

// Decode this lane's block from words w*64 of `lds` into x[64] (natural order).
template <bool STAGES>
__device__ inline void decode_lane64(const uint64_t* lds, int rate, double (&x)[64], LaneDecOut st = {}, int64_t b = 0)
{
    codec::LaneReader r{lds, rate, 0, 0, 0, 0, 0, 0};
    r.init();
    if (r.get(1) == 0) {
#pragma unroll
        for (int i = 0; i < 64; ++i) x[i] = 0.0;
        if (STAGES) {
            if (st.emax) st.emax[b] = INT32_MIN;
            for (int i = 0; i < 64; ++i) {
                if (st.u) st.u[64 * b + i] = 0;
                if (st.q) st.q[64 * b + i] = 0;
                if (st.planes) st.planes[64 * b + i] = 0;
            }
        }
        return;
    }
    const int emax = (int)r.get(11) - 1023;
    int budget = 64 * rate - 12;
    int n = 0;
    uint32_t alo[32], ahi[32], clo[32], chi[32];
    for (int p = 31; p >= 0; --p) {  // planes 63..32
        const uint64_t X = lane_decode_plane(n, budget, r);
        const int pu = __builtin_amdgcn_readfirstlane(p);
        clo[pu] = (uint32_t)X;
        chi[pu] = (uint32_t)(X >> 32);
        if (STAGES && st.planes) st.planes[64 * b + 32 + p] = X;
    }
    for (int p = 31; p >= 0; --p) {  // planes 31..0
        const uint64_t X = lane_decode_plane(n, budget, r);
        const int pu = __builtin_amdgcn_readfirstlane(p);
        alo[pu] = (uint32_t)X;
        ahi[pu] = (uint32_t)(X >> 32);
        if (STAGES && st.planes) st.planes[64 * b + p] = X;
    }
    uint32_t ulo[64], uhi[64];
    codec::coefficients_of(alo, ahi, ulo);
    codec::coefficients_of(clo, chi, uhi);
    int64_t t[64];
    lane_from_sequency(ulo, uhi, t, std::make_integer_sequence<int, 64>{});
    lane_inv_xform(t);
    if (STAGES) {
        if (st.emax) st.emax[b] = emax;
        for (int i = 0; i < 64; ++i) {
            if (st.u) st.u[64 * b + i] = ((uint64_t)uhi[i] << 32) | ulo[i];
            if (st.q) st.q[64 * b + i] = t[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = ldexp((double)t[i], emax - 62);
}

}  // namespace codec64
}  // namespace oocs
