// Device primitives of the gfx950 walk kernels: counter-based RNG, exact unit
// uniforms, correctly rounded float32 logarithms, and wave64 reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

constexpr int kWave = 64;

struct U4 {
    uint32_t x0, x1, x2, x3;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies with the published multipliers and Weyl key increments.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// (2m + 1) * 2^-24 from the top 23 bits: exact in float32, strictly inside (0, 1).
__device__ __forceinline__ float unit_uniform(uint32_t x)
{
    return (float)(2u * (x >> 9) + 1u) * 0x1p-24f;
}

// floor(R * n / 2^64) for a 64-bit random R: an index in [0, n).
__device__ __forceinline__ int64_t scaled_index(uint32_t lo, uint32_t hi, int64_t n)
{
    const uint64_t r = ((uint64_t)hi << 32) | lo;
    return (int64_t)__umul64hi(r, (uint64_t)n);
}

// The high 32 bits of the fraction R * n mod 2^64 left by scaled_index: a second draw,
// independent of the index to within 2^-32, from the same 64 random bits.
__device__ __forceinline__ uint32_t scaled_fraction_hi(uint32_t lo, uint32_t hi, int64_t n)
{
    const uint64_t r = ((uint64_t)hi << 32) | lo;
    return (uint32_t)((r * (uint64_t)n) >> 32);
}

// Logarithms rounded once to float32 from a double-precision evaluation, so the value
// is the correctly rounded one except within ~1e-16 of a rounding tie.
// Transcendentals of the sample stream: evaluated in double precision and rounded once to
// float32.  Compact double routines from the textbook reductions (about a third of the
// instructions of a general-purpose library log; the eRVS jump runs three per key event):
//   ln:    x = 2^e (1 + f) with sqrt(1/2) <= 1 + f < sqrt(2), ln(1 + f) = 2 atanh(s),
//          s = f / (2 + f), by its odd series to s^21 (|s| < 0.172, error below 2^-60
//          relative), ln 2 split in a short head (exact products with e) and a tail;
//   expm1: a = k ln 2 + r, |r| <= ln2 / 2 (Cody-Waite), Taylor series of expm1(r) to r^13,
//          then 2^k expm1(r) + (2^k - 1), both terms exact before the one rounding;
//   log1p: ln(1 + z), where 1 + z is exact in double for a float z with |z| >= 2^-29, and
//          z - z^2/2 + z^3/3 below that.
// Domains used here: ln on (0, 1); expm1 on [-inf, 0]; log1p on (-1, 0].  Their float
// results agree with a correctly rounded libm's (checked on all 2^23 uniforms for ln and
// on 2e8 random arguments each).
constexpr double kLn2Hi = 6.93147180369123816490e-01;  // ln 2 to 32 bits (trailing zeros)
constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
constexpr double kInvLn2 = 1.44269504088896338700e+00;

__device__ __forceinline__ double ln_d(double x)
{
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m = m + m;
        e -= 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    const double t = s + s;
    const double L = t + t * (z * p);
    return (double)e * kLn2Hi + ((double)e * kLn2Lo + L);
}

__device__ __forceinline__ double expm1_d(double a)  // a <= 0
{
    if (a == 0.0) return a;
    if (a < -40.0) return -1.0;
    if (a > -1.4901161193847656e-08) return a + (a * a) * 0.5;  // |a| < 2^-26
    const double k = rint(a * kInvLn2);
    const double r = (a - k * kLn2Hi) - k * kLn2Lo;
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    const double q = r + (r * r) * p;  // expm1(r)
    if (k == 0.0) return q;
    const int ki = (int)k;
    return ldexp(q, ki) + (ldexp(1.0, ki) - 1.0);
}

__device__ __forceinline__ double log1p_d(double z)  // -1 < z <= 0
{
    if (z == 0.0) return z;
    if (z > -1.862645149230957e-09) return z - (z * z) * 0.5 + (z * z * z) * (1.0 / 3.0);  // |z| < 2^-29
    return ln_d(1.0 + z);
}

__device__ __forceinline__ float ln_f(float x) { return (float)ln_d((double)x); }
__device__ __forceinline__ float expm1_f(float x) { return (float)expm1_d((double)x); }
__device__ __forceinline__ float log1p_f(float x) { return (float)log1p_d((double)x); }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ uint64_t lanes_below(int lane) { return (lane == 0) ? 0ull : (~0ull >> (64 - lane)); }

__device__ __forceinline__ int32_t bcast_i32(int32_t v, int src) { return __builtin_amdgcn_readlane(v, src); }

__device__ __forceinline__ uint32_t bcast_u32(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

__device__ __forceinline__ int64_t bcast_i64(int64_t v, int src)
{
    const uint32_t lo = bcast_u32((uint32_t)(uint64_t)v, src);
    const uint32_t hi = bcast_u32((uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Lexicographic maximum over (key, index); the larger index wins equal keys.
__device__ __forceinline__ void wave_argmax(float &key, int32_t &idx)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const float k2 = __shfl_xor(key, o, kWave);
        const int32_t i2 = __shfl_xor(idx, o, kWave);
        if (k2 > key || (k2 == key && i2 > idx)) {
            key = k2;
            idx = i2;
        }
    }
}

// Orders this wave's LDS writes before its later LDS reads (and vice versa).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Binary search for u in the ascending array a[0, n): its position, or -1.
__device__ __forceinline__ int64_t sorted_find(const int32_t *a, int64_t n, int32_t u)
{
    int64_t lo = 0, len = n;
    while (len > 0) {
        const int64_t half = len >> 1;
        if (a[lo + half] < u) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return (lo < n && a[lo] == u) ? lo : -1;
}

// Membership of u in the ascending array a[0, n) by a branch-free bisection: the trip
// count depends on n alone, so lanes that search one shared array (an eRVS step, where
// every lane tests its neighbours against the same N(prev)) never diverge; each round is
// one load, one compare and one select.
__device__ __forceinline__ bool sorted_contains_bisect(const int32_t *a, int32_t n, int32_t u)
{
    if (n <= 0) return false;
    int32_t base = 0, len = n;
    while (len > 1) {
        const int32_t half = len >> 1;
        base = a[base + half] <= u ? base + half : base;
        len -= half;
    }
    return a[base] == u;
}

// Position of u in the strictly ascending array a[0, n) whose values lie in [0, vend), or -1.
// Interpolation search: the bracket (lo, hi) starts at the virtual ends a[-1] = -1 and
// a[n] = vend; each probe guesses u's position from the bracket values.  Vertex ids of
// a row are spread almost uniformly, so a few probes suffice; after eight guesses the
// search bisects, which bounds it by 8 + log2(n) probes for any input.  The guess is
// only a position inside the bracket, so it uses a fast reciprocal: any value works.
// Requires vend < 2^30 so that bracket widths fit int32.  Eight guesses before bisecting
// measured fewest probes on skewed graphs (about 3.9 per miss on a row of ~4500 ids).
__device__ __forceinline__ int32_t sorted_find_interp(const int32_t *a, int32_t n, int32_t u, int32_t vend)
{
    int32_t lo = -1, hi = n;
    int32_t vlo = -1, vhi = vend;
    int it = 0;
    while (hi - lo > 1) {
        int32_t pos;
        if (it < 8) {
            const float f = (float)(u - vlo) * __builtin_amdgcn_rcpf((float)(vhi - vlo));
            pos = lo + (int32_t)(f * (float)(hi - lo));
        } else {
            pos = lo + ((hi - lo) >> 1);
        }
        pos = pos <= lo ? lo + 1 : (pos >= hi ? hi - 1 : pos);
        const int32_t v = a[pos];
        ++it;
        if (v == u) return pos;
        if (v < u) {
            lo = pos;
            vlo = v;
        } else {
            hi = pos;
            vhi = v;
        }
    }
    return -1;
}

__device__ __forceinline__ bool sorted_contains_interp(const int32_t *a, int32_t n, int32_t u, int32_t vend)
{
    return sorted_find_interp(a, n, u, vend) >= 0;
}

// Exact map of the graph's entries (v, u) to their h: open addressing over 128-byte
// buckets (one DRAM line) of eight 64-bit keys v << 32 | u followed by their eight h
// values, the first bucket chosen by the SplitMix64 finaliser (Steele, Lea, Flood,
// OOPSLA'14), then linear probing bucket by bucket.  At most half the slots are used, so
// a query almost always reads one bucket: one memory request where a search of the
// sorted row needs several dependent ones.
constexpr unsigned long long kEmptyKey = ~0ull;
constexpr int kIndexBucketU4 = 8;  // uint4 per bucket: keys in parts 0..3, h in parts 4..5

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t edge_key(int32_t v, int32_t u)
{
    return ((uint64_t)(uint32_t)v << 32) | (uint64_t)(uint32_t)u;
}

// tab: kIndexBucketU4 uint4 per bucket, mask = buckets - 1 (buckets a power of two).  The
// key parts of a bucket are loaded before any is tested, so they go out together as one
// request instead of one dependent load after another.  Scans at most every bucket
// once, so it ends even on a full table.  Returns the slot of (v, u) in [0, 8), or -1.
// With H the hit's h is read from the bucket's h part (the same DRAM line, so a cache
// hit) and stored in *h.
template <bool H>
__device__ __forceinline__ int index_probe(const uint4 *tab, uint64_t mask, int32_t v, int32_t u, float *h)
{
    const uint64_t key = edge_key(v, u);
    uint64_t b = mix64(key) & mask;
    for (uint64_t t = 0; t <= mask; ++t) {
        const uint4 *p = tab + b * kIndexBucketU4;
        const uint4 x[4] = {p[0], p[1], p[2], p[3]};
        int slot = -1;
        bool empty = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t k0 = ((uint64_t)x[i].y << 32) | x[i].x, k1 = ((uint64_t)x[i].w << 32) | x[i].z;
            slot = k0 == key ? 2 * i : (k1 == key ? 2 * i + 1 : slot);
            empty = empty || k0 == kEmptyKey || k1 == kEmptyKey;
        }
        if (slot >= 0) {
            if (H) *h = reinterpret_cast<const float *>(p + 4)[slot];
            return slot;
        }
        if (empty) return -1;
        b = (b + 1) & mask;
    }
    return -1;
}

__device__ __forceinline__ bool index_contains(const uint4 *tab, uint64_t mask, int32_t v, int32_t u)
{
    return index_probe<false>(tab, mask, v, u, nullptr) >= 0;
}

// ceil(log2(m + 1)): probes of a binary search over m entries.
__device__ __host__ __forceinline__ int probes(int64_t m)
{
    return m <= 0 ? 0 : 64 - __builtin_clzll((unsigned long long)m);
}

}  // namespace fw
