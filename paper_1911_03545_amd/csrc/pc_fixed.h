// pc_fixed.h -- exact fixed-point accumulation of pair weights (the
// deterministic weight sums).
//
// The paper adds weight_func(w_i, w_j) into a binary64 bin per pair (section
// 2.1 and the histogram update of section "Finding and updating the
// histogram bins"); with atomics that sum depends on the order of the adds.
// Here every pair weight p = fl(w_i * w_j) or fl(w_i + w_j) is instead an
// exact integer multiple P = p 2^-Q of one power of two 2^Q common to the
// whole call, with |P| < 2^94.  |P| is split into three 32-bit limbs
//     |P| = m0 + m1 2^32 + m2 2^64,   m0, m1 in [0, 2^32), m2 < 2^30,
// which carry the sign of P (l_k = +-m_k) into three int64 LDS sums, and the
// sums are merged into a 192-bit two's complement integer per bin with
// carries.  Integer addition is associative, so the total is the exact sum
// whatever the order, and it is rounded to binary64 once at the end: the
// exact sum of the binary64 pair weights, correctly rounded, in every run.
//
// The grid 2^Q (found on the device, k_wfixed_plan): every weight w is a
// multiple of 2^low(w), the lowest set bit of its significand; a product of
// two weights is a multiple of 2^(low_i + low_j), a sum a multiple of
// 2^min(low_i, low_j), and rounding a multiple of 2^q to binary64 keeps it a
// multiple of 2^q (the result is either exact or a multiple of its own ulp,
// which is then at least 2^q).  A product is also a multiple of its own
// ulp, at least 2^(e_min - 52) with e_min the exponent of fl(min|w_1| *
// min|w_2|).  So Q = max(low_1 + low_2, e_min - 52) for products and
// Q = min(low_1, low_2) for sums.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc {

// Per-call grid of the fixed-point weight sums, in the misc buffer.  The
// scan kernels fill the first fields with atomic maxima over every nonzero
// weight of each side (zero-initialised), the plan kernel the rest.
struct pc_wfixed {
    uint32_t lowkey[2];             // 2100 - min low(w) (0: no nonzero weight)
    uint32_t pad[2];
    unsigned long long maxbits[2];  // bits of max |w|
    unsigned long long notmin[2];   // ~bits of min |w| (max of the complements)
    double scale;                   // 2^-Q: the lane weights are prescaled by it
    double unscale;                 // 2^Q
    int32_t q;                      // Q
    int32_t ok;                     // 1 when every pair weight fits the grid
};

// Signed limbs of P (an integer-valued double, |P| < 2^94), as two's
// complement words ready for uint64 adds.  The split works on |P| (each step
// exact: the remainders keep a subset of |P|'s significand bits) and the
// sign goes to every limb.
__host__ __device__ __forceinline__ void fixed_limbs(double P, unsigned long long &l0,
                                            unsigned long long &l1, unsigned long long &l2)
{
    const double a = fabs(P);
    const double h2 = floor(a * 0x1p-64);
    const double r1 = fma(h2, -0x1p64, a);   // in [0, 2^64)
    const double h1 = floor(r1 * 0x1p-32);
    const double r0 = fma(h1, -0x1p32, r1);  // in [0, 2^32)
    const unsigned long long m0 = (unsigned)r0, m1 = (unsigned)h1, m2 = (unsigned)h2;
    const bool neg = P < 0.0;
    l0 = neg ? 0ull - m0 : m0;
    l1 = neg ? 0ull - m1 : m1;
    l2 = neg ? 0ull - m2 : m2;
}

// Sign extension of an int64 into the upper words of a 192-bit integer.
__host__ __device__ __forceinline__ unsigned long long fixed_ext(long long x)
{
    return x < 0 ? ~0ull : 0ull;
}

// w += b (192-bit, modulo 2^192)
__host__ __device__ __forceinline__ void fixed_add(unsigned long long w[3],
                                                   const unsigned long long b[3])
{
    const unsigned long long s0 = w[0] + b[0];
    const unsigned long long c0 = s0 < w[0] ? 1ull : 0ull;
    const unsigned long long t1 = w[1] + b[1];
    const unsigned long long c1 = t1 < w[1] ? 1ull : 0ull;
    const unsigned long long s1 = t1 + c0;
    const unsigned long long c1b = s1 < t1 ? 1ull : 0ull;
    w[0] = s0;
    w[1] = s1;
    w[2] = w[2] + b[2] + c1 + c1b;
}

// Limb sums (int64 each, |s| < 2^63) as a 192-bit two's complement integer
// v0 + v1 2^64 + v2 2^128 = s0 + s1 2^32 + s2 2^64.
__host__ __device__ __forceinline__ void fixed_words(long long s0, long long s1, long long s2,
                                            unsigned long long v[3])
{
    v[0] = (unsigned long long)s0;
    v[1] = fixed_ext(s0);
    v[2] = fixed_ext(s0);
    // s1 2^32: low word s1 << 32, middle word the arithmetic shift s1 >> 32
    const unsigned long long t1[3] = {(unsigned long long)s1 << 32,
                                      (unsigned long long)(s1 >> 32), fixed_ext(s1)};
    fixed_add(v, t1);
    const unsigned long long t2[3] = {0ull, (unsigned long long)s2, fixed_ext(s2)};
    fixed_add(v, t2);
}

// g (3 words) += v modulo 2^192 with device-scope atomics: each word's carry
// out is detected by the thread whose add produced it and passed up, so the
// total is exact in any interleaving.
__device__ __forceinline__ void fixed_atomic_add(unsigned long long *g,
                                                 const unsigned long long v[3])
{
    unsigned long long carry = 0;
    if (v[0]) {
        const unsigned long long old = atomicAdd(&g[0], v[0]);
        carry = (old + v[0] < old) ? 1ull : 0ull;
    }
    const unsigned long long u1 = v[1] + carry;
    unsigned long long carry2 = (u1 < v[1]) ? 1ull : 0ull;
    if (u1) {
        const unsigned long long old = atomicAdd(&g[1], u1);
        carry2 += (old + u1 < old) ? 1ull : 0ull;
    }
    const unsigned long long u2 = v[2] + carry2;
    if (u2)
        atomicAdd(&g[2], u2);
}

// The 192-bit two's complement integer w times 2^q, rounded once to the
// nearest binary64 (ties to even).  q >= -1022 keeps every nonzero result
// normal (|w| >= 1).
__host__ __device__ __forceinline__ double fixed_to_double(const unsigned long long win[3],
                                                           int q)
{
    unsigned long long w[3] = {win[0], win[1], win[2]};
    const bool neg = (long long)w[2] < 0;
    if (neg) {
        // two's complement negation
        w[0] = ~w[0];
        w[1] = ~w[1];
        w[2] = ~w[2];
        const unsigned long long one[3] = {1ull, 0ull, 0ull};
        fixed_add(w, one);
    }
    int top;
    if (w[2])
        top = 128 + 63 - __builtin_clzll(w[2]);
    else if (w[1])
        top = 64 + 63 - __builtin_clzll(w[1]);
    else if (w[0])
        top = 63 - __builtin_clzll(w[0]);
    else
        return 0.0;
    double r;
    if (top <= 52) {
        r = ldexp((double)w[0], q);   // exact: fewer than 54 bits
    } else {
        const int sh = top - 52;      // bits below the 53-bit significand
        // significand: bits [sh, sh + 52]
        const int k = sh >> 6, o = sh & 63;
        unsigned long long m = w[k] >> o;
        if (o && k + 1 < 3)
            m |= w[k + 1] << (64 - o);
        m &= (1ull << 53) - 1ull;
        // round bit (sh - 1) and sticky bits below it
        const int rb = sh - 1;
        const bool round = (w[rb >> 6] >> (rb & 63)) & 1ull;
        bool sticky = false;
        for (int t = 0; t < 3; t++) {
            const int lo = t * 64;
            if (lo >= rb)
                break;
            const int nbits = rb - lo;   // bits of word t below the round bit
            const unsigned long long mask = nbits >= 64 ? ~0ull : ((1ull << nbits) - 1ull);
            if (w[t] & mask)
                sticky = true;
        }
        int e = sh;
        if (round && (sticky || (m & 1ull))) {
            m++;
            if (m == (1ull << 53)) {
                m >>= 1;
                e++;
            }
        }
        r = ldexp((double)m, e + q);
    }
    return neg ? -r : r;
}

}  // namespace pc
