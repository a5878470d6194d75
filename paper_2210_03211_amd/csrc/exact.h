// exact.h -- order-free exact summation of FP64 values on the GPU.
//
// Every sum that feeds a LazyFox decision (per-community sums of the WCC-hat node terms,
// the join/leave corrections, the global cc) and the partition score are accumulated
// exactly in fixed point and rounded once to the nearest double (ties to even).  The
// result therefore does not depend on summation order, thread count or reduction shape.
//
//  X192  two's-complement 192-bit integer, weight of the lowest bit 2^-120.  Holds the node
//        terms g in (2^-62, 1] (lowest set bit >= 2^-114), local CCs, and any sum of up to
//        2^31 of them.
//  X256  two's-complement 256-bit integer, lowest bit 2^-192.  Holds community scores
//        p * R(sum g) in (2^-124, 2^31) (lowest set bit >= 2^-176) and their sum.
//  Digits: for atomics, a signed 128-bit term is split into four 32-bit digits (three
//        unsigned, the top one signed) that are added into four signed 64-bit counters;
//        the counters are folded back into an X192 once all terms are in.
//
// A value that cannot be represented exactly sets a flag that the host turns into an error.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned long long u64;
typedef long long i64;

struct X192 { u64 w0, w1, w2; };
struct X256 { u64 w0, w1, w2, w3; };

__device__ __forceinline__ u64 addc64(u64 a, u64 b, u64 &carry)
{
    u64 s = a + b;
    u64 c1 = s < a;
    u64 s2 = s + carry;
    u64 c2 = s2 < s;
    carry = c1 | c2;
    return s2;
}

__device__ __forceinline__ X192 x192_zero() { X192 r = {0, 0, 0}; return r; }
__device__ __forceinline__ X256 x256_zero() { X256 r = {0, 0, 0, 0}; return r; }

__device__ __forceinline__ void x192_add(X192 &a, const X192 &b)
{
    u64 c = 0;
    a.w0 = addc64(a.w0, b.w0, c);
    a.w1 = addc64(a.w1, b.w1, c);
    a.w2 = addc64(a.w2, b.w2, c);
}

__device__ __forceinline__ void x256_add(X256 &a, const X256 &b)
{
    u64 c = 0;
    a.w0 = addc64(a.w0, b.w0, c);
    a.w1 = addc64(a.w1, b.w1, c);
    a.w2 = addc64(a.w2, b.w2, c);
    a.w3 = addc64(a.w3, b.w3, c);
}

__device__ __forceinline__ X192 x192_neg(X192 a)
{
    X192 r;
    u64 c = 1;
    r.w0 = addc64(~a.w0, 0, c);
    r.w1 = addc64(~a.w1, 0, c);
    r.w2 = addc64(~a.w2, 0, c);
    return r;
}

__device__ __forceinline__ void x192_sub(X192 &a, const X192 &b)
{
    X192 nb = x192_neg(b);
    x192_add(a, nb);
}

// Split a double into (53-bit integer mantissa, shift) relative to a fixed point whose
// lowest bit weighs 2^-lsb.  Returns false for zero.  *bad is set if inexact / too large.
__device__ __forceinline__ bool fx_split(double v, int lsb, u64 &mant, int &sh, bool &neg, int &bad)
{
    u64 bits = (u64)__double_as_longlong(v);
    neg = (bits >> 63) != 0;
    int e = (int)((bits >> 52) & 0x7ff);
    u64 m = bits & 0xFFFFFFFFFFFFFull;
    if (e == 0) {
        if (m != 0) bad = 1;      // subnormal: far below any representable lowest bit
        return false;
    }
    if (e == 0x7ff) { bad = 1; return false; }
    mant = m | (1ull << 52);
    sh = e - 1075 + lsb;          // weight of mant's lowest bit, in bits above the fixed LSB
    if (sh < 0) {
        // exact only if the bits shifted out are zero
        if (sh <= -53 || (mant & ((1ull << (-sh)) - 1)) != 0) bad = 1;
        mant = (sh <= -53) ? 0 : (mant >> (-sh));
        sh = 0;
    }
    return true;
}

// v -> X192 (lowest bit 2^-120); |v| < 2^70
__device__ __forceinline__ X192 x192_from_double(double v, int &bad)
{
    X192 r = x192_zero();
    u64 mant; int sh; bool neg;
    if (!fx_split(v, 120, mant, sh, neg, bad)) return r;
    int li = sh >> 6, bi = sh & 63;
    u64 lo = mant << bi;
    u64 hi = bi > 11 ? (mant >> (64 - bi)) : 0;
    if (li == 0) { r.w0 = lo; r.w1 = hi; }
    else if (li == 1) { r.w1 = lo; r.w2 = hi; }
    else if (li == 2 && hi == 0) { r.w2 = lo; }
    else { bad = 1; }
    if ((i64)r.w2 < 0) bad = 1;
    return neg ? x192_neg(r) : r;
}

// v >= 0 -> X256 (lowest bit 2^-192); v < 2^62
__device__ __forceinline__ X256 x256_from_double(double v, int &bad)
{
    X256 r = x256_zero();
    u64 mant; int sh; bool neg;
    if (!fx_split(v, 192, mant, sh, neg, bad)) return r;
    if (neg) { bad = 1; return r; }
    int li = sh >> 6, bi = sh & 63;
    u64 lo = mant << bi;
    u64 hi = bi > 11 ? (mant >> (64 - bi)) : 0;
    if (li == 0) { r.w0 = lo; r.w1 = hi; }
    else if (li == 1) { r.w1 = lo; r.w2 = hi; }
    else if (li == 2) { r.w2 = lo; r.w3 = hi; }
    else if (li == 3 && hi == 0) { r.w3 = lo; }
    else { bad = 1; }
    if ((i64)r.w3 < 0) bad = 1;
    return r;
}

// Round the non-negative magnitude (h = bits [top-63, top], sticky = any lower bit) to a
// double: keep 53 bits, round to nearest, ties to even.  value = H * 2^(top - 63 - lsb).
__device__ __forceinline__ double fx_round_top64(u64 H, bool sticky, int top, int lsb)
{
    u64 mant = H >> 11;
    u64 rbit = (H >> 10) & 1;
    bool st = sticky || (H & 0x3ffull) != 0;
    if (rbit && (st || (mant & 1))) mant++;
    int E = top - 52 - lsb;       // value = mant * 2^E
    if (mant == (1ull << 53)) { mant >>= 1; E++; }
    u64 bits = ((u64)(E + 52 + 1023) << 52) | (mant & 0xFFFFFFFFFFFFFull);
    return __longlong_as_double((i64)bits);
}

__device__ __forceinline__ double x192_round(X192 a)
{
    bool neg = (i64)a.w2 < 0;
    if (neg) a = x192_neg(a);
    int top;
    if (a.w2) top = 128 + 63 - __clzll((i64)a.w2);
    else if (a.w1) top = 64 + 63 - __clzll((i64)a.w1);
    else if (a.w0) top = 63 - __clzll((i64)a.w0);
    else return 0.0;
    // left-normalise so that bit `top` lands on bit 191
    int s = 191 - top;
    int q = s >> 6, r = s & 63;
    u64 a0 = a.w0, a1 = a.w1, a2 = a.w2;
    if (q == 1) { a2 = a1; a1 = a0; a0 = 0; }
    else if (q == 2) { a2 = a0; a1 = 0; a0 = 0; }
    if (r) { a2 = (a2 << r) | (a1 >> (64 - r)); a1 = (a1 << r) | (a0 >> (64 - r)); a0 <<= r; }
    double d = fx_round_top64(a2, (a1 | a0) != 0, top, 120);
    return neg ? -d : d;
}

__device__ __forceinline__ double x256_round(X256 a)   // a >= 0
{
    int top;
    if (a.w3) top = 192 + 63 - __clzll((i64)a.w3);
    else if (a.w2) top = 128 + 63 - __clzll((i64)a.w2);
    else if (a.w1) top = 64 + 63 - __clzll((i64)a.w1);
    else if (a.w0) top = 63 - __clzll((i64)a.w0);
    else return 0.0;
    int s = 255 - top;
    int q = s >> 6, r = s & 63;
    u64 a0 = a.w0, a1 = a.w1, a2 = a.w2, a3 = a.w3;
    for (int k = 0; k < q; k++) { a3 = a2; a2 = a1; a1 = a0; a0 = 0; }
    if (r) {
        a3 = (a3 << r) | (a2 >> (64 - r));
        a2 = (a2 << r) | (a1 >> (64 - r));
        a1 = (a1 << r) | (a0 >> (64 - r));
        a0 <<= r;
    }
    return fx_round_top64(a3, (a2 | a1 | a0) != 0, top, 192);
}

// ---- digit form (for atomics) ----------------------------------------------------------
// A term t with |t| < 2^127 (in units of 2^-120) as four 32-bit digits: d0..d2 unsigned,
// d3 signed, t = d0 + d1 2^32 + d2 2^64 + d3 2^96.
__device__ __forceinline__ void x192_digits(const X192 &t, i64 &d0, i64 &d1, i64 &d2, i64 &d3)
{
    d0 = (i64)(t.w0 & 0xffffffffull);
    d1 = (i64)(t.w0 >> 32);
    d2 = (i64)(t.w1 & 0xffffffffull);
    d3 = (i64)(int)(unsigned)(t.w1 >> 32);
}

__device__ __forceinline__ X192 x192_sext(i64 v)
{
    X192 r;
    r.w0 = (u64)v;
    r.w1 = r.w2 = (v < 0) ? ~0ull : 0ull;
    return r;
}

// sum_k D_k 2^(32k), each D_k a signed 64-bit digit counter
__device__ __forceinline__ X192 x192_from_digits(i64 D0, i64 D1, i64 D2, i64 D3)
{
    X192 r = x192_sext(D0);
    u64 s1 = (D1 < 0) ? ~0ull : 0ull, s3 = (D3 < 0) ? ~0ull : 0ull;
    X192 t1 = {(u64)D1 << 32, (u64)(D1 >> 32), s1};
    X192 t2 = {0, (u64)D2, (D2 < 0) ? ~0ull : 0ull};
    X192 t3 = {0, (u64)D3 << 32, (u64)(D3 >> 32)};
    (void)s3;
    x192_add(r, t1);
    x192_add(r, t2);
    x192_add(r, t3);
    return r;
}

// ---- wave-level reductions (wave64) ----------------------------------------------------
__device__ __forceinline__ u64 shfl_xor_u64(u64 v, int m)
{
    return (u64)__shfl_xor((long long)v, m, 64);
}

__device__ __forceinline__ X192 wave_sum_x192(X192 v)
{
    for (int m = 32; m >= 1; m >>= 1) {
        X192 o = {shfl_xor_u64(v.w0, m), shfl_xor_u64(v.w1, m), shfl_xor_u64(v.w2, m)};
        x192_add(v, o);
    }
    return v;
}

__device__ __forceinline__ X256 wave_sum_x256(X256 v)
{
    for (int m = 32; m >= 1; m >>= 1) {
        X256 o = {shfl_xor_u64(v.w0, m), shfl_xor_u64(v.w1, m), shfl_xor_u64(v.w2, m),
                  shfl_xor_u64(v.w3, m)};
        x256_add(v, o);
    }
    return v;
}

__device__ __forceinline__ i64 wave_sum_i64(i64 v)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
