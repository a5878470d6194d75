// method.h -- device arithmetic of the LazyFox method (WCC-hat node terms, community
// density, candidate changes), shared by the initialisation and the iteration kernels.
//
// WCC-hat (Methods, WCC-hat subsection): for a member x of community C with
// d = deg(x,V), i = deg(x,C), s = |C| and density p,
//     WCC-hat(x,C) = E[t(x,C)] / E[t(x,V)] * deg(x,V) / (|C\{x}| + deg(x,V\C))
// with E[t(x,C)] = C(i,2) p and E[t(x,V)] = C(d,2) cc, i.e. p * g(i,d,s) / cc with
//     g(i,d,s) = i(i-1) / ((d-1)(s-1+d-i)),   0 if i < 2 or d < 2 (E[t] = 0).
// cc is a positive constant, so the method's comparisons use the cc-free score
// W(C) = fl(p * R(sum_{y in C} g)), R = exact sum rounded once to nearest-even.
#pragma once
#include "lf_internal.h"

#define WAVE 64

#define WAVE_SYNC()                                                                        \
    do {                                                                                   \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");                             \
        __builtin_amdgcn_wave_barrier();                                                   \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");                             \
    } while (0)

__device__ __forceinline__ double g_term(long long i, long long d, long long s)
{
    if (d < 2 || i < 2) return 0.0;
    long long num = i * (i - 1);
    long long den = (d - 1) * (s - 1 + d - i);
    return (double)num / (double)den;
}

// density of a community with s members and m internal edges
__device__ __forceinline__ double density(long long s, long long m)
{
    if (s < 2) return 0.0;
    return (double)(2 * m) / (double)(s * (s - 1));
}

__device__ __forceinline__ X192 rec_load(const unsigned *p)
{
    X192 r;
    r.w0 = (u64)p[0] | ((u64)p[1] << 32);
    r.w1 = (u64)p[2] | ((u64)p[3] << 32);
    r.w2 = (u64)p[4];
    return r;
}

__device__ __forceinline__ void rec_store(unsigned *p, const X192 &v, int &bad)
{
    p[0] = (unsigned)v.w0;
    p[1] = (unsigned)(v.w0 >> 32);
    p[2] = (unsigned)v.w1;
    p[3] = (unsigned)(v.w1 >> 32);
    p[4] = (unsigned)v.w2;
    if (v.w2 >> 32) bad = 1;           // a stored sum is never negative nor >= 2^40
}

// write a re-summed community (members' exact sums at sizes s, s+1, s-1 and in-count sum)
__device__ __forceinline__ void store_comm(const Ctx &cx, int C, long long s, X192 a0, X192 ap, X192 am,
                                           long long sumi, int &bad)
{
    if (sumi & 1) atomicOr(&cx.ctr->error, LF_DEVERR_ODD);
    long long m = sumi / 2;
    CommRec *r = &cx.cr[C];
    r->m = m;
    r->W = density(s, m) * x192_round(a0);
    rec_store(r->Sp, ap, bad);
    rec_store(r->Sm, am, bad);
    cx.tflag[C] = 0;
}

// position of community c among a node's cnt slots (-1 if absent); *in gets its in-count
__device__ __forceinline__ int find_slot_in(const Slot *slot, long long off, int cnt, int c, int *in)
{
    for (int t = 0; t < cnt; t += 4) {         // four independent loads per round trip
        const Slot s0 = slot[off + t];
        Slot s1 = {-2, 0}, s2 = {-2, 0}, s3 = {-2, 0};
        if (t + 1 < cnt) s1 = slot[off + t + 1];
        if (t + 2 < cnt) s2 = slot[off + t + 2];
        if (t + 3 < cnt) s3 = slot[off + t + 3];
        if (s0.comm == c) { *in = s0.in; return t; }
        if (s1.comm == c) { *in = s1.in; return t + 1; }
        if (s2.comm == c) { *in = s2.in; return t + 2; }
        if (s3.comm == c) { *in = s3.in; return t + 3; }
    }
    return -1;
}

__device__ __forceinline__ int find_slot(const Slot *slot, long long off, int cnt, int c)
{
    // four independent loads per round trip (a node holds a handful of memberships)
    for (int t = 0; t < cnt; t += 4) {
        const int c0 = slot[off + t].comm;
        const int c1 = t + 1 < cnt ? slot[off + t + 1].comm : -2;
        const int c2 = t + 2 < cnt ? slot[off + t + 2].comm : -2;
        const int c3 = t + 3 < cnt ? slot[off + t + 3].comm : -2;
        if (c0 == c) return t;
        if (c1 == c) return t + 1;
        if (c2 == c) return t + 2;
        if (c3 == c) return t + 3;
    }
    return -1;
}

// correction of one neighbour y (in C with in-count i, degree dy) when x joins C (its
// in-count rises by one, the size to s+1) or leaves C (falls by one, size s-1)
__device__ __forceinline__ X192 visit_term(bool leave, long long i, long long dy, long long s, int &bad)
{
    double gn, go;
    if (leave) { gn = g_term(i - 1, dy, s - 1); go = g_term(i, dy, s - 1); }
    else { gn = g_term(i + 1, dy, s + 1); go = g_term(i, dy, s + 1); }
    X192 t = x192_from_double(gn, bad);
    X192 o = x192_from_double(go, bad);
    x192_sub(t, o);
    return t;
}

// the fields of C's record a candidate evaluation needs (S = S- for a leave, S+ for a join)
struct CandRec {
    long long m;
    double W;
    unsigned S[5];
    int s;
};

__device__ __forceinline__ void load_cand(const Ctx &cx, int C, bool leave, CandRec &r)
{
    const CommRec *p = &cx.cr[C];
    r.s = p->s;
    r.m = p->m;
    r.W = p->W;
    const unsigned *S = leave ? p->Sm : p->Sp;
#pragma unroll
    for (int k = 0; k < 5; k++) r.S[k] = S[k];
}

// change of C's cc-free score when x (degree dx, k neighbours in C) joins / leaves C;
// corr = exact sum of the neighbours' corrections
__device__ __forceinline__ double cand_delta(const CandRec &r, bool leave, long long k, long long dx, X192 corr,
                                             int &bad)
{
    long long s = r.s;
    long long m = r.m;
    X192 S = rec_load(r.S);
    x192_add(S, corr);
    double p;
    if (leave) {
        X192 own = x192_from_double(g_term(k, dx, s - 1), bad);
        x192_sub(S, own);
        p = density(s - 1, m - k);
    } else {
        X192 own = x192_from_double(g_term(k, dx, s + 1), bad);
        x192_add(S, own);
        p = density(s + 1, m + k);
    }
    double pS = p * x192_round(S);
    return pS - r.W;
}

__device__ __forceinline__ double candidate_delta(const Ctx &cx, int C, bool leave, long long k, long long dx,
                                                  X192 corr, int &bad)
{
    CandRec r;
    load_cand(cx, C, leave, r);
    return cand_delta(r, leave, k, dx, corr, bad);
}

// strictly positive changes only; larger wins; equal -> lower community id
__device__ __forceinline__ void better(double d, int c, double &bd, int &bc)
{
    if (!(d > 0.0)) return;
    if (bc < 0 || d > bd || (d == bd && c < bc)) { bd = d; bc = c; }
}

__device__ __forceinline__ void wave_best(double &bd, int &bc)
{
    for (int m = 32; m >= 1; m >>= 1) {
        double od = __shfl_xor(bd, m, WAVE);
        int oc = __shfl_xor(bc, m, WAVE);
        if (oc >= 0 && (bc < 0 || od > bd || (od == bd && oc < bc))) { bd = od; bc = oc; }
    }
}

// the g-terms of one member of C with in-count i and degree d at sizes s, s+1, s-1
__device__ __forceinline__ void member_add(long long i, long long d, long long s, X192 &a0, X192 &ap, X192 &am,
                                           long long &sumi, int &bad)
{
    sumi += i;
    X192 v = x192_from_double(g_term(i, d, s), bad);
    x192_add(a0, v);
    v = x192_from_double(g_term(i, d, s + 1), bad);
    x192_add(ap, v);
    v = x192_from_double(g_term(i, d, s - 1), bad);
    x192_add(am, v);
}

// exact g-sums of one member y of C (at sizes s, s+1, s-1) if y is still in C
__device__ __forceinline__ void member_terms(const Ctx &cx, int y, int C, long long s, X192 &a0, X192 &ap,
                                             X192 &am, long long &sumi, int &bad)
{
    NodeHdr hy = cx.nh[y];
    int in = 0;
    int t = find_slot_in(cx.slot, hy.off, hy.cnt, C, &in);
    if (t < 0) return;                       // left C earlier in this iteration
    member_add(in, hy.deg, s, a0, ap, am, sumi, bad);
}

// ---- membership lines (the queue kernels' view of the memberships) --------------------
// first membership slot of a node whose line is l
__device__ __forceinline__ Slot *line_slots(const Ctx &cx, int x, const NodeLine &l)
{
    return l.off < 0 ? cx.ln[x].s : cx.slot + l.off;
}

// position of community c among the memberships of the node with line l (-1 if absent)
// and its in-count: inline memberships come from the line itself
__device__ __forceinline__ int line_find(const Ctx &cx, const NodeLine &l, int c, int *in)
{
    if (l.off < 0) {
        int a = -1, iv = 0;
#pragma unroll
        for (int t = 0; t < LINE_SLOTS; t++)
            if (t < l.cnt && l.s[t].comm == c) {
                a = t;
                iv = l.s[t].in;
            }
        *in = iv;
        return a;
    }
    return find_slot_in(cx.slot, l.off, l.cnt, c, in);
}

// member_terms on the membership lines
__device__ __forceinline__ void member_terms_line(const Ctx &cx, int y, int C, long long s, X192 &a0, X192 &ap,
                                                  X192 &am, long long &sumi, int &bad)
{
    const NodeLine ly = cx.ln[y];
    int in = 0;
    if (line_find(cx, ly, C, &in) < 0) return;   // left C earlier in this iteration
    member_add(in, ly.deg, s, a0, ap, am, sumi, bad);
}

// The lanes executing this call with want = true receive consecutive indices from *ctr,
// with a single atomic per wave (the leader is an active lane, so divergent callers are
// fine); returns -1 for the others.
__device__ __forceinline__ int wave_reserve(int *ctr, bool want)
{
    unsigned long long m = __ballot(want);
    if (!m) return -1;
    int lane = threadIdx.x & (WAVE - 1);
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(ctr, __popcll(m));
    base = __shfl(base, leader, WAVE);
    return want ? base + __popcll(m & ((1ull << lane) - 1)) : -1;
}

__device__ __forceinline__ unsigned hash_tab(int c) { return (unsigned)c * 0x9E3779B1u; }

__device__ __forceinline__ unsigned long long hash64(unsigned long long k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}
