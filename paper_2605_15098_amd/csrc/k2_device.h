// Device code shared by the compiled kernels (kernels.hip) and the pass
// kernels generated at run time (jit.cpp): complex arithmetic, the block-pass
// op handlers, the persistent block-pass skeleton and the op interpreter.
// Every gate's arithmetic lives here once, so the plain sweep, the
// interpreted block pass and a generated block pass compute the same bits.
#pragma once

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#endif

#include "k2_abi.h"

namespace svk {

template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };

__device__ __forceinline__ float xfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double xfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename C> __host__ __device__ __forceinline__ C mk(double re, double im)
{
    C r;
    r.x = (decltype(r.x))re;
    r.y = (decltype(r.y))im;
    return r;
}

// z * a
template <typename C> __device__ __forceinline__ C cmul(C z, C a)
{
    C r;
    r.x = xfma(z.x, a.x, -(z.y * a.y));
    r.y = xfma(z.x, a.y, z.y * a.x);
    return r;
}

// u0 * a + u1 * b
template <typename C> __device__ __forceinline__ C cmad2(C u0, C a, C u1, C b)
{
    C r;
    r.x = xfma(u0.x, a.x, xfma(-u0.y, a.y, xfma(u1.x, b.x, -(u1.y * b.y))));
    r.y = xfma(u0.x, a.y, xfma(u0.y, a.x, xfma(u1.x, b.y, u1.y * b.x)));
    return r;
}

// Component-wise select (a whole-struct ?: on double2 is lowered through
// scratch memory).
template <typename C> __device__ __forceinline__ C csel(bool p, C x, C y)
{
    C r;
    r.x = p ? x.x : y.x;
    r.y = p ? x.y : y.y;
    return r;
}

// Hadamard butterfly: ((a+b)/sqrt2, (a-b)/sqrt2)
template <typename C> __device__ __forceinline__ void hbfly(C &a, C &b)
{
    using T = decltype(a.x);
    const T s = (T)0.70710678118654752440;
    C x, y;
    x.x = (a.x + b.x) * s;
    x.y = (a.y + b.y) * s;
    y.x = (a.x - b.x) * s;
    y.y = (a.y - b.y) * s;
    a = x;
    b = y;
}

__device__ __forceinline__ uint64_t insert0(uint64_t x, int b)
{
    const uint64_t lo = x & ((1ull << b) - 1ull);
    return ((x >> b) << (b + 1)) | lo;
}

__device__ __forceinline__ uint32_t insert0_32(uint32_t x, int b)
{
    return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1u));
}

// Storage order of the state in HBM: amplitude i (physical index, after the
// qubit layout) is kept at sto(i), which XORs index bits S0 .. S0+8 (byte
// address bits 8..16: S0 = 5 for complex64, 4 for complex128) with a fold of
// the bits above them. A block whose local bits are the low S0 bits plus
// high bits (the block pass's scattered runs) then spreads its runs over
// the HBM channels instead of drawing them all from the few that its fixed
// middle address bits select; runs of 2^S0 amplitudes and aligned ranges of
// 2^(S0+9) amplitudes stay contiguous. The map is linear over GF(2)
// (sto(x ^ y) = sto(x) ^ sto(y)) and is its own inverse; states below
// 2^(S0+10) amplitudes are stored in plain order.
template <typename C> __host__ __device__ __forceinline__ uint64_t sto(uint64_t i)
{
    constexpr int S0 = sizeof(C) == 8 ? 5 : 4;
    const uint64_t h = i >> (S0 + 9);
    return i ^ (((h ^ (h >> 9) ^ (h >> 18) ^ (h >> 27) ^ (h >> 36)) & 511ull) << S0);
}

// LDS index swizzle: the low bits that span one 128-byte bank row are XORed
// with a fold of the higher bits, so lanes whose local indices differ only in
// high bits still spread over the banks. The map is linear over GF(2) (shifts,
// XORs and a constant mask), so for disjoint bit sets
// swz(a | b) = swz(a) ^ swz(b): a thread swizzles its own bits once and each
// register slot adds a block-uniform term.
template <typename C> __host__ __device__ __forceinline__ uint32_t swz(uint32_t x)
{
    constexpr int E = (sizeof(C) == 8) ? 4 : 3;  // log2(elements per 128 B)
    constexpr uint32_t M = (1u << E) - 1u;
    const uint32_t h = x >> E;
    return x ^ ((h ^ (h >> E) ^ (h >> (2 * E))) & M);
}

// A non-register condition bit: 0..l-1 = local bit (tested on the thread's
// local index), 64 + p = memory bit p outside the block (the block base).
__device__ __forceinline__ bool code_bit(uint32_t tloc, uint64_t base, int code)
{
    return code >= 64 ? (bool)((base >> (code - 64)) & 1ull) : (bool)((tloc >> code) & 1u);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Work-group barrier that waits only for this wave's LDS (and scalar)
// accesses. Outstanding global loads stay in flight, so the next block,
// prefetched into registers, keeps streaming across re-layouts.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ------------------------------------------------------------ op handlers

// Dense, Hadamard or exchange gate on register slot J, optionally controlled
// by another slot (ckind CK_SLOT) or a per-thread predicate (tpred).
template <int J, int R, typename C>
__device__ __forceinline__ void k2_pairs(C *a, int kind, const double *v, bool tpred, int ckind, int cslot)
{
    const C u00 = mk<C>(v[0], v[1]), u01 = mk<C>(v[2], v[3]);
    const C u10 = mk<C>(v[4], v[5]), u11 = mk<C>(v[6], v[7]);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (k & (1 << J)) continue;
        if (ckind == svp::CK_SLOT && !((k >> cslot) & 1)) continue;
        constexpr int H = 1 << J;
        C x = a[k], y = a[k + H], nx, ny;
        if (kind == svp::K2_H) {
            nx = x;
            ny = y;
            hbfly(nx, ny);
        } else if (kind == svp::K2_X) {
            nx = y;
            ny = x;
        } else {
            nx = cmad2(u00, x, u01, y);
            ny = cmad2(u10, x, u11, y);
        }
        a[k] = csel(tpred, nx, x);
        a[k + H] = csel(tpred, ny, y);
    }
}

// Unnormalized Hadamard on register slot J: (a, b) -> (a + b, a - b).
template <int J, int R, typename C> __device__ __forceinline__ void k2_hu(C *a)
{
    constexpr int H = 1 << J;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (k & H) continue;
        const C x = a[k], y = a[k + H];
        a[k].x = x.x + y.x;
        a[k].y = x.y + y.y;
        a[k + H].x = x.x - y.x;
        a[k + H].y = x.y - y.y;
    }
}

// Per-block state a program sees.
struct K2Ctx {
    uint32_t tid;
    uint64_t base;
    uint32_t tloc;               // local index of the thread's slot-0 amplitude
    unsigned char *lds;          // block buffer for re-layouts
    const double2 *ufac;         // block-uniform factors
    const unsigned char *table;  // plan table
    const unsigned char *tabs;   // the pass's lane/wave factors in LDS (type C)
};

// Local index x with bit b taken out (the bits above it move down one).
__device__ __forceinline__ uint32_t drop_bit(uint32_t x, int b)
{
    return (x & ((1u << b) - 1u)) | ((x >> (b + 1)) << b);
}

// Re-layout through LDS: the amplitudes leave registers in layout rb_old and
// come back in layout rb_new (local bit of each register slot, any order).
// With split < 0 the whole block passes through LDS at once. Otherwise the
// block moves in two halves, local bit x = 0 then x = 1, each stored at its
// local index with bit x taken out, so LDS holds 2^(l-1) amplitudes:
//  - split = x < 32: slot s holds x in both layouts; round h writes and
//    reads the registers whose slot-s bit is h (the first round's reads do
//    not overwrite the registers the second round writes);
//  - split = 32 + x: x is the thread-id bit p in both layouts; round h is
//    done by the threads whose bit p is h (whole waves when p >= 6), all of
//    their registers.
template <int LOGR, typename C>
__device__ __forceinline__ void k2_layout(C *a, K2Ctx &cx, const int *rb_old, const int *rb_new, int split)
{
    constexpr int R = 1 << LOGR;
    // The thread's indices are laundered here so that each re-layout derives
    // its LDS addresses when it runs, instead of the program computing every
    // re-layout's addresses at the start of the block and holding them.
    asm volatile("" : "+v"(cx.tid), "+v"(cx.tloc));
    // the new thread local index: the thread-id bits spread over the
    // non-register bits, zeros inserted at the register bits in ascending order
    uint32_t rmask = 0;
#pragma unroll
    for (int j = 0; j < LOGR; ++j) rmask |= 1u << rb_new[j];
    uint32_t tnew = cx.tid;
#pragma unroll
    for (int j = 0; j < LOGR; ++j) {
        tnew = insert0_32(tnew, __builtin_ctz(rmask));
        rmask &= rmask - 1u;
    }
    if (split < 0) {
        const uint32_t tsw = swz<C>(cx.tloc) * (uint32_t)sizeof(C);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint32_t kp = 0;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if ((k >> j) & 1) kp |= 1u << rb_old[j];
            *reinterpret_cast<C *>(cx.lds + (tsw ^ (swz<C>(kp) * (uint32_t)sizeof(C)))) = a[k];
        }
        lds_barrier();
        cx.tloc = tnew;
        const uint32_t tsn = swz<C>(cx.tloc) * (uint32_t)sizeof(C);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint32_t kp = 0;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if ((k >> j) & 1) kp |= 1u << rb_new[j];
            a[k] = *reinterpret_cast<const C *>(cx.lds + (tsn ^ (swz<C>(kp) * (uint32_t)sizeof(C))));
        }
        lds_barrier();
        return;
    }
    if (split >= 32) {
        const int x = split - 32;
        uint32_t om = 0;
#pragma unroll
        for (int j = 0; j < LOGR; ++j) om |= 1u << rb_old[j];
        const int p = x - __builtin_popcount(om & ((1u << x) - 1u));
        const uint32_t mine = (cx.tid >> p) & 1u;
        const uint32_t tso = swz<C>(drop_bit(cx.tloc, x)) * (uint32_t)sizeof(C);
        const uint32_t tsn = swz<C>(drop_bit(tnew, x)) * (uint32_t)sizeof(C);
#pragma unroll
        for (uint32_t h = 0; h < 2; ++h) {
            if (mine == h) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    uint32_t kp = 0;
#pragma unroll
                    for (int j = 0; j < LOGR; ++j)
                        if ((k >> j) & 1) kp |= 1u << rb_old[j];
                    *reinterpret_cast<C *>(cx.lds + (tso ^ (swz<C>(drop_bit(kp, x)) * (uint32_t)sizeof(C)))) = a[k];
                }
            }
            lds_barrier();
            if (mine == h) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    uint32_t kp = 0;
#pragma unroll
                    for (int j = 0; j < LOGR; ++j)
                        if ((k >> j) & 1) kp |= 1u << rb_new[j];
                    a[k] = *reinterpret_cast<const C *>(cx.lds + (tsn ^ (swz<C>(drop_bit(kp, x)) * (uint32_t)sizeof(C))));
                }
            }
            lds_barrier();
        }
        cx.tloc = tnew;
        return;
    }
    int s = 0;
#pragma unroll
    for (int j = 0; j < LOGR; ++j)
        if (rb_old[j] == split) s = j;
    const uint32_t tso = swz<C>(drop_bit(cx.tloc, split)) * (uint32_t)sizeof(C);
    const uint32_t tsn = swz<C>(drop_bit(tnew, split)) * (uint32_t)sizeof(C);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (((k >> s) & 1) != h) continue;
            uint32_t kp = 0;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if (j != s && ((k >> j) & 1)) kp |= 1u << rb_old[j];
            *reinterpret_cast<C *>(cx.lds + (tso ^ (swz<C>(drop_bit(kp, split)) * (uint32_t)sizeof(C)))) = a[k];
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (((k >> s) & 1) != h) continue;
            uint32_t kp = 0;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if (j != s && ((k >> j) & 1)) kp |= 1u << rb_new[j];
            a[k] = *reinterpret_cast<const C *>(cx.lds + (tsn ^ (swz<C>(drop_bit(kp, split)) * (uint32_t)sizeof(C))));
        }
        lds_barrier();
    }
    cx.tloc = tnew;
}

// ---- dense window through the matrix cores (16x16x4 MFMA)

typedef float k2_f4 __attribute__((ext_vector_type(4)));
typedef double k2_d4 __attribute__((ext_vector_type(4)));

template <typename T> struct K2Mfma;
template <> struct K2Mfma<float> {
    using V = k2_f4;
    static __device__ __forceinline__ V mma(float x, float y, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
    }
};
template <> struct K2Mfma<double> {
    using V = k2_d4;
    static __device__ __forceinline__ V mma(double x, double y, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
    }
};

// A KW-qubit unitary on local bits w[0] < ... < w[KW-1], applied to every
// one of the block's 2^(l-KW) vectors through the LDS copy of the block.
// The window's complex 2^KW matrix acts as the real matrix M' of size
// D = 2^(KW+1) on interleaved vectors (real index 2 j + c: amplitude j of
// the window, component c). Wave-level 16x16x4 MFMA: 16 vectors per group
// (lane % 16), operand B[k][n] from lane 16 k + n, output D[4 q + r][n] in
// register r of lane 16 q + n for FP32, D[4 r + q][n] for FP64 (the FP64
// instruction interleaves its output rows). mat holds M' in A-operand order:
// mat[(t * D/4 + s) * 64 + lane] = M'[16 t + lane % 16][4 s + lane / 16].
// The register layout rb is the same before and after. Needs full waves
// (2^(l - LOGR) >= 64 threads).
template <int LOGR, int KW, typename C>
__device__ __forceinline__ void k2_mfma(C *a, K2Ctx &cx, const int *rb, const int *w, int l, const void *mat)
{
    using T = decltype(C::x);
    using V = typename K2Mfma<T>::V;
    constexpr int R = 1 << LOGR;
    constexpr int D = 2 << KW;
    constexpr int TILES = D / 16, STEPS = D / 4;
    {
        const uint32_t tsw = swz<C>(cx.tloc) * (uint32_t)sizeof(C);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint32_t kp = 0;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if ((k >> j) & 1) kp |= 1u << rb[j];
            *reinterpret_cast<C *>(cx.lds + (tsw ^ (swz<C>(kp) * (uint32_t)sizeof(C)))) = a[k];
        }
    }
    lds_barrier();
    // whole waves only: the planner emits this op for blocks of 64 or more
    // threads (every lane supplies an operand)
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    const int nwaves = blockDim.x >= 64u ? (int)(blockDim.x >> 6) : 1;
    const int col = lane & 15, q = lane >> 4;
    uint32_t wsw[KW], wmask = 0;
#pragma unroll
    for (int i = 0; i < KW; ++i) {
        wsw[i] = swz<C>(1u << w[i]);
        wmask |= 1u << w[i];
    }
    const uint32_t nvec = 1u << (l - KW);
    const int groups = (int)((nvec + 15u) >> 4);
    // The table address is laundered so that its loads stay inside this op:
    // they do not depend on the block, and hoisting every window's operands
    // out of the block loop would need hundreds of registers. It is read as
    // a uniform value first (it is one), so that the scalar-register operand
    // holds wherever the compiler cannot prove it uniform by itself.
    const T *M = reinterpret_cast<const T *>(uniform64(reinterpret_cast<uint64_t>(mat)));
    asm volatile("" : "+s"(M));
    // The lane's A operand for every (tile, step) of a 4-qubit window is
    // loaded once per op (16 or 32 registers) while the block's own registers
    // are parked in LDS; a 5-qubit window would take 64 or 128 registers, so
    // its steps read the table, which stays in the caches.
    constexpr bool AREG = KW == 4;
    T areg[AREG ? TILES * STEPS : 1];
    if constexpr (AREG) {
#pragma unroll
        for (int i = 0; i < TILES * STEPS; ++i) areg[i] = M[i * 64 + lane];
    }
    // input element of lane: amplitude j = 2 s + (q >> 1), component q & 1
    const uint32_t in_lane = (q >> 1) ? wsw[0] : 0u;
    for (int g = wave; g < groups; g += nwaves) {
        const uint32_t n = (uint32_t)g * 16u + (uint32_t)col;
        const bool valid = n < nvec;
        uint32_t vb = 0, m = n;
        for (int b = 0; b < l; ++b)
            if (!((wmask >> b) & 1u)) {
                vb |= (m & 1u) << b;
                m >>= 1;
            }
        const uint32_t vsw = swz<C>(vb);
        V acc[TILES];
#pragma unroll
        for (int t = 0; t < TILES; ++t) acc[t] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            uint32_t jsw = in_lane;
#pragma unroll
            for (int i = 1; i < KW; ++i)
                if (((2 * s) >> i) & 1) jsw ^= wsw[i];
            const T *src = reinterpret_cast<const T *>(cx.lds + (vsw ^ jsw) * (uint32_t)sizeof(C));
            const T bv = valid ? src[q & 1] : T(0);
#pragma unroll
            for (int t = 0; t < TILES; ++t) {
                T av;
                if constexpr (AREG) av = areg[t * STEPS + s];
                else av = M[(t * STEPS + s) * 64 + lane];
                acc[t] = K2Mfma<T>::mma(av, bv, acc[t]);
            }
        }
        if (valid) {
#pragma unroll
            for (int t = 0; t < TILES; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // output row of (lane, register): amplitude row >> 1, component row & 1
                    const int row = 16 * t + (sizeof(T) == 4 ? 4 * q + r : 4 * r + q);
                    const int jo = row >> 1;
                    uint32_t osw = 0;
#pragma unroll
                    for (int i = 0; i < KW; ++i)
                        if ((jo >> i) & 1) osw ^= wsw[i];
                    T *dst = reinterpret_cast<T *>(cx.lds + (vsw ^ osw) * (uint32_t)sizeof(C));
                    dst[row & 1] = acc[t][r];
                }
        }
    }
    lds_barrier();
    {
        const uint32_t tsw = swz<C>(cx.tloc) * (uint32_t)sizeof(C);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint32_t kp = 0;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if ((k >> j) & 1) kp |= 1u << rb[j];
            a[k] = *reinterpret_cast<const C *>(cx.lds + (tsw ^ (swz<C>(kp) * (uint32_t)sizeof(C))));
        }
    }
    lds_barrier();
}

// Thread factor of a diagonal-run group: block-uniform factor (FP64, cast
// once) times the wave and lane entries of the pass's factor table in LDS,
// in the state's precision.
template <typename C>
__device__ __forceinline__ C k2_group_factor(const svp::DiagGroup &G, const K2Ctx &cx)
{
    // keeps the scheduler from starting many runs' factors at once, which
    // would raise register use past the two-work-groups-per-CU budget
    __builtin_amdgcn_sched_barrier(0);
    C f = mk<C>(1.0, 0.0);
    bool on = true;
    if (G.cond_kind == 1) on = (cx.base >> G.cond_bit) & 1ull;
    else if (G.cond_kind == 2) on = (cx.tid >> G.cond_bit) & 1u;
    if (on) {
        const C *tab = reinterpret_cast<const C *>(cx.tabs);
        if (G.uidx >= 0) f = mk<C>(cx.ufac[G.uidx].x, cx.ufac[G.uidx].y);
        if (G.wave_off >= 0) f = cmul(f, tab[G.wave_off + (cx.tid >> 6)]);
        if (G.lane_off >= 0) f = cmul(f, tab[G.lane_off + (cx.tid & 63u)]);
    }
    return f;
}

// One factor of a run's fold (DiagRun): T = g for the first, T = T * g after.
template <typename C> __device__ __forceinline__ C k2_fold(bool first, C T, C g)
{
    return first ? g : cmul(T, g);
}

// Slot k's multiply of a diagonal run: F = Q[k] * T (or Q[k] when no group
// covers k, or T without a constant), a[k] = F * a[k].
template <typename C> __device__ __forceinline__ void k2_diag_apply(C &ak, bool with_q, double2 q, bool have_t, C T)
{
    const C qc = mk<C>(q.x, q.y);
    const C F = with_q ? (have_t ? cmul(qc, T) : qc) : T;
    ak = cmul(F, ak);
}

// A diagonal run evaluated slot by slot (the interpreter): each slot folds
// its groups in the record's canonical order (see DiagRun), recomputing the
// group factors it needs.
template <int LOGR, typename C>
__device__ __forceinline__ void k2_diagrun(C *a, const K2Ctx &cx, const svp::DiagRun *rec)
{
    constexpr int R = 1 << LOGR;
    const svp::DiagGroup *gs = reinterpret_cast<const svp::DiagGroup *>(rec + 1);
    const int ng = rec->ngroups;
    const double2 *qt = reinterpret_cast<const double2 *>(gs + ng);
    const uint32_t kmask = rec->kmask, qmask = rec->qmask;
    // The groups are stored by ascending top register bit (rmask = 0 first),
    // so one walk over them in record order hands every slot its factors in
    // the order the record defines: a group whose top bit is not in k has
    // rmask outside k and is skipped for that slot.
    if constexpr (sizeof(C) * R <= 128) {
        // Each group's factor once per block. Slot k with top bit b starts
        // from the finished product of slot k - 2^b (the groups of lower
        // levels that lie within k are exactly those within k - 2^b) and
        // folds only the groups of level b that lie within k.
        C T[R];
        bool have[R];
        T[0] = mk<C>(1.0, 0.0);
        have[0] = false;
        int i = 0;
        for (; i < ng && gs[i].rmask == 0; ++i) {
            T[0] = k2_fold(!have[0], T[0], k2_group_factor<C>(gs[i], cx));
            have[0] = true;
        }
#pragma unroll
        for (int b = 0; b < LOGR; ++b) {
#pragma unroll
            for (int k = 1 << b; k < (2 << b); ++k) {
                T[k] = T[k - (1 << b)];
                have[k] = have[k - (1 << b)];
            }
            for (; i < ng && (31 - __builtin_clz((uint32_t)gs[i].rmask)) == b; ++i) {
                const int rm = gs[i].rmask;
                const C f = k2_group_factor<C>(gs[i], cx);
#pragma unroll
                for (int k = 1 << b; k < (2 << b); ++k) {
                    if (rm & ~k) continue;
                    T[k] = k2_fold(!have[k], T[k], f);
                    have[k] = true;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k)
            if ((kmask >> k) & 1u) k2_diag_apply(a[k], ((qmask >> k) & 1u) != 0, qt[k], have[k], T[k]);
    } else {
        // larger tiles: slot by slot (the accumulators would not fit)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (!((kmask >> k) & 1u)) continue;
            C T = mk<C>(1.0, 0.0);
            bool have = false;
            for (int i = 0; i < ng; ++i) {
                if (gs[i].rmask & ~k) continue;
                T = k2_fold(!have, T, k2_group_factor<C>(gs[i], cx));
                have = true;
            }
            k2_diag_apply(a[k], ((qmask >> k) & 1u) != 0, qt[k], have, T);
        }
    }
}

template <int R, typename C>
__device__ __forceinline__ void k2_phase(C *a, const K2Ctx &cx, int rmask, uint32_t lmask, uint64_t gmask, C z)
{
    const bool tpred = ((cx.tloc & lmask) == lmask) && ((cx.base & gmask) == gmask);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if ((k & rmask) != rmask) continue;
        a[k] = csel(tpred, cmul(z, a[k]), a[k]);
    }
}

template <int R, typename C>
__device__ __forceinline__ void k2_diag(C *a, const K2Ctx &cx, int slot, int code, int rmask, uint32_t lmask,
                                        uint64_t gmask, C d0, C d1)
{
    const bool tpred = ((cx.tloc & lmask) == lmask) && ((cx.base & gmask) == gmask);
    if (slot >= 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if ((k & rmask) != rmask) continue;
            const C d = csel(((k >> slot) & 1) != 0, d1, d0);
            a[k] = csel(tpred, cmul(d, a[k]), a[k]);
        }
    } else {
        const C d = csel(code_bit(cx.tloc, cx.base, code), d1, d0);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if ((k & rmask) != rmask) continue;
            a[k] = csel(tpred, cmul(d, a[k]), a[k]);
        }
    }
}

template <int R, typename C> __device__ __forceinline__ void k2_scale(C *a, double s)
{
    using T = decltype(a[0].x);
    const T sc = (T)s;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        a[k].x *= sc;
        a[k].y *= sc;
    }
}

// ------------------------------------------------------------ skeleton

template <typename T, int LOGR> constexpr int k2_max_threads()
{
    return (LOGR + (sizeof(T) == 8 ? 1 : 0)) >= 5 ? (LOGR + (sizeof(T) == 8 ? 1 : 0) >= 6 ? 256 : 512) : 1024;
}

// Memory bits outside the block, from the block number (work-group uniform).
// Deposit the low bits of v at the set bits of mask, in ascending order. With
// v and mask uniform this stays on the scalar unit.
__device__ __forceinline__ uint64_t k2_deposit(uint64_t v, uint64_t mask)
{
    uint64_t out = 0;
    for (uint64_t m = mask; m != 0; m &= m - 1) {
        if (v & 1ull) out |= m & (~m + 1ull);
        v >>= 1;
    }
    return out;
}

// Register slot k of the thread is amplitude tbase ^ (XOR of roff[j] over
// the set bits j of k): tbase and roff are already in storage order (sto is
// linear), so the storage order costs nothing per access.
template <int LOGR, typename C>
__device__ __forceinline__ void k2_load(C *a, const C *__restrict__ S, uint64_t tbase, const uint64_t *roff, bool vec2)
{
    constexpr int R = 1 << LOGR;
    if (sizeof(C) == 8 && vec2) {
        // memory bit 0 is local bit 0 = slot 0: slots k, k+1 are adjacent
#pragma unroll
        for (int k = 0; k < R; k += 2) {
            uint64_t addr = tbase;
#pragma unroll
            for (int j = 1; j < LOGR; ++j)
                if ((k >> j) & 1) addr ^= roff[j];
            const float4 v = *reinterpret_cast<const float4 *>(S + addr);
            a[k] = mk<C>(v.x, v.y);
            a[k + 1] = mk<C>(v.z, v.w);
        }
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint64_t addr = tbase;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if ((k >> j) & 1) addr ^= roff[j];
            a[k] = S[addr];
        }
    }
}

template <int LOGR, typename C>
__device__ __forceinline__ void k2_store(const C *a, C *__restrict__ S, uint64_t tbase, const uint64_t *roff, bool vec2)
{
    constexpr int R = 1 << LOGR;
    if (sizeof(C) == 8 && vec2) {
#pragma unroll
        for (int k = 0; k < R; k += 2) {
            uint64_t addr = tbase;
#pragma unroll
            for (int j = 1; j < LOGR; ++j)
                if ((k >> j) & 1) addr ^= roff[j];
            float4 v;
            v.x = (float)a[k].x;
            v.y = (float)a[k].y;
            v.z = (float)a[k + 1].x;
            v.w = (float)a[k + 1].y;
            *reinterpret_cast<float4 *>(S + addr) = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint64_t addr = tbase;
#pragma unroll
            for (int j = 0; j < LOGR; ++j)
                if ((k >> j) & 1) addr ^= roff[j];
            S[addr] = a[k];
        }
    }
}

// Block-resident pass, persistent: a work-group handles blocks first,
// first + stride, ... and loads the next one into registers while it runs the
// program on block i. A block is 2^l amplitudes: local bit i is memory bit
// args.bits[i]; the other memory bits come from the block number. Each thread
// holds R = 2^LOGR amplitudes in registers; register slot j stands for local
// bit rb[j]; the remaining local bits, in ascending order, are the bits of
// threadIdx. A program starts and ends in the canonical layout
// (k2_canon_bit: slot 0 = local bit 0, slots 1.. = local bits l-r .. l-2),
// so lanes walk consecutive memory and, for complex64, slots 0 and 1 form
// one 16-byte access. lds is laid out by k2_lds_layout.
//
// V2 must equal args.vec2: a compile-time access width keeps one load path in
// the loop, so the wait for the current block counts only its own loads and
// the next block's prefetch stays in flight.
//
// PF = 2 issues the next block's loads on every iteration (the last re-reads
// the current block) so their count is the same on every path; PF = 1 (a
// work-group with few blocks, the batched passes) skips it after the last
// block; PF = 0 does not prefetch: the next block is loaded after the store,
// for passes that keep two work-groups on a CU (half the registers each) and
// let one compute while the other waits.
template <typename T, int LOGR, bool V2, int PF, class Prog>
__device__ __forceinline__ void k2_body(typename CT<T>::type *__restrict__ S, const svp::K2Args &args,
                                        unsigned char *lds, const Prog &prog, uint64_t first, uint64_t stride)
{
    using C = typename CT<T>::type;
    constexpr int R = 1 << LOGR;
    const int l = args.l;
    const int tb = l - LOGR;
    const uint32_t tid = threadIdx.x;
    // The wave number is wave-uniform (a scalar register) and the lane comes
    // back from two lane-count instructions, so the thread index is rebuilt
    // per block instead of being held in a vector register (or spilled) for
    // the whole launch.
    const uint32_t wave_no = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t nblocks = 1ull << args.nblk_bits;
    constexpr bool vec2 = V2;
    // (offsets read as wave-uniform values: they stay in scalar registers)
    const svp::K2Lds L = svp::k2_lds_layout(l, (int)sizeof(C), args.nug, args.tab_count, args.nut, args.half_lds);
    double2 *ufac = reinterpret_cast<double2 *>(lds + __builtin_amdgcn_readfirstlane(L.ufac));
    C *tabs = reinterpret_cast<C *>(lds + __builtin_amdgcn_readfirstlane(L.tabs));
    svp::UTerm *uterm = reinterpret_cast<svp::UTerm *>(lds + __builtin_amdgcn_readfirstlane(L.uterm));
    svp::UGroup *ugrp = reinterpret_cast<svp::UGroup *>(lds + __builtin_amdgcn_readfirstlane(L.ugrp));
    // memory bits outside the block, as a mask (the block number is deposited there)
    uint64_t gmask = 0;
    for (int i = 0; i < args.nblk_bits; ++i) gmask |= 1ull << args.nbits[i];
    gmask = uniform64(gmask);
    const uint64_t base_or = uniform64(args.base_or);

    // canonical-layout addressing, the same for every block: the thread-id
    // bits go, in ascending order, to the local bits that are not register bits
    uint32_t canon_regs = 0;
#pragma unroll
    for (int j = 0; j < LOGR; ++j) canon_regs |= 1u << svp::k2_canon_bit(j, l, LOGR);
    uint64_t tmem_local = 0;
    for (int i = 0, c = 0; i < l; ++i) {
        if ((canon_regs >> i) & 1u) continue;
        tmem_local |= (uint64_t)((tid >> c) & 1u) << args.bits[i];
        ++c;
    }
    tmem_local = sto<C>(tmem_local);
    // (read as wave-uniform values: they stay in scalar registers)
    uint64_t roff[LOGR];
#pragma unroll
    for (int j = 0; j < LOGR; ++j) roff[j] = uniform64(sto<C>(1ull << args.bits[svp::k2_canon_bit(j, l, LOGR)]));

    uint64_t bid = first;
    if (bid >= nblocks) return;
    // the pass's lane/wave factors, once per launch: LDS reads keep the
    // program clear of vector-memory waits, which would also wait for the
    // next block's prefetch
    // (the block-uniform terms likewise)
    if (args.tab_count > 0 || args.nug > 0) {
        const double2 *src = reinterpret_cast<const double2 *>(args.table + args.tab_off);
        for (int i = (int)tid; i < args.tab_count; i += (int)blockDim.x) tabs[i] = mk<C>(src[i].x, src[i].y);
        const svp::UTerm *ts = reinterpret_cast<const svp::UTerm *>(args.table + args.ut_off);
        for (int i = (int)tid; i < args.nut; i += (int)blockDim.x) uterm[i] = ts[i];
        const svp::UGroup *gs = reinterpret_cast<const svp::UGroup *>(args.table + args.ug_off);
        for (int i = (int)tid; i < args.nug; i += (int)blockDim.x) ugrp[i] = gs[i];
        __syncthreads();
    }
    uint64_t base = uniform64(k2_deposit(bid, gmask) | base_or);
    C a[R], b[PF ? R : 1];
    k2_load<LOGR>(a, S, sto<C>(base) ^ tmem_local, roff, vec2);

    for (;;) {
        const uint64_t next = bid + stride;
        const bool has_next = next < nblocks;
        // With a path-independent count of loads in flight, the wait for
        // this block's data does not also wait for the prefetch.
        const uint64_t nbase = has_next ? uniform64(k2_deposit(next, gmask) | base_or) : base;
        if constexpr (PF > 0)
            if (PF == 2 || has_next) k2_load<LOGR>(b, S, sto<C>(nbase) ^ tmem_local, roff, vec2);

        // Block-uniform phase factors of the diagonal runs: each is
        // e^{2 pi i sum angle_j [base covers tmask_j]}, summed exactly in
        // 64-bit fixed-point turns and evaluated once per block.
        if (args.nug > 0) {
            const int gtid = (int)((wave_no << 6) | __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)));
            for (int g = gtid; g < args.nug; g += blockDim.x) {
                const svp::UTerm *tm = uterm + ugrp[g].term_off;
                if constexpr (sizeof(T) == 4) {
                    // complex64: the factor is rounded to FP32 anyway; the
                    // exact sum of the turns, its top 32 bits to 2^-31
                    // half-turns, one FP32 sincospi
                    uint64_t acc = 0;
                    for (int j = 0; j < ugrp[g].nterms; ++j)
                        if ((base & tm[j].tmask) == tm[j].tmask) acc += tm[j].angle;
                    float sn, cs;
                    sincospif(ldexpf((float)(int32_t)(acc >> 32), -31), &sn, &cs);
                    ufac[g] = make_double2(cs, sn);
                } else {
                    // complex128: product of the covered terms' FP64
                    // factors (no transcendental in the block loop)
                    double2 f = make_double2(1.0, 0.0);
                    for (int j = 0; j < ugrp[g].nterms; ++j)
                        if ((base & tm[j].tmask) == tm[j].tmask) f = cmul(f, make_double2(tm[j].re, tm[j].im));
                    ufac[g] = f;
                }
            }
            lds_barrier();
        }

        // The thread index is laundered per block so that the programs' LDS
        // addresses and per-thread table factors are recomputed for each
        // block instead of being hoisted out of the block loop, where they
        // would pin dozens of registers and halve the resident work-groups.
        uint32_t tid_b = (wave_no << 6) | __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        asm volatile("" : "+v"(tid_b));
        // canonical local index of the thread: tid bits 0 .. tb-2 on local
        // bits 1 .. tb-1, the top tid bit on local bit l-1
        const uint32_t tloc0 = tb == 0 ? 0u
                                       : ((tid_b & ((1u << (tb - 1)) - 1u)) << 1) |
                                             (((tid_b >> (tb - 1)) & 1u) << (l - 1));
        K2Ctx cx{tid_b, base, tloc0, lds, ufac, args.table, reinterpret_cast<const unsigned char *>(tabs)};
        prog.template run<T, LOGR>(a, cx);

        // the program ends in the canonical layout. The thread's address bits
        // are laundered so that the store recomputes its addresses instead of
        // keeping the load's live across the program (dozens of registers).
        uint64_t tm_st = tmem_local;
        asm volatile("" : "+v"(tm_st));
        k2_store<LOGR>(a, S, sto<C>(base) ^ tm_st, roff, vec2);
        if (!has_next) break;
        if (args.nug > 0) lds_barrier();  // the next block's factors overwrite ufac
        if constexpr (PF > 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) a[k] = b[k];
        } else {
            uint64_t tm_ld = tmem_local;
            asm volatile("" : "+v"(tm_ld));
            k2_load<LOGR>(a, S, sto<C>(nbase) ^ tm_ld, roff, vec2);
        }
        base = nbase;
        bid = next;
    }
}

// k2_body with the access width chosen once, outside the block loop.
template <typename T, int LOGR, class Prog, int PF = 1>
__device__ __forceinline__ void k2_body_any(typename CT<T>::type *__restrict__ S, const svp::K2Args &args,
                                            unsigned char *lds, const Prog &prog, uint64_t first, uint64_t stride)
{
    if (args.vec2) k2_body<T, LOGR, true, PF>(S, args, lds, prog, first, stride);
    else k2_body<T, LOGR, false, PF>(S, args, lds, prog, first, stride);
}

// ------------------------------------------------------------ interpreter

// Runs the op list of a pass (ops[0..nops)) on one block. MFMA selects the
// build that also runs matrix-core windows: their registers would otherwise
// weigh on every program the interpreter runs.
template <bool MFMA>
struct K2Interp {
    const svp::K2Op *__restrict__ ops;
    int nops;
    int l;

    template <typename T, int LOGR>
    __device__ __forceinline__ void run(typename CT<T>::type *a, K2Ctx &cx) const
    {
        using C = typename CT<T>::type;
        constexpr int R = 1 << LOGR;
        int rb[LOGR];
        rb[0] = 0;
#pragma unroll
        for (int j = 1; j < LOGR; ++j) rb[j] = svp::k2_canon_bit(j, l, LOGR);
        for (int oi = 0; oi < nops; ++oi) {
            const svp::K2Op &op = ops[oi];
            const int kind = op.kind;
            if (kind == svp::K2_HU) {
                switch (op.a) {
                case 0: k2_hu<0, R>(a); break;
                case 1: if constexpr (LOGR > 1) k2_hu<1, R>(a); break;
                case 2: if constexpr (LOGR > 2) k2_hu<2, R>(a); break;
                case 3: if constexpr (LOGR > 3) k2_hu<3, R>(a); break;
                case 4: if constexpr (LOGR > 4) k2_hu<4, R>(a); break;
                default: break;
                }
            } else if (kind == svp::K2_DIAGRUN) {
                k2_diagrun<LOGR>(a, cx, reinterpret_cast<const svp::DiagRun *>(cx.table + op.a));
            } else if (kind == svp::K2_LAYOUT) {
                int nrb[LOGR];
#pragma unroll
                for (int j = 0; j < LOGR; ++j) nrb[j] = (op.a >> (5 * j)) & 31;
                k2_layout<LOGR>(a, cx, rb, nrb, op.b);
#pragma unroll
                for (int j = 0; j < LOGR; ++j) rb[j] = nrb[j];
            } else if (kind == svp::K2_MFMA) {
                if constexpr (MFMA) {
                    int wb[5];
#pragma unroll
                    for (int i = 0; i < 5; ++i) wb[i] = (op.c >> (5 * i)) & 31;
                    if (op.b == 4) k2_mfma<LOGR, 4>(a, cx, rb, wb, l, cx.table + op.a);
                    else k2_mfma<LOGR, 5>(a, cx, rb, wb, l, cx.table + op.a);
                }
            } else if (kind == svp::K2_SCALE) {
                k2_scale<R>(a, op.v[0]);
            } else if (kind == svp::K2_PHASE) {
                k2_phase<R>(a, cx, op.a, (uint32_t)op.m0, op.m1, mk<C>(op.v[0], op.v[1]));
            } else if (kind == svp::K2_DIAG) {
                k2_diag<R>(a, cx, op.a, op.b, op.c, (uint32_t)op.m0, op.m1, mk<C>(op.v[0], op.v[1]),
                           mk<C>(op.v[2], op.v[3]));
            } else {
                const int ckind = op.b;
                const bool tpred = (ckind == svp::CK_MEM) ? code_bit(cx.tloc, cx.base, op.c) : true;
                const int cslot = op.c;
                switch (op.a) {
                case 0: k2_pairs<0, R>(a, kind, op.v, tpred, ckind, cslot); break;
                case 1: if constexpr (LOGR > 1) k2_pairs<1, R>(a, kind, op.v, tpred, ckind, cslot); break;
                case 2: if constexpr (LOGR > 2) k2_pairs<2, R>(a, kind, op.v, tpred, ckind, cslot); break;
                case 3: if constexpr (LOGR > 3) k2_pairs<3, R>(a, kind, op.v, tpred, ckind, cslot); break;
                case 4: if constexpr (LOGR > 4) k2_pairs<4, R>(a, kind, op.v, tpred, ckind, cslot); break;
                default: break;
                }
            }
        }
    }
};

}  // namespace svk
