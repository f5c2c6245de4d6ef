// gfx950 kernels of the state-vector simulator.
//
//  k1  plain sweep: one gate over the whole state (Algorithm 1, Section III-A,
//      with the single-control predicate). Pairs are enumerated by inserting
//      the fixed bits into a dense counter, so consecutive lanes touch
//      consecutive amplitudes and every sweep is a coalesced HBM stream.
//  k2  block-resident pass (the flush of Section III-B): one work-group owns
//      one block of 2^l amplitudes gathered by address from its l local
//      memory bits, keeps 2^r of them per thread in registers, applies the
//      whole deferred gate run and writes the block back.
//  k3  explicit qubit exchange (the SWAP of Section III-B) as an in-place
//      pass over the amplitudes whose two bits differ.
//  k5  FP64 readouts: probabilities, marginals, argmax, norm, and
//      logical-order gather/scatter.
//
// Complex values are interleaved (re, im): float2 for complex64 and double2
// for complex128. Gate matrices arrive in binary64 and are rounded once.
// The single-gate arithmetic (cmul, cmad2, hbfly in k2_device.h) is shared by
// k1 and k2 so an unfused partitioned run reproduces the plain run bit for
// bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "k2_device.h"
#include "launch.h"
#include "plan.h"

namespace svk {

// ---------------------------------------------------------------- init

template <typename C> __global__ void __launch_bounds__(256) init_kernel(C *S, uint64_t N)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        C z;
        z.x = (i == 0) ? 1 : 0;
        z.y = 0;
        S[i] = z;
    }
}

static unsigned grid_for(uint64_t work, unsigned block, unsigned cap)
{
    uint64_t g = (work + block - 1) / block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t init_zero_state(void *S, int n, int dtype, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const unsigned g = grid_for(N, 256, 8192);
    if (dtype == 0) init_kernel<float2><<<g, 256, 0, st>>>((float2 *)S, N);
    else init_kernel<double2><<<g, 256, 0, st>>>((double2 *)S, N);
    return hipGetLastError();
}

// Logical-to-storage order in place (sto is its own inverse, so each pair
// {i, sto(i)} is swapped once, by the thread of the smaller index).
template <typename C> __global__ void __launch_bounds__(256) sto_inplace_kernel(C *S, uint64_t N)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const uint64_t j = sto<C>(i);
        if (j <= i) continue;
        const C a = S[i];
        S[i] = S[j];
        S[j] = a;
    }
}

hipError_t to_storage_order(void *S, int n, int dtype, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const int s0 = dtype == 0 ? 5 : 4;
    if (n < s0 + 10) return hipSuccess;  // stored in plain order
    const unsigned g = grid_for(N, 256, 8192);
    if (dtype == 0) sto_inplace_kernel<float2><<<g, 256, 0, st>>>((float2 *)S, N);
    else sto_inplace_kernel<double2><<<g, 256, 0, st>>>((double2 *)S, N);
    return hipGetLastError();
}

bool plain_storage(int n, int dtype) { return n < (dtype == 0 ? 5 : 4) + 10; }

// ---------------------------------------------------------------- k1

constexpr int K1_BLOCK = 256;
constexpr int K1_PER = 4;

enum { K1_DENSE = 0, K1_H = 1, K1_X = 2 };

// Pairs (j, j + 2^t) with bit t of j clear and, if c >= 0, bit c set.
template <typename C>
__global__ void __launch_bounds__(K1_BLOCK)
k1_pair_kernel(C *__restrict__ S, uint64_t npairs, int t, int c, int kind, C u00, C u01, C u10, C u11)
{
    const uint64_t base = (uint64_t)blockIdx.x * (K1_BLOCK * K1_PER) + threadIdx.x;
    const int lo = (c >= 0 && c < t) ? c : t;
    const int hi = (c >= 0 && c > t) ? c : t;
    const uint64_t cbit = c >= 0 ? (1ull << c) : 0ull;
    const uint64_t h = 1ull << t;
#pragma unroll
    for (int i = 0; i < K1_PER; ++i) {
        const uint64_t p = base + (uint64_t)i * K1_BLOCK;
        if (p >= npairs) break;
        uint64_t j = insert0(p, lo);
        if (c >= 0) j = insert0(j, hi);
        j |= cbit;
        // storage order: sto(j + h) = sto(j) ^ sto(h), bit t of j being clear
        const uint64_t sj = sto<C>(j), sk = sj ^ sto<C>(h);
        C a = S[sj], b = S[sk];
        if (kind == K1_H) {
            hbfly(a, b);
            S[sj] = a;
            S[sk] = b;
        } else if (kind == K1_X) {
            S[sj] = b;
            S[sk] = a;
        } else {
            S[sj] = cmad2(u00, a, u01, b);
            S[sk] = cmad2(u10, a, u11, b);
        }
    }
}

// Diagonal gates. Amplitudes with every bit of `ones` (at most two bits, lo
// <= hi) set are multiplied by d1 when tsel < 0, else by d0 or d1 according
// to bit tsel.
template <typename C>
__global__ void __launch_bounds__(K1_BLOCK)
k1_diag_kernel(C *__restrict__ S, uint64_t namps, int nones, int lo, int hi, int tsel, C d0, C d1)
{
    const uint64_t base = (uint64_t)blockIdx.x * (K1_BLOCK * K1_PER) + threadIdx.x;
    uint64_t ones = 0;
    if (nones >= 1) ones |= 1ull << lo;
    if (nones >= 2) ones |= 1ull << hi;
#pragma unroll
    for (int i = 0; i < K1_PER; ++i) {
        const uint64_t p = base + (uint64_t)i * K1_BLOCK;
        if (p >= namps) break;
        uint64_t j = p;
        if (nones >= 1) j = insert0(j, lo);
        if (nones >= 2) j = insert0(j, hi);
        j |= ones;
        const uint64_t sj = sto<C>(j);
        C a = S[sj];
        const C d = csel(tsel >= 0 && !((j >> tsel) & 1ull), d0, d1);
        S[sj] = cmul(d, a);
    }
}

template <typename T> static hipError_t k1_launch(void *Sv, int n, const svp::MGate &g, hipStream_t st)
{
    using C = typename CT<T>::type;
    C *S = (C *)Sv;
    const double *u = g.u;
    if (g.cls == svp::GC_DIAG) {
        const bool ptype = (u[0] == 1.0 && u[1] == 0.0);
        int bits[2], nb = 0;
        if (g.c >= 0) bits[nb++] = g.c;
        if (ptype) bits[nb++] = g.t;
        if (nb == 2 && bits[0] > bits[1]) { int x = bits[0]; bits[0] = bits[1]; bits[1] = x; }
        const uint64_t namps = 1ull << (n - nb);
        const unsigned grid = (unsigned)((namps + K1_BLOCK * K1_PER - 1) / (K1_BLOCK * K1_PER));
        k1_diag_kernel<C><<<grid, K1_BLOCK, 0, st>>>(S, namps, nb, nb > 0 ? bits[0] : 0,
                                                     nb > 1 ? bits[1] : 0, ptype ? -1 : g.t,
                                                     mk<C>(u[0], u[1]), mk<C>(u[6], u[7]));
        return hipGetLastError();
    }
    const uint64_t npairs = 1ull << (n - 1 - (g.c >= 0 ? 1 : 0));
    const unsigned grid = (unsigned)((npairs + K1_BLOCK * K1_PER - 1) / (K1_BLOCK * K1_PER));
    const int kind = g.op == 0 ? K1_H : (g.cls == svp::GC_PERM ? K1_X : K1_DENSE);
    k1_pair_kernel<C><<<grid, K1_BLOCK, 0, st>>>(S, npairs, g.t, g.c, kind, mk<C>(u[0], u[1]),
                                                 mk<C>(u[2], u[3]), mk<C>(u[4], u[5]),
                                                 mk<C>(u[6], u[7]));
    return hipGetLastError();
}

hipError_t k1_gate(void *S, int n, int dtype, const svp::MGate &g, hipStream_t st)
{
    return dtype == 0 ? k1_launch<float>(S, n, g, st) : k1_launch<double>(S, n, g, st);
}

// ---------------------------------------------------------------- extended gates

// A k-qubit unitary (2^k x 2^k, row-major, the state's precision; bit b of
// the row index = target b) on physical target bits where every physical
// bit of cmask is 1: one thread per group of 2^k amplitudes. The group base
// inserts zeros at the fixed bits (targets and controls, ascending) into
// the thread number and sets the controls; the matrix is read at uniform
// addresses (scalar loads), the 2^k outputs are stored after all inputs are
// in registers.
template <typename C, int K>
__global__ void __launch_bounds__(128) kq_kernel(C *__restrict__ S, uint64_t ngroups, KqArg a, const C *__restrict__ U)
{
    constexpr int D = 1 << K;
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
    uint64_t j = g;
    for (int i = 0; i < a.nfixed; ++i) j = insert0(j, a.fixed[i]);
    j |= a.cmask;
    const uint64_t sj = sto<C>(j);
    // storage offset of group member x (the order is linear, so offsets XOR)
    auto at = [&](int x) {
        uint64_t off = sj;
#pragma unroll
        for (int b = 0; b < K; ++b)
            if ((x >> b) & 1) off ^= a.toff[b];
        return off;
    };
    C v[D];
#pragma unroll
    for (int x = 0; x < D; ++x) v[x] = S[at(x)];
#pragma unroll
    for (int x = 0; x < D; ++x) {
        C acc = mk<C>(0.0, 0.0);
#pragma unroll
        for (int y = 0; y < D; ++y) {
            const C u = U[x * D + y];
            acc.x = xfma(u.x, v[y].x, xfma(-u.y, v[y].y, acc.x));
            acc.y = xfma(u.x, v[y].y, xfma(u.y, v[y].x, acc.y));
        }
        S[at(x)] = acc;
    }
}

template <typename C> static hipError_t kq_launch(void *S, int n, const KqArg &a, const void *U, hipStream_t st)
{
    const uint64_t ngroups = 1ull << (n - a.nfixed);
    const unsigned grid = (unsigned)((ngroups + 127) / 128);
    switch (a.k) {
    case 1: kq_kernel<C, 1><<<grid, 128, 0, st>>>((C *)S, ngroups, a, (const C *)U); break;
    case 2: kq_kernel<C, 2><<<grid, 128, 0, st>>>((C *)S, ngroups, a, (const C *)U); break;
    case 3: kq_kernel<C, 3><<<grid, 128, 0, st>>>((C *)S, ngroups, a, (const C *)U); break;
    case 4: kq_kernel<C, 4><<<grid, 128, 0, st>>>((C *)S, ngroups, a, (const C *)U); break;
    case 5: kq_kernel<C, 5><<<grid, 128, 0, st>>>((C *)S, ngroups, a, (const C *)U); break;
    case 6: kq_kernel<C, 6><<<grid, 128, 0, st>>>((C *)S, ngroups, a, (const C *)U); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t kq_gate(void *S, int n, int dtype, const int *tbits, int k, const int *cbits, int nc, const void *U,
                   hipStream_t st)
{
    if (k < 1 || k > 6 || nc < 0 || k + nc > n || k + nc > 24) return hipErrorInvalidValue;
    KqArg a{};
    a.k = k;
    int fixed[24];
    for (int b = 0; b < k; ++b) fixed[b] = tbits[b];
    for (int b = 0; b < nc; ++b) {
        fixed[k + b] = cbits[b];
        a.cmask |= 1ull << cbits[b];
    }
    a.nfixed = k + nc;
    std::sort(fixed, fixed + a.nfixed);
    for (int i = 0; i < a.nfixed; ++i) a.fixed[i] = (int8_t)fixed[i];
    for (int b = 0; b < k; ++b)
        a.toff[b] = dtype == 0 ? sto<float2>(1ull << tbits[b]) : sto<double2>(1ull << tbits[b]);
    return dtype == 0 ? kq_launch<float2>(S, n, a, U, st) : kq_launch<double2>(S, n, a, U, st);
}

// ---------------------------------------------------------------- k3

// Exchange memory bits p and v: amplitude i with bit p = 1, bit v = 0 trades
// places with i ^ 2^p ^ 2^v. Pure data movement, exact.
template <typename C>
__global__ void __launch_bounds__(K1_BLOCK) k3_kernel(C *__restrict__ S, uint64_t npairs, int p, int v)
{
    const uint64_t base = (uint64_t)blockIdx.x * (K1_BLOCK * K1_PER) + threadIdx.x;
    const int lo = p < v ? p : v, hi = p < v ? v : p;
    const uint64_t flip = (1ull << p) | (1ull << v);
#pragma unroll
    for (int i = 0; i < K1_PER; ++i) {
        const uint64_t q = base + (uint64_t)i * K1_BLOCK;
        if (q >= npairs) break;
        uint64_t j = insert0(insert0(q, lo), hi) | (1ull << p);
        const uint64_t sj = sto<C>(j), sk = sto<C>(j ^ flip);
        C a = S[sj], b = S[sk];
        S[sj] = b;
        S[sk] = a;
    }
}

hipError_t k3_swap(void *S, int n, int dtype, int p, int v, hipStream_t st)
{
    const uint64_t npairs = 1ull << (n - 2);
    const unsigned grid = (unsigned)((npairs + K1_BLOCK * K1_PER - 1) / (K1_BLOCK * K1_PER));
    if (dtype == 0) k3_kernel<float2><<<grid, K1_BLOCK, 0, st>>>((float2 *)S, npairs, p, v);
    else k3_kernel<double2><<<grid, K1_BLOCK, 0, st>>>((double2 *)S, npairs, p, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k2

// Interpreted block pass: the op list of the pass runs on every block (see
// k2_body and K2Interp in k2_device.h).
template <typename T, int LOGR, bool MFMA>
__global__ void __launch_bounds__((k2_max_threads<T, LOGR>()))
k2_kernel(typename CT<T>::type *__restrict__ S, const svp::K2Op *__restrict__ ops, svp::K2Args args)
{
    extern __shared__ unsigned char lds_raw[];
    // the build with matrix-core windows keeps no prefetch set (registers)
    k2_body_any<T, LOGR, K2Interp<MFMA>, MFMA ? 0 : 1>(S, args, lds_raw, K2Interp<MFMA>{ops, args.nops, args.l},
                                                        blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- k6

// Barrier of the work-groups that share one instance. Thread 0 releases the
// group's stores device-wide, counts itself in, and waits (bounded) until the
// count reaches `target`; a wait that exceeds `limit` polls, or an error
// raised by another group, sets *err and makes every waiter leave, so the
// grid always drains.
__device__ __forceinline__ bool group_barrier(unsigned *ctr, unsigned target, int *err, unsigned limit, int *ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(ctr, 1u);
        unsigned spins = 0;
        int good = 1;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                atomicExch(err, 1);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        __threadfence();
        *ok = good;
    }
    __syncthreads();
    // the same for every thread after the barrier: read as a uniform value,
    // so that code after a barrier stays uniform for the compiler too
    return __builtin_amdgcn_readfirstlane(*ok) != 0;
}

// The passes of one instance on this work-group's share of its blocks
// (rank among group_size work-groups). Work-groups that share an instance
// meet at the counter barrier between passes; a work-group that runs an
// instance alone meets its own waves there, since the next pass reads what
// other waves stored.
template <typename T, int LOGR, bool MFMA>
__device__ __forceinline__ bool k6_run(const svp::BatchInst &I, uint64_t rank, const svp::BatchPass *__restrict__ passes,
                       const svp::K2Op *__restrict__ ops, unsigned *ctrs, int *err, unsigned limit,
                       unsigned char *lds, int *ok)
{
    using C = typename CT<T>::type;
    for (int p = 0; p < I.npass; ++p) {
        const svp::BatchPass &P = passes[I.pass_off + p];
        // no prefetch of the next block: measured no faster here, and its
        // registers would push the interpreter into spills
        k2_body_any<T, LOGR, K2Interp<MFMA>, 0>((C *)I.S, P.args, lds,
                                                 K2Interp<MFMA>{ops + P.op_begin, P.args.nops, P.args.l}, rank,
                                                 (uint64_t)I.group_size);
        if (p + 1 == I.npass) break;
        if (I.group_size > 1) {
            if (!group_barrier(&ctrs[I.ctr], (unsigned)((p + 1) * I.group_size), err, limit, ok)) return false;
        } else {
            __syncthreads();
        }
    }
    return true;
}

// Many states in one persistent launch. Work-group w runs the jobs
// wg_off[w] .. wg_off[w+1]-1 in order; a job is (instance, rank). An
// instance spread over several work-groups is their only job; small
// instances are packed several to a work-group. Every instance uses the
// launch's work-group size: its block has l = r + log2(threads) local qubits
// with its own register tile r (I.logr, 3 .. LMAX), so a small state runs
// with smaller tiles instead of shrinking every instance's block.
template <typename T, int LMAX, bool MFMA>
__global__ void __launch_bounds__((k2_max_threads<T, LMAX>()))
k6_batch_kernel(const svp::BatchInst *__restrict__ insts, const int32_t *__restrict__ wg_off,
                const int2 *__restrict__ jobs, const svp::BatchPass *__restrict__ passes,
                const svp::K2Op *__restrict__ ops, unsigned *ctrs, int *err, unsigned limit)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ int ok;
    const int j0 = wg_off[blockIdx.x], j1 = wg_off[blockIdx.x + 1];
    for (int j = j0; j < j1; ++j) {
        if (j > j0) __syncthreads();  // the previous job's last reads of LDS
        const int2 J = jobs[j];
        const svp::BatchInst I = insts[J.x];
        bool good = true;
        if (I.logr == 3) good = k6_run<T, 3, MFMA>(I, (uint64_t)J.y, passes, ops, ctrs, err, limit, lds_raw, &ok);
        if constexpr (LMAX >= 4)
            if (I.logr == 4) good = k6_run<T, 4, MFMA>(I, (uint64_t)J.y, passes, ops, ctrs, err, limit, lds_raw, &ok);
        if constexpr (LMAX >= 5)
            if (I.logr == 5) good = k6_run<T, 5, MFMA>(I, (uint64_t)J.y, passes, ops, ctrs, err, limit, lds_raw, &ok);
        if (!good) return;
    }
}

__global__ void __launch_bounds__(256) zero_u32_kernel(unsigned *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t zero_u32(unsigned *p, uint32_t n, hipStream_t st)
{
    zero_u32_kernel<<<grid_for(n, 256, 1024), 256, 0, st>>>(p, n);
    return hipGetLastError();
}

template <typename T>
static const void *k6_fn(int lmax, bool mfma)
{
    switch (lmax * 2 + (mfma ? 1 : 0)) {
    case 6: return (const void *)k6_batch_kernel<T, 3, false>;
    case 7: return (const void *)k6_batch_kernel<T, 3, true>;
    case 8: return (const void *)k6_batch_kernel<T, 4, false>;
    case 9: return (const void *)k6_batch_kernel<T, 4, true>;
    case 10: return (const void *)k6_batch_kernel<T, 5, false>;
    case 11: return (const void *)k6_batch_kernel<T, 5, true>;
    default: return nullptr;
    }
}

int k6_max_threads(int dtype, int lmax)
{
    if (lmax < 3 || lmax > 5) return 0;
    const int bumped = lmax + (dtype == 0 ? 0 : 1);
    return bumped >= 5 ? (bumped >= 6 ? 256 : 512) : 1024;
}

int k6_occupancy(int dtype, int lmax, unsigned threads, size_t lds, bool mfma)
{
    const void *fn = dtype == 0 ? k6_fn<float>(lmax, mfma) : k6_fn<double>(lmax, mfma);
    if (!fn) return 0;
    if (lds > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)threads, lds) != hipSuccess) return 0;
    return per_cu;
}

hipError_t k6_batch(int dtype, int lmax, unsigned grid, unsigned threads, size_t lds, const svp::BatchInst *insts,
                    const int32_t *wg_off, const void *jobs, const svp::BatchPass *passes, const svp::K2Op *ops,
                    unsigned *ctrs, int *err, unsigned limit, bool mfma, hipStream_t st)
{
    const void *fn = dtype == 0 ? k6_fn<float>(lmax, mfma) : k6_fn<double>(lmax, mfma);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {&insts, &wg_off, &jobs, &passes, &ops, &ctrs, &err, &limit};
    return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, st);
}

template <typename T, int LOGR, bool MFMA>
static hipError_t k2_launch_t(void *S, const K2Args &a, const svp::K2Op *ops, hipStream_t st)
{
    using C = typename CT<T>::type;
    const size_t lds = svp::k2_lds_layout(a.l, (int)sizeof(C), a.nug, a.tab_count, a.nut, a.half_lds).total;
    static size_t attr_bytes = 64 * 1024;
    if (lds > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)k2_kernel<T, LOGR, MFMA>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_bytes = lds;
    }
    const unsigned threads = 1u << (a.l - LOGR);
    const uint64_t blocks = 1ull << a.nblk_bits;
    if (threads > (unsigned)k2_max_threads<T, LOGR>()) return hipErrorInvalidConfiguration;
    // persistent grid: as many work-groups as fit on the device at once
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k2_kernel<T, LOGR, MFMA>,
                                                                (int)threads, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const uint64_t grid = svp::k2_grid((uint64_t)per_cu * (uint64_t)cus, blocks);
    k2_kernel<T, LOGR, MFMA><<<(unsigned)grid, threads, lds, st>>>((C *)S, ops, a);
    return hipGetLastError();
}

template <typename T, bool MFMA>
static hipError_t k2_dispatch(void *S, int logr, const K2Args &a, const svp::K2Op *ops, hipStream_t st)
{
    switch (logr) {
    case 1: return k2_launch_t<T, 1, MFMA>(S, a, ops, st);
    case 2: return k2_launch_t<T, 2, MFMA>(S, a, ops, st);
    case 3: return k2_launch_t<T, 3, MFMA>(S, a, ops, st);
    case 4: return k2_launch_t<T, 4, MFMA>(S, a, ops, st);
    case 5: return k2_launch_t<T, 5, MFMA>(S, a, ops, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t k2_pass(void *S, int n, int dtype, int logr, const K2Args &a, const svp::K2Op *ops, bool mfma,
                   hipStream_t st)
{
    if (a.l < logr || a.l > n || logr < 1) return hipErrorInvalidValue;
    if (mfma)
        return dtype == 0 ? k2_dispatch<float, true>(S, logr, a, ops, st)
                          : k2_dispatch<double, true>(S, logr, a, ops, st);
    return dtype == 0 ? k2_dispatch<float, false>(S, logr, a, ops, st)
                      : k2_dispatch<double, false>(S, logr, a, ops, st);
}

// ---------------------------------------------------------------- measurement

// Inclusive prefix sums of FP64 values in a fixed order (deterministic):
// tiles of SCAN_TILE values, each thread summing SCAN_PER consecutive values,
// a work-group scan of the thread sums, then the tiles' totals scanned the
// same way (recursively) and added back.
constexpr int SCAN_THREADS = 256, SCAN_PER = 8, SCAN_TILE = SCAN_THREADS * SCAN_PER;

__device__ double block_exclusive_scan(double v, double *sh, double *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_THREADS; d <<= 1) {
        const double x = t >= d ? sh[t - d] : 0.0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    const double incl = sh[t];
    *total = sh[SCAN_THREADS - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) scan_tiles(const double *__restrict__ in, double *__restrict__ out,
                                                            uint64_t m, double *__restrict__ tile_sums)
{
    __shared__ double sh[SCAN_THREADS];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER;
    double v[SCAN_PER], s = 0.0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
        v[k] = base + k < m ? in[base + k] : 0.0;
        s += v[k];
        v[k] = s;
    }
    double total;
    const double off = block_exclusive_scan(s, sh, &total);
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k)
        if (base + k < m) out[base + k] = off + v[k];
    if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_THREADS) scan_add(double *__restrict__ out, uint64_t m,
                                                          const double *__restrict__ tile_incl)
{
    if (blockIdx.x == 0) return;
    const double off = tile_incl[blockIdx.x - 1];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k)
        if (base + k < m) out[base + k] += off;
}

size_t scan_scratch_bytes(uint64_t m)
{
    size_t b = 0;
    for (uint64_t x = (m + SCAN_TILE - 1) / SCAN_TILE; x > 1; x = (x + SCAN_TILE - 1) / SCAN_TILE) b += x * 8;
    return b + 64;
}

hipError_t scan_inclusive(const double *in, double *out, uint64_t m, void *scratch, hipStream_t st)
{
    const uint64_t tiles = (m + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles > 0xffffffffull) return hipErrorInvalidValue;
    double *sums = tiles > 1 ? (double *)scratch : nullptr;
    scan_tiles<<<(unsigned)tiles, SCAN_THREADS, 0, st>>>(in, out, m, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || tiles <= 1) return e;
    e = scan_inclusive(sums, sums, tiles, (double *)scratch + tiles, st);
    if (e != hipSuccess) return e;
    scan_add<<<(unsigned)tiles, SCAN_THREADS, 0, st>>>(out, m, sums);
    return hipGetLastError();
}

// Inverse CDF: the smallest m with cdf[m] > u * cdf[M - 1] (clamped to M - 1).
__global__ void __launch_bounds__(256) sample_search(const double *__restrict__ cdf, uint64_t M,
                                                     const double *__restrict__ u, uint64_t shots,
                                                     uint64_t *__restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= shots) return;
    const double target = u[i] * cdf[M - 1];
    uint64_t lo = 0, hi = M;  // first index in [lo, hi) with cdf > target
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    out[i] = lo < M ? lo : M - 1;
}

hipError_t sample_outcomes(const double *cdf, uint64_t M, const double *u, uint64_t shots, uint64_t *out,
                           hipStream_t st)
{
    if (shots == 0) return hipSuccess;
    sample_search<<<grid_for(shots, 256, 0x7fffffffu), 256, 0, st>>>(cdf, M, u, shots, out);
    return hipGetLastError();
}

// Projective collapse over the storage order: amplitudes whose physical
// bits in `mask` differ from `val` become 0, the others are scaled.
template <typename C>
__global__ void __launch_bounds__(256) collapse_kernel(C *__restrict__ S, uint64_t N, uint64_t mask, uint64_t val,
                                                       double scale)
{
    using T = decltype(C::x);
    const T sc = (T)scale;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const uint64_t p = sto<C>(i);  // storage position i holds physical index sto(i)
        C a = S[i];
        if ((p & mask) != val) {
            a.x = 0;
            a.y = 0;
        } else {
            a.x *= sc;
            a.y *= sc;
        }
        S[i] = a;
    }
}

hipError_t collapse(void *S, int n, int dtype, uint64_t mask, uint64_t val, double scale, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const unsigned g = grid_for(N, 256, 16384);
    if (dtype == 0) collapse_kernel<float2><<<g, 256, 0, st>>>((float2 *)S, N, mask, val, scale);
    else collapse_kernel<double2><<<g, 256, 0, st>>>((double2 *)S, N, mask, val, scale);
    return hipGetLastError();
}

// ---------------------------------------------------------------- bandwidth probe

// Plain HBM streams, the reference for the block passes' bandwidth: mode 0
// copies src to dst, mode 1 rewrites dst in place (read and write of the
// same addresses, as a block pass does). 16-byte accesses, four in flight
// per thread, grid-stride over whole-device work-groups.
__global__ void __launch_bounds__(256) stream_probe_kernel(float4 *__restrict__ dst, const float4 *__restrict__ src,
                                                            uint64_t n16, float scale)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        float4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k].x *= scale;
            v[k].y *= scale;
            v[k].z *= scale;
            v[k].w *= scale;
            dst[i + k * stride] = v[k];
        }
    }
    for (; i < n16; i += stride) {
        float4 v = src[i];
        v.x *= scale;
        v.y *= scale;
        v.z *= scale;
        v.w *= scale;
        dst[i] = v;
    }
}

hipError_t stream_probe(void *dst, const void *src, uint64_t bytes, int mode, hipStream_t st)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const uint64_t n16 = bytes / 16;
    const unsigned grid = grid_for(n16, 256, (unsigned)cus * 8u);
    stream_probe_kernel<<<grid, 256, 0, st>>>((float4 *)dst, (const float4 *)(mode == 1 ? dst : src), n16, 1.0f);
    return hipGetLastError();
}

// ---------------------------------------------------------------- k5 readouts

struct PermArg {
    int8_t p[48];
    int n;
    int ident;
};

static PermArg make_perm(const int *perm, int n)
{
    PermArg pa{};
    pa.n = n;
    pa.ident = 1;
    for (int q = 0; q < n; ++q) {
        pa.p[q] = (int8_t)(perm ? perm[q] : q);
        if (pa.p[q] != q) pa.ident = 0;
    }
    return pa;
}

__device__ __forceinline__ uint64_t phys_of(uint64_t x, const PermArg &pa)
{
    if (pa.ident) return x;
    uint64_t p = 0;
    for (int q = 0; q < pa.n; ++q) p |= ((x >> q) & 1ull) << pa.p[q];
    return p;
}

template <typename C> __device__ __forceinline__ double prob(C a)
{
    const double re = (double)a.x, im = (double)a.y;
    return re * re + im * im;
}

template <typename C>
__global__ void __launch_bounds__(256)
probs_kernel(const C *__restrict__ S, PermArg pa, double *__restrict__ out, uint64_t off, uint64_t cnt)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        out[i] = prob(S[sto<C>(phys_of(off + i, pa))]);
}

hipError_t probabilities(const void *S, int n, int dtype, const int *perm, double *out,
                         uint64_t offset, uint64_t count, hipStream_t st)
{
    const PermArg pa = make_perm(perm, n);
    const unsigned g = grid_for(count, 256, 16384);
    if (dtype == 0) probs_kernel<float2><<<g, 256, 0, st>>>((const float2 *)S, pa, out, offset, count);
    else probs_kernel<double2><<<g, 256, 0, st>>>((const double2 *)S, pa, out, offset, count);
    return hipGetLastError();
}

struct BitList {
    int8_t b[48];
    int cnt;
    int low;  // 1: b[k] == k + first (the bits form one contiguous run), first = b[0]
};

// Place bit k of v at position bl.b[k]. A contiguous run is one shift.
__device__ __forceinline__ uint64_t deposit(uint64_t v, const BitList &bl)
{
    if (bl.low) return bl.cnt ? (v << bl.b[0]) : 0ull;
    uint64_t r = 0;
    for (int k = 0; k < bl.cnt; ++k) r |= ((v >> k) & 1ull) << bl.b[k];
    return r;
}

// Each thread owns one marginal entry m and sums its 2^(n-nq) terms in order.
template <typename C>
__global__ void __launch_bounds__(256)
marg_direct_kernel(const C *__restrict__ S, BitList qb, BitList ob, double *__restrict__ out)
{
    const uint64_t M = 1ull << qb.cnt, O = 1ull << ob.cnt;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += stride) {
        const uint64_t bm = deposit(m, qb);
        double s = 0.0;
        for (uint64_t o = 0; o < O; ++o) s += prob(S[sto<C>(bm | deposit(o, ob))]);
        out[m] = s;
    }
}

// Small marginals: work-group (m, g) reduces chunk g of m's terms; the
// partials are then summed in fixed order. Deterministic.
constexpr int MARG_G = 256;

template <typename C>
__global__ void __launch_bounds__(256)
marg_chunk_kernel(const C *__restrict__ S, BitList qb, BitList ob, double *__restrict__ part)
{
    __shared__ double red[256];
    const uint64_t m = blockIdx.y;
    const uint64_t O = 1ull << ob.cnt;
    const uint64_t per = (O + MARG_G - 1) / MARG_G;
    const uint64_t o0 = (uint64_t)blockIdx.x * per;
    uint64_t o1 = o0 + per;
    if (o1 > O) o1 = O;
    const uint64_t bm = deposit(m, qb);
    double s = 0.0;
    for (uint64_t o = o0 + threadIdx.x; o < o1; o += blockDim.x) s += prob(S[sto<C>(bm | deposit(o, ob))]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[m * MARG_G + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) marg_finish_kernel(const double *__restrict__ part, uint64_t M,
                                                          double *__restrict__ out)
{
    const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double s = 0.0;
    for (int g = 0; g < MARG_G; ++g) s += part[m * MARG_G + g];
    out[m] = s;
}

static BitList make_bits(const int *b, int cnt)
{
    BitList bl{};
    bl.cnt = cnt;
    bl.low = 1;
    for (int k = 0; k < cnt; ++k) {
        bl.b[k] = (int8_t)b[k];
        if (b[k] != b[0] + k) bl.low = 0;
    }
    return bl;
}

size_t marginal_scratch_bytes(int n, int nq)
{
    if (n - nq <= 12) return 0;
    return (size_t)sizeof(double) * MARG_G << nq;
}

template <typename C>
static hipError_t marginal_t(const C *S, int n, const int *qbits, int nq, const int *obits,
                             double *out, void *scratch, hipStream_t st)
{
    const BitList qb = make_bits(qbits, nq), ob = make_bits(obits, n - nq);
    const uint64_t M = 1ull << nq;
    if (n - nq <= 12) {
        marg_direct_kernel<C><<<grid_for(M, 256, 65535), 256, 0, st>>>(S, qb, ob, out);
        return hipGetLastError();
    }
    if (M > 65535) return hipErrorInvalidValue;
    double *part = (double *)scratch;
    dim3 grid(MARG_G, (unsigned)M);
    marg_chunk_kernel<C><<<grid, 256, 0, st>>>(S, qb, ob, part);
    marg_finish_kernel<<<grid_for(M, 256, 65535), 256, 0, st>>>(part, M, out);
    return hipGetLastError();
}

hipError_t marginal(const void *S, int n, int dtype, const int *qbits, int nq, const int *obits,
                    double *out, void *scratch, hipStream_t st)
{
    return dtype == 0 ? marginal_t((const float2 *)S, n, qbits, nq, obits, out, scratch, st)
                      : marginal_t((const double2 *)S, n, qbits, nq, obits, out, scratch, st);
}

// argmax with the lowest index winning ties
__device__ __forceinline__ bool better(double v1, uint64_t i1, double v2, uint64_t i2)
{
    return v1 > v2 || (v1 == v2 && i1 < i2);
}

constexpr int AM_BLOCKS = 8192;

__device__ void block_argmax(double v, uint64_t i, double *rv, uint64_t *ri, double *outv, uint64_t *outi)
{
    __shared__ double sv[256];
    __shared__ uint64_t si[256];
    sv[threadIdx.x] = v;
    si[threadIdx.x] = i;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double v2 = sv[threadIdx.x + w];
            const uint64_t i2 = si[threadIdx.x + w];
            if (better(v2, i2, sv[threadIdx.x], si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *outv = sv[0];
        *outi = si[0];
    }
    (void)rv;
    (void)ri;
}

__global__ void __launch_bounds__(256) argmax_stage1(const double *__restrict__ p, uint64_t len,
                                                     double *pv, uint64_t *pi)
{
    double bv = -1.0;
    uint64_t bi = ~0ull;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
        if (better(p[i], i, bv, bi)) { bv = p[i]; bi = i; }
    block_argmax(bv, bi, nullptr, nullptr, &pv[blockIdx.x], &pi[blockIdx.x]);
}

__global__ void __launch_bounds__(256) argmax_stage2(const double *pv, const uint64_t *pi, int nparts,
                                                     uint64_t *res_idx, double *res_val)
{
    double bv = -1.0;
    uint64_t bi = ~0ull;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x)
        if (better(pv[i], pi[i], bv, bi)) { bv = pv[i]; bi = pi[i]; }
    block_argmax(bv, bi, nullptr, nullptr, res_val, res_idx);
}

size_t argmax_scratch_bytes(uint64_t) { return (size_t)AM_BLOCKS * (sizeof(double) + sizeof(uint64_t)); }

hipError_t argmax(const double *p, uint64_t len, void *scratch, uint64_t *res_idx, double *res_val,
                  hipStream_t st)
{
    double *pv = (double *)scratch;
    uint64_t *pi = (uint64_t *)(pv + AM_BLOCKS);
    const unsigned g = grid_for(len, 256, AM_BLOCKS);
    argmax_stage1<<<g, 256, 0, st>>>(p, len, pv, pi);
    argmax_stage2<<<1, 256, 0, st>>>(pv, pi, (int)g, res_idx, res_val);
    return hipGetLastError();
}

// The marginal's physical bits in ascending order, as runs of consecutive
// bits (a permuted layout usually leaves one or two), and the logical bit of
// each: the marginal is walked in memory order so that neighbouring threads
// read neighbouring amplitudes, and the logical index is formed only for
// entries that can win.
struct PhysMarg {
    int8_t src[48], dst[48], len[48];  // run r: bits src..src+len-1 of p -> dst..
    int8_t lbit[48];                   // logical bit of the k-th physical bit (ascending)
    int nruns, cnt;
};

__device__ __forceinline__ uint64_t deposit_runs(uint64_t p, const PhysMarg &q)
{
    uint64_t r = 0;
    for (int k = 0; k < q.nruns; ++k) r |= ((p >> q.src[k]) & ((1ull << q.len[k]) - 1ull)) << q.dst[k];
    return r;
}

template <typename C>
__global__ void __launch_bounds__(256) marg_argmax_stage1(const C *__restrict__ S, PhysMarg qm, BitList ob,
                                                          double *pv, uint64_t *pi)
{
    const uint64_t M = 1ull << qm.cnt, O = 1ull << ob.cnt;
    double bv = -1.0;
    uint64_t bi = ~0ull;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += stride) {
        const uint64_t bm = deposit_runs(p, qm);
        double s = 0.0;
        for (uint64_t o = 0; o < O; ++o) s += prob(S[sto<C>(bm | deposit(o, ob))]);
        if (s >= bv) {
            uint64_t m = 0;
            for (int k = 0; k < qm.cnt; ++k) m |= ((p >> k) & 1ull) << qm.lbit[k];
            if (better(s, m, bv, bi)) { bv = s; bi = m; }
        }
    }
    block_argmax(bv, bi, nullptr, nullptr, &pv[blockIdx.x], &pi[blockIdx.x]);
}

// Scratch of the allocation-free readout: partial maxima of the fused
// marginal/argmax kernels, then the result (index, value). One copy per GPU
// for the life of the process; in host code the name below is not a device
// address: kernels get the per-device address from static_scratch().
constexpr size_t kStaticScratchBytes = (size_t)AM_BLOCKS * (sizeof(double) + sizeof(uint64_t)) + 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t static_scratch(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t marginal_argmax(const void *S, int n, int dtype, const int *qbits, int nq, const int *obits,
                           void *scratch, uint64_t *res_idx, double *res_val, hipStream_t st)
{
    const BitList ob = make_bits(obits, n - nq);
    PhysMarg qm{};
    qm.cnt = nq;
    {
        int order[64];
        for (int j = 0; j < nq; ++j) order[j] = j;
        for (int a = 1; a < nq; ++a)  // ascending physical bit
            for (int b = a; b > 0 && qbits[order[b]] < qbits[order[b - 1]]; --b) {
                const int t = order[b];
                order[b] = order[b - 1];
                order[b - 1] = t;
            }
        for (int k = 0; k < nq; ++k) {
            qm.lbit[k] = (int8_t)order[k];
            const int phys = qbits[order[k]];
            if (qm.nruns > 0 && qm.dst[qm.nruns - 1] + qm.len[qm.nruns - 1] == phys) {
                qm.len[qm.nruns - 1] += 1;
            } else {
                qm.src[qm.nruns] = (int8_t)k;
                qm.dst[qm.nruns] = (int8_t)phys;
                qm.len[qm.nruns] = 1;
                qm.nruns += 1;
            }
        }
    }
    double *pv = (double *)scratch;
    uint64_t *pi = (uint64_t *)(pv + AM_BLOCKS);
    const unsigned g = grid_for(1ull << nq, 256, AM_BLOCKS);
    if (dtype == 0) marg_argmax_stage1<float2><<<g, 256, 0, st>>>((const float2 *)S, qm, ob, pv, pi);
    else marg_argmax_stage1<double2><<<g, 256, 0, st>>>((const double2 *)S, qm, ob, pv, pi);
    argmax_stage2<<<1, 256, 0, st>>>(pv, pi, (int)g, res_idx, res_val);
    return hipGetLastError();
}

template <typename C>
__global__ void __launch_bounds__(256) norm_stage1(const C *__restrict__ S, uint64_t N, double *part)
{
    __shared__ double red[256];
    double s = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) s += prob(S[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) norm_stage2(const double *part, int nparts, double *res)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *res = red[0];
}

size_t norm_scratch_bytes(int) { return (size_t)AM_BLOCKS * sizeof(double); }

hipError_t norm2(const void *S, int n, int dtype, void *scratch, double *res, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const unsigned g = grid_for(N, 256, AM_BLOCKS);
    double *part = (double *)scratch;
    if (dtype == 0) norm_stage1<float2><<<g, 256, 0, st>>>((const float2 *)S, N, part);
    else norm_stage1<double2><<<g, 256, 0, st>>>((const double2 *)S, N, part);
    norm_stage2<<<1, 256, 0, st>>>(part, (int)g, res);
    return hipGetLastError();
}

template <typename C>
__global__ void __launch_bounds__(256) gather_kernel(const C *__restrict__ S, PermArg pa, C *__restrict__ out,
                                                     uint64_t off, uint64_t cnt)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        out[i] = S[sto<C>(phys_of(off + i, pa))];
}

template <typename C>
__global__ void __launch_bounds__(256) scatter_kernel(C *__restrict__ S, PermArg pa, const C *__restrict__ in,
                                                      uint64_t off, uint64_t cnt)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
        S[sto<C>(phys_of(off + i, pa))] = in[i];
}

hipError_t gather_logical(const void *S, int n, int dtype, const int *perm, void *out, uint64_t offset,
                          uint64_t count, hipStream_t st)
{
    const PermArg pa = make_perm(perm, n);
    const unsigned g = grid_for(count, 256, 16384);
    if (dtype == 0) gather_kernel<float2><<<g, 256, 0, st>>>((const float2 *)S, pa, (float2 *)out, offset, count);
    else gather_kernel<double2><<<g, 256, 0, st>>>((const double2 *)S, pa, (double2 *)out, offset, count);
    return hipGetLastError();
}

hipError_t scatter_logical(void *S, int n, int dtype, const int *perm, const void *in, uint64_t offset,
                           uint64_t count, hipStream_t st)
{
    const PermArg pa = make_perm(perm, n);
    const unsigned g = grid_for(count, 256, 16384);
    if (dtype == 0) scatter_kernel<float2><<<g, 256, 0, st>>>((float2 *)S, pa, (const float2 *)in, offset, count);
    else scatter_kernel<double2><<<g, 256, 0, st>>>((double2 *)S, pa, (const double2 *)in, offset, count);
    return hipGetLastError();
}

}  // namespace svk
