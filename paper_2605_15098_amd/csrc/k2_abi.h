// Plain-data records shared by the host planner, the block-pass kernels and
// the pass kernels generated at run time. Only fixed-width integers and
// doubles; no library types.
#pragma once

#if defined(__HIPCC_RTC__)
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::int8_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
using __hip_internal::uint8_t;
#else
#include <cstdint>
#endif

namespace svp {

// Block-pass ops (device program).
enum K2Kind {
    K2_LAYOUT = 0,   // a: packed local bit of each register slot (5 bits
                     // each, slot 0 lowest; any order); b: how the block
                     // moves through LDS: -1 whole; 0..31 in two halves by
                     // that local bit, held by the same slot before and
                     // after; 32 + x in two halves by local bit x, a
                     // thread-id bit at the same position before and after
    K2_DENSE = 1,    // a: slot; b: control kind; c: control slot or bit code;
                     // v[0..7]: row-major 2x2 (re, im)
    K2_H = 2,        // as K2_DENSE, Hadamard
    K2_X = 3,        // as K2_DENSE, exchange
    K2_PHASE = 4,    // a: slot mask; m0: local-bit mask; m1: block-base mask;
                     // v[0..1]: factor
    K2_DIAG = 5,     // a: target slot or -1; b: target bit code when a < 0;
                     // c: slot mask; m0/m1 as K2_PHASE; v[0..1] d0, v[2..3] d1
    K2_DIAGRUN = 6,  // a: byte offset of a DiagRun in the table buffer
    K2_HU = 7,       // unnormalized Hadamard (a+b, a-b) on slot a, no control
    K2_SCALE = 8,    // every amplitude times v[0]
    K2_MFMA = 9,     // dense window unitary through the matrix cores: a: byte
                     // offset of the operand-ordered matrix in the table;
                     // b: window qubits (4 or 5); c: packed window local bits
                     // (5 bits each, ascending); m0: window local-bit mask
};
// Control of a dense op: none, a register slot, or a bit code (0..l-1 =
// local bit tested on the thread's local index, 64 + p = memory bit p of the
// block base).
enum CtlKind { CK_NONE = 0, CK_SLOT = 1, CK_MEM = 2 };

struct K2Op {
    int32_t kind, a, b, c;
    uint64_t m0, m1;
    double v[8];
};

// One thread-dependent factor of a diagonal run: applied to the amplitudes
// whose register slots cover rmask, when the block-uniform or wave-uniform
// condition holds. factor = U[uidx] * wave_table[wave] * lane_table[lane].
struct DiagGroup {
    int32_t rmask;
    int32_t cond_kind;  // 0 none, 1 memory bit of the block base, 2 thread-id bit (>= 6)
    int32_t cond_bit;
    int32_t uidx;       // block-uniform factor index, -1 none
    int32_t lane_off;   // index of 64 entries in the pass's factor table, -1 none
    int32_t wave_off;   // index of 2^(waves) entries in that table, -1 none
    int32_t pad0, pad1;
};

// A run of diagonal gates as one multiply per register slot. Followed in the
// table by ngroups DiagGroup records (sorted by the highest bit of rmask,
// groups with rmask = 0 first) and then 2^r complex doubles Q[k], the
// constant factor of register pattern k. Register slot k is multiplied (when
// k is in kmask) by F(k) = Q[k] * T(k) if k is in qmask, else T(k), where the
// thread factor T(k) folds, in this order, the groups with rmask = 0 and then,
// for each set bit b of k ascending, the groups whose highest rmask bit is b
// and whose rmask lies within k (each in record order; T = g for the first
// factor, T = T * g after). Folding in this fixed order lets a compiled pass
// share T between slots along a walk of the subsets of the register bits and
// still give the same bits as a slot-by-slot evaluation.
struct DiagRun {
    uint32_t kmask;
    uint32_t qmask;
    int32_t ngroups;
    int32_t pad;
};

// Block-uniform factor: e^{2 pi i sum angle_j [base covers tmask_j]} with
// angles as 64-bit fixed-point turns; computed once per block (complex64:
// from the exact sum of the angles; complex128: as the product of the
// covered terms' factors re + i im, formed in binary64 on the host).
struct UGroup {
    int32_t term_off;   // index of the group's first term in the pass's UTerm array
    int32_t nterms;
};
struct UTerm {
    uint64_t tmask;
    uint64_t angle;
    double re, im;      // e^{2 pi i angle}
};

// Arguments of one block pass, passed by value.
struct K2Args {
    int32_t n;
    int32_t l;
    int32_t nops;
    int32_t nug;               // block-uniform factor groups
    const uint8_t *table;      // device copy of the plan's table buffer
    int32_t ug_off;            // byte offset of the UGroup array
    int32_t vec2;              // 1: memory bit 0 is local bit 0 (16-byte complex64 pairs)
    int8_t bits[48];           // memory bit of each local bit, ascending
    int8_t nbits[48];          // memory bits outside the block, ascending
    int32_t tab_off;           // byte offset of the pass's lane/wave factor
    int32_t tab_count;         // table (tab_count complex doubles), staged in LDS
    int32_t ut_off;            // byte offset of the pass's UTerm array
    int32_t nut;               // its length (staged in LDS with the UGroups)
    // Blocks of this launch: block number b (0 <= b < 2^nblk_bits) is
    // deposited into memory bits nbits[0..nblk_bits) and OR-ed with base_or.
    // A whole-state pass has nblk_bits = n - l and base_or = 0; the outer
    // tier launches a pass on one chunk of outer blocks at a time.
    uint64_t base_or;
    int32_t nblk_bits;
    int32_t half_lds;          // 1: every re-layout is split, so LDS holds
                               // half the block (2^(l-1) amplitudes)
};

// LDS of a block pass, in this order (16-byte aligned pieces): the block
// (2^l amplitudes, or 2^(l-1) when every re-layout goes in halves), nug
// block-uniform factors (double2), the lane/wave factor table (tab_count
// amplitudes), nut UTerms, nug UGroups.
struct K2Lds {
    uint32_t ufac, tabs, uterm, ugrp, total;
};
#if defined(__HIPCC_RTC__) || defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
__host__ __device__
#endif
inline K2Lds k2_lds_layout(int l, int amp, int nug, int tab_count, int nut, int half_lds)
{
    auto up = [](uint32_t x) { return (x + 15u) & ~15u; };
    K2Lds o;
    o.ufac = up(((uint32_t)amp << l) >> (half_lds ? 1 : 0));
    o.tabs = up(o.ufac + 16u * (uint32_t)nug);
    o.uterm = up(o.tabs + (uint32_t)amp * (uint32_t)tab_count);
    o.ugrp = up(o.uterm + 32u * (uint32_t)nut);
    o.total = up(o.ugrp + 8u * (uint32_t)nug);
    return o;
}

// Canonical layout of a block pass (its load and store): register slot 0
// holds local bit 0 and slots 1..r-1 hold local bits l-r .. l-2, so the
// thread id spreads over local bits 1 .. l-r-1 (lanes walk consecutive
// memory) and the top local bit l-1. Keeping the top bit a thread-id bit
// lets most re-layouts split the block by it into halves of whole waves. A
// block of r bits is all registers.
#if defined(__HIPCC_RTC__) || defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
__host__ __device__ __attribute__((always_inline))
#endif
constexpr int k2_canon_bit(int j, int l, int r)
{
    return j == 0 ? 0 : (l == r ? j : l - r - 1 + j);
}

// Batched passes (one persistent launch over many states). Instance i is
// served by group_size work-groups (ranks 0 .. group_size-1), which run its
// passes in order and meet at a counter barrier between passes.
struct BatchInst {
    void *S;             // the instance's state
    int32_t npass;
    int32_t pass_off;    // first BatchPass of this instance
    int32_t logr;        // register tile (2^logr amplitudes per thread)
    int32_t group_size;  // work-groups sharing the instance
    int32_t ctr;         // barrier counter index (group_size > 1)
    int32_t l;           // block qubits of its passes
};
struct BatchPass {
    K2Args args;         // args.table points to the batch table
    int32_t op_begin;    // first op in the batch op array
    int32_t pad[3];
};

}  // namespace svp
