// Host-side planner: turns a gate list into the device work of one
// sv_apply_circuit call. Pure C++17, no HIP types, so it runs and is tested
// without a GPU.
//
// Two schedules:
//  - plain: one whole-state sweep per gate (Algorithm 1 of Section III-A);
//  - partitioned (Section III-B): the state is split into blocks of 2^l
//    amplitudes; gates whose target is local are deferred and, when a gate
//    with a global target arrives (or the circuit ends), the deferred run is
//    applied block by block in one block-resident pass; the global target is
//    then brought into the block in place of a victim chosen by LRU (the
//    paper) or by furthest next use, and the logical-to-physical map is
//    updated. A global control is decided per block.
//
// Device program of one block-resident pass: every work-group holds one
// block, 2^r amplitudes per thread in registers ("register slots"), the
// other l-r local bits spread over the thread id (lanes = thread-id bits
// 0..5, waves above). Gates target register slots; a layout op moves the
// block through LDS so that other local bits become register slots.
// Diagonal gates act on any bit; a run of them becomes one phase multiply per
// amplitude whose factor is assembled from host-built tables.
#pragma once

#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "k2_abi.h"

namespace svp {

// Gate classes after matrix construction.
enum GateClass { GC_DENSE = 0, GC_DIAG = 1, GC_PERM = 2 };

// A gate in memory-bit coordinates with its FP64 matrix.
struct MGate {
    int cls;        // GateClass
    int op;         // original op code (SV_H ...)
    int t;          // memory bit of the target
    int c;          // memory bit of the control, -1 for none
    double u[8];    // row-major 2x2 (re, im)
    // diagonal gates with unit-modulus entries: d0 = e^{2 pi i th0},
    // d1 = e^{2 pi i th1} (angles in turns); unit = 0 otherwise
    int unit;
    double th0, th1;
};

static_assert(sizeof(K2Op) == 96, "K2Op layout");
static_assert(sizeof(DiagGroup) == 32, "DiagGroup layout");
static_assert(sizeof(DiagRun) == 16, "DiagRun layout");

enum StepKind {
    ST_K1 = 0,  // one plain sweep for one gate
    ST_K2 = 1,  // one block-resident pass
    ST_K3 = 2,  // explicit exchange of memory bits p and v
};

struct Step {
    int kind = 0;
    MGate g{};              // ST_K1
    int l = 0;              // ST_K2: local bits
    int logr = 0;           // ST_K2: register bits per thread
    int bits[64] = {0};     // ST_K2: memory bit of each local bit (ascending)
    int op_begin = 0, op_count = 0;
    int ug_off = 0, nug = 0;  // ST_K2: block-uniform factor groups
    int tab_off = 0, tab_count = 0;  // ST_K2: lane/wave factor table (complex doubles)
    int ut_off = 0, nut = 0;         // ST_K2: UTerm array of the block-uniform groups
    int half_lds = 0;                // ST_K2: every re-layout split (LDS holds half the block)
    int p = 0, v = 0;       // ST_K3
    int ngates = 0;         // gates applied by this step
};

struct PlanConfig {
    int n = 0;
    int dtype = 0;            // 0 = complex64, 1 = complex128
    int mode = 1;             // 0 plain, 1 partitioned
    int l = 0;                // block qubits (0 = default)
    int logr = 0;             // register bits per thread (0 = default for the dtype)
    int policy = 0;           // 0 LRU, 1 look-ahead
    int remap = 0;            // 0 virtual, 1 explicit
    int diag_free = 0;        // diagonal gates never force a SWAP
    int pin_low = -1;         // low memory bits kept in every block (-1 = auto)
    int fuse_k = 1;           // 0: one op per gate; 1: diagonal runs combined,
                              // Hadamard normalization deferred
    int half_lds = 1;         // re-layouts in two halves: 0 never, 1 for blocks
                              // above 64 KiB, 2 whenever possible
};

struct PlanStats {
    int64_t gates = 0, swaps = 0, phases = 0, passes = 0, fused = 0;
    double bytes = 0.0;
};

struct Plan {
    std::vector<Step> steps;
    std::vector<K2Op> ops;
    std::vector<uint8_t> table;      // DiagRun, lane/wave tables, UGroup, UTerm
    PlanStats stats;
    std::vector<int> l2p_after;      // layout after the plan
    int l = 0;
};

// Default block size for a dtype (complex64 / complex128).
int default_block_qubits(int dtype);
int max_block_qubits(int dtype);
// Default low memory qubits kept in every block (virtual remap) and default
// register qubits per thread.
int default_pin_qubits(int dtype);
int default_reg_qubits(int dtype);

// Build the 2x2 FP64 matrix and class of a gate. Returns false for an
// unknown op.
bool gate_matrix(int op, double theta, const double *u_in, double *u_out, int *cls);

// Raw gate record, laid out as sv_gate.
struct RawGate {
    int32_t op, target, control, target2;
    double theta;
    double u[8];
};
std::string validate(int n, const RawGate *gates, size_t m);
// Validate and plan. l2p: layout at entry (size n); the layout after the plan
// is plan.l2p_after. Returns "" or an error message.
std::string make_plan(const PlanConfig &cfg, const RawGate *gates, size_t m,
                      const std::vector<int> &l2p, Plan &plan);

// Angle in turns -> 64-bit fixed point (mod one turn).
uint64_t turns_fixed(double turns);

// Work-groups of one block-pass launch: the resident work-groups (the
// persistent grid), at most one per block, and at most SV_K2_MAX_GRID when
// that is set to a positive number, so that each work-group walks many
// blocks even on a small state (tests of the block loop's reload paths).
inline uint64_t k2_grid(uint64_t resident, uint64_t blocks)
{
    uint64_t g = resident < blocks ? resident : blocks;
    if (const char *e = std::getenv("SV_K2_MAX_GRID")) {
        const long long cap = std::atoll(e);
        if (cap > 0 && (uint64_t)cap < g) g = (uint64_t)cap;
    }
    return g < 1 ? 1 : g;
}

}  // namespace svp
