// Test-only host emulator of the planner's device programs.
//
// It runs the steps that make_plan produces (plain sweeps, explicit exchange
// passes and block-resident passes with their op programs and tables) on a
// complex<double> state, re-implementing the kernels' index arithmetic
// (register slots, thread-id deposit, LDS re-layout, lane/wave/block-uniform
// factors) on the CPU. Tests compare it with the FP64 oracle, so a wrong op
// or table emitted by the planner is caught without a GPU. It is not linked
// into the simulator library.
#include <cmath>
#include <cstdio>
#include <complex>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <cstdlib>
#include <vector>

#ifndef SV_EMU_NO_JIT
#include "../../paper_2605_15098_amd/csrc/jit.h"
#endif
#include "../../paper_2605_15098_amd/csrc/plan.h"
#include "../../paper_2605_15098_amd/csrc/plan.h"

using cd = std::complex<double>;
using namespace svp;

namespace {

// Writes per amplitude in the current step (every kernel is checked to write
// each amplitude it owns exactly once per step) and the steps that broke it.
std::vector<uint32_t> g_writes;
bool g_plant_double_write = false;  // tests: one block pass stores an amplitude twice
int64_t g_write_faults = 0, g_writes_total = 0;

void note_write(uint64_t i)
{
    g_writes[i] += 1;
    g_writes_total += 1;
}

// After a step: every amplitude written exactly `expect(i)` times (0 or 1).
template <class F>
void check_writes(uint64_t N, F expect)
{
    for (uint64_t i = 0; i < N; ++i) {
        if (g_writes[i] != expect(i)) {
            ++g_write_faults;
            break;
        }
    }
    std::fill(g_writes.begin(), g_writes.end(), 0u);
}

void apply_pair_gate(std::vector<cd> &S, int n, const MGate &g)
{
    const uint64_t N = 1ull << n;
    const cd u00(g.u[0], g.u[1]), u01(g.u[2], g.u[3]), u10(g.u[4], g.u[5]), u11(g.u[6], g.u[7]);
    for (uint64_t j = 0; j < N; ++j) {
        if ((j >> g.t) & 1ull) continue;
        if (g.c >= 0 && !((j >> g.c) & 1ull)) continue;
        const uint64_t k = j | (1ull << g.t);
        const cd a = S[j], b = S[k];
        S[j] = u00 * a + u01 * b;
        S[k] = u10 * a + u11 * b;
        note_write(j);
        note_write(k);
    }
}

cd expturn(uint64_t a)
{
    const double x = std::ldexp((double)(int64_t)a, -63);
    return cd(std::cos(M_PI * x), std::sin(M_PI * x));
}

bool return_error = false;
int g_dtype = 0;  // dtype of the plan being emulated (table precision)

void run_k2(std::vector<cd> &S, int n, const Step &st, const Plan &plan)
{
    const int l = st.l, r = st.logr, R = 1 << r, tb = l - r;
    const int NT = 1 << tb;
    std::vector<int> nb;
    {
        std::vector<bool> in(n, false);
        for (int i = 0; i < l; ++i) in[st.bits[i]] = true;
        for (int p = 0; p < n; ++p)
            if (!in[p]) nb.push_back(p);
    }
    const uint64_t nblocks = 1ull << (n - l);
    std::vector<cd> lds(1ull << l);
    const uint8_t *table = plan.table.data();
    for (uint64_t bid = 0; bid < nblocks; ++bid) {
        uint64_t base = 0;
        for (int i = 0; i < n - l; ++i) base |= ((bid >> i) & 1ull) << nb[i];
        std::vector<cd> ufac(st.nug);
        for (int g = 0; g < st.nug; ++g) {
            const UGroup *ug = reinterpret_cast<const UGroup *>(table + st.ug_off) + g;
            const UTerm *tm = reinterpret_cast<const UTerm *>(table + st.ut_off) + ug->term_off;
            uint64_t acc = 0;
            for (int j = 0; j < ug->nterms; ++j)
                if ((base & tm[j].tmask) == tm[j].tmask) acc += tm[j].angle;
            ufac[g] = expturn(acc);
        }
        // per-thread registers; canonical layout: slot 0 = local bit 0,
        // slots 1.. = top local bits
        std::vector<std::vector<cd>> a(NT, std::vector<cd>(R));
        std::vector<int> rb(r);
        rb[0] = 0;
        for (int j = 1; j < r; ++j) rb[j] = k2_canon_bit(j, l, r);
        std::vector<uint32_t> tloc(NT);
        auto set_layout = [&]() {
            uint32_t rmask = 0;
            for (int j = 0; j < r; ++j) rmask |= 1u << rb[j];
            for (int tid = 0; tid < NT; ++tid) {
                uint32_t tl = 0;
                int cnt = 0;
                for (int i = 0; i < l; ++i) {
                    if ((rmask >> i) & 1u) continue;
                    tl |= ((uint32_t)(tid >> cnt) & 1u) << i;
                    ++cnt;
                }
                tloc[tid] = tl;
            }
        };
        set_layout();
        auto code_bit = [&](int tid, int code) {
            return code >= 64 ? (bool)((base >> (code - 64)) & 1ull) : (bool)((tloc[tid] >> code) & 1u);
        };
        auto tpred_of = [&](int tid, const K2Op &op) {
            return ((tloc[tid] & (uint32_t)op.m0) == (uint32_t)op.m0) && ((base & op.m1) == op.m1);
        };
        auto amp_mem = [&](int tid, int k) {
            uint32_t x = tloc[tid];
            for (int j = 0; j < r; ++j)
                if ((k >> j) & 1) x |= 1u << rb[j];
            uint64_t addr = base;
            for (int i = 0; i < l; ++i)
                if ((x >> i) & 1u) addr |= 1ull << st.bits[i];
            return addr;
        };
        auto amp_loc = [&](int tid, int k) {
            uint32_t x = tloc[tid];
            for (int j = 0; j < r; ++j)
                if ((k >> j) & 1) x |= 1u << rb[j];
            return x;
        };
        for (int tid = 0; tid < NT; ++tid)
            for (int k = 0; k < R; ++k) a[tid][k] = S[amp_mem(tid, k)];
        for (int oi = 0; oi < st.op_count; ++oi) {
            const K2Op &op = plan.ops[st.op_begin + oi];
            if (op.kind == K2_LAYOUT && op.b >= 32) {
                // split by a thread-id bit: round h is done by the threads
                // whose id bit p is h, all their registers, through half the LDS
                const int x = op.b - 32;
                std::vector<int> nrb(r);
                uint32_t om = 0, nm = 0;
                for (int j = 0; j < r; ++j) {
                    nrb[j] = (op.a >> (5 * j)) & 31;
                    om |= 1u << rb[j];
                    nm |= 1u << nrb[j];
                }
                const uint32_t below = (1u << x) - 1u;
                const int p = x - __builtin_popcount(om & below);
                if (((om | nm) >> x) & 1u || p != x - __builtin_popcount(nm & below)) {
                    return_error = true;
                    return;
                }
                auto drop = [](uint32_t v, int b) { return (v & ((1u << b) - 1u)) | ((v >> (b + 1)) << b); };
                std::vector<uint32_t> old_loc(NT * R);
                for (int tid = 0; tid < NT; ++tid)
                    for (int k = 0; k < R; ++k) old_loc[tid * R + k] = amp_loc(tid, k);
                rb = nrb;
                set_layout();
                std::vector<cd> half(1ull << (l - 1));
                for (int h = 0; h < 2; ++h) {
                    std::vector<int> filled(half.size(), 0);
                    for (int tid = 0; tid < NT; ++tid) {
                        if (((tid >> p) & 1) != h) continue;
                        for (int k = 0; k < R; ++k) {
                            const uint32_t i = drop(old_loc[tid * R + k], x);
                            if (i >= half.size() || filled[i]++) return_error = true;
                            else half[i] = a[tid][k];
                        }
                    }
                    for (int tid = 0; tid < NT; ++tid) {
                        if (((tid >> p) & 1) != h) continue;
                        for (int k = 0; k < R; ++k) {
                            const uint32_t i = drop(amp_loc(tid, k), x);
                            if (i >= half.size() || filled[i]-- != 1) return_error = true;
                            else a[tid][k] = half[i];
                        }
                    }
                }
            } else if (op.kind == K2_LAYOUT && op.b >= 0) {
                // split re-layout: two rounds through half the LDS, as the
                // kernel does it (bit op.b taken out of the local index);
                // every cell of a round is written once and read once
                const int sb = op.b;
                std::vector<int> nrb(r);
                for (int j = 0; j < r; ++j) nrb[j] = (op.a >> (5 * j)) & 31;
                int s = -1;
                for (int j = 0; j < r; ++j)
                    if (rb[j] == sb && nrb[j] == sb) s = j;
                if (s < 0) {
                    return_error = true;
                    return;
                }
                auto drop = [](uint32_t x, int b) { return (x & ((1u << b) - 1u)) | ((x >> (b + 1)) << b); };
                const std::vector<int> old_rb = rb;
                const std::vector<uint32_t> old_tloc = tloc;
                rb = nrb;
                set_layout();
                const std::vector<uint32_t> new_tloc = tloc;
                std::vector<cd> half(1ull << (l - 1));
                for (int h = 0; h < 2; ++h) {
                    std::vector<int> filled(half.size(), 0);
                    for (int tid = 0; tid < NT; ++tid)
                        for (int k = 0; k < R; ++k) {
                            if (((k >> s) & 1) != h) continue;
                            uint32_t x = old_tloc[tid];
                            for (int j = 0; j < r; ++j)
                                if (j != s && ((k >> j) & 1)) x |= 1u << old_rb[j];
                            const uint32_t i = drop(x, sb);
                            if (i >= half.size() || filled[i]++) return_error = true;
                            else half[i] = a[tid][k];
                        }
                    for (int tid = 0; tid < NT; ++tid)
                        for (int k = 0; k < R; ++k) {
                            if (((k >> s) & 1) != h) continue;
                            uint32_t x = new_tloc[tid];
                            for (int j = 0; j < r; ++j)
                                if (j != s && ((k >> j) & 1)) x |= 1u << nrb[j];
                            const uint32_t i = drop(x, sb);
                            if (i >= half.size() || filled[i]-- != 1) return_error = true;
                            else a[tid][k] = half[i];
                        }
                }
            } else if (op.kind == K2_LAYOUT) {
                if (st.half_lds) return_error = true;  // LDS holds only half the block
                for (int tid = 0; tid < NT; ++tid)
                    for (int k = 0; k < R; ++k) lds[amp_loc(tid, k)] = a[tid][k];
                for (int j = 0; j < r; ++j) rb[j] = (op.a >> (5 * j)) & 31;
                set_layout();
                for (int tid = 0; tid < NT; ++tid)
                    for (int k = 0; k < R; ++k) a[tid][k] = lds[amp_loc(tid, k)];
            } else if (op.kind == K2_PHASE) {
                const cd z(op.v[0], op.v[1]);
                for (int tid = 0; tid < NT; ++tid) {
                    if (!tpred_of(tid, op)) continue;
                    for (int k = 0; k < R; ++k)
                        if ((k & op.a) == op.a) a[tid][k] *= z;
                }
            } else if (op.kind == K2_DIAG) {
                const cd d0(op.v[0], op.v[1]), d1(op.v[2], op.v[3]);
                for (int tid = 0; tid < NT; ++tid) {
                    if (!tpred_of(tid, op)) continue;
                    for (int k = 0; k < R; ++k) {
                        if ((k & op.c) != op.c) continue;
                        bool sel = op.a >= 0 ? (bool)((k >> op.a) & 1) : code_bit(tid, op.b);
                        a[tid][k] *= sel ? d1 : d0;
                    }
                }
            } else if (op.kind == K2_DIAGRUN) {
                const DiagRun *rec = reinterpret_cast<const DiagRun *>(table + op.a);
                const DiagGroup *gs = reinterpret_cast<const DiagGroup *>(rec + 1);
                const double *qt = reinterpret_cast<const double *>(gs + rec->ngroups);
                // record invariants: groups sorted by their highest register
                // bit, every slot a group or a constant touches is multiplied
                auto top = [](int m) { return m ? 31 - __builtin_clz((uint32_t)m) : -1; };
                for (int i = 1; i < rec->ngroups; ++i)
                    if (top(gs[i - 1].rmask) > top(gs[i].rmask)) return_error = true;
                if ((rec->qmask & ~rec->kmask) != 0) return_error = true;
                for (int i = 0; i < rec->ngroups; ++i)
                    for (int k = 0; k < R; ++k)
                        if ((k & gs[i].rmask) == gs[i].rmask && !((rec->kmask >> k) & 1u)) return_error = true;
                const double *ptab = reinterpret_cast<const double *>(table + st.tab_off);
                for (int tid = 0; tid < NT; ++tid) {
                    std::vector<cd> gf(rec->ngroups, cd(1, 0));
                    for (int i = 0; i < rec->ngroups; ++i) {
                        const DiagGroup &G = gs[i];
                        bool on = true;
                        if (G.cond_kind == 1) on = (base >> G.cond_bit) & 1ull;
                        else if (G.cond_kind == 2) on = (tid >> G.cond_bit) & 1;
                        if (!on) continue;
                        cd f(1, 0);
                        if (G.uidx >= 0) f = ufac[G.uidx];
                        if (G.wave_off >= 0) {
                            const double *w = ptab + 2 * G.wave_off;
                            f *= cd(w[2 * (tid >> 6)], w[2 * (tid >> 6) + 1]);
                        }
                        if (G.lane_off >= 0) {
                            const double *w = ptab + 2 * G.lane_off;
                            f *= cd(w[2 * (tid & 63)], w[2 * (tid & 63) + 1]);
                        }
                        gf[i] = f;
                    }
                    for (int k = 0; k < R; ++k) {
                        if (!((rec->kmask >> k) & 1u)) continue;
                        cd F(1, 0);
                        for (int i = 0; i < rec->ngroups; ++i)
                            if ((k & gs[i].rmask) == gs[i].rmask) F *= gf[i];
                        if ((rec->qmask >> k) & 1u) F *= cd(qt[2 * k], qt[2 * k + 1]);
                        a[tid][k] *= F;
                    }
                }
            } else if (op.kind == K2_SCALE) {
                for (int tid = 0; tid < NT; ++tid)
                    for (int k = 0; k < R; ++k) a[tid][k] *= op.v[0];
            } else if (op.kind == K2_MFMA) {
                if (st.half_lds) return_error = true;  // windows read the whole block from LDS
                // unpack the operand-ordered real matrix and apply it to every
                // vector of the window bits, in FP64
                const int K = op.b, W = 1 << K, D = 2 * W, steps = D / 4;
                std::vector<int> w(K);
                uint32_t wm = 0;
                for (int i = 0; i < K; ++i) {
                    w[i] = (op.c >> (5 * i)) & 31;
                    wm |= 1u << w[i];
                }
                if ((uint64_t)wm != op.m0) return_error = true;
                std::vector<double> M((size_t)D * D);
                for (int t = 0; t < D / 16; ++t)
                    for (int s = 0; s < steps; ++s)
                        for (int lane = 0; lane < 64; ++lane) {
                            const size_t idx = ((size_t)t * steps + s) * 64 + lane;
                            const double v = g_dtype == 0 ? (double)reinterpret_cast<const float *>(table + op.a)[idx]
                                                          : reinterpret_cast<const double *>(table + op.a)[idx];
                            M[(size_t)(16 * t + lane % 16) * D + 4 * s + lane / 16] = v;
                        }
                for (int tid = 0; tid < NT; ++tid)
                    for (int k = 0; k < R; ++k) lds[amp_loc(tid, k)] = a[tid][k];
                for (uint32_t v = 0; v < (1u << (l - K)); ++v) {
                    uint32_t vb = 0, mm = v;
                    for (int b = 0; b < l; ++b)
                        if (!((wm >> b) & 1u)) {
                            vb |= (mm & 1u) << b;
                            mm >>= 1;
                        }
                    auto addr = [&](int j) {
                        uint32_t x = vb;
                        for (int i = 0; i < K; ++i)
                            if ((j >> i) & 1) x |= 1u << w[i];
                        return x;
                    };
                    std::vector<double> in(D), out(D, 0.0);
                    for (int j = 0; j < W; ++j) {
                        in[2 * j] = lds[addr(j)].real();
                        in[2 * j + 1] = lds[addr(j)].imag();
                    }
                    for (int rr = 0; rr < D; ++rr)
                        for (int cc = 0; cc < D; ++cc) out[rr] += M[(size_t)rr * D + cc] * in[cc];
                    for (int j = 0; j < W; ++j) lds[addr(j)] = cd(out[2 * j], out[2 * j + 1]);
                }
                for (int tid = 0; tid < NT; ++tid)
                    for (int k = 0; k < R; ++k) a[tid][k] = lds[amp_loc(tid, k)];
            } else {
                const int J = op.a, H = 1 << J;
                const cd u00(op.v[0], op.v[1]), u01(op.v[2], op.v[3]), u10(op.v[4], op.v[5]),
                    u11(op.v[6], op.v[7]);
                for (int tid = 0; tid < NT; ++tid) {
                    const bool tpred = op.b == CK_MEM ? code_bit(tid, op.c) : true;
                    if (!tpred) continue;
                    for (int k = 0; k < R; ++k) {
                        if (k & H) continue;
                        if (op.b == CK_SLOT && !((k >> op.c) & 1)) continue;
                        cd x = a[tid][k], y = a[tid][k + H];
                        if (op.kind == K2_H) {
                            const double s = 0.70710678118654752440;
                            a[tid][k] = (x + y) * s;
                            a[tid][k + H] = (x - y) * s;
                        } else if (op.kind == K2_HU) {
                            a[tid][k] = x + y;
                            a[tid][k + H] = x - y;
                        } else if (op.kind == K2_X) {
                            a[tid][k] = y;
                            a[tid][k + H] = x;
                        } else {
                            a[tid][k] = u00 * x + u01 * y;
                            a[tid][k + H] = u10 * x + u11 * y;
                        }
                    }
                }
            }
        }
        for (int tid = 0; tid < NT; ++tid)
            for (int k = 0; k < R; ++k) {
                const uint64_t addr = amp_mem(tid, k);
                S[addr] = a[tid][k];
                note_write(addr);
            }
        if (g_plant_double_write && bid == 0) note_write(amp_mem(0, 0));  // planted mistake (tests)
    }
}

}  // namespace

extern "C" int emu_apply(int n, int dtype, int mode, int l, int logr, int policy, int remap, int diag_free,
                         int pin_low, int fuse_k, const void *gates, size_t m, double *state_inout,
                         int64_t *counts_out)
{
    PlanConfig c;
    g_dtype = dtype;
    if (const char *e = std::getenv("SV_HALF_LDS")) c.half_lds = std::atoi(e);
    c.n = n;
    c.dtype = dtype;
    c.mode = mode;
    c.l = l;
    c.logr = logr;
    c.policy = policy;
    c.remap = remap;
    c.diag_free = diag_free;
    c.pin_low = pin_low;
    c.fuse_k = fuse_k;
    std::vector<int> l2p(n);
    for (int q = 0; q < n; ++q) l2p[q] = q;
    Plan plan;
    return_error = false;
    std::string err = make_plan(c, reinterpret_cast<const RawGate *>(gates), m, l2p, plan);
    if (!err.empty()) return -1;
    const uint64_t N = 1ull << n;
    std::vector<cd> S(N);
    for (uint64_t i = 0; i < N; ++i) S[i] = cd(state_inout[2 * i], state_inout[2 * i + 1]);
    g_writes.assign(N, 0u);
    g_plant_double_write = std::getenv("EMU_PLANT_DOUBLE_WRITE") != nullptr;
    g_write_faults = 0;
    g_writes_total = 0;
    for (const Step &st : plan.steps) {
        if (st.kind == ST_K1) {
            apply_pair_gate(S, n, st.g);
            // the pairs whose control holds, once each
            const MGate g = st.g;
            check_writes(N, [&](uint64_t i) { return (uint32_t)(g.c < 0 || ((i >> g.c) & 1ull)); });
        } else if (st.kind == ST_K3) {
            for (uint64_t i = 0; i < N; ++i) {
                if (((i >> st.p) & 1ull) && !((i >> st.v) & 1ull)) {
                    const uint64_t k = i ^ (1ull << st.p) ^ (1ull << st.v);
                    std::swap(S[i], S[k]);
                    note_write(i);
                    note_write(k);
                }
            }
            // the exchanged pairs, once each
            check_writes(N, [&](uint64_t i) { return (uint32_t)(((i >> st.p) ^ (i >> st.v)) & 1ull); });
        } else {
            run_k2(S, n, st, plan);
            // a block pass stores every amplitude once
            check_writes(N, [](uint64_t) { return 1u; });
        }
    }
    for (uint64_t x = 0; x < N; ++x) {
        uint64_t p = 0;
        for (int q = 0; q < n; ++q) p |= ((x >> q) & 1ull) << plan.l2p_after[q];
        state_inout[2 * x] = S[p].real();
        state_inout[2 * x + 1] = S[p].imag();
    }
    if (return_error) return -2;
    counts_out[0] = plan.stats.passes;
    counts_out[1] = plan.stats.swaps;
    counts_out[2] = (int64_t)plan.ops.size();
    counts_out[3] = (int64_t)plan.table.size();
    counts_out[4] = 0;  // block passes that stage half the block
    for (const Step &st : plan.steps) counts_out[4] += st.kind == ST_K2 && st.half_lds;
    counts_out[5] = g_write_faults;  // steps that wrote an amplitude other than once
    counts_out[6] = g_writes_total;
    return 0;
}

// Plan the circuit and compile every generated block-pass kernel (no GPU
// needed). Returns the number of kernels compiled, or -1 with the first
// compiler log copied to log_out.
#ifndef SV_EMU_NO_JIT  // the sanitizer build leaves the run-time compiler out
extern "C" int emu_jit_check(int n, int dtype, int l, int logr, int policy, int remap, int diag_free, int fuse_k,
                             const void *gates, size_t m, char *log_out, size_t log_cap)
{
    PlanConfig c;
    if (const char *e = std::getenv("SV_HALF_LDS")) c.half_lds = std::atoi(e);
    c.n = n;
    c.dtype = dtype;
    c.mode = 1;
    c.l = l;
    c.logr = logr;
    c.policy = policy;
    c.remap = remap;
    c.diag_free = diag_free;
    c.fuse_k = fuse_k;
    std::vector<int> l2p(n);
    for (int q = 0; q < n; ++q) l2p[q] = q;
    Plan plan;
    if (!make_plan(c, reinterpret_cast<const RawGate *>(gates), m, l2p, plan).empty()) return -2;
    int count = 0;
    for (const Step &st : plan.steps) count += st.kind == ST_K2;
    const std::string src = svj::generate_plan(plan, dtype);
    const std::string log = svj::compile_check(src);
    if (!log.empty()) {
        std::snprintf(log_out, log_cap, "%s\n---- source ----\n%s", log.c_str(), src.c_str());
        return -1;
    }
    return count;
}
#endif
