// Host planner: gate list -> device steps. See plan.h for the model.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <queue>
#include <limits>

namespace svp {

namespace {
enum { OP_H = 0, OP_X, OP_Y, OP_Z, OP_RX, OP_RY, OP_RZ, OP_P, OP_U2, OP_SWAP };

int amp_bytes(int dtype) { return dtype == 0 ? 8 : 16; }
// Low memory bits spanning one 128-byte segment.
int segment_bits(int dtype) { return dtype == 0 ? 4 : 3; }
}  // namespace

// Defaults measured on the 32-qubit QPE (the largest blocks, 256-byte runs
// and 32 amplitudes per thread for complex64; 128-byte runs and 16 per
// thread for complex128).
int default_block_qubits(int dtype) { return dtype == 0 ? 14 : 13; }
int max_block_qubits(int dtype) { return dtype == 0 ? 14 : 13; }
int default_pin_qubits(int dtype) { return dtype == 0 ? 5 : 3; }
int default_reg_qubits(int dtype) { return dtype == 0 ? 5 : 4; }

bool gate_matrix(int op, double theta, const double *u_in, double *u, int *cls)
{
    const double s = 0.70710678118654752440;  // 1/sqrt(2)
    const double ch = std::cos(0.5 * theta), sh = std::sin(0.5 * theta);
    std::memset(u, 0, 8 * sizeof(double));
    int k = GC_DENSE;
    switch (op) {
    case OP_H: u[0] = s; u[2] = s; u[4] = s; u[6] = -s; break;
    case OP_X: u[2] = 1.0; u[4] = 1.0; k = GC_PERM; break;
    case OP_Y: u[3] = -1.0; u[5] = 1.0; break;
    case OP_Z: u[0] = 1.0; u[6] = -1.0; k = GC_DIAG; break;
    case OP_RX: u[0] = ch; u[3] = -sh; u[5] = -sh; u[6] = ch; break;
    case OP_RY: u[0] = ch; u[2] = -sh; u[4] = sh; u[6] = ch; break;
    case OP_RZ: u[0] = ch; u[1] = -sh; u[6] = ch; u[7] = sh; k = GC_DIAG; break;
    case OP_P: u[0] = 1.0; u[6] = std::cos(theta); u[7] = std::sin(theta); k = GC_DIAG; break;
    case OP_U2:
        std::memcpy(u, u_in, 8 * sizeof(double));
        if (u[2] == 0.0 && u[3] == 0.0 && u[4] == 0.0 && u[5] == 0.0) k = GC_DIAG;
        break;
    default: return false;
    }
    *cls = k;
    return true;
}

uint64_t turns_fixed(double turns)
{
    double r = turns - std::floor(turns);  // [0, 1]
    if (r >= 1.0) r = 0.0;
    return (uint64_t)std::ldexp(r, 64);
}

// Angles (turns) of the two diagonal entries of a diagonal gate, exact for
// the gate kinds defined by an angle. Entries that are not of unit modulus
// mark the gate as non-unit.
static void diag_angles(const RawGate &x, MGate &g)
{
    g.unit = 0;
    g.th0 = g.th1 = 0.0;
    if (g.cls != GC_DIAG) return;
    const double tw = 1.0 / (2.0 * M_PI);
    switch (x.op) {
    case OP_Z: g.th1 = 0.5; g.unit = 1; return;
    case OP_P: g.th1 = x.theta * tw; g.unit = 1; return;
    case OP_RZ: g.th0 = -0.5 * x.theta * tw; g.th1 = 0.5 * x.theta * tw; g.unit = 1; return;
    default: break;
    }
    const double m0 = std::hypot(g.u[0], g.u[1]), m1 = std::hypot(g.u[6], g.u[7]);
    if (std::fabs(m0 - 1.0) > 1e-14 || std::fabs(m1 - 1.0) > 1e-14) return;
    g.th0 = std::atan2(g.u[1], g.u[0]) * tw;
    g.th1 = std::atan2(g.u[7], g.u[6]) * tw;
    g.unit = 1;
}

std::string validate(int n, const RawGate *g, size_t m)
{
    if (m > 0 && !g) return "gate array is null";
    for (size_t i = 0; i < m; ++i) {
        const RawGate &x = g[i];
        const std::string at = " (gate " + std::to_string(i) + ")";
        if (x.op < OP_H || x.op > OP_SWAP) return "unknown op" + at;
        if (x.target < 0 || x.target >= n) return "target out of range" + at;
        if (x.op == OP_SWAP) {
            if (x.target2 < 0 || x.target2 >= n || x.target2 == x.target)
                return "SWAP needs two distinct qubits" + at;
            if (x.control >= 0) return "SWAP takes no control" + at;
            continue;
        }
        if (x.control < -1 || x.control >= n) return "control out of range" + at;
        if (x.control == x.target) return "control equals target" + at;
        if (!std::isfinite(x.theta)) return "non-finite angle" + at;
        if (x.op == OP_U2)
            for (int k = 0; k < 8; ++k)
                if (!std::isfinite(x.u[k])) return "non-finite matrix entry" + at;
    }
    return "";
}

namespace {

struct Builder {
    const PlanConfig &cfg;
    Plan &plan;
    int n, l, logr, ab, sbits;
    double state_bytes;

    Builder(const PlanConfig &c, Plan &p) : cfg(c), plan(p)
    {
        n = c.n;
        ab = amp_bytes(c.dtype);
        sbits = segment_bits(c.dtype);
        state_bytes = std::ldexp((double)ab, n);
        l = 0;
        logr = 0;
    }

    // Algorithmic bytes of one plain sweep: a condition bit at or above the
    // segment size halves the segments touched.
    double k1_bytes(const MGate &g) const
    {
        double b = 2.0 * state_bytes;
        if (g.c >= sbits) b *= 0.5;
        if (g.cls == GC_DIAG && g.u[0] == 1.0 && g.u[1] == 0.0 && g.t >= sbits) b *= 0.5;
        return b;
    }

    void add_k1(const MGate &g)
    {
        Step s;
        s.kind = ST_K1;
        s.g = g;
        s.ngates = 1;
        plan.steps.push_back(s);
        plan.stats.passes += 1;
        plan.stats.bytes += k1_bytes(g);
    }

    // ---- block-pass compilation ---------------------------------------

    // Lane/wave factor tables of the pass being compiled (re, im pairs);
    // stored once per pass and staged into LDS by the kernel.
    std::vector<double> ptab;

    // Append raw bytes to the table buffer at a 16-byte aligned offset.
    int table_put(const void *p, size_t bytes)
    {
        size_t off = (plan.table.size() + 15) & ~size_t(15);
        plan.table.resize(off + bytes);
        std::memcpy(plan.table.data() + off, p, bytes);
        return (int)off;
    }

    // One diagonal term: the amplitude gains angle turns (fixed point) when
    // every register slot of rmask and every memory bit of tmask is 1.
    struct Term {
        int rmask;
        uint64_t tmask;
        uint64_t angle;
    };

    // Emit a run of unit-modulus diagonal gates as one K2_DIAGRUN op for the
    // current layout.
    void emit_diag_run(const std::vector<MGate> &run, const std::vector<int> &rank,
                       const std::vector<int> &rb, std::vector<UGroup> &ugroups,
                       std::vector<UTerm> &uterms)
    {
        const int r = logr;
        // thread-id bit of each non-register local bit (lanes: 0..5)
        std::vector<int> tbit(64, -1);
        {
            std::vector<bool> isreg(l, false);
            for (int j = 0; j < r; ++j) isreg[rb[j]] = true;
            int cnt = 0;
            for (int i = 0; i < l; ++i)
                if (!isreg[i]) tbit[i] = cnt++;
        }
        const int nthread_bits = l - r;
        const int nwave_bits = nthread_bits > 6 ? nthread_bits - 6 : 0;
        auto slot_of_mem = [&](int p) -> int {
            const int lb = rank[p];
            if (lb < 0) return -1;
            for (int j = 0; j < r; ++j)
                if (rb[j] == lb) return j;
            return -1;
        };
        std::vector<Term> terms;
        auto add = [&](std::vector<int> bits, double turns) {
            Term t{0, 0, turns_fixed(turns)};
            if (t.angle == 0) return;
            for (int p : bits) {
                const int s = slot_of_mem(p);
                if (s >= 0) t.rmask |= 1 << s;
                else t.tmask |= 1ull << p;
            }
            terms.push_back(t);
        };
        for (const MGate &g : run) {
            std::vector<int> cb;
            if (g.c >= 0) cb.push_back(g.c);
            add(cb, g.th0);
            cb.push_back(g.t);
            add(cb, g.th1 - g.th0);
        }
        // classify the memory bits of a term's thread part
        enum { CL_LANE = 0, CL_WAVE = 1, CL_GLOBAL = 2 };
        auto cls = [&](int p) {
            const int lb = rank[p];
            if (lb < 0) return (int)CL_GLOBAL;
            return tbit[lb] < 6 ? (int)CL_LANE : (int)CL_WAVE;
        };
        struct GroupAcc {
            int rmask, cond_kind, cond_bit;
            std::vector<std::pair<uint64_t, uint64_t>> lane, wave, glob;  // (mask, angle)
        };
        std::vector<GroupAcc> groups;
        std::vector<uint64_t> qang(size_t(1) << r, 0);
        for (const Term &t : terms) {
            if (t.tmask == 0) {
                for (size_t k = 0; k < qang.size(); ++k)
                    if ((int(k) & t.rmask) == t.rmask) qang[k] += t.angle;
                continue;
            }
            std::vector<int> bits;
            for (int p = 0; p < 64; ++p)
                if ((t.tmask >> p) & 1ull) bits.push_back(p);
            int ck = 0, cbit = 0;
            uint64_t rest = t.tmask;
            if (bits.size() == 2 && cls(bits[0]) != cls(bits[1])) {
                // the non-lane bit (global before wave) becomes a condition
                int a = bits[0], b2 = bits[1];
                int pick = (cls(a) == CL_GLOBAL) ? a : (cls(b2) == CL_GLOBAL ? b2 : (cls(a) == CL_WAVE ? a : b2));
                if (cls(pick) == CL_GLOBAL) { ck = 1; cbit = pick; }
                else { ck = 2; cbit = tbit[rank[pick]]; }
                rest &= ~(1ull << pick);
            }
            int part = -1;
            for (int p = 0; p < 64; ++p)
                if ((rest >> p) & 1ull) part = cls(p);
            GroupAcc *G = nullptr;
            for (auto &x : groups)
                if (x.rmask == t.rmask && x.cond_kind == ck && x.cond_bit == cbit) G = &x;
            if (!G) {
                groups.push_back(GroupAcc{t.rmask, ck, cbit, {}, {}, {}});
                G = &groups.back();
            }
            if (part == CL_LANE) G->lane.push_back({rest, t.angle});
            else if (part == CL_WAVE) G->wave.push_back({rest, t.angle});
            else G->glob.push_back({rest, t.angle});
        }
        auto cexp = [](uint64_t a, double *out) {
            const double x = std::ldexp((double)(int64_t)a, -63);  // half-turns in [-1, 1)
            out[0] = std::cos(M_PI * x);
            out[1] = std::sin(M_PI * x);
        };
        // tables over lane / wave thread-id bits
        auto build_table = [&](const std::vector<std::pair<uint64_t, uint64_t>> &ts, int first, int nbits) {
            const int N = 1 << nbits;
            std::vector<double> tab(2 * std::max(N, 1));
            for (int x = 0; x < N; ++x) {
                uint64_t acc = 0;
                for (auto &pr : ts) {
                    bool on = true;
                    for (int p = 0; p < 64; ++p)
                        if ((pr.first >> p) & 1ull) {
                            const int tb = tbit[rank[p]] - first;
                            if (!((x >> tb) & 1)) on = false;
                        }
                    if (on) acc += pr.second;
                }
                cexp(acc, &tab[2 * x]);
            }
            const int idx = (int)(ptab.size() / 2);
            ptab.insert(ptab.end(), tab.begin(), tab.end());
            return idx;
        };
        // One op for the whole run (DiagRun): its groups sorted by the
        // highest register bit they need (groups without one first), the
        // slots any group or constant touches, and the constants.
        const uint32_t all = (uint32_t)((1ull << qang.size()) - 1ull);
        auto cover = [&](int rmask) {
            uint32_t m = 0;
            for (size_t k = 0; k < qang.size(); ++k)
                if ((int(k) & rmask) == rmask) m |= 1u << k;
            return m;
        };
        auto top_bit = [](int rmask) { return rmask ? 31 - __builtin_clz((uint32_t)rmask) : -1; };
        std::stable_sort(groups.begin(), groups.end(),
                         [&](const GroupAcc &x, const GroupAcc &y) { return top_bit(x.rmask) < top_bit(y.rmask); });
        DiagRun head{};
        std::vector<DiagGroup> recs;
        for (GroupAcc &G : groups) {
            DiagGroup d{};
            d.rmask = G.rmask;
            d.cond_kind = G.cond_kind;
            d.cond_bit = G.cond_bit;
            d.uidx = -1;
            d.lane_off = -1;
            d.wave_off = -1;
            if (!G.lane.empty()) d.lane_off = build_table(G.lane, 0, std::min(6, nthread_bits));
            if (!G.wave.empty()) d.wave_off = build_table(G.wave, 6, nwave_bits);
            if (!G.glob.empty()) {
                UGroup ug{(int)uterms.size(), (int)G.glob.size()};
                for (auto &pr : G.glob) {
                    double c[2];
                    cexp(pr.second, c);
                    uterms.push_back(UTerm{pr.first, pr.second, c[0], c[1]});
                }
                d.uidx = (int)ugroups.size();
                ugroups.push_back(ug);
            }
            head.kmask |= cover(G.rmask) & all;
            recs.push_back(d);
        }
        for (size_t k = 0; k < qang.size(); ++k)
            if (qang[k] != 0) head.qmask |= 1u << k;
        head.kmask |= head.qmask;
        head.ngroups = (int)recs.size();
        if (head.kmask == 0) return;
        std::vector<double> q(2 * qang.size());
        for (size_t k = 0; k < qang.size(); ++k) cexp(qang[k], &q[2 * k]);
        std::vector<uint8_t> blob(sizeof(DiagRun) + recs.size() * sizeof(DiagGroup) + q.size() * sizeof(double));
        uint8_t *w = blob.data();
        std::memcpy(w, &head, sizeof(DiagRun));
        w += sizeof(DiagRun);
        if (!recs.empty()) std::memcpy(w, recs.data(), recs.size() * sizeof(DiagGroup));
        w += recs.size() * sizeof(DiagGroup);
        std::memcpy(w, q.data(), q.size() * sizeof(double));
        K2Op op{};
        op.kind = K2_DIAGRUN;
        op.a = table_put(blob.data(), blob.size());
        plan.ops.push_back(op);
    }

    // LDS of one work-group on gfx950.
    static constexpr uint32_t kLdsLimit = 160 * 1024;
    // blocks above this many bytes stage half at a time (one 2^14 complex64
    // block would otherwise take 128 KiB of the CU's 160 KiB)
    static constexpr size_t kHalfFrom = 64 * 1024;

    // A pass is compiled with lane/wave factor tables and split re-layouts
    // when it can be; a pass whose LDS would overflow drops the tables (one
    // op per diagonal gate), and one whose re-layouts cannot all be split
    // stages the whole block.
    void compile_block(const std::vector<MGate> &q, const std::vector<int> &B)
    {
        const size_t ops0 = plan.ops.size(), tab0 = plan.table.size(), steps0 = plan.steps.size();
        const PlanStats st0 = plan.stats;
        for (int attempt = 0; attempt < 4; ++attempt) {
            const bool tables = attempt < 2, allow_half = (attempt & 1) == 0;
            const bool split_ok = compile_block_impl(q, B, tables, allow_half);
            const Step &s = plan.steps.back();
            if (attempt == 3 ||
                (split_ok && k2_lds_layout(s.l, ab, s.nug, s.tab_count, s.nut, s.half_lds).total <= kLdsLimit))
                return;
            plan.ops.resize(ops0);
            plan.table.resize(tab0);
            plan.steps.resize(steps0);
            plan.stats = st0;
        }
    }

    // Returns false when the pass was to stage half the block but a
    // re-layout had no slot that keeps its bit.
    bool compile_block_impl(const std::vector<MGate> &q, const std::vector<int> &B, bool tables, bool allow_half)
    {
        const int r = logr;
        const bool combine = cfg.fuse_k >= 1;
        const bool combine_diag = combine && tables;
        ptab.clear();
        std::vector<int> rank(64, -1);
        for (int i = 0; i < (int)B.size(); ++i) rank[B[i]] = i;
        // canonical layout (load and store): slot 0 = local bit 0, the other
        // slots = the local bits below the top one
        std::vector<int> canon(r);
        for (int j = 0; j < r; ++j) canon[j] = k2_canon_bit(j, l, r);
        std::vector<int> rb = canon;  // register slot j holds local bit rb[j]
        std::vector<UGroup> ugroups;
        std::vector<UTerm> uterms;
        auto slot_of = [&](int local) {
            for (int j = 0; j < r; ++j)
                if (rb[j] == local) return j;
            return -1;
        };
        // Split re-layouts (half): the block moves through LDS in two halves,
        // so LDS holds 2^(l-1) amplitudes and two work-groups fit on a CU.
        // The halves are split by a local bit that one register slot holds
        // before and after, or by a local bit that is the same thread-id bit
        // before and after (a wave bit, so each half is whole waves). Slot
        // order is free: a kept bit stays in its slot and a new canonical bit
        // goes to its canonical slot when that is free (so the return to the
        // canonical layout usually shares a slot); when no split exists a
        // layout keeps one current bit.
        bool half = false, split_ok = true;
        auto canon_slot = [&](int b) {
            for (int j = 0; j < r; ++j)
                if (canon[j] == b) return j;
            return -1;
        };
        auto push_layout = [&](const std::vector<int> &nrb, int split) {
            K2Op op{};
            op.kind = K2_LAYOUT;
            int packed = 0;
            for (int j = 0; j < r; ++j) packed |= nrb[j] << (5 * j);
            op.a = packed;
            op.b = split;
            plan.ops.push_back(op);
            rb = nrb;
        };
        // the split code of a re-layout rb -> nrb (K2_LAYOUT's b), -1 if none
        auto split_of = [&](const std::vector<int> &nrb) {
            for (int j = 0; j < r; ++j)
                if (nrb[j] == rb[j]) return rb[j];
            uint32_t om = 0, nm = 0;
            for (int j = 0; j < r; ++j) {
                om |= 1u << rb[j];
                nm |= 1u << nrb[j];
            }
            for (int x = l - 1; x >= 0; --x) {
                if (((om | nm) >> x) & 1u) continue;
                const uint32_t below = (1u << x) - 1u;
                const int po = x - __builtin_popcount(om & below), pn = x - __builtin_popcount(nm & below);
                // a lane bit splits within waves: only blocks of one wave or less
                if (po == pn && (po >= 6 || l - r <= 6)) return 32 + x;
            }
            return -1;
        };
        auto emit_split = [&](const std::vector<int> &nrb) {
            if (nrb == rb) return;
            const int sb = half ? split_of(nrb) : -1;
            if (half && sb < 0) split_ok = false;
            push_layout(nrb, sb);
        };
        // a layout in exactly this slot order (the canonical one); without a
        // split one of its bits is brought in first, in its slot
        auto emit_fixed = [&](const std::vector<int> &nrb) {
            if (half && nrb != rb && split_of(nrb) < 0) {
                for (int j = 0; j < r; ++j)
                    if (std::find(rb.begin(), rb.end(), nrb[j]) == rb.end()) {
                        std::vector<int> mid = rb;
                        mid[j] = nrb[j];
                        emit_split(mid);
                        break;
                    }
            }
            emit_split(nrb);
        };
        auto arrange = [&](const std::vector<int> &S) {
            std::vector<int> nrb(r, -1), rest;
            for (int b : S)
                if (slot_of(b) >= 0) nrb[slot_of(b)] = b;
            for (int b : S) {
                if (slot_of(b) >= 0) continue;
                const int j = canon_slot(b);
                if (j >= 0 && nrb[j] < 0) nrb[j] = b;
                else rest.push_back(b);
            }
            std::sort(rest.begin(), rest.end());
            size_t ri = 0;
            for (int j = 0; j < r; ++j)
                if (nrb[j] < 0) nrb[j] = rest[ri++];
            return nrb;
        };
        // a layout holding the bits S (in priority order), slots arranged
        auto emit_layout = [&](std::vector<int> S) {
            std::vector<int> nrb = arrange(S);
            if (half && nrb != rb && split_of(nrb) < 0) {
                bool keeps = false;
                for (int b : S) keeps = keeps || slot_of(b) >= 0;
                if (!keeps) {
                    // keep a canonical bit if one is held, else slot 0's bit
                    int keep = rb[0];
                    for (int j = r - 1; j >= 0; --j)
                        if (canon_slot(rb[j]) >= 0) keep = rb[j];
                    S.back() = keep;
                    nrb = arrange(S);
                }
            }
            emit_split(nrb);
        };
        // a non-register bit as the kernel tests it: local bit index, or
        // 64 + memory bit for a bit of the block base
        auto code_of = [&](int p) { return rank[p] >= 0 ? rank[p] : 64 + p; };
        auto emit_single_diag = [&](const MGate &g) {
            K2Op op{};
            const bool ptype = (g.u[0] == 1.0 && g.u[1] == 0.0);
            int rmask = 0;
            uint64_t lmask = 0, gmask = 0;
            auto cond = [&](int p) {
                const int lb = rank[p];
                const int sl = lb >= 0 ? slot_of(lb) : -1;
                if (sl >= 0) rmask |= 1 << sl;
                else if (lb >= 0) lmask |= 1ull << lb;
                else gmask |= 1ull << p;
            };
            if (g.c >= 0) cond(g.c);
            if (ptype) {
                cond(g.t);
                op.kind = K2_PHASE;
                op.a = rmask;
                op.m0 = lmask;
                op.m1 = gmask;
                op.v[0] = g.u[6];
                op.v[1] = g.u[7];
            } else {
                const int lb = rank[g.t];
                const int sl = lb >= 0 ? slot_of(lb) : -1;
                op.kind = K2_DIAG;
                op.a = sl;
                op.b = code_of(g.t);
                op.c = rmask;
                op.m0 = lmask;
                op.m1 = gmask;
                op.v[0] = g.u[0]; op.v[1] = g.u[1];
                op.v[2] = g.u[6]; op.v[3] = g.u[7];
            }
            plan.ops.push_back(op);
        };
        std::vector<MGate> pending;
        auto flush_diag = [&]() {
            if (pending.empty()) return;
            if (!combine_diag) {
                for (const MGate &g : pending) emit_single_diag(g);
            } else {
                std::vector<MGate> unit_run;
                for (const MGate &g : pending) {
                    if (g.unit) { unit_run.push_back(g); continue; }
                    // a non-unit diagonal ends the combinable run
                    if (!unit_run.empty()) emit_diag_run(unit_run, rank, rb, ugroups, uterms);
                    unit_run.clear();
                    emit_single_diag(g);
                }
                if (!unit_run.empty()) emit_diag_run(unit_run, rank, rb, ugroups, uterms);
            }
            pending.clear();
        };
        // Dense windows (fuse_k 4 or 5), formed over the pass's gate order:
        // starting at a gate on local qubits, later gates join while the
        // union of local qubits stays within fuse_k; a gate that cannot join
        // but shares no qubit with the window is set aside and its qubits
        // may no longer join (so it commutes with every window gate after
        // it), which keeps diagonal runs whole. A window needs 4 or 5
        // qubits of its own (no padding), a non-diagonal gate, and an
        // estimated vector-ALU cost of its gates above the matrix-core
        // cost of a 2^k x 2^k product (SV_FUSE_ALL=1 takes every such window:
        // tests). `items` is the pass's gate order with windows as units.
        struct Item {
            bool window;
            uint32_t bits;               // window local bits
            std::vector<MGate> gates;    // the window's gates in order, or one gate
        };
        std::vector<Item> items;
        bool any_window = false;
        {
            const bool fusing = cfg.fuse_k >= 4 && l >= 4 && l - logr >= 6;  // whole waves for the matrix op
            const bool force = [] {
                const char *e = std::getenv("SV_FUSE_ALL");
                return e && e[0] == '1';
            }();
            const int kmax = std::min(cfg.fuse_k, l);
            auto local_bits = [&](const MGate &g) -> int64_t {
                if (rank[g.t] < 0 || (g.c >= 0 && rank[g.c] < 0)) return -1;
                uint32_t m = 1u << rank[g.t];
                if (g.c >= 0) m |= 1u << rank[g.c];
                return m;
            };
            auto mem_bits = [](const MGate &g) {
                uint64_t m = 1ull << g.t;
                if (g.c >= 0) m |= 1ull << g.c;
                return m;
            };
            // vector-ALU work per amplitude of a gate in a block pass, in
            // instructions (a 2x2 product: 8; controlled: half; Hadamard: 2;
            // exchange: 1; a diagonal gate, folded into a run: 1), and the
            // measured cost of a matrix-core window in the same units. The
            // window's 2^k x 2^k product is 8 * 2^k flop per amplitude, at the
            // vector rate on this GPU for FP32 and FP64 alike, plus two LDS
            // round trips of the block and operand reads. Set from circuits
            // that keep D layers of dense gates inside 5-qubit groups (28
            // qubits, two rounds, windows growing across rounds): complex128
            // windows won only at D = 8 and complex64 windows lost at every
            // depth up to 8, so a 5-qubit window needs about 780 units of
            // replaced work in complex128 and about 1540 in complex64.
            auto valu = [&](const MGate &g) {
                double c = g.cls == GC_DIAG ? 1.0 : (g.cls == GC_PERM ? 1.0 : (g.op == 0 ? 2.0 : 8.0));
                return g.c >= 0 && g.cls != GC_DIAG ? 0.5 * c : c;
            };
            auto mfma_cost = [&](int k) { return (double)((cfg.dtype == 0 ? 48 : 24) << k) + 8.0; };
            std::vector<MGate> rest(q.begin(), q.end());
            size_t pos = 0;
            while (pos < rest.size()) {
                const int64_t m0 = fusing ? local_bits(rest[pos]) : -1;
                if (m0 < 0) {
                    items.push_back(Item{false, 0, {rest[pos]}});
                    ++pos;
                    continue;
                }
                uint32_t W = (uint32_t)m0;
                uint64_t Wmem = mem_bits(rest[pos]), blocked = 0;
                std::vector<size_t> win{pos}, aside;
                size_t j = pos + 1;
                for (; j < rest.size(); ++j) {
                    const MGate &h = rest[j];
                    const int64_t mh = local_bits(h);
                    const uint64_t hm = mem_bits(h);
                    if (mh >= 0 && (hm & blocked) == 0 && __builtin_popcount(W | (uint32_t)mh) <= kmax) {
                        W |= (uint32_t)mh;
                        Wmem |= hm;
                        win.push_back(j);
                        continue;
                    }
                    if ((hm & Wmem) == 0 && aside.size() < 64) {
                        aside.push_back(j);
                        blocked |= hm;
                        continue;
                    }
                    break;
                }
                bool dense = false;
                double cost = 0.0;
                for (size_t x : win) {
                    dense = dense || rest[x].cls != GC_DIAG;
                    cost += valu(rest[x]);
                }
                const int K = __builtin_popcount(W);
                if (win.size() < 2 || !dense || K < 4 || (!force && cost <= mfma_cost(K))) {
                    items.push_back(Item{false, 0, {rest[pos]}});
                    ++pos;
                    continue;
                }
                Item it{true, W, {}};
                for (size_t x : win) it.gates.push_back(rest[x]);
                items.push_back(std::move(it));
                any_window = true;
                // continue with the set-aside gates, then the unscanned ones
                std::vector<MGate> next;
                for (size_t x : aside) next.push_back(rest[x]);
                next.insert(next.end(), rest.begin() + (std::ptrdiff_t)j, rest.end());
                rest.swap(next);
                pos = 0;
            }
        }
        // matrix-core windows read the whole block from LDS
        half = allow_half && r >= 2 && (cfg.half_lds == 2 || (cfg.half_lds == 1 && ((size_t)ab << l) > kHalfFrom)) &&
               !any_window;
        auto emit_mfma = [&](const std::vector<MGate> &wg, uint32_t m) {
            std::vector<int> wl;
            for (int b = 0; b < l; ++b)
                if ((m >> b) & 1u) wl.push_back(b);
            const int K = (int)wl.size();
            const int W = 1 << K;
            auto pos = [&](int memb) {
                const int lb = rank[memb];
                for (int i = 0; i < K; ++i)
                    if (wl[i] == lb) return i;
                return -1;
            };
            // U (row-major, interleaved re/im) = product of the gates, later gates on the left
            std::vector<double> U(2 * (size_t)W * W, 0.0);
            for (int x = 0; x < W; ++x) U[2 * ((size_t)x * W + x)] = 1.0;
            for (const MGate &g : wg) {
                const int tp = pos(g.t), cp = g.c >= 0 ? pos(g.c) : -1;
                for (int col = 0; col < W; ++col)
                    for (int x = 0; x < W; ++x) {
                        if ((x >> tp) & 1) continue;
                        if (cp >= 0 && !((x >> cp) & 1)) continue;
                        const int y = x | (1 << tp);
                        double *a = &U[2 * ((size_t)x * W + col)], *b = &U[2 * ((size_t)y * W + col)];
                        const double ar = a[0], ai = a[1], br = b[0], bi = b[1];
                        a[0] = g.u[0] * ar - g.u[1] * ai + g.u[2] * br - g.u[3] * bi;
                        a[1] = g.u[0] * ai + g.u[1] * ar + g.u[2] * bi + g.u[3] * br;
                        b[0] = g.u[4] * ar - g.u[5] * ai + g.u[6] * br - g.u[7] * bi;
                        b[1] = g.u[4] * ai + g.u[5] * ar + g.u[6] * bi + g.u[7] * br;
                    }
            }
            // real form: M'[2 jo + co][2 ji + ci]; A-operand order of the
            // 16x16x4 MFMA: [tile][step][lane] = M'[16 t + lane % 16][4 s + lane / 16]
            const int D = 2 * W, steps = D / 4, tiles = D / 16;
            auto mreal = [&](int R, int C) {
                const double ur = U[2 * ((size_t)(R >> 1) * W + (C >> 1))];
                const double ui = U[2 * ((size_t)(R >> 1) * W + (C >> 1)) + 1];
                if ((R & 1) == 0) return (C & 1) ? -ui : ur;
                return (C & 1) ? ur : ui;
            };
            std::vector<double> md((size_t)tiles * steps * 64);
            for (int t = 0; t < tiles; ++t)
                for (int st = 0; st < steps; ++st)
                    for (int lane = 0; lane < 64; ++lane)
                        md[((size_t)t * steps + st) * 64 + lane] = mreal(16 * t + lane % 16, 4 * st + lane / 16);
            K2Op op{};
            op.kind = K2_MFMA;
            if (cfg.dtype == 0) {
                std::vector<float> mf(md.begin(), md.end());
                op.a = table_put(mf.data(), mf.size() * sizeof(float));
            } else {
                op.a = table_put(md.data(), md.size() * sizeof(double));
            }
            op.b = K;
            int packed = 0;
            uint64_t mask = 0;
            for (int i = 0; i < K; ++i) {
                packed |= wl[i] << (5 * i);
                mask |= 1ull << wl[i];
            }
            op.c = packed;
            op.m0 = mask;
            plan.ops.push_back(op);
            plan.stats.fused += (int64_t)wg.size();
        };
        int hscale = 0;  // unnormalized Hadamards applied in this pass
        const int begin = (int)plan.ops.size();
        for (size_t i = 0; i < items.size(); ++i) {
            if (items[i].window) {
                flush_diag();
                emit_mfma(items[i].gates, items[i].bits);
                continue;
            }
            const MGate &g = items[i].gates[0];
            if (g.cls == GC_DIAG) {
                pending.push_back(g);
                continue;
            }
            const int lt = rank[g.t];
            if (slot_of(lt) < 0) {
                // new register set: this target, then the next distinct
                // non-diagonal targets of the run, then current slots. The
                // re-layout is placed before the pending diagonal run (pure
                // data movement commutes with it), so the run sees this
                // target as a register slot.
                std::vector<int> nrb{lt};
                for (size_t k = i + 1; k < items.size() && (int)nrb.size() < r; ++k) {
                    if (items[k].window) continue;  // windows need no register slots
                    const MGate &y = items[k].gates[0];
                    if (y.cls == GC_DIAG) continue;
                    const int x = rank[y.t];
                    if (std::find(nrb.begin(), nrb.end(), x) == nrb.end()) nrb.push_back(x);
                }
                for (int j = 0; j < r && (int)nrb.size() < r; ++j)
                    if (std::find(nrb.begin(), nrb.end(), rb[j]) == nrb.end()) nrb.push_back(rb[j]);
                for (int x = l - 1; x >= 0 && (int)nrb.size() < r; --x)
                    if (std::find(nrb.begin(), nrb.end(), x) == nrb.end()) nrb.push_back(x);
                emit_layout(nrb);
            }
            flush_diag();
            K2Op op{};
            op.kind = g.op == OP_H ? K2_H : (g.cls == GC_PERM ? K2_X : K2_DENSE);
            op.a = slot_of(lt);
            if (g.c < 0) {
                op.b = CK_NONE;
                if (combine && op.kind == K2_H) {
                    op.kind = K2_HU;
                    ++hscale;
                }
            } else {
                const int lc = rank[g.c];
                const int sc = lc >= 0 ? slot_of(lc) : -1;
                if (sc >= 0) { op.b = CK_SLOT; op.c = sc; }
                else { op.b = CK_MEM; op.c = code_of(g.c); }
            }
            for (int k = 0; k < 8; ++k) op.v[k] = g.u[k];
            plan.ops.push_back(op);
        }
        flush_diag();
        if (hscale > 0) {
            K2Op op{};
            op.kind = K2_SCALE;
            op.v[0] = std::ldexp(1.0, -(hscale / 2)) * ((hscale & 1) ? 0.70710678118654752440 : 1.0);
            plan.ops.push_back(op);
        }
        emit_fixed(canon);
        Step s;
        s.kind = ST_K2;
        s.l = l;
        s.logr = r;
        s.half_lds = half ? 1 : 0;
        for (int i = 0; i < l; ++i) s.bits[i] = B[i];
        s.op_begin = begin;
        s.op_count = (int)plan.ops.size() - begin;
        s.ngates = (int)q.size();
        if (!ptab.empty()) {
            s.tab_off = table_put(ptab.data(), ptab.size() * sizeof(double));
            s.tab_count = (int)(ptab.size() / 2);
        }
        if (!ugroups.empty()) {
            s.ut_off = table_put(uterms.data(), uterms.size() * sizeof(UTerm));
            s.nut = (int)uterms.size();
            s.ug_off = table_put(ugroups.data(), ugroups.size() * sizeof(UGroup));
            s.nug = (int)ugroups.size();
        }
        plan.steps.push_back(s);
        plan.stats.phases += 1;
        plan.stats.passes += 1;
        plan.stats.bytes += 2.0 * state_bytes;
        return split_ok;
    }
};

// Partitioned schedule over the gate dependence graph (virtual remap only).
//
// Circuit SWAPs are relabels, so they are taken out first: every later gate
// is renamed onto the memory bits the SWAPs leave its qubits on. Two of the
// remaining gates are ordered only when they share a qubit on which at least
// one of them is not diagonal (a control and a diagonal gate act diagonally
// on their qubits); gates that are diagonal on every qubit they share
// commute, so any order the graph allows gives the same state up to
// rounding. Deferral then works on the graph instead of the list: every
// ready gate whose target is local (or that needs no local target) joins the
// current block pass, lowest circuit index first, and when only gates with
// a global target are ready the pass is flushed and the next block's local
// qubits are chosen by look-ahead: starting from the pinned bits, the target
// of the ready gate with the longest chain of dependent local-target gates
// is added, everything that the bits chosen so far let run is run on a copy
// of the graph, and this repeats until the block is full.
std::string schedule_graph(const PlanConfig &cfg, const RawGate *gates, size_t m, int l, int pin, Plan &plan, std::vector<int> &l2p, std::vector<int> &slot_mem,
                           std::vector<int> &mem_slot, std::vector<MGate> &queue,
                           const std::function<void()> &flush)
{
    std::vector<MGate> G;
    G.reserve(m);
    for (size_t i = 0; i < m; ++i) {
        const RawGate &x = gates[i];
        if (x.op == OP_SWAP) {
            std::swap(l2p[x.target], l2p[x.target2]);
            continue;
        }
        MGate g;
        g.op = x.op;
        gate_matrix(x.op, x.theta, x.u, g.u, &g.cls);
        g.t = l2p[x.target];
        g.c = x.control >= 0 ? l2p[x.control] : -1;
        diag_angles(x, g);
        G.push_back(g);
    }
    const int M = (int)G.size();
    std::vector<int> indeg(M, 0), prio(M, 0);
    std::vector<std::vector<int>> succ(M);
    std::vector<char> blocking(M);
    {
        std::vector<int> last_nd(64, -1);
        std::vector<std::vector<int>> diag_since(64);
        auto edge = [&](int a, int c) {
            succ[a].push_back(c);
            ++indeg[c];
        };
        for (int i = 0; i < M; ++i) {
            const MGate &g = G[i];
            blocking[i] = !(cfg.diag_free && g.cls == GC_DIAG);
            const int qs[2] = {g.t, g.c};
            const bool nd[2] = {g.cls != GC_DIAG, false};
            for (int k = 0; k < 2; ++k) {
                const int q = qs[k];
                if (q < 0) continue;
                if (last_nd[q] >= 0) edge(last_nd[q], i);
                if (nd[k]) {
                    for (int d : diag_since[q]) edge(d, i);
                    diag_since[q].clear();
                    last_nd[q] = i;
                } else {
                    diag_since[q].push_back(i);
                }
            }
        }
    }
    // longest chain of local-target gates starting at each gate
    for (int i = M - 1; i >= 0; --i) {
        int best = 0;
        for (int s : succ[i]) best = std::max(best, prio[s]);
        prio[i] = best + blocking[i];
    }
    auto runnable = [&](int i, const std::vector<char> &local) { return !blocking[i] || local[G[i].t]; };

    // look-ahead choice of the next block's free local bits from the ready set
    auto choose = [&](const std::vector<int> &ready) {
        std::vector<char> in(64, 0);
        for (int p = 0; p < pin; ++p) in[p] = 1;
        std::vector<int> want, work = ready, held, undo;
        for (;;) {
            while (!work.empty()) {
                const int i = work.back();
                work.pop_back();
                if (!runnable(i, in)) {
                    held.push_back(i);
                    continue;
                }
                for (int s : succ[i]) {
                    undo.push_back(s);
                    if (--indeg[s] == 0) work.push_back(s);
                }
            }
            if (held.empty() || pin + (int)want.size() >= l) break;
            int best = -1;
            for (int i : held)
                if (best < 0 || prio[i] > prio[best] || (prio[i] == prio[best] && i < best)) best = i;
            in[G[best].t] = 1;
            want.push_back(G[best].t);
            work.swap(held);
        }
        for (int s : undo) ++indeg[s];
        return want;
    };
    // gather the chosen bits, keeping the pinned bits and, in the places left,
    // the bits already local; new bits take the freed slots in slot order
    auto gather = [&](const std::vector<int> &want) {
        std::vector<char> keep(64, 0);
        int kept = 0;
        for (int p = 0; p < pin; ++p) keep[p] = 1, ++kept;
        for (int p : want) keep[p] = 1, ++kept;
        for (int v = 0; v < l && kept < l; ++v)
            if (!keep[slot_mem[v]]) keep[slot_mem[v]] = 1, ++kept;
        std::vector<int> incoming;
        for (int p : want)
            if (mem_slot[p] < 0) incoming.push_back(p);
        size_t next = 0;
        for (int v = 0; v < l && next < incoming.size(); ++v) {
            if (keep[slot_mem[v]]) continue;
            mem_slot[slot_mem[v]] = -1;
            slot_mem[v] = incoming[next++];
            mem_slot[slot_mem[v]] = v;
            plan.stats.swaps += 1;
        }
        std::vector<char> local(64, 0);
        for (int v = 0; v < l; ++v) local[slot_mem[v]] = 1;
        return local;
    };

    std::priority_queue<int, std::vector<int>, std::greater<int>> ready;
    std::vector<int> held;
    for (int i = 0; i < M; ++i)
        if (indeg[i] == 0) held.push_back(i);
    // the first block costs nothing to choose either
    std::vector<char> local = gather(choose(held));
    for (;;) {
        for (int i : held) ready.push(i);
        held.clear();
        while (!ready.empty()) {
            const int i = ready.top();
            ready.pop();
            if (!runnable(i, local)) {
                held.push_back(i);
                continue;
            }
            queue.push_back(G[i]);
            plan.stats.gates += 1;
            for (int s : succ[i])
                if (--indeg[s] == 0) ready.push(s);
        }
        if (held.empty()) break;
        flush();
        local = gather(choose(held));
    }
    flush();
    plan.l2p_after = l2p;
    return "";
}

}  // namespace

std::string make_plan(const PlanConfig &cfg, const RawGate *gates, size_t m,
                      const std::vector<int> &l2p_in, Plan &plan)
{
    plan = Plan();
    const int n = cfg.n;
    if (n < 1 || n > 40) return "n out of range";
    if ((int)l2p_in.size() != n) return "layout size mismatch";
    std::string err = validate(n, gates, m);
    if (!err.empty()) return err;
    Builder b(cfg, plan);
    std::vector<int> l2p = l2p_in, p2l(n);
    for (int q = 0; q < n; ++q) p2l[l2p[q]] = q;

    auto to_mgate = [&](const RawGate &x, MGate &g) {
        g.op = x.op;
        gate_matrix(x.op, x.theta, x.u, g.u, &g.cls);
        g.t = l2p[x.target];
        g.c = x.control >= 0 ? l2p[x.control] : -1;
        diag_angles(x, g);
    };
    auto relabel = [&](int a, int bq) {
        const int pa = l2p[a], pb = l2p[bq];
        l2p[a] = pb; l2p[bq] = pa;
        p2l[pb] = a; p2l[pa] = bq;
    };

    int l = cfg.l > 0 ? cfg.l : default_block_qubits(cfg.dtype);
    if (l > n) l = n;
    const bool partitioned = cfg.mode == 1;
    if (!partitioned) {
        for (size_t i = 0; i < m; ++i) {
            if (gates[i].op == 9) { relabel(gates[i].target, gates[i].target2); continue; }
            MGate g;
            to_mgate(gates[i], g);
            b.add_k1(g);
            plan.stats.gates += 1;
        }
        plan.l2p_after = l2p;
        plan.l = n;
        return "";
    }
    if (l > max_block_qubits(cfg.dtype)) return "block_qubits above the on-chip maximum";
    b.l = l;
    b.logr = std::min(cfg.logr > 0 ? cfg.logr : default_reg_qubits(cfg.dtype), l);
    if (l - b.logr > 10) b.logr = l - 10;  // at most 1024 threads per block
    plan.l = l;
    const bool explicit_remap = cfg.remap == 1;
    int pin = 0;
    if (!explicit_remap) {
        pin = cfg.pin_low >= 0 ? cfg.pin_low : default_pin_qubits(cfg.dtype);
        pin = std::min(pin, l - 1);
        if (pin < 0) pin = 0;
    }

    // slots 0..l-1; slot v holds memory bit slot_mem[v]
    std::vector<int> slot_mem(l), mem_slot(64, -1);
    std::vector<int64_t> last_use(l, -1);
    for (int v = 0; v < l; ++v) { slot_mem[v] = v; mem_slot[v] = v; }
    std::vector<MGate> queue;
    std::vector<int> cls(m, 0);
    for (size_t i = 0; i < m; ++i) {
        double tmp[8];
        if (gates[i].op != 9) gate_matrix(gates[i].op, gates[i].theta, gates[i].u, tmp, &cls[i]);
    }
    auto needs_local = [&](size_t i) { return !(cfg.diag_free && cls[i] == GC_DIAG); };

    auto flush = [&]() {
        if (queue.empty()) return;
        std::vector<int> B(slot_mem.begin(), slot_mem.end());
        std::sort(B.begin(), B.end());
        b.compile_block(queue, B);
        queue.clear();
    };

    if (cfg.policy == 2) {
        if (explicit_remap) return "the dependence-graph schedule needs virtual remap";
        return schedule_graph(cfg, gates, m, l, pin, plan, l2p, slot_mem, mem_slot, queue, flush);
    }

    // next time (gate index > i) the data now at memory bit p is the target of
    // a gate that needs it local; circuit SWAPs rename it on the way
    auto next_use = [&](size_t i, int p) -> int64_t {
        int name = p2l[p];
        for (size_t k = i + 1; k < m; ++k) {
            const RawGate &x = gates[k];
            if (x.op == 9) {
                if (name == x.target) name = x.target2;
                else if (name == x.target2) name = x.target;
                continue;
            }
            if (x.target == name && needs_local(k)) return (int64_t)k;
        }
        return std::numeric_limits<int64_t>::max();
    };

    // Bulk remap (virtual remap + look-ahead): when a flush is forced, the
    // next block gathers the pinned bits plus the memory bits that the
    // upcoming gates target first, so one pass serves as many targets as
    // fit. No data moves, so replacing many local qubits costs nothing.
    const bool bulk = !explicit_remap && cfg.policy == 1;
    auto bulk_remap = [&](size_t i) {
        std::vector<int> want;
        std::vector<int> l2p_f = l2p;
        std::vector<bool> chosen(64, false);
        for (int p = 0; p < pin; ++p) chosen[p] = true;
        for (size_t k = i; k < m && (int)want.size() < l - pin; ++k) {
            const RawGate &y = gates[k];
            if (y.op == 9) {
                std::swap(l2p_f[y.target], l2p_f[y.target2]);
                continue;
            }
            if (!needs_local(k)) continue;
            const int p = l2p_f[y.target];
            if (!chosen[p]) { chosen[p] = true; want.push_back(p); }
        }
        // keep current local bits in the remaining places
        for (int v = 0; v < l && (int)want.size() < l - pin; ++v)
            if (!chosen[slot_mem[v]]) { chosen[slot_mem[v]] = true; want.push_back(slot_mem[v]); }
        std::vector<bool> keep(64, false);
        for (int p : want) keep[p] = true;
        for (int p = 0; p < pin; ++p) keep[p] = true;
        // slots whose bit is not kept receive the new bits, in slot order
        std::vector<int> incoming;
        for (int p : want)
            if (mem_slot[p] < 0) incoming.push_back(p);
        size_t next = 0;
        for (int v = 0; v < l && next < incoming.size(); ++v) {
            if (keep[slot_mem[v]]) continue;
            mem_slot[slot_mem[v]] = -1;
            slot_mem[v] = incoming[next++];
            mem_slot[slot_mem[v]] = v;
            last_use[v] = (int64_t)i;
            plan.stats.swaps += 1;
        }
    };

    for (size_t i = 0; i < m; ++i) {
        const RawGate &x = gates[i];
        if (x.op == 9) { relabel(x.target, x.target2); continue; }
        MGate g;
        to_mgate(x, g);
        if (bulk && needs_local(i) && mem_slot[g.t] < 0) {
            flush();
            bulk_remap(i);
        } else if (needs_local(i) && mem_slot[g.t] < 0) {
            flush();
            int victim = -1;
            int64_t best_key = 0, best_lru = 0;
            for (int v = 0; v < l; ++v) {
                if (slot_mem[v] < pin) continue;
                int64_t key = cfg.policy == 1 ? -next_use(i, slot_mem[v]) : 0;
                if (victim < 0 || key < best_key || (key == best_key && last_use[v] < best_lru)) {
                    victim = v;
                    best_key = key;
                    best_lru = last_use[v];
                }
            }
            if (victim < 0) return "no local slot can be evicted (block too small)";
            plan.stats.swaps += 1;
            if (explicit_remap) {
                // exchange memory bits g.t and victim (slot v == memory bit v)
                const int pv = victim, pt = g.t;
                Step s;
                s.kind = ST_K3;
                s.p = pt;
                s.v = pv;
                plan.steps.push_back(s);
                plan.stats.passes += 1;
                plan.stats.bytes += 2.0 * b.state_bytes * (pv < b.sbits ? 1.0 : 0.5);
                const int qa = p2l[pt], qb = p2l[pv];
                l2p[qa] = pv; l2p[qb] = pt;
                p2l[pv] = qa; p2l[pt] = qb;
                to_mgate(x, g);
            } else {
                mem_slot[slot_mem[victim]] = -1;
                slot_mem[victim] = g.t;
                mem_slot[g.t] = victim;
            }
            last_use[victim] = (int64_t)i;
        }
        queue.push_back(g);
        plan.stats.gates += 1;
        if (mem_slot[g.t] >= 0) last_use[mem_slot[g.t]] = (int64_t)i;
    }
    flush();
    plan.l2p_after = l2p;
    return "";
}

}  // namespace svp
