// Host-side sanitizer driver (test infrastructure): built with
// -fsanitize=address,undefined together with the planner, the emulator of the
// planner's device programs and the C oracle, it plans and emulates many
// circuits under every schedule option and runs the oracle's entry points,
// so an out-of-bounds access, use after free, leak or undefined operation in
// that host code fails the build's run.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2605_15098_amd/csrc/plan.h"

extern "C" int emu_apply(int n, int dtype, int mode, int l, int logr, int policy, int remap, int diag_free,
                         int pin_low, int fuse_k, const void *gates, size_t m, double *state_inout,
                         int64_t *counts_out);
extern "C" int or_apply(int n, double *S, int m, const int *op, const int *tgt, const int *ctl, const int *tgt2,
                        const double *theta, const double *u);
extern "C" int or_apply_partitioned(int n, int l, double *S, int m, const int *op, const int *tgt, const int *ctl,
                                    const int *tgt2, const double *theta, const double *u, int *l2p_out,
                                    int64_t *swaps, int64_t *phases);

using svp::RawGate;

static std::vector<RawGate> qpe(int n, double phi)
{
    std::vector<RawGate> g;
    auto add = [&](int op, int t, int c, double th, int t2 = -1) {
        RawGate r{};
        r.op = op; r.target = t; r.control = c; r.target2 = t2; r.theta = th;
        g.push_back(r);
    };
    const int t = n - 1;
    add(1, t, -1, 0);
    for (int q = 0; q < t; ++q) add(0, q, -1, 0);
    for (int j = 0; j < t; ++j) add(7, t, j, 2 * M_PI * std::fmod(std::ldexp(phi, j), 1.0));
    for (int q = 0; q < t / 2; ++q) add(9, q, -1, 0, t - 1 - q);
    for (int q = 0; q < t; ++q) {
        for (int p = 0; p < q; ++p) add(7, q, p, -2 * M_PI / std::ldexp(1.0, q - p + 1));
        add(0, q, -1, 0);
    }
    return g;
}

static std::vector<RawGate> random_circuit(int n, int depth, std::mt19937_64 &rng, bool u2)
{
    std::vector<RawGate> g;
    std::uniform_real_distribution<double> ang(0, 2 * M_PI);
    for (int i = 0; i < depth; ++i) {
        RawGate r{};
        r.op = (int)(rng() % (u2 ? 10 : 9));
        if (n == 1 && r.op == 9) r.op = 0;  // a SWAP needs two qubits
        r.target = (int)(rng() % n);
        r.control = -1;
        r.target2 = -1;
        if (r.op == 9) {
            do r.target2 = (int)(rng() % n); while (r.target2 == r.target);
        } else if (rng() % 2 && n > 1) {
            do r.control = (int)(rng() % n); while (r.control == r.target);
        }
        r.theta = ang(rng);
        if (r.op == 8) {  // a unitary: rotation composition
            const double a = ang(rng), b = ang(rng);
            r.u[0] = std::cos(a); r.u[1] = 0; r.u[2] = -std::sin(a) * std::cos(b); r.u[3] = -std::sin(a) * std::sin(b);
            r.u[4] = std::sin(a) * std::cos(b); r.u[5] = -std::sin(a) * std::sin(b); r.u[6] = std::cos(a); r.u[7] = 0;
        }
        g.push_back(r);
    }
    return g;
}

int main()
{
    std::mt19937_64 rng(12345);
    int plans = 0, emulated = 0;
    for (int n : {1, 2, 5, 9, 13, 16, 20, 24}) {
        std::vector<std::vector<RawGate>> circuits;
        if (n >= 2) circuits.push_back(qpe(n, 0.318));
        circuits.push_back(random_circuit(n, 120, rng, true));
        for (const auto &g : circuits)
            for (int dtype : {0, 1})
                for (int mode : {0, 1})
                    for (int policy : {0, 1, 2})
                        for (int remap : {0, 1})
                            for (int fuse : {0, 1, 4, 5})
                                for (int l : {0, 3, 8, 13}) {
                                    if (policy == 2 && remap == 1) continue;
                                    if (mode == 0 && (policy || remap || fuse != 1 || l)) continue;
                                    svp::PlanConfig c;
                                    c.n = n; c.dtype = dtype; c.mode = mode; c.l = l; c.policy = policy;
                                    c.remap = remap; c.diag_free = policy == 2; c.fuse_k = fuse;
                                    std::vector<int> l2p(n);
                                    for (int q = 0; q < n; ++q) l2p[q] = q;
                                    svp::Plan plan;
                                    const std::string err = svp::make_plan(c, g.data(), g.size(), l2p, plan);
                                    (void)err;
                                    ++plans;
                                }
        // emulate a few plans on small states and run the oracle
        if (n <= 13) {
            for (const auto &g : circuits) {
                const size_t N = size_t(1) << n;
                std::vector<double> S(2 * N, 0.0), O(2 * N, 0.0), P(2 * N, 0.0);
                S[0] = O[0] = P[0] = 1.0;
                int64_t counts[8] = {};
                for (int policy : {0, 2})
                    for (int fuse : {0, 1, 5}) {
                        std::vector<double> T = S;
                        if (emu_apply(n, 1, 1, std::min(n, 8), 0, policy, policy == 2 ? 0 : 1, policy == 2, -1, fuse,
                                      g.data(), g.size(), T.data(), counts) == 0)
                            ++emulated;
                    }
                std::vector<int> op, tg, ct, t2;
                std::vector<double> th, u;
                for (const RawGate &r : g) {
                    op.push_back(r.op); tg.push_back(r.target); ct.push_back(r.control); t2.push_back(r.target2);
                    th.push_back(r.theta);
                    u.insert(u.end(), r.u, r.u + 8);
                }
                if (or_apply(n, O.data(), (int)g.size(), op.data(), tg.data(), ct.data(), t2.data(), th.data(),
                             u.data()) != 0)
                    return 2;
                std::vector<int> l2p(64);
                int64_t sw = 0, ph = 0;
                if (or_apply_partitioned(n, std::max(1, n / 2), P.data(), (int)g.size(), op.data(), tg.data(),
                                         ct.data(), t2.data(), th.data(), u.data(), l2p.data(), &sw, &ph) != 0)
                    return 3;
                for (size_t i = 0; i < 2 * N; ++i)
                    if (O[i] != P[i]) return 4;  // the partitioned method is the plain method bit for bit
            }
        }
    }
    std::printf("sanitized run: %d plans, %d emulated programs\n", plans, emulated);
    return 0;
}
