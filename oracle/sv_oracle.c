/*
 * FP64 CPU oracle for the state-vector gate-application path.
 *
 * TEST INFRASTRUCTURE ONLY. It is called by the tests, by the smoke check and
 * by the CPU-baseline leg of the benchmark; the simulator library never links,
 * loads or calls it, and it shares no code, header or table with it.
 *
 * What it computes (paper: "Accelerating State-Vector Quantum Simulation on
 * Integrated GPUs via Cache Locality Optimization", arXiv 2605.15098):
 *   - Section III-A, Algorithm 1 (single-qubit gate application): for every i
 *     stepping by 2^(t+1) and every j in [i, i+2^t), with a = S[j] and
 *     b = S[j+2^t], write S[j] = U11 a + U12 b and S[j+2^t] = U21 a + U22 b.
 *   - Section III-A, controlled gates: iteration j runs only when bit c of j
 *     is 1.
 *   - Section III-B (dividing the quantum state), applied literally in
 *     or_apply_partitioned: local qubits 0..l-1, a SWAP of a global target into
 *     the least-recently-used local position, the logical-to-physical map,
 *     deferred local gates flushed block by block, and global controls decided
 *     by the block index.
 * Conventions (readings of the paper, listed with the design notes): qubit q
 * is index bit q (little-endian, the bit order Algorithm 1 uses); U is indexed
 * row = output, column = input; all arithmetic is binary64 with explicit real
 * and imaginary parts and no contraction into FMA (built with
 * -ffp-contract=off).
 *
 * State arrays are 2^n interleaved (re, im) doubles in logical order.
 *
 * Built with -DOR_FLOAT the same source keeps the state in binary32 (gate
 * matrices still formed in binary64, rounded once): that build exists only to
 * time the method at the precision of the complex64 GPU path (the paper ran
 * single precision throughout); it is never used as a reference.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef OR_FLOAT
typedef float or_real;
#else
typedef double or_real;
#endif

/* Gate kinds, numbered as in the gate records the workload generator writes. */
enum { OR_H = 0, OR_X, OR_Y, OR_Z, OR_RX, OR_RY, OR_RZ, OR_P, OR_U2, OR_SWAP };

/* Planted-mistake switch for the mutation tests (tests/test_oracle_pins.py):
 * a build with -DOR_MUTANT=k must be caught by the pins. 0 = correct. */
#ifndef OR_MUTANT
#define OR_MUTANT 0
#endif

/* Build the 2x2 matrix of one gate in binary64, row-major (re, im) pairs.
 * Definitions: H = [[1,1],[1,-1]]/sqrt(2); X, Y, Z the Pauli matrices;
 * RX/RY/RZ(theta) = exp(-i theta sigma/2); P(theta) = diag(1, e^{i theta})
 * (the phase gate of Eq. 2). Returns 0, or -1 for an unknown kind. */
int or_gate_matrix(int op, double theta, const double *u_in, double *u)
{
    const double s = 1.0 / sqrt(2.0);
    const double c2 = cos(0.5 * theta), s2 = sin(0.5 * theta);
    memset(u, 0, 8 * sizeof(double));
    switch (op) {
    case OR_H: u[0] = s; u[2] = s; u[4] = s; u[6] = -s; break;
    case OR_X: u[2] = 1.0; u[4] = 1.0; break;
    case OR_Y: u[3] = -1.0; u[5] = 1.0; break;
    case OR_Z: u[0] = 1.0; u[6] = -1.0; break;
    case OR_RX: u[0] = c2; u[3] = -s2; u[5] = -s2; u[6] = c2; break;
    case OR_RY: u[0] = c2; u[2] = -s2; u[4] = s2; u[6] = c2; break;
    case OR_RZ: u[0] = c2; u[1] = -s2; u[6] = c2; u[7] = s2; break;
    case OR_P: u[0] = 1.0; u[6] = cos(theta); u[7] = sin(theta); break;
    case OR_U2: memcpy(u, u_in, 8 * sizeof(double)); break;
    default: return -1;
    }
#if OR_MUTANT == 1
    { double t0 = u[2], t1 = u[3]; u[2] = u[4]; u[3] = u[5]; u[4] = t0; u[5] = t1; } /* transposed U */
#elif OR_MUTANT == 2
    if (op == OR_RZ) { u[1] = -u[1]; u[7] = -u[7]; } /* wrong rotation sign */
#elif OR_MUTANT == 3
    if (op == OR_H) u[6] = s; /* wrong sign in H */
#endif
    return 0;
}

/* One Algorithm-1 iteration body on the pair (j, j + 2^t). */
static inline void pair_update(or_real *S, uint64_t j, uint64_t h, const or_real *u)
{
    const or_real ar = S[2 * j], ai = S[2 * j + 1];
    const or_real br = S[2 * (j + h)], bi = S[2 * (j + h) + 1];
    /* S[j] = U11 a + U12 b ; S[j+h] = U21 a + U22 b */
    const or_real r0 = (u[0] * ar - u[1] * ai) + (u[2] * br - u[3] * bi);
    const or_real i0 = (u[0] * ai + u[1] * ar) + (u[2] * bi + u[3] * br);
#if OR_MUTANT == 4
    const or_real r1 = (u[4] * ar - u[5] * ai) + (u[6] * br + u[7] * bi); /* dropped conj sign */
#else
    const or_real r1 = (u[4] * ar - u[5] * ai) + (u[6] * br - u[7] * bi);
#endif
    const or_real i1 = (u[4] * ai + u[5] * ar) + (u[6] * bi + u[7] * br);
    S[2 * j] = r0; S[2 * j + 1] = i0;
    S[2 * (j + h)] = r1; S[2 * (j + h) + 1] = i1;
}

/* Algorithm 1 with the optional control predicate, on a state of 2^n
 * amplitudes. The pair index p enumerates exactly the (i, j) iterations of
 * the two loops (j = i + low part, i = high part shifted past bit t); the
 * iterations are independent, so they are distributed over threads. */
static void apply_alg1(or_real *S, int n, int t, int c, const or_real *u)
{
    const uint64_t h = 1ull << t;
    const int64_t npairs = (int64_t)(1ull << (n - 1));
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t p = 0; p < npairs; ++p) {
        const uint64_t lo = (uint64_t)p & (h - 1);
        const uint64_t i = ((uint64_t)p >> t) << (t + 1);
        const uint64_t j = i + lo;
#if OR_MUTANT == 5
        (void)c;
#else
        if (c >= 0 && !((j >> c) & 1ull)) continue;
#endif
        pair_update(S, j, h, u);
    }
}

/* SWAP of qubits a and b: exchange the amplitudes whose bits a and b differ. */
static void apply_swap(or_real *S, int n, int a, int b)
{
    const uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t x = 0; x < (int64_t)N; ++x) {
        const uint64_t i = (uint64_t)x;
        const uint64_t ba = (i >> a) & 1ull, bb = (i >> b) & 1ull;
        if (ba == 1 && bb == 0) {
            const uint64_t k = i ^ (1ull << a) ^ (1ull << b);
            or_real tr = S[2 * i], ti = S[2 * i + 1];
            S[2 * i] = S[2 * k]; S[2 * i + 1] = S[2 * k + 1];
            S[2 * k] = tr; S[2 * k + 1] = ti;
        }
    }
}

static int check_gate(int n, int op, int t, int c, int t2)
{
    if (op < 0 || op > OR_SWAP) return -1;
    if (t < 0 || t >= n) return -1;
    if (op == OR_SWAP) return (t2 >= 0 && t2 < n && t2 != t) ? 0 : -1;
    if (c >= n || c == t) return -1;
    return 0;
}

/* Apply m gates in order to S (2^n interleaved complex, modified in place).
 * Gate g is (op[g], tgt[g], ctl[g] (-1 none), tgt2[g] (SWAP), theta[g],
 * u[8g..8g+7] for OR_U2). Returns 0, or -1 on a malformed gate (nothing
 * after it is applied). */
int or_apply(int n, or_real *S, int m, const int *op, const int *tgt, const int *ctl,
             const int *tgt2, const double *theta, const double *u)
{
    double U[8];
    or_real Ur[8];
    if (n < 1 || n > 40) return -1;
    for (int g = 0; g < m; ++g) {
        if (check_gate(n, op[g], tgt[g], ctl[g], tgt2[g])) return -1;
        if (op[g] == OR_SWAP) { apply_swap(S, n, tgt[g], tgt2[g]); continue; }
        if (or_gate_matrix(op[g], theta[g], u + 8 * g, U)) return -1;
        for (int k = 0; k < 8; ++k) Ur[k] = (or_real)U[k];
        apply_alg1(S, n, tgt[g], ctl[g], Ur);
    }
    return 0;
}

/* |0...0> in S, written by the same static thread partition that the gate
 * loops use, so each page is first touched by the thread (and NUMA node)
 * that later sweeps it. */
void or_zero_state(int n, or_real *S)
{
    const int64_t N = (int64_t)(1ull << n);
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t i = 0; i < N; ++i) { S[2 * i] = 0; S[2 * i + 1] = 0; }
    S[0] = 1;
}

#ifndef OR_FLOAT
/* ---- General gates (a wider front end than the paper's single control) ----
 *
 * A k-qubit unitary U (2^k x 2^k, row-major (re, im) pairs, row = output)
 * on targets t[0..k-1], applied where every control bit c[0..nc-1] is 1:
 * for each index j whose target bits are 0 and whose control bits are 1,
 * the 2^k amplitudes a_x = S[j + sum_b x_b 2^t[b]] (x over 0 .. 2^k - 1, bit
 * b of x = qubit t[b]) become sum_y U[x][y] a_y. This is Algorithm 1's pair
 * update widened from 2 amplitudes to 2^k, with the control predicate over
 * several bits. Returns 0, or -1 for a malformed gate. */
int or_apply_kq(int n, or_real *S, int k, const int *t, int nc, const int *c, const double *U)
{
    if (n < 1 || n > 40 || k < 1 || k > 6 || nc < 0 || nc > 16 || k + nc > n) return -1;
    uint64_t tmask = 0, cmask = 0;
    for (int b = 0; b < k; ++b) {
        if (t[b] < 0 || t[b] >= n || ((tmask >> t[b]) & 1ull)) return -1;
        tmask |= 1ull << t[b];
    }
    for (int b = 0; b < nc; ++b) {
        if (c[b] < 0 || c[b] >= n || (((tmask | cmask) >> c[b]) & 1ull)) return -1;
        cmask |= 1ull << c[b];
    }
    const int K = 1 << k;
    const uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t ji = 0; ji < (int64_t)N; ++ji) {
        const uint64_t j = (uint64_t)ji;
        if ((j & tmask) != 0 || (j & cmask) != cmask) continue;
        double ar[64], ai[64];
        uint64_t idx[64];
        for (int x = 0; x < K; ++x) {
            uint64_t off = 0;
            for (int b = 0; b < k; ++b)
                if ((x >> b) & 1) off |= 1ull << t[b];
            idx[x] = j | off;
            ar[x] = S[2 * idx[x]];
            ai[x] = S[2 * idx[x] + 1];
        }
        for (int x = 0; x < K; ++x) {
            double re = 0.0, im = 0.0;
            for (int y = 0; y < K; ++y) {
                const double ur = U[2 * (x * K + y)], ui = U[2 * (x * K + y) + 1];
                re += ur * ar[y] - ui * ai[y];
                im += ur * ai[y] + ui * ar[y];
            }
            S[2 * idx[x]] = (or_real)re;
            S[2 * idx[x] + 1] = (or_real)im;
        }
    }
    return 0;
}

/* |S_i|^2 in binary64. */
void or_probabilities(int n, const double *S, double *P)
{
    const int64_t N = (int64_t)(1ull << n);
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t i = 0; i < N; ++i) P[i] = S[2 * i] * S[2 * i] + S[2 * i + 1] * S[2 * i + 1];
}

/* Marginal probability over the listed qubits: out[m] = sum of |S_i|^2 over
 * all i whose bits qubits[0..nq-1] spell m (qubits[k] is bit k of m).
 * Serial summation in index order, so the result is deterministic. */
void or_marginal(int n, const double *S, int nq, const int *qubits, double *out)
{
    const uint64_t N = 1ull << n, M = 1ull << nq;
    memset(out, 0, M * sizeof(double));
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t m = 0;
        for (int k = 0; k < nq; ++k) m |= ((i >> qubits[k]) & 1ull) << k;
        out[m] += S[2 * i] * S[2 * i] + S[2 * i + 1] * S[2 * i + 1];
    }
}

/* Index of the largest entry; the lowest index wins ties. */
int64_t or_argmax(int64_t len, const double *P)
{
    int64_t best = 0;
    for (int64_t i = 1; i < len; ++i)
        if (P[i] > P[best]) best = i;
    return best;
}

/* ---- Section III-B, applied literally ------------------------------------ */

typedef struct { double u[8]; int pt; int pc; } or_queued;

/* Flush the deferred queue: every queued gate runs on block 0, then on block 1,
 * and so on; inside a block the queue order is kept. A control at a physical
 * position >= l is decided by the block index. */
static void flush(double *S, int n, int l, or_queued *q, int nq)
{
    if (nq == 0) return;
    const int64_t nblocks = (int64_t)(1ull << (n - l));
    const uint64_t bsize = 1ull << l;
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t b = 0; b < nblocks; ++b) {
        double *blk = S + 2 * (uint64_t)b * bsize;
        for (int k = 0; k < nq; ++k) {
            const int t = q[k].pt, c = q[k].pc;
            if (c >= l && !(((uint64_t)b >> (c - l)) & 1ull)) continue; /* block-index control */
            const uint64_t h = 1ull << t;
            for (uint64_t i = 0; i < bsize; i += 2 * h)
                for (uint64_t j = i; j < i + h; ++j) {
                    if (c >= 0 && c < l && !((j >> c) & 1ull)) continue;
                    pair_update(blk, j, h, q[k].u);
                }
        }
    }
}

/* Apply the circuit with the paper's partitioning: blocks of 2^l amplitudes.
 * Readings of points the paper leaves open (all amplitudes are unaffected by
 * them; only the counts are):
 *   - a local slot is "used" when its qubit is a gate's target or is swapped in;
 *     every slot starts as never used (-1); the least recently used slot is the
 *     victim, the lowest slot winning ties;
 *   - the queue is flushed before the SWAP, and the triggering gate starts the
 *     next queue; a final flush ends the circuit;
 *   - a SWAP gate of the circuit itself only relabels the map.
 * On return S is in logical order (the final map is undone), l2p_out[q] holds
 * the physical position of qubit q before that, and *swaps / *phases count the
 * state SWAPs and the non-empty flushes. */
int or_apply_partitioned(int n, int l, double *S, int m, const int *op, const int *tgt,
                         const int *ctl, const int *tgt2, const double *theta, const double *u,
                         int *l2p_out, int64_t *swaps, int64_t *phases)
{
    int l2p[64], p2l[64];
    int64_t last_use[64];
    if (n < 1 || n > 40 || l < 1 || l > n) return -1;
    for (int q = 0; q < n; ++q) { l2p[q] = q; p2l[q] = q; }
    for (int s = 0; s < l; ++s) last_use[s] = -1;
    or_queued *queue = (or_queued *)malloc(sizeof(or_queued) * (size_t)(m > 0 ? m : 1));
    if (!queue) return -2;
    int nq = 0;
    *swaps = 0; *phases = 0;
    for (int g = 0; g < m; ++g) {
        if (check_gate(n, op[g], tgt[g], ctl[g], tgt2[g])) { free(queue); return -1; }
        if (op[g] == OR_SWAP) {
            const int a = tgt[g], b = tgt2[g];
            const int pa = l2p[a], pb = l2p[b];
            l2p[a] = pb; l2p[b] = pa; p2l[pb] = a; p2l[pa] = b;
            continue;
        }
        int pt = l2p[tgt[g]];
        if (pt >= l) {
            if (nq) { flush(S, n, l, queue, nq); ++*phases; nq = 0; }
            int v = 0;
            for (int s = 1; s < l; ++s)
                if (last_use[s] < last_use[v]) v = s;
            apply_swap(S, n, pt, v);
            ++*swaps;
            const int qa = p2l[pt], qb = p2l[v];
            l2p[qa] = v; l2p[qb] = pt; p2l[v] = qa; p2l[pt] = qb;
            last_use[v] = g;
            pt = v;
        }
        or_queued *e = &queue[nq++];
        if (or_gate_matrix(op[g], theta[g], u + 8 * g, e->u)) { free(queue); return -1; }
        e->pt = pt;
        e->pc = ctl[g] >= 0 ? l2p[ctl[g]] : -1;
        last_use[pt] = g;
    }
    if (nq) { flush(S, n, l, queue, nq); ++*phases; }
    free(queue);
    /* undo the map: logical index x lives at the physical index whose bit
     * l2p[q] equals bit q of x */
    const uint64_t N = 1ull << n;
    double *tmp = (double *)malloc(2 * N * sizeof(double));
    if (!tmp) return -2;
#pragma omp parallel for schedule(static) if (n >= 14)
    for (int64_t xi = 0; xi < (int64_t)N; ++xi) {
        const uint64_t x = (uint64_t)xi;
        uint64_t p = 0;
        for (int q = 0; q < n; ++q) p |= ((x >> q) & 1ull) << l2p[q];
        tmp[2 * x] = S[2 * p]; tmp[2 * x + 1] = S[2 * p + 1];
    }
    memcpy(S, tmp, 2 * N * sizeof(double));
    free(tmp);
    for (int q = 0; q < n; ++q) l2p_out[q] = l2p[q];
    return 0;
}

#endif /* !OR_FLOAT: readouts and the partitioned method are binary64 only */

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel loops (timing a one-thread reference). */
void or_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
