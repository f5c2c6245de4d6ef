// C ABI of the simulator (include/sv.h): handles, validation, plan
// execution on a HIP stream, FP64 readouts. No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/sv.h"
#include "jit.h"
#include "launch.h"
#include "mlp.h"
#include "plan.h"
#include "qasm.h"

namespace {

thread_local std::string g_err;
std::mutex g_live_mu;
std::unordered_set<const void *> g_live;
int g_fault = 0;  // 1: next device allocation fails; 2: next launch fails

sv_status fail(sv_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

sv_status hip_fail(hipError_t e, const char *what)
{
    return fail(SV_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define SV_HIP(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

hipError_t dev_alloc(void **p, size_t bytes)
{
    if (g_fault == 1) {
        g_fault = 0;
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

bool launch_fault()
{
    if (g_fault == 2) {
        g_fault = 0;
        return true;
    }
    return false;
}

size_t amp_bytes(int dtype) { return dtype == SV_COMPLEX64 ? 8 : 16; }

}  // namespace

struct sv_handle_s {
    int n = 0;
    int dtype = 0;
    void *buf = nullptr;
    size_t bytes = 0;
    bool owns = false;
    hipStream_t stream = nullptr;
    std::vector<int> l2p;
    svp::K2Op *dops = nullptr;
    size_t dops_cap = 0;
    uint8_t *dtab = nullptr;
    size_t dtab_cap = 0;
    void *scratch = nullptr;
    size_t scratch_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    bool kernel_timing = false;
    std::vector<hipEvent_t> kev;   // pairs around each launch when kernel_timing
    std::vector<int> kev_kind;
    sv_stats st{};
};

namespace {

sv_status check_handle(sv_handle h)
{
    if (!h) return fail(SV_ERR_BAD_HANDLE, "null handle");
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!g_live.count(h)) return fail(SV_ERR_BAD_HANDLE, "handle is not live");
    return SV_OK;
}

sv_status ensure_scratch(sv_handle h, size_t bytes)
{
    if (bytes <= h->scratch_cap) return SV_OK;
    if (h->scratch) {
        hipStreamSynchronize(h->stream);
        hipFree(h->scratch);
        h->scratch = nullptr;
        h->scratch_cap = 0;
    }
    void *p = nullptr;
    if (dev_alloc(&p, bytes) != hipSuccess) return fail(SV_ERR_OUT_OF_MEMORY, "scratch allocation failed");
    h->scratch = p;
    h->scratch_cap = bytes;
    return SV_OK;
}

// true when p is device (or managed) memory
bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

bool identity(const std::vector<int> &l2p)
{
    for (size_t q = 0; q < l2p.size(); ++q)
        if (l2p[q] != (int)q) return false;
    return true;
}

sv_status new_handle(int n, sv_dtype dtype, sv_handle *out, sv_handle_s **hp)
{
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (n < 1 || n > 36) return fail(SV_ERR_INVALID_ARG, "n must be in [1, 36]");
    if (dtype != SV_COMPLEX64 && dtype != SV_COMPLEX128) return fail(SV_ERR_INVALID_ARG, "unknown dtype");
    sv_handle_s *h = new (std::nothrow) sv_handle_s();
    if (!h) return fail(SV_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->n = n;
    h->dtype = dtype;
    h->l2p.resize(n);
    for (int q = 0; q < n; ++q) h->l2p[q] = q;
    *hp = h;
    return SV_OK;
}

void free_handle(sv_handle_s *h)
{
    for (hipEvent_t e : h->kev) hipEventDestroy(e);
    if (h->ev0) hipEventDestroy(h->ev0);
    if (h->ev1) hipEventDestroy(h->ev1);
    if (h->dops) hipFree(h->dops);
    if (h->dtab) hipFree(h->dtab);
    if (h->scratch) hipFree(h->scratch);
    if (h->owns && h->buf) hipFree(h->buf);
    delete h;
}

sv_status finish_handle(sv_handle_s *h, sv_handle *out)
{
    hipError_t e = hipEventCreate(&h->ev0);
    if (e == hipSuccess) e = hipEventCreate(&h->ev1);
    if (e != hipSuccess) {
        free_handle(h);
        return hip_fail(e, "hipEventCreate");
    }
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(h);
    }
    *out = h;
    return SV_OK;
}

svp::PlanConfig config_from(sv_handle h, const sv_schedule *s)
{
    svp::PlanConfig c;
    c.n = h->n;
    c.dtype = h->dtype;
    if (!s) {
        c.mode = 1;
        c.l = 0;
        c.policy = SV_SWAP_GRAPH;
        c.remap = SV_REMAP_VIRTUAL;
        c.diag_free = 1;
        c.fuse_k = 1;
    } else {
        c.mode = s->mode;
        c.l = s->block_qubits;
        c.policy = s->swap_policy;
        c.remap = s->remap;
        c.diag_free = s->diag_free;
        c.fuse_k = s->fuse_k;
        if (s->reg_qubits > 0) c.logr = s->reg_qubits;
        if (s->pin_qubits > 0) c.pin_low = s->pin_qubits;
    }
    if (const char *e = std::getenv("SV_PIN_BITS")) c.pin_low = std::atoi(e);
    if (const char *e = std::getenv("SV_LOGR")) c.logr = std::atoi(e);
    if (const char *e = std::getenv("SV_HALF_LDS")) c.half_lds = std::atoi(e);
    return c;
}

sv_status check_schedule(const sv_schedule *s, int dtype)
{
    if (!s) return SV_OK;
    if (s->mode != SV_PLAIN && s->mode != SV_PARTITIONED) return fail(SV_ERR_INVALID_ARG, "unknown mode");
    if (s->block_qubits < 0) return fail(SV_ERR_INVALID_ARG, "block_qubits < 0");
    if (s->block_qubits > svp::max_block_qubits(dtype))
        return fail(SV_ERR_UNSUPPORTED, "block_qubits above the on-chip maximum for this dtype");
    if (s->swap_policy != SV_SWAP_LRU && s->swap_policy != SV_SWAP_LOOKAHEAD && s->swap_policy != SV_SWAP_GRAPH)
        return fail(SV_ERR_INVALID_ARG, "unknown swap policy");
    if (s->remap != SV_REMAP_VIRTUAL && s->remap != SV_REMAP_EXPLICIT)
        return fail(SV_ERR_INVALID_ARG, "unknown remap");
    if (s->swap_policy == SV_SWAP_GRAPH && s->remap != SV_REMAP_VIRTUAL && s->mode == SV_PARTITIONED)
        return fail(SV_ERR_UNSUPPORTED, "the dependence-graph schedule needs virtual remap");
    if (s->fuse_k < 0) return fail(SV_ERR_INVALID_ARG, "fuse_k < 0");
    if (s->fuse_k > 6) return fail(SV_ERR_UNSUPPORTED, "fuse_k above 6");
    if (s->fuse_k == 2 || s->fuse_k == 3 || s->fuse_k == 6)
        return fail(SV_ERR_UNSUPPORTED, "dense fusion windows have 4 or 5 qubits");
    if (s->fuse_k >= 4 && s->mode != SV_PARTITIONED)
        return fail(SV_ERR_UNSUPPORTED, "dense fusion runs inside block passes (partitioned mode)");
    if (s->outer_qubits < 0 || s->outer_qubits > 40) return fail(SV_ERR_INVALID_ARG, "outer_qubits out of range");
    if (s->outer_qubits > 0 && s->mode != SV_PARTITIONED)
        return fail(SV_ERR_UNSUPPORTED, "the outer tier chains block passes (partitioned mode)");
    if (s->tuner != SV_TUNER_NONE && s->tuner != SV_TUNER_EXHAUSTIVE && s->tuner != SV_TUNER_LEARNED)
        return fail(SV_ERR_INVALID_ARG, "unknown tuner");
    if (s->reg_qubits < 0) return fail(SV_ERR_INVALID_ARG, "reg_qubits < 0");
    if (s->pin_qubits < 0 || s->pin_qubits > 16) return fail(SV_ERR_INVALID_ARG, "pin_qubits out of range");
    if (s->reg_qubits > (dtype == SV_COMPLEX64 ? 5 : 4))
        return fail(SV_ERR_UNSUPPORTED, "reg_qubits above the register budget for this dtype");
    return SV_OK;
}

sv_status run_plan(sv_handle h, const svp::Plan &plan, int outer_qubits, bool record = true)
{
    const auto tu0 = std::chrono::steady_clock::now();
    if (!plan.ops.empty()) {
        const size_t need = plan.ops.size();
        if (need > h->dops_cap) {
            if (h->dops) {
                hipStreamSynchronize(h->stream);
                hipFree(h->dops);
                h->dops = nullptr;
                h->dops_cap = 0;
            }
            size_t cap = std::max<size_t>(need, 1024);
            void *p = nullptr;
            if (dev_alloc(&p, cap * sizeof(svp::K2Op)) != hipSuccess)
                return fail(SV_ERR_OUT_OF_MEMORY, "program buffer allocation failed");
            h->dops = (svp::K2Op *)p;
            h->dops_cap = cap;
        }
        SV_HIP(hipMemcpyAsync(h->dops, plan.ops.data(), need * sizeof(svp::K2Op), hipMemcpyHostToDevice,
                              h->stream),
               "program upload");
    }
    if (!plan.table.empty()) {
        const size_t need = plan.table.size();
        if (need > h->dtab_cap) {
            if (h->dtab) {
                hipStreamSynchronize(h->stream);
                hipFree(h->dtab);
                h->dtab = nullptr;
                h->dtab_cap = 0;
            }
            size_t cap = std::max<size_t>(need, 1 << 16);
            void *p = nullptr;
            if (dev_alloc(&p, cap) != hipSuccess) return fail(SV_ERR_OUT_OF_MEMORY, "table allocation failed");
            h->dtab = (uint8_t *)p;
            h->dtab_cap = cap;
        }
        SV_HIP(hipMemcpyAsync(h->dtab, plan.table.data(), need, hipMemcpyHostToDevice, h->stream), "table upload");
    }
    // Block passes run as kernels compiled for their op lists (cached), unless
    // SV_JIT=0 selects the op interpreter. Compilation happens before the
    // first event so device time covers only the kernels.
    const char *jenv = std::getenv("SV_JIT");
    const bool use_jit = !(jenv && jenv[0] == '0');
    const bool trace = std::getenv("SV_TRACE_HOST") != nullptr;
    const auto tp0 = std::chrono::steady_clock::now();
    if (trace)
        std::fprintf(stderr, "[sv] upload %.3f ms\n", std::chrono::duration<double, std::milli>(tp0 - tu0).count());
    std::vector<const void *> jit(plan.steps.size(), nullptr);
    if (use_jit) {
        std::string err;
        hipError_t e = svj::prepare_plan(plan, h->dtype, jit, &err);
        if (e != hipSuccess)
            return fail(SV_ERR_DEVICE, err.empty() ? std::string("pass compilation: ") + hipGetErrorString(e) : err);
    }
    const auto tp1 = std::chrono::steady_clock::now();
    h->kev_kind.clear();
    // One launch of block pass si over 2^nblk blocks: the bits of the block
    // number are `vary` (ascending), every block also carries base_or.
    auto launch_k2 = [&](size_t si, const std::vector<int> &vary, uint64_t base_or) -> hipError_t {
        const svp::Step &s = plan.steps[si];
        svk::K2Args a{};
        a.n = h->n;
        a.l = s.l;
        a.nops = s.op_count;
        a.nug = s.nug;
        a.ug_off = s.ug_off;
        a.tab_off = s.tab_off;
        a.tab_count = s.tab_count;
        a.ut_off = s.ut_off;
        a.nut = s.nut;
        a.table = h->dtab;
        a.vec2 = (s.l >= 2 && s.logr >= 2 && s.bits[0] == 0) ? 1 : 0;
        a.half_lds = s.half_lds;
        for (int i = 0; i < s.l; ++i) a.bits[i] = (int8_t)s.bits[i];
        for (size_t k = 0; k < vary.size(); ++k) a.nbits[k] = (int8_t)vary[k];
        a.nblk_bits = (int32_t)vary.size();
        a.base_or = base_or;
        if (jit[si]) return svj::launch(jit[si], h->buf, a, h->stream);
        bool mf = false;
        for (int i = 0; i < s.op_count && !mf; ++i) mf = plan.ops[s.op_begin + i].kind == svp::K2_MFMA;
        return svk::k2_pass(h->buf, h->n, h->dtype, s.logr, a, h->dops + s.op_begin, mf, h->stream);
    };
    auto local_mask = [&](const svp::Step &s) {
        uint64_t m = 0;
        for (int i = 0; i < s.l; ++i) m |= 1ull << s.bits[i];
        return m;
    };
    auto timed = [&](int kind, auto &&fn) -> sv_status {
        if (h->kernel_timing) {
            while (h->kev.size() < 2 * h->kev_kind.size() + 2) {
                hipEvent_t ev;
                SV_HIP(hipEventCreate(&ev), "hipEventCreate");
                h->kev.push_back(ev);
            }
            SV_HIP(hipEventRecord(h->kev[2 * h->kev_kind.size()], h->stream), "hipEventRecord");
        }
        if (launch_fault()) return fail(SV_ERR_DEVICE, "injected launch failure");
        hipError_t e = fn();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        if (h->kernel_timing) {
            SV_HIP(hipEventRecord(h->kev[2 * h->kev_kind.size() + 1], h->stream), "hipEventRecord");
            h->kev_kind.push_back(kind);
        }
        return SV_OK;
    };
    if (record) SV_HIP(hipEventRecord(h->ev0, h->stream), "hipEventRecord");
    for (size_t si = 0; si < plan.steps.size();) {
        const svp::Step &s = plan.steps[si];
        if (s.kind == svp::ST_K1) {
            if (sv_status st = timed(0, [&] { return svk::k1_gate(h->buf, h->n, h->dtype, s.g, h->stream); })) return st;
            ++si;
            continue;
        }
        if (s.kind == svp::ST_K3) {
            if (sv_status st = timed(2, [&] { return svk::k3_swap(h->buf, h->n, h->dtype, s.p, s.v, h->stream); }))
                return st;
            ++si;
            continue;
        }
        // Outer tier: consecutive block passes whose local bits together fit
        // in outer_qubits bits run outer block by outer block (2^outer_qubits
        // amplitudes), every pass of the chain on one outer block before the
        // next, so the later passes find the block in the Infinity Cache.
        uint64_t U = local_mask(s);
        size_t sj = si + 1;
        if (outer_qubits > 0)
            while (sj < plan.steps.size() && plan.steps[sj].kind == svp::ST_K2 &&
                   __builtin_popcountll(U | local_mask(plan.steps[sj])) <= outer_qubits) {
                U |= local_mask(plan.steps[sj]);
                ++sj;
            }
        if (sj - si < 2) {
            std::vector<int> vary;
            for (int p = 0; p < h->n; ++p)
                if (!((local_mask(s) >> p) & 1ull)) vary.push_back(p);
            if (sv_status st = timed(1, [&] { return launch_k2(si, vary, 0); })) return st;
            ++si;
            continue;
        }
        const int u = __builtin_popcountll(U);
        std::vector<int> rest;  // memory bits outside the outer block, ascending
        for (int p = 0; p < h->n; ++p)
            if (!((U >> p) & 1ull)) rest.push_back(p);
        // an outer block is 2^outer_qubits amplitudes: the chain's local bits
        // and the lowest c remaining bits; one launch per pass and outer block
        const int c = std::min((int)rest.size(), outer_qubits - u);
        const std::vector<int> chunk(rest.begin(), rest.begin() + c), high(rest.begin() + c, rest.end());
        const uint64_t nchunks = 1ull << high.size();
        for (uint64_t j = 0; j < nchunks; ++j) {
            uint64_t base_or = 0;
            for (size_t k = 0; k < high.size(); ++k)
                if ((j >> k) & 1ull) base_or |= 1ull << high[k];
            for (size_t sk = si; sk < sj; ++sk) {
                const uint64_t lm = local_mask(plan.steps[sk]);
                std::vector<int> vary;
                for (int p = 0; p < h->n; ++p)
                    if (((U >> p) & 1ull) && !((lm >> p) & 1ull)) vary.push_back(p);
                vary.insert(vary.end(), chunk.begin(), chunk.end());
                if (sv_status st = timed(1, [&] { return launch_k2(sk, vary, base_or); })) return st;
            }
        }
        si = sj;
    }
    if (record) {
        SV_HIP(hipEventRecord(h->ev1, h->stream), "hipEventRecord");
        h->timed = true;
    }
    if (trace) {
        const auto tp2 = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[sv] prepare %.3f ms, launch %.3f ms, %zu steps\n",
                     std::chrono::duration<double, std::milli>(tp1 - tp0).count(),
                     std::chrono::duration<double, std::milli>(tp2 - tp1).count(), plan.steps.size());
    }
    return SV_OK;
}

void fill_stats(sv_stats *o, const svp::PlanConfig &c, const svp::Plan &p)
{
    o->gates = p.stats.gates;
    o->swaps = p.stats.swaps;
    o->phases = p.stats.phases;
    o->passes = p.stats.passes;
    o->fused = p.stats.fused;
    o->bytes = p.stats.bytes;
    o->block_qubits = p.l;
    o->fuse_k = c.fuse_k;
    o->swap_policy = c.policy;
    o->mode = c.mode;
}

// complement of the physical bits in `q` among 0..n-1, ascending
std::vector<int> complement(int n, const std::vector<int> &q)
{
    std::vector<bool> in(n, false);
    for (int b : q) in[b] = true;
    std::vector<int> o;
    for (int p = 0; p < n; ++p)
        if (!in[p]) o.push_back(p);
    return o;
}

}  // namespace

extern "C" {

const char *sv_version(void) { return "svmi 0.1 (gfx950)"; }

const char *sv_last_error(void) { return g_err.c_str(); }

sv_status sv_stream_probe(void *dst, const void *src, size_t bytes, int mode, void *stream)
{
    if (!dst || (mode == 0 && !src)) return fail(SV_ERR_INVALID_ARG, "null buffer");
    if (mode != 0 && mode != 1) return fail(SV_ERR_INVALID_ARG, "mode must be 0 (copy) or 1 (in place)");
    if (bytes % 16 != 0 || ((uintptr_t)dst % 16) != 0 || (mode == 0 && ((uintptr_t)src % 16) != 0))
        return fail(SV_ERR_INVALID_ARG, "buffers and size must be 16-byte aligned");
    SV_HIP(svk::stream_probe(dst, src, bytes, mode, (hipStream_t)stream), "stream probe");
    return SV_OK;
}

sv_status sv_debug_inject_fault(int kind)
{
    if (kind < 0 || kind > 2) return fail(SV_ERR_INVALID_ARG, "unknown fault kind");
    g_fault = kind;
    return SV_OK;
}

sv_status sv_create(int n, sv_dtype dtype, sv_handle *out)
{
    sv_handle_s *h = nullptr;
    sv_status s = new_handle(n, dtype, out, &h);
    if (s) return s;
    h->bytes = amp_bytes(dtype) << n;
    h->owns = true;
    hipError_t e = dev_alloc(&h->buf, h->bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->buf = nullptr;
        free_handle(h);
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            return fail(SV_ERR_OUT_OF_MEMORY, "device allocation of the state failed");
        return hip_fail(e, "hipMalloc");
    }
    e = svk::init_zero_state(h->buf, n, dtype, h->stream);
    if (e != hipSuccess) {
        free_handle(h);
        return hip_fail(e, "init");
    }
    return finish_handle(h, out);
}

sv_status sv_wrap(int n, sv_dtype dtype, void *dev_buf, size_t bytes, void *hip_stream, sv_handle *out)
{
    sv_handle_s *h = nullptr;
    sv_status s = new_handle(n, dtype, out, &h);
    if (s) return s;
    if (!dev_buf) {
        delete h;
        return fail(SV_ERR_INVALID_ARG, "buffer is null");
    }
    if (bytes < (amp_bytes(dtype) << n)) {
        delete h;
        return fail(SV_ERR_INVALID_ARG, "buffer smaller than 2^n amplitudes");
    }
    h->buf = dev_buf;
    h->bytes = bytes;
    h->owns = false;
    h->stream = (hipStream_t)hip_stream;
    // the buffer holds the state in logical order: bring it to storage order
    hipError_t e = svk::to_storage_order(h->buf, n, dtype, h->stream);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "storage order");
    }
    return finish_handle(h, out);
}

sv_status sv_destroy(sv_handle h)
{
    if (!h) return SV_OK;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!g_live.erase(h)) return fail(SV_ERR_BAD_HANDLE, "handle is not live");
    }
    hipStreamSynchronize(h->stream);
    free_handle(h);
    return SV_OK;
}

sv_status sv_reset(sv_handle h)
{
    if (sv_status s = check_handle(h)) return s;
    for (int q = 0; q < h->n; ++q) h->l2p[q] = q;
    SV_HIP(svk::init_zero_state(h->buf, h->n, h->dtype, h->stream), "init");
    return SV_OK;
}

sv_status sv_set_stream(sv_handle h, void *hip_stream)
{
    if (sv_status s = check_handle(h)) return s;
    h->stream = (hipStream_t)hip_stream;
    return SV_OK;
}

sv_status sv_set_kernel_timing(sv_handle h, int on)
{
    if (sv_status s = check_handle(h)) return s;
    h->kernel_timing = on != 0;
    return SV_OK;
}

sv_status sv_layout(sv_handle h, int *l2p)
{
    if (sv_status s = check_handle(h)) return s;
    if (!l2p) return fail(SV_ERR_INVALID_ARG, "out is null");
    for (int q = 0; q < h->n; ++q) l2p[q] = h->l2p[q];
    return SV_OK;
}

sv_status sv_plan(int n, sv_dtype dtype, const sv_gate *gates, size_t m, const sv_schedule *s, sv_stats *out)
{
    if (n < 1 || n > 36) return fail(SV_ERR_INVALID_ARG, "n must be in [1, 36]");
    if (dtype != SV_COMPLEX64 && dtype != SV_COMPLEX128) return fail(SV_ERR_INVALID_ARG, "unknown dtype");
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    if (sv_status st = check_schedule(s, dtype)) return st;
    sv_handle_s tmp;
    tmp.n = n;
    tmp.dtype = dtype;
    svp::PlanConfig c = config_from(&tmp, s);
    std::vector<int> l2p(n);
    for (int q = 0; q < n; ++q) l2p[q] = q;
    svp::Plan plan;
    std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, l2p, plan);
    if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
    std::memset(out, 0, sizeof(*out));
    fill_stats(out, c, plan);
    return SV_OK;
}

sv_status sv_apply_circuit(sv_handle h, const sv_gate *gates, size_t m, const sv_schedule *s)
{
    if (sv_status st = check_handle(h)) return st;
    if (sv_status st = check_schedule(s, h->dtype)) return st;
    sv_schedule tuned;
    if (s && s->tuner != SV_TUNER_NONE) {
        if (sv_status st = sv_tune(h, gates, m, s->tuner, &tuned)) return st;
        s = &tuned;
    }
    const auto t0 = std::chrono::steady_clock::now();
    svp::PlanConfig c = config_from(h, s);
    svp::Plan plan;
    std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, h->l2p, plan);
    if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
    const auto t1 = std::chrono::steady_clock::now();
    if (sv_status st = run_plan(h, plan, s ? s->outer_qubits : 0)) return st;
    h->l2p = plan.l2p_after;
    std::memset(&h->st, 0, sizeof(h->st));
    fill_stats(&h->st, c, plan);
    h->st.plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return SV_OK;
}

static bool finite_all(const double *x, size_t k)
{
    for (size_t i = 0; i < k; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// An extended gate that sv_gate can express, as that record (else false).
static bool as_plain_gate(const sv_gate_ex &g, svp::RawGate &r)
{
    if (g.op == SV_UK) return false;
    if (g.op == SV_SWAP) {
        if (g.ncontrols != 0) return false;
        r = svp::RawGate{SV_SWAP, g.targets[0], -1, g.targets[1], 0.0, {0}};
        return true;
    }
    if (g.ncontrols > 1) return false;
    r = svp::RawGate{g.op, g.targets[0], g.ncontrols ? g.controls[0] : -1, -1, g.theta, {0}};
    std::memcpy(r.u, g.u, sizeof r.u);
    return true;
}

static sv_status check_gate_ex(const sv_gate_ex &g, int n, size_t i)
{
    const std::string at = " (gate " + std::to_string(i) + ")";
    if (g.op < SV_H || g.op > SV_UK) return fail(SV_ERR_INVALID_ARG, "unknown op" + at);
    const int want = g.op == SV_SWAP ? 2 : (g.op == SV_UK ? g.ntargets : 1);
    if (g.op == SV_UK && g.ntargets > SV_MAX_TARGETS) return fail(SV_ERR_UNSUPPORTED, "more than 6 targets" + at);
    if (g.ntargets != want || want < 1) return fail(SV_ERR_INVALID_ARG, "wrong number of targets" + at);
    if (g.ncontrols > SV_MAX_CONTROLS) return fail(SV_ERR_UNSUPPORTED, "more than 16 controls" + at);
    if (g.ncontrols < 0) return fail(SV_ERR_INVALID_ARG, "negative control count" + at);
    uint64_t seen = 0;
    for (int b = 0; b < g.ntargets + g.ncontrols; ++b) {
        const int q = b < g.ntargets ? g.targets[b] : g.controls[b - g.ntargets];
        if (q < 0 || q >= n || ((seen >> q) & 1ull)) return fail(SV_ERR_INVALID_ARG, "qubit out of range or repeated" + at);
        seen |= 1ull << q;
    }
    if (!std::isfinite(g.theta)) return fail(SV_ERR_INVALID_ARG, "non-finite angle" + at);
    if (g.op == SV_U2 && !finite_all(g.u, 8)) return fail(SV_ERR_INVALID_ARG, "non-finite matrix entry" + at);
    if (g.op == SV_UK) {
        if (!g.uk) return fail(SV_ERR_INVALID_ARG, "null unitary" + at);
        if (!finite_all(g.uk, (size_t)2 << (2 * g.ntargets))) return fail(SV_ERR_INVALID_ARG, "non-finite matrix entry" + at);
    }
    return SV_OK;
}

sv_status sv_apply_circuit_ex(sv_handle h, const sv_gate_ex *gates, size_t m, const sv_schedule *s)
{
    if (sv_status st = check_handle(h)) return st;
    if (sv_status st = check_schedule(s, h->dtype)) return st;
    if (s && s->tuner != SV_TUNER_NONE) return fail(SV_ERR_UNSUPPORTED, "the tuner takes sv_gate circuits");
    if (m > 0 && !gates) return fail(SV_ERR_INVALID_ARG, "gate array is null");
    for (size_t i = 0; i < m; ++i)
        if (sv_status st = check_gate_ex(gates[i], h->n, i)) return st;
    svp::PlanConfig c = config_from(h, s);
    sv_stats tot{};
    double plan_ms = 0.0;
    std::vector<svp::RawGate> seg;
    auto flush = [&]() -> sv_status {
        if (seg.empty()) return SV_OK;
        const auto p0 = std::chrono::steady_clock::now();
        svp::Plan plan;
        std::string err = svp::make_plan(c, seg.data(), seg.size(), h->l2p, plan);
        if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
        plan_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - p0).count();
        if (sv_status st = run_plan(h, plan, s ? s->outer_qubits : 0, false)) return st;
        h->l2p = plan.l2p_after;
        sv_stats one{};
        fill_stats(&one, c, plan);
        tot.gates += one.gates;
        tot.swaps += one.swaps;
        tot.phases += one.phases;
        tot.passes += one.passes;
        tot.fused += one.fused;
        tot.bytes += one.bytes;
        tot.block_qubits = one.block_qubits;
        seg.clear();
        return SV_OK;
    };
    // the matrices of the extended gates, formed in binary64 and rounded
    // once to the state's precision, uploaded together before any gate runs
    const size_t ab = amp_bytes(h->dtype);
    std::vector<size_t> moff(m, 0);
    std::vector<unsigned char> mats;
    for (size_t i = 0; i < m; ++i) {
        const sv_gate_ex &g = gates[i];
        svp::RawGate r;
        if (as_plain_gate(g, r)) continue;
        const int k = g.op == SV_UK ? g.ntargets : (g.op == SV_SWAP ? 2 : 1);
        const int D = 1 << k;
        std::vector<double> U(2 * (size_t)D * D, 0.0);
        if (g.op == SV_UK) {
            std::memcpy(U.data(), g.uk, U.size() * sizeof(double));
        } else if (g.op == SV_SWAP) {
            for (int x = 0; x < 4; ++x) U[2 * (x * 4 + ((x & 1) << 1 | (x >> 1)))] = 1.0;
        } else {
            int cls = 0;
            svp::gate_matrix(g.op, g.theta, g.u, U.data(), &cls);
        }
        moff[i] = mats.size();
        mats.resize(mats.size() + (((size_t)D * D * ab + 255) & ~(size_t)255));
        unsigned char *dst = mats.data() + moff[i];
        if (h->dtype == SV_COMPLEX64) {
            for (size_t e = 0; e < U.size(); ++e) {
                const float f = (float)U[e];
                std::memcpy(dst + e * sizeof(float), &f, sizeof f);
            }
        } else {
            std::memcpy(dst, U.data(), U.size() * sizeof(double));
        }
    }
    if (!mats.empty()) {
        if (sv_status st = ensure_scratch(h, mats.size())) return st;
        SV_HIP(hipMemcpyAsync(h->scratch, mats.data(), mats.size(), hipMemcpyHostToDevice, h->stream), "upload");
        SV_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    }
    SV_HIP(hipEventRecord(h->ev0, h->stream), "hipEventRecord");
    for (size_t i = 0; i < m; ++i) {
        const sv_gate_ex &g = gates[i];
        svp::RawGate r;
        if (as_plain_gate(g, r)) {
            seg.push_back(r);
            continue;
        }
        if (sv_status st = flush()) return st;
        const int k = g.op == SV_UK ? g.ntargets : (g.op == SV_SWAP ? 2 : 1);
        int tb[SV_MAX_TARGETS], cb[SV_MAX_CONTROLS];
        for (int b = 0; b < k; ++b) tb[b] = h->l2p[g.targets[b]];
        for (int b = 0; b < g.ncontrols; ++b) cb[b] = h->l2p[g.controls[b]];
        if (launch_fault()) return fail(SV_ERR_DEVICE, "injected launch failure");
        SV_HIP(svk::kq_gate(h->buf, h->n, h->dtype, tb, k, cb, g.ncontrols, (char *)h->scratch + moff[i], h->stream),
               "kernel launch");
        tot.gates += 1;
        tot.passes += 1;
        tot.bytes += std::ldexp(2.0 * (double)ab, h->n - g.ncontrols);
    }
    if (sv_status st = flush()) return st;
    SV_HIP(hipEventRecord(h->ev1, h->stream), "hipEventRecord");
    h->timed = true;
    std::memset(&h->st, 0, sizeof(h->st));
    fill_stats(&h->st, c, svp::Plan());
    h->st.gates = tot.gates;
    h->st.swaps = tot.swaps;
    h->st.phases = tot.phases;
    h->st.passes = tot.passes;
    h->st.fused = tot.fused;
    h->st.bytes = tot.bytes;
    h->st.block_qubits = tot.block_qubits;
    h->st.plan_ms = plan_ms;
    return SV_OK;
}

sv_status sv_qasm_parse(const char *text, sv_gate_ex *gates, size_t cap, size_t *count, int *nqubits)
{
    if (!text || !count || !nqubits) return fail(SV_ERR_INVALID_ARG, "null text, count or nqubits");
    if (cap > 0 && !gates) return fail(SV_ERR_INVALID_ARG, "null gate array with nonzero capacity");
    std::vector<sv_gate_ex> out;
    int nq = 0;
    std::string err;
    const sv_status st = svq::parse(text, out, nq, err);
    if (st != SV_OK) return fail(st, err);
    *count = out.size();
    *nqubits = nq;
    if (cap > 0) std::memcpy(gates, out.data(), std::min(cap, out.size()) * sizeof(sv_gate_ex));
    return SV_OK;
}

sv_status sv_prepare(sv_handle h, const sv_gate *gates, size_t m, const sv_schedule *s, int repeats)
{
    if (sv_status st = check_handle(h)) return st;
    if (sv_status st = check_schedule(s, h->dtype)) return st;
    if (repeats < 1 || repeats > 64) return fail(SV_ERR_INVALID_ARG, "repeats must be in [1, 64]");
    const char *jenv = std::getenv("SV_JIT");
    if (jenv && jenv[0] == '0') return SV_OK;
    svp::PlanConfig c = config_from(h, s);
    std::vector<int> l2p = h->l2p;
    for (int r = 0; r < repeats; ++r) {
        svp::Plan plan;
        std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, l2p, plan);
        if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
        std::vector<const void *> handles;
        hipError_t e = svj::prepare_plan(plan, h->dtype, handles, &err);
        if (e != hipSuccess)
            return fail(SV_ERR_DEVICE, err.empty() ? std::string("pass compilation: ") + hipGetErrorString(e) : err);
        l2p = plan.l2p_after;
    }
    return SV_OK;
}

sv_status sv_stats_get(sv_handle h, sv_stats *out)
{
    if (sv_status s = check_handle(h)) return s;
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    if (h->timed) {
        SV_HIP(hipEventSynchronize(h->ev1), "hipEventSynchronize");
        float ms = 0.f;
        SV_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1), "hipEventElapsedTime");
        h->st.device_ms = ms;
        for (int k = 0; k < 3; ++k) {
            h->st.kernel_ms[k] = 0.0;
            h->st.kernel_launches[k] = 0;
        }
        for (size_t i = 0; i < h->kev_kind.size(); ++i) {
            float kms = 0.f;
            SV_HIP(hipEventElapsedTime(&kms, h->kev[2 * i], h->kev[2 * i + 1]), "hipEventElapsedTime");
            h->st.kernel_ms[h->kev_kind[i]] += kms;
            h->st.kernel_launches[h->kev_kind[i]] += 1;
        }
    }
    *out = h->st;
    return SV_OK;
}

sv_status sv_norm(sv_handle h, double *norm2)
{
    if (sv_status s = check_handle(h)) return s;
    if (!norm2) return fail(SV_ERR_INVALID_ARG, "out is null");
    const size_t need = svk::norm_scratch_bytes(h->n) + 64;
    if (sv_status s = ensure_scratch(h, need)) return s;
    double *res = (double *)((char *)h->scratch + svk::norm_scratch_bytes(h->n));
    SV_HIP(svk::norm2(h->buf, h->n, h->dtype, h->scratch, res, h->stream), "norm");
    SV_HIP(hipMemcpyAsync(norm2, res, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
    SV_HIP(hipStreamSynchronize(h->stream), "sync");
    h->st.norm_drift = std::fabs(*norm2 - 1.0);
    return SV_OK;
}

sv_status sv_probabilities(sv_handle h, const int *qubits, int nq, double *out)
{
    if (sv_status s = check_handle(h)) return s;
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    if (nq < 0 || nq > h->n) return fail(SV_ERR_INVALID_ARG, "nq out of range");
    if (nq > 0 && !qubits) return fail(SV_ERR_INVALID_ARG, "qubits is null");
    std::vector<int> qb;
    std::vector<bool> seen(h->n, false);
    for (int k = 0; k < nq; ++k) {
        if (qubits[k] < 0 || qubits[k] >= h->n || seen[qubits[k]])
            return fail(SV_ERR_INVALID_ARG, "qubit list has an out-of-range or repeated entry");
        seen[qubits[k]] = true;
        qb.push_back(h->l2p[qubits[k]]);
    }
    const bool dev = is_device_ptr(out);
    if (nq == 0 || nq == h->n) {
        // all probabilities in logical order (nq == n with a permuted list is a marginal)
        bool plain_order = (nq == 0);
        if (nq == h->n) {
            plain_order = true;
            for (int k = 0; k < nq; ++k)
                if (qubits[k] != k) plain_order = false;
        }
        if (plain_order) {
            const uint64_t N = 1ull << h->n;
            if (dev) {
                SV_HIP(svk::probabilities(h->buf, h->n, h->dtype, h->l2p.data(), out, 0, N, h->stream), "probs");
                return SV_OK;
            }
            const uint64_t chunk = std::min<uint64_t>(N, 1ull << 24);
            if (sv_status s = ensure_scratch(h, chunk * sizeof(double))) return s;
            for (uint64_t off = 0; off < N; off += chunk) {
                const uint64_t cnt = std::min(chunk, N - off);
                SV_HIP(svk::probabilities(h->buf, h->n, h->dtype, h->l2p.data(), (double *)h->scratch, off, cnt,
                                          h->stream),
                       "probs");
                SV_HIP(hipMemcpyAsync(out + off, h->scratch, cnt * sizeof(double), hipMemcpyDeviceToHost,
                                      h->stream),
                       "copy");
                SV_HIP(hipStreamSynchronize(h->stream), "sync");
            }
            return SV_OK;
        }
    }
    const std::vector<int> ob = complement(h->n, qb);
    const uint64_t M = 1ull << nq;
    if (h->n - nq > 12 && M > 65535) return fail(SV_ERR_UNSUPPORTED, "marginal shape not supported");
    const size_t sb = svk::marginal_scratch_bytes(h->n, nq);
    const size_t outb = dev ? 0 : M * sizeof(double);
    if (sv_status s = ensure_scratch(h, sb + outb + 256)) return s;
    double *dst = dev ? out : (double *)((char *)h->scratch + ((sb + 255) / 256) * 256);
    SV_HIP(svk::marginal(h->buf, h->n, h->dtype, qb.data(), nq, ob.data(), dst, h->scratch, h->stream), "marginal");
    if (!dev) {
        SV_HIP(hipMemcpyAsync(out, dst, M * sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
        SV_HIP(hipStreamSynchronize(h->stream), "sync");
    }
    return SV_OK;
}

sv_status sv_qpe_readout(sv_handle h, int t, uint64_t *m, double *phi, double *pmax)
{
    if (sv_status s = check_handle(h)) return s;
    if (t < 1 || t > h->n) return fail(SV_ERR_INVALID_ARG, "t out of range");
    if (!m || !phi || !pmax) return fail(SV_ERR_INVALID_ARG, "null output");
    std::vector<int> qb(t);
    for (int k = 0; k < t; ++k) qb[k] = h->l2p[k];
    const std::vector<int> ob = complement(h->n, qb);
    const size_t am = svk::argmax_scratch_bytes(1ull << t);
    const size_t resb = 64;
    if (h->n - t <= 4) {
        if (sv_status s = ensure_scratch(h, am + resb)) return s;
        char *base = (char *)h->scratch;
        uint64_t *ri = (uint64_t *)(base + am);
        double *rv = (double *)(base + am + 8);
        SV_HIP(svk::marginal_argmax(h->buf, h->n, h->dtype, qb.data(), t, ob.data(), h->scratch, ri, rv, h->stream),
               "qpe readout");
        uint64_t hi = 0;
        double hv = 0;
        SV_HIP(hipMemcpyAsync(&hi, ri, 8, hipMemcpyDeviceToHost, h->stream), "copy");
        SV_HIP(hipMemcpyAsync(&hv, rv, 8, hipMemcpyDeviceToHost, h->stream), "copy");
        SV_HIP(hipStreamSynchronize(h->stream), "sync");
        *m = hi;
        *pmax = hv;
    } else {
        const uint64_t M = 1ull << t;
        if (h->n - t > 12 && M > 65535) return fail(SV_ERR_UNSUPPORTED, "marginal shape not supported");
        const size_t sb = ((svk::marginal_scratch_bytes(h->n, t) + 255) / 256) * 256;
        const size_t mb = ((M * sizeof(double) + 255) / 256) * 256;
        if (sv_status s = ensure_scratch(h, sb + mb + am + resb)) return s;
        char *base = (char *)h->scratch;
        double *marg = (double *)(base + sb);
        void *ams = base + sb + mb;
        uint64_t *ri = (uint64_t *)(base + sb + mb + am);
        double *rv = (double *)(base + sb + mb + am + 8);
        SV_HIP(svk::marginal(h->buf, h->n, h->dtype, qb.data(), t, ob.data(), marg, base, h->stream), "marginal");
        SV_HIP(svk::argmax(marg, M, ams, ri, rv, h->stream), "argmax");
        uint64_t hi = 0;
        double hv = 0;
        SV_HIP(hipMemcpyAsync(&hi, ri, 8, hipMemcpyDeviceToHost, h->stream), "copy");
        SV_HIP(hipMemcpyAsync(&hv, rv, 8, hipMemcpyDeviceToHost, h->stream), "copy");
        SV_HIP(hipStreamSynchronize(h->stream), "sync");
        *m = hi;
        *pmax = hv;
    }
    *phi = std::ldexp((double)*m, -t);
    return SV_OK;
}

// Outcome probabilities of the listed qubits (all qubits in order when
// nq = 0) into device memory at dst (2^nq doubles, or 2^n); work is device
// scratch of outcome_work_bytes.
static size_t outcome_work_bytes(sv_handle h, int nq)
{
    return nq == 0 ? 0 : svk::marginal_scratch_bytes(h->n, nq);
}

static sv_status outcome_probs(sv_handle h, const int *qubits, int nq, double *dst, void *work)
{
    if (nq == 0) {
        SV_HIP(svk::probabilities(h->buf, h->n, h->dtype, h->l2p.data(), dst, 0, 1ull << h->n, h->stream), "probs");
        return SV_OK;
    }
    std::vector<int> qb;
    for (int k = 0; k < nq; ++k) qb.push_back(h->l2p[qubits[k]]);
    const std::vector<int> ob = complement(h->n, qb);
    SV_HIP(svk::marginal(h->buf, h->n, h->dtype, qb.data(), nq, ob.data(), dst, work, h->stream), "marginal");
    return SV_OK;
}

static sv_status check_measured(sv_handle h, const int *qubits, int nq)
{
    if (nq < 0 || nq > h->n) return fail(SV_ERR_INVALID_ARG, "nq out of range");
    if (nq > 0 && !qubits) return fail(SV_ERR_INVALID_ARG, "qubits is null");
    std::vector<bool> seen(h->n, false);
    for (int k = 0; k < nq; ++k) {
        if (qubits[k] < 0 || qubits[k] >= h->n || seen[qubits[k]])
            return fail(SV_ERR_INVALID_ARG, "qubit list has an out-of-range or repeated entry");
        seen[qubits[k]] = true;
    }
    const int m = nq == 0 ? h->n : nq;
    if (m > 32) return fail(SV_ERR_UNSUPPORTED, "more than 32 measured qubits");
    if (nq > 0 && h->n - nq > 12 && nq > 16) return fail(SV_ERR_UNSUPPORTED, "marginal shape not supported");
    return SV_OK;
}

sv_status sv_sample(sv_handle h, const int *qubits, int nq, const double *uniforms, size_t shots, uint64_t *out)
{
    if (sv_status s = check_handle(h)) return s;
    if (sv_status s = check_measured(h, qubits, nq)) return s;
    if (shots > 0 && (!uniforms || !out)) return fail(SV_ERR_INVALID_ARG, "null uniforms or output");
    if (shots == 0) return SV_OK;
    const bool du = is_device_ptr(uniforms), dout = is_device_ptr(out);
    const uint64_t M = 1ull << (nq == 0 ? h->n : nq);
    const size_t chunk = std::min<size_t>(shots, size_t(1) << 22);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_p = 0, o_c = up(M * 8), o_w = o_c + up(M * 8);
    const size_t o_u = o_w + up(std::max(outcome_work_bytes(h, nq), svk::scan_scratch_bytes(M)));
    const size_t o_o = o_u + up(chunk * 8), need = o_o + up(chunk * 8);
    if (sv_status st = ensure_scratch(h, need)) return st;
    char *base = (char *)h->scratch;
    double *P = (double *)(base + o_p), *cdf = (double *)(base + o_c);
    if (sv_status st = outcome_probs(h, qubits, nq, P, base + o_w)) return st;
    SV_HIP(svk::scan_inclusive(P, cdf, M, base + o_w, h->stream), "scan");
    for (size_t off = 0; off < shots; off += chunk) {
        const size_t c = std::min(chunk, shots - off);
        const double *u = uniforms + off;
        if (!du) {
            SV_HIP(hipMemcpyAsync(base + o_u, u, c * 8, hipMemcpyHostToDevice, h->stream), "copy");
            u = (const double *)(base + o_u);
        }
        uint64_t *o = dout ? out + off : (uint64_t *)(base + o_o);
        SV_HIP(svk::sample_outcomes(cdf, M, u, c, o, h->stream), "sample");
        if (!dout) {
            SV_HIP(hipMemcpyAsync(out + off, o, c * 8, hipMemcpyDeviceToHost, h->stream), "copy");
            SV_HIP(hipStreamSynchronize(h->stream), "sync");
        }
    }
    return SV_OK;
}

sv_status sv_measure(sv_handle h, const int *qubits, int nq, double u, uint64_t *outcome, double *prob)
{
    if (sv_status s = check_handle(h)) return s;
    if (sv_status s = check_measured(h, qubits, nq)) return s;
    if (!outcome || !prob) return fail(SV_ERR_INVALID_ARG, "null output");
    if (!(u >= 0.0 && u < 1.0)) return fail(SV_ERR_INVALID_ARG, "u must be in [0, 1)");
    const uint64_t M = 1ull << (nq == 0 ? h->n : nq);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t o_p = 0, o_c = up(M * 8), o_w = o_c + up(M * 8);
    const size_t o_u = o_w + up(std::max(outcome_work_bytes(h, nq), svk::scan_scratch_bytes(M)));
    const size_t need = o_u + 256;
    if (sv_status st = ensure_scratch(h, need)) return st;
    char *base = (char *)h->scratch;
    double *P = (double *)(base + o_p), *cdf = (double *)(base + o_c);
    if (sv_status st = outcome_probs(h, qubits, nq, P, base + o_w)) return st;
    SV_HIP(svk::scan_inclusive(P, cdf, M, base + o_w, h->stream), "scan");
    SV_HIP(hipMemcpyAsync(base + o_u, &u, 8, hipMemcpyHostToDevice, h->stream), "copy");
    uint64_t *dm = (uint64_t *)(base + o_u + 64);
    SV_HIP(svk::sample_outcomes(cdf, M, (const double *)(base + o_u), 1, dm, h->stream), "sample");
    uint64_t m = 0;
    SV_HIP(hipMemcpyAsync(&m, dm, 8, hipMemcpyDeviceToHost, h->stream), "copy");
    SV_HIP(hipStreamSynchronize(h->stream), "sync");
    double pm = 0.0;
    SV_HIP(hipMemcpyAsync(&pm, P + m, 8, hipMemcpyDeviceToHost, h->stream), "copy");
    SV_HIP(hipStreamSynchronize(h->stream), "sync");
    if (!(pm > 0.0)) return fail(SV_ERR_INVALID_ARG, "the drawn outcome has zero probability (state is zero)");
    // the measured qubits' physical bits must equal m's bits
    uint64_t mask = 0, val = 0;
    const int cnt = nq == 0 ? h->n : nq;
    for (int k = 0; k < cnt; ++k) {
        const int pb = h->l2p[nq == 0 ? k : qubits[k]];
        mask |= 1ull << pb;
        if ((m >> k) & 1ull) val |= 1ull << pb;
    }
    SV_HIP(svk::collapse(h->buf, h->n, h->dtype, mask, val, 1.0 / std::sqrt(pm), h->stream), "collapse");
    *outcome = m;
    *prob = pm;
    return SV_OK;
}

sv_status sv_qpe_readout_noalloc(sv_handle h, int t, uint64_t *m, double *phi, double *pmax)
{
    if (sv_status s = check_handle(h)) return s;
    if (t < 1 || t > h->n) return fail(SV_ERR_INVALID_ARG, "t out of range");
    if (!m || !phi || !pmax) return fail(SV_ERR_INVALID_ARG, "null output");
    if (h->n - t > 4)
        return fail(SV_ERR_UNSUPPORTED, "allocation-free readout needs n - t <= 4 (the counting marginal of a state "
                                        "with more than 4 other qubits needs a marginal buffer beyond the static "
                                        "scratch)");
    const size_t am = svk::argmax_scratch_bytes(1ull << t);
    if (am + 16 > svk::static_scratch_bytes())
        return fail(SV_ERR_UNSUPPORTED, "readout scratch larger than the static scratch");
    // counting qubits' physical bits and the others, ascending (no host allocation)
    int qb[64], ob[64], no = 0;
    bool inq[64] = {};
    for (int k = 0; k < t; ++k) {
        qb[k] = h->l2p[k];
        inq[qb[k]] = true;
    }
    for (int p = 0; p < h->n; ++p)
        if (!inq[p]) ob[no++] = p;
    void *base = nullptr;
    SV_HIP(svk::static_scratch(&base), "hipGetSymbolAddress");
    uint64_t *ri = (uint64_t *)((char *)base + am);
    double *rv = (double *)((char *)base + am + 8);
    SV_HIP(svk::marginal_argmax(h->buf, h->n, h->dtype, qb, t, ob, base, ri, rv, h->stream), "qpe readout");
    uint64_t hi = 0;
    double hv = 0;
    SV_HIP(hipMemcpyAsync(&hi, ri, 8, hipMemcpyDeviceToHost, h->stream), "copy");
    SV_HIP(hipMemcpyAsync(&hv, rv, 8, hipMemcpyDeviceToHost, h->stream), "copy");
    SV_HIP(hipStreamSynchronize(h->stream), "sync");
    *m = hi;
    *pmax = hv;
    *phi = std::ldexp((double)hi, -t);
    return SV_OK;
}

static sv_status state_io(sv_handle h, uint64_t offset, uint64_t count, void *out, const void *in)
{
    const uint64_t N = 1ull << h->n;
    if (offset > N || count > N - offset) return fail(SV_ERR_INVALID_ARG, "range outside the state");
    if (count == 0) return SV_OK;
    const size_t ab = amp_bytes(h->dtype);
    void *user = out ? out : const_cast<void *>(in);
    const bool dev = is_device_ptr(user);
    // a plain copy only where the physical layout and the storage order are both the identity
    const bool ident = identity(h->l2p) && svk::plain_storage(h->n, h->dtype);
    char *sbase = (char *)h->buf + offset * ab;
    if (ident) {
        if (out) {
            SV_HIP(hipMemcpyAsync(out, sbase, count * ab, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                  h->stream),
                   "copy");
        } else {
            SV_HIP(hipMemcpyAsync(sbase, in, count * ab, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  h->stream),
                   "copy");
        }
        if (!dev) SV_HIP(hipStreamSynchronize(h->stream), "sync");
        return SV_OK;
    }
    if (dev) {
        if (out) SV_HIP(svk::gather_logical(h->buf, h->n, h->dtype, h->l2p.data(), out, offset, count, h->stream), "gather");
        else SV_HIP(svk::scatter_logical(h->buf, h->n, h->dtype, h->l2p.data(), in, offset, count, h->stream), "scatter");
        return SV_OK;
    }
    const uint64_t chunk = std::min<uint64_t>(count, (1ull << 27) / ab);
    if (sv_status s = ensure_scratch(h, chunk * ab)) return s;
    for (uint64_t o = 0; o < count; o += chunk) {
        const uint64_t c = std::min(chunk, count - o);
        if (out) {
            SV_HIP(svk::gather_logical(h->buf, h->n, h->dtype, h->l2p.data(), h->scratch, offset + o, c, h->stream),
                   "gather");
            SV_HIP(hipMemcpyAsync((char *)out + o * ab, h->scratch, c * ab, hipMemcpyDeviceToHost, h->stream), "copy");
            SV_HIP(hipStreamSynchronize(h->stream), "sync");
        } else {
            SV_HIP(hipMemcpyAsync(h->scratch, (const char *)in + o * ab, c * ab, hipMemcpyHostToDevice, h->stream),
                   "copy");
            SV_HIP(svk::scatter_logical(h->buf, h->n, h->dtype, h->l2p.data(), h->scratch, offset + o, c, h->stream),
                   "scatter");
            SV_HIP(hipStreamSynchronize(h->stream), "sync");
        }
    }
    return SV_OK;
}

sv_status sv_state(sv_handle h, void *out)
{
    if (sv_status s = check_handle(h)) return s;
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    return state_io(h, 0, 1ull << h->n, out, nullptr);
}

sv_status sv_state_range(sv_handle h, uint64_t offset, uint64_t count, void *out)
{
    if (sv_status s = check_handle(h)) return s;
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    return state_io(h, offset, count, out, nullptr);
}

sv_status sv_set_state_range(sv_handle h, uint64_t offset, uint64_t count, const void *in)
{
    if (sv_status s = check_handle(h)) return s;
    if (!in) return fail(SV_ERR_INVALID_ARG, "in is null");
    return state_io(h, offset, count, nullptr, in);
}

}  // extern "C"

// ------------------------------------------------------------------ tuning

namespace {

struct CostModel {
    int in = 0;
    std::vector<float> params, norm;
};
std::mutex g_model_mu;
CostModel g_model;

std::vector<sv_schedule> candidates(int n, int dtype)
{
    std::vector<sv_schedule> out;
    const int top = std::min(n, svp::max_block_qubits(dtype));
    const int r0 = dtype == SV_COMPLEX64 ? 4 : 3;
    const int p0 = dtype == SV_COMPLEX64 ? 4 : 3;  // 128-byte segments
    for (int l = std::max(1, top - 2); l <= top; ++l)
        for (int r = r0; r <= r0 + 1; ++r) {
            if (r > l && r != r0) continue;  // small blocks: one tile of 2^l
            for (int p = p0; p <= p0 + 1; ++p) {
                if (p >= l && p != p0) continue;
                for (int fk : {1, 5}) {
                    sv_schedule c{};
                    c.mode = SV_PARTITIONED;
                    c.block_qubits = l;
                    c.fuse_k = fk;
                    c.swap_policy = SV_SWAP_GRAPH;
                    c.remap = SV_REMAP_VIRTUAL;
                    c.diag_free = 1;
                    c.reg_qubits = std::min(r, l);
                    c.pin_qubits = p;
                    out.push_back(c);
                }
            }
        }
    return out;
}

svp::PlanConfig config_for(int n, int dtype, const sv_schedule *s)
{
    sv_handle_s tmp;
    tmp.n = n;
    tmp.dtype = dtype;
    return config_from(&tmp, s);
}

void plan_features(int n, int dtype, const svp::PlanConfig &c, const svp::Plan &p, float *f)
{
    double k2 = 0, k3 = 0, k1 = 0, ops = 0, maxops = 0, dense = 0, diag = 0, layout = 0;
    int logr = 0;
    for (const svp::Step &st : p.steps) {
        if (st.kind == svp::ST_K1) k1 += 1;
        else if (st.kind == svp::ST_K3) k3 += 1;
        else {
            k2 += 1;
            logr = st.logr;
            ops += st.op_count;
            maxops = std::max(maxops, (double)st.op_count);
            for (int i = 0; i < st.op_count; ++i) {
                const int kind = p.ops[st.op_begin + i].kind;
                if (kind == svp::K2_DENSE || kind == svp::K2_H || kind == svp::K2_X || kind == svp::K2_HU) dense += 1;
                else if (kind == svp::K2_PHASE || kind == svp::K2_DIAG || kind == svp::K2_DIAGRUN) diag += 1;
                else if (kind == svp::K2_LAYOUT) layout += 1;
            }
        }
    }
    f[0] = (float)n;
    f[1] = (float)amp_bytes(dtype);
    f[2] = (float)(c.mode == 1 ? p.l : 0);
    f[3] = (float)logr;
    // low memory qubits kept local in every block (virtual remap): the
    // length of the contiguous runs every access covers
    int pin = 0;
    if (c.mode == 1 && c.remap == SV_REMAP_VIRTUAL)
        pin = std::max(0, std::min(c.pin_low >= 0 ? c.pin_low : svp::default_pin_qubits(dtype), p.l - 1));
    f[4] = (float)pin;
    f[5] = (float)c.fuse_k;
    f[6] = (float)p.stats.gates;
    f[7] = (float)k2;
    f[8] = (float)k3;
    f[9] = (float)k1;
    f[10] = (float)std::log2(std::max(1.0, p.stats.bytes));
    f[11] = (float)ops;
    f[12] = (float)maxops;
    f[13] = (float)dense;
    f[14] = (float)diag;
    f[15] = (float)layout;
}

sv_status status_of(hipError_t e, const char *what)
{
    return e == hipSuccess ? SV_OK : hip_fail(e, what);
}

}  // namespace

extern "C" {

sv_status sv_tune_candidates(int n, sv_dtype dtype, sv_schedule *out, int cap, int *count)
{
    if (n < 1 || n > 36) return fail(SV_ERR_INVALID_ARG, "n must be in [1, 36]");
    if (dtype != SV_COMPLEX64 && dtype != SV_COMPLEX128) return fail(SV_ERR_INVALID_ARG, "unknown dtype");
    if (!count) return fail(SV_ERR_INVALID_ARG, "count is null");
    if (cap < 0) return fail(SV_ERR_INVALID_ARG, "cap < 0");
    const std::vector<sv_schedule> c = candidates(n, dtype);
    if (out)
        for (int i = 0; i < (int)c.size() && i < cap; ++i) out[i] = c[i];
    *count = (int)c.size();
    return SV_OK;
}

sv_status sv_features(int n, sv_dtype dtype, const sv_gate *gates, size_t m, const sv_schedule *s, float *out)
{
    if (n < 1 || n > 36) return fail(SV_ERR_INVALID_ARG, "n must be in [1, 36]");
    if (dtype != SV_COMPLEX64 && dtype != SV_COMPLEX128) return fail(SV_ERR_INVALID_ARG, "unknown dtype");
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    if (sv_status st = check_schedule(s, dtype)) return st;
    const svp::PlanConfig c = config_for(n, dtype, s);
    std::vector<int> l2p(n);
    for (int q = 0; q < n; ++q) l2p[q] = q;
    svp::Plan plan;
    std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, l2p, plan);
    if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
    plan_features(n, dtype, c, plan, out);
    return SV_OK;
}

sv_status sv_jit_precompile(int n, sv_dtype dtype, const sv_gate *gates, size_t m, const sv_schedule *s)
{
    if (n < 1 || n > 36) return fail(SV_ERR_INVALID_ARG, "n must be in [1, 36]");
    if (dtype != SV_COMPLEX64 && dtype != SV_COMPLEX128) return fail(SV_ERR_INVALID_ARG, "unknown dtype");
    if (sv_status st = check_schedule(s, dtype)) return st;
    const svp::PlanConfig c = config_for(n, dtype, s);
    std::vector<int> l2p(n);
    for (int q = 0; q < n; ++q) l2p[q] = q;
    svp::Plan plan;
    std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, l2p, plan);
    if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
    if (svj::precompile(plan, dtype, &err) != hipSuccess)
        return fail(SV_ERR_DEVICE, err.empty() ? std::string("pass compilation failed") : err);
    return SV_OK;
}

sv_status sv_tune_time(sv_handle h, const sv_gate *gates, size_t m, const sv_schedule *cands, int ncand,
                       int repeats, double *ms_out, double *compile_ms)
{
    if (sv_status st = check_handle(h)) return st;
    if (!cands || ncand < 1) return fail(SV_ERR_INVALID_ARG, "no candidates");
    if (!ms_out) return fail(SV_ERR_INVALID_ARG, "ms_out is null");
    if (repeats < 1 || repeats > 100) return fail(SV_ERR_INVALID_ARG, "repeats must be in [1, 100]");
    std::vector<sv_schedule> cs(cands, cands + ncand);
    for (sv_schedule &c : cs) {
        if (sv_status st = check_schedule(&c, h->dtype)) return st;
        c.tuner = SV_TUNER_NONE;
    }
    {
        svp::Plan probe;
        std::string err = svp::make_plan(config_from(h, &cs[0]), reinterpret_cast<const svp::RawGate *>(gates), m,
                                         h->l2p, probe);
        if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
    }
    if (svj::cache_size() > 256) {
        if (hipError_t e = svj::trim_cache(128); e != hipSuccess) return hip_fail(e, "kernel cache trim");
    }
    const size_t nb = amp_bytes(h->dtype) << h->n;
    void *scratch = nullptr;
    if (dev_alloc(&scratch, nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SV_ERR_OUT_OF_MEMORY, "tuner scratch state does not fit");
    }
    sv_handle tmp = nullptr;
    sv_status rc = status_of(hipMemcpyAsync(scratch, h->buf, nb, hipMemcpyDeviceToDevice, h->stream), "copy");
    if (rc == SV_OK) rc = sv_wrap(h->n, (sv_dtype)h->dtype, scratch, nb, h->stream, &tmp);
    for (int i = 0; i < ncand && rc == SV_OK; ++i) {
        const svp::PlanConfig c = config_from(h, &cs[i]);
        svp::Plan plan;
        std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, h->l2p, plan);
        if (!err.empty()) {
            rc = fail(SV_ERR_INVALID_ARG, err);
            break;
        }
        double cms = 0.0;
        const char *jenv = std::getenv("SV_JIT");
        if (!(jenv && jenv[0] == '0')) {
            std::vector<const void *> handles;
            if (svj::prepare_plan(plan, h->dtype, handles, &err, &cms) != hipSuccess) {
                rc = fail(SV_ERR_DEVICE, err.empty() ? std::string("pass compilation failed") : err);
                break;
            }
        }
        if (compile_ms) compile_ms[i] = cms;
        std::vector<double> t;
        for (int rep = 0; rep <= repeats && rc == SV_OK; ++rep) {
            // every run starts from the caller's layout so all runs share one
            // plan; the scratch contents are not needed afterwards
            tmp->l2p = h->l2p;
            rc = sv_apply_circuit(tmp, gates, m, &cs[i]);
            sv_stats st{};
            if (rc == SV_OK) rc = sv_stats_get(tmp, &st);
            if (rc == SV_OK && rep > 0) t.push_back(st.device_ms);
        }
        if (rc != SV_OK) break;
        std::sort(t.begin(), t.end());
        ms_out[i] = t[t.size() / 2];
    }
    if (tmp) sv_destroy(tmp);
    hipStreamSynchronize(h->stream);
    hipFree(scratch);
    return rc;
}

sv_status sv_tune(sv_handle h, const sv_gate *gates, size_t m, int mode, sv_schedule *out)
{
    if (sv_status st = check_handle(h)) return st;
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    if (mode != SV_TUNER_EXHAUSTIVE && mode != SV_TUNER_LEARNED) return fail(SV_ERR_INVALID_ARG, "unknown tuner mode");
    const std::vector<sv_schedule> cs = candidates(h->n, h->dtype);
    CostModel model;
    if (mode == SV_TUNER_LEARNED) {
        std::lock_guard<std::mutex> lk(g_model_mu);
        model = g_model;
    }
    if (mode == SV_TUNER_LEARNED && !model.params.empty()) {
        const int in = model.in, nc = (int)cs.size();
        const svk::MlpLayout L = svk::mlp_layout(in);
        // host layout of the device buffer: params | norm | X | y | argmin
        std::vector<float> host((size_t)L.count + 2 * in + (size_t)nc * in + nc + 1, 0.f);
        std::copy(model.params.begin(), model.params.end(), host.begin());
        std::copy(model.norm.begin(), model.norm.end(), host.begin() + L.count);
        float *X = host.data() + L.count + 2 * in;
        for (int i = 0; i < nc; ++i) {
            const svp::PlanConfig c = config_from(h, &cs[i]);
            svp::Plan plan;
            std::string err = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates), m, h->l2p, plan);
            if (!err.empty()) return fail(SV_ERR_INVALID_ARG, err);
            plan_features(h->n, h->dtype, c, plan, X + (size_t)i * in);
        }
        float *d = nullptr;
        if (dev_alloc((void **)&d, host.size() * sizeof(float)) != hipSuccess)
            return fail(SV_ERR_OUT_OF_MEMORY, "cost model buffer");
        int best = -1;
        sv_status rc = status_of(hipMemcpyAsync(d, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice,
                                                h->stream), "upload");
        float *dy = d + L.count + 2 * in + (size_t)nc * in;
        if (rc == SV_OK)
            rc = status_of(svk::mlp_forward(d, in, d + L.count, d + L.count + 2 * in, nc, dy, (int *)(dy + nc),
                                            h->stream), "cost model");
        if (rc == SV_OK)
            rc = status_of(hipMemcpyAsync(&best, dy + nc, sizeof(int), hipMemcpyDeviceToHost, h->stream), "readback");
        if (rc == SV_OK) rc = status_of(hipStreamSynchronize(h->stream), "sync");
        hipFree(d);
        if (rc != SV_OK) return rc;
        if (best < 0 || best >= nc) return fail(SV_ERR_DEVICE, "cost model returned no candidate");
        *out = cs[best];
        return SV_OK;
    }
    std::vector<double> ms(cs.size(), 0.0);
    if (sv_status st = sv_tune_time(h, gates, m, cs.data(), (int)cs.size(), 3, ms.data(), nullptr)) return st;
    size_t best = 0;
    for (size_t i = 1; i < ms.size(); ++i)
        if (ms[i] < ms[best]) best = i;
    *out = cs[best];
    return SV_OK;
}

sv_status sv_set_cost_model(const float *params, int in, const float *norm)
{
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (!params) {
        g_model = CostModel{};
        return SV_OK;
    }
    if (in != SV_FEATURES) return fail(SV_ERR_INVALID_ARG, "the cost model reads SV_FEATURES inputs");
    const svk::MlpLayout L = svk::mlp_layout(in);
    CostModel m;
    m.in = in;
    m.params.assign(params, params + L.count);
    for (float v : m.params)
        if (!std::isfinite(v)) return fail(SV_ERR_INVALID_ARG, "non-finite parameter");
    m.norm.resize(2 * (size_t)in);
    for (int i = 0; i < in; ++i) {
        m.norm[i] = norm ? norm[i] : 0.f;
        m.norm[in + i] = norm ? norm[in + i] : 1.f;
    }
    g_model = std::move(m);
    return SV_OK;
}

size_t sv_mlp_param_count(int in)
{
    if (in < 1 || in > svk::kMlpMaxIn) return 0;
    return (size_t)svk::mlp_layout(in).count;
}

size_t sv_mlp_workspace_bytes(int in, int batch)
{
    if (in < 1 || in > svk::kMlpMaxIn || batch < 1) return 0;
    return sizeof(float) * (size_t)svk::mlp_grad_groups(batch) * (size_t)(svk::mlp_layout(in).count + 1);
}

sv_status sv_mlp_forward(const float *params, int in, const float *norm, const float *x, int batch, float *y,
                         void *stream)
{
    if (in < 1 || in > svk::kMlpMaxIn) return fail(SV_ERR_INVALID_ARG, "in must be in [1, 32]");
    if (batch < 1) return fail(SV_ERR_INVALID_ARG, "batch < 1");
    if (!params || !x || !y) return fail(SV_ERR_INVALID_ARG, "null pointer");
    return status_of(svk::mlp_forward(params, in, norm, x, batch, y, nullptr, (hipStream_t)stream), "mlp forward");
}

sv_status sv_mlp_grad(const float *params, int in, const float *norm, const float *x, const float *target,
                      int batch, float *grad, float *loss, void *workspace, void *stream)
{
    if (in < 1 || in > svk::kMlpMaxIn) return fail(SV_ERR_INVALID_ARG, "in must be in [1, 32]");
    if (batch < 1) return fail(SV_ERR_INVALID_ARG, "batch < 1");
    if (!params || !x || !target || !grad || !workspace) return fail(SV_ERR_INVALID_ARG, "null pointer");
    return status_of(svk::mlp_grad(params, in, norm, x, target, batch, grad, loss, (float *)workspace,
                                   (hipStream_t)stream),
                     "mlp grad");
}

sv_status sv_mlp_adam(float *params, float *m, float *v, const float *grad, size_t count, float lr, float beta1,
                      float beta2, float eps, int step, void *stream)
{
    if (!params || !m || !v || !grad) return fail(SV_ERR_INVALID_ARG, "null pointer");
    if (count < 1 || count > (size_t)svk::kMlpMaxParams) return fail(SV_ERR_INVALID_ARG, "count out of range");
    if (step < 1) return fail(SV_ERR_INVALID_ARG, "step counts from 1");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(SV_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    return status_of(svk::mlp_adam(params, m, v, grad, (int)count, lr, beta1, beta2, eps, step, (hipStream_t)stream),
                     "mlp adam");
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

// One prepared batch: its device arrays and captured graph, keyed by a hash
// of everything its plans depend on.
struct BatchEntry {
    uint64_t key = 0;
    int dtype = 0, lmax = 4, count = 0;
    unsigned grid = 0, threads = 0;
    size_t lds = 0;
    void *dbuf = nullptr;
    unsigned *ctrs = nullptr;  // count barrier counters, then the error flag
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::vector<int>> l2p_after;
    std::vector<svp::PlanStats> stats;
    std::vector<int> l;        // block qubits per instance
    ~BatchEntry()
    {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (dbuf) hipFree(dbuf);
    }
};

std::mutex g_batch_mu;
std::vector<BatchEntry *> g_batches;  // most recent last
int *g_err_host = nullptr;

uint64_t mix64(uint64_t h, uint64_t x)
{
    h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h *= 0xff51afd7ed558ccdull;
    return h ^ (h >> 33);
}

uint64_t hash_bytes(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        std::memcpy(&w, b + i, 8);
        h = mix64(h, w);
    }
    uint64_t tail = 0;
    std::memcpy(&tail, b + i, n - i);
    return mix64(h, tail ^ n);
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Build (or fetch) the batch for these handles; nullptr + message on failure.
// *sequential is set when the schedule does not run as one launch.
BatchEntry *get_batch(sv_handle *hs, int count, const sv_gate *const *gates, const size_t *m, const sv_schedule *s,
                      bool *sequential, std::string *err)
{
    *sequential = false;
    const int dtype = hs[0]->dtype;
    svp::PlanConfig base = config_from(hs[0], s);
    int min_n = 64;
    for (int i = 0; i < count; ++i) min_n = std::min(min_n, hs[i]->n);
    // One work-group size for the launch, 2^tbits threads; instance i runs
    // blocks of l_i = min(n_i, tbits + rmax) qubits with a register tile of
    // l_i - tbits (3 .. rmax) amplitude bits.
    const int lreq = base.l > 0 ? base.l : svp::default_block_qubits(dtype);
    // default tile: one below the single-state default (the batched kernel
    // runs the interpreter, whose largest tile needs twice the registers and
    // halves the resident work-groups)
    const int rmax = std::min(s && s->reg_qubits > 0 ? s->reg_qubits : svp::default_reg_qubits(dtype) - 1, lreq);
    if (base.mode != 1 || base.remap != 0 || rmax < 3 || rmax > (dtype == 0 ? 5 : 4) || min_n < 3) {
        *sequential = true;
        return nullptr;
    }
    int tbits = std::min(lreq - rmax, min_n - 3);
    while ((1 << tbits) > svk::k6_max_threads(dtype, rmax)) --tbits;
    std::vector<int> li(count), ri(count);
    int lmax_tile = 3;
    for (int i = 0; i < count; ++i) {
        li[i] = std::min(hs[i]->n, tbits + rmax);
        ri[i] = li[i] - tbits;
        lmax_tile = std::max(lmax_tile, ri[i]);
    }
    uint64_t key = mix64(0x5eed, (uint64_t)count);
    key = mix64(key, (uint64_t)tbits);
    if (const char *env = std::getenv("SV_BATCH_MAX_GRID")) key = mix64(key, (uint64_t)std::atol(env));
    key = hash_bytes(key, &base, sizeof(base));
    for (int i = 0; i < count; ++i) {
        key = mix64(key, (uint64_t)(uintptr_t)hs[i]->buf);
        key = mix64(key, (uint64_t)hs[i]->n);
        key = hash_bytes(key, hs[i]->l2p.data(), hs[i]->l2p.size() * sizeof(int));
        key = hash_bytes(key, gates[i], m[i] * sizeof(sv_gate));
    }
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        for (size_t k = 0; k < g_batches.size(); ++k)
            if (g_batches[k]->key == key && g_batches[k]->count == count) {
                BatchEntry *e = g_batches[k];
                g_batches.erase(g_batches.begin() + k);
                g_batches.push_back(e);
                return e;
            }
    }
    // plan every instance with its own block size and tile
    std::vector<svp::Plan> plans(count);
    for (int i = 0; i < count; ++i) {
        svp::PlanConfig c = config_from(hs[i], s);
        c.l = li[i];
        c.logr = ri[i];
        std::string e = svp::make_plan(c, reinterpret_cast<const svp::RawGate *>(gates[i]), m[i], hs[i]->l2p, plans[i]);
        if (!e.empty()) {
            *err = "instance " + std::to_string(i) + ": " + e;
            return nullptr;
        }
        for (const svp::Step &st : plans[i].steps)
            if (st.kind != svp::ST_K2) {
                *sequential = true;
                return nullptr;
            }
    }
    // concatenate ops and tables, rebasing table offsets
    std::vector<svp::K2Op> ops;
    std::vector<uint8_t> table;
    std::vector<svp::BatchPass> passes;
    std::vector<svp::BatchInst> insts(count);
    std::vector<double> work(count);
    size_t max_lds = 0;
    bool all_half = true;
    const size_t amp = dtype == 0 ? 8 : 16;
    for (int i = 0; i < count; ++i) {
        const svp::Plan &P = plans[i];
        const size_t tb = align16(table.size());
        table.resize(tb + P.table.size());
        if (!P.table.empty()) std::memcpy(table.data() + tb, P.table.data(), P.table.size());
        const int ob = (int)ops.size();
        for (svp::K2Op op : P.ops) {
            if (op.kind == svp::K2_DIAGRUN) {
                op.a += (int)tb;
            } else if (op.kind == svp::K2_MFMA) {
                op.a += (int)tb;
            }
            ops.push_back(op);
        }
        insts[i].S = hs[i]->buf;
        insts[i].pass_off = (int)passes.size();
        insts[i].npass = 0;
        insts[i].logr = ri[i];
        insts[i].l = li[i];
        insts[i].ctr = i;
        for (const svp::Step &st : P.steps) {
            svp::BatchPass bp{};
            bp.args.n = hs[i]->n;
            bp.args.l = st.l;
            bp.args.nops = st.op_count;
            bp.args.nug = st.nug;
            bp.args.ug_off = st.nug ? (int)(st.ug_off + tb) : 0;
            bp.args.tab_off = st.tab_count ? (int)(st.tab_off + tb) : 0;
            bp.args.tab_count = st.tab_count;
            bp.args.ut_off = st.nut ? (int)(st.ut_off + tb) : 0;
            bp.args.nut = st.nut;
            max_lds = std::max<size_t>(
                max_lds, svp::k2_lds_layout(st.l, (int)amp, st.nug, st.tab_count, st.nut, st.half_lds).total);
            all_half = all_half && st.half_lds;
            bp.args.vec2 = (st.l >= 2 && st.logr >= 2 && st.bits[0] == 0) ? 1 : 0;
            bp.args.half_lds = st.half_lds;
            std::vector<bool> in(hs[i]->n, false);
            for (int b = 0; b < st.l; ++b) {
                bp.args.bits[b] = (int8_t)st.bits[b];
                in[st.bits[b]] = true;
            }
            int k = 0;
            for (int p = 0; p < hs[i]->n; ++p)
                if (!in[p]) bp.args.nbits[k++] = (int8_t)p;
            bp.args.nblk_bits = hs[i]->n - st.l;
            bp.args.base_or = 0;
            bp.op_begin = ob + st.op_begin;
            passes.push_back(bp);
            insts[i].npass += 1;
        }
        // work in amplitudes moved: every pass reads and writes the state
        work[i] = (double)insts[i].npass * std::ldexp(1.0, hs[i]->n);
    }
    // resident capacity
    const unsigned threads = 1u << tbits;
    int lmax_blk = 0;
    for (int x : li) lmax_blk = std::max(lmax_blk, x);
    const size_t lds = std::max<size_t>(max_lds, svp::k2_lds_layout(lmax_blk, (int)amp, 0, 0, 0, all_half).total);
    bool mfma = false;
    for (const svp::K2Op &op : ops) mfma = mfma || op.kind == svp::K2_MFMA;
    const int per_cu = svk::k6_occupancy(dtype, lmax_tile, threads, lds, mfma);
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1) {
        *err = "cannot size the batch launch";
        return nullptr;
    }
    long cap = (long)per_cu * cus;
    if (const char *env = std::getenv("SV_BATCH_MAX_GRID")) {
        const long v = std::atol(env);
        if (v > 0) cap = std::min(cap, v);
    }
    // Work-groups: an instance with more than one work-group's share of the
    // work gets ceil(share) of its own (at most one per block; the largest
    // groups shrink until everything fits the resident capacity); the
    // others are packed, largest first, onto the least loaded of the
    // remaining work-groups, one after another without barriers.
    double wsum = 0;
    for (double w : work) wsum += w;
    const double target = wsum > 0 ? wsum / (double)cap : 1.0;
    std::vector<int> gsz(count, 1);
    for (int i = 0; i < count; ++i) {
        const double blocks = std::ldexp(1.0, hs[i]->n - li[i]);
        const double share = work[i] / target;
        gsz[i] = share > 1.0 ? (int)std::min(std::ceil(share), blocks) : 1;
    }
    auto packing = [&](long *ded, long *bins, double *single_work, long *nsingle) {
        *ded = 0;
        *single_work = 0;
        *nsingle = 0;
        for (int i = 0; i < count; ++i) {
            if (gsz[i] > 1) {
                *ded += gsz[i];
            } else {
                *single_work += work[i];
                *nsingle += 1;
            }
        }
        *bins = *nsingle == 0 ? 0 : std::min(*nsingle, std::max(1L, (long)std::ceil(*single_work / target)));
    };
    long ded, bins, nsingle;
    double single_work;
    packing(&ded, &bins, &single_work, &nsingle);
    while (ded + bins > cap) {
        const int big = (int)(std::max_element(gsz.begin(), gsz.end()) - gsz.begin());
        if (gsz[big] <= 1) break;
        gsz[big] -= 1;
        packing(&ded, &bins, &single_work, &nsingle);
    }
    if (ded + bins > cap) bins = cap - ded;
    if (nsingle > 0 && bins < 1) {
        *sequential = true;
        return nullptr;
    }
    std::vector<std::vector<std::pair<int, int>>> wg;  // per work-group: (instance, rank)
    for (int i = 0; i < count; ++i) {
        insts[i].group_size = gsz[i];
        if (gsz[i] > 1)
            for (int r = 0; r < gsz[i]; ++r) wg.push_back({{i, r}});
    }
    {
        std::vector<int> order;
        for (int i = 0; i < count; ++i)
            if (gsz[i] == 1) order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
        std::vector<double> load(bins, 0.0);
        const size_t first = wg.size();
        wg.resize(first + bins);
        for (int i : order) {
            const size_t b = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            load[b] += work[i];
            wg[first + b].push_back({i, 0});
        }
    }
    std::vector<int32_t> wg_off(1, 0);
    std::vector<int32_t> jobs;  // int2 pairs
    for (const auto &w : wg) {
        for (const auto &j : w) {
            jobs.push_back(j.first);
            jobs.push_back(j.second);
        }
        wg_off.push_back((int32_t)(jobs.size() / 2));
    }
    // one device buffer: insts | wg_off | jobs | passes | ops | table | counters
    BatchEntry *e = new (std::nothrow) BatchEntry();
    if (!e) {
        *err = "host allocation failed";
        return nullptr;
    }
    const size_t o_inst = 0, o_wg = align16(o_inst + insts.size() * sizeof(svp::BatchInst));
    const size_t o_jobs = align16(o_wg + wg_off.size() * sizeof(int32_t));
    const size_t o_pass = align16(o_jobs + jobs.size() * sizeof(int32_t));
    const size_t o_ops = align16(o_pass + passes.size() * sizeof(svp::BatchPass));
    const size_t o_tab = align16(o_ops + ops.size() * sizeof(svp::K2Op));
    const size_t o_ctr = align16(o_tab + table.size());
    const size_t bytes = o_ctr + (size_t)(count + 1) * sizeof(unsigned);
    if (dev_alloc(&e->dbuf, bytes) != hipSuccess) {
        delete e;
        *err = "batch buffer allocation failed";
        return nullptr;
    }
    char *d = static_cast<char *>(e->dbuf);
    for (svp::BatchPass &bp : passes) bp.args.table = reinterpret_cast<const uint8_t *>(d + o_tab);
    hipStream_t st = hs[0]->stream;
    hipError_t he = hipSuccess;
    auto up = [&](size_t off, const void *src, size_t n) {
        if (he == hipSuccess && n) he = hipMemcpyAsync(d + off, src, n, hipMemcpyHostToDevice, st);
    };
    up(o_inst, insts.data(), insts.size() * sizeof(svp::BatchInst));
    up(o_wg, wg_off.data(), wg_off.size() * sizeof(int32_t));
    up(o_jobs, jobs.data(), jobs.size() * sizeof(int32_t));
    up(o_pass, passes.data(), passes.size() * sizeof(svp::BatchPass));
    up(o_ops, ops.data(), ops.size() * sizeof(svp::K2Op));
    up(o_tab, table.data(), table.size());
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    e->ctrs = reinterpret_cast<unsigned *>(d + o_ctr);
    e->key = key;
    e->dtype = dtype;
    e->lmax = lmax_tile;
    e->count = count;
    e->grid = (unsigned)wg.size();
    e->threads = threads;
    e->lds = lds;
    e->l = li;
    for (int i = 0; i < count; ++i) {
        e->l2p_after.push_back(plans[i].l2p_after);
        e->stats.push_back(plans[i].stats);
    }
    // capture on a private stream (the handle's stream may be the legacy
    // default stream, which cannot be captured); the graph is then launched on
    // the handle's stream. Counters and the error flag are cleared by a kernel.
    hipStream_t cap_st = nullptr;
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
        hipError_t h1 = svk::zero_u32(e->ctrs, (uint32_t)(count + 1), cap_st);
        hipError_t h2 = svk::k6_batch(dtype, lmax_tile, e->grid, threads, lds,
                                      reinterpret_cast<const svp::BatchInst *>(d + o_inst),
                                      reinterpret_cast<const int32_t *>(d + o_wg), d + o_jobs,
                                      reinterpret_cast<const svp::BatchPass *>(d + o_pass),
                                      reinterpret_cast<const svp::K2Op *>(d + o_ops), e->ctrs,
                                      reinterpret_cast<int *>(e->ctrs + count), 1u << 24, mfma, cap_st);
        he = hipStreamEndCapture(cap_st, &e->graph);
        if (he == hipSuccess) he = h1 != hipSuccess ? h1 : h2;
    }
    if (cap_st) hipStreamDestroy(cap_st);
    if (he == hipSuccess) he = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        *err = std::string("batch graph: ") + hipGetErrorString(he);
        delete e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batches.push_back(e);
    while (g_batches.size() > 8) {
        delete g_batches.front();
        g_batches.erase(g_batches.begin());
    }
    return e;
}

sv_status check_batch(sv_handle *hs, int count, const sv_gate *const *gates, const size_t *m)
{
    if (count < 0 || (count > 0 && (!hs || !gates || !m))) return fail(SV_ERR_INVALID_ARG, "bad batch arrays");
    std::unordered_set<const void *> seen;
    for (int i = 0; i < count; ++i) {
        if (sv_status st = check_handle(hs[i])) return st;
        if (!seen.insert(hs[i]).second) return fail(SV_ERR_INVALID_ARG, "a handle appears twice in the batch");
        if (hs[i]->dtype != hs[0]->dtype) return fail(SV_ERR_INVALID_ARG, "mixed dtypes in one batch");
        if (m[i] > 0 && !gates[i]) return fail(SV_ERR_INVALID_ARG, "null gate list");
        std::string e = svp::validate(hs[i]->n, reinterpret_cast<const svp::RawGate *>(gates[i]), m[i]);
        if (!e.empty()) return fail(SV_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": " + e);
    }
    return SV_OK;
}

}  // namespace

extern "C" {

sv_status sv_apply_batch(sv_handle *hs, int count, const sv_gate *const *gates, const size_t *m,
                         const sv_schedule *s)
{
    if (sv_status st = check_batch(hs, count, gates, m)) return st;
    if (count == 0) return SV_OK;
    if (sv_status st = check_schedule(s, hs[0]->dtype)) return st;
    if (s && s->tuner != SV_TUNER_NONE)
        return fail(SV_ERR_UNSUPPORTED, "batches are tuned with sv_tune_batch, not through the schedule");
    bool sequential = false;
    std::string err;
    BatchEntry *e = get_batch(hs, count, gates, m, s, &sequential, &err);
    if (sequential) {
        for (int i = 0; i < count; ++i)
            if (sv_status st = sv_apply_circuit(hs[i], gates[i], m[i], s)) return st;
        return SV_OK;
    }
    if (!e) return fail(SV_ERR_DEVICE, err);
    if (!g_err_host) {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(int), 0) != hipSuccess) return fail(SV_ERR_OUT_OF_MEMORY, "pinned flag");
        g_err_host = static_cast<int *>(p);
    }
    sv_handle h0 = hs[0];
    hipStream_t st = h0->stream;
    if (launch_fault()) return fail(SV_ERR_DEVICE, "injected launch failure");
    SV_HIP(hipEventRecord(h0->ev0, st), "hipEventRecord");
    SV_HIP(hipGraphLaunch(e->exec, st), "hipGraphLaunch");
    SV_HIP(hipEventRecord(h0->ev1, st), "hipEventRecord");
    SV_HIP(hipMemcpyAsync(g_err_host, e->ctrs + count, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    SV_HIP(hipStreamSynchronize(st), "sync");
    if (*g_err_host != 0) return fail(SV_ERR_DEVICE, "batch pass barrier did not complete (timed out)");
    float ms = 0.f;
    SV_HIP(hipEventElapsedTime(&ms, h0->ev0, h0->ev1), "hipEventElapsedTime");
    for (int i = 0; i < count; ++i) {
        sv_handle h = hs[i];
        h->l2p = e->l2p_after[i];
        std::memset(&h->st, 0, sizeof(h->st));
        h->st.gates = e->stats[i].gates;
        h->st.swaps = e->stats[i].swaps;
        h->st.phases = e->stats[i].phases;
        h->st.passes = e->stats[i].passes;
        h->st.fused = e->stats[i].fused;
        h->st.bytes = e->stats[i].bytes;
        h->st.device_ms = ms;
        h->st.block_qubits = e->l[i];
        h->st.mode = 1;
        h->st.fuse_k = s ? s->fuse_k : 1;
        h->st.swap_policy = s ? s->swap_policy : SV_SWAP_GRAPH;
        h->timed = false;
    }
    return SV_OK;
}

sv_status sv_tune_batch(sv_handle *hs, int count, const sv_gate *const *gates, const size_t *m, sv_schedule *out)
{
    if (sv_status st = check_batch(hs, count, gates, m)) return st;
    if (!out) return fail(SV_ERR_INVALID_ARG, "out is null");
    if (count == 0) return fail(SV_ERR_INVALID_ARG, "empty batch");
    const int dtype = hs[0]->dtype;
    int max_n = 0;
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        max_n = std::max(max_n, hs[i]->n);
        total += align16(hs[i]->bytes);
    }
    // scratch copies of every state, wrapped in temporary handles
    void *scratch = nullptr;
    if (dev_alloc(&scratch, total) != hipSuccess) return fail(SV_ERR_OUT_OF_MEMORY, "tuner scratch");
    std::vector<sv_handle> tmp(count, nullptr);
    sv_status rc = SV_OK;
    size_t off = 0;
    for (int i = 0; i < count && rc == SV_OK; ++i) {
        char *dst = static_cast<char *>(scratch) + off;
        off += align16(hs[i]->bytes);
        const size_t nb = amp_bytes(dtype) << hs[i]->n;
        if (hipMemcpyAsync(dst, hs[i]->buf, nb, hipMemcpyDeviceToDevice, hs[0]->stream) != hipSuccess) rc = SV_ERR_DEVICE;
        else rc = sv_wrap(hs[i]->n, (sv_dtype)dtype, dst, nb, hs[0]->stream, &tmp[i]);
        if (rc == SV_OK) tmp[i]->l2p = hs[i]->l2p;
    }
    sv_schedule best{};
    double best_ms = 1e30;
    if (rc == SV_OK) {
        const int lmax = std::min(max_n, svp::max_block_qubits(dtype));
        static const int fuse_ks[] = {1, 4, 5};
        const int rdef = svp::default_reg_qubits(dtype);
        for (int l = std::max(7, lmax - 5); l <= lmax && rc == SV_OK; ++l)
            for (int r = rdef - 1; r <= rdef && rc == SV_OK; ++r)
            for (int fuse : fuse_ks) {
                if (rc != SV_OK) break;
                sv_schedule c{};
                c.mode = SV_PARTITIONED;
                c.block_qubits = l;
                c.reg_qubits = r;
                c.fuse_k = fuse;
                c.swap_policy = SV_SWAP_GRAPH;
                c.remap = SV_REMAP_VIRTUAL;
                c.diag_free = 1;
                std::vector<double> t;
                for (int rep = 0; rep < 4 && rc == SV_OK; ++rep) {
                    rc = sv_apply_batch(tmp.data(), count, gates, m, &c);
                    if (rc == SV_OK && rep > 0) t.push_back(tmp[0]->st.device_ms);
                }
                if (rc != SV_OK) break;
                std::sort(t.begin(), t.end());
                const double med = t[t.size() / 2];
                if (med < best_ms) {
                    best_ms = med;
                    best = c;
                }
            }
    }
    for (sv_handle h : tmp)
        if (h) sv_destroy(h);
    hipStreamSynchronize(hs[0]->stream);
    hipFree(scratch);
    if (rc != SV_OK) return rc;
    *out = best;
    return SV_OK;
}

}  // extern "C"
