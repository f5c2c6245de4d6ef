// Pass kernels generated at run time.
//
// A block pass's op list is known once the planner has run, so instead of
// interpreting it on every block, the library writes it out as straight-line
// device code (register slots, masks, tables and constants all fixed),
// compiles it for gfx950 with hipRTC and launches it through the module API.
// The generated code calls the same handlers as the interpreter
// (k2_device.h), in the same order with the same operands, so both produce
// the same bits. Compiled kernels are cached by their source text.
#include "jit.h"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <unistd.h>
#include <cstring>
#include <functional>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

namespace {

#include "jit_src.inc"  // kJitAbiH, kJitDeviceH: text of k2_abi.h and k2_device.h

struct Kernel {
    hipFunction_t fn = nullptr;
    int per_cu = 0;
    unsigned threads = 0;
};
struct Entry {
    hipModule_t mod = nullptr;
    std::vector<Kernel> kernels;
    uint64_t last_use = 0;
};

std::mutex g_mu;
std::unordered_map<std::string, Entry> g_cache;
uint64_t g_clock = 0;
int g_cus = 0;

std::string hexd(double x)
{
    char buf[64];
    std::snprintf(buf, sizeof buf, "%a", x);
    return buf;
}

std::string u64s(uint64_t x) { return std::to_string(x) + "ull"; }

// The compile options of every pass module.
const char *const kRtcOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                                "-target-feature", "-Xclang", "-packed-fp32-ops"};
constexpr int kRtcNopts = (int)(sizeof kRtcOpts / sizeof kRtcOpts[0]);

}  // namespace

namespace svj {

static std::string generate_pass(const svp::Step &s, const svp::Plan &plan, int dtype, int idx)
{
    const int r = s.logr, l = s.l;
    std::ostringstream o;
    o << "struct Prog" << idx << " {\n  template <typename T, int LOGR>\n"
         "  __device__ __forceinline__ void run(typename CT<T>::type *a, K2Ctx &cx) const {\n"
         "    using C = typename CT<T>::type;\n    constexpr int R = 1 << LOGR;\n    (void)R;\n";
    std::vector<int> rb(r);
    rb[0] = 0;
    for (int j = 1; j < r; ++j) rb[j] = svp::k2_canon_bit(j, l, r);
    for (int i = 0; i < s.op_count; ++i) {
        const svp::K2Op &op = plan.ops[s.op_begin + i];
        switch (op.kind) {
        case svp::K2_HU:
            o << "    k2_hu<" << op.a << ", R>(a);\n";
            break;
        case svp::K2_LAYOUT: {
            std::vector<int> nrb(r);
            for (int j = 0; j < r; ++j) nrb[j] = (op.a >> (5 * j)) & 31;
            o << "    { const int ro[" << r << "] = {";
            for (int j = 0; j < r; ++j) o << (j ? ", " : "") << rb[j];
            o << "}; const int rn[" << r << "] = {";
            for (int j = 0; j < r; ++j) o << (j ? ", " : "") << nrb[j];
            o << "}; k2_layout<LOGR>(a, cx, ro, rn, " << op.b << "); }\n";
            rb = nrb;
            break;
        }
        case svp::K2_DIAGRUN: {
            // Thread factors shared along a depth-first walk of the subsets
            // of the register bits: slot k's product extends its parent's
            // (k without its highest bit) by the groups whose highest bit is
            // that bit, which is the fold order DiagRun defines, so the
            // interpreter's slot-by-slot products have the same bits.
            const svp::DiagRun *rec = reinterpret_cast<const svp::DiagRun *>(plan.table.data() + op.a);
            const svp::DiagGroup *gs = reinterpret_cast<const svp::DiagGroup *>(rec + 1);
            const double *qt = reinterpret_cast<const double *>(gs + rec->ngroups);
            auto top_bit = [](int m) { return m ? 31 - __builtin_clz((uint32_t)m) : -1; };
            o << "    {\n";
            for (int i = 0; i < rec->ngroups; ++i) {
                const svp::DiagGroup &G = gs[i];
                o << "      const svp::DiagGroup G" << i << "{" << G.rmask << ", " << G.cond_kind << ", " << G.cond_bit
                  << ", " << G.uidx << ", " << G.lane_off << ", " << G.wave_off << ", 0, 0};\n"
                  << "      const C g" << i << " = k2_group_factor<C>(G" << i << ", cx);\n";
            }
            int tmp = 0;
            auto fold = [&](std::string t, int i) -> std::string {
                if (t.empty()) return "g" + std::to_string(i);
                const std::string name = "t" + std::to_string(tmp++);
                o << "      const C " << name << " = cmul(" << t << ", g" << i << ");\n";
                return name;
            };
            std::string troot;
            for (int i = 0; i < rec->ngroups; ++i)
                if (gs[i].rmask == 0) troot = fold(troot, i);
            std::function<void(int, const std::string &)> visit = [&](int k, const std::string &tk) {
                if ((rec->kmask >> k) & 1u) {
                    const bool q = (rec->qmask >> k) & 1u;
                    o << "      k2_diag_apply(a[" << k << "], " << (q ? "true" : "false") << ", make_double2("
                      << hexd(qt[2 * k]) << ", " << hexd(qt[2 * k + 1]) << "), " << (tk.empty() ? "false" : "true")
                      << ", " << (tk.empty() ? std::string("mk<C>(1.0, 0.0)") : tk) << ");\n";
                }
                for (int j = top_bit(k) + 1; j < r; ++j) {
                    const int c = k | (1 << j);
                    std::string tc = tk;
                    for (int i = 0; i < rec->ngroups; ++i)
                        if (top_bit(gs[i].rmask) == j && (gs[i].rmask & ~c) == 0) tc = fold(tc, i);
                    visit(c, tc);
                }
            };
            visit(0, troot);
            o << "    }\n";
            break;
        }
        case svp::K2_SCALE:
            o << "    k2_scale<R>(a, " << hexd(op.v[0]) << ");\n";
            break;
        case svp::K2_MFMA: {
            o << "    { const int ro[" << r << "] = {";
            for (int j = 0; j < r; ++j) o << (j ? ", " : "") << rb[j];
            o << "}; const int w[5] = {";
            for (int j = 0; j < 5; ++j) o << (j ? ", " : "") << ((op.c >> (5 * j)) & 31);
            o << "}; k2_mfma<LOGR, " << op.b << ">(a, cx, ro, w, " << l << ", cx.table + " << op.a << "); }\n";
            break;
        }
        case svp::K2_PHASE:
            o << "    k2_phase<R>(a, cx, " << op.a << ", " << (uint32_t)op.m0 << "u, " << u64s(op.m1) << ", mk<C>("
              << hexd(op.v[0]) << ", " << hexd(op.v[1]) << "));\n";
            break;
        case svp::K2_DIAG:
            o << "    k2_diag<R>(a, cx, " << op.a << ", " << op.b << ", " << op.c << ", " << (uint32_t)op.m0 << "u, "
              << u64s(op.m1) << ", mk<C>(" << hexd(op.v[0]) << ", " << hexd(op.v[1]) << "), mk<C>("
              << hexd(op.v[2]) << ", " << hexd(op.v[3]) << "));\n";
            break;
        default: {
            o << "    { const double v[8] = {";
            for (int k = 0; k < 8; ++k) o << (k ? ", " : "") << hexd(op.v[k]);
            o << "}; ";
            const std::string tpred =
                op.b == svp::CK_MEM ? "code_bit(cx.tloc, cx.base, " + std::to_string(op.c) + ")" : "true";
            o << "k2_pairs<" << op.a << ", R>(a, " << op.kind << ", v, " << tpred << ", " << op.b << ", "
              << (op.b == svp::CK_SLOT ? op.c : 0) << "); }\n";
            break;
        }
        }
    }
    o << "  }\n};\n";
    const char *T = dtype == 0 ? "float" : "double";
    const bool vec2 = s.l >= 2 && s.logr >= 2 && s.bits[0] == 0;  // as the launcher sets args.vec2
    const unsigned threads = 1u << (l - r);
    const size_t amp = dtype == 0 ? 8 : 16;
    const size_t lds = svp::k2_lds_layout(l, (int)amp, s.nug, s.tab_count, s.nut, s.half_lds).total;
    // A pass that stages half the block keeps two work-groups on a CU: the
    // register budget is that of four waves per SIMD and the next block is not
    // prefetched (the other work-group computes while one waits). The others
    // prefetch into a second register set.
    const bool two = s.half_lds && threads * 2 <= 1024;
    // a pass with matrix-core windows keeps no prefetch set either: the
    // windows' operands and accumulators take those registers
    bool windows = false;
    for (int i = 0; i < s.op_count; ++i) windows = windows || plan.ops[s.op_begin + i].kind == svp::K2_MFMA;
    o << "extern \"C\" __global__ void __launch_bounds__(" << threads << ")";
    if (two) o << " __attribute__((amdgpu_waves_per_eu(" << (threads / 64 * 2 + 3) / 4 << ")))";
    o << " svk2_pass_" << idx << "(CT<" << T << ">::type *__restrict__ S, svp::K2Args args) {\n"
      << "  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[" << (lds > 0 ? lds : 16) << "];\n"
      << "  k2_body<" << T << ", " << r << ", " << (vec2 ? "true" : "false") << ", " << (two || windows ? 0 : 2)
      << ">(S, args, lds_raw, Prog" << idx << "{}, blockIdx.x, gridDim.x);\n}\n";
    return o.str();
}

std::string generate(const svp::Step &s, const svp::Plan &plan, int dtype)
{
    return "#include \"k2_device.h\"\nusing namespace svk;\n" + generate_pass(s, plan, dtype, 0);
}

// All block passes of a plan in one translation unit (one compile); kernel
// i is svk2_pass_<i> for the i-th block pass.
std::string generate_plan(const svp::Plan &plan, int dtype)
{
    std::string src = "#include \"k2_device.h\"\nusing namespace svk;\n";
    int idx = 0;
    for (const svp::Step &s : plan.steps)
        if (s.kind == svp::ST_K2) src += generate_pass(s, plan, dtype, idx++);
    return src;
}

static hipError_t compile_rtc(const std::string &src, std::vector<char> &code, std::string *err)
{
    hiprtcProgram prog;
    const char *headers[] = {kJitAbiH, kJitDeviceH};
    const char *names[] = {"k2_abi.h", "k2_device.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "svk2_pass.hip", 2, headers, names) != HIPRTC_SUCCESS) {
        if (err) *err = "hiprtcCreateProgram failed";
        return hipErrorInvalidValue;
    }
    const hiprtcResult rc = hiprtcCompileProgram(prog, kRtcNopts, kRtcOpts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        if (err) *err = "pass compilation failed: " + log.substr(0, 2000);
        hiprtcDestroyProgram(&prog);
        return hipErrorInvalidImage;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return hipSuccess;
}

// Optional on-disk cache of compiled passes, shared by processes: with
// SV_JIT_CACHE_DIR set, a pass module is stored as <dir>/svk2-<key>.co where
// the key is two independent 64-bit FNV-1a hashes of the source text (which
// embeds every constant) and the compiler version; a file is written under a
// temporary name and renamed into place, so readers never see a partial one.
static uint64_t fnv1a(const std::string &s, uint64_t h)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 0x100000001b3ull;
    }
    return h;
}

// Hash of everything a module depends on besides its generated source: the
// embedded header texts (handlers, skeleton, K2Args layout) and the options.
static uint64_t toolchain_hash()
{
    std::string t = kJitAbiH;
    t += '\0';
    t += kJitDeviceH;
    for (int i = 0; i < kRtcNopts; ++i) {
        t += '\0';
        t += kRtcOpts[i];
    }
    return fnv1a(t, 0xcbf29ce484222325ull);
}

// <dir>/svk2-<source hash x2>-<toolchain hash>.co; the source hashes also
// cover the hipRTC version.
static std::string cache_path(const std::string &src)
{
    const char *dir = std::getenv("SV_JIT_CACHE_DIR");
    if (!dir || !*dir) return "";
    int major = 0, minor = 0;
    hiprtcVersion(&major, &minor);
    const std::string tag = src + "|hiprtc " + std::to_string(major) + "." + std::to_string(minor);
    char name[96];
    std::snprintf(name, sizeof name, "/svk2-%016llx%016llx-%016llx.co",
                  (unsigned long long)fnv1a(tag, 0xcbf29ce484222325ull),
                  (unsigned long long)fnv1a(tag, 0x84222325cbf29ce4ull), (unsigned long long)toolchain_hash());
    return std::string(dir) + name;
}

static hipError_t compile(const std::string &src, std::vector<char> &code, std::string *err)
{
    const std::string path = cache_path(src);
    if (!path.empty()) {
        if (FILE *f = std::fopen(path.c_str(), "rb")) {
            std::fseek(f, 0, SEEK_END);
            const long size = std::ftell(f);
            std::fseek(f, 0, SEEK_SET);
            code.resize(size > 0 ? (size_t)size : 0);
            const bool ok = size > 0 && std::fread(code.data(), 1, code.size(), f) == code.size();
            std::fclose(f);
            if (ok) return hipSuccess;
        }
    }
    hipError_t e = compile_rtc(src, code, err);
    if (e == hipSuccess && !path.empty()) {
        const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
        if (FILE *f = std::fopen(tmp.c_str(), "wb")) {
            const bool ok = std::fwrite(code.data(), 1, code.size(), f) == code.size();
            std::fclose(f);
            if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
        }
    }
    return e;
}

std::string compile_check(const std::string &src)
{
    hiprtcProgram prog;
    const char *headers[] = {kJitAbiH, kJitDeviceH};
    const char *names[] = {"k2_abi.h", "k2_device.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "svk2_pass.hip", 2, headers, names) != HIPRTC_SUCCESS)
        return "hiprtcCreateProgram failed";
    std::string out;
    if (hiprtcCompileProgram(prog, kRtcNopts, kRtcOpts) != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        out.assign(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &out[0]);
        if (out.empty()) out = "compile failed";
    }
    hiprtcDestroyProgram(&prog);
    return out;
}

hipError_t prepare_plan(const svp::Plan &plan, int dtype, std::vector<const void *> &handles, std::string *err,
                        double *compile_ms)
{
    if (compile_ms) *compile_ms = 0.0;
    handles.assign(plan.steps.size(), nullptr);
    bool any = false;
    for (const svp::Step &s : plan.steps) any = any || s.kind == svp::ST_K2;
    if (!any) return hipSuccess;
    const std::string src = generate_plan(plan, dtype);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_cus == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
    }
    auto it = g_cache.find(src);
    if (it == g_cache.end()) {
        std::vector<char> code;
        const auto t0 = std::chrono::steady_clock::now();
        hipError_t he = compile(src, code, err);
        if (compile_ms)
            *compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (he != hipSuccess) return he;
        Entry e;
        he = hipModuleLoadData(&e.mod, code.data());
        if (he != hipSuccess) return he;
        int idx = 0;
        for (const svp::Step &s : plan.steps) {
            if (s.kind != svp::ST_K2) continue;
            Kernel k;
            const std::string name = "svk2_pass_" + std::to_string(idx++);
            he = hipModuleGetFunction(&k.fn, e.mod, name.c_str());
            if (he != hipSuccess) return he;
            k.threads = 1u << (s.l - s.logr);
            he = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&k.per_cu, k.fn, (int)k.threads, 0);
            if (he != hipSuccess) return he;
            if (k.per_cu < 1) return hipErrorInvalidConfiguration;
            e.kernels.push_back(k);
        }
        it = g_cache.emplace(src, std::move(e)).first;
    }
    it->second.last_use = ++g_clock;
    size_t k = 0;
    for (size_t i = 0; i < plan.steps.size(); ++i)
        if (plan.steps[i].kind == svp::ST_K2) handles[i] = &it->second.kernels[k++];
    return hipSuccess;
}

hipError_t launch(const void *handle, void *S, const svp::K2Args &a, hipStream_t st)
{
    const Kernel &e = *static_cast<const Kernel *>(handle);
    const uint64_t blocks = 1ull << a.nblk_bits;
    const uint64_t grid = svp::k2_grid((uint64_t)e.per_cu * (uint64_t)g_cus, blocks);
    svp::K2Args args = a;
    void *params[] = {&S, &args};
    return hipModuleLaunchKernel(e.fn, (unsigned)grid, 1, 1, e.threads, 1, 1, 0, st, params, nullptr);
}

hipError_t precompile(const svp::Plan &plan, int dtype, std::string *err)
{
    bool any = false;
    for (const svp::Step &s : plan.steps) any = any || s.kind == svp::ST_K2;
    if (!any) return hipSuccess;
    std::vector<char> code;
    return compile(generate_plan(plan, dtype), code, err);
}

hipError_t trim_cache(size_t keep)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_cache.size() <= keep) return hipSuccess;
    // kernels of an evicted module may still be queued on some stream
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    std::vector<std::pair<uint64_t, const std::string *>> order;
    for (auto &kv : g_cache) order.emplace_back(kv.second.last_use, &kv.first);
    std::sort(order.begin(), order.end());
    const size_t drop = g_cache.size() - keep;
    std::vector<std::string> victims;
    for (size_t i = 0; i < drop; ++i) victims.push_back(*order[i].second);
    for (const std::string &v : victims) {
        auto it = g_cache.find(v);
        if (it->second.mod) e = hipModuleUnload(it->second.mod);
        g_cache.erase(it);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t cache_size()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_cache.size();
}

}  // namespace svj
