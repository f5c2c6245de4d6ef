// OpenQASM 2.0 front end: program text to extended gate records.
//
// The paper's circuits (Section IV) are gate lists over one control; this
// reader widens the front end to the exchange format most circuit sources
// emit. It follows the OpenQASM 2.0 grammar: registers, the built-in U and
// CX, the standard library's gate names (enabled by including "qelib1.inc";
// the library is built in, no file is read), user gate definitions with
// angle parameters, expressions over pi and the six standard functions,
// and register broadcast. Measurement and barriers are accepted and
// dropped (the state is what the library returns); reset, classically
// conditioned gates and opaque gates are refused. Qubits are numbered over
// the quantum registers in declaration order.
//
// Matrix conventions (the language fixes gates only up to a global phase;
// a state-vector simulator has to pick one):
//   U(theta, phi, lambda) = [[cos(theta/2), -e^{i lambda} sin(theta/2)],
//                            [e^{i phi} sin(theta/2), e^{i(phi+lambda)} cos(theta/2)]]
//   rx, ry, rz = exp(-i theta sigma / 2); p = u1 = diag(1, e^{i lambda});
//   rzz, rxx = exp(-i theta P (x) P / 2); controlled gates apply the named
//   one-qubit matrix where every control is 1 (cu adds e^{i gamma}).
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/sv.h"
#include "qasm.h"

namespace svq {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kMaxGates = size_t(1) << 24;  // 16 Mi records (3 GiB)
constexpr int kMaxDepth = 64;

enum TokKind { T_ID, T_NUM, T_STR, T_SYM, T_END };
struct Tok {
    TokKind kind;
    std::string text;
    double num = 0.0;
    bool integer = false;
    int line = 0;
};

struct Error {
    sv_status status;
    std::string msg;
};

[[noreturn]] void raise(sv_status s, int line, const std::string &m)
{
    throw Error{s, "qasm line " + std::to_string(line) + ": " + m};
}

std::vector<Tok> lex(const char *src)
{
    std::vector<Tok> out;
    int line = 1;
    const char *p = src;
    while (*p) {
        const char c = *p;
        if (c == '\n') { ++line; ++p; continue; }
        if (std::isspace((unsigned char)c)) { ++p; continue; }
        if (c == '/' && p[1] == '/') {
            while (*p && *p != '\n') ++p;
            continue;
        }
        if (c == '/' && p[1] == '*') {
            p += 2;
            while (*p && !(p[0] == '*' && p[1] == '/')) {
                if (*p == '\n') ++line;
                ++p;
            }
            if (!*p) raise(SV_ERR_INVALID_ARG, line, "unterminated comment");
            p += 2;
            continue;
        }
        Tok t;
        t.line = line;
        if (std::isalpha((unsigned char)c) || c == '_') {
            const char *b = p;
            while (std::isalnum((unsigned char)*p) || *p == '_') ++p;
            t.kind = T_ID;
            t.text.assign(b, p);
        } else if (std::isdigit((unsigned char)c) || (c == '.' && std::isdigit((unsigned char)p[1]))) {
            const char *b = p;
            bool integer = true;
            while (std::isdigit((unsigned char)*p)) ++p;
            if (*p == '.') {
                integer = false;
                ++p;
                while (std::isdigit((unsigned char)*p)) ++p;
            }
            if ((*p == 'e' || *p == 'E') &&
                (std::isdigit((unsigned char)p[1]) ||
                 ((p[1] == '+' || p[1] == '-') && std::isdigit((unsigned char)p[2])))) {
                integer = false;
                p += 2;
                while (std::isdigit((unsigned char)*p)) ++p;
            }
            t.kind = T_NUM;
            t.text.assign(b, p);
            t.num = std::strtod(t.text.c_str(), nullptr);
            t.integer = integer;
        } else if (c == '"') {
            const char *b = ++p;
            while (*p && *p != '"' && *p != '\n') ++p;
            if (*p != '"') raise(SV_ERR_INVALID_ARG, line, "unterminated string");
            t.kind = T_STR;
            t.text.assign(b, p);
            ++p;
        } else if ((c == '-' && p[1] == '>') || (c == '=' && p[1] == '=')) {
            t.kind = T_SYM;
            t.text.assign(p, p + 2);
            p += 2;
        } else if (std::strchr(";,()[]{}+-*/^", c)) {
            t.kind = T_SYM;
            t.text.assign(1, c);
            ++p;
        } else {
            raise(SV_ERR_INVALID_ARG, line, std::string("unexpected character '") + c + "'");
        }
        out.push_back(std::move(t));
    }
    Tok e;
    e.kind = T_END;
    e.line = line;
    out.push_back(e);
    return out;
}

// A user gate: parameter names, qubit argument names, body tokens.
struct GateDef {
    std::vector<std::string> params, args;
    std::vector<Tok> body;
    bool opaque = false;
};

struct Reg {
    int offset, size;
};

class Reader {
public:
    explicit Reader(std::vector<sv_gate_ex> &out) : out_(out) {}

    int nqubits() const { return nq_; }

    void program(const std::vector<Tok> &toks)
    {
        Cursor c{&toks, 0};
        if (c.is_id("OPENQASM")) {
            c.next();
            const Tok &v = c.expect(T_NUM, "version");
            if (v.num < 2.0 || v.num >= 3.0) raise(SV_ERR_UNSUPPORTED, v.line, "only OpenQASM 2.x is read");
            c.sym(";");
        }
        while (c.peek().kind != T_END) statement(c);
    }

private:
    struct Cursor {
        const std::vector<Tok> *t;
        size_t i;
        const Tok &peek(size_t k = 0) const { return (*t)[std::min(i + k, t->size() - 1)]; }
        const Tok &next()
        {
            const Tok &x = peek();
            if (x.kind != T_END) ++i;
            return x;
        }
        bool is_sym(const char *s, size_t k = 0) const { return peek(k).kind == T_SYM && peek(k).text == s; }
        bool is_id(const char *s) const { return peek().kind == T_ID && peek().text == s; }
        void sym(const char *s)
        {
            if (!is_sym(s)) raise(SV_ERR_INVALID_ARG, peek().line, std::string("expected '") + s + "'");
            next();
        }
        const Tok &expect(TokKind k, const char *what)
        {
            if (peek().kind != k) raise(SV_ERR_INVALID_ARG, peek().line, std::string("expected ") + what);
            return next();
        }
    };

    using Env = std::map<std::string, double>;

    // ---- expressions
    double expr(Cursor &c, const Env &env)
    {
        double v = term(c, env);
        while (c.is_sym("+") || c.is_sym("-")) {
            const bool add = c.next().text == "+";
            const double r = term(c, env);
            v = add ? v + r : v - r;
        }
        return v;
    }
    double term(Cursor &c, const Env &env)
    {
        double v = unary(c, env);
        while (c.is_sym("*") || c.is_sym("/")) {
            const bool mul = c.next().text == "*";
            const double r = unary(c, env);
            v = mul ? v * r : v / r;
        }
        return v;
    }
    double unary(Cursor &c, const Env &env)
    {
        if (c.is_sym("-")) {
            c.next();
            return -unary(c, env);
        }
        if (c.is_sym("+")) {
            c.next();
            return unary(c, env);
        }
        const double b = primary(c, env);
        if (c.is_sym("^")) {
            c.next();
            return std::pow(b, unary(c, env));  // right-associative
        }
        return b;
    }
    double primary(Cursor &c, const Env &env)
    {
        const Tok &t = c.next();
        if (t.kind == T_NUM) return t.num;
        if (t.kind == T_SYM && t.text == "(") {
            const double v = expr(c, env);
            c.sym(")");
            return v;
        }
        if (t.kind == T_ID) {
            if (t.text == "pi") return kPi;
            static const std::map<std::string, double (*)(double)> fn = {
                {"sin", [](double x) { return std::sin(x); }},  {"cos", [](double x) { return std::cos(x); }},
                {"tan", [](double x) { return std::tan(x); }},  {"exp", [](double x) { return std::exp(x); }},
                {"ln", [](double x) { return std::log(x); }},   {"sqrt", [](double x) { return std::sqrt(x); }}};
            auto f = fn.find(t.text);
            if (f != fn.end()) {
                c.sym("(");
                const double v = expr(c, env);
                c.sym(")");
                return f->second(v);
            }
            auto e = env.find(t.text);
            if (e != env.end()) return e->second;
            raise(SV_ERR_INVALID_ARG, t.line, "unknown identifier '" + t.text + "' in expression");
        }
        raise(SV_ERR_INVALID_ARG, t.line, "expected an expression");
    }

    // ---- statements
    void statement(Cursor &c)
    {
        const Tok &t = c.peek();
        if (t.kind != T_ID) raise(SV_ERR_INVALID_ARG, t.line, "expected a statement");
        const std::string &w = t.text;
        if (w == "include") {
            c.next();
            const Tok &f = c.expect(T_STR, "a file name");
            if (f.text != "qelib1.inc") raise(SV_ERR_UNSUPPORTED, f.line, "only qelib1.inc can be included");
            qelib_ = true;
            c.sym(";");
        } else if (w == "qreg" || w == "creg") {
            c.next();
            const Tok &name = c.expect(T_ID, "a register name");
            c.sym("[");
            const Tok &sz = c.expect(T_NUM, "a register size");
            if (!sz.integer || sz.num < 1 || sz.num > 4096) raise(SV_ERR_INVALID_ARG, sz.line, "bad register size");
            c.sym("]");
            c.sym(";");
            if (qregs_.count(name.text) || cregs_.count(name.text))
                raise(SV_ERR_INVALID_ARG, name.line, "register '" + name.text + "' declared twice");
            if (w == "qreg") {
                qregs_[name.text] = Reg{nq_, (int)sz.num};
                nq_ += (int)sz.num;
            } else {
                cregs_[name.text] = Reg{0, (int)sz.num};
            }
        } else if (w == "gate" || w == "opaque") {
            definition(c, w == "opaque");
        } else if (w == "measure") {
            c.next();
            auto q = arg(c, true);
            c.sym("->");
            auto b = arg(c, false);
            if (q.size() != b.size()) raise(SV_ERR_INVALID_ARG, t.line, "measure: register sizes differ");
            c.sym(";");
        } else if (w == "barrier") {
            c.next();
            arglist(c);
            c.sym(";");
        } else if (w == "reset") {
            raise(SV_ERR_UNSUPPORTED, t.line, "reset is not supported");
        } else if (w == "if") {
            raise(SV_ERR_UNSUPPORTED, t.line, "classically conditioned gates are not supported");
        } else {
            call(c, Env{}, nullptr, 0);
        }
    }

    // register or register[index] (qubit register when quantum), as qubit numbers
    std::vector<int> arg(Cursor &c, bool quantum)
    {
        const Tok &name = c.expect(T_ID, "a register");
        const auto &regs = quantum ? qregs_ : cregs_;
        auto r = regs.find(name.text);
        if (r == regs.end())
            raise(SV_ERR_INVALID_ARG, name.line,
                  std::string("unknown ") + (quantum ? "quantum" : "classical") + " register '" + name.text + "'");
        if (c.is_sym("[")) {
            c.next();
            const Tok &ix = c.expect(T_NUM, "an index");
            if (!ix.integer || ix.num < 0 || ix.num >= r->second.size)
                raise(SV_ERR_INVALID_ARG, ix.line, "index out of range for '" + name.text + "'");
            c.sym("]");
            return {r->second.offset + (int)ix.num};
        }
        std::vector<int> all(r->second.size);
        for (int i = 0; i < r->second.size; ++i) all[i] = r->second.offset + i;
        return all;
    }
    std::vector<std::vector<int>> arglist(Cursor &c)
    {
        std::vector<std::vector<int>> a;
        a.push_back(arg(c, true));
        while (c.is_sym(",")) {
            c.next();
            a.push_back(arg(c, true));
        }
        return a;
    }

    void definition(Cursor &c, bool opaque)
    {
        c.next();
        const Tok &name = c.expect(T_ID, "a gate name");
        if (defs_.count(name.text) || name.text == "U" || name.text == "CX" || (qelib_ && is_lib(name.text)))
            raise(SV_ERR_INVALID_ARG, name.line, "gate '" + name.text + "' already defined");
        GateDef d;
        d.opaque = opaque;
        if (c.is_sym("(")) {
            c.next();
            if (!c.is_sym(")")) {
                d.params.push_back(c.expect(T_ID, "a parameter name").text);
                while (c.is_sym(",")) {
                    c.next();
                    d.params.push_back(c.expect(T_ID, "a parameter name").text);
                }
            }
            c.sym(")");
        }
        d.args.push_back(c.expect(T_ID, "a qubit argument").text);
        while (c.is_sym(",")) {
            c.next();
            d.args.push_back(c.expect(T_ID, "a qubit argument").text);
        }
        for (size_t i = 0; i < d.args.size(); ++i)
            for (size_t j = 0; j < i; ++j)
                if (d.args[i] == d.args[j]) raise(SV_ERR_INVALID_ARG, name.line, "repeated gate argument");
        if (opaque) {
            c.sym(";");
        } else {
            c.sym("{");
            int depth = 1;
            while (true) {
                const Tok &t = c.next();
                if (t.kind == T_END) raise(SV_ERR_INVALID_ARG, name.line, "unterminated gate body");
                if (t.kind == T_SYM && t.text == "{") ++depth;
                if (t.kind == T_SYM && t.text == "}" && --depth == 0) break;
                d.body.push_back(t);
            }
        }
        defs_[name.text] = std::move(d);
    }

    // A gate call: at top level (qmap == nullptr) the arguments are registers
    // and broadcast; inside a body they are the definition's argument names.
    void call(Cursor &c, const Env &env, const std::map<std::string, int> *qmap, int depth)
    {
        const Tok &name = c.expect(T_ID, "a gate name");
        if (qmap && name.text == "barrier") {
            while (!c.is_sym(";")) c.next();
            c.sym(";");
            return;
        }
        std::vector<double> par;
        if (c.is_sym("(")) {
            c.next();
            if (!c.is_sym(")")) {
                par.push_back(expr(c, env));
                while (c.is_sym(",")) {
                    c.next();
                    par.push_back(expr(c, env));
                }
            }
            c.sym(")");
        }
        std::vector<std::vector<int>> qa;
        if (qmap) {
            do {
                if (!qa.empty()) c.next();
                const Tok &a = c.expect(T_ID, "a qubit argument");
                auto it = qmap->find(a.text);
                if (it == qmap->end()) raise(SV_ERR_INVALID_ARG, a.line, "unknown qubit argument '" + a.text + "'");
                qa.push_back({it->second});
            } while (c.is_sym(","));
        } else {
            qa = arglist(c);
        }
        c.sym(";");
        size_t width = 1;
        for (auto &a : qa)
            if (a.size() > 1) {
                if (width > 1 && a.size() != width) raise(SV_ERR_INVALID_ARG, name.line, "register sizes differ");
                width = a.size();
            }
        for (size_t k = 0; k < width; ++k) {
            std::vector<int> q;
            for (auto &a : qa) q.push_back(a.size() > 1 ? a[k] : a[0]);
            apply(name, par, q, depth);
        }
    }

    void apply(const Tok &name, const std::vector<double> &par, const std::vector<int> &q, int depth)
    {
        for (size_t i = 0; i < q.size(); ++i)
            for (size_t j = 0; j < i; ++j)
                if (q[i] == q[j]) raise(SV_ERR_INVALID_ARG, name.line, "repeated qubit in '" + name.text + "'");
        auto d = defs_.find(name.text);
        if (d != defs_.end()) {
            const GateDef &g = d->second;
            if (g.opaque) raise(SV_ERR_UNSUPPORTED, name.line, "opaque gate '" + name.text + "' has no definition");
            if (par.size() != g.params.size() || q.size() != g.args.size())
                raise(SV_ERR_INVALID_ARG, name.line, "wrong number of parameters or qubits for '" + name.text + "'");
            if (depth >= kMaxDepth) raise(SV_ERR_UNSUPPORTED, name.line, "gate definitions nest too deep");
            Env env;
            for (size_t i = 0; i < par.size(); ++i) env[g.params[i]] = par[i];
            std::map<std::string, int> qmap;
            for (size_t i = 0; i < q.size(); ++i) qmap[g.args[i]] = q[i];
            std::vector<Tok> body = g.body;
            Tok e;
            e.kind = T_END;
            e.line = name.line;
            body.push_back(e);
            Cursor bc{&body, 0};
            while (bc.peek().kind != T_END) call(bc, env, &qmap, depth + 1);
            return;
        }
        if (!builtin(name, par, q)) raise(SV_ERR_INVALID_ARG, name.line, "unknown gate '" + name.text + "'");
    }

    // ---- records
    void emit(int op, std::vector<int> t, std::vector<int> ctl, double theta = 0.0, const double *u = nullptr)
    {
        if (out_.size() >= kMaxGates) raise(SV_ERR_UNSUPPORTED, 0, "circuit too long");
        sv_gate_ex g;
        std::memset(&g, 0, sizeof g);
        g.op = op;
        g.ntargets = (int)t.size();
        g.ncontrols = (int)ctl.size();
        for (size_t i = 0; i < t.size(); ++i) g.targets[i] = t[i];
        for (size_t i = 0; i < ctl.size(); ++i) g.controls[i] = ctl[i];
        g.theta = theta;
        if (u) std::memcpy(g.u, u, sizeof g.u);
        g.uk = nullptr;
        out_.push_back(g);
    }
    static void u3(double th, double ph, double la, double gamma, double *u)
    {
        const double c = std::cos(0.5 * th), s = std::sin(0.5 * th);
        auto put = [&](int e, double mag, double ang) {
            u[2 * e] = mag * std::cos(ang);
            u[2 * e + 1] = mag * std::sin(ang);
        };
        put(0, c, gamma);
        put(1, -s, gamma + la);
        put(2, s, gamma + ph);
        put(3, c, gamma + ph + la);
    }
    static void sqrt_x(bool dagger, double *u)
    {
        // (1/2) [[1 + i, 1 - i], [1 - i, 1 + i]], or its adjoint
        const double sg = dagger ? -0.5 : 0.5;
        const double m[8] = {0.5, sg, 0.5, -sg, 0.5, -sg, 0.5, sg};
        std::memcpy(u, m, sizeof m);
    }

    static bool is_lib(const std::string &n)
    {
        static const char *names[] = {"u3", "u2", "u1", "u0", "u", "p", "cx", "id", "x", "y", "z", "h", "s", "sdg",
                                      "t", "tdg", "rx", "ry", "rz", "sx", "sxdg", "cz", "cy", "swap", "ch", "ccx",
                                      "cswap", "crx", "cry", "crz", "cu1", "cp", "cu3", "csx", "cu", "rxx", "rzz",
                                      "c3x", "c4x", "c3sqrtx", "rccx", "rc3x"};
        for (const char *x : names)
            if (n == x) return true;
        return false;
    }

    bool builtin(const Tok &name, const std::vector<double> &p, const std::vector<int> &q)
    {
        const std::string &n = name.text;
        auto need = [&](size_t np, size_t nqb) {
            if (p.size() != np || q.size() != nqb)
                raise(SV_ERR_INVALID_ARG, name.line, "wrong number of parameters or qubits for '" + n + "'");
        };
        double u[8];
        if (n == "U" || n == "CX") {
        } else if (!qelib_ || !is_lib(n)) {
            return false;
        }
        if (n == "U" || n == "u3" || n == "u") {
            need(3, 1);
            u3(p[0], p[1], p[2], 0.0, u);
            emit(SV_U2, {q[0]}, {}, 0.0, u);
        } else if (n == "u2") {
            need(2, 1);
            u3(0.5 * kPi, p[0], p[1], 0.0, u);
            emit(SV_U2, {q[0]}, {}, 0.0, u);
        } else if (n == "u1" || n == "p") {
            need(1, 1);
            emit(SV_P, {q[0]}, {}, p[0]);
        } else if (n == "u0") {
            need(1, 1);  // identity (an idle of the given length)
        } else if (n == "id") {
            need(0, 1);
        } else if (n == "CX" || n == "cx") {
            need(0, 2);
            emit(SV_X, {q[1]}, {q[0]});
        } else if (n == "x" || n == "y" || n == "z" || n == "h") {
            need(0, 1);
            emit(n == "x" ? SV_X : n == "y" ? SV_Y : n == "z" ? SV_Z : SV_H, {q[0]}, {});
        } else if (n == "s" || n == "sdg" || n == "t" || n == "tdg") {
            need(0, 1);
            const double a = (n[0] == 's' ? 0.5 : 0.25) * kPi;
            emit(SV_P, {q[0]}, {}, n.size() == 3 ? -a : a);
        } else if (n == "rx" || n == "ry" || n == "rz") {
            need(1, 1);
            emit(n == "rx" ? SV_RX : n == "ry" ? SV_RY : SV_RZ, {q[0]}, {}, p[0]);
        } else if (n == "sx" || n == "sxdg") {
            need(0, 1);
            sqrt_x(n == "sxdg", u);
            emit(SV_U2, {q[0]}, {}, 0.0, u);
        } else if (n == "cz" || n == "cy" || n == "ch") {
            need(0, 2);
            emit(n == "cz" ? SV_Z : n == "cy" ? SV_Y : SV_H, {q[1]}, {q[0]});
        } else if (n == "swap") {
            need(0, 2);
            emit(SV_SWAP, {q[0], q[1]}, {});
        } else if (n == "cswap") {
            need(0, 3);
            emit(SV_SWAP, {q[1], q[2]}, {q[0]});
        } else if (n == "ccx" || n == "c3x" || n == "c4x") {
            const size_t nc = n == "ccx" ? 2 : n == "c3x" ? 3 : 4;
            need(0, nc + 1);
            emit(SV_X, {q[nc]}, std::vector<int>(q.begin(), q.begin() + nc));
        } else if (n == "c3sqrtx") {
            need(0, 4);
            sqrt_x(false, u);
            emit(SV_U2, {q[3]}, {q[0], q[1], q[2]}, 0.0, u);
        } else if (n == "crx" || n == "cry" || n == "crz") {
            need(1, 2);
            emit(n == "crx" ? SV_RX : n == "cry" ? SV_RY : SV_RZ, {q[1]}, {q[0]}, p[0]);
        } else if (n == "cu1" || n == "cp") {
            need(1, 2);
            emit(SV_P, {q[1]}, {q[0]}, p[0]);
        } else if (n == "cu3") {
            need(3, 2);
            u3(p[0], p[1], p[2], 0.0, u);
            emit(SV_U2, {q[1]}, {q[0]}, 0.0, u);
        } else if (n == "cu") {
            need(4, 2);
            u3(p[0], p[1], p[2], p[3], u);
            emit(SV_U2, {q[1]}, {q[0]}, 0.0, u);
        } else if (n == "csx") {
            need(0, 2);
            sqrt_x(false, u);
            emit(SV_U2, {q[1]}, {q[0]}, 0.0, u);
        } else if (n == "rzz" || n == "rxx") {
            // exp(-i theta/2 Z(x)Z) = CX . (RZ(theta) on the second) . CX, and
            // conjugating by H on both qubits turns Z(x)Z into X(x)X
            need(1, 2);
            const bool xx = n == "rxx";
            if (xx) {
                emit(SV_H, {q[0]}, {});
                emit(SV_H, {q[1]}, {});
            }
            emit(SV_X, {q[1]}, {q[0]});
            emit(SV_RZ, {q[1]}, {}, p[0]);
            emit(SV_X, {q[1]}, {q[0]});
            if (xx) {
                emit(SV_H, {q[0]}, {});
                emit(SV_H, {q[1]}, {});
            }
        } else {
            raise(SV_ERR_UNSUPPORTED, name.line, "relative-phase gate '" + n + "' is not supported");
        }
        return true;
    }

    std::vector<sv_gate_ex> &out_;
    std::map<std::string, Reg> qregs_, cregs_;
    std::map<std::string, GateDef> defs_;
    bool qelib_ = false;
    int nq_ = 0;
};

}  // namespace

sv_status parse(const char *text, std::vector<sv_gate_ex> &out, int &nqubits, std::string &err)
{
    out.clear();
    nqubits = 0;
    try {
        Reader r(out);
        r.program(lex(text));
        nqubits = r.nqubits();
        return SV_OK;
    } catch (const Error &e) {
        err = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        err = "out of host memory while reading the program";
        return SV_ERR_OUT_OF_MEMORY;
    }
}

}  // namespace svq
