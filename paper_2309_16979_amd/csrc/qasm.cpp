// OpenQASM 2.0 importer: circuit text -> msv_gate list (host only).
//
// The paper presents the method as a module that state-vector simulators
// plug in (Sec. 1, modularity; Sec. 2, Qiskit / Cirq / UniQ backends); a
// circuit format those frameworks export is the natural way in. The subset
// read here is the language of OpenQASM 2.0: the header, `include` of the
// standard gate library (recognised by name, no file is read), qreg / creg,
// user `gate` definitions (expanded inline, parameters substituted),
// register broadcasting, parameter expressions (pi, + - * / ^, unary minus,
// sin cos tan exp ln sqrt), and the standard gates by their matrices as the
// language defines them:
//   U(t,p,l) = u3(t,p,l) = u(t,p,l) = [[cos t/2, -e^{il} sin t/2],
//                                      [e^{ip} sin t/2, e^{i(p+l)} cos t/2]]
//   u2(p,l) = u3(pi/2,p,l); u1(l) = p(l) = rz(l) = diag(1, e^{il})
//   (in OpenQASM 2.0, rz is u1: it differs from exp(-i l Z/2) by a global
//   phase); rx(t) = u3(t,-pi/2,pi/2) = exp(-i t X/2); ry(t) = u3(t,0,0);
//   x y z h s t, sdg = u1(-pi/2), tdg = u1(-pi/4), sx = sqrt(X), sxdg, id;
//   CX / cx, cz, cy, ch, swap, cu1 / cp, crz(l) = controlled diag(e^{-il/2},
//   e^{il/2}), crx, cry, cu3, rxx(t) = exp(-i t XX/2), rzz(t) =
//   exp(-i t ZZ/2); ccx and cswap through two-qubit gates (Barenco et al.
//   1995: a Toffoli is CV(b,t) CX(a,b) CV^dagger(b,t) CX(a,b) CV(a,t) with
//   V = sqrt(X)).
// `barrier` and `measure` are skipped (the simulator returns the state before
// measurement); `reset`, `if` and `opaque` are refused.
#include <cctype>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace msv {
namespace {

using cplx = std::complex<double>;
const double kPi = 3.14159265358979323846;

struct Tok {
    enum Kind { ID, NUM, STR, SYM, END } k;
    std::string s;
    double v = 0.0;
    int line = 0;
};

struct QErr {
    int code;
    std::string msg;
};

[[noreturn]] void qfail(int line, const std::string &m, int code = MSV_E_ARG)
{
    char buf[64];
    snprintf(buf, sizeof buf, "qasm line %d: ", line);
    throw QErr{code, buf + m};
}

std::vector<Tok> lex(const char *text)
{
    std::vector<Tok> out;
    int line = 1;
    const char *p = text;
    while (*p) {
        const char c = *p;
        if (c == '\n') { ++line; ++p; continue; }
        if (isspace((unsigned char)c)) { ++p; continue; }
        if (c == '/' && p[1] == '/') {
            while (*p && *p != '\n') ++p;
            continue;
        }
        Tok t;
        t.line = line;
        if (isalpha((unsigned char)c) || c == '_') {
            const char *b = p;
            while (isalnum((unsigned char)*p) || *p == '_') ++p;
            t.k = Tok::ID;
            t.s.assign(b, p);
        } else if (isdigit((unsigned char)c) || (c == '.' && isdigit((unsigned char)p[1]))) {
            char *e = nullptr;
            t.v = strtod(p, &e);
            t.k = Tok::NUM;
            t.s.assign(p, (size_t)(e - p));
            p = e;
        } else if (c == '"') {
            const char *b = ++p;
            while (*p && *p != '"' && *p != '\n') ++p;
            if (*p != '"') qfail(line, "unterminated string");
            t.k = Tok::STR;
            t.s.assign(b, p);
            ++p;
        } else if (c == '-' && p[1] == '>') {
            t.k = Tok::SYM;
            t.s = "->";
            p += 2;
        } else if (c == '=' && p[1] == '=') {
            t.k = Tok::SYM;
            t.s = "==";
            p += 2;
        } else if (strchr(";,()[]{}+-*/^", c)) {
            t.k = Tok::SYM;
            t.s = std::string(1, c);
            ++p;
        } else {
            qfail(line, std::string("unexpected character '") + c + "'");
        }
        out.push_back(t);
    }
    Tok e;
    e.k = Tok::END;
    e.line = line;
    out.push_back(e);
    return out;
}

// A gate call inside a user definition, kept as tokens of its parameter
// expressions and its argument names.
struct BodyCall {
    std::string name;
    std::vector<std::vector<Tok>> params;
    std::vector<std::string> args;
    int line;
};

struct GateDef {
    std::vector<std::string> params, args;
    std::vector<BodyCall> body;
};

struct Emitted {
    uint32_t kind;
    int q0, q1;
    double theta;
    int nmat;                   // 0, 8 (2x2) or 32 (4x4) doubles
    double m[32];
};

class Parser {
  public:
    explicit Parser(std::vector<Tok> t) : t_(std::move(t)) {}

    void run()
    {
        expect_id("OPENQASM");
        const Tok v = next();
        if (v.k != Tok::NUM || v.v != 2.0) qfail(v.line, "only OpenQASM 2.0 is read");
        expect_sym(";");
        while (peek().k != Tok::END) statement();
    }

    int n_qubits() const { return nq_; }
    const std::vector<Emitted> &gates() const { return out_; }

  private:
    std::vector<Tok> t_;
    size_t i_ = 0;
    std::map<std::string, std::pair<int, int>> qreg_;   // name -> (offset, size)
    std::map<std::string, int> creg_;
    std::map<std::string, GateDef> defs_;
    int nq_ = 0;
    std::vector<Emitted> out_;

    const Tok &peek() const { return t_[i_]; }
    Tok next() { return t_[i_ < t_.size() - 1 ? i_++ : i_]; }
    bool is_sym(const char *s) const { return peek().k == Tok::SYM && peek().s == s; }
    void expect_sym(const char *s)
    {
        const Tok t = next();
        if (t.k != Tok::SYM || t.s != s) qfail(t.line, std::string("expected '") + s + "'");
    }
    void expect_id(const char *s)
    {
        const Tok t = next();
        if (t.k != Tok::ID || t.s != s) qfail(t.line, std::string("expected '") + s + "'");
    }
    std::string ident()
    {
        const Tok t = next();
        if (t.k != Tok::ID) qfail(t.line, "expected a name");
        return t.s;
    }
    int integer()
    {
        const Tok t = next();
        if (t.k != Tok::NUM || t.v != std::floor(t.v) || t.v < 0 || t.v > 1e9) qfail(t.line, "expected an index");
        return (int)t.v;
    }

    // ---- expressions over a parameter environment
    double expr(const std::map<std::string, double> &env)
    {
        double v = term(env);
        while (is_sym("+") || is_sym("-")) {
            const bool add = next().s == "+";
            const double r = term(env);
            v = add ? v + r : v - r;
        }
        return v;
    }
    double term(const std::map<std::string, double> &env)
    {
        double v = power(env);
        while (is_sym("*") || is_sym("/")) {
            const bool mul = next().s == "*";
            const double r = power(env);
            v = mul ? v * r : v / r;
        }
        return v;
    }
    double power(const std::map<std::string, double> &env)
    {
        const double b = unary(env);
        if (is_sym("^")) {
            next();
            return std::pow(b, power(env));
        }
        return b;
    }
    double unary(const std::map<std::string, double> &env)
    {
        if (is_sym("-")) { next(); return -unary(env); }
        if (is_sym("+")) { next(); return unary(env); }
        return primary(env);
    }
    double primary(const std::map<std::string, double> &env)
    {
        const Tok t = next();
        if (t.k == Tok::NUM) return t.v;
        if (t.k == Tok::SYM && t.s == "(") {
            const double v = expr(env);
            expect_sym(")");
            return v;
        }
        if (t.k != Tok::ID) qfail(t.line, "bad expression");
        if (t.s == "pi") return kPi;
        static const char *fn[] = {"sin", "cos", "tan", "exp", "ln", "sqrt"};
        for (int f = 0; f < 6; ++f)
            if (t.s == fn[f]) {
                expect_sym("(");
                const double a = expr(env);
                expect_sym(")");
                switch (f) {
                case 0: return std::sin(a);
                case 1: return std::cos(a);
                case 2: return std::tan(a);
                case 3: return std::exp(a);
                case 4: return std::log(a);
                default: return std::sqrt(a);
                }
            }
        auto it = env.find(t.s);
        if (it == env.end()) qfail(t.line, "unknown parameter '" + t.s + "'");
        return it->second;
    }
    // parameter list `( e, e, ... )` evaluated now (top level) or kept as tokens (definitions)
    std::vector<double> params_now(const std::map<std::string, double> &env)
    {
        std::vector<double> v;
        if (!is_sym("(")) return v;
        next();
        if (is_sym(")")) { next(); return v; }
        for (;;) {
            v.push_back(expr(env));
            if (is_sym(",")) { next(); continue; }
            expect_sym(")");
            return v;
        }
    }
    std::vector<std::vector<Tok>> params_tokens()
    {
        std::vector<std::vector<Tok>> v;
        if (!is_sym("(")) return v;
        next();
        if (is_sym(")")) { next(); return v; }
        std::vector<Tok> cur;
        int depth = 0;
        for (;;) {
            const Tok t = next();
            if (t.k == Tok::END) qfail(t.line, "unterminated parameter list");
            if (t.k == Tok::SYM && t.s == "(") ++depth;
            if (t.k == Tok::SYM && t.s == ")" && depth-- == 0) {
                v.push_back(cur);
                return v;
            }
            if (t.k == Tok::SYM && t.s == "," && depth == 0) {
                v.push_back(cur);
                cur.clear();
                continue;
            }
            cur.push_back(t);
        }
    }
    double eval_tokens(const std::vector<Tok> &toks, const std::map<std::string, double> &env, int line)
    {
        if (toks.empty()) qfail(line, "empty parameter");
        Parser sub(toks);
        Tok e;
        e.k = Tok::END;
        e.line = line;
        sub.t_.push_back(e);
        const double v = sub.expr(env);
        if (sub.peek().k != Tok::END) qfail(line, "bad parameter expression");
        return v;
    }

    // ---- statements
    void statement()
    {
        const Tok t = peek();
        if (t.k != Tok::ID) qfail(t.line, "expected a statement");
        if (t.s == "include") {
            next();
            const Tok f = next();
            if (f.k != Tok::STR || f.s != "qelib1.inc") qfail(f.line, "only the standard gate library can be included");
            expect_sym(";");
        } else if (t.s == "qreg" || t.s == "creg") {
            next();
            const std::string name = ident();
            expect_sym("[");
            const int size = integer();
            expect_sym("]");
            expect_sym(";");
            if (qreg_.count(name) || creg_.count(name)) qfail(t.line, "register '" + name + "' declared twice");
            if (t.s == "qreg") {
                if (size < 1 || nq_ + size > 64) qfail(t.line, "qubit count out of range");
                qreg_[name] = {nq_, size};
                nq_ += size;
            } else {
                creg_[name] = size;
            }
        } else if (t.s == "gate") {
            next();
            define();
        } else if (t.s == "barrier") {
            while (!is_sym(";") && peek().k != Tok::END) next();
            expect_sym(";");
        } else if (t.s == "measure") {
            // the state before measurement is what the simulator returns
            while (!is_sym(";") && peek().k != Tok::END) next();
            expect_sym(";");
        } else if (t.s == "reset" || t.s == "if" || t.s == "opaque") {
            qfail(t.line, "'" + t.s + "' is not supported (a pass applies unitary gates only)", MSV_E_UNSUPPORTED);
        } else {
            apply_top();
        }
    }

    void define()
    {
        const int line = peek().line;
        const std::string name = ident();
        GateDef d;
        if (is_sym("(")) {
            next();
            if (!is_sym(")"))
                for (;;) {
                    d.params.push_back(ident());
                    if (is_sym(",")) { next(); continue; }
                    break;
                }
            expect_sym(")");
        }
        for (;;) {
            d.args.push_back(ident());
            if (is_sym(",")) { next(); continue; }
            break;
        }
        expect_sym("{");
        while (!is_sym("}")) {
            if (peek().k == Tok::END) qfail(line, "unterminated gate body");
            BodyCall c;
            c.line = peek().line;
            c.name = ident();
            if (c.name == "barrier") {
                while (!is_sym(";")) next();
                expect_sym(";");
                continue;
            }
            c.params = params_tokens();
            for (;;) {
                c.args.push_back(ident());
                if (is_sym(",")) { next(); continue; }
                break;
            }
            expect_sym(";");
            d.body.push_back(c);
        }
        expect_sym("}");
        defs_[name] = d;
    }

    // one operand of a top-level call: a qubit, or every qubit of a register
    std::vector<int> operand()
    {
        const Tok t = peek();
        const std::string name = ident();
        auto it = qreg_.find(name);
        if (it == qreg_.end()) qfail(t.line, "unknown quantum register '" + name + "'");
        if (is_sym("[")) {
            next();
            const int i = integer();
            expect_sym("]");
            if (i >= it->second.second) qfail(t.line, "index beyond register '" + name + "'");
            return {it->second.first + i};
        }
        std::vector<int> all;
        for (int i = 0; i < it->second.second; ++i) all.push_back(it->second.first + i);
        return all;
    }

    void apply_top()
    {
        const int line = peek().line;
        const std::string name = ident();
        const std::vector<double> ps = params_now({});
        std::vector<std::vector<int>> ops;
        for (;;) {
            ops.push_back(operand());
            if (is_sym(",")) { next(); continue; }
            break;
        }
        expect_sym(";");
        size_t width = 1;
        for (auto &o : ops)
            if (o.size() > 1) {
                if (width > 1 && o.size() != width) qfail(line, "registers of different sizes");
                width = o.size();
            }
        for (size_t j = 0; j < width; ++j) {
            std::vector<int> q;
            for (auto &o : ops) q.push_back(o.size() > 1 ? o[j] : o[0]);
            call(name, ps, q, line, 0);
        }
    }

    void call(const std::string &name, const std::vector<double> &ps, const std::vector<int> &q, int line, int depth)
    {
        if (depth > 64) qfail(line, "gate definitions nest too deeply");
        for (size_t a = 0; a < q.size(); ++a)
            for (size_t b = a + 1; b < q.size(); ++b)
                if (q[a] == q[b]) qfail(line, "repeated qubit in '" + name + "'");
        auto d = defs_.find(name);
        if (d != defs_.end()) {
            const GateDef &g = d->second;
            if (ps.size() != g.params.size() || q.size() != g.args.size())
                qfail(line, "wrong parameter or qubit count for '" + name + "'");
            std::map<std::string, double> env;
            for (size_t k = 0; k < ps.size(); ++k) env[g.params[k]] = ps[k];
            std::map<std::string, int> qa;
            for (size_t k = 0; k < q.size(); ++k) qa[g.args[k]] = q[k];
            for (const BodyCall &c : g.body) {
                std::vector<double> cp;
                for (auto &toks : c.params) cp.push_back(eval_tokens(toks, env, c.line));
                std::vector<int> cq;
                for (auto &a : c.args) {
                    auto it = qa.find(a);
                    if (it == qa.end()) qfail(c.line, "unknown gate argument '" + a + "'");
                    cq.push_back(it->second);
                }
                call(c.name, cp, cq, c.line, depth + 1);
            }
            return;
        }
        builtin(name, ps, q, line);
    }

    // ---- standard gates
    void need(const std::string &name, const std::vector<double> &ps, const std::vector<int> &q, size_t np,
              size_t nq, int line)
    {
        if (ps.size() != np || q.size() != nq) qfail(line, "wrong parameter or qubit count for '" + name + "'");
    }
    void emit(uint32_t kind, int q0, int q1 = -1, double theta = 0.0)
    {
        Emitted e{};
        e.kind = kind;
        e.q0 = q0;
        e.q1 = q1;
        e.theta = theta;
        out_.push_back(e);
    }
    void emit1(int q, const cplx U[4])
    {
        Emitted e{};
        e.kind = MSV_U1;
        e.q0 = q;
        e.q1 = -1;
        e.nmat = 8;
        for (int k = 0; k < 4; ++k) { e.m[2 * k] = U[k].real(); e.m[2 * k + 1] = U[k].imag(); }
        out_.push_back(e);
    }
    // 4x4 matrix on (q0, q1), row-major, index s = b(q0) + 2 b(q1)
    void emit2(int q0, int q1, const cplx M[16])
    {
        Emitted e{};
        e.kind = MSV_U2;
        e.q0 = q0;
        e.q1 = q1;
        e.nmat = 32;
        for (int k = 0; k < 16; ++k) { e.m[2 * k] = M[k].real(); e.m[2 * k + 1] = M[k].imag(); }
        out_.push_back(e);
    }
    // controlled U: control c, target t (matrix qubits (t, c): the control is
    // the high index bit)
    void emit_controlled(int c, int t, const cplx U[4])
    {
        cplx M[16] = {};
        M[0] = M[5] = 1.0;
        M[10] = U[0];
        M[11] = U[1];
        M[14] = U[2];
        M[15] = U[3];
        emit2(t, c, M);
    }
    static void u3(double th, double ph, double la, cplx U[4])
    {
        const double c = std::cos(th / 2), s = std::sin(th / 2);
        U[0] = c;
        U[1] = -std::polar(1.0, la) * s;
        U[2] = std::polar(1.0, ph) * s;
        U[3] = std::polar(1.0, ph + la) * c;
    }
    static void sqrt_x(bool dagger, cplx V[4])
    {
        const cplx a(0.5, dagger ? -0.5 : 0.5), b(0.5, dagger ? 0.5 : -0.5);
        V[0] = a; V[1] = b; V[2] = b; V[3] = a;
    }
    void toffoli(int a, int b, int t)
    {
        cplx V[4], Vd[4];
        sqrt_x(false, V);
        sqrt_x(true, Vd);
        emit_controlled(b, t, V);
        emit(MSV_CX, a, b);
        emit_controlled(b, t, Vd);
        emit(MSV_CX, a, b);
        emit_controlled(a, t, V);
    }

    void builtin(const std::string &n, const std::vector<double> &ps, const std::vector<int> &q, int line)
    {
        cplx U[4];
        if (n == "U" || n == "u3" || n == "u") {
            need(n, ps, q, 3, 1, line);
            u3(ps[0], ps[1], ps[2], U);
            emit1(q[0], U);
        } else if (n == "u2") {
            need(n, ps, q, 2, 1, line);
            u3(kPi / 2, ps[0], ps[1], U);
            emit1(q[0], U);
        } else if (n == "u1" || n == "p" || n == "rz") {
            need(n, ps, q, 1, 1, line);
            emit(MSV_P, q[0], -1, ps[0]);
        } else if (n == "CX" || n == "cx") {
            need(n, ps, q, 0, 2, line);
            emit(MSV_CX, q[0], q[1]);
        } else if (n == "id") {
            need(n, ps, q, 0, 1, line);
        } else if (n == "x" || n == "y" || n == "z" || n == "h" || n == "s" || n == "t") {
            need(n, ps, q, 0, 1, line);
            const uint32_t k = n == "x" ? MSV_X : n == "y" ? MSV_Y : n == "z" ? MSV_Z : n == "h" ? MSV_H
                                                                            : n == "s" ? MSV_S : MSV_T;
            emit(k, q[0]);
        } else if (n == "sdg" || n == "tdg") {
            need(n, ps, q, 0, 1, line);
            emit(MSV_P, q[0], -1, n == "sdg" ? -kPi / 2 : -kPi / 4);
        } else if (n == "sx" || n == "sxdg") {
            need(n, ps, q, 0, 1, line);
            sqrt_x(n == "sxdg", U);
            emit1(q[0], U);
        } else if (n == "rx" || n == "ry") {
            need(n, ps, q, 1, 1, line);
            emit(n == "rx" ? MSV_RX : MSV_RY, q[0], -1, ps[0]);
        } else if (n == "cz" || n == "swap") {
            need(n, ps, q, 0, 2, line);
            emit(n == "cz" ? MSV_CZ : MSV_SWAP, q[0], q[1]);
        } else if (n == "cu1" || n == "cp") {
            need(n, ps, q, 1, 2, line);
            emit(MSV_CP, q[0], q[1], ps[0]);
        } else if (n == "cy" || n == "ch") {
            need(n, ps, q, 0, 2, line);
            if (n == "cy") { U[0] = 0.0; U[1] = cplx(0, -1); U[2] = cplx(0, 1); U[3] = 0.0; }
            else { const double r = 1.0 / std::sqrt(2.0); U[0] = r; U[1] = r; U[2] = r; U[3] = -r; }
            emit_controlled(q[0], q[1], U);
        } else if (n == "crz") {
            need(n, ps, q, 1, 2, line);
            U[0] = std::polar(1.0, -ps[0] / 2);
            U[1] = U[2] = 0.0;
            U[3] = std::polar(1.0, ps[0] / 2);
            emit_controlled(q[0], q[1], U);
        } else if (n == "crx" || n == "cry") {
            need(n, ps, q, 1, 2, line);
            const double c = std::cos(ps[0] / 2), s = std::sin(ps[0] / 2);
            if (n == "crx") { U[0] = c; U[1] = cplx(0, -s); U[2] = cplx(0, -s); U[3] = c; }
            else { U[0] = c; U[1] = -s; U[2] = s; U[3] = c; }
            emit_controlled(q[0], q[1], U);
        } else if (n == "cu3") {
            need(n, ps, q, 3, 2, line);
            u3(ps[0], ps[1], ps[2], U);
            emit_controlled(q[0], q[1], U);
        } else if (n == "rxx" || n == "rzz") {
            need(n, ps, q, 1, 2, line);
            const double c = std::cos(ps[0] / 2), s = std::sin(ps[0] / 2);
            cplx M[16] = {};
            if (n == "rzz") {
                // exp(-i t ZZ/2): phase e^{-it/2} where the bits agree, e^{it/2} where they differ
                M[0] = M[15] = std::polar(1.0, -ps[0] / 2);
                M[5] = M[10] = std::polar(1.0, ps[0] / 2);
            } else {
                // exp(-i t XX/2) = cos(t/2) I - i sin(t/2) XX; XX maps s to 3 - s
                for (int r = 0; r < 4; ++r) {
                    M[5 * r] = c;
                    M[4 * r + (3 - r)] = cplx(0, -s);
                }
            }
            emit2(q[0], q[1], M);
        } else if (n == "ccx") {
            need(n, ps, q, 0, 3, line);
            toffoli(q[0], q[1], q[2]);
        } else if (n == "cswap") {
            need(n, ps, q, 0, 3, line);
            emit(MSV_CX, q[2], q[1]);
            toffoli(q[0], q[1], q[2]);
            emit(MSV_CX, q[2], q[1]);
        } else {
            qfail(line, "unknown gate '" + n + "'");
        }
    }
};

}  // namespace
}  // namespace msv

using namespace msv;

extern "C" int msv_qasm_parse(const char *text, int *n_qubits, msv_gate *gates, size_t gate_cap, size_t *n_gates,
                              double *mats, size_t mat_cap, size_t *n_mat)
{
    if (!text || !n_qubits || !n_gates || !n_mat) return fail_global(MSV_E_ARG, "msv_qasm_parse: null argument");
    try {
        Parser p(lex(text));
        p.run();
        const std::vector<Emitted> &g = p.gates();
        size_t need_m = 0;
        for (const Emitted &e : g) need_m += (size_t)e.nmat;
        *n_qubits = p.n_qubits();
        *n_gates = g.size();
        *n_mat = need_m;
        if (!gates && !mats) return MSV_OK;   // sizing call
        if (!gates || gate_cap < g.size() || (need_m && (!mats || mat_cap < need_m)))
            return fail_global(MSV_E_ARG, "msv_qasm_parse: output buffers too small");
        size_t m = 0;
        for (size_t i = 0; i < g.size(); ++i) {
            const Emitted &e = g[i];
            gates[i] = msv_gate{e.kind, e.q0, e.q1, e.theta, -1, nullptr};
            if (e.nmat) {
                memcpy(mats + m, e.m, sizeof(double) * (size_t)e.nmat);
                gates[i].mat = mats + m;
                m += (size_t)e.nmat;
            }
        }
        return MSV_OK;
    } catch (const QErr &e) {
        return fail_global(e.code, e.msg.c_str());
    } catch (const std::exception &e) {
        return fail_global(MSV_E_ARG, e.what());
    }
}
