#include "planner.h"

#include <algorithm>
#include <cmath>

namespace msv {

namespace {

const double kPi = 3.14159265358979323846;

cd expi(double a) { return cd(std::cos(a), std::sin(a)); }

bool is_diagonal(const std::vector<cd> &m, int d)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && m[r * d + c] != cd(0.0)) return false;
    return true;
}

std::vector<cd> dagger(const std::vector<cd> &m, int d)
{
    std::vector<cd> o(d * d);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) o[c * d + r] = std::conj(m[r * d + c]);
    return o;
}

// Matrix of a k-qubit op (qubits q, D x D) embedded on the ordered qubit list Q
// (a superset of q).
std::vector<cd> embed(const std::vector<int> &q, const std::vector<cd> &m, const std::vector<int> &Q)
{
    const int k = (int)q.size(), K = (int)Q.size(), d = 1 << k, D = 1 << K;
    std::vector<int> at(k);
    int qmask = 0;
    for (int i = 0; i < k; ++i) {
        at[i] = (int)(std::find(Q.begin(), Q.end(), q[i]) - Q.begin());
        qmask |= 1 << at[i];
    }
    auto sub = [&](int s) {
        int v = 0;
        for (int i = 0; i < k; ++i) v |= ((s >> at[i]) & 1) << i;
        return v;
    };
    std::vector<cd> e((size_t)D * D, cd(0.0));
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if ((r & ~qmask) == (c & ~qmask)) e[(size_t)r * D + c] = m[sub(r) * d + sub(c)];
    return e;
}

std::vector<cd> matmul(const std::vector<cd> &a, const std::vector<cd> &b, int D)
{
    std::vector<cd> o((size_t)D * D, cd(0.0));
    for (int r = 0; r < D; ++r)
        for (int k = 0; k < D; ++k) {
            const cd x = a[(size_t)r * D + k];
            if (x == cd(0.0)) continue;
            for (int c = 0; c < D; ++c) o[(size_t)r * D + c] += x * b[(size_t)k * D + c];
        }
    return o;
}

std::vector<int> unite(const std::vector<int> &a, const std::vector<int> &b)
{
    std::vector<int> o = a;
    for (int x : b)
        if (std::find(o.begin(), o.end(), x) == o.end()) o.push_back(x);
    return o;
}

bool subset(const std::vector<int> &a, const std::vector<int> &b)
{
    for (int x : a)
        if (std::find(b.begin(), b.end(), x) == b.end()) return false;
    return true;
}

}  // namespace

int gate_to_prim(const msv_gate &g, int n, bool inverse, Prim &p, std::string &err)
{
    const bool two = g.kind == MSV_CX || g.kind == MSV_CZ || g.kind == MSV_CP || g.kind == MSV_SWAP ||
                     g.kind == MSV_U2;
    if (g.kind > MSV_U2) { err = "unknown gate kind"; return MSV_E_ARG; }
    if (g.q0 < 0 || g.q0 >= n) { err = "qubit out of range"; return MSV_E_ARG; }
    if (two && (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0)) { err = "bad second qubit"; return MSV_E_ARG; }
    if ((g.kind == MSV_U1 || g.kind == MSV_U2) && !g.mat) { err = "U1/U2 gate without matrix"; return MSV_E_ARG; }
    if (!std::isfinite(g.theta)) { err = "non-finite angle"; return MSV_E_RANGE; }
    p = Prim();
    p.param = g.param;
    p.kind = (int)g.kind;
    const double t = g.theta, c = std::cos(t / 2), s = std::sin(t / 2), h = 1.0 / std::sqrt(2.0);
    const cd I(0.0, 1.0);
    switch (g.kind) {
    case MSV_H: p.q = {g.q0}; p.m = {h, h, h, -h}; break;
    case MSV_X: p.q = {g.q0}; p.m = {0.0, 1.0, 1.0, 0.0}; break;
    case MSV_Y: p.q = {g.q0}; p.m = {0.0, -I, I, 0.0}; break;
    case MSV_RX: p.q = {g.q0}; p.m = {c, -I * s, -I * s, c}; break;
    case MSV_RY: p.q = {g.q0}; p.m = {c, -s, s, c}; break;
    case MSV_U1:
        p.q = {g.q0};
        p.m.resize(4);
        for (int i = 0; i < 4; ++i) p.m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
        break;
    case MSV_Z: p.diag = true; p.q = {g.q0}; p.m = {1.0, -1.0}; break;
    case MSV_S: p.diag = true; p.q = {g.q0}; p.m = {1.0, I}; break;
    case MSV_T: p.diag = true; p.q = {g.q0}; p.m = {1.0, expi(kPi / 4)}; break;
    case MSV_RZ: p.diag = true; p.q = {g.q0}; p.m = {expi(-t / 2), expi(t / 2)}; break;
    case MSV_P: p.diag = true; p.q = {g.q0}; p.m = {1.0, expi(t)}; break;
    case MSV_CX: p.q = {g.q1}; p.ctrl = g.q0; p.m = {0.0, 1.0, 1.0, 0.0}; break;
    case MSV_CZ: p.diag = true; p.q = {g.q0, g.q1}; p.m = {1.0, 1.0, 1.0, -1.0}; break;
    case MSV_CP: p.diag = true; p.q = {g.q0, g.q1}; p.m = {1.0, 1.0, 1.0, expi(t)}; break;
    case MSV_SWAP:
        p.q = {g.q0, g.q1};
        p.m.assign(16, 0.0);
        p.m[0] = p.m[1 * 4 + 2] = p.m[2 * 4 + 1] = p.m[15] = 1.0;
        break;
    case MSV_U2:
        p.q = {g.q0, g.q1};
        p.m.resize(16);
        for (int i = 0; i < 16; ++i) p.m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
        break;
    default: err = "unknown gate kind"; return MSV_E_ARG;
    }
    for (const cd &v : p.m)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) { err = "non-finite matrix"; return MSV_E_RANGE; }
    const int d = 1 << (int)p.q.size();
    if (!p.diag && p.ctrl < 0 && is_diagonal(p.m, d)) {
        std::vector<cd> dv(d);
        for (int i = 0; i < d; ++i) dv[i] = p.m[i * d + i];
        p.m = dv;
        p.diag = true;
    }
    if (inverse) {
        if (p.diag)
            for (cd &v : p.m) v = std::conj(v);
        else
            p.m = dagger(p.m, d);
    }
    return MSV_OK;
}

namespace {

// Accumulates the ops of one pass, fusing as it goes.
struct Fuser {
    const PlanOptions &o;
    const std::vector<int> &local;   // tile qubits of the pass
    std::vector<HostOp> out;
    enum { NONE, DENSE, DIAGS } open = NONE;
    std::vector<int> Q;
    std::vector<cd> M;
    std::vector<Prim> diags;          // pending diagonal prims
    // The pending run's qubits, and its controlled-linear-phase form built up
    // one prim at a time (phase_ok false once a prim does not fit it), so
    // that testing one more prim costs O(1) instead of a pass over the run.
    uint64_t diag_mask = 0;
    struct PhaseAcc {
        HostOp op;
        int pend_a = -1, pend_b = -1;
        double pend_g = 0.0;
    } acc;
    bool phase_ok = false;

    Fuser(const PlanOptions &opt, const std::vector<int> &loc) : o(opt), local(loc) {}

    bool is_local(int q) const { return std::find(local.begin(), local.end(), q) != local.end(); }

    void flush_dense()
    {
        HostOp op;
        op.type = OP_DENSE;
        op.q = Q;
        op.m = M;
        out.push_back(op);
        open = NONE;
    }

    // A pending run of diagonal gates as a table over <= 5 qubits, or as a
    // controlled linear phase; returns false when neither fits.
    static bool diag_union(const std::vector<Prim> &ds, std::vector<int> &U)
    {
        U.clear();
        for (const Prim &p : ds) U = unite(U, p.q);
        return U.size() <= 5;
    }

    void phase_start(PhaseAcc &a) const
    {
        a = PhaseAcc();
        a.op.type = OP_PHASE;
        a.op.mu.assign(o.n, 0.0);
        a.op.lam.assign(o.n, 0.0);
    }

    // One more diagonal prim in the controlled-linear-phase form; false when
    // it does not fit (a's contents are then undefined).
    static bool phase_add(PhaseAcc &a, const Prim &p)
    {
        HostOp &op = a.op;
        if (p.q.size() == 1) {
            op.global *= p.m[0];
            op.mu[p.q[0]] += std::arg(p.m[1] / p.m[0]);
            return true;
        }
        const int x = p.q[0], y = p.q[1];
        const cd d0 = p.m[0], d1 = p.m[1], d2 = p.m[2], d3 = p.m[3];
        op.global *= d0;
        op.mu[x] += std::arg(d1 / d0);
        op.mu[y] += std::arg(d2 / d0);
        const double gam = std::arg(d3 * d0 / (d1 * d2));
        if (gam == 0.0) return true;
        if (op.hub < 0 && a.pend_a < 0) {
            a.pend_a = x;
            a.pend_b = y;
            a.pend_g = gam;
            return true;
        }
        if (op.hub < 0) {
            if (x == a.pend_a || x == a.pend_b) op.hub = x;
            else if (y == a.pend_a || y == a.pend_b) op.hub = y;
            else return false;
            op.lam[op.hub == a.pend_a ? a.pend_b : a.pend_a] += a.pend_g;
        }
        if (x == op.hub) op.lam[y] += gam;
        else if (y == op.hub) op.lam[x] += gam;
        else return false;
        return true;
    }

    // The finished form: a lone pending pair takes its second qubit as hub.
    static void phase_finish(PhaseAcc &a)
    {
        if (a.op.hub < 0 && a.pend_a >= 0) {
            a.op.hub = a.pend_b;
            a.op.lam[a.pend_a] += a.pend_g;
        }
    }

    bool phase_form(const std::vector<Prim> &ds, HostOp &op) const
    {
        PhaseAcc a;
        phase_start(a);
        for (const Prim &p : ds)
            if (!phase_add(a, p)) return false;
        phase_finish(a);
        op = a.op;
        return true;
    }

    static uint64_t mask_of(const Prim &p)
    {
        uint64_t m = 0;
        for (int q : p.q) m |= 1ull << q;
        return m;
    }

    // Start a run of diagonal prims with p.
    void diags_begin(const Prim &p)
    {
        diags.clear();
        diags.push_back(p);
        diag_mask = mask_of(p);
        phase_start(acc);
        phase_ok = phase_add(acc, p);
        open = DIAGS;
    }

    // Add p to the pending run if the extended run still fits a table over
    // <= 5 qubits or the controlled-linear-phase form (the test on the
    // whole extended run, without a pass over it).
    bool diags_try(const Prim &p)
    {
        const uint64_t m = diag_mask | mask_of(p);
        bool ph = false;
        PhaseAcc next;
        if (phase_ok) {
            next = acc;
            ph = phase_add(next, p);
        }
        if (__builtin_popcountll(m) > 5 && !ph) return false;
        diags.push_back(p);
        diag_mask = m;
        phase_ok = ph;
        if (ph) acc = std::move(next);
        return true;
    }

    void flush_diags()
    {
        std::vector<int> U;
        if (diag_union(diags, U)) {
            // explicit table over U
            const int k = (int)U.size(), D = 1 << k;
            std::vector<cd> t(D, cd(1.0));
            for (const Prim &p : diags) {
                std::vector<int> at;
                for (int q : p.q) at.push_back((int)(std::find(U.begin(), U.end(), q) - U.begin()));
                for (int s = 0; s < D; ++s) {
                    int v = 0;
                    for (size_t i = 0; i < at.size(); ++i) v |= ((s >> at[i]) & 1) << i;
                    t[s] *= p.m[v];
                }
            }
            HostOp op;
            op.type = OP_DIAG;
            op.q = U;
            op.m = t;
            out.push_back(op);
        } else {
            HostOp op;
            phase_form(diags, op);
            out.push_back(op);
        }
        diags.clear();
        open = NONE;
    }

    void flush()
    {
        if (open == DENSE) flush_dense();
        else if (open == DIAGS) flush_diags();
    }

    void add(const Prim &p)
    {
        if (p.probe || p.obs) {
            flush();
            HostOp op;
            op.type = p.obs ? OP_OBS : OP_GRAD;
            op.q = p.q;
            op.m = p.m;
            op.slot = p.slot;
            op.diag = p.diag;
            out.push_back(op);
            return;
        }
        if (p.diag) {
            if (open == DENSE && subset(p.q, Q)) {
                std::vector<cd> dm((size_t)1 << (2 * p.q.size()), cd(0.0));
                const int d = 1 << (int)p.q.size();
                for (int i = 0; i < d; ++i) dm[(size_t)i * d + i] = p.m[i];
                M = matmul(embed(p.q, dm, Q), M, 1 << (int)Q.size());
                return;
            }
            if (open == DIAGS) {
                if (diags_try(p)) return;
                flush_diags();
            } else {
                flush();
            }
            diags_begin(p);
            return;
        }
        std::vector<int> qs = p.q;
        std::vector<cd> m = p.m;
        if (p.ctrl >= 0) {
            if (!is_local(p.ctrl)) {
                flush();
                HostOp op;
                op.type = OP_DENSE;
                op.q = p.q;
                op.m = p.m;
                op.ctrl_mask = 1ull << p.ctrl;
                out.push_back(op);
                return;
            }
            // controlled 1q U on target with local control: 4x4 on (ctrl, target)
            qs = {p.ctrl, p.q[0]};
            m.assign(16, 0.0);
            m[0] = 1.0;                       // s = 0: ctrl 0, target 0
            m[2 * 4 + 2] = 1.0;               // s = 2: ctrl 0, target 1
            m[1 * 4 + 1] = p.m[0];            // ctrl 1: U on target bit (s = 1, 3)
            m[1 * 4 + 3] = p.m[1];
            m[3 * 4 + 1] = p.m[2];
            m[3 * 4 + 3] = p.m[3];
        }
        if (open == DENSE) {
            std::vector<int> U = unite(Q, qs);
            if ((int)U.size() <= std::max(o.k_max, (int)qs.size()) && (int)U.size() <= kMaxFuse) {
                const int D = 1 << (int)U.size();
                M = matmul(embed(qs, m, U), embed(Q, M, U), D);
                Q = U;
                return;
            }
        }
        flush();
        Q = qs;
        M = m;
        open = DENSE;
    }
};

}  // namespace

std::vector<Prim> relabel_swaps(const std::vector<Prim> &prims, int n, std::vector<int> &pos)
{
    pos.resize(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    std::vector<Prim> out;
    out.reserve(prims.size());
    for (const Prim &p : prims) {
        if (p.kind == MSV_SWAP && p.ctrl < 0 && !p.probe && !p.obs && p.q.size() == 2 && pos[p.q[0]] >= 6 &&
            pos[p.q[1]] >= 6) {
            std::swap(pos[p.q[0]], pos[p.q[1]]);
            continue;
        }
        Prim r = p;
        for (int &q : r.q) q = pos[q];
        if (r.ctrl >= 0) r.ctrl = pos[r.ctrl];
        out.push_back(std::move(r));
    }
    return out;
}

void restore_order(std::vector<Pass> &passes, const std::vector<int> &pos, const PlanOptions &o)
{
    bool ident = true;
    for (int q = 0; q < (int)pos.size(); ++q) ident &= pos[q] == q;
    if (ident) return;
    if (passes.empty()) {
        Pass ps;
        for (int q = 0; q < o.tb; ++q) ps.tile_q.push_back(q);
        passes.push_back(ps);
    }
    // the qubit stored at position pos[q] goes back to position q
    std::vector<int> &oq = passes.back().out_q;
    oq.assign(pos.size(), 0);
    for (int q = 0; q < (int)pos.size(); ++q) oq[pos[q]] = q;
}

std::vector<Pass> plan_passes(const std::vector<Prim> &prims, const PlanOptions &o)
{
    std::vector<Pass> passes;
    const int tb = o.tb;
    // Qubit masks: q (the dense / diagonal qubits) and support (q and control).
    std::vector<uint64_t> qm(prims.size()), sm(prims.size());
    for (size_t i = 0; i < prims.size(); ++i) {
        uint64_t m = 0;
        for (int q : prims[i].q) m |= 1ull << q;
        qm[i] = m;
        sm[i] = prims[i].ctrl >= 0 ? m | (1ull << prims[i].ctrl) : m;
    }
    // Gates not yet placed, in list order. Each pass takes every gate that
    // fits the tile and commutes with all gates deferred before it in this
    // pass, scanning a bounded window ahead of the first deferred gate. Two
    // gates are taken to commute when their supports (targets and control)
    // are disjoint, when both are diagonal, or when one is diagonal on qubits
    // the other does not transform; probes and observables commute with
    // nothing. Against every deferred gate at once this reduces to unions of
    // the deferred gates' masks: a diagonal p must avoid the targets of the
    // deferred dense gates; a dense p must avoid their supports and the
    // qubits of the deferred diagonals.
    std::vector<size_t> rest(prims.size());
    for (size_t i = 0; i < prims.size(); ++i) rest[i] = i;
    const size_t window = (size_t)std::max(0, o.lookahead);
    const uint64_t low6 = o.n >= 6 ? 63ull : ((1ull << o.n) - 1);
    while (!rest.empty()) {
        uint64_t L = low6;
        uint64_t nd_q = 0, nd_s = 0, d_q = 0;   // deferred: dense targets, dense supports, diagonal qubits
        bool def_special = false;               // a probe / observable was deferred
        std::vector<size_t> take, defer;
        size_t scanned_after_defer = 0;
        size_t pos = 0;
        for (; pos < rest.size(); ++pos) {
            const size_t i = rest[pos];
            const Prim &p = prims[i];
            if (!defer.empty() && (p.probe || p.obs || ++scanned_after_defer > window)) break;
            uint64_t U = L;
            bool fits = true;
            if (!(p.diag || p.obs || p.probe) || (p.probe && !p.diag)) {
                U = L | qm[i];
                fits = __builtin_popcountll(U) <= tb;
            }
            bool ok = fits;
            if (ok && !defer.empty()) {
                if (def_special || p.probe || p.obs) ok = false;
                else if (p.diag) ok = (qm[i] & nd_q) == 0;
                else ok = (sm[i] & nd_s) == 0 && (qm[i] & d_q) == 0;
            }
            if (ok) {
                take.push_back(i);
                L = U;
            } else {
                defer.push_back(i);
                if (p.probe || p.obs) def_special = true;
                else if (p.diag) d_q |= qm[i];
                else { nd_q |= qm[i]; nd_s |= sm[i]; }
            }
        }
        if (take.empty()) {   // cannot happen for tb >= 8; keep progress regardless
            take.push_back(rest[0]);
            defer.erase(defer.begin());
            L |= qm[rest[0]];
        }
        std::vector<size_t> next = defer;
        next.insert(next.end(), rest.begin() + pos, rest.end());
        rest.swap(next);
        // fill the tile with the lowest remaining qubits
        for (int q = 0; __builtin_popcountll(L) < tb && q < o.n; ++q) L |= 1ull << q;
        Pass ps;
        for (int q = 0; q < o.n; ++q)
            if ((L >> q) & 1ull) ps.tile_q.push_back(q);
        ps.gate_begin = prims[take.front()].gate;
        ps.gate_end = prims[take.back()].gate + 1;
        Fuser f(o, ps.tile_q);
        for (size_t k : take) f.add(prims[k]);
        f.flush();
        ps.ops = f.out;
        passes.push_back(ps);
    }
    return passes;
}

template <typename R>
bool lower_passes(const std::vector<Pass> &passes, const PlanOptions &o, std::vector<OpDesc> &ops,
                  std::vector<R> &pool, std::vector<PassGeom> &geoms)
{
    const int n = o.n, tb = o.tb, NH = 1 << (tb - 6);
    bool ok = tb >= kMinTileBits && tb <= kMaxTileBits && tb <= n;
    auto push = [&](cd v) {
        pool.push_back((R)v.real());
        pool.push_back((R)v.imag());
    };
    for (const Pass &ps : passes) {
        PassGeom g{};
        g.n = n;
        g.tb = tb;
        g.op_begin = (int32_t)ops.size();
        g.n_ops = (int32_t)ps.ops.size();
        uint64_t tmask = 0;
        for (int i = 0; i < tb; ++i) {
            g.tile_q[i] = ps.tile_q[i];
            tmask |= 1ull << ps.tile_q[i];
        }
        const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
        g.nontile_mask = all & ~tmask;
        g.tile_begin = 0;
        g.n_tiles = 1ull << (n - tb);
        if (!ps.out_q.empty()) {
            g.out_perm = 1;
            for (int q = 0; q < n; ++q) {
                g.out_q[q] = (uint8_t)ps.out_q[q];
                ok = ok && (q < 6 ? ps.out_q[q] == q : (ps.out_q[q] >= 6 && ps.out_q[q] < n));
            }
        }
        auto tpos = [&](int q) {
            for (int i = 0; i < tb; ++i)
                if (ps.tile_q[i] == q) return i;
            return -1;
        };
        // Register segments: maximal runs of ops that can act on per-thread
        // registers (dense ops of <= 2 qubits whose tile bits fit in R register
        // bits together with the run's other dense ops, diagonals, controlled
        // phases). Each run costs one LDS round trip instead of one per op.
        const int RB = tb - 8;   // register bits per thread
        const bool use_seg = o.segments && RB >= 2 && RB <= 5;
        std::vector<int> seg_id(ps.ops.size(), -1);
        std::vector<uint32_t> seg_mask;
        if (use_seg) {
            int cur = -1;
            for (size_t i = 0; i < ps.ops.size(); ++i) {
                const HostOp &h = ps.ops[i];
                uint32_t P = 0;
                bool joinable = false;
                if (h.type == OP_DENSE && h.q.size() <= 2 && !h.q.empty()) {
                    joinable = true;
                    for (int q : h.q) {
                        const int p = tpos(q);
                        if (p < 0) joinable = false;
                        else P |= 1u << p;
                    }
                } else if (h.type == OP_DIAG || h.type == OP_PHASE) {
                    joinable = true;
                }
                if (!joinable) {
                    cur = -1;
                    continue;
                }
                if (cur >= 0 && __builtin_popcount(seg_mask[cur] | P) <= RB) {
                    seg_mask[cur] |= P;
                } else {
                    cur = (int)seg_mask.size();
                    seg_mask.push_back(P);
                }
                seg_id[i] = cur;
            }
            // complete each register set with the highest free tile bits, so
            // that the low tile bits (consecutive LDS words) stay thread bits
            for (uint32_t &m : seg_mask)
                for (int p = tb - 1; p >= 0 && __builtin_popcount(m) < RB; --p) m |= 1u << p;
        }
        int open_seg = -1;
        for (size_t hi = 0; hi < ps.ops.size(); ++hi) {
            const HostOp &h = ps.ops[hi];
            const int sid = seg_id[hi];
            if (sid >= 0 && sid != open_seg) {
                open_seg = sid;
                OpDesc sd{};
                sd.type = OP_SEG;
                int cnt = 0;
                for (size_t j = hi; j < ps.ops.size() && seg_id[j] == sid; ++j) ++cnt;
                sd.k = cnt;
                for (int m = 0; m < 5; ++m) { sd.pos[m] = -1; sd.gq[m] = -1; }
                int r = 0;
                for (int p = 0; p < tb; ++p)
                    if ((seg_mask[sid] >> p) & 1u) sd.pos[r++] = p;
                sd.ctrl_local = seg_mask[sid];
                sd.ctrl_pos = -1;
                sd.ctrl_q = -1;
                sd.slot = -1;
                ops.push_back(sd);
            }
            OpDesc d{};
            d.type = h.type;
            d.mat = (int32_t)(pool.size() / 2);
            d.ctrl_pos = -1;
            d.ctrl_q = -1;
            d.slot = -1;
            d.diag = 0;
            d.real = 0;
            for (int m = 0; m < 5; ++m) { d.pos[m] = -1; d.gq[m] = -1; }
            if (h.type == OP_DENSE) {
                d.k = (int32_t)h.q.size();
                // matrix cores need k >= 3 and 16 columns of 2^k amplitudes per tile
                if (o.mma != 0 && d.k >= 3 && d.k >= o.mfma_min_k && tb - d.k >= 4) d.type = OP_MFMA;
                ok = ok && d.k >= 1 && d.k <= kMaxFuse && (int)h.m.size() == (1 << (2 * d.k));
                for (int m = 0; m < d.k; ++m) {
                    d.pos[m] = tpos(h.q[m]);
                    ok = ok && d.pos[m] >= 0;
                }
                ok = ok && (h.ctrl_mask & tmask) == 0;
                d.real = 1;
                for (const cd &v : h.m)
                    if (v.imag() != 0.0) d.real = 0;
                d.ctrl_fixed = h.ctrl_mask;
                if (d.k == 2 && d.type == OP_DENSE && d.pos[0] > d.pos[1]) {
                    // two-qubit ops take their tile bits ascending (register
                    // segments need it; the LDS path uses the same matrix so
                    // that both sum in the same order): swap the index bits
                    std::swap(d.pos[0], d.pos[1]);
                    auto sw = [](int v) { return ((v & 1) << 1) | ((v >> 1) & 1); };
                    for (int r = 0; r < 4; ++r)
                        for (int c = 0; c < 4; ++c) push(h.m[sw(r) * 4 + sw(c)]);
                } else {
                    for (const cd &v : h.m) push(v);
                }
            } else if (h.type == OP_GRAD) {
                d.k = (int32_t)h.q.size();
                d.slot = h.slot;
                d.diag = h.diag ? 1 : 0;
                ok = ok && d.k >= 1 && d.k <= 2 && h.slot >= 0 &&
                     (int)h.m.size() == (h.diag ? (1 << d.k) : (1 << (2 * d.k)));
                for (int m = 0; m < d.k; ++m) {
                    d.gq[m] = h.q[m];
                    d.pos[m] = tpos(h.q[m]);
                    ok = ok && (h.diag || d.pos[m] >= 0);
                }
                for (const cd &v : h.m) push(v);
            } else if (h.type == OP_OBS) {
                d.k = 0;
            } else if (h.type == OP_DIAG && sid >= 0) {
                // diagonal on registers: the table is reordered so that a
                // thread's entries for its register elements are one contiguous
                // row, selected by its thread bits and the tile's fixed bits
                d.type = OP_RDIAG;
                d.k = (int32_t)h.q.size();
                ok = ok && d.k >= 1 && d.k <= 5 && (int)h.m.size() == (1 << d.k);
                const uint32_t S = seg_mask[sid];
                std::vector<int> rb, tb_, ub;   // table bits m by kind
                for (int m = 0; m < d.k; ++m) {
                    const int p = tpos(h.q[m]);
                    (p >= 0 && ((S >> p) & 1u) ? rb : p >= 0 ? tb_ : ub).push_back(m);
                }
                std::sort(rb.begin(), rb.end(), [&](int a, int b) { return tpos(h.q[a]) < tpos(h.q[b]); });
                std::vector<int> order(rb);
                order.insert(order.end(), tb_.begin(), tb_.end());
                order.insert(order.end(), ub.begin(), ub.end());
                d.slot = (int32_t)rb.size();
                d.diag = (int32_t)tb_.size();
                d.ctrl_local = 0;
                for (int j = 0; j < d.k; ++j) {
                    d.gq[j] = h.q[order[j]];
                    d.pos[j] = tpos(h.q[order[j]]);
                }
                for (int m : rb) {
                    const int p = tpos(h.q[m]);
                    d.ctrl_local |= 1u << __builtin_popcount(S & ((1u << p) - 1u));
                }
                for (int v = 0; v < (1 << d.k); ++v) {
                    int s = 0;
                    for (int j = 0; j < d.k; ++j) s |= ((v >> j) & 1) << order[j];
                    push(h.m[s]);
                }
            } else if (h.type == OP_DIAG) {
                d.k = (int32_t)h.q.size();
                ok = ok && d.k >= 1 && d.k <= 5 && (int)h.m.size() == (1 << d.k);
                for (int m = 0; m < d.k; ++m) {
                    d.gq[m] = h.q[m];
                    d.pos[m] = tpos(h.q[m]);
                }
                for (const cd &v : h.m) push(v);
            } else if (sid >= 0) {
                // controlled phase on registers: factor = F(thread, tile id) U(register index)
                d.type = OP_RPHASE;
                d.ctrl_q = h.hub;
                d.ctrl_pos = h.hub >= 0 ? tpos(h.hub) : -1;
                const int G = (n - tb + 7) / 8;
                d.k = G;
                const uint32_t S = seg_mask[sid];
                std::vector<int> sp, tp, nq;
                for (int p = 0; p < tb; ++p) ((S >> p) & 1u ? sp : tp).push_back(ps.tile_q[p]);
                for (int q = 0; q < n; ++q)
                    if ((g.nontile_mask >> q) & 1ull) nq.push_back(q);
                // per-qubit factors, then every table as subset products
                // (entry v = entry of v without its lowest bit times that bit's factor)
                std::vector<cd> fa(n), fab(n);
                for (int q = 0; q < n; ++q) {
                    fa[q] = expi(h.mu[q]);
                    fab[q] = expi(h.mu[q] + h.lam[q]);
                }
                auto subset_table = [&](const std::vector<int> &qs, int size, const std::vector<cd> &f, cd first) {
                    std::vector<cd> t(size);
                    t[0] = first;
                    for (int v = 1; v < size; ++v) {
                        const int b = __builtin_ctz(v);
                        t[v] = b < (int)qs.size() ? t[v & (v - 1)] * f[qs[b]] : t[v & (v - 1)];
                    }
                    return t;
                };
                for (int on = 0; on < 2; ++on)
                    for (const cd &v : subset_table(sp, 1 << RB, on ? fab : fa, h.global)) push(v);
                for (int on = 0; on < 2; ++on)
                    for (const cd &v : subset_table(tp, 256, on ? fab : fa, 1.0)) push(v);
                for (int on = 0; on < 2; ++on)
                    for (int gg = 0; gg < G; ++gg) {
                        std::vector<int> qs;
                        for (int j = 0; j < 8 && 8 * gg + j < (int)nq.size(); ++j) qs.push_back(nq[8 * gg + j]);
                        for (const cd &v : subset_table(qs, 256, on ? fab : fa, 1.0)) push(v);
                    }
                ok = ok && (int)sp.size() == RB && (int)tp.size() == 8;
            } else {
                d.k = 0;
                d.ctrl_q = h.hub;
                d.ctrl_pos = h.hub >= 0 ? tpos(h.hub) : -1;
                d.ctrl_fixed = g.nontile_mask;
                // loA (with the global factor), hiA, loB, hiB, fixA[n], fixB[n]
                for (int a = 0; a < 64; ++a) {
                    double ph = 0.0;
                    for (int i = 0; i < 6; ++i)
                        if ((a >> i) & 1) ph += h.mu[ps.tile_q[i]];
                    push(h.global * expi(ph));
                }
                for (int a = 0; a < NH; ++a) {
                    double ph = 0.0;
                    for (int i = 0; i < tb - 6; ++i)
                        if ((a >> i) & 1) ph += h.mu[ps.tile_q[6 + i]];
                    push(expi(ph));
                }
                for (int a = 0; a < 64; ++a) {
                    double ph = 0.0;
                    for (int i = 0; i < 6; ++i)
                        if ((a >> i) & 1) ph += h.lam[ps.tile_q[i]];
                    push(expi(ph));
                }
                for (int a = 0; a < NH; ++a) {
                    double ph = 0.0;
                    for (int i = 0; i < tb - 6; ++i)
                        if ((a >> i) & 1) ph += h.lam[ps.tile_q[6 + i]];
                    push(expi(ph));
                }
                for (int q = 0; q < n; ++q) push((g.nontile_mask >> q) & 1 ? expi(h.mu[q]) : cd(1.0));
                for (int q = 0; q < n; ++q) push((g.nontile_mask >> q) & 1 ? expi(h.lam[q]) : cd(1.0));
            }
            ops.push_back(d);
        }
        ok = ok && (int)ps.tile_q.size() == tb && ps.tile_q[0] == 0 && ps.tile_q[5] == 5;
        g.n_ops = (int32_t)(ops.size() - (size_t)g.op_begin);   // segment markers included
        g.max_k = 0;
        g.mma = 0;
        for (int i = g.op_begin; i < (int)ops.size(); ++i) {
            if (ops[i].type == OP_DENSE) g.max_k = std::max<int>(g.max_k, ops[i].k);
            if (ops[i].type == OP_MFMA) g.mma = o.mma;
        }
        geoms.push_back(g);
    }
    return ok;
}

template bool lower_passes<float>(const std::vector<Pass> &, const PlanOptions &, std::vector<OpDesc> &,
                                  std::vector<float> &, std::vector<PassGeom> &);
template bool lower_passes<double>(const std::vector<Pass> &, const PlanOptions &, std::vector<OpDesc> &,
                                   std::vector<double> &, std::vector<PassGeom> &);

}  // namespace msv
