// msv_adjoint: expectation and gradient by the adjoint method with compressed
// checkpoints.
//
//   forward:  psi_0 -> psi_N, saving psi at each checkpoint gate index in the
//             canonical compressed chunk format (its compressed size in HBM);
//   lambda := O psi_N (one pass with the observable op);
//   reverse:  for each segment, last first: restore psi from the segment's
//             checkpoint and run the segment forward (fresh psi at its end),
//             then one two-state sweep backwards through the segment: probe
//             <lambda| A_k |psi_k> for parameterised gates, apply U_k^dagger to
//             psi and lambda;
//   grad[p] = sum over the gates fed by p of 2 Re <lambda_k| A_k |psi_k>;
//   finally psi is restored from the first checkpoint (the input state).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>
#include <thread>

#include "internal.h"

namespace msv {

namespace {

struct Ckpt {
    DevMem blob, sizes, offsets;
};

uint64_t n_chunks_of(const msv_sim *s) { return 1ull << (s->n - s->log2c); }
uint64_t nb_of(const msv_sim *s) { return (2ull << s->log2c) / 64; }

struct Scratch {
    DevMem dst_off, kinds, flags, grad_part, grad_out, psi_part, lam_part, pstats;
};

int save_ckpt(msv_sim *s, Ckpt &c, Scratch &w)
{
    hipStream_t cs = s->stream();
    int st;
    if (!s->compressed()) {
        if ((st = dev_alloc(s, c.blob, s->elt() << s->n))) return st;
        HIPCHK(s, hipMemcpyAsync(c.blob.p, s->amps.p, s->elt() << s->n, hipMemcpyDeviceToDevice, cs));
        return MSV_OK;
    }
    const uint64_t nc = n_chunks_of(s), nb = nb_of(s);
    if ((st = dev_alloc(s, c.sizes, 8 * nc))) return st;
    if ((st = dev_alloc(s, c.offsets, 8 * (nc + 1)))) return st;
    const DevStore &d = s->st[s->cur];
    HIPCHK(s, launch_scan_chunks((const uint8_t *)d.W.p, (const int32_t *)d.A.p, nb, nc, (uint32_t *)w.dst_off.p,
                                 (uint64_t *)c.sizes.p, (uint32_t *)w.kinds.p, (uint32_t *)w.flags.p, cs));
    HIPCHK(s, launch_scan_sizes((const uint64_t *)c.sizes.p, nc, (uint64_t *)c.offsets.p, cs));
    uint64_t total = 0;
    HIPCHK(s, hipMemcpyAsync(&total, (const uint64_t *)c.offsets.p + nc, 8, hipMemcpyDeviceToHost, cs));
    HIPCHK(s, hipStreamSynchronize(cs));
    if ((st = dev_alloc(s, c.blob, std::max<uint64_t>(total, 256)))) return st;
    HIPCHK(s, launch_assemble_chunks(s->is_double() ? 0 : 1, s->log2c, s->eb, s->export_pred_mode(),
                                     (const uint8_t *)d.W.p,
                                     (const int32_t *)d.A.p, (const uint32_t *)d.OFF.p, (const uint64_t *)d.heap.p,
                                     (const uint32_t *)w.dst_off.p, (const uint64_t *)c.sizes.p,
                                     (const uint32_t *)w.kinds.p, (const uint64_t *)c.offsets.p, nc,
                                     (uint8_t *)c.blob.p, cs));
    return MSV_OK;
}

// Identity pass geometry with no ops (decode -> encode copy).
PassGeom copy_geom(const msv_sim *s, int tb)
{
    PassGeom g{};
    g.n = s->n;
    g.tb = tb;
    g.n_ops = 0;
    g.op_begin = 0;
    uint64_t tm = 0;
    for (int i = 0; i < tb; ++i) {
        g.tile_q[i] = i;
        tm |= 1ull << i;
    }
    g.nontile_mask = (s->n >= 64 ? ~0ull : ((1ull << s->n) - 1)) & ~tm;
    g.n_tiles = 1ull << (s->n - tb);
    return g;
}

int restore_ckpt(msv_sim *s, Ckpt &c, Scratch &w, int tb)
{
    hipStream_t cs = s->stream();
    if (!s->compressed()) {
        HIPCHK(s, hipMemcpyAsync(s->amps.p, c.blob.p, s->elt() << s->n, hipMemcpyDeviceToDevice, cs));
        return MSV_OK;
    }
    const uint64_t nc = n_chunks_of(s);
    DevStore &d = s->st[s->cur];
    HIPCHK(s, launch_parse_chunks((const uint8_t *)c.blob.p, (const uint64_t *)c.offsets.p,
                                  (const uint64_t *)c.sizes.p, nc, s->log2c, (uint8_t *)d.W.p, (int32_t *)d.A.p,
                                  (uint32_t *)d.OFF.p, (uint32_t *)w.flags.p, cs));
    PassBuffers b{};
    b.in = BlockStore{(uint8_t *)d.W.p, (int32_t *)d.A.p, (uint32_t *)d.OFF.p, (uint64_t *)c.blob.p, nullptr, 0};
    b.out = s->st[s->cur ^ 1].view();
    b.inv_step = s->inv_step();
    b.step = s->step();
    b.scale = 1.0;
    b.flags = (uint32_t *)w.flags.p;
    b.check_err = 0;
    b.pred_mode = s->pred_mode;
    b.in_pred = s->in_pred();
    b.ops = (const OpDesc *)s->ws.ops.p;
    b.pool = s->ws.pool.p;
    HIPCHK(s, launch_pass(s->is_double(), true, true, copy_geom(s, tb), b, cs));
    s->cur ^= 1;
    return MSV_OK;
}

// lambda := O psi (one pass: load psi, multiply by the observable, store lambda).
int init_lambda(msv_sim *s, const uint64_t *masks, const double *coeffs, size_t n_terms, Scratch &w, int tb)
{
    hipStream_t cs = s->stream();
    int st;
    if ((st = dev_alloc(s, s->ws.masks, 16 * std::max<size_t>(n_terms, 1)))) return st;
    if ((st = pin_stage(s, 16 * n_terms + sizeof(OpDesc) + 64))) return st;
    HIPCHK(s, hipStreamSynchronize(cs));
    uint8_t *pin = (uint8_t *)s->ws.pin.p;
    memcpy(pin, masks, 8 * n_terms);
    memcpy(pin + 8 * n_terms, coeffs, 8 * n_terms);
    OpDesc od{};
    od.type = OP_OBS;
    od.slot = -1;
    memcpy(pin + 16 * n_terms, &od, sizeof od);
    if (n_terms) HIPCHK(s, hipMemcpyAsync(s->ws.masks.p, pin, 16 * n_terms, hipMemcpyHostToDevice, cs));
    if ((st = dev_alloc(s, s->ws.ops, std::max<size_t>(sizeof od, 256)))) return st;
    HIPCHK(s, hipMemcpyAsync(s->ws.ops.p, pin + 16 * n_terms, sizeof od, hipMemcpyHostToDevice, cs));
    PassGeom g = copy_geom(s, tb);
    g.n_ops = 1;
    PassBuffers b{};
    const bool c = s->compressed();
    b.amps_in = s->amps.p;
    b.amps_out = s->lam_amps.p;
    if (c) {
        b.in = s->st[s->cur].view();
        b.out = s->lam[0].view();
    }
    b.inv_step = c ? s->inv_step() : 0.0;
    b.step = c ? s->step() : 0.0;
    b.scale = 1.0;
    b.flags = (uint32_t *)w.flags.p;
    b.check_err = 0;
    b.pred_mode = s->pred_mode;
    b.in_pred = s->in_pred();
    b.ops = (const OpDesc *)s->ws.ops.p;
    b.pool = s->ws.pool.p;
    b.obs_masks = (const uint64_t *)s->ws.masks.p;
    b.obs_coeffs = (const double *)((uint8_t *)s->ws.masks.p + 8 * n_terms);
    b.obs_terms = (int32_t)n_terms;
    HIPCHK(s, launch_pass(s->is_double(), c, c, g, b, cs));
    s->lcur = 0;
    HIPCHK(s, hipStreamSynchronize(cs));   // the pinned staging is reused next
    return MSV_OK;
}

// Reverse two-state passes over the planned probe / U^dagger list.
int run_adjoint_passes(msv_sim *s, const std::vector<Pass> &passes, const PlanOptions &o, Scratch &w,
                       uint64_t stride, uint64_t *violations)
{
    hipStream_t cs = s->stream();
    std::vector<OpDesc> ops;
    std::vector<PassGeom> geoms;
    std::vector<float> pf;
    std::vector<double> pd;
    const bool ok = s->is_double() ? lower_passes<double>(passes, o, ops, pd, geoms)
                                   : lower_passes<float>(passes, o, ops, pf, geoms);
    if (!ok) return fail_sim(s, MSV_E_ARG, "internal planner error (adjoint)");
    const size_t ops_bytes = ops.size() * sizeof(OpDesc);
    const size_t pool_bytes = s->is_double() ? pd.size() * 8 : pf.size() * 4;
    int st;
    if ((st = dev_alloc(s, s->ws.ops, std::max<size_t>(ops_bytes, 256)))) return st;
    if ((st = dev_alloc(s, s->ws.pool, std::max<size_t>(pool_bytes, 256)))) return st;
    if ((st = pin_stage(s, ops_bytes + pool_bytes + 512))) return st;
    HIPCHK(s, hipStreamSynchronize(cs));
    uint8_t *pin = (uint8_t *)s->ws.pin.p;
    const size_t a1 = (ops_bytes + 255) & ~(size_t)255;
    if (ops_bytes) memcpy(pin, ops.data(), ops_bytes);
    if (pool_bytes) memcpy(pin + a1, s->is_double() ? (const void *)pd.data() : (const void *)pf.data(), pool_bytes);
    if (ops_bytes) HIPCHK(s, hipMemcpyAsync(s->ws.ops.p, pin, ops_bytes, hipMemcpyHostToDevice, cs));
    if (pool_bytes) HIPCHK(s, hipMemcpyAsync(s->ws.pool.p, pin + a1, pool_bytes, hipMemcpyHostToDevice, cs));
    const uint64_t tiles = geoms.empty() ? 0 : geoms[0].n_tiles;
    if ((st = dev_alloc(s, w.psi_part, 3 * 8 * std::max<uint64_t>(tiles, 1)))) return st;
    if ((st = dev_alloc(s, w.lam_part, 3 * 8 * std::max<uint64_t>(tiles, 1)))) return st;
    if ((st = dev_alloc(s, w.pstats, 6 * 8 * std::max<size_t>(geoms.size(), 1)))) return st;
    if ((st = dev_alloc(s, s->ws.pass_off, 64))) return st;
    const uint64_t offs2[2] = {0, tiles};
    HIPCHK(s, hipMemcpyAsync(s->ws.pass_off.p, offs2, 16, hipMemcpyHostToDevice, cs));
    const bool c = s->compressed();
    for (size_t p = 0; p < geoms.size(); ++p) {
        AdjointBuffers ab{};
        for (int which = 0; which < 2; ++which) {
            PassBuffers &b = which ? ab.lam : ab.psi;
            b.amps_in = b.amps_out = which ? s->lam_amps.p : s->amps.p;
            if (c) {
                const DevStore *dv = which ? s->lam : s->st;
                const int cur = which ? s->lcur : s->cur;
                b.in = dv[cur].view();
                b.out = dv[cur ^ 1].view();
            }
            b.inv_step = c ? s->inv_step() : 0.0;
            b.step = c ? s->step() : 0.0;
            b.scale = 1.0;
            b.part = (double *)(which ? w.lam_part.p : w.psi_part.p);
            b.flags = (uint32_t *)w.flags.p;
            b.check_err = s->check_bound;
            b.pred_mode = s->pred_mode;
            b.in_pred = s->in_pred();
            b.ops = (const OpDesc *)s->ws.ops.p;
            b.pool = s->ws.pool.p;
        }
        ab.grad_part = (double *)w.grad_part.p;
        ab.grad_stride = stride;
        HIPCHK(s, launch_adjoint_pass(s->is_double(), c, geoms[p], ab, cs));
        HIPCHK(s, launch_pass_stats((const double *)w.psi_part.p, (const uint64_t *)s->ws.pass_off.p, 1,
                                    (double *)w.pstats.p + 6 * p, cs));
        HIPCHK(s, launch_pass_stats((const double *)w.lam_part.p, (const uint64_t *)s->ws.pass_off.p, 1,
                                    (double *)w.pstats.p + 6 * p + 3, cs));
        if (c) {
            s->cur ^= 1;
            s->lcur ^= 1;
        }
    }
    std::vector<double> hs(6 * geoms.size() + 6, 0.0);
    if (!geoms.empty())
        HIPCHK(s, hipMemcpyAsync(hs.data(), w.pstats.p, 6 * 8 * geoms.size(), hipMemcpyDeviceToHost, cs));
    HIPCHK(s, hipStreamSynchronize(cs));
    if (c)
        for (size_t p = 0; p < geoms.size(); ++p) {
            if (hs[6 * p + 1] > bound_for(s, hs[6 * p])) ++*violations;
            if (hs[6 * p + 4] > bound_for(s, hs[6 * p + 3])) ++*violations;
            s->max_err_all = std::max(s->max_err_all, std::max(hs[6 * p + 1], hs[6 * p + 4]));
        }
    s->stats.passes += geoms.size();
    return MSV_OK;
}

// Derivative operator A with dU/dtheta = A U for a parameterised gate.
int probe_prim(const msv_gate &g, int n, Prim &p, std::string &err)
{
    p = Prim();
    p.probe = true;
    const cd I(0.0, 1.0);
    switch (g.kind) {
    case MSV_RX: p.q = {g.q0}; p.m = {0.0, -0.5 * I, -0.5 * I, 0.0}; break;     // -i X / 2
    case MSV_RY: p.q = {g.q0}; p.m = {0.0, -0.5, 0.5, 0.0}; break;               // -i Y / 2
    case MSV_RZ: p.q = {g.q0}; p.diag = true; p.m = {-0.5 * I, 0.5 * I}; break;  // -i Z / 2
    case MSV_P: p.q = {g.q0}; p.diag = true; p.m = {0.0, I}; break;              // i |1><1|
    case MSV_CP:
        if (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0) { err = "bad CP qubits"; return MSV_E_ARG; }
        p.q = {g.q0, g.q1};
        p.diag = true;
        p.m = {0.0, 0.0, 0.0, I};                                                // i |11><11|
        break;
    default: err = "only RX, RY, RZ, P and CP may be parameterised"; return MSV_E_ARG;
    }
    if (g.q0 < 0 || g.q0 >= n) { err = "qubit out of range"; return MSV_E_ARG; }
    return MSV_OK;
}

}  // namespace

}  // namespace msv

using namespace msv;

extern "C" int msv_adjoint(msv_sim *s, const msv_gate *gates, size_t n_gates, const double *params, size_t n_params,
                           const uint64_t *masks, const double *coeffs, size_t n_terms, const size_t *ckpt_at,
                           size_t n_ckpt, double *expval, double *grad)
{
    if (!s) return fail_global(MSV_E_ARG, "null handle");
    if (s->poisoned) return fail_sim(s, MSV_E_STATE, "handle poisoned by an earlier device error");
    if (!s->inited) return fail_sim(s, MSV_E_STATE, "state not initialised");
    if (s->store != MSV_STORE_DEVICE) return fail_sim(s, MSV_E_UNSUPPORTED, "adjoint runs on the device store");
    if (s->renorm || s->scale != 1.0) return fail_sim(s, MSV_E_UNSUPPORTED, "adjoint with renormalisation");
    if ((n_gates && !gates) || (n_params && !params) || !expval || (n_params && !grad) ||
        (n_terms && (!masks || !coeffs)) || (n_ckpt && !ckpt_at) || n_terms > 4096)
        return fail_sim(s, MSV_E_ARG, "bad argument");
    const auto t0 = std::chrono::steady_clock::now();
    // bind parameters; build forward, inverse and probe prims
    std::vector<Prim> fwd(n_gates), inv(n_gates), prb(n_gates);
    std::vector<int> slot_of(n_gates, -1), slot_param;
    std::string err;
    for (size_t k = 0; k < n_gates; ++k) {
        msv_gate g = gates[k];
        if (g.param >= 0) {
            if ((size_t)g.param >= n_params) return fail_sim(s, MSV_E_ARG, "parameter index out of range");
            g.theta = params[g.param];
            int st = probe_prim(g, s->n, prb[k], err);
            if (st) return fail_sim(s, st, err.c_str());
            slot_of[k] = (int)slot_param.size();
            prb[k].slot = slot_of[k];
            slot_param.push_back(g.param);
        }
        int st = gate_to_prim(g, s->n, false, fwd[k], err);
        if (st) return fail_sim(s, st, err.c_str());
        st = gate_to_prim(g, s->n, true, inv[k], err);
        if (st) return fail_sim(s, st, err.c_str());
        fwd[k].gate = inv[k].gate = prb[k].gate = k;
    }
    std::vector<size_t> cps{0};
    for (size_t i = 0; i < n_ckpt; ++i)
        if (ckpt_at[i] < n_gates) cps.push_back(ckpt_at[i]);
    std::sort(cps.begin(), cps.end());
    cps.erase(std::unique(cps.begin(), cps.end()), cps.end());
    const size_t n_seg = cps.size();
    auto seg_end = [&](size_t j) { return j + 1 < n_seg ? cps[j + 1] : n_gates; };

    int st;
    PlanOptions o;
    o.n = s->n;
    o.tb = std::min(choose_tile_bits(s), 12);
    o.k_max = s->k_max;
    o.mfma_min_k = s->mfma_min_k;
    o.lookahead = s->lookahead;
    const uint64_t stride = 1ull << (s->n - o.tb);
    Scratch w;
    struct Free {
        msv_sim *s;
        Scratch &w;
        std::vector<Ckpt> ck;
        ~Free()
        {
            for (DevMem *m : {&w.dst_off, &w.kinds, &w.flags, &w.grad_part, &w.grad_out, &w.psi_part, &w.lam_part,
                              &w.pstats})
                dev_free(s, *m);
            for (auto &c : ck) {
                dev_free(s, c.blob);
                dev_free(s, c.sizes);
                dev_free(s, c.offsets);
            }
        }
    } fr{s, w, std::vector<Ckpt>(n_seg)};
    const uint64_t total_blocks = 2ull << (s->n - 6);
    if ((st = dev_alloc(s, w.dst_off, 4 * total_blocks))) return st;
    if ((st = dev_alloc(s, w.kinds, 4 * n_chunks_of(s) + 64))) return st;
    if ((st = dev_alloc(s, w.flags, 256))) return st;
    const size_t n_slots = slot_param.size();
    if ((st = dev_alloc(s, w.grad_part, 16 * stride * std::max<size_t>(n_slots, 1)))) return st;
    if ((st = dev_alloc(s, w.grad_out, 16 * std::max<size_t>(n_slots, 1)))) return st;
    if (s->compressed()) {
        for (auto &d : s->lam) {
            const uint64_t nblk = 2ull << (s->n - 6);
            if ((st = dev_alloc(s, d.W, nblk)) || (st = dev_alloc(s, d.A, 4 * nblk)) ||
                (st = dev_alloc(s, d.OFF, 4 * nblk)) || (st = dev_alloc(s, d.heap, 8ull << s->n)))
                return st;
        }
    } else if ((st = dev_alloc(s, s->lam_amps, s->elt() << s->n))) {
        return st;
    }
    if ((st = dev_alloc(s, s->ws.ops, 256)) || (st = dev_alloc(s, s->ws.pool, 256))) return st;
    hipStream_t cs = s->stream();
    HIPCHK(s, hipMemsetAsync(w.flags.p, 0, 16, cs));
    s->stats = msv_stats{};

    // forward with checkpoints
    double nrm = 0, el = 0, wl = 0;
    for (size_t j = 0; j < n_seg; ++j) {
        if ((st = save_ckpt(s, fr.ck[j], w))) return st;
        std::vector<Prim> seg(fwd.begin() + cps[j], fwd.begin() + seg_end(j));
        if (!seg.empty()) {
            std::vector<Pass> ps = plan_passes(seg, o);
            if ((st = run_passes_device(s, ps, o, &nrm, &el, &wl, nullptr))) return st;
            s->stats.passes += ps.size();
        }
    }
    // expectation of the final state
    {
        if ((st = dev_alloc(s, s->ws.masks, 16 * std::max<size_t>(n_terms, 1)))) return st;
        if ((st = dev_alloc(s, s->ws.red, 4 * 8 * 2048)) || (st = dev_alloc(s, s->ws.red_out, 256))) return st;
        if ((st = pin_stage(s, 16 * n_terms + 64))) return st;
        HIPCHK(s, hipStreamSynchronize(cs));
        memcpy(s->ws.pin.p, masks, 8 * n_terms);
        memcpy((uint8_t *)s->ws.pin.p + 8 * n_terms, coeffs, 8 * n_terms);
        if (n_terms) HIPCHK(s, hipMemcpyAsync(s->ws.masks.p, s->ws.pin.p, 16 * n_terms, hipMemcpyHostToDevice, cs));
        ReduceArgs a{};
        a.kind = RED_EXPZ;
        a.amp_begin = 0;
        a.amp_count = 1ull << s->n;
        a.masks = (const uint64_t *)s->ws.masks.p;
        a.coeffs = (const double *)((uint8_t *)s->ws.masks.p + 8 * n_terms);
        a.n_terms = (int32_t)n_terms;
        a.partials = (double *)s->ws.red.p;
        a.scale = 1.0;
        int groups = 0;
        HIPCHK(s, launch_reduce(s->is_double(), s->decode_comp(), s->amps.p, s->st[s->cur].view(),
                                s->compressed() ? s->step() : 0.0, a, &groups, cs));
        HIPCHK(s, launch_reduce_final(a.partials, groups, (double *)s->ws.red_out.p, cs));
        double o4[4];
        HIPCHK(s, hipMemcpyAsync(o4, s->ws.red_out.p, 32, hipMemcpyDeviceToHost, cs));
        HIPCHK(s, hipStreamSynchronize(cs));
        *expval = o4[1];
    }
    if ((st = init_lambda(s, masks, coeffs, n_terms, w, o.tb))) return st;

    // reverse sweep, one segment at a time
    uint64_t violations = 0;
    for (size_t jj = n_seg; jj-- > 0;) {
        const size_t b = cps[jj], e = seg_end(jj);
        if (jj + 1 < n_seg) {
            if ((st = restore_ckpt(s, fr.ck[jj], w, o.tb))) return st;
            std::vector<Prim> seg(fwd.begin() + b, fwd.begin() + e);
            if (!seg.empty()) {
                std::vector<Pass> ps = plan_passes(seg, o);
                if ((st = run_passes_device(s, ps, o, &nrm, &el, &wl, nullptr))) return st;
                s->stats.passes += ps.size();
            }
        }
        std::vector<Prim> rev;
        for (size_t k = e; k-- > b;) {
            if (slot_of[k] >= 0) rev.push_back(prb[k]);
            rev.push_back(inv[k]);
        }
        if (rev.empty()) continue;
        std::vector<Pass> ps = plan_passes(rev, o);
        if ((st = run_adjoint_passes(s, ps, o, w, stride, &violations))) return st;
    }
    // gradients
    std::vector<double> gv(2 * std::max<size_t>(n_slots, 1), 0.0);
    if (n_slots) {
        HIPCHK(s, launch_grad_reduce((const double *)w.grad_part.p, stride, (int)n_slots, (double *)w.grad_out.p, cs));
        HIPCHK(s, hipMemcpyAsync(gv.data(), w.grad_out.p, 16 * n_slots, hipMemcpyDeviceToHost, cs));
    }
    // back to the input state
    if ((st = restore_ckpt(s, fr.ck[0], w, o.tb))) return st;
    uint32_t flags = 0;
    HIPCHK(s, hipMemcpyAsync(&flags, w.flags.p, 4, hipMemcpyDeviceToHost, cs));
    HIPCHK(s, hipStreamSynchronize(cs));
    for (size_t p = 0; p < n_params; ++p) grad[p] = 0.0;
    for (size_t k = 0; k < n_slots; ++k) grad[slot_param[k]] += 2.0 * gv[2 * k];
    s->stats.bound_violations += violations;
    s->stats.gates = n_gates;
    s->stats.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (flags & 4u) return fail_sim(s, MSV_E_CORRUPT, "checkpoint failed validation");
    if (flags & 1u) {
        s->inited = false;
        return fail_sim(s, MSV_E_RANGE, "a value left the codec range during the adjoint sweep");
    }
    return MSV_OK;
}

// ---------------------------------------------------------------------------
// Batched adjoint: many parameter sets of one ansatz, every sweep of every
// set as work items of persistent launches.
//
// Per set the stores are: the checkpoints CK_0 .. CK_(S-1) (CK_0 the input
// state, CK_j the state at the start of segment j), two work stores A and B
// for psi (one, updated in place, for plain amplitudes) and two for lambda
// (one for plain amplitudes). Launches, each over all sets:
//   1. forward through every segment (the last pass of segment j writes
//      CK_(j+1); an empty segment copies with an op-less pass), then
//      lambda := O psi (the observable pass) - one persistent launch;
//   2. the expectation of each final state (one reduction launch);
//   3. per segment, last first: a persistent launch recomputing psi over the
//      segment from its checkpoint (not for the last segment), then a
//      persistent launch of its two-state reverse passes;
//   4. the gradient partials of every set summed (one launch).
// Launches are O(segments), independent of the number of sets.

namespace msv {
namespace {

struct Slot {
    DevStore st;       // compressed
    void *amps = nullptr;   // plain
};

}  // namespace
}  // namespace msv

extern "C" int msv_batch_adjoint(const msv_circuit *ansatz, const double *params, size_t n_sets, size_t n_params,
                                 const uint64_t *masks, const double *coeffs, size_t n_terms, const size_t *ckpt_at,
                                 size_t n_ckpt, int dtype, double eb, double *expvals, double *grads)
{
    if (!ansatz || !params || !expvals || (n_params && !grads) || n_sets == 0 || n_sets > (1u << 16) ||
        (n_terms && (!masks || !coeffs)) || n_terms > 4096 || (n_ckpt && !ckpt_at) || (ansatz->n_gates && !ansatz->gates))
        return fail_global(MSV_E_ARG, "msv_batch_adjoint: bad argument");
    if (dtype != MSV_C128 && dtype != MSV_C64) return fail_global(MSV_E_ARG, "bad dtype");
    if (!(eb >= 0.0) || !std::isfinite(eb)) return fail_global(MSV_E_ARG, "bad error bound");
    const int n = ansatz->n_qubits;
    if (n < 8 || n > 30) return fail_global(MSV_E_ARG, "batched adjoint: qubits must be in [8, 30]");
    const bool dbl = dtype == MSV_C128, comp = eb > 0.0;
    const size_t G = ansatz->n_gates;
    const msv_gate *gates = ansatz->gates;

    // segments
    std::vector<size_t> cps{0};
    for (size_t i = 0; i < n_ckpt; ++i)
        if (ckpt_at[i] > 0 && ckpt_at[i] < G) cps.push_back(ckpt_at[i]);
    std::sort(cps.begin(), cps.end());
    cps.erase(std::unique(cps.begin(), cps.end()), cps.end());
    const size_t S = cps.size();
    auto seg_end = [&](size_t j) { return j + 1 < S ? cps[j + 1] : G; };

    // probe slots (the same for every set: they follow the gates' parameter indices)
    std::vector<int> slot_of(G, -1), slot_param;
    for (size_t k = 0; k < G; ++k)
        if (gates[k].param >= 0) {
            if ((size_t)gates[k].param >= n_params) return fail_global(MSV_E_ARG, "parameter index out of range");
            slot_of[k] = (int)slot_param.size();
            slot_param.push_back(gates[k].param);
        }
    const size_t n_slots = slot_param.size();

    const int tb = std::min(dbl ? 11 : 12, n);
    PlanOptions of;   // forward: register segments, VALU ops only
    of.n = n;
    of.tb = tb;
    of.k_max = 2;
    of.mfma_min_k = 6;
    of.segments = true;
    PlanOptions orv = of;   // reverse: the two-state kernel runs plain ops
    orv.segments = false;
    const uint64_t stride = 1ull << (n - tb);

    // bound prims and plans per set, sets in parallel on the host
    std::vector<std::vector<std::vector<Pass>>> fplan(n_sets, std::vector<std::vector<Pass>>(S)),
        rplan(n_sets, std::vector<std::vector<Pass>>(S));
    std::vector<int> pstat(n_sets, MSV_OK);
    std::vector<std::string> perr(n_sets);
    {
        auto plan_set = [&](size_t k) {
            std::vector<Prim> fwd(G), inv(G), prb(G);
            for (size_t i = 0; i < G; ++i) {
                msv_gate g = gates[i];
                int st;
                if (g.param >= 0) {
                    g.theta = params[k * n_params + g.param];
                    if ((st = probe_prim(g, n, prb[i], perr[k]))) { pstat[k] = st; return; }
                    prb[i].slot = slot_of[i];
                }
                if ((st = gate_to_prim(g, n, false, fwd[i], perr[k])) || (st = gate_to_prim(g, n, true, inv[i], perr[k]))) {
                    pstat[k] = st;
                    return;
                }
                fwd[i].gate = inv[i].gate = prb[i].gate = i;
            }
            for (size_t j = 0; j < S; ++j) {
                const size_t b = cps[j], e = seg_end(j);
                std::vector<Prim> seg(fwd.begin() + b, fwd.begin() + e), rev;
                if (!seg.empty()) fplan[k][j] = plan_passes(seg, of);
                for (size_t i = e; i-- > b;) {
                    if (slot_of[i] >= 0) rev.push_back(prb[i]);
                    rev.push_back(inv[i]);
                }
                if (!rev.empty()) rplan[k][j] = plan_passes(rev, orv);
            }
        };
        const size_t nt = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        auto worker = [&](size_t t) { for (size_t k = t; k < n_sets; k += nt) plan_set(k); };
        for (size_t t = 1; t < nt; ++t) pool.emplace_back(worker, t);
        worker(0);
        for (auto &th : pool) th.join();
        for (size_t k = 0; k < n_sets; ++k)
            if (pstat[k]) return fail_global(pstat[k], ("batched adjoint gate: " + perr[k]).c_str());
    }

    // lowering: one op buffer and one pool for every set; an empty segment
    // of the forward sweep becomes one op-less (copy) pass
    std::vector<OpDesc> ops;
    std::vector<float> pf;
    std::vector<double> pd;
    std::vector<std::vector<std::vector<PassGeom>>> fgeo(n_sets, std::vector<std::vector<PassGeom>>(S)),
        rgeo(n_sets, std::vector<std::vector<PassGeom>>(S));
    auto lower_into = [&](const std::vector<Pass> &ps, const PlanOptions &o, std::vector<PassGeom> &geoms) -> bool {
        std::vector<OpDesc> oi;
        std::vector<float> pfi;
        std::vector<double> pdi;
        const bool ok = dbl ? lower_passes<double>(ps, o, oi, pdi, geoms) : lower_passes<float>(ps, o, oi, pfi, geoms);
        if (!ok) return false;
        const int32_t op0 = (int32_t)ops.size(), m0 = (int32_t)((dbl ? pd.size() : pf.size()) / 2);
        for (OpDesc &d : oi) d.mat += m0;
        for (auto &g : geoms) g.op_begin += op0;
        ops.insert(ops.end(), oi.begin(), oi.end());
        if (dbl) pd.insert(pd.end(), pdi.begin(), pdi.end());
        else pf.insert(pf.end(), pfi.begin(), pfi.end());
        return true;
    };
    PassGeom copy_g{};
    {
        copy_g.n = n;
        copy_g.tb = tb;
        uint64_t tm = 0;
        for (int i = 0; i < tb; ++i) {
            copy_g.tile_q[i] = i;
            tm |= 1ull << i;
        }
        copy_g.nontile_mask = (n >= 64 ? ~0ull : ((1ull << n) - 1)) & ~tm;
        copy_g.n_tiles = stride;
    }
    for (size_t k = 0; k < n_sets; ++k)
        for (size_t j = 0; j < S; ++j) {
            if (!lower_into(fplan[k][j], of, fgeo[k][j]) || !lower_into(rplan[k][j], orv, rgeo[k][j]))
                return fail_global(MSV_E_ARG, "internal planner error (batched adjoint)");
            if (fgeo[k][j].empty() && j + 1 < S) fgeo[k][j].push_back(copy_g);
        }
    PassGeom obs_g = copy_g;
    obs_g.n_ops = 1;
    obs_g.op_begin = (int32_t)ops.size();
    {
        OpDesc od{};
        od.type = OP_OBS;
        od.slot = -1;
        ops.push_back(od);
    }

    // simulators (stores), one stream, one arena for every store
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
        return fail_global(MSV_E_DEVICE, "stream creation failed");
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{stream};
    StoreArena arena;
    const uint64_t nblk = 2ull << (n - 6);
    const size_t elt = dbl ? 16 : 8;
    const size_t store_bytes = comp ? ((nblk + 255) & ~255ull) + 2 * ((4 * nblk + 255) & ~255ull) + (8ull << n) + 1024
                                    : (elt << n) + 256;
    const size_t per_set = (S + (comp ? 4 : 2)) * store_bytes + 4096;
    if (arena.reserve(per_set * n_sets + (1 << 20)) != MSV_OK)
        return fail_global(MSV_E_NOMEM, "batched adjoint store allocation failed");
    // the sets share the stream: one wait for it, then each simulator is
    // destroyed without its own
    struct Sims {
        hipStream_t stream;
        std::vector<msv_sim *> v;
        std::vector<std::vector<DevMem>> extra;
        ~Sims()
        {
            (void)hipStreamSynchronize(stream);
            for (size_t i = 0; i < v.size(); ++i) {
                for (auto &m : extra[i]) dev_free(v[i], m);
                v[i]->stream_drained = true;
                msv_destroy(v[i]);
            }
        }
    } sims{stream, {}, {}};
    // slot ids per set: 0 .. S-1 checkpoints, then A, B, L0, L1
    const int A = (int)S, B = (int)S + 1, L0 = (int)S + 2, L1 = (int)S + 3;
    std::vector<std::vector<Slot>> slots(n_sets, std::vector<Slot>(S + 4));
    int st;
    for (size_t k = 0; k < n_sets; ++k) {
        msv_sim *s = nullptr;
        if ((st = msv_create(n, dtype, &s))) return st;
        sims.v.push_back(s);
        sims.extra.emplace_back();
        msv_set_stream(s, stream);
        if ((st = msv_set_device_allocator(s, &StoreArena::alloc, &StoreArena::release, &arena)) ||
            (st = msv_set_error_bound(s, eb)) || (st = msv_set_chunk_qubits(s, std::min(n, 20))) ||
            (st = msv_init_basis(s, ansatz->init_basis)))
            return st;
        auto &sl = slots[k];
        auto &ex = sims.extra.back();
        if (comp) {
            sl[0].st = s->st[s->cur];   // the input state
            sl[A].st = s->st[s->cur ^ 1];
            for (int id : {B, L0, L1}) {
                ex.resize(ex.size() + 4);
                DevMem *m = &ex[ex.size() - 4];
                if ((st = dev_alloc(s, m[0], nblk)) || (st = dev_alloc(s, m[1], 4 * nblk)) ||
                    (st = dev_alloc(s, m[2], 4 * nblk)) || (st = dev_alloc(s, m[3], 8ull << n)))
                    return st;
            }
            for (size_t j = 1; j < S; ++j) {
                ex.resize(ex.size() + 4);
                DevMem *m = &ex[ex.size() - 4];
                if ((st = dev_alloc(s, m[0], nblk)) || (st = dev_alloc(s, m[1], 4 * nblk)) ||
                    (st = dev_alloc(s, m[2], 4 * nblk)) || (st = dev_alloc(s, m[3], 8ull << n)))
                    return st;
            }
            // ex holds B, L0, L1, CK_1 .. CK_(S-1), four arrays each
            auto store_of = [&](size_t idx) {
                DevStore d;
                d.W = ex[4 * idx];
                d.A = ex[4 * idx + 1];
                d.OFF = ex[4 * idx + 2];
                d.heap = ex[4 * idx + 3];
                return d;
            };
            sl[B].st = store_of(0);
            sl[L0].st = store_of(1);
            sl[L1].st = store_of(2);
            for (size_t j = 1; j < S; ++j) sl[j].st = store_of(2 + j);
        } else {
            sl[0].amps = s->amps.p;
            const size_t nb_extra = 2 + (S - 1);   // A, L0, CK_1 .. CK_(S-1)
            ex.resize(nb_extra);
            for (size_t i = 0; i < nb_extra; ++i)
                if ((st = dev_alloc(s, ex[i], elt << n))) return st;
            sl[A].amps = ex[0].p;
            sl[B].amps = ex[0].p;
            sl[L0].amps = ex[1].p;
            sl[L1].amps = ex[1].p;
            for (size_t j = 1; j < S; ++j) sl[j].amps = ex[1 + j].p;
        }
    }
    // the store a pass writes when psi is in `cur` (never a checkpoint)
    auto work = [&](int cur) { return comp ? (cur == A ? B : A) : A; };

    // device buffers: ops, pool, masks / coeffs, flags, queue, grad partials,
    // reduction partials and outputs, descriptors and prefixes
    struct Bufs {
        std::vector<void *> p;
        ~Bufs() { for (void *x : p) if (x) (void)hipFree(x); }
        void *get(size_t b)
        {
            void *x = nullptr;
            if (hipMalloc(&x, std::max<size_t>(b, 256)) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            p.push_back(x);
            return x;
        }
    } bufs;
    const size_t pool_bytes = dbl ? pd.size() * 8 : pf.size() * 4;
    const size_t queue_bytes = 256 + 4 * n_sets;
    OpDesc *d_ops = (OpDesc *)bufs.get(ops.size() * sizeof(OpDesc));
    void *d_pool = bufs.get(pool_bytes);
    double *d_obs = (double *)bufs.get(16 * std::max<size_t>(n_terms, 1));
    uint32_t *d_flags = (uint32_t *)bufs.get(256);
    uint8_t *d_queue = (uint8_t *)bufs.get(queue_bytes);
    double *d_grad = (double *)bufs.get(16 * stride * std::max<size_t>(n_slots, 1) * n_sets);
    double *d_gout = (double *)bufs.get(16 * std::max<size_t>(n_slots, 1) * n_sets);
    if (!d_ops || !d_pool || !d_obs || !d_flags || !d_queue || !d_grad || !d_gout)
        return fail_global(MSV_E_NOMEM, "batched adjoint buffer allocation failed");
    // uploads copy from host buffers kept alive until the final synchronisation
    std::deque<std::vector<uint8_t>> keep;
    auto h2d = [&](void *dst, const void *src, size_t b) -> int {
        if (!b) return MSV_OK;
        keep.emplace_back((const uint8_t *)src, (const uint8_t *)src + b);
        if (hipMemcpyAsync(dst, keep.back().data(), b, hipMemcpyHostToDevice, stream) != hipSuccess)
            return hip_fail(nullptr, hipErrorInvalidValue, "batched adjoint upload");
        return MSV_OK;
    };
    std::vector<double> obs_host(2 * n_terms);
    if (n_terms) {
        memcpy(obs_host.data(), masks, 8 * n_terms);
        memcpy(obs_host.data() + n_terms, coeffs, 8 * n_terms);
    }
    if ((st = h2d(d_ops, ops.data(), ops.size() * sizeof(OpDesc))) ||
        (st = h2d(d_pool, dbl ? (const void *)pd.data() : (const void *)pf.data(), pool_bytes)) ||
        (st = h2d(d_obs, obs_host.data(), 16 * n_terms)))
        return st;
    if (hipMemsetAsync(d_flags, 0, 16, stream) != hipSuccess) return hip_fail(nullptr, hipErrorUnknown, "memset");

    auto buffers = [&](size_t k, int in, int out) {
        PassBuffers b{};
        const Slot &si = slots[k][in], &so = slots[k][out];
        if (comp) {
            b.in = si.st.view();
            b.out = so.st.view();
        } else {
            b.amps_in = si.amps;
            b.amps_out = so.amps;
        }
        b.inv_step = comp ? 1.0 / (2.0 * eb) : 0.0;
        b.step = comp ? 2.0 * eb : 0.0;
        b.scale = 1.0;
        b.flags = d_flags;
        b.ops = d_ops;
        b.pool = d_pool;
        return b;
    };
    const uint64_t spin_limit = 1ull << 22;
    auto run_batch = [&](std::vector<BatchDesc> &descs, const char *what) -> int {
        if (descs.empty()) return MSV_OK;
        std::vector<uint64_t> prefix(descs.size());
        uint64_t items = 0;
        int max_k = 0;
        for (size_t i = 0; i < descs.size(); ++i) {
            descs[i].group = queue_group(descs[i].geo.n_tiles);
            prefix[i] = items;
            items += (descs[i].geo.n_tiles + descs[i].group - 1) / descs[i].group;
            max_k = std::max(max_k, (int)descs[i].geo.max_k);
        }
        BatchDesc *dd = (BatchDesc *)bufs.get(descs.size() * sizeof(BatchDesc));
        uint64_t *dp = (uint64_t *)bufs.get(8 * prefix.size());
        if (!dd || !dp) return fail_global(MSV_E_NOMEM, "batched adjoint descriptor allocation failed");
        int e;
        if ((e = h2d(dd, descs.data(), descs.size() * sizeof(BatchDesc))) || (e = h2d(dp, prefix.data(), 8 * prefix.size())))
            return e;
        if (hipMemsetAsync(d_queue, 0, queue_bytes, stream) != hipSuccess)
            return hip_fail(nullptr, hipErrorUnknown, "memset");
        int grid = 0;
        hipError_t he = launch_batch_persistent(dbl, comp, tb, max_k, dd, dp, (int)descs.size(), items,
                                                (unsigned long long *)d_queue, (unsigned int *)(d_queue + 256),
                                                d_flags, spin_limit, &grid, stream);
        if (he != hipSuccess) return hip_fail(nullptr, he, what);
        return MSV_OK;
    };
    auto run_adjoint = [&](std::vector<AdjointDesc> &descs) -> int {
        if (descs.empty()) return MSV_OK;
        std::vector<uint64_t> prefix(descs.size());
        uint64_t items = 0;
        for (size_t i = 0; i < descs.size(); ++i) {
            descs[i].group = queue_group(descs[i].geo.n_tiles);
            prefix[i] = items;
            items += (descs[i].geo.n_tiles + descs[i].group - 1) / descs[i].group;
        }
        AdjointDesc *dd = (AdjointDesc *)bufs.get(descs.size() * sizeof(AdjointDesc));
        uint64_t *dp = (uint64_t *)bufs.get(8 * prefix.size());
        if (!dd || !dp) return fail_global(MSV_E_NOMEM, "batched adjoint descriptor allocation failed");
        int e;
        if ((e = h2d(dd, descs.data(), descs.size() * sizeof(AdjointDesc))) ||
            (e = h2d(dp, prefix.data(), 8 * prefix.size())))
            return e;
        if (hipMemsetAsync(d_queue, 0, queue_bytes, stream) != hipSuccess)
            return hip_fail(nullptr, hipErrorUnknown, "memset");
        int grid = 0;
        hipError_t he = launch_adjoint_persistent(dbl, comp, tb, dd, dp, (int)descs.size(), items,
                                                  (unsigned long long *)d_queue, (unsigned int *)(d_queue + 256),
                                                  d_flags, spin_limit, &grid, stream);
        if (he != hipSuccess) return hip_fail(nullptr, he, "launch_adjoint_persistent");
        return MSV_OK;
    };

    // 1. forward sweep and lambda := O psi, every set in one launch
    std::vector<int> psi(n_sets, 0), lam(n_sets, L0);
    {
        std::vector<BatchDesc> descs;
        std::vector<std::vector<BatchDesc>> per(n_sets);
        for (size_t k = 0; k < n_sets; ++k) {
            int cur = 0;
            uint64_t need = 0;
            for (size_t j = 0; j < S; ++j)
                for (size_t p = 0; p < fgeo[k][j].size(); ++p) {
                    const bool to_ck = p + 1 == fgeo[k][j].size() && j + 1 < S;
                    const int out = to_ck ? (int)(j + 1) : work(cur);
                    BatchDesc d{};
                    d.geo = fgeo[k][j][p];
                    d.buf = buffers(k, cur, out);
                    d.circuit = (uint32_t)k;
                    d.need = need;
                    need += d.geo.n_tiles;
                    per[k].push_back(d);
                    cur = out;
                }
            BatchDesc d{};
            d.geo = obs_g;
            d.buf = buffers(k, cur, L0);
            d.buf.obs_masks = (const uint64_t *)d_obs;
            d.buf.obs_coeffs = d_obs + n_terms;
            d.buf.obs_terms = (int32_t)n_terms;
            d.circuit = (uint32_t)k;
            d.need = need;
            per[k].push_back(d);
            psi[k] = cur;
        }
        // level-major order: items only wait on items queued before them
        for (size_t l = 0;; ++l) {
            bool any = false;
            for (size_t k = 0; k < n_sets; ++k)
                if (l < per[k].size()) {
                    descs.push_back(per[k][l]);
                    any = true;
                }
            if (!any) break;
        }
        if ((st = run_batch(descs, "forward sweep"))) return st;
    }
    // 2. expectation of every final state
    {
        std::vector<ReduceJob> jobs(n_sets);
        const uint64_t groups_max = 2048;
        double *d_part = (double *)bufs.get(32 * groups_max * n_sets);
        double *d_red = (double *)bufs.get(32 * n_sets);
        ReduceJob *d_jobs = (ReduceJob *)bufs.get(sizeof(ReduceJob) * n_sets);
        if (!d_part || !d_red || !d_jobs) return fail_global(MSV_E_NOMEM, "batched adjoint reduction buffers");
        int groups = 0;
        for (size_t k = 0; k < n_sets; ++k) {
            const Slot &sl = slots[k][psi[k]];
            ReduceJob &jb = jobs[k];
            jb.amps = comp ? nullptr : sl.amps;
            if (comp) jb.st = sl.st.view();
            jb.step = comp ? 2.0 * eb : 0.0;
            jb.a.kind = RED_EXPZ;
            jb.a.amp_begin = 0;
            jb.a.amp_count = 1ull << n;
            jb.a.masks = (const uint64_t *)d_obs;
            jb.a.coeffs = d_obs + n_terms;
            jb.a.n_terms = (int32_t)n_terms;
            jb.a.scale = 1.0;
        }
        // every job has the same length, so the same number of groups
        {
            uint64_t g = (((1ull << n) >> 6) + 3) / 4;
            groups = (int)std::max<uint64_t>(1, std::min<uint64_t>(g, groups_max));
        }
        for (size_t k = 0; k < n_sets; ++k) jobs[k].a.partials = d_part + 4 * (uint64_t)groups * k;
        if ((st = h2d(d_jobs, jobs.data(), sizeof(ReduceJob) * n_sets))) return st;
        int g2 = 0;
        hipError_t he = launch_reduce_multi(dbl, comp ? 1 : 0, d_jobs, (int)n_sets, 1ull << n, &g2, stream);
        if (he != hipSuccess || g2 != groups) return hip_fail(nullptr, he != hipSuccess ? he : hipErrorUnknown, "reduce");
        if ((he = launch_reduce_final_multi(d_part, groups, (int)n_sets, d_red, stream)) != hipSuccess)
            return hip_fail(nullptr, he, "reduce final");
        std::vector<double> red(4 * n_sets);
        if (hipMemcpyAsync(red.data(), d_red, 32 * n_sets, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return hip_fail(nullptr, hipErrorUnknown, "expectation read-back");
        for (size_t k = 0; k < n_sets; ++k) expvals[k] = red[4 * k + 1];
    }
    // 3. reverse, one segment at a time, every set in each launch
    for (size_t jj = S; jj-- > 0;) {
        if (jj + 1 < S) {
            std::vector<std::vector<BatchDesc>> per(n_sets);
            for (size_t k = 0; k < n_sets; ++k) {
                int cur = (int)jj;
                uint64_t need = 0;
                for (size_t p = 0; p < fplan[k][jj].size(); ++p) {   // an empty segment needs no recompute
                    const int out = work(cur);
                    BatchDesc d{};
                    d.geo = fgeo[k][jj][p];
                    d.buf = buffers(k, cur, out);
                    d.circuit = (uint32_t)k;
                    d.need = need;
                    need += d.geo.n_tiles;
                    per[k].push_back(d);
                    cur = out;
                }
                psi[k] = cur;
            }
            std::vector<BatchDesc> descs;
            for (size_t l = 0;; ++l) {
                bool any = false;
                for (size_t k = 0; k < n_sets; ++k)
                    if (l < per[k].size()) {
                        descs.push_back(per[k][l]);
                        any = true;
                    }
                if (!any) break;
            }
            if ((st = run_batch(descs, "segment recompute"))) return st;
        }
        std::vector<std::vector<AdjointDesc>> per(n_sets);
        for (size_t k = 0; k < n_sets; ++k) {
            uint64_t need = 0;
            for (const PassGeom &g : rgeo[k][jj]) {
                const int pout = work(psi[k]);
                const int lout = comp ? (lam[k] == L0 ? L1 : L0) : L0;
                AdjointDesc d{};
                d.geo = g;
                d.buf.psi = buffers(k, psi[k], pout);
                d.buf.lam = buffers(k, lam[k], lout);
                d.buf.grad_part = d_grad + 2 * stride * std::max<size_t>(n_slots, 1) * k;
                d.buf.grad_stride = stride;
                d.circuit = (uint32_t)k;
                d.need = need;
                need += g.n_tiles;
                per[k].push_back(d);
                psi[k] = pout;
                lam[k] = lout;
            }
        }
        std::vector<AdjointDesc> descs;
        for (size_t l = 0;; ++l) {
            bool any = false;
            for (size_t k = 0; k < n_sets; ++k)
                if (l < per[k].size()) {
                    descs.push_back(per[k][l]);
                    any = true;
                }
            if (!any) break;
        }
        if ((st = run_adjoint(descs))) return st;
    }
    // 4. gradients
    std::vector<double> gv(2 * std::max<size_t>(n_slots, 1) * n_sets, 0.0);
    if (n_slots) {
        hipError_t he = launch_grad_reduce_multi(d_grad, stride, (int)n_slots, (int)n_sets, d_gout, stream);
        if (he != hipSuccess) return hip_fail(nullptr, he, "grad reduce");
        if (hipMemcpyAsync(gv.data(), d_gout, 16 * n_slots * n_sets, hipMemcpyDeviceToHost, stream) != hipSuccess)
            return hip_fail(nullptr, hipErrorUnknown, "gradient read-back");
    }
    uint32_t flags = 0;
    if (hipMemcpyAsync(&flags, d_flags, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return hip_fail(nullptr, hipErrorUnknown, "batched adjoint read-back");
    if (flags & kFlagQueueTimeout)
        return fail_global(MSV_E_DEVICE, "batched adjoint: a dependency wait exceeded its limit");
    if (flags & 1u) return fail_global(MSV_E_RANGE, "a value left the codec range in the batched adjoint");
    for (size_t k = 0; k < n_sets; ++k) {
        double *g = grads + k * n_params;
        for (size_t p = 0; p < n_params; ++p) g[p] = 0.0;
        for (size_t i = 0; i < n_slots; ++i) g[slot_param[i]] += 2.0 * gv[2 * (k * n_slots + i)];
    }
    return MSV_OK;
}
