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
