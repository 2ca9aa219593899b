// Host-core co-processing of the host store (the paper's online stage step
// (5): CPU cores left idle while the GPU works update a share of the chunks).
//
// A pass over the host store streams chunk groups through the GPU; with the
// option "cpu_share" > 0 a share of the groups instead runs on host threads,
// in the same pass and at the same time: each thread reads a group's
// canonical chunks from the input arena, decodes them, applies the pass's
// fused ops (the planner's host ops: dense k-qubit matrices with controls,
// diagonal tables, controlled linear phases) in FP64, rounds to the state's
// type, encodes, and writes canonical chunks to the output arena. Nothing of
// such a group crosses the host link.
//
// This is the library's own CPU implementation of the chunk format (block by
// block, bit planes packed a word at a time, the three predictors of the
// width byte); it shares nothing with the test oracle.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "internal.h"

namespace msv {

namespace {

using cpx = std::complex<double>;

constexpr uint32_t kMagic = 0x4356534Du;

uint64_t pad8(uint64_t x) { return (x + 7) & ~7ull; }

// Decode one canonical chunk into out[0 .. 2^log2c) (FP64). False when the
// chunk is malformed.
template <typename T>
bool decode_chunk(const uint8_t *p, uint64_t bytes, int log2c, double step, cpx *out)
{
    const uint64_t C = 1ull << log2c, nb = 2 * C / 64;
    if (bytes < 32) return false;
    uint32_t magic;
    memcpy(&magic, p, 4);
    if (magic != kMagic || p[4] != 1 || p[6] != log2c) return false;
    if (p[5] == 0) {
        for (uint64_t i = 0; i < C; ++i) out[i] = 0.0;
        return true;
    }
    uint32_t mode;
    memcpy(&mode, p + 28, 4);
    if (mode > 1) return false;
    const uint8_t *W = p + 32;
    const int32_t *A = (const int32_t *)(p + 32 + pad8(nb));
    const uint64_t *pay = (const uint64_t *)(p + 32 + pad8(nb) + pad8(4 * nb));
    uint64_t words = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        if ((W[b] & 63) > 32 || (W[b] >> 6) > (mode ? 2 : 0)) return false;
        words += W[b] & 63;
    }
    if (32 + pad8(nb) + pad8(4 * nb) + 8 * words != bytes) return false;
    uint64_t off = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        const uint64_t j = b >> 1, plane = b & 1;
        const uint32_t w = W[b] & 63, pred = W[b] >> 6;
        uint32_t q = (uint32_t)A[b], e = 0;   // code and first difference, mod 2^32
        for (int i = 0; i < 64; ++i) {
            uint32_t u = 0;
            for (uint32_t k = 0; k < w; ++k) u |= (uint32_t)((pay[off + k] >> i) & 1ull) << k;
            const uint32_t d = (u >> 1) ^ (0u - (u & 1u));   // zigzag inverse
            if (i > 0) {
                if (pred == 0) q += d;
                else if (pred == 1) q = d;
                else {
                    e += d;
                    q += e;
                }
            }
            const T x = (T)((double)(int32_t)q * step);
            cpx &o = out[j * 64 + (uint64_t)i];
            o = plane ? cpx(o.real(), (double)x) : cpx((double)x, o.imag());
        }
        off += w;
    }
    return true;
}

struct EncodeStats {
    double norm = 0.0, err = 0.0, words = 0.0;
    bool bad = false;
};

// Zigzagged residuals of one block's codes under predictor pred (u[0] = 0)
// and their width.
uint32_t block_residuals(const int32_t *q, uint32_t pred, uint32_t *u)
{
    uint32_t any = 0;
    u[0] = 0;
    for (int i = 1; i < 64; ++i) {
        uint32_t d;
        if (pred == 0) d = (uint32_t)q[i] - (uint32_t)q[i - 1];
        else if (pred == 1) d = (uint32_t)q[i];
        else if (i == 1) d = (uint32_t)q[1] - (uint32_t)q[0];
        else d = (uint32_t)q[i] - 2u * (uint32_t)q[i - 1] + (uint32_t)q[i - 2];
        u[i] = (d << 1) ^ (0u - (d >> 31));
        any |= u[i];
    }
    return any ? 32u - (uint32_t)__builtin_clz(any) : 0u;
}

// Encode C = 2^log2c values (rounded to T first) as a canonical chunk into
// out (capacity: the chunk bound) in predictor mode pred_mode; returns its
// size.
template <typename T>
uint64_t encode_chunk(const cpx *v, int log2c, int dtype, double eb, double inv_step, double step, int pred_mode,
                      uint8_t *out, EncodeStats &st)
{
    const uint64_t C = 1ull << log2c, nb = 2 * C / 64;
    uint8_t *W = out + 32;
    int32_t *A = (int32_t *)(out + 32 + pad8(nb));
    uint64_t *pay = (uint64_t *)(out + 32 + pad8(nb) + pad8(4 * nb));
    memset(out + 32, 0, pad8(nb) + pad8(4 * nb));
    uint64_t off = 0;
    bool zero = true;
    for (uint64_t b = 0; b < nb; ++b) {
        const uint64_t j = b >> 1, plane = b & 1;
        int32_t q[64];
        uint32_t u[64];
        for (int i = 0; i < 64; ++i) {
            const cpx &c = v[j * 64 + (uint64_t)i];
            const T x = (T)(plane ? c.imag() : c.real());
            const double xd = (double)x;
            if (!plane) st.norm += xd * xd + (double)(T)c.imag() * (double)(T)c.imag();
            const double r = std::rint(xd * inv_step);
            if (!std::isfinite(xd) || std::fabs(r) > 1073741823.0) {
                st.bad = true;
                q[i] = 0;
            } else {
                q[i] = (int32_t)r;
            }
            const T xr = (T)((double)q[i] * step);
            st.err = std::max(st.err, (double)std::fabs(x - xr));
        }
        uint32_t w = block_residuals(q, 0, u), pred = 0;
        if (pred_mode) {
            for (uint32_t p = 1; p <= 2; ++p) {
                const uint32_t wp = block_residuals(q, p, u);
                if (wp < w) {
                    w = wp;
                    pred = p;
                }
            }
            block_residuals(q, pred, u);
        }
        W[b] = (uint8_t)(w | (pred << 6));
        A[b] = q[0];
        if (w || q[0]) zero = false;
        for (uint32_t k = 0; k < w; ++k) {
            uint64_t plane_word = 0;
            for (int i = 0; i < 64; ++i) plane_word |= (uint64_t)((u[i] >> k) & 1u) << i;
            pay[off + k] = plane_word;
        }
        off += w;
    }
    st.words += (double)off;
    const uint64_t total = zero ? 32 : 32 + pad8(nb) + pad8(4 * nb) + 8 * off;
    const uint32_t magic = kMagic, nbl = (uint32_t)nb, mode32 = (uint32_t)pred_mode;
    memcpy(out, &magic, 4);
    out[4] = 1;
    out[5] = zero ? 0 : 1;
    out[6] = (uint8_t)log2c;
    out[7] = (uint8_t)dtype;
    memcpy(out + 8, &eb, 8);
    memcpy(out + 16, &total, 8);
    memcpy(out + 24, &nbl, 4);
    memcpy(out + 28, &mode32, 4);
    return total;
}

// Global qubit -> bit of the group-local index (in-chunk bits, then the
// group's crossing qubits Hq), or -1 when the qubit is fixed for the group.
struct GroupMap {
    int c;
    std::vector<int> lb;   // per qubit
    uint64_t base;         // global index bits of the fixed qubits
    uint64_t global(uint64_t li) const
    {
        uint64_t g = base | (li & ((1ull << c) - 1));
        for (size_t q = (size_t)c; q < lb.size(); ++q)
            if (lb[q] >= 0 && ((li >> lb[q]) & 1ull)) g |= 1ull << q;
        return g;
    }
};

void apply_ops(const Pass &pass, const GroupMap &gm, std::vector<cpx> &a)
{
    const uint64_t L = a.size();
    std::vector<uint64_t> gidx(L);
    for (uint64_t li = 0; li < L; ++li) gidx[li] = gm.global(li);
    for (const HostOp &h : pass.ops) {
        if (h.type == OP_DENSE) {
            const int k = (int)h.q.size(), D = 1 << k;
            std::vector<int> bits(k);
            uint64_t mask = 0;
            for (int m = 0; m < k; ++m) {
                bits[m] = gm.lb[h.q[m]];
                mask |= 1ull << bits[m];
            }
            std::vector<cpx> in(D);
            std::vector<uint64_t> idx(D);
            for (uint64_t li = 0; li < L; ++li) {
                if (li & mask) continue;   // visit each group of 2^k once, from its all-zero member
                if ((gidx[li] & h.ctrl_mask) != h.ctrl_mask) continue;
                for (int s = 0; s < D; ++s) {
                    uint64_t x = li;
                    for (int m = 0; m < k; ++m)
                        if ((s >> m) & 1) x |= 1ull << bits[m];
                    idx[s] = x;
                    in[s] = a[x];
                }
                for (int r = 0; r < D; ++r) {
                    cpx acc = 0.0;
                    for (int s = 0; s < D; ++s) acc += h.m[(size_t)r * D + s] * in[s];
                    a[idx[r]] = acc;
                }
            }
        } else if (h.type == OP_DIAG) {
            for (uint64_t li = 0; li < L; ++li) {
                uint64_t s = 0;
                for (size_t m = 0; m < h.q.size(); ++m) s |= ((gidx[li] >> h.q[m]) & 1ull) << m;
                a[li] *= h.m[s];
            }
        } else if (h.type == OP_PHASE) {
            for (uint64_t li = 0; li < L; ++li) {
                const uint64_t g = gidx[li];
                double ph = 0.0;
                for (size_t q = 0; q < h.mu.size(); ++q)
                    if ((g >> q) & 1ull) ph += h.mu[q];
                if (h.hub >= 0 && ((g >> h.hub) & 1ull))
                    for (size_t q = 0; q < h.lam.size(); ++q)
                        if ((g >> q) & 1ull) ph += h.lam[q];
                a[li] *= h.global * cpx(std::cos(ph), std::sin(ph));
            }
        }
    }
}

template <typename T>
int run_group(msv_sim *s, const Pass &pass, const std::vector<uint64_t> &chunks, const std::vector<int> &Hq,
              int in_side, int out_side, double scale, EncodeStats &st)
{
    HostStore &h = s->hs;
    const int c = s->log2c;
    const uint64_t C = 1ull << c;
    GroupMap gm;
    gm.c = c;
    gm.lb.assign(s->n, -1);
    for (int q = 0; q < c; ++q) gm.lb[q] = q;
    for (size_t j = 0; j < Hq.size(); ++j) gm.lb[Hq[j]] = c + (int)j;
    gm.base = chunks[0] << c;   // chunk 0 of the group has every Hq bit 0
    std::vector<cpx> a(C * chunks.size());
    for (size_t k = 0; k < chunks.size(); ++k) {
        const uint64_t ch = chunks[k];
        if (!decode_chunk<T>(h.arena[in_side].at(h.pos[in_side][ch]), h.bytes[in_side][ch], c, s->step(),
                             a.data() + k * C))
            return MSV_E_CORRUPT;
    }
    if (scale != 1.0)
        for (cpx &x : a) x = cpx((double)(T)((T)x.real() * (T)scale), (double)(T)((T)x.imag() * (T)scale));
    apply_ops(pass, gm, a);
    const uint64_t nb = 2 * C / 64;
    std::vector<uint8_t> buf(32 + pad8(nb) + pad8(4 * nb) + 8 * 32 * nb);
    for (size_t k = 0; k < chunks.size(); ++k) {
        const uint64_t bytes = encode_chunk<T>(a.data() + k * C, c, s->is_double() ? 0 : 1, s->eb, s->inv_step(),
                                               s->step(), s->pred_mode, buf.data(), st);
        uint64_t pos = 0;
        int e = host_arena_alloc(s, out_side, bytes, &pos);   // serialised inside
        if (e) return e;
        memcpy(h.arena[out_side].at(pos), buf.data(), bytes);
        h.pos[out_side][chunks[k]] = pos;
        h.bytes[out_side][chunks[k]] = bytes;
    }
    return MSV_OK;
}

}  // namespace

int cpu_group_pass(msv_sim *s, const Pass &pass, const std::vector<uint64_t> &chunks, const std::vector<int> &Hq,
                   int in_side, int out_side, double scale, double *norm, double *err, double *words, bool *bad)
{
    EncodeStats st;
    const int r = s->is_double() ? run_group<double>(s, pass, chunks, Hq, in_side, out_side, scale, st)
                                 : run_group<float>(s, pass, chunks, Hq, in_side, out_side, scale, st);
    *norm += st.norm;
    *err = std::max(*err, st.err);
    *words += st.words;
    *bad = *bad || st.bad;
    return r;
}

}  // namespace msv
