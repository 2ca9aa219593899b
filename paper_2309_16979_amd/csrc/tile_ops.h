// Device-side building blocks of a tile pass, shared by the single-state pass
// kernel and the two-state adjoint kernel.
//
// A tile is 2^TB amplitudes held in LDS as two planes (re, im). Tile-local bit
// i is global qubit geo.tile_q[i]; bits 0..5 are qubits 0..5, so a tile is a
// set of whole 64-amplitude codec blocks. Every function here is called by
// all threads of the workgroup.
#pragma once
#include <hip/hip_runtime.h>

#include "codec_device.h"
#include "kernels.h"

namespace msv {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using V = float2; };
template <> struct Cplx<double> { using V = double2; };

// Op coefficients (matrices, diagonal tables) are read-only for the whole
// launch and, per op, the same for every thread: reading them through the
// constant address space lets the compiler fetch them with scalar loads into
// SGPRs instead of one vector load per thread into VGPRs.
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ ConstPtr<T> as_const(const T *p)
{
    return (ConstPtr<T>)p;
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float absT(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double absT(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float maxT(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double maxT(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ uint64_t block_index(const BlockStore &s, uint64_t B)
{
    if (!s.chunk_slot) return B;
    const uint64_t nbm = (1ull << s.log2_nb) - 1;
    return ((uint64_t)s.chunk_slot[B >> s.log2_nb] << s.log2_nb) | (B & nbm);
}

// One op descriptor through the constant address space: the index is the
// same for every thread, so the words arrive by scalar loads in SGPRs.
__device__ __forceinline__ OpDesc load_op(const OpDesc *p)
{
    static_assert(sizeof(OpDesc) % 4 == 0, "OpDesc is read as 32-bit words");
    OpDesc o;
    const ConstPtr<uint32_t> w = as_const(reinterpret_cast<const uint32_t *>(p));
    uint32_t *d = reinterpret_cast<uint32_t *>(&o);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(OpDesc) / 4); ++i) d[i] = w[i];
    return o;
}

// Workgroups go to the 8 XCDs in turn (workgroup b to XCD b mod 8), each
// with its own L2. Tile b' = (b mod 8) (n / 8) + b / 8 of a grid of n gives
// every XCD one contiguous eighth of the tiles, so neighbouring tiles, whose
// block records and payloads share cache lines, meet in the same L2.
__device__ __forceinline__ uint32_t xcd_tile()
{
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    return (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
}

// ------------------------------------------------------------- geometry

// LDS position of tile element l within its plane: bits 6.. are XOR-folded
// onto bits 0..5. The map is its own inverse and linear over XOR, so
// swz(a | b) = swz(a) ^ swz(b) for disjoint a, b. Accesses whose 64 lanes
// vary over tile bits above 5 (register segments and dense ops on low
// qubits) then spread over the LDS banks instead of hitting a few.
__device__ __forceinline__ int swz(int l) { return l ^ ((l >> 6) & 63); }

// Global index of the tile's amplitude 0: the tile id's bits deposited into
// the non-tile positions in ascending order.
__device__ __forceinline__ uint64_t tile_base(const PassGeom &geo, uint64_t tile)
{
    uint64_t base = 0, m = geo.nontile_mask, t = tile;
    while (m) {
        const uint64_t low = m & (~m + 1ull);
        if (t & 1ull) base |= low;
        t >>= 1;
        m &= m - 1;
    }
    return base;
}

// sG[jb] = global 64-amplitude block index of tile block jb.
template <int TB>
__device__ __forceinline__ void tile_blocks(const PassGeom &geo, uint64_t base, uint64_t *sG)
{
    constexpr int NAB = 1 << (TB - 6);
    for (int jb = threadIdx.x; jb < NAB; jb += kThreads) {
        uint64_t G = base >> 6;
#pragma unroll
        for (int i = 0; i < TB - 6; ++i)
            if ((jb >> i) & 1) G |= 1ull << (geo.tile_q[6 + i] - 6);
        sG[jb] = G;
    }
}

// ------------------------------------------------------------------ load

// stage: 128 words of LDS for this wave, through which the compressed decode
// broadcasts plane words (unpack_codes4_lds). PRED = false: every block of
// the input uses predictor 0.
template <typename T, int TB, bool LOADC, bool PRED = true, bool XP = true>
__device__ __forceinline__ void tile_load(T *sre, T *sim, const uint64_t *sG, const void *amps, const BlockStore &in,
                                          double step, double sc, int wave, int lane, uint64_t *stage)
{
    constexpr int NAB = 1 << (TB - 6), NSB = 2 * NAB, NW = kThreads / 64;
    using V2 = typename Cplx<T>::V;
    const T scale = (T)sc;
    if (!LOADC) {
        // every load of the wave in flight before the first LDS write
        constexpr int PER = (NAB + NW - 1) / NW;
        const V2 *a = (const V2 *)amps;
        V2 v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int jb = wave + NW * i;
            if (jb < NAB) v[i] = a[(sG[jb] << 6) | (uint64_t)lane];
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int jb = wave + NW * i;
            if (jb < NAB) {
                v[i].x *= scale;   // exact when scale is 1
                v[i].y *= scale;
                const int p = swz(jb * 64 + lane);
                sre[p] = v[i].x;
                sim[p] = v[i].y;
            }
        }
        return;
    }
    // Compressed: the wave decodes amplitude blocks jb = wave + NW * a, both
    // planes together, in rounds of up to 16. Lane j < 32 fetches the width,
    // anchor and payload offset of amplitude block a = r0 + j / 2, plane j & 1;
    // then every block's payload word `lane` is loaded, and one wait covers
    // all of them before the bit planes are unpacked.
    constexpr int APW = (NAB + NW - 1) / NW;   // amplitude blocks per wave
    constexpr int RA = APW < 16 ? APW : 16;
    for (int r0 = 0; r0 < APW; r0 += RA) {
        uint32_t wv = 0, ov = 0;
        int32_t av = 0;
        {
            const int a = r0 + (lane >> 1);
            const int jb = wave + NW * a;
            if (lane < 2 * RA && a < APW && jb < NAB) {
                const uint64_t bi = block_index(in, 2 * sG[jb] + (uint64_t)(lane & 1));
                wv = in.W[bi];
                av = in.A[bi];
                if (wv) ov = in.OFF[bi];
            }
        }
        uint64_t mine[2 * RA];
#pragma unroll
        for (int j = 0; j < 2 * RA; ++j) {
            const uint32_t wj = (uint32_t)__builtin_amdgcn_readlane((int)wv, j);
            const uint32_t W = PRED ? wbyte_width(wj) : wj;   // without PRED the byte is the width
            const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)ov, j);
            mine[j] = 0;
            if ((uint32_t)lane < W) mine[j] = in.heap[(uint64_t)off + lane];
        }
        if constexpr (RA % 2 == 0 && APW % RA == 0 && NAB % NW == 0) {
            // two amplitude blocks (four stream blocks) per unpack loop
#pragma unroll
            for (int a = 0; a < RA; a += 2) {
                const int jb = wave + NW * (r0 + a);
                uint32_t W4[4];
                int32_t A4[4], q4[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    W4[p] = (uint32_t)__builtin_amdgcn_readlane((int)wv, 2 * a + p);
                    A4[p] = __builtin_amdgcn_readlane(av, 2 * a + p);
                }
                if (lane < 32) {
#pragma unroll
                    for (int p = 0; p < 4; ++p) stage[32 * p + lane] = mine[2 * a + p];
                }
                unpack_codes4_lds<PRED, XP>(stage, W4, A4, q4);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    T xr = dequantize<T>(q4[2 * h], step), xi = dequantize<T>(q4[2 * h + 1], step);
                    xr *= scale;   // exact when scale is 1
                    xi *= scale;
                    const int p = swz((jb + NW * h) * 64 + lane);
                    sre[p] = xr;
                    sim[p] = xi;
                }
            }
        } else {
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const int jb = wave + NW * (r0 + a);
                if (r0 + a >= APW || jb >= NAB) break;
                int32_t qr, qi;
                unpack_codes2<PRED>(mine[2 * a], (uint32_t)__builtin_amdgcn_readlane((int)wv, 2 * a),
                              __builtin_amdgcn_readlane(av, 2 * a), mine[2 * a + 1],
                              (uint32_t)__builtin_amdgcn_readlane((int)wv, 2 * a + 1),
                              __builtin_amdgcn_readlane(av, 2 * a + 1), qr, qi);
                T xr = dequantize<T>(qr, step), xi = dequantize<T>(qi, step);
                xr *= scale;   // exact when scale is 1
                xi *= scale;
                const int p = swz(jb * 64 + lane);
                sre[p] = xr;
                sim[p] = xi;
            }
        }
    }
}

// ----------------------------------------------------------- expectation

// This thread's share of sum_t c_t <psi| Z(m_t) |psi> (t < n_terms <= 64)
// over the tile, taken on the values the store will hold: the decoder's
// values (T)(q * 2 eb) when storing compressed, the amplitudes themselves
// otherwise. Per 64-amplitude block G (lane = index bits 0..5) the sum is
// sum_t c_t (-1)^popcount(G & h_t) P^(l_t) with l_t / h_t the low 6 / high
// bits of m_t and P^ the Walsh-Hadamard transform of the block's
// probabilities over the lanes, the same form as the reduction kernel.
template <typename T, int TB, bool STOREC>
__device__ __forceinline__ double tile_expect(const T *sre, const T *sim, const uint64_t *sG, const uint64_t *masks,
                                              const double *coeffs, int n_terms, double inv_step, double step,
                                              int wave, int lane)
{
    constexpr int NAB = 1 << (TB - 6), NW = kThreads / 64;
    double ct = 0.0;
    uint64_t mhi = 0;
    int lsrc = 0;
    if (lane < n_terms) {
        ct = coeffs[lane];
        mhi = masks[lane] >> 6;
        lsrc = (int)(masks[lane] & 63u);
    }
    const double s0 = (lane & 1) ? -1.0 : 1.0, s1 = (lane & 2) ? -1.0 : 1.0, s2 = (lane & 4) ? -1.0 : 1.0,
                 s3 = (lane & 8) ? -1.0 : 1.0, s4 = (lane & 16) ? -1.0 : 1.0, s5 = (lane & 32) ? -1.0 : 1.0;
    double acc = 0.0;
    for (int jb = wave; jb < NAB; jb += NW) {
        const int l = swz(jb * 64 + lane);
        double xr = (double)sre[l], xi = (double)sim[l];
        if (STOREC) {
            const double rr = __builtin_rint(xr * inv_step), ri = __builtin_rint(xi * inv_step);
            xr = __builtin_fabs(rr) <= 1073741823.0 ? (double)(T)(rr * step) : 0.0;
            xi = __builtin_fabs(ri) <= 1073741823.0 ? (double)(T)(ri * step) : 0.0;
        }
        double P = xr * xr + xi * xi;
        P = __builtin_fma(s0, P, __shfl_xor(P, 1, 64));
        P = __builtin_fma(s1, P, __shfl_xor(P, 2, 64));
        P = __builtin_fma(s2, P, __shfl_xor(P, 4, 64));
        P = __builtin_fma(s3, P, __shfl_xor(P, 8, 64));
        P = __builtin_fma(s4, P, __shfl_xor(P, 16, 64));
        P = __builtin_fma(s5, P, __shfl_xor(P, 32, 64));
        const double ph = __shfl(P, lsrc, 64);
        acc += ((__popcll(sG[jb] & mhi) & 1) ? -ct : ct) * ph;
    }
    return acc;
}

// ----------------------------------------------------------------- store

// Predictor mode 1 for one block held as Lorenzo-1 zigzags (*u_p, this
// lane's value) with width byte *w_p and anchor A: the codes come back as A
// plus the prefix sums of the residuals; when predictor 1 or 2 needs fewer
// bits, its zigzags replace *u_p and *w_p becomes width | predictor << 8
// (lane 0 writes it).
__device__ __forceinline__ void repredict(uint32_t *u_p, uint32_t *w_p, int32_t A, int lane)
{
    const uint32_t u = *u_p;
    const uint32_t d = (u >> 1) ^ (0u - (u & 1u));
    const int32_t q = (int32_t)((uint32_t)A + wave_inclusive_sum(d));
    uint32_t un, u2;
    residuals_alt(q, (int32_t)d, un, u2);
    const uint32_t w1 = *w_p, wn = block_width(un), w2 = block_width(u2);
    uint32_t w = w1, pred = 0, best = u;
    if (wn < w) {
        w = wn;
        pred = 1;
        best = un;
    }
    if (w2 < w) {
        w = w2;
        pred = 2;
        best = u2;
    }
    if (pred) {
        *u_p = best;
        if (lane == 0) *w_p = w | (pred << 8);
    }
}

// Store the tile (plain or encoded). nrm / err accumulate this thread's FP64
// sum |x|^2 and max |x - x'|; the return value is the tile's payload words
// (valid in every thread). The codec scratch sW / sA / sOff holds NSB entries;
// sW holds width | predictor << 8. pred_mode 0: Lorenzo-1 for every block;
// 1: per block the predictor of smallest width (compiled in when PRED; the
// variants without it keep the register budget of the Lorenzo-1 path).
// OWN_OFF: `own_off` (2^(TB-5) words of LDS for this wave) receives the
// payload offsets: every wave scans the widths itself (E2), so E3 needs no
// second barrier. Otherwise wave 0 scans into sOff.
// XP: bit planes of four blocks whose widths are all <= 8 by one half-wave
// transpose (store_planes4_bytes); false keeps one ballot per plane and block.
template <typename T, int TB, bool STOREC, bool OWN_OFF = false, bool PRED = true, bool XP = true>
__device__ __forceinline__ uint32_t tile_store(T *sre, T *sim, const uint64_t *sG, uint32_t *sW, int32_t *sA,
                                               uint32_t *sOff, void *amps, const BlockStore &out, uint64_t slot,
                                               double inv_step, double step, int check, int pred_mode,
                                               uint32_t *flags,
                                               double &nrm, double &err, int wave, int lane,
                                               uint32_t *own_off = nullptr)
{
    constexpr int NAB = 1 << (TB - 6), NSB = 2 * NAB, NW = kThreads / 64;
    constexpr int VPT = sizeof(T) / 4;
    using V2 = typename Cplx<T>::V;
    if (!STOREC) {
        V2 *a = (V2 *)amps;
        for (int jb = wave; jb < NAB; jb += NW) {
            V2 v;
            const int p = swz(jb * 64 + lane);
            v.x = sre[p];
            v.y = sim[p];
            const double xr = v.x, xi = v.y;
            nrm += xr * xr + xi * xi;
            a[(sG[jb] << 6) | (uint64_t)lane] = v;
        }
        return 0;
    }
    bool bad = false;
    // |x - x'| in T is exact: x' = 0 when the code is 0, and otherwise x and
    // x' have the same sign and are within a factor of two of each other
    // (|x - q step| <= step / 2 with |q| >= 1), so the subtraction loses
    // nothing (Sterbenz). The FP64 maximum equals the maximum taken in T.
    T errt = 0;
    // E1 (per amplitude block, both planes): codes, residuals, widths; the
    // zigzag residuals replace the values in LDS. Two amplitude blocks per
    // iteration when the wave has an even number of them (independent
    // chains for the scheduler; sums keep the one-block order).
    constexpr bool E1_PAIR = NAB % (2 * NW) == 0;
    double nrm_im = 0.0;   // second FMA chain of the norm (imaginary parts)
    if constexpr (E1_PAIR) for (int jb = wave; jb < NAB; jb += 2 * NW) {
        const int jc = jb + NW;
        const int l0 = swz(jb * 64 + lane), l1 = swz(jc * 64 + lane);
        const T x[4] = {sre[l0], sim[l0], sre[l1], sim[l1]};
        double d[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) d[p] = (double)x[p];
        nrm = __builtin_fma(d[0], d[0], nrm);
        nrm_im = __builtin_fma(d[1], d[1], nrm_im);
        nrm = __builtin_fma(d[2], d[2], nrm);
        nrm_im = __builtin_fma(d[3], d[3], nrm_im);
        // codes (quantize, written out so that the check below reuses the
        // rounded FP64 value: q = r exactly whenever r is in range)
        int32_t q[4];
        double r[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            r[p] = __builtin_rint(d[p] * inv_step);
            const bool ok = __builtin_fabs(r[p]) <= 1073741823.0;
            bad |= !ok;
            q[p] = ok ? (int32_t)r[p] : 0;
        }
        if (check) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T yr = (T)(r[2 * h] * step), yi = (T)(r[2 * h + 1] * step);
                errt = maxT(errt, maxT(absT(x[2 * h] - yr), absT(x[2 * h + 1] - yi)));
            }
        }
        uint32_t u[4], W4[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) u[p] = residual_zigzag(q[p]);
        // widths: when every zigzag of the four blocks fits a byte, one OR
        // reduction over the four packed side by side gives all four
        if (__builtin_amdgcn_ballot_w64((u[0] | u[1] | u[2] | u[3]) > 255u) == 0) {
            const uint32_t o = wave_or(u[0] | (u[1] << 8) | (u[2] << 16) | (u[3] << 24));
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t b = (o >> (8 * p)) & 255u;
                W4[p] = b ? 32u - (uint32_t)__builtin_clz(b) : 0u;
            }
        } else {
            block_width4(u, W4);
        }
        reinterpret_cast<uint32_t *>(sre)[l0 * VPT] = u[0];
        reinterpret_cast<uint32_t *>(sim)[l0 * VPT] = u[1];
        reinterpret_cast<uint32_t *>(sre)[l1 * VPT] = u[2];
        reinterpret_cast<uint32_t *>(sim)[l1 * VPT] = u[3];
        if (lane == 0) {   // lane 0 holds the anchors q_0 itself
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                sW[2 * jb + (p & 1) + 2 * NW * (p >> 1)] = W4[p];
                sA[2 * jb + (p & 1) + 2 * NW * (p >> 1)] = q[p];
            }
        }
    }
    if constexpr (!E1_PAIR) for (int jb = wave; jb < NAB; jb += NW) {
        const int l = swz(jb * 64 + lane);
        const T xr = sre[l], xi = sim[l];
        const double dr = (double)xr, di = (double)xi;
        nrm += dr * dr + di * di;
        const int32_t qr = quantize<T>(xr, inv_step, bad);
        const int32_t qi = quantize<T>(xi, inv_step, bad);
        if (check) {
            const T yr = dequantize<T>(qr, step), yi = dequantize<T>(qi, step);
            errt = maxT(errt, maxT(absT(xr - yr), absT(xi - yi)));
        }
        const uint32_t ur = residual_zigzag(qr);
        const uint32_t ui = residual_zigzag(qi);
        uint32_t Wr, Wi;
        block_width2(ur, ui, Wr, Wi);
        const int32_t Ar = __builtin_amdgcn_readlane(qr, 0);
        const int32_t Ai = __builtin_amdgcn_readlane(qi, 0);
        reinterpret_cast<uint32_t *>(sre)[l * VPT] = ur;
        reinterpret_cast<uint32_t *>(sim)[l * VPT] = ui;
        if (lane == 0) {
            sW[2 * jb] = Wr;
            sW[2 * jb + 1] = Wi;
            sA[2 * jb] = Ar;
            sA[2 * jb + 1] = Ai;
        }
    }
    // E1b (predictor mode 1): each wave revisits its own blocks; the codes come
    // back from the Lorenzo-1 zigzags in LDS (prefix sums from the anchor), the
    // other two predictors' residuals and widths are formed, and a block whose
    // width shrinks takes the better predictor (ties to the lower id)
    if (PRED && pred_mode) {
#pragma unroll 1
        for (int jb = wave; jb < NAB; jb += NW) {
            const int l = swz(jb * 64 + lane);
            uint32_t *ur_p = reinterpret_cast<uint32_t *>(sre) + l * VPT;
            uint32_t *ui_p = reinterpret_cast<uint32_t *>(sim) + l * VPT;
            repredict(ur_p, sW + 2 * jb, sA[2 * jb], lane);
            repredict(ui_p, sW + 2 * jb + 1, sA[2 * jb + 1], lane);
        }
    }
    nrm += nrm_im;
    err = fmax(err, (double)errt);
    if (bad) atomicOr(flags, 1u);
    __syncthreads();
    // E2: exclusive scan of the widths over the tile's blocks
    uint32_t *const so = OWN_OFF ? own_off : sOff;
    if (OWN_OFF || wave == 0) {
        constexpr int PER = (NSB + 63) / 64;
        uint32_t v[PER];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = lane * PER + i;
            v[i] = idx < NSB ? (PRED ? sW[idx] & 0xffu : sW[idx]) : 0u;
            s += v[i];
        }
        uint32_t ex = wave_inclusive_sum(s) - s;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = lane * PER + i;
            if (idx < NSB) so[idx] = ex;
            ex += v[i];
        }
    }
    if (!OWN_OFF) __syncthreads();
    // E3: bit planes of both planes into this tile's heap slot; then lane j
    // of the wave writes width, anchor and offset of the wave's stream block j
    if constexpr (NAB % (2 * NW) == 0) {
        for (int jb = wave; jb < NAB; jb += 2 * NW) {
            const int jc = jb + NW;
            const int l0 = swz(jb * 64 + lane), l1 = swz(jc * 64 + lane);
            const uint32_t u[4] = {reinterpret_cast<const uint32_t *>(sre)[l0 * VPT],
                                   reinterpret_cast<const uint32_t *>(sim)[l0 * VPT],
                                   reinterpret_cast<const uint32_t *>(sre)[l1 * VPT],
                                   reinterpret_cast<const uint32_t *>(sim)[l1 * VPT]};
            constexpr uint32_t WM = PRED ? 0xffu : ~0u;   // without PRED sW holds the width alone
            const uint32_t W4[4] = {sW[2 * jb] & WM, sW[2 * jb + 1] & WM, sW[2 * jc] & WM, sW[2 * jc + 1] & WM};
            const uint32_t o4[4] = {so[2 * jb], so[2 * jb + 1], so[2 * jc], so[2 * jc + 1]};
            if (XP && max(max(W4[0], W4[1]), max(W4[2], W4[3])) <= 8u) {
                store_planes4_bytes(u, W4[0], W4[1], W4[2], W4[3], o4[0], o4[1], o4[2], o4[3], out.heap + slot,
                                    (uint32_t)lane);
            } else {
                uint64_t m[4];
                pack_planes4(u, W4, m);
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if ((uint32_t)lane < W4[p]) out.heap[slot + o4[p] + lane] = m[p];
            }
        }
    } else {
        for (int jb = wave; jb < NAB; jb += NW) {
            const int l = swz(jb * 64 + lane);
            const uint32_t ur = reinterpret_cast<const uint32_t *>(sre)[l * VPT];
            const uint32_t ui = reinterpret_cast<const uint32_t *>(sim)[l * VPT];
            constexpr uint32_t WM = PRED ? 0xffu : ~0u;
            const uint32_t Wr = sW[2 * jb] & WM, Wi = sW[2 * jb + 1] & WM;
            const uint64_t mr = pack_planes(ur, Wr);
            const uint64_t mi = pack_planes(ui, Wi);
            if ((uint32_t)lane < Wr) out.heap[slot + so[2 * jb] + lane] = mr;
            if ((uint32_t)lane < Wi) out.heap[slot + so[2 * jb + 1] + lane] = mi;
        }
    }
    constexpr int APW = (NAB + NW - 1) / NW;
    for (int j0 = 0; j0 < 2 * APW; j0 += 64) {
        const int j = j0 + lane;                 // stream block j of the wave: amplitude block j / 2
        const int jb = wave + NW * (j >> 1);
        if (j < 2 * APW && jb < NAB) {
            const int bt = 2 * jb + (j & 1);
            const uint64_t bi = block_index(out, 2 * sG[jb] + (uint64_t)(j & 1));
            out.W[bi] = PRED ? (uint8_t)((sW[bt] & 63u) | ((sW[bt] >> 8) << 6)) : (uint8_t)sW[bt];
            out.A[bi] = sA[bt];
            out.OFF[bi] = (uint32_t)(slot + so[bt]);
        }
    }
    return so[NSB - 1] + (PRED ? sW[NSB - 1] & 0xffu : sW[NSB - 1]);
}

// ------------------------------------------------------------------- ops

// Dense 2^K x 2^K complex matrix on tile-local bits op.pos[0..K), matrix index
// s = sum_m b(pos[m]) 2^m. Each work item loads its group of 2^K amplitudes
// into registers and writes RPT output rows; when there are fewer groups than
// threads, adjacent lanes of one wave share a group (all loads of a wave are
// issued before its stores, so sharing is race-free).
template <typename T, int TB, int K, bool REAL>
__device__ __forceinline__ void op_dense(T *__restrict__ sre, T *__restrict__ sim, const OpDesc &op,
                                         const T *__restrict__ M)
{
    constexpr int D = 1 << K;
    constexpr int NG = (1 << TB) >> K;
    constexpr int TPG0 = NG >= kThreads ? 1 : kThreads / NG;
    constexpr int TPG = TPG0 < D ? TPG0 : D;
    constexpr int RPT = D / TPG;
    int sp[K];
#pragma unroll
    for (int m = 0; m < K; ++m) sp[m] = op.pos[m];
#pragma unroll
    for (int i = 1; i < K; ++i)
#pragma unroll
        for (int j = i; j > 0; --j)
            if (sp[j - 1] > sp[j]) { int t = sp[j]; sp[j] = sp[j - 1]; sp[j - 1] = t; }
    int offs[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        int o = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if ((s >> m) & 1) o |= 1 << op.pos[m];
        offs[s] = swz(o);
    }
    const int cl = (int)op.ctrl_local;
    for (int w = threadIdx.x; w < NG * TPG; w += kThreads) {
        const int g = w / TPG, rb = w % TPG;
        int l0 = g;
#pragma unroll
        for (int m = 0; m < K; ++m) l0 = ((l0 >> sp[m]) << (sp[m] + 1)) | (l0 & ((1 << sp[m]) - 1));
        if ((l0 & cl) != cl) continue;
        const int p0 = swz(l0);
        T vr[D], vi[D];
#pragma unroll
        for (int s = 0; s < D; ++s) { vr[s] = sre[p0 ^ offs[s]]; vi[s] = sim[p0 ^ offs[s]]; }
#pragma unroll
        for (int rr = 0; rr < RPT; ++rr) {
            const int r = rb * RPT + rr;
            T ar = 0, ai = 0;
            if (REAL) {
#pragma unroll
                for (int s = 0; s < D; ++s) {
                    const T mr = M[2 * (r * D + s)];
                    ar = fmaT(mr, vr[s], ar);
                    ai = fmaT(mr, vi[s], ai);
                }
            } else {
#pragma unroll
                for (int s = 0; s < D; ++s) {
                    const T mr = M[2 * (r * D + s)], mi = M[2 * (r * D + s) + 1];
                    ar = fmaT(mr, vr[s], ar);
                    ar = fmaT(-mi, vi[s], ar);
                    ai = fmaT(mr, vi[s], ai);
                    ai = fmaT(mi, vr[s], ai);
                }
            }
            int lr = p0;
#pragma unroll
            for (int s = 0; s < D; ++s)
                if (s == r) lr = p0 ^ offs[s];
            sre[lr] = ar;
            sim[lr] = ai;
        }
    }
}

// Bit s of a diagonal table index: table bit m is global qubit gq[m], taken
// from the tile-local index (pos[m] >= 0) or from the tile's base.
template <int K>
__device__ __forceinline__ int diag_fixed_bits(const OpDesc &op, uint64_t base)
{
    int fixed_s = 0;
#pragma unroll
    for (int m = 0; m < K; ++m)
        if (op.pos[m] < 0) fixed_s |= (int)((base >> op.gq[m]) & 1ull) << m;
    return fixed_s;
}

template <int K>
__device__ __forceinline__ int diag_index(const OpDesc &op, int fixed_s, int l)
{
    int s = fixed_s;
#pragma unroll
    for (int m = 0; m < K; ++m)
        if (op.pos[m] >= 0) s |= ((l >> op.pos[m]) & 1) << m;
    return s;
}

// Diagonal over K qubits: amplitude *= d[s].
template <typename T, int TB, int K>
__device__ __forceinline__ void op_diag(T *__restrict__ sre, T *__restrict__ sim, const OpDesc &op,
                                        const T *__restrict__ dv, uint64_t base)
{
    const int fixed_s = diag_fixed_bits<K>(op, base);
    for (int l = threadIdx.x; l < (1 << TB); l += kThreads) {
        const int s = diag_index<K>(op, fixed_s, l);
        const T dr = dv[2 * s], di = dv[2 * s + 1];
        const int p = swz(l);
        const T xr = sre[p], xi = sim[p];
        sre[p] = fmaT(xr, dr, -xi * di);
        sim[p] = fmaT(xr, di, xi * dr);
    }
}

// Controlled linear phase (a run of diagonal gates sharing one control c):
//   factor(g) = A(g) * (b_c(g) ? B(g) : 1),
// A and B products of per-qubit phases. Tile-local qubits factor through two
// tables indexed by the low 6 bits and by the high TB-6 bits; qubits outside
// the tile contribute a per-tile constant built from per-qubit factors.
template <typename T, int TB>
__device__ __forceinline__ void op_phase(T *__restrict__ sre, T *__restrict__ sim, const OpDesc &op,
                                         const T *__restrict__ tab, uint64_t base, int n, T *__restrict__ scratch)
{
    constexpr int NH = 1 << (TB - 6);
    const T *loA = tab, *hiA = tab + 2 * 64, *loB = tab + 2 * (64 + NH), *hiB = tab + 2 * (128 + NH);
    const T *fixA = tab + 2 * (128 + 2 * NH), *fixB = fixA + 2 * n;
    T ar = 1, ai = 0, br = 1, bi = 0;
    const uint64_t fm = base & op.ctrl_fixed;  // ctrl_fixed holds the non-tile qubit mask here
    for (int q = 0; q < n; ++q) {
        if (!((fm >> q) & 1ull)) continue;
        T fr = fixA[2 * q], fi = fixA[2 * q + 1];
        T tr = ar * fr - ai * fi;
        ai = ar * fi + ai * fr;
        ar = tr;
        fr = fixB[2 * q];
        fi = fixB[2 * q + 1];
        tr = br * fr - bi * fi;
        bi = br * fi + bi * fr;
        br = tr;
    }
    bool ctrl_fixed_on = true;
    if (op.ctrl_q >= 0 && op.ctrl_pos < 0) ctrl_fixed_on = (base >> op.ctrl_q) & 1ull;
    // scratch: lo0 = loA * A_fix (control 0), lo1 = loA * loB * A_fix * B_fix, hi1 = hiA * hiB
    T *lo0 = scratch, *lo1 = scratch + 128, *hi0 = scratch + 256, *hi1 = scratch + 256 + 2 * NH;
    for (int i = threadIdx.x; i < 64; i += kThreads) {
        const T xr = loA[2 * i], xi = loA[2 * i + 1];
        const T r0 = xr * ar - xi * ai, i0 = xr * ai + xi * ar;
        lo0[2 * i] = r0;
        lo0[2 * i + 1] = i0;
        const T yr = loB[2 * i], yi = loB[2 * i + 1];
        const T cr = br * yr - bi * yi, ci = br * yi + bi * yr;
        lo1[2 * i] = r0 * cr - i0 * ci;
        lo1[2 * i + 1] = r0 * ci + i0 * cr;
    }
    for (int i = threadIdx.x; i < NH; i += kThreads) {
        const T xr = hiA[2 * i], xi = hiA[2 * i + 1];
        const T yr = hiB[2 * i], yi = hiB[2 * i + 1];
        hi0[2 * i] = xr;
        hi0[2 * i + 1] = xi;
        hi1[2 * i] = xr * yr - xi * yi;
        hi1[2 * i + 1] = xr * yi + xi * yr;
    }
    __syncthreads();
    const int cp = op.ctrl_pos;
    const bool has_ctrl = op.ctrl_q >= 0;
    for (int l = threadIdx.x; l < (1 << TB); l += kThreads) {
        const bool on = has_ctrl && (cp >= 0 ? ((l >> cp) & 1) != 0 : ctrl_fixed_on);
        const T *lo = on ? lo1 : lo0;
        const T *hi = on ? hi1 : hi0;
        const int a = l & 63, h = l >> 6;
        const T fr = lo[2 * a], fi = lo[2 * a + 1];
        const T gr = hi[2 * h], gi = hi[2 * h + 1];
        const T pr = fr * gr - fi * gi, pi = fr * gi + fi * gr;
        const int p = swz(l);
        const T xr = sre[p], xi = sim[p];
        sre[p] = fmaT(xr, pr, -xi * pi);
        sim[p] = fmaT(xr, pi, xi * pr);
    }
}

// LDS scratch (in T) needed by op_phase.
template <int TB> struct PhaseScratch { static constexpr int size = 2 * (128 + 2 * (1 << (TB - 6))); };

// Multiply every amplitude by the real diagonal sum_k c_k (-1)^popcount(g & m_k).
template <typename T, int TB>
__device__ __forceinline__ void op_obs(T *__restrict__ sre, T *__restrict__ sim, const uint64_t *sG,
                                       const uint64_t *__restrict__ masks, const double *__restrict__ coeffs,
                                       int n_terms)
{
    for (int l = threadIdx.x; l < (1 << TB); l += kThreads) {
        const uint64_t g = (sG[l >> 6] << 6) | (uint64_t)(l & 63);
        double v = 0.0;
        for (int t = 0; t < n_terms; ++t) v += (__popcll(g & masks[t]) & 1) ? -coeffs[t] : coeffs[t];
        const int p = swz(l);
        sre[p] = (T)(sre[p] * v);
        sim[p] = (T)(sim[p] * v);
    }
}

// One op (dense, diagonal, phase) on one tile. Ends without a barrier.
// KMAX bounds the dense width compiled in (register use grows with it).
template <typename T, int TB, int KMAX = 5>
__device__ __forceinline__ void apply_op(T *sre, T *sim, const OpDesc &op, const T *M, uint64_t base, int n,
                                         T *sph)
{
    if (op.type == OP_DENSE || op.type == OP_MFMA) {
        if (op.ctrl_fixed == 0 || (base & op.ctrl_fixed) == op.ctrl_fixed) {
            if (op.real) {
                switch (op.k) {
                case 1: op_dense<T, TB, 1, true>(sre, sim, op, M); break;
                case 2: op_dense<T, TB, 2, true>(sre, sim, op, M); break;
                case 3: op_dense<T, TB, (KMAX >= 3 ? 3 : 1), true>(sre, sim, op, M); break;
                case 4: op_dense<T, TB, (KMAX >= 4 ? 4 : 1), true>(sre, sim, op, M); break;
                default: op_dense<T, TB, (KMAX >= 5 ? 5 : 1), true>(sre, sim, op, M); break;
                }
            } else {
                switch (op.k) {
                case 1: op_dense<T, TB, 1, false>(sre, sim, op, M); break;
                case 2: op_dense<T, TB, 2, false>(sre, sim, op, M); break;
                case 3: op_dense<T, TB, (KMAX >= 3 ? 3 : 1), false>(sre, sim, op, M); break;
                case 4: op_dense<T, TB, (KMAX >= 4 ? 4 : 1), false>(sre, sim, op, M); break;
                default: op_dense<T, TB, (KMAX >= 5 ? 5 : 1), false>(sre, sim, op, M); break;
                }
            }
        }
    } else if (op.type == OP_DIAG) {
        switch (op.k) {
        case 1: op_diag<T, TB, 1>(sre, sim, op, M, base); break;
        case 2: op_diag<T, TB, 2>(sre, sim, op, M, base); break;
        case 3: op_diag<T, TB, 3>(sre, sim, op, M, base); break;
        case 4: op_diag<T, TB, 4>(sre, sim, op, M, base); break;
        default: op_diag<T, TB, 5>(sre, sim, op, M, base); break;
        }
    } else if (op.type == OP_PHASE) {
        op_phase<T, TB>(sre, sim, op, M, base, n, sph);
    }
}

// Per-thread FP64 partial of <lambda| A |psi> over the tile for a probe op:
// A dense on tile bits (k <= 2) or diagonal (table of 2^k entries).
template <typename T, int TB, int K>
__device__ __forceinline__ void probe_dense(const T *pre, const T *pim, const T *lre, const T *lim, const OpDesc &op,
                                            const T *__restrict__ M, double &accr, double &acci)
{
    constexpr int D = 1 << K;
    constexpr int NG = (1 << TB) >> K;
    int sp[K];
#pragma unroll
    for (int m = 0; m < K; ++m) sp[m] = op.pos[m];
    if (K == 2 && sp[0] > sp[1]) { int t = sp[0]; sp[0] = sp[1]; sp[1] = t; }
    int offs[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
        int o = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if ((s >> m) & 1) o |= 1 << op.pos[m];
        offs[s] = swz(o);
    }
    for (int g = threadIdx.x; g < NG; g += kThreads) {
        int l0 = g;
#pragma unroll
        for (int m = 0; m < K; ++m) l0 = ((l0 >> sp[m]) << (sp[m] + 1)) | (l0 & ((1 << sp[m]) - 1));
        const int p0 = swz(l0);
        double vr[D], vi[D];
#pragma unroll
        for (int s = 0; s < D; ++s) { vr[s] = pre[p0 ^ offs[s]]; vi[s] = pim[p0 ^ offs[s]]; }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int s = 0; s < D; ++s) {
                const double mr = M[2 * (r * D + s)], mi = M[2 * (r * D + s) + 1];
                ar += mr * vr[s] - mi * vi[s];
                ai += mr * vi[s] + mi * vr[s];
            }
            const double yr = lre[p0 ^ offs[r]], yi = lim[p0 ^ offs[r]];
            accr += yr * ar + yi * ai;   // conj(lambda) * (A psi)
            acci += yr * ai - yi * ar;
        }
    }
}

template <typename T, int TB, int K>
__device__ __forceinline__ void probe_diag(const T *pre, const T *pim, const T *lre, const T *lim, const OpDesc &op,
                                           const T *__restrict__ dv, uint64_t base, double &accr, double &acci)
{
    const int fixed_s = diag_fixed_bits<K>(op, base);
    for (int l = threadIdx.x; l < (1 << TB); l += kThreads) {
        const int s = diag_index<K>(op, fixed_s, l);
        const double dr = dv[2 * s], di = dv[2 * s + 1];
        const int p = swz(l);
        const double xr = pre[p], xi = pim[p];
        const double ar = dr * xr - di * xi, ai = dr * xi + di * xr;
        const double yr = lre[p], yi = lim[p];
        accr += yr * ar + yi * ai;
        acci += yr * ai - yi * ar;
    }
}

template <typename T, int TB>
__device__ __forceinline__ void probe(const T *pre, const T *pim, const T *lre, const T *lim, const OpDesc &op,
                                      const T *M, uint64_t base, double &accr, double &acci)
{
    if (op.diag) {
        if (op.k == 1) probe_diag<T, TB, 1>(pre, pim, lre, lim, op, M, base, accr, acci);
        else probe_diag<T, TB, 2>(pre, pim, lre, lim, op, M, base, accr, acci);
    } else {
        if (op.k == 1) probe_dense<T, TB, 1>(pre, pim, lre, lim, op, M, accr, acci);
        else probe_dense<T, TB, 2>(pre, pim, lre, lim, op, M, accr, acci);
    }
}

}  // namespace msv
