// Wave-level building blocks of the chunk codec on gfx950 (wave64).
//
// One 64-lane wave handles one 64-value block of one plane: lane i holds value
// i. Prediction residuals use a DPP wave shift, the decode prefix sum a DPP
// Hillis-Steele scan within rows of 16 plus two row broadcasts, the width an
// OR reduction, and bit-plane packing one ballot per plane.
//
// A block's width byte holds its width (bits 0..5, 0..32) and its predictor
// (bits 6..7): 0 Lorenzo-1 (d_i = q_i - q_(i-1)), 1 none (d_i = q_i),
// 2 Lorenzo-2 (d_1 = q_1 - q_0, d_i = q_i - 2 q_(i-1) + q_(i-2)); d_0 = 0 and
// the anchor is q_0 for all three; arithmetic wraps modulo 2^32. Predictor
// mode 0 uses Lorenzo-1 only; mode 1 keeps, per block, the predictor with the
// smallest width (ties to the lower id).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msv {

template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes (uint32 wrap-around arithmetic).
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x)
{
    x += dpp_u32<0x111, 0xf, 0xf, true>(x);   // row_shr:1
    x += dpp_u32<0x112, 0xf, 0xf, true>(x);   // row_shr:2
    x += dpp_u32<0x114, 0xf, 0xf, true>(x);   // row_shr:4
    x += dpp_u32<0x118, 0xf, 0xf, true>(x);   // row_shr:8
    x += dpp_u32<0x142, 0xa, 0xf, false>(x);  // row_bcast:15 -> rows 1, 3
    x += dpp_u32<0x143, 0xc, 0xf, false>(x);  // row_bcast:31 -> rows 2, 3
    return x;
}

// Bitwise OR of all 64 lanes, returned uniformly.
__device__ __forceinline__ uint32_t wave_or(uint32_t x)
{
    x |= dpp_u32<0x111, 0xf, 0xf, true>(x);
    x |= dpp_u32<0x112, 0xf, 0xf, true>(x);
    x |= dpp_u32<0x114, 0xf, 0xf, true>(x);
    x |= dpp_u32<0x118, 0xf, 0xf, true>(x);
    x |= dpp_u32<0x142, 0xa, 0xf, false>(x);
    x |= dpp_u32<0x143, 0xc, 0xf, false>(x);
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Value of lane i-1 (0 for lane 0).
__device__ __forceinline__ uint32_t wave_shift_up1(uint32_t x)
{
    return dpp_u32<0x138, 0xf, 0xf, true>(x);  // wave_shr:1
}

// Code of this lane's value: q = rint(x * inv_step) in FP64, round half to
// even. `bad` is set when x is not finite or |q| > 2^30 - 1 (the code is then 0).
template <typename T>
__device__ __forceinline__ int32_t quantize(T x, double inv_step, bool &bad)
{
    const double r = __builtin_rint((double)x * inv_step);
    const bool ok = __builtin_fabs(r) <= 1073741823.0;
    bad |= !ok;
    return ok ? (int32_t)r : 0;
}

// Decoded value of a code: (T)((double)q * step).
template <typename T>
__device__ __forceinline__ T dequantize(int32_t q, double step)
{
    return (T)((double)q * step);
}

__device__ __forceinline__ uint32_t zigzag(int32_t d) { return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31); }

// Width and predictor fields of a width byte.
__device__ __forceinline__ uint32_t wbyte_width(uint32_t wb) { return wb & 63u; }
__device__ __forceinline__ uint32_t wbyte_pred(uint32_t wb) { return wb >> 6; }

// Lorenzo-1 residual d_i = q_i - q_(i-1), d_0 = 0. The shifted copy stays a
// separate v_mov_dpp (the empty asm hides it from the DPP combiner), so the
// subtraction is an ordinary VALU op whose operand order is explicit.
__device__ __forceinline__ int32_t residual1(int32_t q)
{
    uint32_t prev = wave_shift_up1((uint32_t)q);
    asm("" : "+v"(prev));
    return lane_id() == 0 ? 0 : (int32_t)((uint32_t)q - prev);
}

// Zigzag of the Lorenzo-1 residual.
__device__ __forceinline__ uint32_t residual_zigzag(int32_t q) { return zigzag(residual1(q)); }

// Zigzagged residuals of predictors 1 (none) and 2 (Lorenzo-2) from the codes
// q and their Lorenzo-1 residuals d1 (d1_0 = 0, so the Lorenzo-2 residual
// d1_i - d1_(i-1) is d1_1 at lane 1 and 0 at lane 0).
__device__ __forceinline__ void residuals_alt(int32_t q, int32_t d1, uint32_t &u_none, uint32_t &u_l2)
{
    uint32_t prev = wave_shift_up1((uint32_t)d1);
    asm("" : "+v"(prev));
    u_none = lane_id() == 0 ? 0u : zigzag(q);
    u_l2 = zigzag((int32_t)((uint32_t)d1 - prev));
}

// Bits needed for every lane's u (0..32), uniform.
__device__ __forceinline__ uint32_t block_width(uint32_t u)
{
    const uint32_t o = wave_or(u);
    return o ? 32u - (uint32_t)__builtin_clz(o) : 0u;
}

// Lane k (< W) receives bit-plane word k: bit i = bit k of lane i's u.
__device__ __forceinline__ uint64_t pack_planes(uint32_t u, uint32_t W)
{
    uint64_t mine = 0;
    const uint32_t lane = lane_id();
    for (uint32_t k = 0; k < W; ++k) {
        const uint64_t bal = __builtin_amdgcn_ballot_w64(((u >> k) & 1u) != 0u);
        if (lane == k) mine = bal;
    }
    return mine;
}

// Two independent inclusive prefix sums, interleaved so that each DPP step of
// one chain fills the other's hazard slots.
__device__ __forceinline__ void wave_inclusive_sum2(uint32_t &x, uint32_t &y)
{
    x += dpp_u32<0x111, 0xf, 0xf, true>(x);
    y += dpp_u32<0x111, 0xf, 0xf, true>(y);
    x += dpp_u32<0x112, 0xf, 0xf, true>(x);
    y += dpp_u32<0x112, 0xf, 0xf, true>(y);
    x += dpp_u32<0x114, 0xf, 0xf, true>(x);
    y += dpp_u32<0x114, 0xf, 0xf, true>(y);
    x += dpp_u32<0x118, 0xf, 0xf, true>(x);
    y += dpp_u32<0x118, 0xf, 0xf, true>(y);
    x += dpp_u32<0x142, 0xa, 0xf, false>(x);
    y += dpp_u32<0x142, 0xa, 0xf, false>(y);
    x += dpp_u32<0x143, 0xc, 0xf, false>(x);
    y += dpp_u32<0x143, 0xc, 0xf, false>(y);
}

// Widths of two blocks (OR reductions interleaved).
__device__ __forceinline__ void block_width2(uint32_t u, uint32_t v, uint32_t &wu, uint32_t &wv)
{
    u |= dpp_u32<0x111, 0xf, 0xf, true>(u);
    v |= dpp_u32<0x111, 0xf, 0xf, true>(v);
    u |= dpp_u32<0x112, 0xf, 0xf, true>(u);
    v |= dpp_u32<0x112, 0xf, 0xf, true>(v);
    u |= dpp_u32<0x114, 0xf, 0xf, true>(u);
    v |= dpp_u32<0x114, 0xf, 0xf, true>(v);
    u |= dpp_u32<0x118, 0xf, 0xf, true>(u);
    v |= dpp_u32<0x118, 0xf, 0xf, true>(v);
    u |= dpp_u32<0x142, 0xa, 0xf, false>(u);
    v |= dpp_u32<0x142, 0xa, 0xf, false>(v);
    u |= dpp_u32<0x143, 0xc, 0xf, false>(u);
    v |= dpp_u32<0x143, 0xc, 0xf, false>(v);
    const uint32_t ou = (uint32_t)__builtin_amdgcn_readlane((int)u, 63);
    const uint32_t ov = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    wu = ou ? 32u - (uint32_t)__builtin_clz(ou) : 0u;
    wv = ov ? 32u - (uint32_t)__builtin_clz(ov) : 0u;
}

// Codes of one block from its first-order sums: d holds the zigzag-decoded
// residuals, e their inclusive prefix sums (e_0 = 0). Predictor 0: A + e;
// 1: the residuals themselves (A at lane 0); 2: A + the prefix sums of e (the
// caller passes them as e2).
__device__ __forceinline__ int32_t codes_from_sums(uint32_t pred, int32_t A, uint32_t d, uint32_t e, uint32_t e2)
{
    if (pred == 1) return lane_id() == 0 ? A : (int32_t)d;
    return (int32_t)((uint32_t)A + (pred == 2 ? e2 : e));
}

// Codes of two blocks (the re and im planes of one amplitude block) from
// their width bytes Wr / Wi. Lane k holds word k of each block in mr / mi and
// 0 for k at or beyond its width, so both unpack in one loop up to the larger
// width. PRED = false: the blocks are known to use predictor 0.
template <bool PRED = true>
__device__ __forceinline__ void unpack_codes2(uint64_t mr, uint32_t Wr, int32_t Ar, uint64_t mi, uint32_t Wi,
                                              int32_t Ai, int32_t &qr, int32_t &qi)
{
    // planes from the most significant down: word << (63 - lane) puts this
    // lane's bit on top, and a funnel shift appends it to u
    const uint32_t up = 63u - lane_id();
    const uint32_t Pr = PRED ? wbyte_pred(Wr) : 0u, Pi = PRED ? wbyte_pred(Wi) : 0u;
    if (PRED) {
        Wr = wbyte_width(Wr);
        Wi = wbyte_width(Wi);
    }
    const uint32_t Wm = Wr > Wi ? Wr : Wi;
    uint32_t ur = 0, ui = 0;
    for (uint32_t k = Wm; k-- > 0;) {
        const uint32_t r_lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mr, (int)k);
        const uint32_t r_hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mr >> 32), (int)k);
        const uint32_t i_lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mi, (int)k);
        const uint32_t i_hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mi >> 32), (int)k);
        const uint64_t tr = (((uint64_t)r_hi << 32) | r_lo) << up;
        const uint64_t ti = (((uint64_t)i_hi << 32) | i_lo) << up;
        ur = __builtin_amdgcn_alignbit(ur, (uint32_t)(tr >> 32), 31u);
        ui = __builtin_amdgcn_alignbit(ui, (uint32_t)(ti >> 32), 31u);
    }
    if (!PRED || (Pr | Pi) == 0) {
        // Lorenzo-1 only: one scan in place
        uint32_t dr = (ur >> 1) ^ (0u - (ur & 1u));
        uint32_t di = (ui >> 1) ^ (0u - (ui & 1u));
        if (Wm) wave_inclusive_sum2(dr, di);
        qr = (int32_t)((uint32_t)Ar + dr);
        qi = (int32_t)((uint32_t)Ai + di);
        return;
    }
    const uint32_t dr = (ur >> 1) ^ (0u - (ur & 1u));
    const uint32_t di = (ui >> 1) ^ (0u - (ui & 1u));
    uint32_t er = dr, ei = di;
    wave_inclusive_sum2(er, ei);
    uint32_t fr = er, fi = ei;
    if (Pr == 2 || Pi == 2) wave_inclusive_sum2(fr, fi);
    qr = codes_from_sums(Pr, Ar, dr, er, fr);
    qi = codes_from_sums(Pi, Ai, di, ei, fi);
}

// Four independent inclusive prefix sums, interleaved.
__device__ __forceinline__ void wave_inclusive_sum4(uint32_t *x)
{
#define MSV_SCAN_STEP(C, R, B, Z)                                              \
    _Pragma("unroll") for (int p = 0; p < 4; ++p) x[p] += dpp_u32<C, R, B, Z>(x[p]);
    MSV_SCAN_STEP(0x111, 0xf, 0xf, true)
    MSV_SCAN_STEP(0x112, 0xf, 0xf, true)
    MSV_SCAN_STEP(0x114, 0xf, 0xf, true)
    MSV_SCAN_STEP(0x118, 0xf, 0xf, true)
    MSV_SCAN_STEP(0x142, 0xa, 0xf, false)
    MSV_SCAN_STEP(0x143, 0xc, 0xf, false)
#undef MSV_SCAN_STEP
}

// Widths of four blocks (OR reductions interleaved).
__device__ __forceinline__ void block_width4(const uint32_t *u_in, uint32_t *w)
{
    uint32_t u[4] = {u_in[0], u_in[1], u_in[2], u_in[3]};
#define MSV_OR_STEP(C, R, B, Z)                                                \
    _Pragma("unroll") for (int p = 0; p < 4; ++p) u[p] |= dpp_u32<C, R, B, Z>(u[p]);
    MSV_OR_STEP(0x111, 0xf, 0xf, true)
    MSV_OR_STEP(0x112, 0xf, 0xf, true)
    MSV_OR_STEP(0x114, 0xf, 0xf, true)
    MSV_OR_STEP(0x118, 0xf, 0xf, true)
    MSV_OR_STEP(0x142, 0xa, 0xf, false)
    MSV_OR_STEP(0x143, 0xc, 0xf, false)
#undef MSV_OR_STEP
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)u[p], 63);
        w[p] = o ? 32u - (uint32_t)__builtin_clz(o) : 0u;
    }
}

// One step of a 32 x 32 bit transpose within each half-wave: lanes l and
// l ^ J exchange the bit groups the other one needs. The lower lane keeps its
// bits at positions with bit J clear (mask M) and takes the upper lane's bits
// there, shifted up by J, into the others; the upper lane keeps its bits at
// positions with bit J set and takes the lower lane's, shifted down by J.
// Branch-free: both shifts are one rotate by a per-lane amount, and one bit
// select merges.
template <int J, uint32_t M>
__device__ __forceinline__ uint32_t transpose_step(uint32_t x, uint32_t lane)
{
    const uint32_t p = (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (J << 10) | 0x1f);   // lane ^ J
    const uint32_t up = 0u - ((lane / J) & 1u);                                     // all ones on the upper lane
    const uint32_t keep = M ^ up;                                                   // M, or ~M on the upper lane
    const uint32_t rot = (32u - J) + (up & (uint32_t)(2 * J - 32));                 // 32 - J, or J on the upper lane
    const uint32_t sh = __builtin_amdgcn_alignbit(p, p, rot);                       // p rotated right by rot
    return (x & keep) | (sh & ~keep);
}

// Transpose of the 32 x 32 bit matrix held by each half-wave (row = lane,
// column = bit): afterwards bit i of lane 32h + j is bit j of the input of
// lane 32h + i.
__device__ __forceinline__ uint32_t transpose32_halves(uint32_t x, uint32_t lane)
{
    x = transpose_step<16, 0x0000ffffu>(x, lane);
    x = transpose_step<8, 0x00ff00ffu>(x, lane);
    x = transpose_step<4, 0x0f0f0f0fu>(x, lane);
    x = transpose_step<2, 0x33333333u>(x, lane);
    x = transpose_step<1, 0x55555555u>(x, lane);
    return x;
}

// Codes of four blocks (two amplitude blocks, both planes each) from their
// width bytes Wb, unpacked in one loop up to the largest width. The words are
// staged in LDS: stage[32 p + k] holds word k of block p (0 at or beyond its
// width), so each plane word reaches all lanes by one broadcast LDS read
// instead of two v_readlane. Planes go from the most significant down, as in
// unpack_codes2. Blocks of predictor 0 only (every block of mode 0) take one
// scan; other predictors take a second scan (Lorenzo-2) or none (none).
// PRED = false: the blocks are known to use predictor 0.
// XP = false keeps the plane-by-plane unpack for every width (fewer live
// registers, for kernels that are short of them).
template <bool PRED = true, bool XP = true>
__device__ __forceinline__ void unpack_codes4_lds(const uint64_t *stage, const uint32_t *Wb, const int32_t *A,
                                                  int32_t *q)
{
    const uint32_t up = 63u - lane_id();
    uint32_t W[4], P[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        W[p] = PRED ? wbyte_width(Wb[p]) : Wb[p];
        P[p] = PRED ? wbyte_pred(Wb[p]) : 0u;
    }
    const uint32_t Wm = max(max(W[0], W[1]), max(W[2], W[3]));
    uint32_t u[4] = {0u, 0u, 0u, 0u};
    if (XP && Wm <= 8u) {
        // every zigzag fits a byte: lane 8p + k of each half-wave takes its
        // half of block p's plane k (staged words beyond a block's width are
        // zero), and the half-wave transpose hands every lane its four values
        // as u0 | u1 << 8 | u2 << 16 | u3 << 24
        const uint32_t lane = lane_id(), j = lane & 31u;
        const uint32_t y = reinterpret_cast<const uint32_t *>(stage)[2u * (32u * (j >> 3) + (j & 7u)) + (lane >> 5)];
        const uint32_t x = transpose32_halves(y, lane);
#pragma unroll
        for (int p = 0; p < 4; ++p) u[p] = (x >> (8 * p)) & 255u;
    } else {
        for (uint32_t k = Wm; k-- > 0;) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint64_t t = stage[32 * p + k] << up;
                u[p] = __builtin_amdgcn_alignbit(u[p], (uint32_t)(t >> 32), 31u);
            }
        }
    }
    if (!PRED || (P[0] | P[1] | P[2] | P[3]) == 0) {
        // Lorenzo-1 only: one scan in place
        uint32_t d[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) d[p] = (u[p] >> 1) ^ (0u - (u[p] & 1u));
        if (Wm) wave_inclusive_sum4(d);
#pragma unroll
        for (int p = 0; p < 4; ++p) q[p] = (int32_t)((uint32_t)A[p] + d[p]);
        return;
    }
    uint32_t d[4], e[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) e[p] = d[p] = (u[p] >> 1) ^ (0u - (u[p] & 1u));
    wave_inclusive_sum4(e);
    uint32_t f[4] = {e[0], e[1], e[2], e[3]};
    if (P[0] == 2 || P[1] == 2 || P[2] == 2 || P[3] == 2) wave_inclusive_sum4(f);
#pragma unroll
    for (int p = 0; p < 4; ++p) q[p] = codes_from_sums(P[p], A[p], d[p], e[p], f[p]);
}

// Lane k (< W[p]) receives bit-plane word k of block p, for four blocks.
__device__ __forceinline__ void pack_planes4(const uint32_t *u, const uint32_t *W, uint64_t *mine)
{
    const uint32_t lane = lane_id();
    const uint32_t Wm = max(max(W[0], W[1]), max(W[2], W[3]));
#pragma unroll
    for (int p = 0; p < 4; ++p) mine[p] = 0;
    for (uint32_t k = 0; k < Wm; ++k) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint64_t bal = __builtin_amdgcn_ballot_w64(((u[p] >> k) & 1u) != 0u);
            if (lane == k) mine[p] = bal;
        }
    }
}

// Bit planes of four blocks whose zigzags all fit a byte (widths w0..w3 <= 8),
// written to heap[o_p + k] for k < w_p: the same words as pack_planes4. The
// four values of a lane travel as one word u0 | u1 << 8 | u2 << 16 | u3 << 24;
// after the half-wave transposes, lane 8p + k of the low half holds the low 32
// bits of block p's plane k and the same lane of the high half its high 32
// bits. Widths and offsets (< 2^16 words within a tile) are picked per lane
// from packed words (shifts, not an indexed array, which would go to scratch).
__device__ __forceinline__ void store_planes4_bytes(const uint32_t *u, uint32_t w0, uint32_t w1, uint32_t w2,
                                                    uint32_t w3, uint32_t o0, uint32_t o1, uint32_t o2, uint32_t o3,
                                                    uint64_t *heap, uint32_t lane)
{
    uint32_t x = u[0] | (u[1] << 8) | (u[2] << 16) | (u[3] << 24);
    x = transpose32_halves(x, lane);
    const uint32_t hi = (uint32_t)__shfl_xor((int)x, 32, 64);
    const uint32_t wp = w0 | (w1 << 8) | (w2 << 16) | (w3 << 24);
    const uint32_t w = (wp >> (lane & 24u)) & 255u;                          // block (lane >> 3) & 3
    const uint32_t oa = (lane & 16u) ? (o2 | (o3 << 16)) : (o0 | (o1 << 16));
    const uint32_t off = (oa >> ((lane & 8u) << 1)) & 0xffffu;
    const uint32_t k = lane & 7u;
    if (lane < 32 && k < w) heap[off + k] = (uint64_t)x | ((uint64_t)hi << 32);
}

// Predictor mode 1 for two blocks: given the codes q, their Lorenzo-1
// residuals d1 and the Lorenzo-1 zigzags u with widths W (P = 0), keep per
// block the predictor of smallest width (ties to the lower id), updating u, W
// and P.
__device__ __forceinline__ void choose_predictors2(const int32_t *q, const int32_t *d1, uint32_t *u, uint32_t *W,
                                                   uint32_t *P)
{
    uint32_t un[2], u2[2], wn[2], w2[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) residuals_alt(q[p], d1[p], un[p], u2[p]);
    block_width2(un[0], un[1], wn[0], wn[1]);
    block_width2(u2[0], u2[1], w2[0], w2[1]);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        if (wn[p] < W[p]) {
            W[p] = wn[p];
            P[p] = 1;
            u[p] = un[p];
        }
        if (w2[p] < W[p]) {
            W[p] = w2[p];
            P[p] = 2;
            u[p] = u2[p];
        }
    }
}

// FP64 sum over the 64 lanes, returned to every lane (butterfly: the same
// order on every call, so the result is reproducible).
__device__ __forceinline__ double wave_sum_f64(double x)
{
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ double wave_max_f64(double x)
{
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

}  // namespace msv
