// Fused dense ops on the matrix cores (gfx950 MFMA).
//
// A dense K-qubit unitary U = Ur + i Ui acting on the tile is the real GEMM
//   [Yr; Yi] = R [Xr; Xi],   R = [[Ur, -Ui], [Ui, Ur]]   (2D x 2D, D = 2^K)
// whose columns are the tile's groups of D amplitudes (the group index fills
// the tile bits that are not op positions, lowest first) and whose rows are
// the group's real parts (rows 0..D-1) and imaginary parts (rows D..2D-1),
// row s of a group sitting at tile offset sum_m bit_m(s) << pos[m].
// This is Sec. 2's gate application for a fused group, 8 D flops per amplitude.
//
// Each wave owns 16 columns at a time: the 16x16 output blocks of R X are
// accumulated with 16x16xKK MFMAs; R is held in registers for the whole op in
// the A-operand layout, X is read from LDS in the B-operand layout, and the
// results are written back in place (a wave reads all of its columns before it
// writes any, and columns of different waves are disjoint).
//
// Operand layouts (lane l, q = l / 16, j = l % 16; checked on the device):
//   A: lane holds A[j][KK t + EPL q + e], e < EPL
//   B: lane holds B[KK t + EPL q + e][j]
//   C: lane, register r holds C[4 q + r][j] (FP32 accumulators) or
//      C[4 r + q][j] (FP64 16x16x4)
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "tile_ops.h"

namespace msv {

typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef short mf_s4 __attribute__((ext_vector_type(4)));

template <typename T, int MF> struct MfmaTraits;

template <> struct MfmaTraits<float, MMA_NATIVE> {
    static constexpr int KK = 4, EPL = 1;
    static constexpr __device__ int crow(int q, int r) { return 4 * q + r; }
    using Op = float;
    using Acc = mf_f4;
    static __device__ __forceinline__ Op pack(const float *v) { return v[0]; }
    static __device__ __forceinline__ Acc mma(Op a, Op b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <> struct MfmaTraits<double, MMA_NATIVE> {
    static constexpr int KK = 4, EPL = 1;
    static constexpr __device__ int crow(int q, int r) { return 4 * r + q; }
    using Op = double;
    using Acc = mf_d4;
    static __device__ __forceinline__ Op pack(const double *v) { return v[0]; }
    static __device__ __forceinline__ Acc mma(Op a, Op b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Round-to-nearest-even FP32 -> BF16 bits.
__device__ __forceinline__ short bf16_bits(float x)
{
    const __bf16 b = (__bf16)x;
    return __builtin_bit_cast(short, b);
}

template <> struct MfmaTraits<float, MMA_BF16> {
    static constexpr int KK = 16, EPL = 4;
    static constexpr __device__ int crow(int q, int r) { return 4 * q + r; }
    using Op = mf_s4;
    using Acc = mf_f4;
    static __device__ __forceinline__ Op pack(const float *v)
    {
        Op o;
        o[0] = bf16_bits(v[0]);
        o[1] = bf16_bits(v[1]);
        o[2] = bf16_bits(v[2]);
        o[3] = bf16_bits(v[3]);
        return o;
    }
    static __device__ __forceinline__ Acc mma(Op a, Op b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

// Tile offset of matrix index s: bit m of s goes to tile bit pos[m].
template <int K>
__device__ __forceinline__ int op_offset(const int *pos, int s)
{
    int o = 0;
#pragma unroll
    for (int m = 0; m < K; ++m) o |= ((s >> m) & 1) << pos[m];
    return o;
}

// samp holds the tile as re[2^TB] followed by im[2^TB]. M is the complex
// matrix (row r, column s at 2 (r D + s)). Requires 2^(TB-K) >= 16.
template <typename T, int TB, int K, int MF>
__device__ __forceinline__ void op_mfma(T *__restrict__ samp, const OpDesc &op, const T *__restrict__ M, int wave,
                                        int lane)
{
    using Tr = MfmaTraits<T, MF>;
    using Op = typename Tr::Op;
    using Acc = typename Tr::Acc;
    constexpr int D = 1 << K, D2 = 2 * D, TILE = 1 << TB;
    constexpr int KK = Tr::KK, EPL = Tr::EPL;
    constexpr int RB = D2 / 16, KS = D2 / KK;
    constexpr int NCT = (TILE >> K) / 16;
    constexpr int NW = kThreads / 64;
    static_assert(NCT >= 1, "tile too small for a 16-column block");
    static_assert(D2 % KK == 0 && D2 % 16 == 0, "matrix does not tile");

    const int q = lane >> 4, j = lane & 15;
    int pos[K], sp[K];
#pragma unroll
    for (int m = 0; m < K; ++m) pos[m] = sp[m] = op.pos[m];
#pragma unroll
    for (int i = 1; i < K; ++i)
#pragma unroll
        for (int jj = i; jj > 0; --jj)
            if (sp[jj - 1] > sp[jj]) { const int t = sp[jj]; sp[jj] = sp[jj - 1]; sp[jj - 1] = t; }

    // R in the A-operand layout: row 16 rb + j, column KK t + EPL q + e.
    Op a[RB][KS];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int i = 16 * rb + j;
        const int ii = i & (D - 1);
        const bool ilo = i < D;
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            T v[EPL];
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int c = KK * t + EPL * q + e;
                const int cc = c & (D - 1);
                const bool clo = c < D;
                const T ur = M[2 * (ii * D + cc)], ui = M[2 * (ii * D + cc) + 1];
                v[e] = ilo ? (clo ? ur : -ui) : (clo ? ui : ur);
            }
            a[rb][t] = Tr::pack(v);
        }
    }
    // LDS offsets (relative to a group's base) of this lane's B rows and C rows.
    int pb[KS][EPL], pc[RB][4];
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int rho = KK * t + EPL * q + e;
            pb[t][e] = (rho < D ? 0 : TILE) | swz(op_offset<K>(pos, rho & (D - 1)));
        }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * rb + Tr::crow(q, r);
            pc[rb][r] = (row < D ? 0 : TILE) | swz(op_offset<K>(pos, row & (D - 1)));
        }

    for (int ct = wave; ct < NCT; ct += NW) {
        int l0 = ct * 16 + j;
#pragma unroll
        for (int m = 0; m < K; ++m) l0 = ((l0 >> sp[m]) << (sp[m] + 1)) | (l0 & ((1 << sp[m]) - 1));
        l0 = swz(l0);
        Op b[KS];
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            T v[EPL];
#pragma unroll
            for (int e = 0; e < EPL; ++e) v[e] = samp[l0 ^ pb[t][e]];
            b[t] = Tr::pack(v);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            Acc c = {0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < KS; ++t) c = Tr::mma(a[rb][t], b[t], c);
#pragma unroll
            for (int r = 0; r < 4; ++r) samp[l0 ^ pc[rb][r]] = (T)c[r];
        }
    }
}

// Dispatch on the op's width; widths below 3 or tiles too small for 16
// columns never reach here (the planner keeps them on the VALU).
template <typename T, int TB, int MF>
__device__ __forceinline__ void apply_mfma(T *samp, const OpDesc &op, const T *M, uint64_t base, int wave, int lane)
{
    if (op.ctrl_fixed != 0 && (base & op.ctrl_fixed) != op.ctrl_fixed) return;
    if constexpr (MF != MMA_NONE) {
        switch (op.k) {
        case 3:
            if constexpr (TB >= 7) op_mfma<T, TB, 3, MF>(samp, op, M, wave, lane);
            break;
        case 4:
            if constexpr (TB >= 8) op_mfma<T, TB, 4, MF>(samp, op, M, wave, lane);
            break;
        case 5:
            if constexpr (TB >= 9) op_mfma<T, TB, 5, MF>(samp, op, M, wave, lane);
            break;
        default: break;
        }
    }
}

}  // namespace msv
