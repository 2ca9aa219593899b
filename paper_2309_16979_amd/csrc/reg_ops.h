// Register-resident op segments of a tile pass.
//
// A segment is a run of consecutive ops of one pass that all act on the same
// R = TB - 8 "register" tile bits S[0] < ... < S[R-1]: dense ops of one or two
// qubits whose tile bits lie in S, diagonal tables and controlled linear
// phases (which act elementwise, so any bits will do). For the segment each
// of the 256 threads holds 2^R amplitudes in registers: register index i
// (bit r = tile bit S[r]), the thread id deposited into the other TB - R = 8
// tile bits in ascending order. The segment costs one LDS read and one write
// of the tile however many ops it holds; the ops themselves are the gate
// applications of Sec. 2, evaluated in the same order and with the same
// operation order as the LDS-resident kernels (dense and diagonal ops give
// bit-identical results).
#pragma once
#include <hip/hip_runtime.h>

#include "tile_ops.h"

namespace msv {

// An empty asm statement carrying the variant's id: the variants of a
// dispatch then end in different instructions, so the compiler cannot merge
// their (otherwise identical) tails into one block with run-time register
// indices, which would move the register arrays to scratch memory.
template <int ID>
__device__ __forceinline__ void variant_end()
{
    asm volatile("; register op variant %0" ::"n"(ID));
}

// Tile offset of register index i: bit r of i goes to tile bit S[r].
template <int R>
__device__ __forceinline__ int reg_offset(const int *S, int i)
{
    int o = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if ((i >> r) & 1) o |= 1 << S[r];
    return o;
}

// Register bit of tile position p (p must be in S): rank of p in S.
__device__ __forceinline__ int reg_rank(uint32_t smask, int p)
{
    return __builtin_popcount(smask & ((1u << p) - 1u));
}

// ---------------------------------------------------------------- dense

template <typename T, int R, int RB, bool REAL>
__device__ __forceinline__ void reg_dense1(T *re, T *im, const T *__restrict__ Mg)
{
    const ConstPtr<T> M = as_const(Mg);
    T mr[4], mi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        mr[e] = M[2 * e];
        mi[e] = REAL ? T(0) : M[2 * e + 1];
    }
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if ((i >> RB) & 1) continue;
        const int j = i | (1 << RB);
        const T vr[2] = {re[i], re[j]}, vi[2] = {im[i], im[j]};
        T outr[2], outi[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            T ar = 0, ai = 0;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                ar = fmaT(mr[2 * r + s], vr[s], ar);
                if (!REAL) ar = fmaT(-mi[2 * r + s], vi[s], ar);
                ai = fmaT(mr[2 * r + s], vi[s], ai);
                if (!REAL) ai = fmaT(mi[2 * r + s], vr[s], ai);
            }
            outr[r] = ar;
            outi[r] = ai;
        }
        re[i] = outr[0];
        im[i] = outi[0];
        re[j] = outr[1];
        im[j] = outi[1];
    }
    variant_end<RB + (REAL ? 100 : 0)>();
}

// Matrix index s = b(register bit A) + 2 b(register bit B), A < B.
template <typename T, int R, int A, int B, bool REAL>
__device__ __forceinline__ void reg_dense2(T *re, T *im, const T *__restrict__ Mg)
{
    const ConstPtr<T> M = as_const(Mg);
    T mr[16], mi[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        mr[e] = M[2 * e];
        mi[e] = REAL ? T(0) : M[2 * e + 1];
    }
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if (((i >> A) & 1) || ((i >> B) & 1)) continue;
        const int idx[4] = {i, i | (1 << A), i | (1 << B), i | (1 << A) | (1 << B)};
        T vr[4], vi[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            vr[s] = re[idx[s]];
            vi[s] = im[idx[s]];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T ar = 0, ai = 0;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                ar = fmaT(mr[4 * r + s], vr[s], ar);
                if (!REAL) ar = fmaT(-mi[4 * r + s], vi[s], ar);
                ai = fmaT(mr[4 * r + s], vi[s], ai);
                if (!REAL) ai = fmaT(mi[4 * r + s], vr[s], ai);
            }
            re[idx[r]] = ar;
            im[idx[r]] = ai;
        }
    }
    variant_end<1000 + 10 * A + B + (REAL ? 100 : 0)>();
}

template <typename T, int R, bool REAL, int RB = 0>
__device__ __forceinline__ void reg_dense1_at(int rb, T *re, T *im, const T *M)
{
    if constexpr (RB < R) {
        if (rb == RB) reg_dense1<T, R, RB, REAL>(re, im, M);
        else reg_dense1_at<T, R, REAL, RB + 1>(rb, re, im, M);
    }
}

template <typename T, int R, bool REAL, int P = 0>
__device__ __forceinline__ void reg_dense2_at(int a, int b, T *re, T *im, const T *M)
{
    if constexpr (P < R * R) {
        constexpr int A = P / R, B = P % R;
        if constexpr (A < B) {
            if (a == A && b == B) {
                reg_dense2<T, R, A, B, REAL>(re, im, M);
                return;
            }
        }
        reg_dense2_at<T, R, REAL, P + 1>(a, b, re, im, M);
    }
}

// Dense op of k <= 2 qubits with tile positions pos[0] < pos[1] in S.
template <typename T, int R>
__device__ __forceinline__ void reg_dense(T *re, T *im, const OpDesc &op, uint32_t smask, const T *M)
{
    const int a = reg_rank(smask, op.pos[0]);
    if (op.k == 1) {
        if (op.real) reg_dense1_at<T, R, true>(a, re, im, M);
        else reg_dense1_at<T, R, false>(a, re, im, M);
    } else {
        const int b = reg_rank(smask, op.pos[1]);
        if (op.real) reg_dense2_at<T, R, true>(a, b, re, im, M);
        else reg_dense2_at<T, R, false>(a, b, re, im, M);
    }
}

// ------------------------------------------------------------- diagonal

// The bits of i at the set positions of m, packed from bit 0 up.
__host__ __device__ constexpr int extract_bits(int i, int m)
{
    int r = 0, j = 0;
    for (int b = 0; b < 8; ++b)
        if ((m >> b) & 1) r |= ((i >> b) & 1) << j++;
    return r;
}

// Diagonal with the table reordered by the planner (OP_RDIAG): the thread's
// 2^popcount(RM) entries form one row, entry v for the register elements whose
// register bits in RM (ascending) spell v. The row is uniform when the op has
// no thread bits (scalar loads), else per thread. The products keep the FMA
// order of op_diag, so a diagonal gives the same bits in both paths.
template <typename T, int R, int RM, bool UNIFORM>
__device__ __forceinline__ void reg_rdiag_apply(T *re, T *im, const T *__restrict__ row)
{
    constexpr int NV = 1 << __builtin_popcount(RM);
    T dr[NV], di[NV];
    if (UNIFORM) {
        const ConstPtr<T> rc = as_const(row);
#pragma unroll
        for (int v = 0; v < NV; ++v) { dr[v] = rc[2 * v]; di[v] = rc[2 * v + 1]; }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) { dr[v] = row[2 * v]; di[v] = row[2 * v + 1]; }
    }
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        const int v = extract_bits(i, RM);
        const T xr = re[i], xi = im[i];
        re[i] = fmaT(xr, dr[v], -xi * di[v]);
        im[i] = fmaT(xr, di[v], xi * dr[v]);
    }
    variant_end<3000 + RM + (UNIFORM ? 100 : 0)>();
}

template <typename T, int R, bool UNIFORM, int RM = 0>
__device__ __forceinline__ void reg_rdiag_at(int rm, T *re, T *im, const T *row)
{
    if constexpr (RM < (1 << R)) {
        if (rm == RM) reg_rdiag_apply<T, R, RM, UNIFORM>(re, im, row);
        else reg_rdiag_at<T, R, UNIFORM, RM + 1>(rm, re, im, row);
    }
}

template <typename T, int R>
__device__ __forceinline__ void reg_rdiag(T *re, T *im, const OpDesc &op, int tbase, const T *__restrict__ dv,
                                          uint64_t base)
{
    // (loops over every descriptor field with constant indices: a run-time
    // index into the descriptor would move it to scratch memory)
    const int br = op.slot, bt = op.diag;
    int u = 0;   // the tile's fixed bits (uniform)
#pragma unroll
    for (int j = 0; j < 5; ++j)
        if (j >= br + bt && j < op.k) u |= (int)((base >> op.gq[j]) & 1ull) << (j - br - bt);
    if (bt == 0) {
        reg_rdiag_at<T, R, true>((int)op.ctrl_local, re, im, dv + 2 * (u << br));
    } else {
        int t = u << bt;
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if (j >= br && j < br + bt) t |= ((tbase >> op.pos[j]) & 1) << (j - br);
        reg_rdiag_at<T, R, false>((int)op.ctrl_local, re, im, dv + 2 * (t << br));
    }
}

// ------------------------------------------------------ controlled phase

// RC: register bit of the control (0 <= RC < R, so every element knows its
// control statically), or -1 when the control is a thread bit, a bit of the
// tile's base, or absent (then `on_t` holds it per thread).
template <typename T, int R, int RC>
__device__ __forceinline__ void reg_phase_apply(T *re, T *im, T f0r, T f0i, T f1r, T f1i, bool on_t,
                                                const ConstPtr<T> U0, const ConstPtr<T> U1)
{
    constexpr int NR = 1 << R;
    if (RC < 0) {
        // one thread factor for all of the thread's elements
        const T fr = on_t ? f1r : f0r, fi = on_t ? f1i : f0i;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const T u0r = U0[2 * i], u0i = U0[2 * i + 1], u1r = U1[2 * i], u1i = U1[2 * i + 1];
            const T ur = on_t ? u1r : u0r, ui = on_t ? u1i : u0i;
            const T pr = fmaT(fr, ur, -(fi * ui)), pi = fmaT(fr, ui, fi * ur);
            const T xr = re[i], xi = im[i];
            re[i] = fmaT(xr, pr, -xi * pi);
            im[i] = fmaT(xr, pi, xi * pr);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const bool on = ((i >> RC) & 1) != 0;
            const T fr = on ? f1r : f0r, fi = on ? f1i : f0i;
            const T ur = on ? U1[2 * i] : U0[2 * i], ui = on ? U1[2 * i + 1] : U0[2 * i + 1];
            const T pr = fmaT(fr, ur, -(fi * ui)), pi = fmaT(fr, ui, fi * ur);
            const T xr = re[i], xi = im[i];
            re[i] = fmaT(xr, pr, -xi * pi);
            im[i] = fmaT(xr, pi, xi * pr);
        }
    }
    variant_end<2000 + RC>();
}

template <typename T, int R, int RC = -1>
__device__ __forceinline__ void reg_phase_at(int rc, T *re, T *im, T f0r, T f0i, T f1r, T f1i, bool on_t,
                                             const ConstPtr<T> U0, const ConstPtr<T> U1)
{
    if constexpr (RC < R) {
        if (rc == RC) reg_phase_apply<T, R, RC>(re, im, f0r, f0i, f1r, f1i, on_t, U0, U1);
        else reg_phase_at<T, R, RC + 1>(rc, re, im, f0r, f0i, f1r, f1i, on_t, U0, U1);
    }
}

// factor(l) = A(l) (b_c(l) ? B(l) : 1) with A, B products of per-qubit phases
// (and a global factor in A), split as F(thread bits, tile bits outside the
// tile) * U(register index). Pool layout (complex entries): U0[2^R], U1[2^R]
// (register part for control off / on, global factor included), P0[256],
// P1[256] (thread part, indexed by thread id), then for each of the
// op.k = ceil((n - TB) / 8) bytes g of the tile id TA[g][256] and afterwards
// TAB[g][256] (off / on). ctrl_pos: tile position of the control (-1 when it
// lies outside the tile), ctrl_q: its qubit (-1 = no control).
template <typename T, int R>
__device__ __forceinline__ void reg_phase(T *re, T *im, const OpDesc &op, uint32_t smask, int tbase,
                                          const T *__restrict__ tab, uint64_t base, uint64_t tile)
{
    constexpr int NR = 1 << R;
    const ConstPtr<T> U0 = as_const(tab), U1 = as_const(tab + 2 * NR);
    const T *P0 = tab + 4 * NR, *P1 = P0 + 512;
    const ConstPtr<T> TA = as_const(P1 + 512), TAB = as_const(P1 + 512 + 512 * op.k);
    const int tid = threadIdx.x;
    T f0r = P0[2 * tid], f0i = P0[2 * tid + 1], f1r = P1[2 * tid], f1i = P1[2 * tid + 1];
    for (int g = 0; g < op.k; ++g) {
        const int v = (int)((tile >> (8 * g)) & 255ull);
        const T ar = TA[512 * g + 2 * v], ai = TA[512 * g + 2 * v + 1];
        const T br = TAB[512 * g + 2 * v], bi = TAB[512 * g + 2 * v + 1];
        T t = f0r * ar - f0i * ai;
        f0i = f0r * ai + f0i * ar;
        f0r = t;
        t = f1r * br - f1i * bi;
        f1i = f1r * bi + f1i * br;
        f1r = t;
    }
    const int cp = op.ctrl_pos;
    const bool has_ctrl = op.ctrl_q >= 0;
    const bool ctrl_reg = has_ctrl && cp >= 0 && ((smask >> cp) & 1u);
    bool on_t = false;   // control from the thread's bits or the tile base
    if (has_ctrl && !ctrl_reg) on_t = cp >= 0 ? ((tbase >> cp) & 1) != 0 : ((base >> op.ctrl_q) & 1ull) != 0;
    if (ctrl_reg) reg_phase_at<T, R, 0>(reg_rank(smask, cp), re, im, f0r, f0i, f1r, f1i, false, U0, U1);
    else reg_phase_apply<T, R, -1>(re, im, f0r, f0i, f1r, f1i, on_t, U0, U1);
}

// ---------------------------------------------------------------- segment

// seg: the OP_SEG marker (k = ops in the segment, pos[0..R) = S ascending,
// ctrl_local = mask of S); sops: the segment's ops. Ends without a barrier.
template <typename T, int TB>
__device__ __forceinline__ void run_segment(T *samp, const OpDesc &seg, const OpDesc *__restrict__ sops,
                                            const T *__restrict__ pool, uint64_t base, uint64_t tile)
{
    constexpr int R = TB - 8, NR = 1 << R, TILE = 1 << TB;
    static_assert(R >= 2 && R <= 5, "segments need 2..5 register bits");
    int S[R];
#pragma unroll
    for (int r = 0; r < R; ++r) S[r] = seg.pos[r];
    const uint32_t smask = seg.ctrl_local;
    int tbase = threadIdx.x;
#pragma unroll
    for (int r = 0; r < R; ++r) tbase = ((tbase >> S[r]) << (S[r] + 1)) | (tbase & ((1 << S[r]) - 1));
    const int pbase = swz(tbase);
    T re[NR], im[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int l = pbase ^ swz(reg_offset<R>(S, i));
        re[i] = samp[l];
        im[i] = samp[TILE + l];
    }
    for (int k = 0; k < seg.k; ++k) {
        const OpDesc op = load_op(sops + k);
        const T *M = pool + 2 * (int64_t)op.mat;
        if (op.type == OP_DENSE) {
            if (op.ctrl_fixed == 0 || (base & op.ctrl_fixed) == op.ctrl_fixed) reg_dense<T, R>(re, im, op, smask, M);
        } else if (op.type == OP_RDIAG) {
            reg_rdiag<T, R>(re, im, op, tbase, M, base);
        } else if (op.type == OP_RPHASE) {
            reg_phase<T, R>(re, im, op, smask, tbase, M, base, tile);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int l = pbase ^ swz(reg_offset<R>(S, i));
        samp[l] = re[i];
        samp[TILE + l] = im[i];
    }
}

}  // namespace msv
