// Kernels around the pass: basis-state init, FP64 reductions for
// measurement / expectation / fidelity, range decode, and the canonical chunk
// format (encode into per-block slots, per-chunk scan, assembly, parsing).
#include <hip/hip_runtime.h>

#include "codec_device.h"
#include "kernels.h"

namespace msv {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using V = float2; };
template <> struct Vec2<double> { using V = double2; };

static __device__ __forceinline__ uint64_t bidx(const BlockStore &s, uint64_t B)
{
    if (!s.chunk_slot) return B;
    const uint64_t nbm = (1ull << s.log2_nb) - 1;
    return ((uint64_t)s.chunk_slot[B >> s.log2_nb] << s.log2_nb) | (B & nbm);
}

// ------------------------------------------------------------------ init

template <typename T>
__global__ __launch_bounds__(64) void init_basis_block_kernel(BlockStore st, uint64_t index,
                                                              double inv_step)
{
    const uint32_t lane = lane_id();
    bool bad = false;
    const T x = lane == (uint32_t)(index & 63u) ? (T)1 : (T)0;
    const int32_t q = quantize<T>(x, inv_step, bad);
    const uint32_t u = residual_zigzag(q);
    const uint32_t W = block_width(u);
    const int32_t A = __builtin_amdgcn_readlane(q, 0);
    const uint64_t mine = pack_planes(u, W);
    const uint64_t bi = bidx(st, 2 * (index >> 6));
    if (lane < W) st.heap[lane] = mine;
    if (lane == 0) { st.W[bi] = (uint8_t)W; st.A[bi] = A; st.OFF[bi] = 0; }
}

hipError_t launch_init_basis_block(bool is_double, BlockStore st, uint64_t index, double inv_step,
                                   hipStream_t stream)
{
    if (is_double)
        hipLaunchKernelGGL(init_basis_block_kernel<double>, dim3(1), dim3(64), 0, stream, st, index, inv_step);
    else
        hipLaunchKernelGGL(init_basis_block_kernel<float>, dim3(1), dim3(64), 0, stream, st, index, inv_step);
    return hipGetLastError();
}

// ------------------------------------------------------------- reductions

constexpr int kRedGroups = 2048;

// Amplitude blocks G = first + k, k = blockIdx.x * NW + wave + stride * j,
// decoded both planes at a time in rounds of up to 16 per wave: lane 2a + p
// fetches the metadata of round block a, plane p, then every block's payload
// word `lane` is loaded before one wait. f(G, xr, xi) runs per decoded block.
template <typename T, bool COMP, bool PRED, typename F>
// stage: 128 words of LDS for this wave, through which the decode broadcasts
// plane words (unpack_codes4_lds). PRED = false: every block uses predictor 0.
static __device__ __forceinline__ void for_amp_blocks(const void *amps, const BlockStore &st, double step,
                                                      uint64_t first, uint64_t nab, int wave, int lane,
                                                      uint64_t *stage, F &&f)
{
    using V2 = typename Vec2<T>::V;
    constexpr int NW = kThreads / 64;
    constexpr int RA = 16;
    const uint64_t stride = (uint64_t)gridDim.x * NW;
    for (uint64_t k0 = (uint64_t)blockIdx.x * NW + wave; k0 < nab; k0 += stride * RA) {
        if (!COMP) {
            V2 v[RA];
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const uint64_t k = k0 + stride * a;
                if (k < nab) v[a] = ((const V2 *)amps)[((first + k) << 6) | (uint64_t)lane];
            }
#pragma unroll
            for (int a = 0; a < RA; ++a) {
                const uint64_t k = k0 + stride * a;
                if (k < nab) f(first + k, (double)v[a].x, (double)v[a].y);
            }
            continue;
        }
        uint32_t wv = 0, ov = 0;
        int32_t av = 0;
        {
            const uint64_t k = k0 + stride * (uint64_t)(lane >> 1);
            if (lane < 2 * RA && k < nab) {
                const uint64_t bi = bidx(st, 2 * (first + k) + (uint64_t)(lane & 1));
                wv = st.W[bi];
                av = st.A[bi];
                if (wv) ov = st.OFF[bi];
            }
        }
        uint64_t mine[2 * RA];
#pragma unroll
        for (int j = 0; j < 2 * RA; ++j) {
            const uint32_t wj = (uint32_t)__builtin_amdgcn_readlane((int)wv, j);
            const uint32_t W = PRED ? wbyte_width(wj) : wj;   // without PRED the byte is the width
            const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)ov, j);
            mine[j] = 0;
            if ((uint32_t)lane < W) mine[j] = st.heap[(uint64_t)off + lane];
        }
        // two amplitude blocks per unpack loop; a block beyond the range has
        // width 0 and anchor 0 and is not handed to f
#pragma unroll
        for (int a = 0; a < RA; a += 2) {
            const uint64_t k = k0 + stride * a;
            if (k >= nab) break;
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
            unpack_codes4_lds<PRED>(stage, W4, A4, q4);
            f(first + k, (double)dequantize<T>(q4[0], step), (double)dequantize<T>(q4[1], step));
            if (k + stride < nab)
                f(first + k + stride, (double)dequantize<T>(q4[2], step), (double)dequantize<T>(q4[3], step));
        }
    }
}

// One workgroup's share (group blockIdx.x of gridDim.x) of a reduction.
template <typename T, int COMP>
__device__ __forceinline__ void reduce_body(const void *amps, const BlockStore &st, double step, const ReduceArgs &a)
{
    constexpr int NW = kThreads / 64;
    __shared__ double sacc[4][NW];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t nab = a.amp_count >> 6, first = a.amp_begin >> 6;
    // four named accumulators (an array here ends up in scratch memory,
    // indexed at run time by the reduction kind)
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    // Z-strings (up to 64 terms): per block G (64 amplitudes, lane = index
    // bits 0..5) the expectation is sum_t c_t (-1)^popcount(G & h_t) P^(l_t),
    // with l_t / h_t the low 6 / high bits of mask m_t and P^ the 64-point
    // Walsh-Hadamard transform of the block's probabilities over the lanes,
    // P^(l) = sum_j p_j (-1)^popcount(l & j). Six butterfly stages leave P^(l)
    // in lane l; lane t then gathers P^(l_t) for term t and weights it with
    // its own block sign, so the cost per block does not grow with the terms.
    const bool fast = a.kind == RED_EXPZ && a.n_terms <= 64;
    double ct = 0.0;        // lane t: coefficient of term t (0 beyond n_terms)
    uint64_t mhi = 0;       // lane t: block-index part of m_t
    int lsrc = 0;           // lane t: l_t, the lane holding P^(l_t)
    if (fast && lane < a.n_terms) {
        ct = a.coeffs[lane];
        mhi = a.masks[lane] >> 6;
        lsrc = (int)(a.masks[lane] & 63u);
    }
    // butterfly stage k: lanes with bit k set take o - P, the others o + P;
    // as fma(+-1, P, o) this is one rounding, the same as the add it replaces
    const double s0 = (lane & 1) ? -1.0 : 1.0, s1 = (lane & 2) ? -1.0 : 1.0, s2 = (lane & 4) ? -1.0 : 1.0,
                 s3 = (lane & 8) ? -1.0 : 1.0, s4 = (lane & 16) ? -1.0 : 1.0, s5 = (lane & 32) ? -1.0 : 1.0;
    __shared__ uint64_t stage[NW * 128];
    for_amp_blocks<T, COMP != 0, COMP == 2>(amps, st, step, first, nab, wave, lane, stage + 128 * wave,
                            [&](uint64_t G, double xr, double xi) {
        xr *= a.scale;
        xi *= a.scale;
        const uint64_t i = (G << 6) | (uint64_t)lane;
        const double p = xr * xr + xi * xi;
        acc0 += p;
        if (a.kind == RED_PROB1) {
            acc1 += ((i >> a.qubit) & 1ull) ? p : 0.0;
        } else if (a.kind == RED_EXPZ) {
            if (fast) {
                double P = p;
                P = fma(s0, P, __shfl_xor(P, 1, 64));
                P = fma(s1, P, __shfl_xor(P, 2, 64));
                P = fma(s2, P, __shfl_xor(P, 4, 64));
                P = fma(s3, P, __shfl_xor(P, 8, 64));
                P = fma(s4, P, __shfl_xor(P, 16, 64));
                P = fma(s5, P, __shfl_xor(P, 32, 64));
                const double ph = __shfl(P, lsrc, 64);
                acc1 += ((__popcll(G & mhi) & 1) ? -ct : ct) * ph;
            } else {
                double v = 0.0;
                for (int t = 0; t < a.n_terms; ++t)
                    v += (__popcll(i & a.masks[t]) & 1) ? -a.coeffs[t] : a.coeffs[t];
                acc1 += p * v;
            }
        } else if (a.kind == RED_OVERLAP) {
            const uint64_t r = i - a.amp_begin;
            const double rr = a.ref[2 * r], ri = a.ref[2 * r + 1];
            acc1 += rr * xr + ri * xi;   // Re(conj(ref) psi)
            acc2 += rr * xi - ri * xr;   // Im(conj(ref) psi)
            acc3 += rr * rr + ri * ri;
        }
    });
    const double sums[4] = {wave_sum_f64(acc0), wave_sum_f64(acc1), wave_sum_f64(acc2), wave_sum_f64(acc3)};
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) sacc[j][wave] = sums[j];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += sacc[threadIdx.x][w];
        a.partials[4 * blockIdx.x + threadIdx.x] = s;
    }
}

template <typename T, int COMP>
__global__ __launch_bounds__(kThreads) void reduce_kernel(const void *amps, BlockStore st, double step,
                                                          ReduceArgs a)
{
    reduce_body<T, COMP>(amps, st, step, a);
}

// Several reductions of equal length in one launch: job blockIdx.y.
template <typename T, int COMP>
__global__ __launch_bounds__(kThreads) void reduce_multi_kernel(const ReduceJob *jobs)
{
    const ReduceJob &j = jobs[blockIdx.y];
    reduce_body<T, COMP>(j.amps, j.st, j.step, j.a);
}

template <typename T>
static void reduce_comp(int comp, dim3 grid, dim3 block, hipStream_t stream, const void *amps, const BlockStore &st,
                        double step, const ReduceArgs &a)
{
    if (comp == 2) hipLaunchKernelGGL((reduce_kernel<T, 2>), grid, block, 0, stream, amps, st, step, a);
    else if (comp == 1) hipLaunchKernelGGL((reduce_kernel<T, 1>), grid, block, 0, stream, amps, st, step, a);
    else hipLaunchKernelGGL((reduce_kernel<T, 0>), grid, block, 0, stream, amps, st, step, a);
}

static uint64_t reduce_groups(uint64_t amp_count)
{
    uint64_t g = ((amp_count >> 6) + 3) / 4;
    if (g > (uint64_t)kRedGroups) g = kRedGroups;
    return g == 0 ? 1 : g;
}

hipError_t launch_reduce_multi(bool is_double, int comp, const ReduceJob *jobs, int n_jobs, uint64_t amp_count,
                               int *n_groups, hipStream_t stream)
{
    const uint64_t g = reduce_groups(amp_count);
    *n_groups = (int)g;
    if (n_jobs <= 0) return hipSuccess;
    const dim3 grid((unsigned)g, (unsigned)n_jobs), block(kThreads);
    if (is_double) {
        if (comp == 2) hipLaunchKernelGGL((reduce_multi_kernel<double, 2>), grid, block, 0, stream, jobs);
        else if (comp == 1) hipLaunchKernelGGL((reduce_multi_kernel<double, 1>), grid, block, 0, stream, jobs);
        else hipLaunchKernelGGL((reduce_multi_kernel<double, 0>), grid, block, 0, stream, jobs);
    } else {
        if (comp == 2) hipLaunchKernelGGL((reduce_multi_kernel<float, 2>), grid, block, 0, stream, jobs);
        else if (comp == 1) hipLaunchKernelGGL((reduce_multi_kernel<float, 1>), grid, block, 0, stream, jobs);
        else hipLaunchKernelGGL((reduce_multi_kernel<float, 0>), grid, block, 0, stream, jobs);
    }
    return hipGetLastError();
}

hipError_t launch_reduce(bool is_double, int comp, const void *amps, BlockStore st,
                         double step, const ReduceArgs &a, int *n_groups, hipStream_t stream)
{
    const uint64_t g = reduce_groups(a.amp_count);
    *n_groups = (int)g;
    const dim3 grid((unsigned)g), block(kThreads);
    if (is_double) reduce_comp<double>(comp, grid, block, stream, amps, st, step, a);
    else reduce_comp<float>(comp, grid, block, stream, amps, st, step, a);
    return hipGetLastError();
}

// Job blockIdx.x: out[4 job + j] = sum_g partials[4 (job n + g) + j].
__global__ __launch_bounds__(kThreads) void reduce_final_kernel(const double *partials, int n, double *out)
{
    __shared__ double s[4][kThreads];
    partials += (uint64_t)blockIdx.x * 4 * (uint64_t)n;
    out += 4 * blockIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = threadIdx.x; g < n; g += kThreads)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] += partials[4 * g + j];
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = kThreads / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int j = 0; j < 4; ++j) s[j][threadIdx.x] += s[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

hipError_t launch_reduce_final(const double *partials, int n_groups, double *out, hipStream_t stream)
{
    return launch_reduce_final_multi(partials, n_groups, 1, out, stream);
}

hipError_t launch_reduce_final_multi(const double *partials, int n_groups, int n_jobs, double *out,
                                     hipStream_t stream)
{
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_final_kernel, dim3((unsigned)n_jobs), dim3(kThreads), 0, stream, partials, n_groups,
                       out);
    return hipGetLastError();
}

// One workgroup of kStatThreads per pass (a pass has up to 2^(n - TB)
// workgroup partials, 65536 at n = 28).
constexpr int kStatThreads = 1024;

__global__ __launch_bounds__(kStatThreads) void pass_stats_kernel(const double *part, const uint64_t *offs,
                                                                  double *out)
{
    __shared__ double sn[kStatThreads], se[kStatThreads], sw[kStatThreads];
    const int p = blockIdx.x;
    double a = 0.0, e = 0.0, w = 0.0;
    for (uint64_t i = offs[p] + threadIdx.x; i < offs[p + 1]; i += kStatThreads) {
        a += part[3 * i];
        e = fmax(e, part[3 * i + 1]);
        w += part[3 * i + 2];
    }
    sn[threadIdx.x] = a;
    se[threadIdx.x] = e;
    sw[threadIdx.x] = w;
    __syncthreads();
    for (int h = kStatThreads / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sn[threadIdx.x] += sn[threadIdx.x + h];
            se[threadIdx.x] = fmax(se[threadIdx.x], se[threadIdx.x + h]);
            sw[threadIdx.x] += sw[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[3 * p] = sn[0]; out[3 * p + 1] = se[0]; out[3 * p + 2] = sw[0]; }
}

hipError_t launch_pass_stats(const double *part, const uint64_t *pass_offsets, int n_passes, double *out,
                             hipStream_t stream)
{
    if (n_passes <= 0) return hipSuccess;
    hipLaunchKernelGGL(pass_stats_kernel, dim3(n_passes), dim3(kStatThreads), 0, stream, part, pass_offsets, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ range decode

template <typename T, int COMP>
__global__ __launch_bounds__(kThreads) void decode_range_kernel(const void *amps, BlockStore st, double step,
                                                                double scale, uint64_t first, uint64_t nab, void *out)
{
    using V2 = typename Vec2<T>::V;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int NW = kThreads / 64;
    __shared__ uint64_t stage[NW * 128];
    for_amp_blocks<T, COMP != 0, COMP == 2>(amps, st, step, first, nab, wave, lane, stage + 128 * wave,
                            [&](uint64_t G, double xr, double xi) {
        V2 v;
        v.x = (T)xr;
        v.y = (T)xi;
        if (scale != 1.0) { v.x = (T)(v.x * (T)scale); v.y = (T)(v.y * (T)scale); }
        ((V2 *)out)[((G - first) << 6) | (uint64_t)lane] = v;
    });
}

template <typename T>
static void decode_range_comp(int comp, dim3 grid, dim3 block, hipStream_t stream, const void *amps,
                              const BlockStore &st, double step, double scale, uint64_t first, uint64_t nab,
                              void *out)
{
    if (comp == 2)
        hipLaunchKernelGGL((decode_range_kernel<T, 2>), grid, block, 0, stream, amps, st, step, scale, first, nab,
                           out);
    else if (comp == 1)
        hipLaunchKernelGGL((decode_range_kernel<T, 1>), grid, block, 0, stream, amps, st, step, scale, first, nab,
                           out);
    else
        hipLaunchKernelGGL((decode_range_kernel<T, 0>), grid, block, 0, stream, amps, st, step, scale, first, nab,
                           out);
}

hipError_t launch_decode_range(bool is_double, int comp, const void *amps, BlockStore st, double step,
                               double scale, uint64_t amp_begin, uint64_t amp_count, void *out, hipStream_t stream)
{
    const uint64_t nab = amp_count >> 6;
    uint64_t g = (nab + 3) / 4;
    if (g > 65536) g = 65536;
    if (g == 0) return hipSuccess;
    const dim3 grid((unsigned)g), block(kThreads);
    if (is_double) decode_range_comp<double>(comp, grid, block, stream, amps, st, step, scale, amp_begin >> 6, nab, out);
    else decode_range_comp<float>(comp, grid, block, stream, amps, st, step, scale, amp_begin >> 6, nab, out);
    return hipGetLastError();
}

// ---------------------------------------------------- canonical chunk format

template <typename T>
__global__ __launch_bounds__(kThreads) void encode_chunks_kernel(const T *vals, uint64_t n_blocks,
                                                                 double inv_step, double step, int pred_mode,
                                                                 uint8_t *W, int32_t *A, uint64_t *slots,
                                                                 unsigned long long *err_bits, uint32_t *flags)
{
    constexpr int NW = kThreads / 64;
    const uint32_t lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double err = 0.0;
    bool bad = false;
    for (uint64_t b = (uint64_t)blockIdx.x * NW + wave; b < n_blocks; b += (uint64_t)gridDim.x * NW) {
        const uint64_t j = b >> 1, p = b & 1;
        const T x = vals[2 * ((j << 6) | lane) + p];
        const int32_t q = quantize<T>(x, inv_step, bad);
        const T xr = dequantize<T>(q, step);
        err = fmax(err, __builtin_fabs((double)x - (double)xr));
        const int32_t d1 = residual1(q);
        uint32_t u = zigzag(d1);
        uint32_t w = block_width(u), pred = 0;
        if (pred_mode) {
            uint32_t un, u2;
            residuals_alt(q, d1, un, u2);
            const uint32_t wn = block_width(un), w2 = block_width(u2);
            if (wn < w) { w = wn; pred = 1; u = un; }
            if (w2 < w) { w = w2; pred = 2; u = u2; }
        }
        const uint64_t mine = pack_planes(u, w);
        const int32_t a0 = __builtin_amdgcn_readlane(q, 0);
        if (lane < w) slots[b * 32 + lane] = mine;
        if (lane == 0) { W[b] = (uint8_t)(w | (pred << 6)); A[b] = a0; }
    }
    err = wave_max_f64(err);
    if (lane == 0) atomicMax(err_bits, (unsigned long long)__double_as_longlong(err));
    if (bad) atomicOr(flags, 1u);
}

hipError_t launch_encode_chunks(bool is_double, const void *vals, uint64_t n_blocks_total, double inv_step,
                                uint8_t *W, int32_t *A, uint64_t *slot_words, double *err_max_bits,
                                uint32_t *flags, double step, int pred_mode, hipStream_t stream)
{
    uint64_t g = (n_blocks_total + 3) / 4;
    if (g > 65536) g = 65536;
    if (g == 0) return hipSuccess;
    unsigned long long *eb = reinterpret_cast<unsigned long long *>(err_max_bits);
    if (is_double)
        hipLaunchKernelGGL(encode_chunks_kernel<double>, dim3((unsigned)g), dim3(kThreads), 0, stream,
                           (const double *)vals, n_blocks_total, inv_step, step, pred_mode, W, A, slot_words, eb,
                           flags);
    else
        hipLaunchKernelGGL(encode_chunks_kernel<float>, dim3((unsigned)g), dim3(kThreads), 0, stream,
                           (const float *)vals, n_blocks_total, inv_step, step, pred_mode, W, A, slot_words, eb,
                           flags);
    return hipGetLastError();
}

static __device__ __forceinline__ uint64_t pad8(uint64_t x) { return (x + 7) & ~7ull; }

// Block-wide exclusive scan of one uint64 per thread; returns the total.
static __device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *ex, uint64_t *sbuf)
{
    sbuf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const uint64_t t = threadIdx.x >= (unsigned)off ? sbuf[threadIdx.x - off] : 0ull;
        __syncthreads();
        sbuf[threadIdx.x] += t;
        __syncthreads();
    }
    const uint64_t incl = sbuf[threadIdx.x];
    const uint64_t total = sbuf[kThreads - 1];
    __syncthreads();
    *ex = incl - v;
    return total;
}

// Block-wide sum of one uint64 per thread (every thread gets it).
static __device__ uint64_t block_sum(uint64_t v, uint64_t *sbuf)
{
    uint64_t ex;
    return block_exclusive_scan(v, &ex, sbuf);
}

// Four width bytes packed in a word (width in bits 0..5, predictor in bits
// 6..7): the sum of their widths (v_sad_u8 against zero) and whether any is
// malformed: a width above 32 (bit 5 set together with any of bits 0..4), or
// a predictor the chunk's mode does not allow (mode 0: none but 0; mode 1:
// 0..2).
static __device__ __forceinline__ uint32_t width4_sum(uint32_t x, uint32_t acc)
{
    return __builtin_amdgcn_sad_u8(x & 0x3F3F3F3Fu, 0u, acc);
}
static __device__ __forceinline__ uint32_t width4_bad(uint32_t x, uint32_t mode)
{
    const uint32_t low = ((x & 0x1F1F1F1Fu) + 0x1F1F1F1Fu) & 0x20202020u;
    const uint32_t pred_bad = mode ? (x & 0x80808080u & ((x & 0x40404040u) << 1)) : (x & 0xC0C0C0C0u);
    return pred_bad | (x & low);
}
static __device__ __forceinline__ bool width_bad(uint32_t v, uint32_t mode)
{
    return (v & 63u) > 32u || (v >> 6) > (mode ? 2u : 0u);
}

// Sum of the widths of the width bytes w[0..n) over the workgroup's threads
// (per-thread part returned; the caller reduces), with bit flags of malformed
// bytes (for predictor mode `mode`) in *bad.
// n and the address of w must be multiples of 16 for the wide path.
static __device__ __forceinline__ uint64_t widths_part(const uint8_t *w, uint64_t n, uint32_t mode, uint32_t *bad)
{
    uint64_t s = 0;
    uint32_t b = 0;
    if ((((uintptr_t)w) & 15u) == 0 && (n & 15u) == 0) {
        const uint4 *w16 = reinterpret_cast<const uint4 *>(w);
        for (uint64_t i = threadIdx.x; i < n / 16; i += kThreads) {
            const uint4 x = w16[i];
            uint32_t t = width4_sum(x.x, 0u);
            t = width4_sum(x.y, t);
            t = width4_sum(x.z, t);
            t = width4_sum(x.w, t);
            s += t;
            b |= width4_bad(x.x, mode) | width4_bad(x.y, mode) | width4_bad(x.z, mode) | width4_bad(x.w, mode);
        }
    } else {
        for (uint64_t i = threadIdx.x; i < n; i += kThreads) {
            const uint32_t v = w[i];
            s += v & 63u;
            b |= width_bad(v, mode) ? 1u : 0u;
        }
    }
    *bad |= b;
    return s;
}

// Grid: x = chunk, y = segment of the chunk's blocks. Each workgroup sums the
// widths before its segment and scans its segment in tiles of 4 * kThreads
// blocks; the first one also sums the whole chunk and decides its kind (all
// widths and anchors zero: ZERO).
__global__ __launch_bounds__(kThreads) void scan_chunks_kernel(const uint8_t *W, const int32_t *A, uint64_t nb,
                                                               uint32_t *off, uint64_t *sizes, uint32_t *kinds,
                                                               uint32_t *flags)
{
    __shared__ uint64_t sbuf[kThreads];
    __shared__ int snz;
    const uint64_t c = blockIdx.x;
    const uint64_t seg_len = (nb + gridDim.y - 1) / gridDim.y;
    const uint64_t s0 = (uint64_t)blockIdx.y * seg_len;
    if (s0 >= nb) return;   // whole workgroup, before any barrier
    const uint64_t s1 = s0 + seg_len < nb ? s0 + seg_len : nb;
    const bool first = blockIdx.y == 0;
    const uint8_t *w = W + c * nb;
    const int32_t *a = A + c * nb;
    uint32_t bad = 0;
    const uint64_t before = block_sum(widths_part(w, s0, 1u, &bad), sbuf);
    bad = 0;   // widths outside the segment are checked by their own workgroup
    uint64_t carry = before;
    // tiles of 4 * kThreads blocks, four consecutive blocks per thread
    for (uint64_t t0 = s0; t0 < s1; t0 += 4 * kThreads) {
        const uint64_t b = t0 + 4 * (uint64_t)threadIdx.x;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t wb = b + k < s1 ? w[b + k] : 0u;
            bad |= width_bad(wb, 1u) ? 1u : 0u;
            v[k] = wb & 63u;
            sum += v[k];
        }
        uint64_t ex;
        const uint64_t tsum = block_exclusive_scan(sum, &ex, sbuf);
        uint64_t run = carry + ex;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (b + k < s1) off[c * nb + b + k] = (uint32_t)run;
            run += v[k];
        }
        carry += tsum;
    }
    if (bad) atomicOr(flags, 2u);
    if (!first) return;   // whole workgroup
    // first segment: the whole chunk's total (widths from s1 on) and kind
    uint32_t ignore = 0;
    const uint64_t rest = block_sum(widths_part(w + s1, nb - s1, 1u, &ignore), sbuf);
    const uint64_t total = carry + rest;   // the same in every thread
    bool general = total != 0;
    if (!general) {
        // no payload: the chunk is ZERO unless an anchor is nonzero
        if (threadIdx.x == 0) snz = 0;
        __syncthreads();
        bool nz = false;
        for (uint64_t i = threadIdx.x; i < nb; i += kThreads) nz |= a[i] != 0;
        if (nz) snz = 1;
        __syncthreads();
        general = snz != 0;
    }
    if (threadIdx.x == 0) {
        kinds[c] = general ? 1u : 0u;
        sizes[c] = general ? 32 + pad8(nb) + pad8(4 * nb) + 8 * total : 32;
    }
}

hipError_t launch_scan_chunks(const uint8_t *W, const int32_t *A, uint64_t nb, uint64_t n_chunks, uint32_t *off,
                              uint64_t *sizes, uint32_t *kinds, uint32_t *flags, hipStream_t stream)
{
    if (n_chunks == 0) return hipSuccess;
    if (n_chunks > 0x7fffffffull) return hipErrorInvalidValue;
    // segments of at least 2048 blocks, at most 64 per chunk
    uint64_t segs = nb / 2048;
    if (segs < 1) segs = 1;
    if (segs > 64) segs = 64;
    hipLaunchKernelGGL(scan_chunks_kernel, dim3((unsigned)n_chunks, (unsigned)segs), dim3(kThreads), 0, stream, W,
                       A, nb, off, sizes, kinds, flags);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void scan_sizes_kernel(const uint64_t *sizes, uint64_t n, uint64_t *offsets)
{
    __shared__ uint64_t sbuf[kThreads];
    const uint64_t per = (n + kThreads - 1) / kThreads;
    const uint64_t i0 = threadIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    uint64_t s = 0;
    for (uint64_t i = i0; i < i1; ++i) s += (sizes[i] + 255) & ~255ull;
    uint64_t ex;
    const uint64_t total = block_exclusive_scan(s, &ex, sbuf);
    for (uint64_t i = i0; i < i1; ++i) {
        offsets[i] = ex;
        ex += (sizes[i] + 255) & ~255ull;
    }
    if (threadIdx.x == 0) offsets[n] = total;
}

__global__ __launch_bounds__(kThreads) void zero_words_kernel(uint64_t *p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        p[i] = 0;
}

hipError_t launch_zero_words(uint64_t *p, uint64_t n_words, hipStream_t stream)
{
    if (n_words == 0) return hipSuccess;
    uint64_t g = (n_words + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)g), dim3(kThreads), 0, stream, p, n_words);
    return hipGetLastError();
}

hipError_t launch_scan_sizes(const uint64_t *sizes, uint64_t n, uint64_t *offsets, hipStream_t stream)
{
    hipLaunchKernelGGL(scan_sizes_kernel, dim3(1), dim3(kThreads), 0, stream, sizes, n, offsets);
    return hipGetLastError();
}

// One wave per 64 consecutive blocks (lane = block): the lanes write their
// blocks' widths and anchors side by side, the lane of a chunk's first block
// writes that chunk's header, then the wave copies the payload of its blocks
// one block at a time (lanes = the block's plane words). nb is a power of two.
__global__ __launch_bounds__(kThreads) void assemble_chunks_kernel(int dtype, int log2c, double eb, int pred_mode,
                                                                   const uint8_t *W, const int32_t *A,
                                                                   const uint32_t *src_off, const uint64_t *src,
                                                                   const uint32_t *dst_off, const uint64_t *sizes,
                                                                   const uint32_t *kinds, const uint64_t *offsets,
                                                                   uint64_t nb, uint64_t n_chunks, uint8_t *out)
{
    constexpr int NW = kThreads / 64;
    const uint32_t lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t total_blocks = nb * n_chunks;
    const int lnb = __builtin_ctzll(nb);
    const uint64_t a_off = 32 + pad8(nb), p_off = a_off + pad8(4 * nb);
    const uint64_t stride = (uint64_t)gridDim.x * NW * 64;
    for (uint64_t g0 = ((uint64_t)blockIdx.x * NW + wave) * 64; g0 < total_blocks; g0 += stride) {
        const uint64_t gb = g0 + lane;
        const bool in = gb < total_blocks;
        const uint64_t c = in ? gb >> lnb : 0, b = gb & (nb - 1);
        uint8_t *o = out + (in ? offsets[c] : 0);
        const bool general = in && kinds[c] != 0;
        if (in && b == 0) {
            uint32_t *h = reinterpret_cast<uint32_t *>(o);
            const uint64_t ebits = (uint64_t)__double_as_longlong(eb);
            h[0] = 0x4356534Du;
            h[1] = 1u | ((general ? 1u : 0u) << 8) | ((uint32_t)log2c << 16) | ((uint32_t)dtype << 24);
            h[2] = (uint32_t)(ebits & 0xffffffffull);
            h[3] = (uint32_t)(ebits >> 32);
            h[4] = (uint32_t)(sizes[c] & 0xffffffffull);
            h[5] = (uint32_t)(sizes[c] >> 32);
            h[6] = (uint32_t)nb;
            h[7] = (uint32_t)pred_mode;
            if (general) {
                // zero padding after W and after A
                for (uint64_t i = 32 + nb; i < a_off; ++i) o[i] = 0;
                for (uint64_t i = a_off + 4 * nb; i < p_off; ++i) o[i] = 0;
            }
        }
        uint32_t w = 0;
        uint64_t d = 0, so = 0;
        if (general) {
            const uint32_t wb = W[gb];
            o[32 + b] = (uint8_t)wb;
            w = wb & 63u;
            reinterpret_cast<int32_t *>(o + a_off)[b] = A[gb];
            d = (uint64_t)(uintptr_t)(reinterpret_cast<uint64_t *>(o) + p_off / 8 + dst_off[gb]);
            so = src_off ? (uint64_t)src_off[gb] : gb * 32;
        }
        uint64_t m = __ballot(w != 0);
        while (m) {
            const int j = __builtin_ctzll(m);
            m &= m - 1;
            const uint32_t wj = (uint32_t)__builtin_amdgcn_readlane((int)w, j);
            const uint64_t dj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(d >> 32), j) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)d, j);
            const uint64_t sj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(so >> 32), j) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)so, j);
            if (lane < wj) reinterpret_cast<uint64_t *>((uintptr_t)dj)[lane] = src[sj + lane];
        }
    }
}

hipError_t launch_assemble_chunks(int dtype, int log2c, double eb, int pred_mode, const uint8_t *W, const int32_t *A,
                                  const uint32_t *src_off, const uint64_t *src_heap, const uint32_t *dst_off,
                                  const uint64_t *sizes, const uint32_t *kinds, const uint64_t *offsets,
                                  uint64_t n_chunks, uint8_t *out, hipStream_t stream)
{
    const uint64_t nb = (2ull << log2c) / 64;
    if (log2c < 6 || (nb & (nb - 1)) != 0) return hipErrorInvalidValue;
    uint64_t g = (nb * n_chunks + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_chunks_kernel, dim3((unsigned)g), dim3(kThreads), 0, stream, dtype, log2c, eb,
                       pred_mode, W, A, src_off, src_heap, dst_off, sizes, kinds, offsets, nb, n_chunks, out);
    return hipGetLastError();
}


// Grid: x = chunk, y = segment of the chunk's blocks. Every workgroup checks
// the header and the widths of the whole chunk (so all of a chunk's
// workgroups take the same accept/reject decision), sums the widths before
// its segment, then scans its own segment in tiles of 4 * kThreads blocks.
__global__ __launch_bounds__(kThreads) void parse_chunks_kernel(const uint8_t *base, const uint64_t *offsets,
                                                                const uint64_t *staged, int log2c, uint64_t nb,
                                                                uint8_t *W, int32_t *A, uint32_t *OFF,
                                                                uint32_t *flags)
{
    __shared__ uint64_t sbuf[kThreads];
    __shared__ int sbad;
    const uint64_t c = blockIdx.x;
    const uint64_t seg_len = (nb + gridDim.y - 1) / gridDim.y;
    const uint64_t s0 = (uint64_t)blockIdx.y * seg_len;
    if (s0 >= nb) return;   // whole workgroup, before any barrier
    const uint64_t s1 = s0 + seg_len < nb ? s0 + seg_len : nb;
    const uint8_t *o = base + offsets[c];
    const uint64_t have = staged[c];
    const uint64_t a_off = 32 + pad8(nb), p_off = a_off + pad8(4 * nb);
    // header first: nothing past it is read unless the header is consistent
    // with the bytes actually staged for this chunk
    bool hdr_bad = have < 32;
    uint32_t kind = 0, mode = 0;
    uint64_t total = 0;
    if (!hdr_bad) {
        const uint32_t *h = reinterpret_cast<const uint32_t *>(o);
        const uint32_t meta = h[1];
        kind = (meta >> 8) & 0xffu;
        mode = h[7];
        total = (uint64_t)h[4] | ((uint64_t)h[5] << 32);
        hdr_bad = h[0] != 0x4356534Du || (meta & 0xffu) != 1u || kind > 1u ||
                  ((meta >> 16) & 0xffu) != (uint32_t)log2c || h[6] != (uint32_t)nb || mode > 1u ||
                  total != have || (kind == 0 && total != 32) || (kind == 1 && total < p_off);
    }
    const bool general = !hdr_bad && kind == 1;
    if (threadIdx.x == 0) sbad = hdr_bad ? 1 : 0;
    __syncthreads();
    const uint8_t *wb = o + 32;
    uint32_t wbad = 0;
    uint64_t pre = 0, all = 0;
    if (general) {
        pre = widths_part(wb, s0, mode, &wbad);
        all = pre + widths_part(wb + s0, nb - s0, mode, &wbad);
    }
    if (wbad) sbad = 1;
    const uint64_t words = block_sum(all, sbuf);
    const uint64_t before = block_sum(pre, sbuf);
    if (threadIdx.x == 0 && general && p_off + 8 * words != total) sbad = 1;
    __syncthreads();
    const bool ok = general && sbad == 0;
    uint64_t carry = (offsets[c] + p_off) / 8 + before;
    // tiles of 4 * kThreads blocks, four consecutive blocks per thread
    for (uint64_t t0 = s0; t0 < s1; t0 += 4 * kThreads) {
        const uint64_t b = t0 + 4 * (uint64_t)threadIdx.x;
        uint32_t w[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w[k] = ok && b + k < s1 ? wb[b + k] : 0u;
            sum += w[k] & 63u;
        }
        uint64_t ex;
        const uint64_t tsum = block_exclusive_scan(sum, &ex, sbuf);
        uint64_t run = carry + ex;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (b + k < s1) {
                const uint64_t gb = c * nb + b + k;
                W[gb] = (uint8_t)w[k];
                A[gb] = ok ? reinterpret_cast<const int32_t *>(o + a_off)[b + k] : 0;
                OFF[gb] = ok ? (uint32_t)run : 0u;
            }
            run += w[k] & 63u;
        }
        carry += tsum;
    }
    if (threadIdx.x == 0 && blockIdx.y == 0 && sbad) atomicOr(flags, 4u);
}

hipError_t launch_parse_chunks(const uint8_t *base, const uint64_t *offsets, const uint64_t *staged,
                               uint64_t n_chunks, int log2c, uint8_t *W, int32_t *A, uint32_t *OFF,
                               uint32_t *flags, hipStream_t stream)
{
    if (n_chunks == 0) return hipSuccess;
    if (n_chunks > 0x7fffffffull) return hipErrorInvalidValue;
    const uint64_t nb = (2ull << log2c) / 64;
    // segments of at least 2048 blocks, at most 64 per chunk
    uint64_t segs = nb / 2048;
    if (segs < 1) segs = 1;
    if (segs > 64) segs = 64;
    hipLaunchKernelGGL(parse_chunks_kernel, dim3((unsigned)n_chunks, (unsigned)segs), dim3(kThreads), 0, stream, base,
                       offsets, staged, log2c, nb, W, A, OFF, flags);
    return hipGetLastError();
}

}  // namespace msv
