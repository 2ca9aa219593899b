// The fused streamed pass: load (decode) -> apply every op of the pass in LDS
// -> store (encode), one workgroup per tile of 2^TB amplitudes.
//
// A pass (one stage of the paper's online loop, Sec. 2) is a run of gates whose
// non-diagonal qubits all fit into one tile: the tile's first six bits are
// qubits 0..5 (so it consists of whole 64-amplitude codec blocks) and its other
// TB-6 bits are the pass's qubits, which may lie inside a chunk or cross chunks
// (then the workgroup gathers blocks from 2^h chunks: the chunk-pair exchange).
// Every workgroup decodes its blocks into LDS (planar re / im), runs the op
// list with a barrier between ops, and re-encodes its blocks. Encoded payload
// goes to the workgroup's own heap slot (worst case 32 words per block), so
// no cross-workgroup scan is needed; W / A / OFF record where each block went.
#include <hip/hip_runtime.h>

#include "codec_device.h"
#include "kernels.h"

namespace msv {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using V = float2; };
template <> struct Cplx<double> { using V = double2; };

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ uint64_t block_index(const BlockStore &s, uint64_t B)
{
    if (!s.chunk_slot) return B;
    const uint64_t nbm = (1ull << s.log2_nb) - 1;
    return ((uint64_t)s.chunk_slot[B >> s.log2_nb] << s.log2_nb) | (B & nbm);
}

// Dense 2^K x 2^K complex matrix on tile-local bits op.pos[0..K), matrix index
// s = sum_m b(pos[m]) 2^m. Each work item loads its group of 2^K amplitudes
// into registers and writes RPT output rows; when there are fewer groups than
// threads, adjacent lanes of one wave share a group (all loads of a wave are
// issued before its stores, so sharing is race-free).
template <typename T, int TB, int K>
__device__ __forceinline__ void op_dense(T *__restrict__ sre, T *__restrict__ sim,
                                         const OpDesc &op, const T *__restrict__ M)
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
        offs[s] = o;
    }
    const int cl = (int)op.ctrl_local;
    for (int w = threadIdx.x; w < NG * TPG; w += kThreads) {
        const int g = w / TPG, rb = w % TPG;
        int l0 = g;
#pragma unroll
        for (int m = 0; m < K; ++m) l0 = ((l0 >> sp[m]) << (sp[m] + 1)) | (l0 & ((1 << sp[m]) - 1));
        if ((l0 & cl) != cl) continue;
        T vr[D], vi[D];
#pragma unroll
        for (int s = 0; s < D; ++s) { vr[s] = sre[l0 + offs[s]]; vi[s] = sim[l0 + offs[s]]; }
#pragma unroll
        for (int rr = 0; rr < RPT; ++rr) {
            const int r = rb * RPT + rr;
            T ar = 0, ai = 0;
#pragma unroll
            for (int s = 0; s < D; ++s) {
                const T mr = M[2 * (r * D + s)], mi = M[2 * (r * D + s) + 1];
                ar = fmaT(mr, vr[s], ar);
                ar = fmaT(-mi, vi[s], ar);
                ai = fmaT(mr, vi[s], ai);
                ai = fmaT(mi, vr[s], ai);
            }
            int lr = l0;
#pragma unroll
            for (int s = 0; s < D; ++s)
                if (s == r) lr = l0 + offs[s];
            sre[lr] = ar;
            sim[lr] = ai;
        }
    }
}

// Diagonal over K qubits: amplitude *= d[s], s = sum_m b(q_m) 2^m, each bit
// taken from the tile-local index or, for qubits outside the tile, from base.
template <typename T, int TB, int K>
__device__ __forceinline__ void op_diag(T *__restrict__ sre, T *__restrict__ sim, const OpDesc &op,
                                        const T *__restrict__ dv, uint64_t base)
{
    int fixed_s = 0;
#pragma unroll
    for (int m = 0; m < K; ++m)
        if (op.pos[m] < 0) fixed_s |= (int)((base >> op.gq[m]) & 1ull) << m;
    for (int l = threadIdx.x; l < (1 << TB); l += kThreads) {
        int s = fixed_s;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if (op.pos[m] >= 0) s |= ((l >> op.pos[m]) & 1) << m;
        const T dr = dv[2 * s], di = dv[2 * s + 1];
        const T xr = sre[l], xi = sim[l];
        sre[l] = fmaT(xr, dr, -xi * di);
        sim[l] = fmaT(xr, di, xi * dr);
    }
}

// Controlled linear phase (a run of diagonal gates sharing one control c):
//   factor(g) = A(g) * (b_c(g) ? B(g) : 1),
// A and B products of per-qubit phases. Tile-local qubits factor through two
// tables indexed by the low 6 bits and by the high TB-6 bits; qubits outside
// the tile contribute a per-tile constant built from per-qubit factors.
template <typename T, int TB>
__device__ __forceinline__ void op_phase(T *__restrict__ sre, T *__restrict__ sim,
                                         const OpDesc &op, const T *__restrict__ tab,
                                         uint64_t base, int n, T *__restrict__ scratch)
{
    constexpr int NH = 1 << (TB - 6);
    const T *loA = tab, *hiA = tab + 2 * 64, *loB = tab + 2 * (64 + NH), *hiB = tab + 2 * (128 + NH);
    const T *fixA = tab + 2 * (128 + 2 * NH), *fixB = fixA + 2 * n;
    // per-tile constants: product over set fixed bits (bit of base) of the factor
    T ar = 1, ai = 0, br = 1, bi = 0;
    const uint64_t fm = base & op.ctrl_fixed;  // ctrl_fixed holds the non-tile qubit mask here
    for (int q = 0; q < n; ++q) {
        if (!((fm >> q) & 1ull)) continue;
        T fr = fixA[2 * q], fi = fixA[2 * q + 1];
        T tr = ar * fr - ai * fi; ai = ar * fi + ai * fr; ar = tr;
        fr = fixB[2 * q]; fi = fixB[2 * q + 1];
        tr = br * fr - bi * fi; bi = br * fi + bi * fr; br = tr;
    }
    bool ctrl_fixed_on = true;
    if (op.ctrl_q >= 0 && op.ctrl_pos < 0) ctrl_fixed_on = (base >> op.ctrl_q) & 1ull;
    // scratch tables: lo' = (loA * A_fix) for ctrl 0, (loA*loB * A_fix*B_fix) for ctrl 1
    T *lo0 = scratch, *lo1 = scratch + 128, *hi1 = scratch + 256;
    for (int i = threadIdx.x; i < 64; i += kThreads) {
        T xr = loA[2 * i], xi = loA[2 * i + 1];
        T r0 = xr * ar - xi * ai, i0 = xr * ai + xi * ar;
        lo0[2 * i] = r0; lo0[2 * i + 1] = i0;
        T yr = loB[2 * i], yi = loB[2 * i + 1];
        T cr = br * yr - bi * yi, ci = br * yi + bi * yr;
        lo1[2 * i] = r0 * cr - i0 * ci; lo1[2 * i + 1] = r0 * ci + i0 * cr;
    }
    for (int i = threadIdx.x; i < NH; i += kThreads) {
        T xr = hiA[2 * i], xi = hiA[2 * i + 1];
        T yr = hiB[2 * i], yi = hiB[2 * i + 1];
        hi1[2 * i] = xr * yr - xi * yi; hi1[2 * i + 1] = xr * yi + xi * yr;
    }
    __syncthreads();
    const int cp = op.ctrl_pos;
    const bool has_ctrl = op.ctrl_q >= 0;
    for (int l = threadIdx.x; l < (1 << TB); l += kThreads) {
        bool on = has_ctrl && (cp >= 0 ? ((l >> cp) & 1) != 0 : ctrl_fixed_on);
        const T *lo = on ? lo1 : lo0;
        const T *hi = on ? hi1 : hiA;
        const int a = l & 63, h = l >> 6;
        T fr = lo[2 * a], fi = lo[2 * a + 1];
        T gr = hi[2 * h], gi = hi[2 * h + 1];
        T pr = fr * gr - fi * gi, pi = fr * gi + fi * gr;
        const T xr = sre[l], xi = sim[l];
        sre[l] = fmaT(xr, pr, -xi * pi);
        sim[l] = fmaT(xr, pi, xi * pr);
    }
}

template <typename T, int TB, bool LOADC, bool STOREC>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassGeom geo, PassBuffers buf)
{
    constexpr int TILE = 1 << TB;
    constexpr int NAB = TILE >> 6;   // 64-amplitude blocks per tile
    constexpr int NSB = 2 * NAB;     // stream blocks (re + im planes)
    constexpr int NW = kThreads / 64;
    constexpr int VPT = sizeof(T) / 4;   // uint32 words per LDS value
    using V2 = typename Cplx<T>::V;

    __shared__ T sre[TILE];
    __shared__ T sim[TILE];
    __shared__ uint64_t sG[NAB];
    __shared__ uint32_t sW[NSB];
    __shared__ int32_t sA[NSB];
    __shared__ uint32_t sOff[NSB];
    __shared__ double sred[2 * NW];
    __shared__ T sph[2 * (128 + (1 << (TB - 6)))];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform for the compiler
    const uint64_t tile = geo.tile_begin + blockIdx.x;

    // global index of the tile's amplitude 0: tile bits deposited into the
    // non-tile positions in ascending order
    uint64_t base = 0;
    {
        uint64_t m = geo.nontile_mask, t = tile;
        while (m) {
            const uint64_t low = m & (~m + 1ull);
            if (t & 1ull) base |= low;
            t >>= 1;
            m &= m - 1;
        }
    }
    for (int jb = tid; jb < NAB; jb += kThreads) {
        uint64_t G = base >> 6;
#pragma unroll
        for (int i = 0; i < TB - 6; ++i)
            if ((jb >> i) & 1) G |= 1ull << (geo.tile_q[6 + i] - 6);
        sG[jb] = G;
    }
    __syncthreads();

    // ---------------------------------------------------------------- load
    if (!LOADC) {
        const V2 *a = (const V2 *)buf.amps_in;
        for (int jb = wave; jb < NAB; jb += NW) {
            const V2 v = a[(sG[jb] << 6) | (uint64_t)lane];
            sre[jb * 64 + lane] = v.x;
            sim[jb * 64 + lane] = v.y;
        }
    } else {
        const double sc = buf.scale_src ? 1.0 / __builtin_sqrt(*buf.scale_src) : buf.scale;
        const T scale = (T)sc;
        for (int bt = wave; bt < NSB; bt += NW) {
            const int jb = bt >> 1, p = bt & 1;
            const uint64_t bi = block_index(buf.in, 2 * sG[jb] + (uint64_t)p);
            const uint32_t W = buf.in.W[bi];
            const int32_t A = buf.in.A[bi];
            uint64_t mine = 0;
            if (W) {
                const uint64_t off = buf.in.OFF[bi];
                if ((uint32_t)lane < W) mine = buf.in.heap[off + lane];
            }
            const int32_t q = unpack_codes(mine, W, A);
            T x = dequantize<T>(q, buf.step);
            if (sc != 1.0) x *= scale;
            (p ? sim : sre)[jb * 64 + lane] = x;
        }
    }
    __syncthreads();

    // ----------------------------------------------------------------- ops
    const T *pool = (const T *)buf.pool;
    for (int oi = 0; oi < geo.n_ops; ++oi) {
        const OpDesc op = buf.ops[geo.op_begin + oi];
        const T *M = pool + 2 * (int64_t)op.mat;
        if (op.type == OP_DENSE) {
            if (op.ctrl_fixed == 0 || (base & op.ctrl_fixed) == op.ctrl_fixed) {
                switch (op.k) {
                case 1: op_dense<T, TB, 1>(sre, sim, op, M); break;
                case 2: op_dense<T, TB, 2>(sre, sim, op, M); break;
                case 3: op_dense<T, TB, 3>(sre, sim, op, M); break;
                case 4: op_dense<T, TB, 4>(sre, sim, op, M); break;
                default: op_dense<T, TB, 5>(sre, sim, op, M); break;
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
            op_phase<T, TB>(sre, sim, op, M, base, geo.n, sph);
        }
        __syncthreads();
    }

    // --------------------------------------------------------------- store
    double nrm = 0.0, err = 0.0;
    if (!STOREC) {
        V2 *a = (V2 *)buf.amps_out;
        for (int jb = wave; jb < NAB; jb += NW) {
            V2 v;
            v.x = sre[jb * 64 + lane];
            v.y = sim[jb * 64 + lane];
            const double xr = v.x, xi = v.y;
            nrm += xr * xr + xi * xi;
            a[(sG[jb] << 6) | (uint64_t)lane] = v;
        }
    } else {
        bool bad = false;
        const double inv_step = buf.inv_step, step = buf.step;
        // E1: codes, residuals, widths; the zigzag residual replaces the value in LDS
        for (int bt = wave; bt < NSB; bt += NW) {
            const int jb = bt >> 1, p = bt & 1;
            T *plane = p ? sim : sre;
            const T x = plane[jb * 64 + lane];
            const double xd = (double)x;
            nrm += xd * xd;
            const int32_t q = quantize<T>(x, inv_step, bad);
            if (buf.check_err) {
                const T xr = dequantize<T>(q, step);
                err = fmax(err, __builtin_fabs(xd - (double)xr));
            }
            const uint32_t u = residual_zigzag(q);
            const uint32_t W = block_width(u);
            const int32_t A = __builtin_amdgcn_readlane(q, 0);
            reinterpret_cast<uint32_t *>(plane)[(jb * 64 + lane) * VPT] = u;
            if (lane == 0) { sW[bt] = W; sA[bt] = A; }
        }
        if (bad) atomicOr(buf.flags, 1u);
        __syncthreads();
        // E2: exclusive scan of the widths over the tile's blocks
        if (wave == 0) {
            constexpr int PER = (NSB + 63) / 64;
            uint32_t v[PER];
            uint32_t s = 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int idx = lane * PER + i;
                v[i] = idx < NSB ? sW[idx] : 0u;
                s += v[i];
            }
            uint32_t ex = wave_inclusive_sum(s) - s;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int idx = lane * PER + i;
                if (idx < NSB) sOff[idx] = ex;
                ex += v[i];
            }
        }
        __syncthreads();
        // E3: bit planes into this tile's heap slot
        const uint64_t slot = (tile - buf.slot_tile0) * (uint64_t)(32 * NSB);
        for (int bt = wave; bt < NSB; bt += NW) {
            const int jb = bt >> 1, p = bt & 1;
            const T *plane = p ? sim : sre;
            const uint32_t u = reinterpret_cast<const uint32_t *>(plane)[(jb * 64 + lane) * VPT];
            const uint32_t W = sW[bt];
            const uint64_t mine = pack_planes(u, W);
            const uint64_t off = slot + sOff[bt];
            if ((uint32_t)lane < W) buf.out.heap[off + lane] = mine;
            if (lane == 0) {
                const uint64_t bi = block_index(buf.out, 2 * sG[jb] + (uint64_t)p);
                buf.out.W[bi] = (uint8_t)W;
                buf.out.A[bi] = sA[bt];
                buf.out.OFF[bi] = (uint32_t)off;
            }
        }
    }
    // per-workgroup statistics (fixed reduction order)
    nrm = wave_sum_f64(nrm);
    err = wave_max_f64(err);
    if (lane == 0) { sred[wave] = nrm; sred[NW + wave] = err; }
    __syncthreads();
    if (tid == 0 && buf.part) {
        double a = 0.0, e = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) { a += sred[w]; e = fmax(e, sred[NW + w]); }
        buf.part[3 * blockIdx.x] = a;
        buf.part[3 * blockIdx.x + 1] = e;
        buf.part[3 * blockIdx.x + 2] = STOREC ? (double)(sOff[NSB - 1] + sW[NSB - 1]) : 0.0;
    }
}

template <typename T, int TB>
static hipError_t launch_tb(bool load_c, bool store_c, const PassGeom &geo, const PassBuffers &buf,
                            hipStream_t stream)
{
    const dim3 grid((unsigned)geo.n_tiles), block(kThreads);
    if (load_c && store_c)
        hipLaunchKernelGGL((pass_kernel<T, TB, true, true>), grid, block, 0, stream, geo, buf);
    else if (load_c)
        hipLaunchKernelGGL((pass_kernel<T, TB, true, false>), grid, block, 0, stream, geo, buf);
    else if (store_c)
        hipLaunchKernelGGL((pass_kernel<T, TB, false, true>), grid, block, 0, stream, geo, buf);
    else
        hipLaunchKernelGGL((pass_kernel<T, TB, false, false>), grid, block, 0, stream, geo, buf);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(bool load_c, bool store_c, const PassGeom &geo, const PassBuffers &buf,
                           hipStream_t stream)
{
    switch (geo.tb) {
    case 6: return launch_tb<T, 6>(load_c, store_c, geo, buf, stream);
    case 7: return launch_tb<T, 7>(load_c, store_c, geo, buf, stream);
    case 8: return launch_tb<T, 8>(load_c, store_c, geo, buf, stream);
    case 9: return launch_tb<T, 9>(load_c, store_c, geo, buf, stream);
    case 10: return launch_tb<T, 10>(load_c, store_c, geo, buf, stream);
    case 11: return launch_tb<T, 11>(load_c, store_c, geo, buf, stream);
    case 12: return launch_tb<T, 12>(load_c, store_c, geo, buf, stream);
    case 13: return launch_tb<T, 13>(load_c, store_c, geo, buf, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass(bool is_double, bool load_c, bool store_c, const PassGeom &geo,
                       const PassBuffers &buf, hipStream_t stream)
{
    if (geo.n_tiles == 0) return hipSuccess;
    if (geo.n_tiles > 0x7fffffffull) return hipErrorInvalidValue;
    return is_double ? launch_t<double>(load_c, store_c, geo, buf, stream)
                     : launch_t<float>(load_c, store_c, geo, buf, stream);
}

}  // namespace msv
