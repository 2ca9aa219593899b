/*
 * Oracle: scalar CPU reference of the chunk codec (format "MSVC" version 1).
 *
 * TEST INFRASTRUCTURE ONLY. The product library never links or calls this
 * file. It exists so that the GPU codec can be checked byte for byte.
 *
 * The paper compresses every state chunk independently (Sec. 2, "Offline
 * stage") with an unnamed lossy compressor and names the codec as pluggable
 * (Sec. 2, end of "Online stage"). The codec here is the project's own
 * specification, implemented one value at a time:
 *
 *  input   C = 2^c complex values (f64 or f32, interleaved), c >= 6. Plane p=0
 *          holds the real parts, p=1 the imaginary parts. Block j of plane p
 *          covers amplitudes 64j..64j+63; its stream index is b = 2j + p.
 *  quantize  q = (int32) rint((double)x * inv_step), inv_step = 1/(2 eb) in
 *          FP64, round half to even. Non-finite x, or |rint(.)| > 2^30 - 1,
 *          rejects the chunk.
 *  predict   anchor A_b = q_0; d_0 = 0; for i >= 1, in 32-bit wrap-around
 *          arithmetic, one of
 *            predictor 0 (Lorenzo-1)  d_i = q_i - q_(i-1)
 *            predictor 1 (none)       d_i = q_i
 *            predictor 2 (Lorenzo-2)  d_1 = q_1 - q_0,
 *                                     d_i = q_i - 2 q_(i-1) + q_(i-2) (i >= 2).
 *          Mode 0 (header field `mode`) uses predictor 0 for every block;
 *          mode 1 picks, per block, the predictor whose residuals need the
 *          fewest bits (ties to the lower id).
 *  zigzag    u_i = (d_i << 1) ^ (d_i >> 31)   (as uint32).
 *  width     W_b = bits needed for OR_i u_i (0..32).
 *  pack      W_b 64-bit words; bit i of word k is bit k of u_i.
 *  kind      ZERO when every A_b and W_b is 0, else GENERAL.
 *  layout    32-byte header
 *              u32 magic 0x4356534D | u8 version 1 | u8 kind | u8 log2C |
 *              u8 dtype (0 f64, 1 f32) | f64 eb | u64 total_bytes |
 *              u32 n_blocks (= 2C/64) | u32 mode (0 or 1)
 *            ZERO chunks end here. GENERAL chunks continue with
 *              u8 W[n_blocks]: W_b | predictor << 6 (zero-padded to 8 bytes),
 *              i32 A[n_blocks] (zero-padded to 8 bytes),
 *              the payload words of all blocks in stream order.
 *  decode    predictor 0: q_i = A_b + sum_{1<=m<=i} d_m;
 *            predictor 1: q_0 = A_b, q_i = d_i;
 *            predictor 2: e_i = sum_{1<=m<=i} d_m, q_i = A_b + sum_{1<=m<=i} e_m
 *            (wrap-around sums, d_m = unzigzag(u_m));
 *            x' = (T)((double)q_i * step), step = 2 eb.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define ORC_MAGIC 0x4356534Du
#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_RANGE (-4)
#define ORC_E_CORRUPT (-6)

static size_t pad8(size_t x) { return (x + 7u) & ~(size_t)7u; }

static void put_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

/* Quantize one value; returns 0 or ORC_E_RANGE. */
int orc_quantize(double x, double inv_step, int32_t *q)
{
    if (!isfinite(x)) return ORC_E_RANGE;
    double r = rint(x * inv_step);
    if (fabs(r) > 1073741823.0) return ORC_E_RANGE;
    *q = (int32_t)r;
    return ORC_OK;
}

/* Worst-case encoded size of one chunk of 2^log2c values. */
size_t orc_codec_bound(int log2c)
{
    size_t nb = ((size_t)2 << log2c) / 64;
    return 32 + pad8(nb) + pad8(4 * nb) + nb * 32 * 8;
}

/* Residuals of one block under predictor `pred`, zigzagged, into u[64]
 * (u[0] = 0); returns the block's width. */
static int block_residuals(const int32_t *q, int pred, uint32_t *u)
{
    uint32_t acc = 0;
    u[0] = 0;
    for (int i = 1; i < 64; ++i) {
        uint32_t d;
        if (pred == 0) d = (uint32_t)q[i] - (uint32_t)q[i - 1];
        else if (pred == 1) d = (uint32_t)q[i];
        else if (i == 1) d = (uint32_t)q[1] - (uint32_t)q[0];
        else d = (uint32_t)q[i] - 2u * (uint32_t)q[i - 1] + (uint32_t)q[i - 2];
        int32_t ds = (int32_t)d;
        u[i] = (d << 1) ^ (uint32_t)(ds >> 31);
        acc |= u[i];
    }
    return acc ? 32 - __builtin_clz(acc) : 0;
}

/* The predictor of one block in `mode` and its width. */
static int block_choice(const int32_t *q, int mode, uint32_t *u, int *pred)
{
    int best = block_residuals(q, 0, u), bp = 0;
    if (mode == 1) {
        for (int p = 1; p <= 2; ++p) {
            int w = block_residuals(q, p, u);
            if (w < best) { best = w; bp = p; }
        }
        block_residuals(q, bp, u);
    }
    *pred = bp;
    return best;
}

static int block_codes(int dtype, const void *in, size_t b, double inv_step, int32_t *q)
{
    size_t j = b / 2, p = b % 2;
    for (int i = 0; i < 64; ++i) {
        size_t comp = 2 * (64 * j + (size_t)i) + p;
        double x = dtype == 0 ? ((const double *)in)[comp]
                              : (double)((const float *)in)[comp];
        if (orc_quantize(x, inv_step, &q[i]) != ORC_OK) return ORC_E_RANGE;
    }
    return ORC_OK;
}

/*
 * Encode one chunk in predictor mode `mode` (0 or 1). dtype 0: in is
 * double[2C]; dtype 1: float[2C]. Writes at most cap bytes to out and the
 * encoded size to *out_bytes.
 */
int orc_codec_encode_mode(int dtype, int log2c, double eb, int mode, const void *in,
                          void *out, size_t cap, size_t *out_bytes)
{
    if ((dtype != 0 && dtype != 1) || log2c < 6 || log2c > 40 || !(eb > 0.0) || !isfinite(eb) ||
        (mode != 0 && mode != 1))
        return ORC_E_ARG;
    const double inv_step = 1.0 / (2.0 * eb);
    const size_t C = (size_t)1 << log2c;
    const size_t nb = 2 * C / 64;
    const size_t w_off = 32, a_off = 32 + pad8(nb), p_off = a_off + pad8(4 * nb);
    uint8_t *o = (uint8_t *)out;
    if (cap < 32) return ORC_E_ARG;

    /* first sweep: codes, anchors, widths */
    int all_zero = 1;
    size_t words = 0;
    for (size_t b = 0; b < nb; ++b) {
        int32_t q[64];
        uint32_t u[64];
        int pred;
        if (block_codes(dtype, in, b, inv_step, q) != ORC_OK) return ORC_E_RANGE;
        int w = block_choice(q, mode, u, &pred);
        if (w || q[0]) all_zero = 0;
        words += (size_t)w;
    }
    size_t total = all_zero ? 32 : p_off + 8 * words;
    if (total > cap) return ORC_E_ARG;
    memset(o, 0, all_zero ? 32 : p_off);
    put_u32(o + 0, ORC_MAGIC);
    o[4] = 1;
    o[5] = all_zero ? 0 : 1;
    o[6] = (uint8_t)log2c;
    o[7] = (uint8_t)dtype;
    memcpy(o + 8, &eb, 8);
    put_u64(o + 16, (uint64_t)total);
    put_u32(o + 24, (uint32_t)nb);
    put_u32(o + 28, (uint32_t)mode);
    *out_bytes = total;
    if (all_zero) return ORC_OK;

    /* second sweep: write W, A and the bit planes */
    size_t wpos = 0;
    for (size_t b = 0; b < nb; ++b) {
        int32_t q[64];
        uint32_t u[64];
        int pred;
        block_codes(dtype, in, b, inv_step, q);
        int w = block_choice(q, mode, u, &pred);
        o[w_off + b] = (uint8_t)(w | (pred << 6));
        memcpy(o + a_off + 4 * b, &q[0], 4);
        for (int k = 0; k < w; ++k) {
            uint64_t word = 0;
            for (int i = 0; i < 64; ++i)
                word |= (uint64_t)((u[i] >> k) & 1u) << i;
            put_u64(o + p_off + 8 * (wpos + (size_t)k), word);
        }
        wpos += (size_t)w;
    }
    return ORC_OK;
}

/* Mode 0 (Lorenzo-1 for every block). */
int orc_codec_encode(int dtype, int log2c, double eb, const void *in,
                     void *out, size_t cap, size_t *out_bytes)
{
    return orc_codec_encode_mode(dtype, log2c, eb, 0, in, out, cap, out_bytes);
}

/* Read the header fields of an encoded chunk; returns 0 or ORC_E_CORRUPT. */
int orc_codec_header(const void *in, size_t in_bytes, int *dtype, int *log2c,
                     int *kind, double *eb, uint64_t *total)
{
    const uint8_t *p = (const uint8_t *)in;
    if (in_bytes < 32 || get_u32(p) != ORC_MAGIC || p[4] != 1 || p[5] > 1 || p[7] > 1)
        return ORC_E_CORRUPT;
    int c = p[6];
    if (c < 6 || c > 40) return ORC_E_CORRUPT;
    uint64_t nb = ((uint64_t)2 << c) / 64;
    if (get_u32(p + 24) != (uint32_t)nb || get_u32(p + 28) > 1) return ORC_E_CORRUPT;
    double e;
    memcpy(&e, p + 8, 8);
    if (!(e > 0.0) || !isfinite(e)) return ORC_E_CORRUPT;
    uint64_t t = get_u64(p + 16);
    if (t > in_bytes) return ORC_E_CORRUPT;
    if (p[5] == 0 && t != 32) return ORC_E_CORRUPT;
    *dtype = p[7]; *log2c = c; *kind = p[5]; *eb = e; *total = t;
    return ORC_OK;
}

/* Decode one chunk into out (double[2C] or float[2C] by the header's dtype). */
int orc_codec_decode(const void *in, size_t in_bytes, void *out)
{
    int dtype, log2c, kind;
    double eb;
    uint64_t total;
    int st = orc_codec_header(in, in_bytes, &dtype, &log2c, &kind, &eb, &total);
    if (st) return st;
    const uint8_t *p = (const uint8_t *)in;
    const size_t C = (size_t)1 << log2c, nb = 2 * C / 64;
    const double step = 2.0 * eb;
    if (kind == 0) {
        if (dtype == 0) memset(out, 0, 2 * C * sizeof(double));
        else memset(out, 0, 2 * C * sizeof(float));
        return ORC_OK;
    }
    const size_t w_off = 32, a_off = 32 + pad8(nb), p_off = a_off + pad8(4 * nb);
    if (total < p_off) return ORC_E_CORRUPT;
    const int mode = (int)get_u32(p + 28);
    size_t words = 0;
    for (size_t b = 0; b < nb; ++b) {
        int w = p[w_off + b] & 63, pred = p[w_off + b] >> 6;
        if (w > 32 || pred > (mode == 1 ? 2 : 0)) return ORC_E_CORRUPT;
        words += (size_t)w;
    }
    if (p_off + 8 * words != total) return ORC_E_CORRUPT;
    size_t wpos = 0;
    for (size_t b = 0; b < nb; ++b) {
        size_t j = b / 2, pl = b % 2;
        int w = p[w_off + b] & 63, pred = p[w_off + b] >> 6;
        int32_t a;
        memcpy(&a, p + a_off + 4 * b, 4);
        uint32_t q = (uint32_t)a, e = 0;
        for (int i = 0; i < 64; ++i) {
            uint32_t u = 0;
            for (int k = 0; k < w; ++k) {
                uint64_t word = get_u64(p + p_off + 8 * (wpos + (size_t)k));
                u |= (uint32_t)((word >> i) & 1u) << k;
            }
            uint32_t d = (u >> 1) ^ (0u - (u & 1u));
            if (i > 0) {
                if (pred == 0) q += d;
                else if (pred == 1) q = d;
                else { e += d; q += e; }
            }
            double x = (double)(int32_t)q * step;
            size_t comp = 2 * (64 * j + (size_t)i) + pl;
            if (dtype == 0) ((double *)out)[comp] = x;
            else ((float *)out)[comp] = (float)x;
        }
        wpos += (size_t)w;
    }
    return ORC_OK;
}
