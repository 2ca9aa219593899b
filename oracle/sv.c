/*
 * Oracle: plain FP64 state-vector simulator on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.
 *
 * What it computes is the plain definition of state-vector simulation that the
 * compressed method reproduces when its error bound is zero (paper, Sec. 2,
 * "Online stage": every stage updates all 2^n amplitudes): the state
 * psi in C^(2^n) starts at a basis state and each gate, in list order, maps
 *
 *   psi'[base | sum_m s'_m 2^q_m] = sum_s U[s', s] psi[base | sum_m s_m 2^q_m]
 *
 * with little-endian qubits (index i = sum_q b_q 2^q) and the sub-index of a
 * two-qubit gate on (q0, q1) being s = b(q0) + 2 b(q1). No fusion, no
 * blocking, no special cases: every gate is a dense 2x2 or 4x4 complex matrix
 * applied to every amplitude group.
 *
 * Gate matrices (standard definitions):
 *   H = [[1,1],[1,-1]]/sqrt2, X, Y = [[0,-i],[i,0]], Z = diag(1,-1),
 *   S = diag(1,i), T = diag(1,e^{i pi/4}), RX(t) = exp(-i t X/2),
 *   RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2), P(l) = diag(1, e^{il}),
 *   CX (control q0, target q1), CZ = diag(1,1,1,-1), CP(l) = diag(1,1,1,e^{il}),
 *   SWAP, U1 / U2 = caller-given 2x2 / 4x4.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

enum {
    ORC_H = 0, ORC_X, ORC_Y, ORC_Z, ORC_S, ORC_T, ORC_RX, ORC_RY, ORC_RZ, ORC_P,
    ORC_CX, ORC_CZ, ORC_CP, ORC_SWAP, ORC_U1, ORC_U2
};

typedef struct {
    int32_t kind, q0, q1, pad;
    double theta;
    const double *mat; /* U1 / U2: row-major, interleaved (re, im) */
} orc_gate;

/* Fill U (row-major, interleaved re/im) for gate g; return its qubit count, or
 * 0 for an unknown kind. */
static int gate_matrix(const orc_gate *g, double U[32])
{
    memset(U, 0, 32 * sizeof(double));
#define SET(r, c, re, im) do { U[2 * ((r) * d + (c))] = (re); U[2 * ((r) * d + (c)) + 1] = (im); } while (0)
    int d = 2;
    const double h = 1.0 / sqrt(2.0);
    const double c = cos(g->theta / 2.0), s = sin(g->theta / 2.0);
    switch (g->kind) {
    case ORC_H: SET(0, 0, h, 0); SET(0, 1, h, 0); SET(1, 0, h, 0); SET(1, 1, -h, 0); return 1;
    case ORC_X: SET(0, 1, 1, 0); SET(1, 0, 1, 0); return 1;
    case ORC_Y: SET(0, 1, 0, -1); SET(1, 0, 0, 1); return 1;
    case ORC_Z: SET(0, 0, 1, 0); SET(1, 1, -1, 0); return 1;
    case ORC_S: SET(0, 0, 1, 0); SET(1, 1, 0, 1); return 1;
    case ORC_T: SET(0, 0, 1, 0); SET(1, 1, cos(M_PI / 4), sin(M_PI / 4)); return 1;
    /* exp(-i t X/2) = cos(t/2) I - i sin(t/2) X */
    case ORC_RX: SET(0, 0, c, 0); SET(0, 1, 0, -s); SET(1, 0, 0, -s); SET(1, 1, c, 0); return 1;
    /* exp(-i t Y/2) = cos(t/2) I - i sin(t/2) Y */
    case ORC_RY: SET(0, 0, c, 0); SET(0, 1, -s, 0); SET(1, 0, s, 0); SET(1, 1, c, 0); return 1;
    /* exp(-i t Z/2) = diag(e^{-it/2}, e^{it/2}) */
    case ORC_RZ: SET(0, 0, c, -s); SET(1, 1, c, s); return 1;
    case ORC_P: SET(0, 0, 1, 0); SET(1, 1, cos(g->theta), sin(g->theta)); return 1;
    case ORC_U1:
        for (int i = 0; i < 8; ++i) U[i] = g->mat[i];
        return 1;
    default: break;
    }
    d = 4;
    switch (g->kind) {
    case ORC_CX: /* s = b(q0) + 2 b(q1); flip q1 when q0 = 1: s=1 <-> s=3 */
        SET(0, 0, 1, 0); SET(2, 2, 1, 0); SET(1, 3, 1, 0); SET(3, 1, 1, 0); return 2;
    case ORC_CZ: SET(0, 0, 1, 0); SET(1, 1, 1, 0); SET(2, 2, 1, 0); SET(3, 3, -1, 0); return 2;
    case ORC_CP:
        SET(0, 0, 1, 0); SET(1, 1, 1, 0); SET(2, 2, 1, 0);
        SET(3, 3, cos(g->theta), sin(g->theta)); return 2;
    case ORC_SWAP: SET(0, 0, 1, 0); SET(1, 2, 1, 0); SET(2, 1, 1, 0); SET(3, 3, 1, 0); return 2;
    case ORC_U2:
        for (int i = 0; i < 32; ++i) U[i] = g->mat[i];
        return 2;
    default: break;
    }
#undef SET
    return 0;
}

/* Export the matrix the oracle uses for one gate (for tests). */
int orc_gate_matrix(const orc_gate *g, double *out32)
{
    return gate_matrix(g, out32);
}

/* Insert a zero bit at position p of x. */
static inline uint64_t insert_zero(uint64_t x, int p)
{
    uint64_t lo = x & ((1ull << p) - 1);
    return ((x >> p) << (p + 1)) | lo;
}

/* Apply a gate list to psi (2^n complex doubles, interleaved). Returns 0, or -1
 * for a bad gate (unknown kind, qubit out of range, repeated qubit). */
int orc_apply(int n, double *psi, const orc_gate *gates, size_t n_gates)
{
    for (size_t gi = 0; gi < n_gates; ++gi) {
        const orc_gate *g = &gates[gi];
        double U[32];
        int k = gate_matrix(g, U);
        if (k == 0) return -1;
        int q[2] = {g->q0, g->q1};
        for (int m = 0; m < k; ++m)
            if (q[m] < 0 || q[m] >= n) return -1;
        if (k == 2 && q[0] == q[1]) return -1;
        const int d = 1 << k;
        int lo = q[0], hi = q[0];
        if (k == 2) { lo = q[0] < q[1] ? q[0] : q[1]; hi = q[0] < q[1] ? q[1] : q[0]; }
        const int64_t n_groups = (int64_t)1 << (n - k);
        #pragma omp parallel for schedule(static)
        for (int64_t grp = 0; grp < n_groups; ++grp) {
            uint64_t base = insert_zero((uint64_t)grp, lo);
            if (k == 2) base = insert_zero(base, hi);
            uint64_t idx[4];
            double vr[4], vi[4];
            for (int s = 0; s < d; ++s) {
                uint64_t i = base;
                for (int m = 0; m < k; ++m)
                    if ((s >> m) & 1) i |= 1ull << q[m];
                idx[s] = i;
                vr[s] = psi[2 * i];
                vi[s] = psi[2 * i + 1];
            }
            for (int r = 0; r < d; ++r) {
                double accr = 0.0, acci = 0.0;
                for (int s = 0; s < d; ++s) {
                    double ur = U[2 * (r * d + s)], ui = U[2 * (r * d + s) + 1];
                    accr += ur * vr[s] - ui * vi[s];
                    acci += ur * vi[s] + ui * vr[s];
                }
                psi[2 * idx[r]] = accr;
                psi[2 * idx[r] + 1] = acci;
            }
        }
    }
    return 0;
}

/* psi = |x> */
void orc_init_basis(int n, double *psi, uint64_t x)
{
    const int64_t N = (int64_t)1 << n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) { psi[2 * i] = 0.0; psi[2 * i + 1] = 0.0; }
    psi[2 * x] = 1.0;
}

/* <psi| sum_k c_k Z(m_k) |psi> = sum_i |psi_i|^2 sum_k c_k (-1)^popcount(i & m_k) */
double orc_expect_z(int n, const double *psi, const uint64_t *masks,
                    const double *coeffs, size_t n_terms)
{
    const int64_t N = (int64_t)1 << n;
    double total = 0.0;
    #pragma omp parallel for reduction(+ : total) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        double v = 0.0;
        for (size_t k = 0; k < n_terms; ++k)
            v += (__builtin_popcountll((uint64_t)i & masks[k]) & 1) ? -coeffs[k] : coeffs[k];
        total += p * v;
    }
    return total;
}
