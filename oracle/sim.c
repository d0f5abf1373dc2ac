/*
 * Oracle state-vector simulator: plain, slow, obviously correct.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The product path
 * never links or calls it, and it shares no code with the device path.
 *
 * Conventions (paper, Section 2): qubit q is bit q of the basis index,
 * i = sum_q i_q 2^q.  A state of n qubits is 2^n complex128 amplitudes stored as
 * interleaved (re, im) doubles.  Every operation below is written directly from
 * its definition, one amplitude pair at a time, with no blocking or fusion.
 *
 * Gate semantics (paper, Section 2: arbitrary one-qubit gates and controlled
 * one-qubit gates, which update amplitudes in pairs):
 *   U(t):      for every index i with bit t = 0 and j = i | 2^t,
 *              (a_i, a_j) <- (u00 a_i + u01 a_j, u10 a_i + u11 a_j)
 *   CU(c, t):  the same update restricted to indices with bit c = 1
 *   CX(c, t):  CU with U = X, i.e. a_i <-> a_j where bit c = 1
 *   CZ(a, b):  a_i <- -a_i where bits a and b are both 1
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t kind, q0, q1, pad;
    double u[8];
} orc_gate;

enum { ORC_U = 0, ORC_CX = 1, ORC_CZ = 2, ORC_CU = 3 };

/* (a, b) <- (m00 a + m01 b, m10 a + m11 b) with complex arithmetic spelled out */
static void pair_update(double *s, uint64_t i, uint64_t j, const double *m)
{
    double ar = s[2 * i], ai = s[2 * i + 1];
    double br = s[2 * j], bi = s[2 * j + 1];
    s[2 * i]     = m[0] * ar - m[1] * ai + m[2] * br - m[3] * bi;
    s[2 * i + 1] = m[0] * ai + m[1] * ar + m[2] * bi + m[3] * br;
    s[2 * j]     = m[4] * ar - m[5] * ai + m[6] * br - m[7] * bi;
    s[2 * j + 1] = m[4] * ai + m[5] * ar + m[6] * bi + m[7] * br;
}

void orc_apply_u(double *s, int n, int t, const double *m)
{
    const uint64_t N = 1ull << n, tb = 1ull << t;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i)
        if (!(i & tb))
            pair_update(s, i, i | tb, m);
}

void orc_apply_cu(double *s, int n, int c, int t, const double *m)
{
    const uint64_t N = 1ull << n, tb = 1ull << t, cb = 1ull << c;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i)
        if ((i & cb) && !(i & tb))
            pair_update(s, i, i | tb, m);
}

void orc_apply_cx(double *s, int n, int c, int t)
{
    const uint64_t N = 1ull << n, tb = 1ull << t, cb = 1ull << c;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i)
        if ((i & cb) && !(i & tb)) {
            uint64_t j = i | tb;
            double r = s[2 * i], im = s[2 * i + 1];
            s[2 * i] = s[2 * j];
            s[2 * i + 1] = s[2 * j + 1];
            s[2 * j] = r;
            s[2 * j + 1] = im;
        }
}

void orc_apply_cz(double *s, int n, int a, int b)
{
    const uint64_t N = 1ull << n, ab = 1ull << a, bb = 1ull << b;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i)
        if ((i & ab) && (i & bb)) {
            s[2 * i] = -s[2 * i];
            s[2 * i + 1] = -s[2 * i + 1];
        }
}

/* Apply one gate record with its qubits read as bit positions p0, p1. */
int orc_apply_gate(double *s, int n, int kind, int p0, int p1, const double *m)
{
    switch (kind) {
    case ORC_U:  orc_apply_u(s, n, p0, m); return 0;
    case ORC_CX: orc_apply_cx(s, n, p0, p1); return 0;
    case ORC_CZ: orc_apply_cz(s, n, p0, p1); return 0;
    case ORC_CU: orc_apply_cu(s, n, p0, p1, m); return 0;
    }
    return -1;
}

/* Run gates g[0..ng) in program order on logical state s. */
int orc_run(double *s, int n, const orc_gate *g, int64_t ng)
{
    for (int64_t k = 0; k < ng; ++k)
        if (orc_apply_gate(s, n, g[k].kind, g[k].q0, g[k].q1, g[k].u))
            return -1;
    return 0;
}

void orc_set_basis(double *s, int n, uint64_t x)
{
    memset(s, 0, sizeof(double) * 2 * (1ull << n));
    s[2 * x] = 1.0;
}

#define ORC_BLOCK 4096ull

/* Sum of f(i) over all 2^n indices taken as fixed 4096-term block sums (each
 * in index order) added in block order, so the value is independent of the
 * number of threads. */
static double block_sum(const double *s, int n, uint64_t qb, int signed_by_bit)
{
    const uint64_t N = 1ull << n, nb = (N + ORC_BLOCK - 1) / ORC_BLOCK;
    double *part = (double *)malloc(sizeof(double) * nb);
    if (!part)
        return NAN;
#pragma omp parallel for schedule(static)
    for (uint64_t b = 0; b < nb; ++b) {
        double acc = 0.0;
        uint64_t e = (b + 1) * ORC_BLOCK < N ? (b + 1) * ORC_BLOCK : N;
        for (uint64_t i = b * ORC_BLOCK; i < e; ++i) {
            double p = s[2 * i] * s[2 * i] + s[2 * i + 1] * s[2 * i + 1];
            acc += (signed_by_bit && (i & qb)) ? -p : p;
        }
        part[b] = acc;
    }
    double total = 0.0;
    for (uint64_t b = 0; b < nb; ++b)
        total += part[b];
    free(part);
    return total;
}

double orc_norm(const double *s, int n)
{
    return block_sum(s, n, 0, 0);
}

/* <Z_q> = sum_i |a_i|^2 (1 - 2 i_q) for every qubit q. */
void orc_expect_z(const double *s, int n, double *out)
{
    for (int q = 0; q < n; ++q)
        out[q] = block_sum(s, n, 1ull << q, 1);
}

/* Physical index of logical basis index i under qubit placement sigma:
 * j(i, sigma) = sum_q i_q 2^{sigma(q)} (paper, Section 2). */
uint64_t orc_index_map(uint64_t i, int n, const int *sigma)
{
    uint64_t j = 0;
    for (int q = 0; q < n; ++q)
        if ((i >> q) & 1)
            j |= 1ull << sigma[q];
    return j;
}

/* dst[j(i, sigma_to)] = src[j(i, sigma_from)] for every logical i: the data
 * movement of PermuteQubits from placement sigma_from to sigma_to. */
void orc_permute(const double *src, double *dst, int n, const int *sigma_from, const int *sigma_to)
{
    const uint64_t N = 1ull << n;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t a = orc_index_map(i, n, sigma_from), b = orc_index_map(i, n, sigma_to);
        dst[2 * b] = src[2 * a];
        dst[2 * b + 1] = src[2 * a + 1];
    }
}

/* OpenMP threads the loops above run with. */
int orc_threads(void)
{
    return omp_get_max_threads();
}

/* Run the loops above with n threads (n >= 1). */
void orc_set_threads(int n)
{
    if (n >= 1)
        omp_set_num_threads(n);
}
