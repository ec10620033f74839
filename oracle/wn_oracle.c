/*
 * FP64 CPU oracle for the generalized winding number of a triangle mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg load it; the GPU library never does, and
 * the two share no code, headers, tables or helpers.
 *
 * Paper: "Differentiable Voxelization and Mesh Morphing" (arXiv 2407.11272).
 *   - Section 2.1, Eq. 2: W(q, S) = 1/(4 pi) * flux of (x - q)/|x - q|^3 through S.
 *   - Section 2.2, Eq. 5: W(q) = 1/(4 pi) * sum over faces of the solid angle.
 *   - Section 2.2, Eq. 7: triangle solid angle from the unit vectors e_j = (v_j - q)/|v_j - q|,
 *       det(e0, e1, e2) over 1 + e0.e1 + e1.e2 + e2.e0.
 *   - Section 2.2, Eq. 8: the ATAN2 case table, including ATAN2(0, 0) = 0.
 *   - Algorithm 1: per face, normalise, form alpha and beta, accumulate ATAN2(alpha, beta).
 *
 * Readings (where the paper is silent or garbled):
 *   - The half-angle identity: tan(Omega / 2) = det / (1 + sum of dots) for unit vectors,
 *     so Omega = 2 * ATAN2(alpha, beta) and W = sum ATAN2(alpha, beta) / (2 pi).
 *     Eq. 7 as printed lacks the factor 2; the octant pin (Omega = 4 pi / 8) fixes it.
 *   - A vertex that coincides with q has no direction: its unit vector is taken as 0, so
 *     alpha = 0 and the face contributes ATAN2(0, beta >= 0) = 0.
 *   - Eq. 8 is applied literally: y = -0 counts as y >= 0, and x = 0, y = 0 gives 0
 *     whatever the signs of the zeros.
 *   - The gradient is not given in the paper.  It is the chain rule through
 *     Omega = 2 ATAN2(alpha, beta) and e_j = R_j / |R_j|; at alpha = beta = 0 (q on an
 *     edge) the face contributes 0.
 *
 * Summation: every sum over faces (or points, for the gradient) is Neumaier-compensated
 * in FP64.  Parallelism: OpenMP over independent outputs only; every output's own sum
 * runs in index order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- helpers --- */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int wno_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ Eq. 8 --- */

/* ATAN2(y, x) exactly as the case table of Section 2.2, Eq. 8. */
double wno_atan2_eq8(double y, double x)
{
    if (x > 0) return atan(y / x);
    if (x < 0) {
        if (y >= 0) return atan(y / x) + M_PI;
        return atan(y / x) - M_PI;
    }
    /* x == 0 (either sign of zero) */
    if (y > 0) return M_PI / 2;
    if (y < 0) return -M_PI / 2;
    return 0.0;
}

/* ------------------------------------------------------------------ Eq. 7 --- */

/* alpha = det(e0, e1, e2) and beta = 1 + e0.e1 + e1.e2 + e2.e0 for one face seen from q. */
void wno_alpha_beta(const double *v0, const double *v1, const double *v2, const double *q,
                    double *alpha, double *beta)
{
    const double *v[3] = {v0, v1, v2};
    double e[3][3];
    for (int j = 0; j < 3; ++j) {
        double r[3] = {v[j][0] - q[0], v[j][1] - q[1], v[j][2] - q[2]};
        double len = sqrt(dot3(r, r));
        for (int c = 0; c < 3; ++c) e[j][c] = len > 0 ? r[c] / len : 0.0;
    }
    double x12[3];
    cross3(e[1], e[2], x12);
    *alpha = dot3(e[0], x12);
    *beta = 1.0 + dot3(e[0], e[1]) + dot3(e[1], e[2]) + dot3(e[2], e[0]);
}

/* Solid angle Omega of one triangle at q: 2 * ATAN2(alpha, beta). */
double wno_solid_angle(const double *v0, const double *v1, const double *v2, const double *q)
{
    double a, b;
    wno_alpha_beta(v0, v1, v2, q, &a, &b);
    return 2.0 * wno_atan2_eq8(a, b);
}

/* ------------------------------------------------------------------ Eq. 5 --- */

/*
 * W[i] = 1/(4 pi) * sum_f Omega_f(Q[i]) for every query point.
 * V: [nV][3], F: [nF][3] (indices into V), Q: [nQ][3], W: [nQ].
 * Returns 0, or -1 if a face index is out of range (W is then unspecified).
 */
int wno_winding(const double *V, int64_t nV, const int64_t *F, int64_t nF,
                const double *Q, int64_t nQ, double *W, int nthreads)
{
    for (int64_t f = 0; f < 3 * nF; ++f)
        if (F[f] < 0 || F[f] >= nV) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nQ; ++i) {
        const double *q = Q + 3 * i;
        nsum s = {0.0, 0.0};
        for (int64_t f = 0; f < nF; ++f) {
            double a, b;
            wno_alpha_beta(V + 3 * F[3 * f], V + 3 * F[3 * f + 1], V + 3 * F[3 * f + 2], q, &a, &b);
            nsum_add(&s, 2.0 * wno_atan2_eq8(a, b));
        }
        W[i] = nsum_get(&s) / (4.0 * M_PI);
    }
    return 0;
}

/* Voxel centres lo + (idx + 1/2) (hi - lo) / n, flat index (i n1 + j) n2 + k (z fastest). */
void wno_grid_points(const double *lo, const double *hi, const int64_t *n, double *Q)
{
    for (int64_t i = 0; i < n[0]; ++i)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t k = 0; k < n[2]; ++k) {
                int64_t idx = (i * n[1] + j) * n[2] + k;
                int64_t ijk[3] = {i, j, k};
                for (int d = 0; d < 3; ++d)
                    Q[3 * idx + d] = lo[d] + ((double)ijk[d] + 0.5) * (hi[d] - lo[d]) / (double)n[d];
            }
}

/* ------------------------------------------------------------- gradient ---- */

/*
 * dOmega/dv_j for one face (out[3 j + c]).  With alpha = e0.(e1 x e2) and
 * beta = 1 + sum of pairwise dots:
 *   dOmega = 2 (beta dalpha - alpha dbeta) / (alpha^2 + beta^2)
 *   dalpha/de_j = e_k x e_l (j, k, l cyclic),  dbeta/de_j = e_k + e_l
 *   de_j/dv_j  = (I - e_j e_j^T) / |R_j|
 * A vertex at q (|R_j| = 0) or alpha = beta = 0 gives 0.
 */
void wno_solid_angle_grad(const double *v0, const double *v1, const double *v2, const double *q,
                          double *out)
{
    const double *v[3] = {v0, v1, v2};
    double e[3][3], len[3];
    memset(out, 0, 9 * sizeof(double));
    for (int j = 0; j < 3; ++j) {
        double r[3] = {v[j][0] - q[0], v[j][1] - q[1], v[j][2] - q[2]};
        len[j] = sqrt(dot3(r, r));
        for (int c = 0; c < 3; ++c) e[j][c] = len[j] > 0 ? r[c] / len[j] : 0.0;
    }
    double x12[3];
    cross3(e[1], e[2], x12);
    double alpha = dot3(e[0], x12);
    double beta = 1.0 + dot3(e[0], e[1]) + dot3(e[1], e[2]) + dot3(e[2], e[0]);
    double den = alpha * alpha + beta * beta;
    if (den == 0.0) return;
    for (int j = 0; j < 3; ++j) {
        if (len[j] == 0.0) continue;
        int k = (j + 1) % 3, l = (j + 2) % 3;
        double u[3], g[3];
        cross3(e[k], e[l], u);
        for (int c = 0; c < 3; ++c) g[c] = 2.0 * (beta * u[c] - alpha * (e[k][c] + e[l][c])) / den;
        /* project out the radial component and divide by |R_j| */
        double ge = dot3(g, e[j]);
        for (int c = 0; c < 3; ++c) out[3 * j + c] = (g[c] - ge * e[j][c]) / len[j];
    }
}

/*
 * Adjoint of Eq. 5 for given dL/dW at every query point:
 *   dLdT[f][j][c] = sum_i dLdW[i] * (1/(4 pi)) dOmega_f(Q[i]) / dv_{F[f][j]}[c]
 *   dLdV[v][c]    = sum of dLdT over the corners (f, j) with F[f][j] = v, in face order.
 * dLdT ([nF][9]) or dLdV ([nV][3]) may be NULL.  Returns 0, or -1 on a bad index.
 */
int wno_grad(const double *V, int64_t nV, const int64_t *F, int64_t nF,
             const double *Q, int64_t nQ, const double *dLdW, double *dLdT, double *dLdV, int nthreads)
{
    for (int64_t f = 0; f < 3 * nF; ++f)
        if (F[f] < 0 || F[f] >= nV) return -1;
    set_threads(nthreads);
    double *T = dLdT;
    double *own = NULL;
    if (!T) {
        own = (double *)calloc((size_t)(nF > 0 ? nF : 1) * 9, sizeof(double));
        if (!own) return -2;
        T = own;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t f = 0; f < nF; ++f) {
        nsum s[9];
        for (int c = 0; c < 9; ++c) s[c].s = s[c].c = 0.0;
        const double *a = V + 3 * F[3 * f], *b = V + 3 * F[3 * f + 1], *d = V + 3 * F[3 * f + 2];
        for (int64_t i = 0; i < nQ; ++i) {
            double g[9];
            wno_solid_angle_grad(a, b, d, Q + 3 * i, g);
            for (int c = 0; c < 9; ++c) nsum_add(&s[c], dLdW[i] * g[c]);
        }
        for (int c = 0; c < 9; ++c) T[9 * f + c] = nsum_get(&s[c]) / (4.0 * M_PI);
    }
    if (dLdV) {
        nsum *acc = (nsum *)calloc((size_t)(nV > 0 ? nV : 1) * 3, sizeof(nsum));
        if (!acc) { free(own); return -2; }
        for (int64_t f = 0; f < nF; ++f)
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 3; ++c) nsum_add(&acc[3 * F[3 * f + j] + c], T[9 * f + 3 * j + c]);
        for (int64_t x = 0; x < 3 * nV; ++x) dLdV[x] = nsum_get(&acc[x]);
        free(acc);
    }
    free(own);
    return 0;
}

/* --------------------------------------------------- naive integral (Eq. 4) --- */

/*
 * Section 2.1, Eq. 4: the naive discretisation of the flux integral, one sample per
 * face at its centroid c_i with the area-weighted normal n_i Delta_i = N_i / 2,
 * N_i = (v1 - v0) x (v2 - v0):
 *   W(q) ~= 1/(4 pi) sum_i <n_i, (c_i - q)/|c_i - q|^3> Delta_i
 *        = 1/(8 pi) sum_i <N_i, c_i - q> / |c_i - q|^3.
 * A face whose centroid coincides with q contributes 0 (reading: the sample is
 * undefined there).  `S` (optional) receives 1/(8 pi) sum_i |term_i|, the scale of
 * the rounding error of any evaluation of this sum.
 */
static double naive_term(const double *a, const double *b, const double *c, const double *q)
{
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double N[3], r[3];
    cross3(e1, e2, N);
    for (int d = 0; d < 3; ++d) r[d] = (a[d] + b[d] + c[d]) / 3.0 - q[d];
    double r2 = dot3(r, r);
    if (r2 == 0.0) return 0.0;
    return dot3(N, r) / (r2 * sqrt(r2));
}

int wno_winding_naive(const double *V, int64_t nV, const int64_t *F, int64_t nF,
                      const double *Q, int64_t nQ, double *W, double *S, int nthreads)
{
    for (int64_t f = 0; f < 3 * nF; ++f)
        if (F[f] < 0 || F[f] >= nV) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nQ; ++i) {
        nsum s = {0.0, 0.0}, sa = {0.0, 0.0};
        for (int64_t f = 0; f < nF; ++f) {
            double t = naive_term(V + 3 * F[3 * f], V + 3 * F[3 * f + 1], V + 3 * F[3 * f + 2], Q + 3 * i);
            nsum_add(&s, t);
            nsum_add(&sa, fabs(t));
        }
        W[i] = nsum_get(&s) / (8.0 * M_PI);
        if (S) S[i] = nsum_get(&sa) / (8.0 * M_PI);
    }
    return 0;
}

/*
 * Gradient of one naive term g = <N, r> / |r|^3 (r = c - q, c the centroid) with
 * respect to v_j: dc/dv_j = I/3 and d<a, N>/dv_j = (v_{j+1} - v_{j+2}) x a, so
 *   dg/dv_j = (N/|r|^3 - 3 <N, r> r/|r|^5) / 3 + (v_{j+1} - v_{j+2}) x r/|r|^3.
 */
void wno_naive_term_grad(const double *v0, const double *v1, const double *v2, const double *q, double *out)
{
    const double *v[3] = {v0, v1, v2};
    double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    double N[3], r[3];
    cross3(e1, e2, N);
    for (int d = 0; d < 3; ++d) r[d] = (v0[d] + v1[d] + v2[d]) / 3.0 - q[d];
    memset(out, 0, 9 * sizeof(double));
    double r2 = dot3(r, r);
    if (r2 == 0.0) return;
    double ir3 = 1.0 / (r2 * sqrt(r2));
    double nr = dot3(N, r);
    double a[3];
    for (int d = 0; d < 3; ++d) a[d] = r[d] * ir3;
    for (int j = 0; j < 3; ++j) {
        const double *p = v[(j + 1) % 3], *m = v[(j + 2) % 3];
        double e[3] = {p[0] - m[0], p[1] - m[1], p[2] - m[2]}, x[3];
        cross3(e, a, x);
        for (int d = 0; d < 3; ++d) out[3 * j + d] = (N[d] * ir3 - 3.0 * nr * r[d] * ir3 / r2) / 3.0 + x[d];
    }
}

/* Adjoint of wno_winding_naive: dLdT[f][j][c] = sum_i dLdW[i] dW_i/dv_{F[f][j]}[c] and
 * its per-vertex gather (face order).  Either output may be NULL. */
int wno_grad_naive(const double *V, int64_t nV, const int64_t *F, int64_t nF,
                   const double *Q, int64_t nQ, const double *dLdW, double *dLdT, double *dLdV, int nthreads)
{
    for (int64_t f = 0; f < 3 * nF; ++f)
        if (F[f] < 0 || F[f] >= nV) return -1;
    set_threads(nthreads);
    double *T = dLdT;
    double *own = NULL;
    if (!T) {
        own = (double *)calloc((size_t)(nF > 0 ? nF : 1) * 9, sizeof(double));
        if (!own) return -2;
        T = own;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t f = 0; f < nF; ++f) {
        nsum s[9];
        for (int c = 0; c < 9; ++c) s[c].s = s[c].c = 0.0;
        for (int64_t i = 0; i < nQ; ++i) {
            double g[9];
            wno_naive_term_grad(V + 3 * F[3 * f], V + 3 * F[3 * f + 1], V + 3 * F[3 * f + 2], Q + 3 * i, g);
            for (int c = 0; c < 9; ++c) nsum_add(&s[c], dLdW[i] * g[c]);
        }
        for (int c = 0; c < 9; ++c) T[9 * f + c] = nsum_get(&s[c]) / (8.0 * M_PI);
    }
    if (dLdV) {
        nsum *acc = (nsum *)calloc((size_t)(nV > 0 ? nV : 1) * 3, sizeof(nsum));
        if (!acc) { free(own); return -2; }
        for (int64_t f = 0; f < nF; ++f)
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 3; ++c) nsum_add(&acc[3 * F[3 * f + j] + c], T[9 * f + 3 * j + c]);
        for (int64_t x = 0; x < 3 * nV; ++x) dLdV[x] = nsum_get(&acc[x]);
        free(acc);
    }
    free(own);
    return 0;
}

/* ------------------------------------------------------- guard-band distances */

/* Distance from p to the segment [a, b] (a vertex when a == b). */
static double seg_dist(const double *p, const double *a, const double *b)
{
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double L = dot3(ab, ab);
    double t = L > 0 ? dot3(ap, ab) / L : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double d[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
    return sqrt(dot3(d, d));
}

/* Distance from p to the closed triangle (a, b, c): plane distance if the projection
 * falls inside (barycentric test), otherwise the nearest edge. */
static double tri_dist(const double *p, const double *a, const double *b, const double *c)
{
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double n[3];
    cross3(ab, ac, n);
    double nn = dot3(n, n);
    if (nn > 0) {
        double t = dot3(ap, n) / nn;
        double x[3] = {ap[0] - t * n[0], ap[1] - t * n[1], ap[2] - t * n[2]}; /* in-plane offset from a */
        double d00 = dot3(ab, ab), d01 = dot3(ab, ac), d11 = dot3(ac, ac);
        double d20 = dot3(x, ab), d21 = dot3(x, ac);
        double den = d00 * d11 - d01 * d01;
        if (den > 0) {
            double v = (d11 * d20 - d01 * d21) / den;
            double w = (d00 * d21 - d01 * d20) / den;
            if (v >= 0 && w >= 0 && v + w <= 1) return fabs(t) * sqrt(nn);
        }
    }
    double d1 = seg_dist(p, a, b), d2 = seg_dist(p, b, c), d3 = seg_dist(p, c, a);
    double m = d1 < d2 ? d1 : d2;
    return m < d3 ? m : d3;
}

/* Per query point: the smallest distance to any face edge (vertices included) and
 * to any face.  Used to exclude points where FP32 cannot resolve the sign. */
int wno_min_dist(const double *V, int64_t nV, const int64_t *F, int64_t nF,
                 const double *Q, int64_t nQ, double *d_edge, double *d_face, int nthreads)
{
    for (int64_t f = 0; f < 3 * nF; ++f)
        if (F[f] < 0 || F[f] >= nV) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nQ; ++i) {
        const double *p = Q + 3 * i;
        double de = INFINITY, df = INFINITY;
        for (int64_t f = 0; f < nF; ++f) {
            const double *a = V + 3 * F[3 * f], *b = V + 3 * F[3 * f + 1], *c = V + 3 * F[3 * f + 2];
            double x = seg_dist(p, a, b);
            if (x < de) de = x;
            x = seg_dist(p, b, c);
            if (x < de) de = x;
            x = seg_dist(p, c, a);
            if (x < de) de = x;
            x = tri_dist(p, a, b, c);
            if (x < df) df = x;
        }
        d_edge[i] = de;
        d_face[i] = df;
    }
    return 0;
}

/* Evaluation chain (Section 3): nearest-neighbour distance from every point of A to
 * the point set B, d[i] = min_j |A_i - B_j|, by brute force in FP64. */
int wno_nn_dist(const double *A, int64_t nA, const double *B, int64_t nB, double *d, int nthreads)
{
    if (nB <= 0 && nA > 0) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nA; ++i) {
        double best = INFINITY;
        for (int64_t j = 0; j < nB; ++j) {
            const double dx = A[3 * i] - B[3 * j], dy = A[3 * i + 1] - B[3 * j + 1], dz = A[3 * i + 2] - B[3 * j + 2];
            const double s = dx * dx + dy * dy + dz * dz;
            if (s < best) best = s;
        }
        d[i] = sqrt(best);
    }
    return 0;
}
