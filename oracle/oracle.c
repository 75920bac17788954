/*
 * FP64 reference ("oracle") for short-range pair forces, energy and virial in
 * a deforming periodic box, following Dobson, Fox & Saracino, "Cell List
 * Algorithms for Nonequilibrium Molecular Dynamics" (arXiv:1412.3784).
 *
 * TEST INFRASTRUCTURE ONLY.  It exists to check the GPU library; only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header or table with the GPU library.
 *
 * Conventions
 *   3x3 matrices are row-major double[9]; a lattice basis L has the basis
 *   vectors v1, v2, v3 as its COLUMNS (Sec. 2, L = [v1 v2 v3]), so
 *   L[3*r + c] is component r of v_c.  Positions are N x 3 row-major.
 *   Images of a particle at q are q + L m, m in Z^3 (Sec. 2).
 *
 * What is computed (the plain definition the cell lists must reproduce):
 *   P = {(i, j, m) : (i < j, or i == j and m > 0 lexicographically),
 *                    |x_j + L m - x_i| < r_c}            (Sec. 2 images, Sec. 3 cut-off)
 *   U = sum_P phi(r),  f_ij = -phi'(r) r_ij / r  with r_ij = x_i - x_j - L m,
 *   F_i = sum f_ij, F_j -= f_ij,  W = sum_P r_ij (x) f_ij.
 *   phi is the Lennard-Jones form truncated at r_c and (optionally) shifted
 *   to zero there; WCA is the truncation at 2^(1/6) sigma (named in Sec. 5).
 *   The cut-off test is strict, r^2 < r_c^2, evaluated in FP64 as
 *   d_k = (x_j,k - x_i,k) + (L m)_k,  r^2 = d0*d0 + d1*d1 + d2*d2.
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */
static void mm3(const double *a, const double *b, double *c)
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += a[3 * r + q] * b[3 * q + k];
            t[3 * r + k] = s;
        }
    memcpy(c, t, sizeof t);
}

static double det3(const double *a)
{
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
           a[2] * (a[3] * a[7] - a[4] * a[6]);
}

/* inverse by the adjugate (cofactor transpose) over the determinant */
static int inv3(const double *a, double *out)
{
    double d = det3(a);
    if (d == 0.0 || !isfinite(d)) return -1;
    double c[9];
    c[0] = a[4] * a[8] - a[5] * a[7];
    c[1] = a[2] * a[7] - a[1] * a[8];
    c[2] = a[1] * a[5] - a[2] * a[4];
    c[3] = a[5] * a[6] - a[3] * a[8];
    c[4] = a[0] * a[8] - a[2] * a[6];
    c[5] = a[2] * a[3] - a[0] * a[5];
    c[6] = a[3] * a[7] - a[4] * a[6];
    c[7] = a[1] * a[6] - a[0] * a[7];
    c[8] = a[0] * a[4] - a[1] * a[3];
    for (int k = 0; k < 9; ++k) out[k] = c[k] / d;
    return 0;
}

static void imm3(const int64_t *a, const int64_t *b, int64_t *c)
{
    int64_t t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            int64_t s = 0;
            for (int q = 0; q < 3; ++q) s += a[3 * r + q] * b[3 * q + k];
            t[3 * r + k] = s;
        }
    memcpy(c, t, sizeof t);
}

/* inverse of an integer matrix with determinant 1 (its adjugate) */
static int iinv3(const int64_t *a, int64_t *out)
{
    int64_t d = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                a[2] * (a[3] * a[7] - a[4] * a[6]);
    if (d != 1) return -1;
    out[0] = a[4] * a[8] - a[5] * a[7];
    out[1] = a[2] * a[7] - a[1] * a[8];
    out[2] = a[1] * a[5] - a[2] * a[4];
    out[3] = a[5] * a[6] - a[3] * a[8];
    out[4] = a[0] * a[8] - a[2] * a[6];
    out[5] = a[2] * a[3] - a[0] * a[5];
    out[6] = a[3] * a[7] - a[4] * a[6];
    out[7] = a[1] * a[6] - a[0] * a[7];
    out[8] = a[0] * a[4] - a[1] * a[3];
    return 0;
}

static void ipow3(const int64_t *m, int64_t p, int64_t *out)
{
    int64_t r[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    int64_t b[9];
    if (p < 0) { iinv3(m, b); p = -p; } else memcpy(b, m, sizeof b);
    for (int64_t k = 0; k < p; ++k) imm3(r, b, r);
    memcpy(out, r, sizeof r);
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && (a < 0)) --q;
    return q;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: the lattice moves with the flow, dL/dt = A L, L_t = exp(At) L0  */
/* ------------------------------------------------------------------------ */
/* E = exp(tA).  A diagonal: closed form.  Otherwise the Taylor series with
 * scaling and squaring (Moler & Van Loan's "Taylor + scaling-and-squaring"
 * method); for a nilpotent A (shear) the series terminates exactly.       */
int orc_expm(const double *A, double t, double *E)
{
    int diag = 1;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            if (r != c && A[3 * r + c] != 0.0) diag = 0;
    if (diag) {
        memset(E, 0, 9 * sizeof(double));
        for (int k = 0; k < 3; ++k) E[4 * k] = exp(t * A[4 * k]);
        return 0;
    }
    double X[9], nrm = 0.0;
    for (int k = 0; k < 9; ++k) { X[k] = t * A[k]; nrm = fmax(nrm, fabs(X[k])); }
    int s = 0;
    while (nrm * 3.0 > 0.5 && s < 60) { nrm *= 0.5; ++s; }
    double scale = ldexp(1.0, -s);
    for (int k = 0; k < 9; ++k) X[k] *= scale;
    double term[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, S[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int n = 1; n <= 30; ++n) {
        mm3(term, X, term);
        for (int k = 0; k < 9; ++k) term[k] /= (double)n;
        for (int k = 0; k < 9; ++k) S[k] += term[k];
    }
    for (int q = 0; q < s; ++q) mm3(S, S, S);
    memcpy(E, S, sizeof S);
    return 0;
}

int orc_lattice_at(const double *L0, const double *A, double t, double *L)
{
    double E[9];
    orc_expm(A, t, E);
    mm3(E, L0, L);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2: remapping by SL(3;Z), KR and generalised KR                     */
/* ------------------------------------------------------------------------ */
/* For a diagonal flow A and automorphisms M_k chosen so that L0 M_k L0^-1 is
 * the diagonal matrix exp(diag(mu_k)) (eq:kr: exp(A t*) L0 = L0 M), the
 * stretch theta = t diag(A) is written theta = sum_k alpha_k mu_k; with
 * p_k = floor(alpha_k + 1/2) the reduced basis is
 *     Lred = exp(diag(theta - sum_k p_k mu_k)) L0 = L_t prod_k M_k^{-p_k},
 * the bounded-stretch form of the generalised KR section, and the integer
 * matrix Mtot = prod_k M_k^{-p_k} satisfies Lred = L_t Mtot.
 * naut = 0: no remap (Lred = L_t).  Returns 0, -1 (bad automorphism),
 * -2 (flow not diagonal / not in the span of the log-eigenvalues).        */
/* Sec. 2.2, planar shear (Lees-Edwards): for the shear flow A (A^2 = 0) the
 * lattice is L_t = (I + tA) L0, and the automorphism M = I - N with N^2 = 0
 * resets it.  In lattice coordinates L0^-1 A L0 = s N for a scalar s, so
 * L_t M^p = L0 (I + (s t - p) N); applying M each time the box has been
 * sheared by half a lattice spacing means p = floor(s t + 1/2) (the reset the
 * paper recommends, bounding the deformation angle by 90 - atan 2 degrees).
 * Mtot = M^p = I - p N.  Returns 0, -1 (bad automorphism) or -2 (A is not a
 * shear of the lattice along N).                                          */
static int reduce_shear(const double *L0, const double *A, double t, const int32_t *aut, double *Lred,
                        int32_t *Mtot, int32_t *coef)
{
    int64_t M[9], N[9], NN[9], tmp[9];
    for (int q = 0; q < 9; ++q) M[q] = aut[q];
    if (iinv3(M, tmp)) return -1;
    for (int q = 0; q < 9; ++q) N[q] = (q % 4 == 0 ? 1 : 0) - M[q];
    imm3(N, N, NN);
    for (int q = 0; q < 9; ++q)
        if (NN[q] != 0) return -1;
    double L0i[9], X[9];
    if (inv3(L0, L0i)) return -1;
    mm3(L0i, A, X);
    mm3(X, L0, X);
    double xn = 0.0, nn = 0.0, xmax = 0.0;
    for (int q = 0; q < 9; ++q) {
        xn += X[q] * (double)N[q];
        nn += (double)(N[q] * N[q]);
        xmax = fmax(xmax, fabs(X[q]));
    }
    if (nn == 0.0) return -1;
    double sr = xn / nn;
    for (int q = 0; q < 9; ++q)
        if (fabs(X[q] - sr * (double)N[q]) > 1e-9 * (xmax + 1e-300)) return -2;
    int64_t p = (int64_t)floor(sr * t + 0.5);
    int64_t P[9];
    for (int q = 0; q < 9; ++q) P[q] = (q % 4 == 0 ? 1 : 0) - p * N[q];
    double Lt[9], Pd[9];
    orc_lattice_at(L0, A, t, Lt);
    for (int q = 0; q < 9; ++q) Pd[q] = (double)P[q];
    mm3(Lt, Pd, Lred);
    if (Mtot)
        for (int q = 0; q < 9; ++q) Mtot[q] = (int32_t)P[q];
    if (coef) coef[0] = (int32_t)p;
    return 0;
}

int orc_reduce(const double *L0, const double *A, double t, int naut, const int32_t *aut,
               double *Lred, int32_t *Mtot, int32_t *coef)
{
    if (coef) coef[0] = coef[1] = 0;
    if (naut == 0) {
        orc_lattice_at(L0, A, t, Lred);
        if (Mtot) { memset(Mtot, 0, 9 * sizeof(int32_t)); Mtot[0] = Mtot[4] = Mtot[8] = 1; }
        return 0;
    }
    if (naut < 0 || naut > 2) return -1;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            if (r != c && A[3 * r + c] != 0.0) return naut == 1 ? reduce_shear(L0, A, t, aut, Lred, Mtot, coef) : -2;
    double L0i[9];
    if (inv3(L0, L0i)) return -1;
    double mu[2][3];
    int64_t Mi[2][9];
    for (int k = 0; k < naut; ++k) {
        double Md[9], D[9];
        for (int q = 0; q < 9; ++q) { Md[q] = (double)aut[9 * k + q]; Mi[k][q] = aut[9 * k + q]; }
        int64_t tmp[9];
        if (iinv3(Mi[k], tmp)) return -1; /* det must be exactly 1 */
        mm3(L0, Md, D);
        mm3(D, L0i, D);
        double dmax = 0.0;
        for (int q = 0; q < 9; ++q) dmax = fmax(dmax, fabs(D[q]));
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                if (r != c && fabs(D[3 * r + c]) > 1e-9 * dmax) return -1;
        for (int r = 0; r < 3; ++r) {
            if (!(D[4 * r] > 0.0)) return -1;
            mu[k][r] = log(D[4 * r]);
        }
    }
    double th[3] = {t * A[0], t * A[4], t * A[8]};
    double al[2] = {0.0, 0.0};
    if (naut == 1) {
        double mm = 0.0, mt = 0.0;
        for (int r = 0; r < 3; ++r) { mm += mu[0][r] * mu[0][r]; mt += mu[0][r] * th[r]; }
        al[0] = mt / mm;
    } else {
        double g00 = 0, g01 = 0, g11 = 0, b0 = 0, b1 = 0;
        for (int r = 0; r < 3; ++r) {
            g00 += mu[0][r] * mu[0][r];
            g01 += mu[0][r] * mu[1][r];
            g11 += mu[1][r] * mu[1][r];
            b0 += mu[0][r] * th[r];
            b1 += mu[1][r] * th[r];
        }
        double dd = g00 * g11 - g01 * g01;
        if (fabs(dd) < 1e-12 * g00 * g11) return -1;
        al[0] = (g11 * b0 - g01 * b1) / dd;
        al[1] = (g00 * b1 - g01 * b0) / dd;
    }
    double res = 0.0, tn = 0.0;
    for (int r = 0; r < 3; ++r) {
        double v = th[r] - al[0] * mu[0][r] - (naut == 2 ? al[1] * mu[1][r] : 0.0);
        res = fmax(res, fabs(v));
        tn = fmax(tn, fabs(th[r]));
    }
    if (res > 1e-9 * (1.0 + tn)) return -2;
    int64_t p[2] = {0, 0};
    double e[3] = {th[0], th[1], th[2]};
    for (int k = 0; k < naut; ++k) {
        p[k] = (int64_t)floor(al[k] + 0.5);
        for (int r = 0; r < 3; ++r) e[r] -= (double)p[k] * mu[k][r];
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Lred[3 * r + c] = exp(e[r]) * L0[3 * r + c];
    int64_t M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, P[9];
    for (int k = 0; k < naut; ++k) {
        ipow3(Mi[k], -p[k], P);
        imm3(M, P, M);
    }
    if (Mtot)
        for (int q = 0; q < 9; ++q) Mtot[q] = (int32_t)M[q];
    if (coef) { coef[0] = (int32_t)p[0]; coef[1] = (int32_t)p[1]; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1: box heights (Fig. "bh": distance between opposite faces)        */
/* h_i is the spacing of the lattice planes spanned by the other two vectors */
/* = 1 / |row i of L^-1|.                                                    */
/* ------------------------------------------------------------------------ */
int orc_heights(const double *L, double *h)
{
    double Li[9];
    if (inv3(L, Li)) return -1;
    for (int r = 0; r < 3; ++r)
        h[r] = 1.0 / sqrt(Li[3 * r] * Li[3 * r] + Li[3 * r + 1] * Li[3 * r + 1] +
                          Li[3 * r + 2] * Li[3 * r + 2]);
    return 0;
}

/* c_i = floor(h_i / d_cut) (Sec. 4.1) */
int orc_ds_counts(const double *L, double rc, int32_t *c)
{
    double h[3];
    if (orc_heights(L, h)) return -1;
    for (int k = 0; k < 3; ++k) c[k] = (int32_t)floor(h[k] / rc);
    return (c[0] >= 1 && c[1] >= 1 && c[2] >= 1) ? 0 : -3;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2: rotate the box so v1 lies on the x axis and v2 in the xy plane: */
/* the QR decomposition L = Q R, R upper triangular with positive diagonal.  */
/* Classical Gram-Schmidt on the columns.                                    */
/* ------------------------------------------------------------------------ */
int orc_qr(const double *L, double *Q, double *R)
{
    double v[3][3], q[3][3];
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) v[c][r] = L[3 * r + c];
    memset(R, 0, 9 * sizeof(double));
    for (int c = 0; c < 3; ++c) {
        double w[3] = {v[c][0], v[c][1], v[c][2]};
        for (int p = 0; p < c; ++p) {
            double d = q[p][0] * v[c][0] + q[p][1] * v[c][1] + q[p][2] * v[c][2];
            R[3 * p + c] = d;
            for (int r = 0; r < 3; ++r) w[r] -= d * q[p][r];
        }
        double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (!(nrm > 0.0)) return -1;
        R[3 * c + c] = nrm;
        for (int r = 0; r < 3; ++r) q[c][r] = w[r] / nrm;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Q[3 * r + c] = q[c][r];
    return 0;
}

/* l_i = floor(r_ii / d_cut) (Sec. 5.2) */
int orc_do_counts(const double *L, double rc, int32_t *l)
{
    double Q[9], R[9];
    if (orc_qr(L, Q, R)) return -1;
    for (int k = 0; k < 3; ++k) l[k] = (int32_t)floor(R[4 * k] / rc);
    return (l[0] >= 1 && l[1] >= 1 && l[2] >= 1) ? 0 : -3;
}

/* Dynamic-offset neighbourhood of cell (a,b,c) (Sec. 4.2, the four cases).
 * Rectangular cells of widths w_i = r_ii / l_i tile the rearranged box
 * [0,r11) x [0,r22) x [0,r33); the replica reached by the lattice vector
 * R (i,j,k) is shifted by j r12 + k r13 in x and k r23 in y.  A cell (in any
 * replica) belongs to the neighbourhood if it overlaps the home cell grown
 * on every side by one cell width (grow = 0: the paper's rule, which gives
 * 27 / 30 / 34 / 36 cells for generic offsets) or by d_cut (grow = 1: the
 * tight rule, a subset that still covers the cut-off sphere because
 * w_i >= d_cut).  Layers (z) are never offset; within layer k the rows (y)
 * are offset by k r23 and within row (j, k) the cells (x) by j r12 + k r13.
 * Each entry is (a', b', c', i, j, k): the cell in the box and the lattice
 * image.  Returns the number of entries (at most maxout are written).     */
int orc_do_neighbourhood(const double *R, const int32_t *l, double rc, int32_t a, int32_t b,
                         int32_t c, int32_t grow, int32_t *out, int32_t maxout)
{
    double w[3] = {R[0] / l[0], R[4] / l[1], R[8] / l[2]};
    double g0 = grow ? rc / w[0] : 1.0, g1 = grow ? rc / w[1] : 1.0;
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        int64_t C = c + dz, k = floor_div(C, l[2]), cz = C - k * l[2];
        double fy = -(double)k * R[5] / w[1]; /* row offset of layer k, in rows */
        int64_t B0 = (int64_t)floor(b - g1 + fy), B1 = (int64_t)ceil(b + 1 + g1 + fy) - 1;
        for (int64_t B = B0; B <= B1; ++B) {
            int64_t j = floor_div(B, l[1]), by = B - j * l[1];
            double fx = -((double)j * R[1] + (double)k * R[2]) / w[0]; /* cell offset of row */
            int64_t A0 = (int64_t)floor(a - g0 + fx), A1 = (int64_t)ceil(a + 1 + g0 + fx) - 1;
            for (int64_t Ax = A0; Ax <= A1; ++Ax) {
                int64_t i = floor_div(Ax, l[0]), ax = Ax - i * l[0];
                if (cnt < maxout && out) {
                    int32_t *o = out + 6 * cnt;
                    o[0] = (int32_t)ax; o[1] = (int32_t)by; o[2] = (int32_t)cz;
                    o[3] = (int32_t)i; o[4] = (int32_t)j; o[5] = (int32_t)k;
                }
                ++cnt;
            }
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* pair potential (Sec. 3: zero past the cut-off; WCA named in Sec. 5)       */
/* pot = {eps, sigma, r_c, shift_flag}                                       */
/* ------------------------------------------------------------------------ */
static double pot_shift(const double *pot)
{
    if (pot[3] == 0.0) return 0.0;
    double s2 = pot[1] * pot[1] / (pot[2] * pot[2]);
    double s6 = s2 * s2 * s2;
    return 4.0 * pot[0] * (s6 * s6 - s6);
}

/* for r2 < rc^2: phi(r) and fs with f_ij = fs * r_ij, i.e. fs = -phi'(r)/r */
static void pair_eval(const double *pot, double shift, double r2, double *phi, double *fs)
{
    double s2 = pot[1] * pot[1] / r2;
    double s6 = s2 * s2 * s2;
    double s12 = s6 * s6;
    *phi = 4.0 * pot[0] * (s12 - s6) - shift;
    *fs = 24.0 * pot[0] * (2.0 * s12 - s6) / r2;
}

/* order-independent pair key hash: SplitMix64's output function (Steele,
 * Lea & Flood 2014) applied to (j << 32) | 10-bit biased image components */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static uint64_t pair_key(int64_t j, const int64_t *m)
{
    uint64_t k = ((uint64_t)j) << 32;
    k |= ((uint64_t)((m[0] + 512) & 0x3ff)) << 20;
    k |= ((uint64_t)((m[1] + 512) & 0x3ff)) << 10;
    k |= ((uint64_t)((m[2] + 512) & 0x3ff));
    return mix64(k);
}

/* image m (relative to L, input positions) mapped through Mkey for keys */
static void key_image(const int32_t *Mkey, const int64_t *m, int64_t *out)
{
    if (!Mkey) { out[0] = m[0]; out[1] = m[1]; out[2] = m[2]; return; }
    for (int r = 0; r < 3; ++r)
        out[r] = (int64_t)Mkey[3 * r] * m[0] + (int64_t)Mkey[3 * r + 1] * m[1] +
                 (int64_t)Mkey[3 * r + 2] * m[2];
}

static int lex_positive(const int64_t *m)
{
    if (m[0] != 0) return m[0] > 0;
    if (m[1] != 0) return m[1] > 0;
    return m[2] > 0;
}

/* d = (x_j - x_i) + L m, the separation of x_i from image m of x_j */
static double sep2(const double *L, const double *xi, const double *xj, const int64_t *m, double *d)
{
    for (int k = 0; k < 3; ++k) {
        double lm = L[3 * k] * (double)m[0] + L[3 * k + 1] * (double)m[1] + L[3 * k + 2] * (double)m[2];
        d[k] = (xj[k] - xi[k]) + lm;
    }
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

/* range of image components that can reach within r_c: with u = s_j - s_i + m
 * (fractional separation), |L u| < r_c implies |u_k| <= r_c / h_k.           */
static void image_range(const double *Li, const double *h, double rc, const double *xi,
                        const double *xj, int64_t *lo, int64_t *hi)
{
    for (int k = 0; k < 3; ++k) {
        double ds = Li[3 * k] * (xj[0] - xi[0]) + Li[3 * k + 1] * (xj[1] - xi[1]) +
                    Li[3 * k + 2] * (xj[2] - xi[2]);
        lo[k] = (int64_t)ceil(-ds - rc / h[k]) - 1;
        hi[k] = (int64_t)floor(-ds + rc / h[k]) + 1;
    }
}

/* ------------------------------------------------------------------------ */
/* Brute force over all particle pairs and all reachable lattice images.     */
/* Writes up to maxp pairs as (i, j, m0, m1, m2); returns |P|.               */
/* ------------------------------------------------------------------------ */
int64_t orc_pairs_brute(const double *x, int64_t n, const double *L, double rc, int64_t maxp,
                        int64_t *out)
{
    double Li[9], h[3];
    if (inv3(L, Li) || orc_heights(L, h)) return -1;
    double rc2 = rc * rc;
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j) {
            int64_t lo[3], hi[3], m[3];
            image_range(Li, h, rc, x + 3 * i, x + 3 * j, lo, hi);
            for (m[0] = lo[0]; m[0] <= hi[0]; ++m[0])
                for (m[1] = lo[1]; m[1] <= hi[1]; ++m[1])
                    for (m[2] = lo[2]; m[2] <= hi[2]; ++m[2]) {
                        if (i == j && !lex_positive(m)) continue;
                        double d[3];
                        if (sep2(L, x + 3 * i, x + 3 * j, m, d) < rc2) {
                            if (np < maxp && out) {
                                int64_t *o = out + 5 * np;
                                o[0] = i; o[1] = j; o[2] = m[0]; o[3] = m[1]; o[4] = m[2];
                            }
                            ++np;
                        }
                    }
        }
    return np;
}

/* accumulate one pair of P into the outputs (full per-particle bookkeeping) */
static void add_pair(const double *pot, double shift, int64_t i, int64_t j, const int64_t *m,
                     const double *d, double r2, const int32_t *Mkey, double *F, double *u,
                     double *U, double *W, int64_t *cnt, uint64_t *hash)
{
    double phi, fs;
    pair_eval(pot, shift, r2, &phi, &fs);
    double rij[3] = {-d[0], -d[1], -d[2]};
    double f[3] = {fs * rij[0], fs * rij[1], fs * rij[2]};
    if (F)
        for (int k = 0; k < 3; ++k) { F[3 * i + k] += f[k]; F[3 * j + k] -= f[k]; }
    if (u) { u[i] += 0.5 * phi; u[j] += 0.5 * phi; }
    *U += phi;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) W[3 * a + b] += rij[a] * f[b];
    if (cnt) { cnt[i] += 1; cnt[j] += 1; }
    if (hash) {
        int64_t km[3], mneg[3] = {-m[0], -m[1], -m[2]}, kn[3];
        key_image(Mkey, m, km);
        key_image(Mkey, mneg, kn);
        hash[i] += pair_key(j, km);
        hash[j] += pair_key(i, kn);
    }
}

/* Forces, energy, virial and per-particle (count, hash) over the brute-force
 * pair set P.  Any output may be NULL except U and W.  Mkey (optional) maps
 * the image vector before hashing.                                          */
int orc_forces_brute(const double *x, int64_t n, const double *L, const double *pot,
                     const int32_t *Mkey, double *F, double *u, double *U, double *W,
                     int64_t *cnt, uint64_t *hash)
{
    double Li[9], h[3];
    if (inv3(L, Li) || orc_heights(L, h)) return -1;
    double rc = pot[2], rc2 = rc * rc, shift = pot_shift(pot);
    if (F) memset(F, 0, 3 * n * sizeof(double));
    if (u) memset(u, 0, n * sizeof(double));
    if (cnt) memset(cnt, 0, n * sizeof(int64_t));
    if (hash) memset(hash, 0, n * sizeof(uint64_t));
    *U = 0.0;
    memset(W, 0, 9 * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j) {
            int64_t lo[3], hi[3], m[3];
            image_range(Li, h, rc, x + 3 * i, x + 3 * j, lo, hi);
            for (m[0] = lo[0]; m[0] <= hi[0]; ++m[0])
                for (m[1] = lo[1]; m[1] <= hi[1]; ++m[1])
                    for (m[2] = lo[2]; m[2] <= hi[2]; ++m[2]) {
                        if (i == j && !lex_positive(m)) continue;
                        double d[3];
                        double r2 = sep2(L, x + 3 * i, x + 3 * j, m, d);
                        if (r2 < rc2) add_pair(pot, shift, i, j, m, d, r2, Mkey, F, u, U, W, cnt, hash);
                    }
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1, the dynamic-size cell list, written plainly: cells congruent to */
/* the box, c_i = floor(h_i / d_cut), particles assigned in the lattice      */
/* basis, 27-cell neighbourhood visited as (cell, image) pairs.  Every       */
/* particle visits its whole neighbourhood (each pair is seen from both      */
/* ends); per-particle sums run in a fixed order, and the global U and W are */
/* summed over fixed chunks in index order, so results do not depend on the  */
/* thread count.  stats = {candidates visited, in-range (directed) pairs}.   */
/* ------------------------------------------------------------------------ */
#define ORC_CHUNK 4096

int orc_forces_cells(const double *x, int64_t n, const double *L, const double *pot,
                     const int32_t *Mkey, int nthreads, const int64_t *sub, int64_t nsub, double *F,
                     double *u, double *U, double *W, int64_t *cnt, uint64_t *hash, int64_t *stats,
                     double *fmag)
{
    double Li[9];
    int32_t c[3];
    if (inv3(L, Li)) return -1;
    int rcode = orc_ds_counts(L, pot[2], c);
    if (rcode) return rcode;
    double rc2 = pot[2] * pot[2], shift = pot_shift(pot);
    if (sub)
        for (int64_t q = 0; q < nsub; ++q)
            if (sub[q] < 0 || sub[q] >= n) return -5;
    int64_t nc = (int64_t)c[0] * c[1] * c[2];
    int64_t *img = (int64_t *)malloc(3 * n * sizeof(int64_t));
    int64_t *cell = (int64_t *)malloc(n * sizeof(int64_t));
    int64_t *start = (int64_t *)calloc(nc + 1, sizeof(int64_t));
    int64_t *members = (int64_t *)malloc(n * sizeof(int64_t));
    const int64_t nrows = sub ? nsub : n;
    int64_t nchunks = (nrows + ORC_CHUNK - 1) / ORC_CHUNK;
    double *cU = (double *)calloc(nchunks > 0 ? nchunks : 1, sizeof(double));
    double *cW = (double *)calloc(9 * (nchunks > 0 ? nchunks : 1), sizeof(double));
    int64_t *cS = (int64_t *)calloc(2 * (nchunks > 0 ? nchunks : 1), sizeof(int64_t));
    if (!img || !cell || !start || !members || !cU || !cW || !cS) {
        free(img); free(cell); free(start); free(members); free(cU); free(cW); free(cS);
        return -4;
    }
    /* assignment: s = L^-1 x, wrap s into [0,1), cell = floor(c s) */
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + 3 * i;
        int64_t a[3];
        for (int k = 0; k < 3; ++k) {
            double s = Li[3 * k] * xi[0] + Li[3 * k + 1] * xi[1] + Li[3 * k + 2] * xi[2];
            double fl = floor(s);
            double w = s - fl;
            int64_t nk = (int64_t)fl;
            if (w >= 1.0) { w = 0.0; nk += 1; }
            img[3 * i + k] = nk;
            int64_t ak = (int64_t)floor(w * c[k]);
            if (ak < 0) ak = 0;
            if (ak > c[k] - 1) ak = c[k] - 1;
            a[k] = ak;
        }
        cell[i] = a[0] + (int64_t)c[0] * (a[1] + (int64_t)c[1] * a[2]);
        start[cell[i] + 1] += 1;
    }
    for (int64_t q = 0; q < nc; ++q) start[q + 1] += start[q];
    {
        int64_t *fill = (int64_t *)malloc((nc > 0 ? nc : 1) * sizeof(int64_t));
        if (!fill) { free(img); free(cell); free(start); free(members); free(cU); free(cW); free(cS); return -4; }
        memcpy(fill, start, nc * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) members[fill[cell[i]]++] = i; /* stable: index order */
        free(fill);
    }
    /* thread count for this call only (0: the OpenMP default) */
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        double Uc = 0.0, Wc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        int64_t cand = 0, inr = 0;
        int64_t iend = (ch + 1) * ORC_CHUNK < nrows ? (ch + 1) * ORC_CHUNK : nrows;
        for (int64_t row = ch * ORC_CHUNK; row < iend; ++row) {
            const int64_t i = sub ? sub[row] : row;
            int64_t ci = cell[i];
            int64_t a[3] = {ci % c[0], (ci / c[0]) % c[1], ci / ((int64_t)c[0] * c[1])};
            double Fi[3] = {0, 0, 0}, ui = 0.0, mi = 0.0;
            int64_t ki = 0;
            uint64_t hi = 0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int64_t Au[3] = {a[0] + dx, a[1] + dy, a[2] + dz}, mc[3], ap[3];
                        for (int k = 0; k < 3; ++k) {
                            mc[k] = floor_div(Au[k], c[k]);
                            ap[k] = Au[k] - mc[k] * c[k];
                        }
                        int64_t cj = ap[0] + (int64_t)c[0] * (ap[1] + (int64_t)c[1] * ap[2]);
                        for (int64_t q = start[cj]; q < start[cj + 1]; ++q) {
                            int64_t j = members[q];
                            /* image relative to the input positions */
                            int64_t m[3] = {mc[0] - img[3 * j] + img[3 * i],
                                            mc[1] - img[3 * j + 1] + img[3 * i + 1],
                                            mc[2] - img[3 * j + 2] + img[3 * i + 2]};
                            if (j == i && m[0] == 0 && m[1] == 0 && m[2] == 0) continue;
                            ++cand;
                            double d[3];
                            double r2 = sep2(L, x + 3 * i, x + 3 * j, m, d);
                            if (!(r2 < rc2)) continue;
                            ++inr;
                            double phi, fs;
                            pair_eval(pot, shift, r2, &phi, &fs);
                            double rij[3] = {-d[0], -d[1], -d[2]};
                            for (int k = 0; k < 3; ++k) Fi[k] += fs * rij[k];
                            mi += fabs(fs) * sqrt(r2);
                            ui += 0.5 * phi;
                            for (int p = 0; p < 3; ++p)
                                for (int s = 0; s < 3; ++s) Wc[3 * p + s] += 0.5 * rij[p] * fs * rij[s];
                            ++ki;
                            if (hash) {
                                int64_t km[3];
                                key_image(Mkey, m, km);
                                hi += pair_key(j, km);
                            }
                        }
                    }
            if (F) for (int k = 0; k < 3; ++k) F[3 * row + k] = Fi[k];
            if (u) u[row] = ui;
            if (fmag) fmag[row] = mi;
            if (cnt) cnt[row] = ki;
            if (hash) hash[row] = hi;
            Uc += ui;
        }
        cU[ch] = Uc;
        for (int k = 0; k < 9; ++k) cW[9 * ch + k] = Wc[k];
        cS[2 * ch] = cand;
        cS[2 * ch + 1] = inr;
    }
    *U = 0.0;
    memset(W, 0, 9 * sizeof(double));
    int64_t s0 = 0, s1 = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        *U += cU[ch];
        for (int k = 0; k < 9; ++k) W[k] += cW[9 * ch + k];
        s0 += cS[2 * ch];
        s1 += cS[2 * ch + 1];
    }
    if (stats) { stats[0] = s0; stats[1] = s1; }
    free(img); free(cell); free(start); free(members); free(cU); free(cW); free(cS);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SLLOD dynamics in the deforming box (Sec. 2.1: the box follows the flow,  */
/* dL/dt = A L; particles stream with it).  The paper states the lab-frame   */
/* equations with image momenta; this oracle uses the equivalent peculiar-   */
/* momentum form                                                             */
/*     dq/dt = p/m + A q,      dp/dt = F(q) - A p,                           */
/* whose images q + L m carry the same p.  One step of length h is the       */
/* symmetric splitting                                                       */
/*     p <- e^{-Ah/2} p,  p <- p + (h/2) F(q),                               */
/*     q <- e^{Ah} q + h phi1(Ah) p / m         (exact flow of dq/dt, p fixed) */
/*     t <- t + h, F <- F(q) in the lattice at t,                            */
/*     p <- p + (h/2) F,  p <- e^{-Ah/2} p,                                  */
/* with phi1(z) = (e^z - 1)/z, for a diagonal A.  Positions are kept in the  */
/* unit cell of the reduced basis (a lattice translation, Sec. 2).  Each     */
/* record (after the start and after every step) holds                       */
/*     t, U, W_xx, W_yy, W_zz, K_xx, K_yy, K_zz   with K_aa = sum_i p_ia^2/m,  */
/* W as in orc_forces_cells.  Total energy H = sum_a K_aa/2 + U obeys        */
/*     dH/dt = -sum_a A_aa (K_aa + W_aa)                                     */
/* along exact solutions, which the tests use as a pin.                     */
/* Returns 0, or the first failing code of orc_reduce / orc_forces_cells.   */
/* ------------------------------------------------------------------------ */
static double phi1(double z) { return z != 0.0 ? expm1(z) / z : 1.0; }

static void wrap_into(const double *L, double *x, int64_t n)
{
    double Li[9];
    if (inv3(L, Li)) return;
    for (int64_t i = 0; i < n; ++i) {
        double *q = x + 3 * i, f[3];
        for (int k = 0; k < 3; ++k)
            f[k] = floor(Li[3 * k] * q[0] + Li[3 * k + 1] * q[1] + Li[3 * k + 2] * q[2]);
        for (int k = 0; k < 3; ++k) q[k] -= L[3 * k] * f[0] + L[3 * k + 1] * f[1] + L[3 * k + 2] * f[2];
    }
}

static int sllod_forces(const double *x, int64_t n, const double *L0, const double *A, double t, int naut,
                        const int32_t *aut, const double *pot, int nthreads, double *Lred, double *F,
                        double *U, double *W)
{
    int32_t M[9];
    int rc = orc_reduce(L0, A, t, naut, aut, Lred, M, NULL);
    if (rc) return rc;
    return orc_forces_cells(x, n, Lred, pot, NULL, nthreads, NULL, 0, F, NULL, U, W, NULL, NULL, NULL, NULL);
}

static void sllod_record(double *o, double t, double U, const double *W, const double *p, int64_t n, double m)
{
    double K[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) K[a] += p[3 * i + a] * p[3 * i + a] / m;
    o[0] = t;
    o[1] = U;
    o[2] = W[0];
    o[3] = W[4];
    o[4] = W[8];
    for (int a = 0; a < 3; ++a) o[5 + a] = K[a];
}

int orc_sllod(double *x, double *p, int64_t n, const double *L0, const double *A, double t0, int naut,
              const int32_t *aut, const double *pot, double h, double mass, int64_t nsteps, int nthreads,
              double *hist)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            if (r != c && A[3 * r + c] != 0.0) return -2;
    double *F = (double *)malloc((n > 0 ? 3 * n : 1) * sizeof(double));
    if (!F) return -4;
    double Lred[9], U, W[9];
    double a[3] = {A[0], A[4], A[8]};
    double t = t0;
    int rc = sllod_forces(x, n, L0, A, t, naut, aut, pot, nthreads, Lred, F, &U, W);
    if (rc) { free(F); return rc; }
    wrap_into(Lred, x, n);
    if (hist) sllod_record(hist, t, U, W, p, n, mass);
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k)
                p[3 * i + k] = exp(-0.5 * h * a[k]) * p[3 * i + k] + 0.5 * h * F[3 * i + k];
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k)
                x[3 * i + k] = exp(h * a[k]) * x[3 * i + k] + h * phi1(h * a[k]) * p[3 * i + k] / mass;
        t = t0 + (double)(s + 1) * h;
        rc = sllod_forces(x, n, L0, A, t, naut, aut, pot, nthreads, Lred, F, &U, W);
        if (rc) { free(F); return rc; }
        wrap_into(Lred, x, n);
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k)
                p[3 * i + k] = exp(-0.5 * h * a[k]) * (p[3 * i + k] + 0.5 * h * F[3 * i + k]);
        if (hist) sllod_record(hist + 8 * (s + 1), t, U, W, p, n, mass);
    }
    free(F);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
