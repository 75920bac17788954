// FP64 lattice geometry shared by the host API and the device kernels.
//
// Everything here is O(1) per box: the reduced basis at strain time t
// (Sec. 2.1-2.2 of Dobson, Fox & Saracino, arXiv:1412.3784), the box heights
// and dynamic-size cell counts (Sec. 4.1), the QR rotation and dynamic-offset
// cell widths (Sec. 4.2), and the per-box record ("CellGeom") the binning and
// sweep kernels take by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define NCL_HD __host__ __device__ inline

namespace ncl {

// ---------------------------------------------------------------------------
// 3x3 helpers (row-major)
// ---------------------------------------------------------------------------
NCL_HD void mat_mul(const double* a, const double* b, double* c) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      t[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
  for (int k = 0; k < 9; ++k) c[k] = t[k];
}

NCL_HD double mat_det(const double* m) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// inverse through the cofactor matrix; returns false when singular
NCL_HD bool mat_inv(const double* m, double* out) {
  const double det = mat_det(m);
  if (!(det != 0.0) || det != det) return false;
  const double r = 1.0 / det;
  double t[9] = {m[4] * m[8] - m[5] * m[7], m[2] * m[7] - m[1] * m[8], m[1] * m[5] - m[2] * m[4],
                 m[5] * m[6] - m[3] * m[8], m[0] * m[8] - m[2] * m[6], m[2] * m[3] - m[0] * m[5],
                 m[3] * m[7] - m[4] * m[6], m[1] * m[6] - m[0] * m[7], m[0] * m[4] - m[1] * m[3]};
  for (int k = 0; k < 9; ++k) out[k] = t[k] * r;
  return true;
}

NCL_HD void imat_mul(const int64_t* a, const int64_t* b, int64_t* c) {
  int64_t t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      t[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
  for (int k = 0; k < 9; ++k) c[k] = t[k];
}

// adjugate of a determinant-one integer matrix = its inverse
NCL_HD int64_t imat_det(const int64_t* m) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}
NCL_HD void imat_adj(const int64_t* m, int64_t* out) {
  int64_t t[9] = {m[4] * m[8] - m[5] * m[7], m[2] * m[7] - m[1] * m[8], m[1] * m[5] - m[2] * m[4],
                  m[5] * m[6] - m[3] * m[8], m[0] * m[8] - m[2] * m[6], m[2] * m[3] - m[0] * m[5],
                  m[3] * m[7] - m[4] * m[6], m[1] * m[6] - m[0] * m[7], m[0] * m[4] - m[1] * m[3]};
  for (int k = 0; k < 9; ++k) out[k] = t[k];
}

NCL_HD int64_t idiv_floor(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (q * b > a) ? q - 1 : q;
}
NCL_HD int idiv_floor32(int a, int b) {  // b > 0
  int q = a / b;
  return (q * b > a) ? q - 1 : q;
}
// floor(a / b), b > 0, by two comparisons when -b <= a < 2b (a cell index
// plus or minus a few cells), else by a division
// floor(a / b) for b > 0 from inv_b = 1 / b rounded to FP64: the product
// (a + 1/2) inv_b is within a relative 2^-52 of (a + 1/2) / b, i.e. within
// |a + 1/2| 2^-52 / b < 1 / (2 b) of it for |a| < 2^51, while (a + 1/2) / b
// lies at least 1 / (2 b) from every integer; its floor is floor(a / b)
NCL_HD int idiv_floor_f(int a, double inv_b) { return (int)floor(((double)a + 0.5) * inv_b); }

NCL_HD int idiv_floor_near(int a, int b) {
  if (a >= -b && a < 2 * b) return (int)(a >= b) - (int)(a < 0);
  return idiv_floor32(a, b);
}

// ---------------------------------------------------------------------------
// reduction of the deforming basis (Sec. 2.2)
// ---------------------------------------------------------------------------
// Constants of a remapping policy that do not depend on t: the log-eigenvalue
// vectors mu_k of L0 M_k L0^-1 (diagonal by construction of L0, eq:kr), the
// Gram matrix of the mu_k, and the automorphisms and their inverses.
struct RemapPolicy {
  int naut;            // 0, 1 (KR / Lees-Edwards) or 2 (generalised KR)
  int shear;           // 1: planar shear, A^2 = 0 (Sec. 2.2, Lees-Edwards)
  double L0[9];
  double adiag[3];     // diagonal of A
  double mu[2][3];
  double gram_inv[4];  // inverse of the 2x2 (or 1x1) Gram matrix of the mu_k
  int64_t M[2][9];
  int64_t Minv[2][9];
  // shear: L_t = L0 (I + s t N), N = I - M (N^2 = 0), L0N = L0 N; without an
  // automorphism N is replaced by X = L0^-1 A L0 itself (s = 1)
  double s;
  double L0N[9];
  int64_t N[9];
};

enum { GEOM_OK = 0, GEOM_E_AUT = -1, GEOM_E_FLOW = -2, GEOM_E_SMALL = -3, GEOM_E_SINGULAR = -4 };

// host-only set-up; returns GEOM_* code
// Planar shear (Sec. 2.2): A nilpotent (A^2 = 0), L_t = (I + tA) L0.  With
// the automorphism M, N = I - M must satisfy N^2 = 0 and L0^-1 A L0 = s N;
// the reset M^p, p = floor(s t + 1/2), is applied whenever the box has been
// sheared by half a lattice spacing, so Lred = L0 (I + (s t - p) N) and
// Mtot = M^p = I - p N.
inline int shear_policy_init(RemapPolicy* p, const double* A, int naut, const int32_t* aut) {
  double AA[9], amax = 0.0;
  mat_mul(A, A, AA);
  for (int k = 0; k < 9; ++k) amax = fmax(amax, fabs(A[k]));
  for (int k = 0; k < 9; ++k)
    if (fabs(AA[k]) > 1e-12 * amax * amax) return GEOM_E_FLOW;
  double L0i[9], X[9];
  if (!mat_inv(p->L0, L0i)) return GEOM_E_SINGULAR;
  mat_mul(L0i, A, X);
  mat_mul(X, p->L0, X);
  p->shear = 1;
  if (naut == 0) {
    // no reset: L_t = L0 (I + t X)
    p->s = 1.0;
    mat_mul(p->L0, X, p->L0N);
    for (int k = 0; k < 9; ++k) p->N[k] = 0;
    return GEOM_OK;
  }
  if (naut != 1) return GEOM_E_FLOW;
  int64_t M[9], NN[9];
  for (int k = 0; k < 9; ++k) M[k] = aut[k];
  if (imat_det(M) != 1) return GEOM_E_AUT;
  for (int k = 0; k < 9; ++k) p->N[k] = (k % 4 == 0 ? 1 : 0) - M[k];
  imat_mul(p->N, p->N, NN);
  for (int k = 0; k < 9; ++k)
    if (NN[k] != 0) return GEOM_E_AUT;
  double xn = 0.0, nn = 0.0, xmax = 0.0;
  for (int k = 0; k < 9; ++k) {
    xn += X[k] * (double)p->N[k];
    nn += (double)(p->N[k] * p->N[k]);
    xmax = fmax(xmax, fabs(X[k]));
  }
  if (nn == 0.0) return GEOM_E_AUT;
  p->s = xn / nn;
  for (int k = 0; k < 9; ++k)
    if (fabs(X[k] - p->s * (double)p->N[k]) > 1e-9 * (xmax + 1e-300)) return GEOM_E_FLOW;
  double Nd[9];
  for (int k = 0; k < 9; ++k) Nd[k] = (double)p->N[k];
  mat_mul(p->L0, Nd, p->L0N);
  return GEOM_OK;
}

inline int remap_policy_init(RemapPolicy* p, const double* L0, const double* A, int naut,
                             const int32_t* aut) {
  for (int k = 0; k < 9; ++k) p->L0[k] = L0[k];
  p->naut = naut;
  p->shear = 0;
  for (int k = 0; k < 3; ++k) p->adiag[k] = A[4 * k];
  if (naut < 0 || naut > 2) return GEOM_E_AUT;
  bool diag = true;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (i != j && A[3 * i + j] != 0.0) diag = false;
  if (!diag) return shear_policy_init(p, A, naut, aut);
  if (naut == 0) return GEOM_OK;
  double L0i[9];
  if (!mat_inv(L0, L0i)) return GEOM_E_SINGULAR;
  for (int a = 0; a < naut; ++a) {
    double Md[9], D[9];
    for (int k = 0; k < 9; ++k) {
      p->M[a][k] = aut[9 * a + k];
      Md[k] = (double)aut[9 * a + k];
    }
    if (imat_det(p->M[a]) != 1) return GEOM_E_AUT;
    imat_adj(p->M[a], p->Minv[a]);
    mat_mul(L0, Md, D);
    mat_mul(D, L0i, D);
    double big = 0.0;
    for (int k = 0; k < 9; ++k) big = fmax(big, fabs(D[k]));
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (i != j && fabs(D[3 * i + j]) > 1e-9 * big) return GEOM_E_AUT;
    for (int i = 0; i < 3; ++i) {
      if (!(D[4 * i] > 0.0)) return GEOM_E_AUT;
      p->mu[a][i] = log(D[4 * i]);
    }
  }
  // Gram matrix of the mu vectors and its inverse
  double g00 = 0, g01 = 0, g11 = 0;
  for (int i = 0; i < 3; ++i) {
    g00 += p->mu[0][i] * p->mu[0][i];
    if (naut == 2) {
      g01 += p->mu[0][i] * p->mu[1][i];
      g11 += p->mu[1][i] * p->mu[1][i];
    }
  }
  if (naut == 1) {
    if (!(g00 > 0.0)) return GEOM_E_AUT;
    p->gram_inv[0] = 1.0 / g00;
  } else {
    const double det = g00 * g11 - g01 * g01;
    if (!(fabs(det) > 1e-12 * g00 * g11)) return GEOM_E_AUT;
    p->gram_inv[0] = g11 / det;
    p->gram_inv[1] = -g01 / det;
    p->gram_inv[2] = -g01 / det;
    p->gram_inv[3] = g00 / det;
  }
  // the flow must lie in the span of the mu_k
  double a[2];
  double b0 = 0, b1 = 0;
  for (int i = 0; i < 3; ++i) {
    b0 += p->mu[0][i] * p->adiag[i];
    if (naut == 2) b1 += p->mu[1][i] * p->adiag[i];
  }
  if (naut == 1) {
    a[0] = b0 * p->gram_inv[0];
    a[1] = 0.0;
  } else {
    a[0] = p->gram_inv[0] * b0 + p->gram_inv[1] * b1;
    a[1] = p->gram_inv[2] * b0 + p->gram_inv[3] * b1;
  }
  double res = 0.0, an = 0.0;
  for (int i = 0; i < 3; ++i) {
    double r = p->adiag[i] - a[0] * p->mu[0][i] - (naut == 2 ? a[1] * p->mu[1][i] : 0.0);
    res = fmax(res, fabs(r));
    an = fmax(an, fabs(p->adiag[i]));
  }
  if (res > 1e-9 * (an + 1e-300) && an > 0.0) return GEOM_E_FLOW;
  return GEOM_OK;
}

// Reduced basis at time t: Lred = exp(diag(eps)) L0 with eps = t diag(A) -
// sum_k p_k mu_k, p_k = floor(alpha_k + 1/2) (the bounded-stretch form of the
// generalised-KR boundary conditions).  Without automorphisms, Lred =
// exp(tA) L0 for diagonal A.  coef receives (p1, p2).
NCL_HD void remap_at(const RemapPolicy& p, double t, double* Lred, int64_t* coef) {
  double th[3] = {t * p.adiag[0], t * p.adiag[1], t * p.adiag[2]};
  coef[0] = coef[1] = 0;
  if (p.shear) {
    // Lred = L0 + (s t - p) L0 N
    const double st = p.s * t;
    if (p.naut == 1) coef[0] = (int64_t)floor(st + 0.5);
    const double f = st - (double)coef[0];
    for (int k = 0; k < 9; ++k) Lred[k] = p.L0[k] + f * p.L0N[k];
    return;
  }
  if (p.naut >= 1) {
    double b0 = 0, b1 = 0;
    for (int i = 0; i < 3; ++i) {
      b0 += p.mu[0][i] * th[i];
      if (p.naut == 2) b1 += p.mu[1][i] * th[i];
    }
    double a0, a1 = 0.0;
    if (p.naut == 1) {
      a0 = b0 * p.gram_inv[0];
    } else {
      a0 = p.gram_inv[0] * b0 + p.gram_inv[1] * b1;
      a1 = p.gram_inv[2] * b0 + p.gram_inv[3] * b1;
    }
    coef[0] = (int64_t)floor(a0 + 0.5);
    coef[1] = (p.naut == 2) ? (int64_t)floor(a1 + 0.5) : 0;
    for (int i = 0; i < 3; ++i) {
      th[i] -= (double)coef[0] * p.mu[0][i];
      if (p.naut == 2) th[i] -= (double)coef[1] * p.mu[1][i];
    }
  }
  for (int i = 0; i < 3; ++i) {
    const double e = exp(th[i]);
    for (int j = 0; j < 3; ++j) Lred[3 * i + j] = e * p.L0[3 * i + j];
  }
}

// Mtot = M1^-p1 M2^-p2 (elongation) or M^p (shear), so that Lred = L_t Mtot
NCL_HD void remap_matrix(const RemapPolicy& p, const int64_t* coef, int64_t* Mtot) {
  if (p.shear) {
    // M^p = I - p N
    for (int k = 0; k < 9; ++k) Mtot[k] = (k % 4 == 0 ? 1 : 0) - coef[0] * p.N[k];
    return;
  }
  int64_t R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int a = 0; a < p.naut; ++a) {
    const int64_t* step = coef[a] > 0 ? p.Minv[a] : p.M[a];
    const int64_t n = coef[a] > 0 ? coef[a] : -coef[a];
    for (int64_t q = 0; q < n; ++q) imat_mul(R, step, R);
  }
  for (int k = 0; k < 9; ++k) Mtot[k] = R[k];
}

// Reduced basis at time t for a policy set up by remap_policy_init (host):
// with automorphisms, the remapped basis L_t M_tot (Sec. 2.2) and its
// coefficients; without, L_t = exp(tA) L0 itself (Sec. 2.1), in closed form
// for diagonal A, else by a Taylor series with scaling and squaring.
inline void reduced_lattice(const RemapPolicy& p, const double* A, double t, double* Lred, int64_t* coef,
                            int64_t* Mtot) {
  if (p.naut > 0) {
    remap_at(p, t, Lred, coef);
    remap_matrix(p, coef, Mtot);
    return;
  }
  bool diag = true;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (i != j && A[3 * i + j] != 0.0) diag = false;
  double E[9];
  if (diag) {
    for (int k = 0; k < 9; ++k) E[k] = 0.0;
    for (int i = 0; i < 3; ++i) E[4 * i] = exp(t * A[4 * i]);
  } else {
    double X[9], big = 0.0;
    for (int k = 0; k < 9; ++k) {
      X[k] = t * A[k];
      big = fmax(big, fabs(X[k]));
    }
    int sq = 0;
    while (big > 0.125 && sq < 64) {
      big *= 0.5;
      ++sq;
    }
    const double sc = ldexp(1.0, -sq);
    for (int k = 0; k < 9; ++k) X[k] *= sc;
    double term[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int k = 0; k < 9; ++k) E[k] = term[k];
    for (int q = 1; q <= 24; ++q) {
      mat_mul(term, X, term);
      for (int k = 0; k < 9; ++k) {
        term[k] /= (double)q;
        E[k] += term[k];
      }
    }
    for (int q = 0; q < sq; ++q) mat_mul(E, E, E);
  }
  mat_mul(E, p.L0, Lred);
  coef[0] = coef[1] = 0;
  for (int k = 0; k < 9; ++k) Mtot[k] = (k % 4 == 0) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// cell geometry of one box (Sec. 4.1 dynamic size, Sec. 4.2 dynamic offset)
// ---------------------------------------------------------------------------
enum { VAR_DS = 0, VAR_DO = 1 };

struct CellGeom {
  // frame: DS -> Cartesian; DO -> rotated frame x' = Q^T x
  double B[9];      // basis in the frame: DS Lred, DO R (upper triangular)
  double Binv[9];   // B^-1
  double Finv[9];   // DS: Lred^-1 (Cartesian -> fractional); DO: Q^T
  double Q[9];      // DO: rotation (Lred = Q R); DS: identity
  double cen[9];    // DS: Lred diag(1/c) (cell step vectors as columns); DO: diag(w)
  double ds_delta[27][3];  // DS: Lred diag(1/c) delta for the 27 stencil offsets
  double w[3];      // DO cell widths r_ii / l_i; DS: 1/c_i (fractional cell size)
  double inv_w[2];  // DO: 1 / w[0], 1 / w[1]
  double inv_nc[3]; // 1 / nc[i] (idiv_floor_f)
  double grow[2];   // DO: neighbourhood growth (in cells) along x and y
  double rc2_lo64, rc2_hi64;  // per-particle screen: rc^2 minus / plus its rounding band
  int32_t nc[3];    // cells per axis (c_i or l_i)
  int32_t variant;
  int64_t Mtot[9];  // Lred = L_t Mtot (used only for pair keys)
};

// heights h_i = 1 / |row i of Lred^-1|
NCL_HD void box_heights(const double* Linv, double* h) {
  for (int i = 0; i < 3; ++i)
    h[i] = 1.0 / sqrt(Linv[3 * i] * Linv[3 * i] + Linv[3 * i + 1] * Linv[3 * i + 1] +
                      Linv[3 * i + 2] * Linv[3 * i + 2]);
}

// Householder-free QR of a 3x3 basis by modified Gram-Schmidt on its columns
NCL_HD bool basis_qr(const double* L, double* Q, double* R) {
  double q[3][3];
  for (int k = 0; k < 9; ++k) R[k] = 0.0;
  for (int c = 0; c < 3; ++c) {
    double v[3] = {L[c], L[3 + c], L[6 + c]};
    for (int p = 0; p < c; ++p) {
      const double d = q[p][0] * v[0] + q[p][1] * v[1] + q[p][2] * v[2];
      R[3 * p + c] = d;
      v[0] -= d * q[p][0];
      v[1] -= d * q[p][1];
      v[2] -= d * q[p][2];
    }
    const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!(nv > 0.0)) return false;
    R[4 * c] = nv;
    for (int r = 0; r < 3; ++r) q[c][r] = v[r] / nv;
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Q[3 * r + c] = q[c][r];
  return true;
}

// Fill the record for one box; returns GEOM_OK or GEOM_E_SMALL / SINGULAR.
NCL_HD int cell_geom_init(CellGeom* g, const double* Lred, const int64_t* Mtot, double rc,
                          int variant, int do_tight) {
  g->variant = variant;
  for (int k = 0; k < 9; ++k) g->Mtot[k] = Mtot[k];
  double Linv[9];
  if (!mat_inv(Lred, Linv)) return GEOM_E_SINGULAR;
  if (variant == VAR_DS) {
    double h[3];
    box_heights(Linv, h);
    for (int i = 0; i < 3; ++i) {
      const double c = floor(h[i] / rc);
      g->nc[i] = (c >= 1.0 && c < 2147483647.0) ? (int32_t)c : 0;
    }
    if (g->nc[0] < 1 || g->nc[1] < 1 || g->nc[2] < 1) return GEOM_E_SMALL;
    for (int k = 0; k < 9; ++k) {
      g->B[k] = Lred[k];
      g->Binv[k] = Linv[k];
      g->Finv[k] = Linv[k];
      g->Q[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    for (int i = 0; i < 3; ++i) {
      g->w[i] = 1.0 / g->nc[i];
      for (int j = 0; j < 3; ++j) g->cen[3 * i + j] = Lred[3 * i + j] / g->nc[j];
    }
    int q = 0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx, ++q)
          for (int i = 0; i < 3; ++i)
            g->ds_delta[q][i] = g->cen[3 * i] * dx + g->cen[3 * i + 1] * dy + g->cen[3 * i + 2] * dz;
    g->grow[0] = g->grow[1] = 1.0;
    g->inv_w[0] = g->inv_w[1] = 0.0;
  } else {
    double Q[9], R[9];
    if (!basis_qr(Lred, Q, R)) return GEOM_E_SINGULAR;
    for (int i = 0; i < 3; ++i) {
      const double l = floor(R[4 * i] / rc);
      g->nc[i] = (l >= 1.0 && l < 2147483647.0) ? (int32_t)l : 0;
    }
    if (g->nc[0] < 1 || g->nc[1] < 1 || g->nc[2] < 1) return GEOM_E_SMALL;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        g->B[3 * r + c] = R[3 * r + c];
        g->Finv[3 * r + c] = Q[3 * c + r];  // Q^T
        g->Q[3 * r + c] = Q[3 * r + c];
        g->cen[3 * r + c] = 0.0;
      }
    for (int i = 0; i < 3; ++i) {
      g->w[i] = R[4 * i] / g->nc[i];
      g->cen[4 * i] = g->w[i];
    }
    g->inv_w[0] = 1.0 / g->w[0];
    g->inv_w[1] = 1.0 / g->w[1];
    if (!mat_inv(g->B, g->Binv)) return GEOM_E_SINGULAR;
    g->grow[0] = do_tight ? rc / g->w[0] : 1.0;
    g->grow[1] = do_tight ? rc / g->w[1] : 1.0;
    for (int q = 0; q < 27; ++q) g->ds_delta[q][0] = g->ds_delta[q][1] = g->ds_delta[q][2] = 0.0;
  }
  for (int i = 0; i < 3; ++i) g->inv_nc[i] = 1.0 / (double)g->nc[i];
  return GEOM_OK;
}

// unit in the last place of an FP32 number of magnitude |x|
NCL_HD double ulp32(double x) {
  x = fabs(x);
  if (x < 1e-30) return 1e-37;
  int e;
  frexp(x, &e);  // x = f 2^e, f in [0.5, 1)
  return ldexp(1.0, e - 24);
}

// Band around rc^2 for the per-particle screen: candidates carry FP32
// offsets from their cell centre (at most half a cell diagonal per
// component, so off by half an FP32 ulp of that), compared with an FP64 home
// vector; r^2 within four times that error bound of rc^2 is re-decided from
// FP64 positions.
NCL_HD void cell_geom_bands(CellGeom* g, double rc) {
  double omax = 0.0;
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) s += 0.5 * fabs(g->cen[3 * r + c]);
    omax = fmax(omax, s);
  }
  // dynamic offset: plus the FP64 rounding of a home x placed relative to the
  // first cell of the id numbering (at most ncells w0 + 8 rc from it)
  const double big = (double)g->nc[0] * g->nc[1] * g->nc[2] * g->w[0] + 8.0 * rc;
  const double od = 0.5 * ulp32(omax) * 1.7320508075688772 + (g->variant == VAR_DO ? ldexp(big, -52) : 0.0);
  const double er = 2.0 * rc * od + od * od + 1e-15 * rc * rc;
  g->rc2_lo64 = rc * rc - 4.0 * er;
  g->rc2_hi64 = rc * rc + 4.0 * er;
}

// ---------------------------------------------------------------------------
// particle location: wrap into the box and find the cell (Sec. 4.1, 4.2)
// ---------------------------------------------------------------------------
// Returns the linear cell id a + c0 (b + c1 c), writes the wrapped position
// in the variant's frame (xw) and the lattice image n with
// x = (frame^-1 xw) + Lred n.  Non-finite input sets *bad and lands in cell 0.
NCL_HD uint32_t locate(const CellGeom& g, const double* x, double* xw, int32_t* img, bool* bad) {
  int32_t a[3];
  const bool finite = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
  if (!finite) {
    *bad = true;
    xw[0] = xw[1] = xw[2] = 0.0;
    img[0] = img[1] = img[2] = 0;
    return 0u;
  }
  if (g.variant == VAR_DS) {
    // fractional coordinates s = Lred^-1 x, wrapped into [0,1)
    double s[3], n[3];
    for (int i = 0; i < 3; ++i) s[i] = g.Finv[3 * i] * x[0] + g.Finv[3 * i + 1] * x[1] + g.Finv[3 * i + 2] * x[2];
    for (int i = 0; i < 3; ++i) {
      double fl = floor(s[i]);
      double f = s[i] - fl;
      if (f >= 1.0) { f = 0.0; fl += 1.0; }
      n[i] = fl;
      // the recorded image (pair keys only) saturates beyond 2^30
      img[i] = (int32_t)fmin(fmax(fl, -1073741824.0), 1073741824.0);
      int32_t ai = (int32_t)(f * g.nc[i]);
      a[i] = ai < 0 ? 0 : (ai >= g.nc[i] ? g.nc[i] - 1 : ai);
    }
    for (int i = 0; i < 3; ++i)
      xw[i] = x[i] - (g.B[3 * i] * n[0] + g.B[3 * i + 1] * n[1] + g.B[3 * i + 2] * n[2]);
  } else {
    // rotate (x' = Q^T x), then the rectangular rearrangement: reduce z by
    // r_z, then y by r_y, then x by r_x; the result lies in
    // [0,r11) x [0,r22) x [0,r33), a fundamental domain of the lattice.
    double y[3];
    for (int i = 0; i < 3; ++i) y[i] = g.Finv[3 * i] * x[0] + g.Finv[3 * i + 1] * x[1] + g.Finv[3 * i + 2] * x[2];
    const double k = floor(y[2] / g.B[8]);
    y[0] -= k * g.B[2];
    y[1] -= k * g.B[5];
    y[2] -= k * g.B[8];
    const double j = floor(y[1] / g.B[4]);
    y[0] -= j * g.B[1];
    y[1] -= j * g.B[4];
    const double i = floor(y[0] / g.B[0]);
    y[0] -= i * g.B[0];
    // the recorded image (pair keys only) saturates beyond 2^30
    img[0] = (int32_t)fmin(fmax(i, -1073741824.0), 1073741824.0);
    img[1] = (int32_t)fmin(fmax(j, -1073741824.0), 1073741824.0);
    img[2] = (int32_t)fmin(fmax(k, -1073741824.0), 1073741824.0);
    for (int d = 0; d < 3; ++d) {
      int32_t ad = (int32_t)floor(y[d] / g.w[d]);
      a[d] = ad < 0 ? 0 : (ad >= g.nc[d] ? g.nc[d] - 1 : ad);
      xw[d] = y[d];
    }
  }
  return (uint32_t)a[0] + (uint32_t)g.nc[0] * ((uint32_t)a[1] + (uint32_t)g.nc[1] * (uint32_t)a[2]);
}

// centre of cell (a,b,c) in the variant's frame
NCL_HD void cell_centre(const CellGeom& g, int a, int b, int c, double* out) {
  const double u[3] = {a + 0.5, b + 0.5, c + 0.5};
  for (int i = 0; i < 3; ++i) out[i] = g.cen[3 * i] * u[0] + g.cen[3 * i + 1] * u[1] + g.cen[3 * i + 2] * u[2];
}

}  // namespace ncl
