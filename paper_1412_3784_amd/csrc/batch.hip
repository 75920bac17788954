// Batched form: many independent boxes ("replicas") of uneven size, each
// with its own flow, rate and strain time, binned and swept by kernels that
// each cover every replica in one launch; plus the steps of a SLLOD
// integrator for NEMD runs of such a batch.
//
// Layout (concatenated over replicas r = 0..R-1):
//   input order   particles n_off[r] .. n_off[r+1]-1 (x, p, F as given)
//   slot order    replica r owns slots slot_off[r] .. slot_off[r+1]-1, a
//                 multiple of the 256-thread workgroup, so every sweep
//                 workgroup belongs to one replica; unused slots hold
//                 perm = PAD and are never read as neighbours
//   cells         replica r owns cells cell_off[r] .. cell_off[r+1]-1, its
//                 static capacity floor(V_r / d_cut^3) + 1 (cells never
//                 outnumber that, Sec. 4.1 / 5.2 counts), so nothing is
//                 allocated while stepping
//   geometry      one CellGeom per replica, recomputed on the device from the
//                 replica's remap policy at its current time (Sec. 2.1-2.2)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.hpp"
#include "geometry.hpp"
#include "kernels.hpp"
#include "sweep_common.hpp"

namespace ncl {

constexpr uint32_t PAD_SLOT = 0xffffffffu;

__device__ inline uint32_t find_rep(const uint32_t* __restrict__ off, uint32_t nrep, uint32_t i) {
  // last r with off[r] <= i
  uint32_t lo = 0, hi = nrep - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void kb_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// lattice of every replica at t = t0[r] + (step + off) h, on the device in FP64
__global__ void kb_prologue(BatchDev D, int off, double h) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.nrep) return;
  const double t = D.t0[r] + (double)(D.step[0] + off) * h;
  double Lred[9];
  int64_t coef[2], Mtot[9];
  remap_at(D.pol[r], t, Lred, coef);
  remap_matrix(D.pol[r], coef, Mtot);
  CellGeom g;
  const int rc = cell_geom_init(&g, Lred, Mtot, D.rc, D.variant, D.do_tight);
  int bad = 0;
  if (rc != GEOM_OK) {
    bad = rc == GEOM_E_SMALL ? 2 : 4;
  } else {
    cell_geom_bands(&g, D.rc);
    const uint64_t nc = (uint64_t)g.nc[0] * g.nc[1] * g.nc[2];
    if (nc > (uint64_t)(D.cell_off[r + 1] - D.cell_off[r])) bad = 8;
  }
  if (bad) {
    // a zero one-cell geometry marked invalid: binning puts every particle in
    // cell 0, the sweep skips the replica and writes zero forces
    atomicOr(D.err, bad);
    g = CellGeom{};
    g.nc[0] = g.nc[1] = g.nc[2] = 1;
    g.variant = -1;
  }
  D.geom[r] = g;
}

__global__ void kb_cell_index(BatchDev D, const double* __restrict__ x) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  const uint32_t r = find_rep(D.n_off, D.nrep, i);
  const double p[3] = {x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2]};
  double xw[3];
  int32_t img[3];
  bool bad = false;
  const uint32_t c = locate(D.geom[r], p, xw, img, &bad) + D.cell_off[r];
  if (bad) atomicOr(D.err, 1);
  D.cell_of[i] = c;
  D.rep[i] = r;
}

// sorted position s (replica-major, cells in order) -> slot in the
// replica's padded range
__global__ void kb_place(BatchDev D, const uint32_t* __restrict__ keys) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= D.n) return;
  const uint32_t r = find_rep(D.cell_off, D.nrep, keys[s]);
  D.perm[s + (D.slot_off[r] - D.n_off[r])] = D.rs_va[s];
}

__global__ void kb_gather(BatchDev D, const double* __restrict__ x) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= D.nslots) return;
  const uint32_t i = D.perm[s];
  if (i == PAD_SLOT) return;
  const uint32_t r = D.blk_rep[s / SW_THREADS];
  const CellGeom& g = D.geom[r];
  const double p[3] = {x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2]};
  double xw[3];
  int32_t img[3];
  bool bad = false;
  const uint32_t c = locate(g, p, xw, img, &bad);
  const int a = (int)(c % (uint32_t)g.nc[0]);
  const int b = (int)((c / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
  const int cz = (int)(c / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
  double cen[3];
  cell_centre(g, a, b, cz, cen);
  D.pos64[s] = make_double4(xw[0], xw[1], xw[2], 0.0);
  const double o[3] = {xw[0] - cen[0], xw[1] - cen[1], xw[2] - cen[2]};
  const float hi[3] = {(float)o[0], (float)o[1], (float)o[2]};
  D.pos32[s] = make_float4(hi[0], hi[1], hi[2], __uint_as_float(c));
  D.pos32lo[s] = make_float4((float)(o[0] - hi[0]), (float)(o[1] - hi[1]), (float)(o[2] - hi[2]), 0.f);
  if (D.wrap) D.wrap[s] = make_int4(img[0], img[1], img[2], 0);
}

// one thread per slot; the workgroup's replica fixes the geometry
template <int VAR, int PREC, bool DEBUG>
__global__ void __launch_bounds__(SW_THREADS) kb_sweep(SweepArgs A0, BatchDev D) {
  __shared__ float plist[PL_K * SW_THREADS_P * 3];
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t r = D.blk_rep[lb];
  const CellGeom& g = D.geom[r];
  SweepArgs A = A0;
  A.cell0 = D.cell_off[r];
  A.pad = (int32_t)(D.slot_off[r] - D.n_off[r]);
  A.jbase = D.n_off[r];
  const uint32_t s = lb * SW_THREADS + threadIdx.x;
  const uint32_t send = D.slot_off[r] + (D.n_off[r + 1] - D.n_off[r]);
  Acc<PREC, DEBUG> acc;
  uint32_t nbh = 0;
  // an invalid replica geometry, or a non-finite position anywhere (whose
  // cell could hold arbitrarily many particles): zero forces, no sweep
  const bool skip = g.variant < 0 || (D.err[0] & 1) != 0;
  if (s < send) {
    if (!skip) {
      PairList L{plist + 3 * threadIdx.x, 0};
      sweep_particle<VAR, PREC, DEBUG>(A, g, s, acc, nbh, L);
    }
    write_particle<VAR, PREC, DEBUG>(A, g, s, acc);
  }
  double v[7];
  acc_energy(acc, v);
  const uint32_t st4[4] = {acc.cand, acc.pairs, acc.fp64, nbh};
  block_commit(A, lb, v, st4);
}

// per replica: U = 1/2 sum u, W = 1/2 sum w over its workgroups, in order;
// DO rotates W back to Cartesian
__global__ void kb_finalize(BatchDev D, const double* __restrict__ partial, double* __restrict__ U,
                            double* __restrict__ W, unsigned long long* __restrict__ stats) {
  __shared__ double red[4][PART_STRIDE];
  const uint32_t r = blockIdx.x;
  const uint32_t b0 = D.slot_off[r] / SW_THREADS, b1 = D.slot_off[r + 1] / SW_THREADS;
  double v[PART_STRIDE] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (uint32_t b = b0 + threadIdx.x; b < b1; b += blockDim.x)
    for (int k = 0; k < PART_STRIDE; ++k)
      if (k != 7) v[k] += partial[PART_STRIDE * (size_t)b + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < PART_STRIDE; ++k) {
    const double t = warp_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4) {  // one addition per replica and counter (statistics are exact in FP64)
    const double c = ((red[0][8 + threadIdx.x] + red[1][8 + threadIdx.x]) + red[2][8 + threadIdx.x]) + red[3][8 + threadIdx.x];
    if (c != 0.0) atomicAdd(&stats[threadIdx.x], (unsigned long long)c);
  }
  if (threadIdx.x == 0) {
    double s[7];
    for (int k = 0; k < 7; ++k) s[k] = 0.5 * (((red[0][k] + red[1][k]) + red[2][k]) + red[3][k]);
    const CellGeom& g = D.geom[r];
    U[r] = s[0];
    const double Wp[9] = {s[1], s[4], s[5], s[4], s[2], s[6], s[5], s[6], s[3]};
    double* Wr = W + 9 * (size_t)r;
    if (g.variant == VAR_DO) {
      double T[9];
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c)
          T[3 * i + c] = g.Q[3 * i] * Wp[c] + g.Q[3 * i + 1] * Wp[3 + c] + g.Q[3 * i + 2] * Wp[6 + c];
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c)
          Wr[3 * i + c] = T[3 * i] * g.Q[3 * c] + T[3 * i + 1] * g.Q[3 * c + 1] + T[3 * i + 2] * g.Q[3 * c + 2];
    } else {
      for (int k = 0; k < 9; ++k) Wr[k] = Wp[k];
    }
  }
}

// ---------------------------------------------------------------------------
// SLLOD with peculiar momenta: dq/dt = p/m + A q, dp/dt = F - A p, split
// symmetrically per step h:
//   p <- exp(-A h/2) p ; p += (h/2) F ; q <- exp(A h) q + h phi1(A h) p/m ;
//   (new lattice, cells, F) ; p += (h/2) F ; p <- exp(-A h/2) p
// with phi1(z) = (e^z - 1)/z.  A is diagonal per replica.  Positions are put
// back into the reduced box after the drift (a lattice translation, which
// leaves peculiar momenta unchanged).
// ---------------------------------------------------------------------------
template <typename FT>
__global__ void kb_kick(BatchDev D, double* __restrict__ p, const FT* __restrict__ F, double h, double mass,
                        int second) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = D.blk_rep[s / SW_THREADS];
  const uint32_t i = (s < D.nslots) ? D.perm[s] : PAD_SLOT;
  double k2[3] = {0.0, 0.0, 0.0};
  if (i != PAD_SLOT) {
    const double* a = D.adiag + 3 * (size_t)r;
    for (int d = 0; d < 3; ++d) {
      double v = p[3 * (size_t)i + d];
      const double e = exp(-0.5 * h * a[d]);
      if (second) {
        v = (v + 0.5 * h * (double)F[3 * (size_t)i + d]) * e;
        k2[d] = v * v / mass;
      } else {
        v = v * e + 0.5 * h * (double)F[3 * (size_t)i + d];
      }
      p[3 * (size_t)i + d] = v;
    }
  }
  if (second) {
    // per-workgroup sums of p_d^2 / m (diagonal of the kinetic tensor)
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
      const double t = warp_sum(k2[d]);
      if (lane == 0) red[wid][d] = t;
    }
    __syncthreads();
    if (threadIdx.x < 3 && s - threadIdx.x < D.nslots) {
      const int d = threadIdx.x;
      D.kpart[3 * (size_t)(s / SW_THREADS) + d] = ((red[0][d] + red[1][d]) + red[2][d]) + red[3][d];
    }
  }
}

__global__ void kb_drift(BatchDev D, double* __restrict__ x, const double* __restrict__ p, double h, double mass) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= D.nslots) return;
  const uint32_t i = D.perm[s];
  if (i == PAD_SLOT) return;
  const uint32_t r = D.blk_rep[s / SW_THREADS];
  const double* a = D.adiag + 3 * (size_t)r;
  double q[3];
  for (int d = 0; d < 3; ++d) {
    const double z = a[d] * h;
    const double phi1 = (z != 0.0) ? expm1(z) / z : 1.0;
    q[d] = exp(z) * x[3 * (size_t)i + d] + h * phi1 * p[3 * (size_t)i + d] / mass;
  }
  // back into the reduced box of the new lattice: q - Lred floor(Lred^-1 q)
  double Linv[9], L[9];
  for (int k = 0; k < 9; ++k) L[k] = D.lred[9 * (size_t)r + k];
  mat_inv(L, Linv);
  double n[3];
  for (int d = 0; d < 3; ++d) n[d] = floor(Linv[3 * d] * q[0] + Linv[3 * d + 1] * q[1] + Linv[3 * d + 2] * q[2]);
  for (int d = 0; d < 3; ++d) x[3 * (size_t)i + d] = q[d] - (L[3 * d] * n[0] + L[3 * d + 1] * n[1] + L[3 * d + 2] * n[2]);
}

// reduced basis of every replica at the prologue's time (for the drift's wrap)
__global__ void kb_lattice(BatchDev D, int off, double h) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.nrep) return;
  const double t = D.t0[r] + (double)(D.step[0] + off) * h;
  int64_t coef[2];
  remap_at(D.pol[r], t, D.lred + 9 * (size_t)r, coef);
}

// per replica, after the second kick: record (t, U, W diag, K diag) at the
// current step
__global__ void kb_observe(BatchDev D, const double* __restrict__ U, const double* __restrict__ W, double h,
                           double* __restrict__ hist, uint32_t hist_cap) {
  const uint32_t r = blockIdx.x;
  __shared__ double red[4][4];
  const uint32_t b0 = D.slot_off[r] / SW_THREADS, b1 = D.slot_off[r + 1] / SW_THREADS;
  double k[3] = {0, 0, 0};
  for (uint32_t b = b0 + threadIdx.x; b < b1; b += blockDim.x)
    for (int d = 0; d < 3; ++d) k[d] += D.kpart[3 * (size_t)b + d];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    const double t = warp_sum(k[d]);
    if (lane == 0) red[wid][d] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t step = D.step[0];
    if (step < hist_cap) {
      double* o = hist + 8 * ((size_t)step * D.nrep + r);
      o[0] = D.t0[r] + (double)step * h;
      o[1] = U[r];
      o[2] = W[9 * (size_t)r];
      o[3] = W[9 * (size_t)r + 4];
      o[4] = W[9 * (size_t)r + 8];
      for (int d = 0; d < 3; ++d) o[5 + d] = ((red[0][d] + red[1][d]) + red[2][d]) + red[3][d];
    }
  }
}

__global__ void kb_step_advance(BatchDev D) {
  if (threadIdx.x == 0 && blockIdx.x == 0) D.step[0] += 1;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline uint32_t cdivb(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t batch_prologue(const BatchDev& D, int off, double h, hipStream_t st) {
  kb_prologue<<<cdivb(D.nrep, 64), 64, 0, st>>>(D, off, h);
  kb_lattice<<<cdivb(D.nrep, 64), 64, 0, st>>>(D, off, h);
  return hipGetLastError();
}

hipError_t batch_build(const BatchDev& D, const double* x, hipStream_t st) {
  kb_fill_u32<<<cdivb(D.nslots, 256), 256, 0, st>>>(D.perm, D.nslots, PAD_SLOT);
  if (D.n > 0) kb_cell_index<<<cdivb(D.n, 256), 256, 0, st>>>(D, x);
  const uint32_t* keys = D.cell_of;
  hipError_t e = radix_sort_cells(D.cell_of, D.rank, D.rs_va, D.rs_vb, D.n, D.ncells, D.rs_hist, D.rs_off,
                                  D.scan_tmp, &keys, st);
  if (e == hipSuccess) e = cell_starts(keys, D.n, D.ncells, D.cstart, st);
  if (e != hipSuccess) return e;
  if (D.n > 0) {
    kb_place<<<cdivb(D.n, 256), 256, 0, st>>>(D, keys);
    kb_gather<<<cdivb(D.nslots, 256), 256, 0, st>>>(D, x);
  }
  return hipGetLastError();
}

template <int VAR, int PREC, bool DEBUG>
static void bsweep_t(const SweepArgs& A, const BatchDev& D, hipStream_t st) {
  kb_sweep<VAR, PREC, DEBUG><<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(A, D);
}

hipError_t batch_sweep(const SweepArgs& A, const BatchDev& D, int precision, bool debug, double* U, double* W,
                       hipStream_t st) {
  kb_fill_u32<<<1, 64, 0, st>>>((uint32_t*)A.stats, 8, 0u);
  if (D.nslots > 0) {
#define NCL_BSW(V, P)                                   \
  if (D.variant == V && precision == P) {               \
    if (debug) bsweep_t<V, P, true>(A, D, st);          \
    else bsweep_t<V, P, false>(A, D, st);               \
  }
    NCL_BSW(VAR_DS, 0) NCL_BSW(VAR_DS, 1) NCL_BSW(VAR_DS, 2)
    NCL_BSW(VAR_DO, 0) NCL_BSW(VAR_DO, 1) NCL_BSW(VAR_DO, 2)
#undef NCL_BSW
  }
  kb_finalize<<<D.nrep, 256, 0, st>>>(D, A.partial, U, W, A.stats);
  return hipGetLastError();
}

hipError_t batch_kick(const BatchDev& D, double* p, const void* F, bool f64, double h, double mass, int second,
                      hipStream_t st) {
  const uint32_t nb = D.nslots / SW_THREADS;
  if (nb == 0) return hipSuccess;
  if (f64)
    kb_kick<double><<<nb, SW_THREADS, 0, st>>>(D, p, (const double*)F, h, mass, second);
  else
    kb_kick<float><<<nb, SW_THREADS, 0, st>>>(D, p, (const float*)F, h, mass, second);
  return hipGetLastError();
}

hipError_t batch_drift(const BatchDev& D, double* x, const double* p, double h, double mass, hipStream_t st) {
  if (D.nslots) kb_drift<<<cdivb(D.nslots, 256), 256, 0, st>>>(D, x, p, h, mass);
  return hipGetLastError();
}

hipError_t batch_observe(const BatchDev& D, const double* U, const double* W, double h, double* hist,
                         uint32_t hist_cap, bool advance, hipStream_t st) {
  if (advance) kb_step_advance<<<1, 64, 0, st>>>(D);
  kb_observe<<<D.nrep, 256, 0, st>>>(D, U, W, h, hist, hist_cap);
  return hipGetLastError();
}

}  // namespace ncl
