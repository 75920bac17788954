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

#include <algorithm>

#include "batch.hpp"
#include "geometry.hpp"
#include "kernels.hpp"
#include "sweep_common.hpp"

namespace ncl {

constexpr uint32_t PAD_SLOT = 0xffffffffu;

// replica of particle i (input order, or position i of the sorted keys,
// which are replica-major): the replica of its 256-particle block, then a
// short forward step (replicas hold far more particles than a block)
__device__ inline uint32_t rep_of(const BatchDev& D, uint32_t i) {
  uint32_t r = D.in_rep[i >> 8];
  while (r + 1 < D.nrep && D.n_off[r + 1] <= i) ++r;
  return r;
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
  if (D.pcur) {
    D.pcur[2 * r] = coef[0];
    D.pcur[2 * r + 1] = coef[1];
  }
  CellGeom g;
  const int rc = cell_geom_init(&g, Lred, Mtot, D.rc_cells, D.variant, D.do_tight);
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
  if (i == 0) D.cstart[D.ncells + 1] = 0u;  // no runs of empty cells queued yet
  if (i >= D.n) return;
  const uint32_t r = rep_of(D, i);
  const double p[3] = {x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2]};
  double xw[3];
  int32_t img[3];
  bool bad = false;
  uint32_t c;
  const uint32_t rf = __builtin_amdgcn_readfirstlane(r);
  if (__ballot(r != rf) == 0)  // one replica in the wave: scalar geometry loads
    c = locate(D.geom[rf], p, xw, img, &bad) + D.cell_off[rf];
  else
    c = locate(D.geom[r], p, xw, img, &bad) + D.cell_off[r];
  if (bad) atomicOr(D.err, 1);
  D.cell_of[i] = c;
}

__global__ void kb_gather(BatchDev D, const double* __restrict__ x) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= D.nslots) return;
  // a block's slots belong to one replica: its offsets and geometry are read
  // through scalar loads.  Every key lies in its replica's cell range (an
  // invalid replica's particles all in its cell 0), so the sorted positions
  // n_off[r] .. n_off[r + 1] - 1 hold replica r's particles in cell order:
  // slot s takes sorted position n_off[r] + (s - slot_off[r]); the slots past
  // the replica's count are padding.
  const uint32_t r = __builtin_amdgcn_readfirstlane(D.blk_rep[s / SW_THREADS]);
  const uint32_t q = s - D.slot_off[r];
  if (q >= D.n_off[r + 1] - D.n_off[r]) {
    D.perm[s] = PAD_SLOT;
    return;
  }
  const uint32_t i = D.rs_va[D.n_off[r] + q];
  D.perm[s] = i;
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
  if (D.wrap) D.wrap[s] = make_int4(img[0], img[1], img[2], 0);
}

// the per-particle sweep of one BT-slot block lb (BT divides 256, the
// replicas' slot padding); the replica of the block fixes the geometry
template <int VAR, int PREC, bool DEBUG, int BT = SW_THREADS>
__device__ inline void sweep_block(const SweepArgs& A0, const BatchDev& D, uint32_t lb, SweepSmemT<BT>& sm) {
  static_assert(256 % BT == 0, "blocks of a replica's padded slots");
  const uint32_t r = D.blk_rep[lb / (256 / BT)];
  const CellGeom& g = D.geom[r];
  SweepArgs A = A0;
  A.cell0 = D.cell_off[r];
  A.pad = (int32_t)(D.slot_off[r] - D.n_off[r]);
  A.jbase = D.n_off[r];
  const uint32_t s = lb * BT + threadIdx.x;
  const uint32_t send = D.slot_off[r] + (D.n_off[r + 1] - D.n_off[r]);
  Acc<PREC, DEBUG> acc;
  uint32_t nbh = 0;
  // an invalid replica geometry, or a non-finite position anywhere (whose
  // cell could hold arbitrarily many particles): zero forces, no sweep
  const bool skip = g.variant < 0 || (D.err[0] & 1) != 0;
  if (s < send) {
    if (!skip) {
      PairListS<BT> L(sm.plist + threadIdx.x);
      sweep_particle<VAR, PREC, DEBUG, true>(A, g, s, acc, nbh, L);
    }
    write_particle<VAR, PREC, DEBUG>(A, g, s, acc);
  }
  double v[7];
  acc_energy(acc, v);
  const uint32_t st4[4] = {acc.cand, acc.pairs, acc.fp64, nbh};
  block_commit<BT / 64>(A, lb, v, st4, sm.red);
}

// one thread per slot, workgroups of swp_threads(VAR) lanes (one partial
// slot each), four waves per SIMD
template <int VAR, int PREC, bool DEBUG>
__global__ void __launch_bounds__(swp_threads(VAR), 4) kb_sweep(SweepArgs A0, BatchDev D) {
  constexpr int BT = swp_threads(VAR);
  __shared__ SweepSmemT<BT> sm;
  sweep_block<VAR, PREC, DEBUG, BT>(A0, D, xcd_block(blockIdx.x, gridDim.x), sm);
}

// ---------------------------------------------------------------------------
// Fused bin + force launch.  Each workgroup takes the next item of a queue
// when it starts: first one bin item per replica (smallest replicas first),
// then the sweep items (256-slot blocks) in the same replica order.  A bin item sorts its
// whole replica inside one workgroup (a stable LSD radix sort of the cell
// keys whose digits are ranked with wave ballots in LDS; keys and values
// ping-pong through the replica's range of the staged sort buffers, which
// stay in L2), writes the replica's cell starts, slot permutation and sorted
// positions, then releases the replica's ready flag.  A sweep item waits
// (bounded) for its replica's flag and runs the per-particle sweep of its
// block.  The wait cannot deadlock: a sweep item is taken only after every
// bin item has been taken by a running workgroup, and bin items wait on
// nothing.  Workgroups are not persistent (one item each): a loop over items
// kept the sweep's invariant state live across items and spilled registers.  The replicas' geometry comes from the lattice prologue launched
// before, so no workgroup reads geometry written in this launch.
// ---------------------------------------------------------------------------
constexpr int FB_SUB = 4;                        // sub-rounds of 64 keys per wave and tile
constexpr uint32_t FB_TILE = SW_THREADS * FB_SUB;  // keys ranked per tile
constexpr uint32_t FB_SPIN_LIMIT = 1u << 20;     // polls (at least 0.2 s) before giving up

struct FusedSmem {
  uint32_t base[256];       // running output offset of each digit
  uint32_t wcnt[4][256];    // per-wave digit counts of the current tile
  uint32_t hist[4][256];    // digit histograms of up to four passes
  uint32_t item;
  int32_t wait_ok;
};
union FusedLds {
  SweepSmem sw;
  FusedSmem fb;
};

// mask of the lanes of this wave whose digit equals this lane's (valid lanes only)
__device__ inline uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t eq = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t B = __ballot(bit);
    eq &= bit ? B : ~B;
  }
  return eq;
}

__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// stable sort of n (key, value) pairs in ka/va by the low nbits of the keys;
// returns 0 if the result is in ka/va, 1 if in kb/vb
__device__ int wg_radix_sort(uint32_t* __restrict__ ka, uint32_t* __restrict__ va, uint32_t* __restrict__ kb,
                             uint32_t* __restrict__ vb, uint32_t n, int nbits, FusedSmem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int npass = (nbits + 7) / 8;
  if (npass == 0 || n == 0) return 0;
  // every pass's digit histogram from one read of the keys
  for (int q = tid; q < 4 * 256; q += SW_THREADS) (&S.hist[0][0])[q] = 0u;
  __syncthreads();
  for (uint32_t e = tid; e < n; e += SW_THREADS) {
    const uint32_t k = ka[e];
    for (int p = 0; p < npass; ++p) atomicAdd(&S.hist[p][(k >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  int cur = 0;
  for (int p = 0; p < npass; ++p) {
    const uint32_t* ks = cur ? kb : ka;
    const uint32_t* vs = cur ? vb : va;
    uint32_t* kd = cur ? ka : kb;
    uint32_t* vd = cur ? va : vb;
    const int sh = 8 * p;
    // exclusive scan of the histogram (wave 0, four digits per lane)
    if (wid == 0) {
      uint32_t h[4], sum = 0;
      for (int q = 0; q < 4; ++q) {
        h[q] = S.hist[p][4 * lane + q];
        sum += h[q];
      }
      uint32_t incl = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
      }
      uint32_t run = incl - sum;
      for (int q = 0; q < 4; ++q) {
        S.base[4 * lane + q] = run;
        run += h[q];
      }
    }
    for (int q = tid; q < 4 * 256; q += SW_THREADS) (&S.wcnt[0][0])[q] = 0u;
    __syncthreads();
    for (uint32_t t0 = 0; t0 < n; t0 += FB_TILE) {
      // wave w ranks keys t0 + 256 w + 64 q + lane, q = 0..3, in that order
      uint32_t key[FB_SUB], val[FB_SUB], dig[FB_SUB], pos[FB_SUB];
#pragma unroll
      for (int q = 0; q < FB_SUB; ++q) {
        const uint32_t e = t0 + (uint32_t)(256 * wid + 64 * q + lane);
        const bool valid = e < n;
        key[q] = valid ? ks[e] : 0u;
        val[q] = valid ? vs[e] : 0u;
        dig[q] = (key[q] >> sh) & 255u;
        const uint64_t eq = match_digit(dig[q], valid);
        const uint32_t before = S.wcnt[wid][dig[q]];  // this wave's earlier keys with the digit
        pos[q] = valid ? before + lanes_below(eq) : 0xffffffffu;
        // the highest lane of each digit group advances the wave's count
        if (valid && (eq >> lane) == 1ull) S.wcnt[wid][dig[q]] = before + (uint32_t)__popcll(eq);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < FB_SUB; ++q) {
        if (pos[q] != 0xffffffffu) {
          const uint32_t d = dig[q];
          uint32_t off = S.base[d] + pos[q];
          for (int w = 0; w < wid; ++w) off += S.wcnt[w][d];
          kd[off] = key[q];
          vd[off] = val[q];
        }
      }
      __syncthreads();
      {
        const int d = tid;  // 256 threads, one digit each
        S.base[d] += ((S.wcnt[0][d] + S.wcnt[1][d]) + S.wcnt[2][d]) + S.wcnt[3][d];
        S.wcnt[0][d] = S.wcnt[1][d] = S.wcnt[2][d] = S.wcnt[3][d] = 0u;
      }
      __syncthreads();
    }
    cur ^= 1;
  }
  return cur;
}

// bin replica r inside this workgroup
__device__ void fused_bin(const BatchDev& D, const double* __restrict__ x, uint32_t r, FusedSmem& S) {
  const int tid = threadIdx.x;
  const CellGeom& g = D.geom[r];
  const uint32_t i0 = D.n_off[r], n = D.n_off[r + 1] - i0;
  const uint32_t s0 = D.slot_off[r], ns = D.slot_off[r + 1] - s0;
  const uint32_t cell0 = D.cell_off[r];
  const uint32_t nc = (uint32_t)g.nc[0] * (uint32_t)g.nc[1] * (uint32_t)g.nc[2];
  uint32_t* ka = D.cell_of + i0;
  uint32_t* va = D.rank + i0;
  uint32_t* kb = D.rs_va + i0;
  uint32_t* vb = D.rs_vb + i0;
  // cell keys (replica-local cell ids) and local indices
  for (uint32_t k = tid; k < n; k += SW_THREADS) {
    const size_t i = (size_t)i0 + k;
    const double p[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    double xw[3];
    int32_t img[3];
    bool bad = false;
    const uint32_t c = locate(g, p, xw, img, &bad);
    if (bad) atomicOr(D.err, 1);
    ka[k] = c;
    va[k] = k;
  }
  __syncthreads();
  const int nbits = nc > 1 ? 32 - __clz((int)(nc - 1)) : 0;
  const int where = wg_radix_sort(ka, va, kb, vb, n, nbits, S);
  const uint32_t* sk = where ? kb : ka;
  const uint32_t* sv = where ? vb : va;
  // cell starts (global sorted positions, as the staged build writes them):
  // each first particle of a cell fills the cells from the previous key
  for (uint32_t s = tid; s <= n; s += SW_THREADS) {
    const uint32_t lo = s == 0 ? 0u : sk[s - 1] + 1u;
    const uint32_t hi = s == n ? nc : sk[s];
    for (uint32_t c = lo; c <= hi && (s == 0 || s == n || sk[s] != sk[s - 1]); ++c) D.cstart[cell0 + c] = i0 + s;
  }
  // the rest of the replica's cell capacity, up to the next replica's first
  // cell, holds the replica's end (as the staged build leaves it)
  const uint32_t cap = D.cell_off[r + 1] - cell0;
  for (uint32_t c = nc + 1 + tid; c <= cap; c += SW_THREADS) D.cstart[cell0 + c] = i0 + n;
  // slots: permutation and sorted positions; padding slots marked
  for (uint32_t s = tid; s < ns; s += SW_THREADS) {
    if (s >= n) {
      D.perm[s0 + s] = PAD_SLOT;
      continue;
    }
    const uint32_t i = i0 + sv[s];
    D.perm[s0 + s] = i;
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
    D.pos64[s0 + s] = make_double4(xw[0], xw[1], xw[2], 0.0);
    D.pos32[s0 + s] = make_float4((float)(xw[0] - cen[0]), (float)(xw[1] - cen[1]), (float)(xw[2] - cen[2]),
                                  __uint_as_float(c));
    if (D.wrap) D.wrap[s0 + s] = make_int4(img[0], img[1], img[2], 0);
  }
}

template <int VAR, int PREC>
__global__ void __launch_bounds__(SW_THREADS, 4) kb_fused(SweepArgs A0, BatchDev D, const double* __restrict__ x,
                                                         uint32_t* __restrict__ queue, uint32_t* __restrict__ ready,
                                                         const uint32_t* __restrict__ order,
                                                         const uint32_t* __restrict__ blk_order) {
  __shared__ FusedLds sm;
  const uint32_t R = D.nrep, nitems = R + D.nslots / SW_THREADS;
  // items in the order workgroups start, not by block index
  if (threadIdx.x == 0) sm.fb.item = atomicAdd(queue, 1u);
  __syncthreads();
  // wave-uniform (scalar registers): the geometry and ranges it selects are
  // then scalar too
  const uint32_t item = __builtin_amdgcn_readfirstlane(sm.fb.item);
  __syncthreads();
  if (item >= nitems) return;  // uniform per workgroup
  if (item < R) {
    const uint32_t r = __builtin_amdgcn_readfirstlane(order[item]);
    // a replica's build is the critical path of its sweep blocks, which may
    // be spinning on other CUs: its waves issue ahead of the sweep waves
    // sharing this CU
    __builtin_amdgcn_s_setprio(3);
    fused_bin(D, x, r, sm.fb);
    // publish the replica: every thread's writes, then the flag
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&ready[r], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const uint32_t lb = __builtin_amdgcn_readfirstlane(blk_order[item - R]);
  if (threadIdx.x == 0) {
    const uint32_t r = D.blk_rep[lb];
    uint32_t spins = 0;
    int ok = 1;
    while (__hip_atomic_load(&ready[r], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      __builtin_amdgcn_s_sleep(8);
      if (++spins > FB_SPIN_LIMIT) {
        atomicOr(D.err, 16);
        ok = 0;
        break;
      }
    }
    sm.fb.wait_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const bool waited = sm.fb.wait_ok != 0;
  __syncthreads();
  if (!waited) return;  // flagged; the replica's forces are not written
  sweep_block<VAR, PREC, false>(A0, D, lb, sm.sw);
}

// partials of one-wave workgroups -> one partial per 256-slot block, the
// four waves summed in the order a 256-lane workgroup sums them (so the
// per-replica sums do not depend on the sweep's workgroup size)
__global__ void kb_combine4(const double* __restrict__ in, uint32_t nblk, double* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblk * PART_STRIDE) return;
  const uint32_t b = i / PART_STRIDE, k = i % PART_STRIDE;
  const double* p = in + 4 * PART_STRIDE * (size_t)b + k;
  out[i] = ((p[0] + p[PART_STRIDE]) + p[2 * PART_STRIDE]) + p[3 * PART_STRIDE];
}

// per replica: U = 1/2 sum u, W = 1/2 sum w over its workgroups, in order;
// DO rotates W back to Cartesian
// cart: the partials are already Cartesian (neighbour-list forces), so the
// dynamic-offset rotation back from the cell frame is skipped
__global__ void kb_finalize(BatchDev D, const double* __restrict__ partial, double* __restrict__ U,
                            double* __restrict__ W, unsigned long long* __restrict__ stats, int cart) {
  __shared__ double red[4][PART_STRIDE];
  const uint32_t r = blockIdx.x;
  const uint32_t b0 = D.slot_off[r] / 256, b1 = D.slot_off[r + 1] / 256;
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
    if (g.variant == VAR_DO && !cart) {
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
// Per-particle kernels of the integrator walk the caller's order padded like
// the slots: position u of replica r is input index n_off[r] + (u -
// slot_off[r]) while that is below n_off[r+1], so loads and stores are
// coalesced and a workgroup never straddles two replicas.
__device__ inline uint32_t padded_input(const BatchDev& D, uint32_t u, uint32_t r) {
  const uint32_t q = u - D.slot_off[r];
  return (u < D.nslots && q < D.n_off[r + 1] - D.n_off[r]) ? D.n_off[r] + q : PAD_SLOT;
}

template <typename FT>
__global__ void kb_kick(BatchDev D, double* __restrict__ p, const FT* __restrict__ F, double h, double mass,
                        int second) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = D.blk_rep[s / SW_THREADS];
  const uint32_t i = padded_input(D, s, r);
  // the workgroup's replica's factors exp(-A h / 2), once per workgroup
  __shared__ double ek[3];
  if (threadIdx.x < 3) ek[threadIdx.x] = exp(-0.5 * h * D.adiag[3 * (size_t)r + threadIdx.x]);
  __syncthreads();
  double k2[3] = {0.0, 0.0, 0.0};
  if (i != PAD_SLOT) {
    for (int d = 0; d < 3; ++d) {
      double v = p[3 * (size_t)i + d];
      const double e = ek[d];
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

// the workgroup's replica's drift factors exp(A h) and h phi1(A h), phi1(z) =
// (e^z - 1) / z, once per workgroup (a workgroup never straddles replicas)
__device__ inline void drift_factors(const BatchDev& D, uint32_t r, double h, double* ez, double* hphi) {
  if (threadIdx.x < 3) {
    const double z = D.adiag[3 * (size_t)r + threadIdx.x] * h;
    ez[threadIdx.x] = exp(z);
    hphi[threadIdx.x] = h * ((z != 0.0) ? expm1(z) / z : 1.0);
  }
  __syncthreads();
}

// q <- exp(A h) q + h phi1(A h) p / m in the padded input order, left
// unwrapped until the next list rebuild (the cell-list steps drift and wrap
// in kb_kick_drift)
__global__ void kb_drift(BatchDev D, double* __restrict__ x, const double* __restrict__ p, double h, double mass) {
  __shared__ double ez[3], hphi[3];
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = D.blk_rep[blockIdx.x];
  drift_factors(D, r, h, ez, hphi);
  const uint32_t i = padded_input(D, s, r);
  if (i == PAD_SLOT) return;
  for (int d = 0; d < 3; ++d) x[3 * (size_t)i + d] = ez[d] * x[3 * (size_t)i + d] + hphi[d] * p[3 * (size_t)i + d] / mass;
}

// The end of step n - 1 and the start of step n in one pass (both use the
// forces of step n - 1): if kick2, p <- (p + h/2 F) exp(-A h/2) with the
// kinetic partial sums of step n - 1; then p <- p exp(-A h/2) + h/2 F and
// the drift q <- exp(A h) q + h phi1(A h) p / m into the reduced box of the
// lattice the prologue set for step n.  The arithmetic is that of a second
// kick, a first kick and a drift in that order, so the trajectory does not
// depend on the fusion; it reads x, p and F once and writes x and p once.
// A workgroup's valid slots are a prefix of it and map to consecutive input
// particles, so their coordinates are moved between HBM and LDS as three
// contiguous runs of 8-byte words (a wave's access covers 512 contiguous
// bytes, not every third word of 1.5 KB).
template <typename FT>
__global__ void kb_kick_drift(BatchDev D, double* __restrict__ x, double* __restrict__ p, const FT* __restrict__ F,
                              double h, double mass, int kick2) {
  const uint32_t t = threadIdx.x;
  const uint32_t r = D.blk_rep[blockIdx.x];
  // slots q0 .. q0 + nv - 1 of replica r are its input particles n_off[r] + q
  const uint32_t q0 = blockIdx.x * SW_THREADS - D.slot_off[r], nr = D.n_off[r + 1] - D.n_off[r];
  const uint32_t nv = q0 < nr ? min(nr - q0, (uint32_t)SW_THREADS) : 0u;
  const size_t b0 = 3 * ((size_t)D.n_off[r] + q0);
  __shared__ double sx[3 * SW_THREADS], sp[3 * SW_THREADS];
  __shared__ FT sf[3 * SW_THREADS];
  for (uint32_t k = t; k < 3 * nv; k += SW_THREADS) {
    sx[k] = x[b0 + k];
    sp[k] = p[b0 + k];
    sf[k] = F[b0 + k];
  }
  __shared__ double ek[3], ez[3], hphi[3], Ls[9], Lis[9];
  if (threadIdx.x < 3) ek[threadIdx.x] = exp(-0.5 * h * D.adiag[3 * (size_t)r + threadIdx.x]);
  // the replica's reduced basis and its inverse, once per workgroup (by the
  // second wave, beside the first wave's factors)
  static_assert(SW_THREADS > 64, "the basis is inverted by the second wave");
  if (threadIdx.x == 64) {
    double L[9], Li[9];
    for (int k = 0; k < 9; ++k) L[k] = D.lred[9 * (size_t)r + k];
    mat_inv(L, Li);
    for (int k = 0; k < 9; ++k) {
      Ls[k] = L[k];
      Lis[k] = Li[k];
    }
  }
  drift_factors(D, r, h, ez, hphi);  // synchronises the workgroup (the staged runs too)
  double k2[3] = {0.0, 0.0, 0.0};
  if (t < nv) {
    double v[3], q[3];
    for (int d = 0; d < 3; ++d) {
      const double f = (double)sf[3 * t + d];
      v[d] = sp[3 * t + d];
      if (kick2) {
        v[d] = (v[d] + 0.5 * h * f) * ek[d];
        k2[d] = v[d] * v[d] / mass;
      }
      v[d] = v[d] * ek[d] + 0.5 * h * f;
      sp[3 * t + d] = v[d];
    }
    for (int d = 0; d < 3; ++d) q[d] = ez[d] * sx[3 * t + d] + hphi[d] * v[d] / mass;
    double n[3];
    for (int d = 0; d < 3; ++d) n[d] = floor(Lis[3 * d] * q[0] + Lis[3 * d + 1] * q[1] + Lis[3 * d + 2] * q[2]);
    for (int d = 0; d < 3; ++d) sx[3 * t + d] = q[d] - (Ls[3 * d] * n[0] + Ls[3 * d + 1] * n[1] + Ls[3 * d + 2] * n[2]);
  }
  __syncthreads();
  for (uint32_t k = t; k < 3 * nv; k += SW_THREADS) {
    x[b0 + k] = sx[k];
    p[b0 + k] = sp[k];
  }
  if (kick2) {
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int d = 0; d < 3; ++d) {
      const double t = warp_sum(k2[d]);
      if (lane == 0) red[wid][d] = t;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      const int d = threadIdx.x;
      D.kpart[3 * (size_t)blockIdx.x + d] = ((red[0][d] + red[1][d]) + red[2][d]) + red[3][d];
    }
  }
}

// list steps: the slot-ordered Cartesian copy takes the same affine step
__global__ void kb_drift_slots(BatchDev D, const double* __restrict__ p, double h, double mass) {
  __shared__ double ez[3], hphi[3];
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  drift_factors(D, D.blk_rep[blockIdx.x], h, ez, hphi);
  const uint32_t i = D.perm[s];
  if (i == PAD_SLOT) return;
  const double4 y = D.ysl[s];
  const double yv[3] = {y.x, y.y, y.z};
  double yn[3];
  for (int d = 0; d < 3; ++d) yn[d] = ez[d] * yv[d] + hphi[d] * p[3 * (size_t)i + d] / mass;
  D.ysl[s] = make_double4(yn[0], yn[1], yn[2], 0.0);
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
  if (D.n > 0) kb_cell_index<<<cdivb(D.n, 256), 256, 0, st>>>(D, x);
  const uint32_t* keys = D.cell_of;
  hipError_t e = radix_sort_cells(D.cell_of, D.rank, D.rs_va, D.rs_vb, D.n, D.ncells, D.rs_hist, D.rs_off,
                                  &keys, st);
  if (e == hipSuccess) e = cell_starts(keys, D.n, D.ncells, D.cstart, st);
  // the replicas' unused cell ranges: one queued run each, filled by a
  // launch of their own (measured faster here than inside kb_gather)
  if (e == hipSuccess) e = fill_empty_runs(D.cstart, D.ncells, st);
  if (e != hipSuccess) return e;
  if (D.nslots > 0) kb_gather<<<cdivb(D.nslots, 256), 256, 0, st>>>(D, x);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Verlet lists with a skin (neighbour lists reused between rebuilds).
// Between two rebuilds at t_b and t no remap occurs, so the reduced lattice
// is L(t) = E L(t_b) with E = exp(A (t - t_b)) (diagonal), and the unwrapped
// positions are x(t) = E x(t_b) + delta.  A pair (i, j, m) then has
// r(t) = E r(t_b) + delta_j - delta_i, so every pair closer than d_cut at t
// was closer than d_cut + skin at t_b as long as
//   max_k exp(-a_k (t - t_b)) (d_cut + 2 max|delta|) < d_cut + skin.
// Entry k of slot s sits at ((k / 4) * nslots + s) * 4 + k % 4: a lane
// appends to its own 32-byte group, and a wave reading group k / 4 of 64
// consecutive slots reads one contiguous 2 KB block.  An entry is the
// neighbour's slot and its lattice image m (three 10-bit biased components), with r = y_j - y_i + L m for the slot-ordered Cartesian
// positions y, which are the wrapped positions at the rebuild advanced by the
// same drift as the caller's positions (y - x stays a lattice vector).
// ---------------------------------------------------------------------------
__device__ inline uint32_t pack_image(int m0, int m1, int m2) {
  return ((uint32_t)(m0 + 512) & 0x3ffu) | (((uint32_t)(m1 + 512) & 0x3ffu) << 10) |
         (((uint32_t)(m2 + 512) & 0x3ffu) << 20);
}

// positions into the current reduced box (input order)
__global__ void kb_wrap(BatchDev D, double* __restrict__ x) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  const uint32_t r = rep_of(D, i);
  double L[9], Linv[9];
  for (int k = 0; k < 9; ++k) L[k] = D.lred[9 * (size_t)r + k];
  mat_inv(L, Linv);
  double q[3], n[3];
  for (int d = 0; d < 3; ++d) q[d] = x[3 * (size_t)i + d];
  if (!(isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]))) return;
  for (int d = 0; d < 3; ++d) n[d] = floor(Linv[3 * d] * q[0] + Linv[3 * d + 1] * q[1] + Linv[3 * d + 2] * q[2]);
  for (int d = 0; d < 3; ++d) x[3 * (size_t)i + d] = q[d] - (L[3 * d] * n[0] + L[3 * d + 1] * n[1] + L[3 * d + 2] * n[2]);
}

// group g of slot s's list entries <- this lane's four staged entries
__device__ inline void store_group(const BatchDev& D, uint32_t s, uint32_t grp, const uint2 (*stage)[SW_THREADS]) {
  const uint32_t t = threadIdx.x;
  uint4* dst = reinterpret_cast<uint4*>(D.vl + (((size_t)grp * D.nslots + s) << 2));
  dst[0] = make_uint4(stage[0][t].x, stage[0][t].y, stage[1][t].x, stage[1][t].y);
  dst[1] = make_uint4(stage[2][t].x, stage[2][t].y, stage[3][t].x, stage[3][t].y);
}

// neighbour lists within d_cut + skin (the cut-off the cells were built for),
// from the FP64 wrapped positions, both directions of every pair
template <int VAR>
__global__ void __launch_bounds__(SW_THREADS) kb_list_build(BatchDev D) {
  // entries are staged per lane in LDS (entry q of the open group of lane t
  // at stage[q][t]) and stored a whole 32-byte group at a time
  __shared__ uint2 stage[4][SW_THREADS];
  // XCD-aware block order: neighbouring slots share an L2
  const uint32_t s = xcd_block(blockIdx.x, gridDim.x) * SW_THREADS + threadIdx.x;
  if (s >= D.nslots) return;
  const uint32_t r = D.blk_rep[s / SW_THREADS];
  const uint32_t send = D.slot_off[r] + (D.n_off[r + 1] - D.n_off[r]);
  if (s >= send) return;
  const CellGeom& g = D.geom[r];
  uint32_t cnt = 0;
  const uint32_t kmax = D.kmax;
  if (g.variant >= 0 && !(D.err[0] & 1)) {
    const uint32_t cell0 = D.cell_off[r], pad = D.slot_off[r] - D.n_off[r];
    const double rl2 = D.rc_cells * D.rc_cells;
    const double4 pi = D.pos64[s];
    const uint32_t hc = __float_as_uint(D.pos32[s].w);
    // slot-ordered Cartesian position for the force passes
    if (g.variant == VAR_DO) {
      D.ysl[s] = make_double4(g.Q[0] * pi.x + g.Q[1] * pi.y + g.Q[2] * pi.z,
                              g.Q[3] * pi.x + g.Q[4] * pi.y + g.Q[5] * pi.z,
                              g.Q[6] * pi.x + g.Q[7] * pi.y + g.Q[8] * pi.z, 0.0);
    } else {
      D.ysl[s] = pi;
    }
    const int l0 = g.nc[0], l1 = g.nc[1], l2 = g.nc[2];
    const int a = (int)(hc % (uint32_t)l0);
    const int b = (int)((hc / (uint32_t)l0) % (uint32_t)l1);
    const int c = (int)(hc / ((uint32_t)l0 * (uint32_t)l1));
    // every slot of local cells [c0, c1) seen through image m
    auto visit = [&](uint32_t c0, uint32_t c1, int m0, int m1, int m2) {
      const double sx = g.B[0] * m0 + g.B[1] * m1 + g.B[2] * m2;
      const double sy = g.B[3] * m0 + g.B[4] * m1 + g.B[5] * m2;
      const double sz = g.B[6] * m0 + g.B[7] * m1 + g.B[8] * m2;
      const double xo = pi.x - sx, yo = pi.y - sy, zo = pi.z - sz;
      const bool zero = (m0 | m1 | m2) == 0;
      const uint32_t st = D.cstart[cell0 + c0] + pad, en = D.cstart[cell0 + c1] + pad;
      const uint32_t self = zero ? s : 0xffffffffu;
      // four candidate loads in flight per step (indices past the run are
      // clamped to its last particle and masked out); entries keep the
      // candidates' order
      for (uint32_t j0 = st; j0 < en; j0 += 4) {
        double4 pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = D.pos64[min(j0 + u, en - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t js = j0 + u;
          const double dx = pj[u].x - xo, dy = pj[u].y - yo, dz = pj[u].z - zo;
          if (fma(dz, dz, fma(dy, dy, dx * dx)) < rl2 && js < en && js != self) {
            if (cnt < kmax) {
              stage[cnt & 3u][threadIdx.x] = make_uint2(js, pack_image(m0, m1, m2));
              if ((cnt & 3u) == 3u) store_group(D, s, cnt >> 2, stage);
            }
            ++cnt;
          }
        }
      }
    };
    if (VAR == VAR_DS) {
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int u[3] = {a + dx, b + dy, c + dz};
            int m[3], w[3];
            for (int k = 0; k < 3; ++k) {
              m[k] = idiv_floor32(u[k], g.nc[k]);
              w[k] = u[k] - m[k] * g.nc[k];
            }
            const uint32_t cj = (uint32_t)w[0] + (uint32_t)l0 * ((uint32_t)w[1] + (uint32_t)l1 * (uint32_t)w[2]);
            visit(cj, cj + 1, m[0], m[1], m[2]);
          }
    } else {
      for (int dz = -1; dz <= 1; ++dz) {
        const int C = c + dz;
        const int k = idiv_floor32(C, l2);
        const int cz = C - k * l2;
        const double fy = -(double)k * g.B[5] / g.w[1];
        const int B0 = (int)floor(b - g.grow[1] + fy);
        const int B1 = (int)ceil(b + 1 + g.grow[1] + fy) - 1;
        for (int Bq = B0; Bq <= B1; ++Bq) {
          const int j = idiv_floor32(Bq, l1);
          const int by = Bq - j * l1;
          const double fx = -((double)j * g.B[1] + (double)k * g.B[2]) / g.w[0];
          const int A0 = (int)floor(a - g.grow[0] + fx);
          const int A1 = (int)ceil(a + 1 + g.grow[0] + fx) - 1;
          const uint32_t rowbase = (uint32_t)l0 * ((uint32_t)by + (uint32_t)l1 * (uint32_t)cz);
          for (int i = idiv_floor32(A0, l0); i <= idiv_floor32(A1, l0); ++i) {
            const int axlo = max(A0 - i * l0, 0), axhi = min(A1 - i * l0, l0 - 1);
            visit(rowbase + (uint32_t)axlo, rowbase + (uint32_t)axhi + 1, i, j, k);
          }
        }
      }
    }
    // the open group (entries past cnt are never read); kmax is a multiple
    // of four, so an open group exists only below kmax
    if (cnt < kmax && (cnt & 3u) != 0u) store_group(D, s, cnt >> 2, stage);
    if (cnt > kmax) atomicOr(D.need, 4u);
  }
  D.vl_cnt[s] = cnt < kmax ? cnt : kmax;
}

// largest |x - E x_b| per replica (slot order: a workgroup never straddles
// two replicas; one atomic per workgroup on the replica's counter)
__global__ void __launch_bounds__(SW_THREADS) kb_disp(BatchDev D, const double* __restrict__ x, int off, double h) {
  __shared__ double red[SW_THREADS / 64];
  const uint32_t s = blockIdx.x * SW_THREADS + threadIdx.x;
  const uint32_t r = D.blk_rep[blockIdx.x];
  const uint32_t i = padded_input(D, s, r);
  double d = 0.0;
  if (i != PAD_SLOT) {
    const double dt = D.t0[r] + (double)(D.step[0] + off) * h - D.tb[r];
    double e2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double u = x[3 * (size_t)i + k] - exp(D.adiag[3 * (size_t)r + k] * dt) * D.xb[3 * (size_t)i + k];
      e2 = fma(u, u, e2);
    }
    d = sqrt(e2);
    if (!(d == d)) d = 1e300;  // a non-finite position forces a rebuild (which flags it)
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_down(d, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < SW_THREADS / 64; ++w) d = fmax(d, red[w]);
    atomicMax(&D.dmax[r], (unsigned long long)__double_as_longlong(d));
  }
}

// per replica: does the skin still cover the interval since the last
// rebuild, and has no remap occurred?  (bit 0: skin, bit 1: remap)
__global__ void kb_need(BatchDev D, int off, double h, double skin) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.nrep) return;
  const double dt = D.t0[r] + (double)(D.step[0] + off) * h - D.tb[r];
  double emax = 0.0;
  for (int k = 0; k < 3; ++k) emax = fmax(emax, exp(-D.adiag[3 * (size_t)r + k] * dt));
  const double dm = __longlong_as_double((long long)D.dmax[r]);
  uint32_t need = 0;
  if (!(emax * (D.rc + 2.0 * dm) < D.rc + skin)) need |= 1u;
  if (D.pcur[2 * r] != D.pb[2 * r] || D.pcur[2 * r + 1] != D.pb[2 * r + 1]) need |= 2u;
  if (need) atomicOr(D.need, need);
}

// record the state of a rebuild: positions, time and remap coefficients
__global__ void kb_mark(BatchDev D, const double* __restrict__ x, int off, double h) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < 3 * (size_t)D.n) D.xb[i] = x[i];
  if (i < D.nrep) {
    D.tb[i] = D.t0[i] + (double)(D.step[0] + off) * h;
    D.pb[2 * i] = D.pcur[2 * i];
    D.pb[2 * i + 1] = D.pcur[2 * i + 1];
  }
}

// forces, energy and virial from the lists at the current positions and
// lattice; separations in FP64 from the slot-ordered positions.  Entries are
// taken four at a time (their neighbour loads issued together), and the 27
// lattice shifts L m with m in {-1,0,1}^3 come from LDS.
template <int PREC>
__global__ void __launch_bounds__(SW_THREADS) kb_list_force(SweepArgs A, BatchDev D) {
  __shared__ double shift[27][3];
  // XCD-aware block order: the neighbours of a range of slots stay in one L2
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t r = D.blk_rep[lb];
  const CellGeom& g = D.geom[r];
  double L[9];
  for (int k = 0; k < 9; ++k) L[k] = D.lred[9 * (size_t)r + k];
  if (threadIdx.x < 27) {
    const int m0 = (int)(threadIdx.x % 3) - 1, m1 = (int)((threadIdx.x / 3) % 3) - 1, m2 = (int)(threadIdx.x / 9) - 1;
    for (int d = 0; d < 3; ++d) shift[threadIdx.x][d] = L[3 * d] * m0 + L[3 * d + 1] * m1 + L[3 * d + 2] * m2;
  }
  __syncthreads();
  const uint32_t s = lb * SW_THREADS + threadIdx.x;
  const uint32_t send = D.slot_off[r] + (D.n_off[r + 1] - D.n_off[r]);
  Acc<PREC, false> acc;
  if (s < send) {
    if (g.variant >= 0 && !(D.err[0] & 1)) {
      const double4 yi = D.ysl[s];
      const uint32_t n = D.vl_cnt[s];
      const uint4* grp = reinterpret_cast<const uint4*>(D.vl);
      // the next group's entries are loaded while the current group's
      // neighbours are evaluated (the last prefetch re-reads group 0)
      uint4 n01 = make_uint4(0u, 0u, 0u, 0u), n23 = n01;
      if (n > 0) {
        n01 = grp[(size_t)s * 2];
        n23 = grp[(size_t)s * 2 + 1];
      }
      for (uint32_t k0 = 0; k0 < n; k0 += 4) {
        const uint4 e01 = n01, e23 = n23;
        const size_t gn = ((size_t)((k0 + 4 < n ? k0 + 4 : 0) >> 2) * D.nslots + s) * 2;
        n01 = grp[gn];
        n23 = grp[gn + 1];
        const uint32_t js[4] = {e01.x, e01.z, e23.x, e23.z}, mc[4] = {e01.y, e01.w, e23.y, e23.w};
        double4 yj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) yj[u] = D.ysl[(k0 + u < n) ? js[u] : s];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (k0 + u >= n) break;
          const int m0 = (int)(mc[u] & 0x3ffu) - 512, m1 = (int)((mc[u] >> 10) & 0x3ffu) - 512,
                    m2 = (int)((mc[u] >> 20) & 0x3ffu) - 512;
          double sx, sy, sz;
          if (((unsigned)(m0 + 1) | (unsigned)(m1 + 1) | (unsigned)(m2 + 1)) <= 2u) {
            const int q = (m0 + 1) + 3 * (m1 + 1) + 9 * (m2 + 1);
            sx = shift[q][0];
            sy = shift[q][1];
            sz = shift[q][2];
          } else {
            sx = L[0] * m0 + L[1] * m1 + L[2] * m2;
            sy = L[3] * m0 + L[4] * m1 + L[5] * m2;
            sz = L[6] * m0 + L[7] * m1 + L[8] * m2;
          }
          const double dx = yj[u].x - yi.x + sx, dy = yj[u].y - yi.y + sy, dz = yj[u].z - yi.z + sz;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          acc.cand += 1;
          if (r2 < A.rc2) {
            if (PREC == 0 || r2 < A.rclose2_64)
              pair64(acc, A.p64, dx, dy, dz, r2);
            else
              pair32(acc, A.p32, A.p64, (float)dx, (float)dy, (float)dz, (float)r2, r2);
            acc.pairs += 1;
          }
        }
      }
    }
    write_particle<VAR_DS, PREC, false>(A, g, s, acc);  // Cartesian frame: no rotation
  }
  double v[7];
  acc_energy(acc, v);
  const uint32_t st4[4] = {acc.cand, acc.pairs, 0u, 0u};
  block_commit(A, lb, v, st4);
}

template <int VAR, int PREC, bool DEBUG>
static void bsweep_t(const SweepArgs& A, const BatchDev& D, hipStream_t st) {
  kb_sweep<VAR, PREC, DEBUG><<<D.nslots / swp_threads(VAR), swp_threads(VAR), 0, st>>>(A, D);
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
  const double* part = A.partial;
  static_assert(256 / SWP_MIN_THREADS == 4, "kb_combine4 sums four one-wave partials");
  if (swp_threads(D.variant) == SWP_MIN_THREADS && D.nslots > 0) {
    // the combined partials follow the one-wave ones (nslots / 64 slots)
    double* comb = A.partial + PART_STRIDE * (size_t)(D.nslots / SWP_MIN_THREADS);
    const uint32_t nblk = D.nslots / 256;
    kb_combine4<<<cdivb((uint64_t)nblk * PART_STRIDE, 256), 256, 0, st>>>(A.partial, nblk, comb);
    part = comb;
  }
  kb_finalize<<<D.nrep, 256, 0, st>>>(D, part, U, W, A.stats, 0);
  return hipGetLastError();
}

__global__ void kb_copy_f64(double* dst, const double* src, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t batch_copy(double* dst, const double* src, uint64_t n, hipStream_t st) {
  if (n > 0) kb_copy_f64<<<cdivb(n, 256), 256, 0, st>>>(dst, src, n);
  return hipGetLastError();
}

template <int VAR, int PREC>
static hipError_t fused_t(const SweepArgs& A, const BatchDev& D, const double* x, uint32_t* fstate,
                          const uint32_t* order, const uint32_t* blk_order, hipStream_t st) {
  // one workgroup per item; each takes the next item from the queue
  const uint32_t nitems = D.nrep + D.nslots / SW_THREADS;
  kb_fused<VAR, PREC><<<nitems, SW_THREADS, 0, st>>>(A, D, x, fstate, fstate + 1, order, blk_order);
  return hipGetLastError();
}

// fused bin + force of every replica (the lattice prologue must have run):
// fstate holds the queue counter and one ready flag per replica
hipError_t batch_fused(const SweepArgs& A, const BatchDev& D, const double* x, int precision, uint32_t* fstate,
                       const uint32_t* order, const uint32_t* blk_order, double* U, double* W, hipStream_t st) {
  kb_fill_u32<<<1, 64, 0, st>>>((uint32_t*)A.stats, 8, 0u);
  kb_fill_u32<<<cdivb(D.nrep + 1, 256), 256, 0, st>>>(fstate, D.nrep + 1, 0u);
  if (D.nslots > 0) {
    hipError_t e = hipSuccess;
    if (D.variant == VAR_DS && precision == 0) e = fused_t<VAR_DS, 0>(A, D, x, fstate, order, blk_order, st);
    if (D.variant == VAR_DS && precision == 1) e = fused_t<VAR_DS, 1>(A, D, x, fstate, order, blk_order, st);
    if (D.variant == VAR_DS && precision == 2) e = fused_t<VAR_DS, 2>(A, D, x, fstate, order, blk_order, st);
    if (D.variant == VAR_DO && precision == 0) e = fused_t<VAR_DO, 0>(A, D, x, fstate, order, blk_order, st);
    if (D.variant == VAR_DO && precision == 1) e = fused_t<VAR_DO, 1>(A, D, x, fstate, order, blk_order, st);
    if (D.variant == VAR_DO && precision == 2) e = fused_t<VAR_DO, 2>(A, D, x, fstate, order, blk_order, st);
    if (e != hipSuccess) return e;
  }
  kb_finalize<<<D.nrep, 256, 0, st>>>(D, A.partial, U, W, A.stats, 0);
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

hipError_t batch_kick_drift(const BatchDev& D, double* x, double* p, const void* F, bool f64, double h, double mass,
                            bool kick2, hipStream_t st) {
  const uint32_t nb = D.nslots / SW_THREADS;
  if (nb == 0) return hipSuccess;
  if (f64)
    kb_kick_drift<double><<<nb, SW_THREADS, 0, st>>>(D, x, p, (const double*)F, h, mass, kick2 ? 1 : 0);
  else
    kb_kick_drift<float><<<nb, SW_THREADS, 0, st>>>(D, x, p, (const float*)F, h, mass, kick2 ? 1 : 0);
  return hipGetLastError();
}

hipError_t batch_drift(const BatchDev& D, double* x, const double* p, double h, double mass, hipStream_t st) {
  if (D.nslots) {
    kb_drift<<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(D, x, p, h, mass);
    kb_drift_slots<<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(D, p, h, mass);
  }
  return hipGetLastError();
}

hipError_t batch_observe(const BatchDev& D, const double* U, const double* W, double h, double* hist,
                         uint32_t hist_cap, bool advance, hipStream_t st) {
  if (advance) kb_step_advance<<<1, 64, 0, st>>>(D);
  kb_observe<<<D.nrep, 256, 0, st>>>(D, U, W, h, hist, hist_cap);
  return hipGetLastError();
}


// Verlet lists: rebuild (wrap, cells for d_cut + skin, lists, mark) and the
// per-step check; the caller reads D.need on the host between the two
hipError_t batch_list_rebuild(const BatchDev& D, double* x, int off, double h, hipStream_t st) {
  if (D.n > 0) kb_wrap<<<cdivb(D.n, 256), 256, 0, st>>>(D, x);
  hipError_t e = batch_build(D, x, st);
  if (e != hipSuccess) return e;
  if (D.nslots) {
    if (D.variant == VAR_DS) kb_list_build<VAR_DS><<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(D);
    else kb_list_build<VAR_DO><<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(D);
  }
  const size_t nm = 3 * (size_t)D.n > D.nrep ? 3 * (size_t)D.n : D.nrep;
  kb_mark<<<(uint32_t)((nm + 255) / 256), 256, 0, st>>>(D, x, off, h);
  return hipGetLastError();
}

hipError_t batch_wrap(const BatchDev& D, double* x, hipStream_t st) {
  if (D.n > 0) kb_wrap<<<cdivb(D.n, 256), 256, 0, st>>>(D, x);
  return hipGetLastError();
}

hipError_t batch_list_check(const BatchDev& D, const double* x, int off, double h, double skin, hipStream_t st) {
  kb_fill_u32<<<cdivb(2 * D.nrep, 256), 256, 0, st>>>((uint32_t*)D.dmax, 2 * D.nrep, 0u);
  if (D.nslots) kb_disp<<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(D, x, off, h);
  kb_need<<<cdivb(D.nrep, 64), 64, 0, st>>>(D, off, h, skin);
  return hipGetLastError();
}

hipError_t batch_list_force(const SweepArgs& A, const BatchDev& D, int precision, double* U, double* W,
                            hipStream_t st) {
  kb_fill_u32<<<1, 64, 0, st>>>((uint32_t*)A.stats, 8, 0u);
  if (D.nslots) {
    if (precision == 0) kb_list_force<0><<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(A, D);
    else if (precision == 2) kb_list_force<2><<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(A, D);
    else kb_list_force<1><<<D.nslots / SW_THREADS, SW_THREADS, 0, st>>>(A, D);
  }
  kb_finalize<<<D.nrep, 256, 0, st>>>(D, A.partial, U, W, A.stats, 1);
  return hipGetLastError();
}

}  // namespace ncl
