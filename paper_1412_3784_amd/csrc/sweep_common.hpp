// Device-side pieces shared by the single-box and the batched kernels: the
// per-particle accumulators, the pair force (Sec. 3: zero past the cut-off),
// the visit of one neighbour cell, the per-particle neighbourhood sweep of
// both cell-list variants (Sec. 4.1, 4.2), and fixed-order reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "geometry.hpp"
#include "kernels.hpp"

namespace ncl {

constexpr int SW_THREADS = 256;
constexpr int SCAN_THREADS = 256;

// blockIdx -> logical block so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of cells and keeps
// its neighbour data in its own L2.
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nb) {
  const uint32_t nx = 8, per = nb / nx, rem = nb % nx;
  const uint32_t x = bid % nx, idx = bid / nx;
  return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}


__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[SCAN_THREADS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < SCAN_THREADS / 64; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}


// order-independent pair key hash: SplitMix64's output function (Steele, Lea
// & Flood 2014) on (j << 32) | three 10-bit biased image components
__device__ inline uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <int PREC, bool DEBUG>
struct Acc {
  // FP32 modes: per-particle FP32 force and virial sums (+ Kahan terms for
  // the force); the energy of every pair is summed in FP64 in gu (the half
  // list also keeps the forces of its FP64-path pairs in gx, gy, gz).  FP64
  // mode uses only the double fields.
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float kx = 0.f, ky = 0.f, kz = 0.f;
  float w[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  double gx = 0.0, gy = 0.0, gz = 0.0, gu = 0.0;
  double gw[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  uint32_t cand = 0, pairs = 0, fp64 = 0;
  int64_t dcount = 0;
  uint64_t dhash = 0;
};

__device__ inline void kahan_add(float& s, float& c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// one FP64 pair (FP64 mode, and the FP32 modes' band / close pairs)
template <int PREC, bool DEBUG>
__device__ inline void pair64(Acc<PREC, DEBUG>& acc, const Pot64& p, double dx, double dy, double dz, double r2) {
  const double r2i = 1.0 / r2;
  const double s2 = p.sig2 * r2i;
  const double s6 = s2 * s2 * s2;
  const double fs = r2i * s6 * (p.eps48 * s6 - p.eps24);
  const double phi = s6 * (p.eps4 * s6 - p.eps4) - p.shift;
  if (PREC == 0) {
    acc.gx -= fs * dx;
    acc.gy -= fs * dy;
    acc.gz -= fs * dz;
  } else if (PREC == 2) {
    kahan_add(acc.fx, acc.kx, (float)(-fs * dx));
    kahan_add(acc.fy, acc.ky, (float)(-fs * dy));
    kahan_add(acc.fz, acc.kz, (float)(-fs * dz));
  } else {
    // FP32 modes: the pair's force is rounded once and joins the FP32 sums
    // (the tolerance is relative to sum_j |f_ij|, which holds this pair);
    // the energy keeps an FP64 sum, its bound being 1e-7 of sum |u|
    acc.fx += (float)(-fs * dx);
    acc.fy += (float)(-fs * dy);
    acc.fz += (float)(-fs * dz);
  }
  acc.gu += phi;
  if (PREC == 0) {
    acc.gw[0] += fs * dx * dx;
    acc.gw[1] += fs * dy * dy;
    acc.gw[2] += fs * dz * dz;
    acc.gw[3] += fs * dx * dy;
    acc.gw[4] += fs * dx * dz;
    acc.gw[5] += fs * dy * dz;
  } else {
    acc.w[0] += (float)(fs * dx * dx);
    acc.w[1] += (float)(fs * dy * dy);
    acc.w[2] += (float)(fs * dz * dz);
    acc.w[3] += (float)(fs * dx * dy);
    acc.w[4] += (float)(fs * dx * dz);
    acc.w[5] += (float)(fs * dy * dz);
  }
}

// Pair energy of the FP32 modes, evaluated in FP64 from r^2: the FP32
// reciprocal r2i of r^2 is refined by one Newton step (relative error about
// 1e-14).  The shifted energy cancels to zero at the cut-off (for WCA every
// pair sits near it), where an FP32 evaluation is off by ~1e-8 eps per pair
// with a bias that does not average out; the 1e-7 energy bound (relative to
// sum |u_i|) then fails for boxes whose pairs are all near r_c.
__device__ inline double phi64(const Pot64& p, double r2, float r2i) {
  double y = (double)r2i;
  y = fma(y, fma(-r2, y, 1.0), y);
  const double s2 = p.sig2 * y;
  const double s6 = s2 * s2 * s2;
  return fma(s6, fma(p.eps4, s6, -p.eps4), -p.shift);
}

// one FP32 pair: force and virial in FP32 from the FP32 separation and r2
// (r^2 rounded once from an FP64 value), energy in FP64 from r2e, the FP64
// r^2 where the caller has it (else r2 widened); the force is added to
// (bx, by, bz) in FP32
template <int PREC, bool DEBUG>
__device__ inline void pair32_to(Acc<PREC, DEBUG>& acc, const Pot32& p, const Pot64& p64, float dx, float dy,
                                 float dz, float r2, double r2e, float& bx, float& by, float& bz) {
  const float r2i = __builtin_amdgcn_rcpf(r2);
  const float s2 = p.sig2 * r2i;
  const float s6 = s2 * s2 * s2;
  const float fs = r2i * s6 * fmaf(p.eps48, s6, -p.eps24);
  bx = fmaf(-fs, dx, bx);
  by = fmaf(-fs, dy, by);
  bz = fmaf(-fs, dz, bz);
  acc.gu += phi64(p64, r2e, r2i);
  const float fdx = fs * dx, fdy = fs * dy;
  acc.w[0] = fmaf(fdx, dx, acc.w[0]);
  acc.w[1] = fmaf(fdy, dy, acc.w[1]);
  acc.w[2] = fmaf(fs * dz, dz, acc.w[2]);
  acc.w[3] = fmaf(fdx, dy, acc.w[3]);
  acc.w[4] = fmaf(fdx, dz, acc.w[4]);
  acc.w[5] = fmaf(fdy, dz, acc.w[5]);
}

// one FP32 pair into the particle's sums (Kahan mode: compensated)
template <int PREC, bool DEBUG>
__device__ inline void pair32(Acc<PREC, DEBUG>& acc, const Pot32& p, const Pot64& p64, float dx, float dy, float dz,
                              float r2, double r2e) {
  if (PREC == 2) {
    float bx = 0.f, by = 0.f, bz = 0.f;
    pair32_to(acc, p, p64, dx, dy, dz, r2, r2e, bx, by, bz);
    kahan_add(acc.fx, acc.kx, bx);
    kahan_add(acc.fy, acc.ky, by);
    kahan_add(acc.fz, acc.kz, bz);
  } else {
    pair32_to(acc, p, p64, dx, dy, dz, r2, r2e, acc.fx, acc.fy, acc.fz);
  }
}

template <bool DEBUG>
__device__ inline void debug_pair(int64_t& cnt, uint64_t& hsh, const SweepArgs& A, const CellGeom& g, uint32_t j,
                                  const int* mcell, const int4& wi) {
  if (!DEBUG) return;
  const int4 wj = A.wrap[j];
  // image relative to the positions as given: x_j + Lred m - x_i
  const int64_t m[3] = {(int64_t)mcell[0] - wj.x + wi.x, (int64_t)mcell[1] - wj.y + wi.y,
                        (int64_t)mcell[2] - wj.z + wi.z};
  int64_t mk[3];
  for (int r = 0; r < 3; ++r) mk[r] = g.Mtot[3 * r] * m[0] + g.Mtot[3 * r + 1] * m[1] + g.Mtot[3 * r + 2] * m[2];
  uint64_t key = ((uint64_t)(A.perm[j] - A.jbase)) << 32;
  key |= ((uint64_t)((mk[0] + 512) & 0x3ff)) << 20;
  key |= ((uint64_t)((mk[1] + 512) & 0x3ff)) << 10;
  key |= ((uint64_t)((mk[2] + 512) & 0x3ff));
  hsh += splitmix_out(key);
  cnt += 1;
}

// Per-lane list of in-range pairs waiting for evaluation (LDS, entry e of
// lane t at base[e * S + t] for a workgroup of S lanes); evaluated by whole
// waves so that no lane runs the pair code alone.  An entry holds the separation in FP32 and
// r^2 rounded once from the FP64 screening value: recomputing r^2 from the
// three rounded components instead would add their rounding, which the WCA
// force near its cut-off (|f'| about 75 eps/sigma^2 at r = 1.11 sigma)
// magnifies to ~1e-5 eps/sigma for an isolated pair.  `q` is the lane's next
// free entry; the pairs are counted when the list is evaluated.
//
// Pairs that need the FP64 path (within the rounding band of d_cut, or
// closer than the close-pair radius) wait at the other end of the same
// list, from entry PL_K - 1 down, holding the neighbour's slot and lattice
// image; they are evaluated when the particle's sweep ends (or when they
// and the ordinary entries leave no room), all lanes together.  Evaluated
// where they are met, the wave ran the FP64 path once for every lane that
// met one (about 0.3 close pairs per particle in a uniform random liquid).
constexpr int PL_K = 10;
constexpr int SW_THREADS_P = 256;
typedef float pl_entry __attribute__((ext_vector_type(4)));      // (d_x, d_y, d_z, r^2)
typedef __attribute__((address_space(3))) pl_entry lds_entry;  // 32-bit LDS pointer
// S: lanes of the workgroup (the stride between a lane's entries)
template <int S>
struct PairListS {
  static constexpr int stride = S;  // in entries
  lds_entry* base;
  lds_entry* q;    // next ordinary entry (growing up)
  lds_entry* top;  // last FP64-path entry (growing down from base + PL_K)
  __device__ explicit PairListS(pl_entry* p)
      : base((lds_entry*)p), q((lds_entry*)p), top((lds_entry*)p + PL_K * S) {}
};
using PairList = PairListS<SW_THREADS_P>;

// lattice image of a deferred pair, three 10-bit biased components
__device__ inline uint32_t pack_image(const int* m) {
  return ((uint32_t)(m[0] + 512) & 0x3ffu) | (((uint32_t)(m[1] + 512) & 0x3ffu) << 10) |
         (((uint32_t)(m[2] + 512) & 0x3ffu) << 20);
}

// a pair within the rounding band or closer than the close-pair radius:
// decided and evaluated from the FP64 wrapped positions exactly as FP64 mode
template <int PREC, bool DEBUG>
__device__ inline void exact_pair(Acc<PREC, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, uint32_t s,
                                  uint32_t j, uint32_t code, const int4& wi) {
  const int m[3] = {(int)(code & 0x3ffu) - 512, (int)((code >> 10) & 0x3ffu) - 512, (int)((code >> 20) & 0x3ffu) - 512};
  const double sx = g.B[0] * m[0] + g.B[1] * m[1] + g.B[2] * m[2];
  const double sy = g.B[3] * m[0] + g.B[4] * m[1] + g.B[5] * m[2];
  const double sz = g.B[6] * m[0] + g.B[7] * m[1] + g.B[8] * m[2];
  const double4 ph64 = A.pos64[s];
  const double xo64 = ph64.x - sx, yo64 = ph64.y - sy, zo64 = ph64.z - sz;
  const double4 pj64 = A.pos64[j];
  const double ex = pj64.x - xo64, ey = pj64.y - yo64, ez = pj64.z - zo64;
  const double e2 = fma(ez, ez, fma(ey, ey, ex * ex));
  acc.fp64 += 1;
  if (e2 < A.rc2) {
    if (e2 < A.rclose2_64)
      pair64(acc, A.p64, ex, ey, ez, e2);
    else
      pair32(acc, A.p32, A.p64, (float)ex, (float)ey, (float)ez, (float)e2, e2);
    acc.pairs += 1;
    debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
  }
}

// the lane's ordinary entries (Kahan mode: the round's forces, at most PL_K
// pairs, are summed in FP32 and join the compensated sums once per round)
template <int PREC, bool DEBUG, class PL>
__device__ inline void flush_list(Acc<PREC, DEBUG>& acc, const SweepArgs& A, PL& L) {
  if constexpr (PREC == 2) {
    float bx = 0.f, by = 0.f, bz = 0.f;
    for (const lds_entry* e = L.base; e != L.q; e += PL::stride) {
      const pl_entry v = *e;
      pair32_to(acc, A.p32, A.p64, v.x, v.y, v.z, v.w, (double)v.w, bx, by, bz);
      acc.pairs += 1;
    }
    kahan_add(acc.fx, acc.kx, bx);
    kahan_add(acc.fy, acc.ky, by);
    kahan_add(acc.fz, acc.kz, bz);
  } else {
    for (const lds_entry* e = L.base; e != L.q; e += PL::stride) {
      const pl_entry v = *e;
      pair32(acc, A.p32, A.p64, v.x, v.y, v.z, v.w, (double)v.w);
      acc.pairs += 1;
    }
  }
  L.q = L.base;
}

// the lane's FP64-path entries
template <int PREC, bool DEBUG, class PL>
__device__ inline void flush_exact(Acc<PREC, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, uint32_t s,
                                   const int4& wi, PL& L) {
  const lds_entry* end = L.base + PL_K * PL::stride;
  for (const lds_entry* e = L.top; e != end; e += PL::stride) {
    const pl_entry v = *e;
    exact_pair(acc, A, g, s, __float_as_uint(v.x), __float_as_uint(v.y), wi);
  }
  L.top = L.base + PL_K * PL::stride;
}

// room for the next group of four candidates in every lane's list
template <int PREC, bool DEBUG, class PL>
__device__ inline void make_room(Acc<PREC, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, uint32_t s,
                                 const int4& wi, PL& L) {
  if (__ballot(L.q + 4 * PL::stride > L.top) != 0) {
    flush_list(acc, A, L);
    if (__ballot(L.q + 4 * PL::stride > L.top) != 0) flush_exact(acc, A, g, s, wi, L);
  }
}

// Visit one neighbour cell `cj` seen through lattice image `m` (in the
// basis Lred); `dc` is the FP64 vector from the home cell's centre to the
// centre of that image of cj (the FP64 paths form the shift B m from m).
//
// FLAT: the slots [cstart[cj], cstart[cj + ncell]) of ncell consecutive x
// cells of one row (cells are stored x-fastest), for the rectangular cells
// of the dynamic-offset list, whose x step (w0, 0, 0) only changes d_x; dc
// is then the centre offset of the row's x cell 0 and each candidate adds
// ax_j w0, ax_j being its cell's x index (cell id - row base).
template <int PREC, bool DEBUG, bool FLAT = false, class PL = PairList>
__device__ inline void visit_cell(Acc<PREC, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, uint32_t s,
                                  uint32_t cj, bool zero_image, const double* dc, const int* m,
                                  const double* oi, const double4& pi64, const int4& wi, PL& L,
                                  uint32_t ncell = 1, uint32_t rowbase = 0) {
  const uint32_t st = A.cstart[A.cell0 + cj] + A.pad, en = A.cstart[A.cell0 + cj + ncell] + A.pad;
  const uint32_t self = zero_image ? s : 0xffffffffu;
  acc.cand += (en - st) - ((zero_image && s >= st && s < en) ? 1u : 0u);
  if (PREC == 0) {
    const double sx = g.B[0] * m[0] + g.B[1] * m[1] + g.B[2] * m[2];
    const double sy = g.B[3] * m[0] + g.B[4] * m[1] + g.B[5] * m[2];
    const double sz = g.B[6] * m[0] + g.B[7] * m[1] + g.B[8] * m[2];
    const double xo = pi64.x - sx, yo = pi64.y - sy, zo = pi64.z - sz;
    for (uint32_t j0 = st; j0 < en; j0 += 2) {
      const double4 pa = A.pos64[j0];
      const double4 pb = A.pos64[min(j0 + 1, en - 1)];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double4 pj = u ? pb : pa;
        const uint32_t j = j0 + u;
        const double dx = pj.x - xo, dy = pj.y - yo, dz = pj.z - zo;
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        if (r2 < A.rc2 && j < en && j != self) {
          pair64(acc, A.p64, dx, dy, dz, r2);
          acc.pairs += 1;
          debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
        }
      }
    }
  } else {
    // FP64 home position relative to the centre of this image of cj; the
    // candidates' FP32 offsets are widened to FP64, so the separation is
    // exact up to the rounding of the stored FP32 offsets
    const double xo = oi[0] - dc[0], yo = oi[1] - dc[1], zo = oi[2] - dc[2];
    // FLAT runs: the home x relative to the centre of x cell 0 of the cell
    // id numbering, so that a candidate's cell id times w0 gives its cell's
    // centre directly (rounding of this sum at most 2^-53 of ncells w0, kept
    // inside the screen's band)
    const double xo2 = FLAT ? xo + (double)rowbase * g.w[0] : 0.0;
    // run-end and self tests of candidate j0 + u against bounds shifted by u
    // (en - u saturated at 0: no slot precedes it then; j0 < en holds inside
    // the loop)
    const uint32_t enu[4] = {en, en > 1u ? en - 1u : 0u, en > 2u ? en - 2u : 0u, en > 3u ? en - 3u : 0u};
    const uint32_t selfu[4] = {self, self - 1u, self - 2u, self - 3u};
    // four candidate loads in flight per step from one address; entries
    // past the run (up to three; the array has four spare entries at its
    // end) are read and masked out
    // dynamic size: the self-exclusion test is compiled in only for the
    // visits (wave-wide) that hold some lane's own particle (measured 3 %
    // faster).  The dynamic-offset runs take the plain copy of the loop
    // below, with the test: a second copy cost them registers and time, and
    // routing them through this lambda changed their code (the batched sweep
    // ran 2-3 % slower).
    auto run = [&](auto check_self) {
      constexpr bool CHECK_SELF = decltype(check_self)::value;
      const float4* pp = A.pos32 + st;
      for (uint32_t j0 = st; j0 < en; j0 += 4, pp += 4) {
        float4 pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = pp[u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t j = j0 + u;
          // FLAT: x-cell index times w0 from the cell id (xo2 = xo + rowbase w0)
          const double dx = FLAT ? fma((double)__float_as_uint(pj[u].w), g.w[0], -xo2) + (double)pj[u].x
                                 : (double)pj[u].x - xo;
          const double dy = (double)pj[u].y - yo, dz = (double)pj[u].z - zo;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          if (r2 < g.rc2_hi64 && (u == 0 || j0 < enu[u]) && (!CHECK_SELF || j0 != selfu[u])) {
            if (r2 > g.rc2_lo64 || r2 < A.rclose2_64) {
              // within the rounding band of d_cut, or a close pair: deferred
              // to the FP64 path (see flush_exact)
              L.top -= PL::stride;
              *L.top = pl_entry{__uint_as_float(j), __uint_as_float(pack_image(m)), 0.0f, 0.0f};
            } else {
              *L.q = pl_entry{(float)dx, (float)dy, (float)dz, (float)r2};
              L.q += PL::stride;
              debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
            }
          }
        }
        // the next group appends at most four entries per lane
        make_room(acc, A, g, s, wi, L);
      }
    };
    if constexpr (!FLAT) {
      if (__ballot(self >= st && self < en) != 0) run(std::true_type{});
      else run(std::false_type{});
    } else {
      const float4* pp = A.pos32 + st;
      for (uint32_t j0 = st; j0 < en; j0 += 4, pp += 4) {
        float4 pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = pp[u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t j = j0 + u;
          // FLAT: x-cell index times w0 from the cell id (xo2 = xo + rowbase w0)
          const double dx = FLAT ? fma((double)__float_as_uint(pj[u].w), g.w[0], -xo2) + (double)pj[u].x
                                 : (double)pj[u].x - xo;
          const double dy = (double)pj[u].y - yo, dz = (double)pj[u].z - zo;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          if (r2 < g.rc2_hi64 && (u == 0 || j0 < enu[u]) && j0 != selfu[u]) {
            if (r2 > g.rc2_lo64 || r2 < A.rclose2_64) {
              // within the rounding band of d_cut, or a close pair: deferred
              // to the FP64 path (see flush_exact)
              L.top -= PL::stride;
              *L.top = pl_entry{__uint_as_float(j), __uint_as_float(pack_image(m)), 0.0f, 0.0f};
            } else {
              *L.q = pl_entry{(float)dx, (float)dy, (float)dz, (float)r2};
              L.q += PL::stride;
              debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
            }
          }
        }
        // the next group appends at most four entries per lane
        make_room(acc, A, g, s, wi, L);
      }
    }
  }
}

// Cell starts: runs of empty cells longer than a span are not filled by
// the cell-start kernel but queued after cstart[nc] as (first cell, length,
// value) triples behind a count; a later kernel fills them, each workgroup
// taking runs blockIdx.x, blockIdx.x + gridDim.x, ...  The count is cleared
// by the cell-index kernel that precedes the sort.
__device__ inline void cs_fill_runs(uint32_t* __restrict__ cstart, uint32_t nc) {
  const uint32_t* runs = cstart + nc + 1;
  const uint32_t nr = runs[0];
  for (uint32_t q = blockIdx.x; q < nr; q += gridDim.x) {
    const uint32_t c0 = runs[1 + 3 * q], len = runs[2 + 3 * q], v = runs[3 + 3 * q];
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) cstart[c0 + i] = v;
  }
}

__device__ inline double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// per-particle sweep straight from global memory (used for bricks whose
// neighbourhood does not fit the LDS tile)
// ---------------------------------------------------------------------------
template <int VAR, int PREC, bool DEBUG, bool DIVFREE = false, class PL = PairList>
__device__ void sweep_particle(const SweepArgs& A, const CellGeom& g, uint32_t s, Acc<PREC, DEBUG>& acc,
                               uint32_t& nbh, PL& L) {
  const float4 pi = A.pos32[s];
  const double4 pi64 = A.pos64[s];
  const int4 wi = DEBUG ? A.wrap[s] : make_int4(0, 0, 0, 0);
  const uint32_t hc = __float_as_uint(pi.w);
  const int a = (int)(hc % (uint32_t)g.nc[0]);
  const int b = (int)((hc / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
  const int c = (int)(hc / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
  double oi[3];
  cell_centre(g, a, b, c, oi);
  oi[0] = pi64.x - oi[0];
  oi[1] = pi64.y - oi[1];
  oi[2] = pi64.z - oi[2];
  if (VAR == VAR_DS) {
    // 27 cells congruent to the box; the unwrapped index a + delta gives
    // the cell (a + delta) mod c and the lattice image floor((a + delta)/c)
    int q = 0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx, ++q) {
          const int u[3] = {a + dx, b + dy, c + dz};
          int m[3], w[3];
          for (int k = 0; k < 3; ++k) {  // u[k] in [-1, nc[k]]
            m[k] = (int)(u[k] >= g.nc[k]) - (int)(u[k] < 0);
            w[k] = u[k] - m[k] * g.nc[k];
          }
          const uint32_t cj = (uint32_t)w[0] + (uint32_t)g.nc[0] * ((uint32_t)w[1] + (uint32_t)g.nc[1] * (uint32_t)w[2]);
          const bool zero = (dx == 0 && dy == 0 && dz == 0);
          visit_cell<PREC, DEBUG>(acc, A, g, s, cj, zero, g.ds_delta[q], m, oi, pi64, wi, L);
          ++nbh;
        }
  } else {
    // rectangular cells of the rotated box; layer k (z) is offset by
    // k r23 in y, row (j, k) by j r12 + k r13 in x.  The row and x image
    // indices are exact floor divisions by the FP64 reciprocal cell counts
    // (idiv_floor_f).  DIVFREE: the layer image by comparisons and the
    // shifts in cells by the reciprocal widths (a cell only touched at the
    // range's edge may then be visited or not; it holds no pair in range);
    // otherwise by an FP64 division.  Which is faster depends on the
    // kernel's register allocation (measured: the batched sweep gains 5 %,
    // the single-box sweep loses to spilled scalar registers).
    const double w0 = g.w[0], w1 = g.w[1], w2 = g.w[2];
    for (int dz = -1; dz <= 1; ++dz) {
      const int C = c + dz;  // in [-1, nc[2]]
      const int k = DIVFREE ? (int)(C >= g.nc[2]) - (int)(C < 0) : idiv_floor_f(C, g.inv_nc[2]);
      const int cz = C - k * g.nc[2];
      const double fy = DIVFREE ? -(double)k * g.B[5] * g.inv_w[1] : -(double)k * g.B[5] / w1;
      const int B0 = (int)floor(b - g.grow[1] + fy);
      const int B1 = (int)ceil(b + 1 + g.grow[1] + fy) - 1;
      for (int Bq = B0; Bq <= B1; ++Bq) {
        const int j = idiv_floor_f(Bq, g.inv_nc[1]);
        const int by = Bq - j * g.nc[1];
        const double xs = (double)j * g.B[1] + (double)k * g.B[2];
        const double fx = DIVFREE ? -xs * g.inv_w[0] : -xs / w0;
        const int A0 = (int)floor(a - g.grow[0] + fx);
        const int A1 = (int)ceil(a + 1 + g.grow[0] + fx) - 1;
        const uint32_t rowbase = (uint32_t)g.nc[0] * ((uint32_t)by + (uint32_t)g.nc[1] * (uint32_t)cz);
        // the row's cells A0..A1, one contiguous run per x image i
        const int i0 = idiv_floor_f(A0, g.inv_nc[0]);
        const int i1 = idiv_floor_f(A1, g.inv_nc[0]);
        for (int i = i0; i <= i1; ++i) {
          const int axlo = max(A0 - i * g.nc[0], 0), axhi = min(A1 - i * g.nc[0], g.nc[0] - 1);
          const int m[3] = {i, j, k};
          // centre offset of x cell 0 of this image of the row
          const double dcv[3] = {(double)(i * g.nc[0] - a) * w0 + xs, (Bq - b) * w1 + (double)k * g.B[5], (C - c) * w2};
          const bool zero = (i == 0 && j == 0 && k == 0);
          visit_cell<PREC, DEBUG, PREC != 0>(acc, A, g, s, rowbase + (uint32_t)axlo, zero, dcv, m, oi, pi64, wi, L,
                                             (uint32_t)(axhi - axlo + 1), rowbase);
          nbh += (uint32_t)(axhi - axlo + 1);
        }
      }
    }
  }
  if (PREC != 0) {
    flush_list(acc, A, L);
    flush_exact(acc, A, g, s, wi, L);
  }
}

// per-particle outputs: force rotated back to Cartesian for DO, written in
// the caller's order; debug digest
template <int VAR, int PREC, bool DEBUG>
__device__ inline void write_particle(const SweepArgs& A, const CellGeom& g, uint32_t s, const Acc<PREC, DEBUG>& acc) {
  double F[3];
  if (PREC == 0) {
    F[0] = acc.gx; F[1] = acc.gy; F[2] = acc.gz;
  } else if (PREC == 2) {
    F[0] = (double)acc.fx - (double)acc.kx;
    F[1] = (double)acc.fy - (double)acc.ky;
    F[2] = (double)acc.fz - (double)acc.kz;
  } else {
    F[0] = (double)acc.fx;
    F[1] = (double)acc.fy;
    F[2] = (double)acc.fz;
  }
  double Fc[3];
  if (VAR == VAR_DO) {
    for (int r = 0; r < 3; ++r) Fc[r] = g.Q[3 * r] * F[0] + g.Q[3 * r + 1] * F[1] + g.Q[3 * r + 2] * F[2];
  } else {
    Fc[0] = F[0]; Fc[1] = F[1]; Fc[2] = F[2];
  }
  const uint32_t io = A.perm[s];
  if (PREC == 0) {
    double* Fo = (double*)A.F;
    Fo[3 * (size_t)io] = Fc[0];
    Fo[3 * (size_t)io + 1] = Fc[1];
    Fo[3 * (size_t)io + 2] = Fc[2];
  } else {
    float* Fo = (float*)A.F;
    Fo[3 * (size_t)io] = (float)Fc[0];
    Fo[3 * (size_t)io + 1] = (float)Fc[1];
    Fo[3 * (size_t)io + 2] = (float)Fc[2];
  }
  if (DEBUG) {
    A.dbg_count[io] = acc.dcount;
    A.dbg_hash[io] = acc.dhash;
  }
}

// energy and virial of one thread as FP64 (u, wxx, wyy, wzz, wxy, wxz, wyz)
template <int PREC, bool DEBUG>
__device__ inline void acc_energy(const Acc<PREC, DEBUG>& acc, double* v) {
  if (PREC == 0) {
    v[0] = acc.gu;
    for (int k = 0; k < 6; ++k) v[1 + k] = acc.gw[k];
  } else {
    v[0] = acc.gu;
    for (int k = 0; k < 6; ++k) v[1 + k] = (double)acc.w[k];
  }
}

// block-wide sums of v[7] (FP64, fixed order) and of the integer statistics
// -> partial[PART_STRIDE * slot], summed over slots by the finalisation.
// (Statistics are not added atomically: one counter hit by every wave of a
// launch serialises in one L2 channel and cost a quarter of the sweep.)
// Every thread of the block (NW waves) must call it.  `red` is LDS for the
// waves' sums; it may alias memory the block has finished with (the pair
// lists), since the block synchronises before writing it.
template <int NW = 4>
__device__ inline void block_commit(const SweepArgs& A, uint32_t slot, const double* v, const uint32_t* st4,
                                    double (*red)[PART_STRIDE]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double t = warp_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned long long c = st4[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if (lane == 0) red[wid][8 + k] = (double)c;
  }
  __syncthreads();
  if (threadIdx.x < PART_STRIDE && threadIdx.x != 7) {
    double t = red[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < NW; ++w) t += red[w][threadIdx.x];
    A.partial[PART_STRIDE * (size_t)slot + threadIdx.x] = t;
  }
}

__device__ inline void block_commit(const SweepArgs& A, uint32_t slot, const double* v, const uint32_t* st4) {
  __shared__ double red[4][PART_STRIDE];
  block_commit(A, slot, v, st4, red);
}

// LDS of the per-particle sweeps: the per-lane pair lists, reused for the
// block's reduction once every lane has flushed its list
template <int BT>
union SweepSmemT {
  pl_entry plist[PL_K * BT];
  double red[BT / 64][PART_STRIDE];
};
using SweepSmem = SweepSmemT<SW_THREADS_P>;


}  // namespace ncl
