// Half-list sweep: every interacting pair is evaluated once and its force is
// applied to both particles (Newton's third law), with the FP32-offset
// precision of the per-particle sweep.
//
// Ownership.  A particle visits only the forward half of its stencil: the
// layer above (dz = +1) whole; in its own layer the rows above (dy > 0); in
// its own row the cells to its right (dx > 0); in its own cell the particles
// of larger slot.  Offsets are taken in unwrapped cell indices, so for a pair
// (i, j, m) the reverse pair (j, i, -m) has the opposite offset and exactly one
// of the two is forward.  This holds for the 27 (cell, image) stencil of the
// dynamic-size list (Sec. 4.1) and for the dynamic-offset neighbourhood
// (Sec. 4.2), whose rows and cells are included by a test that is symmetric in
// the offset between cell centres.
//
// Scatter.  A workgroup sweeps 256 consecutive slots, which lie in at most a
// few rows of cells.  The forward rows of each home row ("windows": at most 6
// per home row) are assigned LDS accumulators, one triple per particle, laid
// out segment by segment (a segment is a run of one x image of one row, i.e.
// a contiguous range of slots).  Forces on the neighbour go to these
// accumulators with LDS atomics, as 64-bit fixed point in units of
// q = 2^-20 eps/sigma (integer LDS atomics run at the LDS read rate on gfx950,
// FP32 ones about 14 times slower; integer sums are also exact and
// order-independent; each addition is off by at most q/2, and the range,
// 2^43 eps/sigma, is far beyond the forces of the FP32 path, whose pairs are
// never closer than 0.3 sigma).  At the end the workgroup adds them, and the
// home particles' own sums, to an FP64 force array in slot order with global
// atomics (coalesced: consecutive slots).  Pairs on the exact FP64 path, and
// rows without a window, add the neighbour's force to the FP64 array directly.
// A last kernel writes the forces in the caller's order.  The order of the
// atomic additions varies from run to run, so forces are not bit-reproducible;
// the pair set, and U and W (summed per workgroup in a fixed order), are.
#include "sweep_common.hpp"

namespace ncl {

constexpr int HL_K = 7;        // per-lane list of pairs waiting for evaluation
constexpr int HW_CAP = 1984;   // window accumulators per workgroup (particles; two workgroups per CU)
constexpr int HW_ROWS = 4;     // home rows per workgroup that get windows
constexpr int HW_WPR = 6;      // windows per home row
constexpr int HW_SEGS = 64;    // segments over all windows of a workgroup
constexpr int NO_WIN = INT32_MIN;  // run without a window (a real base may be negative)

struct HalfSmem {
  unsigned long long fx[HW_CAP], fy[HW_CAP], fz[HW_CAP];  // fixed point, units of q
  pl_entry list[HL_K * SW_THREADS];  // (d_x, d_y, d_z, r^2) as in the full sweep's list
  uint16_t tgt[HL_K * SW_THREADS];
  int32_t seg_off[HW_SEGS + 1];        // first accumulator of each segment
  int32_t seg_base[HW_SEGS];           // accumulator of slot j = j + seg_base
  int32_t seg_slot0[HW_SEGS], seg_len[HW_SEGS];
  int32_t win_seg0[HW_ROWS * HW_WPR];  // first segment of the window (-1: none)
  int32_t win_ilo[HW_ROWS * HW_WPR];   // x image of that segment
  int32_t win_ns[HW_ROWS * HW_WPR];    // segments of the window
  int32_t row_lo, nrow, nseg, total, ok;
};

struct HList {
  pl_entry* base;
  uint16_t* tgt;
  int cnt;
};

__device__ inline int half_wave_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// dynamic offset (Sec. 4.2): rows [B0, B1] of layer image k seen from home
// row b, and x cells [A0, A1] of row image (j, k) seen from home x cell a;
// the same expressions as the full per-particle sweep
__device__ inline void do_rows(const CellGeom& g, int b, int k, int& B0, int& B1) {
  const double fy = -(double)k * g.B[5] / g.w[1];
  B0 = (int)floor(b - g.grow[1] + fy);
  B1 = (int)ceil(b + 1 + g.grow[1] + fy) - 1;
}
__device__ inline void do_cols(const CellGeom& g, int a, int j, int k, int& A0, int& A1) {
  const double xs = (double)j * g.B[1] + (double)k * g.B[2];
  const double fx = -xs / g.w[0];
  A0 = (int)floor(a - g.grow[0] + fx);
  A1 = (int)ceil(a + 1 + g.grow[0] + fx) - 1;
}

// Windows of the workgroup's slots [s0, s1): computed by wave 0, then the
// accumulators are cleared.  Every thread of the block must call it.
template <int VAR>
__device__ void build_windows(const SweepArgs& A, const CellGeom& g, HalfSmem& S, uint32_t s0, uint32_t s1) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int l0 = g.nc[0], l1 = g.nc[1], l2 = g.nc[2];
  if (tid < 64) {
    const uint32_t clo = __float_as_uint(A.pos32[s0].w), chi = __float_as_uint(A.pos32[s1 - 1].w);
    const int rlo = (int)(clo / (uint32_t)l0), rhi = (int)(chi / (uint32_t)l0);
    const int nrow = rhi - rlo + 1;
    int ns = 0, X0 = 0, X1 = -1, ilo = 0, rowbase = 0;
    if (nrow <= HW_ROWS && lane < nrow * HW_WPR) {
      const int h = lane / HW_WPR, wl = lane - h * HW_WPR;
      const int R = rlo + h;
      const int b = R % l1, c = R / l1;
      const int xa = (h == 0) ? (int)(clo % (uint32_t)l0) : 0;
      const int xb = (h == nrow - 1) ? (int)(chi % (uint32_t)l0) : l0 - 1;
      int Bq = 0, C = c;
      bool use = false;
      if (VAR == VAR_DS) {
        if (wl < 5) {
          use = true;
          const int dz = wl < 2 ? 0 : 1, dy = wl < 2 ? wl : wl - 3;
          Bq = b + dy;
          C = c + dz;
          X0 = (wl == 0) ? xa : xa - 1;
          X1 = xb + 1;
        }
      } else {
        int k, B0, B1;
        if (wl < 2) {
          k = 0;
          do_rows(g, b, 0, B0, B1);
          Bq = b + wl;
        } else {
          C = c + 1;
          k = idiv_floor32(C, l2);
          do_rows(g, b, k, B0, B1);
          Bq = B0 + (wl - 2);
        }
        use = Bq <= B1;
        if (use) {
          const int j = idiv_floor32(Bq, l1);
          int A0, A1, D0, D1;
          do_cols(g, xa, j, k, A0, A1);
          do_cols(g, xb, j, k, D0, D1);
          X0 = (wl == 0) ? xa : A0;
          X1 = D1;
        }
      }
      if (use) {
        const int jy = idiv_floor32(Bq, l1), kz = idiv_floor32(C, l2);
        rowbase = l0 * ((Bq - jy * l1) + l1 * (C - kz * l2));
        ilo = idiv_floor32(X0, l0);
        ns = idiv_floor32(X1, l0) - ilo + 1;
      }
    }
    const int incl = half_wave_scan(ns);
    const int sbeg = incl - ns;
    const int nseg = __shfl(incl, 63, 64);
    const bool ok = nrow <= HW_ROWS && nseg <= HW_SEGS;
    if (lane < HW_ROWS * HW_WPR) {
      S.win_seg0[lane] = (ok && ns > 0) ? sbeg : -1;
      S.win_ilo[lane] = ilo;
      S.win_ns[lane] = ns;
    }
    if (ok)
      for (int q = 0; q < ns; ++q) {
        const int i = ilo + q;
        const int axlo = max(X0 - i * l0, 0), axhi = min(X1 - i * l0, l0 - 1);
        const uint32_t st = A.cstart[rowbase + axlo], en = A.cstart[rowbase + axhi + 1];
        S.seg_slot0[sbeg + q] = (int32_t)st;
        S.seg_len[sbeg + q] = (int32_t)(en - st);
      }
    if (lane == 0) {
      S.row_lo = rlo;
      S.nrow = nrow;
      S.nseg = ok ? nseg : 0;
      S.ok = ok ? 1 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // accumulator offsets of the segments
    const int ns2 = ok ? nseg : 0;
    const int len = lane < ns2 ? S.seg_len[lane] : 0;
    const int inc2 = half_wave_scan(len);
    const int total = __shfl(inc2, 63, 64);
    if (lane < ns2) {
      S.seg_off[lane] = inc2 - len;
      S.seg_base[lane] = (inc2 - len) - S.seg_slot0[lane];
    }
    if (lane == 0) {
      S.seg_off[ns2] = total;
      const bool fit = ok && total <= HW_CAP;
      S.total = fit ? total : 0;
      if (!fit) S.ok = 0;
    }
  }
  __syncthreads();
  for (int p = tid; p < S.total; p += SW_THREADS) {
    S.fx[p] = 0ull;
    S.fy[p] = 0ull;
    S.fz[p] = 0ull;
  }
  __syncthreads();
}

// LDS base for a run of slots [st, en) of x image i in window wl of the home
// row hrow (accumulator of slot j = j + base); NO_WIN when the run has no
// window (its neighbour forces then go to the FP64 array directly)
__device__ inline int run_base(const HalfSmem& S, int hrow, int wl, int i, uint32_t st, uint32_t en) {
  if (!S.ok || wl >= HW_WPR) return NO_WIN;
  const int w = hrow * HW_WPR + wl;
  const int s0 = S.win_seg0[w];
  const int q = i - S.win_ilo[w];
  if (s0 < 0 || q < 0 || q >= S.win_ns[w]) return NO_WIN;
  const int sg = s0 + q;
  if ((int32_t)st < S.seg_slot0[sg] || (int32_t)en > S.seg_slot0[sg] + S.seg_len[sg]) return NO_WIN;
  return S.seg_base[sg];
}

// one FP32 pair: accumulates the home particle's force, energy and virial
// and returns fs, the neighbour's force being fs * d (d = x_j - x_i)
template <bool DEBUG>
__device__ inline float hpair32(Acc<1, DEBUG>& acc, const Pot32& p, const Pot64& p64, float dx, float dy, float dz,
                               float r2, double r2e) {
  const float r2i = __builtin_amdgcn_rcpf(r2);
  const float s2 = p.sig2 * r2i;
  const float s6 = s2 * s2 * s2;
  const float fs = r2i * s6 * fmaf(p.eps48, s6, -p.eps24);
  acc.fx = fmaf(-fs, dx, acc.fx);
  acc.fy = fmaf(-fs, dy, acc.fy);
  acc.fz = fmaf(-fs, dz, acc.fz);
  acc.gu += phi64(p64, r2e, r2i);  // energy in FP64, as in the full list
  const float fdx = fs * dx, fdy = fs * dy;
  acc.w[0] = fmaf(fdx, dx, acc.w[0]);
  acc.w[1] = fmaf(fdy, dy, acc.w[1]);
  acc.w[2] = fmaf(fs * dz, dz, acc.w[2]);
  acc.w[3] = fmaf(fdx, dy, acc.w[3]);
  acc.w[4] = fmaf(fdx, dz, acc.w[4]);
  acc.w[5] = fmaf(fdy, dz, acc.w[5]);
  return fs;
}

__device__ inline void add_f64(double* Facc, uint32_t j, double fx, double fy, double fz) {
  unsafeAtomicAdd(&Facc[3 * (size_t)j], fx);
  unsafeAtomicAdd(&Facc[3 * (size_t)j + 1], fy);
  unsafeAtomicAdd(&Facc[3 * (size_t)j + 2], fz);
}

// pair digests of both particles (test builds): the neighbour's key names
// the home particle with the opposite image
template <bool DEBUG>
__device__ inline void debug_both(Acc<1, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, uint32_t s, uint32_t j,
                                  const int* mcell, const int4& wi) {
  if (!DEBUG) return;
  const int4 wj = A.wrap[j];
  const int64_t m[3] = {(int64_t)mcell[0] - wj.x + wi.x, (int64_t)mcell[1] - wj.y + wi.y,
                        (int64_t)mcell[2] - wj.z + wi.z};
  int64_t mk[3];
  for (int r = 0; r < 3; ++r) mk[r] = g.Mtot[3 * r] * m[0] + g.Mtot[3 * r + 1] * m[1] + g.Mtot[3 * r + 2] * m[2];
  auto key = [](uint32_t id, const int64_t* v) {
    uint64_t k = ((uint64_t)id) << 32;
    k |= ((uint64_t)((v[0] + 512) & 0x3ff)) << 20;
    k |= ((uint64_t)((v[1] + 512) & 0x3ff)) << 10;
    k |= ((uint64_t)((v[2] + 512) & 0x3ff));
    return k;
  };
  const uint32_t ij = A.perm[j], is = A.perm[s];
  acc.dhash += splitmix_out(key(ij - A.jbase, mk));
  acc.dcount += 1;
  const int64_t mr[3] = {-mk[0], -mk[1], -mk[2]};
  atomicAdd((unsigned long long*)&A.dbg_count[ij], 1ull);
  atomicAdd((unsigned long long*)&A.dbg_hash[ij], (unsigned long long)splitmix_out(key(is - A.jbase, mr)));
}

// FP32 force component -> fixed point (units of q), rounded to nearest
__device__ inline unsigned long long to_fix(float v, double inv_q) {
  return (unsigned long long)__double2ll_rn((double)v * inv_q);
}

template <bool DEBUG>
__device__ inline void hflush(Acc<1, DEBUG>& acc, const SweepArgs& A, HalfSmem& S, HList& L) {
  for (int e = 0; e < L.cnt; ++e) {
    const pl_entry q = L.base[e * SW_THREADS];
    const float dx = q.x, dy = q.y, dz = q.z;
    const int t = L.tgt[e * SW_THREADS];
    const float fs = hpair32(acc, A.p32, A.p64, dx, dy, dz, q.w, (double)q.w);
    atomicAdd(&S.fx[t], to_fix(fs * dx, A.fix_inv));
    atomicAdd(&S.fy[t], to_fix(fs * dy, A.fix_inv));
    atomicAdd(&S.fz[t], to_fix(fs * dz, A.fix_inv));
  }
  L.cnt = 0;
}

// Visit the forward part of one run of neighbour cells: cells
// [cj, cj + ncell) seen through image m, dc the FP64 centre offset as in the
// full sweep.  On the zero image only slots after the home particle count.
template <bool DEBUG, bool FLAT>
__device__ inline void hvisit(Acc<1, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, HalfSmem& S, uint32_t s,
                              uint32_t cj, bool zero_image, const double* dc, const int* m, const double* oi,
                              const double4& pi64, const int4& wi, HList& L, double* Facc, int hrow, int wl,
                              uint32_t ncell, uint32_t rowbase) {
  const uint32_t st0 = A.cstart[cj], en = A.cstart[cj + ncell];
  const uint32_t st = zero_image ? max(st0, s + 1) : st0;
  const int rb = run_base(S, hrow, wl, m[0], st0, en);
  if (st < en) acc.cand += en - st;
  const double xo = oi[0] - dc[0], yo = oi[1] - dc[1], zo = oi[2] - dc[2];
  for (uint32_t j0 = st; j0 < en; j0 += 4) {
    const uint32_t jl = en - 1;
    float4 pj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pj[u] = A.pos32[min(j0 + u, jl)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t j = j0 + u;
      double dx = (double)pj[u].x - xo;
      if (FLAT) dx = fma((double)(int32_t)(__float_as_uint(pj[u].w) - rowbase), g.w[0], dx);
      const double dy = (double)pj[u].y - yo, dz = (double)pj[u].z - zo;
      const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      if (r2 < g.rc2_hi64 && j < en) {
        const bool exact = r2 > g.rc2_lo64 || r2 < A.rclose2_64;
        if (exact || rb == NO_WIN || r2 < A.rwin2_64) {
          double fj[3];
          bool hit = true;
          if (exact) {
            // as the full sweep: re-evaluated from the FP64 positions
            const double sx = g.B[0] * m[0] + g.B[1] * m[1] + g.B[2] * m[2];
            const double sy = g.B[3] * m[0] + g.B[4] * m[1] + g.B[5] * m[2];
            const double sz = g.B[6] * m[0] + g.B[7] * m[1] + g.B[8] * m[2];
            const double4 pj64 = A.pos64[j];
            const double ex = pj64.x - (pi64.x - sx), ey = pj64.y - (pi64.y - sy), ez = pj64.z - (pi64.z - sz);
            const double e2 = fma(ez, ez, fma(ey, ey, ex * ex));
            acc.fp64 += 1;
            hit = e2 < A.rc2;
            if (hit) {
              if (e2 < A.rclose2_64) {
                const double r2i = 1.0 / e2;
                const double s2 = A.p64.sig2 * r2i;
                const double s6 = s2 * s2 * s2;
                const double fs = r2i * s6 * (A.p64.eps48 * s6 - A.p64.eps24);
                acc.gx -= fs * ex;
                acc.gy -= fs * ey;
                acc.gz -= fs * ez;
                acc.gu += s6 * (A.p64.eps4 * s6 - A.p64.eps4) - A.p64.shift;
                acc.w[0] += (float)(fs * ex * ex);
                acc.w[1] += (float)(fs * ey * ey);
                acc.w[2] += (float)(fs * ez * ez);
                acc.w[3] += (float)(fs * ex * ey);
                acc.w[4] += (float)(fs * ex * ez);
                acc.w[5] += (float)(fs * ey * ez);
                fj[0] = fs * ex; fj[1] = fs * ey; fj[2] = fs * ez;
              } else {
                const float fx = (float)ex, fy = (float)ey, fz = (float)ez;
                const float fs = hpair32(acc, A.p32, A.p64, fx, fy, fz, (float)e2, e2);
                fj[0] = (double)(fs * fx); fj[1] = (double)(fs * fy); fj[2] = (double)(fs * fz);
              }
              debug_both<DEBUG>(acc, A, g, s, j, m, wi);
            }
          } else {
            const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
            const float fs = hpair32(acc, A.p32, A.p64, fx, fy, fz, (float)r2, r2);
            fj[0] = (double)(fs * fx); fj[1] = (double)(fs * fy); fj[2] = (double)(fs * fz);
            debug_both<DEBUG>(acc, A, g, s, j, m, wi);
          }
          if (hit) {
            add_f64(Facc, j, fj[0], fj[1], fj[2]);
            acc.pairs += 2;
          }
        } else {
          L.base[L.cnt * SW_THREADS] = pl_entry{(float)dx, (float)dy, (float)dz, (float)r2};
          L.tgt[L.cnt * SW_THREADS] = (uint16_t)(rb + (int)j);
          L.cnt += 1;
          acc.pairs += 2;
          debug_both<DEBUG>(acc, A, g, s, j, m, wi);
        }
      }
    }
    if (__ballot(L.cnt > HL_K - 4) != 0) hflush(acc, A, S, L);  // a group appends at most four
  }
}

template <int VAR, bool DEBUG>
__device__ void sweep_half(const SweepArgs& A, const CellGeom& g, HalfSmem& S, uint32_t s, Acc<1, DEBUG>& acc,
                           uint32_t& nbh, HList& L, double* Facc) {
  const float4 pi = A.pos32[s];
  const double4 pi64 = A.pos64[s];
  const int4 wi = DEBUG ? A.wrap[s] : make_int4(0, 0, 0, 0);
  const uint32_t hc = __float_as_uint(pi.w);
  const int l0 = g.nc[0], l1 = g.nc[1], l2 = g.nc[2];
  const int a = (int)(hc % (uint32_t)l0);
  const int b = (int)((hc / (uint32_t)l0) % (uint32_t)l1);
  const int c = (int)(hc / ((uint32_t)l0 * (uint32_t)l1));
  const int hrow = (int)(hc / (uint32_t)l0) - S.row_lo;
  double oi[3];
  cell_centre(g, a, b, c, oi);
  oi[0] = pi64.x - oi[0];
  oi[1] = pi64.y - oi[1];
  oi[2] = pi64.z - oi[2];
  if (VAR == VAR_DS) {
    for (int dz = 0; dz <= 1; ++dz)
      for (int dy = dz ? -1 : 0; dy <= 1; ++dy)
        for (int dx = (dz == 0 && dy == 0) ? 0 : -1; dx <= 1; ++dx) {
          const int q = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          const int u[3] = {a + dx, b + dy, c + dz};
          int m[3], w[3];
          for (int k = 0; k < 3; ++k) {
            m[k] = idiv_floor32(u[k], g.nc[k]);
            w[k] = u[k] - m[k] * g.nc[k];
          }
          const uint32_t cj = (uint32_t)w[0] + (uint32_t)l0 * ((uint32_t)w[1] + (uint32_t)l1 * (uint32_t)w[2]);
          const bool zero = (m[0] | m[1] | m[2]) == 0;
          hvisit<DEBUG, false>(acc, A, g, S, s, cj, zero, g.ds_delta[q], m, oi, pi64, wi, L, Facc, hrow,
                               dz == 0 ? dy : 3 + dy, 1, 0);
          ++nbh;
        }
  } else {
    const double w0 = g.w[0], w1 = g.w[1], w2 = g.w[2];
    for (int dz = 0; dz <= 1; ++dz) {
      const int C = c + dz;
      const int k = idiv_floor32(C, l2);
      const int cz = C - k * l2;
      int B0, B1;
      do_rows(g, b, k, B0, B1);
      for (int Bq = dz ? B0 : b; Bq <= B1; ++Bq) {
        const int j = idiv_floor32(Bq, l1);
        const int by = Bq - j * l1;
        const double xs = (double)j * g.B[1] + (double)k * g.B[2];
        int A0, A1;
        do_cols(g, a, j, k, A0, A1);
        if (dz == 0 && Bq == b) A0 = a;
        const int wl = dz ? ((Bq - B0 < 4) ? 2 + (Bq - B0) : HW_WPR) : ((Bq - b < 2) ? Bq - b : HW_WPR);
        const uint32_t rowbase = (uint32_t)l0 * ((uint32_t)by + (uint32_t)l1 * (uint32_t)cz);
        for (int i = idiv_floor32(A0, l0); i <= idiv_floor32(A1, l0); ++i) {
          const int axlo = max(A0 - i * l0, 0), axhi = min(A1 - i * l0, l0 - 1);
          const int m[3] = {i, j, k};
          const double dcv[3] = {(double)(i * l0 - a) * w0 + xs, (Bq - b) * w1 + (double)k * g.B[5], (C - c) * w2};
          const bool zero = (i == 0 && j == 0 && k == 0);
          hvisit<DEBUG, true>(acc, A, g, S, s, rowbase + (uint32_t)axlo, zero, dcv, m, oi, pi64, wi, L, Facc, hrow,
                              wl, (uint32_t)(axhi - axlo + 1), rowbase);
          nbh += (uint32_t)(axhi - axlo + 1);
        }
      }
    }
  }
}

template <int VAR, bool DEBUG>
__global__ void __launch_bounds__(SW_THREADS) k_sweep_half(SweepArgs A, CellGeom g, double* __restrict__ Facc) {
  __shared__ HalfSmem S;
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t s0 = lb * SW_THREADS, s1 = min(s0 + SW_THREADS, A.n);
  build_windows<VAR>(A, g, S, s0, s1);
  const uint32_t s = s0 + threadIdx.x;
  Acc<1, DEBUG> acc;
  uint32_t nbh = 0;
  if (s < s1) {
    HList L{S.list + threadIdx.x, S.tgt + threadIdx.x, 0};
    sweep_half<VAR, DEBUG>(A, g, S, s, acc, nbh, L, Facc);
    hflush(acc, A, S, L);
    add_f64(Facc, s, (double)acc.fx + acc.gx, (double)acc.fy + acc.gy, (double)acc.fz + acc.gz);
    if (DEBUG) {
      const uint32_t io = A.perm[s];
      atomicAdd((unsigned long long*)&A.dbg_count[io], (unsigned long long)acc.dcount);
      atomicAdd((unsigned long long*)&A.dbg_hash[io], (unsigned long long)acc.dhash);
    }
  }
  __syncthreads();
  // the windows' neighbour forces, one particle per thread
  const int nseg = S.nseg;
  for (int p = threadIdx.x; p < S.total; p += SW_THREADS) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {  // last segment starting at or before p
      const int mid = (lo + hi + 1) >> 1;
      if (S.seg_off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const long long vx = (long long)S.fx[p], vy = (long long)S.fy[p], vz = (long long)S.fz[p];
    if ((vx | vy | vz) != 0)
      add_f64(Facc, (uint32_t)(p - S.seg_base[lo]), (double)vx * A.fix_q, (double)vy * A.fix_q, (double)vz * A.fix_q);
  }
  double v[7];
  acc_energy(acc, v);
  const uint32_t st4[4] = {acc.cand, acc.pairs, acc.fp64, nbh};
  block_commit(A, lb, v, st4);
}

__global__ void k_fill_f64(double* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// slot-order FP64 sums -> caller's order, rotated back for the dynamic offset
__global__ void k_half_out(const double* __restrict__ Facc, const uint32_t* __restrict__ perm, uint32_t n, CellGeom g,
                           float* __restrict__ F) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double f[3] = {Facc[3 * (size_t)s], Facc[3 * (size_t)s + 1], Facc[3 * (size_t)s + 2]};
  double o[3];
  if (g.variant == VAR_DO) {
    for (int r = 0; r < 3; ++r) o[r] = g.Q[3 * r] * f[0] + g.Q[3 * r + 1] * f[1] + g.Q[3 * r + 2] * f[2];
  } else {
    o[0] = f[0]; o[1] = f[1]; o[2] = f[2];
  }
  const size_t io = perm[s];
  F[3 * io] = (float)o[0];
  F[3 * io + 1] = (float)o[1];
  F[3 * io + 2] = (float)o[2];
}

// launched by launch_sweep for SWEEP_HALF (FP32 precision); the caller has
// cleared the statistics and launches the finalisation with scale 1
hipError_t launch_half(const SweepLaunch& L, hipStream_t st, uint32_t nblocks) {
  const SweepArgs& A = *L.args;
  const size_t n = A.n;
  const uint32_t zb = (uint32_t)((3 * n + 255) / 256 < 8192 ? (3 * n + 255) / 256 : 8192);
  k_fill_f64<<<zb, 256, 0, st>>>(L.facc, 3 * n);
  if (L.debug) {
    const uint32_t db = (uint32_t)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    k_fill_u64<<<db, 256, 0, st>>>((unsigned long long*)A.dbg_count, n);
    k_fill_u64<<<db, 256, 0, st>>>((unsigned long long*)A.dbg_hash, n);
  }
  const int var = L.g->variant;
  if (var == VAR_DS) {
    if (L.debug) k_sweep_half<VAR_DS, true><<<nblocks, SW_THREADS, 0, st>>>(A, *L.g, L.facc);
    else k_sweep_half<VAR_DS, false><<<nblocks, SW_THREADS, 0, st>>>(A, *L.g, L.facc);
  } else {
    if (L.debug) k_sweep_half<VAR_DO, true><<<nblocks, SW_THREADS, 0, st>>>(A, *L.g, L.facc);
    else k_sweep_half<VAR_DO, false><<<nblocks, SW_THREADS, 0, st>>>(A, *L.g, L.facc);
  }
  k_half_out<<<(uint32_t)((n + 255) / 256), 256, 0, st>>>(L.facc, A.perm, A.n, *L.g, (float*)A.F);
  return hipGetLastError();
}

}  // namespace ncl
