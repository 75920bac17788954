// HIP kernels for gfx950: the neighbourhood sweep that evaluates forces,
// energy and virial over the cell lists of Sec. 4.1 / 4.2 of Dobson, Fox &
// Saracino, arXiv:1412.3784 (the cells are built every step by build.hip).
//
// Data layout in HBM (sorted = cell order, x fastest, particles of a cell by
// ascending input index):
//   cell_of[N], rank[N]    u32, radix-sort keys (cell ids, ping-pong)
//   rs_val[N]              u32, radix-sort values
//   cstart[Nc+1]           u32, first sorted slot of each cell
//   perm[N]                u32  sorted slot -> input index
//   pos64[N]               double4 (x, y, z, -) wrapped FP64 position in the
//                          variant's frame (Cartesian for DS, rotated for DO)
//   pos32[N + 4]           float4 (ox, oy, oz, cell id bits): FP32 offset from
//                          the FP64 centre of the particle's cell (high word);
//                          four spare entries for reads past a run's end
//   pos32lo[N]             float4 (ox, oy, oz, -): low word, offset - high
//                          (read by the tiled sweep only)
//   wrap[N]                int4 lattice image of the wrap (debug only)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geometry.hpp"
#include "batch.hpp"
#include "kernels.hpp"
#include "sweep_common.hpp"

namespace ncl {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_zero_f64(double* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// the neighbourhood sweep
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// the LDS-tiled sweep
// ---------------------------------------------------------------------------
// One workgroup takes a brick of Sx x Sy x Sz home cells.  It stages the
// union of the home cells' neighbourhoods (every (cell, lattice image) any
// home cell needs) in LDS, each particle as FP32 coordinates in a frame
// centred on the brick (image shift folded in) plus a 16-bit fixed-point
// residual, so hi + residual carries the FP64 position to ~2^-40 of the
// brick size.  Each lane then screens its own neighbourhood from LDS with
// FP32 hi coordinates against a slightly widened cut-off, lists the
// survivors, and evaluates them with a separation rebuilt in FP64 from
// hi + residual.  Pairs whose rebuilt r^2 lies within a thin band of
// d_cut^2 (and, in FP32 modes, pairs closer than the close-pair radius; in
// FP64 mode, every pair) are re-evaluated from the FP64 wrapped positions
// exactly as the FP64 per-particle path does, so every mode decides the
// interacting set identically.
constexpr int TILE_CAP = 2240;
constexpr int LIST_K = 32;
constexpr int MAX_LAYERS = 8;
constexpr int MAX_ROWS = 64;
constexpr int MAX_CELLS = 896;
constexpr int MAX_HOME_ROWS = 48;
constexpr int CELLS_PT = (MAX_CELLS + SW_THREADS - 1) / SW_THREADS;

struct TileSmem {
  float4 hi[TILE_CAP];          // brick-frame FP32 coordinates, .w = sorted index bits
  uint2 res[TILE_CAP];          // int16 residuals (x | y << 16, z)
  uint16_t list[LIST_K * SW_THREADS];
  uint16_t cell_off[MAX_CELLS + 1];
  uint32_t cell_g0[MAX_CELLS];  // global sorted start of each tile cell
  uint8_t cell_row[MAX_CELLS];
  int32_t rowA0[MAX_ROWS], rowN[MAX_ROWS], rowCell0[MAX_ROWS + 1], rowB[MAX_ROWS], rowJ[MAX_ROWS], rowL[MAX_ROWS];
  int32_t layerRow0[MAX_LAYERS + 1], layerC[MAX_LAYERS], layerK[MAX_LAYERS], layerB0[MAX_LAYERS],
      layerNB[MAX_LAYERS];
  int32_t homeP0[MAX_HOME_ROWS], homeCum[MAX_HOME_ROWS + 1], homeB[MAX_HOME_ROWS], homeC[MAX_HOME_ROWS],
      homeCell0[MAX_HOME_ROWS];
  int32_t ntile, nrows, ncells, nhome, overflow;
};

__device__ inline int iclamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// separation of home i from image m of j exactly as the FP64 path forms it
__device__ inline double sep64(const CellGeom& g, const double4& pi64, const double4& pj64, const int* m,
                               double& dx, double& dy, double& dz) {
  const double sx = g.B[0] * m[0] + g.B[1] * m[1] + g.B[2] * m[2];
  const double sy = g.B[3] * m[0] + g.B[4] * m[1] + g.B[5] * m[2];
  const double sz = g.B[6] * m[0] + g.B[7] * m[1] + g.B[8] * m[2];
  const double xo = pi64.x - sx, yo = pi64.y - sy, zo = pi64.z - sz;
  dx = pj64.x - xo;
  dy = pj64.y - yo;
  dz = pj64.z - zo;
  return fma(dz, dz, fma(dy, dy, dx * dx));
}

// inclusive scan across one wave (64 lanes)
__device__ inline int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

template <int VAR, int PREC, bool DEBUG>
__global__ void __launch_bounds__(SW_THREADS) k_sweep_tile(SweepArgs A, CellGeom g) {
  __shared__ TileSmem S;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t nbrick = (uint32_t)A.nbx * A.nby * A.nbz;
  const uint32_t brick = xcd_block(blockIdx.x, gridDim.x);
  if (brick >= nbrick) return;  // grid == nbrick; uniform per block
  const int l0 = g.nc[0], l1 = g.nc[1], l2 = g.nc[2];
  const int bxi = (int)(brick % (uint32_t)A.nbx);
  const int byi = (int)((brick / (uint32_t)A.nbx) % (uint32_t)A.nby);
  const int bzi = (int)(brick / ((uint32_t)A.nbx * A.nby));
  const int a0 = bxi * A.sx, b0 = byi * A.sy, c0 = bzi * A.sz;
  const int sx = min(A.sx, l0 - a0), sy = min(A.sy, l1 - b0), sz = min(A.sz, l2 - c0);
  const int nlay = sz + 2;
  // brick-frame origin: the centre of the brick, in cell-index units
  const double uO[3] = {a0 + 0.5 * sx, b0 + 0.5 * sy, c0 + 0.5 * sz};
  // ---- tile layout: layers (z), rows (y) per layer, cells (x) per row ----
  if (wid == 0) {
    int nb = 0;
    if (lane < nlay && lane < MAX_LAYERS) {
      const int C = c0 - 1 + lane;
      const int kk = idiv_floor32(C, l2);
      int B0, B1;
      if (VAR == VAR_DS) {
        B0 = b0 - 1;
        B1 = b0 + sy;
      } else {
        const double fy = -(double)kk * g.B[5] / g.w[1];
        B0 = (int)floor(b0 - g.grow[1] + fy);
        B1 = (int)ceil(b0 + sy + g.grow[1] + fy) - 1;
      }
      nb = B1 - B0 + 1;
      S.layerC[lane] = C;
      S.layerK[lane] = kk;
      S.layerB0[lane] = B0;
      S.layerNB[lane] = nb;
    }
    const int inc = wave_incl_scan(nb);
    if (lane <= nlay && lane <= MAX_LAYERS) S.layerRow0[lane] = inc - nb;
    if (lane == 63) {
      S.nrows = inc;
      S.overflow = (inc > MAX_ROWS || nlay > MAX_LAYERS) ? 1 : 0;
    }
  }
  __syncthreads();
  if (S.overflow) goto overflow;
  // rows: x range of every row, then the prefix of cells over rows
  if (wid == 0) {
    int n = 0;
    if (lane < S.nrows) {
      const int r = lane;
      int L = 0;
      while (L + 1 < nlay && S.layerRow0[L + 1] <= r) ++L;
      const int B = S.layerB0[L] + (r - S.layerRow0[L]);
      const int j = idiv_floor32(B, l1);
      const int kk = S.layerK[L];
      int A0, A1;
      if (VAR == VAR_DS) {
        A0 = a0 - 1;
        A1 = a0 + sx;
      } else {
        const double fx = -((double)j * g.B[1] + (double)kk * g.B[2]) / g.w[0];
        A0 = (int)floor(a0 - g.grow[0] + fx);
        A1 = (int)ceil(a0 + sx + g.grow[0] + fx) - 1;
      }
      n = A1 - A0 + 1;
      S.rowA0[r] = A0;
      S.rowN[r] = n;
      S.rowB[r] = B;
      S.rowJ[r] = j;
      S.rowL[r] = L;
    }
    const int inc = wave_incl_scan(n);
    if (lane < S.nrows) S.rowCell0[lane] = inc - n;
    if (lane == 63) {
      S.rowCell0[S.nrows] = inc;
      S.ncells = inc;
      if (inc > MAX_CELLS) S.overflow = 1;
    }
  }
  __syncthreads();
  if (S.overflow) goto overflow;
  // cells: global id and particle count, CELLS_PT consecutive cells per
  // thread, offsets by a block-wide scan
  {
    uint32_t cntv[CELLS_PT], sum = 0;
#pragma unroll
    for (int q = 0; q < CELLS_PT; ++q) {
      const int t = tid * CELLS_PT + q;
      cntv[q] = 0;
      if (t < S.ncells) {
        int lo = 0, hi = S.nrows - 1;
        while (lo < hi) {  // last row with rowCell0 <= t
          const int mid = (lo + hi + 1) >> 1;
          if (S.rowCell0[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int r = lo, L = S.rowL[r];
        const int Aq = S.rowA0[r] + (t - S.rowCell0[r]);
        const int i = idiv_floor32(Aq, l0);
        const int ax = Aq - i * l0;
        const int by = S.rowB[r] - S.rowJ[r] * l1;
        const int cz = S.layerC[L] - S.layerK[L] * l2;
        const uint32_t gid = (uint32_t)ax + (uint32_t)l0 * ((uint32_t)by + (uint32_t)l1 * (uint32_t)cz);
        const uint32_t st = A.cstart[gid], en = A.cstart[gid + 1];
        S.cell_g0[t] = st;
        S.cell_row[t] = (uint8_t)r;
        cntv[q] = en - st;
        sum += en - st;
      }
    }
    uint32_t total;
    uint32_t run = block_excl_scan(sum, &total);
#pragma unroll
    for (int q = 0; q < CELLS_PT; ++q) {
      const int t = tid * CELLS_PT + q;
      if (t < S.ncells) S.cell_off[t] = (uint16_t)min(run, 65535u);
      run += cntv[q];
    }
    if (tid == 0) {
      S.cell_off[S.ncells] = (uint16_t)min(total, 65535u);
      S.ntile = (int)min(total, 1u << 30);
      if (total > (uint32_t)TILE_CAP) S.overflow = 1;
    }
  }
  __syncthreads();
  if (S.overflow) goto overflow;
  // ---- stage positions, one row per wave at a time: X = (offset from own
  //      cell centre) + (centre of the cell image) - (brick centre), kept as
  //      FP32 hi + int16 residual in units of res_unit ----
  {
    const double ru_inv = 1.0 / A.res_unit;
    for (int r = wid; r < S.nrows; r += SW_THREADS / 64) {
      const int L = S.rowL[r];
      const int cbeg = S.rowCell0[r], cend = S.rowCell0[r + 1];
      const int pbeg = S.cell_off[cbeg], pend = S.cell_off[cend];
      const int Bq = S.rowB[r], Cq = S.layerC[L];
      const double shx = (VAR == VAR_DO) ? ((double)S.rowJ[r] * g.B[1] + (double)S.layerK[L] * g.B[2]) : 0.0;
      const double shy = (VAR == VAR_DO) ? (double)S.layerK[L] * g.B[5] : 0.0;
      for (int p = pbeg + lane; p < pend; p += 64) {
        int t = cbeg;
        while (t + 1 < cend && (int)S.cell_off[t + 1] <= p) ++t;
        const uint32_t gj = S.cell_g0[t] + (uint32_t)(p - S.cell_off[t]);
        const float4 h4 = A.pos32[gj];
        const float4 l4 = A.pos32lo[gj];
        const int Aq = S.rowA0[r] + (t - cbeg);
        // cell-image centre minus the brick centre, from exact index offsets
        const double du[3] = {(Aq + 0.5) - uO[0], (Bq + 0.5) - uO[1], (Cq + 0.5) - uO[2]};
        double X[3];
        if (VAR == VAR_DS) {
          for (int d = 0; d < 3; ++d)
            X[d] = g.cen[3 * d] * du[0] + g.cen[3 * d + 1] * du[1] + g.cen[3 * d + 2] * du[2];
        } else {
          X[0] = du[0] * g.w[0] + shx;
          X[1] = du[1] * g.w[1] + shy;
          X[2] = du[2] * g.w[2];
        }
        X[0] += (double)h4.x + (double)l4.x;
        X[1] += (double)h4.y + (double)l4.y;
        X[2] += (double)h4.z + (double)l4.z;
        const float hx = (float)X[0], hy = (float)X[1], hz = (float)X[2];
        const int rx = iclamp((int)rint((X[0] - hx) * ru_inv), -32767, 32767);
        const int ry = iclamp((int)rint((X[1] - hy) * ru_inv), -32767, 32767);
        const int rz = iclamp((int)rint((X[2] - hz) * ru_inv), -32767, 32767);
        S.hi[p] = make_float4(hx, hy, hz, __uint_as_float(gj));
        S.res[p] = make_uint2(((uint32_t)rx & 0xffffu) | ((uint32_t)ry << 16), (uint32_t)rz & 0xffffu);
      }
    }
  }
  // home rows: (b, c) rows of the brick, each a contiguous run of tile cells
  if (wid == 0) {
    const int nhr = sy * sz;
    int cntr = 0;
    if (lane < nhr && lane < MAX_HOME_ROWS) {
      const int cc = lane / sy, bb = lane - cc * sy;
      const int L = cc + 1;
      const int r = S.layerRow0[L] + (b0 + bb - S.layerB0[L]);
      const int t0 = S.rowCell0[r] + (a0 - S.rowA0[r]);
      S.homeCell0[lane] = t0;
      S.homeP0[lane] = S.cell_off[t0];
      S.homeB[lane] = b0 + bb;
      S.homeC[lane] = c0 + cc;
      cntr = S.cell_off[t0 + sx] - S.cell_off[t0];
    }
    const int inc = wave_incl_scan(cntr);
    if (lane <= nhr && lane <= MAX_HOME_ROWS) S.homeCum[lane] = inc - cntr;
    if (lane == 63) {
      S.nhome = inc;
      if (nhr > MAX_HOME_ROWS) S.overflow = 1;
    }
  }
  __syncthreads();
  if (S.overflow) goto overflow;
  {
    const int nhr = sy * sz;
    const float rc2c = A.rc2c;
    const double res_unit = A.res_unit;
    uint32_t st4[4] = {0, 0, 0, 0};
    double v7[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int hbase = 0; hbase < S.nhome; hbase += SW_THREADS) {
      const int h = hbase + tid;
      const bool active = h < S.nhome;
      Acc<PREC, DEBUG> acc;
      if (active) {
        int hr = 0;
        while (hr + 1 < nhr && S.homeCum[hr + 1] <= h) ++hr;
        const int pi = S.homeP0[hr] + (h - S.homeCum[hr]);
        // home cell: which cell of the home row holds pi
        int tc = S.homeCell0[hr];
        while ((int)S.cell_off[tc + 1] <= pi) ++tc;
        const int a = a0 + (tc - S.homeCell0[hr]);
        const int b = S.homeB[hr], c = S.homeC[hr];
        const float4 hi4 = S.hi[pi];
        const uint2 rs = S.res[pi];
        const uint32_t gi = __float_as_uint(hi4.w);
        const double4 pi64 = A.pos64[gi];
        const int4 wi = DEBUG ? A.wrap[gi] : make_int4(0, 0, 0, 0);
        const double xih = hi4.x, yih = hi4.y, zih = hi4.z;
        const double xir = (double)(int16_t)(rs.x & 0xffffu), yir = (double)(int16_t)(rs.x >> 16),
                     zir = (double)(int16_t)(rs.y & 0xffffu);
        const float xi = hi4.x, yi = hi4.y, zi = hi4.z;
        // one listed candidate: separation rebuilt in FP64 from hi + residual
        auto eval = [&](const float4& q, const uint2& qr) {
          const double dx = ((double)q.x - xih) + ((double)(int16_t)(qr.x & 0xffffu) - xir) * res_unit;
          const double dy = ((double)q.y - yih) + ((double)(int16_t)(qr.x >> 16) - yir) * res_unit;
          const double dz = ((double)q.z - zih) + ((double)(int16_t)(qr.y & 0xffffu) - zir) * res_unit;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const bool band = fabs(r2 - A.rc2) <= A.band64;
          const bool close = r2 < A.rclose2_64;
          if (PREC == 0 || band || close) {
            // exact path: recover the lattice image and re-form the
            // separation from FP64 wrapped positions
            const uint32_t gj = __float_as_uint(q.w);
            const double4 pj64 = A.pos64[gj];
            const double vx = dx - (pj64.x - pi64.x), vy = dy - (pj64.y - pi64.y), vz = dz - (pj64.z - pi64.z);
            int m[3];
            for (int d = 0; d < 3; ++d)
              m[d] = (int)rint(g.Binv[3 * d] * vx + g.Binv[3 * d + 1] * vy + g.Binv[3 * d + 2] * vz);
            double ex, ey, ez;
            const double e2 = sep64(g, pi64, pj64, m, ex, ey, ez);
            acc.fp64 += (PREC == 0) ? 0u : 1u;
            if (e2 < A.rc2) {
              if (PREC == 0 || close)
                pair64(acc, A.p64, ex, ey, ez, e2);
              else
                pair32(acc, A.p32, A.p64, (float)ex, (float)ey, (float)ez, (float)e2, e2);
              acc.pairs += 1;
              debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, gj, m, wi);
            }
          } else if (r2 < A.rc2) {
            pair32(acc, A.p32, A.p64, (float)dx, (float)dy, (float)dz, (float)r2, r2);
            acc.pairs += 1;
            if (DEBUG) {
              // digest of the pair as accepted here: its image, recovered as
              // on the exact path
              const uint32_t gj = __float_as_uint(q.w);
              const double4 pj64 = A.pos64[gj];
              const double vx = dx - (pj64.x - pi64.x), vy = dy - (pj64.y - pi64.y), vz = dz - (pj64.z - pi64.z);
              int m[3];
              for (int d = 0; d < 3; ++d)
                m[d] = (int)rint(g.Binv[3 * d] * vx + g.Binv[3 * d + 1] * vy + g.Binv[3 * d + 2] * vz);
              debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, gj, m, wi);
            }
          }
        };
        for (int dzl = 0; dzl < 3; ++dzl) {
          const int L = (c - c0) + dzl;
          const int nr = S.layerNB[L] - (sy - 1);
          const int r0 = S.layerRow0[L] + (b - b0);
          int cnt = 0;
          // evaluate this lane's listed candidates, two at a time
          auto flush = [&]() {
            int e = 0;
            for (; e + 1 < cnt; e += 2) {
              const int p0 = S.list[e * SW_THREADS + tid], p1 = S.list[(e + 1) * SW_THREADS + tid];
              const float4 q0 = S.hi[p0], q1 = S.hi[p1];
              const uint2 r0v = S.res[p0], r1v = S.res[p1];
              if (p0 != pi) eval(q0, r0v);
              if (p1 != pi) eval(q1, r1v);
            }
            if (e < cnt) {
              const int p0 = S.list[e * SW_THREADS + tid];
              if (p0 != pi) eval(S.hi[p0], S.res[p0]);
            }
            cnt = 0;
          };
          for (int rq = 0; rq < nr; ++rq) {
            const int r = r0 + rq;
            const int nc1 = S.rowN[r] - (sx - 1);
            const int t0 = S.rowCell0[r] + (a - a0);
            const int plo = S.cell_off[t0], phi = S.cell_off[t0 + nc1];
            acc.cand += (uint32_t)(phi - plo);
            st4[3] += (uint32_t)nc1;
            // four independent LDS reads in flight per step; every
            // candidate is written to the list slot and the count advanced
            // only for survivors (no branch per candidate)
            int p = plo;
            for (; p + 4 <= phi; p += 4) {
              const float4 q0 = S.hi[p], q1 = S.hi[p + 1], q2 = S.hi[p + 2], q3 = S.hi[p + 3];
              float d0 = q0.x - xi, d1 = q0.y - yi, d2 = q0.z - zi;
              const float s0 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
              d0 = q1.x - xi; d1 = q1.y - yi; d2 = q1.z - zi;
              const float s1 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
              d0 = q2.x - xi; d1 = q2.y - yi; d2 = q2.z - zi;
              const float s2 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
              d0 = q3.x - xi; d1 = q3.y - yi; d2 = q3.z - zi;
              const float s3 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
              S.list[cnt * SW_THREADS + tid] = (uint16_t)p;
              cnt += (s0 < rc2c) ? 1 : 0;
              S.list[cnt * SW_THREADS + tid] = (uint16_t)(p + 1);
              cnt += (s1 < rc2c) ? 1 : 0;
              S.list[cnt * SW_THREADS + tid] = (uint16_t)(p + 2);
              cnt += (s2 < rc2c) ? 1 : 0;
              S.list[cnt * SW_THREADS + tid] = (uint16_t)(p + 3);
              cnt += (s3 < rc2c) ? 1 : 0;
              // the whole wave evaluates together as soon as one lane's list
              // is nearly full (a lane flushing alone would idle the rest)
              if (__ballot(cnt > LIST_K - 5) != 0) flush();
            }
            for (; p < phi; ++p) {
              const float4 q0 = S.hi[p];
              const float d0 = q0.x - xi, d1 = q0.y - yi, d2 = q0.z - zi;
              const float s0 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
              S.list[cnt * SW_THREADS + tid] = (uint16_t)p;
              cnt += (s0 < rc2c) ? 1 : 0;
            }
            if (__ballot(cnt > LIST_K - 5) != 0) flush();
          }
          flush();
        }
        acc.cand -= 1;  // the home particle itself
        write_particle<VAR, PREC, DEBUG>(A, g, gi, acc);
      }
      double v[7];
      acc_energy(acc, v);
      for (int kq = 0; kq < 7; ++kq) v7[kq] += v[kq];
      st4[0] += acc.cand;
      st4[1] += acc.pairs;
      st4[2] += acc.fp64;
    }
    block_commit(A, brick, v7, st4);
    return;
  }
overflow:
  // the neighbourhood does not fit: hand the brick to the fallback kernel
  if (tid == 0) {
    const uint32_t q = atomicAdd(A.overflow, 1u);
    A.overflow[1 + q] = brick;
  }
}

// bricks listed by k_sweep_tile, one per workgroup iteration, swept per
// particle from global memory
template <int VAR, int PREC, bool DEBUG>
__global__ void __launch_bounds__(SW_THREADS) k_sweep_fallback(SweepArgs A, CellGeom g) {
  __shared__ pl_entry plist[PL_K * SW_THREADS_P];
  const uint32_t nover = A.overflow[0];
  const int l0 = g.nc[0], l1 = g.nc[1], l2 = g.nc[2];
  for (uint32_t q = blockIdx.x; q < nover; q += gridDim.x) {
    const uint32_t brick = A.overflow[1 + q];
    const int bxi = (int)(brick % (uint32_t)A.nbx);
    const int byi = (int)((brick / (uint32_t)A.nbx) % (uint32_t)A.nby);
    const int bzi = (int)(brick / ((uint32_t)A.nbx * A.nby));
    const int a0 = bxi * A.sx, b0 = byi * A.sy, c0 = bzi * A.sz;
    const int sx = min(A.sx, l0 - a0), sy = min(A.sy, l1 - b0), sz = min(A.sz, l2 - c0);
    double v7[7] = {0, 0, 0, 0, 0, 0, 0};
    uint32_t st4[4] = {0, 0, 0, 0};
    for (int cc = 0; cc < sz; ++cc)
      for (int bb = 0; bb < sy; ++bb) {
        const uint32_t id0 = (uint32_t)a0 + (uint32_t)l0 * ((uint32_t)(b0 + bb) + (uint32_t)l1 * (uint32_t)(c0 + cc));
        const uint32_t s0 = A.cstart[id0], s1 = A.cstart[id0 + sx];
        for (uint32_t s = s0 + threadIdx.x; s < s1; s += SW_THREADS) {
          Acc<PREC, DEBUG> acc;
          uint32_t nbh = 0;
          PairList L(plist + threadIdx.x);
          sweep_particle<VAR, PREC, DEBUG>(A, g, s, acc, nbh, L);
          write_particle<VAR, PREC, DEBUG>(A, g, s, acc);
          double v[7];
          acc_energy(acc, v);
          for (int k = 0; k < 7; ++k) v7[k] += v[k];
          st4[0] += acc.cand;
          st4[1] += acc.pairs;
          st4[2] += acc.fp64;
          st4[3] += nbh;
        }
      }
    block_commit(A, brick, v7, st4);
  }
}

// one thread per particle in cell order, neighbour data straight from
// global memory (L1/L2); partial sums per workgroup (swp_threads(VAR)
// lanes).  Four waves per SIMD (at most 128 VGPRs; the 10-deep list of
// 16-byte entries, whose LDS the block's reduction reuses, makes 160 bytes
// per lane, so 16 waves fill the CU's 160 KB) hide more load latency than
// three: measured 0.80 -> 0.70 ms at 1 M LJ.
template <int VAR, int PREC, bool DEBUG>
__global__ void __launch_bounds__(swp_threads(VAR), 4) k_sweep_particle(SweepArgs A, CellGeom g) {
  constexpr int BT = swp_threads(VAR);
  __shared__ SweepSmemT<BT> sm;
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t s = lb * BT + threadIdx.x;
  Acc<PREC, DEBUG> acc;
  uint32_t nbh = 0;
  if (s < A.n) {
    PairListS<BT> L(sm.plist + threadIdx.x);
    sweep_particle<VAR, PREC, DEBUG>(A, g, s, acc, nbh, L);
    write_particle<VAR, PREC, DEBUG>(A, g, s, acc);
  }
  double v[7];
  acc_energy(acc, v);
  const uint32_t st4[4] = {acc.cand, acc.pairs, acc.fp64, nbh};
  block_commit<BT / 64>(A, lb, v, st4, sm.red);
}

// first level of the fixed-order reduction: block r sums partial slots
// [256 r, 256 r + 256) into out[r]
__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partial, uint32_t nb,
                                                         double* __restrict__ out) {
  __shared__ double red[4][PART_STRIDE];
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < PART_STRIDE; ++k) {
    const double t = warp_sum((b < nb && k != 7) ? partial[PART_STRIDE * (size_t)b + k] : 0.0);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < PART_STRIDE)
    out[PART_STRIDE * (size_t)blockIdx.x + threadIdx.x] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// U = scale sum u, W = scale sum w (scale 1/2 for the full list, which counts
// each pair twice; 1 for the half list); DO's W is rotated back,
// W_cart = Q W' Q^T.
__global__ void k_finalize(const double* __restrict__ partial, uint32_t nb, CellGeom g, double* __restrict__ U,
                           double* __restrict__ W, double scale, unsigned long long* __restrict__ stats) {
  __shared__ double red[4][PART_STRIDE];
  double v[PART_STRIDE] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
    for (int k = 0; k < PART_STRIDE; ++k)
      if (k != 7) v[k] += partial[PART_STRIDE * (size_t)b + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < PART_STRIDE; ++k) {
    const double t = warp_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4)  // statistics: integers, exact in FP64
    stats[threadIdx.x] = (unsigned long long)(((red[0][8 + threadIdx.x] + red[1][8 + threadIdx.x]) +
                                               red[2][8 + threadIdx.x]) + red[3][8 + threadIdx.x]);
  if (threadIdx.x == 0) {
    double s[7];
    for (int k = 0; k < 7; ++k) s[k] = scale * (((red[0][k] + red[1][k]) + red[2][k]) + red[3][k]);
    U[0] = s[0];
    const double Wp[9] = {s[1], s[4], s[5], s[4], s[2], s[6], s[5], s[6], s[3]};
    if (g.variant == VAR_DO) {
      double T[9], Wc[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          T[3 * r + c] = g.Q[3 * r] * Wp[c] + g.Q[3 * r + 1] * Wp[3 + c] + g.Q[3 * r + 2] * Wp[6 + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Wc[3 * r + c] = T[3 * r] * g.Q[3 * c] + T[3 * r + 1] * g.Q[3 * c + 1] + T[3 * r + 2] * g.Q[3 * c + 2];
      for (int k = 0; k < 9; ++k) W[k] = Wc[k];
    } else {
      for (int k = 0; k < 9; ++k) W[k] = Wp[k];
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }


// two-level fixed-order reduction of the nb partial slots into U, W, stats
static void finalize(const SweepLaunch& L, hipStream_t st, uint32_t nb, double scale) {
  const uint32_t nr = cdiv(nb, 256);
  k_reduce_partials<<<nr, 256, 0, st>>>(L.args->partial, nb, L.args->partial2);
  k_finalize<<<1, 256, 0, st>>>(L.args->partial2, nr, *L.g, L.U, L.W, scale, L.args->stats);
}

template <int VAR, int PREC, bool DEBUG>
static void sweep_t(const SweepLaunch& L, hipStream_t st, uint32_t nslots) {
  if (L.mode == SWEEP_TILED) {
    k_sweep_tile<VAR, PREC, DEBUG><<<nslots, SW_THREADS, 0, st>>>(*L.args, *L.g);
    k_sweep_fallback<VAR, PREC, DEBUG><<<min(nslots, 1024u), SW_THREADS, 0, st>>>(*L.args, *L.g);
  } else {
    k_sweep_particle<VAR, PREC, DEBUG><<<nslots, swp_threads(VAR), 0, st>>>(*L.args, *L.g);
  }
}

hipError_t launch_sweep(const SweepLaunch& L, hipStream_t st) {
  const uint32_t n = L.args->n;
  const uint32_t nbrick = (L.mode == SWEEP_TILED)  ? (uint32_t)L.args->nbx * L.args->nby * L.args->nbz
                          : (L.mode == SWEEP_HALF) ? cdiv(n, SW_THREADS)
                                                   : cdiv(n, swp_threads(L.g->variant));
  if (L.mode == SWEEP_HALF) {
    k_fill_u32<<<1, 64, 0, st>>>((uint32_t*)L.args->stats, 8, 0u);
    if (n > 0) {
      const hipError_t e = launch_half(L, st, nbrick);
      if (e != hipSuccess) return e;
      finalize(L, st, nbrick, 1.0);
    } else {
      k_zero_f64<<<1, 64, 0, st>>>(L.U, 1);
      k_zero_f64<<<1, 64, 0, st>>>(L.W, 9);
    }
    return hipGetLastError();
  }
  if (n > 0 && nbrick > 0) {
    // the finalisation writes every statistic; the overflow queue exists for
    // the tiled sweep only
    if (L.mode == SWEEP_TILED) k_fill_u32<<<1, 64, 0, st>>>(L.args->overflow, 1, 0u);
    const int var = L.g->variant, prec = L.precision;
    const bool dbg = L.debug;
#define NCL_SW(V, P)                                      \
  if (var == V && prec == P) {                            \
    if (dbg) sweep_t<V, P, true>(L, st, nbrick);          \
    else sweep_t<V, P, false>(L, st, nbrick);             \
  }
    NCL_SW(VAR_DS, 0) NCL_SW(VAR_DS, 1) NCL_SW(VAR_DS, 2)
    NCL_SW(VAR_DO, 0) NCL_SW(VAR_DO, 1) NCL_SW(VAR_DO, 2)
#undef NCL_SW
    finalize(L, st, nbrick, 0.5);
  } else {
    k_fill_u32<<<1, 64, 0, st>>>((uint32_t*)L.args->stats, 8, 0u);
    k_zero_f64<<<1, 64, 0, st>>>(L.U, 1);
    k_zero_f64<<<1, 64, 0, st>>>(L.W, 9);
  }
  return hipGetLastError();
}

}  // namespace ncl
