// HIP kernels for gfx950: cell build (Sec. 4.1 / 4.2 of Dobson, Fox &
// Saracino, arXiv:1412.3784: particles are assigned to cells at every step)
// and the neighbourhood sweep that evaluates forces, energy and virial.
//
// Data layout in HBM (sorted = cell order, x fastest, particles of a cell by
// ascending input index):
//   cell_of[N], rank[N]    u32, input order      (bin_count)
//   count[Nc], cstart[Nc+1] u32                  (histogram, exclusive scan)
//   perm[N]                u32  sorted slot -> input index
//   pos64[N]               double4 (x, y, z, -) wrapped FP64 position in the
//                          variant's frame (Cartesian for DS, rotated for DO)
//   pos32[N]               float4 (ox, oy, oz, cell id bits): FP32 offset from
//                          the FP64 centre of the particle's cell (high word)
//   pos32lo[N]             float4 (ox, oy, oz, -): low word, offset - high
//   wrap[N]                int4 lattice image of the wrap (debug only)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geometry.hpp"
#include "kernels.hpp"

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

// blockIdx -> logical block so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of cells and keeps
// its neighbour data in its own L2.
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nb) {
  const uint32_t nx = 8, per = nb / nx, rem = nb % nx;
  const uint32_t x = bid % nx, idx = bid / nx;
  return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__global__ void k_bin_count(const double* __restrict__ x, uint32_t n, CellGeom g, uint32_t* __restrict__ cell_of,
                            uint32_t* __restrict__ rank, uint32_t* __restrict__ count, int* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double p[3] = {x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2]};
  double xw[3];
  int32_t img[3];
  bool bad = false;
  const uint32_t c = locate(g, p, xw, img, &bad);
  if (bad) atomicOr(err, 1);
  cell_of[i] = c;
  rank[i] = atomicAdd(&count[c], 1u);
}

// exclusive scan of u32 counts, three passes: per-block totals, a scan of
// the totals in one block, then the per-block scan with its offset.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

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

__global__ void k_scan_totals(const uint32_t* __restrict__ in, uint32_t n, uint32_t* __restrict__ tot) {
  const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) s += (base + k < n) ? in[base + k] : 0u;
  uint32_t total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

__global__ void k_scan_top(uint32_t* __restrict__ tot, uint32_t nb) {
  // one block: exclusive scan of the block totals in place, in chunks
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nb; base += SCAN_THREADS) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? tot[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan(v, &total);
    if (i < nb) tot[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, uint32_t n, const uint32_t* __restrict__ tot,
                             uint32_t* __restrict__ out) {
  const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS], s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = tot[blockIdx.x] + block_excl_scan(s, &total);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (base < n && base + SCAN_ITEMS >= n) out[n] = run;  // the thread holding the last element
}

__global__ void k_scatter(const uint32_t* __restrict__ cell_of, const uint32_t* __restrict__ rank, uint32_t n,
                          const uint32_t* __restrict__ cstart, uint32_t* __restrict__ perm) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  perm[cstart[cell_of[i]] + rank[i]] = i;
}

// order each cell's particles by input index (insertion sort; cells hold a
// handful of particles), and record the largest occupancy
__global__ void k_cell_sort(const uint32_t* __restrict__ cstart, uint32_t ncells, uint32_t* __restrict__ perm,
                            uint32_t* __restrict__ maxocc) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const uint32_t b = cstart[c], e = cstart[c + 1];
  for (uint32_t k = b + 1; k < e; ++k) {
    const uint32_t v = perm[k];
    uint32_t q = k;
    while (q > b && perm[q - 1] > v) {
      perm[q] = perm[q - 1];
      --q;
    }
    perm[q] = v;
  }
  atomicMax(maxocc, e - b);
}

__global__ void k_gather(const double* __restrict__ x, const uint32_t* __restrict__ perm, uint32_t n, CellGeom g,
                         double4* __restrict__ pos64, float4* __restrict__ pos32, float4* __restrict__ pos32lo,
                         int4* __restrict__ wrap) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t i = perm[s];
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
  pos64[s] = make_double4(xw[0], xw[1], xw[2], 0.0);
  // FP32 offset from the cell centre as a hi + lo pair (hi + lo carries the
  // FP64 offset to ~48 bits); the sweep screens with hi alone
  const double o[3] = {xw[0] - cen[0], xw[1] - cen[1], xw[2] - cen[2]};
  const float hi[3] = {(float)o[0], (float)o[1], (float)o[2]};
  pos32[s] = make_float4(hi[0], hi[1], hi[2], __uint_as_float(c));
  pos32lo[s] = make_float4((float)(o[0] - hi[0]), (float)(o[1] - hi[1]), (float)(o[2] - hi[2]), 0.f);
  if (wrap) wrap[s] = make_int4(img[0], img[1], img[2], 0);
}

// ---------------------------------------------------------------------------
// the neighbourhood sweep
// ---------------------------------------------------------------------------
// order-independent pair key hash: SplitMix64's output function (Steele, Lea
// & Flood 2014) on (j << 32) | three 10-bit biased image components
__device__ inline uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <int PREC, bool DEBUG>
struct Acc {
  // FP32 modes: per-particle FP32 sums (+ Kahan terms), FP64 sums for the
  // pairs taken on the FP64 path.  FP64 mode uses only the double fields.
  float fx = 0.f, fy = 0.f, fz = 0.f, u = 0.f;
  float kx = 0.f, ky = 0.f, kz = 0.f, ku = 0.f;
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
  acc.gx -= fs * dx;
  acc.gy -= fs * dy;
  acc.gz -= fs * dz;
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

template <int PREC, bool DEBUG>
__device__ inline void pair32(Acc<PREC, DEBUG>& acc, const Pot32& p, float dx, float dy, float dz, float r2) {
  const float r2i = __builtin_amdgcn_rcpf(r2);
  const float s2 = p.sig2 * r2i;
  const float s6 = s2 * s2 * s2;
  const float fs = r2i * s6 * fmaf(p.eps48, s6, -p.eps24);
  const float phi = fmaf(s6, fmaf(p.eps4, s6, -p.eps4), -p.shift);
  if (PREC == 2) {
    kahan_add(acc.fx, acc.kx, -fs * dx);
    kahan_add(acc.fy, acc.ky, -fs * dy);
    kahan_add(acc.fz, acc.kz, -fs * dz);
    kahan_add(acc.u, acc.ku, phi);
  } else {
    acc.fx = fmaf(-fs, dx, acc.fx);
    acc.fy = fmaf(-fs, dy, acc.fy);
    acc.fz = fmaf(-fs, dz, acc.fz);
    acc.u += phi;
  }
  const float fdx = fs * dx, fdy = fs * dy;
  acc.w[0] = fmaf(fdx, dx, acc.w[0]);
  acc.w[1] = fmaf(fdy, dy, acc.w[1]);
  acc.w[2] = fmaf(fs * dz, dz, acc.w[2]);
  acc.w[3] = fmaf(fdx, dy, acc.w[3]);
  acc.w[4] = fmaf(fdx, dz, acc.w[4]);
  acc.w[5] = fmaf(fdy, dz, acc.w[5]);
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
  uint64_t key = ((uint64_t)A.perm[j]) << 32;
  key |= ((uint64_t)((mk[0] + 512) & 0x3ff)) << 20;
  key |= ((uint64_t)((mk[1] + 512) & 0x3ff)) << 10;
  key |= ((uint64_t)((mk[2] + 512) & 0x3ff));
  hsh += splitmix_out(key);
  cnt += 1;
}

// Visit one neighbour cell `cj` seen through lattice image `m` (in the
// basis Lred); `dc` is the FP64 vector from the home cell's centre to the
// centre of that image of cj, `sh` the lattice shift B m in the frame.
template <int PREC, bool DEBUG>
__device__ inline void visit_cell(Acc<PREC, DEBUG>& acc, const SweepArgs& A, const CellGeom& g, uint32_t s,
                                  uint32_t cj, bool zero_image, const double* dc, const int* m,
                                  const double* oi, const double4& pi64, const int4& wi) {
  const uint32_t st = A.cstart[cj], en = A.cstart[cj + 1];
  const uint32_t self = zero_image ? s : 0xffffffffu;
  acc.cand += (en - st) - ((zero_image && s >= st && s < en) ? 1u : 0u);
  if (PREC == 0) {
    const double sx = g.B[0] * m[0] + g.B[1] * m[1] + g.B[2] * m[2];
    const double sy = g.B[3] * m[0] + g.B[4] * m[1] + g.B[5] * m[2];
    const double sz = g.B[6] * m[0] + g.B[7] * m[1] + g.B[8] * m[2];
    const double xo = pi64.x - sx, yo = pi64.y - sy, zo = pi64.z - sz;
    for (uint32_t j = st; j < en; ++j) {
      const double4 pj = A.pos64[j];
      const double dx = pj.x - xo, dy = pj.y - yo, dz = pj.z - zo;
      const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      if (r2 < A.rc2 && j != self) {
        pair64(acc, A.p64, dx, dy, dz, r2);
        acc.pairs += 1;
        debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
      }
    }
  } else {
    // home position relative to the centre of this image of cj, FP64 split
    // into FP32 hi + lo
    const double vx = oi[0] - dc[0], vy = oi[1] - dc[1], vz = oi[2] - dc[2];
    const float xo = (float)vx, yo = (float)vy, zo = (float)vz;
    const float xl = (float)(vx - xo), yl = (float)(vy - yo), zl = (float)(vz - zo);
    for (uint32_t j = st; j < en; ++j) {
      const float4 pj = A.pos32[j];
      float dx = pj.x - xo, dy = pj.y - yo, dz = pj.z - zo;
      float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
      if (r2 < A.rc2_hi && j != self) {
        if (r2 > A.rc2_lo || r2 < A.rclose2) {
          // re-evaluate from the FP64 positions exactly as the FP64 mode does
          const double sx = g.B[0] * m[0] + g.B[1] * m[1] + g.B[2] * m[2];
          const double sy = g.B[3] * m[0] + g.B[4] * m[1] + g.B[5] * m[2];
          const double sz = g.B[6] * m[0] + g.B[7] * m[1] + g.B[8] * m[2];
          const double xo64 = pi64.x - sx, yo64 = pi64.y - sy, zo64 = pi64.z - sz;
          const double4 pj64 = A.pos64[j];
          const double ex = pj64.x - xo64, ey = pj64.y - yo64, ez = pj64.z - zo64;
          const double e2 = fma(ez, ez, fma(ey, ey, ex * ex));
          acc.fp64 += 1;
          if (e2 < A.rc2) {
            pair64(acc, A.p64, ex, ey, ez, e2);
            acc.pairs += 1;
            debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
          }
        } else {
          // refine the separation with the low words: d = (hi_j - hi_i) + (lo_j - lo_i)
          const float4 pl = A.pos32lo[j];
          dx += pl.x - xl;
          dy += pl.y - yl;
          dz += pl.z - zl;
          r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
          pair32(acc, A.p32, dx, dy, dz, r2);
          acc.pairs += 1;
          debug_pair<DEBUG>(acc.dcount, acc.dhash, A, g, j, m, wi);
        }
      }
    }
  }
}

__device__ inline double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int VAR, int PREC, bool DEBUG>
__global__ void __launch_bounds__(256) k_sweep(SweepArgs A, CellGeom g) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t s = lb * blockDim.x + threadIdx.x;
  const bool active = s < A.n;
  Acc<PREC, DEBUG> acc;
  uint32_t nbh = 0;
  if (active) {
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
            for (int k = 0; k < 3; ++k) {
              m[k] = idiv_floor32(u[k], g.nc[k]);
              w[k] = u[k] - m[k] * g.nc[k];
            }
            const uint32_t cj = (uint32_t)w[0] + (uint32_t)g.nc[0] * ((uint32_t)w[1] + (uint32_t)g.nc[1] * (uint32_t)w[2]);
            const bool zero = (dx == 0 && dy == 0 && dz == 0);
            visit_cell<PREC, DEBUG>(acc, A, g, s, cj, zero, g.ds_delta[q], m, oi, pi64, wi);
            ++nbh;
          }
    } else {
      // rectangular cells of the rotated box; layer k (z) is offset by
      // k r23 in y, row (j, k) by j r12 + k r13 in x
      const double w0 = g.w[0], w1 = g.w[1], w2 = g.w[2];
      for (int dz = -1; dz <= 1; ++dz) {
        const int C = c + dz;
        const int k = idiv_floor32(C, g.nc[2]);
        const int cz = C - k * g.nc[2];
        const double fy = -(double)k * g.B[5] / w1;
        const int B0 = (int)floor(b - g.grow[1] + fy);
        const int B1 = (int)ceil(b + 1 + g.grow[1] + fy) - 1;
        for (int Bq = B0; Bq <= B1; ++Bq) {
          const int j = idiv_floor32(Bq, g.nc[1]);
          const int by = Bq - j * g.nc[1];
          const double xs = (double)j * g.B[1] + (double)k * g.B[2];
          const double fx = -xs / w0;
          const int A0 = (int)floor(a - g.grow[0] + fx);
          const int A1 = (int)ceil(a + 1 + g.grow[0] + fx) - 1;
          for (int Aq = A0; Aq <= A1; ++Aq) {
            const int i = idiv_floor32(Aq, g.nc[0]);
            const int ax = Aq - i * g.nc[0];
            const uint32_t cj = (uint32_t)ax + (uint32_t)g.nc[0] * ((uint32_t)by + (uint32_t)g.nc[1] * (uint32_t)cz);
            const int m[3] = {i, j, k};
            // centre of this image of cj minus the home centre
            const double dcv[3] = {(Aq - a) * w0 + xs, (Bq - b) * w1 + (double)k * g.B[5], (C - c) * w2};
            const bool zero = (i == 0 && j == 0 && k == 0 && cj == hc);
            visit_cell<PREC, DEBUG>(acc, A, g, s, cj, zero, dcv, m, oi, pi64, wi);
            ++nbh;
          }
        }
      }
    }
    // per-particle outputs, rotated back to Cartesian for DO
    double F[3];
    if (PREC == 0) {
      F[0] = acc.gx; F[1] = acc.gy; F[2] = acc.gz;
    } else if (PREC == 2) {
      F[0] = ((double)acc.fx - (double)acc.kx) + acc.gx;
      F[1] = ((double)acc.fy - (double)acc.ky) + acc.gy;
      F[2] = ((double)acc.fz - (double)acc.kz) + acc.gz;
    } else {
      F[0] = (double)acc.fx + acc.gx;
      F[1] = (double)acc.fy + acc.gy;
      F[2] = (double)acc.fz + acc.gz;
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
  // block partial sums of u and W in FP64, fixed order
  double v[7];
  if (PREC == 0) {
    v[0] = acc.gu;
    for (int k = 0; k < 6; ++k) v[1 + k] = acc.gw[k];
  } else {
    v[0] = (PREC == 2 ? ((double)acc.u - (double)acc.ku) : (double)acc.u) + acc.gu;
    for (int k = 0; k < 6; ++k) v[1 + k] = (double)acc.w[k];
  }
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double t = warp_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  // integer statistics
  unsigned long long st[4] = {acc.cand, acc.pairs, acc.fp64, nbh};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) st[k] += __shfl_down(st[k], o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (st[k]) atomicAdd(&A.stats[k], st[k]);
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const double t = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    A.partial[8 * (size_t)lb + threadIdx.x] = t;
  }
}

// U = 1/2 sum u, W = 1/2 sum w (full list counts each pair twice); DO's W is
// rotated back, W_cart = Q W' Q^T.
__global__ void k_finalize(const double* __restrict__ partial, uint32_t nb, CellGeom g, double* __restrict__ U,
                           double* __restrict__ W) {
  __shared__ double red[4][8];
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
    for (int k = 0; k < 7; ++k) v[k] += partial[8 * (size_t)b + k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < 7; ++k) {
    const double t = warp_sum(v[k]);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[7];
    for (int k = 0; k < 7; ++k) s[k] = 0.5 * (((red[0][k] + red[1][k]) + red[2][k]) + red[3][k]);
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

hipError_t launch_build(const BuildLaunch& L, hipStream_t st) {
  const uint32_t n = L.n, nc = L.ncells;
  if (nc > 0) k_fill_u32<<<cdiv(nc, 256), 256, 0, st>>>(L.count, nc, 0u);
  k_fill_u32<<<1, 64, 0, st>>>(L.maxocc, 1, 0u);
  if (n > 0) k_bin_count<<<cdiv(n, 256), 256, 0, st>>>(L.x, n, *L.g, L.cell_of, L.rank, L.count, L.err);
  const uint32_t nb = cdiv(nc, SCAN_TILE);
  k_scan_totals<<<nb, SCAN_THREADS, 0, st>>>(L.count, nc, L.scan_tmp);
  k_scan_top<<<1, SCAN_THREADS, 0, st>>>(L.scan_tmp, nb);
  k_scan_apply<<<nb, SCAN_THREADS, 0, st>>>(L.count, nc, L.scan_tmp, L.cstart);
  if (n > 0) {
    k_scatter<<<cdiv(n, 256), 256, 0, st>>>(L.cell_of, L.rank, n, L.cstart, L.perm);
    k_cell_sort<<<cdiv(nc, 256), 256, 0, st>>>(L.cstart, nc, L.perm, L.maxocc);
    k_gather<<<cdiv(n, 256), 256, 0, st>>>(L.x, L.perm, n, *L.g, L.pos64, L.pos32, L.pos32lo, L.wrap);
  }
  return hipGetLastError();
}

template <int VAR, int PREC, bool DEBUG>
static void sweep_t(const SweepLaunch& L, hipStream_t st, uint32_t nb) {
  k_sweep<VAR, PREC, DEBUG><<<nb, 256, 0, st>>>(*L.args, *L.g);
}

hipError_t launch_sweep(const SweepLaunch& L, hipStream_t st) {
  const uint32_t n = L.args->n;
  const uint32_t nb = n > 0 ? cdiv(n, 256) : 0;
  k_fill_u32<<<1, 64, 0, st>>>((uint32_t*)L.args->stats, 8, 0u);
  if (nb > 0) {
    const int var = L.g->variant, prec = L.precision;
    const bool dbg = L.debug;
#define NCL_SW(V, P)                                      \
  if (var == V && prec == P) {                            \
    if (dbg) sweep_t<V, P, true>(L, st, nb);              \
    else sweep_t<V, P, false>(L, st, nb);                 \
  }
    NCL_SW(VAR_DS, 0) NCL_SW(VAR_DS, 1) NCL_SW(VAR_DS, 2)
    NCL_SW(VAR_DO, 0) NCL_SW(VAR_DO, 1) NCL_SW(VAR_DO, 2)
#undef NCL_SW
    k_finalize<<<1, 256, 0, st>>>(L.args->partial, nb, *L.g, L.U, L.W);
  } else {
    k_zero_f64<<<1, 64, 0, st>>>(L.U, 1);
    k_zero_f64<<<1, 64, 0, st>>>(L.W, 9);
  }
  return hipGetLastError();
}

}  // namespace ncl
