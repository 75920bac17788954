// HIP kernels for gfx950: the cell build of every step (Sec. 4.1 / 4.2 of
// Dobson, Fox & Saracino, arXiv:1412.3784: particles are assigned to cells
// at every step): cell index and wrap of each particle, the permutation into
// cell order (particles of a cell by ascending input index), the cell starts
// and the gather of the sorted position arrays.  The array layout is
// described at the top of kernels.hip.
//
// The permutation is a stable least-significant-digit radix sort of the
// (cell, input index) pairs, 8 bits per pass: per tile of 2048 keys an LDS
// histogram of the digit, one exclusive scan over (digit, tile), then a
// scatter in which each key's rank among equal digits of its tile comes from
// wave ballots.  Stability makes the order within a cell the input order, with
// no atomics on global memory (scattered global atomics run at about 25 G/s
// on MI355X, which bounded a count-and-scatter build).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geometry.hpp"
#include "batch.hpp"
#include "kernels.hpp"
#include "sweep_common.hpp"

namespace ncl {

__global__ void k_bfill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__global__ void k_cell_index(const double* __restrict__ x, uint32_t n, CellGeom g, uint32_t* __restrict__ cell_of,
                             int* __restrict__ err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double p[3] = {x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2]};
  double xw[3];
  int32_t img[3];
  bool bad = false;
  const uint32_t c = locate(g, p, xw, img, &bad);
  if (bad) atomicOr(err, 1);
  cell_of[i] = c;
}

// radix sort of the cell keys: RS_THREADS x RS_ITEMS keys per tile
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr uint32_t RS_TILE = RS_THREADS * RS_ITEMS;

// digit histogram of each tile -> hist[digit * ntiles + tile]
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint32_t* __restrict__ key, uint32_t n, int shift,
                                                       uint32_t* __restrict__ hist, uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t t0 = blockIdx.x * RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e = t0 + r * RS_THREADS + threadIdx.x;
    if (e < n) atomicAdd(&h[(key[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// stable scatter of one digit pass: key e of the tile goes to
// off[digit * ntiles + tile] + (number of earlier keys of the tile with the
// same digit).  Keys are ranked in the order of e (rounds of 256, waves,
// lanes; ties by wave ballots), staged in LDS in digit order, then written
// out so that consecutive lanes store consecutive addresses of a digit's run.
// vin == nullptr means the values are the indices e.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, uint32_t n, int shift,
                                                          const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ off, uint32_t ntiles,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  __shared__ uint32_t off0[256], run[256], tstart[256];
  __shared__ uint32_t wcnt[RS_THREADS / 64][256];
  __shared__ uint32_t sk[RS_TILE], sv[RS_TILE];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t t0 = blockIdx.x * RS_TILE;
  off0[tid] = off[(size_t)tid * ntiles + blockIdx.x];
  uint32_t total;
  tstart[tid] = block_excl_scan(hist[(size_t)tid * ntiles + blockIdx.x], &total);  // digit order
  run[tid] = 0u;
  for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0u;
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e = t0 + r * RS_THREADS + tid;
    const bool valid = e < n;
    const uint32_t k = valid ? kin[e] : 0u;
    const uint32_t v = valid ? (vin ? vin[e] : e) : 0u;
    const uint32_t d = (k >> shift) & 255u;
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t rk = (uint32_t)__popcll(peers & lt);
    if (valid && rk == 0) wcnt[wid][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t q = tstart[d] + run[d] + rk;
      for (int w = 0; w < wid; ++w) q += wcnt[w][d];
      sk[q] = k;
      sv[q] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < RS_THREADS / 64; ++w) {
      add += wcnt[w][tid];
      wcnt[w][tid] = 0u;
    }
    run[tid] += add;
    __syncthreads();
  }
  // the tile in digit order: slot q of digit d goes to off0[d] + q - tstart[d]
  const uint32_t cnt = total;
  for (uint32_t q = tid; q < cnt; q += RS_THREADS) {
    const uint32_t k = sk[q];
    const uint32_t d = (k >> shift) & 255u;
    const uint32_t pos = off0[d] + (q - tstart[d]);
    kout[pos] = k;
    vout[pos] = sv[q];
  }
}

// cell starts from the sorted keys: cstart[c] = first slot whose key is >= c
// (empty cells get the start of the next occupied one; cstart[nc] = n)
__global__ void k_rs_cstart(const uint32_t* __restrict__ key, uint32_t n, uint32_t nc, uint32_t* __restrict__ cstart) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t k = key[s];
  const uint32_t c0 = (s == 0) ? 0u : key[s - 1] + 1u;
  for (uint32_t c = c0; c <= k; ++c) cstart[c] = s;
  if (s == n - 1)
    for (uint32_t c = k + 1; c <= nc; ++c) cstart[c] = n;
}

// largest cell occupancy, for the statistics only (one block: a counter
// updated by every wave of a launch serialises in one L2 channel)
__global__ void __launch_bounds__(1024) k_max_occ(const uint32_t* __restrict__ cstart, uint32_t nc,
                                                  uint32_t* __restrict__ maxocc) {
  __shared__ uint32_t red[16];
  uint32_t m = 0;
  for (uint32_t c = threadIdx.x; c < nc; c += blockDim.x) m = max(m, cstart[c + 1] - cstart[c]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) m = max(m, red[w]);
    *maxocc = m;
  }
}

// exclusive scan of u32 counts, three passes: per-block totals, a scan of
// the totals in one block, then the per-block scan with its offset.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

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
// host launchers
// ---------------------------------------------------------------------------
static inline uint32_t bdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// exclusive scan of n counts into out[0..n] (out[n] = total); tmp holds
// ceil(n / SCAN_TILE) block totals
static hipError_t scan_counts(const uint32_t* count, uint32_t n, uint32_t* tmp, uint32_t* out, hipStream_t st) {
  const uint32_t nb = bdiv(n, SCAN_TILE);
  if (nb == 0) return hipSuccess;
  k_scan_totals<<<nb, SCAN_THREADS, 0, st>>>(count, n, tmp);
  k_scan_top<<<1, SCAN_THREADS, 0, st>>>(tmp, nb);
  k_scan_apply<<<nb, SCAN_THREADS, 0, st>>>(count, n, tmp, out);
  return hipGetLastError();
}

hipError_t launch_max_occupancy(const uint32_t* cstart, uint32_t nc, uint32_t* out, hipStream_t st) {
  k_max_occ<<<1, 1024, 0, st>>>(cstart, nc, out);
  return hipGetLastError();
}

// tiles of the radix sort and the size of its (digit, tile) offset array
uint32_t rs_tiles(uint32_t n) { return bdiv(n, RS_TILE); }
size_t rs_offsets(uint32_t n) { return (size_t)256 * rs_tiles(n) + 1; }

hipError_t radix_sort_cells(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, uint32_t n,
                            uint32_t nkeys, uint32_t* hist, uint32_t* off, uint32_t* scan_tmp,
                            const uint32_t** sorted_keys, hipStream_t st) {
  // 8-bit digits over the bits of the largest key
  int bits = 1;
  while (bits < 32 && ((nkeys - 1u) >> bits) != 0u) ++bits;
  const int passes = (bits + 7) / 8;
  const uint32_t nt = rs_tiles(n), nh = 256u * nt;
  // keys ping-pong between keys and keys_alt; values end in vals
  uint32_t* kb[2] = {keys, keys_alt};
  uint32_t* vb[2] = {(passes & 1) ? vals : vals_alt, (passes & 1) ? vals_alt : vals};
  for (int p = 0; p < passes && n > 0; ++p) {
    k_rs_hist<<<nt, RS_THREADS, 0, st>>>(kb[p & 1], n, 8 * p, hist, nt);
    const hipError_t e = scan_counts(hist, nh, scan_tmp, off, st);
    if (e != hipSuccess) return e;
    k_rs_scatter<<<nt, RS_THREADS, 0, st>>>(kb[p & 1], p ? vb[(p - 1) & 1] : nullptr, n, 8 * p, hist, off, nt,
                                            kb[(p + 1) & 1], vb[p & 1]);
  }
  *sorted_keys = kb[passes & 1];
  return hipGetLastError();
}

hipError_t cell_starts(const uint32_t* sorted_keys, uint32_t n, uint32_t nc, uint32_t* cstart, hipStream_t st) {
  if (n == 0) k_bfill_u32<<<bdiv(nc + 1, 256), 256, 0, st>>>(cstart, nc + 1, 0u);
  else k_rs_cstart<<<bdiv(n, 256), 256, 0, st>>>(sorted_keys, n, nc, cstart);
  return hipGetLastError();
}

hipError_t launch_build(const BuildLaunch& L, hipStream_t st) {
  const uint32_t n = L.n, nc = L.ncells;
  if (n > 0) k_cell_index<<<bdiv(n, 256), 256, 0, st>>>(L.x, n, *L.g, L.cell_of, L.err);
  const uint32_t* keys = L.cell_of;
  hipError_t e = radix_sort_cells(L.cell_of, L.rank, L.perm, L.rs_val, n, nc, L.rs_hist, L.rs_off, L.scan_tmp, &keys, st);
  if (e == hipSuccess) e = cell_starts(keys, n, nc, L.cstart, st);
  if (e != hipSuccess) return e;
  if (n > 0) k_gather<<<bdiv(n, 256), 256, 0, st>>>(L.x, L.perm, n, *L.g, L.pos64, L.pos32, L.pos32lo, L.wrap);
  return hipGetLastError();
}

}  // namespace ncl
