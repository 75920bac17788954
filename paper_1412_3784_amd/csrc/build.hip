// HIP kernels for gfx950: the cell build of every step (Sec. 4.1 / 4.2 of
// Dobson, Fox & Saracino, arXiv:1412.3784: particles are assigned to cells
// at every step): cell index and wrap of each particle, the permutation into
// cell order (particles of a cell by ascending input index), the cell starts
// and the gather of the sorted position arrays.  The array layout is
// described at the top of kernels.hip.
//
// The permutation is a stable least-significant-digit radix sort of the
// (cell, input index) pairs, in as few passes of at most 10 bits as the
// largest cell index needs: per tile of 2048 keys an LDS histogram of the
// digit, a two-level scan of each digit's counts over the tiles, then a
// scatter in which each key's rank among equal digits of its tile comes from
// wave ballots.  The (tile, digit) counters are stored one contiguous row per
// tile (a layout by digit made every tile touch 2^10 scattered words, which
// cost more than its keys).  Stability makes the order within a cell the
// input order, with no atomics on global memory (scattered global atomics
// run at about 25 G/s on MI355X, which bounded a count-and-scatter build).
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
                             int* __restrict__ err, uint32_t* __restrict__ cs_runs) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *cs_runs = 0u;  // no runs of empty cells queued yet (k_rs_cstart)
  if (i >= n) return;
  const double p[3] = {x[3 * (size_t)i], x[3 * (size_t)i + 1], x[3 * (size_t)i + 2]};
  double xw[3];
  int32_t img[3];
  bool bad = false;
  const uint32_t c = locate(g, p, xw, img, &bad);
  if (bad) atomicOr(err, 1);
  cell_of[i] = c;
}

// radix sort of the cell keys: RS_THREADS x RS_ITEMS keys per tile, each
// wave ranking a contiguous quarter of its tile; digits of up to RS_MAXLOG
// bits (the passes split the key's bits evenly), kernels instantiated for
// 2^8, 2^9 and 2^10 digit values.  Every (tile, digit) array is stored tile
// by tile, so that a tile reads and writes its counters as one contiguous
// row; the column scan over tiles runs in segments of RS_SEG tiles.
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 8;
constexpr uint32_t RS_TILE = RS_THREADS * RS_ITEMS;
constexpr uint32_t RS_WTILE = 64 * RS_ITEMS;  // keys of one wave
constexpr int RS_MAXLOG = 10;
constexpr uint32_t RS_SEG = 64;
constexpr uint32_t RS_BIG_N = 1u << 22;
constexpr int RS_TOP_THREADS = 1024;

// the lanes of the wave holding a valid key with this lane's digit
template <int LOGND>
__device__ inline uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < LOGND; ++bit) {
    const uint64_t bb = __ballot((d >> bit) & 1u);
    peers &= ((d >> bit) & 1u) ? bb : ~bb;
  }
  return peers;
}

// digit histogram of each tile -> hist[tile * ND + digit].  Keys in cell
// order come in runs of one digit, and LDS atomics on one address
// serialise, so the first lane of each run of equal digits (consecutive
// lanes of a round of 64 keys) adds the run's length.
template <int LOGND>
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint32_t* __restrict__ key, uint32_t n, int shift,
                                                       uint32_t mask, uint32_t* __restrict__ hist) {
  constexpr int ND = 1 << LOGND;
  __shared__ uint32_t h[ND];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t w0 = blockIdx.x * RS_TILE + wid * RS_WTILE;
  uint32_t kk[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e = w0 + r * 64 + lane;
    kk[r] = e < n ? key[e] : 0u;
  }
  for (int d = tid; d < ND; d += RS_THREADS) h[d] = 0u;
  __syncthreads();
  const uint64_t above = lane == 63 ? 0ull : ~0ull << (lane + 1);
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e0 = w0 + r * 64;
    const uint32_t nv = e0 >= n ? 0u : min(64u, n - e0);  // valid lanes 0 .. nv - 1
    const uint32_t d = (kk[r] >> shift) & mask;
    const uint32_t dp = (uint32_t)__shfl_up((int)d, 1, 64);
    const bool head = (uint32_t)lane < nv && (lane == 0 || dp != d);
    const uint64_t heads = __ballot(head);
    const uint64_t next = heads & above;
    const uint32_t end = next ? (uint32_t)__ffsll((long long)next) - 1u : nv;
    if (head) atomicAdd(&h[d], end - (uint32_t)lane);
  }
  __syncthreads();
  for (int d = tid; d < ND; d += RS_THREADS) hist[(size_t)blockIdx.x * ND + d] = h[d];
}

// column scan, first level: block (segment, group of 64 digits); each wave
// takes a quarter of the segment's tiles.  pre[tile * ND + d] = keys of
// digit d in the earlier tiles of the segment; seg[segment * ND + d] = the
// segment's count.
template <int LOGND>
__global__ void __launch_bounds__(RS_THREADS) k_rs_segscan(const uint32_t* __restrict__ hist, uint32_t nt,
                                                          uint32_t* __restrict__ pre, uint32_t* __restrict__ seg) {
  constexpr int ND = 1 << LOGND;
  constexpr uint32_t PER = RS_SEG / RS_WAVES;
  __shared__ uint32_t ws[RS_WAVES][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t d = blockIdx.y * 64 + lane;
  const uint32_t t0 = blockIdx.x * RS_SEG + wid * PER;
  uint32_t v[PER], s = 0;
#pragma unroll
  for (uint32_t i = 0; i < PER; ++i) v[i] = t0 + i < nt ? hist[(size_t)(t0 + i) * ND + d] : 0u;
#pragma unroll
  for (uint32_t i = 0; i < PER; ++i) s += v[i];
  ws[wid][lane] = s;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < RS_WAVES; ++w) {
    if (w < wid) off += ws[w][lane];
    tot += ws[w][lane];
  }
#pragma unroll
  for (uint32_t i = 0; i < PER; ++i) {
    if (t0 + i < nt) pre[(size_t)(t0 + i) * ND + d] = off;
    off += v[i];
  }
  if (wid == 0) seg[(size_t)blockIdx.x * ND + d] = tot;
}

// column scan, second level: block per 64 digits, its waves splitting the
// segments.  seg[segment * ND + d] becomes the keys of digit d in the earlier
// segments (in place); dtot[d] = the digit's total.
template <int LOGND>
__global__ void __launch_bounds__(RS_TOP_THREADS) k_rs_segtop(uint32_t* __restrict__ seg, uint32_t nseg,
                                                             uint32_t* __restrict__ dtot) {
  constexpr int ND = 1 << LOGND, NW = RS_TOP_THREADS / 64;
  __shared__ uint32_t ws[NW][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t d = blockIdx.x * 64 + lane;
  const uint32_t per = (nseg + NW - 1) / NW;
  const uint32_t s0 = min(nseg, wid * per), s1 = min(nseg, s0 + per);
  uint32_t s = 0;
#pragma unroll 8
  for (uint32_t q = s0; q < s1; ++q) s += seg[(size_t)q * ND + d];
  ws[wid][lane] = s;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < NW; ++w) {
    if (w < wid) off += ws[w][lane];
    tot += ws[w][lane];
  }
#pragma unroll 8
  for (uint32_t q = s0; q < s1; ++q) {
    const uint32_t v = seg[(size_t)q * ND + d];
    seg[(size_t)q * ND + d] = off;
    off += v;
  }
  if (wid == 0) dtot[d] = tot;
}

// stable scatter of one digit pass: key e of tile t goes to (keys of smaller
// digits) + (keys of its digit in earlier segments) + (in earlier tiles of
// its segment) + (earlier keys of the tile with the same digit).  Each wave
// ranks its contiguous 512 keys round by round (ties within a round by wave
// ballots) against a running count per digit in its own LDS row; the rows
// are then turned into per-wave offsets.  Keys are staged in LDS in digit
// order and written out so that consecutive lanes store consecutive
// addresses of a digit's run.  vin == nullptr means the values are the
// indices e.
template <int LOGND>
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, uint32_t n, int shift,
                                                          uint32_t mask, const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ pre,
                                                          const uint32_t* __restrict__ seg,
                                                          const uint32_t* __restrict__ dtot,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  constexpr int ND = 1 << LOGND, DPT = ND / RS_THREADS;
  __shared__ uint32_t off0[ND], tstart[ND];
  __shared__ uint32_t wc[RS_WAVES][ND];
  __shared__ uint32_t sk[RS_TILE], sv[RS_TILE];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // each XCD takes a contiguous range of tiles, so that the partial lines
  // of a digit's run written by consecutive tiles merge in one L2
  const uint32_t t = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t w0 = t * RS_TILE + wid * RS_WTILE;
  uint32_t kk[RS_ITEMS], vv[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t e = w0 + r * 64 + lane;
    kk[r] = e < n ? kin[e] : 0u;
    vv[r] = e < n ? (vin ? vin[e] : e) : 0u;
  }
  // thread tid holds digits tid * DPT .. tid * DPT + DPT - 1: the digit's
  // base (exclusive scan of the digit totals) and its start in the tile
  // (exclusive scan of the tile's counts)
  const uint32_t* hrow = hist + (size_t)t * ND;
  const uint32_t* prow = pre + (size_t)t * ND;
  const uint32_t* srow = seg + (size_t)(t / RS_SEG) * ND;
  // every load of the tile is issued before the first use of any
  uint32_t dt[DPT], hc[DPT], sp[DPT], sd = 0, sh = 0;
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int d = tid * DPT + q;
    dt[q] = dtot[d];
    hc[q] = hrow[d];
    sp[q] = srow[d] + prow[d];
  }
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int d = tid * DPT + q;
    sd += dt[q];
    sh += hc[q];
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) wc[w][d] = 0u;
  }
  uint32_t all, total;
  uint32_t bd = block_excl_scan(sd, &all);
  uint32_t bh = block_excl_scan(sh, &total);
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int d = tid * DPT + q;
    off0[d] = bd + sp[q];
    tstart[d] = bh;
    bd += dt[q];
    bh += hc[q];
  }
  __syncthreads();
  // rank of each key among the wave's earlier keys of its digit
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t rk[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const bool valid = w0 + r * 64 + lane < n;
    const uint32_t d = (kk[r] >> shift) & mask;
    const uint64_t peers = digit_peers<LOGND>(d, valid);
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    rk[r] = wc[wid][d] + below;
    if (valid && below == 0) wc[wid][d] = rk[r] + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: counts of the waves -> keys of the digit in earlier waves
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int d = tid * DPT + q;
    uint32_t a = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
      const uint32_t c = wc[w][d];
      wc[w][d] = a;
      a += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    if (w0 + r * 64 + lane < n) {
      const uint32_t d = (kk[r] >> shift) & mask;
      const uint32_t q = tstart[d] + wc[wid][d] + rk[r];
      sk[q] = kk[r];
      sv[q] = vv[r];
    }
  }
  __syncthreads();
  // the tile in digit order: slot q of digit d goes to off0[d] + q - tstart[d]
  for (uint32_t q = tid; q < total; q += RS_THREADS) {
    const uint32_t k = sk[q];
    const uint32_t d = (k >> shift) & mask;
    const uint32_t pos = off0[d] + (q - tstart[d]);
    kout[pos] = k;
    vout[pos] = sv[q];
  }
}

// cell starts from the sorted keys: cstart[c] = first slot whose key is >= c
// (empty cells get the start of the next occupied one; cstart[nc] = n).  The
// first particle of each occupied cell writes its cell and the empty cells
// before it; a run of more than CS_SPAN empty cells (the unused cell range of
// a batched replica, or a sparse box) is queued instead, as (first cell,
// length, value) after cstart[nc], and filled by a later kernel
// (cs_fill_runs: one workgroup per run; one thread writing a run of
// thousands of cells held the whole build).  Such runs are disjoint and
// longer than CS_SPAN, so at most nc / CS_SPAN + 1 of them exist.
constexpr uint32_t CS_SPAN = 64;

__device__ inline void cs_fill(uint32_t* __restrict__ cstart, uint32_t* __restrict__ runs, uint32_t c0, uint32_t c1,
                               uint32_t v) {  // cells c0 .. c1 - 1
  if (c1 <= c0) return;
  if (c1 - c0 <= CS_SPAN) {
    for (uint32_t c = c0; c < c1; ++c) cstart[c] = v;
  } else {
    const uint32_t q = atomicAdd(runs, 1u);
    runs[1 + 3 * q] = c0;
    runs[2 + 3 * q] = c1 - c0;
    runs[3 + 3 * q] = v;
  }
}

__global__ void k_rs_cstart(const uint32_t* __restrict__ key, uint32_t n, uint32_t nc, uint32_t* __restrict__ cstart) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t* runs = cstart + nc + 1;
  const uint32_t k = key[s];
  const uint32_t c0 = (s == 0) ? 0u : key[s - 1] + 1u;
  if (c0 <= k) {
    cstart[k] = s;
    cs_fill(cstart, runs, c0, k, s);
  }
  if (s == n - 1) {
    cstart[nc] = n;
    cs_fill(cstart, runs, k + 1, nc, n);
  }
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

__global__ void k_gather(const double* __restrict__ x, const uint32_t* __restrict__ perm, uint32_t n, CellGeom g,
                         double4* __restrict__ pos64, float4* __restrict__ pos32, float4* __restrict__ pos32lo,
                         int4* __restrict__ wrap, uint32_t* __restrict__ cstart, uint32_t nc) {
  cs_fill_runs(cstart, nc);
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
  if (pos32lo) pos32lo[s] = make_float4((float)(o[0] - hi[0]), (float)(o[1] - hi[1]), (float)(o[2] - hi[2]), 0.f);
  if (wrap) wrap[s] = make_int4(img[0], img[1], img[2], 0);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline uint32_t bdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_max_occupancy(const uint32_t* cstart, uint32_t nc, uint32_t* out, hipStream_t st) {
  k_max_occ<<<1, 1024, 0, st>>>(cstart, nc, out);
  return hipGetLastError();
}

// tiles and segments of the radix sort and the size of its (tile, digit)
// arrays: the histogram; then the per-tile prefixes, the per-segment
// prefixes and the digit totals
uint32_t rs_tiles(uint32_t n) { return bdiv(n, RS_TILE); }
static uint32_t rs_segs(uint32_t nt) { return bdiv(nt, RS_SEG); }
size_t rs_offsets(uint32_t n) {
  const uint32_t nt = rs_tiles(n);
  return ((size_t)nt + rs_segs(nt) + 1) << RS_MAXLOG;
}

template <int LOGND>
static void rs_pass(const uint32_t* kin, const uint32_t* vin, uint32_t n, int shift, uint32_t mask, uint32_t* hist,
                    uint32_t* off, uint32_t nt, uint32_t* kout, uint32_t* vout, hipStream_t st) {
  constexpr uint32_t ND = 1u << LOGND;
  const uint32_t ns = rs_segs(nt);
  uint32_t* pre = off;
  uint32_t* seg = pre + (size_t)nt * ND;
  uint32_t* dtot = seg + (size_t)ns * ND;
  k_rs_hist<LOGND><<<nt, RS_THREADS, 0, st>>>(kin, n, shift, mask, hist);
  k_rs_segscan<LOGND><<<dim3(ns, ND / 64), RS_THREADS, 0, st>>>(hist, nt, pre, seg);
  k_rs_segtop<LOGND><<<ND / 64, RS_TOP_THREADS, 0, st>>>(seg, ns, dtot);
  k_rs_scatter<LOGND><<<nt, RS_THREADS, 0, st>>>(kin, vin, n, shift, mask, hist, pre, seg, dtot, kout, vout);
}

hipError_t radix_sort_cells(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, uint32_t n,
                            uint32_t nkeys, uint32_t* hist, uint32_t* off, const uint32_t** sorted_keys,
                            hipStream_t st) {
  // the bits of the largest key, split evenly over the fewest passes of at
  // most RS_MAXLOG bits (17 bits: two passes of 9); from RS_BIG_N keys on,
  // at most 8 bits (a 2,048-key tile then writes runs of about 8 keys per
  // digit instead of 2, and three passes of 7 bits sort 16 M keys of 20
  // bits faster than two of 10: 0.25 against 0.29 ms)
  int bits = 1;
  while (bits < 32 && ((nkeys - 1u) >> bits) != 0u) ++bits;
  const int maxlog = n >= RS_BIG_N ? 8 : RS_MAXLOG;
  const int passes = (bits + maxlog - 1) / maxlog;
  const int db = (bits + passes - 1) / passes;
  const uint32_t mask = (1u << db) - 1u;
  const int logn = db < 8 ? 8 : db;
  const uint32_t nt = rs_tiles(n);
  // keys ping-pong between keys and keys_alt; values end in vals
  uint32_t* kb[2] = {keys, keys_alt};
  uint32_t* vb[2] = {(passes & 1) ? vals : vals_alt, (passes & 1) ? vals_alt : vals};
  for (int p = 0; p < passes && n > 0; ++p) {
    const uint32_t* vin = p ? vb[(p - 1) & 1] : nullptr;
    if (logn == 8)
      rs_pass<8>(kb[p & 1], vin, n, db * p, mask, hist, off, nt, kb[(p + 1) & 1], vb[p & 1], st);
    else if (logn == 9)
      rs_pass<9>(kb[p & 1], vin, n, db * p, mask, hist, off, nt, kb[(p + 1) & 1], vb[p & 1], st);
    else
      rs_pass<10>(kb[p & 1], vin, n, db * p, mask, hist, off, nt, kb[(p + 1) & 1], vb[p & 1], st);
  }
  *sorted_keys = kb[passes & 1];
  return hipGetLastError();
}

__global__ void k_cs_runs(uint32_t* __restrict__ cstart, uint32_t nc) { cs_fill_runs(cstart, nc); }

hipError_t fill_empty_runs(uint32_t* cstart, uint32_t nc, hipStream_t st) {
  k_cs_runs<<<512, 256, 0, st>>>(cstart, nc);
  return hipGetLastError();
}

size_t cstart_words(uint32_t nc) { return (size_t)nc + 1 + 1 + 3 * ((size_t)nc / CS_SPAN + 2); }

hipError_t cell_starts(const uint32_t* sorted_keys, uint32_t n, uint32_t nc, uint32_t* cstart, hipStream_t st) {
  if (n == 0) k_bfill_u32<<<bdiv(nc + 1, 256), 256, 0, st>>>(cstart, nc + 1, 0u);
  else k_rs_cstart<<<bdiv(n, 256), 256, 0, st>>>(sorted_keys, n, nc, cstart);
  return hipGetLastError();
}

hipError_t launch_build(const BuildLaunch& L, hipStream_t st) {
  const uint32_t n = L.n, nc = L.ncells;
  if (n > 0) k_cell_index<<<bdiv(n, 256), 256, 0, st>>>(L.x, n, *L.g, L.cell_of, L.err, L.cstart + nc + 1);
  const uint32_t* keys = L.cell_of;
  hipError_t e = radix_sort_cells(L.cell_of, L.rank, L.perm, L.rs_val, n, nc, L.rs_hist, L.rs_off, &keys, st);
  if (e == hipSuccess) e = cell_starts(keys, n, nc, L.cstart, st);
  if (e != hipSuccess) return e;
  if (n > 0)
    k_gather<<<bdiv(n, 256), 256, 0, st>>>(L.x, L.perm, n, *L.g, L.pos64, L.pos32, L.pos32lo, L.wrap, L.cstart, nc);
  return hipGetLastError();
}

}  // namespace ncl
