// Launch descriptors shared between the C-ABI layer and the kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geometry.hpp"

namespace ncl {

// per-workgroup partial sums of a sweep: [0..6] u, wxx, wyy, wzz, wxy, wxz,
// wyz; [8..11] statistics (candidates, pairs, FP64 pairs, cells visited),
// exact as doubles
constexpr int PART_STRIDE = 12;

struct Pot32 {
  float sig2, eps4, eps24, eps48, shift;
};
struct Pot64 {
  double sig2, eps4, eps24, eps48, shift;
};

struct SweepArgs {
  const double4* pos64;
  const float4* pos32;
  const float4* pos32lo;
  const uint32_t* cstart;
  const uint32_t* perm;
  const int4* wrap;
  void* F;
  double* partial;
  double* partial2;        // second-level sums of partial, one per 256 slots
  unsigned long long* stats;
  int64_t* dbg_count;
  uint64_t* dbg_hash;
  uint32_t* overflow;      // [0] = count, then brick ids handed to the fallback
  uint32_t n;
  uint32_t cell0;          // batched form: first cell of the replica in cstart
  int32_t pad;             // batched form: slot offset added to cstart values
  uint32_t jbase;          // batched form: first input index of the replica (pair keys are replica-local)
  float rc2_lo, rc2_hi, rclose2;  // FP32 band and close radius (reported options)
  double rc2;
  // LDS-tiled path: brick of sx x sy x sz home cells, nbx x nby x nbz bricks
  int32_t sx, sy, sz, nbx, nby, nbz;
  float rc2c;        // FP32 screening threshold: rc^2 plus the FP32 frame error bound
  double band64;     // |r^2 - rc^2| below this is re-decided from FP64 positions
  double res_unit;   // value of one unit of the int16 residual
  double rclose2_64; // FP32 modes: pairs closer than this are evaluated in FP64
  double fix_q, fix_inv;  // half list: fixed-point unit of the LDS force sums and its inverse
  double rwin2_64;        // half list: pairs closer than this bypass the fixed-point sums
  Pot32 p32;
  Pot64 p64;
};


struct BuildLaunch {
  const CellGeom* g;
  const double* x;
  uint32_t n, ncells;
  // cell_of, rank: radix-sort keys (ping-pong); rs_val: values; rs_hist,
  // rs_off: rs_offsets(n) words each
  uint32_t *cell_of, *rank, *rs_val, *rs_hist, *rs_off, *cstart, *perm;
  double4* pos64;
  float4* pos32;
  float4* pos32lo;  // may be null when no tiled sweep reads this build
  int4* wrap;  // may be null
  int* err;
};

enum { SWEEP_TILED = 0, SWEEP_PARTICLE = 1, SWEEP_AUTO = 2, SWEEP_HALF = 3 };

// Workgroup size of the single-box per-particle sweep, by cell-list variant.
// Dynamic offset: one wave, so that a wave's LDS is freed when it ends
// rather than when the slowest of its workgroup's waves ends (measured at
// 1 M LJ: 0.683 -> 0.639 ms; 16 M: 7.96 -> 7.73 ms); dynamic size keeps
// four (1 M equal, 16 M 9.76 against 9.88 ms).  The sweep writes one
// partial slot per workgroup, so a launch holds ceil(n / size) slots, at
// most ceil(n / SWP_MIN_THREADS).
constexpr int swp_threads(int variant) { return variant == VAR_DO ? 64 : 256; }
constexpr int SWP_MIN_THREADS = 64;

struct SweepLaunch {
  int mode;  // SWEEP_TILED, SWEEP_PARTICLE or SWEEP_HALF
  const CellGeom* g;
  SweepArgs* args;
  int precision;
  bool debug;
  double *U, *W;
  double* facc;  // SWEEP_HALF: FP64 forces in slot order (3 n)
};

hipError_t launch_build(const BuildLaunch& L, hipStream_t st);
uint32_t rs_tiles(uint32_t n);
// Stable sort of n cell keys (all < nkeys) with their indices 0..n-1 (radix,
// passes of at most 10 bits): the indices end in vals, *sorted_keys points at
// the sorted keys (keys or keys_alt); hist and off hold rs_offsets(n) words.
hipError_t radix_sort_cells(uint32_t* keys, uint32_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, uint32_t n,
                            uint32_t nkeys, uint32_t* hist, uint32_t* off, const uint32_t** sorted_keys,
                            hipStream_t st);
// cstart[c] = first sorted position with key >= c, c = 0..nc; cstart holds
// cstart_words(nc) words (the cell starts, then a queue of long runs of empty
// cells).  The queue's count cstart[nc + 1] must be zero before the call (the
// cell-index kernels clear it) and the queued runs are written by
// cs_fill_runs in a later kernel (k_gather, or fill_empty_runs).
size_t cstart_words(uint32_t nc);
hipError_t cell_starts(const uint32_t* sorted_keys, uint32_t n, uint32_t nc, uint32_t* cstart, hipStream_t st);
hipError_t fill_empty_runs(uint32_t* cstart, uint32_t nc, hipStream_t st);
// largest of cstart[c + 1] - cstart[c] over c < nc into *out (statistics)
hipError_t launch_max_occupancy(const uint32_t* cstart, uint32_t nc, uint32_t* out, hipStream_t st);
size_t rs_offsets(uint32_t n);
hipError_t launch_sweep(const SweepLaunch& L, hipStream_t st);
hipError_t launch_half(const SweepLaunch& L, hipStream_t st, uint32_t nblocks);

}  // namespace ncl
