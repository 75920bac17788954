// Device view of a batch of replicas, passed by value to the batched kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geometry.hpp"
#include "kernels.hpp"

namespace ncl {

struct BatchDev {
  uint32_t nrep, n, nslots, ncells;
  int32_t variant, do_tight;
  double rc;
  double rc_cells;           // cut-off the cells are built for: rc, or rc + skin with neighbour lists
  const uint32_t* n_off;     // [nrep+1] particles, input order
  const uint32_t* slot_off;  // [nrep+1] slots (multiples of 256)
  const uint32_t* cell_off;  // [nrep+1] cell capacity offsets
  const uint32_t* blk_rep;   // [nslots / 256] replica of each 256-slot block
  const uint32_t* in_rep;    // [ceil(n / 256)] replica of particle 256 b (input and sorted order alike)
  const RemapPolicy* pol;    // [nrep]
  const double* t0;          // [nrep] strain time at step 0
  const double* adiag;       // [nrep*3] diagonal of each flow matrix
  CellGeom* geom;            // [nrep] current cell geometry
  double* lred;              // [nrep*9] current reduced basis
  uint32_t* step;            // device step counter
  int* err;
  uint32_t *cell_of, *rank, *cstart, *perm;
  uint32_t *rs_va, *rs_vb, *rs_hist, *rs_off;  // radix sort of the cell keys
  double4* pos64;
  float4* pos32;
  int4* wrap;                // debug only
  double* kpart;             // [nslots/256*3] kinetic partial sums
  int64_t* pcur;             // [nrep*2] remap coefficients at the current time
  // neighbour lists with a skin (entry k of slot s at k * nslots + s)
  uint32_t kmax;
  uint2* vl;                 // [nslots * kmax] (neighbour slot, packed image)
  uint32_t* vl_cnt;
  double4* ysl;              // [nslots] slot-ordered Cartesian positions (see batch.hip)
  double* xb;                // positions at the last rebuild (input order)
  double* tb;                // [nrep] time of the last rebuild
  int64_t* pb;               // [nrep*2] remap coefficients at the last rebuild
  unsigned long long* dmax;  // [nrep] largest peculiar displacement since (double bits)
  uint32_t* need;            // rebuild flags: 1 skin, 2 remap, 4 list capacity
};

hipError_t batch_prologue(const BatchDev& D, int off, double h, hipStream_t st);
hipError_t batch_build(const BatchDev& D, const double* x, hipStream_t st);
hipError_t batch_sweep(const SweepArgs& A, const BatchDev& D, int precision, bool debug, double* U, double* W,
                       hipStream_t st);
// fused bin + force in one persistent launch (see batch.hip); the lattice
// prologue must precede it
hipError_t batch_fused(const SweepArgs& A, const BatchDev& D, const double* x, int precision, uint32_t* fstate,
                       const uint32_t* order, const uint32_t* blk_order, double* U, double* W, hipStream_t st);
// dst[i] = src[i], i < n (a kernel, so that graph captures record no copy node)
hipError_t batch_copy(double* dst, const double* src, uint64_t n, hipStream_t st);
hipError_t batch_kick(const BatchDev& D, double* p, const void* F, bool f64, double h, double mass, int second,
                      hipStream_t st);
// list steps: unwrapped drift of x and of the slot-ordered copy
hipError_t batch_drift(const BatchDev& D, double* x, const double* p, double h, double mass, hipStream_t st);
// optional second kick of the previous step (with its kinetic sums), first
// kick and wrapped drift of this step in one pass (see batch.hip)
hipError_t batch_kick_drift(const BatchDev& D, double* x, double* p, const void* F, bool f64, double h, double mass,
                            bool kick2, hipStream_t st);
hipError_t batch_wrap(const BatchDev& D, double* x, hipStream_t st);
hipError_t batch_list_rebuild(const BatchDev& D, double* x, int off, double h, hipStream_t st);
hipError_t batch_list_check(const BatchDev& D, const double* x, int off, double h, double skin, hipStream_t st);
hipError_t batch_list_force(const SweepArgs& A, const BatchDev& D, int precision, double* U, double* W,
                            hipStream_t st);
hipError_t batch_observe(const BatchDev& D, const double* U, const double* W, double h, double* hist,
                         uint32_t hist_cap, bool advance, hipStream_t st);

}  // namespace ncl
