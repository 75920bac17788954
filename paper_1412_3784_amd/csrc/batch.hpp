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
  const uint32_t* n_off;     // [nrep+1] particles, input order
  const uint32_t* slot_off;  // [nrep+1] slots (multiples of the workgroup)
  const uint32_t* cell_off;  // [nrep+1] cell capacity offsets
  const uint32_t* blk_rep;   // [nslots / 256] replica of each sweep workgroup
  const RemapPolicy* pol;    // [nrep]
  const double* t0;          // [nrep] strain time at step 0
  const double* adiag;       // [nrep*3] diagonal of each flow matrix
  CellGeom* geom;            // [nrep] current cell geometry
  double* lred;              // [nrep*9] current reduced basis
  uint32_t* step;            // device step counter
  int* err;
  uint32_t *cell_of, *rank, *rep, *cstart, *scan_tmp, *perm;
  uint32_t *rs_va, *rs_vb, *rs_hist, *rs_off;  // radix sort of the cell keys
  double4* pos64;
  float4* pos32;
  float4* pos32lo;
  int4* wrap;                // debug only
  double* kpart;             // [nslots/256*3] kinetic partial sums
};

hipError_t batch_prologue(const BatchDev& D, int off, double h, hipStream_t st);
hipError_t batch_build(const BatchDev& D, const double* x, hipStream_t st);
hipError_t batch_sweep(const SweepArgs& A, const BatchDev& D, int precision, bool debug, double* U, double* W,
                       hipStream_t st);
hipError_t batch_kick(const BatchDev& D, double* p, const void* F, bool f64, double h, double mass, int second,
                      hipStream_t st);
hipError_t batch_drift(const BatchDev& D, double* x, const double* p, double h, double mass, hipStream_t st);
hipError_t batch_observe(const BatchDev& D, const double* U, const double* W, double h, double* hist,
                         uint32_t hist_cap, bool advance, hipStream_t st);

}  // namespace ncl
