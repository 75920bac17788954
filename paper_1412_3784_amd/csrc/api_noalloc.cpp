// ncl_forces_noalloc: lattice at time t, cell build and force pass of one
// box in a single call that allocates nothing (declared in
// include/nemdcl.h).  It runs the same kernels as ncl_set_lattice +
// ncl_build_cells + ncl_compute_forces with the per-particle sweep; every
// scratch array (sort keys, cell starts, sorted positions, block partials,
// statistics) lives in one file-scope device array of fixed size, so boxes
// are limited to NCL_NOALLOC_MAX_N particles and NCL_NOALLOC_MAX_CELLS
// cells.  Each device holds its own copy of the array; calls on one device
// share it, keep the last call's contents, and race if they overlap.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "../../include/nemdcl.h"
#include "geometry.hpp"
#include "kernels.hpp"

using namespace ncl;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_ptr[MAX_DEVICES];  // device address of `scratch`, per device

// word 0..3 statistics (u64), 4 occupancy, 5 error flag (see launch_sweep and
// the cell-index kernel); cleared by a kernel so that the call can be captured
__global__ void kn_clear(unsigned long long* w, int n) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = 0ull;
}

// a non-finite position, flagged by the cell-index kernel, makes U NaN
__global__ void kn_flag(const unsigned long long* w, double* U) {
  if (threadIdx.x == 0 && (w[5] & 0xffffffffull) != 0ull) U[0] = __longlong_as_double(0x7ff8000000000000ll);
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// byte offsets of the scratch arrays for n particles and nc cells
struct Layout {
  size_t small, cell_of, rank, perm, rs_val, rs_hist, rs_off, cstart, pos64, pos32, pos32lo, partial, overflow, end;
  uint32_t nblk;
};

Layout layout(uint32_t n, uint32_t nc) {
  Layout L;
  const size_t m = n > 0 ? n : 1;
  L.nblk = (uint32_t)((m + SWP_MIN_THREADS - 1) / SWP_MIN_THREADS);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += up256(bytes);
    return at;
  };
  L.small = take(8 * sizeof(unsigned long long));
  L.cell_of = take(m * 4);
  L.rank = take(m * 4);
  L.perm = take(m * 4);
  L.rs_val = take(m * 4);
  L.rs_hist = take(rs_offsets((uint32_t)m) * 4);
  L.rs_off = take(rs_offsets((uint32_t)m) * 4);
  L.cstart = take(cstart_words(nc) * 4);
  L.pos64 = take(m * sizeof(double4));
  L.pos32 = take((m + 4) * sizeof(float4));
  L.pos32lo = take(m * sizeof(float4));
  L.partial = take((size_t)PART_STRIDE * (L.nblk + 2 + (L.nblk + 2) / 256 + 1) * sizeof(double));
  L.overflow = take((L.nblk + 2) * 4);
  L.end = o;
  return L;
}

// set-up once per device, with that device current: the array's device
// address (the host-side name `scratch` is not one)
int scratch_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= MAX_DEVICES) return NCL_E_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NCL_E_HIP;
    g_ptr[device] = (unsigned char*)p;
  }
  *out = g_ptr[device];
  return NCL_OK;
}

}  // namespace

extern "C" {

int ncl_forces_noalloc(int device, void* stream, const double L0[9], const double A[9], double t, int naut,
                       const int32_t* aut, const double pot[4], int variant, int precision, const double* x,
                       int64_t n, void* F, double* U, double* W) {
  if (!L0 || !A || !pot || !U || !W) return NCL_E_ARG;
  if (variant != NCL_DYNAMIC_SIZE && variant != NCL_DYNAMIC_OFFSET) return NCL_E_ARG;
  if (precision < NCL_PREC_FP64 || precision > NCL_PREC_FP32_KAHAN) return NCL_E_ARG;
  if (naut < 0 || naut > 2 || (naut > 0 && !aut)) return NCL_E_ARG;
  if (n < 0 || (n > 0 && (!x || !F))) return NCL_E_ARG;
  const double eps = pot[0], sigma = pot[1], rc = pot[2];
  if (!(eps > 0.0) || !(sigma > 0.0) || !(rc > 0.0) || !isfinite(eps + sigma + rc) || !isfinite(t)) return NCL_E_ARG;
  for (int k = 0; k < 9; ++k)
    if (!isfinite(L0[k]) || !isfinite(A[k])) return NCL_E_ARG;
  if (n > NCL_NOALLOC_MAX_N) return NCL_E_CAPACITY;
  // lattice at t and cell geometry, on the host
  RemapPolicy pol;
  const int prc = remap_policy_init(&pol, L0, A, naut, aut);
  if (prc != GEOM_OK) return NCL_E_LATTICE;
  double Lred[9];
  int64_t coef[2], Mtot[9];
  reduced_lattice(pol, A, t, Lred, coef, Mtot);
  CellGeom g;
  const int grc = cell_geom_init(&g, Lred, Mtot, rc, variant == NCL_DYNAMIC_OFFSET ? VAR_DO : VAR_DS, 1);
  if (grc == GEOM_E_SMALL) return NCL_E_BOX_TOO_SMALL;
  if (grc != GEOM_OK) return NCL_E_LATTICE;
  cell_geom_bands(&g, rc);
  const double ncd = (double)g.nc[0] * g.nc[1] * g.nc[2];
  if (ncd > (double)NCL_NOALLOC_MAX_CELLS) return NCL_E_CAPACITY;
  const uint32_t nc = (uint32_t)ncd;
  const Layout lay = layout((uint32_t)n, nc);
  const Layout cap = layout(NCL_NOALLOC_MAX_N, NCL_NOALLOC_MAX_CELLS);
  if (lay.end > SCRATCH_BYTES || cap.end > SCRATCH_BYTES) return NCL_E_CAPACITY;

  if (hipSetDevice(device) != hipSuccess) return NCL_E_HIP;
  unsigned char* base = nullptr;
  const int src = scratch_ptr(device, &base);
  if (src != NCL_OK) return src;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* small = (unsigned long long*)(base + lay.small);
  kn_clear<<<1, 64, 0, st>>>(small, 8);

  BuildLaunch B;
  B.g = &g;
  B.x = x;
  B.n = (uint32_t)n;
  B.ncells = nc;
  B.cell_of = (uint32_t*)(base + lay.cell_of);
  B.rank = (uint32_t*)(base + lay.rank);
  B.rs_val = (uint32_t*)(base + lay.rs_val);
  B.rs_hist = (uint32_t*)(base + lay.rs_hist);
  B.rs_off = (uint32_t*)(base + lay.rs_off);
  B.cstart = (uint32_t*)(base + lay.cstart);
  B.perm = (uint32_t*)(base + lay.perm);
  B.pos64 = (double4*)(base + lay.pos64);
  B.pos32 = (float4*)(base + lay.pos32);
  B.pos32lo = (float4*)(base + lay.pos32lo);
  B.wrap = nullptr;
  B.err = (int*)(small + 5);
  if (launch_build(B, st) != hipSuccess) return NCL_E_HIP;

  // sweep arguments as the handle path fills them (default close radius)
  const double s2 = sigma * sigma, close_r = 0.45;
  double shift = 0.0;
  if (pot[3] != 0.0) {
    const double q = s2 / (rc * rc), q6 = q * q * q;
    shift = 4.0 * eps * (q6 * q6 - q6);
  }
  SweepArgs S{};
  S.pos64 = B.pos64;
  S.pos32 = B.pos32;
  S.pos32lo = B.pos32lo;
  S.cstart = B.cstart;
  S.perm = B.perm;
  S.wrap = nullptr;
  S.F = F;
  S.partial = (double*)(base + lay.partial);
  S.partial2 = S.partial + PART_STRIDE * (size_t)(lay.nblk + 2);
  S.stats = small;
  S.dbg_count = nullptr;
  S.dbg_hash = nullptr;
  S.overflow = (uint32_t*)(base + lay.overflow);
  S.n = (uint32_t)n;
  S.cell0 = 0;
  S.pad = 0;
  S.jbase = 0;
  S.rc2 = rc * rc;
  S.rc2_lo = (float)(rc * rc * (1.0 - 1e-5));
  S.rc2_hi = (float)(rc * rc * (1.0 + 1e-5));
  S.rclose2_64 = close_r * close_r * s2;
  S.rclose2 = (float)S.rclose2_64;
  S.p64.sig2 = s2;
  S.p64.eps4 = 4.0 * eps;
  S.p64.eps24 = 24.0 * eps;
  S.p64.eps48 = 48.0 * eps;
  S.p64.shift = shift;
  S.p32.sig2 = (float)s2;
  S.p32.eps4 = (float)(4.0 * eps);
  S.p32.eps24 = (float)(24.0 * eps);
  S.p32.eps48 = (float)(48.0 * eps);
  S.p32.shift = (float)shift;
  SweepLaunch L;
  L.mode = SWEEP_PARTICLE;
  L.g = &g;
  L.args = &S;
  L.precision = precision;
  L.debug = false;
  L.U = U;
  L.W = W;
  L.facc = nullptr;
  if (launch_sweep(L, st) != hipSuccess) return NCL_E_HIP;
  kn_flag<<<1, 64, 0, st>>>(small, U);
  return hipGetLastError() == hipSuccess ? NCL_OK : NCL_E_HIP;
}

}  // extern "C"
