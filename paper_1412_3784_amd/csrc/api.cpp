// C-ABI of the nemdcl library (declared in include/nemdcl.h).
//
// Host side: argument checks, the FP64 lattice at time t (Sec. 2.1-2.2 of
// Dobson, Fox & Saracino, arXiv:1412.3784), the cell geometry (Sec. 4.1,
// 4.2), scratch management, and the kernel launches on the handle's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

#include "../../include/nemdcl.h"
#include "geometry.hpp"
#include "kernels.hpp"

using namespace ncl;

struct ncl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // potential
  double eps = 1.0, sigma = 1.0, rc = 1.122462048309373, shift_on = 1.0;
  // options
  int do_tight = 1;
  int sweep_mode = SWEEP_AUTO;
  int deterministic = 1;
  double close_r = 0.45, band = 1e-5;
  // lattice
  bool have_lattice = false;
  RemapPolicy pol;
  double t = 0.0;
  double Lred[9];
  int64_t Mtot[9];
  int64_t coef[2] = {0, 0};
  // build state
  bool built = false;
  int variant = 0, precision = 0, debug = 0;
  uint32_t n = 0, ncells = 0;
  const double* x = nullptr;
  CellGeom geom;
  // scratch
  size_t cap_n = 0, cap_cells = 0, cap_blocks = 0, cap_wrap = 0, cap_dbgF = 0;
  uint32_t *cell_of = nullptr, *rank = nullptr, *cstart = nullptr, *perm = nullptr,
           *rs_val = nullptr, *rs_hist = nullptr, *rs_off = nullptr;
  size_t cap_rs = 0;
  double4* pos64 = nullptr;
  float4* pos32 = nullptr;
  float4* pos32lo = nullptr;
  int4* wrap = nullptr;
  double* partial = nullptr;
  uint32_t* overflow = nullptr;
  size_t cap_bricks = 0;
  int brick[6] = {1, 1, 1, 1, 1, 1};  // sx, sy, sz, nbx, nby, nbz
  // autotuner: candidate brick shapes of the current build (best first) and
  // the schedule chosen per workload class
  int ncand = 0;
  int cand[3][6];
  struct Tuned {
    uint64_t key;
    int mode;
    int brick[6];
    float ms[5];
  };
  std::vector<Tuned> tuned;
  Tuned last{};
  int used_mode = SWEEP_PARTICLE;  // schedule of the last force pass
  int used_brick[3] = {0, 0, 0};
  double* dbgF = nullptr;  // internal F/U/W for ncl_debug_pairs
  double* facc = nullptr;  // half-list sweep: FP64 forces in slot order
  size_t cap_facc = 0;
  // small device words: [0..3] stats (u64), then maxocc (u32), err (i32)
  unsigned long long* small = nullptr;
  std::string err;
};

static int fail(ncl_ctx* h, int code, const char* fmt, const char* a = "") {
  if (h) {
    char buf[512];
    snprintf(buf, sizeof buf, fmt, a);
    h->err = buf;
  }
  return code;
}

static int hip_fail(ncl_ctx* h, hipError_t e, const char* where) {
  if (h) h->err = std::string(where) + ": " + hipGetErrorString(e);
  return NCL_E_HIP;
}

#define HIPCHK(h, call)                          \
  do {                                           \
    hipError_t _e = (call);                      \
    if (_e != hipSuccess) return hip_fail(h, _e, #call); \
  } while (0)

template <class T>
static hipError_t grow(T** p, size_t* cap, size_t need) {
  if (*cap >= need && *p) return hipSuccess;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
    *p = nullptr;
  }
  size_t n = need > 0 ? need : 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e == hipSuccess) *cap = n;
  return e;
}

extern "C" {

int ncl_create(ncl_handle* out, int device, void* stream) {
  if (!out) return NCL_E_ARG;
  *out = nullptr;
  ncl_ctx* h = new (std::nothrow) ncl_ctx();
  if (!h) return NCL_E_CAPACITY;
  h->device = device;
  h->stream = (hipStream_t)stream;
  // no device work here: memory is allocated by the first ncl_build_cells, so
  // the host-only calls (lattice, cell counts) work without a GPU
  memset(h->Lred, 0, sizeof h->Lred);
  memset(h->Mtot, 0, sizeof h->Mtot);
  *out = h;
  return NCL_OK;
}

int ncl_destroy(ncl_handle h) {
  if (!h) return NCL_E_ARG;
  int code = NCL_OK;
  if (h->small) {  // device state exists only after a build
    if (hipSetDevice(h->device) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) code = NCL_E_HIP;
    void* bufs[] = {h->cell_of, h->rank,   h->cstart,  h->perm,     h->pos64,
                    h->pos32,   h->pos32lo, h->wrap,  h->partial,  h->overflow, h->dbgF,
                    h->facc,    h->rs_val,  h->rs_hist, h->rs_off, h->small};
    for (void* b : bufs)
      if (b && hipFree(b) != hipSuccess) code = NCL_E_HIP;
  }
  delete h;
  return code;
}

int ncl_set_potential(ncl_handle h, double eps, double sigma, double rc, int shift_energy) {
  if (!h) return NCL_E_ARG;
  if (!(eps > 0.0) || !(sigma > 0.0) || !(rc > 0.0) || !isfinite(eps + sigma + rc))
    return fail(h, NCL_E_ARG, "potential parameters must be positive and finite");
  h->eps = eps;
  h->sigma = sigma;
  h->rc = rc;
  h->shift_on = shift_energy ? 1.0 : 0.0;
  h->built = false;
  return NCL_OK;
}

int ncl_set_option(ncl_handle h, int option, double value) {
  if (!h) return NCL_E_ARG;
  switch (option) {
    case NCL_OPT_DO_TIGHT: h->do_tight = value != 0.0; break;
    case NCL_OPT_CLOSE_RADIUS:
      if (!(value >= 0.0)) return fail(h, NCL_E_ARG, "close radius must be >= 0");
      h->close_r = value;
      break;
    case NCL_OPT_SWEEP:
      if (value != 0.0 && value != 1.0 && value != 2.0 && value != 3.0)
        return fail(h, NCL_E_ARG, "sweep mode must be 0 (tiled), 1 (per particle), 2 (autotuned) or 3 (half list)");
      h->sweep_mode = (int)value;
      break;
    case NCL_OPT_DETERMINISTIC:
      if (value != 0.0 && value != 1.0) return fail(h, NCL_E_ARG, "deterministic must be 0 or 1");
      h->deterministic = (int)value;
      break;
    case NCL_OPT_BAND:
      if (!(value >= 0.0 && value < 0.1)) return fail(h, NCL_E_ARG, "band must be in [0, 0.1)");
      h->band = value;
      break;
    default: return fail(h, NCL_E_ARG, "unknown option");
  }
  h->built = false;
  return NCL_OK;
}

int ncl_set_lattice(ncl_handle h, const double L0[9], const double A[9], double t, int naut, const int32_t* aut) {
  if (!h || !L0 || !A) return NCL_E_ARG;
  if (naut < 0 || naut > 2 || (naut > 0 && !aut)) return fail(h, NCL_E_ARG, "naut must be 0, 1 or 2 with automorphisms");
  for (int k = 0; k < 9; ++k)
    if (!isfinite(L0[k]) || !isfinite(A[k])) return fail(h, NCL_E_ARG, "non-finite L0 or A");
  if (!isfinite(t)) return fail(h, NCL_E_ARG, "non-finite t");
  RemapPolicy p;
  int rc = remap_policy_init(&p, L0, A, naut, aut);
  if (rc == GEOM_E_SINGULAR) return fail(h, NCL_E_LATTICE, "singular L0");
  if (rc != GEOM_OK) return fail(h, NCL_E_LATTICE, "automorphism not unimodular / not diagonalised by L0, or flow incompatible");
  reduced_lattice(p, A, t, h->Lred, h->coef, h->Mtot);
  h->pol = p;
  h->t = t;
  h->have_lattice = true;
  h->built = false;
  return NCL_OK;
}

int ncl_get_lattice(ncl_handle h, double Lred[9], int32_t Mtot[9], int32_t coef[2]) {
  if (!h) return NCL_E_ARG;
  if (!h->have_lattice) return fail(h, NCL_E_STATE, "no lattice set");
  if (Lred)
    for (int k = 0; k < 9; ++k) Lred[k] = h->Lred[k];
  if (Mtot)
    for (int k = 0; k < 9; ++k) {
      if (h->Mtot[k] > INT32_MAX || h->Mtot[k] < INT32_MIN) return fail(h, NCL_E_CAPACITY, "Mtot overflows int32");
      Mtot[k] = (int32_t)h->Mtot[k];
    }
  if (coef) {
    coef[0] = (int32_t)h->coef[0];
    coef[1] = (int32_t)h->coef[1];
  }
  return NCL_OK;
}

static int make_geom(ncl_ctx* h, int variant, CellGeom* g) {
  int rc = cell_geom_init(g, h->Lred, h->Mtot, h->rc, variant == NCL_DYNAMIC_OFFSET ? VAR_DO : VAR_DS, h->do_tight);
  if (rc == GEOM_OK) cell_geom_bands(g, h->rc);
  if (rc == GEOM_E_SMALL) return fail(h, NCL_E_BOX_TOO_SMALL, "box too small for the cut-off: a cell count is below 1");
  if (rc != GEOM_OK) return fail(h, NCL_E_LATTICE, "singular basis");
  const double nc = (double)g->nc[0] * g->nc[1] * g->nc[2];
  if (nc > 2147483647.0) return fail(h, NCL_E_CAPACITY, "more than 2^31-1 cells");
  return NCL_OK;
}

int ncl_cell_counts(ncl_handle h, int variant, int32_t counts[3]) {
  if (!h || !counts) return NCL_E_ARG;
  if (variant != NCL_DYNAMIC_SIZE && variant != NCL_DYNAMIC_OFFSET) return fail(h, NCL_E_ARG, "bad variant");
  if (!h->have_lattice) return fail(h, NCL_E_STATE, "no lattice set");
  CellGeom g;
  int rc = make_geom(h, variant, &g);
  if (rc) return rc;
  for (int k = 0; k < 3; ++k) counts[k] = g.nc[k];
  return NCL_OK;
}

// Brick of home cells per workgroup of the tiled sweep: as many home
// particles as the 256 lanes can hold while the staged neighbourhood (home
// cells plus a rim of one or two cells, per variant) stays well inside the
// LDS tile.  Sizes come from the mean cell occupancy.
// Brick shapes for the LDS-tiled sweep, ranked by a model of useful home
// particles against staged neighbourhood size; the best three are kept as
// candidates for the autotuner and the best one is the default.
static void choose_brick(ncl_ctx* h, const CellGeom& g, size_t n, uint32_t nc) {
  const double occ = nc ? (double)n / nc : 1.0;
  // staged rim: DS adds one cell each side; DO adds the cells overlapping a
  // band of d_cut (about 2.5-3 cells per axis with offset rows)
  const double rim = (g.variant == VAR_DO) ? 2.6 : 2.0;
  double best[3] = {-1e300, -1e300, -1e300};
  int bs[3][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}};
  int found = 0;
  for (int sz = 1; sz <= g.nc[2] && sz <= 6; ++sz)
    for (int sy = 1; sy <= g.nc[1] && sy <= 12; ++sy)
      for (int sx = 1; sx <= g.nc[0] && sx <= 24; ++sx) {
        const double home = occ * sx * sy * sz;
        const double rows = (double)(sz + 2) * (sy + rim);
        const double cells = rows * (sx + rim);
        const double tile = occ * cells;
        if (rows > 56 || cells > 800 || sy * sz > 48 || tile > 0.86 * 2240) continue;
        const double score = fmin(home, 244.0) - 0.03 * tile;
        ++found;
        for (int r = 0; r < 3; ++r)
          if (score > best[r]) {
            for (int q = 2; q > r; --q) {
              best[q] = best[q - 1];
              for (int k = 0; k < 3; ++k) bs[q][k] = bs[q - 1][k];
            }
            best[r] = score;
            bs[r][0] = sx; bs[r][1] = sy; bs[r][2] = sz;
            break;
          }
      }
  h->ncand = found < 1 ? 1 : (found < 3 ? found : 3);
  for (int r = 0; r < h->ncand; ++r)
    for (int k = 0; k < 3; ++k) {
      h->cand[r][k] = bs[r][k];
      h->cand[r][3 + k] = (g.nc[k] + bs[r][k] - 1) / bs[r][k];
    }
  for (int k = 0; k < 6; ++k) h->brick[k] = h->cand[0][k];
}

static uint64_t tune_key(const ncl_ctx* h);

int ncl_build_cells(ncl_handle h, int variant, const double* x, int64_t n, int precision, int debug) {
  if (!h) return NCL_E_ARG;
  if (variant != NCL_DYNAMIC_SIZE && variant != NCL_DYNAMIC_OFFSET) return fail(h, NCL_E_ARG, "bad variant");
  if (precision < NCL_PREC_FP64 || precision > NCL_PREC_FP32_KAHAN) return fail(h, NCL_E_ARG, "bad precision");
  if (n < 0) return fail(h, NCL_E_ARG, "n < 0");
  if (n > 0 && !x) return fail(h, NCL_E_ARG, "null positions");
  if (n > 0x7fffff00LL) return fail(h, NCL_E_CAPACITY, "more than 2^31 particles");
  if (!h->have_lattice) return fail(h, NCL_E_STATE, "no lattice set");
  HIPCHK(h, hipSetDevice(h->device));
  if (!h->small) {
    HIPCHK(h, hipMalloc((void**)&h->small, 8 * sizeof(unsigned long long)));
    HIPCHK(h, hipMemsetAsync(h->small, 0, 8 * sizeof(unsigned long long), h->stream));
  }
  CellGeom g;
  int rc = make_geom(h, variant, &g);
  if (rc) return rc;
  const uint32_t nc = (uint32_t)((uint64_t)g.nc[0] * g.nc[1] * g.nc[2]);
  // capacity: cells never exceed V / rc^3 for a box of this volume
  const double vcap = fabs(mat_det(h->Lred)) / (h->rc * h->rc * h->rc);
  size_t want_cells = (size_t)nc + 1;
  if (h->cap_cells < want_cells) {
    const size_t bound = (size_t)fmin(vcap + 2.0, 2147483647.0);
    want_cells = want_cells > bound ? want_cells : bound;
  }
  const size_t un = (size_t)n;
  if (un > h->cap_n || !h->perm) {
    // per-particle arrays, all sized for cap_n particles
    void** bufs[] = {(void**)&h->cell_of, (void**)&h->rank,    (void**)&h->perm,  (void**)&h->pos64,
                     (void**)&h->pos32,   (void**)&h->pos32lo, (void**)&h->rs_val};
    for (void** b : bufs)
      if (*b) {
        HIPCHK(h, hipFree(*b));
        *b = nullptr;
      }
    h->cap_n = 0;
    const size_t m = un > 0 ? un : 1;
    HIPCHK(h, hipMalloc((void**)&h->cell_of, m * sizeof(uint32_t)));
    HIPCHK(h, hipMalloc((void**)&h->rank, m * sizeof(uint32_t)));
    HIPCHK(h, hipMalloc((void**)&h->perm, m * sizeof(uint32_t)));
    HIPCHK(h, hipMalloc((void**)&h->pos64, m * sizeof(double4)));
    // four spare entries: the per-particle sweep reads candidates in groups
    // of four and masks out those past a cell's run
    HIPCHK(h, hipMalloc((void**)&h->pos32, (m + 4) * sizeof(float4)));
    HIPCHK(h, hipMalloc((void**)&h->pos32lo, m * sizeof(float4)));
    HIPCHK(h, hipMalloc((void**)&h->rs_val, m * sizeof(uint32_t)));
    h->cap_n = m;
  }
  if (debug) HIPCHK(h, grow(&h->wrap, &h->cap_wrap, un));
  if (want_cells > h->cap_cells || !h->cstart) {
    if (h->cstart) HIPCHK(h, hipFree(h->cstart));
    h->cstart = nullptr;
    h->cap_cells = 0;
    HIPCHK(h, hipMalloc((void**)&h->cstart, cstart_words((uint32_t)(want_cells - 1)) * sizeof(uint32_t)));
    h->cap_cells = want_cells;
  }
  // radix sort of the cell keys: (digit, tile) counts and offsets
  {
    const size_t nrs = rs_offsets((uint32_t)un);
    if (nrs > h->cap_rs || !h->rs_hist) {
      if (h->rs_hist) HIPCHK(h, hipFree(h->rs_hist));
      if (h->rs_off) HIPCHK(h, hipFree(h->rs_off));
      h->rs_hist = h->rs_off = nullptr;
      h->cap_rs = 0;
      HIPCHK(h, hipMalloc((void**)&h->rs_hist, nrs * sizeof(uint32_t)));
      HIPCHK(h, hipMalloc((void**)&h->rs_off, nrs * sizeof(uint32_t)));
      h->cap_rs = nrs;
    }
  }
  choose_brick(h, g, (size_t)n, nc);
  {
    // one partial slot per sweep workgroup (the per-particle sweep's are the
    // smallest)
    size_t nbr = ((size_t)n + SWP_MIN_THREADS - 1) / SWP_MIN_THREADS;
    for (int r = 0; r < h->ncand; ++r)
      nbr = std::max(nbr, (size_t)h->cand[r][3] * h->cand[r][4] * h->cand[r][5]);
    if (nbr + 2 > h->cap_bricks || !h->overflow) {
      if (h->overflow) HIPCHK(h, hipFree(h->overflow));
      if (h->partial) HIPCHK(h, hipFree(h->partial));
      h->overflow = nullptr;
      h->partial = nullptr;
      h->cap_bricks = 0;
      HIPCHK(h, hipMalloc((void**)&h->overflow, (nbr + 2) * sizeof(uint32_t)));
      // block partials, then their second-level sums (one per 256 blocks)
      HIPCHK(h, hipMalloc((void**)&h->partial, PART_STRIDE * (nbr + 2 + (nbr + 2) / 256 + 1) * sizeof(double)));
      h->cap_bricks = nbr + 2;
    }
  }
  if (precision == NCL_PREC_FP32 &&
      (h->sweep_mode == SWEEP_HALF || (h->sweep_mode == SWEEP_AUTO && !h->deterministic)))
    HIPCHK(h, grow(&h->facc, &h->cap_facc, 3 * un));

  h->geom = g;
  h->variant = variant;
  h->precision = precision;
  h->debug = debug ? 1 : 0;
  h->n = (uint32_t)n;
  h->ncells = nc;
  h->x = x;
  BuildLaunch L;
  L.g = &h->geom;
  L.x = x;
  L.n = (uint32_t)n;
  L.ncells = nc;
  L.cell_of = h->cell_of;
  L.rank = h->rank;
  L.rs_val = h->rs_val;
  L.rs_hist = h->rs_hist;
  L.rs_off = h->rs_off;
  L.cstart = h->cstart;
  L.perm = h->perm;
  L.pos64 = h->pos64;
  L.pos32 = h->pos32;
  // the FP32 residuals are read by the tiled sweep only: skipped when the
  // force pass of this build cannot be tiled (an explicit other schedule,
  // or an autotuned class already tuned to another; an untuned class is
  // timed with tiled candidates).  Options and lattices change only with a
  // new build, so the choice made here holds for this build's force pass.
  bool need_lo = h->sweep_mode == SWEEP_TILED;
  if (h->sweep_mode == SWEEP_AUTO) {
    need_lo = true;
    const uint64_t key = tune_key(h);
    for (const auto& t : h->tuned)
      if (t.key == key) need_lo = t.mode == SWEEP_TILED;
  }
  L.pos32lo = need_lo ? h->pos32lo : nullptr;
  L.wrap = debug ? h->wrap : nullptr;
  L.err = (int*)(h->small + 5);
  hipError_t e = launch_build(L, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "cell build launch");
  h->built = true;
  return NCL_OK;
}

// brick-dependent fields of the LDS-tiled sweep: the brick shape and the
// FP32 screening band and residual unit that follow from its extent
static void brick_args(const ncl_ctx* h, SweepArgs* A) {
  const double rc2 = h->rc * h->rc;
  A->sx = h->brick[0];
  A->sy = h->brick[1];
  A->sz = h->brick[2];
  A->nbx = h->brick[3];
  A->nby = h->brick[4];
  A->nbz = h->brick[5];
  // largest brick-frame coordinate: half the brick plus the rim of staged
  // cells, per axis, through the cell step vectors
  const CellGeom& g = h->geom;
  const double ext[3] = {0.5 * A->sx + 4.0, 0.5 * A->sy + 4.0, 0.5 * A->sz + 3.0};
  double xmax = 0.0;
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
    for (int c = 0; c < 3; ++c) s += fabs(g.cen[3 * r + c]) * ext[c];
    xmax = fmax(xmax, s);
  }
  const double rc = h->rc;
  // FP32 screening: each coordinate is off by at most half an ulp of xmax,
  // the difference by one more half ulp; bound the r^2 error and double it
  const double dd = ulp32(xmax) + 0.5 * ulp32(2.0 * rc);
  const double dr2 = 2.0 * rc * sqrt(3.0) * dd + 3.0 * dd * dd + 2.0 * ulp32(rc2);
  A->rc2c = nextafterf((float)(rc2 + 2.0 * dr2), INFINITY);
  // residual unit: half an ulp of xmax spans 16384 units of the int16
  A->res_unit = ulp32(xmax) / 32768.0;
  const double dfine = A->res_unit + 4e-16 * xmax;
  A->band64 = 4.0 * (2.0 * rc * sqrt(3.0) * dfine + 1e-15 * rc2);
}

static void fill_sweep_args(ncl_ctx* h, SweepArgs* A, void* F) {
  const double s2 = h->sigma * h->sigma;
  double shift = 0.0;
  if (h->shift_on != 0.0) {
    const double q = s2 / (h->rc * h->rc);
    const double q6 = q * q * q;
    shift = 4.0 * h->eps * (q6 * q6 - q6);
  }
  A->pos64 = h->pos64;
  A->pos32 = h->pos32;
  A->pos32lo = h->pos32lo;
  A->cstart = h->cstart;
  A->perm = h->perm;
  A->wrap = h->wrap;
  A->F = F;
  A->partial = h->partial;
  A->partial2 = h->partial + PART_STRIDE * h->cap_bricks;
  A->stats = h->small;
  A->dbg_count = nullptr;
  A->dbg_hash = nullptr;
  A->n = h->n;
  A->cell0 = 0;
  A->pad = 0;
  A->jbase = 0;
  const double rc2 = h->rc * h->rc;
  A->rc2 = rc2;
  A->rc2_lo = (float)(rc2 * (1.0 - h->band));
  A->rc2_hi = (float)(rc2 * (1.0 + h->band));
  A->rclose2 = (float)(h->close_r * h->close_r * s2);
  A->p64.sig2 = s2;
  A->p64.eps4 = 4.0 * h->eps;
  A->p64.eps24 = 24.0 * h->eps;
  A->p64.eps48 = 48.0 * h->eps;
  A->p64.shift = shift;
  A->overflow = h->overflow;
  brick_args(h, A);
  A->rclose2_64 = h->close_r * h->close_r * s2;
  A->fix_q = ldexp(h->eps / h->sigma, -20);
  A->fix_inv = 1.0 / A->fix_q;
  A->rwin2_64 = fmax(A->rclose2_64, 0.09 * s2);
  A->p32.sig2 = (float)s2;
  A->p32.eps4 = (float)(4.0 * h->eps);
  A->p32.eps24 = (float)(24.0 * h->eps);
  A->p32.eps48 = (float)(48.0 * h->eps);
  A->p32.shift = (float)shift;
}

// Workload class for the autotuner: variant, precision, cells per axis and
// occupancy in quarter-octaves; a schedule is re-tuned when any changes.
static uint64_t tune_key(const ncl_ctx* h) {
  const double occ = h->ncells ? (double)h->n / h->ncells : 0.0;
  const int ob = occ > 0.0 ? (int)floor(4.0 * log2(occ)) + 64 : 0;
  uint64_t k = (uint64_t)h->geom.variant | ((uint64_t)h->precision << 2) | ((uint64_t)(ob & 0xff) << 4);
  for (int a = 0; a < 3; ++a) k |= (uint64_t)(h->geom.nc[a] & 0xffff) << (12 + 16 * a);
  return k | ((uint64_t)(h->deterministic & 1) << 60);
}

static hipError_t sweep_with(ncl_ctx* h, SweepArgs* A, int mode, const int* brick, double* U, double* W) {
  for (int k = 0; k < 6; ++k) h->brick[k] = brick[k];
  brick_args(h, A);
  SweepLaunch L;
  L.mode = mode;
  L.g = &h->geom;
  L.args = A;
  L.precision = h->precision;
  L.debug = false;
  L.U = U;
  L.W = W;
  L.facc = h->facc;
  return launch_sweep(L, h->stream);
}

// the half-list sweep runs in FP32 precision and needs its force array
static bool half_ok(const ncl_ctx* h) {
  return h->precision == NCL_PREC_FP32 && h->facc && h->cap_facc >= 3 * (size_t)h->n;
}

// Autotuner: time each candidate schedule once on the caller's stream (after
// one untimed launch) with HIP events; the fastest is cached for the class.
// The half list is a candidate only when run-to-run identical forces are not
// required.
static int autotune(ncl_ctx* h, SweepArgs* A, double* U, double* W, ncl_ctx::Tuned* out) {
  int modes[5], bricks[5][6], nc = 0;
  modes[nc] = SWEEP_PARTICLE;
  for (int k = 0; k < 6; ++k) bricks[nc][k] = h->cand[0][k];
  ++nc;
  for (int r = 0; r < h->ncand && nc < 4; ++r, ++nc) {
    modes[nc] = SWEEP_TILED;
    for (int k = 0; k < 6; ++k) bricks[nc][k] = h->cand[r][k];
  }
  if (!h->deterministic && half_ok(h)) {
    modes[nc] = SWEEP_HALF;
    for (int k = 0; k < 6; ++k) bricks[nc][k] = h->cand[0][k];
    ++nc;
  }
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  int best = 0;
  float bms = 3.0e38f;
  out->key = tune_key(h);
  for (int c = 0; c < 5; ++c) out->ms[c] = -1.0f;
  for (int c = 0; c < nc; ++c) {
    hipError_t e = sweep_with(h, A, modes[c], bricks[c], U, W);
    if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
    if (e == hipSuccess) e = sweep_with(h, A, modes[c], bricks[c], U, W);
    if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return hip_fail(h, e, "autotune");
    }
    out->ms[modes[c] == SWEEP_HALF ? 4 : c] = ms;
    if (ms < bms) {
      bms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  out->mode = modes[best];
  for (int k = 0; k < 6; ++k) out->brick[k] = bricks[best][k];
  return NCL_OK;
}

int ncl_compute_forces(ncl_handle h, void* F, double* U, double* W) {
  if (!h) return NCL_E_ARG;
  if (!h->built) return fail(h, NCL_E_STATE, "ncl_build_cells must precede ncl_compute_forces");
  if (!U || !W || (h->n > 0 && !F)) return fail(h, NCL_E_ARG, "null output");
  HIPCHK(h, hipSetDevice(h->device));
  SweepArgs A;
  fill_sweep_args(h, &A, F);
  int mode = h->sweep_mode;
  if (mode == SWEEP_HALF && !half_ok(h))
    return fail(h, NCL_E_ARG, "the half-list sweep needs NCL_PREC_FP32 (set the sweep option before ncl_build_cells)");
  int brick[6];
  for (int k = 0; k < 6; ++k) brick[k] = h->cand[0][k];
  if (mode == SWEEP_AUTO) {
    const uint64_t key = tune_key(h);
    const ncl_ctx::Tuned* t = nullptr;
    for (const auto& e : h->tuned)
      if (e.key == key) t = &e;
    // the autotuner times schedules with a host wait on events, which a
    // stream under graph capture cannot do: a class first met during a
    // capture runs the per-particle sweep and is tuned on a later,
    // uncaptured call
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(h, hipStreamIsCapturing(h->stream, &cap));
    if (!t && cap != hipStreamCaptureStatusNone) {
      mode = SWEEP_PARTICLE;
    } else {
      if (!t) {
        ncl_ctx::Tuned nt{};
        const int rc = autotune(h, &A, U, W, &nt);
        if (rc) return rc;
        h->tuned.push_back(nt);
        t = &h->tuned.back();
      }
      h->last = *t;
      mode = t->mode;
      for (int k = 0; k < 6; ++k) brick[k] = t->brick[k];
    }
  }
  hipError_t e = sweep_with(h, &A, mode, brick, U, W);
  if (e != hipSuccess) return hip_fail(h, e, "sweep launch");
  h->used_mode = mode;
  for (int k = 0; k < 3; ++k) h->used_brick[k] = mode == SWEEP_TILED ? brick[k] : 0;
  return NCL_OK;
}

int ncl_debug_pairs(ncl_handle h, int64_t* count, uint64_t* hash) {
  if (!h) return NCL_E_ARG;
  if (!h->built || !h->debug) return fail(h, NCL_E_STATE, "ncl_build_cells(..., debug=1) must precede ncl_debug_pairs");
  if (h->n > 0 && (!count || !hash)) return fail(h, NCL_E_ARG, "null output");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, grow(&h->dbgF, &h->cap_dbgF, 3 * (size_t)h->n + 10));
  SweepArgs A;
  fill_sweep_args(h, &A, h->dbgF);
  A.dbg_count = count;
  A.dbg_hash = hash;
  SweepLaunch L;
  L.mode = h->sweep_mode == SWEEP_AUTO ? (h->last.key == tune_key(h) ? h->last.mode : SWEEP_PARTICLE) : h->sweep_mode;
  if (L.mode == SWEEP_TILED) {
    const int* b = h->sweep_mode == SWEEP_AUTO ? h->last.brick : h->cand[0];
    for (int k = 0; k < 6; ++k) h->brick[k] = b[k];
    brick_args(h, &A);
  }
  L.g = &h->geom;
  L.args = &A;
  L.precision = h->precision;
  L.debug = true;
  L.U = h->dbgF + 3 * (size_t)h->n;
  L.W = h->dbgF + 3 * (size_t)h->n + 1;
  L.facc = h->facc;
  if (L.mode == SWEEP_HALF && !half_ok(h)) return fail(h, NCL_E_ARG, "the half-list sweep needs NCL_PREC_FP32");
  hipError_t e = launch_sweep(L, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "debug sweep launch");
  return NCL_OK;
}

int ncl_get_stats(ncl_handle h, ncl_stats* out) {
  if (!h || !out) return NCL_E_ARG;
  if (!h->small) return fail(h, NCL_E_STATE, "nothing built yet");
  HIPCHK(h, hipSetDevice(h->device));
  if (h->built && h->cstart) {
    const hipError_t e = launch_max_occupancy(h->cstart, h->ncells, (uint32_t*)(h->small + 4), h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "occupancy");
  }
  unsigned long long w[8];
  HIPCHK(h, hipMemcpyAsync(w, h->small, sizeof w, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  memset(out, 0, sizeof *out);
  out->n = h->n;
  out->variant = h->variant;
  out->precision = h->precision;
  for (int k = 0; k < 3; ++k) out->cells[k] = h->geom.nc[k];
  out->ncells = h->ncells;
  out->candidates = (int64_t)w[0];
  out->pairs = (int64_t)w[1];
  out->fp64_pairs = (int64_t)w[2];
  out->neighbourhood = (int64_t)w[3];
  out->max_occupancy = (int32_t)(uint32_t)(w[4] & 0xffffffffull);
  out->sweep = h->used_mode;
  for (int k = 0; k < 3; ++k) out->brick[k] = h->used_brick[k];
  for (int k = 0; k < 5; ++k) out->tune_ms[k] = -1.0f;
  for (const auto& t : h->tuned)
    if (t.key == tune_key(h))
      for (int k = 0; k < 5; ++k) out->tune_ms[k] = t.ms[k];
  const int errw = (int)(uint32_t)(w[5] & 0xffffffffull);
  if (errw) {
    int zero = 0;
    HIPCHK(h, hipMemcpyAsync((char*)(h->small + 5), &zero, sizeof zero, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return fail(h, NCL_E_DEVICE_FLAG, "a kernel flagged a non-finite position");
  }
  return NCL_OK;
}

const char* ncl_last_error(ncl_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
