// C-ABI of the batched form (declared in include/nemdcl.h): many independent
// boxes of uneven size, each with its own flow, rate and strain time, binned
// and swept together, and SLLOD steps over such a batch, optionally replayed
// as one captured HIP graph per step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/nemdcl.h"
#include "batch.hpp"
#include "geometry.hpp"
#include "kernels.hpp"

using namespace ncl;

struct ncl_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own = nullptr;       // private stream for graph capture
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int32_t nrep = 0;
  std::vector<int64_t> n;
  uint64_t ntot = 0, nslots = 0, ncells = 0;
  double eps = 1.0, sigma = 1.0, rc = 1.122462048309373, shift_on = 1.0, close_r = 0.45;
  int do_tight = 1, variant = NCL_DYNAMIC_OFFSET, precision = NCL_PREC_FP32, debug = 0;
  double skin = 0.0;  // > 0: SLLOD reuses neighbour lists within d_cut + skin
  uint32_t kmax = 0;
  int64_t rebuilds = 0;  // list rebuilds of the last SLLOD run
  bool have_lattice = false, built = false;
  // schedule of the force pass: staged launches (SWEEP_PARTICLE), one fused
  // persistent bin + force launch (NCL_SWEEP_FUSED) or the autotuner's
  // choice (SWEEP_AUTO, timed once per variant and precision)
  int sweep_mode = SWEEP_AUTO;
  struct Tuned {
    int key, mode;
    float ms[2];  // staged, fused
  };
  std::vector<Tuned> tuned;
  int used_mode = SWEEP_PARTICLE;
  float used_ms[2] = {-1.0f, -1.0f};
  bool pending = false;          // fused schedule: cells not built yet, the force pass bins
  const double* x = nullptr;     // positions of the last build (xcopy for the fused schedule)
  double* xcopy = nullptr;       // fused schedule: the build's positions, read by the force pass
  uint32_t* fstate = nullptr;    // fused: queue counter, then one ready flag per replica
  uint32_t *order = nullptr, *blk_order = nullptr;  // fused: bin order, sweep block order
  std::vector<double> t0;
  // device memory (one allocation per array)
  uint32_t *n_off = nullptr, *slot_off = nullptr, *cell_off = nullptr, *blk_rep = nullptr, *in_rep = nullptr;
  RemapPolicy* pol = nullptr;
  double *t0_d = nullptr, *adiag = nullptr, *lred = nullptr, *kpart = nullptr, *partial = nullptr;
  CellGeom* geom = nullptr;
  uint32_t* small = nullptr;  // [0..7] stats (4 u64), [8] maxocc, [9] err, [10] step
  uint32_t *rs_va = nullptr, *rs_vb = nullptr, *rs_hist = nullptr, *rs_off = nullptr;
  uint32_t *cell_of = nullptr, *rank = nullptr, *cstart = nullptr,
           *perm = nullptr;
  double4* pos64 = nullptr;
  float4* pos32 = nullptr;
  int4* wrap = nullptr;
  double* dbgF = nullptr;
  int64_t *pcur = nullptr, *pb = nullptr;
  uint2* vl = nullptr;
  uint32_t* vl_cnt = nullptr;
  double4* ysl = nullptr;
  double *xb = nullptr, *tb = nullptr;
  unsigned long long* dmax = nullptr;
  std::string err;
};

static int bfail(ncl_batch* b, int code, const char* msg) {
  if (b) b->err = msg;
  return code;
}
static int bhip(ncl_batch* b, hipError_t e, const char* where) {
  if (b) b->err = std::string(where) + ": " + hipGetErrorString(e);
  return NCL_E_HIP;
}
#define BCHK(b, call)                                 \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return bhip(b, _e, #call);  \
  } while (0)

template <class T>
static hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, (n > 0 ? n : 1) * sizeof(T));
}

static BatchDev view(ncl_batch* b) {
  BatchDev D;
  D.nrep = (uint32_t)b->nrep;
  D.n = (uint32_t)b->ntot;
  D.nslots = (uint32_t)b->nslots;
  D.ncells = (uint32_t)b->ncells;
  D.variant = b->variant == NCL_DYNAMIC_OFFSET ? VAR_DO : VAR_DS;
  D.do_tight = b->do_tight;
  D.rc = b->rc;
  D.rc_cells = b->rc + b->skin;
  D.n_off = b->n_off;
  D.slot_off = b->slot_off;
  D.cell_off = b->cell_off;
  D.blk_rep = b->blk_rep;
  D.in_rep = b->in_rep;
  D.pol = b->pol;
  D.t0 = b->t0_d;
  D.adiag = b->adiag;
  D.geom = b->geom;
  D.lred = b->lred;
  D.step = b->small + 10;
  D.err = (int*)(b->small + 9);
  D.cell_of = b->cell_of;
  D.rank = b->rank;
  D.rs_va = b->rs_va;
  D.rs_vb = b->rs_vb;
  D.rs_hist = b->rs_hist;
  D.rs_off = b->rs_off;
  D.cstart = b->cstart;
  D.perm = b->perm;
  D.pos64 = b->pos64;
  D.pos32 = b->pos32;
  D.wrap = (b->debug || b->skin > 0.0) ? b->wrap : nullptr;
  D.pcur = b->pcur;
  D.kmax = b->kmax;
  D.vl = b->vl;
  D.vl_cnt = b->vl_cnt;
  D.ysl = b->ysl;
  D.xb = b->xb;
  D.tb = b->tb;
  D.pb = b->pb;
  D.dmax = b->dmax;
  D.need = b->small + 11;
  D.kpart = b->kpart;
  return D;
}

static void sweep_args(ncl_batch* b, SweepArgs* A, void* F) {
  memset(A, 0, sizeof *A);
  const double s2 = b->sigma * b->sigma, rc2 = b->rc * b->rc;
  double shift = 0.0;
  if (b->shift_on != 0.0) {
    const double q = s2 / rc2, q6 = q * q * q;
    shift = 4.0 * b->eps * (q6 * q6 - q6);
  }
  A->pos64 = b->pos64;
  A->pos32 = b->pos32;
  A->pos32lo = nullptr;  // read by the single-box tiled sweep only
  A->cstart = b->cstart;
  A->perm = b->perm;
  A->wrap = b->wrap;
  A->F = F;
  A->partial = b->partial;
  A->partial2 = nullptr;  // per-replica finalisation reads the block partials directly
  A->stats = (unsigned long long*)b->small;
  A->n = (uint32_t)b->nslots;
  A->rc2 = rc2;
  A->rclose2_64 = b->close_r * b->close_r * s2;
  A->fix_q = A->fix_inv = A->rwin2_64 = 0.0;  // half list: single-box only
  A->rclose2 = (float)A->rclose2_64;
  A->p64.sig2 = s2;
  A->p64.eps4 = 4.0 * b->eps;
  A->p64.eps24 = 24.0 * b->eps;
  A->p64.eps48 = 48.0 * b->eps;
  A->p64.shift = shift;
  A->p32.sig2 = (float)s2;
  A->p32.eps4 = (float)(4.0 * b->eps);
  A->p32.eps24 = (float)(24.0 * b->eps);
  A->p32.eps48 = (float)(48.0 * b->eps);
  A->p32.shift = (float)shift;
}

static int tune_key(const ncl_batch* b) { return b->variant * 4 + b->precision; }

static const ncl_batch::Tuned* tuned_entry(const ncl_batch* b) {
  for (const auto& t : b->tuned)
    if (t.key == tune_key(b)) return &t;
  return nullptr;
}

// schedule the next force pass runs with
static int sched_mode(const ncl_batch* b) {
  if (b->sweep_mode != SWEEP_AUTO) return b->sweep_mode;
  const ncl_batch::Tuned* t = tuned_entry(b);
  return t ? t->mode : SWEEP_PARTICLE;
}

// Batched autotuner: the staged build + sweep against the fused launch, each
// timed once after an untimed run, with HIP events on the caller's stream;
// the faster is kept for this variant and precision.  Both leave the same
// cells and the same forces (the sort order and the sweep are identical).
// largest replica the autotuner tries the fused schedule on: one workgroup
// bins a replica, about 1 ms per 65,536 particles
constexpr int64_t FUSED_TUNE_MAX_N = 131072;

static int tune(ncl_batch* b, const SweepArgs& A, double* U, double* W) {
  const BatchDev D = view(b);
  if (*std::max_element(b->n.begin(), b->n.end()) > FUSED_TUNE_MAX_N) {
    // the fused schedule is not a candidate: the staged pass only
    BCHK(b, batch_prologue(D, 0, 0.0, b->stream));
    BCHK(b, batch_build(D, b->x, b->stream));
    BCHK(b, batch_sweep(A, D, b->precision, false, U, W, b->stream));
    ncl_batch::Tuned t{tune_key(b), SWEEP_PARTICLE, {-1.0f, -1.0f}};
    b->tuned.push_back(t);
    b->used_mode = SWEEP_PARTICLE;
    return NCL_OK;
  }
  hipEvent_t ev[3];
  for (auto& e : ev) BCHK(b, hipEventCreate(&e));
  float ms[2] = {0.0f, 0.0f};
  hipError_t e = hipSuccess;
  for (int m = 0; m < 2 && e == hipSuccess; ++m)
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      if (rep == 1) e = hipEventRecord(ev[0], b->stream);
      // the fused schedule pays a copy of the positions at every build: its
      // cost is timed by copying the copy onto itself (same bytes moved)
      if (m == 1 && e == hipSuccess) e = batch_copy(b->xcopy, b->xcopy, 3 * b->ntot, b->stream);
      if (e == hipSuccess) e = batch_prologue(D, 0, 0.0, b->stream);
      if (m == 0) {
        if (e == hipSuccess) e = batch_build(D, b->x, b->stream);
        if (e == hipSuccess) e = batch_sweep(A, D, b->precision, false, U, W, b->stream);
      } else {
        if (e == hipSuccess) e = batch_fused(A, D, b->x, b->precision, b->fstate, b->order, b->blk_order, U, W, b->stream);
      }
      if (rep == 1 && e == hipSuccess) e = hipEventRecord(ev[1], b->stream);
      if (rep == 1 && e == hipSuccess) e = hipEventSynchronize(ev[1]);
      if (rep == 1 && e == hipSuccess) e = hipEventElapsedTime(&ms[m], ev[0], ev[1]);
    }
  for (auto& q : ev) (void)hipEventDestroy(q);
  if (e != hipSuccess) return bhip(b, e, "batched autotuner");
  ncl_batch::Tuned t{tune_key(b), ms[1] < ms[0] ? NCL_SWEEP_FUSED : SWEEP_PARTICLE, {ms[0], ms[1]}};
  b->tuned.push_back(t);
  b->used_mode = t.mode;  // the schedule of this workload from now on
  b->used_ms[0] = ms[0];
  b->used_ms[1] = ms[1];
  return NCL_OK;
}

static void free_all(ncl_batch* b) {
  void* bufs[] = {b->n_off,  b->slot_off, b->cell_off, b->blk_rep, b->pol,     b->t0_d,    b->adiag,
                  b->lred,   b->kpart,    b->partial,  b->geom,    b->small,   b->cell_of, b->rank,
                  b->cstart, b->perm,     b->pos64,    b->pos32,
                  b->wrap,   b->dbgF,     b->rs_va,    b->rs_vb,   b->rs_hist, b->rs_off,
                  b->pcur,   b->pb,       b->vl,       b->ysl,     b->vl_cnt,  b->xb,
                  b->tb,     b->dmax,     b->fstate,   b->order,   b->blk_order, b->xcopy, b->in_rep};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
}

extern "C" {

int ncl_batch_create(ncl_batch_handle* out, int device, void* stream, int32_t nrep, const int64_t* n) {
  if (!out || nrep <= 0 || !n) return NCL_E_ARG;
  *out = nullptr;
  uint64_t tot = 0, slots = 0;
  for (int r = 0; r < nrep; ++r) {
    if (n[r] < 1) return NCL_E_ARG;
    tot += (uint64_t)n[r];
    slots += (uint64_t)((n[r] + 255) / 256) * 256;
  }
  if (slots >= 0xffffff00ull) return NCL_E_CAPACITY;
  ncl_batch* b = new (std::nothrow) ncl_batch();
  if (!b) return NCL_E_CAPACITY;
  b->device = device;
  b->stream = (hipStream_t)stream;
  b->nrep = nrep;
  b->n.assign(n, n + nrep);
  b->ntot = tot;
  b->nslots = slots;
  hipError_t e = hipSetDevice(device);
  std::vector<uint32_t> noff(nrep + 1), soff(nrep + 1), brep(slots / 256), irep((tot + 255) / 256);
  noff[0] = soff[0] = 0;
  for (int r = 0; r < nrep; ++r) {
    noff[r + 1] = noff[r] + (uint32_t)n[r];
    soff[r + 1] = soff[r] + (uint32_t)(((n[r] + 255) / 256) * 256);
    for (uint32_t q = soff[r] / 256; q < soff[r + 1] / 256; ++q) brep[q] = (uint32_t)r;
  }
  // replica of particle 256 q: the last r with noff[r] <= 256 q
  for (size_t q = 0, r = 0; q < irep.size(); ++q) {
    while (r + 1 < (size_t)nrep && noff[r + 1] <= 256 * q) ++r;
    irep[q] = (uint32_t)r;
  }
  if (e == hipSuccess) e = dalloc(&b->n_off, nrep + 1);
  if (e == hipSuccess) e = dalloc(&b->slot_off, nrep + 1);
  if (e == hipSuccess) e = dalloc(&b->blk_rep, brep.size());
  if (e == hipSuccess) e = dalloc(&b->in_rep, irep.size());
  if (e == hipSuccess) e = dalloc(&b->small, 16);
  if (e == hipSuccess) e = dalloc(&b->perm, slots);
  if (e == hipSuccess) e = dalloc(&b->pos64, slots);
  if (e == hipSuccess) e = dalloc(&b->pos32, slots + 4);  // + 4: groups of four candidate reads
  if (e == hipSuccess) e = dalloc(&b->cell_of, tot);
  if (e == hipSuccess) e = dalloc(&b->rank, tot);
  if (e == hipSuccess) e = dalloc(&b->rs_va, tot);
  if (e == hipSuccess) e = dalloc(&b->rs_vb, tot);
  if (e == hipSuccess) e = dalloc(&b->rs_hist, rs_offsets((uint32_t)tot));
  if (e == hipSuccess) e = dalloc(&b->rs_off, rs_offsets((uint32_t)tot));
  // one partial per sweep workgroup, then (one-wave workgroups) their sums per
  // 256-slot block
  if (e == hipSuccess) e = dalloc(&b->partial, PART_STRIDE * (slots / SWP_MIN_THREADS + slots / 256 + 1));
  if (e == hipSuccess) e = dalloc(&b->kpart, 3 * (slots / 256 + 1));
  if (e == hipSuccess) e = dalloc(&b->pol, nrep);
  if (e == hipSuccess) e = dalloc(&b->t0_d, nrep);
  if (e == hipSuccess) e = dalloc(&b->adiag, 3 * (size_t)nrep);
  if (e == hipSuccess) e = dalloc(&b->lred, 9 * (size_t)nrep);
  if (e == hipSuccess) e = dalloc(&b->geom, nrep);
  if (e == hipSuccess) e = dalloc(&b->pcur, 2 * (size_t)nrep);
  // fused schedule: replicas binned smallest first, their sweep blocks in the
  // same order (a block's replica is then usually binned when it is taken)
  std::vector<uint32_t> ord(nrep), bord;
  for (int r = 0; r < nrep; ++r) ord[r] = (uint32_t)r;
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t c) { return n[a] < n[c]; });
  bord.reserve(slots / 256);
  for (uint32_t r : ord)
    for (uint32_t q = soff[r] / 256; q < soff[r + 1] / 256; ++q) bord.push_back(q);
  if (e == hipSuccess) e = dalloc(&b->fstate, (size_t)nrep + 1);
  if (e == hipSuccess) e = dalloc(&b->order, (size_t)nrep);
  if (e == hipSuccess) e = dalloc(&b->blk_order, bord.size());
  if (e == hipSuccess) e = hipMemcpy(b->order, ord.data(), ord.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && !bord.empty()) e = hipMemcpy(b->blk_order, bord.data(), bord.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->n_off, noff.data(), noff.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->slot_off, soff.data(), soff.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && !brep.empty()) e = hipMemcpy(b->blk_rep, brep.data(), brep.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && !irep.empty()) e = hipMemcpy(b->in_rep, irep.data(), irep.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->small, 0, 16 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    free_all(b);
    delete b;
    return NCL_E_HIP;
  }
  *out = b;
  return NCL_OK;
}

int ncl_batch_destroy(ncl_batch_handle b) {
  if (!b) return NCL_E_ARG;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  if (b->own) (void)hipStreamSynchronize(b->own);
  free_all(b);
  if (b->own) (void)hipStreamDestroy(b->own);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  delete b;
  return NCL_OK;
}

int ncl_batch_set_potential(ncl_batch_handle b, double eps, double sigma, double rc, int shift_energy) {
  if (!b) return NCL_E_ARG;
  if (!(eps > 0.0) || !(sigma > 0.0) || !(rc > 0.0) || !isfinite(eps + sigma + rc))
    return bfail(b, NCL_E_ARG, "potential parameters must be positive and finite");
  if (b->have_lattice && rc != b->rc) return bfail(b, NCL_E_STATE, "set the potential before the lattices");
  b->eps = eps;
  b->sigma = sigma;
  b->rc = rc;
  b->shift_on = shift_energy ? 1.0 : 0.0;
  return NCL_OK;
}

int ncl_batch_set_option(ncl_batch_handle b, int option, double value) {
  if (!b) return NCL_E_ARG;
  if (option == NCL_OPT_DO_TIGHT) {
    b->do_tight = value != 0.0;
  } else if (option == NCL_OPT_CLOSE_RADIUS) {
    if (!(value >= 0.0)) return bfail(b, NCL_E_ARG, "close radius must be >= 0");
    b->close_r = value;
  } else if (option == NCL_OPT_SWEEP) {
    if (value != 1.0 && value != 2.0 && value != 4.0)
      return bfail(b, NCL_E_ARG, "batch sweep mode must be 1 (staged), 2 (autotuned) or 4 (fused)");
    b->sweep_mode = (int)value;
  } else if (option == NCL_OPT_SKIN) {
    if (!(value >= 0.0) || !isfinite(value)) return bfail(b, NCL_E_ARG, "skin must be >= 0");
    if (b->have_lattice) return bfail(b, NCL_E_STATE, "set the skin before ncl_batch_set_lattices");
    b->skin = value;
  } else {
    return bfail(b, NCL_E_ARG, "option not available for batches");
  }
  b->built = false;
  return NCL_OK;
}

int ncl_batch_set_lattices(ncl_batch_handle b, int variant, const double* L0, const double* A, const double* t,
                           const int32_t* naut, const int32_t* aut) {
  if (!b || !L0 || !A || !t || !naut) return NCL_E_ARG;
  if (variant != NCL_DYNAMIC_SIZE && variant != NCL_DYNAMIC_OFFSET) return bfail(b, NCL_E_ARG, "bad variant");
  BCHK(b, hipSetDevice(b->device));
  const int R = b->nrep;
  std::vector<RemapPolicy> pol(R);
  std::vector<double> ad(3 * (size_t)R);
  std::vector<uint32_t> coff(R + 1);
  coff[0] = 0;
  const double rc3 = b->rc * b->rc * b->rc;
  for (int r = 0; r < R; ++r) {
    if (naut[r] < 0 || naut[r] > 2 || (naut[r] > 0 && !aut)) return bfail(b, NCL_E_ARG, "naut must be 0, 1 or 2");
    for (int k = 0; k < 9; ++k)
      if (!isfinite(L0[9 * r + k]) || !isfinite(A[9 * r + k])) return bfail(b, NCL_E_ARG, "non-finite L0 or A");
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (i != j && A[9 * r + 3 * i + j] != 0.0) return bfail(b, NCL_E_LATTICE, "batched flows must be diagonal");
    const int rcode = remap_policy_init(&pol[r], L0 + 9 * r, A + 9 * r, naut[r], naut[r] ? aut + 18 * r : nullptr);
    if (rcode != GEOM_OK) return bfail(b, NCL_E_LATTICE, "automorphism not unimodular / not diagonalised, or flow incompatible");
    const double tr = A[9 * r] + A[9 * r + 4] + A[9 * r + 8];
    if (fabs(tr) > 1e-12 * (fabs(A[9 * r]) + fabs(A[9 * r + 4]) + fabs(A[9 * r + 8]) + 1e-300))
      return bfail(b, NCL_E_LATTICE, "batched flows must be traceless (constant box volume)");
    for (int d = 0; d < 3; ++d) ad[3 * r + d] = A[9 * r + 4 * d];
    // cells never exceed V / rc^3 (product of heights <= volume)
    const double cap = floor(fabs(mat_det(L0 + 9 * r)) / rc3) + 1.0;
    if (coff[r] + cap > 2.0e9) return bfail(b, NCL_E_CAPACITY, "too many cells");
    coff[r + 1] = coff[r] + (uint32_t)cap;
  }
  const uint64_t ncells = coff[R];
  if (ncells != b->ncells || !b->cstart) {
    if (b->cstart) (void)hipFree(b->cstart);
    if (b->cell_off) (void)hipFree(b->cell_off);
    b->cstart = b->cell_off = nullptr;
    BCHK(b, dalloc(&b->cstart, cstart_words((uint32_t)ncells)));
    BCHK(b, dalloc(&b->cell_off, (size_t)R + 1));
    b->ncells = ncells;
  }
  BCHK(b, hipMemcpy(b->cell_off, coff.data(), coff.size() * 4, hipMemcpyHostToDevice));
  if (b->skin > 0.0) {
    // list capacity: 1.5 times the mean count within d_cut + skin of the
    // densest replica, plus 24 (a rebuild that needs more fails with
    // NCL_E_CAPACITY)
    const double rl = b->rc + b->skin;
    double most = 0.0;
    for (int r = 0; r < R; ++r)
      most = fmax(most, (double)b->n[r] / fabs(mat_det(L0 + 9 * r)) * 4.0 / 3.0 * M_PI * rl * rl * rl);
    const double km = 4.0 * ceil((1.5 * most + 24.0) / 4.0);  // entries come in groups of four
    if (km * (double)b->nslots > 4.0e10 || b->nslots >= (1ull << 31))
      return bfail(b, NCL_E_CAPACITY, "neighbour lists would not fit");
    const uint32_t kmax = (uint32_t)km;
    if (kmax != b->kmax || !b->vl) {
      void* old[] = {b->vl, b->ysl, b->vl_cnt, b->xb, b->tb, b->pb, b->dmax};
      for (void* q : old)
        if (q) (void)hipFree(q);
      b->vl = nullptr;
      b->ysl = nullptr;
      b->vl_cnt = nullptr;
      b->xb = b->tb = nullptr;
      b->pb = nullptr;
      b->dmax = nullptr;
      b->kmax = 0;
      BCHK(b, dalloc(&b->vl, (size_t)kmax * b->nslots));
      BCHK(b, dalloc(&b->ysl, b->nslots));
      BCHK(b, dalloc(&b->vl_cnt, b->nslots));
      BCHK(b, dalloc(&b->xb, 3 * b->ntot));
      BCHK(b, dalloc(&b->tb, (size_t)R));
      BCHK(b, dalloc(&b->pb, 2 * (size_t)R));
      BCHK(b, dalloc(&b->dmax, (size_t)R));
      b->kmax = kmax;
    }
    if (!b->wrap) BCHK(b, dalloc(&b->wrap, b->nslots));
  }
  BCHK(b, hipMemcpy(b->pol, pol.data(), pol.size() * sizeof(RemapPolicy), hipMemcpyHostToDevice));
  BCHK(b, hipMemcpy(b->t0_d, t, (size_t)R * sizeof(double), hipMemcpyHostToDevice));
  BCHK(b, hipMemcpy(b->adiag, ad.data(), ad.size() * sizeof(double), hipMemcpyHostToDevice));
  b->t0.assign(t, t + R);
  b->variant = variant;
  b->have_lattice = true;
  b->built = false;
  return NCL_OK;
}

int ncl_batch_build_cells(ncl_batch_handle b, const double* x, int precision, int debug) {
  if (!b || !x) return NCL_E_ARG;
  if (!b->have_lattice) return bfail(b, NCL_E_STATE, "no lattices set");
  if (precision < NCL_PREC_FP64 || precision > NCL_PREC_FP32_KAHAN) return bfail(b, NCL_E_ARG, "bad precision");
  BCHK(b, hipSetDevice(b->device));
  if (debug && !b->wrap) BCHK(b, dalloc(&b->wrap, b->nslots));
  b->precision = precision;
  b->debug = debug ? 1 : 0;
  b->x = x;
  // The fused schedule bins inside the force pass, and the autotuner's first
  // force pass builds again: both read a copy of the positions taken here,
  // so the caller's array is read only by this call, as with the staged
  // build.  Debug builds are staged.
  const bool fused = !debug && sched_mode(b) == NCL_SWEEP_FUSED;
  const bool tuning = !debug && b->sweep_mode == SWEEP_AUTO && !tuned_entry(b);
  if (fused || tuning) {
    if (!b->xcopy) BCHK(b, dalloc(&b->xcopy, 3 * b->ntot));
    BCHK(b, batch_copy(b->xcopy, x, 3 * b->ntot, b->stream));
    b->x = b->xcopy;
  }
  BatchDev D = view(b);
  BCHK(b, batch_prologue(D, 0, 0.0, b->stream));
  b->pending = fused;
  if (!b->pending) BCHK(b, batch_build(D, x, b->stream));
  b->built = true;
  return NCL_OK;
}

int ncl_batch_compute_forces(ncl_batch_handle b, void* F, double* U, double* W) {
  if (!b || !F || !U || !W) return NCL_E_ARG;
  if (!b->built) return bfail(b, NCL_E_STATE, "ncl_batch_build_cells must precede ncl_batch_compute_forces");
  BCHK(b, hipSetDevice(b->device));
  SweepArgs A;
  sweep_args(b, &A, F);
  const BatchDev D = view(b);
  if (b->pending) {
    BCHK(b, batch_fused(A, D, b->x, b->precision, b->fstate, b->order, b->blk_order, U, W, b->stream));
    b->pending = false;
    b->used_mode = NCL_SWEEP_FUSED;
    return NCL_OK;
  }
  if (b->sweep_mode == SWEEP_AUTO && !b->debug && !tuned_entry(b)) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    BCHK(b, hipStreamIsCapturing(b->stream, &cap));
    if (cap == hipStreamCaptureStatusNone) return tune(b, A, U, W);
  }
  BCHK(b, batch_sweep(A, D, b->precision, false, U, W, b->stream));
  b->used_mode = SWEEP_PARTICLE;
  return NCL_OK;
}

int ncl_batch_debug_pairs(ncl_batch_handle b, int64_t* count, uint64_t* hash) {
  if (!b || !count || !hash) return NCL_E_ARG;
  if (!b->built || !b->debug) return bfail(b, NCL_E_STATE, "ncl_batch_build_cells(..., debug=1) must come first");
  BCHK(b, hipSetDevice(b->device));
  if (!b->dbgF) BCHK(b, dalloc(&b->dbgF, 3 * b->ntot + 10 * (size_t)b->nrep + 16));
  SweepArgs A;
  sweep_args(b, &A, b->dbgF);
  A.dbg_count = count;
  A.dbg_hash = hash;
  BCHK(b, batch_sweep(A, view(b), b->precision, true, b->dbgF + 3 * b->ntot, b->dbgF + 3 * b->ntot + b->nrep,
                      b->stream));
  return NCL_OK;
}

int ncl_batch_get_stats(ncl_batch_handle b, ncl_stats* out) {
  if (!b || !out) return NCL_E_ARG;
  BCHK(b, hipSetDevice(b->device));
  if (b->built && b->pending) {
    // fused schedule, force pass not run yet: build the cells now
    BCHK(b, batch_build(view(b), b->x, b->stream));
    b->pending = false;
  }
  if (b->built && b->cstart) BCHK(b, launch_max_occupancy(b->cstart, b->ncells, b->small + 8, b->stream));
  uint32_t w[16];
  BCHK(b, hipMemcpyAsync(w, b->small, sizeof w, hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  memset(out, 0, sizeof *out);
  const unsigned long long* s = (const unsigned long long*)w;
  out->n = (int64_t)b->ntot;
  out->variant = b->variant;
  out->precision = b->precision;
  out->ncells = (int64_t)b->ncells;
  out->candidates = (int64_t)s[0];
  out->pairs = (int64_t)s[1];
  out->fp64_pairs = (int64_t)s[2];
  out->neighbourhood = (int64_t)s[3];
  out->list_rebuilds = b->rebuilds;
  out->sweep = b->used_mode;
  for (int k = 0; k < 5; ++k) out->tune_ms[k] = -1.0f;
  if (const ncl_batch::Tuned* t = tuned_entry(b))
    for (int k = 0; k < 2; ++k) out->tune_ms[k] = t->ms[k];
  out->max_occupancy = (int32_t)w[8];
  if (w[9]) {
    const int code = (int)w[9];
    const uint32_t z = 0;
    BCHK(b, hipMemcpyAsync(b->small + 9, &z, 4, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    if (code & 2) return bfail(b, NCL_E_BOX_TOO_SMALL, "a replica's box became too small for the cut-off");
    if (code & 8) return bfail(b, NCL_E_CAPACITY, "a replica exceeded its cell capacity");
    return bfail(b, NCL_E_DEVICE_FLAG, "a kernel flagged a non-finite position or a singular lattice");
  }
  return NCL_OK;
}

int ncl_batch_get_lattices(ncl_batch_handle b, double* Lred, int32_t* cells) {
  if (!b) return NCL_E_ARG;
  if (!b->built) return bfail(b, NCL_E_STATE, "nothing built yet");
  BCHK(b, hipSetDevice(b->device));
  std::vector<CellGeom> g(b->nrep);
  std::vector<double> L(9 * (size_t)b->nrep);
  BCHK(b, hipMemcpyAsync(g.data(), b->geom, g.size() * sizeof(CellGeom), hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipMemcpyAsync(L.data(), b->lred, L.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  for (int r = 0; r < b->nrep; ++r) {
    if (cells)
      for (int k = 0; k < 3; ++k) cells[3 * r + k] = g[r].nc[k];
    if (Lred)
      for (int k = 0; k < 9; ++k) Lred[9 * r + k] = L[9 * r + k];
  }
  return NCL_OK;
}

// SLLOD steps of every replica, each step's second kick done with the next
// step's first kick and drift in one pass.  Step n from the forces of step
// n - 1: lattice at t_n, [second kick of n - 1,] first kick and drift,
// [observables of n - 1 and the step count,] cells, forces of step n.  The
// first step of a run has no pending second kick; the steps after it are
// all alike (the sequence a graph captures, lattice offset 2 since the
// step count then lags one step behind); the run ends with the last step's
// second kick and observables.
static hipError_t sllod_step(ncl_batch* b, const BatchDev& D, const SweepArgs& A, double* x, double* p, void* F,
                             double* U, double* W, double h, double mass, double* hist, uint32_t hist_cap,
                             bool first, hipStream_t st) {
  const bool f64 = b->precision == NCL_PREC_FP64;
  hipError_t e;
  if ((e = batch_prologue(D, first ? 1 : 2, h, st)) != hipSuccess) return e;
  if ((e = batch_kick_drift(D, x, p, F, f64, h, mass, !first, st)) != hipSuccess) return e;
  if (!first && (e = batch_observe(D, U, W, h, hist, hist_cap, true, st)) != hipSuccess) return e;
  if ((e = batch_build(D, x, st)) != hipSuccess) return e;
  return batch_sweep(A, D, b->precision, false, U, W, st);
}

static hipError_t sllod_finish(ncl_batch* b, const BatchDev& D, double* p, void* F, double* U, double* W, double h,
                               double mass, double* hist, uint32_t hist_cap, hipStream_t st) {
  hipError_t e = batch_kick(D, p, F, b->precision == NCL_PREC_FP64, h, mass, 1, st);
  if (e == hipSuccess) e = batch_observe(D, U, W, h, hist, hist_cap, true, st);
  return e;
}

// SLLOD with neighbour lists (skin > 0): each step checks on the device
// whether the lists still cover every pair within d_cut (skin bound and no
// remap since the last rebuild), reads that one flag on the host and
// rebuilds only when needed; positions stay unwrapped between rebuilds and
// are put back into the reduced box at the end
static int sllod_run_lists(ncl_batch* b, const BatchDev& D, const SweepArgs& A, double* x, double* p, void* F,
                           double* U, double* W, double h, double mass, int64_t nsteps, double* hist,
                           uint32_t hist_cap, hipStream_t st) {
  const bool f64 = b->precision == NCL_PREC_FP64;
  uint32_t* need_h = nullptr;
  BCHK(b, hipHostMalloc((void**)&need_h, sizeof(uint32_t), hipHostMallocDefault));
  auto read_need = [&](uint32_t* out) -> hipError_t {
    hipError_t e = hipMemcpyAsync(need_h, D.need, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    *out = *need_h;
    return e;
  };
  int code = NCL_OK;
  hipError_t e = hipSuccess;
  uint32_t need = 0;
  b->rebuilds = 0;
  auto rebuild = [&](int off) -> int {
    if ((e = hipMemsetAsync(D.need, 0, sizeof(uint32_t), st)) != hipSuccess) return bhip(b, e, "flag");
    if ((e = batch_list_rebuild(D, x, off, h, st)) != hipSuccess) return bhip(b, e, "list rebuild");
    if ((e = read_need(&need)) != hipSuccess) return bhip(b, e, "list rebuild");
    if (need & 4u) return bfail(b, NCL_E_CAPACITY, "a particle has more neighbours than the lists hold");
    ++b->rebuilds;
    return NCL_OK;
  };
  if (e == hipSuccess) e = batch_prologue(D, 0, h, st);
  if (e == hipSuccess) code = rebuild(0);
  if (e == hipSuccess && code == NCL_OK) e = batch_list_force(A, D, b->precision, U, W, st);
  if (e == hipSuccess && code == NCL_OK) e = batch_kick(D, p, F, f64, 0.0, mass, 1, st);
  if (e == hipSuccess && code == NCL_OK) e = batch_observe(D, U, W, h, hist, hist_cap, false, st);
  for (int64_t k = 0; k < nsteps && e == hipSuccess && code == NCL_OK; ++k) {
    if ((e = batch_kick(D, p, F, f64, h, mass, 0, st)) != hipSuccess) break;
    if ((e = batch_prologue(D, 1, h, st)) != hipSuccess) break;
    if ((e = batch_drift(D, x, p, h, mass, st)) != hipSuccess) break;
    if ((e = hipMemsetAsync(D.need, 0, sizeof(uint32_t), st)) != hipSuccess) break;
    if ((e = batch_list_check(D, x, 1, h, b->skin, st)) != hipSuccess) break;
    if ((e = read_need(&need)) != hipSuccess) break;
    if (need && (code = rebuild(1)) != NCL_OK) break;
    if ((e = batch_list_force(A, D, b->precision, U, W, st)) != hipSuccess) break;
    if ((e = batch_kick(D, p, F, f64, h, mass, 1, st)) != hipSuccess) break;
    e = batch_observe(D, U, W, h, hist, hist_cap, true, st);
  }
  // positions back into the reduced box, and cells that match them
  if (e == hipSuccess && code == NCL_OK && D.n > 0) e = batch_wrap(D, x, st);
  if (e == hipSuccess && code == NCL_OK) e = batch_build(D, x, st);
  const hipError_t se = hipStreamSynchronize(st);
  (void)hipHostFree(need_h);
  if (code != NCL_OK) return code;
  if (e != hipSuccess) return bhip(b, e, "sllod with neighbour lists");
  if (se != hipSuccess) return bhip(b, se, "sllod with neighbour lists");
  return NCL_OK;
}

int ncl_batch_sllod_run(ncl_batch_handle b, double* x, double* p, void* F, double* U, double* W, double h,
                        double mass, int64_t nsteps, int use_graph, double* hist) {
  if (!b || !x || !p || !F || !U || !W) return NCL_E_ARG;
  if (!(h > 0.0) || !(mass > 0.0) || nsteps < 0) return bfail(b, NCL_E_ARG, "need h > 0, mass > 0, nsteps >= 0");
  if (!b->have_lattice) return bfail(b, NCL_E_STATE, "no lattices set");
  if (b->debug) return bfail(b, NCL_E_STATE, "rebuild without debug before stepping");
  BCHK(b, hipSetDevice(b->device));
  const uint32_t hist_cap = hist ? (uint32_t)std::min<int64_t>(nsteps + 1, 0x7fffffff) : 0;
  hipStream_t st = b->own;
  // order the private stream after the caller's work
  BCHK(b, hipEventRecord(b->ev_in, b->stream));
  BCHK(b, hipStreamWaitEvent(st, b->ev_in, 0));
  BatchDev D = view(b);
  SweepArgs A;
  sweep_args(b, &A, F);
  const bool f64 = b->precision == NCL_PREC_FP64;
  // step counter to zero, forces and observables at the starting time
  BCHK(b, hipMemsetAsync(b->small + 10, 0, 4, st));
  if (b->skin > 0.0) {
    const int code = sllod_run_lists(b, D, A, x, p, F, U, W, h, mass, nsteps, hist, hist_cap, st);
    if (code != NCL_OK) {
      // steps may have run: x and p are then advanced by an unknown number
      // of steps (x unwrapped), and the lattices and cells no longer match
      // them, so the batch needs ncl_batch_set_lattices again
      b->built = false;
      b->have_lattice = false;
      return code;
    }
  } else {
  BCHK(b, batch_prologue(D, 0, h, st));
  BCHK(b, batch_build(D, x, st));
  BCHK(b, batch_sweep(A, D, b->precision, false, U, W, st));
  BCHK(b, batch_kick(D, p, F, f64, 0.0, mass, 1, st));  // p unchanged; kinetic sums
  BCHK(b, batch_observe(D, U, W, h, hist, hist_cap, false, st));
  if (nsteps > 0) BCHK(b, sllod_step(b, D, A, x, p, F, U, W, h, mass, hist, hist_cap, true, st));
  if (use_graph && nsteps > 1) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BCHK(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t ce = sllod_step(b, D, A, x, p, F, U, W, h, mass, hist, hist_cap, false, st);
    hipError_t ee = hipStreamEndCapture(st, &graph);
    if (ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return bhip(b, ce, "sllod step capture");
    }
    if (ee != hipSuccess) return bhip(b, ee, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return bhip(b, ie, "hipGraphInstantiate");
    }
    hipError_t le = hipSuccess;
    for (int64_t k = 1; k < nsteps && le == hipSuccess; ++k) le = hipGraphLaunch(exec, st);
    hipError_t se = hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (le != hipSuccess) return bhip(b, le, "hipGraphLaunch");
    if (se != hipSuccess) return bhip(b, se, "graph replay");
  } else {
    for (int64_t k = 1; k < nsteps; ++k)
      BCHK(b, sllod_step(b, D, A, x, p, F, U, W, h, mass, hist, hist_cap, false, st));
  }
  if (nsteps > 0) BCHK(b, sllod_finish(b, D, p, F, U, W, h, mass, hist, hist_cap, st));
  }
  // the caller's stream continues after the run
  BCHK(b, hipEventRecord(b->ev_out, st));
  BCHK(b, hipStreamWaitEvent(b->stream, b->ev_out, 0));
  // the batch now sits at t0 + nsteps h
  for (int r = 0; r < b->nrep; ++r) b->t0[r] += (double)nsteps * h;
  BCHK(b, hipMemcpyAsync(b->t0_d, b->t0.data(), b->t0.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemsetAsync(b->small + 10, 0, 4, b->stream));
  b->built = true;
  b->pending = false;
  return NCL_OK;
}

const char* ncl_batch_last_error(ncl_batch_handle b) { return b ? b->err.c_str() : "null handle"; }

}  // extern "C"
