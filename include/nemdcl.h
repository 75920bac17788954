/*
 * nemdcl -- short-range pair forces in a deforming periodic box on AMD MI355X
 * (gfx950), with the dynamic-size and dynamic-offset cell lists of Dobson,
 * Fox & Saracino, "Cell List Algorithms for Nonequilibrium Molecular
 * Dynamics" (arXiv:1412.3784).
 *
 * Problem (Sec. 2): a lattice with basis L = [v1 v2 v3] (columns), images
 * q + L n of every particle, a homogeneous flow u = A x that deforms the
 * lattice as L_t = exp(tA) L0 (Sec. 2.1), remapped by integer matrices of
 * determinant one (Sec. 2.2).  Pairs interact through a Lennard-Jones form
 * truncated at d_cut (zero beyond it, Sec. 3).  The library bins particles
 * into the cells of the dynamic-size list (cells congruent to the box, Sec.
 * 4.1) or of the dynamic-offset list (rectangular cells of the rotated box,
 * Sec. 4.2) and sweeps each cell's neighbourhood on the GPU.
 *
 * Conventions for every entry point
 *   - 3x3 matrices are row-major double[9]; a basis has the basis vectors as
 *     its COLUMNS, so M[3*r + c] is component r of vector c.
 *   - Positions are N x 3 row-major FP64 in DEVICE memory; forces are N x 3
 *     row-major in DEVICE memory, FP64 for NCL_PREC_FP64 and FP32 otherwise,
 *     in the caller's particle order.  U and W are DEVICE pointers.
 *   - The caller owns every buffer it passes.  The handle owns its scratch
 *     (cell arrays, sorted particle copies, partial sums), allocated by
 *     ncl_build_cells only when N or the cell count exceeds what it holds.
 *   - All GPU work is enqueued on the handle's stream; calls return without
 *     waiting unless stated.  One handle per stream; handles are independent.
 *   - Every call returns NCL_OK (0) or a negative NCL_E_* code; the text of
 *     the last error is available from ncl_last_error.  No exceptions cross
 *     this interface.
 */
#ifndef NEMDCL_H
#define NEMDCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NCL_OK 0
#define NCL_E_ARG (-1)           /* null pointer, bad enum, n < 0, ...            */
#define NCL_E_BOX_TOO_SMALL (-2) /* some cell count c_i or l_i is below 1         */
#define NCL_E_LATTICE (-3)       /* automorphism not unimodular / not diagonalised
                                    by L0, or flow incompatible with the remap    */
#define NCL_E_CAPACITY (-4)      /* a size exceeds a fixed limit of the library   */
#define NCL_E_HIP (-5)           /* a HIP runtime call failed                      */
#define NCL_E_DEVICE_FLAG (-6)   /* a kernel raised its error word (e.g. a
                                    non-finite position); reported by the next
                                    synchronising call                             */
#define NCL_E_STATE (-7)         /* calls out of order (e.g. forces before cells)  */

/* cell-list variant (Sec. 4.1 and 4.2) */
#define NCL_DYNAMIC_SIZE 0
#define NCL_DYNAMIC_OFFSET 1

/* arithmetic of the pair sweep.
 * FP64:        positions, distances, forces and sums in FP64.
 * FP32:        FP32 offsets of each particle from its FP64 cell centre, FP32
 *              pair maths and per-particle FP32 sums; the pair maths take
 *              r^2 rounded once from the FP64 screen of the separation (not
 *              recomputed from its FP32 components, whose rounding the WCA
 *              force near d_cut would magnify).  Pairs whose r^2 lies
 *              within the rounding band of d_cut^2 are re-decided from FP64
 *              positions exactly as in FP64 mode, so the interacting set
 *              equals the FP64 one; pairs closer than a close-pair radius
 *              take their separation and pair terms in FP64 (the force is
 *              then added to the FP32 sums, the energy to an FP64 sum).
 * FP32_KAHAN:  as FP32, with Kahan-compensated per-particle force sums (the
 *              per-particle sweep compensates once per evaluation round of
 *              at most ten pairs summed in FP32, the other schedules once
 *              per pair).                                                   */
#define NCL_PREC_FP64 0
#define NCL_PREC_FP32 1
#define NCL_PREC_FP32_KAHAN 2

/* options for ncl_set_option */
#define NCL_OPT_DO_TIGHT 0       /* 1: dynamic-offset neighbourhood grown by d_cut
                                    instead of one cell width (default 1)         */
#define NCL_OPT_CLOSE_RADIUS 1   /* FP32 modes: pairs with r below this (in sigma)
                                    are evaluated in FP64 (default 0.45)          */
#define NCL_OPT_BAND 2           /* FP32 modes: relative half-width of the r^2 band
                                    re-decided in FP64 (default 1e-5)             */
#define NCL_OPT_SWEEP 3          /* sweep kernel: 0 = LDS-tiled bricks of cells,
                                    1 = one thread per particle, 2 = autotuned
                                    (default): the first force pass of each
                                    workload class (variant, precision, cells per
                                    axis, occupancy) times the per-particle sweep
                                    and the tiled sweep with its three best-ranked
                                    bricks (and, when NCL_OPT_DETERMINISTIC is 0,
                                    the half list) on the handle's stream,
                                    synchronising once, and keeps the fastest;
                                    3 = half list: each pair evaluated once and
                                    applied to both particles with atomic sums
                                    (NCL_PREC_FP32 only; forces are then not
                                    bit-identical from run to run).
                                    Batches: 1 = staged launches (lattice
                                    prologue, cell build, per-particle sweep);
                                    4 = one persistent fused bin + force launch
                                    after the prologue: workgroups take one
                                    replica's whole cell build each, then sweep
                                    blocks whose replica is built; 2 = autotuned
                                    (default): the first force pass of each
                                    variant and precision times both and keeps
                                    the faster (the staged schedule only, when
                                    a replica holds more than 131,072
                                    particles).  The fused schedule (and the
                                    autotuner) copies the positions at
                                    ncl_batch_build_cells, which stays the only
                                    call that reads the caller's array          */
#define NCL_SWEEP_FUSED 4        /* batch sweep schedule, see NCL_OPT_SWEEP      */
#define NCL_OPT_SKIN 5           /* batches only: skin (in length units, default 0)
                                    of the neighbour lists that
                                    ncl_batch_sllod_run reuses between rebuilds;
                                    0 rebuilds cells every step.  Set before
                                    ncl_batch_set_lattices                        */
#define NCL_OPT_DETERMINISTIC 4  /* 1 (default): the autotuner only picks
                                    schedules whose forces are bit-identical from
                                    run to run; 0: it may pick the half list.
                                    Set sweep options before ncl_build_cells,
                                    which sizes the half list's FP64 force array
                                    (24 bytes per particle)                       */

typedef struct ncl_ctx *ncl_handle;

typedef struct {
    int64_t n;              /* particles binned                                   */
    int32_t variant;        /* NCL_DYNAMIC_SIZE / NCL_DYNAMIC_OFFSET              */
    int32_t precision;      /* NCL_PREC_*                                         */
    int32_t cells[3];       /* c_i (Sec. 4.1) or l_i (Sec. 4.2)                   */
    int32_t max_occupancy;  /* most particles in one cell                         */
    int64_t ncells;
    int64_t candidates;     /* distance checks, each ordered (i, j-image) once
                               (half list: each unordered pair once)           */
    int64_t pairs;          /* in-range ordered pairs: twice the interacting set  */
    int64_t fp64_pairs;     /* FP32 modes: pairs re-evaluated in FP64 (ordered;
                               half list: unordered)                           */
    int64_t neighbourhood;  /* sum over particles of neighbourhood cells visited   */
    int32_t sweep;          /* schedule of the last force pass: 0 tiled, 1 per
                               particle, 3 half list                           */
    int32_t brick[3];       /* its brick of cells when tiled                      */
    float tune_ms[5];       /* autotuner timings of this workload class: per
                               particle, tiled with the three best-ranked
                               bricks, half list (-1: not timed)               */
    int64_t list_rebuilds;  /* batches: neighbour-list builds of the last
                               ncl_batch_sllod_run with a skin (0 otherwise)   */
} ncl_stats;

/* Create a handle on HIP device `device` that enqueues on `stream` (a
 * hipStream_t owned by the caller; NULL means the default stream). */
int ncl_create(ncl_handle *out, int device, void *stream);

/* Free the handle and its scratch (synchronises its stream). */
int ncl_destroy(ncl_handle h);

/* Pair potential phi(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] - shift for
 * r < rc and 0 beyond (Sec. 3: forces identically zero past the cut-off);
 * shift = phi_LJ(rc) if shift_energy != 0, else 0.  WCA (Sec. 5) is
 * rc = 2^(1/6) sigma with shift_energy = 1.  Forces are not shifted. */
int ncl_set_potential(ncl_handle h, double eps, double sigma, double rc, int shift_energy);

int ncl_set_option(ncl_handle h, int option, double value);

/* Lattice at strain time t (host pointers).  L_t = exp(tA) L0 (Sec. 2.1).
 * A is either diagonal (elongational flows) or a planar shear with A^2 = 0
 * (Sec. 2.2), for which L_t = (I + tA) L0; other flows return NCL_E_LATTICE.
 * naut = 0: no remap, the basis is L_t.
 * Diagonal A, naut = 1 (Kraynik-Reinelt, eq:kr) or 2 (generalised KR,
 * Sec. 2.2): `aut` holds M1 (and M2) as int32[9] row-major, each of
 * determinant 1 and such that L0 M_k L0^-1 is diagonal with positive entries
 * exp(mu_k); t diag(A) must lie in the span of the mu_k.  The stretch
 * t diag(A) = sum_k alpha_k mu_k is reduced to eps = t diag(A) -
 * sum_k p_k mu_k with p_k = floor(alpha_k + 1/2), and the basis used is
 * Lred = exp(diag(eps)) L0 = L_t M1^-p1 M2^-p2.
 * Shear A, naut = 1 (Lees-Edwards, eq:Mshear): M = I - N with N^2 = 0 and
 * L0^-1 A L0 = s N; M is applied each time the box has been sheared by half
 * a lattice spacing: Lred = L_t M^p = L0 (I + (s t - p) N), p = floor(s t +
 * 1/2).  Host-side FP64; no GPU work. */
int ncl_set_lattice(ncl_handle h, const double L0[9], const double A[9], double t, int naut,
                    const int32_t *aut);

/* The basis in use and the integer matrix with Lred = L_t Mtot (host
 * pointers; any may be NULL).  coef receives (p1, p2). */
int ncl_get_lattice(ncl_handle h, double Lred[9], int32_t Mtot[9], int32_t coef[2]);

/* Cell counts the current lattice gives for a variant: c_i = floor(h_i/d_cut)
 * with h_i the box heights (Sec. 4.1), or l_i = floor(r_ii/d_cut) with R from
 * the QR decomposition Lred = Q R (Sec. 4.2, 5.2).  Host only. */
int ncl_cell_counts(ncl_handle h, int variant, int32_t counts[3]);

/* Bin the n positions x (device, N x 3 FP64, any image) into the cells of
 * `variant` for the current lattice (Sec. 4.1: every step, from the current
 * box): wrap into the box, assign cells, counting-sort, and write the sorted
 * copies the sweep reads (FP64 wrapped positions, FP32 offsets from the FP64
 * cell centres, cell ids, the permutation).  Within a cell the order is by
 * particle index, so results are run-to-run deterministic.  `x` must stay
 * valid until ncl_compute_forces has run.  debug != 0 also keeps each
 * particle's wrap vector for ncl_debug_pairs.  n == 0 is allowed. */
int ncl_build_cells(ncl_handle h, int variant, const double *x, int64_t n, int precision, int debug);

/* Sweep every cell's neighbourhood (27 cells, Sec. 4.1; 27/30/34/36 cells,
 * Sec. 4.2) and write F (device, N x 3, FP64 or FP32 per precision, input
 * order), U = sum over interacting pairs of phi (device double[1]) and
 * W = sum over interacting pairs of r_ij (x) f_ij (device double[9],
 * row-major, r_ij = x_i - image of x_j, f_ij the force on i from j). */
int ncl_compute_forces(ncl_handle h, void *F, double *U, double *W);

/* Per-particle pair-set digest (test aid, device int64[N] and uint64[N], input
 * order): count_i = number of neighbour images (j, m) of i within d_cut and
 * hash_i = sum of SplitMix64(key(j, Mtot m)) over them, m being the image in
 * the basis Lred relative to the positions as given, so keys refer to the
 * unreduced basis L_t.  Requires ncl_build_cells(..., debug=1). */
int ncl_debug_pairs(ncl_handle h, int64_t *count, uint64_t *hash);

/* Copy the statistics of the last build / force pass (synchronises the
 * stream; reports NCL_E_DEVICE_FLAG if a kernel raised its error word). */
int ncl_get_stats(ncl_handle h, ncl_stats *out);

/* Text of the last error on this handle ("" if none). */
const char *ncl_last_error(ncl_handle h);

/* ------------------------------------------------------------------------ */
/* Batched form: R independent boxes ("replicas") of uneven size, each with */
/* its own basis, diagonal traceless flow, automorphisms and strain time,   */
/* sharing one potential and one cell-list variant.  Every kernel covers all */
/* replicas in one launch; each replica's lattice at its current time is    */
/* computed on the GPU in FP64 (Sec. 2.1-2.2).  Arrays are concatenated in  */
/* replica order: positions, momenta and forces are (sum_r n_r) x 3; U is   */
/* double[R] and W double[R*9] on the device.  Per-replica cell storage is  */
/* sized once from floor(V_r / d_cut^3) + 1, which bounds the cell count of */
/* both variants at any strain (Sec. 4.1 heights, Sec. 5.2 counts), so no   */
/* call after ncl_batch_set_lattices allocates.                              */
/* ------------------------------------------------------------------------ */
typedef struct ncl_batch *ncl_batch_handle;

/* nrep replicas of n[r] >= 1 particles (host array). */
int ncl_batch_create(ncl_batch_handle *out, int device, void *stream, int32_t nrep, const int64_t *n);
int ncl_batch_destroy(ncl_batch_handle b);
/* As ncl_set_potential; call before ncl_batch_set_lattices. */
int ncl_batch_set_potential(ncl_batch_handle b, double eps, double sigma, double rc, int shift_energy);
/* NCL_OPT_DO_TIGHT, NCL_OPT_CLOSE_RADIUS, NCL_OPT_SWEEP (1, 2 or 4) and
 * NCL_OPT_SKIN. */
int ncl_batch_set_option(ncl_batch_handle b, int option, double value);
/* Per replica r (host arrays): L0 + 9r, A + 9r (diagonal, traceless), strain
 * time t[r], naut[r] automorphisms at aut + 18r (as in ncl_set_lattice). */
int ncl_batch_set_lattices(ncl_batch_handle b, int variant, const double *L0, const double *A, const double *t,
                           const int32_t *naut, const int32_t *aut);
/* Lattices at the current times, then the cell build of every replica. */
int ncl_batch_build_cells(ncl_batch_handle b, const double *x, int precision, int debug);
/* Forces (FP64 or FP32 per precision), U[r], W[r*9] of every replica. */
int ncl_batch_compute_forces(ncl_batch_handle b, void *F, double *U, double *W);
/* Per-particle pair digest as ncl_debug_pairs, with j the index within the
 * replica (device int64[sum n] and uint64[sum n], concatenated input order);
 * requires debug = 1 at build. */
int ncl_batch_debug_pairs(ncl_batch_handle b, int64_t *count, uint64_t *hash);
/* Aggregate statistics (synchronises). */
int ncl_batch_get_stats(ncl_batch_handle b, ncl_stats *out);
/* Reduced bases (host double[R*9], may be NULL) and cell counts (host
 * int32[R*3], may be NULL) in use (synchronises). */
int ncl_batch_get_lattices(ncl_batch_handle b, double *Lred, int32_t *cells);
/* nsteps SLLOD steps of every replica with peculiar momenta p (device,
 * FP64): dq/dt = p/m + A q, dp/dt = F - A p, split symmetrically per step
 * (half kick with stretch, drift, rebuild and forces, half kick), positions
 * x (device, FP64) put back into the reduced box after every drift.  F (FP32
 * or FP64 per the build precision), U and W hold the final forces.  With
 * use_graph != 0 one step is captured as a HIP graph and replayed for all
 * steps but the first (a step's second half kick is done in one pass with
 * the next step's first half kick and drift, so the first step and the last
 * half kick run outside the graph).  hist (device, may be NULL) receives (nsteps + 1) x R records of 8
 * doubles: t, U, W_xx, W_yy, W_zz, K_xx, K_yy, K_zz with K = sum p p^T / m.
 * Afterwards the replicas' strain times have advanced by nsteps h.
 * With NCL_OPT_SKIN = s > 0, forces come from neighbour lists within
 * d_cut + s, rebuilt only when a step could break them: between rebuilds at
 * t_b and t (no remap) the lattice is E L(t_b), E = exp(A (t - t_b)), and
 * positions E x(t_b) + delta, so the lists hold every pair within d_cut as
 * long as max_k exp(-a_k (t - t_b)) (d_cut + 2 max|delta|) < d_cut + s; each
 * step checks that (and remaps) on the device and reads one flag on the host,
 * so steps are not graph-replayed; positions stay unwrapped between rebuilds
 * and are put back into the reduced box at the end.  NCL_E_CAPACITY if a
 * particle has more neighbours than the lists hold (1.5 times the mean of the
 * densest replica plus 24, rounded up to a multiple of 4).  After any error
 * of a run with a skin, x and p may have advanced by an unknown number of
 * steps (x possibly unwrapped): the batch forgets its lattices and cells,
 * and every later call except ncl_batch_set_lattices returns NCL_E_STATE. */
int ncl_batch_sllod_run(ncl_batch_handle b, double *x, double *p, void *F, double *U, double *W, double h,
                        double mass, int64_t nsteps, int use_graph, double *hist);
const char *ncl_batch_last_error(ncl_batch_handle b);

/* ---- entry point that allocates nothing ----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One call
 * does what ncl_set_lattice + ncl_build_cells + ncl_compute_forces do with the
 * per-particle sweep (NCL_OPT_SWEEP = 1) and the default options, for a box
 * of at most NCL_NOALLOC_MAX_N particles whose cell list has at most
 * NCL_NOALLOC_MAX_CELLS cells; its results are those of that sequence, bit
 * for bit.  Every scratch array lives in one file-scope device array of the
 * library (8 MiB per device, held until the process ends); the call makes
 * no hipMalloc, hipFree or allocating library call and synchronises nothing,
 * so it can be captured into a graph.
 *   device, stream  HIP device and stream (hipStream_t) to enqueue on
 *   L0, A, t, naut, aut  as ncl_set_lattice
 *   pot             eps, sigma, r_c, shift flag (as ncl_set_potential)
 *   variant, precision, x, n  as ncl_build_cells (no debug digests)
 *   F, U, W         as ncl_compute_forces (device, caller-owned)
 * Returns NCL_E_CAPACITY when n or the cell count exceeds its maximum (nothing
 * is enqueued), NCL_E_ARG / NCL_E_LATTICE / NCL_E_BOX_TOO_SMALL as the calls it
 * replaces.  A non-finite position sets *U to NaN (there is no handle to
 * report it through).  All calls on one device share its array and leave
 * their contents there: calls that overlap on one device (two streams, or
 * threads) race and must be ordered by the caller. */
#define NCL_NOALLOC_MAX_N 65536
#define NCL_NOALLOC_MAX_CELLS 65536
int ncl_forces_noalloc(int device, void *stream, const double L0[9], const double A[9], double t, int naut,
                       const int32_t *aut, const double pot[4], int variant, int precision, const double *x,
                       int64_t n, void *F, double *U, double *W);

#ifdef __cplusplus
}
#endif
#endif /* NEMDCL_H */
