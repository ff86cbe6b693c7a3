// Internal declarations of the batched (multi-scenario) sweep.
#pragma once
#include "mrsdc_internal.h"

namespace mrsdc {

constexpr int kMaxS = 64;  // scenarios per batch = lanes of a wavefront

// Shared operators of the batch, row-major: each row lists its K entries and
// then its nonzero R entries (the Robin rows), at most 64 in all, so one
// coalesced load fetches a row.  Entries address LDS-staged rows: tiles of TR
// consecutive rows; the union of the columns of a tile's rows is copied into
// at most kStageSlots LDS rows; slot_row[t][sl] = global row staged in slot
// sl of tile t, slot[e] = slot of entry e's column within its row's tile.
struct BatchOp {
  int64_t N = 0;
  const int64_t *rowptr = nullptr;  // [N+1] over the merged entries, by tile position
  const int *nk = nullptr;          // [N] K entries of the row (the rest are R)
  const double *val = nullptr;      // entry values
  const float *val32 = nullptr;     // FP32 copy (FP32 form)
  const int *slot32 = nullptr;      // entry -> LDS slot within the row's tile
  const uint16_t *oslot = nullptr;  // [N] slot of the row itself within its tile
  int TR = 0, ntiles = 0;
  const int *nslots = nullptr;    // [ntiles]
  const int *slot_row = nullptr;  // [ntiles][kStageSlots]
  // rows in tile order: tile t holds positions [tstart[t], tstart[t+1]);
  // rowptr, nk and oslot are indexed by position, prow[pos] is the row
  const int64_t *tstart = nullptr;  // [ntiles + 1]
  const int64_t *prow = nullptr;    // [N]
  const double *pmass = nullptr;    // [N] lumped mass of row prow[pos]
  // Column sweep (every body a box of the 27-point pattern): FP64 records,
  // and FP32 ones in FP32 contexts.  Work items are footprints of kColFX x
  // kColFY nodes of one body over a run of z planes.  Each plane of an item
  // has one record of its footprint rows' K stencils (kColRows rows of
  // kStencil values, row r = node (x0 + r % kColFX, y0 + r / kColFX)): value
  // k is the entry of neighbour k = (dz+1) 9 + (dy+1) 3 + (dx+1), 0 where
  // there is none, and value 27 is the row's lumped mass, negated when the
  // row has an R stencil (rows outside the body are all zeros).  Rows with R
  // entries or a boundary load g have an R stencil: the planes where some
  // row has one also have one record of the rows' R stencils (same layout,
  // value 27 the row's g).
  int ncol_items = 0;
  // [ncol_items][kColItem]: row offset, nx, ny, nz, x0, y0, z0, z1, first K
  // record, first R record, R plane mask (bit z - z0; two words)
  const int *col_items = nullptr;
  const float *kcol32 = nullptr;   // [K records][kColRows][kStencil], then the R records:
  const float *rcol32 = nullptr;   // [R records][kColRows][kStencil] (same buffer)
  const double *kcol64 = nullptr;  // the same in FP64
  const double *rcol64 = nullptr;
  int64_t col_rec_bytes32 = 0, col_rec_bytes64 = 0;  // bytes of both, per form
};
constexpr int kColFX = 4, kColFY = 4;                // footprint of a column item
constexpr int kColZeroRow = 64;  // zeros after the direction p and the node states
constexpr int kColRows = kColFX * kColFY;            // rows of a plane of an item
constexpr int kColPL = (kColFX + 2) * (kColFY + 2);  // staged rows per plane (halo included)
constexpr int kColDepth = 2;                         // stages in flight beyond the one read
constexpr int kColItem = 12;                         // ints per work item
constexpr int kStencil = 28;                         // 27 neighbours + the mass
constexpr int kMaxR = 8;  // tiles hold at most 4 kMaxR rows

// Staging buffer of the tiled kernels: 64 KB per workgroup (two workgroups
// fit in one CU's LDS), rows of up to 64 FP64 scenario values.
constexpr int kStageBytes = 65536;
constexpr int kStageSlots = (kStageBytes / 8 - 64) / 64;  // 127, with a 64-value tail
constexpr int kMaxTileEntries = 1024;                      // matrix entries of a tile
constexpr int kBatchMaxGrid = 1024;  // workgroups of the batched kernels (a multiple of 8)

// Per-scenario solver scalars (index s fastest).  In the FP32 form, tol2 and
// done belong to the inner FP32 solve and ref_* to the FP64 refinement around
// it; the FP64 form never sets ref_done.
struct BatchScalars {
  double rz[2][kMaxS];
  double tol2[kMaxS];
  double alpha[kMaxS];
  double beta[kMaxS];
  double ref_tol2[kMaxS];
  double resid[17][kMaxS];
  int active[kMaxS];
  int done[kMaxS];
  int done_it[kMaxS];             // iteration whose check found the solve converged (-1: none)
  int ref_done[kMaxS];
  int fail[kMaxS];
  int stop[kMaxS];                // residual control: no further sweeps this step
  int sweeps[kMaxS];              // sweeps run when stop was set
  long long iters_total[kMaxS];   // CG iterations of the step (inner ones in FP32)
  long long refine_total[kMaxS];  // refinement rounds of the step
  int slot_iters[kSlots][kMaxS];  // FP64: iterations (-1 budget hit); FP32: largest inner count
  int slot_rounds[kSlots][kMaxS]; // FP32: refinement rounds (-1: not converged)
};

// One implicit node solve of the batch.
struct BSolve {
  int m = 0;
  bool pred = false;
  int slot = 0;
  int budget = 0;  // CG launches (inner CG launches per round in FP32)
  int rounds = 0;  // refinement rounds (FP32)
  double rtol = 0.0, refine_rtol = 0.0, inner_rtol = 0.0;
};

struct BatchArgs {
  int S = 0, M = 0, P = 0, grid = 0;
  int sgrid64 = 0, sgrid32 = 0;  // workgroups of the tiled kernels (FP64 / FP32 staging)
  int cgrid = 0;    // workgroups of the column-sweep CG operator (0: tiles)
  int cgrid_f = 0;  // of the FP64 column sweep of F (0: tiles)
  int bgrid64 = 0, bgrid32 = 0;  // workgroups of the CG update (b): all resident
  // launch variants (every one gives the same results): stages in flight of
  // the column sweep (1 or kColDepth), row groups in flight of the CG
  // updates (b: 2 or 4, c: 4 or 8)
  int col_depth = kColDepth, groups_b = 4, groups_c = 4;
  int64_t N = 0;
  double dtau_h[kMaxM + 1] = {};
  BatchOp op;
  const double *mass = nullptr, *Kd = nullptr, *Rd = nullptr, *gbase = nullptr;
  const double *h = nullptr, *alpha = nullptr, *Pf = nullptr, *period = nullptr;  // [S]
  double *tn = nullptr;                                                           // [S]
  const Weights *w = nullptr;
  const int *ifpos = nullptr;
  IfaceDev f;
  double *T[kMaxM + 1] = {};
  double *F[kMaxM + 1] = {};
  double *I[kMaxM + 1] = {};
  double *r = nullptr, *p = nullptr, *q = nullptr;  // FP64 form
  // FP32 form: inner CG vectors and the FP64 refinement residual
  float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
  double *r64 = nullptr;
  int fp32 = 0;
  double sweep_tol = 0.0;  // > 0: residual-controlled sweeps, per scenario
  double *partial = nullptr;  // [3][pgrid][S]: per-workgroup partial sums
  int pgrid = 0;              // workgroups whose three partial sums the buffer holds
  BatchScalars *sc = nullptr;
  double *Eold = nullptr, *Enew = nullptr;  // [(M+1)(P+1)][n_if][S]
  double *Tbuf[2] = {};                     // [n_if][S]
  double *fst = nullptr;                    // [n_if][S]
  double *coefD = nullptr;                  // [(M+1)(P+1)][dstride][S]
  int *coefI = nullptr;
  int n_if = 0;
};

void blaunch_clear(const BatchArgs &a, hipStream_t st);
void blaunch_iface_coeffs(const BatchArgs &a, hipStream_t st);
void blaunch_f_multi(const BatchArgs &a, int j0, int j1, hipStream_t st);
void blaunch_quad_resid(const BatchArgs &a, int k, hipStream_t st);
void blaunch_solve(const BatchArgs &a, const BSolve &sv, hipStream_t st);
void blaunch_iface(const BatchArgs &a, int m, bool corr, hipStream_t st);
void blaunch_operator_timing(const BatchArgs &a, int m, int reps, hipStream_t st);
// For the autotuner: reps launches of the column-sweep or tiled operator
// (which 0, timing variant; either form), the FP32 update (b) (1) or the FP32
// update (c) (2) with the launch variants in a; b and c overwrite only inner
// CG vectors
void blaunch_tune(const BatchArgs &a, int which, int reps, hipStream_t st);
void blaunch_commit(const BatchArgs &a, double dt, hipStream_t st);
void blaunch_scatter(double *dst, const double *src, int64_t n, int S, int s, hipStream_t st);
void blaunch_gather(double *dst, const double *src, int64_t n, int S, int s, hipStream_t st);
// workgroups of the column-sweep operator resident per CU (set by its LDS
// ring) in the FP32 (fp32 = 1) or FP64 form with depth stages in flight
int col_workgroups_per_cu(int fp32, int depth);
// bgrid64 / bgrid32 from the occupancy of the update kernels (device current)
void set_resident_grids(BatchArgs &a);

}  // namespace mrsdc
