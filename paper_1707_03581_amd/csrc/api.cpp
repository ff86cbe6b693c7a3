// C-ABI of the MRSDC library and the host-side driver of the time step.
//
// Per time step [t_n, t_n + dt] (paper §3, Alg. 1 then K times Alg. 2):
//   predictor, for each interval m:  init solve (one SpMV) -> CG -> interface
//                                    substeps (f^E at the embedded nodes)
//   sweep k = 1..K:  F_j = f^I(T_j) + g at all standard nodes (one multi-RHS
//                    SpMV), I_{m-1}^m and the residual (one fused pass), then
//                    for each interval m: init (no SpMV) -> CG -> substeps
//   commit T_{n+1} = T_M on the device, unless a solve ran out of budget.
// Every kernel of a step is enqueued without host round trips; the host reads
// a small counter block once per step.  CG iterations are launched in a
// per-solve budget taken from the previous step; kernels of a converged solve
// return at once.  A solve that exhausts its budget makes the step uncommitted
// and the step is repeated with doubled budgets, up to pcg_maxit (ENOCONV).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <queue>
#include <unordered_map>
#include <vector>

#include "batch_internal.h"
#include "deform_internal.h"
#include "mrsdc_internal.h"

using namespace mrsdc;

namespace {

struct HostBody {
  bool set = false;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> K, R, mass, rload;
  double h = 0.0, Tenv = 0.0;
  std::vector<double> T;
  bool hasT = false;
};

struct HostFace {
  bool set = false;
  int nu = 0, nv = 0;
  std::vector<double> u, v;
  std::vector<int32_t> ids;
};

struct Coupling {
  int kind = 0;  // 0 none, 1 contact, 2 patch
  int fix_body = 0, fix_face = 0, mov_body = 1, mov_face = 0;
  double du = 0, dv = 0, alpha = 0, Pf = 0, split = 0.5;
  int body = 0, face = 0;
  double wu = 0, wv = 0, uc = 0, q0 = 0, Tfix = 0;
};

struct Motion {
  double s0 = 0, a = 0, period = 1, phase = 0;
};

}  // namespace

struct mrsdc_ctx {
  mrsdc_config cfg;
  mrsdc_allocator allocator = {};  // copy of cfg.alloc (cfg.alloc points here when set)
  std::string err;
  HostBody body[2];
  HostFace face[2][8];
  Coupling cpl;
  Motion motion;
  double t = 0.0;
  bool prepared = false;
  bool dirty_T = true;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void *> allocs;
  int64_t footprint = 0;
  int64_t scen_bytes = 0;  // part of footprint that grows with the scenario count
  DevState d;
  Weights w;
  int nbody = 0;
  int64_t off[3] = {0, 0, 0};
  StepCounters *ctr_host = nullptr;  // pinned
  int budget[kSlots];   // CG launch budget per solve slot (inner CG for FP32_REFINE)
  int last_it[kSlots];      // the slot's iteration count one step earlier
  int last_rounds[kSlots];  // FP32: the slot's refinement rounds one step earlier
  int expect[kSlots];   // iterations the slot took in the last step
  int rounds[kSlots];   // refinement round budget per slot
  int64_t matrix_bytes = 0;
  int64_t nnz = 0;
  int64_t batch_entries = 0;  // merged K and R entries of a batched operator
  int64_t col_stored_bytes = 0;  // stencil records and work items of the column sweep
  // captured time step (use_graph): valid for the budgets in graph_key
  hipGraphExec_t graph_exec = nullptr;
  std::vector<int> graph_key;
  bool graph_off = false;
  int64_t graph_captures = 0, graph_replays = 0;
  int graph_warm = 0;  // steps run directly (to learn the budgets) before the first capture
  bool tuned = false;  // autotune: launch variants chosen for this device state
  int op_form_used = 0;       // MRSDC_OP_* the CG product reads (single contexts)
  int col_bytes = 0;          // 2: 16-bit column offsets, 4: int32 columns
  // event timing of kernel classes
  bool prof = false;
  std::vector<hipEvent_t> ev;   // pairs
  std::vector<int> ev_class;    // 0 cg spmv, 1 iface
  int ev_used = 0;
  mrsdc_kernel_times times = {};
  // batched contexts: S > 0 scenarios sharing the operators
  int S = 0;
  std::vector<double> sc_h, sc_alpha, sc_Pf, sc_period, sc_t;
  std::vector<int> sc_active;
  // a scenario joined since the last step: its solves may need more than the
  // budgets learned from the others, so the next step widens them
  bool batch_joined = false;
  std::vector<std::vector<double>> sc_T;  // pending host temperatures (empty: none)
  BatchArgs ba;
  BatchScalars *bsc_host = nullptr;       // pinned
  double *stage = nullptr;                // device staging vector [N]
  // thermo-elastic deformation of one body (independent of the stepper's
  // device state: kept when the operators change)
  DeformDev df;
  bool df_ready = false;
  int df_body = 0;
  int64_t df_nodes = 0;
  std::vector<void *> df_allocs;
  int64_t df_bytes = 0;
  double df_factor_ms = 0.0;
  int64_t df_dispatches = 0;  // kernels the factorisation launched
};

namespace {

mrsdc_status fail(mrsdc_ctx *c, mrsdc_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
mrsdc_status fail(mrsdc_ctx *c, mrsdc_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(c, MRSDC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// per_scenario: the allocation grows with the batch's scenario count (its
// bytes are counted apart for admission by footprint)
// Device memory of a context: through the caller's allocator when one was
// given, else hipMalloc / hipFree.
void *dev_malloc(mrsdc_ctx *c, size_t bytes) {
  if (c->cfg.alloc) return c->allocator.alloc(bytes, (void *)c->stream, c->allocator.user);
  void *q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    hipGetLastError();
    return nullptr;
  }
  return q;
}
void dev_free(mrsdc_ctx *c, void *p) {
  if (!p) return;
  if (c->cfg.alloc) c->allocator.release(p, (void *)c->stream, c->allocator.user);
  else hipFree(p);
}

template <typename T>
mrsdc_status dalloc(mrsdc_ctx *c, T **p, size_t count, bool per_scenario = false) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void *q = dev_malloc(c, bytes);
  if (!q) return fail(c, MRSDC_ENOMEM, "device allocation of %zu bytes failed", bytes);
  c->allocs.push_back(q);
  c->footprint += (int64_t)bytes;
  if (per_scenario) c->scen_bytes += (int64_t)bytes;
  *p = static_cast<T *>(q);
  return MRSDC_OK;
}

template <typename T>
mrsdc_status upload(mrsdc_ctx *c, T **p, const std::vector<T> &h, bool per_scenario = false) {
  mrsdc_status s = dalloc(c, p, h.size(), per_scenario);
  if (s) return s;
  if (!h.empty()) HIPCHK(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return MRSDC_OK;
}

void free_device(mrsdc_ctx *c) {
  // keep the device-resident temperature and time when the operators change
  if (c->prepared && c->S > 0) {
    if (c->stream) hipStreamSynchronize(c->stream);
    const int64_t N = c->ba.N;
    for (int s = 0; s < c->S; ++s) {
      if (!c->sc_T[s].empty()) continue;  // a newer host value is pending
      std::vector<double> col(N);
      blaunch_gather(c->stage, c->d.T[0], N, c->S, s, c->stream);
      hipMemcpyAsync(col.data(), c->stage, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream);
      hipStreamSynchronize(c->stream);
      c->sc_T[s] = std::move(col);
    }
  } else if (c->prepared && !c->dirty_T) {
    if (c->stream) hipStreamSynchronize(c->stream);
    for (int b = 0; b < c->nbody; ++b) {
      if (!c->body[b].set || !c->body[b].hasT) continue;
      c->body[b].T.resize(c->body[b].n);
      hipMemcpy(c->body[b].T.data(), c->d.T[0] + c->off[b], sizeof(double) * c->body[b].n,
                hipMemcpyDeviceToHost);
    }
    c->dirty_T = true;
  }
  // a captured step refers to the buffers freed below
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  c->graph_exec = nullptr;
  c->graph_key.clear();
  c->graph_warm = 0;
  c->tuned = false;
  for (void *p : c->allocs) dev_free(c, p);
  c->allocs.clear();
  c->footprint = 0;
  c->scen_bytes = 0;
  c->prepared = false;
}

bool valid_scheme(const mrsdc_config *cfg) {
  if (cfg->M < 1 || cfg->M > kMaxM || cfg->P < 1 || cfg->P > kMaxP) return false;
  if (cfg->M < 2 && cfg->node_family == MRSDC_LOBATTO) return false;
  if (cfg->method != MRSDC_MULTIRATE && cfg->method != MRSDC_SINGLE_RATE) return false;
  if (cfg->method == MRSDC_SINGLE_RATE && cfg->precision != MRSDC_FP64) return false;
  if (cfg->K < 0 || cfg->K > 16 || !(cfg->dt > 0) || !std::isfinite(cfg->dt)) return false;
  if (cfg->node_family != MRSDC_LOBATTO && cfg->node_family != MRSDC_EQUI_NOLEFT) return false;
  if ((cfg->op_form & ~(0xff | MRSDC_OP_COL32)) != 0 || (cfg->op_form & 0xff) > MRSDC_OP_PATTERNS)
    return false;
  if (cfg->precision != MRSDC_FP64 && cfg->precision != MRSDC_FP32_REFINE) return false;
  if (!(cfg->pcg_rtol > 0) || cfg->pcg_maxit < 1) return false;
  if (!(cfg->sweep_tol >= 0) || !std::isfinite(cfg->sweep_tol)) return false;
  if (cfg->precision == MRSDC_FP32_REFINE &&
      (!(cfg->refine_rtol > 0) || cfg->refine_maxit < 1 || !(cfg->inner_rtol > 0)))
    return false;
  return true;
}

// first node c of grid y (shifted by sy) whose hat support ends after t
int first_hat_after_h(const std::vector<double> &y, double sy, double t) {
  const int n = (int)y.size();
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    double end = y[mid < n - 1 ? mid + 1 : mid] + sy;
    if (end > t) hi = mid; else lo = mid + 1;
  }
  return lo;
}

double min_spacing(const std::vector<double> &x) {
  double m = INFINITY;
  for (size_t i = 1; i < x.size(); ++i) m = std::min(m, x[i] - x[i - 1]);
  return m;
}
double max_support(const std::vector<double> &x) {
  double m = 0;
  const int n = (int)x.size();
  for (int a = 0; a < n; ++a) m = std::max(m, x[a < n - 1 ? a + 1 : a] - x[a > 0 ? a - 1 : a]);
  return m;
}

// Band of hats of y overlapping each hat of x along one (static) direction.
mrsdc_status band_coeffs(mrsdc_ctx *c, const std::vector<double> &x, const std::vector<double> &y,
                         double lo, double hi, std::vector<double> &C, std::vector<int> &lo_idx,
                         std::vector<int> &cnt) {
  const int nx = (int)x.size(), ny = (int)y.size();
  C.assign((size_t)nx * kBand, 0.0);
  lo_idx.assign(nx, 0);
  cnt.assign(nx, 0);
  for (int a = 0; a < nx; ++a) {
    double start = x[a > 0 ? a - 1 : a], end = x[a < nx - 1 ? a + 1 : a];
    int c0 = first_hat_after_h(y, 0.0, start);
    lo_idx[a] = c0;
    for (int i = 0; i < kBand; ++i) {
      int cc = c0 + i;
      if (cc >= ny) break;
      C[(size_t)kBand * a + i] =
          hat_product_integral(x.data(), nx, a, y.data(), ny, cc, 0.0, lo, hi);
      if (C[(size_t)kBand * a + i] != 0.0) cnt[a] = i + 1;
    }
    int cn = c0 + kBand;
    if (cn < ny && y[cn > 0 ? cn - 1 : cn] < end)
      return fail(c, MRSDC_EINVAL, "face grids too dissimilar: more than %d coupled nodes", kBand);
  }
  return MRSDC_OK;
}

// Batched contexts: shared operators in row-major form (one row per
// wavefront), per-scenario parameters, and the argument block of the batch
// kernels over the scenario-interleaved vectors allocated by prepare().
// Tiles for the LDS-staged operator: the largest TR (rows per tile) whose
// every tile has at most kStageSlots distinct columns over its entries (K
// and R).  The tiling depends on the mesh only (not on S or precision), so a
// scenario's arithmetic is the same in any batch.  col: global column of
// every merged entry.
// Grid dimensions of a body whose pattern is the 27-point stencil of an
// nx x ny x nz node grid numbered x fastest (the box bodies), else false.
bool box_dims(const HostBody &B, int64_t dims[3]) {
  if (B.n < 8 || B.rowptr[1] - B.rowptr[0] != 8) return false;
  const int64_t nx = B.col[B.rowptr[0] + 2], nxy = B.col[B.rowptr[0] + 4];
  if (nx < 2 || nxy % nx != 0 || B.n % nxy != 0) return false;
  const int64_t ny = nxy / nx, nz = B.n / nxy;
  if (ny < 2 || nz < 2) return false;
  for (int64_t i = 0; i < B.n; ++i) {
    const int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    int64_t e = B.rowptr[i];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t x = ix + dx, y = iy + dy, z = iz + dz;
          if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) continue;
          if (e >= B.rowptr[i + 1] || B.col[e] != x + nx * (y + ny * z)) return false;
          ++e;
        }
    if (e != B.rowptr[i + 1]) return false;
  }
  dims[0] = nx;
  dims[1] = ny;
  dims[2] = nz;
  return true;
}

// Tiles of the staged products and the operator stored in tile order.  On
// box bodies a tile is a block of up to 3 x 3 x 3 nodes: its column union is
// at most 5 x 5 x 5 = 125 rows for 27 rows (about 4.6 staged rows per row,
// against 10.5 for a run of 12 consecutive rows); otherwise tiles are runs of
// consecutive rows.  rowptr / col / val / nk are by row; the device gets them
// by tile position (row prow[pos]), tile t holding positions
// [tstart[t], tstart[t+1]).
mrsdc_status build_stage_tiles(mrsdc_ctx *c, int64_t N, const std::vector<int64_t> &rowptr,
                               const std::vector<int64_t> &col, const std::vector<double> &val,
                               const std::vector<int> &nk, BatchArgs &a) {
  std::vector<int64_t> order, tstart;
  // block tiling when every body is a box
  bool blocks = true;
  for (int b = 0; b < c->nbody && blocks; ++b) {
    int64_t dm[3];
    if (!box_dims(c->body[b], dm)) {
      blocks = false;
      break;
    }
    for (int64_t bz = 0; bz < dm[2]; bz += 3)
      for (int64_t by = 0; by < dm[1]; by += 3)
        for (int64_t bx = 0; bx < dm[0]; bx += 3) {
          tstart.push_back((int64_t)order.size());
          for (int64_t z = bz; z < std::min(bz + 3, dm[2]); ++z)
            for (int64_t y = by; y < std::min(by + 3, dm[1]); ++y)
              for (int64_t x = bx; x < std::min(bx + 3, dm[0]); ++x)
                order.push_back(c->off[b] + x + dm[0] * (y + dm[1] * z));
        }
  }
  static const int kTry[] = {32, 24, 16, 12, 10, 8, 6, 4, 3, 2, 1};  // at most 4 kMaxR rows
  std::vector<int64_t> cols;
  for (int attempt = blocks ? -1 : 0; attempt < (int)(sizeof kTry / sizeof kTry[0]); ++attempt) {
    if (attempt >= 0) {  // runs of consecutive rows
      const int TR = kTry[attempt];
      order.resize(N);
      for (int64_t r = 0; r < N; ++r) order[r] = r;
      tstart.clear();
      for (int64_t r = 0; r < N; r += TR) tstart.push_back(r);
    }
    if (tstart.empty() || tstart.back() != N) tstart.push_back(N);
    const int64_t T = (int64_t)tstart.size() - 1;
    std::vector<int> nslots(T, 0), slot_row((size_t)T * kStageSlots, 0);
    std::vector<int64_t> prp(N + 1, 0);
    std::vector<int> pnk(N), slot;
    std::vector<uint16_t> oslot(N);
    std::vector<double> pval, pmass(N), rmass(N);
    for (int b = 0; b < c->nbody; ++b)
      for (int64_t i = 0; i < c->body[b].n; ++i) rmass[c->off[b] + i] = c->body[b].mass[i];
    slot.reserve(col.size());
    pval.reserve(col.size());
    bool fits = true;
    for (int64_t t = 0; t < T && fits; ++t) {
      if (tstart[t + 1] - tstart[t] > 4 * kMaxR) fits = false;
      cols.clear();
      int64_t ne = 0;
      for (int64_t q = tstart[t]; q < tstart[t + 1]; ++q) {
        const int64_t r = order[q];
        ne += rowptr[r + 1] - rowptr[r];
        cols.insert(cols.end(), col.begin() + rowptr[r], col.begin() + rowptr[r + 1]);
      }
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      if (ne > kMaxTileEntries || (int64_t)cols.size() > kStageSlots) {
        fits = false;
        break;
      }
      nslots[t] = (int)cols.size();
      for (size_t k = 0; k < cols.size(); ++k) slot_row[(size_t)t * kStageSlots + k] = (int)cols[k];
      for (int64_t q = tstart[t]; q < tstart[t + 1]; ++q) {
        const int64_t r = order[q];
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          slot.push_back((int)(std::lower_bound(cols.begin(), cols.end(), col[e]) - cols.begin()));
          pval.push_back(val[e]);
        }
        prp[q + 1] = (int64_t)slot.size();
        pnk[q] = nk[r];
        pmass[q] = rmass[r];
        const auto it = std::lower_bound(cols.begin(), cols.end(), r);
        if (it == cols.end() || *it != r)
          return fail(c, MRSDC_EINVAL, "row %lld has no diagonal entry", (long long)r);
        oslot[q] = (uint16_t)(it - cols.begin());
      }
    }
    if (!fits) continue;
    mrsdc_status st;
    int *pi;
    int64_t *pl;
    uint16_t *pu;
    double *pv;
    if ((st = upload(c, &pl, prp))) return st;
    a.op.rowptr = pl;
    if ((st = upload(c, &pi, pnk))) return st;
    a.op.nk = pi;
    if ((st = upload(c, &pv, pval))) return st;
    a.op.val = pv;
    if (c->cfg.precision == MRSDC_FP32_REFINE) {
      std::vector<float> v32(pval.begin(), pval.end());
      float *pf32;
      if ((st = upload(c, &pf32, v32))) return st;
      a.op.val32 = pf32;
    }
    if ((st = upload(c, &pi, nslots))) return st;
    a.op.nslots = pi;
    if ((st = upload(c, &pi, slot_row))) return st;
    a.op.slot_row = pi;
    if ((st = upload(c, &pi, slot))) return st;
    a.op.slot32 = pi;
    if ((st = upload(c, &pu, oslot))) return st;
    a.op.oslot = pu;
    if ((st = upload(c, &pl, tstart))) return st;
    a.op.tstart = pl;
    if ((st = upload(c, &pl, order))) return st;
    a.op.prow = pl;
    if ((st = upload(c, &pv, pmass))) return st;
    a.op.pmass = pv;
    a.op.TR = attempt >= 0 ? kTry[attempt] : 0;  // 0: node blocks
    a.op.ntiles = (int)T;
    c->batch_entries = (int64_t)slot.size();
    // every workgroup resident: two FP64 or three FP32 staging buffers per CU
    // on 256 CUs
    a.sgrid64 = (int)std::min<int64_t>((T + 7) / 8 * 8, 512);
    a.sgrid32 = (int)std::min<int64_t>((T + 7) / 8 * 8, 768);
    return MRSDC_OK;
  }
  return fail(c, MRSDC_EINVAL, "a row block exceeds the staging capacity of %d columns", kStageSlots);
}

// Column sweeps when every body is a box of the 27-point pattern: work items
// of kColFX x kColFY nodes of one body over a run of z planes, and per item
// plane a record of the footprint rows' K stencils (value k = entry of
// neighbour (dz+1) 9 + (dy+1) 3 + (dx+1); value 27 = the row's mass,
// negated where the row has an R stencil) plus, for the planes where a row
// has one (R entries or a boundary load g), a record of their R stencils
// (value 27 = g).  Items run body by body, then by z run, then by footprint
// row and column, so neighbouring footprints (which share halo rows) are
// dealt to the same XCD and run side by side.  The CG operator sweeps in
// the context's form (cgrid; FP32 records in FP32 contexts), F = h g - L T
// in FP64 (cgrid_f; FP64 records); an FP64 sweep takes each item as two work
// units (the two halves of the scenarios).
// Leaves cgrid = cgrid_f = 0 (tiles only) for any other mesh and where the
// context asks for the stored values (MRSDC_OP_VALUES), and either one at 0
// where its vectors hold 2 GB or more.
mrsdc_status build_columns(mrsdc_ctx *c, int64_t N, const std::vector<double> &gbase,
                           BatchArgs &a) {
  if (c->cfg.op_form == MRSDC_OP_VALUES) return MRSDC_OK;  // stored values: tiles
  const bool fp32 = c->cfg.precision == MRSDC_FP32_REFINE;
  const int64_t vb = fp32 ? 4 : 8, units = fp32 ? 1 : 2;
  const bool cg = (N * c->S + kColZeroRow) * vb < ((int64_t)1 << 31);
  const bool fsweep = (N * c->S + kColZeroRow) * 8 < ((int64_t)1 << 31);
  if (!cg && !fsweep) return MRSDC_OK;
  int64_t dm[2][3];
  for (int b = 0; b < c->nbody; ++b)
    if (!box_dims(c->body[b], dm[b])) return MRSDC_OK;
  // per-row stencils in natural row order
  std::vector<double> ks((size_t)N * kStencil, 0.0), rs;
  std::vector<int> ridx(N, -1);
  std::vector<double> mass(N);
  int64_t colplanes = 0;
  for (int b = 0; b < c->nbody; ++b) {
    const HostBody &B = c->body[b];
    const int64_t nx = dm[b][0], ny = dm[b][1];
    colplanes += ((dm[b][0] + kColFX - 1) / kColFX) * ((dm[b][1] + kColFY - 1) / kColFY) * dm[b][2];
    for (int64_t i = 0; i < B.n; ++i) {
      const int64_t row = c->off[b] + i;
      const int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
      mass[row] = B.mass[i];
      bool hasR = false;
      for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e) {
        const int64_t j = B.col[e];
        const int64_t jx = j % nx, jy = (j / nx) % ny, jz = j / (nx * ny);
        const int k = (int)((jz - iz + 1) * 9 + (jy - iy + 1) * 3 + (jx - ix + 1));
        ks[(size_t)row * kStencil + k] = B.K[e];
        hasR |= !B.R.empty() && B.R[e] != 0.0;
      }
      if (!hasR && gbase[row] == 0.0) continue;
      ridx[row] = (int)(rs.size() / kStencil);
      rs.resize(rs.size() + kStencil, 0.0);
      double *r = rs.data() + rs.size() - kStencil;
      r[27] = gbase[row];
      for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e) {
        const int64_t j = B.col[e];
        const int64_t jx = j % nx, jy = (j / nx) % ny, jz = j / (nx * ny);
        r[(jz - iz + 1) * 9 + (jy - iy + 1) * 3 + (jx - ix + 1)] = B.R[e];
      }
    }
  }
  // Run length: the one (8 .. 64 planes) with the shortest simulated
  // makespan when XCD x deals its eighth of the items, in order, to its
  // resident workgroups as they come free, an item costing its planes plus
  // the steps that fill its pipeline (for the CG operator's sweep, else F's).
  const bool sim32 = fp32 && cg;
  const int64_t slots =
      std::max<int64_t>(1, 256 * (int64_t)col_workgroups_per_cu(sim32, a.col_depth) / 8);
  auto makespan = [&](int64_t zr) {
    std::vector<int64_t> cost;
    for (int b = 0; b < c->nbody; ++b) {
      const int64_t fp = ((dm[b][0] + kColFX - 1) / kColFX) * ((dm[b][1] + kColFY - 1) / kColFY);
      for (int64_t z0 = 0; z0 < dm[b][2]; z0 += zr)
        cost.insert(cost.end(), fp * (sim32 ? 1 : 2),
                    std::min(dm[b][2], z0 + zr) - z0 + 3 + a.col_depth);
    }
    const int64_t T = (int64_t)cost.size();
    int64_t worst = 0;
    for (int x = 0; x < 8; ++x) {
      std::priority_queue<int64_t, std::vector<int64_t>, std::greater<int64_t>> free_at;
      for (int64_t i = 0; i < slots; ++i) free_at.push(0);
      for (int64_t t = T * x / 8; t < T * (x + 1) / 8; ++t) {
        const int64_t s0 = free_at.top();
        free_at.pop();
        free_at.push(s0 + cost[t]);
        worst = std::max(worst, s0 + cost[t]);
      }
    }
    return worst;
  };
  int64_t zrun = 64, best = makespan(64);
  for (int64_t zr = 63; zr >= 8; --zr) {
    const int64_t ms = makespan(zr);
    if (ms < best) best = ms, zrun = zr;
  }
  std::vector<int> items;
  std::vector<double> krec, rrec;
  const size_t rec = (size_t)kColRows * kStencil;
  for (int b = 0; b < c->nbody; ++b)
    for (int64_t z0 = 0; z0 < dm[b][2]; z0 += zrun)
      for (int64_t y0 = 0; y0 < dm[b][1]; y0 += kColFY)
        for (int64_t x0 = 0; x0 < dm[b][0]; x0 += kColFX) {
          const int64_t z1 = std::min(dm[b][2], z0 + zrun);
          const int kb = (int)(krec.size() / rec), rb = (int)(rrec.size() / rec);
          uint64_t mask = 0;
          for (int64_t z = z0; z < z1; ++z) {
            krec.resize(krec.size() + rec, 0.0);
            double *kr = krec.data() + krec.size() - rec;
            std::vector<double> rr(rec, 0.0);
            bool anyR = false;
            for (int r = 0; r < kColRows; ++r) {
              const int64_t gx = x0 + r % kColFX, gy = y0 + r / kColFX;
              if (gx >= dm[b][0] || gy >= dm[b][1]) continue;  // outside the body: zeros
              const int64_t row = c->off[b] + gx + dm[b][0] * (gy + dm[b][1] * z);
              for (int k = 0; k < 27; ++k) kr[r * kStencil + k] = ks[(size_t)row * kStencil + k];
              const bool hasR = ridx[row] >= 0;
              kr[r * kStencil + 27] = hasR ? -mass[row] : mass[row];
              if (!hasR) continue;
              anyR = true;
              for (int k = 0; k < kStencil; ++k)
                rr[r * kStencil + k] = rs[(size_t)ridx[row] * kStencil + k];
            }
            if (anyR) {
              mask |= 1ull << (z - z0);
              rrec.insert(rrec.end(), rr.begin(), rr.end());
            }
          }
          const int it[kColItem] = {(int)c->off[b], (int)dm[b][0], (int)dm[b][1], (int)dm[b][2],
                                    (int)x0, (int)y0, (int)z0, (int)z1, kb, rb,
                                    (int)(uint32_t)mask, (int)(uint32_t)(mask >> 32)};
          items.insert(items.end(), it, it + kColItem);
        }
  c->col_stored_bytes = cg ? (int64_t)(krec.size() + rrec.size()) * vb + (int64_t)items.size() * 4 : 0;
  if (rrec.empty()) rrec.assign(rec, 0.0);
  mrsdc_status st;
  int *pi;
  if ((st = upload(c, &pi, items))) return st;
  a.op.col_items = pi;
  a.op.ncol_items = (int)(items.size() / kColItem);
  // K records then R records in one buffer (one buffer resource in the kernel)
  const size_t nk = krec.size();
  krec.insert(krec.end(), rrec.begin(), rrec.end());
  if (krec.size() * 8 >= ((size_t)1 << 31))
    return fail(c, MRSDC_EINVAL, "column records above 2 GB");
  if (fp32 && cg) {
    float *pf;
    if ((st = upload(c, &pf, std::vector<float>(krec.begin(), krec.end())))) return st;
    a.op.kcol32 = pf;
    a.op.rcol32 = pf + nk;
    a.op.col_rec_bytes32 = (int64_t)krec.size() * 4;
  }
  double *pd;
  if ((st = upload(c, &pd, krec))) return st;
  a.op.kcol64 = pd;
  a.op.rcol64 = pd + nk;
  a.op.col_rec_bytes64 = (int64_t)krec.size() * 8;
  // one workgroup per work unit: the dispatcher balances them over the CUs
  const int64_t nit = a.op.ncol_items;
  a.cgrid = cg ? (int)((nit * units + 7) / 8 * 8 + 8) : 0;
  a.cgrid_f = fsweep ? (int)((nit * 2 + 7) / 8 * 8 + 8) : 0;
  return MRSDC_OK;
}

mrsdc_status prepare_batch(mrsdc_ctx *c, int64_t N) {
  DevState &d = c->d;
  const int S = c->S;
  mrsdc_status st;
  // merged rows: the row's K entries, then its nonzero R entries (nk[row] = K
  // count); columns stay on the host (the device addresses staged slots)
  std::vector<int64_t> rowptr(N + 1, 0), col;
  std::vector<int> nk(N, 0);
  std::vector<double> val, Kd(N, 0.0), Rd(N, 0.0), gbase(N, 0.0);
  for (int b = 0; b < c->nbody; ++b) {
    const HostBody &B = c->body[b];
    for (int64_t i = 0; i < B.n; ++i) {
      const int64_t row = c->off[b] + i, base = c->off[b];
      gbase[row] = B.Tenv * (B.rload.empty() ? 0.0 : B.rload[i]);
      for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e) {
        if (B.col[e] == i) {
          Kd[row] += B.K[e];
          if (!B.R.empty()) Rd[row] += B.R[e];
        } else if (B.K[e] == 0.0) {
          continue;  // stored zero (e.g. face neighbours on cubic cells): no arithmetic
        }
        col.push_back(base + B.col[e]);
        val.push_back(B.K[e]);
      }
      nk[row] = (int)(col.size() - rowptr[row]);
      if (!B.R.empty())
        for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e) {
          if (B.R[e] == 0.0) continue;
          col.push_back(base + B.col[e]);
          val.push_back(B.R[e]);
        }
      rowptr[row + 1] = (int64_t)col.size();
      if (rowptr[row + 1] - rowptr[row] > 64)
        return fail(c, MRSDC_EINVAL, "batched contexts need at most 64 K and R entries per row");
    }
  }
  BatchArgs &a = c->ba;
  a = BatchArgs();
  a.S = S;
  a.N = N;
  a.M = c->cfg.M;
  a.P = c->cfg.P;
  a.sweep_tol = c->cfg.sweep_tol;
  // blocks of 4 rows, a multiple of the 8 XCDs
  a.grid = (int)std::min<int64_t>(((N + 3) / 4 + 7) / 8 * 8, kBatchMaxGrid);
  set_resident_grids(a);
  for (int m = 0; m <= c->cfg.M; ++m) a.dtau_h[m] = c->w.dtau[m];
  double *pv;
  a.op.N = N;
  if ((st = build_stage_tiles(c, N, rowptr, col, val, nk, a))) return st;
  if ((st = build_columns(c, N, gbase, a))) return st;
  if ((st = upload(c, &pv, Kd))) return st;
  a.Kd = pv;
  if ((st = upload(c, &pv, Rd))) return st;
  a.Rd = pv;
  if ((st = upload(c, &pv, gbase))) return st;
  a.gbase = pv;
  a.mass = d.mass;
  // per-scenario parameters (unset ones take the context-wide values)
  std::vector<double> h(S), al(S), pf(S), per(S), t(S);
  std::vector<int> act(S);
  for (int s = 0; s < S; ++s) {
    h[s] = std::isnan(c->sc_h[s]) ? c->body[0].h : c->sc_h[s];
    al[s] = std::isnan(c->sc_alpha[s]) ? c->cpl.alpha : c->sc_alpha[s];
    pf[s] = std::isnan(c->sc_Pf[s]) ? c->cpl.Pf : c->sc_Pf[s];
    per[s] = std::isnan(c->sc_period[s]) ? c->motion.period : c->sc_period[s];
    t[s] = c->sc_t[s];
    act[s] = c->sc_active[s];
  }
  if ((st = upload(c, &pv, h, true))) return st;
  a.h = pv;
  if ((st = upload(c, &pv, al, true))) return st;
  a.alpha = pv;
  if ((st = upload(c, &pv, pf, true))) return st;
  a.Pf = pv;
  if ((st = upload(c, &pv, per, true))) return st;
  a.period = pv;
  if ((st = upload(c, &pv, t, true))) return st;
  a.tn = pv;
  if ((st = dalloc(c, &a.sc, 1))) return st;
  HIPCHK(hipMemset(a.sc, 0, sizeof(BatchScalars)));
  HIPCHK(hipMemcpy(a.sc->active, act.data(), sizeof(int) * S, hipMemcpyHostToDevice));
  // partial sums: up to three per scenario from every workgroup of any
  // launch that publishes them (the grids of the tiled, row, column-sweep
  // and F / predictor-sweep kernels; the updates' resident grids are at
  // most a.grid)
  const int maxgrid = std::max({a.grid, a.sgrid64, a.sgrid32, a.cgrid, a.cgrid_f});
  a.pgrid = maxgrid;
  if ((st = dalloc(c, &a.partial, 3 * (size_t)maxgrid * S, true)))
    return st;
  if ((st = dalloc(c, &c->stage, N))) return st;
  a.w = d.w;
  a.ifpos = d.ifc.kind ? d.ifpos : nullptr;
  a.f = d.ifc;
  a.n_if = d.ifc.n_if;
  for (int m = 0; m <= c->cfg.M; ++m) {
    a.T[m] = d.T[m];
    a.F[m] = d.F[m];
    a.I[m] = d.I[m];
  }
  a.r = d.r;
  a.p = d.p;
  a.q = d.q;
  if (c->cfg.precision == MRSDC_FP32_REFINE) {
    // FP32 copies of the shared operator values for the inner solves; FP32
    // inner vectors and the FP64 refinement residual, scenario-interleaved
    a.fp32 = 1;
    const size_t NS = (size_t)N * S;
    // p32 and x32 end in one row of 64 zeros (shared, not per scenario): the
    // column sweeps of the CG operator and of the refinement stage halo rows
    // outside a body from it
    if ((st = dalloc(c, &a.x32, NS + kColZeroRow, true)) || (st = dalloc(c, &a.r32, NS, true)) ||
        (st = dalloc(c, &a.p32, NS + kColZeroRow, true)) || (st = dalloc(c, &a.q32, NS, true)) ||
        (st = dalloc(c, &a.r64, NS, true)))
      return st;
    c->scen_bytes -= 2 * (int64_t)kColZeroRow * sizeof(float);
    HIPCHK(hipMemset(a.x32, 0, (NS + kColZeroRow) * sizeof(float)));
    HIPCHK(hipMemset(a.r32, 0, NS * sizeof(float)));
    HIPCHK(hipMemset(a.p32, 0, (NS + kColZeroRow) * sizeof(float)));
    HIPCHK(hipMemset(a.q32, 0, NS * sizeof(float)));
    HIPCHK(hipMemset(a.r64, 0, NS * sizeof(double)));
  }
  a.Eold = d.Eold;
  a.Enew = d.Enew;
  a.Tbuf[0] = d.Tbuf[0];
  a.Tbuf[1] = d.Tbuf[1];
  a.fst = d.fst;
  a.coefD = d.coefD;
  a.coefI = d.coefI;
  if (!c->bsc_host) HIPCHK(hipHostMalloc((void **)&c->bsc_host, sizeof(BatchScalars), 0));
  return MRSDC_OK;
}

mrsdc_status prepare(mrsdc_ctx *c) {
  if (c->prepared) return MRSDC_OK;
  if (!c->body[0].set) return fail(c, MRSDC_ESTATE, "body 0 not set");
  c->nbody = c->body[1].set ? 2 : 1;
  c->off[0] = 0;
  c->off[1] = c->body[0].n;
  c->off[2] = c->off[1] + (c->nbody == 2 ? c->body[1].n : 0);
  const int64_t N = c->off[c->nbody];
  if (c->S == 0)
    for (int b = 0; b < c->nbody; ++b)
      if (!c->body[b].hasT) return fail(c, MRSDC_ESTATE, "temperature of body %d not set", b);
  const mrsdc_config &cfg = c->cfg;
  if (!build_weights(cfg.M, cfg.node_family, cfg.P, cfg.dt, &c->w))
    return fail(c, MRSDC_EINVAL, "bad quadrature");
  hipError_t he = hipSetDevice(cfg.device);
  if (he != hipSuccess) return fail(c, MRSDC_EDEVICE, "hipSetDevice: %s", hipGetErrorString(he));
  if (!c->stream) {
    if (cfg.stream) {
      c->stream = (hipStream_t)cfg.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
  }

  DevState &d = c->d;
  d = DevState();
  d.N = N;
  d.M = cfg.M;
  d.P = cfg.P;
  d.K = cfg.K;
  d.sweep_tol = cfg.sweep_tol;
  d.single_rate = cfg.method == MRSDC_SINGLE_RATE;
  for (int m = 0; m <= cfg.M; ++m) d.dtau_h[m] = c->w.dtau[m];
  // a multiple of the 8 XCDs (the solve kernels deal their rows per XCD)
  d.grid = (int)std::min<int64_t>((N + kBlock - 1) / kBlock, kMaxGrid);
  d.grid = (d.grid + 7) / 8 * 8;
  const bool batch = c->S > 0;
  const int S = batch ? c->S : 1;
  if (batch && c->cpl.kind == 2)
    return fail(c, MRSDC_EINVAL, "batched contexts support the contact coupling only");
  if (batch && cfg.method != MRSDC_MULTIRATE)
    return fail(c, MRSDC_EINVAL, "batched contexts run the multi-rate method");
  if (batch && cfg.op_form != MRSDC_OP_AUTO && cfg.op_form != MRSDC_OP_VALUES)
    return fail(c, MRSDC_EINVAL, "batched contexts take MRSDC_OP_AUTO or MRSDC_OP_VALUES");
  const int form = cfg.op_form & 0xff;  // requested operator form of the CG product
  const bool want_dict = form == MRSDC_OP_AUTO || form >= MRSDC_OP_DICT;

  // ---- operator L = K + h R in SELL-64 ----
  const int64_t nslices = (N + kSlice - 1) / kSlice;
  std::vector<int64_t> off(nslices + 1, 0);
  std::vector<int64_t> rowlen(N);
  std::vector<double> Ldiag(N, 0.0), mass(N), g(N);
  int64_t maxdelta = 0;
  for (int b = 0; b < c->nbody; ++b) {
    const HostBody &B = c->body[b];
    for (int64_t i = 0; i < B.n; ++i) {
      const int64_t row = c->off[b] + i;
      rowlen[row] = B.rowptr[i + 1] - B.rowptr[i];
      mass[row] = B.mass[i];
      g[row] = B.h * B.Tenv * (B.rload.empty() ? 0.0 : B.rload[i]);
      for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e) {
        const double v = B.K[e] + (B.R.empty() ? 0.0 : B.h * B.R[e]);
        if (B.col[e] == i) Ldiag[row] += v;
        maxdelta = std::max<int64_t>(maxdelta, std::llabs((int64_t)B.col[e] - i));
      }
    }
  }
  for (int64_t s = 0; s < nslices; ++s) {
    int64_t w = 0;
    for (int64_t r = s * kSlice; r < std::min<int64_t>(N, (s + 1) * kSlice); ++r)
      w = std::max(w, rowlen[r]);
    off[s + 1] = off[s] + w * kSlice;
  }
  const int64_t nelem = off[nslices];
  const bool use16 = maxdelta <= 32767 && !(cfg.op_form & MRSDC_OP_COL32);
  std::vector<double> val(nelem, 0.0);
  std::vector<float> val32;
  std::vector<int16_t> d16;
  std::vector<int32_t> c32;
  if (use16) d16.assign(nelem, 0);
  else c32.assign(nelem, 0);
  int64_t nnz_total = 0;
  for (int b = 0; b < c->nbody; ++b) {
    const HostBody &B = c->body[b];
    nnz_total += B.nnz;
    for (int64_t i = 0; i < B.n; ++i) {
      const int64_t row = c->off[b] + i, s = row / kSlice, lane = row % kSlice;
      int64_t k = 0;
      for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e, ++k) {
        const int64_t el = off[s] + k * kSlice + lane;
        val[el] = B.K[e] + (B.R.empty() ? 0.0 : B.h * B.R[e]);
        if (use16) d16[el] = (int16_t)((int64_t)B.col[e] - i);
        else c32[el] = (int32_t)(c->off[b] + B.col[e]);
      }
      for (; k * kSlice + off[s] < off[s + 1]; ++k) {  // padding: zero times own entry
        const int64_t el = off[s] + k * kSlice + lane;
        if (!use16) c32[el] = (int32_t)row;
      }
    }
  }
  // lanes past the last row keep col 0 / delta 0 and are never read
  if (cfg.precision == MRSDC_FP32_REFINE && !batch) {
    val32.resize(nelem);
    for (int64_t e = 0; e < nelem; ++e) val32[e] = (float)val[e];
  }
  mrsdc_status st;
  d.op.nrows = N;
  d.op.nslices = nslices;
  d.op.nelem = nelem;
  if (!batch) {  // batched contexts keep their own row-major operators
    int64_t *doff;
    double *dval;
    if ((st = upload(c, &doff, off))) return st;
    if ((st = upload(c, &dval, val))) return st;
    d.op.off = doff;
    d.op.val = dval;
    if (use16) {
      int16_t *p;
      if ((st = upload(c, &p, d16))) return st;
      d.op.d16 = p;
    } else {
      int32_t *p;
      if ((st = upload(c, &p, c32))) return st;
      d.op.c32 = p;
    }
  }
  if (!val32.empty()) {
    float *p;
    if ((st = upload(c, &p, val32))) return st;
    d.op.val32 = p;
  }
  // value dictionary for the CG operator: exact, when the operator holds at
  // most kDictMax distinct values (bit patterns), as on structured meshes
  bool dict = false;
  if (!batch && want_dict) {
    std::unordered_map<uint64_t, int> keys;
    std::vector<uint8_t> vid(nelem);
    std::vector<double> vdict;
    dict = true;
    for (int64_t e = 0; e < nelem; ++e) {
      uint64_t k;
      std::memcpy(&k, &val[e], sizeof k);
      auto it = keys.find(k);
      if (it == keys.end()) {
        if ((int)vdict.size() == kDictMax) {
          dict = false;
          break;
        }
        it = keys.emplace(k, (int)vdict.size()).first;
        vdict.push_back(val[e]);
      }
      vid[e] = (uint8_t)it->second;
    }
    if (dict) {
      uint8_t *pv;
      double *pd;
      if ((st = upload(c, &pv, vid)) || (st = upload(c, &pd, vdict))) return st;
      d.op.vid = pv;
      d.op.vdict = pd;
      d.op.ndict = (int)vdict.size();
      if (use16 && (form == MRSDC_OP_AUTO || form == MRSDC_OP_PATTERNS)) {  // row patterns
        std::map<std::vector<int>, int> forms;
        std::vector<uint8_t> rcls(N, 0);
        std::vector<std::vector<int>> list;
        bool ok = true;
        std::vector<int> key;
        for (int64_t r = 0; r < N && ok; ++r) {
          const int64_t s = r / kSlice, lane = r % kSlice;
          key.clear();
          for (int64_t e = off[s] + lane; e < off[s + 1]; e += kSlice)
            key.push_back((int)d16[e] * 256 + (int)vid[e]);
          if ((int)key.size() > kMaxClsWidth) {
            ok = false;
            break;
          }
          auto it = forms.find(key);
          if (it == forms.end()) {
            if ((int)list.size() == kMaxCls) {
              ok = false;
              break;
            }
            it = forms.emplace(key, (int)list.size()).first;
            list.push_back(key);
          }
          rcls[r] = (uint8_t)it->second;
        }
        if (ok) {
          int cw = 1;
          for (auto &l : list) cw = std::max(cw, (int)l.size());
          std::vector<int> ctab(list.size() * (size_t)cw, 0), clen(list.size());
          for (size_t cI = 0; cI < list.size(); ++cI) {
            clen[cI] = (int)list[cI].size();
            std::copy(list[cI].begin(), list[cI].end(), ctab.begin() + cI * cw);
          }
          uint8_t *pr;
          int *pt, *pl;
          if ((st = upload(c, &pr, rcls)) || (st = upload(c, &pt, ctab)) || (st = upload(c, &pl, clen)))
            return st;
          d.op.rcls = pr;
          d.op.ctab = pt;
          d.op.clen = pl;
          d.op.ncls = (int)list.size();
          d.op.cw = cw;
        }
      }
      if (use16 && maxdelta <= 2047 && vdict.size() <= 16 &&
          (form == MRSDC_OP_AUTO || form == MRSDC_OP_PACKED)) {
        std::vector<int16_t> pk(nelem);
        for (int64_t e = 0; e < nelem; ++e) pk[e] = (int16_t)(d16[e] * 16 + vid[e]);
        int16_t *pp;
        if ((st = upload(c, &pp, pk))) return st;
        d.op.pk16 = pp;
      }
      if (cfg.precision == MRSDC_FP32_REFINE) {
        std::vector<float> vd32(vdict.size());
        for (size_t j = 0; j < vdict.size(); ++j) vd32[j] = (float)vdict[j];
        float *pf;
        if ((st = upload(c, &pf, vd32))) return st;
        d.op.vdict32 = pf;
      }
    }
  }
  if (!batch) {
    c->op_form_used = d.op.rcls ? MRSDC_OP_PATTERNS
                      : d.op.pk16 ? MRSDC_OP_PACKED
                      : d.op.vid ? MRSDC_OP_DICT
                                 : MRSDC_OP_VALUES;
    c->col_bytes = use16 ? 2 : 4;
    if (form != MRSDC_OP_AUTO && form != c->op_form_used)
      return fail(c, MRSDC_EINVAL,
                  "operator form %d does not apply to this operator (%zu-value limit, %d row forms,"
                  " |col - row| up to %lld)",
                  form, form == MRSDC_OP_PACKED ? (size_t)16 : (size_t)kDictMax, kMaxCls,
                  (long long)maxdelta);
  }
  c->matrix_bytes = nnz_total * (8 + (use16 ? 2 : 4)) + 8 * (nslices + 1);
  c->nnz = nnz_total;
  // CG operator application: values (1-byte dictionary indices, or FP64 /
  // FP32 for the inner solves of the FP32 path) + column offsets + p, mass, q
  const int64_t vb = dict ? 1 : (cfg.precision == MRSDC_FP32_REFINE ? 4 : 8);
  const int64_t eb = d.op.pk16 ? 2 : vb + (use16 ? 2 : 4);  // bytes per entry
  c->times.cg_spmv_bytes = (d.op.rcls ? N : nnz_total * eb) + 8 * (nslices + 1) +
                           (cfg.precision == MRSDC_FP32_REFINE ? 12 : 24) * N;
  c->times.nnz = nnz_total;
  c->times.n = N;

  double *dmass, *dg, *dLd;
  if ((st = upload(c, &dmass, mass))) return st;
  if ((st = upload(c, &dg, g))) return st;
  if ((st = upload(c, &dLd, Ldiag))) return st;
  d.mass = dmass;
  d.g = dg;
  d.Ldiag = dLd;
  const bool fp32 = cfg.precision == MRSDC_FP32_REFINE;
  for (int m = 1; m <= cfg.M; ++m) {
    if (c->w.dtau[m] == 0.0 || batch) continue;
    std::vector<double> di(N);
    for (int64_t i = 0; i < N; ++i) di[i] = 1.0 / (mass[i] + c->w.dtau[m] * Ldiag[i]);
    if ((st = upload(c, &d.dinv[m], di))) return st;
    if (fp32) {
      std::vector<float> d32(N);
      for (int64_t i = 0; i < N; ++i) d32[i] = (float)di[i];
      if ((st = upload(c, &d.dinv32[m], d32))) return st;
    }
  }
  if (fp32 && !batch) {
    std::vector<float> m32(N);
    for (int64_t i = 0; i < N; ++i) m32[i] = (float)mass[i];
    float *pm;
    if ((st = upload(c, &pm, m32))) return st;
    d.mass32 = pm;
    if ((st = dalloc(c, &d.x32, N)) || (st = dalloc(c, &d.r32, N)) ||
        (st = dalloc(c, &d.p32, N)) || (st = dalloc(c, &d.q32, N)) ||
        (st = dalloc(c, &d.u32, N)) || (st = dalloc(c, &d.s32, N)) ||
        (st = dalloc(c, &d.b64, N)) || (st = dalloc(c, &d.r64, N)))
      return st;
  }

  // ---- weights ----
  Weights *dw;
  if ((st = dalloc(c, &dw, 1))) return st;
  HIPCHK(hipMemcpy(dw, &c->w, sizeof(Weights), hipMemcpyHostToDevice));
  d.w = dw;

  // ---- states ----
  const bool lob = cfg.node_family == MRSDC_LOBATTO;
  const size_t NS = (size_t)N * S;
  for (int m = 0; m <= cfg.M; ++m) {
    if (lob && m == 1) {
      d.T[1] = d.T[0];
    } else if ((st = dalloc(c, &d.T[m], batch ? NS + kColZeroRow : NS, true))) {
      return st;
    }
    if (m >= 1 && (st = dalloc(c, &d.F[m], NS, true))) return st;
    if (m >= 1 && c->w.dtau[m] != 0.0 && (st = dalloc(c, &d.I[m], NS, true))) return st;
  }
  if (!(batch && fp32) &&
      ((st = dalloc(c, &d.r, NS, true)) || (st = dalloc(c, &d.p, batch ? NS + kColZeroRow : NS, true)) ||
       (st = dalloc(c, &d.q, NS, true)) ||
       (!batch && ((st = dalloc(c, &d.u, NS, true)) || (st = dalloc(c, &d.s, NS, true))))))
    return st;
  if (batch) {  // inactive scenarios keep finite zeros
    for (int m = 0; m <= cfg.M; ++m) {
      // (each node state ends in one row of 64 zeros, shared by the
      // scenarios: the column sweep of F stages halo rows from it)
      if (!(lob && m == 1)) {
        c->scen_bytes -= (int64_t)kColZeroRow * sizeof(double);
        HIPCHK(hipMemset(d.T[m], 0, (NS + kColZeroRow) * sizeof(double)));
      }
      if (m >= 1) HIPCHK(hipMemset(d.F[m], 0, NS * sizeof(double)));
      if (d.I[m]) HIPCHK(hipMemset(d.I[m], 0, NS * sizeof(double)));
    }
    if (!fp32) {
      // p ends in one row of 64 zeros (shared, not per scenario): the column
      // sweep stages halo rows outside a body from it
      c->scen_bytes -= (int64_t)kColZeroRow * sizeof(double);
      HIPCHK(hipMemset(d.r, 0, NS * sizeof(double)));
      HIPCHK(hipMemset(d.p, 0, (NS + kColZeroRow) * sizeof(double)));
      HIPCHK(hipMemset(d.q, 0, NS * sizeof(double)));
    }
  }
  if ((st = dalloc(c, &d.partial, 6 * (size_t)d.grid))) return st;
  if ((st = dalloc(c, &d.sc, 1)) || (st = dalloc(c, &d.ctr, 1)) || (st = dalloc(c, &d.tn, 1)))
    return st;
  HIPCHK(hipMemset(d.sc, 0, sizeof(SolveScalars)));

  // ---- coupling ----
  const Coupling &cp = c->cpl;
  IfaceDev &f = d.ifc;
  f = IfaceDev();
  std::vector<int> ifpos;
  if (cp.kind != 0) {
    const int fb = cp.kind == 1 ? cp.fix_body : cp.body;
    const int ff = cp.kind == 1 ? cp.fix_face : cp.face;
    if (fb >= c->nbody || !c->face[fb][ff].set)
      return fail(c, MRSDC_ESTATE, "coupling face (body %d, face %d) not set", fb, ff);
    const HostFace &F = c->face[fb][ff];
    f.kind = cp.kind;
    f.nuf = F.nu;
    f.nvf = F.nv;
    f.nfix = F.nu * F.nv;
    std::vector<int64_t> rows;
    for (int k = 0; k < f.nfix; ++k) rows.push_back(c->off[fb] + F.ids[k]);
    std::vector<double> um, vm;
    if (cp.kind == 1) {
      if (cp.mov_body >= c->nbody || !c->face[cp.mov_body][cp.mov_face].set)
        return fail(c, MRSDC_ESTATE, "moving face not set");
      if (cp.mov_body == cp.fix_body)
        return fail(c, MRSDC_EINVAL, "contact faces must belong to different bodies");
      const HostFace &G = c->face[cp.mov_body][cp.mov_face];
      f.num = G.nu;
      f.nvm = G.nv;
      for (double x : G.u) um.push_back(x + cp.du);
      for (double x : G.v) vm.push_back(x + cp.dv);
      for (int k = 0; k < G.nu * G.nv; ++k) rows.push_back(c->off[cp.mov_body] + G.ids[k]);
      f.ou0 = std::max(F.u.front(), um.front());
      f.ou1 = std::min(F.u.back(), um.back());
      f.alpha = cp.alpha;
      f.Pf = cp.Pf;
      f.split = cp.split;
      // v direction moves: bound the band from the spacings
      if (max_support(F.v) / min_spacing(vm) + 3 > kBand || max_support(vm) / min_spacing(F.v) + 3 > kBand)
        return fail(c, MRSDC_EINVAL, "face grids too dissimilar along v");
    } else {
      f.ou0 = std::max(F.u.front(), cp.uc - 0.5 * cp.wu);
      f.ou1 = std::min(F.u.back(), cp.uc + 0.5 * cp.wu);
      f.alpha = cp.alpha;
      f.q0 = cp.q0;
      f.Tfix = cp.Tfix;
      f.wv = cp.wv;
    }
    f.n_if = (int)rows.size();
    f.s0 = c->motion.s0;
    f.a = c->motion.a;
    f.period = c->motion.period;
    f.phase = c->motion.phase;
    ifpos.assign(N, -1);
    for (int k = 0; k < f.n_if; ++k) {
      if (ifpos[rows[k]] != -1) return fail(c, MRSDC_EINVAL, "node listed twice on the faces");
      ifpos[rows[k]] = k;
    }
    // static u-direction integrals over [ou0, ou1]
    std::vector<double> Mu(3 * (size_t)f.nuf, 0.0), Hu(f.nuf, 0.0);
    for (int a = 0; a < f.nuf; ++a) {
      for (int i = 0; i < 3; ++i) {
        int aa = a - 1 + i;
        if (aa >= 0 && aa < f.nuf && f.ou1 > f.ou0)
          Mu[3 * a + i] = hat_product_integral(F.u.data(), f.nuf, a, F.u.data(), f.nuf, aa, 0.0,
                                               f.ou0, f.ou1);
      }
      if (f.ou1 > f.ou0) Hu[a] = hat_integral(F.u.data(), f.nuf, a, f.ou0, f.ou1);
    }
    double *p;
    int *pi;
    int64_t *pr;
    if ((st = upload(c, &p, F.u))) return st;
    f.uf = p;
    if ((st = upload(c, &p, F.v))) return st;
    f.vf = p;
    if ((st = upload(c, &p, Mu))) return st;
    f.Mu = p;
    if ((st = upload(c, &p, Hu))) return st;
    f.Hu = p;
    if ((st = upload(c, &pr, rows))) return st;
    f.rows = pr;
    if (cp.kind == 1) {
      std::vector<double> Cu, CuT, Nu(3 * (size_t)f.num, 0.0), Gu(f.num, 0.0);
      std::vector<int> clo, alo, ccnt, acnt;
      if ((st = band_coeffs(c, F.u, um, f.ou0, f.ou1, Cu, clo, ccnt))) return st;
      if ((st = band_coeffs(c, um, F.u, f.ou0, f.ou1, CuT, alo, acnt))) return st;
      for (int cc = 0; cc < f.num; ++cc) {
        for (int i = 0; i < 3; ++i) {
          int c2 = cc - 1 + i;
          if (c2 >= 0 && c2 < f.num && f.ou1 > f.ou0)
            Nu[3 * cc + i] = hat_product_integral(um.data(), f.num, cc, um.data(), f.num, c2, 0.0,
                                                  f.ou0, f.ou1);
        }
        if (f.ou1 > f.ou0) Gu[cc] = hat_integral(um.data(), f.num, cc, f.ou0, f.ou1);
      }
      if ((st = upload(c, &p, um))) return st;
      f.um = p;
      if ((st = upload(c, &p, vm))) return st;
      f.vm = p;
      if ((st = upload(c, &p, Cu))) return st;
      f.Cu = p;
      if ((st = upload(c, &p, CuT))) return st;
      f.CuT = p;
      if ((st = upload(c, &p, Nu))) return st;
      f.Nu = p;
      if ((st = upload(c, &p, Gu))) return st;
      f.Gu = p;
      if ((st = upload(c, &pi, clo))) return st;
      f.clo = pi;
      if ((st = upload(c, &pi, alo))) return st;
      f.alo = pi;
      if ((st = upload(c, &pi, ccnt))) return st;
      f.ccnt = pi;
      if ((st = upload(c, &pi, acnt))) return st;
      f.acnt = pi;
    }
    if ((st = upload(c, &pi, ifpos))) return st;
    d.ifpos = pi;
    const size_t ncache = (size_t)(cfg.M + 1) * (cfg.P + 1) * f.n_if * S;
    if ((st = dalloc(c, &d.Eold, ncache, true)) || (st = dalloc(c, &d.Enew, ncache, true)))
      return st;
    HIPCHK(hipMemset(d.Eold, 0, ncache * sizeof(double)));
    HIPCHK(hipMemset(d.Enew, 0, ncache * sizeof(double)));
    if ((st = dalloc(c, &d.Tbuf[0], (size_t)f.n_if * S, true)) ||
        (st = dalloc(c, &d.Tbuf[1], (size_t)f.n_if * S, true)) ||
        (st = dalloc(c, &d.fst, (size_t)f.n_if * S, true)))
      return st;
    if (d.single_rate &&
        ((st = dalloc(c, &d.ifc_lin, (size_t)f.n_if)) || (st = dalloc(c, &d.ifc_src, (size_t)f.n_if))))
      return st;
    if (!batch && !d.single_rate && (st = dalloc(c, &d.Ipre, ncache))) return st;
    const size_t ntab = (size_t)(cfg.M + 1) * (cfg.P + 1) * S;
    if ((st = dalloc(c, &d.coefD, ntab * coef_table_doubles(f), true)) ||
        (st = dalloc(c, &d.coefI, ntab * coef_table_ints(f), true)))
      return st;
  }
  if (!c->ctr_host) HIPCHK(hipHostMalloc((void **)&c->ctr_host, sizeof(StepCounters), 0));
  if (batch && (st = prepare_batch(c, N))) return st;
  const int b0 = std::min(cfg.pcg_maxit, 24);
  for (int i = 0; i < kSlots; ++i) {
    c->budget[i] = b0;
    c->expect[i] = b0;
    c->last_it[i] = 0;
    c->last_rounds[i] = 0;
    c->rounds[i] = std::min(cfg.refine_maxit, 3);
  }
  c->prepared = true;
  c->dirty_T = true;
  return MRSDC_OK;
}

mrsdc_status upload_T(mrsdc_ctx *c) {
  if (!c->dirty_T) return MRSDC_OK;
  for (int b = 0; b < c->nbody; ++b)
    HIPCHK(hipMemcpyAsync(c->d.T[0] + c->off[b], c->body[b].T.data(), sizeof(double) * c->body[b].n,
                          hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->d.tn, &c->t, sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->dirty_T = false;
  return MRSDC_OK;
}

inline int slot_of(int k, int m) { return k * kMaxM + (m - 1); }

bool take_events(mrsdc_ctx *c, int cls, hipEvent_t *e0, hipEvent_t *e1) {
  *e0 = *e1 = nullptr;
  if (!c->prof) return false;
  if (2 * (c->ev_used + 1) > (int)c->ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      c->ev.push_back(e);
    }
    c->ev_class.resize(c->ev.size() / 2);
  }
  *e0 = c->ev[2 * c->ev_used];
  *e1 = c->ev[2 * c->ev_used + 1];
  c->ev_class[c->ev_used] = cls;
  c->ev_used++;
  return true;
}

void collect_events(mrsdc_ctx *c) {
  for (int i = 0; i < c->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) continue;
    if (c->ev_class[i] == 0) {
      c->times.cg_spmv_launches++;
      c->times.cg_spmv_ms += ms;
    } else {
      c->times.iface_launches++;
      c->times.iface_ms += ms;
    }
  }
  c->ev_used = 0;
}

// CG iterations of one solve within its launch budget, which is returned.
// defer: the check after the budget is left to the caller.
int enqueue_cg(mrsdc_ctx *c, int slot, int m, bool fp32, bool defer = false) {
  const DevState &d = c->d;
  const int B = c->budget[slot];
  for (int it = 0; it < B; ++it) {
    const bool tail = it >= c->expect[slot];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!tail) take_events(c, 0, &e0, &e1);
    if (fp32)
      launch_pcg32_iter(d, m, slot, it, it == B - 1, tail, c->cfg.inner_rtol, c->stream, e0, e1);
    else launch_pcg_iter(d, m, slot, it, it == B - 1, tail, c->cfg.pcg_rtol, c->stream, e0, e1);
  }
  if (!defer) launch_pcg_final(d, m, slot, B, fp32, c->stream);
  return B;
}

// One implicit node solve of interval m (x = T[m] in place).  defer: an FP64
// solve leaves its final check to the caller and returns its launch budget
// (-1 when nothing is left to check).
// Learned launch budgets.  A slot's budget follows its recent iteration
// counts both ways until a step is captured; from then on it only grows, so
// the captured launch sequence stays valid (a converged solve's spare
// launches return at once) and the step is re-captured only when a budget
// grows.
void learn_budget(mrsdc_ctx *c, int i, int v) {
  v = std::min(c->cfg.pcg_maxit, v);
  c->budget[i] = c->graph_exec ? std::max(c->budget[i], v) : v;
}
void learn_rounds(mrsdc_ctx *c, int i, int v) {
  v = std::min(c->cfg.refine_maxit, v);
  c->rounds[i] = c->graph_exec ? std::max(c->rounds[i], v) : v;
}

int enqueue_solve(mrsdc_ctx *c, int k, int m, bool defer = false) {
  const DevState &d = c->d;
  const mrsdc_config &cfg = c->cfg;
  const int slot = slot_of(k, m);
  if (cfg.precision == MRSDC_FP64) {
    if (k == 0) launch_init_pred(d, m, slot, cfg.pcg_rtol, c->stream);
    else launch_init_corr(d, m, slot, cfg.pcg_rtol, c->stream);
    const int B = enqueue_cg(c, slot, m, false, defer);
    return defer ? B : -1;
  }
  // FP32 inner CG, FP64 refinement: rounds within a budget
  launch_refine_init(d, m, slot, k == 0, cfg.refine_rtol, c->stream);
  const int R = c->rounds[slot];
  for (int r = 0; r < R; ++r) {
    launch_inner_init(d, m, slot, cfg.inner_rtol, r, cfg.refine_rtol, c->stream);
    const int B = enqueue_cg(c, slot, m, true, true);
    launch_refine_update(d, m, slot, r, r == R - 1, B, c->stream);
  }
  return -1;
}

void enqueue_step(mrsdc_ctx *c) {
  DevState &d = c->d;
  const int M = c->cfg.M, K = c->cfg.K;
  const bool lob = c->cfg.node_family == MRSDC_LOBATTO;
  hipStream_t st = c->stream;
  launch_clear_counters(d, st);
  launch_iface_coeffs(d, st);
  // predictor (Alg. 1)
  for (int m = 1; m <= M; ++m) {
    if (c->w.dtau[m] == 0.0) continue;
    const int chk = enqueue_solve(c, 0, m, true);
    hipEvent_t e0, e1;
    if (take_events(c, 1, &e0, &e1)) hipEventRecord(e0, st);
    launch_iface(d, m, false, slot_of(0, m), chk, st);
    if (e1) hipEventRecord(e1, st);
  }
  std::swap(d.Eold, d.Enew);
  // correction sweeps (Alg. 2)
  const int passes = c->cfg.final_residual ? K + 1 : K;
  for (int k = 1; k <= passes; ++k) {
    // F_j for all standard nodes that changed (Lobatto T_1 = T_n: once per step)
    const int j0 = (lob && k > 1) ? 2 : 1;
    launch_f_multi(d, j0, M, st);
    launch_quad_resid(d, k - 1, st);
    if (k > K) break;
    launch_iface_quad(d, st);
    for (int m = 1; m <= M; ++m) {
      if (c->w.dtau[m] == 0.0) continue;
      const int chk = enqueue_solve(c, k, m, true);
      hipEvent_t e0, e1;
      if (take_events(c, 1, &e0, &e1)) hipEventRecord(e0, st);
      launch_iface(d, m, true, slot_of(k, m), chk, st);
      if (e1) hipEventRecord(e1, st);
    }
    std::swap(d.Eold, d.Enew);
  }
  launch_step_end(d, c->cfg.dt, st);
}

// Single-rate SDC (the comparison method of §5): f^E joins the implicit part,
// so every node solve carries the exchange operator A_c(tau_m) and the
// coupling source at tau_m, and there are no embedded substeps.  The
// predictor is implicit Euler node by node; a sweep evaluates the full right
// hand side F_j = f^I(T_j) + g + f^E(T_j, tau_j) at the standard nodes and
// integrates it with the weights s_mj alone.
void enqueue_step_single(mrsdc_ctx *c) {
  DevState &d = c->d;
  const int M = c->cfg.M, K = c->cfg.K;
  const bool lob = c->cfg.node_family == MRSDC_LOBATTO;
  hipStream_t st = c->stream;
  launch_clear_counters(d, st);
  launch_iface_coeffs(d, st);
  for (int m = 1; m <= M; ++m)
    if (c->w.dtau[m] != 0.0) enqueue_solve(c, 0, m);
  const int passes = c->cfg.final_residual ? K + 1 : K;
  for (int k = 1; k <= passes; ++k) {
    const int j0 = (lob && k > 1) ? 2 : 1;  // Lobatto T_1 = T_n: once per step
    launch_f_multi(d, j0, M, st);
    for (int j = j0; j <= M; ++j) launch_iface_F(d, j, st);
    launch_quad_resid(d, k - 1, st);
    if (k > K) break;
    for (int m = 1; m <= M; ++m)
      if (c->w.dtau[m] != 0.0) enqueue_solve(c, k, m);
  }
  launch_step_end(d, c->cfg.dt, st);
}

// ---- batched contexts ----
mrsdc_status batch_upload_pending(mrsdc_ctx *c) {
  const int64_t N = c->ba.N;
  for (int s = 0; s < c->S; ++s) {
    if (c->sc_T[s].empty()) continue;
    HIPCHK(hipMemcpyAsync(c->stage, c->sc_T[s].data(), sizeof(double) * N, hipMemcpyHostToDevice,
                          c->stream));
    blaunch_scatter(c->d.T[0], c->stage, N, c->S, s, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->sc_T[s].clear();
  }
  return MRSDC_OK;
}

mrsdc_status batch_upload_params(mrsdc_ctx *c) {
  if (!c->prepared) return MRSDC_OK;
  const int S = c->S;
  std::vector<double> h(S), al(S), pf(S), per(S);
  std::vector<int> act(S);
  for (int s = 0; s < S; ++s) {
    h[s] = std::isnan(c->sc_h[s]) ? c->body[0].h : c->sc_h[s];
    al[s] = std::isnan(c->sc_alpha[s]) ? c->cpl.alpha : c->sc_alpha[s];
    pf[s] = std::isnan(c->sc_Pf[s]) ? c->cpl.Pf : c->sc_Pf[s];
    per[s] = std::isnan(c->sc_period[s]) ? c->motion.period : c->sc_period[s];
    act[s] = c->sc_active[s];
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy((void *)c->ba.h, h.data(), sizeof(double) * S, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)c->ba.alpha, al.data(), sizeof(double) * S, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)c->ba.Pf, pf.data(), sizeof(double) * S, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void *)c->ba.period, per.data(), sizeof(double) * S, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->ba.tn, c->sc_t.data(), sizeof(double) * S, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->ba.sc->active, act.data(), sizeof(int) * S, hipMemcpyHostToDevice));
  return MRSDC_OK;
}

BSolve bsolve(const mrsdc_ctx *c, int k, int m) {
  BSolve sv;
  sv.m = m;
  sv.pred = k == 0;
  sv.slot = slot_of(k, m);
  sv.budget = c->budget[sv.slot];
  sv.rounds = c->rounds[sv.slot];
  sv.rtol = c->cfg.pcg_rtol;
  sv.refine_rtol = c->cfg.refine_rtol;
  sv.inner_rtol = c->cfg.inner_rtol;
  return sv;
}

void enqueue_batch_step(mrsdc_ctx *c) {
  BatchArgs &a = c->ba;
  const int M = c->cfg.M, K = c->cfg.K;
  const bool lob = c->cfg.node_family == MRSDC_LOBATTO;
  hipStream_t st = c->stream;
  blaunch_clear(a, st);
  blaunch_iface_coeffs(a, st);
  for (int m = 1; m <= M; ++m) {
    if (c->w.dtau[m] == 0.0) continue;
    blaunch_solve(a, bsolve(c, 0, m), st);
    blaunch_iface(a, m, false, st);
  }
  std::swap(a.Eold, a.Enew);
  const int passes = c->cfg.final_residual ? K + 1 : K;
  for (int k = 1; k <= passes; ++k) {
    blaunch_f_multi(a, (lob && k > 1) ? 2 : 1, M, st);
    blaunch_quad_resid(a, k - 1, st);
    if (k > K) break;
    for (int m = 1; m <= M; ++m) {
      if (c->w.dtau[m] == 0.0) continue;
      blaunch_solve(a, bsolve(c, k, m), st);
      blaunch_iface(a, m, true, st);
    }
    std::swap(a.Eold, a.Enew);
  }
  blaunch_commit(a, c->cfg.dt, st);
}

// Autotuner (batched contexts): time the launch variants of the CG kernels
// on this mesh and keep the fastest: the column sweep's stages in flight,
// and in the FP32 form the row groups in flight of the two CG updates.
// Every variant forms the same sums in the same order (the grids, and so the
// partial sums, stay fixed), so the choice changes time only.  Runs before
// the first step (the launches then overwrite only CG vectors that every
// solve re-initialises); the choice is kept per process for the mesh, form
// and scenario count.
mrsdc_status autotune_batch(mrsdc_ctx *c) {
  c->tuned = true;
  BatchArgs &a = c->ba;
  const bool fp32 = c->cfg.precision == MRSDC_FP32_REFINE;
  if (c->cfg.autotune >= 2) {  // a fixed variant: bits of autotune - 2
    const int v = c->cfg.autotune - 2;
    a.col_depth = (v & 1) ? 1 : kColDepth;
    a.groups_b = (v & 2) ? 2 : 4;
    a.groups_c = (v & 4) ? 8 : 4;
    return MRSDC_OK;
  }
  if (!fp32 && a.cgrid == 0) return MRSDC_OK;
  static std::mutex mu;
  static std::map<std::vector<int64_t>, std::array<int, 3>> cache;
  const std::vector<int64_t> key = {c->cfg.device, a.N,           a.S,
                                    c->batch_entries, a.cgrid,     a.fp32};
  {
    std::lock_guard<std::mutex> g(mu);
    auto f = cache.find(key);
    if (f != cache.end()) {
      a.col_depth = f->second[0];
      a.groups_b = f->second[1];
      a.groups_c = f->second[2];
      return MRSDC_OK;
    }
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto time_it = [&](int which, float *us) -> hipError_t {
    constexpr int kReps = 8;
    blaunch_tune(a, which, 2, c->stream);  // warm
    hipError_t e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) {
      blaunch_tune(a, which, kReps, c->stream);
      e = hipEventRecord(e1, c->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    *us = 1e3f * ms / kReps;
    return e;
  };
  struct Cand {
    int *knob;
    int which;
    std::vector<int> values;
  };
  // (in FP64 the operator only: the updates there would write the states)
  std::vector<Cand> cands;
  if (fp32) cands = {{&a.groups_b, 1, {4, 2}}, {&a.groups_c, 2, {4, 8}}};
  if (a.cgrid > 0) cands.insert(cands.begin(), Cand{&a.col_depth, 0, {kColDepth, 1}});
  hipError_t e = hipSuccess;
  for (const Cand &k : cands) {
    int best = k.values[0];
    float tbest = 0.f;
    for (size_t i = 0; i < k.values.size() && e == hipSuccess; ++i) {
      *k.knob = k.values[i];
      float us = 0.f;
      e = time_it(k.which, &us);
      if (i == 0 || us < tbest) tbest = us, best = k.values[i];
    }
    *k.knob = best;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, MRSDC_EDEVICE, "autotune: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> g(mu);
  cache[key] = {a.col_depth, a.groups_b, a.groups_c};
  return MRSDC_OK;
}

// One time step on the context's stream: its launches directly, or (use_graph)
// the step captured once into a HIP graph and replayed while the launch
// budgets stay as they were at capture.  The first kGraphWarmSteps steps run
// directly, so the capture holds budgets learned from iteration counts rather
// than the initial ones.  A stream that cannot be captured (the legacy
// default stream) turns graphs off for the context.
constexpr int kGraphWarmSteps = 3;
hipError_t run_step(mrsdc_ctx *c, void (*enqueue)(mrsdc_ctx *)) {
  if (!c->cfg.use_graph || c->graph_off || c->prof || c->graph_warm < kGraphWarmSteps) {
    if (c->cfg.use_graph) c->graph_warm++;
    enqueue(c);
    return hipGetLastError();
  }
  std::vector<int> key(c->budget, c->budget + kSlots);
  key.insert(key.end(), c->rounds, c->rounds + kSlots);
  if (!c->graph_exec || key != c->graph_key) {
    if (c->graph_exec) {
      hipGraphExecDestroy(c->graph_exec);
      c->graph_exec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      hipGetLastError();
      c->graph_off = true;
      enqueue(c);
      return hipGetLastError();
    }
    enqueue(c);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph_exec = nullptr;
      return e;
    }
    c->graph_key = key;
    c->graph_captures++;
  }
  c->graph_replays++;
  return hipGraphLaunch(c->graph_exec, c->stream);
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char *mrsdc_version(void) { return "mrsdc-mi355x 0.1"; }

void mrsdc_config_init(mrsdc_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->device = 0;
  cfg->precision = MRSDC_FP64;
  cfg->M = 3;
  cfg->node_family = MRSDC_LOBATTO;
  cfg->P = 2;
  cfg->K = 2;
  cfg->dt = 1.0;
  cfg->pcg_rtol = 1e-13;
  cfg->pcg_maxit = 1000;
  cfg->refine_rtol = 1e-10;
  cfg->refine_maxit = 20;
  cfg->inner_rtol = 1e-6;
  cfg->final_residual = 0;
  cfg->use_graph = 0;
  cfg->stream = nullptr;
}

mrsdc_status mrsdc_create(mrsdc_ctx **out, const mrsdc_config *cfg) {
  if (!out) return MRSDC_EINVAL;
  *out = nullptr;
  if (!cfg || !valid_scheme(cfg)) return MRSDC_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || cfg->device < 0 || cfg->device >= n) {
    hipGetLastError();
    return MRSDC_EDEVICE;
  }
  if (cfg->alloc && (!cfg->alloc->alloc || !cfg->alloc->release)) return MRSDC_EINVAL;
  mrsdc_ctx *c = new (std::nothrow) mrsdc_ctx();
  if (!c) return MRSDC_ENOMEM;
  c->cfg = *cfg;
  if (cfg->alloc) {
    c->allocator = *cfg->alloc;
    c->cfg.alloc = &c->allocator;
  }
  *out = c;
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_body(mrsdc_ctx *c, int body, int64_t n, int64_t nnz, const int64_t *rowptr,
                            const int32_t *col, const double *K, const double *R, const double *mass,
                            const double *robin_load) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1) return fail(c, MRSDC_EINVAL, "body must be 0 or 1");
  if (n <= 0 || nnz < n || !rowptr || !col || !K || !mass)
    return fail(c, MRSDC_EINVAL, "bad body arrays");
  if (rowptr[0] != 0 || rowptr[n] != nnz) return fail(c, MRSDC_EINVAL, "rowptr must run 0..nnz");
  if (n > (int64_t)1 << 30) return fail(c, MRSDC_EINVAL, "body too large");
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] <= rowptr[i]) return fail(c, MRSDC_EINVAL, "row %lld empty or rowptr not increasing", (long long)i);
    bool diag = false;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return fail(c, MRSDC_EINVAL, "column out of range in row %lld", (long long)i);
      if (e > rowptr[i] && col[e] <= col[e - 1]) return fail(c, MRSDC_EINVAL, "columns not sorted in row %lld", (long long)i);
      if (col[e] == i) diag = true;
    }
    if (!diag) return fail(c, MRSDC_EINVAL, "row %lld has no diagonal entry", (long long)i);
    if (!(mass[i] > 0) || !std::isfinite(mass[i])) return fail(c, MRSDC_EINVAL, "mass must be positive");
  }
  if (!finite_all(K, nnz) || (R && !finite_all(R, nnz)) || (robin_load && !finite_all(robin_load, n)))
    return fail(c, MRSDC_EINVAL, "non-finite operator values");
  free_device(c);
  HostBody &B = c->body[body];
  B.set = true;
  B.n = n;
  B.nnz = nnz;
  B.rowptr.assign(rowptr, rowptr + n + 1);
  B.col.assign(col, col + nnz);
  B.K.assign(K, K + nnz);
  if (R) B.R.assign(R, R + nnz); else B.R.clear();
  B.mass.assign(mass, mass + n);
  if (robin_load) B.rload.assign(robin_load, robin_load + n); else B.rload.clear();
  B.hasT = false;
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_robin(mrsdc_ctx *c, int body, double h, double T_env) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1 || !(h >= 0) || !std::isfinite(h) || !std::isfinite(T_env))
    return fail(c, MRSDC_EINVAL, "bad Robin data");
  c->body[body].h = h;
  c->body[body].Tenv = T_env;
  free_device(c);
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_face(mrsdc_ctx *c, int body, int face, int nu, int nv, const double *u,
                            const double *v, const int32_t *ids) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1 || face < 0 || face > 7 || nu < 2 || nv < 2 || !u || !v || !ids)
    return fail(c, MRSDC_EINVAL, "bad face arguments");
  if (!c->body[body].set) return fail(c, MRSDC_ESTATE, "set the body before its faces");
  for (int i = 1; i < nu; ++i)
    if (!(u[i] > u[i - 1])) return fail(c, MRSDC_EINVAL, "face u not increasing");
  for (int i = 1; i < nv; ++i)
    if (!(v[i] > v[i - 1])) return fail(c, MRSDC_EINVAL, "face v not increasing");
  for (int64_t k = 0; k < (int64_t)nu * nv; ++k)
    if (ids[k] < 0 || ids[k] >= c->body[body].n) return fail(c, MRSDC_EINVAL, "face node id out of range");
  HostFace &F = c->face[body][face];
  F.set = true;
  F.nu = nu;
  F.nv = nv;
  F.u.assign(u, u + nu);
  F.v.assign(v, v + nv);
  F.ids.assign(ids, ids + (int64_t)nu * nv);
  free_device(c);
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_motion(mrsdc_ctx *c, double s0, double a, double period, double phase) {
  if (!c) return MRSDC_EINVAL;
  if (!(period > 0) || !std::isfinite(s0) || !std::isfinite(a) || !std::isfinite(phase) || !std::isfinite(period))
    return fail(c, MRSDC_EINVAL, "bad motion");
  c->motion = {s0, a, period, phase};
  free_device(c);
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_contact(mrsdc_ctx *c, int fix_body, int fix_face, int mov_body, int mov_face,
                               double du, double dv, double alpha, double friction_W, double split) {
  if (!c) return MRSDC_EINVAL;
  if (fix_body < 0 || fix_body > 1 || mov_body < 0 || mov_body > 1 || fix_face < 0 || fix_face > 7 ||
      mov_face < 0 || mov_face > 7 || !(alpha >= 0) || !(friction_W >= 0) || !(split >= 0 && split <= 1) ||
      !std::isfinite(du) || !std::isfinite(dv))
    return fail(c, MRSDC_EINVAL, "bad contact arguments");
  Coupling &p = c->cpl;
  p = Coupling();
  p.kind = 1;
  p.fix_body = fix_body;
  p.fix_face = fix_face;
  p.mov_body = mov_body;
  p.mov_face = mov_face;
  p.du = du;
  p.dv = dv;
  p.alpha = alpha;
  p.Pf = friction_W;
  p.split = split;
  free_device(c);
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_patch(mrsdc_ctx *c, int body, int face, double width_u, double width_v,
                             double u_center, double q0, double alpha, double T_fixed) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1 || face < 0 || face > 7 || !(width_u > 0) || !(width_v > 0) ||
      !std::isfinite(u_center) || !std::isfinite(q0) || !(alpha >= 0) || !std::isfinite(T_fixed))
    return fail(c, MRSDC_EINVAL, "bad patch arguments");
  Coupling &p = c->cpl;
  p = Coupling();
  p.kind = 2;
  p.body = body;
  p.face = face;
  p.wu = width_u;
  p.wv = width_v;
  p.uc = u_center;
  p.q0 = q0;
  p.alpha = alpha;
  p.Tfix = T_fixed;
  free_device(c);
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_temperature(mrsdc_ctx *c, int body, const double *T, int64_t n) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1 || !c->body[body].set) return fail(c, MRSDC_ESTATE, "body not set");
  if (!T || n != c->body[body].n) return fail(c, MRSDC_EINVAL, "temperature length mismatch");
  if (!finite_all(T, n)) return fail(c, MRSDC_EINVAL, "temperature not finite");
  c->body[body].T.assign(T, T + n);
  c->body[body].hasT = true;
  c->dirty_T = true;
  return MRSDC_OK;
}

mrsdc_status mrsdc_set_time(mrsdc_ctx *c, double t) {
  if (!c) return MRSDC_EINVAL;
  if (!std::isfinite(t)) return fail(c, MRSDC_EINVAL, "time not finite");
  // device-resident state must be pulled back before the time can be replaced
  if (c->prepared && !c->dirty_T) {
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->nbody; ++b) {
      c->body[b].T.resize(c->body[b].n);
      HIPCHK(hipMemcpy(c->body[b].T.data(), c->d.T[0] + c->off[b], sizeof(double) * c->body[b].n,
                       hipMemcpyDeviceToHost));
    }
  }
  c->t = t;
  c->dirty_T = true;
  return MRSDC_OK;
}

mrsdc_status mrsdc_get_time(const mrsdc_ctx *c, double *t) {
  if (!c || !t) return MRSDC_EINVAL;
  *t = c->t;
  return MRSDC_OK;
}

mrsdc_status mrsdc_advance(mrsdc_ctx *c, double horizon, mrsdc_stats *stats) {
  if (!c) return MRSDC_EINVAL;
  if (c->S > 0) return fail(c, MRSDC_ESTATE, "batched context: use mrsdc_batch_advance");
  if (stats) std::memset(stats, 0, sizeof(*stats));
  const double dt = c->cfg.dt;
  if (!(horizon >= 0) || !std::isfinite(horizon)) return fail(c, MRSDC_EINVAL, "bad horizon");
  const double ns = horizon / dt;
  const int64_t nsteps = (int64_t)std::llround(ns);
  if (std::fabs(ns - (double)nsteps) > 1e-9 * std::max(1.0, ns))
    return fail(c, MRSDC_EINVAL, "horizon %.17g is not a multiple of dt %.17g", horizon, dt);
  mrsdc_status s = prepare(c);
  if (s) return s;
  if ((s = upload_T(c))) return s;
  auto t0 = std::chrono::steady_clock::now();
  mrsdc_stats acc;
  std::memset(&acc, 0, sizeof acc);
  acc.op_form = c->op_form_used;
  acc.col_bytes = c->col_bytes;
  const int64_t cap0 = c->graph_captures, rep0 = c->graph_replays;
  const int Kc = c->cfg.K;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (;;) {
      HIPCHK(run_step(c, c->d.single_rate ? enqueue_step_single : enqueue_step));
      HIPCHK(hipMemcpyAsync(c->ctr_host, c->d.ctr, sizeof(StepCounters), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      const StepCounters &h = *c->ctr_host;
      if (c->prof) collect_events(c);
      const bool fp32 = c->cfg.precision == MRSDC_FP32_REFINE;
      if (h.fail == 0) {
        acc.pcg_iters += h.pcg_iters;
        acc.sweeps += h.stop ? h.sweeps : Kc;
        acc.refine_steps += h.refine_steps;
        acc.max_iters = std::max(acc.max_iters, h.max_iters);
        for (int k = 0; k <= Kc; ++k) acc.residual[k] = h.resid[k];
        for (int i = 0; i < kSlots; ++i) {
          const int it = h.slot_iters[i];
          if (it > 0) {
            // a slot's count repeats from step to step within one or two: one
            // launch pair beyond the larger of its last two counts (FP64: a
            // solve that still runs out repeats the step with a doubled
            // budget; FP32: an inner solve cut short leaves the rest to the
            // refinement, and its budget doubles)
            learn_budget(c, i, std::max(it, c->last_it[i]) + 1);
            c->last_it[i] = it;
            c->expect[i] = it;
          } else if (it < 0 && fp32 && c->budget[i] < c->cfg.pcg_maxit) {
            c->budget[i] = std::min(c->cfg.pcg_maxit, 2 * c->budget[i]);  // inner solve cut short
          }
          if (fp32 && h.slot_rounds[i] > 0) {
            // the larger of the slot's last two round counts; a solve that
            // needs more repeats the step with twice the rounds
            learn_rounds(c, i, std::max(h.slot_rounds[i], c->last_rounds[i]));
            c->last_rounds[i] = h.slot_rounds[i];
          }
        }
        break;
      }
      // some solve ran out of budget: the step was not committed
      bool grow = false;
      for (int i = 0; i < kSlots; ++i) {
        if (!fp32 && h.slot_iters[i] < 0 && c->budget[i] < c->cfg.pcg_maxit) {
          c->budget[i] = std::min(c->cfg.pcg_maxit, 2 * c->budget[i]);
          grow = true;
        }
        if (fp32 && h.slot_rounds[i] < 0) {
          if (c->rounds[i] < c->cfg.refine_maxit) {
            c->rounds[i] = std::min(c->cfg.refine_maxit, 2 * c->rounds[i]);
            grow = true;
          }
          if (c->budget[i] < c->cfg.pcg_maxit) {
            c->budget[i] = std::min(c->cfg.pcg_maxit, 2 * c->budget[i]);
            grow = true;
          }
        }
      }
      acc.redone_steps++;
      if (!grow) {
        acc.steps = n;  // the device state stays at the last committed step
        if (stats) {
          acc.wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          *stats = acc;
        }
        return fail(c, MRSDC_ENOCONV, "implicit solve did not converge in %d iterations (step %lld)",
                    c->cfg.pcg_maxit, (long long)n);
      }
    }
    c->t += dt;
  }
  // count solves from the scheme
  int nint = 0;
  for (int m = 1; m <= c->cfg.M; ++m) nint += c->w.dtau[m] != 0.0;
  acc.steps = nsteps;
  acc.solves = nsteps * nint * (Kc + 1);
  acc.wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // algorithmic bytes: CG iteration = matrix + 14 vector reads/writes per row;
  // init/solve ~ 8 passes; per sweep one multi-RHS SpMV and (3M+2) passes.
  const int64_t N = c->d.N;
  acc.bytes_moved = acc.pcg_iters * (c->times.cg_spmv_bytes + 88 * N) + acc.solves * 64 * N +
                    nsteps * Kc * (c->matrix_bytes + 16 * (int64_t)c->cfg.M * N +
                                   8 * (3 * (int64_t)c->cfg.M + 2) * N);
  acc.graph_captures = (int32_t)(c->graph_captures - cap0);
  acc.graph_launches = (int32_t)(c->graph_replays - rep0);
  if (stats) *stats = acc;
  return MRSDC_OK;
}

}  // extern "C"

namespace {

// Checks and device preparation shared by both stationary entry points.
mrsdc_status stationary_begin(mrsdc_ctx *c, double rtol, int maxit, int *iters) {
  if (iters) *iters = 0;
  if (c->S > 0) return fail(c, MRSDC_ESTATE, "batched context: set each scenario's field instead");
  if (!(rtol > 0) || !std::isfinite(rtol) || maxit < 1)
    return fail(c, MRSDC_EINVAL, "bad tolerance or iteration cap");
  if (!c->body[0].set) return fail(c, MRSDC_ESTATE, "body 0 not set");
  for (int b = 0; b < 2; ++b) {
    const HostBody &B = c->body[b];
    if (!B.set) continue;
    bool robin = B.h > 0 && !B.R.empty() && !B.rload.empty();
    if (robin) {
      robin = false;
      for (double r : B.rload) robin |= r > 0;
    }
    if (!robin) return fail(c, MRSDC_EINVAL, "body %d has no Robin term: the stationary problem is singular", b);
  }
  // start from the current field (zero where none was set)
  for (int b = 0; b < 2; ++b) {
    HostBody &B = c->body[b];
    if (B.set && !B.hasT) {
      B.T.assign(B.n, 0.0);
      B.hasT = true;
      c->dirty_T = true;
    }
  }
  return MRSDC_OK;
}

// Jacobi-PCG on (K + h R) T = g from the current field, with the Jacobi
// inverse ddinv of L and a zero mass vector dzero (device, N values each).
mrsdc_status stationary_iterate(mrsdc_ctx *c, double rtol, int maxit, int *iters,
                                const double *ddinv, const double *dzero) {
  hipError_t he;
  launch_clear_counters(c->d, c->stream);
  if ((he = hipMemsetAsync(c->d.sc, 0, sizeof(SolveScalars), c->stream)))
    return fail(c, MRSDC_EDEVICE, "HIP: %s", hipGetErrorString(he));
  launch_stationary_init(c->d, dzero, ddinv, 0, rtol, c->stream);
  SolveScalars sc;
  int it = 0;
  for (;;) {
    if ((he = hipMemcpyAsync(&sc, c->d.sc, sizeof sc, hipMemcpyDeviceToHost, c->stream)) ||
        (he = hipStreamSynchronize(c->stream)))
      return fail(c, MRSDC_EDEVICE, "HIP: %s", hipGetErrorString(he));
    if (sc.done) break;
    if (it >= maxit)
      return fail(c, MRSDC_ENOCONV, "stationary solve did not converge in %d iterations", maxit);
    const int n = std::min(64, maxit - it);
    launch_stationary_iters(c->d, dzero, ddinv, 0, it, n, maxit - 1, c->stream);
    if ((he = hipGetLastError())) return fail(c, MRSDC_EDEVICE, "HIP: %s", hipGetErrorString(he));
    it += n;
  }
  if (iters) *iters = sc.iters;
  return MRSDC_OK;
}

}  // namespace

extern "C" {

mrsdc_status mrsdc_set_stationary(mrsdc_ctx *c, double rtol, int maxit, int *iters) {
  if (!c) return MRSDC_EINVAL;
  mrsdc_status st = stationary_begin(c, rtol, maxit, iters);
  if (st) return st;
  if ((st = prepare(c))) return st;
  if ((st = upload_T(c))) return st;
  // Jacobi inverse of L = K + h R and a zero mass vector
  const int64_t N = c->d.N;
  std::vector<double> dinv(N, 0.0);
  for (int b = 0; b < c->nbody; ++b) {
    const HostBody &B = c->body[b];
    for (int64_t i = 0; i < B.n; ++i) {
      double dl = 0.0;
      for (int64_t e = B.rowptr[i]; e < B.rowptr[i + 1]; ++e)
        if (B.col[e] == i) dl += B.K[e] + (B.R.empty() ? 0.0 : B.h * B.R[e]);
      dinv[c->off[b] + i] = 1.0 / dl;
    }
  }
  double *ddinv = (double *)dev_malloc(c, sizeof(double) * N);
  double *dzero = (double *)dev_malloc(c, sizeof(double) * N);
  auto release = [&]() {
    dev_free(c, ddinv);
    dev_free(c, dzero);
  };
  if (!ddinv || !dzero) {
    release();
    return fail(c, MRSDC_ENOMEM, "device allocation failed");
  }
  hipError_t he;
  if ((he = hipMemcpy(ddinv, dinv.data(), sizeof(double) * N, hipMemcpyHostToDevice)) ||
      (he = hipMemset(dzero, 0, sizeof(double) * N))) {
    release();
    return fail(c, MRSDC_EDEVICE, "HIP: %s", hipGetErrorString(he));
  }
  st = stationary_iterate(c, rtol, maxit, iters, ddinv, dzero);
  // the loop above synchronised the stream (or failed): nothing still reads them
  hipStreamSynchronize(c->stream);
  release();
  return st;
}

mrsdc_status mrsdc_set_stationary_noalloc(mrsdc_ctx *c, double rtol, int maxit, int *iters) {
  if (!c) return MRSDC_EINVAL;
  mrsdc_status st = stationary_begin(c, rtol, maxit, iters);
  if (st) return st;
  if (!c->prepared)
    return fail(c, MRSDC_ESTATE,
                "device state not prepared: advance (or call mrsdc_set_stationary) once first");
  const int64_t N = c->d.N;
  if (N > MRSDC_NOALLOC_MAX_ROWS)
    return fail(c, MRSDC_EINVAL, "%lld rows exceed the fixed scratch of %lld rows",
                (long long)N, (long long)MRSDC_NOALLOC_MAX_ROWS);
  hipError_t he = hipSetDevice(c->cfg.device);
  double *scr = nullptr;
  if (he == hipSuccess) he = stationary_scratch(c->cfg.device, &scr);
  if (he != hipSuccess) return fail(c, MRSDC_EDEVICE, "HIP: %s", hipGetErrorString(he));
  if ((st = upload_T(c))) return st;
  // the Jacobi inverse of L from its device diagonal and a zero mass vector,
  // written over whatever an earlier call left in the scratch
  double *ddinv = scr, *dzero = scr + N;
  launch_stationary_scratch(ddinv, dzero, c->d.Ldiag, N, c->stream);
  if ((he = hipGetLastError())) return fail(c, MRSDC_EDEVICE, "HIP: %s", hipGetErrorString(he));
  st = stationary_iterate(c, rtol, maxit, iters, ddinv, dzero);
  hipStreamSynchronize(c->stream);  // the scratch is free for the next call on this device
  return st;
}

mrsdc_status mrsdc_get_temperature(mrsdc_ctx *c, int body, double *out, int64_t n) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1 || !c->body[body].set) return fail(c, MRSDC_ESTATE, "body not set");
  if (!out || n != c->body[body].n) return fail(c, MRSDC_EINVAL, "length mismatch");
  if (!c->prepared || c->dirty_T) {
    if (!c->body[body].hasT) return fail(c, MRSDC_ESTATE, "temperature not set");
    std::memcpy(out, c->body[body].T.data(), sizeof(double) * n);
    return MRSDC_OK;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(out, c->d.T[0] + c->off[body], sizeof(double) * n, hipMemcpyDeviceToHost));
  return MRSDC_OK;
}

mrsdc_status mrsdc_get_temperature_device(mrsdc_ctx *c, int body, void *dptr, int64_t n, void *stream) {
  if (!c) return MRSDC_EINVAL;
  if (body < 0 || body > 1 || !c->body[body].set) return fail(c, MRSDC_ESTATE, "body not set");
  if (!dptr || n != c->body[body].n) return fail(c, MRSDC_EINVAL, "length mismatch");
  mrsdc_status s = prepare(c);
  if (s) return s;
  if ((s = upload_T(c))) return s;
  hipStream_t st = stream ? (hipStream_t)stream : c->stream;
  if (st != c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpyAsync(dptr, c->d.T[0] + c->off[body], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  return MRSDC_OK;
}

mrsdc_status mrsdc_profile(mrsdc_ctx *c, int on) {
  if (!c) return MRSDC_EINVAL;
  c->prof = on != 0;
  const int64_t b = c->times.cg_spmv_bytes, nz = c->times.nnz, n = c->times.n;
  c->times = mrsdc_kernel_times();
  c->times.cg_spmv_bytes = b;
  c->times.nnz = nz;
  c->times.n = n;
  c->ev_used = 0;
  return MRSDC_OK;
}

mrsdc_status mrsdc_profile_read(const mrsdc_ctx *c, mrsdc_kernel_times *out) {
  if (!c || !out) return MRSDC_EINVAL;
  *out = c->times;
  return MRSDC_OK;
}

mrsdc_status mrsdc_time_operator(mrsdc_ctx *c, int reps, double *avg_us, int64_t *bytes) {
  if (!c || reps < 1 || !avg_us) return MRSDC_EINVAL;
  if (!c->prepared) return fail(c, MRSDC_ESTATE, "advance at least once before timing");
  int m = 1;
  while (m <= c->cfg.M && c->w.dtau[m] == 0.0) ++m;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool fp32 = c->cfg.precision == MRSDC_FP32_REFINE;
  auto run = [&](int n) {
    if (c->S > 0) blaunch_operator_timing(c->ba, m, n, c->stream);
    else launch_operator_timing(c->d, m, fp32, n, c->stream);
  };
  run(3);  // warm caches and clocks
  HIPCHK(hipEventRecord(e0, c->stream));
  run(reps);
  HIPCHK(hipEventRecord(e1, c->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_us = 1e3 * ms / reps;
  if (bytes) {
    // batched, tiled: every stored entry (4-byte slot + value) once, per row
    // its extent, K count, own slot and mass (22 bytes), and the S right-hand
    // sides read once and written once (FP32 form: FP32 values and vectors);
    // column sweep: the stencil records and work items once, and the S
    // right-hand sides read once and written once
    const bool f32 = c->cfg.precision == MRSDC_FP32_REFINE;
    const int64_t vb = f32 ? 4 : 8, rhs = 2 * vb * (int64_t)c->S * c->ba.N;
    *bytes = c->S == 0                 ? c->times.cg_spmv_bytes
             : c->ba.cgrid > 0         ? c->col_stored_bytes + rhs
                                       : c->batch_entries * (4 + vb) + 22 * c->ba.N + rhs;
  }
  return MRSDC_OK;
}

mrsdc_status mrsdc_footprint_bytes(const mrsdc_ctx *c, int64_t *bytes) {
  if (!c || !bytes) return MRSDC_EINVAL;
  *bytes = c->footprint;
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_slot_bytes(const mrsdc_ctx *c, int64_t *per_scenario, int64_t *shared) {
  if (!c || !per_scenario || !shared) return MRSDC_EINVAL;
  if (c->S <= 0) return MRSDC_ESTATE;
  if (!c->prepared) return MRSDC_ESTATE;
  *per_scenario = (c->scen_bytes + c->S - 1) / c->S;
  *shared = c->footprint - c->scen_bytes;
  return MRSDC_OK;
}

const char *mrsdc_last_error(const mrsdc_ctx *c) { return c ? c->err.c_str() : "null context"; }

mrsdc_status mrsdc_destroy(mrsdc_ctx *c) {
  if (!c) return MRSDC_OK;
  if (c->stream) hipStreamSynchronize(c->stream);
  free_device(c);
  for (void *p : c->df_allocs) dev_free(c, p);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  if (c->ctr_host) hipHostFree(c->ctr_host);
  if (c->bsc_host) hipHostFree(c->bsc_host);
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  delete c;
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_create(mrsdc_ctx **out, const mrsdc_config *cfg, int S) {
  if (!out) return MRSDC_EINVAL;
  *out = nullptr;
  if (S < 1 || S > kMaxS) return MRSDC_EINVAL;
  if (cfg && cfg->method != MRSDC_MULTIRATE) return MRSDC_EINVAL;  // batches run the method of §3
  mrsdc_status st = mrsdc_create(out, cfg);
  if (st) return st;
  mrsdc_ctx *c = *out;
  c->S = S;
  c->sc_h.assign(S, NAN);
  c->sc_alpha.assign(S, NAN);
  c->sc_Pf.assign(S, NAN);
  c->sc_period.assign(S, NAN);
  c->sc_t.assign(S, 0.0);
  c->sc_active.assign(S, 1);
  c->sc_T.assign(S, std::vector<double>());
  return MRSDC_OK;
}

static mrsdc_status need_batch(mrsdc_ctx *c, int s) {
  if (!c) return MRSDC_EINVAL;
  if (c->S == 0) return fail(c, MRSDC_ESTATE, "not a batched context");
  if (s < 0 || s >= c->S) return fail(c, MRSDC_EINVAL, "scenario %d out of range", s);
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_set_scenario(mrsdc_ctx *c, int s, double h, double alpha, double friction_W,
                                      double period) {
  mrsdc_status st = need_batch(c, s);
  if (st) return st;
  if (!(h >= 0) || !(alpha >= 0) || !(friction_W >= 0) || !(period > 0) || !std::isfinite(h) ||
      !std::isfinite(alpha) || !std::isfinite(friction_W) || !std::isfinite(period))
    return fail(c, MRSDC_EINVAL, "bad scenario parameters");
  c->sc_h[s] = h;
  c->sc_alpha[s] = alpha;
  c->sc_Pf[s] = friction_W;
  c->sc_period[s] = period;
  return batch_upload_params(c);
}

mrsdc_status mrsdc_batch_set_temperature(mrsdc_ctx *c, int s, const double *T, int64_t n) {
  mrsdc_status st = need_batch(c, s);
  if (st) return st;
  int64_t N = 0;
  for (int b = 0; b < 2; ++b) N += c->body[b].set ? c->body[b].n : 0;
  if (!T || n != N) return fail(c, MRSDC_EINVAL, "temperature length %lld != %lld", (long long)n, (long long)N);
  if (!finite_all(T, n)) return fail(c, MRSDC_EINVAL, "temperature not finite");
  c->sc_T[s].assign(T, T + n);
  if (c->prepared) return batch_upload_pending(c);
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_set_time(mrsdc_ctx *c, int s, double t) {
  mrsdc_status st = need_batch(c, s);
  if (st) return st;
  if (!std::isfinite(t)) return fail(c, MRSDC_EINVAL, "time not finite");
  c->sc_t[s] = t;
  return batch_upload_params(c);
}

mrsdc_status mrsdc_batch_set_active(mrsdc_ctx *c, int s, int active) {
  mrsdc_status st = need_batch(c, s);
  if (st) return st;
  if (active && !c->sc_active[s]) c->batch_joined = true;
  c->sc_active[s] = active ? 1 : 0;
  return batch_upload_params(c);
}

mrsdc_status mrsdc_batch_get_time(const mrsdc_ctx *c, int s, double *t) {
  if (!c || !t || c->S == 0 || s < 0 || s >= c->S) return MRSDC_EINVAL;
  *t = c->sc_t[s];
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_advance(mrsdc_ctx *c, int nsteps, mrsdc_stats *stats) {
  mrsdc_status st = need_batch(c, 0);
  if (st) return st;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (nsteps < 0) return fail(c, MRSDC_EINVAL, "negative step count");
  for (int s = 0; s < c->S; ++s)
    if (c->sc_active[s] && !c->prepared && c->sc_T[s].empty())
      return fail(c, MRSDC_ESTATE, "temperature of scenario %d not set", s);
  if ((st = prepare(c))) return st;
  if ((st = batch_upload_pending(c))) return st;
  if (c->cfg.autotune && !c->tuned && (st = autotune_batch(c))) return st;
  auto t0 = std::chrono::steady_clock::now();
  mrsdc_stats acc;
  std::memset(&acc, 0, sizeof acc);
  const int64_t cap0 = c->graph_captures, rep0 = c->graph_replays;
  const int S = c->S, Kc = c->cfg.K;
  for (int n = 0; n < nsteps; ++n) {
    if (c->batch_joined) {
      for (int i = 0; i < kSlots; ++i) {
        c->budget[i] = std::min(c->cfg.pcg_maxit, c->budget[i] + std::max(2, c->budget[i] / 5));
        c->rounds[i] = std::min(c->cfg.refine_maxit, c->rounds[i] + 1);
      }
      c->batch_joined = false;
    }
    for (;;) {
      HIPCHK(run_step(c, enqueue_batch_step));
      HIPCHK(hipMemcpyAsync(c->bsc_host, c->ba.sc, sizeof(BatchScalars), hipMemcpyDeviceToHost,
                            c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      const BatchScalars &h = *c->bsc_host;
      const bool fp32 = c->cfg.precision == MRSDC_FP32_REFINE;
      bool failed = false;
      for (int s = 0; s < S; ++s) failed |= (c->sc_active[s] && h.fail[s]);
      if (!failed) {
        for (int i = 0; i < kSlots; ++i) {
          int mx = 0, rmx = 0;
          bool cut = false;  // an inner solve ran out of its budget (FP32)
          for (int s = 0; s < S; ++s) {
            if (!c->sc_active[s]) continue;
            const int it = h.slot_iters[i][s];
            if (it < 0) cut = true;
            else mx = std::max(mx, it);
            rmx = std::max(rmx, h.slot_rounds[i][s]);
          }
          // as for one simulation: one launch pair beyond the larger of the
          // slot's last two counts (largest over the scenarios), and the
          // larger of its last two round counts
          if (cut && fp32) {
            if (c->budget[i] < c->cfg.pcg_maxit)
              c->budget[i] = std::min(c->cfg.pcg_maxit, 2 * c->budget[i]);
          } else if (mx > 0) {
            learn_budget(c, i, std::max(mx, c->last_it[i]) + 1);
            c->last_it[i] = mx;
            c->expect[i] = mx;
          }
          if (fp32 && rmx > 0) {
            learn_rounds(c, i, std::max(rmx, c->last_rounds[i]));
            c->last_rounds[i] = rmx;
          }
          acc.max_iters = std::max(acc.max_iters, mx);
        }
        for (int s = 0; s < S; ++s) {
          if (!c->sc_active[s]) continue;
          acc.pcg_iters += h.iters_total[s];
          acc.refine_steps += h.refine_total[s];
          acc.sweeps += h.stop[s] ? h.sweeps[s] : Kc;
        }
        for (int k = 0; k <= Kc; ++k) {
          double r = 0.0;
          for (int s = 0; s < S; ++s)
            if (c->sc_active[s]) r = std::max(r, h.resid[k][s]);
          acc.residual[k] = r;
        }
        break;
      }
      // some solve of an active scenario failed: nothing was committed
      bool grow = false;
      for (int i = 0; i < kSlots; ++i) {
        bool slot_failed = false;
        for (int s = 0; s < S; ++s) {
          if (!c->sc_active[s]) continue;
          slot_failed |= fp32 ? h.slot_rounds[i][s] < 0 : h.slot_iters[i][s] < 0;
        }
        if (!slot_failed) continue;
        if (fp32 && c->rounds[i] < c->cfg.refine_maxit) {
          c->rounds[i] = std::min(c->cfg.refine_maxit, 2 * c->rounds[i]);
          grow = true;
        }
        if (c->budget[i] < c->cfg.pcg_maxit) {
          c->budget[i] = std::min(c->cfg.pcg_maxit, 2 * c->budget[i]);
          grow = true;
        }
      }
      acc.redone_steps++;
      if (!grow) {
        acc.steps = n;
        acc.wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = acc;
        return fail(c, MRSDC_ENOCONV, "implicit solve did not converge in %d iterations (step %d)",
                    c->cfg.pcg_maxit, n);
      }
    }
    for (int s = 0; s < S; ++s)
      if (c->sc_active[s]) c->sc_t[s] += c->cfg.dt;
  }
  int nint = 0, nact = 0;
  for (int m = 1; m <= c->cfg.M; ++m) nint += c->w.dtau[m] != 0.0;
  for (int s = 0; s < S; ++s) nact += c->sc_active[s];
  acc.steps = nsteps;
  acc.solves = (int64_t)nsteps * nint * (Kc + 1) * nact;
  acc.wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  acc.graph_captures = (int32_t)(c->graph_captures - cap0);
  acc.graph_launches = (int32_t)(c->graph_replays - rep0);
  acc.col_depth = c->ba.cgrid > 0 ? c->ba.col_depth : 0;
  acc.groups_b = c->ba.groups_b;
  acc.groups_c = c->ba.groups_c;
  acc.autotuned = c->tuned ? 1 : 0;
  if (stats) *stats = acc;
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_get_temperature(mrsdc_ctx *c, int s, double *out, int64_t n) {
  mrsdc_status st = need_batch(c, s);
  if (st) return st;
  if (!out) return fail(c, MRSDC_EINVAL, "null output");
  if (!c->prepared || !c->sc_T[s].empty()) {
    if ((int64_t)c->sc_T[s].size() != n) return fail(c, MRSDC_EINVAL, "length mismatch or no state");
    std::memcpy(out, c->sc_T[s].data(), sizeof(double) * n);
    return MRSDC_OK;
  }
  if (n != c->ba.N) return fail(c, MRSDC_EINVAL, "length mismatch");
  blaunch_gather(c->stage, c->d.T[0], n, c->S, s, c->stream);
  HIPCHK(hipMemcpyAsync(out, c->stage, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_get_temperature_device(mrsdc_ctx *c, int s, void *dptr, int64_t n,
                                                void *stream) {
  mrsdc_status st = need_batch(c, s);
  if (st) return st;
  if (!dptr) return fail(c, MRSDC_EINVAL, "null output");
  if (!c->prepared) return fail(c, MRSDC_ESTATE, "no device state yet (advance once first)");
  if ((st = batch_upload_pending(c))) return st;
  if (n != c->ba.N) return fail(c, MRSDC_EINVAL, "length mismatch");
  hipStream_t hs = stream ? (hipStream_t)stream : c->stream;
  if (hs != c->stream) HIPCHK(hipStreamSynchronize(c->stream));  // the state is complete
  blaunch_gather((double *)dptr, c->d.T[0], n, c->S, s, hs);
  HIPCHK(hipGetLastError());
  return MRSDC_OK;
}

mrsdc_status mrsdc_batch_advance_horizons(mrsdc_ctx *c, const double *horizon, mrsdc_stats *stats) {
  mrsdc_status st = need_batch(c, 0);
  if (st) return st;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!horizon) return fail(c, MRSDC_EINVAL, "null horizons");
  const int S = c->S;
  const double dt = c->cfg.dt;
  std::vector<int64_t> n(S, 0);
  int64_t nmax = 0;
  for (int s = 0; s < S; ++s) {
    if (!c->sc_active[s]) continue;
    const double h = horizon[s];
    if (!(h >= 0) || !std::isfinite(h)) return fail(c, MRSDC_EINVAL, "bad horizon of scenario %d", s);
    const double ns = h / dt;
    n[s] = (int64_t)std::llround(ns);
    if (std::fabs(ns - (double)n[s]) > 1e-9 * std::max(1.0, ns))
      return fail(c, MRSDC_EINVAL, "horizon %.17g of scenario %d is not a multiple of dt %.17g",
                  h, s, dt);
    nmax = std::max(nmax, n[s]);
  }
  // a scenario leaves the batch once its horizon is reached; the others go on
  std::vector<int> was(c->sc_active);
  const bool joined = c->batch_joined;
  mrsdc_stats acc;
  std::memset(&acc, 0, sizeof acc);
  for (int64_t k = 0; k < nmax && !st; ++k) {
    for (int s = 0; s < S; ++s)
      if (was[s] && k == n[s] && (st = mrsdc_batch_set_active(c, s, 0))) break;
    if (st) break;
    mrsdc_stats one;
    if ((st = mrsdc_batch_advance(c, 1, &one))) break;
    acc.steps += one.steps;
    acc.solves += one.solves;
    acc.pcg_iters += one.pcg_iters;
    acc.refine_steps += one.refine_steps;
    acc.max_iters = std::max(acc.max_iters, one.max_iters);
    acc.redone_steps += one.redone_steps;
    acc.wall_s += one.wall_s;
    acc.sweeps += one.sweeps;
    acc.graph_captures += one.graph_captures;
    acc.graph_launches += one.graph_launches;
    acc.col_depth = one.col_depth;
    acc.groups_b = one.groups_b;
    acc.groups_c = one.groups_c;
    acc.autotuned = one.autotuned;
    for (int r = 0; r < 17; ++r) acc.residual[r] = one.residual[r];
  }
  for (int s = 0; s < S; ++s)  // every scenario active again as it was
    if (was[s] && !c->sc_active[s]) {
      const mrsdc_status e = mrsdc_batch_set_active(c, s, 1);
      if (!st) st = e;
    }
  c->batch_joined = joined;  // they rejoin with states the learned budgets fit
  if (stats) *stats = acc;
  return st;
}

mrsdc_status mrsdc_quadrature(int M, int node_family, int P, double dt, double *tau, double *s,
                              double *shat, double *stil, double *spq) {
  Weights *w = new (std::nothrow) Weights;
  if (!w) return MRSDC_ENOMEM;
  if (!tau || !s || !shat || !stil || !spq || !build_weights(M, node_family, P, dt, w)) {
    delete w;
    return MRSDC_EINVAL;
  }
  const int M1 = M + 1, P1 = P + 1;
  for (int m = 0; m <= M; ++m) tau[m] = w->tau[m];
  for (int m = 0; m <= M; ++m) {
    for (int j = 0; j <= M; ++j) s[m * M1 + j] = w->s[m][j];
    for (int q = 0; q <= P; ++q) shat[m * P1 + q] = w->shat[m][q];
    for (int p = 0; p <= P; ++p) {
      for (int j = 0; j <= M; ++j) stil[(m * P1 + p) * M1 + j] = w->stil[m][p][j];
      for (int q = 0; q <= P; ++q) spq[(m * P1 + p) * P1 + q] = w->spq[m][p][q];
    }
  }
  delete w;
  return MRSDC_OK;
}

}  // extern "C"

// ---- thermo-elastic deformation ----

static mrsdc_status df_alloc_bytes(mrsdc_ctx *c, void **p, size_t bytes) {
  void *q = dev_malloc(c, std::max<size_t>(bytes, 8));
  if (!q)
    return fail(c, MRSDC_ENOMEM, "device allocation of %zu bytes for the deformation failed",
                bytes);
  c->df_allocs.push_back(q);
  c->df_bytes += (int64_t)bytes;
  *p = q;
  return MRSDC_OK;
}

template <typename T>
static mrsdc_status df_upload(mrsdc_ctx *c, const T **p, const T *h, size_t n) {
  void *q;
  mrsdc_status s = df_alloc_bytes(c, &q, n * sizeof(T));
  if (s) return s;
  if (n) HIPCHK(hipMemcpy(q, h, n * sizeof(T), hipMemcpyHostToDevice));
  *p = static_cast<const T *>(q);
  return MRSDC_OK;
}

static void df_release(mrsdc_ctx *c) {
  if (c->stream) hipStreamSynchronize(c->stream);
  for (void *p : c->df_allocs) dev_free(c, p);
  c->df_allocs.clear();
  c->df_bytes = 0;
  c->df_ready = false;
  c->df = DeformDev();
}

static bool valid_csr(int64_t n, int64_t ncols, int64_t nnz, const int64_t *rowptr,
                      const int32_t *col, bool sorted) {
  if (rowptr[0] != 0 || rowptr[n] != nnz) return false;
  for (int64_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) return false;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= ncols) return false;
      if (sorted && e > rowptr[i] && col[e] <= col[e - 1]) return false;
    }
  }
  return true;
}

extern "C" {

mrsdc_status mrsdc_deform_setup(mrsdc_ctx *c, int body, int64_t n, int64_t nnz,
                                const int64_t *rowptr, const int32_t *col, const double *Ku,
                                int64_t gnnz, const int64_t *growptr, const int32_t *gcol,
                                const double *G, double T_ref) {
  if (!c) return MRSDC_EINVAL;
  if (c->S > 0) return fail(c, MRSDC_ESTATE, "batched context: deformation is per simulation");
  if (body < 0 || body > 1 || !c->body[body].set) return fail(c, MRSDC_ESTATE, "body not set");
  if (n < 1 || nnz < n || gnnz < 0 || !rowptr || !col || !Ku || !growptr || (gnnz && (!gcol || !G)))
    return fail(c, MRSDC_EINVAL, "bad deformation operator arguments");
  const int64_t nodes = c->body[body].n;
  if (!valid_csr(n, n, nnz, rowptr, col, true) || !valid_csr(n, nodes, gnnz, growptr, gcol, false))
    return fail(c, MRSDC_EINVAL, "malformed CSR of the stiffness or the thermal load operator");
  if (!finite_all(Ku, nnz) || !finite_all(G, gnnz) || !std::isfinite(T_ref))
    return fail(c, MRSDC_EINVAL, "non-finite deformation operator values");
  df_release(c);
  // blocks of the half-bandwidth: only neighbouring blocks couple
  int64_t hb = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) hb = std::max<int64_t>(hb, std::llabs(col[e] - i));
  DeformDev D;
  D.n = n;
  D.bs = std::min<int64_t>(n, std::max<int64_t>(hb, 1));
  D.bp = (D.bs + kGjTile - 1) / kGjTile * kGjTile;
  D.nblk = (n + D.bs - 1) / D.bs;
  if (D.bp > kMaxDeformBlock)
    return fail(c, MRSDC_EINVAL, "half-bandwidth %lld exceeds the block limit %lld (renumber the DOFs)",
                (long long)hb, (long long)kMaxDeformBlock);
  D.toff = c->off[body];
  D.T_ref = T_ref;
  // ELL of the couplings to the previous and the next block
  std::vector<int> cntB(n, 0), cntU(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = i / D.bs, lo = k * D.bs, hi = std::min(n, lo + D.bs);
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      cntB[i] += col[e] < lo;
      cntU[i] += col[e] >= hi;
    }
  }
  D.ellB = std::max(1, *std::max_element(cntB.begin(), cntB.end()));
  D.ellU = std::max(1, *std::max_element(cntU.begin(), cntU.end()));
  if (D.ellB > 128 || D.ellU > 128)
    return fail(c, MRSDC_EINVAL, "more than 128 couplings of a row to a neighbouring block");
  const size_t ellB = (size_t)D.nblk * D.ellB * D.bp, ellU = (size_t)D.nblk * D.ellU * D.bp;
  std::vector<int32_t> bcol(ellB, 0), ucol(ellU, 0);
  std::vector<double> bval(ellB, 0.0), uval(ellU, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = i / D.bs, lo = k * D.bs, hi = std::min(n, lo + D.bs), r = i - lo;
    int qb = 0, qu = 0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      if (col[e] < lo) {
        const size_t at = ((size_t)k * D.ellB + qb++) * D.bp + r;
        bcol[at] = (int32_t)(col[e] - (lo - D.bs));
        bval[at] = Ku[e];
      } else if (col[e] >= hi) {
        const size_t at = ((size_t)k * D.ellU + qu++) * D.bp + r;
        ucol[at] = (int32_t)(col[e] - hi);
        uval[at] = Ku[e];
      }
    }
  }
  // device and stream (the stepper's own state is built lazily elsewhere)
  hipError_t he = hipSetDevice(c->cfg.device);
  if (he != hipSuccess) return fail(c, MRSDC_EDEVICE, "hipSetDevice: %s", hipGetErrorString(he));
  if (!c->stream) {
    if (c->cfg.stream) {
      c->stream = (hipStream_t)c->cfg.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
  }
  mrsdc_status st;
  void *q;
  if ((st = df_upload(c, &D.rowptr, rowptr, (size_t)n + 1)) || (st = df_upload(c, &D.col, col, (size_t)nnz)) ||
      (st = df_upload(c, &D.val, Ku, (size_t)nnz)) ||
      (st = df_upload(c, &D.growptr, growptr, (size_t)n + 1)) ||
      (st = df_upload(c, &D.gcol, gcol, (size_t)gnnz)) || (st = df_upload(c, &D.gval, G, (size_t)gnnz)) ||
      (st = df_upload(c, &D.bcol, bcol.data(), ellB)) || (st = df_upload(c, &D.bval, bval.data(), ellB)) ||
      (st = df_upload(c, &D.ucol, ucol.data(), ellU)) || (st = df_upload(c, &D.uval, uval.data(), ellU))) {
    df_release(c);
    return st;
  }
  const size_t blk = (size_t)D.bp * D.bp * sizeof(double);
  if ((st = df_alloc_bytes(c, &q, blk * D.nblk))) { df_release(c); return st; }
  D.W = (double *)q;
  if ((st = df_alloc_bytes(c, &q, blk))) { df_release(c); return st; }
  D.T1 = (double *)q;
  if ((st = df_alloc_bytes(c, &q, sizeof(double) * 2 * kGjTile * kGjTile))) { df_release(c); return st; }
  D.piv = (double *)q;
  if ((st = df_alloc_bytes(c, &q, sizeof(int)))) { df_release(c); return st; }
  D.flag = (int *)q;
  double *vec[4];
  for (int v = 0; v < 4; ++v) {
    if ((st = df_alloc_bytes(c, &q, sizeof(double) * (v == 3 ? D.bp : n)))) { df_release(c); return st; }
    vec[v] = (double *)q;
  }
  D.f = vec[0];
  D.w = vec[1];
  D.x = vec[2];
  D.c = vec[3];
  {  // strips of the symmetric block product and its partials
    const int nt = D.tiles();
    std::vector<int> strip;
    for (int I = 0; I < nt; ++I)
      for (int J0 = I; J0 < nt; J0 += kSymStrip) {
        strip.push_back(I);
        strip.push_back(J0);
      }
    D.nstrip = (int)(strip.size() / 2);
    const int *sp = nullptr;
    if ((st = df_upload(c, &sp, strip.data(), strip.size()))) { df_release(c); return st; }
    D.strip = sp;
    if ((st = df_alloc_bytes(c, &q, sizeof(double) * 64 * (size_t)nt * D.slots()))) {
      df_release(c);
      return st;
    }
    D.part = (double *)q;
  }
  auto t0 = std::chrono::steady_clock::now();
  int64_t dispatches = 0;
  he = deform_factor(D, c->stream, &dispatches);
  if (he != hipSuccess) {
    hipStreamSynchronize(c->stream);
    df_release(c);
    return fail(c, he == hipErrorInvalidValue ? MRSDC_EINVAL : MRSDC_EDEVICE,
                "factorisation (after %lld launches): %s", (long long)dispatches,
                hipGetErrorString(he));
  }
  c->df_dispatches = dispatches;
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, D.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->df_factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (bad) {
    df_release(c);
    return fail(c, MRSDC_EINVAL, "stiffness is not positive definite (%d non-positive pivots)", bad);
  }
  c->df = D;
  c->df_ready = true;
  c->df_body = body;
  c->df_nodes = nodes;
  return MRSDC_OK;
}

static mrsdc_status deform_run(mrsdc_ctx *c, int64_t n, hipEvent_t *ev) {
  if (!c->df_ready) return fail(c, MRSDC_ESTATE, "no deformation problem registered");
  if (n != c->df.n) return fail(c, MRSDC_EINVAL, "length mismatch (%lld DOFs)", (long long)c->df.n);
  if (!c->body[c->df_body].set || c->body[c->df_body].n != c->df_nodes)
    return fail(c, MRSDC_ESTATE, "the body changed since the deformation was registered");
  mrsdc_status s = prepare(c);
  if (s) return s;
  if ((s = upload_T(c))) return s;
  c->df.toff = c->off[c->df_body];
  deform_solve(c->df, c->d.T[0], c->stream, ev);
  HIPCHK(hipGetLastError());
  return MRSDC_OK;
}

mrsdc_status mrsdc_deform(mrsdc_ctx *c, double *u, int64_t n) {
  if (!c) return MRSDC_EINVAL;
  if (!u) return fail(c, MRSDC_EINVAL, "null output");
  mrsdc_status s = deform_run(c, n, nullptr);
  if (s) return s;
  HIPCHK(hipMemcpyAsync(u, c->df.x, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return MRSDC_OK;
}

mrsdc_status mrsdc_deform_device(mrsdc_ctx *c, void *dptr, int64_t n, void *stream) {
  if (!c) return MRSDC_EINVAL;
  if (!dptr) return fail(c, MRSDC_EINVAL, "null output");
  mrsdc_status s = deform_run(c, n, nullptr);
  if (s) return s;
  hipStream_t st = stream ? (hipStream_t)stream : c->stream;
  if (st != c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpyAsync(dptr, c->df.x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  return MRSDC_OK;
}

mrsdc_status mrsdc_deform_get_info(const mrsdc_ctx *c, mrsdc_deform_info *out) {
  if (!c || !out) return MRSDC_EINVAL;
  if (!c->df_ready) return MRSDC_ESTATE;
  out->n = c->df.n;
  out->block = c->df.bs;
  out->padded_block = c->df.bp;
  out->nblocks = c->df.nblk;
  out->factor_bytes = c->df.nblk * c->df.bp * c->df.bp * (int64_t)sizeof(double);
  out->factor_ms = c->df_factor_ms;
  out->factor_launches = c->df_dispatches;
  return MRSDC_OK;
}

mrsdc_status mrsdc_deform_time(mrsdc_ctx *c, int reps, double *solve_us, double *gemv_us,
                               int64_t *gemv_bytes) {
  if (!c) return MRSDC_EINVAL;
  if (reps < 1 || !solve_us || !gemv_us || !gemv_bytes) return fail(c, MRSDC_EINVAL, "bad arguments");
  if (!c->df_ready) return fail(c, MRSDC_ESTATE, "no deformation problem registered");
  const DeformDev &D = c->df;
  const int ng = (int)(2 * D.nblk - 1);
  std::vector<hipEvent_t> ev(2 * (size_t)ng);
  for (auto &e : ev) HIPCHK(hipEventCreate(&e));
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  mrsdc_status s = deform_run(c, D.n, nullptr);  // warm
  if (!s) {
    HIPCHK(hipEventRecord(a, c->stream));
    for (int r = 0; r < reps && !s; ++r) s = deform_run(c, D.n, nullptr);
    HIPCHK(hipEventRecord(b, c->stream));
  }
  if (!s) s = deform_run(c, D.n, ev.data());
  if (!s) HIPCHK(hipStreamSynchronize(c->stream));
  double gsum = 0.0;
  int64_t bytes = 0;
  if (!s) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    *solve_us = 1e3 * ms / reps;
    for (int g = 0; g < ng; ++g) {
      float m = 0.f;
      HIPCHK(hipEventElapsedTime(&m, ev[2 * g], ev[2 * g + 1]));
      gsum += 1e3 * m;
      // forward k = g, backward k = 2 nblk - 2 - g: the upper-triangle tiles of
      // W, v, the partials written and read back, out (+ base)
      const int64_t k = g < D.nblk ? g : 2 * D.nblk - 2 - g;
      const int64_t nt = D.tiles(), nparts = nt * (nt - 1) / 2 + D.nstrip;
      bytes += nt * (nt + 1) / 2 * 64 * 64 * 8 + D.bp * 8 + 2 * nparts * 64 * 8 +
               D.rows(k) * 8 * (g < D.nblk ? 1 : 2);
    }
    *gemv_us = gsum / ng;
    *gemv_bytes = bytes / ng;
  }
  for (auto &e : ev) hipEventDestroy(e);
  hipEventDestroy(a);
  hipEventDestroy(b);
  return s;
}

}  // extern "C"
