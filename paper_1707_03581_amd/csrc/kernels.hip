// HIP kernels of the MRSDC sweep for gfx950 (wave64).
//
// Data layout: one concatenated state vector per standard node (paper §2,
// eq. coupledFEM), operator L = K + h R in SELL-64 (a slice = 64 consecutive
// rows = one wavefront, lane = row, element columns stored slice-major so that
// each value/column load of a wave is one coalesced 512 B / 128 B access).
// All reductions are deterministic: fixed row-to-block assignment, butterfly
// wave sums, per-block partials reduced in a fixed order.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mrsdc_internal.h"

namespace mrsdc {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the block, result broadcast to every thread.  sh: >= 17 doubles.
__device__ inline double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (w == 0) {
    double t = lane < nw ? sh[lane] : 0.0;
    t = wave_sum(t);
    if (lane == 0) sh[16] = t;
  }
  __syncthreads();
  return sh[16];
}
// Two sums at once (the same order as two block_sum calls).  sh: >= 34 doubles.
__device__ inline void block_sum2(double &v0, double &v1, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  __syncthreads();
  if (lane == 0) {
    sh[w] = v0;
    sh[17 + w] = v1;
  }
  __syncthreads();
  if (w == 0) {
    double t0 = lane < nw ? sh[lane] : 0.0, t1 = lane < nw ? sh[17 + lane] : 0.0;
    t0 = wave_sum(t0);
    t1 = wave_sum(t1);
    if (lane == 0) {
      sh[16] = t0;
      sh[33] = t1;
    }
  }
  __syncthreads();
  v0 = sh[16];
  v1 = sh[33];
}
__device__ inline double block_max(double v, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (w == 0) {
    double t = lane < nw ? sh[lane] : 0.0;
    t = wave_max(t);
    if (lane == 0) sh[16] = t;
  }
  __syncthreads();
  return sh[16];
}

// Every block sums the n per-block partials in the same order.
__device__ inline double sum_partials(const double *part, int n, double *sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  return block_sum(v, sh);
}

// ---------------------------------------------------------------------------
// XCD-aware row spans of the solve kernels: workgroup b runs on XCD b % 8
// (round robin), and XCD x takes the x-th eighth of the 64-row slices, so the
// vectors one kernel writes stay in that XCD's L2 for the next, whose
// neighbour reads fall mostly in the same eighth.  Workgroups past the last
// multiple of 8 get nothing (launch grids are multiples of 8).
// ---------------------------------------------------------------------------
constexpr int kXcd = 8;
struct Span {
  int64_t first, end, step;
};
// this wave's slices
__device__ inline Span xcd_slices(int64_t nslices) {
  const int x = blockIdx.x % kXcd, l = blockIdx.x / kXcd, per = gridDim.x / kXcd;
  const int64_t s1 = nslices * (x + 1) / kXcd;
  Span sp;
  sp.first = nslices * x / kXcd + (int64_t)l * (kBlock / 64) + (threadIdx.x >> 6);
  sp.end = (int)blockIdx.x < per * kXcd ? s1 : 0;
  sp.step = (int64_t)per * (kBlock / 64);
  return sp;
}
// this thread's rows: those of the same slices (N rows, ceil(N / 64) slices)
__device__ inline Span xcd_rows(int64_t N) {
  const int64_t ns = (N + kSlice - 1) / kSlice;
  const int x = blockIdx.x % kXcd, l = blockIdx.x / kXcd, per = gridDim.x / kXcd;
  const int64_t r1 = ns * (x + 1) / kXcd * kSlice;
  Span sp;
  sp.first = ns * x / kXcd * kSlice + (int64_t)l * kBlock + threadIdx.x;
  sp.end = (int)blockIdx.x < per * kXcd ? (r1 < N ? r1 : N) : 0;
  sp.step = (int64_t)per * kBlock;
  return sp;
}

// ---------------------------------------------------------------------------
// SELL-64 row product
// ---------------------------------------------------------------------------
template <bool D16>
__device__ inline double sell_row(const SellDev &op, int64_t s, int lane, int64_t row,
                                  const double *__restrict__ x) {
  const int64_t end = op.off[s + 1];
  int64_t e = op.off[s] + lane;
  double acc = 0.0;
  if (D16) {
#pragma unroll 8
    for (; e < end; e += kSlice) acc += op.val[e] * x[row + op.d16[e]];
  } else {
#pragma unroll 8
    for (; e < end; e += kSlice) acc += op.val[e] * x[op.c32[e]];
  }
  return acc;
}

// ---------------------------------------------------------------------------
// F_j = f^I(T_j) + g = g - L T_j for several j at once (matrix read once)
// ---------------------------------------------------------------------------
struct FArgs {
  const double *T[kMaxJ];
  double *F[kMaxJ];
  const double *g;
};

template <bool D16, int J, bool PK = false>
__global__ __launch_bounds__(kBlock) void k_f_multi(SellDev op, FArgs a) {
  __shared__ double sd[PK ? 16 : 1];
  if (PK) {
    if (threadIdx.x < op.ndict) sd[threadIdx.x] = op.vdict[threadIdx.x];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t s = wave; s < op.nslices; s += nw) {
    const int64_t row = s * kSlice + lane;
    if (row >= op.nrows) continue;
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = 0.0;
    const int64_t end = op.off[s + 1];
    for (int64_t e = op.off[s] + lane; e < end; e += kSlice) {
      double v;
      int64_t c;
      if (PK) {  // packed entry: same value, same column
        const int w = op.pk16[e];
        v = sd[w & 15];
        c = row + (w >> 4);
      } else {
        v = op.val[e];
        c = D16 ? row + op.d16[e] : (int64_t)op.c32[e];
      }
#pragma unroll
      for (int j = 0; j < J; ++j) acc[j] += v * a.T[j][c];
    }
    const double gi = a.g[row];
#pragma unroll
    for (int j = 0; j < J; ++j) a.F[j][row] = gi - acc[j];
  }
}

// Row-pattern tables into LDS: the value dictionary, the forms (offset * 256
// + value id) and their lengths; every table load is issued before the
// first store, then one barrier.
template <typename R>
__device__ inline void stage_forms(const SellDev &op, R *sd, int *sct, int *slen) {
  constexpr int kTab = kMaxCls * kMaxClsWidth / kBlock;
  const R *dict = sizeof(R) == 8 ? (const R *)op.vdict : (const R *)op.vdict32;
  const int nt = op.ncls * op.cw;
  int tab[kTab];
  R dv = 0;
  int lv = 0;
  if ((int)threadIdx.x < op.ndict) dv = dict[threadIdx.x];
#pragma unroll
  for (int q = 0; q < kTab; ++q) {
    const int j = (int)threadIdx.x + q * kBlock;
    tab[q] = j < nt ? op.ctab[j] : 0;
  }
  if ((int)threadIdx.x < op.ncls) lv = op.clen[threadIdx.x];
  if ((int)threadIdx.x < op.ndict) sd[threadIdx.x] = dv;
#pragma unroll
  for (int q = 0; q < kTab; ++q) sct[threadIdx.x + q * kBlock] = tab[q];
  if ((int)threadIdx.x < op.ncls) slen[threadIdx.x] = lv;
  __syncthreads();
}

// F_j = g - L T_j for J nodes through the row patterns: each form entry's
// value and column serve all J vectors; entries in the row's order, as in
// the other formats.
template <int J>
__global__ __launch_bounds__(kBlock) void k_f_multi_cls(SellDev op, FArgs a) {
  __shared__ double sd[kDictMax];
  __shared__ int sct[kMaxCls * kMaxClsWidth];
  __shared__ int slen[kMaxCls];
  const int lane = threadIdx.x & 63;
  const Span sp = xcd_slices(op.nslices);
  const int64_t row0 = sp.first * kSlice + lane;
  const int c0 = (sp.first < sp.end && row0 < op.nrows) ? (int)op.rcls[row0] : 0;
  stage_forms<double>(op, sd, sct, slen);
  for (int64_t s = sp.first; s < sp.end; s += sp.step) {
    const int64_t row = s * kSlice + lane;
    if (row >= op.nrows) continue;
    const int c = s == sp.first ? c0 : (int)op.rcls[row];
    const int n = slen[c];
    const int *t = sct + c * op.cw;
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = 0.0;
#pragma unroll 8
    for (int k = 0; k < n; ++k) {
      const int w = t[k];
      const double v = sd[w & 255];
      const int64_t col = row + (w >> 8);
#pragma unroll
      for (int j = 0; j < J; ++j) acc[j] += v * a.T[j][col];
    }
    const double gi = a.g[row];
#pragma unroll
    for (int j = 0; j < J; ++j) a.F[j][row] = gi - acc[j];
  }
}

template <bool D16>
static void f_multi_dispatch(const DevState &d, FArgs a, int J, hipStream_t st) {
  const int grid = d.grid;
  switch (J) {
#define CASE(n) \
  case n:                                                                   \
    if (d.op.rcls) k_f_multi_cls<n><<<grid, kBlock, 0, st>>>(d.op, a);      \
    else if (d.op.pk16) k_f_multi<D16, n, true><<<grid, kBlock, 0, st>>>(d.op, a); \
    else k_f_multi<D16, n><<<grid, kBlock, 0, st>>>(d.op, a);               \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
}

void launch_f_multi(const DevState &d, int j0, int j1, hipStream_t st) {
  // standard nodes j0..j1 (distinct buffers), in chunks of kMaxJ
  for (int jb = j0; jb <= j1; jb += kMaxJ) {
    const int je = jb + kMaxJ - 1 < j1 ? jb + kMaxJ - 1 : j1;
    FArgs a = {};
    int J = 0;
    for (int j = jb; j <= je; ++j, ++J) {
      a.T[J] = d.T[j];
      a.F[J] = d.F[j];
    }
    a.g = d.g;
    if (d.op.d16) f_multi_dispatch<true>(d, a, J, st);
    else f_multi_dispatch<false>(d, a, J, st);
  }
}

// ---------------------------------------------------------------------------
// Quadrature I_{m-1}^m for every interval (eq. standard_quad) and the residual
// max_m |M T_m - M T_n - sum_{l<=m} I_l| (eq. residual), one pass.
// ---------------------------------------------------------------------------
struct QArgs {
  const Weights *w;
  const double *T[kMaxM + 1];
  const double *F[kMaxM + 1];
  double *I[kMaxM + 1];
  const double *mass;
  const int *ifpos;
  const double *Eold;
  int n_if, M, P;
  double *partial;
};

// (the weights come as a restrict-qualified parameter: read-only and alias
// free for the kernel, so they are read through the scalar cache)
__global__ __launch_bounds__(kBlock) void k_quad_resid(int64_t N, QArgs a,
                                                       const Weights *__restrict__ wp) {
  __shared__ double sh[17];
  const Weights &w = *wp;
  const int P1 = a.P + 1;
  double rmax = 0.0;
  const Span sp = xcd_rows(N);
  for (int64_t i = sp.first; i < sp.end; i += sp.step) {
    // every operand of the row is requested before the first store (a store
    // may alias them, which would order the loads after it)
    const double mi = a.mass[i];
    const double Tn = a.T[0][i];
    const int pos = a.ifpos ? a.ifpos[i] : -1;
    double F[kMaxM + 1], T[kMaxM + 1], acc[kMaxM + 1];
#pragma unroll
    for (int j = 1; j <= kMaxM; ++j) {
      F[j] = j <= a.M ? a.F[j][i] : 0.0;
      T[j] = j <= a.M ? a.T[j][i] : 0.0;
    }
#pragma unroll
    for (int m = 1; m <= kMaxM; ++m) {
      acc[m] = 0.0;
      if (m > a.M || w.dtau[m] == 0.0) continue;
#pragma unroll
      for (int j = 1; j <= kMaxM; ++j)
        if (j <= a.M) acc[m] += w.s[m][j] * F[j];
      if (pos >= 0) {
        const double *E = a.Eold + (size_t)m * P1 * a.n_if + pos;
#pragma unroll 4
        for (int q = 1; q <= a.P; ++q) acc[m] += w.shat[m][q] * E[(size_t)q * a.n_if];
      }
    }
    double cum = 0.0;
#pragma unroll
    for (int m = 1; m <= kMaxM; ++m) {
      if (m > a.M || w.dtau[m] == 0.0) continue;
      a.I[m][i] = acc[m];
      cum += acc[m];
      rmax = fmax(rmax, fabs(mi * T[m] - mi * Tn - cum));
    }
  }
  rmax = block_max(rmax, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = rmax;
}

// residual of iterate k; with residual control (tol > 0) the first iterate
// at or below tol ends the step's sweeps
__global__ void k_reduce_max(const double *part, int n, StepCounters *ctr, int k, double tol) {
  __shared__ double sh[17];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v = fmax(v, part[i]);
  v = block_max(v, sh);
  if (threadIdx.x != 0) return;
  ctr->resid[k] = v;
  if (tol > 0 && !ctr->stop && v <= tol) {
    ctr->stop = 1;
    ctr->sweeps = k;
  }
}

void launch_quad_resid(const DevState &d, int k, hipStream_t st) {
  QArgs a = {};
  a.w = d.w;
  for (int m = 0; m <= d.M; ++m) {
    a.T[m] = d.T[m];
    a.F[m] = d.F[m];
    a.I[m] = d.I[m];
  }
  a.mass = d.mass;
  a.ifpos = (d.ifc.kind && !d.single_rate) ? d.ifpos : nullptr;  // embedded terms
  a.Eold = d.Eold;
  a.n_if = d.ifc.n_if;
  a.M = d.M;
  a.P = d.P;
  a.partial = d.partial;
  k_quad_resid<<<d.grid, kBlock, 0, st>>>(d.N, a, d.w);
  k_reduce_max<<<1, kBlock, 0, st>>>(d.partial, d.grid, d.ctr, k, d.sweep_tol);
}

// ---------------------------------------------------------------------------
// Implicit node solve (diag(m) + dtau L) x = b by Jacobi-preconditioned CG
// (the paper leaves the solver open).  Three kernels per iteration:
//   a: q = A p and p.q            -> last block: alpha
//   b: x += alpha p, r -= alpha q -> last block: convergence, beta
//   c: p = z + beta p
// Every kernel returns at once when the solve is done, so a fixed launch
// budget per solve needs no host round trip.  Global sums are deterministic:
// each block publishes its partial, the last block to arrive adds them in
// block order (agent-scope atomics order the partials across XCDs).
// R is the arithmetic type of the iteration: double (FP64 path) or float
// (inner solves of the FP32 path; products summed in double).
// ---------------------------------------------------------------------------
// block sums -> partial[k*grid + block]; consumers read them after the kernel
template <int K>
__device__ inline void publish(double (&v)[K], double *partial, int grid, double *sh) {
  for (int k = 0; k < K; ++k) v[k] = block_sum(v[k], sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) partial[k * grid + blockIdx.x] = v[k];
}

template <typename R>
struct CgArgs {
  SellDev op;
  int64_t N;
  double dtau;
  const R *mass, *dinv;
  const double *g;
  R *x, *r, *p, *q;
  R *u, *s;  // single-reduction form: u = M^{-1} r, s = A p (q holds w = A u)
  double *partial;  // [6*grid]: per-block partial sums of the current solve
  SolveScalars *sc;
  StepCounters *ctr;
  int slot, grid, inner;
  // init_fold: the first operator step of a single-reduction solve also forms
  // the solve's scalars from the init kernel's partials (r.z, r.r, b.b) with
  // the relative tolerance init_rtol, in place of a separate reduction launch
  int init_fold;
  double init_rtol;
  // residual-controlled sweeps: test the stop flag before anything else, so
  // the launches of sweeps that are no longer run return at once
  int early_stop;
  // init / refinement
  double *x64, *b64, *r64;
  const double *Tprev, *F, *I;
  // single-rate method: interface coupling of the implicit operator at this
  // node (ifc_lin = dtau A_c(tau_m) x for the vector x last passed to the
  // interface kernel, ifc_src = dtau times the coupling source), else null
  int m;
  const int *ifpos;
  const double *ifc_lin, *ifc_src;
};

// Row of the operator through the value dictionary held in LDS (sd): the
// same products and sums as the value array, in the same order.
template <bool D16, typename R>
__device__ inline double sell_row_dict(const SellDev &op, int64_t s, int lane, int64_t row,
                                       const R *__restrict__ x, const R *sd) {
  const int64_t end = op.off[s + 1];
  int64_t e = op.off[s] + lane;
  R acc = 0;
  if (D16) {
#pragma unroll 8
    for (; e < end; e += kSlice) acc += sd[op.vid[e]] * x[row + op.d16[e]];
  } else {
#pragma unroll 8
    for (; e < end; e += kSlice) acc += sd[op.vid[e]] * x[op.c32[e]];
  }
  return acc;
}

// Same through the packed entries: offset in the upper 12 bits, dictionary
// index in the lower 4.
template <typename R>
__device__ inline double sell_row_pk(const SellDev &op, int64_t s, int lane, int64_t row,
                                     const R *__restrict__ x, const R *sd) {
  const int64_t end = op.off[s + 1];
  int64_t e = op.off[s] + lane;
  R acc = 0;
#pragma unroll 8
  for (; e < end; e += kSlice) {
    const int w = op.pk16[e];
    acc += sd[w & 15] * x[row + (w >> 4)];
  }
  return acc;
}

// Same through the row patterns (form table in LDS): the same entries, in the
// same order, slice padding included, so the same sums.
template <typename R>
__device__ inline double sell_row_cls(const SellDev &op, int64_t row, int c,
                                      const R *__restrict__ x, const R *sd, const int *sct,
                                      const int *slen) {
  const int n = slen[c];
  const int *t = sct + c * op.cw;
  R acc = 0;
#pragma unroll 8
  for (int k = 0; k < n; ++k) {
    const int w = t[k];
    acc += sd[w & 255] * x[row + (w >> 8)];
  }
  return acc;
}

template <bool D16, typename R>
__device__ inline double sell_row_t(const SellDev &op, int64_t s, int lane, int64_t row,
                                    const R *__restrict__ x);
template <>
__device__ inline double sell_row_t<true, double>(const SellDev &op, int64_t s, int lane,
                                                  int64_t row, const double *__restrict__ x) {
  return sell_row<true>(op, s, lane, row, x);
}
template <>
__device__ inline double sell_row_t<false, double>(const SellDev &op, int64_t s, int lane,
                                                   int64_t row, const double *__restrict__ x) {
  return sell_row<false>(op, s, lane, row, x);
}
// FP32 operator: FP32 values, FP32 products and sums
template <bool D16>
__device__ inline float sell_row32(const SellDev &op, int64_t s, int lane, int64_t row,
                                   const float *__restrict__ x) {
  const int64_t end = op.off[s + 1];
  int64_t e = op.off[s] + lane;
  float acc = 0.0f;
  if (D16) {
#pragma unroll 4
    for (; e < end; e += kSlice) acc += op.val32[e] * x[row + op.d16[e]];
  } else {
#pragma unroll 4
    for (; e < end; e += kSlice) acc += op.val32[e] * x[op.c32[e]];
  }
  return acc;
}
template <>
__device__ inline double sell_row_t<true, float>(const SellDev &op, int64_t s, int lane,
                                                 int64_t row, const float *__restrict__ x) {
  return sell_row32<true>(op, s, lane, row, x);
}
template <>
__device__ inline double sell_row_t<false, float>(const SellDev &op, int64_t s, int lane,
                                                  int64_t row, const float *__restrict__ x) {
  return sell_row32<false>(op, s, lane, row, x);
}
// FP64 operator applied to an FP32 vector (refinement update)
template <bool D16>
__device__ inline double sell_row_mixed(const SellDev &op, int64_t s, int lane, int64_t row,
                                        const float *__restrict__ x) {
  const int64_t end = op.off[s + 1];
  int64_t e = op.off[s] + lane;
  double acc = 0.0;
  if (D16) {
#pragma unroll 4
    for (; e < end; e += kSlice) acc += op.val[e] * (double)x[row + op.d16[e]];
  } else {
#pragma unroll 4
    for (; e < end; e += kSlice) acc += op.val[e] * (double)x[op.c32[e]];
  }
  return acc;
}

__device__ inline bool solve_done(const SolveScalars *sc, const StepCounters *ctr) {
  return sc->done || sc->ref_done || ctr->stop;
}

// scalars of a fresh CG solve from the sums r.z, r.r, b.b
__device__ inline void init_finish(SolveScalars *sc, StepCounters *ctr, int slot, int inner,
                                   double rtol, const double (&o)[3]) {
  sc->rz[0] = o[0];
  sc->rz[1] = 0.0;
  if (inner) {
    sc->tol2 = rtol * rtol * o[1];   // relative to the inner right-hand side
    sc->done = (o[1] == 0.0) ? 1 : 0;
    return;
  }
  sc->bb = o[2];
  sc->tol2 = rtol * rtol * o[2];
  sc->done = (o[1] <= sc->tol2) ? 1 : 0;
  sc->iters = 0;
  if (sc->done) ctr->slot_iters[slot] = 0;
}

// predictor: x0 = T_{m-1}, b = M T_{m-1} + dtau g, r = b - A x0 (one SpMV)
// CLS: row patterns (the tables staged once per block)
template <bool D16, bool PK = false, bool CLS = false>
__global__ __launch_bounds__(kBlock) void k_init_pred(CgArgs<double> a) {
  __shared__ double sh[17];
  __shared__ double sd[CLS ? kDictMax : (PK ? 16 : 1)];
  __shared__ int sct[CLS ? kMaxCls * kMaxClsWidth : 1];
  __shared__ int slen[CLS ? kMaxCls : 1];
  const int lane = threadIdx.x & 63;
  const Span sp = xcd_slices(a.op.nslices);
  if (CLS) {
    stage_forms<double>(a.op, sd, sct, slen);
  } else if (PK) {
    if (threadIdx.x < a.op.ndict) sd[threadIdx.x] = a.op.vdict[threadIdx.x];
    __syncthreads();
  }
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t s = sp.first; s < sp.end; s += sp.step) {
    const int64_t row = s * kSlice + lane;
    if (row >= a.N) continue;
    const double Lx =
        CLS ? sell_row_cls<double>(a.op, row, a.op.rcls[row], a.Tprev, sd, sct, slen)
        : PK ? sell_row_pk<double>(a.op, s, lane, row, a.Tprev, sd)
             : sell_row<D16>(a.op, s, lane, row, a.Tprev);
    const double x0 = a.Tprev[row], mi = a.mass[row];
    double b = mi * x0 + a.dtau * a.g[row];
    double Ax = mi * x0 + a.dtau * Lx;
    if (a.ifc_lin) {
      const int ip = a.ifpos[row];
      if (ip >= 0) {
        b += a.ifc_src[ip];
        Ax += a.ifc_lin[ip];
      }
    }
    const double r = b - Ax;
    const double z = a.dinv[row] * r;
    a.x[row] = x0;
    a.r[row] = r;
    a.p[row] = z;
    if (a.u) a.u[row] = z;
    v[0] += r * z;
    v[1] += r * r;
    v[2] += b * b;
  }
  publish<3>(v, a.partial, a.grid, sh);
}

// correction: x0 = T^k_m (in place), b = M T^{k+1}_{m-1} + dtau (g - F_m) + I_m,
// and since L x0 = g - F_m the initial residual needs no SpMV:
// r = M (T^{k+1}_{m-1} - T^k_m) + I_m.
__global__ __launch_bounds__(kBlock) void k_init_corr(CgArgs<double> a) {
  if (a.ctr->stop) return;
  __shared__ double sh[17];
  double v[3] = {0.0, 0.0, 0.0};
  const Span sp = xcd_rows(a.N);
  for (int64_t i = sp.first; i < sp.end; i += sp.step) {
    const double mi = a.mass[i], tp = a.Tprev[i], x0 = a.x[i], Im = a.I[i];
    double b = mi * tp + a.dtau * (a.g[i] - a.F[i]) + Im;
    if (a.ifc_src) {
      const int ip = a.ifpos[i];
      if (ip >= 0) b += a.ifc_src[ip];
    }
    const double r = mi * (tp - x0) + Im;
    const double z = a.dinv[i] * r;
    a.r[i] = r;
    a.p[i] = z;
    if (a.u) a.u[i] = z;
    v[0] += r * z;
    v[1] += r * r;
    v[2] += b * b;
  }
  publish<3>(v, a.partial, a.grid, sh);
}

// One block: the scalars of a solve from the partials of the previous kernel.
// mode 0: FP64 CG init (r.z, r.r, b.b)   1: refinement init (r.r, b.b)
// mode 2: inner FP32 CG init (r.z, r.r)  3: refinement update (r.r)
__global__ void k_solve_reduce(const double *part, int grid, SolveScalars *sc, StepCounters *ctr,
                               int slot, int mode, double rtol, int round, int last_round) {
  if (ctr->stop) return;  // residual control ended this step's sweeps
  __shared__ double sh[17];
  const int nk = (mode == 0) ? 3 : (mode == 3 ? 1 : 2);
  // the refinement's partials (modes 1, 3) are in slots 2, 3
  const double *base = part + ((mode == 1 || mode == 3) ? 2 * grid : 0);
  double o[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < nk; ++k) o[k] = sum_partials(base + k * grid, grid, sh);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    init_finish(sc, ctr, slot, 0, rtol, o);
  } else if (mode == 1) {
    sc->ref_bb = o[1];
    sc->ref_tol2 = rtol * rtol * o[1];
    sc->ref_done = (o[0] <= sc->ref_tol2) ? 1 : 0;
    sc->ref_rounds = 0;
    sc->done = 0;
    ctr->slot_iters[slot] = 0;  // largest inner iteration count of the solve
    if (sc->ref_done) ctr->slot_rounds[slot] = 0;
  } else if (mode == 2) {
    if (sc->ref_done) return;
    init_finish(sc, ctr, slot, 1, rtol, o);
  } else {
    if (sc->ref_done) return;
    sc->ref_rounds = round + 1;
    ctr->refine_steps += 1;
    if (o[0] <= sc->ref_tol2) {
      sc->ref_done = 1;
      ctr->slot_rounds[slot] = round + 1;
    } else if (last_round) {
      ctr->slot_rounds[slot] = -1;
      ctr->fail += 1;
    }
  }
}

// (a) q = A p, partial p.q.  TAIL = 1 marks launches past the iteration count
// of the previous step (usually early exits), TAIL = 2 the stand-alone timing
// launches (which ignore the convergence flag); both kept apart in profiles.
// FMT: 0 value array, 1 value dictionary, 2 packed entries, 3 row patterns
// CG2: the operator step of the single-reduction iteration (w = A u, partial
// u.w into slot 5), which first ends the solve if ||r_it||^2, summed from
// the previous update's partials, is below the tolerance.
template <typename R>
__device__ inline void cg_converged(const CgArgs<R> &a, int iters) {
  SolveScalars *sc = a.sc;
  StepCounters *ctr = a.ctr;
  sc->done = 1;
  sc->iters = iters;
  ctr->pcg_iters += iters;
  if (!a.inner) ctr->slot_iters[a.slot] = iters;
  else if (ctr->slot_iters[a.slot] >= 0 && iters > ctr->slot_iters[a.slot])
    ctr->slot_iters[a.slot] = iters;
  if (iters > ctr->max_iters) ctr->max_iters = iters;
}

static_assert(kDictMax <= kBlock && kMaxCls <= kBlock && kMaxGrid % kBlock == 0 &&
                  (kMaxCls * kMaxClsWidth) % kBlock == 0,
              "the operator kernel stages one dictionary entry and one form length per thread");

template <bool D16, int TAIL, typename R, bool CPL = false, int FMT = 0, bool CG2 = false>
__global__ __launch_bounds__(kBlock) void k_pcg_a(CgArgs<R> a, int it) {
  constexpr bool DICT = FMT != 0;
  __shared__ double sh[34];
  __shared__ R sd[DICT ? kDictMax : 1];
  __shared__ int sct[FMT == 3 ? kMaxCls * kMaxClsWidth : 1];
  __shared__ int slen[FMT == 3 ? kMaxCls : 1];
  constexpr int kTab = FMT == 3 ? kMaxCls * kMaxClsWidth / kBlock : 1;
  constexpr int kPart = kMaxGrid / kBlock;
  // fresh: the first operator step of a solve, which forms the solve's
  // scalars from the init kernel's partials (r.z, r.r, b.b) and reads none of
  // the previous solve's flags; check: the convergence test on ||r_it||^2
  const bool fresh = CG2 && TAIL != 2 && it == 0 && a.init_fold;
  const bool check = CG2 && TAIL != 2 && it > 0;
  const R *__restrict__ xin = CG2 ? a.u : a.p;
  const int lane = threadIdx.x & 63;
  const Span sp = xcd_slices(a.op.nslices);
  if (a.early_stop && a.ctr->stop) return;
  // Every request that does not depend on another is issued before the first
  // wait: the solve flags, the partials of the reductions, the table entries
  // and the first slice's row data.
  int stop = 0;
  if (TAIL != 2)  // (an inner solve of the refinement also ends with its refinement)
    stop = fresh ? (a.ctr->stop | (a.inner ? a.sc->ref_done : 0))
                 : (a.sc->done | a.sc->ref_done | a.ctr->stop);
  // (loaded first at clamped indices, summed afterwards over the valid ones)
  double t0[kPart], t1[kPart], t2[kPart];
#pragma unroll
  for (int q = 0; q < kPart; ++q) t0[q] = t1[q] = t2[q] = 0.0;
  if (fresh || check) {
    const double *p0 = a.partial + (fresh ? 0 : ((it & 1) ? 4 : 1) * a.grid);
#pragma unroll
    for (int q = 0; q < kPart; ++q) {
      const int j = (int)threadIdx.x + q * kBlock;
      t0[q] = p0[j < a.grid ? j : a.grid - 1];
    }
  }
  if (fresh) {
#pragma unroll
    for (int q = 0; q < kPart; ++q) {
      const int j = (int)threadIdx.x + q * kBlock;
      const int jc = j < a.grid ? j : a.grid - 1;
      t1[q] = a.partial[a.grid + jc];
      t2[q] = a.partial[2 * a.grid + jc];
    }
  }
  int tab[kTab];
  R dv = 0;
  int lv = 0;
  if (DICT) {
    const R *dict = sizeof(R) == 8 ? (const R *)a.op.vdict : (const R *)a.op.vdict32;
    if ((int)threadIdx.x < a.op.ndict) dv = dict[threadIdx.x];
    if (FMT == 3) {
      const int nt = a.op.ncls * a.op.cw;
#pragma unroll
      for (int q = 0; q < kTab; ++q) {
        const int j = (int)threadIdx.x + q * kBlock;
        tab[q] = j < nt ? a.op.ctab[j] : 0;
      }
      if ((int)threadIdx.x < a.op.ncls) lv = a.op.clen[threadIdx.x];
    }
  }
  const int64_t row0 = sp.first * kSlice + lane;
  const bool have0 = sp.first < sp.end && row0 < a.N;
  int c0 = 0;
  R u0 = 0, m0 = 0;
  if (have0) {
    if (FMT == 3) c0 = a.op.rcls[row0];
    u0 = xin[row0];
    m0 = a.mass[row0];
  }
  if (stop) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int q = 0; q < kPart; ++q) {
    if ((int)threadIdx.x + q * kBlock < a.grid) {
      s0 += t0[q];
      s1 += t1[q];
      s2 += t2[q];
    }
  }
  if (fresh) {
    const double rz = s0;
    double rr = s1, bb = s2;
    block_sum2(rr, bb, sh);
    const double o[3] = {block_sum(rz, sh), rr, bb};
    if (blockIdx.x == 0 && threadIdx.x == 0)
      init_finish(a.sc, a.ctr, a.slot, a.inner, a.init_rtol, o);
    // the warm start meets the tolerance (an inner solve: a zero right-hand side)
    if (a.inner ? rr == 0.0 : rr <= a.init_rtol * a.init_rtol * bb) return;
  } else if (check) {
    const double rr = block_sum(s0, sh);
    if (rr <= a.sc->tol2) {
      if (blockIdx.x == 0 && threadIdx.x == 0) cg_converged(a, it);
      return;
    }
  }
  if (DICT) {
    if ((int)threadIdx.x < a.op.ndict) sd[threadIdx.x] = dv;
    if (FMT == 3) {
#pragma unroll
      for (int q = 0; q < kTab; ++q) sct[threadIdx.x + q * kBlock] = tab[q];
      if ((int)threadIdx.x < a.op.ncls) slen[threadIdx.x] = lv;
    }
    __syncthreads();
  }
  double v[1] = {0.0};
  for (int64_t s = sp.first; s < sp.end; s += sp.step) {
    const int64_t row = s * kSlice + lane;
    if (row >= a.N) continue;
    const bool first = s == sp.first;
    const R Lp = FMT == 3 ? (R)sell_row_cls<R>(a.op, row, first ? c0 : (int)a.op.rcls[row], xin,
                                                 sd, sct, slen)
                 : FMT == 2 ? (R)sell_row_pk<R>(a.op, s, lane, row, xin, sd)
                 : FMT == 1 ? (R)sell_row_dict<D16, R>(a.op, s, lane, row, xin, sd)
                            : (R)sell_row_t<D16, R>(a.op, s, lane, row, xin);
    const R pi = first ? u0 : xin[row];
    R qi = (first ? m0 : a.mass[row]) * pi + (R)a.dtau * Lp;
    if (CPL) {  // single-rate method: the coupling of the node operator
      const int ip = a.ifpos[row];
      if (ip >= 0) qi += (R)a.ifc_lin[ip];
    }
    a.q[row] = qi;
    v[0] += (double)pi * (double)qi;
  }
  publish<1>(v, a.partial + (CG2 ? 5 * a.grid : 0), a.grid, sh);
}

// Single-reduction (Chronopoulos-Gear) update of iteration it: with
// gamma = r.u (previous update's partials) and delta = u.w (operator step's):
// beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
// (it = 0: beta = 0, alpha = gamma / delta); p = u + beta p, s = w + beta s,
// x += alpha p, r -= alpha s, u = M^{-1} r; partials of the next r.u, r.r.
// Mathematically the Jacobi-PCG iteration, with one reduction point instead
// of two, so one launch fewer per iteration.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_upd(CgArgs<R> a, int it) {
  if (a.early_stop && a.ctr->stop) return;
  // the solve flags, the first row's operands and the partials are all
  // requested before the first wait
  const int stop = a.sc->done | a.sc->ref_done | a.ctr->stop;
  __shared__ double sh[34];
  const Span sp = xcd_rows(a.N);
  const int64_t i0 = sp.first;
  const bool first = i0 < sp.end;
  R u0 = 0, w0 = 0, p0 = 0, s0 = 0, x0 = 0, r0 = 0, d0 = 0;
  if (first) {
    u0 = a.u[i0];
    w0 = a.q[i0];
    if (it > 0) {
      p0 = a.p[i0];
      s0 = a.s[i0];
    }
    x0 = a.x[i0];
    r0 = a.r[i0];
    d0 = a.dinv[i0];
  }
  const double *pg = a.partial + ((it & 1) ? 3 : 0) * a.grid, *pd = a.partial + 5 * a.grid;
  // loaded first at clamped indices (no branch between the loads), summed
  // afterwards over the valid ones
  double tg[kMaxGrid / kBlock], td[kMaxGrid / kBlock];
#pragma unroll
  for (int q = 0; q < kMaxGrid / kBlock; ++q) {
    const int j = (int)threadIdx.x + q * kBlock;
    const int jc = j < a.grid ? j : a.grid - 1;
    tg[q] = pg[jc];
    td[q] = pd[jc];
  }
  if (stop) return;
  double gam = 0.0, del = 0.0;
#pragma unroll
  for (int q = 0; q < kMaxGrid / kBlock; ++q) {
    if ((int)threadIdx.x + q * kBlock < a.grid) {
      gam += tg[q];
      del += td[q];
    }
  }
  block_sum2(gam, del, sh);
  SolveScalars *sc = a.sc;
  double beta = 0.0, alpha;
  if (it == 0) {
    alpha = gam / del;
  } else {
    beta = gam / sc->gam[(it - 1) & 1];
    alpha = gam / (del - beta * gam / sc->alp[(it - 1) & 1]);
  }
  const R al = (R)alpha, be = (R)beta;
  double v0 = 0.0, v1 = 0.0;
  auto upd = [&](int64_t i, R u, R w, R p, R s, R x, R r, R d) {
    const R pn = it == 0 ? u : u + be * p;
    const R sn = it == 0 ? w : w + be * s;
    a.p[i] = pn;
    a.s[i] = sn;
    a.x[i] = x + al * pn;
    const R rn = r - al * sn;
    a.r[i] = rn;
    const R un = d * rn;
    a.u[i] = un;
    v0 += (double)rn * (double)un;
    v1 += (double)rn * (double)rn;
  };
  if (first) upd(i0, u0, w0, p0, s0, x0, r0, d0);
  for (int64_t i = i0 + sp.step; i < sp.end; i += sp.step)
    upd(i, a.u[i], a.q[i], it > 0 ? a.p[i] : (R)0, it > 0 ? a.s[i] : (R)0, a.x[i], a.r[i],
        a.dinv[i]);
  block_sum2(v0, v1, sh);
  double *po = a.partial + (((it + 1) & 1) ? 3 : 0) * a.grid;  // gamma, rho of it + 1
  if (threadIdx.x == 0) {
    po[blockIdx.x] = v0;
    po[a.grid + blockIdx.x] = v1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->gam[it & 1] = gam;
    sc->alp[it & 1] = alpha;
  }
}

// After the launch budget: converged at iteration it, or the solve failed.
// Executed by one whole block.
template <typename R>
__device__ inline void cg_check_block(const CgArgs<R> &a, int it, double *sh) {
  if (solve_done(a.sc, a.ctr)) return;
  const double rr = sum_partials(a.partial + ((it & 1) ? 4 : 1) * a.grid, a.grid, sh);
  if (threadIdx.x != 0) return;
  if (rr <= a.sc->tol2) {
    cg_converged(a, it);
  } else {  // budget exhausted: the FP64 solve failed; an inner solve only signals it
    a.ctr->slot_iters[a.slot] = -1;
    a.ctr->pcg_iters += it;
    if (!a.inner) a.ctr->fail += 1;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_check(CgArgs<R> a, int it) {
  __shared__ double sh[17];
  cg_check_block(a, it, sh);
}

// (b) alpha = r.z / p.q; x += alpha p; r -= alpha q; partial r.z, r.r
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pcg_b(CgArgs<R> a, int it) {
  if (solve_done(a.sc, a.ctr)) return;
  __shared__ double sh[17];
  // the first row's operands are requested before the reduction of p.q
  const Span sp = xcd_rows(a.N);
  int64_t i = sp.first;
  const bool first = i < sp.end;
  R x0 = 0, p0 = 0, r0 = 0, q0 = 0, d0 = 0;
  if (first) {
    x0 = a.x[i];
    p0 = a.p[i];
    r0 = a.r[i];
    q0 = a.q[i];
    d0 = a.dinv[i];
  }
  const double pq = sum_partials(a.partial, a.grid, sh);
  const R alpha = (R)(a.sc->rz[it & 1] / pq);
  double v[2] = {0.0, 0.0};
  if (first) {
    a.x[i] = x0 + alpha * p0;
    const R r = r0 - alpha * q0;
    a.r[i] = r;
    v[0] += (double)r * (double)(d0 * r);
    v[1] += (double)r * (double)r;
  }
  for (i += sp.step; i < sp.end; i += sp.step) {
    a.x[i] += alpha * a.p[i];
    const R r = a.r[i] - alpha * a.q[i];
    a.r[i] = r;
    v[0] += (double)r * (double)(a.dinv[i] * r);
    v[1] += (double)r * (double)r;
  }
  double *part = a.partial + a.grid;
  for (int k = 0; k < 2; ++k) v[k] = block_sum(v[k], sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v[0];
    part[a.grid + blockIdx.x] = v[1];
  }
}

// (c) convergence test; beta = r.z_new / r.z; p = z + beta p
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pcg_c(CgArgs<R> a, int it, int last) {
  if (solve_done(a.sc, a.ctr)) return;
  __shared__ double sh[34];
  // the first row's operands are requested before the reductions
  const Span sp = xcd_rows(a.N);
  const int64_t i0 = sp.first;
  const bool first = i0 < sp.end;
  R d0 = 0, r0 = 0, p0 = 0;
  if (first) {
    d0 = a.dinv[i0];
    r0 = a.r[i0];
    p0 = a.p[i0];
  }
  double rz = 0.0, rr = 0.0;
  for (int j = threadIdx.x; j < a.grid; j += blockDim.x) {
    rz += a.partial[a.grid + j];
    rr += a.partial[2 * a.grid + j];
  }
  block_sum2(rz, rr, sh);
  SolveScalars *sc = a.sc;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (rr <= sc->tol2) {
    if (lead) {
      StepCounters *ctr = a.ctr;
      sc->done = 1;
      sc->iters = it + 1;
      ctr->pcg_iters += it + 1;
      if (!a.inner) ctr->slot_iters[a.slot] = it + 1;
      else if (ctr->slot_iters[a.slot] >= 0 && it + 1 > ctr->slot_iters[a.slot])
        ctr->slot_iters[a.slot] = it + 1;
      if (it + 1 > ctr->max_iters) ctr->max_iters = it + 1;
    }
    return;
  }
  const R beta = (R)(rz / sc->rz[it & 1]);
  if (first) a.p[i0] = d0 * r0 + beta * p0;
  for (int64_t i = i0 + sp.step; i < sp.end; i += sp.step)
    a.p[i] = a.dinv[i] * a.r[i] + beta * a.p[i];
  if (lead) {
    sc->rz[(it + 1) & 1] = rz;
    if (last) {
      // budget exhausted: the FP64 solve failed; an inner solve only signals it
      a.ctr->slot_iters[a.slot] = -1;
      a.ctr->pcg_iters += it + 1;
      if (!a.inner) a.ctr->fail += 1;
    }
  }
}

// ---- FP64 iterative refinement around FP32 inner solves ----
// init: b and r = b - A x0 in FP64 (corrections without SpMV as above)
template <bool D16, bool PRED, bool PK = false>
__global__ __launch_bounds__(kBlock) void k_rinit(CgArgs<float> a, const double *mass64) {
  if (a.ctr->stop) return;
  __shared__ double sh[17];
  __shared__ double sd[PK ? 16 : 1];
  if (PK) {
    if (threadIdx.x < a.op.ndict) sd[threadIdx.x] = a.op.vdict[threadIdx.x];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  double v[2] = {0.0, 0.0};
  for (int64_t s = wave; s < a.op.nslices; s += nw) {
    const int64_t row = s * kSlice + lane;
    if (row >= a.N) continue;
    const double mi = mass64[row], tp = a.Tprev[row];
    double b, r;
    if (PRED) {
      const double Lx = PK ? sell_row_pk<double>(a.op, s, lane, row, a.Tprev, sd)
                           : sell_row<D16>(a.op, s, lane, row, a.Tprev);
      b = mi * tp + a.dtau * a.g[row];
      r = b - (mi * tp + a.dtau * Lx);
      a.x64[row] = tp;
    } else {
      const double Im = a.I[row];
      b = mi * tp + a.dtau * (a.g[row] - a.F[row]) + Im;
      r = mi * (tp - a.x64[row]) + Im;
    }
    a.b64[row] = b;
    a.r64[row] = r;
    v[0] += r * r;
    v[1] += b * b;
  }
  publish<2>(v, a.partial + 2 * a.grid, a.grid, sh);  // slots 2, 3: r.r, b.b
}

// inner init: r32 = r64, d = 0, p = dinv r32; tolerance relative to ||r32||
// Round 0 first forms the refinement's scalars from the refinement init's
// partials (r.r, b.b in slots 2, 3); a later round first takes the previous
// round's refinement check from the update's partials (r.r in slot 2).  Every
// block decides alike; block 0 stores the scalars.  The last round's check
// stays with k_solve_reduce (mode 3), which also records a failure.
__global__ __launch_bounds__(kBlock) void k_inner_init(CgArgs<float> a, int round,
                                                       double refine_rtol) {
  __shared__ double sh[17];
  if (a.ctr->stop) return;
  if (round > 0 && a.sc->ref_done) return;  // an earlier round met the tolerance
  SolveScalars *sc = a.sc;
  const double rr = sum_partials(a.partial + 2 * a.grid, a.grid, sh);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (round == 0) {
    const double bb = sum_partials(a.partial + 3 * a.grid, a.grid, sh);
    const double tol2 = refine_rtol * refine_rtol * bb;
    const bool met = rr <= tol2;
    if (lead) {
      sc->ref_bb = bb;
      sc->ref_tol2 = tol2;
      sc->ref_done = met ? 1 : 0;
      sc->ref_rounds = 0;
      sc->done = 0;
      a.ctr->slot_iters[a.slot] = 0;  // largest inner iteration count of the solve
      if (met) a.ctr->slot_rounds[a.slot] = 0;
    }
    if (met) return;
  } else {
    const bool met = rr <= sc->ref_tol2;
    if (lead) {
      sc->ref_rounds = round;
      a.ctr->refine_steps += 1;
      if (met) {
        sc->ref_done = 1;
        a.ctr->slot_rounds[a.slot] = round;
      }
    }
    if (met) return;
  }
  double v[2] = {0.0, 0.0};
  const Span sp = xcd_rows(a.N);
  for (int64_t i = sp.first; i < sp.end; i += sp.step) {
    const float r = (float)a.r64[i];
    const float z = a.dinv[i] * r;
    a.r[i] = r;
    a.x[i] = 0.0f;
    a.p[i] = z;
    if (a.u) a.u[i] = z;
    v[0] += (double)r * (double)z;
    v[1] += (double)r * (double)r;
  }
  publish<2>(v, a.partial, a.grid, sh);
}

// FP64 operator on an FP32 vector through the packed entries
__device__ inline double sell_row_pk_mixed(const SellDev &op, int64_t s, int lane, int64_t row,
                                           const float *__restrict__ x, const double *sd) {
  const int64_t end = op.off[s + 1];
  int64_t e = op.off[s] + lane;
  double acc = 0.0;
#pragma unroll 4
  for (; e < end; e += kSlice) {
    const int w = op.pk16[e];
    acc += sd[w & 15] * (double)x[row + (w >> 4)];
  }
  return acc;
}

// FP64 operator on an FP32 vector through the row forms (the same products
// and order as the packed entries)
__device__ inline double sell_row_cls_mixed(const SellDev &op, int64_t row, int c,
                                            const float *__restrict__ x, const double *sd,
                                            const int *sct, const int *slen) {
  const int n = slen[c];
  const int *t = sct + c * op.cw;
  double acc = 0.0;
#pragma unroll 8
  for (int k = 0; k < n; ++k) {
    const int w = t[k];
    acc += sd[w & 255] * (double)x[row + (w >> 8)];
  }
  return acc;
}

// x64 += d; r64 -= A d (FP64 operator); ||r64|| -> refinement converged?
// CLS: row forms (tables staged once per block).  chk_it >= 0: block 0 first
// takes over the check of the inner solve after its launch budget.
template <bool D16, bool PK = false, bool CLS = false>
__global__ __launch_bounds__(kBlock) void k_refine_update(CgArgs<float> a, const double *mass64,
                                                          int chk_it) {
  __shared__ double sh[17];
  if (chk_it >= 0 && blockIdx.x == 0) cg_check_block(a, chk_it, sh);
  if (a.sc->ref_done || a.ctr->stop) return;
  __shared__ double sd[CLS ? kDictMax : (PK ? 16 : 1)];
  __shared__ int sct[CLS ? kMaxCls * kMaxClsWidth : 1];
  __shared__ int slen[CLS ? kMaxCls : 1];
  if (CLS) {
    stage_forms<double>(a.op, sd, sct, slen);
  } else if (PK) {
    if (threadIdx.x < a.op.ndict) sd[threadIdx.x] = a.op.vdict[threadIdx.x];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const Span sp = xcd_slices(a.op.nslices);
  double v[1] = {0.0};
  for (int64_t s = sp.first; s < sp.end; s += sp.step) {
    const int64_t row = s * kSlice + lane;
    if (row >= a.N) continue;
    const double d = (double)a.x[row];
    const double Ld = CLS  ? sell_row_cls_mixed(a.op, row, a.op.rcls[row], a.x, sd, sct, slen)
                      : PK ? sell_row_pk_mixed(a.op, s, lane, row, a.x, sd)
                           : sell_row_mixed<D16>(a.op, s, lane, row, a.x);
    const double Ad = mass64[row] * d + a.dtau * Ld;
    a.x64[row] += d;
    const double r = a.r64[row] - Ad;
    a.r64[row] = r;
    v[0] += r * r;
  }
  publish<1>(v, a.partial + 2 * a.grid, a.grid, sh);  // slot 2: r.r
}

static CgArgs<double> cg64(const DevState &d, int m, int slot) {
  CgArgs<double> a;
  a.init_fold = 0;
  a.init_rtol = 0.0;
  a.early_stop = d.sweep_tol > 0.0 ? 1 : 0;
  a.op = d.op;
  a.N = d.N;
  a.dtau = d.dtau_h[m];
  a.mass = d.mass;
  a.dinv = d.dinv[m];
  a.g = d.g;
  a.x = d.T[m];
  a.r = d.r;
  a.p = d.p;
  a.q = d.q;
  a.u = d.u;
  a.s = d.s;
  a.partial = d.partial;
  a.sc = d.sc;
  a.ctr = d.ctr;
  a.slot = slot;
  a.grid = d.grid;
  a.inner = 0;
  a.x64 = d.T[m];
  a.b64 = nullptr;
  a.r64 = nullptr;
  a.Tprev = d.T[m - 1];
  a.F = d.F[m];
  a.I = d.I[m];
  a.m = m;
  const bool cpl = d.single_rate && d.ifc.kind && d.ifc.n_if > 0;
  a.ifpos = cpl ? d.ifpos : nullptr;
  a.ifc_lin = cpl ? d.ifc_lin : nullptr;
  a.ifc_src = cpl ? d.ifc_src : nullptr;
  return a;
}

static CgArgs<float> cg32(const DevState &d, int m, int slot) {
  CgArgs<float> a;
  a.init_fold = 0;
  a.init_rtol = 0.0;
  a.early_stop = d.sweep_tol > 0.0 ? 1 : 0;
  a.op = d.op;
  a.N = d.N;
  a.dtau = d.dtau_h[m];
  a.mass = d.mass32;
  a.dinv = d.dinv32[m];
  a.g = d.g;
  a.x = d.x32;
  a.r = d.r32;
  a.p = d.p32;
  a.q = d.q32;
  a.u = d.u32;
  a.s = d.s32;
  a.partial = d.partial;
  a.sc = d.sc;
  a.ctr = d.ctr;
  a.slot = slot;
  a.grid = d.grid;
  a.inner = 1;
  a.x64 = d.T[m];
  a.b64 = d.b64;
  a.r64 = d.r64;
  a.Tprev = d.T[m - 1];
  a.F = d.F[m];
  a.I = d.I[m];
  a.m = m;
  a.ifpos = nullptr;
  a.ifc_lin = nullptr;
  a.ifc_src = nullptr;
  return a;
}

static void solve_reduce(const DevState &d, int slot, int mode, double rtol, int round,
                         bool last_round, hipStream_t st) {
  k_solve_reduce<<<1, kBlock, 0, st>>>(d.partial, d.grid, d.sc, d.ctr, slot, mode, rtol, round,
                                       last_round ? 1 : 0);
}

void launch_init_pred(const DevState &d, int m, int slot, double rtol, hipStream_t st) {
  CgArgs<double> a = cg64(d, m, slot);
  if (a.ifc_lin) launch_iface_lin(d, m, d.T[m - 1], st);  // coupling of A x0 and its source
  if (d.op.rcls) k_init_pred<true, false, true><<<d.grid, kBlock, 0, st>>>(a);
  else if (d.op.pk16) k_init_pred<true, true><<<d.grid, kBlock, 0, st>>>(a);
  else if (d.op.d16) k_init_pred<true><<<d.grid, kBlock, 0, st>>>(a);
  else k_init_pred<false><<<d.grid, kBlock, 0, st>>>(a);
  (void)rtol;  // the solve's scalars are formed by its first operator step
}

void launch_init_corr(const DevState &d, int m, int slot, double rtol, hipStream_t st) {
  const CgArgs<double> a = cg64(d, m, slot);
  if (a.ifc_src) launch_iface_lin(d, m, d.T[m], st);  // the coupling source at tau_m
  k_init_corr<<<d.grid, kBlock, 0, st>>>(a);
  (void)rtol;  // the solve's scalars are formed by its first operator step
}

template <typename R>
static void pcg_iter(const DevState &d, const CgArgs<R> &a, int it, bool last, bool tail,
                     hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  // with events: the dispatch's own start/end timestamps (AMD launch extension)
  auto kern = d.op.d16 ? (tail ? k_pcg_a<true, 1, R> : k_pcg_a<true, 0, R>)
                       : (tail ? k_pcg_a<false, 1, R> : k_pcg_a<false, 0, R>);
  if (d.op.rcls)
    kern = tail ? k_pcg_a<true, 1, R, false, 3> : k_pcg_a<true, 0, R, false, 3>;
  else if (d.op.pk16)
    kern = tail ? k_pcg_a<true, 1, R, false, 2> : k_pcg_a<true, 0, R, false, 2>;
  else if (d.op.vid)
    kern = d.op.d16 ? (tail ? k_pcg_a<true, 1, R, false, 1> : k_pcg_a<true, 0, R, false, 1>)
                    : (tail ? k_pcg_a<false, 1, R, false, 1> : k_pcg_a<false, 0, R, false, 1>);
  if (a.ifc_lin)
    kern = d.op.d16 ? (tail ? k_pcg_a<true, 1, R, true> : k_pcg_a<true, 0, R, true>)
                    : (tail ? k_pcg_a<false, 1, R, true> : k_pcg_a<false, 0, R, true>);
  if (a.ifc_lin) launch_iface_lin(d, a.m, (const double *)a.p, st);  // coupling of A p
  if (ev0) hipExtLaunchKernelGGL(kern, dim3(d.grid), dim3(kBlock), 0, st, ev0, ev1, 0, a, it);
  else kern<<<d.grid, kBlock, 0, st>>>(a, it);
  k_pcg_b<R><<<d.grid, kBlock, 0, st>>>(a, it);
  k_pcg_c<R><<<d.grid, kBlock, 0, st>>>(a, it, last ? 1 : 0);
}

// One iteration of the single-reduction form: operator step, then update.
template <typename R>
static void pcg2_iter(const DevState &d, const CgArgs<R> &a, int it, bool tail, hipStream_t st,
                      hipEvent_t ev0, hipEvent_t ev1) {
  void (*kern)(CgArgs<R>, int);
  if (a.ifc_lin)
    kern = d.op.d16 ? (tail ? k_pcg_a<true, 1, R, true, 0, true> : k_pcg_a<true, 0, R, true, 0, true>)
                    : (tail ? k_pcg_a<false, 1, R, true, 0, true> : k_pcg_a<false, 0, R, true, 0, true>);
  else if (d.op.rcls)
    kern = tail ? k_pcg_a<true, 1, R, false, 3, true> : k_pcg_a<true, 0, R, false, 3, true>;
  else if (d.op.pk16)
    kern = tail ? k_pcg_a<true, 1, R, false, 2, true> : k_pcg_a<true, 0, R, false, 2, true>;
  else if (d.op.vid)
    kern = d.op.d16 ? (tail ? k_pcg_a<true, 1, R, false, 1, true> : k_pcg_a<true, 0, R, false, 1, true>)
                    : (tail ? k_pcg_a<false, 1, R, false, 1, true> : k_pcg_a<false, 0, R, false, 1, true>);
  else
    kern = d.op.d16 ? (tail ? k_pcg_a<true, 1, R, false, 0, true> : k_pcg_a<true, 0, R, false, 0, true>)
                    : (tail ? k_pcg_a<false, 1, R, false, 0, true> : k_pcg_a<false, 0, R, false, 0, true>);
  if (a.ifc_lin) launch_iface_lin(d, a.m, (const double *)a.u, st);  // coupling of A u
  if (ev0) hipExtLaunchKernelGGL(kern, dim3(d.grid), dim3(kBlock), 0, st, ev0, ev1, 0, a, it);
  else kern<<<d.grid, kBlock, 0, st>>>(a, it);
  k_cg_upd<R><<<d.grid, kBlock, 0, st>>>(a, it);
}

void launch_pcg_iter(const DevState &d, int m, int slot, int it, bool last, bool tail,
                     double rtol, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  (void)last;  // the budget's end is judged by launch_pcg_final
  CgArgs<double> a = cg64(d, m, slot);
  a.init_fold = 1;
  a.init_rtol = rtol;
  pcg2_iter(d, a, it, tail, st, ev0, ev1);
}

void launch_pcg_final(const DevState &d, int m, int slot, int it, bool fp32, hipStream_t st) {
  if (fp32) k_cg_check<float><<<1, kBlock, 0, st>>>(cg32(d, m, slot), it);
  else k_cg_check<double><<<1, kBlock, 0, st>>>(cg64(d, m, slot), it);
}

// Stationary field (K + h R) T = g: the CG kernels with a zero mass, dtau = 1
// and the Jacobi inverse of L, on T_n in place.
static CgArgs<double> stationary_args(const DevState &d, const double *zeros, const double *dinv,
                                      int slot) {
  CgArgs<double> a = cg64(d, 1, slot);
  a.mass = zeros;
  a.dinv = dinv;
  a.dtau = 1.0;
  a.x = d.T[0];
  a.x64 = d.T[0];
  a.Tprev = d.T[0];
  a.g = d.g;
  a.ifpos = nullptr;  // conduction and Robin part only
  a.ifc_lin = nullptr;
  a.ifc_src = nullptr;
  return a;
}

void launch_stationary_init(const DevState &d, const double *zeros, const double *dinv, int slot,
                            double rtol, hipStream_t st) {
  const CgArgs<double> a = stationary_args(d, zeros, dinv, slot);
  if (d.op.rcls) k_init_pred<true, false, true><<<d.grid, kBlock, 0, st>>>(a);
  else if (d.op.pk16) k_init_pred<true, true><<<d.grid, kBlock, 0, st>>>(a);
  else if (d.op.d16) k_init_pred<true><<<d.grid, kBlock, 0, st>>>(a);
  else k_init_pred<false><<<d.grid, kBlock, 0, st>>>(a);
  solve_reduce(d, slot, 0, rtol, 0, false, st);
}

void launch_stationary_iters(const DevState &d, const double *zeros, const double *dinv, int slot,
                             int it0, int n, int last_it, hipStream_t st) {
  const CgArgs<double> a = stationary_args(d, zeros, dinv, slot);
  for (int it = it0; it < it0 + n; ++it)
    pcg_iter(d, a, it, it == last_it, false, st, nullptr, nullptr);
}

// reps back-to-back operator applications q = A p of interval m (timing only;
// p holds the last solve's direction, q and the partials are scratch)
void launch_operator_timing(const DevState &d, int m, bool fp32, int reps, hipStream_t st) {
  if (fp32) {
    CgArgs<float> a = cg32(d, m, 0);
    for (int i = 0; i < reps; ++i) {
      if (d.op.rcls) k_pcg_a<true, 2, float, false, 3, true><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.pk16) k_pcg_a<true, 2, float, false, 2><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.vid && d.op.d16) k_pcg_a<true, 2, float, false, 1><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.vid) k_pcg_a<false, 2, float, false, 1><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.d16) k_pcg_a<true, 2, float><<<d.grid, kBlock, 0, st>>>(a, 0);
      else k_pcg_a<false, 2, float><<<d.grid, kBlock, 0, st>>>(a, 0);
    }
  } else {
    CgArgs<double> a = cg64(d, m, 0);
    a.x = nullptr;
    for (int i = 0; i < reps; ++i) {
      if (d.op.rcls) k_pcg_a<true, 2, double, false, 3, true><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.pk16) k_pcg_a<true, 2, double, false, 2><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.vid && d.op.d16) k_pcg_a<true, 2, double, false, 1><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.vid) k_pcg_a<false, 2, double, false, 1><<<d.grid, kBlock, 0, st>>>(a, 0);
      else if (d.op.d16) k_pcg_a<true, 2, double><<<d.grid, kBlock, 0, st>>>(a, 0);
      else k_pcg_a<false, 2, double><<<d.grid, kBlock, 0, st>>>(a, 0);
    }
  }
}

void launch_refine_init(const DevState &d, int m, int slot, bool pred, double rtol,
                        hipStream_t st) {
  CgArgs<float> a = cg32(d, m, slot);
  if (d.op.pk16) {
    if (pred) k_rinit<true, true, true><<<d.grid, kBlock, 0, st>>>(a, d.mass);
    else k_rinit<true, false, true><<<d.grid, kBlock, 0, st>>>(a, d.mass);
  } else if (d.op.d16) {
    if (pred) k_rinit<true, true><<<d.grid, kBlock, 0, st>>>(a, d.mass);
    else k_rinit<true, false><<<d.grid, kBlock, 0, st>>>(a, d.mass);
  } else {
    if (pred) k_rinit<false, true><<<d.grid, kBlock, 0, st>>>(a, d.mass);
    else k_rinit<false, false><<<d.grid, kBlock, 0, st>>>(a, d.mass);
  }
  (void)rtol;  // the refinement's scalars are formed by the first round's inner init
}

void launch_inner_init(const DevState &d, int m, int slot, double inner_rtol, int round,
                       double refine_rtol, hipStream_t st) {
  k_inner_init<<<d.grid, kBlock, 0, st>>>(cg32(d, m, slot), round, refine_rtol);
  (void)inner_rtol;  // the inner solve's scalars are formed by its first operator step
}

void launch_pcg32_iter(const DevState &d, int m, int slot, int it, bool last, bool tail,
                       double inner_rtol, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  (void)last;
  CgArgs<float> a = cg32(d, m, slot);
  a.init_fold = 1;
  a.init_rtol = inner_rtol;
  pcg2_iter(d, a, it, tail, st, ev0, ev1);
}

void launch_refine_update(const DevState &d, int m, int slot, int round, bool last_round,
                          int chk_it, hipStream_t st) {
  CgArgs<float> a = cg32(d, m, slot);
  if (d.op.rcls) k_refine_update<true, false, true><<<d.grid, kBlock, 0, st>>>(a, d.mass, chk_it);
  else if (d.op.pk16) k_refine_update<true, true><<<d.grid, kBlock, 0, st>>>(a, d.mass, chk_it);
  else if (d.op.d16) k_refine_update<true><<<d.grid, kBlock, 0, st>>>(a, d.mass, chk_it);
  else k_refine_update<false><<<d.grid, kBlock, 0, st>>>(a, d.mass, chk_it);
  // the other rounds' checks are taken by the next round's inner init
  if (last_round) solve_reduce(d, slot, 3, 0.0, round, last_round, st);
}

// ---------------------------------------------------------------------------
// 1D face integrals of products of hat functions (separable form of the
// rectangle integrals of §2, eqs. femContFix/femContMov and defCB)
// ---------------------------------------------------------------------------
// first node c of grid y (shifted by sy) whose hat support ends after t
__device__ inline int first_hat_after(const double *y, int n, double sy, double t) {
  int lo = 0, hi = n;  // invariant: answer in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double end = y[mid < n - 1 ? mid + 1 : mid] + sy;
    if (end > t) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Embedded explicit substeps of one interval on the interface points (Alg. 1
// and Alg. 2, the inner loops over p).  Off the interface f^E vanishes, so
// those rows end the interval at T* exactly (the weights satisfy
// sum_p tilde s = s and sum_p s_pq = hat s): only interface rows are stepped.
//
// The time-dependent 1D face integrals depend only on the embedded times,
// which are the same for the predictor and every sweep of a step, so they are
// tabulated once per step for all (m, q).  Each substep is then one wide
// launch over the interface points with double-buffered interface state.
// ---------------------------------------------------------------------------
size_t coef_table_doubles(const IfaceDev &f) { return (size_t)CoefLayout{f.nvf, f.nvm}.dstride(); }
size_t coef_table_ints(const IfaceDev &f) { return (size_t)CoefLayout{f.nvf, f.nvm}.istride(); }

__device__ double motion_s(const IfaceDev &f, double t) {
  return f.s0 + f.a * sin(2.0 * M_PI * t / f.period + f.phase);
}

// One block per embedded time point tau_{m,q}: v-direction integrals over the
// v-extent of Gamma_R(t) (contact) or of the patch, and the friction density.
__global__ __launch_bounds__(kBlock) void k_iface_coeffs(IfaceDev f, const Weights *w,
                                                        const double *tn, int P,
                                                        double *coefD, int *coefI,
                                                        int nodes_only) {
  const int P1 = P + 1, tp = blockIdx.x, m = tp / P1, q = tp - m * P1;
  // nodes_only (single-rate method): the tables at the standard node times
  // tau_m = tau_{m-1} + dtau_m (q = P), degenerate first interval included
  if (nodes_only ? (m == 0 || q != P) : (m == 0 || w->dtau[m] == 0.0)) return;
  const CoefLayout L{f.nvf, f.nvm};
  double *D = coefD + (size_t)tp * L.dstride();
  int *I = coefI + (size_t)tp * L.istride();
  const double t = *tn + w->tau[m - 1] + q * (w->dtau[m] / P);
  const double s = motion_s(f, t);
  double ov0, ov1;
  if (f.kind == 1) {
    ov0 = fmax(f.vf[0], f.vm[0] + s);
    ov1 = fmin(f.vf[f.nvf - 1], f.vm[f.nvm - 1] + s);
  } else {
    ov0 = fmax(f.vf[0], s - 0.5 * f.wv);
    ov1 = fmin(f.vf[f.nvf - 1], s + 0.5 * f.wv);
  }
  const bool valid = (f.ou1 > f.ou0) && (ov1 > ov0);
  if (threadIdx.x == 0)
    D[0] = (f.kind == 1 && valid) ? f.Pf / ((f.ou1 - f.ou0) * (ov1 - ov0)) : 0.0;
  for (int b = threadIdx.x; b < f.nvf; b += blockDim.x) {
    for (int i = 0; i < 3; ++i) {
      const int bb = b - 1 + i;
      D[L.Mv() + 3 * b + i] =
          (bb >= 0 && bb < f.nvf && valid)
              ? hat_product_integral(f.vf, f.nvf, b, f.vf, f.nvf, bb, 0.0, ov0, ov1)
              : 0.0;
    }
    D[L.Hv() + b] = valid ? hat_integral(f.vf, f.nvf, b, ov0, ov1) : 0.0;
    if (f.kind == 1) {
      const int d0 = first_hat_after(f.vm, f.nvm, s, f.vf[b > 0 ? b - 1 : b]);
      int cnt = 0;
      for (int i = 0; i < kBand; ++i) {
        const int d = d0 + i;
        const double v = (d < f.nvm && valid)
                             ? hat_product_integral(f.vf, f.nvf, b, f.vm, f.nvm, d, s, ov0, ov1)
                             : 0.0;
        D[L.Cv() + kBand * b + i] = v;
        if (v != 0.0) cnt = i + 1;
      }
      I[L.dlo() + b] = d0;
      I[L.dcnt() + b] = cnt;
    }
  }
  if (f.kind == 1) {
    for (int d = threadIdx.x; d < f.nvm; d += blockDim.x) {
      for (int i = 0; i < 3; ++i) {
        const int dd = d - 1 + i;
        D[L.Nv() + 3 * d + i] = (dd >= 0 && dd < f.nvm && valid)
                                    ? hat_product_integral(f.vm, f.nvm, d, f.vm, f.nvm, dd, 0.0,
                                                           ov0 - s, ov1 - s)
                                    : 0.0;
      }
      D[L.Gv() + d] = valid ? hat_integral(f.vm, f.nvm, d, ov0 - s, ov1 - s) : 0.0;
      const int b0 = first_hat_after(f.vf, f.nvf, 0.0, f.vm[d > 0 ? d - 1 : d] + s);
      int cnt = 0;
      for (int i = 0; i < kBand; ++i) {
        const int b = b0 + i;
        const double v = (b < f.nvf && valid)
                             ? hat_product_integral(f.vf, f.nvf, b, f.vm, f.nvm, d, s, ov0, ov1)
                             : 0.0;
        D[L.CvT() + kBand * d + i] = v;
        if (v != 0.0) cnt = i + 1;
      }
      I[L.blo() + d] = b0;
      I[L.bcnt() + d] = cnt;
    }
  }
}

struct SubArgs {
  IfaceDev f;
  const StepCounters *ctr;
  const Weights *w;
  int m, p, P, M, corr;
  const double *coefD;
  const int *coefI;
  const double *mass;
  const double *Tprev;
  double *Tm;
  const double *Im;
  const double *F[kMaxM + 1];
  const double *Eold;  // [(M+1)(P+1) n_if]
  double *Enew;
  double *Ipre;        // [(M+1)(P+1) n_if] embedded quadratures of the sweep
  double *Tbuf[2];
  double *fst;
  // first substep only: f^E at tau_{m-1} with the previous interval's table
  // (its q = P value; prev_m = 0: none) and the check after the node solve's
  // launch budget (chk_it < 0: none)
  int prev_m;
  int chk_it;
  CgArgs<double> chk;
};

// interface state: on the first substep T_{m,0} = T_{m-1} is read from the
// full vector, afterwards from the interface buffer of the previous substep
template <bool FIRST>
__device__ inline double tif(const SubArgs &A, const double *Tin, int j) {
  return FIRST ? A.Tprev[A.f.rows[j]] : Tin[j];
}

// Separable coupling sums of one interface point.  The 3 x 3 self stencil
// and, when both band counts are at most kFastBand, the cross band are formed
// with fixed trip counts: indices are clamped into the face grid and the
// weights of the clamped terms are zero, so every gather is issued before the
// first is waited for.  A point whose band is wider takes the general loop.
// Every sum adds the same products in the same order as the plain loops
// (a clamped term adds an exact zero).
constexpr int kFastBand = 4;
static_assert(kFastBand <= kBand, "the fast cross band reads kFastBand table entries per point");

template <bool FIRST>
__device__ inline double self_sum(const SubArgs &A, const double *Tin, const double *wu,
                                  const double *wv, int nu, int nv, int base, int a, int b) {
  // (the weights are read unconditionally, their tables hold 3 per point,
  // and masked when used, so no load waits on a branch)
  double w0[3], w1[3];
  int ra[3], cb[3];
  bool ia[3], ib[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int aa = a - 1 + q, bb = b - 1 + q;
    ia[q] = aa >= 0 && aa < nu;
    ib[q] = bb >= 0 && bb < nv;
    ra[q] = ia[q] ? aa : a;
    cb[q] = ib[q] ? bb : b;
    w0[q] = wu[3 * a + q];
    w1[q] = wv[3 * b + q];
  }
  double t[3][3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int r = 0; r < 3; ++r) t[q][r] = tif<FIRST>(A, Tin, base + ra[q] * nv + cb[r]);
  double self = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) acc += (ib[r] ? w1[r] : 0.0) * t[q][r];
    self += (ia[q] ? w0[q] : 0.0) * acc;
  }
  return self;
}

// sum_{i < nu} cu[i] sum_{j < nv} cv[j] T(base + (u0 + i) * ld + v0 + j)
template <bool FIRST>
__device__ inline double cross_sum(const SubArgs &A, const double *Tin, const double *cu,
                                   const double *cv, int u0, int nu, int v0, int nv, int ld,
                                   int base) {
  double cross = 0.0;
  if (nu <= 0 || nv <= 0) return cross;  // no overlap: the band start may lie off the grid
  if (nu <= kFastBand && nv <= kFastBand) {
    // (band tables hold kBand >= kFastBand weights per point: read
    // unconditionally, masked when used)
    double wu[kFastBand], wv[kFastBand], t[kFastBand][kFastBand];
#pragma unroll
    for (int q = 0; q < kFastBand; ++q) {
      wu[q] = cu[q];
      wv[q] = cv[q];
    }
#pragma unroll
    for (int q = 0; q < kFastBand; ++q)
#pragma unroll
      for (int r = 0; r < kFastBand; ++r)
        t[q][r] = tif<FIRST>(A, Tin, base + (u0 + (q < nu ? q : 0)) * ld + v0 + (r < nv ? r : 0));
#pragma unroll
    for (int q = 0; q < kFastBand; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < kFastBand; ++r) acc += (r < nv ? wv[r] : 0.0) * t[q][r];
      cross += (q < nu ? wu[q] : 0.0) * acc;
    }
    return cross;
  }
  for (int q = 0; q < nu; ++q) {
    double acc = 0.0;
    for (int r = 0; r < nv; ++r) acc += cv[r] * tif<FIRST>(A, Tin, base + (u0 + q) * ld + v0 + r);
    cross += cu[q] * acc;
  }
  return cross;
}

// f^E at interface point i (fixed-face points first, then moving-face points)
// as the part linear in T (exchange) and the source (friction, patch flux)
template <bool FIRST>
__device__ void iface_fE_parts(const SubArgs &A, const double *D, const int *I,
                               const double *Tin, int i, double *lin, double *src) {
  const IfaceDev &f = A.f;
  const CoefLayout L{f.nvf, f.nvm};
  const double qf = D[0];
  if (i < f.nfix) {
    const int a = i / f.nvf, b = i - a * f.nvf;
    const double self = self_sum<FIRST>(A, Tin, f.Mu, D + L.Mv(), f.nuf, f.nvf, 0, a, b);
    const double hub = f.Hu[a] * D[L.Hv() + b];
    if (f.kind == 2) {
      *lin = -(f.alpha * self);
      *src = (f.q0 + f.alpha * f.Tfix) * hub;
      return;
    }
    const double cross =
        cross_sum<FIRST>(A, Tin, f.Cu + kBand * a, D + L.Cv() + kBand * b, f.clo[a], f.ccnt[a],
                         I[L.dlo() + b], I[L.dcnt() + b], f.nvm, f.nfix);
    *lin = f.alpha * (cross - self);
    *src = f.split * qf * hub;
    return;
  }
  const int k = i - f.nfix;
  const int c = k / f.nvm, d = k - c * f.nvm;
  const double self = self_sum<FIRST>(A, Tin, f.Nu, D + L.Nv(), f.num, f.nvm, f.nfix, c, d);
  const double cross =
      cross_sum<FIRST>(A, Tin, f.CuT + kBand * c, D + L.CvT() + kBand * d, f.alo[c], f.acnt[c],
                       I[L.blo() + d], I[L.bcnt() + d], f.nvf, 0);
  *lin = f.alpha * (cross - self);
  *src = (1.0 - f.split) * qf * f.Gu[c] * D[L.Gv() + d];
}

template <bool FIRST>
__device__ double iface_fE(const SubArgs &A, const double *D, const int *I, const double *Tin,
                           int i) {
  double lin, src;
  iface_fE_parts<FIRST>(A, D, I, Tin, i, &lin, &src);
  return src + lin;
}

// Substep p of interval m; p = P also writes T^{k+1}_m <- T_{m,P} back.
// p = P+1 (last interval only): f^E at tau_m.  The other intervals' f^E at
// their end point is formed by the next interval's first substep, from the
// same state with the same table.  The first substep launch also takes over
// the convergence check of the node solve it follows (block 0).
//
// The launch has kXcd workgroups per point block and only those on XCD 0
// (b % kXcd == 0) work, so the substeps' state (the interface buffers, the
// f^E cache and the coefficient tables) stays in one L2 from launch to
// launch.
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void k_iface_sub(SubArgs A) {
  if (blockIdx.x % kXcd) return;
  const int bx = blockIdx.x / kXcd;
  if (FIRST && A.chk_it >= 0 && bx == 0) {
    __shared__ double sh[17];
    cg_check_block(A.chk, A.chk_it, sh);
  }
  if (A.ctr->stop) return;
  const int i = bx * blockDim.x + threadIdx.x;
  const IfaceDev &f = A.f;
  const int n = f.n_if;
  if (i >= n) return;
  const Weights &w = *A.w;
  const int m = A.m, p = A.p, P = A.P, P1 = P + 1;
  const CoefLayout L{f.nvf, f.nvm};
  const int tp = m * P1 + (p - 1);
  const double *D = A.coefD + (size_t)tp * L.dstride();
  const int *I = A.coefI + (size_t)tp * L.istride();
  const double *Tin = A.Tbuf[(p - 1) & 1];
  const double E = iface_fE<FIRST>(A, D, I, Tin, i);
  double *En = A.Enew + (size_t)m * P1 * n;
  En[(size_t)(p - 1) * n + i] = E;
  if (FIRST && A.prev_m > 0) {
    const int tq = A.prev_m * P1 + P;
    A.Enew[((size_t)A.prev_m * P1 + P) * n + i] =
        iface_fE<true>(A, A.coefD + (size_t)tq * L.dstride(), A.coefI + (size_t)tq * L.istride(),
                       Tin, i);
  }
  const double Ti = tif<FIRST>(A, Tin, i);
  const int64_t row = f.rows[i];
  if (p == P + 1) {
    A.Tm[row] = Ti;  // T^{k+1}_m <- T_{m,P} (already written by substep P)
    return;
  }
  const double mi = A.mass[row], dtm = w.dtau[m], dtp = dtm / P;
  double fs;
  if (FIRST) {
    // dtau f*_m recovered from the solve: M T* - M T_{m-1} (- I_m)
    fs = (mi * A.Tm[row] - mi * Ti - (A.corr ? A.Im[row] : 0.0)) / dtm;
    A.fst[i] = fs;
  } else {
    fs = A.fst[i];
  }
  double inc;
  if (A.corr) {
    const double *Eo = A.Eold + (size_t)m * P1 * n;
    const double Ip = A.Ipre[((size_t)m * P1 + p) * n + i];
    inc = dtp * (fs + E - Eo[(size_t)(p - 1) * n + i]) + Ip;
  } else {
    inc = dtp * (fs + E);
  }
  const double Tn = Ti + inc / mi;
  A.Tbuf[p & 1][i] = Tn;
  if (p == P) A.Tm[row] = Tn;  // T^{k+1}_m <- T_{m,P}
}

void launch_iface_coeffs(const DevState &d, hipStream_t st) {
  if (!d.ifc.kind || d.ifc.n_if == 0) return;
  k_iface_coeffs<<<(d.M + 1) * (d.P + 1), kBlock, 0, st>>>(d.ifc, d.w, d.tn, d.P, d.coefD,
                                                           d.coefI, d.single_rate);
}

// ---------------------------------------------------------------------------
// single-rate method: the coupling at the standard node times, in the
// implicit part.  MODE 0: F[m] += f^E(x, tau_m) on the interface rows (the
// node values of the quadrature); MODE 1: ifc_lin = -dtau_m (exchange part
// of f^E(x, tau_m)) = dtau_m A_c(tau_m) x and ifc_src = dtau_m (source part).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_iface_node(SubArgs A, double dtau, double *F,
                                                       double *lin, double *src) {
  // node values stay whole after residual control ends the sweeps: the
  // residual of the last iterate is still evaluated from them
  if (MODE == 1 && A.ctr->stop) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.f.n_if) return;
  const CoefLayout L{A.f.nvf, A.f.nvm};
  const int tp = A.m * (A.P + 1) + A.P;
  const double *D = A.coefD + (size_t)tp * L.dstride();
  const int *I = A.coefI + (size_t)tp * L.istride();
  double el, es;
  iface_fE_parts<true>(A, D, I, nullptr, i, &el, &es);
  if (MODE == 0) {
    F[A.f.rows[i]] += es + el;
  } else {
    lin[i] = -(dtau * el);
    src[i] = dtau * es;
  }
}

static SubArgs node_args(const DevState &d, int m, const double *x) {
  SubArgs A{};
  A.f = d.ifc;
  A.ctr = d.ctr;
  A.w = d.w;
  A.m = m;
  A.P = d.P;
  A.M = d.M;
  A.coefD = d.coefD;
  A.coefI = d.coefI;
  A.Tprev = x;
  return A;
}

void launch_iface_F(const DevState &d, int j, hipStream_t st) {
  if (!d.ifc.kind || d.ifc.n_if == 0) return;
  const int grid = (d.ifc.n_if + kBlock - 1) / kBlock;
  k_iface_node<0><<<grid, kBlock, 0, st>>>(node_args(d, j, d.T[j]), 0.0, d.F[j], nullptr,
                                           nullptr);
}

void launch_iface_lin(const DevState &d, int m, const double *x, hipStream_t st) {
  if (!d.ifc.kind || d.ifc.n_if == 0) return;
  const int grid = (d.ifc.n_if + kBlock - 1) / kBlock;
  k_iface_node<1><<<grid, kBlock, 0, st>>>(node_args(d, m, x), d.dtau_h[m], nullptr, d.ifc_lin,
                                           d.ifc_src);
}

// Embedded quadratures I_{m,p} (eq. embedded_quad) of the interface rows for
// every interval and substep of a sweep: they depend only on the previous
// iterate (F_j at the sweep start, the previous sweep's E cache), so one pass
// at the sweep start replaces M + P scattered loads per point and substep.
// (restrict-qualified weights, cache and output: the weights are read
// through the scalar cache, and every operand of a point is loaded before its
// first store)
__global__ __launch_bounds__(kBlock) void k_iface_quad(SubArgs A, const Weights *__restrict__ wp,
                                                       const double *__restrict__ Eold,
                                                       double *__restrict__ Ipre) {
  if (A.ctr->stop) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = A.f.n_if;
  if (i >= n) return;
  const Weights &w = *wp;
  const int P = A.P, P1 = P + 1;
  const int m = blockIdx.y + 1;  // one interval per grid row
  if (w.dtau[m] == 0.0) return;
  const int64_t row = A.f.rows[i];
  const double *Eo = Eold + (size_t)m * P1 * n;
  // loads at clamped indices (no branch between them), zero past M and P
  double F[kMaxM + 1], E[kMaxP + 1];
#pragma unroll
  for (int j = 1; j <= kMaxM; ++j) {
    const double v = A.F[j <= A.M ? j : 1][row];
    F[j] = j <= A.M ? v : 0.0;
  }
#pragma unroll
  for (int q = 1; q <= kMaxP; ++q) {
    const double v = Eo[(size_t)(q <= P ? q : P) * n + i];
    E[q] = q <= P ? v : 0.0;
  }
  for (int p = 1; p <= P; ++p) {
    double Ip = 0.0;
#pragma unroll
    for (int j = 1; j <= kMaxM; ++j)
      if (j <= A.M) Ip += w.stil[m][p][j] * F[j];
#pragma unroll
    for (int q = 1; q <= kMaxP; ++q)
      if (q <= P) Ip += w.spq[m][p][q] * E[q];
    Ipre[((size_t)m * P1 + p) * n + i] = Ip;
  }
}

void launch_iface_quad(const DevState &d, hipStream_t st) {
  if (!d.ifc.kind || d.ifc.n_if == 0) return;
  SubArgs A{};
  A.f = d.ifc;
  A.ctr = d.ctr;
  A.w = d.w;
  A.P = d.P;
  A.M = d.M;
  for (int j = 0; j <= kMaxM; ++j) A.F[j] = d.F[j];
  A.Eold = d.Eold;
  A.Ipre = d.Ipre;
  k_iface_quad<<<dim3((d.ifc.n_if + kBlock - 1) / kBlock, d.M), kBlock, 0, st>>>(A, d.w, d.Eold,
                                                                                 d.Ipre);
}

void launch_iface(const DevState &d, int m, bool corr, int slot, int chk_it, hipStream_t st) {
  if (!d.ifc.kind || d.ifc.n_if == 0) {
    if (chk_it >= 0) launch_pcg_final(d, m, slot, chk_it, false, st);
    return;
  }
  SubArgs A;
  A.f = d.ifc;
  A.ctr = d.ctr;
  A.w = d.w;
  A.m = m;
  A.P = d.P;
  A.M = d.M;
  A.corr = corr ? 1 : 0;
  A.coefD = d.coefD;
  A.coefI = d.coefI;
  A.mass = d.mass;
  A.Tprev = d.T[m - 1];
  A.Tm = d.T[m];
  A.Im = d.I[m];
  for (int j = 0; j <= kMaxM; ++j) A.F[j] = d.F[j];
  A.Eold = d.Eold;
  A.Enew = d.Enew;
  A.Ipre = d.Ipre;
  A.Tbuf[0] = d.Tbuf[0];
  A.Tbuf[1] = d.Tbuf[1];
  A.fst = d.fst;
  A.prev_m = (m > 1 && d.dtau_h[m - 1] != 0.0) ? m - 1 : 0;
  A.chk_it = chk_it;
  A.chk = cg64(d, m, slot);
  const int grid = (d.ifc.n_if + kBlock - 1) / kBlock;
  const int last = m == d.M ? d.P + 1 : d.P;
  for (int p = 1; p <= last; ++p) {
    A.p = p;
    if (p == 1) k_iface_sub<true><<<grid * kXcd, kBlock, 0, st>>>(A);
    else k_iface_sub<false><<<grid * kXcd, kBlock, 0, st>>>(A);
  }
}

// ---------------------------------------------------------------------------
// step end: T_n <- T_M, t_n += dt
// ---------------------------------------------------------------------------
__global__ void k_copy(double *dst, const double *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
// commit the step only if every solve converged within its launch budget
__global__ void k_commit(double *dst, const double *src, int64_t n, const StepCounters *ctr) {
  if (ctr->fail) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_time(double *tn, double dt, const StepCounters *ctr) {
  if (threadIdx.x == 0 && !ctr->fail) *tn += dt;
}
__global__ void k_clear(StepCounters *ctr) {
  int *p = reinterpret_cast<int *>(ctr);
  for (int i = threadIdx.x; i < (int)(sizeof(StepCounters) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

void launch_copy(double *dst, const double *src, int64_t n, hipStream_t st) {
  int grid = (int)((n + kBlock - 1) / kBlock);
  if (grid > 2048) grid = 2048;
  if (grid < 1) grid = 1;
  k_copy<<<grid, kBlock, 0, st>>>(dst, src, n);
}

void launch_step_end(const DevState &d, double dt, hipStream_t st) {
  int grid = (int)((d.N + kBlock - 1) / kBlock);
  if (grid > 2048) grid = 2048;
  k_commit<<<grid, kBlock, 0, st>>>(d.T[0], d.T[d.M], d.N, d.ctr);
  k_time<<<1, 64, 0, st>>>(d.tn, dt, d.ctr);
}

void launch_clear_counters(const DevState &d, hipStream_t st) {
  k_clear<<<1, kBlock, 0, st>>>(d.ctr);
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free stationary solve: the Jacobi
// inverse of L and a zero mass vector, MRSDC_NOALLOC_MAX_ROWS values each
// (64 MiB).  Each device the library runs on holds its own copy until the
// process ends; every call on a device shares it and leaves its contents.
// Host code reaches it only through the address hipGetSymbolAddress returns
// for that device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[2 * (size_t)MRSDC_NOALLOC_MAX_ROWS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t stationary_scratch(int device, double **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {  // first call on this device (the caller made it current)
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<double *>(p);
  }
  *ptr = g_scratch[device];
  return hipSuccess;
}

__global__ void k_stationary_scratch(double *__restrict__ dinv, double *__restrict__ zeros,
                                     const double *__restrict__ Ldiag, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    dinv[i] = 1.0 / Ldiag[i];
    zeros[i] = 0.0;
  }
}

void launch_stationary_scratch(double *dinv, double *zeros, const double *Ldiag, int64_t n,
                               hipStream_t st) {
  int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 2048);
  if (grid < 1) grid = 1;
  k_stationary_scratch<<<grid, kBlock, 0, st>>>(dinv, zeros, Ldiag, n);
}

}  // namespace mrsdc
