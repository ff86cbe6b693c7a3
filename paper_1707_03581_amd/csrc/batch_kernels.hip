// Batched MRSDC sweep: S scenarios (S <= 64) of one machine advanced together.
//
// The scenarios share the mesh operators K and R (per-scenario Robin h_s,
// contact alpha_s, friction power P_s and motion period), so the operator is
// applied as a multi-right-hand-side product.  Layout: every state vector is
// scenario-interleaved, X[row * S + s]; a wavefront handles one row for all
// scenarios (lane = scenario), so the row's matrix entries are wave-uniform
// (scalar loads, read once for S right-hand sides) and every vector access is
// one contiguous line.  Each scenario keeps its own CG scalars and
// convergence flag; arithmetic per scenario does not depend on the others, so
// a scenario's result is the same alone and inside any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "batch_internal.h"

namespace mrsdc {

__device__ inline double bwave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// XCD-aware row ranges: workgroups are dealt to the 8 XCDs round-robin, so
// XCD x = block % 8 walks the contiguous rows [x N/8, (x+1) N/8); stencil
// neighbours of the rows in flight then sit in that XCD's own L2.
constexpr int kXcd = 8;
struct RowRange {
  int64_t row, end, stride;
};
__device__ inline RowRange xcd_rows(int64_t N) {
  const int xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd, per = gridDim.x / kXcd;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  RowRange r;
  r.row = N * xcd / kXcd + (int64_t)local * (kBlock / 64) + w;
  r.end = N * (xcd + 1) / kXcd;
  r.stride = (int64_t)per * (kBlock / 64);
  return r;
}
// The row-parallel updates take the wave's rows (the FOR_ROWS sequence)
// kRowsAhead at a time, every load of the group issued before the first use;
// rows are still accumulated in sequence order.
constexpr int kRowsAhead = 4;

#define FOR_ROWS(row, N)                  \
  for (RowRange rr_ = xcd_rows(N); rr_.row < rr_.end; rr_.row += rr_.stride) \
    if (const int64_t row = rr_.row; true)

// Tiles of the LDS-staged kernels, dealt the same way: XCD x walks the
// contiguous tiles [x T/8, (x+1) T/8), its workgroups side by side.
struct TileRange {
  int t, end, stride;
};
__device__ inline TileRange xcd_tiles(int T) {
  const int xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd, per = gridDim.x / kXcd;
  TileRange r;
  r.t = (int)((int64_t)T * xcd / kXcd) + local;
  r.end = (int)((int64_t)T * (xcd + 1) / kXcd);
  r.stride = per;
  return r;
}
#define FOR_TILES(t, T)                                                        \
  for (TileRange tr_ = xcd_tiles(T); tr_.t < tr_.end; tr_.t += tr_.stride) \
    if (const int t = tr_.t; true)

// sum the per-wave (per-lane = per-scenario) values of the block into
// partial[k][s][blk]
template <int K>
__device__ inline void bpublish(double (&v)[K], double *partial, int grid, int S) {
  __shared__ double sh[kBlock / 64][K][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k = 0; k < K; ++k) sh[w][k][lane] = v[k];
  __syncthreads();
  if (w == 0 && lane < S) {
    for (int k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int ww = 0; ww < kBlock / 64; ++ww) acc += sh[ww][k][lane];
      partial[((size_t)k * S + lane) * grid + blockIdx.x] = acc;
    }
  }
}

__device__ inline double readlane_d(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <typename T>
__device__ inline T readlane_t(T v, int l);
template <>
__device__ inline double readlane_t<double>(double v, int l) {
  return readlane_d(v, l);
}
template <>
__device__ inline float readlane_t<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// one rounding per product-sum, in every kernel that forms a row of the operator
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// LDS-staged multi-RHS operator.  A workgroup takes one tile (TR consecutive
// rows) at a time: it copies the rows of x its tile reads (the union of the
// tile's columns, at most kStageSlots rows of S values) and the tile's matrix
// entries (LDS slot, value) into LDS with direct global-to-LDS loads, then
// forms the rows from LDS.  The union of a hexahedral tile is about nine
// short runs of rows, so each x row is read from L2 about nine times per
// product instead of once per matrix entry.
//
// Lane mapping ("rows per wavefront"): a lane owns VEC consecutive scenarios
// (one 16-byte LDS read: 4 FP32 or 2 FP64 staged values), LPR = 64 / VEC
// lanes cover 64 scenarios of a row, so a wave forms RPW = VEC rows at once,
// each lane walking its own row's entries (no cross-lane broadcast).  The
// mapping does not depend on S, so neither does any summation order.
// ---------------------------------------------------------------------------

template <typename XT>
struct Lanes {
  static constexpr int VEC = 16 / (int)sizeof(XT);
  static constexpr int LPR = 64 / VEC;
  static constexpr int RPW = VEC;
  // wave iterations per tile: tiles hold at most 4 kMaxR rows
  static constexpr int NI = (4 * kMaxR + 4 * RPW - 1) / (4 * RPW);
};

constexpr int kMaxEnt = kMaxTileEntries;

// LDS of a tiled kernel: staged x rows (+ a 64-value tail), the tile's
// entries (+ tail) and its slot rows
template <typename XT, typename VT>
struct StageLds {
  XT x[(kStageSlots + 1) * 64];
  int eslot[kMaxEnt + 64];
  VT eval[kMaxEnt + 64];
  int ssl[kStageSlots + 1];
};

// direct global-to-LDS copy of n contiguous 4-byte units; wave w moves units
// [base, base + 64) for base = 64 w, 64 w + 256, ...; lanes past the end
// repeat a valid unit into the tail
__device__ __attribute__((always_inline)) inline void dma_contig(const void *src, void *dst,
                                                                 int n) {
  const int lane = threadIdx.x & 63;
  const char *sb = reinterpret_cast<const char *>(src);
  char *db = reinterpret_cast<char *>(dst);
  for (int base = (threadIdx.x >> 6) * 64; base < n; base += kBlock) {
    const int u = base + lane < n ? base + lane : base;
    __builtin_amdgcn_global_load_lds((const void *)(sb + (size_t)u * 4),
                                     (__attribute__((address_space(3))) void *)(db + (size_t)base * 4),
                                     4, 0, 0);
  }
}

// Issue the copies of the staged rows of a tile, LDS row sl <- x[ssl[sl]][0..S),
// in UB-byte units (16 when a row of S values is a multiple of 16 bytes, else
// 4); the slot rows come from LDS, so no copy waits on another.  When a row
// holds upr units and upr divides 64, one load instruction moves 64 / upr
// whole rows (lane -> row lane / upr, unit lane % upr); otherwise wave w
// fills units [base, base + 64) for base = 64 w, 64 w + 256, ....  Lanes past
// the end repeat a valid load into the unused tail of the buffer.
template <typename XT, int UB>
__device__ __attribute__((always_inline)) inline void stage_issue(int nslots,
                                                                  const XT *__restrict__ x, int S,
                                                                  XT *lds, const int *ssl) {
  const int upr = S * (int)sizeof(XT) / UB;  // units per row (wave-uniform)
  const char *xb = reinterpret_cast<const char *>(x);
  char *lb = reinterpret_cast<char *>(lds);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  auto issue = [&](const char *src, int base_unit) {
    auto *dst = (__attribute__((address_space(3))) void *)(lb + (size_t)base_unit * UB);
    if constexpr (UB == 16) __builtin_amdgcn_global_load_lds((const void *)src, dst, 16, 0, 0);
    else __builtin_amdgcn_global_load_lds((const void *)src, dst, 4, 0, 0);
  };
  if (64 % upr == 0) {
    const int rpi = 64 / upr;  // rows per load instruction
    const int lr = lane / upr, lu = lane - lr * upr;
    const int step = (kBlock / 64) * rpi;
    // An LDS read after a copy into LDS waits for every copy in flight, so
    // the slot rows of kBatch copies are read first and their copies issued
    // together: one wait per batch instead of one per copy.
    constexpr int kBatch = 8;
    for (int rb = w * rpi; rb < nslots; rb += kBatch * step) {
      int src[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int r0 = rb + k * step;
        src[k] = r0 < nslots ? ssl[r0 + lr < nslots ? r0 + lr : r0] : 0;
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int r0 = rb + k * step;
        if (r0 < nslots) issue(xb + ((size_t)src[k] * upr + lu) * UB, r0 * upr);
      }
    }
    return;
  }
  const int total = nslots * upr;
  for (int base = w * 64; base < total; base += kBlock) {
    const int u = base + lane < total ? base + lane : base;
    const int sl = u / upr;
    issue(xb + ((size_t)ssl[sl] * upr + (u - sl * upr)) * UB, base);
  }
}

// VEC staged values of LDS row sl starting at scenario s0 (AL: 16-byte aligned)
template <typename XT, int VEC, bool AL>
__device__ __attribute__((always_inline)) inline void xrow(const XT *lx, int sl, int S, int s0,
                                                           XT (&o)[VEC]) {
  const XT *q = lx + sl * S + s0;
  if constexpr (AL) {
    if constexpr (VEC == 4) {
      const float4 f = *reinterpret_cast<const float4 *>(q);
      o[0] = f.x; o[1] = f.y; o[2] = f.z; o[3] = f.w;
    } else {
      const double2 d = *reinterpret_cast<const double2 *>(q);
      o[0] = d.x; o[1] = d.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < VEC; ++i) o[i] = q[i];
  }
}

// acc[k] += sum over entries e in [e0, e1) of the row (in order) of
// value_e * x[slot_e][s0 + k]; four entries' LDS reads go out together
template <typename AT, typename VT, typename XT, bool AL>
__device__ __attribute__((always_inline)) inline void entry_sum(const StageLds<XT, VT> &L,
                                                                int rel, int e0, int e1, int S,
                                                                int s0,
                                                                AT (&acc)[Lanes<XT>::VEC]) {
  constexpr int VEC = Lanes<XT>::VEC;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    int sl[4];
    AT v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sl[j] = L.eslot[rel + e + j];
      v[j] = (AT)L.eval[rel + e + j];
    }
    XT xv[4][VEC];
#pragma unroll
    for (int j = 0; j < 4; ++j) xrow<XT, VEC, AL>(L.x, sl[j], S, s0, xv[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < VEC; ++k) acc[k] = fma_t(v[j], (AT)xv[j][k], acc[k]);
  }
  for (; e < e1; ++e) {
    XT xv[VEC];
    xrow<XT, VEC, AL>(L.x, L.eslot[rel + e], S, s0, xv);
    const AT v = (AT)L.eval[rel + e];
#pragma unroll
    for (int k = 0; k < VEC; ++k) acc[k] = fma_t(v, (AT)xv[k], acc[k]);
  }
}

// One tile of a staged product.  For each row of the tile and each of the
// lane's scenarios s = s0 + i < S: epi(row, i, s, y, own, mass) with y =
// (K + h_s R) x (K entries, then R entries, each summed in entry order),
// own = x[row][s] (from LDS) and the lumped mass.  Two memory round trips:
// (1) the tile's slot rows and the extents of the lane's rows; (2) the
// staging copies of x and of the tile's entries.
template <typename AT, typename VT, typename XT, int UB, bool AL, typename Epi>
__device__ __attribute__((always_inline)) inline void tile_apply(
    const BatchArgs &a, int t, const VT *__restrict__ val, const XT *__restrict__ x,
    const AT (&h)[Lanes<XT>::VEC], StageLds<XT, VT> &L, Epi &&epi) {
  using LY = Lanes<XT>;
  constexpr int VEC = LY::VEC, NI = LY::NI;
  const BatchOp &op = a.op;
  const int S = a.S;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane / LY::LPR, s0 = (lane % LY::LPR) * VEC;
  const int64_t r0 = op.tstart[t], r1 = op.tstart[t + 1];  // tile positions
  // (1) slot rows, entry range, and the lane's rows
  int srv = 0;
  if (tid < kStageSlots) srv = op.slot_row[(size_t)t * kStageSlots + tid];
  const int ns = op.nslots[t];
  const int64_t E0 = op.rowptr[r0], E1 = op.rowptr[r1];
  int64_t lo[NI], hi[NI], rw[NI];
  int nk[NI], os[NI];
  double ms[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    int64_t pos = r0 + (int64_t)(w + 4 * i) * LY::RPW + lr;
    pos = pos < r1 ? pos : r1 - 1;
    lo[i] = op.rowptr[pos];
    hi[i] = op.rowptr[pos + 1];
    nk[i] = op.nk[pos];
    os[i] = op.oslot[pos];
    rw[i] = op.prow[pos];
    ms[i] = op.pmass[pos];
  }
  __builtin_amdgcn_s_waitcnt(0);
  if (tid < kStageSlots) L.ssl[tid] = srv;
  __syncthreads();
  // (2) staged rows and the tile's entries
  stage_issue<XT, UB>(ns, x, S, L.x, L.ssl);
  const int ne = (int)(E1 - E0);
  dma_contig(op.slot32 + E0, L.eslot, ne);
  dma_contig(val + E0, L.eval, ne * (int)(sizeof(VT) / 4));
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int64_t pos = r0 + (int64_t)(w + 4 * i) * LY::RPW + lr;
    if (pos >= r1) continue;
    const int64_t row = rw[i];
    const int rel = (int)(lo[i] - E0), n = (int)(hi[i] - lo[i]);
    AT acc[VEC] = {}, accr[VEC] = {};
    entry_sum<AT, VT, XT, AL>(L, rel, 0, nk[i], S, s0, acc);
    entry_sum<AT, VT, XT, AL>(L, rel, nk[i], n, S, s0, accr);
    XT own[VEC];
    xrow<XT, VEC, AL>(L.x, os[i], S, s0, own);
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      if (s0 + k >= S) continue;
      // (one explicit rounding pattern; the column sweep forms the same
      // sums, and y = fma(h, accr, acc) with accr = 0 where there is no R)
      const AT y = n == nk[i] ? acc[k] : fma_t(h[k], accr[k], acc[k]);
      epi(row, k, s0 + k, y, own[k], ms[i]);
    }
  }
  __syncthreads();
}

// per-scenario block sums of the lanes' partials (v[k][i] for scenario
// s0 + i) into partial[k][s][blk]: fixed order over waves and row slots
template <int K, typename XT, typename VT>
__device__ inline void publish_lanes(const double (&v)[K][Lanes<XT>::VEC], double *partial,
                                     int grid, int S, StageLds<XT, VT> &L) {
  using LY = Lanes<XT>;
  double *sh = reinterpret_cast<double *>(L.x);  // [4][RPW][64] per k
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane / LY::LPR, s0 = (lane % LY::LPR) * LY::VEC;
  __syncthreads();
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int i = 0; i < LY::VEC; ++i) sh[(w * LY::RPW + lr) * 64 + s0 + i] = v[k][i];
    __syncthreads();
    if (threadIdx.x < (unsigned)S) {
      double acc = 0.0;
      for (int j = 0; j < 4 * LY::RPW; ++j) acc += sh[j * 64 + threadIdx.x];
      partial[((size_t)k * S + threadIdx.x) * grid + blockIdx.x] = acc;
    }
    __syncthreads();
  }
}

// per-scenario block sums of the lanes' partials (v[k][i] for scenario s0 + i)
// into partial[k][s][blk]: fixed order over waves and row slots
template <int K, int VEC, int RPW>
__device__ inline void publish_groups_in(const double (&v)[K][VEC], double *partial, int grid,
                                         int S, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane / (64 / VEC), s0 = (lane % (64 / VEC)) * VEC;
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) sh[(w * RPW + lr) * 64 + s0 + i] = v[k][i];
    __syncthreads();
    if (threadIdx.x < (unsigned)S) {
      double acc = 0.0;
      for (int j = 0; j < 4 * RPW; ++j) acc += sh[j * 64 + threadIdx.x];
      partial[((size_t)k * S + threadIdx.x) * grid + blockIdx.x] = acc;
    }
    __syncthreads();
  }
}
template <int K, int VEC, int RPW>
__device__ inline void publish_groups(const double (&v)[K][VEC], double *partial, int grid,
                                      int S) {
  __shared__ double sh[4 * RPW * 64];
  publish_groups_in<K, VEC, RPW>(v, partial, grid, S, sh);
}

// ---------------------------------------------------------------------------
// Column-sweep multi-RHS operator (every body a box of the 27-point
// pattern).  A work item is a footprint of kColFX x kColFY nodes of one body
// over a run of z planes.  The workgroup streams up the run one staged plane
// at a time (the footprint and its one-node halo: kColPL rows of 256 bytes
// whatever S is): a lane reads the 3 x 3 neighbourhood of its column in
// plane P once and adds it to the three rows it touches, the
// neighbour-below part (dz = -1) of row P + 1, the dz = 0 part of row P and
// the dz = +1 part of row P - 1, which is then complete.  Each row so gets
// its stencil values in stencil order (dz, then dy, then dx), which is the
// CSR order of its entries, with exact zeros where a neighbour or entry is
// missing (K and R apart, then K + h R).  Each staged value is read from LDS
// once per lane instead of three times, each staged row is copied once per
// item instead of once per tile that touches it, and each matrix entry is
// found from its stencil position instead of a stored column.  The planes
// (and the rows' stencil records) arrive by direct global-to-LDS copies that
// hold no registers, D stages ahead, waited for by count one stage at a time.
//
// A staged row is 64 FP32 or 32 FP64 values, so in FP64 an item is swept
// twice, once per half of the scenarios (by neighbouring workgroups of one
// XCD: the second reads the item's records from L2).  A lane owns the 16
// bytes of four (FP32) or two (FP64) consecutive scenarios of a row, a wave
// the four rows w 4 .. w 4 + 3 of the plane.
// ---------------------------------------------------------------------------
// (XV: the staged values, RV: the stencil records)
template <typename XV, typename RV = XV>
struct ColGeom {
  static constexpr int VB = (int)sizeof(XV);
  static constexpr int VEC = 16 / VB;  // scenarios per lane
  static constexpr int SW = 256 / VB;  // scenarios per workgroup (one staged row)
  static constexpr int H = 64 / SW;    // workgroups per item
  static constexpr int PlaneUnits = kColPL * 16;  // 16-byte units of a plane
  static constexpr int RVB = (int)sizeof(RV);
  static constexpr int RecUnits = kColRows * kStencil * RVB / 16;  // of a K (or R) record
  static constexpr int RecSlot = (2 * RecUnits + 63) / 64 * 64;    // K, R and the copy tail
  static_assert(kColRows == 16 && kBlock == 256, "four waves of four rows");
};
// Wave-wide copies per stage: the staged rows in UB-byte units (16 when a
// row of S values is a multiple of 16 bytes, else 4), then the records in
// 16-byte units; copy j is issued by wave j % 4, so wave w issues C<w> of
// them (C0 the most)
template <typename XV, typename RV, int UB>
struct ColCopies {
  static constexpr int X = ColGeom<XV, RV>::PlaneUnits * 16 / UB / 64;
  static constexpr int N = X + ColGeom<XV, RV>::RecSlot / 64;
  template <int W>
  static constexpr int C = (N - W + 3) / 4;
  static constexpr int C0 = C<0>;
};

// Stage s = staged plane s + 1 (read in step s) and the stencil record of
// plane s + 2 (read in steps s .. s + 2).  With D stages in flight beyond
// the one being read: D + 1 plane slots and D + 3 record slots.
template <typename XV, typename RV, int D>
struct ColLds {
  static constexpr int NX = D + 1, NR = D + 3;
  uint4 x[NX][ColGeom<XV, RV>::PlaneUnits];
  uint4 rec[NR][ColGeom<XV, RV>::RecSlot];
};
// The refinement's sweep also brings the FP64 rows it updates (T and r64 of
// the wave's four rows: 4 KB per wave) into LDS, one step ahead, each lane
// its own values.
constexpr int kColIOBytes = 4 * 4096;
template <typename XV, typename RV, int D>
struct ColLdsIO : ColLds<XV, RV, D> {
  uint4 io[kColIOBytes / 16];
};
// workgroups per CU that the ring leaves room for (160 KB of LDS); four only
// for FP32 with 16-byte copies, at most two for FP64 records with 4-byte
// copies or FP32 staged values (the other forms need more than 128, those
// more than 168 registers)
template <typename XV, typename RV, int D, int UB = 16>
struct ColOcc {
  static constexpr size_t B =
      sizeof(ColLds<XV, RV, D>) + (sizeof(XV) != sizeof(RV) ? kColIOBytes : 0);
  static constexpr bool F32 = sizeof(XV) == 4 && sizeof(RV) == 4;
  static constexpr bool BIG = sizeof(RV) == 8 && (UB == 4 || sizeof(XV) == 4);
  static constexpr int W = F32 && UB == 16 && 4 * B + 1024 <= 160 * 1024 ? 4
                           : !BIG && 3 * B + 768 <= 160 * 1024          ? 3
                           : 2 * B + 512 <= 160 * 1024                  ? 2
                                                                        : 1;
};

struct ColItem {
  int off, nx, ny, nz, x0, y0, z0, z1, kb, rb;
  unsigned mlo, mhi;
};
// (wave-uniform: kept in scalar registers)
__device__ inline ColItem col_item(const BatchOp &op, int t) {
  const int *p = op.col_items + (size_t)kColItem * t;
  int v[kColItem];
#pragma unroll
  for (int k = 0; k < kColItem; ++k) v[k] = __builtin_amdgcn_readfirstlane(p[k]);
  return ColItem{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9],
                 (unsigned)v[10], (unsigned)v[11]};
}

// the stencil records and the vectors of the form
template <typename V>
struct ColVec;
template <>
struct ColVec<float> {
  using V16 = float4;
  __device__ static const float *rec(const BatchOp &op) { return op.kcol32; }
  __device__ static const float *rrec(const BatchOp &op) { return op.rcol32; }
  __device__ static int64_t rec_bytes(const BatchOp &op) { return op.col_rec_bytes32; }
  __device__ static const float *p(const BatchArgs &a) { return a.p32; }
  __device__ static float *q(const BatchArgs &a) { return a.q32; }
  __device__ static void split(const float4 &v, float (&o)[4]) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct ColVec<double> {
  using V16 = double2;
  __device__ static const double *rec(const BatchOp &op) { return op.kcol64; }
  __device__ static const double *rrec(const BatchOp &op) { return op.rcol64; }
  __device__ static int64_t rec_bytes(const BatchOp &op) { return op.col_rec_bytes64; }
  __device__ static const double *p(const BatchArgs &a) { return a.p; }
  __device__ static double *q(const BatchArgs &a) { return a.q; }
  __device__ static void split(const double2 &v, double (&o)[2]) {
    o[0] = v.x;
    o[1] = v.y;
  }
};

// Wave w's copies of the stages of one item: copy j = w + 4 i of a stage
// moves LDS units [64 j', 64 j' + 64) of the staged plane (j' = j < X) or
// of the record slot (j' = j - X).  What a lane copies depends on the stage
// only through the plane and record indices, so the per-lane parts (halo row
// offset, inside flag, record unit) are formed once per item; issuing a
// stage then costs a few instructions per copy.  Every lane copies from
// inside a buffer: halo rows outside the body and the values past S of a
// row come from the row of zeros after the staged vector; the records' tail
// repeats the first K unit.
template <typename XV, typename RV, int UB, int D>
struct ColIssue {
  using G = ColGeom<XV, RV>;
  using CC = ColCopies<XV, RV, UB>;
  static constexpr int UPH = 256 / UB;  // units per staged row
  static constexpr unsigned XB = G::PlaneUnits * 16, RB = G::RecSlot * 16;  // slot bytes
  static constexpr unsigned RECB = G::RecUnits * 16;                        // record bytes
  // buffer resources: x (the staged vector: the CG direction, a node state or
  // the FP32 correction, which ends in a row of zeros) and the records (K,
  // then R)
  __amdgpu_buffer_rsrc_t rx, rrec;
  unsigned off0[CC::C0];  // x copy: the lane's unit at plane 0; record copy: in a record
  unsigned zoff[CC::C0];  // x copy: its offset in the row of zeros
  bool xin[CC::C0];       // x copy: halo row inside the body, unit inside the row
  int rpart[CC::C0];      // record copy: 0 K unit, 1 R unit, 2 tail
  unsigned pstride;       // bytes between planes of x
  unsigned rbase;         // byte offset of the R records
  int w;
  // the next stage (wave-uniform): its plane P and record plane R = P + 1,
  // the byte offsets of its slots, P's offset in x, and R's record indices
  int P, R, kr, rr;
  unsigned xso, rso, pbase;
  unsigned long long rbits;  // R plane bits of the records not issued yet

  // ring slots: stage z0 - 2 + i in plane slot i mod NX, record plane z0 + i
  // in record slot i mod NR; xsrc = the staged vector (N S values, then a
  // row of zeros), hs = this workgroup's first scenario
  __device__ __forceinline__ void init(const BatchArgs &a, const XV *xsrc, const ColItem &it,
                                       int wave, int hs) {
    w = wave;
    const int S = a.S, lane = threadIdx.x & 63;
    const int upr = (min(S - hs, G::SW) * G::VB) / UB;  // units of the row in this half
    const unsigned zrow = (unsigned)(a.N * S) * (unsigned)G::VB;  // the row of zeros
    rx = __builtin_amdgcn_make_buffer_rsrc((void *)xsrc, 0, (int)(zrow + kColZeroRow * G::VB),
                                           0x00020000);
    rrec = __builtin_amdgcn_make_buffer_rsrc((void *)ColVec<RV>::rec(a.op), 0,
                                             (int)ColVec<RV>::rec_bytes(a.op), 0x00020000);
    rbase = (unsigned)((ColVec<RV>::rrec(a.op) - ColVec<RV>::rec(a.op)) * G::RVB);
    pstride = (unsigned)it.nx * (unsigned)it.ny * (unsigned)S * (unsigned)G::VB;
#pragma unroll
    for (int i = 0; i < CC::C0; ++i) {
      const int j = w + 4 * i;
      if (j < CC::X) {
        const int u = j * 64 + lane, hr = u / UPH, part = u % UPH;
        const int hx = hr % (kColFX + 2), hy = hr / (kColFX + 2);
        const int gx = it.x0 - 1 + hx, gy = it.y0 - 1 + hy;
        xin[i] =
            ((unsigned)gx < (unsigned)it.nx) & ((unsigned)gy < (unsigned)it.ny) & (part < upr);
        // (32-bit offsets: the column sweep runs only on vectors below 2 GB)
        const unsigned row = xin[i] ? (unsigned)(it.off + gx + it.nx * gy) : 0u;
        off0[i] = (row * (unsigned)S + (unsigned)hs) * (unsigned)G::VB + (unsigned)(part * UB);
        zoff[i] = zrow + (unsigned)(part * UB);
        rpart[i] = 0;
      } else {
        const int u = (j - CC::X) * 64 + lane;
        rpart[i] = u < G::RecUnits ? 0 : (u < 2 * G::RecUnits ? 1 : 2);
        off0[i] = (unsigned)((rpart[i] == 0 ? u : (rpart[i] == 1 ? u - G::RecUnits : 0)) * 16);
        zoff[i] = 0;
        xin[i] = false;
      }
    }
    P = it.z0 - 1;
    R = it.z0;
    kr = it.kb;
    rr = it.rb;
    rbits = ((unsigned long long)it.mhi << 32) | it.mlo;
    xso = rso = 0;
    pbase = (unsigned)P * pstride;
  }

  // Issue the next stage: plane P (zeros outside the body and past the
  // run's top neighbour z1) and the record of plane R (the run's first record
  // past the run), then step to the stage after it.
  __device__ __forceinline__ void issue(const ColItem &it, ColLds<XV, RV, D> &L) {
    const bool pin = (P >= 0) & (P < it.nz) & (P <= it.z1);
    const bool inrun = R < it.z1;
    const bool hasr = inrun & ((rbits & 1ull) != 0);
    const unsigned ko = (unsigned)(inrun ? kr : it.kb) * RECB;
    const unsigned ro = rbase + (unsigned)(inrun ? rr : it.rb) * RECB;
    char *lx = reinterpret_cast<char *>(&L.x[0][0]) + xso;
    char *lr = reinterpret_cast<char *>(&L.rec[0][0]) + rso;
#pragma unroll
    for (int i = 0; i < CC::C0; ++i) {
      const int j = w + 4 * i;  // wave-uniform
      if (j >= CC::N) break;
      if (j < CC::X) {
        const unsigned off = (pin & xin[i]) ? off0[i] + pbase : zoff[i];
        auto *dst = (__attribute__((address_space(3))) void *)(lx + j * 64 * UB);
        if constexpr (UB == 16) __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, dst, 16, off, 0, 0, 0);
        else __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, dst, 4, off, 0, 0, 0);
      } else {
        const unsigned off = (((rpart[i] == 1) & hasr) ? ro : ko) + off0[i];
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rrec, (__attribute__((address_space(3))) void *)(lr + (j - CC::X) * 1024), 16, off, 0,
            0, 0);
      }
    }
    P += 1;
    pbase += pstride;
    xso = xso + XB == ColLds<XV, RV, D>::NX * XB ? 0u : xso + XB;
    rr += hasr ? 1 : 0;
    kr += 1;
    rbits >>= 1;
    R += 1;
    rso = rso + RB == ColLds<XV, RV, D>::NR * RB ? 0u : rso + RB;
  }
};

// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding: vmcnt in bits 3:0 and 15:14)
template <int N>
__device__ __forceinline__ void col_wait() {
  static_assert(N >= 0 && N < 64, "vmcnt holds six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
}
// Workgroup barrier that orders the LDS accesses around it but leaves the
// copies in flight (a fence would wait for every one of them).
__device__ __forceinline__ void col_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
// Wait until this wave's copies of plane z + 2 have landed, k + 1 planes
// (k = min(z - z0, D - 1)) into the run, with D planes in flight beyond
// z + 1, C copies per plane, ST stores per plane formed and LD loads issued
// per step (before the step's copies) by this wave.  In issue order, what
// follows those copies is exactly: the loads and copies of the D - 1 later
// steps (k of them so far) and the stores of the last k + 1 planes formed
// (the stores and loads are unconditional buffer accesses, so the count is
// exact; if the loads were issued after the copies the wait would only be
// longer), and vmcnt counts them in order.
template <int C, int ST, int D, int LD, int K = 0>
__device__ __forceinline__ void col_wait_plane(int k) {
  if constexpr (K == D - 1) {
    col_wait<(D - 1) * C + ST + K * (ST + LD)>();
  } else {
    if (k == K) col_wait<(D - 1) * C + ST + K * (ST + LD)>();
    else col_wait_plane<C, ST, D, LD, K + 1>(k);
  }
}
// the same for wave w (wave-uniform) issuing CC::C<w> copies per stage and
// LD loads per step just before them
template <typename CC, int ST, int D, int LD>
__device__ __forceinline__ void col_wait_wave(int w, int k) {
  switch (w) {
    case 0: col_wait_plane<CC::template C<0>, ST, D, LD>(k); break;
    case 1: col_wait_plane<CC::template C<1>, ST, D, LD>(k); break;
    case 2: col_wait_plane<CC::template C<2>, ST, D, LD>(k); break;
    default: col_wait_plane<CC::template C<3>, ST, D, LD>(k); break;
  }
}
// Wait until no more than wave w's copies of one stage are in flight.
template <typename CC, int EXTRA>
__device__ __forceinline__ void col_wait_copies(int w) {
  switch (w) {
    case 0: col_wait<CC::template C<0> + EXTRA>(); break;
    case 1: col_wait<CC::template C<1> + EXTRA>(); break;
    case 2: col_wait<CC::template C<2> + EXTRA>(); break;
    default: col_wait<CC::template C<3> + EXTRA>(); break;
  }
}
// Wait until wave w's copies of the first of the D + 1 stages issued have
// landed.
template <typename CC, int D>
__device__ __forceinline__ void col_wait_first(int w) {
  switch (w) {
    case 0: col_wait<D * CC::template C<0>>(); break;
    case 1: col_wait<D * CC::template C<1>>(); break;
    case 2: col_wait<D * CC::template C<2>>(); break;
    default: col_wait<D * CC::template C<3>>(); break;
  }
}

// acc[q] += sum over the nine positions j = 3 dy + dx of one plane (in
// order) of c[j] xv[j][q] (q over the lane's scenarios)
__device__ __forceinline__ void col_part(const __attribute__((address_space(3))) float *c,
                                         const float4 (&xv)[9], float (&acc)[4]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const float w = c[j];
    acc[0] = fma_t(w, xv[j].x, acc[0]);
    acc[1] = fma_t(w, xv[j].y, acc[1]);
    acc[2] = fma_t(w, xv[j].z, acc[2]);
    acc[3] = fma_t(w, xv[j].w, acc[3]);
  }
}
__device__ __forceinline__ void col_part(const __attribute__((address_space(3))) double *c,
                                         const double (&xv)[9][4], double (&acc)[4]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const double w = c[j];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = fma_t(w, xv[j][q], acc[q]);
  }
}
__device__ __forceinline__ void col_part(const __attribute__((address_space(3))) double *c,
                                         const double2 (&xv)[9], double (&acc)[2]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const double w = c[j];
    acc[0] = fma_t(w, xv[j].x, acc[0]);
    acc[1] = fma_t(w, xv[j].y, acc[1]);
  }
}
// CG vectors and stored operator values of the FP64 (double) or FP32 (float) form
template <typename V>
struct BV;
template <>
struct BV<double> {
  __device__ static const double *vals(const BatchArgs &a) { return a.op.val; }
  __device__ static double *x(const BatchArgs &a, int m) { return a.T[m]; }
  __device__ static double *r(const BatchArgs &a) { return a.r; }
  __device__ static double *p(const BatchArgs &a) { return a.p; }
  __device__ static double *q(const BatchArgs &a) { return a.q; }
};
template <>
struct BV<float> {
  __device__ static const float *vals(const BatchArgs &a) { return a.op.val32; }
  __device__ static float *x(const BatchArgs &a, int) { return a.x32; }
  __device__ static float *r(const BatchArgs &a) { return a.r32; }
  __device__ static float *p(const BatchArgs &a) { return a.p32; }
  __device__ static float *q(const BatchArgs &a) { return a.q32; }
};

// (the flags are read at a clamped index without short-circuit evaluation,
// so all of them are requested at once)
__device__ inline bool lane_on(const BatchScalars *sc, int s, int S) {
  const int k = s < S ? s : 0;
  const int off = sc->done[k] | sc->ref_done[k] | sc->stop[k];
  return (s < S) & (sc->active[k] != 0) & (off == 0);
}

// scenario s still sweeping this step (active, not stopped by residual control)
__device__ inline bool sweeping(const BatchScalars *sc, int s, int S) {
  const int k = s < S ? s : 0;
  return (s < S) & (sc->active[k] != 0) & (sc->stop[k] == 0);
}

// the scenario's h, read at a clamped index (zero for a lane past S)
__device__ inline double lane_h(const BatchArgs &a, int s) {
  const double h = a.h[s < a.S ? s : 0];
  return s < a.S ? h : 0.0;
}

// ---------------------------------------------------------------------------
// F_j = g - L_s T_j (several standard nodes j), all scenarios, in LDS tiles
// (meshes without the column sweep; box meshes take its F mode)
// ---------------------------------------------------------------------------
template <int UB, bool AL>
__global__ __launch_bounds__(kBlock) void kb_f_multi(BatchArgs a, int j0, int j1) {
  using LY = Lanes<double>;
  __shared__ StageLds<double, double> L;
  const int S = a.S, s0 = (threadIdx.x & 63) % LY::LPR * LY::VEC;
  double h[LY::VEC];
#pragma unroll
  for (int i = 0; i < LY::VEC; ++i) h[i] = s0 + i < S ? a.h[s0 + i] : 0.0;
  FOR_TILES(t, a.op.ntiles) {
    for (int j = j0; j <= j1; ++j) {
      double *F = a.F[j];
      tile_apply<double, double, double, UB, AL>(
          a, t, a.op.val, a.T[j], h, L,
          [&](int64_t row, int i, int s, double y, double, double) {
            F[row * S + s] = h[i] * a.gbase[row] - y;
          });
    }
  }
}

// ---------------------------------------------------------------------------
// I_{m-1}^m for all m and the residual per scenario (max-norm)
// ---------------------------------------------------------------------------
// (weights as a restrict-qualified parameter, read through the scalar cache;
// every operand of a row is loaded, at clamped node indices, before the
// row's first store)
__global__ __launch_bounds__(kBlock) void kb_quad_resid(BatchArgs a,
                                                        const Weights *__restrict__ wp) {
  const int s = threadIdx.x & 63, S = a.S;
  const Weights &w = *wp;
  const int P1 = a.P + 1;
  double rmax = 0.0;
  if (s < S) {
    FOR_ROWS(row, a.N) {
      const int64_t i = row * S + s;
      const double mi = a.mass[row], Tn = a.T[0][i];
      const int pos = a.ifpos ? a.ifpos[row] : -1;
      double F[kMaxM + 1], T[kMaxM + 1], acc[kMaxM + 1];
#pragma unroll
      for (int j = 1; j <= kMaxM; ++j) {
        const int jj = j <= a.M ? j : 1;
        const double f = a.F[jj][i], t = a.T[jj][i];
        F[j] = j <= a.M ? f : 0.0;
        T[j] = j <= a.M ? t : 0.0;
      }
#pragma unroll
      for (int m = 1; m <= kMaxM; ++m) {
        acc[m] = 0.0;
        if (m > a.M || w.dtau[m] == 0.0) continue;
#pragma unroll
        for (int j = 1; j <= kMaxM; ++j)
          if (j <= a.M) acc[m] += w.s[m][j] * F[j];
        if (pos >= 0) {
          const double *E = a.Eold + ((size_t)m * P1 * a.n_if + pos) * S + s;
#pragma unroll 4
          for (int q = 1; q <= a.P; ++q) acc[m] += w.shat[m][q] * E[(size_t)q * a.n_if * S];
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
  }
  double v[1] = {rmax};
  // per-scenario maxima of the block
  __shared__ double sh[kBlock / 64][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  sh[wv][lane] = v[0];
  __syncthreads();
  if (wv == 0 && lane < S) {
    double mx = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) mx = fmax(mx, sh[k][lane]);
    a.partial[(size_t)blockIdx.x * S + lane] = mx;
  }
}

constexpr int kRedWaves = 16;  // waves of the one-block reductions

__global__ __launch_bounds__(64 * kRedWaves) void kb_resid_reduce(BatchArgs a, int k) {
  __shared__ double sh[kRedWaves][64];
  const int s = threadIdx.x & 63, w = threadIdx.x >> 6;
  double mx = 0.0;
  if (s < a.S)
    for (int b = w; b < a.grid; b += kRedWaves) mx = fmax(mx, a.partial[(size_t)b * a.S + s]);
  sh[w][s] = mx;
  __syncthreads();
  if (w == 0 && s < a.S) {
    for (int ww = 1; ww < kRedWaves; ++ww) mx = fmax(mx, sh[ww][s]);
    BatchScalars *sc = a.sc;
    sc->resid[k][s] = mx;
    // residual control: the first iterate at or below the tolerance ends the
    // scenario's sweeps for this step
    if (a.sweep_tol > 0 && sc->active[s] && !sc->stop[s] && mx <= a.sweep_tol) {
      sc->stop[s] = 1;
      sc->sweeps[s] = k;
    }
  }
}

// ---------------------------------------------------------------------------
// implicit node solve per scenario: Jacobi-PCG, 3 kernels per iteration plus
// one-block scalar reductions
// ---------------------------------------------------------------------------
// Jacobi preconditioner 1 / diag(M + dtau (K + h R)) of a row, one rounding
// pattern in every kernel; where the row has no R part the value does not
// depend on h (fma(h, 0, kd) = kd), so a lane computes it once for its
// scenarios
__device__ __forceinline__ double dinv_of(double ms, double kd, double rd, double h,
                                          double dtau) {
  return 1.0 / __builtin_fma(dtau, __builtin_fma(h, rd, kd), ms);
}
template <typename V, int VEC>
__device__ __forceinline__ void dinv_row(double ms, double kd, double rd, const double (&h)[VEC],
                                         double dtau, V (&d)[VEC]) {
  if (rd == 0.0) {
    const V d0 = (V)dinv_of(ms, kd, 0.0, 0.0, dtau);
#pragma unroll
    for (int k = 0; k < VEC; ++k) d[k] = d0;
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) d[k] = (V)dinv_of(ms, kd, rd, h[k], dtau);
  }
}
__device__ inline double bdinv(const BatchArgs &a, int64_t row, double h, double dtau) {
  return dinv_of(a.mass[row], a.Kd[row], a.Rd[row], h, dtau);
}

// Solve initialisation of one row.  Predictor: x0 = T_{m-1}, b = M T_{m-1} +
// dtau g, r = b - A x0 (Lx = L T_{m-1} from the staged product).
// Correction: b = M T_{m-1} + dtau (g - F_m) + I_m and r = M (T_{m-1} - x0) +
// I_m without a product (L T^k_m = g - F_m).
template <bool PRED>
__device__ inline void init_rhs(const BatchArgs &a, int m, double dtau, int64_t i, int64_t row,
                                double h, double Lx, double *b, double *r) {
  const double mi = a.mass[row], tp = a.T[m - 1][i], g = h * a.gbase[row];
  if (PRED) {
    *b = mi * tp + dtau * g;
    *r = *b - (mi * tp + dtau * Lx);
    a.T[m][i] = tp;
  } else {
    const double Im = a.I[m][i];
    *b = mi * tp + dtau * (g - a.F[m][i]) + Im;
    *r = mi * (tp - a.T[m][i]) + Im;
  }
}

// FP64 form: r, p = z; partial r.z, r.r, b.b
template <bool PRED>
__device__ inline void init64_row(const BatchArgs &a, int m, double dtau, int64_t row, int s,
                                  double h, double Lx, double (&v)[3]) {
  const int64_t i = row * a.S + s;
  double b, r;
  init_rhs<PRED>(a, m, dtau, i, row, h, Lx, &b, &r);
  const double z = bdinv(a, row, h, dtau) * r;
  a.r[i] = r;
  a.p[i] = z;
  v[0] += r * z;
  v[1] += r * r;
  v[2] += b * b;
}

// FP32 form (refinement init): r64; partial r.r, b.b
template <bool PRED>
__device__ inline void init32_row(const BatchArgs &a, int m, double dtau, int64_t row, int s,
                                  double h, double Lx, double (&v)[2]) {
  const int64_t i = row * a.S + s;
  double b, r;
  init_rhs<PRED>(a, m, dtau, i, row, h, Lx, &b, &r);
  a.r64[i] = r;
  v[0] += r * r;
  v[1] += b * b;
}

// predictor initialisation: tiled, L T_{m-1} from the staged rows (meshes
// without the column sweep; box meshes take its predictor modes)
template <int NV, int UB, bool AL>
__global__ __launch_bounds__(kBlock) void kb_init_pred(BatchArgs a, int m, double dtau) {
  using LY = Lanes<double>;
  __shared__ StageLds<double, double> L;
  const int S = a.S, s0 = (threadIdx.x & 63) % LY::LPR * LY::VEC;
  double h[LY::VEC], v[NV][LY::VEC] = {};
  bool on[LY::VEC];
#pragma unroll
  for (int i = 0; i < LY::VEC; ++i) {
    on[i] = s0 + i < S && a.sc->active[s0 + i];
    h[i] = on[i] ? a.h[s0 + i] : 0.0;
  }
  FOR_TILES(t, a.op.ntiles) {
    tile_apply<double, double, double, UB, AL>(
        a, t, a.op.val, a.T[m - 1], h, L,
        [&](int64_t row, int i, int s, double Lx, double, double) {
          if (!on[i]) return;
          double vv[NV] = {};
          if constexpr (NV == 3) init64_row<true>(a, m, dtau, row, s, h[i], Lx, vv);
          else init32_row<true>(a, m, dtau, row, s, h[i], Lx, vv);
#pragma unroll
          for (int k = 0; k < NV; ++k) v[k][i] += vv[k];
        });
  }
  publish_lanes<NV>(v, a.partial, gridDim.x, S, L);
}

// correction initialisation: no product, row-parallel
template <int NV>
__global__ __launch_bounds__(kBlock) void kb_init_corr(BatchArgs a, int m, double dtau) {
  const int s = threadIdx.x & 63, S = a.S;
  double v[NV] = {};
  if (sweeping(a.sc, s, S)) {
    const double h = a.h[s];
    FOR_ROWS(row, a.N) {
      if constexpr (NV == 3) init64_row<false>(a, m, dtau, row, s, h, 0.0, v);
      else init32_row<false>(a, m, dtau, row, s, h, 0.0, v);
    }
  }
  bpublish<NV>(v, a.partial, gridDim.x, S);
}

// x64 += d; r64 -= A d with the FP64 operator on the FP32 correction d
// (staged as FP32); partial r.r.  Tiled (meshes without the column sweep;
// box meshes take its refinement mode).
template <int UB, bool AL>
__global__ __launch_bounds__(kBlock) void kb_refine_update(BatchArgs a, int m, double dtau) {
  using LY = Lanes<float>;
  __shared__ StageLds<float, double> L;
  const int S = a.S, s0 = (threadIdx.x & 63) % LY::LPR * LY::VEC;
  double h[LY::VEC], v[1][LY::VEC] = {};
  bool on[LY::VEC], any = false;
#pragma unroll
  for (int i = 0; i < LY::VEC; ++i) {
    const int s = s0 + i;
    on[i] = sweeping(a.sc, s, S) & (a.sc->ref_done[s < S ? s : 0] == 0);
    const double hs = lane_h(a, s);
    h[i] = on[i] ? hs : 0.0;
    any |= on[i];
  }
  double *x = a.T[m];
  if (__syncthreads_or(any)) {
    FOR_TILES(t, a.op.ntiles) {
      tile_apply<double, double, float, UB, AL>(
          a, t, a.op.val, a.x32, h, L,
          [&](int64_t row, int i, int s, double Ld, float own, double mass) {
            if (!on[i]) return;
            const int64_t ix = row * S + s;
            const double d = (double)own;
            x[ix] += d;
            const double r = a.r64[ix] - (mass * d + dtau * Ld);
            a.r64[ix] = r;
            v[0][i] += r * r;
          });
    }
  }
  publish_lanes<1>(v, a.partial, gridDim.x, S, L);
}

// Per-scenario scalars from the block partials.  Modes:
//   0 FP64 init (r.z, r.r, b.b)      1 alpha (p.q)
//   2 FP64 convergence (r.z, r.r)    3 refinement init (r.r, b.b)
//   4 inner init (r.z, r.r)          5 refinement check (r.r), it = round
//   6 inner convergence (r.z, r.r)
// One workgroup per scenario s = blockIdx.x; np = workgroups of the
// producing kernel, whose partials of scenario s are contiguous.  Fixed-order
// sums: thread j adds blocks j, j + 256, ..., then a fixed halving tree.
__global__ __launch_bounds__(kBlock) void kb_reduce(BatchArgs a, int np, int mode, int it,
                                                    int last, int slot, double rtol) {
  __shared__ double sh[3][kBlock];
  const int s = blockIdx.x, j = threadIdx.x;
  BatchScalars *sc = a.sc;
  const int nk = mode == 0 ? 3 : ((mode == 1 || mode == 5) ? 1 : 2);
  if (np <= kBatchMaxGrid) {  // every partial requested before the first sum
    constexpr int kq = kBatchMaxGrid / kBlock;
    double t[3][kq];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < kq; ++q) {
        const int b = j + q * kBlock;
        t[k][q] = (k < nk && b < np) ? a.partial[((size_t)k * a.S + s) * np + b] : 0.0;
      }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < kq; ++q) acc += t[k][q];
      if (k < nk) sh[k][j] = acc;
    }
  } else {
    for (int k = 0; k < nk; ++k) {
      const double *pp = a.partial + ((size_t)k * a.S + s) * np;
      double acc = 0.0;
      for (int b = j; b < np; b += kBlock) acc += pp[b];
      sh[k][j] = acc;
    }
  }
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (j < h)
      for (int k = 0; k < nk; ++k) sh[k][j] += sh[k][j + h];
    __syncthreads();
  }
  if (j != 0) return;
  double o[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < nk; ++k) o[k] = sh[k][0];
  if (!sweeping(sc, s, a.S)) return;
  if (mode == 0) {
    sc->rz[0][s] = o[0];
    sc->tol2[s] = rtol * rtol * o[2];
    sc->done[s] = (o[1] <= sc->tol2[s]) ? 1 : 0;
    sc->done_it[s] = -1;
    if (sc->done[s]) sc->slot_iters[slot][s] = 0;
    return;
  }
  if (mode == 3) {
    sc->ref_tol2[s] = rtol * rtol * o[1];
    sc->ref_done[s] = (o[0] <= sc->ref_tol2[s]) ? 1 : 0;
    sc->done[s] = 0;
    sc->done_it[s] = -1;
    if (sc->ref_done[s]) sc->slot_rounds[slot][s] = 0;
    return;
  }
  if (sc->ref_done[s]) return;
  if (mode == 4) {
    sc->rz[0][s] = o[0];
    sc->tol2[s] = rtol * rtol * o[1];  // relative to the inner right-hand side
    sc->done[s] = (o[1] == 0.0) ? 1 : 0;
    sc->done_it[s] = -1;
    return;
  }
  if (mode == 5) {
    sc->refine_total[s] += 1;
    if (o[0] <= sc->ref_tol2[s]) {
      sc->ref_done[s] = 1;
      sc->slot_rounds[slot][s] = it + 1;
    } else if (last) {
      sc->slot_rounds[slot][s] = -1;
      sc->fail[s] = 1;
    }
    return;
  }
  if (sc->done[s]) return;
  if (mode == 1) {
    sc->alpha[s] = sc->rz[it & 1][s] / o[0];
    return;
  }
  const bool inner = mode == 6;
  if (o[1] <= sc->tol2[s]) {
    sc->done[s] = 1;
    sc->done_it[s] = it;  // the update (c) of this iteration still moves x
    sc->iters_total[s] += it + 1;
    if (!inner) sc->slot_iters[slot][s] = it + 1;
    else if (sc->slot_iters[slot][s] >= 0 && it + 1 > sc->slot_iters[slot][s])
      sc->slot_iters[slot][s] = it + 1;
    return;
  }
  sc->beta[s] = o[0] / sc->rz[it & 1][s];
  sc->rz[(it + 1) & 1][s] = o[0];
  if (last) {
    // budget exhausted: an FP64 solve failed; an inner solve only signals it
    sc->slot_iters[slot][s] = -1;
    sc->iters_total[s] += it + 1;
    if (!inner) sc->fail[s] = 1;
  }
}

// (a) q = diag(m) p + dtau (K + h R) p, partial p.q.  V = double: the FP64
// form; V = float: the inner solves of the FP32 form (FP32 values, vectors,
// products and row sums; dot products summed in FP64).  TIMING: stand-alone
// timing launches that ignore the convergence flags.  Tiled; a workgroup
// with no scenario left to iterate skips the product.
template <int TIMING, typename V, int UB, bool AL>
__global__ __launch_bounds__(kBlock) void kb_pcg_a(BatchArgs a, int m, double dtau) {
  using LY = Lanes<V>;
  __shared__ StageLds<V, V> L;
  const int S = a.S, s0 = (threadIdx.x & 63) % LY::LPR * LY::VEC;
  V h[LY::VEC];
  double v[1][LY::VEC] = {};
  bool on[LY::VEC], any = false;
#pragma unroll
  for (int i = 0; i < LY::VEC; ++i) {
    const int s = s0 + i;
    on[i] = TIMING ? s < S : lane_on(a.sc, s, S);
    const V hs = (V)lane_h(a, s);
    h[i] = on[i] ? hs : (V)0;
    any |= on[i];
  }
  const V dt = (V)dtau;
  V *q = BV<V>::q(a);
  if (__syncthreads_or(any)) {
    FOR_TILES(t, a.op.ntiles) {
      tile_apply<V, V, V, UB, AL>(a, t, BV<V>::vals(a), BV<V>::p(a), h, L,
                                  [&](int64_t row, int i, int s, V y, V pi, double mass) {
                                    if (!on[i]) return;
                                    const V qi = fma_t((V)mass, pi, dt * y);
                                    q[row * S + s] = qi;
                                    v[0][i] = fma_t((double)pi, (double)qi, v[0][i]);
                                  });
    }
  }
  publish_lanes<1>(v, a.partial, gridDim.x, S, L);
}


// The column sweep's partial p.q: as publish_groups_in, with the lane
// mapping of the sweep (a lane's VEC scenarios start at s0; 16 lanes a row)
// and exact zeros for the scenarios of the other half.
template <typename V, int K>
__device__ inline void publish_col(const double (&v)[K][ColGeom<V>::VEC], double *partial,
                                   int grid, int S, int s0, double *sh) {
  constexpr int VEC = ColGeom<V>::VEC;
  const int j = threadIdx.x >> 4;  // the lane's row of the workgroup
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      sh[j * 64 + s0 + i] = v[k][i];
      if constexpr (ColGeom<V>::H == 2) sh[j * 64 + (s0 ^ 32) + i] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)S) {
      double acc = 0.0;
      for (int r = 0; r < kColRows; ++r) acc += sh[r * 64 + threadIdx.x];
      partial[((size_t)k * S + threadIdx.x) * grid + blockIdx.x] = acc;
    }
    __syncthreads();
  }
}

// The column sweep, one item (or half an item) per workgroup, XCD x taking
// the x-th eighth of the work (neighbouring footprints share halo rows, and
// the two halves of an item its records, in that XCD's L2):
//   MODE kColCG (the CG operator (a)): q = M p + dtau (K + h R) p and the
//     partial p.q (m: the node, dtau its step);
//   MODE kColF: F_m = h g - (K + h R) T_m for every scenario (FP64 only;
//     g of a row is value 27 of its R stencil);
//   MODE kColRefine (the FP32 form's refinement update, V = double): the
//     FP32 correction d = x32 staged, FP64 stencils and sums: T_m += d,
//     r64 -= M d + dtau (K + h R) d and the partial r64.r64, for the
//     scenarios still refining;
//   MODE kColPred32 / kColPred64 (the predictor's solve initialisation,
//     V = double): T_{m-1} staged, x0 = T_m = T_{m-1}, b = M T_{m-1} +
//     dtau h g, r = b - (M + dtau (K + h R)) T_{m-1}; FP32 form: r64 = r and
//     the partials r.r, b.b; FP64 form: r, p = dinv r and r.p, r.r, b.b
//     (dinv from the row's own stencils: mass, K and R centre values), for
//     the active scenarios.
// Where a row of S values is a multiple of 16 bytes, a lane stores its 16
// bytes at once (the values of idle scenarios too, which no later step
// reads, or in kColRefine the values it loaded); otherwise each value apart,
// only where its scenario is on.
constexpr int kColCG = 0, kColF = 1, kColRefine = 2, kColPred32 = 3, kColPred64 = 4;
template <int MODE, typename V>
using ColX = typename std::conditional<MODE == kColRefine, float, V>::type;
template <int TIMING, typename V, int UB, int D, int MODE = kColCG>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(ColOcc<ColX<MODE, V>, V, D, UB>::W)))
void kb_pcg_a_col(BatchArgs a, int m, double dtau) {
  static_assert(MODE == kColCG || sizeof(V) == 8, "F, the refinement and the predictor in FP64");
  using XV = ColX<MODE, V>;  // staged values
  using G = ColGeom<XV, V>;
  using CC = ColCopies<XV, V, UB>;
  using X16 = typename ColVec<XV>::V16;
  constexpr int VEC = G::VEC, VB = G::VB, RVB = G::RVB;
  constexpr bool REF = MODE == kColRefine;
  constexpr bool PRED = MODE == kColPred32 || MODE == kColPred64;
  // output vectors (REF: T_m and r64, also copied into LDS one step ahead;
  // PRED: T_m and r64, or T_m, r and p), partial sums
  constexpr int NOUT = MODE == kColPred64 ? 3 : ((REF || PRED) ? 2 : 1);
  constexpr int NV = MODE == kColPred64 ? 3 : (MODE == kColPred32 ? 2 : 1);
  // stores per step
  constexpr int ST = NOUT * (UB == 16 ? VEC * RVB / 16 : VEC);
  constexpr int LD = REF ? 2 * VEC * RVB / UB : 0;  // copies of the loaded rows
  constexpr int NX = ColLds<XV, V, D>::NX, NR = ColLds<XV, V, D>::NR;
  __shared__ typename std::conditional<REF, ColLdsIO<XV, V, D>, ColLds<XV, V, D>>::type L;
  const int S = a.S, lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int T = a.op.ncol_items * G::H, xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd;
  const int t = (int)((int64_t)T * xcd / kXcd) + local;
  const bool has = t < (int)((int64_t)T * (xcd + 1) / kXcd);
  const int hs = (G::H == 1 ? 0 : t % G::H) * G::SW;  // first scenario of the half
  const int lr = lane >> 4, s0 = hs + (lane & 15) * VEC;
  V h[VEC];
  double v[NV][VEC] = {};
  bool on[VEC], any = false;
#pragma unroll
  for (int i = 0; i < VEC; ++i) {
    const int s = s0 + i, sc = s < S ? s : 0;
    if constexpr (REF) on[i] = has && sweeping(a.sc, s, S) && a.sc->ref_done[sc] == 0;
    else if constexpr (PRED) on[i] = has && s < S && a.sc->active[sc] != 0;
    else on[i] = has && ((TIMING || MODE == kColF) ? s < S : lane_on(a.sc, s, S));
    const V hv = (V)lane_h(a, s);
    h[i] = on[i] ? hv : V(0);
    any |= on[i];
  }
  const V dt = (V)dtau;
  const XV *xsrc;
  V *qdst;
  if constexpr (MODE == kColCG) {
    xsrc = ColVec<V>::p(a);
    qdst = ColVec<V>::q(a);
  } else if constexpr (MODE == kColF) {
    xsrc = reinterpret_cast<const XV *>(a.T[m]);
    qdst = reinterpret_cast<V *>(a.F[m]);
  } else if constexpr (REF) {
    xsrc = a.x32;
    qdst = reinterpret_cast<V *>(a.T[m]);
  } else {
    xsrc = reinterpret_cast<const XV *>(a.T[m - 1]);
    qdst = reinterpret_cast<V *>(a.T[m]);
  }
  // further outputs: REF and kColPred32 r64, kColPred64 r and p
  void *odst1 = (void *)qdst, *odst2 = (void *)qdst;
  if constexpr (REF || MODE == kColPred32) odst1 = (void *)a.r64;
  if constexpr (MODE == kColPred64) {
    odst1 = (void *)a.r;
    odst2 = (void *)a.p;
  }
  const unsigned obytes = (unsigned)(a.N * S) * (unsigned)RVB;  // an output vector
  const __amdgpu_buffer_rsrc_t qres =
      __builtin_amdgcn_make_buffer_rsrc(qdst, 0, (int)obytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rres =
      __builtin_amdgcn_make_buffer_rsrc(odst1, 0, (int)obytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t pres =
      __builtin_amdgcn_make_buffer_rsrc(odst2, 0, (int)obytes, 0x00020000);
  if (__syncthreads_or(any)) {
    const ColItem it = col_item(a.op, G::H == 1 ? t : t / G::H);
    const int r = w * 4 + lr, lx = r % kColFX, ly = r / kColFX;
    // the row's (-1, -1) halo row, in values of the staged rows
    const int lb = (ly * (kColFX + 2) + lx) * G::SW + (lane & 15) * VEC;
    const bool rok = (it.x0 + lx < it.nx) & (it.y0 + ly < it.ny);
    const unsigned pstep = (unsigned)(it.nx * it.ny);  // rows between planes
    // Step z reads plane z + 1 and completes row z; steps z0 - 2 and z0 - 1
    // only start rows z0 and z0 + 1 (what they add to rows below z0 is never
    // used).
    const int zb = it.z0 - 2;
    // REF: T_m and r64 of row z, copied into the wave's LDS area during step
    // z - 1 (a copy outside the run or the body reads past the buffer:
    // zeros, never used).  Copy k moves 16 (UB = 4: 4) bytes per lane: the
    // lane's k-th unit of its T values (k < LD / 2), else of its r64 values,
    // to io + w 4096 + k 64 UB + lane UB.
    auto load_row = [&](int z) {
      if constexpr (REF) {
        const bool in = rok & (z >= it.z0) & (z < it.z1);
        const unsigned row = (unsigned)(it.off + it.x0 + lx + it.nx * (it.y0 + ly + it.ny * z));
        const unsigned off = (row * (unsigned)S + (unsigned)s0) * (unsigned)RVB;
        char *dst = reinterpret_cast<char *>(&L.io[0]) + w * 4096;
#pragma unroll
        for (int k = 0; k < LD; ++k) {
          const int u = k % (LD / 2);  // unit of the lane's values
          const bool ok = in & (UB == 16 || s0 + u * UB / RVB < S);
          const unsigned o = (off + (unsigned)(u * UB)) | ((unsigned)!ok << 31);
          auto *d = (__attribute__((address_space(3))) void *)(dst + k * 64 * UB);
          if constexpr (UB == 16)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(k < LD / 2 ? qres : rres, d, 16, o, 0, 0, 0);
          else
            __builtin_amdgcn_raw_ptr_buffer_load_lds(k < LD / 2 ? qres : rres, d, 4, o, 0, 0, 0);
        }
      }
    };
    ColIssue<XV, V, UB, D> ci;
    ci.init(a, xsrc, it, w, hs);
    load_row(zb);                                  // (never used: keeps the count per step)
    for (int q = 0; q <= D; ++q) ci.issue(it, L);  // stages z0 - 2 .. z0 - 2 + D
    col_wait_first<CC, D>(w);
    col_barrier();
    // K and R sums of rows z, z + 1, z + 2 (a: z, b: z + 1, c: z + 2)
    V ka[VEC] = {}, kb4[VEC] = {}, ra[VEC] = {}, rb4[VEC] = {};
    X16 own = {};  // x of row z (plane z's centre)
    // ring slots as ColIssue lays them out: plane z + 1 (stage z) in plane
    // slot (z - zb) mod NX, the record of plane z in slot (z - z0) mod NR
    constexpr unsigned XB = ColIssue<XV, V, UB, D>::XB, RB = ColIssue<XV, V, UB, D>::RB;
    auto next_r = [&](unsigned o) { return o + RB == NR * RB ? 0u : o + RB; };
    unsigned xro = 0, r0o = (NR - 2) * RB;  // step zb: plane slot 0, record z0 - 2
    const char *lxb = reinterpret_cast<const char *>(&L.x[0][0]) + lb * VB;
    // the row's stencils: an LDS address the compiler may not split into a
    // constant part (else each pair of coefficient reads gets its own add)
    using lds_char = const __attribute__((address_space(3))) char;
    lds_char *lrb = (lds_char *)(reinterpret_cast<const char *>(&L.rec[0][0]) + r * kStencil * RVB);
    lds_char *lrr = lrb + kColRows * kStencil * RVB;  // its R stencils, after the K record
    asm volatile("" : "+v"(lrb), "+v"(lrr));
    for (int z = zb; z < it.z1; ++z) {
      const XV *xs = reinterpret_cast<const XV *>(lxb + xro);
      X16 xv[9];
#pragma unroll
      for (int j = 0; j < 9; ++j)
        xv[j] = *reinterpret_cast<const X16 *>(xs + ((j / 3) * (kColFX + 2) + j % 3) * G::SW);
      const unsigned r1o = next_r(r0o), r2o = next_r(r1o);
      using lds_v = const __attribute__((address_space(3))) V;
      lds_v *c2 = reinterpret_cast<lds_v *>(lrb + r2o);
      lds_v *c1 = reinterpret_cast<lds_v *>(lrb + r1o);
      lds_v *c0 = reinterpret_cast<lds_v *>(lrb + r0o);
      V kc[VEC] = {}, rc[VEC] = {};
      V m2, m1, m0;
      if constexpr (REF) {  // FP32 staged values, FP64 sums: each value widened once
        double xd[9][VEC];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          XV o4[VEC];
          ColVec<XV>::split(xv[j], o4);
#pragma unroll
          for (int q = 0; q < VEC; ++q) xd[j][q] = (double)o4[q];
        }
        col_part(c2, xd, kc);       // row z + 2: dz = -1
        col_part(c1 + 9, xd, kb4);  // row z + 1: dz = 0
        col_part(c0 + 18, xd, ka);  // row z: dz = +1
        m2 = c2[kStencil - 1], m1 = c1[kStencil - 1], m0 = c0[kStencil - 1];
        if (m2 < V(0)) col_part(reinterpret_cast<lds_v *>(lrr + r2o), xd, rc);
        if (m1 < V(0)) col_part(reinterpret_cast<lds_v *>(lrr + r1o) + 9, xd, rb4);
        if (m0 < V(0)) col_part(reinterpret_cast<lds_v *>(lrr + r0o) + 18, xd, ra);
      } else {
        col_part(c2, xv, kc);       // row z + 2: dz = -1
        col_part(c1 + 9, xv, kb4);  // row z + 1: dz = 0
        col_part(c0 + 18, xv, ka);  // row z: dz = +1
        m2 = c2[kStencil - 1], m1 = c1[kStencil - 1], m0 = c0[kStencil - 1];
        // rows with R entries (mass < 0)
        if (m2 < V(0)) col_part(reinterpret_cast<lds_v *>(lrr + r2o), xv, rc);
        if (m1 < V(0)) col_part(reinterpret_cast<lds_v *>(lrr + r1o) + 9, xv, rb4);
        if (m0 < V(0)) col_part(reinterpret_cast<lds_v *>(lrr + r0o) + 18, xv, ra);
      }
      // row z complete
      V ow[VEC];
      {
        XV o4[VEC];
        ColVec<XV>::split(own, o4);
#pragma unroll
        for (int q = 0; q < VEC; ++q) ow[q] = (V)o4[q];
      }
      const V mass = fabs(m0);
      const bool row_in = rok & (z >= it.z0);
      const unsigned row = (unsigned)(it.off + it.x0 + lx + it.nx * (it.y0 + ly + it.ny * z));
      V qv[VEC], rn[VEC], pn[VEC];
      if constexpr (MODE == kColCG) {
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          // (explicit fused forms, so that no instantiation contracts them
          // differently; a row without R entries has ra = 0, so y = ka)
          const V y = fma_t(h[q], ra[q], ka[q]);
          qv[q] = fma_t(mass, ow[q], dt * y);
        }
      } else if constexpr (MODE == kColF) {
        // g of the row: after its R stencil (rows without one have g = 0)
        const V g = m0 < V(0) ? reinterpret_cast<lds_v *>(lrr + r0o)[kStencil - 1] : V(0);
#pragma unroll
        for (int q = 0; q < VEC; ++q) qv[q] = fma_t(h[q], g, -fma_t(h[q], ra[q], ka[q]));
      } else if constexpr (PRED) {
        // the row's g (after its R stencil) and, FP64 form, its Jacobi
        // inverse from the stencils' centre values
        lds_v *cr = reinterpret_cast<lds_v *>(lrr + r0o);
        const V g = m0 < V(0) ? cr[kStencil - 1] : V(0);
        const V kd = c0[13], rd = m0 < V(0) ? cr[13] : V(0);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          const V Lx = fma_t(h[q], ra[q], ka[q]);
          const V mt = mass * ow[q];
          const V bq = fma_t(dt, h[q] * g, mt);
          const V rq = bq - fma_t(dt, Lx, mt);
          qv[q] = ow[q];  // x0 = T_{m-1}
          rn[q] = rq;
          if constexpr (MODE == kColPred64) pn[q] = dinv_of(mass, kd, rd, h[q], dt) * rq;
          if (z >= it.z0) {
            const V on_r = (rok & on[q]) ? rq : V(0), on_b = (rok & on[q]) ? bq : V(0);
            if constexpr (MODE == kColPred64) {
              const V on_p = (rok & on[q]) ? pn[q] : V(0);
              v[0][q] = fma_t(on_r, on_p, v[0][q]);
              v[1][q] = fma_t(on_r, on_r, v[1][q]);
              v[2][q] = fma_t(on_b, on_b, v[2][q]);
            } else {
              v[0][q] = fma_t(on_r, on_r, v[0][q]);
              v[1][q] = fma_t(on_b, on_b, v[1][q]);
            }
          }
        }
      } else {
        // T += d, r -= M d + dtau L d where the scenario still refines; the
        // loaded values elsewhere.  Row z's values landed once no more than
        // the copies of the stage issued after them are in flight.
        col_wait_copies<CC, 0>(w);
        V tl[VEC], rl[VEC];
        {
          const char *src = reinterpret_cast<const char *>(&L.io[0]) + w * 4096 + lane * UB;
#pragma unroll
          for (int k = 0; k < LD; ++k) {
            const int u = k % (LD / 2);
            char *dv = reinterpret_cast<char *>(k < LD / 2 ? tl : rl) + u * UB;
            if constexpr (UB == 16)
              *reinterpret_cast<uint4 *>(dv) = *reinterpret_cast<const uint4 *>(src + k * 64 * UB);
            else
              *reinterpret_cast<unsigned *>(dv) =
                  *reinterpret_cast<const unsigned *>(src + k * 64 * UB);
          }
        }
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          const V y = fma_t(h[q], ra[q], ka[q]);
          const V rq = rl[q] - fma_t(mass, ow[q], dt * y);
          qv[q] = on[q] ? tl[q] + ow[q] : tl[q];
          rn[q] = on[q] ? rq : rl[q];
        }
      }
      // p.q (r.r) over the run's rows (wave-uniform test: the rows below the
      // run come from records that were never copied); a masked lane adds an
      // exact zero (rows outside the body have zero records, so finite q)
      if ((MODE == kColCG || REF) && z >= it.z0) {
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          if constexpr (REF) {
            const V rr = (rok & on[q]) ? rn[q] : V(0);
            v[0][q] = fma_t(rr, rr, v[0][q]);
          } else {
            const V om = (rok & on[q]) ? ow[q] : V(0);
            v[0][q] = fma_t((double)om, (double)qv[q], v[0][q]);
          }
        }
      }
      // a fixed number of stores per step whatever the masks (a masked
      // store's offset lies past the buffer, so it is dropped)
      const unsigned off = (row * (unsigned)S + (unsigned)s0) * (unsigned)RVB;
      typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
      typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
      if constexpr (UB == 16) {
        const bool st = row_in & (s0 < S);
#pragma unroll
        for (int k = 0; k < VEC * RVB / 16; ++k) {
          const int o = (int)((off + 16u * k) | ((unsigned)!st << 31));
          u32x4 val;
          __builtin_memcpy(&val, &qv[k * 16 / RVB], 16);
          __builtin_amdgcn_raw_buffer_store_b128(val, qres, o, 0, 0);
          if constexpr (NOUT >= 2) {
            __builtin_memcpy(&val, &rn[k * 16 / RVB], 16);
            __builtin_amdgcn_raw_buffer_store_b128(val, rres, o, 0, 0);
          }
          if constexpr (NOUT >= 3) {
            __builtin_memcpy(&val, &pn[k * 16 / RVB], 16);
            __builtin_amdgcn_raw_buffer_store_b128(val, pres, o, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          const bool st = row_in & on[q];
          const int o = (int)((off + (unsigned)(RVB * q)) | ((unsigned)!st << 31));
          if constexpr (RVB == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(qv[q]), qres, o, 0, 0);
          } else {
            u32x2 val;
            __builtin_memcpy(&val, &qv[q], 8);
            __builtin_amdgcn_raw_buffer_store_b64(val, qres, o, 0, 0);
            if constexpr (NOUT >= 2) {
              __builtin_memcpy(&val, &rn[q], 8);
              __builtin_amdgcn_raw_buffer_store_b64(val, rres, o, 0, 0);
            }
            if constexpr (NOUT >= 3) {
              __builtin_memcpy(&val, &pn[q], 8);
              __builtin_amdgcn_raw_buffer_store_b64(val, pres, o, 0, 0);
            }
          }
        }
      }
      own = xv[4];
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        ka[q] = kb4[q];
        kb4[q] = kc[q];
        ra[q] = rb4[q];
        rb4[q] = rc[q];
      }
      col_wait_wave<CC, ST, D, LD>(w, min(z - zb, D - 1));
      col_barrier();    // stage z + 1 landed; plane z + 1 and the record of z free
      load_row(z + 1);  // (REF)
      ci.issue(it, L);  // stage z + 1 + D
      xro = xro + XB == NX * XB ? 0u : xro + XB;
      r0o = r1o;
    }
  }
  __syncthreads();  // every copy landed before the LDS is reused (or freed)
  if constexpr (MODE != kColF)
    publish_col<XV, NV>(v, a.partial, gridDim.x, S, s0, reinterpret_cast<double *>(L.x[0]));
}

// ---------------------------------------------------------------------------
// Row-group kernels: the CG vector updates with the lane mapping of the tiled
// kernels (a lane owns VEC consecutive scenarios of a row, a wave RPW
// consecutive rows at once), so each load moves 16 bytes per lane and a wave
// touches RPW whole scenario lines.  Groups of RPW rows are dealt per XCD like
// the rows of xcd_rows; a lane's partial sums run over its own rows in
// sequence, whatever S is.
// ---------------------------------------------------------------------------
struct GroupRange {
  int64_t g, end, stride;
};
__device__ inline GroupRange xcd_groups(int64_t G) {
  const int xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd, per = gridDim.x / kXcd;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  GroupRange r;
  r.g = G * xcd / kXcd + (int64_t)local * (kBlock / 64) + w;
  r.end = G * (xcd + 1) / kXcd;
  r.stride = (int64_t)per * (kBlock / 64);
  return r;
}
constexpr int kGroupsAhead = 4;  // row groups of a lane in flight (default)

// VEC values of scenarios s0.. of element base (AL: one 16-byte access; else
// element by element, lanes past S untouched)
template <typename V, int VEC, bool AL>
__device__ __forceinline__ void vload(const V *p, int64_t base, int s0, int S, V (&o)[VEC]) {
  if constexpr (AL) {
    if constexpr (VEC == 4) {
      const float4 f = *reinterpret_cast<const float4 *>(p + base);
      o[0] = f.x; o[1] = f.y; o[2] = f.z; o[3] = f.w;
    } else {
      const double2 d = *reinterpret_cast<const double2 *>(p + base);
      o[0] = d.x; o[1] = d.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) o[k] = s0 + k < S ? p[base + k] : (V)0;
  }
}
template <typename V, int VEC, bool AL>
__device__ __forceinline__ void vstore(V *p, int64_t base, int s0, int S, const V (&o)[VEC]) {
  if constexpr (AL) {
    if constexpr (VEC == 4) {
      *reinterpret_cast<float4 *>(p + base) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
      *reinterpret_cast<double2 *>(p + base) = make_double2(o[0], o[1]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k)
      if (s0 + k < S) p[base + k] = o[k];
  }
}

// (b) r -= alpha q; partial r.z, r.r; GA row groups of a lane in flight (any
// GA gives the same results).  x += alpha p waits for the update (c), which
// reads p anyway: (b) moves only q and r.
template <typename V, bool AL, int GA>
__global__ __launch_bounds__(kBlock) void kb_pcg_b(BatchArgs a, int m, double dtau) {
  using LY = Lanes<V>;
  constexpr int VEC = LY::VEC, RPW = LY::RPW;
  const int S = a.S, lane = threadIdx.x & 63;
  const int lr = lane / LY::LPR, s0 = (lane % LY::LPR) * VEC;
  bool on[VEC], any = false;
  double h[VEC];
  V alpha[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const int s = s0 + k, sc = s < S ? s : 0;
    on[k] = lane_on(a.sc, s, S);
    h[k] = on[k] ? a.h[sc] : 0.0;
    alpha[k] = on[k] ? (V)a.sc->alpha[sc] : (V)0;
    any |= on[k];
  }
  double v[2][VEC] = {};
  V *rv = BV<V>::r(a);
  const V *q = BV<V>::q(a);
  const int64_t N = a.N, G = (N + RPW - 1) / RPW;
  if (__ballot(any) != 0ull) {  // some lane of the wave has work
    for (GroupRange gr = xcd_groups(G); gr.g < gr.end; gr.g += GA * gr.stride) {
      V qs[GA][VEC], rs[GA][VEC];
      double ms[GA], kd[GA], rd[GA];
      bool ok[GA];
#pragma unroll
      for (int u = 0; u < GA; ++u) {
        const int64_t g = gr.g + u * gr.stride, row = g * RPW + lr;
        ok[u] = (g < gr.end) & (row < N) & (s0 < S);
        const int64_t rw = ok[u] ? row : 0, base = rw * S + (s0 < S ? s0 : 0);
        vload<V, VEC, AL>(q, base, s0, S, qs[u]);
        vload<V, VEC, AL>(rv, base, s0, S, rs[u]);
        ms[u] = a.mass[rw];
        kd[u] = a.Kd[rw];
        rd[u] = a.Rd[rw];
      }
#pragma unroll
      for (int u = 0; u < GA; ++u) {
        if (!ok[u]) continue;
        const int64_t row = (gr.g + u * gr.stride) * RPW + lr, base = row * S + s0;
        V di[VEC];
        dinv_row<V, VEC>(ms[u], kd[u], rd[u], h, dtau, di);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          if (!on[k]) continue;  // idle scenarios keep their values
          // (explicit fused forms: every instantiation rounds alike)
          const V r = fma_t(-alpha[k], qs[u][k], rs[u][k]);
          rs[u][k] = r;
          const V z = di[k] * r;
          v[0][k] = fma_t((double)r, (double)z, v[0][k]);
          v[1][k] = fma_t((double)r, (double)r, v[1][k]);
        }
        vstore<V, VEC, AL>(rv, base, s0, S, rs[u]);
      }
    }
  }
  publish_groups<2, VEC, RPW>(v, a.partial, gridDim.x, S);
}

// p_new = dinv r + beta p with one explicit rounding pattern, whatever code
// path (and therefore contraction choice) computes it
__device__ __forceinline__ float pupdate(float di, float r, float beta, float p) {
  return __builtin_fmaf(di, r, beta * p);
}
__device__ __forceinline__ double pupdate(double di, double r, double beta, double p) {
  return __builtin_fma(di, r, beta * p);
}

// (c) x += alpha p, then p = z + beta p, row groups as in (b), GA of a lane in
// flight.  x moves for every scenario that iterated in this iteration (it),
// including one whose solve the check after (b) has just found converged;
// p only for the scenarios still iterating.
template <typename V, bool AL, int GA>
__global__ __launch_bounds__(kBlock) void kb_pcg_c(BatchArgs a, int m, double dtau, int it) {
  using LY = Lanes<V>;
  constexpr int VEC = LY::VEC, RPW = LY::RPW;
  const int S = a.S, lane = threadIdx.x & 63;
  const int lr = lane / LY::LPR, s0 = (lane % LY::LPR) * VEC;
  bool on[VEC], mv[VEC], any = false;
  double h[VEC];
  V alpha[VEC], beta[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const int s = s0 + k, sc = s < S ? s : 0;
    on[k] = lane_on(a.sc, s, S);
    mv[k] = on[k] | (sweeping(a.sc, s, S) & (a.sc->ref_done[sc] == 0) & (a.sc->done[sc] != 0) &
                     (a.sc->done_it[sc] == it));
    h[k] = on[k] ? a.h[sc] : 0.0;
    alpha[k] = mv[k] ? (V)a.sc->alpha[sc] : (V)0;
    beta[k] = on[k] ? (V)a.sc->beta[sc] : (V)0;
    any |= mv[k];
  }
  if (__ballot(any) == 0ull) return;  // no lane of the wave has work
  V *p = BV<V>::p(a), *x = BV<V>::x(a, m);
  const V *rv = BV<V>::r(a);
  const int64_t N = a.N, G = (N + RPW - 1) / RPW;
  for (GroupRange gr = xcd_groups(G); gr.g < gr.end; gr.g += GA * gr.stride) {
    V ps[GA][VEC], rs[GA][VEC], xs[GA][VEC];
    double ms[GA], kd[GA], rd[GA];
    bool ok[GA];
#pragma unroll
    for (int u = 0; u < GA; ++u) {
      const int64_t g = gr.g + u * gr.stride, row = g * RPW + lr;
      ok[u] = (g < gr.end) & (row < N) & (s0 < S);
      const int64_t rw = ok[u] ? row : 0, base = rw * S + (s0 < S ? s0 : 0);
      vload<V, VEC, AL>(p, base, s0, S, ps[u]);
      vload<V, VEC, AL>(rv, base, s0, S, rs[u]);
      vload<V, VEC, AL>(x, base, s0, S, xs[u]);
      ms[u] = a.mass[rw];
      kd[u] = a.Kd[rw];
      rd[u] = a.Rd[rw];
    }
#pragma unroll
    for (int u = 0; u < GA; ++u) {
      if (!ok[u]) continue;
      const int64_t row = (gr.g + u * gr.stride) * RPW + lr, base = row * S + s0;
      V di[VEC];
      dinv_row<V, VEC>(ms[u], kd[u], rd[u], h, dtau, di);
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        if (mv[k]) xs[u][k] = fma_t(alpha[k], ps[u][k], xs[u][k]);
        if (on[k]) ps[u][k] = pupdate(di[k], rs[u][k], beta[k], ps[u][k]);
      }
      vstore<V, VEC, AL>(x, base, s0, S, xs[u]);
      vstore<V, VEC, AL>(p, base, s0, S, ps[u]);
    }
  }
}

// inner init of the FP32 form: r32 = r64, x32 = 0, p32 = dinv r32; partial
// r.z, r.r.  Row groups as in (b) (16-byte accesses); a lane's values of
// scenarios that do not refine are written too (no later step of theirs
// reads them).
template <bool AL, int GA>
__global__ __launch_bounds__(kBlock) void kb_inner_init(BatchArgs a, double dtau) {
  using LY = Lanes<float>;
  constexpr int VEC = LY::VEC, RPW = LY::RPW;
  const int S = a.S, lane = threadIdx.x & 63;
  const int lr = lane / LY::LPR, s0 = (lane % LY::LPR) * VEC;
  bool on[VEC], any = false;
  double h[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const int s = s0 + k, sc = s < S ? s : 0;
    on[k] = sweeping(a.sc, s, S) & (a.sc->ref_done[sc] == 0);
    h[k] = on[k] ? a.h[sc] : 0.0;
    any |= on[k];
  }
  double v[2][VEC] = {};
  const int64_t N = a.N, G = (N + RPW - 1) / RPW;
  if (__ballot(any) != 0ull) {
    for (GroupRange gr = xcd_groups(G); gr.g < gr.end; gr.g += GA * gr.stride) {
      double rs[GA][VEC], ms[GA], kd[GA], rd[GA];
      bool ok[GA];
#pragma unroll
      for (int u = 0; u < GA; ++u) {
        const int64_t g = gr.g + u * gr.stride, row = g * RPW + lr;
        ok[u] = (g < gr.end) & (row < N) & (s0 < S);
        const int64_t rw = ok[u] ? row : 0, base = rw * S + (s0 < S ? s0 : 0);
        if constexpr (AL) {
          const double2 d0 = *reinterpret_cast<const double2 *>(a.r64 + base);
          const double2 d1 = *reinterpret_cast<const double2 *>(a.r64 + base + 2);
          rs[u][0] = d0.x;
          rs[u][1] = d0.y;
          rs[u][2] = d1.x;
          rs[u][3] = d1.y;
        } else {
#pragma unroll
          for (int k = 0; k < VEC; ++k) rs[u][k] = s0 + k < S ? a.r64[base + k] : 0.0;
        }
        ms[u] = a.mass[rw];
        kd[u] = a.Kd[rw];
        rd[u] = a.Rd[rw];
      }
#pragma unroll
      for (int u = 0; u < GA; ++u) {
        if (!ok[u]) continue;
        const int64_t row = (gr.g + u * gr.stride) * RPW + lr, base = row * S + s0;
        float di[VEC], r[VEC], z[VEC];
        const float zero[VEC] = {};
        dinv_row<float, VEC>(ms[u], kd[u], rd[u], h, dtau, di);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          r[k] = (float)rs[u][k];
          z[k] = di[k] * r[k];
          if (!on[k]) continue;
          v[0][k] = fma_t((double)r[k], (double)z[k], v[0][k]);
          v[1][k] = fma_t((double)r[k], (double)r[k], v[1][k]);
        }
        vstore<float, VEC, AL>(a.r32, base, s0, S, r);
        vstore<float, VEC, AL>(a.x32, base, s0, S, zero);
        vstore<float, VEC, AL>(a.p32, base, s0, S, z);
      }
    }
  }
  publish_groups<2, VEC, RPW>(v, a.partial, gridDim.x, S);
}

// ---------------------------------------------------------------------------
// interface substeps, per scenario (tables with the scenario index fastest)
// ---------------------------------------------------------------------------
__device__ inline void hat3(const double *x, int n, int a, double sft, double *l, double *m,
                            double *h) {
  *l = x[a > 0 ? a - 1 : a] + sft;
  *m = x[a] + sft;
  *h = x[a < n - 1 ? a + 1 : a] + sft;
}

__device__ inline int bfirst_hat_after(const double *y, int n, double sy, double t) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double end = y[mid < n - 1 ? mid + 1 : mid] + sy;
    if (end > t) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// one block per (time point, scenario)
__global__ __launch_bounds__(kBlock) void kb_iface_coeffs(BatchArgs a) {
  const IfaceDev &f = a.f;
  const int S = a.S, P1 = a.P + 1;
  const int tp = blockIdx.x / S, s = blockIdx.x - tp * S;
  const int m = tp / P1, q = tp - m * P1;
  const Weights &w = *a.w;
  if (m == 0 || w.dtau[m] == 0.0 || !a.sc->active[s]) return;
  const CoefLayout L{f.nvf, f.nvm};
  double *D = a.coefD + (size_t)tp * L.dstride() * S;
  int *I = a.coefI + (size_t)tp * L.istride() * S;
  const double t = a.tn[s] + w.tau[m - 1] + q * (w.dtau[m] / a.P);
  const double sv = f.s0 + f.a * sin(2.0 * M_PI * t / a.period[s] + f.phase);
  const double ov0 = fmax(f.vf[0], f.vm[0] + sv), ov1 = fmin(f.vf[f.nvf - 1], f.vm[f.nvm - 1] + sv);
  const bool valid = (f.ou1 > f.ou0) && (ov1 > ov0);
  if (threadIdx.x == 0)
    D[0 * S + s] = valid ? a.Pf[s] / ((f.ou1 - f.ou0) * (ov1 - ov0)) : 0.0;
  for (int b = threadIdx.x; b < f.nvf; b += blockDim.x) {
    for (int i = 0; i < 3; ++i) {
      const int bb = b - 1 + i;
      D[(size_t)(L.Mv() + 3 * b + i) * S + s] =
          (bb >= 0 && bb < f.nvf && valid)
              ? hat_product_integral(f.vf, f.nvf, b, f.vf, f.nvf, bb, 0.0, ov0, ov1)
              : 0.0;
    }
    D[(size_t)(L.Hv() + b) * S + s] = valid ? hat_integral(f.vf, f.nvf, b, ov0, ov1) : 0.0;
    const int d0 = bfirst_hat_after(f.vm, f.nvm, sv, f.vf[b > 0 ? b - 1 : b]);
    int cnt = 0;
    for (int i = 0; i < kBand; ++i) {
      const int d = d0 + i;
      const double v = (d < f.nvm && valid)
                           ? hat_product_integral(f.vf, f.nvf, b, f.vm, f.nvm, d, sv, ov0, ov1)
                           : 0.0;
      D[(size_t)(L.Cv() + kBand * b + i) * S + s] = v;
      if (v != 0.0) cnt = i + 1;
    }
    I[(size_t)(L.dlo() + b) * S + s] = d0;
    I[(size_t)(L.dcnt() + b) * S + s] = cnt;
  }
  for (int d = threadIdx.x; d < f.nvm; d += blockDim.x) {
    for (int i = 0; i < 3; ++i) {
      const int dd = d - 1 + i;
      D[(size_t)(L.Nv() + 3 * d + i) * S + s] =
          (dd >= 0 && dd < f.nvm && valid)
              ? hat_product_integral(f.vm, f.nvm, d, f.vm, f.nvm, dd, 0.0, ov0 - sv, ov1 - sv)
              : 0.0;
    }
    D[(size_t)(L.Gv() + d) * S + s] = valid ? hat_integral(f.vm, f.nvm, d, ov0 - sv, ov1 - sv) : 0.0;
    const int b0 = bfirst_hat_after(f.vf, f.nvf, 0.0, f.vm[d > 0 ? d - 1 : d] + sv);
    int cnt = 0;
    for (int i = 0; i < kBand; ++i) {
      const int b = b0 + i;
      const double v = (b < f.nvf && valid)
                           ? hat_product_integral(f.vf, f.nvf, b, f.vm, f.nvm, d, sv, ov0, ov1)
                           : 0.0;
      D[(size_t)(L.CvT() + kBand * d + i) * S + s] = v;
      if (v != 0.0) cnt = i + 1;
    }
    I[(size_t)(L.blo() + d) * S + s] = b0;
    I[(size_t)(L.bcnt() + d) * S + s] = cnt;
  }
}

template <bool FIRST>
__device__ inline double btif(const BatchArgs &a, const double *Tprev, const double *Tin, int j,
                              int s) {
  return FIRST ? Tprev[a.f.rows[j] * a.S + s] : Tin[(size_t)j * a.S + s];
}

// Coupling sums of one interface point for scenario s, with the fixed trip
// counts of the single-simulation form: clamped indices with zero weights for
// the 3 x 3 self stencil and for a cross band of at most kBFastBand by
// kBFastBand (the general loop otherwise), so every gather is issued before
// the first is waited for; the products are added in the plain loops' order.
constexpr int kBFastBand = 4;

template <bool FIRST>
__device__ inline double bself(const BatchArgs &a, const double *Tprev, const double *Tin,
                               const double *wu, const double *D, int kv, int nu, int nv,
                               int base, int ua, int b, int s) {
  const int S = a.S;
  double w0[3], w1[3];
  int ra[3], cb[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int aa = ua - 1 + q, bb = b - 1 + q;
    const bool ia = aa >= 0 && aa < nu, ib = bb >= 0 && bb < nv;
    ra[q] = ia ? aa : ua;
    cb[q] = ib ? bb : b;
    w0[q] = ia ? wu[3 * ua + q] : 0.0;
    w1[q] = ib ? D[(size_t)(kv + 3 * b + q) * S + s] : 0.0;
  }
  double t[3][3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int r = 0; r < 3; ++r) t[q][r] = btif<FIRST>(a, Tprev, Tin, base + ra[q] * nv + cb[r], s);
  double self = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) acc += w1[r] * t[q][r];
    self += w0[q] * acc;
  }
  return self;
}

// sum_{q < nu} cu[q] sum_{r < nv} D(kv + r) T(base + (u0 + q) * ld + v0 + r)
template <bool FIRST>
__device__ inline double bcross(const BatchArgs &a, const double *Tprev, const double *Tin,
                                const double *cu, const double *D, int kv, int u0, int nu, int v0,
                                int nv, int ld, int base, int s) {
  const int S = a.S;
  double cross = 0.0;
  if (nu <= 0 || nv <= 0) return cross;  // no overlap: the band start may lie off the grid
  if (nu <= kBFastBand && nv <= kBFastBand) {
    double wu[kBFastBand], wv[kBFastBand], t[kBFastBand][kBFastBand];
#pragma unroll
    for (int q = 0; q < kBFastBand; ++q) {
      wu[q] = q < nu ? cu[q] : 0.0;
      wv[q] = q < nv ? D[(size_t)(kv + q) * S + s] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kBFastBand; ++q)
#pragma unroll
      for (int r = 0; r < kBFastBand; ++r)
        t[q][r] = btif<FIRST>(a, Tprev, Tin,
                              base + (u0 + (q < nu ? q : 0)) * ld + v0 + (r < nv ? r : 0), s);
#pragma unroll
    for (int q = 0; q < kBFastBand; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < kBFastBand; ++r) acc += wv[r] * t[q][r];
      cross += wu[q] * acc;
    }
    return cross;
  }
  for (int q = 0; q < nu; ++q) {
    double acc = 0.0;
    for (int r = 0; r < nv; ++r)
      acc += D[(size_t)(kv + r) * S + s] * btif<FIRST>(a, Tprev, Tin, base + (u0 + q) * ld + v0 + r, s);
    cross += cu[q] * acc;
  }
  return cross;
}

template <bool FIRST>
__device__ double bfE(const BatchArgs &a, const double *D, const int *I, const double *Tprev,
                      const double *Tin, int i, int s) {
  const IfaceDev &f = a.f;
  const int S = a.S;
  const CoefLayout L{f.nvf, f.nvm};
  const double alpha = a.alpha[s], qf = D[s];
#define DD(k) D[(size_t)(k) * S + s]
#define II(k) I[(size_t)(k) * S + s]
  if (i < f.nfix) {
    const int ua = i / f.nvf, b = i - ua * f.nvf;
    const double self = bself<FIRST>(a, Tprev, Tin, f.Mu, D, L.Mv(), f.nuf, f.nvf, 0, ua, b, s);
    const double cross =
        bcross<FIRST>(a, Tprev, Tin, f.Cu + kBand * ua, D, L.Cv() + kBand * b, f.clo[ua],
                      f.ccnt[ua], II(L.dlo() + b), II(L.dcnt() + b), f.nvm, f.nfix, s);
    return alpha * (cross - self) + f.split * qf * f.Hu[ua] * DD(L.Hv() + b);
  }
  const int k = i - f.nfix;
  const int c = k / f.nvm, d = k - c * f.nvm;
  const double self = bself<FIRST>(a, Tprev, Tin, f.Nu, D, L.Nv(), f.num, f.nvm, f.nfix, c, d, s);
  const double cross =
      bcross<FIRST>(a, Tprev, Tin, f.CuT + kBand * c, D, L.CvT() + kBand * d, f.alo[c],
                    f.acnt[c], II(L.blo() + d), II(L.bcnt() + d), f.nvf, 0, s);
  return alpha * (cross - self) + (1.0 - f.split) * qf * f.Gu[c] * DD(L.Gv() + d);
#undef DD
#undef II
}

// one wave per interface point, lane = scenario
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void kb_iface_sub(BatchArgs a, int m, int p, int corr) {
  const int s = threadIdx.x & 63, S = a.S;
  const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const IfaceDev &f = a.f;
  const int n = f.n_if;
  if (i >= n || !sweeping(a.sc, s, S)) return;
  const Weights &w = *a.w;
  const int P = a.P, P1 = P + 1;
  const CoefLayout L{f.nvf, f.nvm};
  const int tp = m * P1 + (p - 1);
  const double *D = a.coefD + (size_t)tp * L.dstride() * S;
  const int *I = a.coefI + (size_t)tp * L.istride() * S;
  const double *Tprev = a.T[m - 1];
  double *Tm = a.T[m];
  const double *Tin = a.Tbuf[(p - 1) & 1];
  const double E = bfE<FIRST>(a, D, I, Tprev, Tin, i, s);
  double *En = a.Enew + (size_t)m * P1 * n * S;
  En[((size_t)(p - 1) * n + i) * S + s] = E;
  const double Ti = btif<FIRST>(a, Tprev, Tin, i, s);
  const int64_t row = f.rows[i];
  const int64_t gi = row * S + s;
  if (p == P + 1) {
    Tm[gi] = Ti;
    return;
  }
  const double mi = a.mass[row], dtm = w.dtau[m], dtp = dtm / P;
  double fs;
  if (FIRST) {
    fs = (mi * Tm[gi] - mi * Ti - (corr ? a.I[m][gi] : 0.0)) / dtm;
    a.fst[(size_t)i * S + s] = fs;
  } else {
    fs = a.fst[(size_t)i * S + s];
  }
  double inc;
  if (corr) {
    const double *Eo = a.Eold + (size_t)m * P1 * n * S;
    double Ip = 0.0;
    for (int j = 1; j <= a.M; ++j) Ip += w.stil[m][p][j] * a.F[j][gi];
    for (int q = 1; q <= P; ++q) Ip += w.spq[m][p][q] * Eo[((size_t)q * n + i) * S + s];
    inc = dtp * (fs + E - Eo[((size_t)(p - 1) * n + i) * S + s]) + Ip;
  } else {
    inc = dtp * (fs + E);
  }
  a.Tbuf[p & 1][(size_t)i * S + s] = Ti + inc / mi;
}

// ---------------------------------------------------------------------------
// step bookkeeping
// ---------------------------------------------------------------------------
__global__ void kb_clear(BatchArgs a) {
  BatchScalars *sc = a.sc;
  const int s = threadIdx.x;
  if (s >= a.S) return;
  sc->fail[s] = 0;
  sc->stop[s] = 0;
  sc->sweeps[s] = 0;
  sc->iters_total[s] = 0;
  sc->refine_total[s] = 0;
  for (int k = 0; k < 17; ++k) sc->resid[k][s] = 0.0;
  for (int i = 0; i < kSlots; ++i) {
    sc->slot_iters[i][s] = 0;
    sc->slot_rounds[i][s] = 0;
  }
}

// commit T_n <- T_M and t_n += dt for the active scenarios, unless any failed
__global__ void kb_commit(BatchArgs a, double dt) {
  for (int s = 0; s < a.S; ++s)
    if (a.sc->fail[s]) return;
  const int64_t n = a.N * a.S;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i % a.S);
    if (a.sc->active[s]) a.T[0][i] = a.T[a.M][i];
  }
  if (blockIdx.x == 0 && threadIdx.x < a.S && a.sc->active[threadIdx.x]) a.tn[threadIdx.x] += dt;
}

// column s of an interleaved vector <-> contiguous vector
__global__ void kb_scatter(double *dst, const double *src, int64_t n, int S, int s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i * S + s] = src[i];
}
__global__ void kb_gather(double *dst, const double *src, int64_t n, int S, int s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i * S + s];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void blaunch_clear(const BatchArgs &a, hipStream_t st) { kb_clear<<<1, 64, 0, st>>>(a); }

void blaunch_iface_coeffs(const BatchArgs &a, hipStream_t st) {
  if (!a.f.kind) return;
  kb_iface_coeffs<<<(a.M + 1) * (a.P + 1) * a.S, kBlock, 0, st>>>(a);
}

// 16-byte staging units and aligned lane reads when a row of S values is a
// multiple of 16 bytes
template <typename XT>
static bool vec16(const BatchArgs &a) {
  return (a.S * sizeof(XT)) % 16 == 0;
}

// workgroups of a tiled kernel staging XT values: as many as are resident
// (two FP64 or three FP32 staging buffers per CU), fixed per mesh
template <typename XT>
static int tgrid(const BatchArgs &a) {
  return sizeof(XT) == 8 ? a.sgrid64 : a.sgrid32;
}

#define RED(np, ...) kb_reduce<<<a.S, kBlock, 0, st>>>(a, np, __VA_ARGS__)

void blaunch_f_multi(const BatchArgs &a, int j0, int j1, hipStream_t st) {
  if (a.cgrid_f > 0) {  // the FP64 column sweep, one launch per node
    for (int j = j0; j <= j1; ++j) {
      if (vec16<double>(a))
        kb_pcg_a_col<0, double, 16, kColDepth, kColF><<<a.cgrid_f, kBlock, 0, st>>>(a, j, 0.0);
      else kb_pcg_a_col<0, double, 4, kColDepth, kColF><<<a.cgrid_f, kBlock, 0, st>>>(a, j, 0.0);
    }
    return;
  }
  if (vec16<double>(a)) kb_f_multi<16, true><<<a.sgrid64, kBlock, 0, st>>>(a, j0, j1);
  else kb_f_multi<4, false><<<a.sgrid64, kBlock, 0, st>>>(a, j0, j1);
}

void blaunch_quad_resid(const BatchArgs &a, int k, hipStream_t st) {
  kb_quad_resid<<<a.grid, kBlock, 0, st>>>(a, a.w);
  kb_resid_reduce<<<1, 64 * kRedWaves, 0, st>>>(a, k);
}

int col_workgroups_per_cu(int fp32, int depth) {
  if (fp32) return depth == 1 ? ColOcc<float, float, 1>::W : ColOcc<float, float, kColDepth>::W;
  return depth == 1 ? ColOcc<double, double, 1>::W : ColOcc<double, double, kColDepth>::W;
}

// the column sweep runs the operator of the context's form (its records hold
// that form's values)
template <typename V>
static bool use_columns(const BatchArgs &a) {
  return a.op.ncol_items > 0 && (sizeof(V) == 4) == (a.fp32 != 0);
}

// workgroups of the operator launch
template <typename V>
static int pcg_a_grid(const BatchArgs &a) {
  return use_columns<V>(a) ? a.cgrid : tgrid<V>(a);
}

// the column sweep with D stages in flight (any D gives the same results)
template <typename V, int D>
static void launch_col(const BatchArgs &a, int timing, int g, int m, double dtau, hipStream_t st) {
  if (vec16<V>(a)) {
    if (timing) kb_pcg_a_col<1, V, 16, D><<<g, kBlock, 0, st>>>(a, m, dtau);
    else kb_pcg_a_col<0, V, 16, D><<<g, kBlock, 0, st>>>(a, m, dtau);
  } else {
    if (timing) kb_pcg_a_col<1, V, 4, D><<<g, kBlock, 0, st>>>(a, m, dtau);
    else kb_pcg_a_col<0, V, 4, D><<<g, kBlock, 0, st>>>(a, m, dtau);
  }
}

template <typename V>
static void launch_pcg_a(const BatchArgs &a, int timing, int m, double dtau, hipStream_t st) {
  if (use_columns<V>(a)) {
    const int g = pcg_a_grid<V>(a);
    if (a.col_depth == 1) launch_col<V, 1>(a, timing, g, m, dtau, st);
    else launch_col<V, kColDepth>(a, timing, g, m, dtau, st);
    return;
  }
  const int g = tgrid<V>(a);
  if (vec16<V>(a)) {
    if (timing) kb_pcg_a<1, V, 16, true><<<g, kBlock, 0, st>>>(a, m, dtau);
    else kb_pcg_a<0, V, 16, true><<<g, kBlock, 0, st>>>(a, m, dtau);
  } else {
    if (timing) kb_pcg_a<1, V, 4, false><<<g, kBlock, 0, st>>>(a, m, dtau);
    else kb_pcg_a<0, V, 4, false><<<g, kBlock, 0, st>>>(a, m, dtau);
  }
}

// Workgroups of a grid-stride launch of fn: at most want, every one resident
// at once (a launch larger than what fits runs a second, partial round), a
// multiple of the 8 XCDs
static int resident_grid(const void *fn, int want) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kBlock, 0) != hipSuccess)
    return want;
  const int fit = per * cus / kXcd * kXcd;
  return fit >= kXcd ? std::min(want, fit) : want;
}

void set_resident_grids(BatchArgs &a) {
  // from the default variant, whatever the tuner picks later: the grid sets
  // the partial sums, so it stays fixed
  a.bgrid32 = std::min(resident_grid((const void *)kb_pcg_b<float, true, kGroupsAhead>, a.grid),
                       resident_grid((const void *)kb_pcg_b<float, false, kGroupsAhead>, a.grid));
  a.bgrid64 = std::min(resident_grid((const void *)kb_pcg_b<double, true, kGroupsAhead>, a.grid),
                       resident_grid((const void *)kb_pcg_b<double, false, kGroupsAhead>, a.grid));
}

template <typename V>
static int pcg_b_grid(const BatchArgs &a) {
  return std::is_same<V, float>::value ? a.bgrid32 : a.bgrid64;
}

template <typename V, int GA>
static void launch_pcg_b_ga(const BatchArgs &a, int m, double dtau, hipStream_t st) {
  if (vec16<V>(a)) kb_pcg_b<V, true, GA><<<pcg_b_grid<V>(a), kBlock, 0, st>>>(a, m, dtau);
  else kb_pcg_b<V, false, GA><<<pcg_b_grid<V>(a), kBlock, 0, st>>>(a, m, dtau);
}
template <typename V>
static void launch_pcg_b(const BatchArgs &a, int m, double dtau, hipStream_t st) {
  if (a.groups_b == 2) launch_pcg_b_ga<V, 2>(a, m, dtau, st);
  else launch_pcg_b_ga<V, kGroupsAhead>(a, m, dtau, st);
}
template <typename V, int GA>
static void launch_pcg_c_ga(const BatchArgs &a, int m, double dtau, int it, hipStream_t st) {
  if (vec16<V>(a)) kb_pcg_c<V, true, GA><<<a.grid, kBlock, 0, st>>>(a, m, dtau, it);
  else kb_pcg_c<V, false, GA><<<a.grid, kBlock, 0, st>>>(a, m, dtau, it);
}
template <typename V>
static void launch_pcg_c(const BatchArgs &a, int m, double dtau, int it, hipStream_t st) {
  if (a.groups_c == 8) launch_pcg_c_ga<V, 8>(a, m, dtau, it, st);
  else launch_pcg_c_ga<V, kGroupsAhead>(a, m, dtau, it, st);
}

template <typename V>
static void cg_iterations(const BatchArgs &a, int m, double dtau, int slot, int budget,
                          double rtol, hipStream_t st) {
  const int conv = std::is_same<V, float>::value ? 6 : 2;
  const int gb = pcg_b_grid<V>(a);
  for (int it = 0; it < budget; ++it) {
    launch_pcg_a<V>(a, 0, m, dtau, st);
    RED(pcg_a_grid<V>(a), 1, it, 0, slot, rtol);
    launch_pcg_b<V>(a, m, dtau, st);
    RED(gb, conv, it, it == budget - 1, slot, rtol);
    launch_pcg_c<V>(a, m, dtau, it, st);
  }
}

template <int NV>
static void launch_init(const BatchArgs &a, bool pred, int m, double dtau, hipStream_t st) {
  if (!pred) {
    kb_init_corr<NV><<<a.grid, kBlock, 0, st>>>(a, m, dtau);
    return;
  }
  // the FP64 column sweep of T_{m-1} (its NV partial sums per workgroup must
  // fit the partial-sum buffer)
  if (a.cgrid_f > 0 && (int64_t)NV * a.cgrid_f <= 3 * (int64_t)a.pgrid) {
    constexpr int MODE = NV == 3 ? kColPred64 : kColPred32;
    if (vec16<double>(a))
      kb_pcg_a_col<0, double, 16, kColDepth, MODE><<<a.cgrid_f, kBlock, 0, st>>>(a, m, dtau);
    else kb_pcg_a_col<0, double, 4, kColDepth, MODE><<<a.cgrid_f, kBlock, 0, st>>>(a, m, dtau);
    return;
  }
  if (vec16<double>(a)) kb_init_pred<NV, 16, true><<<a.sgrid64, kBlock, 0, st>>>(a, m, dtau);
  else kb_init_pred<NV, 4, false><<<a.sgrid64, kBlock, 0, st>>>(a, m, dtau);
}

void blaunch_solve(const BatchArgs &a, const BSolve &sv, hipStream_t st) {
  const int m = sv.m;
  const double dtau = a.dtau_h[m];
  // workgroups of the init kernel (as launch_init picks it)
  const int nvi = a.fp32 ? 2 : 3;
  const bool psweep = a.cgrid_f > 0 && (int64_t)nvi * a.cgrid_f <= 3 * (int64_t)a.pgrid;
  const int npi = sv.pred ? (psweep ? a.cgrid_f : a.sgrid64) : a.grid;
  if (!a.fp32) {
    launch_init<3>(a, sv.pred, m, dtau, st);
    RED(npi, 0, 0, 0, sv.slot, sv.rtol);
    cg_iterations<double>(a, m, dtau, sv.slot, sv.budget, sv.rtol, st);
    return;
  }
  // FP32 inner solves inside FP64 refinement rounds
  launch_init<2>(a, sv.pred, m, dtau, st);
  RED(npi, 3, 0, 0, sv.slot, sv.refine_rtol);
  for (int r = 0; r < sv.rounds; ++r) {
    const int gi = pcg_b_grid<float>(a);
    if (vec16<float>(a)) kb_inner_init<true, kGroupsAhead><<<gi, kBlock, 0, st>>>(a, dtau);
    else kb_inner_init<false, kGroupsAhead><<<gi, kBlock, 0, st>>>(a, dtau);
    RED(gi, 4, 0, 0, sv.slot, sv.inner_rtol);
    cg_iterations<float>(a, m, dtau, sv.slot, sv.budget, sv.inner_rtol, st);
    int gr = a.sgrid32;
    if (a.cgrid > 0 && a.op.kcol64) {  // the FP64-stencil column sweep of the correction
      gr = a.cgrid;
      if (vec16<float>(a))
        kb_pcg_a_col<0, double, 16, kColDepth, kColRefine><<<gr, kBlock, 0, st>>>(a, m, dtau);
      else kb_pcg_a_col<0, double, 4, kColDepth, kColRefine><<<gr, kBlock, 0, st>>>(a, m, dtau);
    } else if (vec16<float>(a)) {
      kb_refine_update<16, true><<<gr, kBlock, 0, st>>>(a, m, dtau);
    } else {
      kb_refine_update<4, false><<<gr, kBlock, 0, st>>>(a, m, dtau);
    }
    RED(gr, 5, r, r == sv.rounds - 1, sv.slot, sv.refine_rtol);
  }
}
#undef RED

void blaunch_tune(const BatchArgs &a, int which, int reps, hipStream_t st) {
  int m = 1;
  while (m <= a.M && a.dtau_h[m] == 0.0) ++m;
  const double dtau = a.dtau_h[m];
  for (int i = 0; i < reps; ++i) {
    if (which == 0 && !a.fp32) launch_pcg_a<double>(a, 1, m, dtau, st);
    else if (which == 0) launch_pcg_a<float>(a, 1, m, dtau, st);
    else if (which == 1) launch_pcg_b<float>(a, m, dtau, st);
    else launch_pcg_c<float>(a, m, dtau, 0, st);
  }
}

void blaunch_operator_timing(const BatchArgs &a, int m, int reps, hipStream_t st) {
  for (int i = 0; i < reps; ++i) {
    if (a.fp32) launch_pcg_a<float>(a, 1, m, a.dtau_h[m], st);
    else launch_pcg_a<double>(a, 1, m, a.dtau_h[m], st);
  }
}

void blaunch_iface(const BatchArgs &a, int m, bool corr, hipStream_t st) {
  if (!a.f.kind) return;
  const int grid = (a.f.n_if + kBlock / 64 - 1) / (kBlock / 64);
  for (int p = 1; p <= a.P + 1; ++p) {
    if (p == 1) kb_iface_sub<true><<<grid, kBlock, 0, st>>>(a, m, p, corr ? 1 : 0);
    else kb_iface_sub<false><<<grid, kBlock, 0, st>>>(a, m, p, corr ? 1 : 0);
  }
}

void blaunch_commit(const BatchArgs &a, double dt, hipStream_t st) {
  int grid = (int)std::min<int64_t>((a.N * a.S + kBlock - 1) / kBlock, 4096);
  kb_commit<<<grid, kBlock, 0, st>>>(a, dt);
}

void blaunch_scatter(double *dst, const double *src, int64_t n, int S, int s, hipStream_t st) {
  kb_scatter<<<1024, kBlock, 0, st>>>(dst, src, n, S, s);
}
void blaunch_gather(double *dst, const double *src, int64_t n, int S, int s, hipStream_t st) {
  kb_gather<<<1024, kBlock, 0, st>>>(dst, src, n, S, s);
}

}  // namespace mrsdc
