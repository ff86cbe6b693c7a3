// Thermo-elastic deformation on the device: the stiffness K_u is banded with
// half-bandwidth <= bs, so cut into blocks of bs rows it is block tridiagonal.
// Block LU (block Gaussian elimination):
//   S_0 = A_00,  S_k = A_kk - A_{k,k-1} W_{k-1} A_{k-1,k},  W_k = S_k^{-1}
//   forward   w_k = W_k (f_k - A_{k,k-1} w_{k-1})
//   backward  u_k = w_k - W_k A_{k,k+1} u_{k+1}   (u_last = w_last)
// W_k is dense (the fill of the band), kept padded to bp (a multiple of 64)
// with an identity in the padding.  S_k is inverted in place by blocked
// Gauss-Jordan elimination with 64 x 64 pivot tiles; no pivoting is needed
// because S_k is symmetric positive definite (a Schur complement of an SPD
// matrix).  The solves are bandwidth-bound dense products with the W_k.
#include <hip/hip_ext.h>

#include "deform_internal.h"

namespace mrsdc {

namespace {

constexpr int kT = kGjTile;
constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// factorisation
// ---------------------------------------------------------------------------

// T1 = A_{k,k-1} W_{k-1}: row i of T1 combines the W_{k-1} rows named by the
// entries of row i of the coupling block.
__global__ __launch_bounds__(kThreads) void k_schur_t(DeformDev D, int64_t k) {
  __shared__ double sv[128];
  __shared__ int sc[128];
  const int64_t i = blockIdx.x;
  const int64_t bp = D.bp;
  const int E = D.ellB;
  const int64_t eb = k * (int64_t)E * bp;
  for (int e = threadIdx.x; e < E; e += kThreads) {
    sv[e] = D.bval[eb + e * bp + i];
    sc[e] = D.bcol[eb + e * bp + i];
  }
  __syncthreads();
  const double *Wp = D.W + (k - 1) * bp * bp;
  double *out = D.T1 + i * bp;
  for (int64_t j = threadIdx.x; j < bp; j += kThreads) {
    double a = 0.0;
    for (int e = 0; e < E; ++e) a = fma(sv[e], Wp[(int64_t)sc[e] * bp + j], a);
    out[j] = a;
  }
}

// Row i of S_k = A_kk - T1 A_{k,k-1}^T (k > 0), padded with the identity.
__global__ __launch_bounds__(kThreads) void k_schur_s(DeformDev D, int64_t k) {
  extern __shared__ double trow[];
  const int64_t i = blockIdx.x;
  const int64_t bp = D.bp, bk = D.rows(k), lo = D.lo(k);
  double *S = D.W + k * bp * bp + i * bp;
  if (i >= bk) {
    for (int64_t j = threadIdx.x; j < bp; j += kThreads) S[j] = (j == i) ? 1.0 : 0.0;
    return;
  }
  if (k > 0) {
    for (int64_t j = threadIdx.x; j < bp; j += kThreads) trow[j] = D.T1[i * bp + j];
    __syncthreads();
  }
  const int E = D.ellB;
  const int64_t eb = k * (int64_t)E * bp;
  for (int64_t j = threadIdx.x; j < bp; j += kThreads) {
    double s = 0.0;
    if (k > 0 && j < bk)
      for (int e = 0; e < E; ++e) s = fma(-D.bval[eb + e * bp + j], trow[D.bcol[eb + e * bp + j]], s);
    S[j] = s;
  }
  __syncthreads();  // the row's own entries land after every thread wrote its part
  const int64_t r = lo + i;
  const int64_t e0 = D.rowptr[r], e1 = D.rowptr[r + 1];
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
    const int64_t cidx = D.col[e];
    if (cidx >= lo && cidx < lo + bk) S[cidx - lo] += D.val[e];
  }
}

// Gauss-Jordan inversion of a 64 x 64 tile held in LDS, in place; returns the
// number of pivots that were not positive.  A wavefront owns 16 rows
// i = w + 4q, its lanes the 64 columns j: LDS accesses along a row are
// conflict-free, column values are broadcast.
__device__ inline int gj_invert_tile(double (&A)[kT][kT + 1]) {
  const int t = threadIdx.x;
  const int j = t & 63, w = t >> 6;
  int bad = 0;
  for (int r = 0; r < kT; ++r) {
    const double arr = A[r][r];
    bad += !(arr > 0.0);
    const double pr = 1.0 / arr;
    const double arj = A[r][j];
    double air[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) air[q] = A[w + 4 * q][r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = w + 4 * q;
      double v;
      if (i == r) v = (j == r) ? pr : arj * pr;
      else v = (j == r) ? -air[q] * pr : A[i][j] - air[q] * (arj * pr);
      A[i][j] = v;
    }
    __syncthreads();
  }
  return bad;
}

// Invert the first pivot tile (p, p) of S into piv.
__global__ __launch_bounds__(kThreads) void k_gj_pivot(const double *S, int64_t ld, int p,
                                                       double *piv, int *flag) {
  __shared__ double A[kT][kT + 1];
  const int t = threadIdx.x;
  const double *P = S + (int64_t)p * kT * ld + (int64_t)p * kT;
  for (int e = t; e < kT * kT; e += kThreads) A[e / kT][e % kT] = P[(int64_t)(e / kT) * ld + e % kT];
  __syncthreads();
  const int bad = gj_invert_tile(A);
  for (int e = t; e < kT * kT; e += kThreads) piv[e] = A[e / kT][e % kT];
  if (t == 0 && bad) atomicAdd(flag, bad);
}

// The pivot inverse (contiguous) and a tile of S into LDS: every load is
// issued before the first store, then one barrier.
__device__ inline void stage_pair(const double *piv, const double *tile, int64_t ld,
                                  double (*Pi)[kT + 1], double (*X)[kT + 1]) {
  constexpr int kE = kT * kT / kThreads;
  double pv[kE], xv[kE];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = (int)threadIdx.x + q * kThreads;
    pv[q] = piv[e];
    xv[q] = tile[(int64_t)(e / kT) * ld + e % kT];
  }
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = (int)threadIdx.x + q * kThreads;
    Pi[e / kT][e % kT] = pv[q];
    X[e / kT][e % kT] = xv[q];
  }
  __syncthreads();
}

// Row panel: S(p, j) = piv S(p, j) for every tile column j != p.
__global__ __launch_bounds__(kThreads) void k_gj_row(double *S, int64_t ld, int p,
                                                     const double *piv) {
  __shared__ double Pi[kT][kT + 1];
  __shared__ double X[kT][kT + 1];
  const int t = threadIdx.x;
  const int jt = blockIdx.x < p ? blockIdx.x : blockIdx.x + 1;
  double *tile = S + (int64_t)p * kT * ld + (int64_t)jt * kT;
  stage_pair(piv, tile, ld, Pi, X);
  const int j = t & 63, w = t >> 6;  // rows w + 4q, column j
  double out[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) out[q] = 0.0;
  for (int kk = 0; kk < kT; ++kk) {
    const double x = X[kk][j];
#pragma unroll
    for (int q = 0; q < 16; ++q) out[q] = fma(Pi[w + 4 * q][kk], x, out[q]);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) tile[(int64_t)(w + 4 * q) * ld + j] = out[q];
}

// Trailing update: S(I, J) -= S(I, p) S(p, J) for every tile I != p, J != p.
// The workgroup of tile (p+1, p+1), the next pivot tile, goes first and then
// inverts it into piv_next, hidden behind the other tiles' updates.
static_assert(kT * kT % kThreads == 0, "the update stages whole tiles");
__global__ __launch_bounds__(kThreads) void k_gj_update(double *S, int64_t ld, int p, int nt,
                                                        double *piv_next, int *flag) {
  __shared__ double L[kT][kT + 1];  // L[k][i] = S(I, p)[i][k]
  __shared__ double R[kT][kT + 1];  // R[k][j] = S(p, J)[k][j]
  const int t = threadIdx.x;
  const int m = nt - 1;
  const int rot = p + 1 < nt ? p * m + p : 0;  // position of tile (p+1, p+1)
  const int lin = (int)((blockIdx.x + (unsigned)rot) % (unsigned)(m * m));
  const int bi = lin / m, bj = lin - bi * m;
  const int it = bi < p ? bi : bi + 1, jt = bj < p ? bj : bj + 1;
  const double *SI = S + (int64_t)it * kT * ld + (int64_t)p * kT;
  const double *SJ = S + (int64_t)p * kT * ld + (int64_t)jt * kT;
  double *O = S + (int64_t)it * kT * ld + (int64_t)jt * kT;
  // rows i0 + a (4 consecutive), columns j0 + 16 b (16 lanes side by side:
  // conflict-free LDS reads, 128-byte global runs)
  const int i0 = (t >> 4) * 4, j0 = t & 15;
  // every global load of the workgroup (both operand tiles and this thread's
  // part of the output tile) is issued before the first wait
  constexpr int kE = kT * kT / kThreads;
  double lv[kE], rv[kE], ov[4][4];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = t + q * kThreads, r = e / kT, c = e % kT;
    lv[q] = SI[(int64_t)r * ld + c];
    rv[q] = SJ[(int64_t)r * ld + c];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) ov[a][b] = O[(int64_t)(i0 + a) * ld + j0 + 16 * b];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = t + q * kThreads, r = e / kT, c = e % kT;
    L[c][r] = lv[q];
    R[r][c] = rv[q];
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int kk = 0; kk < kT; ++kk) {
    double av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = L[kk][i0 + a];
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = R[kk][j0 + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
  }
  const bool next = it == p + 1 && jt == p + 1;  // uniform over the workgroup
  if (next) __syncthreads();                     // L is reused below
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double o = ov[a][b] - acc[a][b];
      O[(int64_t)(i0 + a) * ld + j0 + 16 * b] = o;
      if (next) L[i0 + a][j0 + 16 * b] = o;
    }
  if (next) {
    __syncthreads();
    const int bad = gj_invert_tile(L);
    for (int e = t; e < kT * kT; e += kThreads) piv_next[e] = L[e / kT][e % kT];
    if (t == 0 && bad) atomicAdd(flag, bad);
  }
}

// Column panel: S(I, p) = -S(I, p) piv for I != p; S(p, p) = piv.
__global__ __launch_bounds__(kThreads) void k_gj_col(double *S, int64_t ld, int p,
                                                     const double *piv) {
  __shared__ double Pi[kT][kT + 1];
  __shared__ double X[kT][kT + 1];
  const int t = threadIdx.x;
  const int it = blockIdx.x;
  double *tile = S + (int64_t)it * kT * ld + (int64_t)p * kT;
  if (it == p) {
    for (int e = t; e < kT * kT; e += kThreads) tile[(int64_t)(e / kT) * ld + e % kT] = piv[e];
    return;
  }
  stage_pair(piv, tile, ld, Pi, X);
  const int j = t & 63, w = t >> 6;  // rows w + 4q, column j
  double out[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) out[q] = 0.0;
  for (int kk = 0; kk < kT; ++kk) {
    const double pk = Pi[kk][j];
#pragma unroll
    for (int q = 0; q < 16; ++q) out[q] = fma(X[w + 4 * q][kk], pk, out[q]);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) tile[(int64_t)(w + 4 * q) * ld + j] = -out[q];
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------

// f = G (T - T_ref), one thread per displacement DOF; the row's entries are
// taken eight at a time, their columns, values and gathers all requested
// before the first product (the products are added in the row's order).
__global__ __launch_bounds__(kThreads) void k_thermal_load(DeformDev D, const double *T) {
  constexpr int U = 8;
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < D.n;
       r += (int64_t)gridDim.x * kThreads) {
    double a = 0.0;
    int64_t e = D.growptr[r];
    const int64_t e1 = D.growptr[r + 1];
    for (; e + U <= e1; e += U) {
      int c[U];
      double v[U], t[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        c[k] = D.gcol[e + k];
        v[k] = D.gval[e + k];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) t[k] = T[D.toff + c[k]];
#pragma unroll
      for (int k = 0; k < U; ++k) a = fma(v[k], t[k] - D.T_ref, a);
    }
    for (; e < e1; ++e) a = fma(D.gval[e], T[D.toff + D.gcol[e]] - D.T_ref, a);
    D.f[r] = a;
  }
}

// Coupling product of one row of an ELL block with a neighbouring block's
// vector: kSub lanes per row, each over every kSub-th entry (at most 6 of the
// 81 a row can hold), loads issued two at a time, then summed across the
// lanes.
constexpr int kSub = 16;
__device__ inline double ell_row(const double *val, const int32_t *col, int64_t bp, int E,
                                 int64_t i, int sub, const double *x) {
  double a0 = 0.0, a1 = 0.0;
  int e = sub;
  for (; e + kSub < E; e += 2 * kSub) {
    const double v0 = val[e * bp + i], v1 = val[(e + kSub) * bp + i];
    const int c0 = col[e * bp + i], c1 = col[(e + kSub) * bp + i];
    a0 = fma(v0, x[c0], a0);
    a1 = fma(v1, x[c1], a1);
  }
  if (e < E) a0 = fma(val[e * bp + i], x[col[e * bp + i]], a0);
  double s = a0 + a1;
#pragma unroll
  for (int o = 1; o < kSub; o <<= 1) s += __shfl_xor(s, o, 64);
  return s;
}

// Forward right-hand side c = f_k - A_{k,k-1} w_{k-1} (zero in the padding).
__global__ __launch_bounds__(kThreads) void k_fwd_rhs(DeformDev D, int64_t k) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = g / kSub;
  const int sub = (int)(g % kSub);
  if (i >= D.bp) return;
  const int64_t bk = D.rows(k);
  if (i >= bk) {
    if (sub == 0) D.c[i] = 0.0;
    return;
  }
  double a = 0.0;
  if (k > 0) {
    const int64_t eb = k * (int64_t)D.ellB * D.bp;
    a = ell_row(D.bval + eb, D.bcol + eb, D.bp, D.ellB, i, sub, D.w + D.lo(k - 1));
  }
  if (sub == 0) D.c[i] = D.f[D.lo(k) + i] - a;
}

// Backward right-hand side c = A_{k,k+1} u_{k+1} (zero in the padding).
__global__ __launch_bounds__(kThreads) void k_bwd_rhs(DeformDev D, int64_t k) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t i = g / kSub;
  const int sub = (int)(g % kSub);
  if (i >= D.bp) return;
  if (i >= D.rows(k)) {
    if (sub == 0) D.c[i] = 0.0;
    return;
  }
  const int64_t eb = k * (int64_t)D.ellU * D.bp;
  const double a = ell_row(D.uval + eb, D.ucol + eb, D.bp, D.ellU, i, sub, D.x + D.lo(k + 1));
  if (sub == 0) D.c[i] = a;
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
static_assert(kThreads == 256, "k_symv maps 16 x 16 threads onto a 64 x 64 tile");

__global__ __launch_bounds__(kThreads) void k_symv(const double *W, int64_t ld, int nt, int ns,
                                                   const int *strip, const double *v,
                                                   double *part) {
  __shared__ double shc[kSymStrip][kThreads / 64][64];
  const int I = strip[2 * blockIdx.x], J0 = strip[2 * blockIdx.x + 1];
  const int J1 = J0 + kSymStrip < nt ? J0 + kSymStrip : nt;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, cg = t & 15, rg = t >> 4;
  double vi[4], rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 4; ++q) vi[q] = v[I * 64 + rg * 4 + q];
  const double *rowp = W + (int64_t)(I * 64 + rg * 4) * ld + cg * 4;
  for (int J = J0; J < J1; ++J) {
    double a[4][4], vj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const dvec2 lo = *reinterpret_cast<const dvec2 *>(rowp + (int64_t)q * ld + J * 64);
      const dvec2 hi = *reinterpret_cast<const dvec2 *>(rowp + (int64_t)q * ld + J * 64 + 2);
      a[q][0] = lo[0];
      a[q][1] = lo[1];
      a[q][2] = hi[0];
      a[q][3] = hi[1];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) vj[k] = v[J * 64 + cg * 4 + k];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) rs[q] = fma(a[q][k], vj[k], rs[q]);
    if (J > I) {
      double cs[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double c = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) c = fma(a[q][k], vi[q], c);
        c += __shfl_xor(c, 16, 64);
        c += __shfl_xor(c, 32, 64);
        cs[k] = c;
      }
      if (lane < 16)
#pragma unroll
        for (int k = 0; k < 4; ++k) shc[J - J0][w][cg * 4 + k] = cs[k];
    }
  }
  __syncthreads();
  for (int i = t; i < (J1 - J0) * 64; i += kThreads) {
    const int tj = i >> 6, c = i & 63, J = J0 + tj;
    if (J > I)
      part[((int64_t)J * ns + I) * 64 + c] =
          ((shc[tj][0][c] + shc[tj][1][c]) + shc[tj][2][c]) + shc[tj][3][c];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double r = rs[q];
    r += __shfl_xor(r, 1, 64);
    r += __shfl_xor(r, 2, 64);
    r += __shfl_xor(r, 4, 64);
    r += __shfl_xor(r, 8, 64);
    rs[q] = r;
  }
  if (cg == 0) {
    const int sidx = nt + (J0 - I) / kSymStrip;
#pragma unroll
    for (int q = 0; q < 4; ++q) part[((int64_t)I * ns + sidx) * 64 + rg * 4 + q] = rs[q];
  }
}

// out = W v (MODE 0) or base - W v (MODE 1) for the first rows of output
// tile K = blockIdx.x: the transposed contributions of tile rows 0..K-1, then
// the strips of tile row K, in that order; kRedGroups thread groups of 64
// take every kRedGroups-th slot (at most 11 on the 81 tiles of the 1 cm stand,
// requested eight at a time), summed in group order.
constexpr int kRedGroups = 8;
template <int MODE>
__global__ __launch_bounds__(64 * kRedGroups) void k_symv_reduce(const double *part, int nt,
                                                                 int ns, int64_t rows,
                                                                 double *out, const double *base) {
  __shared__ double sg[kRedGroups][64];
  const int K = blockIdx.x, c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int nsK = (nt - K + kSymStrip - 1) / kSymStrip;
  const int n = K + nsK;
  double acc = 0.0;
#pragma unroll 8
  for (int j = g; j < n; j += kRedGroups) {
    const int slot = j < K ? j : nt + (j - K);
    acc += part[((int64_t)K * ns + slot) * 64 + c];
  }
  sg[g][c] = acc;
  __syncthreads();
  if (g != 0) return;
  double y = 0.0;
#pragma unroll
  for (int q = 0; q < kRedGroups; ++q) y += sg[q][c];
  const int64_t r = (int64_t)K * 64 + c;
  if (r < rows) out[r] = MODE == 0 ? y : base[r] - y;
}

__global__ __launch_bounds__(kThreads) void k_copy(double *dst, const double *src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

inline unsigned blocks_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t deform_factor(const DeformDev &D, hipStream_t st, int64_t *dispatches) {
  *dispatches = 0;
  const int nt = (int)(D.bp / kT);
  // launch shapes checked on the host before the first launch: every grid
  // non-empty and within the 32-bit grid limit, the row staged by k_schur_s
  // within the 64 KB of dynamic LDS a workgroup may take without an attribute
  if (D.bp <= 0 || D.bp % kT != 0 || D.bp > kMaxDeformBlock || D.nblk <= 0 || nt < 1 ||
      (int64_t)(nt - 1) * (nt - 1) > 0x7fffffffLL || D.bs <= 0 || D.bs > D.bp ||
      (size_t)D.bp * sizeof(double) > 65536)
    return hipErrorInvalidValue;
  for (int64_t k = 0; k < D.nblk; ++k)
    if (D.rows(k) <= 0 || D.rows(k) > D.bp) return hipErrorInvalidValue;
  hipError_t e = hipMemsetAsync(D.flag, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  int64_t n = 0;
  for (int64_t k = 0; k < D.nblk; ++k) {
    if (k > 0) {
      k_schur_t<<<(unsigned)D.rows(k), kThreads, 0, st>>>(D, k);
      ++n;
    }
    k_schur_s<<<(unsigned)D.bp, kThreads, (size_t)D.bp * sizeof(double), st>>>(D, k);
    double *S = D.W + k * D.bp * D.bp;
    // pivot inverses alternate between two buffers: pass p reads piv[p % 2]
    // while its trailing update inverts the next pivot tile into the other
    k_gj_pivot<<<1, kThreads, 0, st>>>(S, D.bp, 0, D.piv, D.flag);
    n += 2;
    for (int p = 0; p < nt; ++p) {
      double *pc = D.piv + (p & 1) * kT * kT, *pn = D.piv + ((p + 1) & 1) * kT * kT;
      if (nt > 1) {
        k_gj_row<<<nt - 1, kThreads, 0, st>>>(S, D.bp, p, pc);
        k_gj_update<<<(nt - 1) * (nt - 1), kThreads, 0, st>>>(S, D.bp, p, nt, pn, D.flag);
        n += 2;
      }
      k_gj_col<<<nt, kThreads, 0, st>>>(S, D.bp, p, pc);
      ++n;
    }
    // a launch error stops the factorisation at the block it occurred in
    if ((e = hipGetLastError()) != hipSuccess) {
      *dispatches = n;
      return e;
    }
  }
  *dispatches = n;
  return hipSuccess;
}

void deform_solve(const DeformDev &D, const double *T, hipStream_t st, hipEvent_t *ev) {
  k_thermal_load<<<blocks_for(D.n), kThreads, 0, st>>>(D, T);
  const unsigned cb = (unsigned)((D.bp * kSub + kThreads - 1) / kThreads);
  int g = 0;
  // block product: the symmetric form over the upper triangle, then its
  // fixed-order reduction (with events: the pair is timed as one product)
  auto gemv = [&](int mode, int64_t k, double *out, const double *base) {
    const double *W = D.W + k * D.bp * D.bp;
    const int64_t rows = D.rows(k);
    const int nt = D.tiles(), ns = D.slots();
    auto red = mode == 0 ? k_symv_reduce<0> : k_symv_reduce<1>;
    if (ev) {
      hipExtLaunchKernelGGL(k_symv, dim3(D.nstrip), dim3(kThreads), 0, st, ev[2 * g], nullptr, 0,
                            W, D.bp, nt, ns, D.strip, (const double *)D.c, D.part);
      hipExtLaunchKernelGGL(red, dim3(nt), dim3(64 * kRedGroups), 0, st, nullptr, ev[2 * g + 1], 0,
                            (const double *)D.part, nt, ns, rows, out, base);
    } else {
      k_symv<<<D.nstrip, kThreads, 0, st>>>(W, D.bp, nt, ns, D.strip, D.c, D.part);
      red<<<nt, 64 * kRedGroups, 0, st>>>(D.part, nt, ns, rows, out, base);
    }
    ++g;
  };
  for (int64_t k = 0; k < D.nblk; ++k) {
    k_fwd_rhs<<<cb, kThreads, 0, st>>>(D, k);
    gemv(0, k, D.w + D.lo(k), nullptr);
  }
  const int64_t last = D.nblk - 1;
  k_copy<<<blocks_for(D.rows(last)), kThreads, 0, st>>>(D.x + D.lo(last), D.w + D.lo(last),
                                                        D.rows(last));
  for (int64_t k = D.nblk - 2; k >= 0; --k) {
    k_bwd_rhs<<<cb, kThreads, 0, st>>>(D, k);
    gemv(1, k, D.x + D.lo(k), D.w + D.lo(k));
  }
}

}  // namespace mrsdc
