// Device state of the thermo-elastic deformation solve (block LU of the
// banded stiffness, factorised once; forward/backward block solves).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrsdc {

constexpr int kGjTile = 64;              // Gauss-Jordan pivot width and tile size
constexpr int64_t kMaxDeformBlock = 8192;  // padded block: one row of it in LDS (64 KB)
constexpr int kSymStrip = 1;               // tiles per workgroup of the symmetric block product

struct DeformDev {
  int64_t n = 0;     // free displacement DOFs
  int64_t bs = 0;    // block size (>= half-bandwidth)
  int64_t bp = 0;    // bs rounded up to a multiple of kGjTile
  int64_t nblk = 0;  // ceil(n / bs)
  int ellB = 0;      // ELL width of A_{k,k-1}
  int ellU = 0;      // ELL width of A_{k,k+1}
  int64_t toff = 0;  // first node of the body in the temperature vector
  double T_ref = 0.0;
  // K_u (CSR, full symmetric pattern) and the thermal load operator G (CSR)
  const int64_t *rowptr = nullptr;
  const int32_t *col = nullptr;
  const double *val = nullptr;
  const int64_t *growptr = nullptr;
  const int32_t *gcol = nullptr;
  const double *gval = nullptr;
  // couplings of block k to block k-1 (B) and k+1 (U): ELL [nblk][ell][bp],
  // columns local to the neighbouring block, padding entries (0, 0)
  const int32_t *bcol = nullptr;
  const double *bval = nullptr;
  const int32_t *ucol = nullptr;
  const double *uval = nullptr;
  double *W = nullptr;    // [nblk][bp][bp]: S_k^{-1}
  double *T1 = nullptr;   // [bp][bp]: A_{k,k-1} W_{k-1}
  double *piv = nullptr;  // [2][64][64]: inverses of the current and next pivot tiles
  int *flag = nullptr;    // count of non-positive pivots
  double *f = nullptr;    // [n] thermal load
  double *w = nullptr;    // [n] forward results W_k c_k
  double *x = nullptr;    // [n] displacement
  double *c = nullptr;    // [bp] block right-hand side
  // symmetric block product over the upper triangle of 64 x 64 tiles: one
  // workgroup per strip of kSymStrip tiles of a tile row, strip[2 b] = tile
  // row, strip[2 b + 1] = first tile column; part[K][slot][64] holds the
  // contributions to output tile K (slots 0..K-1: the transposed tiles (I, K)
  // of the rows above, slots nt + s: strip s of tile row K)
  const int *strip = nullptr;
  int nstrip = 0;
  double *part = nullptr;

  __host__ __device__ int tiles() const { return (int)(bp / 64); }
  __host__ __device__ int slots() const { return tiles() + (tiles() + kSymStrip - 1) / kSymStrip; }

  __host__ __device__ int64_t lo(int64_t k) const { return k * bs; }
  __host__ __device__ int64_t rows(int64_t k) const { return (k + 1) * bs < n ? bs : n - k * bs; }
};

// Factorise: for every block the Schur complement S_k, inverted in place by
// blocked Gauss-Jordan elimination into W_k.  Checks the launch shapes on the
// host first (hipErrorInvalidValue, nothing launched) and the launches of
// every block; *dispatches counts the kernels launched.
hipError_t deform_factor(const DeformDev &D, hipStream_t st, int64_t *dispatches);
// u = K_u^{-1} G (T - T_ref) into D.x.  With gemv_ev (2 events per dense
// block product, 2 nblk - 1 products) every product is timed.
void deform_solve(const DeformDev &D, const double *T, hipStream_t st, hipEvent_t *gemv_ev);

}  // namespace mrsdc
