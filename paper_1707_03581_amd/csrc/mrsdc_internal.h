// Internal declarations shared by the host driver (api.cpp), the quadrature
// (quadrature.cpp) and the HIP kernels (kernels.hip).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/mrsdc.h"
#include "face_integrals.h"

namespace mrsdc {

constexpr int kMaxM = 8;
constexpr int kMaxP = 32;
constexpr int kBand = 8;        // max coupled nodes per face node and direction
constexpr int kSlice = 64;      // SELL slice height = one wavefront
constexpr int kBlock = 256;     // threads per block of the vector kernels
constexpr int kMaxGrid = 1024;  // blocks (and reduction partials) of a solve's kernels
constexpr int kIfaceBlock = 1024;
constexpr int kMaxJ = 8;        // right-hand sides of the multi-vector SpMV

// Quadrature of one step, 1-based node indices (paper §3 weight definitions).
struct Weights {
  int M, P;
  double dt;
  double tau[kMaxM + 1];   // tau[0] = 0 (t_n), relative to t_n
  double dtau[kMaxM + 1];  // dtau[m] = tau[m] - tau[m-1]
  double s[kMaxM + 1][kMaxM + 1];
  double shat[kMaxM + 1][kMaxP + 1];
  double stil[kMaxM + 1][kMaxP + 1][kMaxM + 1];
  double spq[kMaxM + 1][kMaxP + 1][kMaxP + 1];
};

bool build_weights(int M, int family, int P, double dt, Weights *w);
bool standard_nodes01(int M, int family, long double *x);

// Sliced ELLPACK (SELL-64) operator L = K + h R of the concatenated system.
// Element k of row (64 s + lane) sits at off[s] + 64 k + lane; columns are
// int16 offsets col - row when every |col - row| < 32768, else int32 columns.
struct SellDev {
  int64_t nrows = 0, nslices = 0, nelem = 0;
  const int64_t *off = nullptr;   // [nslices + 1]
  const double *val = nullptr;    // [nelem]
  const float *val32 = nullptr;   // [nelem] (FP32_REFINE)
  const int16_t *d16 = nullptr;   // [nelem] or null
  const int32_t *c32 = nullptr;   // [nelem] or null
  // value dictionary: when the operator holds at most kDictMax distinct
  // values, vid[e] indexes vdict (FP64) / vdict32 (FP32) with vdict[vid[e]]
  // bitwise equal to val[e]; the CG operator then reads 1 byte per entry
  const uint8_t *vid = nullptr;   // [nelem] or null
  const double *vdict = nullptr;  // [ndict]
  const float *vdict32 = nullptr; // [ndict] (FP32_REFINE)
  int ndict = 0;
  // packed entries (at most 16 dictionary values, |col - row| <= 2047):
  // pk16[e] = (col - row) * 16 + vid[e], one 2-byte load per entry
  const int16_t *pk16 = nullptr;  // [nelem] or null
  // row patterns: when the rows' lists of (col - row, dictionary index),
  // slice padding included, take at most kMaxCls distinct forms, row r reads
  // form rcls[r]: clen[c] words ctab[c * cw + k] = (col - row) * 256 + index
  const uint8_t *rcls = nullptr;  // [nrows] or null
  const int *ctab = nullptr;      // [ncls][cw]
  const int *clen = nullptr;      // [ncls]
  int ncls = 0, cw = 0;
};
constexpr int kDictMax = 256;
constexpr int kMaxCls = 128;
constexpr int kMaxClsWidth = 32;

// Per-solve device scalars of the CG iteration and of the refinement loop.
struct SolveScalars {
  double rz[2];      // r.z of the current/next iteration, by parity
  double gam[2];     // single-reduction form: r.u and alpha of iteration it,
  double alp[2];     // by parity (it - 1 is read while it is written)
  double tol2;       // CG stopping threshold on ||r||^2
  double bb;         // ||b||^2
  double alpha, beta;
  double ref_bb, ref_tol2;
  int done, iters;
  int ref_done, ref_rounds;
};

// Device-side counters of one time step, read back once per step.
constexpr int kSlots = 17 * kMaxM;  // (sweep k, interval m) solve slots

struct StepCounters {
  long long pcg_iters;
  long long refine_steps;
  int max_iters;
  int fail;                 // solves that hit their budget
  int stop;                 // residual control: no further sweeps this step
  int sweeps;               // sweeps run when stop was set
  double resid[17];         // residual of iterate k
  int slot_iters[kSlots];   // iterations of each solve of the step (-1: budget hit)
  int slot_rounds[kSlots];  // refinement rounds of each solve (-1: failed)
};

// Coupling data of f^E on device (contact between two face grids, or patch).
struct IfaceDev {
  int kind = 0;            // 0 none, 1 contact, 2 patch
  int nuf = 0, nvf = 0;    // fixed face (or patch face) grid
  int num = 0, nvm = 0;    // moving face grid (contact)
  int nfix = 0, n_if = 0;  // nuf*nvf, total interface points
  const double *uf = nullptr, *vf = nullptr, *um = nullptr, *vm = nullptr;
  const int64_t *rows = nullptr;   // [n_if] global row of each interface point
  // u-direction (time independent) restricted integrals over [ou0, ou1]
  const double *Mu = nullptr;    // [nuf*3] int psi_a psi_{a-1+i}
  const double *Hu = nullptr;    // [nuf]   int psi_a
  const double *Cu = nullptr;    // [nuf*kBand] int psi_a chi_{clo[a]+i}
  const int *clo = nullptr;      // [nuf]
  const int *ccnt = nullptr;     // [nuf] used entries of the band
  const double *Nu = nullptr;    // [num*3] int chi_c chi_{c-1+i}
  const double *Gu = nullptr;    // [num]
  const double *CuT = nullptr;   // [num*kBand] int chi_c psi_{alo[c]+i}
  const int *alo = nullptr;      // [num]
  const int *acnt = nullptr;     // [num]
  double ou0 = 0, ou1 = 0;
  double alpha = 0, Pf = 0, split = 0.5;
  double q0 = 0, Tfix = 0, wv = 0;
  double s0 = 0, a = 0, period = 1, phase = 0;
};

// Layout of one table of time-dependent (v-direction) face integrals:
// doubles [friction density | Mv 3*nvf | Hv nvf | Cv kBand*nvf | Nv 3*nvm |
// Gv nvm | CvT kBand*nvm], ints [dlo nvf | dcnt nvf | blo nvm | bcnt nvm].
struct CoefLayout {
  int nvf, nvm;
  __host__ __device__ int dstride() const { return 1 + (4 + kBand) * (nvf + nvm); }
  __host__ __device__ int istride() const { return 2 * (nvf + nvm); }
  __host__ __device__ int Mv() const { return 1; }
  __host__ __device__ int Hv() const { return 1 + 3 * nvf; }
  __host__ __device__ int Cv() const { return 1 + 4 * nvf; }
  __host__ __device__ int Nv() const { return 1 + (4 + kBand) * nvf; }
  __host__ __device__ int Gv() const { return Nv() + 3 * nvm; }
  __host__ __device__ int CvT() const { return Gv() + nvm; }
  __host__ __device__ int dlo() const { return 0; }
  __host__ __device__ int dcnt() const { return nvf; }
  __host__ __device__ int blo() const { return 2 * nvf; }
  __host__ __device__ int bcnt() const { return 2 * nvf + nvm; }
};


// Everything the kernels of one context touch.
struct DevState {
  int single_rate = 0;        // coupling in the implicit part, no embedded substeps
  double *ifc_lin = nullptr;  // [n_if] single-rate: dtau A_c x of the last interface call
  double *ifc_src = nullptr;  // [n_if] single-rate: dtau times the coupling source
  double sweep_tol = 0.0;  // > 0: residual-controlled sweeps
  int64_t N = 0;
  int M = 0, P = 0, K = 0;
  double dtau_h[kMaxM + 1] = {};      // host copy of the interval lengths
  int grid = 0;                       // blocks of the vector kernels
  SellDev op;
  const double *mass = nullptr, *g = nullptr, *Ldiag = nullptr;
  double *dinv[kMaxM + 1] = {};       // Jacobi inverse per interval
  float *dinv32[kMaxM + 1] = {};
  const float *mass32 = nullptr;
  const Weights *w = nullptr;         // device copy
  const int *ifpos = nullptr;         // [N] interface index or -1
  double *T[kMaxM + 1] = {};          // standard-node states (T[0] = T_n)
  double *F[kMaxM + 1] = {};          // f^I(T_j) + g
  double *I[kMaxM + 1] = {};          // I_{m-1}^m
  double *r = nullptr, *p = nullptr, *q = nullptr;  // CG work
  double *u = nullptr, *s = nullptr;                // single-reduction form
  float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *x32 = nullptr;
  float *u32 = nullptr, *s32 = nullptr;
  double *b64 = nullptr, *r64 = nullptr;  // refinement right-hand side and residual
  double *partial = nullptr;          // [6 * grid]
  SolveScalars *sc = nullptr;
  StepCounters *ctr = nullptr;
  double *tn = nullptr;               // device scalar: t_n of the current step
  IfaceDev ifc;
  double *Eold = nullptr, *Enew = nullptr;  // [(M+1)*(P+1)*n_if]
  double *Ipre = nullptr;  // [(M+1)*(P+1)*n_if] I_{m,p} of the interface rows, per sweep
  double *Tbuf[2] = {};                     // [n_if] interface state, double buffered
  double *fst = nullptr;                    // [n_if] f*_m on the interface
  double *coefD = nullptr;                  // [(M+1)(P+1)] tables of v-direction integrals
  int *coefI = nullptr;
};

// ---- kernel launchers (kernels.hip) ----
void launch_f_multi(const DevState &d, int j0, int j1, hipStream_t st);
void launch_quad_resid(const DevState &d, int k, hipStream_t st);
void launch_init_pred(const DevState &d, int m, int slot, double rtol, hipStream_t st);
void launch_init_corr(const DevState &d, int m, int slot, double rtol, hipStream_t st);
void launch_iface_F(const DevState &d, int j, hipStream_t st);
void launch_pcg_final(const DevState &d, int m, int slot, int it, bool fp32, hipStream_t st);
void launch_iface_quad(const DevState &d, hipStream_t st);
void launch_iface_lin(const DevState &d, int m, const double *x, hipStream_t st);
void launch_stationary_init(const DevState &d, const double *zeros, const double *dinv, int slot,
                            double rtol, hipStream_t st);
void launch_stationary_iters(const DevState &d, const double *zeros, const double *dinv, int slot,
                             int it0, int n, int last_it, hipStream_t st);
// rtol: the solve's relative tolerance; its first launch (it = 0) forms the
// solve's scalars from the partials of launch_init_pred / launch_init_corr
void launch_pcg_iter(const DevState &d, int m, int slot, int it, bool last, bool tail,
                     double rtol, hipStream_t st, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr);
void launch_refine_init(const DevState &d, int m, int slot, bool pred, double rtol,
                        hipStream_t st);
// round 0 also forms the refinement's scalars (tolerance refine_rtol); a later
// round first takes the previous round's refinement check
void launch_inner_init(const DevState &d, int m, int slot, double inner_rtol, int round,
                       double refine_rtol, hipStream_t st);
void launch_pcg32_iter(const DevState &d, int m, int slot, int it, bool last, bool tail,
                       double inner_rtol, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// chk_it >= 0: the check of the round's inner solve after its launch budget
// (launch_pcg_final) is taken over by the update kernel
void launch_refine_update(const DevState &d, int m, int slot, int round, bool last_round,
                          int chk_it, hipStream_t st);
void launch_operator_timing(const DevState &d, int m, bool fp32, int reps, hipStream_t st);
void launch_clear_counters(const DevState &d, hipStream_t st);
size_t coef_table_doubles(const IfaceDev &f);
size_t coef_table_ints(const IfaceDev &f);
void launch_iface_coeffs(const DevState &d, hipStream_t st);
// The embedded substeps of interval m after its node solve; chk_it >= 0: the
// solve's check after its launch budget (launch_pcg_final) is left to this call.
void launch_iface(const DevState &d, int m, bool corr, int slot, int chk_it, hipStream_t st);
void launch_step_end(const DevState &d, double dt, hipStream_t st);
void launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);
// device address of the allocation-free stationary solve's fixed scratch
// (2 MRSDC_NOALLOC_MAX_ROWS doubles) on `device`, which must be current
hipError_t stationary_scratch(int device, double **ptr);
// dinv = 1 / Ldiag, zeros = 0 (n values each)
void launch_stationary_scratch(double *dinv, double *zeros, const double *Ldiag, int64_t n,
                               hipStream_t st);

}  // namespace mrsdc
