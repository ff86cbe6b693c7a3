// Internal declarations of the batched (multi-scenario) sweep.
#pragma once
#include "mrsdc_internal.h"

namespace mrsdc {

constexpr int kMaxS = 64;  // scenarios per batch = lanes of a wavefront

// Shared operators of the batch in row-major form: one row per wavefront, the
// row's entries are wave-uniform.
struct BatchOp {
  int64_t N = 0;
  const int64_t *rowptr = nullptr;  // K: [N+1]
  const int16_t *d16 = nullptr;     // column - row
  const double *Kv = nullptr;
  const int *rrow = nullptr;        // [N] index into rptr, -1 for rows without R entries
  const int64_t *rptr = nullptr;    // R over the Robin rows only
  const int16_t *rd16 = nullptr;
  const double *Rv = nullptr;
  const float *Kv32 = nullptr, *Rv32 = nullptr;
};

// Per-scenario solver scalars (index s fastest).
struct BatchScalars {
  double rz[2][kMaxS];
  double tol2[kMaxS];
  double alpha[kMaxS];
  double beta[kMaxS];
  double resid[17][kMaxS];
  int active[kMaxS];
  int done[kMaxS];
  int fail[kMaxS];
  int pad[kMaxS];
  long long iters_total[kMaxS];
  int slot_iters[kSlots][kMaxS];
};

struct BatchArgs {
  int S = 0, M = 0, P = 0, grid = 0;
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
  double *r = nullptr, *p = nullptr, *q = nullptr;
  double *partial = nullptr;  // [3][grid][S]
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
void blaunch_solve(const BatchArgs &a, int m, bool pred, int slot, int budget, double rtol,
                   hipStream_t st);
void blaunch_iface(const BatchArgs &a, int m, bool corr, hipStream_t st);
void blaunch_operator_timing(const BatchArgs &a, int m, int reps, hipStream_t st);
void blaunch_commit(const BatchArgs &a, double dt, hipStream_t st);
void blaunch_scatter(double *dst, const double *src, int64_t n, int S, int s, hipStream_t st);
void blaunch_gather(double *dst, const double *src, int64_t n, int S, int s, hipStream_t st);

}  // namespace mrsdc
