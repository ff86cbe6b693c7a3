/*
 * mrsdc_oracle.h -- interface of the CPU FP64 oracle.
 *
 * TEST INFRASTRUCTURE, NOT THE PRODUCT.  The oracle is the slow, literal
 * reference implementation of the multi-rate spectral deferred correction
 * (MRSDC) time stepper of Naumann, Ruprecht and Wensch (arXiv 1707.03581),
 * against which the GPU library is checked.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or table with the GPU library.
 *
 * All arrays are caller-owned and only read (except the documented outputs).
 * Temperatures in degrees Celsius, SI units throughout.
 */
#ifndef MRSDC_ORACLE_H
#define MRSDC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LOBATTO = 0, ORC_EQUI_NOLEFT = 1 };
enum { ORC_MULTIRATE = 0, ORC_SINGLE_RATE = 1 };
enum { ORC_NONE = 0, ORC_CONTACT = 1, ORC_PATCH = 2 };

/* One body: linear finite element operators on its own mesh (paper §2). */
typedef struct {
  int64_t n;              /* nodes */
  const int64_t *rowptr;  /* [n+1] */
  const int32_t *col;     /* [nnz] */
  const double *K;        /* stiffness incl. conductivity (= -A_X), [nnz] */
  const double *R;        /* unit Robin boundary mass (B_X,env = -h R), [nnz] */
  const double *mass;     /* row-sum lumped mass, [n] */
  const double *rload;    /* int over the Robin boundary of phi_i, [n] */
  double h;               /* Robin coefficient alpha_X */
  double Tamb;            /* environment temperature T_env */
} orc_body;

/* Tensor grid of face nodes: ids[a*nv+b] is the body-local index of the node
 * at (u[a], v[b]); u and v strictly increasing. */
typedef struct {
  int body;
  int nu, nv;
  const double *u, *v;
  const int32_t *ids;
} orc_face;

typedef struct {
  int kind;          /* ORC_NONE | ORC_CONTACT | ORC_PATCH */
  /* contact (paper §2, Gamma_R(t)): mov coordinates in the fix face frame at
   * zero offset; at time t the mov face's v is shifted by s(t). */
  orc_face fix, mov;
  double alpha;      /* heat exchange coefficient on Gamma_R */
  double Pf;         /* friction power [W], spread uniformly over |Gamma_R(t)| */
  double split;      /* share of the friction heat entering the fixed body */
  /* patch: rigid rectangle of width wu x wv centred at (uc, s(t)) on `face`,
   * flux q0 + alpha (Tfix - T) into the body */
  orc_face face;
  double wu, wv, uc, q0, Tfix;
  /* motion s(t) = s0 + a sin(2 pi t / period + phase) (paper §5) */
  double s0, a, period, phase;
} orc_coupling;

typedef struct {
  int nbody;               /* 1 or 2; bodies are concatenated in this order */
  orc_body body[2];
  orc_coupling cpl;
} orc_problem;

typedef struct {
  int M;          /* standard nodes */
  int family;     /* ORC_LOBATTO | ORC_EQUI_NOLEFT */
  int P;          /* embedded nodes per standard interval */
  int K;          /* correction sweeps after the predictor */
  double dt;      /* time step */
  double pcg_rtol;
  int pcg_maxit;
  double sweep_tol; /* > 0: stop a step's sweeps once its residual is <= sweep_tol */
  int method;       /* ORC_MULTIRATE (Alg. 1/2) | ORC_SINGLE_RATE (single-rate SDC of
                       §3 with the whole coupling f^E in the implicit part; P unused) */
} orc_scheme;

typedef struct {
  int64_t solves, pcg_iters, fE_evals;
  int max_iters;
  double t_pcg, t_embedded, t_total;   /* seconds */
  int threads;
  int64_t sweeps;                      /* correction sweeps run */
} orc_stats;

/* Quadrature nodes and weights for one step of length dt.
 * tau[0..M]   : tau[0] = 0 (= t_n), tau[m] the standard nodes relative to t_n
 * s[(m)*(M+1)+j]            m,j = 1..M      (s_{m,j})
 * shat[m*(P+1)+q]           q = 1..P        (hat s_{m,q})
 * stil[(m*(P+1)+p)*(M+1)+j]                 (tilde s_{m,p,j})
 * spq[(m*(P+1)+p)*(P+1)+q]                  (s_{m,p,q})
 * Index 0 entries are unused (zero).  Returns 0, or -1 on bad arguments. */
int orc_weights(int M, int family, int P, double dt, double *tau, double *s,
                double *shat, double *stil, double *spq);

/* f^E(T, t) on the concatenated vector (zero outside coupled faces). */
int orc_fE(const orc_problem *pb, double t, const double *T, double *out);

/* One implicit node solve (diag(mass) + dtau (K + h R)) x = b by Jacobi-PCG,
 * warm-started from x.  Returns iterations, or -1 on no convergence. */
int orc_solve(const orc_problem *pb, double dtau, const double *b, double *x,
              double rtol, int maxit);

/* Advance T (in/out, concatenated) by nsteps steps of the scheme starting at
 * time t0.  residuals (nullable) receives nsteps*(K+1) values: the residual
 * (paper eq. residual) of iterate k = 0..K of each step.  Returns 0, -1 on
 * bad input, -2 on PCG failure. */
int orc_run(const orc_problem *pb, const orc_scheme *sc, double t0, int nsteps,
            double *T, double *residuals, orc_stats *stats);

/* Stationary field (K + h R) T = g, g = h T_env r (no mass term), by
 * Jacobi-PCG warm-started from T.  Returns iterations, or -1 on no
 * convergence. */
int orc_stationary(const orc_problem *pb, double *T, double rtol, int maxit);

int orc_max_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
