/*
 * mrsdc_oracle.c -- plain FP64 CPU oracle of the MRSDC time stepper.
 *
 * TEST INFRASTRUCTURE, NOT THE PRODUCT: the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it.  It shares no code with
 * the GPU library.
 *
 * What it follows (Naumann, Ruprecht, Wensch, arXiv 1707.03581):
 *   - the split right-hand side f^I, g, f^E of §2 (eq. ivp and the three
 *     definitions before it), with the contact/friction coupling of the weak
 *     form (eqs. femContFix / femContMov) on the overlap Gamma_R(t) and a
 *     row-sum lumped mass;
 *   - standard and embedded nodes and the four weight families s, hat s,
 *     tilde s, s_pq of §3 "Multi-rate SDC" (weight definitions, Table
 *     tab:weights);
 *   - the predictor (Alg. 1) and the correction sweep (Alg. 2), literally,
 *     with every embedded state kept as a full-length vector;
 *   - the residual of eq. residual (max over standard nodes, max-norm).
 * Readings where the paper is silent: Jacobi-preconditioned CG with
 * ||r||_2 <= rtol ||b||_2 for the implicit solves (the solver is not named);
 * Gauss-Lobatto standard nodes have tau_1 = t_n, so their first interval has
 * length zero and is skipped (T_1 = T_n); the friction heat is spread
 * uniformly over |Gamma_R(t)| and split between the bodies.
 */
#include "mrsdc_oracle.h"

#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 q128;

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the following parallel regions (timing at a stated core count) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Quadrature (§3, Multi-rate SDC: node sets and weight definitions)         */
/* ------------------------------------------------------------------------ */

/* Standard nodes on [0,1]: x[1..M]; x[0] = 0 is t_n.
 * Gauss-Lobatto: 0, 1 and the roots of P'_{M-1}, closed forms for M <= 5.
 * Equidistant "no-left" (§3): x_m = m/M, so t_n is not a node. */
static int standard_nodes(int M, int family, q128 *x) {
  x[0] = 0;
  if (family == ORC_EQUI_NOLEFT) {
    if (M < 1) return -1;
    for (int m = 1; m <= M; ++m) x[m] = (q128)m / (q128)M;
    return 0;
  }
  if (family != ORC_LOBATTO) return -1;
  switch (M) {
    case 2: x[1] = 0; x[2] = 1; return 0;
    case 3: x[1] = 0; x[2] = 0.5Q; x[3] = 1; return 0;
    case 4: {
      q128 r = 1 / sqrtq(5.0Q);
      x[1] = 0; x[2] = (1 - r) / 2; x[3] = (1 + r) / 2; x[4] = 1; return 0;
    }
    case 5: {
      q128 r = sqrtq(3.0Q / 7.0Q);
      x[1] = 0; x[2] = (1 - r) / 2; x[3] = 0.5Q; x[4] = (1 + r) / 2; x[5] = 1; return 0;
    }
    default: return -1;
  }
}

/* Integral over [a,b] of the Lagrange polynomial l_j with l_j(nodes[i]) =
 * delta_ij (n nodes), by expanding l_j in monomials and integrating each. */
static q128 lagrange_integral(int n, const q128 *nodes, int j, q128 a, q128 b) {
  q128 c[80];
  for (int k = 0; k < 80; ++k) c[k] = 0;
  c[0] = 1;
  int deg = 0;
  for (int i = 0; i < n; ++i) {
    if (i == j) continue;
    q128 d = nodes[j] - nodes[i];
    for (int k = deg + 1; k >= 1; --k) c[k] = (c[k - 1] - nodes[i] * c[k]) / d;
    c[0] = -nodes[i] * c[0] / d;
    ++deg;
  }
  q128 sum = 0, ak = a, bk = b;
  for (int k = 0; k <= deg; ++k) {
    sum += c[k] * (bk - ak) / (k + 1);
    ak *= a;
    bk *= b;
  }
  return sum;
}

int orc_weights(int M, int family, int P, double dt, double *tau, double *s,
                double *shat, double *stil, double *spq) {
  if (M < 1 || M > 40 || P < 1 || P > 60 || !(dt > 0)) return -1;
  q128 x[64];
  if (standard_nodes(M, family, x)) return -1;
  const int M1 = M + 1, P1 = P + 1;
  memset(s, 0, sizeof(double) * M1 * M1);
  memset(shat, 0, sizeof(double) * M1 * P1);
  memset(stil, 0, sizeof(double) * M1 * P1 * M1);
  memset(spq, 0, sizeof(double) * M1 * P1 * P1);
  q128 Q = dt;
  q128 *std = x + 1; /* the M standard nodes, 0-based */
  q128 emb[64];      /* embedded nodes q/P on the unit interval, 0-based */
  for (int q = 1; q <= P; ++q) emb[q - 1] = (q128)q / (q128)P;
  for (int m = 0; m <= M; ++m) tau[m] = (double)(Q * x[m]);
  for (int m = 1; m <= M; ++m) {
    q128 lo = x[m - 1], hi = x[m], len = hi - lo;
    if (len == 0) continue; /* degenerate interval (Lobatto: tau_1 = t_n) */
    q128 dtm = Q * len;
    for (int j = 1; j <= M; ++j) {
      s[m * M1 + j] = (double)(Q * lagrange_integral(M, std, j - 1, lo, hi));
      for (int p = 1; p <= P; ++p) {
        q128 a = lo + len * (p - 1) / P, b = lo + len * p / P;
        stil[(m * P1 + p) * M1 + j] = (double)(Q * lagrange_integral(M, std, j - 1, a, b));
      }
    }
    for (int q = 1; q <= P; ++q) {
      shat[m * P1 + q] = (double)(dtm * lagrange_integral(P, emb, q - 1, 0, 1));
      for (int p = 1; p <= P; ++p) {
        q128 a = (q128)(p - 1) / P, b = (q128)p / P;
        spq[(m * P1 + p) * P1 + q] = (double)(dtm * lagrange_integral(P, emb, q - 1, a, b));
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side pieces (§2, eq. ivp)                                      */
/* ------------------------------------------------------------------------ */

static int64_t total_n(const orc_problem *pb) {
  int64_t n = 0;
  for (int b = 0; b < pb->nbody; ++b) n += pb->body[b].n;
  return n;
}

static int64_t body_offset(const orc_problem *pb, int body) {
  int64_t off = 0;
  for (int b = 0; b < body; ++b) off += pb->body[b].n;
  return off;
}

/* y = (K + h R) x, i.e. y = -f^I(x) (A_X = -K, B_X,env = -h R). */
static void apply_L(const orc_problem *pb, const double *x, double *y) {
  for (int bi = 0; bi < pb->nbody; ++bi) {
    const orc_body *B = &pb->body[bi];
    int64_t off = body_offset(pb, bi);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < B->n; ++i) {
      double sk = 0, sr = 0;
      for (int64_t e = B->rowptr[i]; e < B->rowptr[i + 1]; ++e) {
        sk += B->K[e] * x[off + B->col[e]];
        sr += B->R[e] * x[off + B->col[e]];
      }
      y[off + i] = sk + B->h * sr;
    }
  }
}

/* g = b_env = h T_env int_{Robin} phi */
static void source_g(const orc_problem *pb, double *g) {
  for (int bi = 0; bi < pb->nbody; ++bi) {
    const orc_body *B = &pb->body[bi];
    int64_t off = body_offset(pb, bi);
    for (int64_t i = 0; i < B->n; ++i) g[off + i] = B->h * B->Tamb * B->rload[i];
  }
}

static double motion_s(const orc_coupling *c, double t) {
  return c->s0 + c->a * sin(2.0 * M_PI * t / c->period + c->phase);
}

/* smallest cell a in [0, n-2] with x[a+1] > lo (n-1 if none) */
static int first_cell_after(const double *x, int n, double lo) {
  int a = 0, b = n - 1; /* search in [a, b) for first a with x[a+1] > lo */
  while (a < b) {
    int mid = (a + b) / 2;
    if (x[mid + 1] > lo) b = mid; else a = mid + 1;
  }
  return a;
}

/* bilinear basis of the cell [x0,x1]x[y0,y1] at (x,y), order (0,0),(1,0),(0,1),(1,1) */
static void bilinear(double x0, double x1, double y0, double y1, double x, double y, double phi[4]) {
  double xi = (x - x0) / (x1 - x0), et = (y - y0) / (y1 - y0);
  phi[0] = (1 - xi) * (1 - et);
  phi[1] = xi * (1 - et);
  phi[2] = (1 - xi) * et;
  phi[3] = xi * et;
}

static void cell_nodes(const orc_face *F, int a, int b, int64_t off, int64_t idx[4]) {
  idx[0] = off + F->ids[a * F->nv + b];
  idx[1] = off + F->ids[(a + 1) * F->nv + b];
  idx[2] = off + F->ids[a * F->nv + b + 1];
  idx[3] = off + F->ids[(a + 1) * F->nv + b + 1];
}

static const double GAUSS2 = 0.57735026918962576451; /* 1/sqrt(3) */

/* Contact and friction on Gamma_R(t) (§2, eqs. femContFix/femContMov):
 * row i of the fixed body receives int phi_i (alpha (T_mov - T_fix) + split q_f),
 * row i of the moving body int phi_i (alpha (T_fix - T_mov) + (1-split) q_f),
 * q_f = P_f / |Gamma_R(t)|.  Integrated exactly with 2x2 Gauss points on every
 * rectangle where a cell of one face overlaps a cell of the other. */
static void fE_contact(const orc_problem *pb, double t, const double *T, double *out) {
  const orc_coupling *c = &pb->cpl;
  const orc_face *F = &c->fix, *G = &c->mov;
  const double s = motion_s(c, t);
  const int64_t offF = body_offset(pb, F->body), offG = body_offset(pb, G->body);
  double ou0 = fmax(F->u[0], G->u[0]), ou1 = fmin(F->u[F->nu - 1], G->u[G->nu - 1]);
  double ov0 = fmax(F->v[0], G->v[0] + s), ov1 = fmin(F->v[F->nv - 1], G->v[G->nv - 1] + s);
  double area = (ou1 > ou0 && ov1 > ov0) ? (ou1 - ou0) * (ov1 - ov0) : 0.0;
  double qf = area > 0 ? c->Pf / area : 0.0;
  for (int cu = 0; cu < G->nu - 1; ++cu) {
    double gu0 = G->u[cu], gu1 = G->u[cu + 1];
    for (int cv = 0; cv < G->nv - 1; ++cv) {
      double gv0 = G->v[cv] + s, gv1 = G->v[cv + 1] + s;
      int64_t gi[4];
      cell_nodes(G, cu, cv, offG, gi);
      for (int a = first_cell_after(F->u, F->nu, gu0); a < F->nu - 1 && F->u[a] < gu1; ++a) {
        for (int b = first_cell_after(F->v, F->nv, gv0); b < F->nv - 1 && F->v[b] < gv1; ++b) {
          double u0 = fmax(F->u[a], gu0), u1 = fmin(F->u[a + 1], gu1);
          double v0 = fmax(F->v[b], gv0), v1 = fmin(F->v[b + 1], gv1);
          if (!(u1 > u0 && v1 > v0)) continue;
          int64_t fi[4];
          cell_nodes(F, a, b, offF, fi);
          double hu = 0.5 * (u1 - u0), hv = 0.5 * (v1 - v0), w = hu * hv;
          for (int gx = -1; gx <= 1; gx += 2) {
            for (int gy = -1; gy <= 1; gy += 2) {
              double x = 0.5 * (u0 + u1) + gx * GAUSS2 * hu;
              double y = 0.5 * (v0 + v1) + gy * GAUSS2 * hv;
              double pf[4], pg[4];
              bilinear(F->u[a], F->u[a + 1], F->v[b], F->v[b + 1], x, y, pf);
              bilinear(gu0, gu1, gv0, gv1, x, y, pg);
              double Tf = 0, Tg = 0;
              for (int k = 0; k < 4; ++k) {
                Tf += pf[k] * T[fi[k]];
                Tg += pg[k] * T[gi[k]];
              }
              double flux_f = c->alpha * (Tg - Tf) + c->split * qf;
              double flux_g = c->alpha * (Tf - Tg) + (1.0 - c->split) * qf;
              for (int k = 0; k < 4; ++k) {
                out[fi[k]] += w * pf[k] * flux_f;
                out[gi[k]] += w * pg[k] * flux_g;
              }
            }
          }
        }
      }
    }
  }
}

/* Rigid patch (the stock of the paper's 2D test, §4, generalised with a
 * prescribed flux): int_{patch(t)} phi_i (q0 + alpha (T_fixed - T)). */
static void fE_patch(const orc_problem *pb, double t, const double *T, double *out) {
  const orc_coupling *c = &pb->cpl;
  const orc_face *F = &c->face;
  const double s = motion_s(c, t);
  const int64_t off = body_offset(pb, F->body);
  double pu0 = c->uc - 0.5 * c->wu, pu1 = c->uc + 0.5 * c->wu;
  double pv0 = s - 0.5 * c->wv, pv1 = s + 0.5 * c->wv;
  for (int a = first_cell_after(F->u, F->nu, pu0); a < F->nu - 1 && F->u[a] < pu1; ++a) {
    for (int b = first_cell_after(F->v, F->nv, pv0); b < F->nv - 1 && F->v[b] < pv1; ++b) {
      double u0 = fmax(F->u[a], pu0), u1 = fmin(F->u[a + 1], pu1);
      double v0 = fmax(F->v[b], pv0), v1 = fmin(F->v[b + 1], pv1);
      if (!(u1 > u0 && v1 > v0)) continue;
      int64_t fi[4];
      cell_nodes(F, a, b, off, fi);
      double hu = 0.5 * (u1 - u0), hv = 0.5 * (v1 - v0), w = hu * hv;
      for (int gx = -1; gx <= 1; gx += 2) {
        for (int gy = -1; gy <= 1; gy += 2) {
          double x = 0.5 * (u0 + u1) + gx * GAUSS2 * hu;
          double y = 0.5 * (v0 + v1) + gy * GAUSS2 * hv;
          double pf[4];
          bilinear(F->u[a], F->u[a + 1], F->v[b], F->v[b + 1], x, y, pf);
          double Tf = 0;
          for (int k = 0; k < 4; ++k) Tf += pf[k] * T[fi[k]];
          double flux = c->q0 + c->alpha * (c->Tfix - Tf);
          for (int k = 0; k < 4; ++k) out[fi[k]] += w * pf[k] * flux;
        }
      }
    }
  }
}

int orc_fE(const orc_problem *pb, double t, const double *T, double *out) {
  int64_t N = total_n(pb);
  memset(out, 0, sizeof(double) * N);
  if (pb->cpl.kind == ORC_CONTACT) fE_contact(pb, t, T, out);
  else if (pb->cpl.kind == ORC_PATCH) fE_patch(pb, t, T, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Implicit node solve: (diag(mass) + dtau (K + h R)) x = b, Jacobi-PCG       */
/* ------------------------------------------------------------------------ */

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

typedef struct {
  const orc_problem *pb;
  int64_t N;
  double *mass, *Ldiag, *r, *z, *p, *q, *diag;
  /* single-rate method: with cpl set, the part of f^E(., t_cpl) linear in T
   * joins the operator; e0 = f^E(0, t_cpl), e1 scratch */
  int cpl;
  double t_cpl;
  double *e0, *e1;
} solver;

static void apply_A(solver *S, double dtau, const double *x, double *y) {
  apply_L(S->pb, x, y);
  if (S->cpl) { /* (K + h R) x - (f^E(x, t) - f^E(0, t)) */
    orc_fE(S->pb, S->t_cpl, x, S->e1);
    for (int64_t i = 0; i < S->N; ++i) y[i] -= S->e1[i] - S->e0[i];
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < S->N; ++i) y[i] = S->mass[i] * x[i] + dtau * y[i];
}

static int pcg(solver *S, double dtau, const double *b, double *x, double rtol, int maxit) {
  const int64_t N = S->N;
  double *r = S->r, *z = S->z, *p = S->p, *q = S->q, *d = S->diag;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) d[i] = S->mass[i] + dtau * S->Ldiag[i];
  apply_A(S, dtau, x, q);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    r[i] = b[i] - q[i];
    z[i] = r[i] / d[i];
    p[i] = z[i];
  }
  double bnorm = sqrt(dot(N, b, b));
  double rz = dot(N, r, z);
  for (int it = 0;; ++it) {
    double rnorm = sqrt(dot(N, r, r));
    if (rnorm <= rtol * bnorm) return it;
    if (it >= maxit) return -1;
    apply_A(S, dtau, p, q);
    double alpha = rz / dot(N, p, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
      z[i] = r[i] / d[i];
    }
    double rz_new = dot(N, r, z);
    double beta = rz_new / rz;
    rz = rz_new;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
  }
}

static int solver_init(solver *S, const orc_problem *pb) {
  int64_t N = total_n(pb);
  S->pb = pb;
  S->N = N;
  S->mass = malloc(sizeof(double) * N);
  S->Ldiag = malloc(sizeof(double) * N);
  S->r = malloc(sizeof(double) * N);
  S->z = malloc(sizeof(double) * N);
  S->p = malloc(sizeof(double) * N);
  S->q = malloc(sizeof(double) * N);
  S->diag = malloc(sizeof(double) * N);
  if (!S->mass || !S->Ldiag || !S->r || !S->z || !S->p || !S->q || !S->diag) return -1;
  for (int bi = 0; bi < pb->nbody; ++bi) {
    const orc_body *B = &pb->body[bi];
    int64_t off = body_offset(pb, bi);
    for (int64_t i = 0; i < B->n; ++i) {
      S->mass[off + i] = B->mass[i];
      double dk = 0, dr = 0;
      for (int64_t e = B->rowptr[i]; e < B->rowptr[i + 1]; ++e)
        if (B->col[e] == i) { dk += B->K[e]; dr += B->R[e]; }
      S->Ldiag[off + i] = dk + B->h * dr;
    }
  }
  return 0;
}

static void solver_free(solver *S) {
  free(S->mass); free(S->Ldiag); free(S->r); free(S->z); free(S->p); free(S->q); free(S->diag);
  free(S->e0); free(S->e1);
}

int orc_solve(const orc_problem *pb, double dtau, const double *b, double *x, double rtol,
              int maxit) {
  solver S;
  memset(&S, 0, sizeof S);
  if (solver_init(&S, pb)) { solver_free(&S); return -1; }
  int it = pcg(&S, dtau, b, x, rtol, maxit);
  solver_free(&S);
  return it;
}

/* Stationary field of the conduction and Robin part (the initial data of the
 * numerical example, section 5, read with the time derivative zero):
 * (K + h R) T = g, g = h T_env r, by the same Jacobi-PCG with no mass term. */
int orc_stationary(const orc_problem *pb, double *T, double rtol, int maxit) {
  solver S;
  memset(&S, 0, sizeof S);
  if (solver_init(&S, pb)) { solver_free(&S); return -1; }
  const int64_t N = S.N;
  for (int64_t i = 0; i < N; ++i) S.mass[i] = 0.0;
  double *g = malloc(sizeof(double) * N);
  if (!g) { solver_free(&S); return -1; }
  source_g(pb, g);
  int it = pcg(&S, 1.0, g, T, rtol, maxit);
  free(g);
  solver_free(&S);
  return it;
}

/* ------------------------------------------------------------------------ */
/* The time stepper: Alg. 1 (predictor) and Alg. 2 (correction sweep)        */
/* ------------------------------------------------------------------------ */

static int validate(const orc_problem *pb, const orc_scheme *sc) {
  if (!pb || !sc || pb->nbody < 1 || pb->nbody > 2) return -1;
  if (sc->M < 1 || sc->P < 1 || sc->K < 0 || !(sc->dt > 0)) return -1;
  if (sc->M < 2 && sc->family == ORC_LOBATTO) return -1;
  if (sc->method != ORC_MULTIRATE && sc->method != ORC_SINGLE_RATE) return -1;
  if (sc->family == ORC_LOBATTO && sc->M > 5) return -1;
  if (pb->cpl.kind != ORC_NONE && !(pb->cpl.period > 0)) return -1;
  return 0;
}

/* Single-rate SDC (§3, "Single-rate spectral deferred correction") in the
 * form the work-precision study of §5 compares against: the part of f^E that
 * is linear in T joins f^I, so the implicit function at node tau_m is
 *     J_m(x) = f^I(x) + f^E(x, tau_m) - f^E(0, tau_m),
 * and the rest, f^E(0, tau_m) (friction or patch flux), is a source taken at
 * the node time like g.  Nothing explicit is left: the predictor is implicit
 * Euler from node to node, and eq. sdc_sweep loses its f^E difference term.
 * The quadrature I_{m-1}^m = sum_j s_{m,j} F(T^k_j, tau_j) uses the full
 * right-hand side.  One equidistant node with K = 0 is implicit Euler for the
 * whole coupled system. */
static int run_single_rate(const orc_problem *pb, const orc_scheme *sc, double t0, int nsteps,
                           double *T, double *residuals, orc_stats *stats) {
  const double tstart = now_s();
  const int M = sc->M, P = sc->P, Ksw = sc->K, M1 = M + 1, P1 = P + 1;
  const int64_t N = total_n(pb);
  const size_t nv = (size_t)N;
  double tau[64], dtau[64];
  double *s = malloc(sizeof(double) * M1 * M1), *shat = malloc(sizeof(double) * M1 * P1);
  double *stil = malloc(sizeof(double) * M1 * P1 * M1), *spq = malloc(sizeof(double) * M1 * P1 * P1);
  double *g = malloc(sizeof(double) * nv), *Tn = malloc(sizeof(double) * nv);
  double *Tst = malloc(sizeof(double) * nv * M1), *Tstn = malloc(sizeof(double) * nv * M1);
  double *F = malloc(sizeof(double) * nv * M1), *Im = malloc(sizeof(double) * nv * M1);
  double *b = malloc(sizeof(double) * nv), *Jk = malloc(sizeof(double) * nv);
  double *zero = calloc(nv, sizeof(double)); /* f^E(0, t) is the coupling source */
  solver S;
  memset(&S, 0, sizeof S);
  int rc = 0;
  if (!s || !shat || !stil || !spq || !g || !Tn || !Tst || !Tstn || !F || !Im || !b || !Jk ||
      !zero || orc_weights(M, sc->family, P, sc->dt, tau, s, shat, stil, spq) ||
      solver_init(&S, pb) || !(S.e0 = malloc(sizeof(double) * nv)) ||
      !(S.e1 = malloc(sizeof(double) * nv))) {
    rc = -1;
    goto done;
  }
  for (int m = 1; m <= M; ++m) dtau[m] = tau[m] - tau[m - 1];
#define V(base, k) ((base) + (size_t)(k) * nv)
  source_g(pb, g);
  S.cpl = 1;
  orc_stats st;
  memset(&st, 0, sizeof st);
  st.threads = orc_max_threads();
  double tp = 0;

  for (int n = 0; n < nsteps; ++n) {
    const double tn = t0 + n * sc->dt;
    memcpy(Tn, T, sizeof(double) * nv);
    /* predictor: M T_m = M T_{m-1} + dtau_m (J_m(T_m) + g + f^E(0, tau_m)) */
    memcpy(V(Tst, 0), Tn, sizeof(double) * nv);
    for (int m = 1; m <= M; ++m) {
      const double *Tprev = V(Tst, m - 1);
      double *xs = V(Tst, m);
      memcpy(xs, Tprev, sizeof(double) * nv);
      if (dtau[m] == 0.0) continue;
      S.t_cpl = tn + tau[m];
      orc_fE(pb, S.t_cpl, zero, S.e0);
      for (int64_t i = 0; i < N; ++i) b[i] = S.mass[i] * Tprev[i] + dtau[m] * (g[i] + S.e0[i]);
      double t1 = now_s();
      int it = pcg(&S, dtau[m], b, xs, sc->pcg_rtol, sc->pcg_maxit);
      tp += now_s() - t1;
      if (it < 0) { rc = -2; goto done; }
      st.solves++; st.pcg_iters += it; if (it > st.max_iters) st.max_iters = it;
    }
    const int passes = residuals ? Ksw + 1 : Ksw;
    for (int k = 1; k <= passes; ++k) {
      /* F_j = f^I(T^k_j) + f^E(T^k_j, tau_j) + g at every standard node */
      for (int j = 1; j <= M; ++j) {
        double *Fj = V(F, j);
        orc_fE(pb, tn + tau[j], V(Tst, j), b);
        st.fE_evals++;
        apply_L(pb, V(Tst, j), Fj);
        for (int64_t i = 0; i < N; ++i) Fj[i] = -Fj[i] + g[i] + b[i];
      }
      /* I_{m-1}^m = sum_j s_{m,j} F_j, and the residual of iterate k-1 */
      for (int m = 1; m <= M; ++m)
        for (int64_t i = 0; i < N; ++i) {
          double acc = 0;
          for (int j = 1; j <= M; ++j) acc += s[m * M1 + j] * F[(size_t)j * nv + i];
          Im[(size_t)m * nv + i] = acc;
        }
      if (residuals || sc->sweep_tol > 0) {
        double rmax = 0;
        for (int64_t i = 0; i < N; ++i) {
          double cum = 0;
          for (int m = 1; m <= M; ++m) {
            if (dtau[m] == 0.0) continue;
            cum += Im[(size_t)m * nv + i];
            double r = fabs(S.mass[i] * Tst[(size_t)m * nv + i] - S.mass[i] * Tn[i] - cum);
            if (r > rmax) rmax = r;
          }
        }
        if (residuals) residuals[(size_t)n * (Ksw + 1) + (k - 1)] = rmax;
        if (sc->sweep_tol > 0 && rmax <= sc->sweep_tol) break;
      }
      if (k > Ksw) break;
      st.sweeps++;
      /* eq. sdc_sweep: M T^{k+1}_m = M T^{k+1}_{m-1}
       *                 + dtau_m (J_m(T^{k+1}_m) - J_m(T^k_m)) + I_{m-1}^m */
      memcpy(V(Tstn, 0), Tn, sizeof(double) * nv);
      for (int m = 1; m <= M; ++m) {
        const double *Tprev = V(Tstn, m - 1), *Tk = V(Tst, m);
        double *xs = V(Tstn, m);
        if (dtau[m] == 0.0) {
          memcpy(xs, Tprev, sizeof(double) * nv);
          continue;
        }
        S.t_cpl = tn + tau[m];
        orc_fE(pb, S.t_cpl, zero, S.e0);
        orc_fE(pb, S.t_cpl, Tk, S.e1);
        apply_L(pb, Tk, Jk);
        for (int64_t i = 0; i < N; ++i) Jk[i] = -Jk[i] + (S.e1[i] - S.e0[i]);
        const double *Imm = V(Im, m);
        for (int64_t i = 0; i < N; ++i) b[i] = S.mass[i] * Tprev[i] - dtau[m] * Jk[i] + Imm[i];
        memcpy(xs, Tk, sizeof(double) * nv);
        double t1 = now_s();
        int it = pcg(&S, dtau[m], b, xs, sc->pcg_rtol, sc->pcg_maxit);
        tp += now_s() - t1;
        if (it < 0) { rc = -2; goto done; }
        st.solves++; st.pcg_iters += it; if (it > st.max_iters) st.max_iters = it;
      }
      double *sw = Tst; Tst = Tstn; Tstn = sw;
    }
    memcpy(T, V(Tst, M), sizeof(double) * nv);
  }
#undef V
  st.t_pcg = tp;
  st.t_total = now_s() - tstart;
  if (stats) *stats = st;
done:
  free(zero);
  solver_free(&S);
  free(s); free(shat); free(stil); free(spq);
  free(g); free(Tn); free(Tst); free(Tstn); free(F); free(Im); free(b); free(Jk);
  return rc;
}

int orc_run(const orc_problem *pb, const orc_scheme *sc, double t0, int nsteps, double *T,
            double *residuals, orc_stats *stats) {
  if (validate(pb, sc) || nsteps < 0) return -1;
  if (sc->method == ORC_SINGLE_RATE) return run_single_rate(pb, sc, t0, nsteps, T, residuals, stats);
  const double tstart = now_s();
  const int M = sc->M, P = sc->P, Ksw = sc->K;
  const int M1 = M + 1, P1 = P + 1;
  const int64_t N = total_n(pb);
  double tau[64], *s = malloc(sizeof(double) * M1 * M1), *shat = malloc(sizeof(double) * M1 * P1);
  double *stil = malloc(sizeof(double) * M1 * P1 * M1), *spq = malloc(sizeof(double) * M1 * P1 * P1);
  solver S;
  memset(&S, 0, sizeof S);
  if (!s || !shat || !stil || !spq || orc_weights(M, sc->family, P, sc->dt, tau, s, shat, stil, spq)) {
    free(s); free(shat); free(stil); free(spq);
    return -1;
  }
  double dtau[64];
  for (int m = 1; m <= M; ++m) dtau[m] = tau[m] - tau[m - 1];

  const size_t nv = (size_t)N;
  double *g = malloc(sizeof(double) * nv), *Tn = malloc(sizeof(double) * nv);
  double *Tst = malloc(sizeof(double) * nv * M1), *Tstn = malloc(sizeof(double) * nv * M1);
  double *Temb = malloc(sizeof(double) * nv * M1 * P1), *Tembn = malloc(sizeof(double) * nv * M1 * P1);
  double *Eold = malloc(sizeof(double) * nv * M1 * P1), *Enew = malloc(sizeof(double) * nv);
  double *F = malloc(sizeof(double) * nv * M1), *Im = malloc(sizeof(double) * nv * M1);
  double *Imp = malloc(sizeof(double) * nv * M1 * P1);
  double *fstar = malloc(sizeof(double) * nv), *b = malloc(sizeof(double) * nv);
  double *LTk = malloc(sizeof(double) * nv);
  int rc = 0;
  if (!g || !Tn || !Tst || !Tstn || !Temb || !Tembn || !Eold || !Enew || !F || !Im || !Imp ||
      !fstar || !b || !LTk || solver_init(&S, pb)) {
    rc = -1;
    goto done;
  }
#define V(base, k) ((base) + (size_t)(k) * nv)
#define EMB(base, m, p) ((base) + ((size_t)(m) * P1 + (p)) * nv)
  source_g(pb, g);
  orc_stats st;
  memset(&st, 0, sizeof st);
  st.threads = orc_max_threads();
  double tp = 0, te = 0;

  for (int n = 0; n < nsteps; ++n) {
    const double tn = t0 + n * sc->dt;
    memcpy(Tn, T, sizeof(double) * nv);

    /* ---- Alg. 1: predictor ---- */
    memcpy(V(Tst, 0), Tn, sizeof(double) * nv);
    for (int m = 1; m <= M; ++m) {
      const double *Tprev = V(Tst, m - 1);
      if (dtau[m] == 0.0) {
        memcpy(V(Tst, m), Tprev, sizeof(double) * nv);
        for (int p = 0; p <= P; ++p) memcpy(EMB(Temb, m, p), Tprev, sizeof(double) * nv);
        continue;
      }
      /* implicit Euler over [tau_{m-1}, tau_m]: M T* = M T_{m-1} + dtau (f^I(T*) + g) */
      for (int64_t i = 0; i < N; ++i) b[i] = S.mass[i] * Tprev[i] + dtau[m] * g[i];
      double *xs = V(Tst, m);
      memcpy(xs, Tprev, sizeof(double) * nv);
      double t1 = now_s();
      int it = pcg(&S, dtau[m], b, xs, sc->pcg_rtol, sc->pcg_maxit);
      tp += now_s() - t1;
      if (it < 0) { rc = -2; goto done; }
      st.solves++; st.pcg_iters += it; if (it > st.max_iters) st.max_iters = it;
      /* f*_m = f^I(T*) + g(tau_m) */
      apply_L(pb, xs, fstar);
      for (int64_t i = 0; i < N; ++i) fstar[i] = -fstar[i] + g[i];
      /* explicit Euler through the embedded nodes */
      t1 = now_s();
      const double dtp = dtau[m] / P;
      memcpy(EMB(Temb, m, 0), Tprev, sizeof(double) * nv);
      for (int p = 1; p <= P; ++p) {
        const double *Tp = EMB(Temb, m, p - 1);
        double *Tq = EMB(Temb, m, p);
        orc_fE(pb, tn + tau[m - 1] + (p - 1) * dtp, Tp, Enew);
        st.fE_evals++;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) Tq[i] = Tp[i] + dtp * (fstar[i] + Enew[i]) / S.mass[i];
      }
      te += now_s() - t1;
      memcpy(V(Tst, m), EMB(Temb, m, P), sizeof(double) * nv);
    }

    /* ---- Alg. 2: K correction sweeps (one extra pass for the last residual) ---- */
    const int passes = residuals ? Ksw + 1 : Ksw;
    for (int k = 1; k <= passes; ++k) {
      /* F_j = f^I(T^k_j) + g(tau_j) at the standard nodes */
      for (int j = 1; j <= M; ++j) {
        double *Fj = V(F, j);
        apply_L(pb, V(Tst, j), Fj);
        for (int64_t i = 0; i < N; ++i) Fj[i] = -Fj[i] + g[i];
      }
      /* f^E(T^k_{m,q}, tau_{m,q}), q = 0..P */
      for (int m = 1; m <= M; ++m) {
        for (int q = 0; q <= P; ++q) {
          if (dtau[m] == 0.0) { memset(EMB(Eold, m, q), 0, sizeof(double) * nv); continue; }
          orc_fE(pb, tn + tau[m - 1] + q * (dtau[m] / P), EMB(Temb, m, q), EMB(Eold, m, q));
          st.fE_evals++;
        }
      }
      /* I_{m-1}^m (eq. standard_quad) and I_{m,p-1}^p (eq. embedded_quad) */
      for (int m = 1; m <= M; ++m) {
        double *Imm = V(Im, m);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
          double acc = 0;
          for (int j = 1; j <= M; ++j) acc += s[m * M1 + j] * F[(size_t)j * nv + i];
          for (int q = 1; q <= P; ++q) acc += shat[m * P1 + q] * EMB(Eold, m, q)[i];
          Imm[i] = acc;
        }
        for (int p = 1; p <= P; ++p) {
          double *Ip = EMB(Imp, m, p);
#pragma omp parallel for schedule(static)
          for (int64_t i = 0; i < N; ++i) {
            double acc = 0;
            for (int j = 1; j <= M; ++j) acc += stil[(m * P1 + p) * M1 + j] * F[(size_t)j * nv + i];
            for (int q = 1; q <= P; ++q) acc += spq[(m * P1 + p) * P1 + q] * EMB(Eold, m, q)[i];
            Ip[i] = acc;
          }
        }
      }
      /* residual of iterate k-1 (eq. residual): max_m |M T_m - M T_n - sum_{l<=m} I_l|;
         with sweep_tol > 0 it also decides whether sweep k runs (the residual
         control of section 3: each sweep should reduce it) */
      if (residuals || sc->sweep_tol > 0) {
        double rmax = 0;
        for (int64_t i = 0; i < N; ++i) {
          double cum = 0;
          for (int m = 1; m <= M; ++m) {
            cum += Im[(size_t)m * nv + i];
            double r = fabs(S.mass[i] * Tst[(size_t)m * nv + i] - S.mass[i] * Tn[i] - cum);
            if (r > rmax) rmax = r;
          }
        }
        if (residuals) residuals[(size_t)n * (Ksw + 1) + (k - 1)] = rmax;
        if (sc->sweep_tol > 0 && rmax <= sc->sweep_tol) break;
      }
      if (k > Ksw) break;
      st.sweeps++;

      memcpy(V(Tstn, 0), Tn, sizeof(double) * nv);
      for (int m = 1; m <= M; ++m) {
        const double *Tprev = V(Tstn, m - 1);
        if (dtau[m] == 0.0) {
          memcpy(V(Tstn, m), Tprev, sizeof(double) * nv);
          for (int p = 0; p <= P; ++p) memcpy(EMB(Tembn, m, p), Tprev, sizeof(double) * nv);
          continue;
        }
        /* M T* = M T^{k+1}_{m-1} + dtau (f^I(T*) - f^I(T^k_m)) + I_{m-1}^m */
        const double *Tk = V(Tst, m);
        apply_L(pb, Tk, LTk); /* = -f^I(T^k_m) */
        const double *Imm = V(Im, m);
        for (int64_t i = 0; i < N; ++i) b[i] = S.mass[i] * Tprev[i] + dtau[m] * LTk[i] + Imm[i];
        double *xs = V(Tstn, m);
        memcpy(xs, Tk, sizeof(double) * nv);
        double t1 = now_s();
        int it = pcg(&S, dtau[m], b, xs, sc->pcg_rtol, sc->pcg_maxit);
        tp += now_s() - t1;
        if (it < 0) { rc = -2; goto done; }
        st.solves++; st.pcg_iters += it; if (it > st.max_iters) st.max_iters = it;
        /* f*_m = f^I(T*) - f^I(T^k_m) */
        apply_L(pb, xs, fstar);
        for (int64_t i = 0; i < N; ++i) fstar[i] = -fstar[i] + LTk[i];
        t1 = now_s();
        const double dtp = dtau[m] / P;
        memcpy(EMB(Tembn, m, 0), Tprev, sizeof(double) * nv);
        for (int p = 1; p <= P; ++p) {
          const double *Tp = EMB(Tembn, m, p - 1);
          double *Tq = EMB(Tembn, m, p);
          const double *Eo = EMB(Eold, m, p - 1), *Ip = EMB(Imp, m, p);
          orc_fE(pb, tn + tau[m - 1] + (p - 1) * dtp, Tp, Enew);
          st.fE_evals++;
#pragma omp parallel for schedule(static)
          for (int64_t i = 0; i < N; ++i)
            Tq[i] = Tp[i] + (dtp * (fstar[i] + Enew[i] - Eo[i]) + Ip[i]) / S.mass[i];
        }
        te += now_s() - t1;
        memcpy(V(Tstn, m), EMB(Tembn, m, P), sizeof(double) * nv);
      }
      double *sw = Tst; Tst = Tstn; Tstn = sw;
      sw = Temb; Temb = Tembn; Tembn = sw;
    }
    memcpy(T, V(Tst, M), sizeof(double) * nv);
  }
#undef V
#undef EMB
  st.t_pcg = tp;
  st.t_embedded = te;
  st.t_total = now_s() - tstart;
  if (stats) *stats = st;
done:
  solver_free(&S);
  free(s); free(shat); free(stil); free(spq);
  free(g); free(Tn); free(Tst); free(Tstn); free(Temb); free(Tembn); free(Eold); free(Enew);
  free(F); free(Im); free(Imp); free(fstar); free(b); free(LTk);
  return rc;
}
