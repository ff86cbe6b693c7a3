// Nodes and weights of one MRSDC step (paper §3, "Multi-rate SDC": standard
// nodes tau_m, equidistant no-left embedded nodes tau_{m,p}, and the integrals
// of Lagrange polynomials s, hat s, tilde s, s_pq of the weight definitions /
// Table tab:weights).
//
// Each weight is an integral of a Lagrange basis polynomial of degree < 32.
// It is evaluated with Gauss-Legendre quadrature of 20 points (exact up to
// degree 39) on the integration interval, the basis polynomial being evaluated
// in product form at the quadrature points; everything in x87 long double.
// Gauss-Lobatto nodes are the end points plus the roots of P'_{M-1}, found by
// Newton's method.
#include <cmath>
#include <cstring>

#include "mrsdc_internal.h"

namespace mrsdc {

namespace {

typedef long double ld;

// Legendre P_n and its derivative at x (three-term recurrence).
void legendre(int n, ld x, ld *p, ld *dp) {
  ld p0 = 1, p1 = x;
  if (n == 0) { *p = 1; *dp = 0; return; }
  for (int k = 2; k <= n; ++k) {
    ld pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1);
}

constexpr int kGL = 20;
ld gl_x[kGL], gl_w[kGL];
bool gl_ready = false;

void gauss_legendre() {
  if (gl_ready) return;
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < kGL; ++i) {
    ld x = std::cos(pi * (i + 0.75L) / (kGL + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre(kGL, x, &p, &dp);
      ld dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-21L) break;
    }
    ld p, dp;
    legendre(kGL, x, &p, &dp);
    gl_x[i] = x;
    gl_w[i] = 2 / ((1 - x * x) * dp * dp);
  }
  gl_ready = true;
}

// Roots of P'_{n} on (-1,1): Newton on P'_n with P''_n from the Legendre ODE.
void lobatto_interior(int M, ld *x01) {
  const int n = M - 1;  // interior nodes are the roots of P'_n, n - 1 of them
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i < n; ++i) {
    ld x = -std::cos(pi * i / n);
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre(n, x, &p, &dp);
      ld d2p = (2 * x * dp - n * (n + 1) * p) / (1 - x * x);
      ld dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-21L) break;
    }
    x01[i] = (1 + x) / 2;
  }
}

// Lagrange basis polynomial j of nodes[0..n-1] at x, product form.
ld lagrange(int n, const ld *nodes, int j, ld x) {
  ld v = 1;
  for (int i = 0; i < n; ++i)
    if (i != j) v *= (x - nodes[i]) / (nodes[j] - nodes[i]);
  return v;
}

ld integrate_basis(int n, const ld *nodes, int j, ld a, ld b) {
  ld half = (b - a) / 2, mid = (a + b) / 2, acc = 0;
  for (int g = 0; g < kGL; ++g) acc += gl_w[g] * lagrange(n, nodes, j, mid + half * gl_x[g]);
  return acc * half;
}

}  // namespace

bool standard_nodes01(int M, int family, long double *x) {
  x[0] = 0;
  if (family == MRSDC_EQUI_NOLEFT) {
    for (int m = 1; m <= M; ++m) x[m] = (ld)m / (ld)M;
    return true;
  }
  if (family != MRSDC_LOBATTO || M < 2) return false;
  ld in[16];
  lobatto_interior(M, in);
  x[1] = 0;
  for (int i = 1; i < M - 1; ++i) x[i + 1] = in[i];
  x[M] = 1;
  return true;
}

bool build_weights(int M, int family, int P, double dt, Weights *w) {
  if (M < 1 || M > kMaxM || P < 1 || P > kMaxP || !(dt > 0)) return false;
  gauss_legendre();
  ld x[kMaxM + 1];
  if (!standard_nodes01(M, family, x)) return false;
  std::memset(w, 0, sizeof(*w));
  w->M = M;
  w->P = P;
  w->dt = dt;
  const ld T = dt;
  ld emb[kMaxP];
  for (int q = 1; q <= P; ++q) emb[q - 1] = (ld)q / (ld)P;
  for (int m = 0; m <= M; ++m) w->tau[m] = (double)(T * x[m]);
  for (int m = 1; m <= M; ++m) {
    ld lo = x[m - 1], hi = x[m], len = hi - lo;
    w->dtau[m] = (double)(T * len);
    if (len == 0) continue;
    for (int j = 1; j <= M; ++j) {
      w->s[m][j] = (double)(T * integrate_basis(M, x + 1, j - 1, lo, hi));
      for (int p = 1; p <= P; ++p)
        w->stil[m][p][j] =
            (double)(T * integrate_basis(M, x + 1, j - 1, lo + len * (p - 1) / P, lo + len * p / P));
    }
    for (int q = 1; q <= P; ++q) {
      w->shat[m][q] = (double)(T * len * integrate_basis(P, emb, q - 1, 0, 1));
      for (int p = 1; p <= P; ++p)
        w->spq[m][p][q] =
            (double)(T * len * integrate_basis(P, emb, q - 1, (ld)(p - 1) / P, (ld)p / P));
    }
  }
  return true;
}

}  // namespace mrsdc
