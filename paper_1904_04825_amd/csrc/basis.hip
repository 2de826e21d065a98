// Host-side construction of the 1D FR tables (Section 3): Gauss-Legendre
// solution points by Newton iteration on the Legendre three-term recurrence,
// barycentric Lagrange differentiation, and the derivatives of the left and
// right Radau correction polynomials g_R = (L_{P+1} + L_P)/2, g_L(x) = g_R(-x).
#include <cmath>

#include "internal.h"

namespace frjf {
namespace {

// L_n(x) and L_n'(x) by the recurrence (k+1) L_{k+1} = (2k+1) x L_k - k L_{k-1}.
void legendre(int n, double x, double* Ln, double* dLn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *Ln = 1.0;
    *dLn = 0.0;
    return;
  }
  double d0 = 0.0, d1 = 1.0;
  for (int k = 1; k < n; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    double d2 = d0 + (2 * k + 1) * p1;  // L'_{k+1} = L'_{k-1} + (2k+1) L_k
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  *Ln = p1;
  *dLn = d1;
}

}  // namespace

Basis make_basis(int P) {
  Basis b{};
  const int n = P + 1;
  b.n = n;
  for (int i = 0; i < n; ++i) {
    // Chebyshev-type initial guess, ascending order
    double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double L, dL;
      legendre(n, x, &L, &dL);
      double dx = L / dL;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double L, dL;
    legendre(n, x, &L, &dL);
    b.x[i] = x;
    b.w[i] = 2.0 / ((1.0 - x * x) * dL * dL);
  }
  // barycentric weights lambda_b = 1 / prod_{c != b} (x_b - x_c)
  double lam[kMaxN];
  for (int i = 0; i < n; ++i) {
    double p = 1.0;
    for (int c = 0; c < n; ++c)
      if (c != i) p *= (b.x[i] - b.x[c]);
    lam[i] = 1.0 / p;
  }
  for (int a = 0; a < n; ++a) {
    double diag = 0.0;
    for (int c = 0; c < n; ++c) {
      if (c == a) continue;
      b.D[a][c] = (lam[c] / lam[a]) / (b.x[a] - b.x[c]);
      diag -= b.D[a][c];
    }
    b.D[a][a] = diag;
  }
  for (int i = 0; i < n; ++i) {
    double pm = 1.0, pp = 1.0;
    for (int c = 0; c < n; ++c) {
      if (c == i) continue;
      pm *= (-1.0 - b.x[c]) / (b.x[i] - b.x[c]);
      pp *= (1.0 - b.x[c]) / (b.x[i] - b.x[c]);
    }
    b.lm[i] = pm;
    b.lp[i] = pp;
  }
  for (int a = 0; a < n; ++a) {
    double L, dP1, dP, x = b.x[a];
    legendre(P + 1, x, &L, &dP1);
    legendre(P, x, &L, &dP);
    b.gR[a] = 0.5 * (dP1 + dP);
    legendre(P + 1, -x, &L, &dP1);
    legendre(P, -x, &L, &dP);
    b.gL[a] = -0.5 * (dP1 + dP);
  }
  b.kLL = b.kLR = b.kRL = b.kRR = 0.0;
  for (int a = 0; a < n; ++a) {
    b.kLL += b.lm[a] * b.gL[a];
    b.kLR += b.lm[a] * b.gR[a];
    b.kRL += b.lp[a] * b.gL[a];
    b.kRR += b.lp[a] * b.gR[a];
  }
  return b;
}

}  // namespace frjf
