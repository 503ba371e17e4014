// Quadrature rules of Appendix D (host code).
//
// Elliptic rule (eq. D.1) in its real-variable form: with k^2 = ell/(1+ell),
// K = K(k^2) and u_q = (q - 1/2) K / Q,
//     s_q = sc^2(u_q | k^2),  r_q = (2K / (pi Q)) dn(u_q | k^2) / cn^2(u_q | k^2),
//     p_q = r_q / (1 + s_q).
// Jacobi's imaginary transformation turns the printed sn(i t | g), cn, dn into
// these real functions of the same modulus k = g.
//
// K is computed by the arithmetic-geometric mean, K(m) = pi / (2 AGM(1, sqrt(1-m)))
// (DLMF 19.8.1), and sn, cn, dn by the descending AGM / Landen scheme of DLMF 22.20(ii)
// (Abramowitz & Stegun 16.4).
//
// Gauss-Legendre rule (eq. D.2): s_q = tan^2(pi lambda_q / 2), p_q = v_q / 2, with the
// Legendre nodes found by Newton's method on P_Q from the Tricomi initial guesses
// (the nodes are the eigenvalues Golub-Welsch would return).
#include <cmath>

#include "../../include/infoesrf.h"

namespace {

const double kPi = 3.14159265358979323846;

double ellipk(double m) {
  double a = 1.0, b = std::sqrt(1.0 - m);
  for (int it = 0; it < 64 && std::fabs(a - b) > 1e-17 * a; ++it) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return kPi / (2.0 * a);
}

void ellipj(double u, double m, double* sn, double* cn, double* dn) {
  if (m == 0.0) {
    *sn = std::sin(u);
    *cn = std::cos(u);
    *dn = 1.0;
    return;
  }
  double a[32], c[32];
  a[0] = 1.0;
  double b = std::sqrt(1.0 - m);
  c[0] = std::sqrt(m);
  int n = 0;
  while (n < 30 && std::fabs(c[n]) > 1e-17 * a[n]) {
    a[n + 1] = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = std::sqrt(a[n] * b);
    ++n;
  }
  double phi = std::ldexp(a[n] * u, n);  // 2^n a_n u
  double phi_next = phi;
  for (int j = n; j > 0; --j) {
    phi_next = phi;
    phi = 0.5 * (phi + std::asin(c[j] / a[j] * std::sin(phi)));
  }
  *sn = std::sin(phi);
  *cn = std::cos(phi);
  *dn = (n > 0) ? std::cos(phi) / std::cos(phi_next - phi) : std::sqrt(1.0 - m * (*sn) * (*sn));
}

}  // namespace

extern "C" int infoesrf_quadrature_elliptic(int32_t Q, double ell, double* s_nodes, double* p_weights) {
  if (Q < 1 || Q > 1024 || !(ell > 0.0) || !std::isfinite(ell) || !s_nodes || !p_weights)
    return INFOESRF_ERR_INVALID_ARG;
  const double m = ell / (1.0 + ell);
  const double K = ellipk(m);
  for (int q = 0; q < Q; ++q) {
    const double u = (q + 0.5) * K / Q;
    double sn, cn, dn;
    ellipj(u, m, &sn, &cn, &dn);
    const double s = (sn / cn) * (sn / cn);
    const double r = (2.0 * K / (kPi * Q)) * dn / (cn * cn);
    s_nodes[q] = s;
    p_weights[q] = r / (1.0 + s);
  }
  return INFOESRF_OK;
}

extern "C" int infoesrf_quadrature_gauss_legendre(int32_t Q, double* s_nodes, double* p_weights) {
  if (Q < 1 || Q > 4096 || !s_nodes || !p_weights) return INFOESRF_ERR_INVALID_ARG;
  for (int i = 0; i < Q; ++i) {
    // i-th root in decreasing order, Tricomi's initial guess
    double x = std::cos(kPi * (i + 0.75) / (Q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= Q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pq = (Q == 1) ? x : p1;
      const double pqm1 = (Q == 1) ? 1.0 : p0;
      dp = Q * (x * pq - pqm1) / (x * x - 1.0);
      const double dx = pq / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    {
      // recompute the derivative at the converged node
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= Q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pq = (Q == 1) ? x : p1;
      const double pqm1 = (Q == 1) ? 1.0 : p0;
      dp = Q * (x * pq - pqm1) / (x * x - 1.0);
    }
    const double w = 2.0 / ((1.0 - x * x) * dp * dp);
    const double t = std::tan(0.5 * kPi * x);
    s_nodes[Q - 1 - i] = t * t;
    p_weights[Q - 1 - i] = 0.5 * w;
  }
  return INFOESRF_OK;
}
