// Host-side FP64 Chebyshev coefficients for an approximation of sign(x) on eps <= |x| <= 1.
//
// The paper approximates the matrix sign function by sum_m alpha_m T_m (Sec. 2, eq. 3) with
// "appropriate coefficients" that it does not list.  This library's rule:
//   1. q(y) interpolates y^{-1/2} on [eps^2, 1] at the n+1 first-kind Chebyshev nodes, n = (N-1)/2;
//   2. p(x) = x q(x^2), an odd polynomial of degree N (the largest odd number <= the request);
//   3. p is re-expanded exactly in T_m(x) from its values at N+1 first-kind nodes (a discrete
//      cosine transform), and the even coefficients, zero up to rounding, are set to zero.
#include <cmath>
#include <vector>

namespace ovl {

namespace {

// Chebyshev interpolation coefficients from samples f(cos(pi (j + 1/2) / n)), j < n
std::vector<double> coeffs_from_samples(const std::vector<double> &f) {
  const int n = (int)f.size();
  std::vector<double> c(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += f[j] * std::cos(M_PI * k * (j + 0.5) / n);
    c[k] = 2.0 * s / n;
  }
  c[0] *= 0.5;
  return c;
}

// sum_k c_k T_k(z) by Clenshaw's backward recurrence
double clenshaw(const std::vector<double> &c, double z) {
  double b1 = 0.0, b2 = 0.0;
  for (int k = (int)c.size() - 1; k >= 1; --k) {
    const double b0 = c[k] + 2.0 * z * b1 - b2;
    b2 = b1;
    b1 = b0;
  }
  return c[0] + z * b1 - b2;
}

}  // namespace

// returns N + 1 coefficients (N odd) in alpha; false on bad arguments
bool cheb_sign_coeffs(int degree, double eps, std::vector<double> &alpha) {
  if (degree < 1 || !(eps > 0.0 && eps < 1.0)) return false;
  const int N = (degree % 2 == 1) ? degree : degree - 1;
  const int nq = (N - 1) / 2 + 1;
  const double a = eps * eps, b = 1.0;
  std::vector<double> fy(nq);
  for (int j = 0; j < nq; ++j) {
    const double z = std::cos(M_PI * (j + 0.5) / nq);
    const double y = 0.5 * (a + b) + 0.5 * (b - a) * z;
    fy[j] = 1.0 / std::sqrt(y);
  }
  const std::vector<double> cq = coeffs_from_samples(fy);
  std::vector<double> px(N + 1);
  for (int j = 0; j <= N; ++j) {
    const double x = std::cos(M_PI * (j + 0.5) / (N + 1));
    const double z = (2.0 * x * x - (a + b)) / (b - a);
    px[j] = x * clenshaw(cq, z);
  }
  alpha = coeffs_from_samples(px);
  for (int m = 0; m <= N; m += 2) alpha[m] = 0.0;
  return true;
}

// sum_m alpha_m T_m(x), Clenshaw, FP64
double cheb_eval(const std::vector<double> &alpha, double x) { return clenshaw(alpha, x); }

}  // namespace ovl
