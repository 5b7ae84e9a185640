// Order-2K Coiflet filters (App. A) derived on the host: the low-pass taps of
// length 6K whose wavelet has vanishing moments 0 .. 2K-1 and whose scaling
// function has vanishing moments 1 .. 2K-1 about the origin of its support
// [-2K, 4K-1] (tap index 2K).
//
// Derivation (independent of any tabulated filter): every orthonormal two-channel
// low-pass filter of length 2m with sum sqrt 2 is reached by the lattice
// recursion H_i(z) = cos t_i H_{i-1}(z) + sin t_i z^-2 G_{i-1}(z),
// G_i(z) = -sin t_i H_{i-1}(z) + cos t_i z^-2 G_{i-1}(z), (H_1, G_1) = (cos t_1 +
// sin t_1 z^-1, -sin t_1 + cos t_1 z^-1), with t_1 + ... + t_m = pi / 4.  Over
// the m - 1 free angles, the moment conditions are solved by Levenberg-Marquardt
// steps (Jacobian by central differences) from a deterministic Halton set of
// starting angles.  The conditions have several isolated solutions; the filter
// returned is the one most nearly symmetric about tap 2K (the regularity and
// symmetry the paper cites for its choice of this family).
#include <cmath>
#include <vector>

#include "efpi.h"

namespace {

void lattice(const std::vector<double>& free_angles, std::vector<double>& h) {
  const int m = (int)free_angles.size() + 1;
  double last = M_PI / 4.0;
  for (double t : free_angles) last -= t;
  std::vector<double> a = {std::cos(free_angles.empty() ? last : free_angles[0]),
                           std::sin(free_angles.empty() ? last : free_angles[0])};
  std::vector<double> b = {-a[1], a[0]};
  for (int i = 1; i < m; ++i) {
    const double t = i < m - 1 ? free_angles[i] : last;
    const double c = std::cos(t), s = std::sin(t);
    const size_t n = a.size() + 2;
    std::vector<double> na(n, 0.0), nb(n, 0.0);
    for (size_t k = 0; k < n; ++k) {
      const double hk = k < a.size() ? a[k] : 0.0;
      const double gk = k >= 2 ? b[k - 2] : 0.0;
      na[k] = c * hk + s * gk;
      nb[k] = -s * hk + c * gk;
    }
    a.swap(na);
    b.swap(nb);
  }
  h = a;
}

// Moment conditions: wavelet moments p = 1 .. 2K-1 of the alternating flip (taken
// about the filter's midpoint, which keeps the terms small; moment 0 holds by
// construction) and scaling moments p = 1 .. 2K-1 about tap 2K.
void residuals(const std::vector<double>& x, int order, std::vector<double>& r) {
  std::vector<double> h;
  lattice(x, h);
  const int n = (int)h.size();
  const double mid = 0.5 * (n - 1);
  const double c0 = (double)order;
  r.clear();
  for (int p = 1; p < order; ++p) {
    double sw = 0.0, ss = 0.0;
    for (int k = 0; k < n; ++k) {
      const double sign = (k & 1) ? -1.0 : 1.0;
      sw += sign * h[k] * std::pow(k - mid, p);
      ss += h[k] * std::pow(k - c0, p);
    }
    r.push_back(sw);
    r.push_back(ss);
  }
}

double max_abs(const std::vector<double>& v) {
  double m = 0.0;
  for (double x : v) m = std::fmax(m, std::fabs(x));
  return m;
}

// Solve (J^T J + mu I) dx = -J^T r by Gaussian elimination with partial pivoting.
bool solve_normal(const std::vector<double>& J, const std::vector<double>& r, int nr, int nx,
                  double mu, std::vector<double>& dx) {
  std::vector<double> A(nx * (nx + 1), 0.0);
  for (int i = 0; i < nx; ++i) {
    for (int j = 0; j < nx; ++j) {
      double s = 0.0;
      for (int k = 0; k < nr; ++k) s += J[k * nx + i] * J[k * nx + j];
      A[i * (nx + 1) + j] = s + (i == j ? mu : 0.0);
    }
    double s = 0.0;
    for (int k = 0; k < nr; ++k) s += J[k * nx + i] * r[k];
    A[i * (nx + 1) + nx] = -s;
  }
  for (int c = 0; c < nx; ++c) {
    int piv = c;
    for (int i = c + 1; i < nx; ++i)
      if (std::fabs(A[i * (nx + 1) + c]) > std::fabs(A[piv * (nx + 1) + c])) piv = i;
    if (A[piv * (nx + 1) + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j <= nx; ++j) std::swap(A[c * (nx + 1) + j], A[piv * (nx + 1) + j]);
    for (int i = c + 1; i < nx; ++i) {
      const double f = A[i * (nx + 1) + c] / A[c * (nx + 1) + c];
      for (int j = c; j <= nx; ++j) A[i * (nx + 1) + j] -= f * A[c * (nx + 1) + j];
    }
  }
  dx.assign(nx, 0.0);
  for (int i = nx - 1; i >= 0; --i) {
    double s = A[i * (nx + 1) + nx];
    for (int j = i + 1; j < nx; ++j) s -= A[i * (nx + 1) + j] * dx[j];
    dx[i] = s / A[i * (nx + 1) + i];
  }
  return true;
}

bool levenberg_marquardt(std::vector<double>& x, int order, double tol) {
  const int nx = (int)x.size();
  std::vector<double> r, rp, rm, xt, dx;
  residuals(x, order, r);
  const int nr = (int)r.size();
  double nrm = 0.0;
  for (double v : r) nrm += v * v;
  double mu = 1e-3;
  std::vector<double> J(nr * nx);
  for (int it = 0; it < 400; ++it) {
    if (max_abs(r) < tol) return true;
    for (int j = 0; j < nx; ++j) {
      xt = x;
      xt[j] += 1e-6;
      residuals(xt, order, rp);
      xt[j] -= 2e-6;
      residuals(xt, order, rm);
      for (int k = 0; k < nr; ++k) J[k * nx + j] = (rp[k] - rm[k]) / 2e-6;
    }
    while (true) {
      if (!solve_normal(J, r, nr, nx, mu, dx)) return false;
      xt = x;
      for (int j = 0; j < nx; ++j) xt[j] += dx[j];
      residuals(xt, order, rp);
      double n2 = 0.0;
      for (double v : rp) n2 += v * v;
      if (n2 < nrm) {
        x = xt;
        r = rp;
        nrm = n2;
        mu = std::fmax(mu / 10.0, 1e-15);
        break;
      }
      mu *= 10.0;
      if (mu > 1e10) return max_abs(r) < tol;
    }
  }
  return max_abs(r) < tol;
}

double halton(int i, int base) {
  double f = 1.0, r = 0.0;
  for (int k = i; k > 0; k /= base) {
    f /= base;
    r += f * (k % base);
  }
  return r;
}

}  // namespace

extern "C" efpi_status efpi_coiflet_taps(int32_t n_taps, double* h_taps) {
  if (n_taps != 6 && n_taps != 12) return EFPI_EINVAL;
  if (!h_taps) return EFPI_EINVAL;
  const int order = n_taps / 3;  // 2K vanishing wavelet moments
  const int nfree = n_taps / 2 - 1;
  static const int primes[] = {2, 3, 5, 7, 11, 13, 17, 19};
  std::vector<std::vector<double>> found;
  for (int s = 1; s <= 400; ++s) {
    std::vector<double> x(nfree);
    for (int j = 0; j < nfree; ++j) x[j] = M_PI * (2.0 * halton(s, primes[j]) - 1.0);
    if (!levenberg_marquardt(x, order, 1e-13)) continue;
    std::vector<double> h;
    lattice(x, h);
    bool seen = false;
    for (const auto& g : found) {
      double d = 0.0;
      for (int k = 0; k < n_taps; ++k) d = std::fmax(d, std::fabs(g[k] - h[k]));
      seen |= d < 1e-8;
    }
    if (!seen) found.push_back(h);
  }
  if (found.empty()) return EFPI_ENUMERIC;
  // asymmetry about tap c0 = 2K: sum_j (h_{c0+j} - h_{c0-j})^2, taps outside 0 .. n-1 zero
  const int c0 = order;
  auto asym = [&](const std::vector<double>& h) {
    double a = 0.0;
    for (int j = 1; j < n_taps; ++j) {
      const double hp = c0 + j < n_taps ? h[c0 + j] : 0.0;
      const double hm = c0 - j >= 0 ? h[c0 - j] : 0.0;
      a += (hp - hm) * (hp - hm);
    }
    return a;
  };
  size_t best = 0;
  for (size_t i = 1; i < found.size(); ++i)
    if (asym(found[i]) < asym(found[best])) best = i;
  for (int k = 0; k < n_taps; ++k) h_taps[k] = found[best][k];
  return EFPI_OK;
}
