// Host construction of the reference-element tables (FP64).
//
// Triangle basis: the orthonormal Dubiner (Koornwinder) basis written in
// collapsed coordinates a = 2 xi / (1 - eta) - 1, b = 2 eta - 1:
//   psi_pq = sqrt(2 (2p+1)(p+q+1)) P_p(a) (1 - eta)^p P_q^(2p+1,0)(b),
// modes ordered by total degree n = p + q, then q ascending.  Gradients by the
// chain rule through (a, b); every point used lies strictly below the top
// vertex, so 1 - eta > 0.
#include "ref_element.hpp"

#include <array>
#include <cmath>

namespace bsw {
namespace {

// General Jacobi polynomial P_n^(al,be)(x) by the three-term recurrence.
double jacobi(int n, double al, double be, double x) {
  if (n == 0) return 1.0;
  double pm = 1.0;
  double p = 0.5 * (al - be + (al + be + 2.0) * x);
  for (int k = 1; k < n; ++k) {
    const double s = 2.0 * k + al + be;
    const double a1 = 2.0 * (k + 1) * (k + al + be + 1) * s;
    const double a2 = (s + 1) * (al * al - be * be);
    const double a3 = s * (s + 1) * (s + 2);
    const double a4 = 2.0 * (k + al) * (k + be) * (s + 2);
    const double pn = ((a2 + a3 * x) * p - a4 * pm) / a1;
    pm = p;
    p = pn;
  }
  return p;
}

// d/dx P_n^(al,be) = (n + al + be + 1)/2 P_{n-1}^(al+1,be+1)
double jacobi_d(int n, double al, double be, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + al + be + 1.0) * jacobi(n - 1, al + 1.0, be + 1.0, x);
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // initial guess (Tricomi), then Newton on P_n
    double z = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
    for (int it = 0; it < 60; ++it) {
      const double p = jacobi(n, 0, 0, z), dp = jacobi_d(n, 0, 0, z);
      const double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * std::fabs(z) + 1e-300) break;
    }
    const double dp = jacobi_d(n, 0, 0, z);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void line_basis(int P, double xi, double* phi, double* dphi) {
  for (int i = 0; i <= P; ++i) {
    const double c = std::sqrt(i + 0.5);
    phi[i] = c * jacobi(i, 0, 0, xi);
    if (dphi) {
      dphi[2 * i] = c * jacobi_d(i, 0, 0, xi);
      dphi[2 * i + 1] = 0.0;
    }
  }
}

void tri_basis(int P, double xi, double eta, double* phi, double* dphi) {
  const double om = 1.0 - eta;          // (1 - b) / 2
  if (om == 0.0) {
    // the collapsed vertex (0, 1): P_p(a) (1 - eta)^p tends to 0 for p >= 1
    // (its homogeneous form is a polynomial in 2 xi + eta - 1 and 1 - eta,
    // both zero here), and only p = 1 keeps a first derivative
    int k = 0;
    for (int n = 0; n <= P; ++n)
      for (int q = 0; q <= n; ++q, ++k) {
        const int p = n - q;
        const double c = std::sqrt(2.0 * (2 * p + 1) * (p + q + 1));
        const double gb = jacobi(q, 2.0 * p + 1, 0, 1.0), dgb = jacobi_d(q, 2.0 * p + 1, 0, 1.0);
        phi[k] = p == 0 ? c * gb : 0.0;
        if (dphi) {
          dphi[2 * k] = p == 1 ? c * 2.0 * gb : 0.0;
          dphi[2 * k + 1] = p == 1 ? c * gb : (p == 0 ? c * 2.0 * dgb : 0.0);
        }
      }
    return;
  }
  const double a = 2.0 * xi / om - 1.0;
  const double b = 2.0 * eta - 1.0;
  int k = 0;
  for (int n = 0; n <= P; ++n)
    for (int q = 0; q <= n; ++q, ++k) {
      const int p = n - q;
      const double c = std::sqrt(2.0 * (2 * p + 1) * (p + q + 1));
      const double fa = jacobi(p, 0, 0, a), dfa = jacobi_d(p, 0, 0, a);
      const double gb = jacobi(q, 2.0 * p + 1, 0, b), dgb = jacobi_d(q, 2.0 * p + 1, 0, b);
      const double omp = std::pow(om, p);
      phi[k] = c * fa * omp * gb;
      if (dphi) {
        const double omp1 = p > 0 ? std::pow(om, p - 1) : 0.0;
        // d/dxi: da/dxi = 2 / (1 - eta)
        dphi[2 * k] = c * 2.0 * dfa * omp1 * gb;
        // d/deta: da/deta = (a + 1) / (1 - eta), d(1-eta)^p/deta = -p (1-eta)^(p-1), db/deta = 2
        dphi[2 * k + 1] = c * (omp1 * ((a + 1.0) * dfa - p * fa) * gb + fa * omp * 2.0 * dgb);
      }
    }
}

struct TriRule {
  std::vector<std::array<double, 2>> x;
  std::vector<double> w;  // normalised to sum 1
};

void add_orbit(TriRule& r, double l1, double l2, double l3, double w) {
  // all distinct permutations of barycentric (l1, l2, l3); point = (l2, l3)
  std::array<std::array<double, 3>, 6> perm = {{{l1, l2, l3}, {l1, l3, l2}, {l2, l1, l3},
                                                 {l2, l3, l1}, {l3, l1, l2}, {l3, l2, l1}}};
  std::vector<std::array<double, 3>> seen;
  for (auto& pm : perm) {
    bool dup = false;
    for (auto& s : seen)
      if (s[0] == pm[0] && s[1] == pm[1] && s[2] == pm[2]) dup = true;
    if (dup) continue;
    seen.push_back(pm);
    r.x.push_back({pm[1], pm[2]});
    r.w.push_back(w);
  }
}

// 12-point degree-6 rule: 2 orbits (a, a, 1-2a) and 1 orbit (b, c, 1-b-c).
// Published parameters are polished by Gauss-Newton on the moments
// int_T xi^i eta^j dA / |T| = 2 i! j! / (i+j+2)!, i + j <= 6.
TriRule rule12() {
  double u[7] = {0.063089014491502, 0.050844906370207, 0.249286745170910, 0.116786275726379,
                 0.053145049844817, 0.310352451033784, 0.082851075618374};
  auto build = [](const double* v) {
    TriRule r;
    add_orbit(r, v[0], v[0], 1.0 - 2.0 * v[0], v[1]);
    add_orbit(r, v[2], v[2], 1.0 - 2.0 * v[2], v[3]);
    add_orbit(r, v[4], v[5], 1.0 - v[4] - v[5], v[6]);
    return r;
  };
  auto fact = [](int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; };
  auto moments = [&](const double* v, std::vector<double>& out) {
    TriRule r = build(v);
    out.clear();
    for (int i = 0; i <= 6; ++i)
      for (int j = 0; i + j <= 6; ++j) {
        double s = 0;
        for (size_t k = 0; k < r.w.size(); ++k) s += r.w[k] * std::pow(r.x[k][0], i) * std::pow(r.x[k][1], j);
        out.push_back(s - 2.0 * fact(i) * fact(j) / fact(i + j + 2));
      }
  };
  for (int it = 0; it < 8; ++it) {
    std::vector<double> f0, fp, fm;
    moments(u, f0);
    const int m = (int)f0.size();
    std::vector<double> J(m * 7);
    for (int c = 0; c < 7; ++c) {
      double up[7], um[7];
      for (int k = 0; k < 7; ++k) up[k] = um[k] = u[k];
      const double h = 1e-7 * std::max(1.0, std::fabs(u[c]));
      up[c] += h; um[c] -= h;
      moments(up, fp); moments(um, fm);
      for (int r = 0; r < m; ++r) J[r * 7 + c] = (fp[r] - fm[r]) / (2 * h);
    }
    // normal equations (7x7), Cholesky-free Gauss-Jordan
    double A[7][8] = {};
    for (int a = 0; a < 7; ++a) {
      for (int b = 0; b < 7; ++b)
        for (int r = 0; r < m; ++r) A[a][b] += J[r * 7 + a] * J[r * 7 + b];
      for (int r = 0; r < m; ++r) A[a][7] -= J[r * 7 + a] * f0[r];
    }
    for (int c = 0; c < 7; ++c) {
      int piv = c;
      for (int r = c + 1; r < 7; ++r) if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      for (int k = 0; k < 8; ++k) std::swap(A[c][k], A[piv][k]);
      for (int r = 0; r < 7; ++r) {
        if (r == c) continue;
        const double f = A[r][c] / A[c][c];
        for (int k = c; k < 8; ++k) A[r][k] -= f * A[c][k];
      }
    }
    for (int c = 0; c < 7; ++c) u[c] += A[c][7] / A[c][c];
  }
  return build(u);
}

TriRule tri_rule(int P) {
  TriRule r;
  if (P == 1) {
    add_orbit(r, 2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 3.0);
  } else if (P == 2) {
    const double s = std::sqrt(15.0);
    add_orbit(r, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 0.225);
    add_orbit(r, (6.0 - s) / 21.0, (6.0 - s) / 21.0, (9.0 + 2.0 * s) / 21.0, (155.0 - s) / 1200.0);
    add_orbit(r, (6.0 + s) / 21.0, (6.0 + s) / 21.0, (9.0 - 2.0 * s) / 21.0, (155.0 + s) / 1200.0);
  } else if (P == 3) {
    r = rule12();
  }
  return r;
}

}  // namespace

void eval_basis(int dim, int P, double xi, double eta, double* phi, double* dphi) {
  if (dim == 1) line_basis(P, xi, phi, dphi);
  else tri_basis(P, xi, eta, phi, dphi);
}

bool build_reference(int dim, int P, RefElement& R) {
  R = RefElement();
  R.dim = dim;
  R.P = P;
  R.nf = 1 + dim + dim * dim;
  std::vector<double> gx, gw;
  if (dim == 1) {
    if (P < 0 || P > 4) return false;
    R.np = P + 1; R.nq = P + 1; R.nfq = 1; R.nfc = 2; R.measure = 2.0;
    gauss_legendre(R.nq, gx, gw);
    R.qxi.resize(2 * R.nq); R.qw = gw;
    for (int q = 0; q < R.nq; ++q) { R.qxi[2 * q] = gx[q]; R.qxi[2 * q + 1] = 0.0; }
    R.fw = {1.0};
    R.fphi.resize(2 * R.np);
    line_basis(P, -1.0, &R.fphi[0], nullptr);
    line_basis(P, 1.0, &R.fphi[R.np], nullptr);
  } else if (dim == 2) {
    if (P < 1 || P > 3) return false;
    TriRule tr = tri_rule(P);
    R.np = (P + 1) * (P + 2) / 2; R.nq = (int)tr.w.size(); R.nfq = P + 1; R.nfc = 3; R.measure = 0.5;
    R.qxi.resize(2 * R.nq); R.qw.resize(R.nq);
    for (int q = 0; q < R.nq; ++q) {
      R.qxi[2 * q] = tr.x[q][0]; R.qxi[2 * q + 1] = tr.x[q][1]; R.qw[q] = 0.5 * tr.w[q];
    }
    gauss_legendre(R.nfq, gx, R.fw);
    const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    R.fphi.resize(3 * R.nfq * R.np);
    for (int f = 0; f < 3; ++f) {
      const double* A = V[f];
      const double* B = V[(f + 1) % 3];
      for (int r = 0; r < R.nfq; ++r) {
        const double s = 0.5 * (1.0 + gx[r]);
        tri_basis(P, A[0] + s * (B[0] - A[0]), A[1] + s * (B[1] - A[1]), &R.fphi[(f * R.nfq + r) * R.np], nullptr);
      }
    }
  } else {
    return false;
  }
  R.phi.resize(R.nq * R.np);
  R.dphi.resize(R.nq * R.np * 2);
  for (int q = 0; q < R.nq; ++q)
    eval_basis(dim, P, R.qxi[2 * q], R.qxi[2 * q + 1], &R.phi[q * R.np], &R.dphi[q * R.np * 2]);
  return true;
}

}  // namespace bsw
