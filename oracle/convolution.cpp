// Discrete contour convolutions, Sec. "Numerical details: convolution
// integrals on C" (Eqs. cm1, cm2, cr1, ctv1-ctv3, cles1-cles3) and
// Sec. "Implementation: convolution". Test infrastructure only.
#include "oracle.hpp"

namespace oracle {

namespace {

// Values outside the stored triangles of a (not necessarily hermitian)
// contour function X are rebuilt from its hermitian conjugate Xc
// (Eq. hermconjg and the continuation of the modified retarded component).
Mat retx(const HM& X, const HM& Xc, int a, int b) {  // X~^R_{a,b}
  int d = X.d();
  if (a >= b) return Mat(X.R(a, b), X.R(a, b) + d * d);
  Mat m = dag(Xc.R(b, a), d);
  for (auto& v : m) v = -v;
  return m;
}
Mat lesx(const HM& X, const HM& Xc, int a, int b) {  // X^<_{a,b}
  int d = X.d();
  if (a <= b) return Mat(X.L(a, b), X.L(a, b) + d * d);
  Mat m = dag(Xc.L(b, a), d);
  for (auto& v : m) v = -v;
  return m;
}
Mat advx(const HM& X, const HM& Xc, int a, int b) {  // X^A_{a,b} = ([Xc]~^R_{b,a})^dag
  return dag(retx(Xc, X, b, a), X.d());
}
Mat vtx(const HM& X, const HM& Xc, int j, int n) {  // X^lceil(tau_j, t_n)
  int d = X.d();
  Mat m = dag(Xc.T(n, X.g.ntau - j), d);
  for (auto& v : m) v *= -(double)X.g.sig;
  return m;
}

// acc += alpha * A f B   (f == nullptr means the unit matrix)
void add3(Mat& acc, const cd* A, const cd* f, const cd* B, int d, cd alpha) {
  if (f == nullptr) {
    gemm_acc(acc.data(), A, B, d, alpha);
    return;
  }
  Mat Af = zeros(d);
  gemm_acc(Af.data(), A, f, d, 1.0);
  gemm_acc(acc.data(), Af.data(), B, d, alpha);
}

const cd* fat(const Fn* f, int n) { return f ? f->at(n) : nullptr; }

// Eq. cm1 + Eq. cm2.
Mat cm12_impl(int m, const HM& A, const HM& B, const cd* f) {
  const Grid& g = A.g;
  int d = g.d, k = g.k, nt = g.ntau;
  const Weights& W = weights(k);
  double ht = g.htau(), xi = g.sig;
  Mat c = zeros(d);
  // C^M_1: int_0^{tau_m} A(tau_m - tau') B(tau')
  if (m <= k) {
    for (int j = 0; j <= k; j++)
      for (int l = 0; l <= k; l++) add3(c, A.M(j), f, B.M(l), d, ht * W.r(m, j, l));
  } else {
    for (int l = 0; l <= m; l++) add3(c, A.M(m - l), f, B.M(l), d, ht * W.w(m, l));
  }
  // C^M_2: int_{tau_m}^beta A(tau_m - tau') B(tau'), A(tau - beta) = xi A(tau)
  if (m >= nt - k) {
    for (int j = 0; j <= k; j++)
      for (int l = 0; l <= k; l++)
        add3(c, A.M(nt - j), f, B.M(nt - l), d, ht * xi * W.r(nt - m, j, l));
  } else {
    for (int l = 0; l <= nt - m; l++)
      add3(c, A.M(nt - l), f, B.M(m + l), d, ht * xi * W.w(nt - m, l));
  }
  return c;
}

// Eq. ctv2 + Eq. ctv3: int_0^beta A^rceil(t_n, tau') B^M(tau' - tau_m).
Mat ctv23_impl(int n, int m, const HM& A, const HM& B, const cd* f) {
  const Grid& g = A.g;
  int d = g.d, k = g.k, nt = g.ntau;
  const Weights& W = weights(k);
  double ht = g.htau(), xi = g.sig;
  Mat c = zeros(d);
  if (m <= k) {
    for (int j = 0; j <= k; j++)
      for (int l = 0; l <= k; l++) add3(c, A.T(n, l), f, B.M(nt - j), d, ht * xi * W.r(m, j, l));
  } else {
    for (int l = 0; l <= m; l++) add3(c, A.T(n, m - l), f, B.M(nt - l), d, ht * xi * W.w(m, l));
  }
  if (m >= nt - k) {
    for (int j = 0; j <= k; j++)
      for (int l = 0; l <= k; l++) add3(c, A.T(n, nt - l), f, B.M(j), d, ht * W.r(nt - m, j, l));
  } else {
    for (int l = 0; l <= nt - m; l++) add3(c, A.T(n, m + l), f, B.M(l), d, ht * W.w(nt - m, l));
  }
  return c;
}

}  // namespace

Mat Rt(const HM& G, int a, int b) { return retx(G, G, a, b); }
Mat Lh(const HM& G, int a, int b) { return lesx(G, G, a, b); }
Mat Adv(const HM& G, int a, int b) { return advx(G, G, a, b); }
Mat Vt(const HM& G, int j, int n) { return vtx(G, G, j, n); }
Mat RtX(const HM& X, const HM& Xc, int a, int b) { return retx(X, Xc, a, b); }
Mat LhX(const HM& X, const HM& Xc, int a, int b) { return lesx(X, Xc, a, b); }
Mat AdvX(const HM& X, const HM& Xc, int a, int b) { return advx(X, Xc, a, b); }
Mat VtX(const HM& X, const HM& Xc, int j, int n) { return vtx(X, Xc, j, n); }

Mat cm12(int m, const HM& A, const HM& B, const cd* f) { return cm12_impl(m, A, B, f); }
Mat ctv23(int n, int m, const HM& A, const HM& B, const cd* f) { return ctv23_impl(n, m, A, B, f); }

void convolution_timestep(int n, const HM& C, const HM& A, const HM& Acc, const HM& B,
                          const HM& Bcc, const Fn* f) {
  const Grid& g = A.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  double h = g.h, ht = g.htau();
  size_t bs = (size_t)d * d;
  if (n == -1) {
    for (int m = 0; m <= ntau; m++) {
      Mat c = cm12_impl(m, A, B, fat(f, -1));
      std::copy(c.begin(), c.end(), C.M(m));
    }
    return;
  }
  // Retarded, Eq. cr1: int_{t_m}^{t_n} A^R(t_n, t) f(t) B^R(t, t_m).
#pragma omp parallel for schedule(dynamic)
  for (int m = 0; m <= n; m++) {
    Mat c = zeros(d);
    if (n > k && n - m > k) {
      for (int j = m; j <= n; j++)
        add3(c, A.R(n, j), fat(f, j), B.R(j, m), d, h * W.w(n - m, j - m));
    } else if (n > k) {
      for (int j = 0; j <= k; j++) {
        Mat b = retx(B, Bcc, n - j, m);
        add3(c, A.R(n, n - j), fat(f, n - j), b.data(), d, h * W.w(n - m, j));
      }
    } else {
      for (int j = 0; j <= k; j++) {
        Mat a = retx(A, Acc, n, j), b = retx(B, Bcc, j, m);
        add3(c, a.data(), fat(f, j), b.data(), d, h * W.i(m, n, j));
      }
    }
    std::copy(c.begin(), c.end(), C.R(n, m));
  }
  // Left-mixing, Eqs. ctv1 + ctv2 + ctv3.
#pragma omp parallel for schedule(static)
  for (int m = 0; m <= ntau; m++) {
    Mat c = ctv23_impl(n, m, A, B, fat(f, -1));
    if (n > k) {
      for (int j = 0; j <= n; j++) add3(c, A.R(n, j), fat(f, j), B.T(j, m), d, h * W.w(n, j));
    } else {
      for (int j = 0; j <= k; j++) {
        Mat a = retx(A, Acc, n, j);
        add3(c, a.data(), fat(f, j), B.T(j, m), d, h * W.s(n, j));
      }
    }
    std::copy(c.begin(), c.end(), C.T(n, m));
  }
  // Lesser C^<(t_m, t_n), m = 0..n, Eqs. cles1 + cles2 + cles3.
#pragma omp parallel for schedule(dynamic)
  for (int m = 0; m <= n; m++) {
    Mat c = zeros(d);
    // cles1: int_0^{t_m} A^R(t_m, t) f(t) B^<(t, t_n)
    if (m > k) {
      for (int j = 0; j <= m; j++) {
        Mat b = lesx(B, Bcc, j, n);
        add3(c, A.R(m, j), fat(f, j), b.data(), d, h * W.w(m, j));
      }
    } else {
      for (int j = 0; j <= k; j++) {
        Mat a = retx(A, Acc, m, j), b = lesx(B, Bcc, j, n);
        add3(c, a.data(), fat(f, j), b.data(), d, h * W.s(m, j));
      }
    }
    // cles2: int_0^{t_n} A^<(t_m, t) f(t) B^A(t, t_n)
    int jmax = n > k ? n : k;
    for (int j = 0; j <= jmax; j++) {
      Mat a = lesx(A, Acc, m, j), b = advx(B, Bcc, j, n);
      add3(c, a.data(), fat(f, j), b.data(), d, h * W.w(n, j));
    }
    // cles3: -i int_0^beta A^rceil(t_m, tau) f(0^-) B^lceil(tau, t_n)
    for (int j = 0; j <= ntau; j++) {
      Mat b = vtx(B, Bcc, j, n);
      add3(c, A.T(m, j), fat(f, -1), b.data(), d, cd(0.0, -1.0) * ht * W.w(ntau, j));
    }
    std::copy(c.begin(), c.end(), C.L(m, n));
  }
  (void)bs;
}

Mat conv_les_diag(int n, const HM& A, const HM& B) {
  const Grid& g = A.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  double h = g.h, ht = g.htau();
  Mat c = zeros(d);
  if (n > k) {
    for (int j = 0; j <= n; j++) gemm_acc(c.data(), A.R(n, j), B.L(j, n), d, h * W.w(n, j));
  } else {
    for (int j = 0; j <= k; j++) {
      Mat a = Rt(A, n, j), b = Lh(B, j, n);
      gemm_acc(c.data(), a.data(), b.data(), d, h * W.s(n, j));
    }
  }
  int jmax = n > k ? n : k;
  for (int j = 0; j <= jmax; j++) {
    Mat a = Lh(A, n, j), b = Adv(B, j, n);
    gemm_acc(c.data(), a.data(), b.data(), d, h * W.w(n, j));
  }
  for (int j = 0; j <= ntau; j++) {
    Mat b = Vt(B, j, n);
    gemm_acc(c.data(), A.T(n, j), b.data(), d, cd(0.0, -1.0) * ht * W.w(ntau, j));
  }
  return c;
}

}  // namespace oracle
