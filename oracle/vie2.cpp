// Dyson equation in integral form on the L-shaped contour,
//   (1 + F) * G = Q  (Eq. vie2),   G * (1 + F^ddagger) = Q  (Eq. vie2_cc),
// for hermitian G and Q: Matsubara, start-up and time stepping
// (Sec. "Implementation: vie2"), built from the second-kind Volterra rules of
// Sec. "Volterra Integral equation of the second kind" (Eqs. MBCVSAMx01_start,
// MBCVSAMx01_t and the conjugate step) and the discrete convolutions of
// Eqs. cm1, cm2, cr1, ctv1-ctv3, cles1-cles3. F and Fcc = F^ddagger are given
// separately: values of F outside its stored triangles come from Fcc and
// vice versa. Test infrastructure only.
#include "oracle.hpp"

namespace oracle {

namespace {

void put(cd* dst, const Mat& m) { std::copy(m.begin(), m.end(), dst); }

Mat blk(const cd* p, int d) { return Mat(p, p + (size_t)d * d); }

// 1 + c X
Mat one_plus(const Mat& X, int d, cd c) {
  Mat m = X;
  for (auto& v : m) v *= c;
  for (int i = 0; i < d; i++) m[i * d + i] += 1.0;
  return m;
}

// A^{-1} B
Mat lsolve(const Mat& A, const Mat& B, int d, bool* ok) {
  Mat a = A, b = B;
  *ok = solve(d, d, a.data(), b.data()) && *ok;
  return b;
}
// B A^{-1} (from A^T X^T = B^T)
Mat rsolve(const Mat& A, const Mat& B, int d, bool* ok) {
  Mat at = zeros(d), bt = zeros(d);
  for (int i = 0; i < d; i++)
    for (int j = 0; j < d; j++) {
      at[i * d + j] = A[j * d + i];
      bt[i * d + j] = B[j * d + i];
    }
  *ok = solve(d, d, at.data(), bt.data()) && *ok;
  Mat x = zeros(d);
  for (int i = 0; i < d; i++)
    for (int j = 0; j < d; j++) x[i * d + j] = bt[j * d + i];
  return x;
}

// Dense block system sum_l A_{p,l} y_l = b_p, p, l = 0..nu-1 (d x d blocks,
// d right-hand-side columns).
struct Blocks {
  int nu, d;
  std::vector<cd> A, B;
  Blocks(int nu_, int d_) : nu(nu_), d(d_), A((size_t)nu_ * d_ * nu_ * d_, 0.0), B((size_t)nu_ * d_ * d_, 0.0) {}
  void set(int p, int l, const Mat& m) {
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) A[(size_t)(p * d + i) * nu * d + l * d + j] = m[i * d + j];
  }
  void rhs(int p, const Mat& m) {
    for (int i = 0; i < d; i++)
      for (int c = 0; c < d; c++) B[(size_t)(p * d + i) * d + c] = m[i * d + c];
  }
  Mat x(int p) const {
    Mat m = zeros(d);
    for (int i = 0; i < d; i++)
      for (int c = 0; c < d; c++) m[i * d + c] = B[(size_t)(p * d + i) * d + c];
    return m;
  }
  bool run() { return solve(nu * d, d, A.data(), B.data()); }
};

// Coefficient of y_l in row p of the start-up of Eq. MBCVSAMx01 with kernel
// k(t, s) = F^R(t, s): M_{p,l} = delta_{pl} + h s_{p,l} F~^R_{p,l}.
Mat start_coef(const HM& F, const HM& Fcc, int p, int l) {
  const Grid& g = F.g;
  int d = g.d;
  Mat f = RtX(F, Fcc, p, l);
  Mat m = zeros(d);
  for (int i = 0; i < d * d; i++) m[i] = g.h * weights(g.k).s(p, l) * f[i];
  if (p == l)
    for (int i = 0; i < d; i++) m[i * d + i] += 1.0;
  return m;
}

// Rows p = 1..k of the start-up (Eq. MBCVSAMx01_start) for y_0 given and
// sources q_p: returns y_1..y_k.
std::vector<Mat> vie_start(const HM& F, const HM& Fcc, const Mat& y0, const std::vector<Mat>& q, bool* ok) {
  int d = F.g.d, k = F.g.k;
  Blocks sys(k, d);
  for (int p = 1; p <= k; p++) {
    for (int l = 1; l <= k; l++) sys.set(p - 1, l - 1, start_coef(F, Fcc, p, l));
    Mat r = q[p];
    Mat m0 = start_coef(F, Fcc, p, 0);
    gemm_acc(r.data(), m0.data(), y0.data(), d, -1.0);
    sys.rhs(p - 1, r);
  }
  *ok = sys.run() && *ok;
  std::vector<Mat> y(k + 1);
  y[0] = y0;
  for (int p = 1; p <= k; p++) y[p] = sys.x(p - 1);
  return y;
}

// Source of the lesser equation Eq. vie2_langreth_les at (m, n):
//   Q^<_{m,n} - C^<_2[F,1,G](m,n) - C^<_3[F,1,G](m,n)  (Eqs. cles2, cles3),
// Q^<_{m,n} for m > n from the hermitian symmetry of Q.
Mat les_source(int m, int n, const HM& G, const HM& F, const HM& Fcc, const HM& Q) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  Mat q = Lh(Q, m, n);
  int jmax = n > k ? n : k;
  for (int j = 0; j <= jmax; j++) {
    Mat f = LhX(F, Fcc, m, j), a = Adv(G, j, n);
    gemm_acc(q.data(), f.data(), a.data(), d, -g.h * W.w(n, j));
  }
  for (int j = 0; j <= ntau; j++) {
    Mat v = Vt(G, j, n);
    gemm_acc(q.data(), F.T(m, j), v.data(), d, -cd(0.0, -1.0) * g.htau() * W.w(ntau, j));
  }
  return q;
}

}  // namespace

bool vie2_mat(const HM& G, const HM& F, const HM& Q) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, nt = g.ntau;
  const Weights& W = weights(k);
  double ht = g.htau(), xi = g.sig;
  // G_m + [F * G]^M(m) = Q_m, the convolution by Eqs. cm1 + cm2 (f = 1):
  // one dense (ntau+1) d system.
  int N = (nt + 1) * d;
  std::vector<cd> A((size_t)N * N, 0.0), rhs((size_t)N * d);
  auto add = [&](int m, int l, const cd* f, double c) {
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) A[(size_t)(m * d + i) * N + l * d + j] += c * f[i * d + j];
  };
  for (int m = 0; m <= nt; m++) {
    if (m <= k) {
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) add(m, l, F.M(j), ht * W.r(m, j, l));
    } else {
      for (int l = 0; l <= m; l++) add(m, l, F.M(m - l), ht * W.w(m, l));
    }
    if (m >= nt - k) {
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) add(m, nt - l, F.M(nt - j), ht * xi * W.r(nt - m, j, l));
    } else {
      for (int l = 0; l <= nt - m; l++) add(m, m + l, F.M(nt - l), ht * xi * W.w(nt - m, l));
    }
  }
  for (int r = 0; r < N; r++) A[(size_t)r * N + r] += 1.0;
  for (int m = 0; m <= nt; m++)
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) rhs[(size_t)(m * d + i) * d + j] = Q.M(m)[i * d + j];
  bool ok = solve(N, d, A.data(), rhs.data());
  for (int m = 0; m <= nt; m++)
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) G.M(m)[i * d + j] = rhs[(size_t)(m * d + i) * d + j];
  return ok;
}

bool vie2_start(const HM& G, const HM& F, const HM& Fcc, const HM& Q) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  double h = g.h, xi = g.sig;
  bool ok = true;
  // Retarded, columns m = 0..k in order (Sec. "Start", first item): with
  // y_p = G^R_{p,m}, y_m = Q^R_{m,m} (Eq. vie2_ini_r) and y_l = -[G^R_{m,l}]^dag
  // for l < m (known from the earlier columns),
  //   y_p + h sum_{l=0..k} I_{m,p,l} F~^R_{p,l} y_l = Q^R_{p,m},  p = m+1..k.
  // Reading: the printed matrix has eps_n where the unit term delta_{pl}
  // belongs, and its right-hand side drops Q^R_{p,m}.
  for (int m = 0; m <= k; m++) {
    Mat ym = blk(Q.R(m, m), d);
    put(G.R(m, m), ym);
    if (m == k) break;
    std::vector<Mat> y(m + 1);
    for (int l = 0; l < m; l++) {
      y[l] = dag(G.R(m, l), d);
      for (auto& v : y[l]) v = -v;
    }
    y[m] = ym;
    auto coef = [&](int p, int l) {
      Mat f = RtX(F, Fcc, p, l);
      for (auto& v : f) v *= h * W.i(m, p, l);
      if (p == l)
        for (int i = 0; i < d; i++) f[i * d + i] += 1.0;
      return f;
    };
    int nu = k - m;
    Blocks sys(nu, d);
    for (int p = m + 1; p <= k; p++) {
      for (int l = m + 1; l <= k; l++) sys.set(p - m - 1, l - m - 1, coef(p, l));
      Mat r = blk(Q.R(p, m), d);
      for (int l = 0; l <= m; l++) {
        Mat c = coef(p, l);
        gemm_acc(r.data(), c.data(), y[l].data(), d, -1.0);
      }
      sys.rhs(p - m - 1, r);
    }
    ok = sys.run() && ok;
    for (int p = m + 1; p <= k; p++) put(G.R(p, m), sys.x(p - m - 1));
  }
  // Left-mixing, each tau index m (second item): Eq. MBCVSAMx01 with
  // k = F^R, y_0 = i xi G^M(beta - tau_m) (Eq. vie2_ini_tv) and
  // q_p = Q^rceil_{p,m} - (C^rceil_2 + C^rceil_3)[F,1,G](p,m) (Eq. map_vie_tv).
#pragma omp parallel for schedule(static) reduction(&& : ok)
  for (int m = 0; m <= ntau; m++) {
    Mat y0 = blk(G.M(ntau - m), d);
    for (auto& v : y0) v *= cd(0.0, xi);
    std::vector<Mat> q(k + 1);
    for (int p = 1; p <= k; p++) {
      q[p] = blk(Q.T(p, m), d);
      Mat c = ctv23(p, m, F, G, nullptr);
      for (int i = 0; i < d * d; i++) q[p][i] -= c[i];
    }
    bool lok = true;
    std::vector<Mat> y = vie_start(F, Fcc, y0, q, &lok);
    ok = ok && lok;
    for (int p = 0; p <= k; p++) put(G.T(p, m), y[p]);
  }
  // Lesser, columns n = 0..k (third item), after R and rceil: Eq. MBCVSAMx01
  // in t_m with k = F^R, y_0 = -[G^rceil_{n,0}]^dag (Eq. vie2_ini_les) and the
  // sources of Eq. map_les_vie2. Rows m <= n are stored.
  for (int n = 0; n <= k; n++) {
    Mat y0 = dag(G.T(n, 0), d);
    for (auto& v : y0) v = -v;
    std::vector<Mat> q(k + 1);
    for (int p = 1; p <= k; p++) q[p] = les_source(p, n, G, F, Fcc, Q);
    std::vector<Mat> y = vie_start(F, Fcc, y0, q, &ok);
    for (int p = 0; p <= n; p++) put(G.L(p, n), y[p]);
  }
  return ok;
}

bool vie2_timestep(int n, const HM& G, const HM& F, const HM& Fcc, const HM& Q) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  double h = g.h, ht = g.htau();
  bool ok = true;
  if (n <= k) return false;
  Mat Fnn = blk(F.R(n, n), d);

  // ---- retarded row n (Sec. "Time stepping", first item). For fixed m,
  // y(t) = G^R(t, t_m) obeys Eq. MBCVSAMx01 with k = F^R; the convolution
  // by Eq. cr1. y_n = G^R_{n,n} = Q^R_{n,n} (Eq. vie2_ini_r).
  put(G.R(n, n), blk(Q.R(n, n), d));
#pragma omp parallel for schedule(dynamic) reduction(&& : ok)
  for (int m = 0; m < n; m++) {
    int N = n - m;
    Mat rhs = blk(Q.R(n, m), d);
    Mat A;
    if (N > k) {
      for (int j = m; j < n; j++) gemm_acc(rhs.data(), F.R(n, j), G.R(j, m), d, -h * W.w(N, j - m));
      A = one_plus(Fnn, d, h * W.w(N, N));
    } else {
      // interval shorter than k+1 points: the k+1 points n-k..n, with G^R
      // continued to t < t' (Eq. y_to_GR)
      for (int j = 1; j <= k; j++) {
        Mat y = Rt(G, n - j, m);
        gemm_acc(rhs.data(), F.R(n, n - j), y.data(), d, -h * W.w(N, j));
      }
      A = one_plus(Fnn, d, h * W.w(N, 0));
    }
    bool lok = true;
    put(G.R(n, m), lsolve(A, rhs, d, &lok));
    ok = ok && lok;
  }

  // ---- left-mixing row n (second item): Eq. MBCVSAMx01_t per tau index,
  // source Q^rceil - (C^rceil_2 + C^rceil_3)[F,1,G].
  Mat AT = one_plus(Fnn, d, h * W.w(n, n));
#pragma omp parallel for schedule(static) reduction(&& : ok)
  for (int m = 0; m <= ntau; m++) {
    Mat rhs = blk(Q.T(n, m), d);
    Mat c = ctv23(n, m, F, G, nullptr);
    for (int i = 0; i < d * d; i++) rhs[i] -= c[i];
    for (int j = 0; j < n; j++) gemm_acc(rhs.data(), F.R(n, j), G.T(j, m), d, -h * W.w(n, j));
    bool lok = true;
    put(G.T(n, m), lsolve(AT, rhs, d, &lok));
    ok = ok && lok;
  }

  // ---- lesser column n (third item, variant B): for fixed m, y(t) =
  // G^<(t_m, t) obeys the conjugate equation with k(s,t) = [F^ddagger]^A(s,t)
  // and source q = Q^< - C^<_1[G,1,F^dd](m,n) - C^<_3[G,1,F^dd](m,n); one step
  // of the conjugate rule at t_n. Every row m < n is independent; the row
  // m = n follows from the finished column (G^<_{n,l} = -[G^<_{l,n}]^dag).
  Mat AL = one_plus(AdvX(Fcc, F, n, n), d, h * W.w(n, n));
  auto row = [&](int m, bool* rok) {
    Mat rhs = blk(Q.L(m, n), d);
    // C^<_1 (Eq. cles1): int_0^{t_m} G^R(t_m, t) Fcc^<(t, t_n)
    if (m > k) {
      for (int j = 0; j <= m; j++) {
        Mat f = LhX(Fcc, F, j, n);
        gemm_acc(rhs.data(), G.R(m, j), f.data(), d, -h * W.w(m, j));
      }
    } else {
      for (int j = 0; j <= k; j++) {
        Mat r = Rt(G, m, j), f = LhX(Fcc, F, j, n);
        gemm_acc(rhs.data(), r.data(), f.data(), d, -h * W.s(m, j));
      }
    }
    // C^<_3 (Eq. cles3): -i int_0^beta G^rceil(t_m, tau) Fcc^lceil(tau, t_n)
    for (int j = 0; j <= ntau; j++) {
      Mat v = VtX(Fcc, F, j, n);
      gemm_acc(rhs.data(), G.T(m, j), v.data(), d, -cd(0.0, -1.0) * ht * W.w(ntau, j));
    }
    // history of the conjugate step: sum_{l<n} w(n,l) G^<_{m,l} Fcc^A_{l,n}
    for (int l = 0; l < n; l++) {
      Mat y = Lh(G, m, l), a = AdvX(Fcc, F, l, n);
      gemm_acc(rhs.data(), y.data(), a.data(), d, -h * W.w(n, l));
    }
    return rsolve(AL, rhs, d, rok);
  };
#pragma omp parallel for schedule(dynamic) reduction(&& : ok)
  for (int m = 0; m < n; m++) {
    bool lok = true;
    put(G.L(m, n), row(m, &lok));
    ok = ok && lok;
  }
  put(G.L(n, n), row(n, &ok));
  return ok;
}

}  // namespace oracle
