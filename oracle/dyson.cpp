// Dyson equation in integro-differential form on the L-shaped contour:
// Matsubara, start-up and time-stepping (Sec. "Implementation: dyson"),
// built from the Volterra start-up and time-step rules of Sec. "Numerical
// details: Volterra integral equations" (Eqs. vdiff_start, MBCVSAMx_t,
// MBCVSAMx_cc_start, MBCVSAMx_cc_t). Test infrastructure only.
//
// Notation: e_n = eps_n - mu (Reading: the equations are printed with eps
// only, the interface takes mu; H - mu N is the operator that evolves the
// contour, so every branch uses eps - mu). xi = sig = -1 fermions, +1 bosons.
#include <cmath>
#include <cstdio>

#include "oracle.hpp"

namespace oracle {

namespace {

Mat ehat(const Fn& eps, int n, double mu) {
  int d = eps.d;
  Mat e(eps.at(n), eps.at(n) + d * d);
  for (int i = 0; i < d; i++) e[i * d + i] -= mu;
  return e;
}

void set(cd* dst, const Mat& m) { std::copy(m.begin(), m.end(), dst); }

Mat scaled(const cd* A, int d, cd a) {
  Mat m(A, A + d * d);
  for (auto& v : m) v *= a;
  return m;
}

// X = A^{-1} B for d x d blocks.
Mat left_solve(const Mat& A, const Mat& B, int d, bool* ok) {
  Mat a = A, b = B;
  *ok = solve(d, d, a.data(), b.data()) && *ok;
  return b;
}
// X = B A^{-1}  (solves A^T X^T = B^T).
Mat right_solve(const Mat& A, const Mat& B, int d, bool* ok) {
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

// Block system sum_{l} A_{p,l} y_l = r_p, p,l = 1..nu (blocks d x d), i.e.
// a (nu d) x (nu d) dense solve with d right-hand-side columns.
struct BlockSys {
  int nu, d;
  std::vector<cd> A, B;
  BlockSys(int nu_, int d_) : nu(nu_), d(d_), A((size_t)nu_ * d_ * nu_ * d_), B((size_t)nu_ * d_ * d_) {}
  cd& a(int p, int l, int i, int j) { return A[((size_t)(p * d + i) * nu * d) + l * d + j]; }
  cd& b(int p, int i, int c) { return B[(size_t)(p * d + i) * d + c]; }
  void set_a(int p, int l, const Mat& m) {
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) a(p, l, i, j) = m[i * d + j];
  }
  void add_b(int p, const Mat& m) {
    for (int i = 0; i < d; i++)
      for (int c = 0; c < d; c++) b(p, i, c) += m[i * d + c];
  }
  Mat x(int p) {
    Mat m = zeros(d);
    for (int i = 0; i < d; i++)
      for (int c = 0; c < d; c++) m[i * d + c] = b(p, i, c);
    return m;
  }
  bool run() { return solve(nu * d, d, A.data(), B.data()); }
};

// Standard Volterra start-up matrix for the rows p = 1..k of the Dyson
// equation with p(t) = i e(t), k(t,s) = i Sigma^R(t,s) (Eq. vdiff_start):
//   B_{p,l} = h^-1 D_{p,l} + delta_{pl} i e_p + i h s_{p,l} Sigma~^R_{p,l}.
Mat start_block(const HM& S, const Fn& eps, int p, int l) {
  const Grid& g = S.g;
  int d = g.d;
  const Weights& W = weights(g.k);
  Mat m = zeros(d);
  for (int i = 0; i < d; i++) m[i * d + i] += W.d(p, l) / g.h;
  if (p == l) {
    Mat e = ehat(eps, p, g.mu);
    for (int i = 0; i < d * d; i++) m[i] += I1 * e[i];
  }
  Mat s = Rt(S, p, l);
  for (int i = 0; i < d * d; i++) m[i] += I1 * g.h * W.s(p, l) * s[i];
  return m;
}

// Source of the lesser equation at row m, column n (Eq. dyson_langreth_les):
//   q_m = -i (C^<_2 + C^<_3)[Sigma, 1, G](m, n),
//   C^<_2 = int_0^{t_n} Sigma^<(t_m,t) G^A(t,t_n),
//   C^<_3 = -i int_0^beta Sigma^rceil(t_m,tau) G^lceil(tau,t_n)  (Eqs. cles2, cles3).
Mat les_source(int m, int n, const HM& G, const HM& S) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  Mat c2 = zeros(d), c3 = zeros(d);
  int jmax = n > k ? n : k;
  for (int j = 0; j <= jmax; j++) {
    Mat s = Lh(S, m, j), a = Adv(G, j, n);
    gemm_acc(c2.data(), s.data(), a.data(), d, g.h * W.w(n, j));
  }
  for (int j = 0; j <= ntau; j++) {
    Mat v = Vt(G, j, n);
    gemm_acc(c3.data(), S.T(m, j), v.data(), d, cd(0.0, -1.0) * g.htau() * W.w(ntau, j));
  }
  Mat q = zeros(d);
  for (int i = 0; i < d * d; i++) q[i] = -I1 * (c2[i] + c3[i]);
  return q;
}

// One step of the lesser column n at row m > k in the serial form (A):
//   [h^-1 a_0 + i e_m + i h w_{m,m} Sigma^R_{m,m}] L_{m,n}
//     = q_m - h^-1 sum_{l=1}^k a_l L_{m-l,n} - i h sum_{j<m} w_{m,j} Sigma^R_{m,j} L_{j,n}.
Mat les_step_A(int m, int n, const HM& G, const HM& S, const Fn& eps, bool* ok) {
  const Grid& g = G.g;
  int d = g.d, k = g.k;
  const Weights& W = weights(k);
  Mat rhs = les_source(m, n, G, S);
  for (int l = 1; l <= k; l++) {
    const cd* y = G.L(m - l, n);
    for (int i = 0; i < d * d; i++) rhs[i] -= W.bdf[l] / g.h * y[i];
  }
  for (int j = 0; j < m; j++) gemm_acc(rhs.data(), S.R(m, j), G.L(j, n), d, -I1 * g.h * W.w(m, j));
  Mat A = zeros(d);
  Mat e = ehat(eps, m, g.mu);
  for (int i = 0; i < d; i++) A[i * d + i] += W.bdf[0] / g.h;
  for (int i = 0; i < d * d; i++) A[i] += I1 * e[i] + I1 * g.h * W.w(m, m) * S.R(m, m)[i];
  return left_solve(A, rhs, d, ok);
}

// Start-up of the lesser column n over rows 1..k (Eq. vdiff_start with
// y_0 = G^<(0, t_n) = -[G^rceil(t_n, 0)]^dag, Eq. dyson_ini_les). Rows up to
// min(n, k) are stored.
bool les_column_start(int n, const HM& G, const HM& S, const Fn& eps) {
  const Grid& g = G.g;
  int d = g.d, k = g.k;
  Mat y0 = dag(G.T(n, 0), d);
  for (auto& v : y0) v = -v;
  set(G.L(0, n), y0);
  BlockSys sys(k, d);
  for (int p = 1; p <= k; p++) {
    for (int l = 1; l <= k; l++) sys.set_a(p - 1, l - 1, start_block(S, eps, p, l));
    Mat q = les_source(p, n, G, S);
    Mat b0 = start_block(S, eps, p, 0);
    gemm_acc(q.data(), b0.data(), y0.data(), d, -1.0);
    sys.add_b(p - 1, q);
  }
  bool ok = sys.run();
  for (int p = 1; p <= k && p <= n; p++) set(G.L(p, n), sys.x(p - 1));
  return ok;
}

// Retarded boundary rows R_{n, n-l}, l = 0..k, of slice n >= k from the
// conjugate start-up (Eq. MBCVSAMx_cc_start) with y(s) = G^R(t_n, t_n - s),
// p(s) = i e(t_n - s), k(s, s') = i Sigma^R(t_n - s, t_n - s'), y_0 = -i:
//   sum_l Y_l [h^-1 D_{p,l} + delta_{pl} i e_{n-p} + i h s_{p,l} Sigma~^R_{n-l,n-p}] = 0.
bool ret_boundary(int n, const HM& G, const HM& S, const Fn& eps) {
  const Grid& g = G.g;
  int d = g.d, k = g.k;
  const Weights& W = weights(k);
  auto C = [&](int l, int p) {
    Mat m = zeros(d);
    for (int i = 0; i < d; i++) m[i * d + i] += W.d(p, l) / g.h;
    if (p == l) {
      Mat e = ehat(eps, n - p, g.mu);
      for (int i = 0; i < d * d; i++) m[i] += I1 * e[i];
    }
    Mat s = Rt(S, n - l, n - p);
    for (int i = 0; i < d * d; i++) m[i] += I1 * g.h * W.s(p, l) * s[i];
    return m;
  };
  Mat Y0 = zeros(d);
  for (int i = 0; i < d; i++) Y0[i * d + i] = -I1;
  // Transpose to column form: sum_l C_{l,p}^T Y_l^T = -C_{0,p}^T Y_0^T.
  BlockSys sys(k, d);
  for (int p = 1; p <= k; p++) {
    for (int l = 1; l <= k; l++) {
      Mat c = C(l, p), ct = zeros(d);
      for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) ct[i * d + j] = c[j * d + i];
      sys.set_a(p - 1, l - 1, ct);
    }
    Mat r = zeros(d);
    Mat c0 = C(0, p);
    gemm_acc(r.data(), Y0.data(), c0.data(), d, -1.0);
    Mat rt = zeros(d);
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) rt[i * d + j] = r[j * d + i];
    sys.add_b(p - 1, rt);
  }
  bool ok = sys.run();
  set(G.R(n, n), Y0);
  for (int l = 1; l <= k; l++) {
    Mat xt = sys.x(l - 1), x = zeros(d);
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) x[i * d + j] = xt[j * d + i];
    set(G.R(n, n - l), x);
  }
  return ok;
}

}  // namespace

void free_mat(const Grid& g, const cd* eps, cd* out) {
  int d = g.d;
  Mat e(eps, eps + d * d);
  for (int i = 0; i < d; i++) e[i * d + i] -= g.mu;
  std::vector<double> x(d);
  Mat V = zeros(d);
  eigh(d, e.data(), x.data(), V.data());
  double xi = g.sig;
  for (int m = 0; m <= g.ntau; m++) {
    double tau = m * g.htau();
    // g(tau) = -exp(-x tau) / (1 - xi exp(-beta x)), 0 <= tau <= beta, the
    // free Matsubara function of Eq. dyson_langreth_m with Sigma = 0
    // (Reading: written with x = eps - mu and an overall minus sign, as the
    // convention C^M(tau) = -i C(-i tau, 0) requires).
    std::vector<double> f(d);
    for (int a = 0; a < d; a++) {
      double xa = x[a];
      if (xa >= 0 || xi > 0)
        f[a] = -std::exp(-xa * tau) / (1.0 - xi * std::exp(-g.beta * xa));
      else
        f[a] = -std::exp(xa * (g.beta - tau)) / (std::exp(g.beta * xa) - xi);
    }
    cd* o = out + (size_t)m * d * d;
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) {
        cd acc = 0.0;
        for (int a = 0; a < d; a++) acc += V[i * d + a] * f[a] * std::conj(V[j * d + a]);
        o[i * d + j] = acc;
      }
  }
}

bool dyson_mat(const HM& G, const HM& Sig, const cd* eps_m1) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, nt = g.ntau;
  const Weights& W = weights(k);
  double ht = g.htau(), xi = g.sig;
  size_t bs = (size_t)d * d;
  // g and K = [g * Sigma]^M
  std::vector<cd> gm((nt + 1) * bs), Km((nt + 1) * bs);
  free_mat(g, eps_m1, gm.data());
  HM gv{g, gm.data(), nullptr, nullptr, nullptr};
  for (int m = 0; m <= nt; m++) {
    Mat c = cm12(m, gv, Sig, nullptr);
    std::copy(c.begin(), c.end(), Km.begin() + m * bs);
  }
  auto K = [&](int m) { return Km.data() + m * bs; };
  // Dense system M_m - sum_l B_{m,l} M_l = g_m with B from Eqs. cm1, cm2.
  int N = (nt + 1) * d;
  std::vector<cd> A((size_t)N * N, 0.0), rhs((size_t)N * d);
  auto addB = [&](int m, int l, const cd* blk, double c) {
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) A[(size_t)(m * d + i) * N + l * d + j] -= c * blk[i * d + j];
  };
  for (int m = 0; m <= nt; m++) {
    if (m <= k) {
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) addB(m, l, K(j), ht * W.r(m, j, l));
    } else {
      for (int l = 0; l <= m; l++) addB(m, l, K(m - l), ht * W.w(m, l));
    }
    if (m >= nt - k) {
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) addB(m, nt - l, K(nt - j), ht * xi * W.r(nt - m, j, l));
    } else {
      for (int l = 0; l <= nt - m; l++) addB(m, m + l, K(nt - l), ht * xi * W.w(nt - m, l));
    }
  }
  for (int r = 0; r < N; r++) A[(size_t)r * N + r] += 1.0;
  for (int m = 0; m <= nt; m++)
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) rhs[(size_t)(m * d + i) * d + j] = gm[m * bs + i * d + j];
  bool ok = solve(N, d, A.data(), rhs.data());
  for (int m = 0; m <= nt; m++)
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) G.M(m)[i * d + j] = rhs[(size_t)(m * d + i) * d + j];
  return ok;
}

bool dyson_start(const HM& G, const HM& S, const Fn& eps) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  double h = g.h, xi = g.sig;
  bool ok = true;
  // Retarded, columns m = 0..k, rows p = m..k (Sec. "Start", first item):
  //   i h^-1 sum_l D_{p,l} y_l - e_p y_p - h sum_l I_{m,p,l} Sigma~^R_{p,l} y_l = 0,
  // y_m = -i, y_l = -[G^R_{m,l}]^dag for l < m.
  // Reading: the printed equation has +eps_n y_n; the sign follows from
  // Eq. dyson_langreth_r, i d_t G^R - e G^R - Sigma^R * G^R = 0.
  for (int m = 0; m <= k; m++) {
    Mat mi = zeros(d);
    for (int i = 0; i < d; i++) mi[i * d + i] = -I1;
    set(G.R(m, m), mi);
    if (m == k) break;
    std::vector<Mat> y(k + 1);
    for (int l = 0; l < m; l++) {
      y[l] = dag(G.R(m, l), d);
      for (auto& v : y[l]) v = -v;
    }
    y[m] = mi;
    auto Ablk = [&](int p, int l) {
      Mat a = zeros(d);
      for (int i = 0; i < d; i++) a[i * d + i] += I1 * W.d(p, l) / h;
      if (p == l) {
        Mat e = ehat(eps, p, g.mu);
        for (int i = 0; i < d * d; i++) a[i] -= e[i];
      }
      Mat s = Rt(S, p, l);
      for (int i = 0; i < d * d; i++) a[i] -= h * W.i(m, p, l) * s[i];
      return a;
    };
    int nu = k - m;
    BlockSys sys(nu, d);
    for (int p = m + 1; p <= k; p++) {
      for (int l = m + 1; l <= k; l++) sys.set_a(p - m - 1, l - m - 1, Ablk(p, l));
      Mat r = zeros(d);
      for (int l = 0; l <= m; l++) {
        Mat a = Ablk(p, l);
        gemm_acc(r.data(), a.data(), y[l].data(), d, -1.0);
      }
      sys.add_b(p - m - 1, r);
    }
    ok = sys.run() && ok;
    for (int p = m + 1; p <= k; p++) set(G.R(p, m), sys.x(p - m - 1));
  }
  // Left-mixing, each tau index m (Sec. "Start", second item): Eq. vdiff_start
  // with y_0 = i xi G^M(beta - tau_m) (Eq. dyson_ini_tv) and
  // q_p = -i (C^rceil_2 + C^rceil_3)[Sigma, 1, G](p, m).
#pragma omp parallel for schedule(static) reduction(&& : ok)
  for (int m = 0; m <= ntau; m++) {
    Mat y0 = scaled(G.M(ntau - m), d, I1 * xi);
    set(G.T(0, m), y0);
    BlockSys sys(k, d);
    for (int p = 1; p <= k; p++) {
      for (int l = 1; l <= k; l++) sys.set_a(p - 1, l - 1, start_block(S, eps, p, l));
      Mat q = ctv23(p, m, S, G, nullptr);
      for (auto& v : q) v *= -I1;
      Mat b0 = start_block(S, eps, p, 0);
      gemm_acc(q.data(), b0.data(), y0.data(), d, -1.0);
      sys.add_b(p - 1, q);
    }
    ok = sys.run() && ok;
    for (int p = 1; p <= k; p++) set(G.T(p, m), sys.x(p - 1));
  }
  // Lesser, columns n = 0..k (Sec. "Start", third item), after R and rceil.
  for (int n = 0; n <= k; n++) ok = les_column_start(n, G, S, eps) && ok;
  return ok;
}

bool dyson_timestep(int n, const HM& G, const HM& S, const Fn& eps, char variant) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  double h = g.h, ht = g.htau(), xi = g.sig;
  bool ok = true;
  if (n <= k) return false;
  Mat e = ehat(eps, n, g.mu);
  // Step matrix shared by every single step at t_n (Eq. MBCVSAMx_t):
  // M_R = h^-1 a_0 + i e_n + i h omega_0 Sigma^R_{n,n}.
  Mat MR = zeros(d);
  for (int i = 0; i < d; i++) MR[i * d + i] += W.bdf[0] / h;
  for (int i = 0; i < d * d; i++) MR[i] += I1 * e[i] + I1 * h * W.w(n, n) * S.R(n, n)[i];

  // ---- retarded row n
  ok = ret_boundary(n, G, S, eps) && ok;
  if (variant == 'B') {
    // (B): for each m < n-k one step of Eq. MBCVSAMx_t for y(s) = G^R(t_m+s, t_m),
    // p = i e(t_m+s), k(s,s') = i Sigma^R(t_m+s, t_m+s'), at s = t_n - t_m.
#pragma omp parallel for schedule(dynamic) reduction(&& : ok)
    for (int m = 0; m < n - k; m++) {
      int N = n - m;
      Mat rhs = zeros(d);
      for (int l = 1; l <= k; l++) {
        const cd* y = G.R(n - l, m);
        for (int i = 0; i < d * d; i++) rhs[i] -= W.bdf[l] / h * y[i];
      }
      for (int j = m; j < n; j++) gemm_acc(rhs.data(), S.R(n, j), G.R(j, m), d, -I1 * h * W.w(N, j - m));
      set(G.R(n, m), left_solve(MR, rhs, d, &ok));
    }
  } else {
    // (A): Eq. MBCVSAMx_cc_t for Y_l = G^R(t_n, t_{n-l}), l = k+1..n.
    for (int l = k + 1; l <= n; l++) {
      Mat rhs = zeros(d);
      for (int r = 1; r <= k; r++) {
        const cd* y = G.R(n, n - (l - r));
        for (int i = 0; i < d * d; i++) rhs[i] -= W.bdf[r] / h * y[i];
      }
      for (int j = 0; j < l; j++)
        gemm_acc(rhs.data(), G.R(n, n - j), S.R(n - j, n - l), d, -I1 * h * W.w(l, j));
      Mat A = zeros(d);
      Mat el = ehat(eps, n - l, g.mu);
      for (int i = 0; i < d; i++) A[i * d + i] += W.bdf[0] / h;
      for (int i = 0; i < d * d; i++) A[i] += I1 * el[i] + I1 * h * W.w(l, l) * S.R(n - l, n - l)[i];
      set(G.R(n, n - l), right_solve(A, rhs, d, &ok));
    }
  }

  // ---- left-mixing row n: Eq. MBCVSAMx_t per tau index (Sec. "Time stepping",
  // second item), q = -i (C^rceil_2 + C^rceil_3)[Sigma, 1, G](n, m).
#pragma omp parallel for schedule(static) reduction(&& : ok)
  for (int m = 0; m <= ntau; m++) {
    Mat rhs = ctv23(n, m, S, G, nullptr);
    for (auto& v : rhs) v *= -I1;
    for (int l = 1; l <= k; l++) {
      const cd* y = G.T(n - l, m);
      for (int i = 0; i < d * d; i++) rhs[i] -= W.bdf[l] / h * y[i];
    }
    for (int j = 0; j < n; j++) gemm_acc(rhs.data(), S.R(n, j), G.T(j, m), d, -I1 * h * W.w(n, j));
    set(G.T(n, m), left_solve(MR, rhs, d, &ok));
  }

  // ---- lesser column n
  if (variant == 'A' || n <= 2 * k) {
    // Reading: for k < n <= 2k the boundary rows n-k..n would overlap the
    // start-up rows 1..k, so the whole column is done in the serial form.
    ok = les_column_start(n, G, S, eps) && ok;
    for (int m = k + 1; m <= n; m++) set(G.L(m, n), les_step_A(m, n, G, S, eps, &ok));
    return ok;
  }
  // (B): rows m < n-k from one step of the conjugate equation (Eq. MBCVSAMx_cc_t)
  // for y(s) = G^<(t_m, s), p = -i e, k(s,s') = -i Sigma^A(s,s'),
  // q = i (C^<_1 + C^<_3)[G, 1, Sigma](m, n).
  // Reading: the printed conjugate lesser equation swaps the G^R Sigma^< and
  // G^< Sigma^A terms; this follows the Langreth rule of Eq. conv_les.
  Mat ML = dag(MR, d);  // h^-1 a_0 - i e_n - i h omega_0 (Sigma^R_{n,n})^dag
#pragma omp parallel for schedule(dynamic) reduction(&& : ok)
  for (int m = 0; m < n - k; m++) {
    Mat c1 = zeros(d), c3 = zeros(d);
    if (m > k) {
      for (int j = 0; j <= m; j++) gemm_acc(c1.data(), G.R(m, j), S.L(j, n), d, h * W.w(m, j));
    } else {
      for (int j = 0; j <= k; j++) {
        Mat r = Rt(G, m, j);
        gemm_acc(c1.data(), r.data(), S.L(j, n), d, h * W.s(m, j));
      }
    }
    for (int j = 0; j <= ntau; j++) {
      Mat v = Vt(S, j, n);
      gemm_acc(c3.data(), G.T(m, j), v.data(), d, cd(0.0, -1.0) * ht * W.w(ntau, j));
    }
    Mat rhs = zeros(d);
    for (int i = 0; i < d * d; i++) rhs[i] = I1 * (c1[i] + c3[i]);
    for (int l = 1; l <= k; l++) {
      const cd* y = G.L(m, n - l);
      for (int i = 0; i < d * d; i++) rhs[i] -= W.bdf[l] / h * y[i];
    }
    for (int l = 0; l < n; l++) {
      Mat y = Lh(G, m, l), sa = dag(S.R(n, l), d);
      gemm_acc(rhs.data(), y.data(), sa.data(), d, I1 * h * W.w(n, l));
    }
    set(G.L(m, n), right_solve(ML, rhs, d, &ok));
  }
  // Boundary rows m = n-k..n by the serial steps (A), in order.
  for (int m = n - k; m <= n; m++) set(G.L(m, n), les_step_A(m, n, G, S, eps, &ok));
  (void)xi;
  return ok;
}

}  // namespace oracle
