// Quadrature and differentiation weights in exact rational arithmetic,
// rounded once to double. Test infrastructure only (see oracle.hpp).
//
// Sec. "Basic integration and differentiation rules":
//   P^{(k)} = M^{-1}, M_{ja} = j^a                       (Eq. integrator_P)
//   D_{m,l} = sum_{a>=1} P_{al} a m^{a-1}                 (Eq. integrator_D)
//   I_{m,n,l} = sum_a P_{al} (n^{a+1} - m^{a+1})/(a+1)    (Eq. integrator_I)
//   a_l = -D_{0,l}                                        (BDF, Tab. integrator_bd)
//   s_{n,j} = I_{0,n,j}  (starting weights, n <= k)       (Eq. integrator_greg)
//   R_{m;r,s} = sum_{a,b} P_{ar} P_{bs} int_0^m (m-x)^a x^b dx   (Eq. integrator_R)
// Gregory weights for n > k. Reading: the paper's verbal definition (BDF
// applied to dI/dt = y) does not reproduce its own Tab. gregory, while the
// classical Gregory rule does: the trapezoidal rule plus k end corrections
// built from forward differences at t=0 and backward differences at t=nh,
// with the Gregory coefficients gamma_r (r = 1..k) read off the series of
// z / ln(1+z). This reproduces every printed entry and has interior
// weights exactly 1, as the paper states.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <map>
#include <mutex>

#include "oracle.hpp"

namespace oracle {
namespace {

using i128 = __int128;

i128 gcd128(i128 a, i128 b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b != 0) {
    i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct Rat {
  i128 n = 0, d = 1;
  Rat() {}
  Rat(i128 a) : n(a), d(1) {}
  Rat(i128 a, i128 b) : n(a), d(b) { norm(); }
  void norm() {
    if (d < 0) {
      n = -n;
      d = -d;
    }
    i128 g = gcd128(n, d);
    if (g > 1) {
      n /= g;
      d /= g;
    }
  }
  double to_double() const { return (double)((long double)n / (long double)d); }
};
Rat operator+(Rat a, Rat b) { return Rat(a.n * b.d + b.n * a.d, a.d * b.d); }
Rat operator-(Rat a, Rat b) { return Rat(a.n * b.d - b.n * a.d, a.d * b.d); }
Rat operator*(Rat a, Rat b) { return Rat(a.n * b.n, a.d * b.d); }
Rat operator/(Rat a, Rat b) { return Rat(a.n * b.d, a.d * b.n); }
Rat operator-(Rat a) { return Rat(-a.n, a.d); }

i128 ipow(i128 b, int e) {
  i128 r = 1;
  for (int i = 0; i < e; i++) r *= b;
  return r;
}
i128 fact(int n) {
  i128 r = 1;
  for (int i = 2; i <= n; i++) r *= i;
  return r;
}
i128 binom(int n, int r) { return fact(n) / (fact(r) * fact(n - r)); }

// Inverse of the Vandermonde matrix M_{ja} = j^a, j,a = 0..k (Gauss-Jordan).
std::vector<Rat> interp_matrix(int k) {
  int n = k + 1;
  std::vector<Rat> A(n * n), X(n * n);
  for (int j = 0; j < n; j++)
    for (int a = 0; a < n; a++) {
      A[j * n + a] = Rat(ipow(j, a));
      X[j * n + a] = Rat(j == a ? 1 : 0);
    }
  for (int c = 0; c < n; c++) {
    int p = c;
    while (A[p * n + c].n == 0) p++;
    if (p != c)
      for (int q = 0; q < n; q++) {
        std::swap(A[p * n + q], A[c * n + q]);
        std::swap(X[p * n + q], X[c * n + q]);
      }
    Rat piv = A[c * n + c];
    for (int q = 0; q < n; q++) {
      A[c * n + q] = A[c * n + q] / piv;
      X[c * n + q] = X[c * n + q] / piv;
    }
    for (int r = 0; r < n; r++) {
      if (r == c || A[r * n + c].n == 0) continue;
      Rat f = A[r * n + c];
      for (int q = 0; q < n; q++) {
        A[r * n + q] = A[r * n + q] - f * A[c * n + q];
        X[r * n + q] = X[r * n + q] - f * X[c * n + q];
      }
    }
  }
  return X;  // X = M^{-1}, indexed [a][l]
}

// Gregory coefficients gamma_r, r = 1..kmax: coefficients of the series
// 1/(ln(1+z)/z) = sum_n b_n z^n, gamma_r = |b_{r+1}|.
std::vector<Rat> gregory_gamma(int kmax) {
  int N = kmax + 2;
  std::vector<Rat> c(N + 1), b(N + 1);
  for (int i = 0; i <= N; i++) c[i] = Rat((i % 2 ? -1 : 1), i + 1);  // ln(1+z)/z
  b[0] = Rat(1);
  for (int n = 1; n <= N; n++) {
    Rat acc(0);
    for (int i = 1; i <= n; i++) acc = acc + c[i] * b[n - i];
    b[n] = -acc;  // c[0] = 1
  }
  std::vector<Rat> g(kmax + 1);
  for (int r = 1; r <= kmax; r++) {
    Rat v = b[r + 1];
    if (v.n < 0) v = -v;
    g[r] = v;
  }
  return g;
}

struct RatWeights {
  int k;
  std::vector<Rat> P, D, I, a, s, omega, R;
};

Rat greg_rat(const RatWeights& W, int n, int j) {
  int k = W.k;
  if (n <= k) return W.s[n * (k + 1) + j];
  if (j < 0 || j > n) return Rat(0);
  // trapezoid
  Rat w = (j == 0 || j == n) ? Rat(1, 2) : Rat(1);
  std::vector<Rat> g = gregory_gamma(k);
  for (int r = 1; r <= k; r++)
    for (int i = 0; i <= r; i++) {
      // -gamma_r (-1)^i C(r,i) at j = i (forward differences at 0) and at
      // j = n - i (backward differences at n).
      Rat t = g[r] * Rat((i % 2 ? -1 : 1) * binom(r, i));
      if (j == i) w = w - t;
      if (j == n - i) w = w - t;
    }
  return w;
}

RatWeights build_rat(int k) {
  RatWeights W;
  W.k = k;
  int n = k + 1;
  W.P = interp_matrix(k);
  W.D.assign(n * n, Rat(0));
  W.I.assign(n * n * n, Rat(0));
  W.a.assign(n, Rat(0));
  W.s.assign(n * n, Rat(0));
  W.R.assign(n * n * n, Rat(0));
  for (int m = 0; m < n; m++)
    for (int l = 0; l < n; l++) {
      Rat acc(0);
      for (int a = 1; a <= k; a++) acc = acc + W.P[a * n + l] * Rat(a * ipow(m, a - 1));
      W.D[m * n + l] = acc;
    }
  for (int m = 0; m < n; m++)
    for (int nn = 0; nn < n; nn++)
      for (int l = 0; l < n; l++) {
        Rat acc(0);
        for (int a = 0; a <= k; a++)
          acc = acc + W.P[a * n + l] * Rat(ipow(nn, a + 1) - ipow(m, a + 1), a + 1);
        W.I[(m * n + nn) * n + l] = acc;
      }
  for (int l = 0; l < n; l++) W.a[l] = -W.D[0 * n + l];
  for (int nn = 0; nn < n; nn++)
    for (int j = 0; j < n; j++) W.s[nn * n + j] = W.I[(0 * n + nn) * n + j];
  for (int m = 0; m < n; m++)
    for (int r = 0; r < n; r++)
      for (int s = 0; s < n; s++) {
        Rat acc(0);
        for (int a = 0; a <= k; a++)
          for (int b = 0; b <= k; b++) {
            // int_0^m (m-x)^a x^b dx = m^{a+b+1} a! b! / (a+b+1)!  (Beta function)
            Rat beta(ipow(m, a + b + 1) * fact(a) * fact(b), fact(a + b + 1));
            acc = acc + W.P[a * n + r] * W.P[b * n + s] * beta;
          }
        W.R[(m * n + r) * n + s] = acc;
      }
  W.omega.assign(n, Rat(0));
  for (int j = 0; j < n; j++) W.omega[j] = greg_rat(W, 2 * k + 2, j);
  return W;
}

std::mutex g_mu;
std::map<int, RatWeights*> g_rat;
std::map<int, Weights*> g_w;

const RatWeights& rat(int k) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_rat.find(k);
  if (it != g_rat.end()) return *it->second;
  RatWeights* W = new RatWeights(build_rat(k));
  g_rat[k] = W;
  return *W;
}

std::vector<double> to_d(const std::vector<Rat>& v) {
  std::vector<double> r(v.size());
  for (size_t i = 0; i < v.size(); i++) r[i] = v[i].to_double();
  return r;
}

}  // namespace

void gregory_rational(int k, int n, int j, int64_t* num, int64_t* den) {
  Rat r = greg_rat(rat(k), n, j);
  *num = (int64_t)r.n;
  *den = (int64_t)r.d;
}

double Weights::w(int n, int j) const {
  if (n <= k) return s(n, j);
  if (j < 0 || j > n) return 0.0;
  // Rows n <= 2k overlap both end corrections: tabulated from the rationals.
  if (n <= 2 * k) return wlow[(size_t)n * (2 * k + 1) + j];
  // From n = 2k+1 on the two ends are disjoint: omega at each end, 1 inside.
  if (j <= k) return omega[j];
  if (n - j <= k) return omega[n - j];
  return 1.0;
}

const Weights& weights(int k) {
  if (k < 0 || k > 6) {
    fprintf(stderr, "oracle: order k=%d out of range\n", k);
    abort();
  }
  const RatWeights& W = rat(k);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_w.find(k);
  if (it != g_w.end()) return *it->second;
  Weights* w = new Weights();
  w->k = k;
  w->P = to_d(W.P);
  w->D = to_d(W.D);
  w->Iw = to_d(W.I);
  w->bdf = to_d(W.a);
  w->start = to_d(W.s);
  w->omega = to_d(W.omega);
  w->R = to_d(W.R);
  w->wlow.assign((size_t)(2 * k + 1) * (2 * k + 1), 0.0);
  for (int n = 0; n <= 2 * k; n++)
    for (int j = 0; j <= std::max(n, k); j++)
      w->wlow[(size_t)n * (2 * k + 1) + j] = greg_rat(W, n, j).to_double();
  g_w[k] = w;
  return *w;
}

}  // namespace oracle
