// Host-side generation of the quadrature and differentiation tables used by
// the kernels. Computed in long double, rounded once to double.
//
// Definitions (Sec. "Basic integration and differentiation rules"):
//   P = M^{-1} with M_{ja} = j^a (Eq. integrator_P), D (Eq. integrator_D),
//   I (Eq. integrator_I), s_{n,j} = I_{0,n,j}, BDF a_l = -D_{0,l}
//   (Eq. integrator_bd), R (Eq. integrator_R).
// Gregory end weights (Eq. integrator_greg, Tab. gregory): the trapezoidal
// rule plus an end correction c_0..c_k on the k+1 points at each end. The
// corrections cancel the end terms of the Euler-Maclaurin expansion for every
// polynomial of degree <= k, which for the left end reads
//   sum_i c_i i^q = B_{q+1} / (q+1)  (q odd),   0  (q even),   q = 0..k,
// a (k+1) x (k+1) Vandermonde system (B_j: Bernoulli numbers). The right end
// mirrors it; where both ends overlap (k < n <= 2k) the corrections add.
#include <cmath>
#include <cstring>

#include "cntr_internal.h"

namespace cntr {

namespace {

typedef long double ld;

// Solve A x = b (n x n, row-major) by Gaussian elimination with pivoting.
void gauss(int n, ld* A, ld* b) {
  for (int c = 0; c < n; c++) {
    int p = c;
    for (int r = c + 1; r < n; r++)
      if (fabsl(A[r * n + c]) > fabsl(A[p * n + c])) p = r;
    if (p != c) {
      for (int q = 0; q < n; q++) {
        ld t = A[p * n + q];
        A[p * n + q] = A[c * n + q];
        A[c * n + q] = t;
      }
      ld t = b[p];
      b[p] = b[c];
      b[c] = t;
    }
    for (int r = c + 1; r < n; r++) {
      ld f = A[r * n + c] / A[c * n + c];
      for (int q = c; q < n; q++) A[r * n + q] -= f * A[c * n + q];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; c--) {
    ld acc = b[c];
    for (int q = c + 1; q < n; q++) acc -= A[c * n + q] * b[q];
    b[c] = acc / A[c * n + c];
  }
}

ld ipow(ld x, int e) {
  ld r = 1;
  for (int i = 0; i < e; i++) r *= x;
  return r;
}

ld factl(int n) {
  ld r = 1;
  for (int i = 2; i <= n; i++) r *= i;
  return r;
}

}  // namespace

void make_weights(int k, KW* W) {
  std::memset(W, 0, sizeof(KW));
  W->k = k;
  int n1 = k + 1;
  // P = inverse Vandermonde, column by column.
  ld P[KP][KP];
  for (int l = 0; l < n1; l++) {
    ld A[KP * KP], b[KP];
    for (int j = 0; j < n1; j++) {
      for (int a = 0; a < n1; a++) A[j * n1 + a] = ipow(j, a);
      b[j] = (j == l) ? 1 : 0;
    }
    gauss(n1, A, b);
    for (int a = 0; a < n1; a++) P[a][l] = b[a];
  }
  for (int p = 0; p < n1; p++)
    for (int l = 0; l < n1; l++) {
      ld acc = 0;
      for (int a = 1; a <= k; a++) acc += P[a][l] * a * ipow(p, a - 1);
      W->D[p][l] = (double)acc;
    }
  for (int m = 0; m < n1; m++)
    for (int n = 0; n < n1; n++)
      for (int l = 0; l < n1; l++) {
        ld acc = 0;
        for (int a = 0; a <= k; a++) acc += P[a][l] * (ipow(n, a + 1) - ipow(m, a + 1)) / (a + 1);
        W->I[m][n][l] = (double)acc;
        if (m == 0) W->s[n][l] = (double)acc;
      }
  for (int l = 0; l < n1; l++) {
    ld acc = 0;
    for (int a = 1; a <= k; a++) acc += P[a][l] * a * ipow(0, a - 1);
    W->a[l] = (double)(-acc);
  }
  for (int m = 0; m < n1; m++)
    for (int r = 0; r < n1; r++)
      for (int s = 0; s < n1; s++) {
        ld acc = 0;
        for (int a = 0; a <= k; a++)
          for (int b = 0; b <= k; b++)
            acc += P[a][r] * P[b][s] * ipow(m, a + b + 1) * factl(a) * factl(b) / factl(a + b + 1);
        W->R[m][r][s] = (double)acc;
      }
  // Bernoulli numbers B_0..B_{k+1}: sum_{j=0}^{m} C(m+1, j) B_j = 0.
  ld B[KP + 2];
  B[0] = 1;
  for (int m = 1; m <= k + 1; m++) {
    ld acc = 0;
    for (int j = 0; j < m; j++) acc += factl(m + 1) / (factl(j) * factl(m + 1 - j)) * B[j];
    B[m] = -acc / (m + 1);
  }
  {
    ld A[KP * KP], b[KP];
    for (int q = 0; q < n1; q++) {
      for (int i = 0; i < n1; i++) A[q * n1 + i] = ipow(i, q);
      b[q] = (q % 2 == 1) ? B[q + 1] / (q + 1) : 0;
    }
    gauss(n1, A, b);
    for (int i = 0; i < n1; i++) W->omega[i] = (double)((i == 0 ? 0.5L : 1.0L) + b[i]);
  }
  // one-step extrapolation: Lagrange basis on nodes 0..k evaluated at k+1;
  // node i carries y_{n-k+i}, so y_{n-l} sits at node k-l.
  for (int l = 0; l < n1; l++) {
    int i = k - l;
    ld acc = 1;
    for (int j = 0; j < n1; j++)
      if (j != i) acc *= (ld)(k + 1 - j) / (ld)(i - j);
    W->ext[l] = (double)acc;
  }
}

}  // namespace cntr
