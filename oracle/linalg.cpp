// Small dense linear algebra for the oracle: block products, Gaussian
// elimination with partial pivoting, hermitian Jacobi eigen-decomposition.
// Test infrastructure only (see oracle.hpp).
#include <cmath>

#include "oracle.hpp"

namespace oracle {

Mat zeros(int d) { return Mat((size_t)d * d, cd(0.0, 0.0)); }

Mat eye(int d) {
  Mat A = zeros(d);
  for (int i = 0; i < d; i++) A[i * d + i] = 1.0;
  return A;
}

Mat dag(const cd* A, int d) {
  Mat B = zeros(d);
  for (int i = 0; i < d; i++)
    for (int j = 0; j < d; j++) B[i * d + j] = std::conj(A[j * d + i]);
  return B;
}

Mat dag(const Mat& A, int d) { return dag(A.data(), d); }

void gemm_acc(cd* C, const cd* A, const cd* B, int d, cd alpha) {
  for (int i = 0; i < d; i++)
    for (int j = 0; j < d; j++) {
      cd acc = 0.0;
      for (int l = 0; l < d; l++) acc += A[i * d + l] * B[l * d + j];
      C[i * d + j] += alpha * acc;
    }
}

bool solve(int n, int nrhs, cd* A, cd* B) {
  for (int c = 0; c < n; c++) {
    int p = c;
    double best = std::abs(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; r++) {
      double v = std::abs(A[(size_t)r * n + c]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    if (best == 0.0) return false;
    if (p != c) {
      for (int q = 0; q < n; q++) std::swap(A[(size_t)p * n + q], A[(size_t)c * n + q]);
      for (int q = 0; q < nrhs; q++) std::swap(B[(size_t)p * nrhs + q], B[(size_t)c * nrhs + q]);
    }
    cd piv = A[(size_t)c * n + c];
#pragma omp parallel for schedule(static) if (n > 256)
    for (int r = c + 1; r < n; r++) {
      cd f = A[(size_t)r * n + c] / piv;
      if (f == cd(0.0, 0.0)) continue;
      for (int q = c; q < n; q++) A[(size_t)r * n + q] -= f * A[(size_t)c * n + q];
      for (int q = 0; q < nrhs; q++) B[(size_t)r * nrhs + q] -= f * B[(size_t)c * nrhs + q];
    }
  }
  for (int c = n - 1; c >= 0; c--) {
    for (int q = 0; q < nrhs; q++) {
      cd acc = B[(size_t)c * nrhs + q];
      for (int l = c + 1; l < n; l++) acc -= A[(size_t)c * n + l] * B[(size_t)l * nrhs + q];
      B[(size_t)c * nrhs + q] = acc / A[(size_t)c * n + c];
    }
  }
  return true;
}

void eigh(int d, const cd* A0, double* w, cd* V) {
  Mat A(A0, A0 + (size_t)d * d);
  for (int i = 0; i < d * d; i++) V[i] = 0.0;
  for (int i = 0; i < d; i++) V[i * d + i] = 1.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) {
        if (i != j) off += std::norm(A[i * d + j]);
        else diag += std::norm(A[i * d + j]);
      }
    if (off <= 1e-32 * (diag + off) || off == 0.0) break;
    for (int p = 0; p < d; p++)
      for (int q = p + 1; q < d; q++) {
        cd apq = A[p * d + q];
        double g = std::abs(apq);
        if (g == 0.0) continue;
        cd e = apq / g;
        double tau = (A[q * d + q].real() - A[p * d + p].real()) / (2.0 * g);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // J = [[c, s e], [-s conj(e), c]] on rows/columns p, q; A <- J^dag A J.
        for (int i = 0; i < d; i++) {
          cd aip = A[i * d + p], aiq = A[i * d + q];
          A[i * d + p] = c * aip - s * std::conj(e) * aiq;
          A[i * d + q] = s * e * aip + c * aiq;
        }
        for (int j = 0; j < d; j++) {
          cd apj = A[p * d + j], aqj = A[q * d + j];
          A[p * d + j] = c * apj - s * e * aqj;
          A[q * d + j] = s * std::conj(e) * apj + c * aqj;
        }
        for (int i = 0; i < d; i++) {
          cd vip = V[i * d + p], viq = V[i * d + q];
          V[i * d + p] = c * vip - s * std::conj(e) * viq;
          V[i * d + q] = s * e * vip + c * viq;
        }
      }
  }
  for (int i = 0; i < d; i++) w[i] = A[i * d + i].real();
}

}  // namespace oracle
