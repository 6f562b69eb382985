// Internal definitions of the HIP Dyson time stepper (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cntr.h"

namespace cntr {

// ------------------------------------------------------------ complex math
struct cplx {
  double x, y;
};
__host__ __device__ inline cplx mk(double a, double b) { return cplx{a, b}; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return cplx{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return cplx{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cplx operator-(cplx a) { return cplx{-a.x, -a.y}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
  return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return cplx{s * a.x, s * a.y}; }
__host__ __device__ inline cplx conj(cplx a) { return cplx{a.x, -a.y}; }
__host__ __device__ inline cplx mul_i(cplx a) { return cplx{-a.y, a.x}; }  // i * a
__host__ __device__ inline double abs2(cplx a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return cplx{(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  }
  double r = b.x / b.y, den = b.x * r + b.y;
  return cplx{(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}
// acc += a * b  (4 real FMAs)
__host__ __device__ inline void cfma(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += a * conj(b)
__host__ __device__ inline void cfma_cb(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// ------------------------------------------------------------ weights
constexpr int KMAX = 5;
constexpr int KP = KMAX + 1;
// Quadrature / differentiation tables for one order k (generated on the
// host by weights.cpp, placed in constant memory).
struct KW {
  int k;
  double a[KP];          // BDF a_l
  double omega[KP];      // Gregory end weights
  double s[KP][KP];      // starting weights s_{n,j} = I_{0,n,j}
  double D[KP][KP];      // polynomial differentiation D_{p,l}
  double I[KP][KP][KP];  // polynomial integration I_{m,n,l}
  double R[KP][KP][KP];  // boundary convolution R_{m;r,s}
  double ext[KP];        // one-step polynomial extrapolation, weight of y_{n-l}
};
void make_weights(int k, KW* out);  // host

extern __constant__ KW c_kw[KMAX + 1];

// Gregory weight w_{n,j}^{(k)}, 0 <= j <= max(n,k).
__device__ inline double greg(const KW& W, int n, int j) {
  int k = W.k;
  if (n <= k) return W.s[n][j];
  bool left = j <= k, right = n - j <= k;
  if (left && right) return W.omega[j] + W.omega[n - j] - 1.0;
  if (left) return W.omega[j];
  if (right) return W.omega[n - j];
  return 1.0;
}

// ------------------------------------------------------------ problem
// One contour problem as seen by the kernels. Pointers are device pointers
// in the canonical layout (see cntr.h).
struct Prob {
  int nt, ntau, d, sig, k;
  double beta, h, mu, htau;
  cplx *Gmat, *Gret, *Gles, *Gtv;
  cplx *Smat, *Sret, *Sles, *Stv;
  const cplx* eps;  // (nt+2) d*d, index n+1
  // optional per-problem inputs of the self-energy / convolution calls
  const double* U;   // (nt+2), index n+1
  const cplx* eps0;  // (nt+2) d*d
  cplx* eps_mf;      // (nt+2) d*d or null
  const cplx* f;     // (nt+2) d*d or null (convolution weight function)
  // Dyson equation in integral form, (1 + F) * G = Q: the S pointers hold
  // F^M, F^R, F^rceil and Fcc^< (Fcc = F^ddagger); the start-up also reads
  // F^< (rows m > j come from Fcc^<) and Fcc^R (F^R continued to t < t')
  const cplx *Qmat, *Qret, *Qles, *Qtv;
  const cplx *Fles, *Fcret;
  // Holstein pieces: a per-problem real series (nt+2, index n+1; entry 0 the
  // Matsubara branch) and a per-problem parameter
  double* aux;
  double par;
};

__host__ __device__ inline size_t tri(int n) { return (size_t)n * (n + 1) / 2; }

// block pointers (d*d complex each)
__device__ inline cplx* blk_R(cplx* base, int n, int j, int d) { return base + (tri(n) + j) * d * d; }
__device__ inline cplx* blk_L(cplx* base, int j, int n, int d) { return base + (tri(n) + j) * d * d; }
__device__ inline cplx* blk_T(cplx* base, int n, int m, int ntau, int d) {
  return base + ((size_t)n * (ntau + 1) + m) * d * d;
}

// status word written by kernels on failure (singular pivot)
struct DevStatus {
  int code;
  int where;
};

}  // namespace cntr
