// Matsubara Dyson equation in integral form (Sec. "Matsubara",
// Eq. Gmat_dyson_integ): G = g + [K * G]^M with K = [g * Sigma]^M. The
// discrete operator of Eqs. cm1/cm2 is assembled as a dense
// (ntau+1)d x (ntau+1)d matrix and solved on the device: an explicit inverse
// by Gauss-Jordan elimination with partial pivoting, then residual
// refinement x <- x + A^-1 (g - A x). Inside a self-consistency loop the
// inverse of an earlier iterate serves as the preconditioner and is only
// rebuilt when the refinement stops contracting.
#include "launch.h"

namespace cntr {

constexpr int NT3 = 256;

// ------------------------------------------------------------ free g^M
// Cyclic Jacobi rotations on the hermitian d x d matrix A (destroyed):
// A = V diag(x) V^dag, V unitary (one thread).
__host__ __device__ inline void herm_jacobi(int d, cplx* A, cplx* V, double* x) {
  for (int e = 0; e < d * d; e++) V[e] = (e / d == e % d) ? mk(1, 0) : mk(0, 0);
  for (int sweep = 0; sweep < 60; sweep++) {
    double off = 0, tot = 0;
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) {
        double v = abs2(A[i * d + j]);
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < d; p++)
      for (int q = p + 1; q < d; q++) {
        cplx apq = A[p * d + q];
        double gabs = sqrt(abs2(apq));
        if (gabs == 0) continue;
        cplx ph = mk(apq.x / gabs, apq.y / gabs);
        double th = (A[q * d + q].x - A[p * d + p].x) / (2 * gabs);
        double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1 + th * th));
        double cs = 1 / sqrt(1 + t * t), sn = t * cs;
        for (int i = 0; i < d; i++) {
          cplx aip = A[i * d + p], aiq = A[i * d + q];
          A[i * d + p] = cs * aip - sn * (conj(ph) * aiq);
          A[i * d + q] = sn * (ph * aip) + cs * aiq;
        }
        for (int j = 0; j < d; j++) {
          cplx apj = A[p * d + j], aqj = A[q * d + j];
          A[p * d + j] = cs * apj - sn * (ph * aqj);
          A[q * d + j] = sn * (conj(ph) * apj) + cs * aqj;
        }
        for (int i = 0; i < d; i++) {
          cplx vip = V[i * d + p], viq = V[i * d + q];
          V[i * d + p] = cs * vip - sn * (conj(ph) * viq);
          V[i * d + q] = sn * (ph * vip) + cs * viq;
        }
      }
  }
  for (int i = 0; i < d; i++) x[i] = A[i * d + i].x;
}

// Cyclic Jacobi rotations on the hermitian d x d matrix A in LDS (destroyed):
// A = V diag(x) V^dag, one wave, the d rows / columns of every rotation
// updated by d lanes at once (the rotation sequence of a one-thread sweep).
__device__ inline void wave_jacobi(int d, cplx* A, cplx* V, double* x, int lane) {
  int dd = d * d;
  if (lane < dd) V[lane] = (lane / d == lane % d) ? mk(1, 0) : mk(0, 0);
  wave_sync();
  for (int sweep = 0; sweep < 60; sweep++) {
    double v = lane < dd ? abs2(A[lane]) : 0.0;
    double off = (lane < dd && lane / d != lane % d) ? v : 0.0;
    for (int o = 32; o >= 1; o >>= 1) {
      v += __shfl_xor(v, o);
      off += __shfl_xor(off, o);
    }
    if (off <= 1e-32 * v) break;
    for (int p = 0; p < d; p++)
      for (int q = p + 1; q < d; q++) {
        cplx apq = A[p * d + q];
        double gabs = sqrt(abs2(apq));
        if (gabs == 0) continue;
        cplx ph = mk(apq.x / gabs, apq.y / gabs);
        double th = (A[q * d + q].x - A[p * d + p].x) / (2 * gabs);
        double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1 + th * th));
        double cs = 1 / sqrt(1 + t * t), sn = t * cs;
        wave_sync();
        if (lane < d) {
          int i = lane;
          cplx aip = A[i * d + p], aiq = A[i * d + q];
          A[i * d + p] = cs * aip - sn * (conj(ph) * aiq);
          A[i * d + q] = sn * (ph * aip) + cs * aiq;
        }
        wave_sync();
        if (lane < d) {
          int j = lane;
          cplx apj = A[p * d + j], aqj = A[q * d + j];
          A[p * d + j] = cs * apj - sn * (ph * aqj);
          A[q * d + j] = sn * (conj(ph) * apj) + cs * aqj;
        } else if (lane >= 32 && lane < 32 + d) {
          int i = lane - 32;
          cplx vip = V[i * d + p], viq = V[i * d + q];
          V[i * d + p] = cs * vip - sn * (conj(ph) * viq);
          V[i * d + q] = sn * (ph * vip) + cs * viq;
        }
        wave_sync();
      }
  }
  if (lane < d) x[lane] = A[lane * d + lane].x;
  wave_sync();
}

// g(tau) = -V diag( e^{-x tau} / (1 - xi e^{-beta x}) ) V^dag for
// eps_{-1} - mu = V diag(x) V^dag, evaluated in the overflow-free form.
__global__ __launch_bounds__(NT3) void k_free_mat(Prob P, cplx* g) {
  __shared__ cplx A[64], V[64];
  __shared__ double x[8];
  int d = P.d, dd = d * d, tid = threadIdx.x;
  if (tid < 64) {
    if (tid < dd) {
      A[tid] = gld(P.eps + tid);
      if (tid / d == tid % d) A[tid].x -= P.mu;
    }
    wave_sync();
    wave_jacobi(d, A, V, x, tid);
  }
  __syncthreads();
  double xi = P.sig, beta = P.beta;
  for (int idx = tid; idx < (P.ntau + 1) * dd; idx += NT3) {
    int m = idx / dd, e = idx % dd, a = e / d, c = e % d;
    double tau = m * P.htau;
    cplx acc = mk(0, 0);
    for (int al = 0; al < d; al++) {
      double xa = x[al], f;
      if (xa >= 0 || xi > 0) f = -exp(-xa * tau) / (1 - xi * exp(-beta * xa));
      else f = -exp(xa * (beta - tau)) / (exp(beta * xa) - xi);
      acc = acc + f * (V[a * d + al] * conj(V[c * d + al]));
    }
    g[idx] = acc;
  }
}

hipError_t launch_free_mat(const Prob& P, cplx* g, hipStream_t s) {
  k_free_mat<<<1, NT3, 0, s>>>(P, g);
  return hipGetLastError();
}

// ------------------------------------------------------ dense operator
// A = 1 + sgn B with B_{m,l} the coefficient of G^M_l in [K * G]^M(m)
// (Eqs. cm1, cm2 with f = 1).
__global__ __launch_bounds__(NT3) void k_mat_build(Prob P, const cplx* K, cplx* Amat, double sgn) {
  int d = P.d, dd = d * d, nt = P.ntau, k = P.k;
  long N = (long)(nt + 1) * d;
  long idx = (long)blockIdx.x * NT3 + threadIdx.x;
  if (idx >= N * N) return;
  long row = idx / N, col = idx % N;
  int m = row / d, a = row % d, l = col / d, b = col % d;
  const KW& W = c_kw[k];
  double ht = P.htau, xi = P.sig;
  cplx v = mk(0, 0);
  if (m <= k) {
    if (l <= k)
      for (int j = 0; j <= k; j++) v = v + (ht * W.R[m][j][l]) * K[(size_t)j * dd + a * d + b];
  } else if (l <= m) {
    v = v + (ht * greg(W, m, l)) * K[(size_t)(m - l) * dd + a * d + b];
  }
  if (m >= nt - k) {
    if (l >= nt - k) {
      int ll = nt - l;
      for (int j = 0; j <= k; j++) v = v + (ht * xi * W.R[nt - m][j][ll]) * K[(size_t)(nt - j) * dd + a * d + b];
    }
  } else if (l >= m) {
    v = v + (ht * xi * greg(W, nt - m, l - m)) * K[(size_t)(nt - (l - m)) * dd + a * d + b];
  }
  v = sgn * v;
  if (row == col) v.x += 1.0;
  Amat[idx] = v;
}

hipError_t launch_mat_build(const Prob& P, const cplx* K, cplx* Amat, hipStream_t s, double sgn) {
  long N = (long)(P.ntau + 1) * P.d;
  long tot = N * N;
  k_mat_build<<<(unsigned)((tot + NT3 - 1) / NT3), NT3, 0, s>>>(P, K, Amat, sgn);
  return hipGetLastError();
}

// ------------------------------------------------- Gauss-Jordan inverse
constexpr int NGJ = 1024;

// pivot search for column c, row interchange, pivot row and column copies
__global__ __launch_bounds__(NGJ) void k_gj_pivot(int N, int c, cplx* A, cplx* col, cplx* prow,
                                                 int* piv, int* status) {
  __shared__ double bv[NGJ];
  __shared__ int bi[NGJ];
  int tid = threadIdx.x;
  double best = -1;
  int bidx = c;
  for (int r = c + tid; r < N; r += NGJ) {
    double v = abs2(A[(long)r * N + c]);
    if (v > best) {
      best = v;
      bidx = r;
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int w = NGJ / 2; w > 0; w >>= 1) {
    if (tid < w) {
      if (bv[tid + w] > bv[tid] || (bv[tid + w] == bv[tid] && bi[tid + w] < bi[tid])) {
        bv[tid] = bv[tid + w];
        bi[tid] = bi[tid + w];
      }
    }
    __syncthreads();
  }
  int p = bi[0];
  if (bv[0] <= 0.0) {
    if (tid == 0) *status = CNTR_ESINGULAR;
    p = c;
  }
  if (tid == 0) piv[c] = p;
  if (p != c)
    for (int q = tid; q < N; q += NGJ) {
      cplx t = A[(long)p * N + q];
      A[(long)p * N + q] = A[(long)c * N + q];
      A[(long)c * N + q] = t;
    }
  __syncthreads();
  cplx pv = A[(long)c * N + c];
  cplx ipv = bv[0] > 0 ? cdiv(mk(1, 0), pv) : mk(0, 0);
  for (int r = tid; r < N; r += NGJ) col[r] = A[(long)r * N + c];
  for (int q = tid; q < N; q += NGJ) prow[q] = (q == c) ? ipv : A[(long)c * N + q] * ipv;
}

__global__ __launch_bounds__(NT3) void k_gj_update(int N, int c, cplx* A, const cplx* col,
                                                   const cplx* prow) {
  long idx = (long)blockIdx.x * NT3 + threadIdx.x;
  if (idx >= (long)N * N) return;
  int r = idx / N, q = idx % N;
  if (r == c) {
    A[idx] = prow[q];
    return;
  }
  cplx f = col[r];
  if (q == c) A[idx] = -(f * prow[c]);
  else A[idx] = A[idx] - f * prow[q];
}

// undo the row interchanges: column swaps in reverse order, row by row
// (grid z: the problems of a batch, matrices N*N apart)
__global__ __launch_bounds__(NT3) void k_gj_unpivot(int N, cplx* A, const int* piv) {
  A += (size_t)blockIdx.z * N * N;
  piv += (size_t)blockIdx.z * N;
  long r = (long)blockIdx.x * NT3 + threadIdx.x;
  if (r >= N) return;
  cplx* row = A + r * N;
  for (int c = N - 1; c >= 0; c--) {
    int p = piv[c];
    if (p != c) {
      cplx t = row[p];
      row[p] = row[c];
      row[c] = t;
    }
  }
}

// ----------------------------------- blocked Gauss-Jordan (N <= GJT GJH)
// Panels of GJB columns. For the panel columns c0..c0+nb-1 the GJ steps run
// in one workgroup with the panel in registers (thread t holds the rows
// t + h GJT, h < GJH): pivot search over the rows r >= c, row interchange,
// and the in-place update of the panel (column c becomes column c of the
// inverse form). The rows that the panel's interchanges move are copied,
// interchanged, to ob. The other columns then take the whole panel as one
// rank-nb update (block identity of the in-place elimination): block rows
// A_1j := A11' A_1j, other rows A_ij += A_i1' A_1j, with the panel ' after
// its steps and A_1j the pivot rows before them.
constexpr int GJB = 8;
constexpr int GJT = 512, GJH = 4;  // panel workgroup: GJT threads, GJH rows each (N <= GJT GJH)
static_assert(GJT * GJH == GJ_BATCH_MAX_N, "blocked inverse size limit");

__device__ inline void gj_argmax(double& v, int& i) {
  // ties: smaller index
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

// (grid z: the problems of a batch; matrices N*N apart, work regions ws
// elements apart, pivots N apart, one status word each)
__global__ __launch_bounds__(GJT) void k_gjb_panel(int N, int c0, int nb, cplx* A, cplx* ob, int* rlist,
                                                   int* piv, int* status, size_t ws) {
  {
    size_t z = blockIdx.z;
    A += z * N * N;
    ob += z * ws;
    rlist = (int*)((cplx*)rlist + z * ws);
    piv += z * N;
    status += z;
  }
  // per-step LDS, double-buffered by the parity of the step (one barrier
  // fewer per step)
  __shared__ double wv[2][GJT / 64];
  __shared__ int wi[2][GJT / 64];
  __shared__ cplx xr[2][2][GJB];  // rows being interchanged
  __shared__ cplx pr[2][GJB];     // pivot row of the step
  __shared__ int s_piv[GJB];
  __shared__ int dst[2 * GJB], src[2 * GJB], s_m;
  int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  cplx L[GJH][GJB];
#pragma unroll
  for (int h = 0; h < GJH; h++) {
    int r = t + h * GJT;
#pragma unroll
    for (int j = 0; j < GJB; j++) L[h][j] = (r < N && j < nb) ? A[(long)r * N + c0 + j] : mk(0, 0);
  }
  for (int b = 0; b < nb; b++) {
    int c = c0 + b, sb = b & 1;
    // pivot: largest |a_rc|^2 over the rows r >= c (ties: smallest row)
    double best = -1;
    int bi = c;
#pragma unroll
    for (int h = 0; h < GJH; h++) {
      int r = t + h * GJT;
      double v = -1;
#pragma unroll
      for (int j = 0; j < GJB; j++)
        if (j == b) v = abs2(L[h][j]);
      if (r >= c && r < N && v > best) {
        best = v;
        bi = r;
      }
    }
    gj_argmax(best, bi);
    if (lane == 0) {
      wv[sb][wave] = best;
      wi[sb][wave] = bi;
    }
    __syncthreads();
    // every thread combines the wave results (same order, same answer)
    double bb = wv[sb][0];
    int p = wi[sb][0];
#pragma unroll
    for (int w = 1; w < GJT / 64; w++)
      if (wv[sb][w] > bb || (wv[sb][w] == bb && wi[sb][w] < p)) {
        bb = wv[sb][w];
        p = wi[sb][w];
      }
    bool ok = bb > 0.0;
    if (!ok) p = c;
    if (t == 0) {
      if (!ok) *status = CNTR_ESINGULAR;
      s_piv[b] = p;
      piv[c] = p;
    }
    // interchange rows c and p of the panel; the pivot row
    if (p != c) {
#pragma unroll
      for (int h = 0; h < GJH; h++) {
        int r = t + h * GJT;
        if (r == c || r == p)
#pragma unroll
          for (int j = 0; j < GJB; j++) xr[sb][r == c ? 0 : 1][j] = L[h][j];
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < GJH; h++) {
        int r = t + h * GJT;
        if (r == c || r == p)
#pragma unroll
          for (int j = 0; j < GJB; j++) L[h][j] = xr[sb][r == c ? 1 : 0][j];
      }
    }
#pragma unroll
    for (int h = 0; h < GJH; h++)
      if (t + h * GJT == c)
#pragma unroll
        for (int j = 0; j < GJB; j++) pr[sb][j] = L[h][j];
    __syncthreads();
    cplx pv = mk(0, 0);
#pragma unroll
    for (int j = 0; j < GJB; j++)
      if (j == b) pv = pr[sb][j];
    cplx ipv = ok ? cdiv(mk(1, 0), pv) : mk(0, 0);
    cplx ps[GJB];  // pivot row times 1 / pivot
#pragma unroll
    for (int j = 0; j < GJB; j++) ps[j] = j == b ? ipv : pr[sb][j] * ipv;
#pragma unroll
    for (int h = 0; h < GJH; h++) {
      int r = t + h * GJT;
      if (r >= N) continue;
      if (r == c) {
#pragma unroll
        for (int j = 0; j < GJB; j++) L[h][j] = ps[j];
      } else {
        cplx f = mk(0, 0);
#pragma unroll
        for (int j = 0; j < GJB; j++)
          if (j == b) f = L[h][j];
#pragma unroll
        for (int j = 0; j < GJB; j++) L[h][j] = j == b ? -(f * ipv) : L[h][j] - f * ps[j];
      }
    }
  }
#pragma unroll
  for (int h = 0; h < GJH; h++) {
    int r = t + h * GJT;
    if (r < N)
#pragma unroll
      for (int j = 0; j < GJB; j++)
        if (j < nb) A[(long)r * N + c0 + j] = L[h][j];
  }
  // the panel's interchanges as one permutation of the rows involved (row
  // dst[i] receives the old row src[i]), built in registers: slots 0..nb-1
  // are the block rows, slot GJB + b the pivot row of step b when it lies
  // outside the block and is new (else empty)
  __syncthreads();  // s_piv
  if (t == 0) {
    int dl[2 * GJB], sl[2 * GJB];
#pragma unroll
    for (int i = 0; i < GJB; i++) dl[i] = i < nb ? c0 + i : -1;
#pragma unroll
    for (int b = 0; b < GJB; b++) {
      int pb = b < nb ? s_piv[b] : -1;
      bool keep = pb >= c0 + nb;
#pragma unroll
      for (int b2 = 0; b2 < GJB; b2++)
        if (b2 < b) keep = keep && dl[GJB + b2] != pb;
      dl[GJB + b] = keep ? pb : -1;
    }
#pragma unroll
    for (int i = 0; i < 2 * GJB; i++) sl[i] = dl[i];
#pragma unroll
    for (int b = 0; b < GJB; b++) {
      int c = c0 + b, pb = b < nb ? s_piv[b] : c;
      if (pb != c) {
        int vc = -1, vp = -1;
#pragma unroll
        for (int i = 0; i < 2 * GJB; i++) {
          if (dl[i] == c) vc = sl[i];
          if (dl[i] == pb) vp = sl[i];
        }
#pragma unroll
        for (int i = 0; i < 2 * GJB; i++) {
          if (dl[i] == c) sl[i] = vp;
          else if (dl[i] == pb) sl[i] = vc;
        }
      }
    }
    int m = 0;
#pragma unroll
    for (int i = 0; i < 2 * GJB; i++)
      if (dl[i] >= 0) {
        dst[m] = dl[i];
        src[m] = sl[i];
        rlist[1 + m] = dl[i];
        m++;
      }
    s_m = m;
    rlist[0] = m;
  }
  __syncthreads();
  // rows dst[i] after the interchanges, columns outside the panel, to ob[i]
  // (the update reads them from there; A itself is rewritten by the update)
  int m = s_m;
  for (int i0 = 0; i0 < m; i0 += 8) {
    cplx v[8][GJH];  // 8 GJH loads in flight
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int h = 0; h < GJH; h++) {
        int i = i0 + u, q = t + h * GJT;
        v[u][h] = (i < m && q < N) ? A[(long)src[i] * N + q] : mk(0, 0);
      }
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int h = 0; h < GJH; h++) {
        int i = i0 + u, q = t + h * GJT;
        if (i < m && q < N && (q < c0 || q >= c0 + nb)) ob[(long)i * N + q] = v[u][h];
      }
  }
}

// Rank-nb update of the columns outside the panel; a workgroup covers NT3
// consecutive columns and GJR rows. Rows involved in the panel's
// interchanges take their (interchanged) old values from ob.
constexpr int GJR = 16;
__global__ __launch_bounds__(NT3) void k_gjb_update(int N, int c0, int nb, cplx* A, const cplx* ob,
                                                    const int* rlist, size_t ws) {
  {
    size_t z = blockIdx.z;
    A += z * N * N;
    ob += z * ws;
    rlist = (const int*)((const cplx*)rlist + z * ws);
  }
  __shared__ cplx ps[GJR][GJB];
  __shared__ int rl[2 * GJB + 1];
  int t = threadIdx.x;
  int q = blockIdx.x * NT3 + t, r0 = blockIdx.y * GJR;
  for (int i = t; i < GJR * GJB; i += NT3) {
    int rr = r0 + i / GJB, j = i % GJB;
    ps[i / GJB][j] = (rr < N && j < nb) ? A[(long)rr * N + c0 + j] : mk(0, 0);
  }
  if (t <= 2 * GJB) rl[t] = rlist[t];
  __syncthreads();
  if (q >= N || (q >= c0 && q < c0 + nb)) return;
  int m = rl[0];
  // pivot rows (block rows c0 + j) after the interchanges
  cplx y[GJB];
#pragma unroll
  for (int j = 0; j < GJB; j++) {
    int ij = 0;
    for (int i = 0; i < m; i++)
      if (rl[1 + i] == c0 + j) ij = i;
    y[j] = j < nb ? ob[(long)ij * N + q] : mk(0, 0);
  }
  for (int i = 0; i < GJR; i++) {
    int r = r0 + i;
    if (r >= N) break;
    bool blk = r >= c0 && r < c0 + nb;
    cplx v = mk(0, 0);
    if (!blk) {
      int ir = -1;
      for (int u = 0; u < m; u++)
        if (rl[1 + u] == r) ir = u;
      v = ir >= 0 ? ob[(long)ir * N + q] : A[(long)r * N + q];
    }
#pragma unroll
    for (int j = 0; j < GJB; j++) v = v + ps[i][j] * y[j];
    A[(long)r * N + q] = v;
  }
}

// ob (2 GJB rows of N) and the list of the rows involved (2 GJB + 1 ints)
size_t gj_work_elems(int N) { return (size_t)(2 * GJB) * N + 4 * GJB; }

hipError_t launch_gj_inverse_batch(int N, int B, cplx* A, cplx* work, int* piv, int* status, hipStream_t s) {
  if (N > GJT * GJH) return hipErrorInvalidValue;
  size_t ws = gj_work_elems(N);
  dim3 gu((N + NT3 - 1) / NT3, (N + GJR - 1) / GJR, B);
  for (int c0 = 0; c0 < N; c0 += GJB) {
    int nb = N - c0 < GJB ? N - c0 : GJB;
    int* rlist = (int*)(work + (size_t)(2 * GJB) * N);
    k_gjb_panel<<<dim3(1, 1, B), GJT, 0, s>>>(N, c0, nb, A, work, rlist, piv, status, ws);
    k_gjb_update<<<gu, NT3, 0, s>>>(N, c0, nb, A, work, rlist, ws);
  }
  k_gj_unpivot<<<dim3((N + NT3 - 1) / NT3, 1, B), NT3, 0, s>>>(N, A, piv);
  return hipGetLastError();
}

hipError_t launch_gj_inverse(int N, cplx* A, cplx* work, int* piv, int* status, hipStream_t s) {
  if (N <= GJT * GJH) return launch_gj_inverse_batch(N, 1, A, work, piv, status, s);
  cplx* col = work;
  cplx* prow = work + N;
  long tot = (long)N * N;
  unsigned nbk = (unsigned)((tot + NT3 - 1) / NT3);
  for (int c = 0; c < N; c++) {
    k_gj_pivot<<<1, NGJ, 0, s>>>(N, c, A, col, prow, piv, status);
    k_gj_update<<<nbk, NT3, 0, s>>>(N, c, A, col, prow);
  }
  k_gj_unpivot<<<(N + NT3 - 1) / NT3, NT3, 0, s>>>(N, A, piv);
  return hipGetLastError();
}

// ------------------------------------------------------------ matvec
// y = X v  or  y = b - X v ; one wavefront per row, lanes stride the row.
// One wavefront per row r: y_r = X_r v (or b_r - X_r v); four row elements
// (and their right-hand sides) are loaded per round.
template <int NR>
__global__ __launch_bounds__(NT3) void k_matvec(int N, const cplx* X, const cplx* v, const cplx* b, cplx* y,
                                                double* zero2) {
  if (zero2 && blockIdx.x == 0 && threadIdx.x < 2) zero2[threadIdx.x] = 0.0;
  int lane = threadIdx.x % 64;
  long r = (long)blockIdx.x * (NT3 / 64) + threadIdx.x / 64;
  if (r >= N) return;
  cplx acc[NR];
#pragma unroll
  for (int c = 0; c < NR; c++) acc[c] = mk(0, 0);
  const cplx* row = X + r * N;
  int q = lane;
  for (; q + 192 < N; q += 256) {
    cplx x[4], w[4][NR];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      x[u] = gld(row + q + 64 * u);
#pragma unroll
      for (int c = 0; c < NR; c++) w[u][c] = gld(v + (long)(q + 64 * u) * NR + c);
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int c = 0; c < NR; c++) cfma(acc[c], x[u], w[u][c]);
  }
  for (; q < N; q += 64) {
    cplx x = gld(row + q);
#pragma unroll
    for (int c = 0; c < NR; c++) cfma(acc[c], x, gld(v + (long)q * NR + c));
  }
#pragma unroll
  for (int c = 0; c < NR; c++) {
    double re = acc[c].x, im = acc[c].y;
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off);
      im += __shfl_xor(im, off);
    }
    if (lane == 0) {
      cplx o = mk(re, im);
      y[r * NR + c] = b ? b[r * NR + c] - o : o;
    }
  }
}

hipError_t launch_matvec(int N, int nrhs, const cplx* X, const cplx* v, const cplx* b, cplx* y,
                         hipStream_t s, double* zero2) {
  int g = (N + 3) / 4;
  switch (nrhs) {
    case 1: k_matvec<1><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 2: k_matvec<2><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 3: k_matvec<3><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 4: k_matvec<4><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 5: k_matvec<5><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 6: k_matvec<6><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 7: k_matvec<7><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    case 8: k_matvec<8><<<g, NT3, 0, s>>>(N, X, v, b, y, zero2); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// x += dx ; norms[0] += sum |r|^2, norms[1] += sum |g|^2
__global__ __launch_bounds__(NT3) void k_axpy_norm(int len, cplx* x, const cplx* dx, const cplx* r,
                                                   const cplx* g, double* norms) {
  __shared__ double s0[NT3], s1[NT3];
  long i = (long)blockIdx.x * NT3 + threadIdx.x;
  double a = 0, b = 0;
  if (i < len) {
    if (dx) x[i] = x[i] + dx[i];
    a = abs2(r[i]);
    b = abs2(g[i]);
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = NT3 / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&norms[0], s0[0]);
    atomicAdd(&norms[1], s1[0]);
  }
}

hipError_t launch_axpy_norm(int len, cplx* x, const cplx* dx, const cplx* r, const cplx* g,
                            double* norms, hipStream_t s) {
  k_axpy_norm<<<(len + NT3 - 1) / NT3, NT3, 0, s>>>(len, x, dx, r, g, norms);
  return hipGetLastError();
}

// Linear mixing of a self-consistency input with the previous input:
// x <- a x + (1-a) keep (unless first), keep <- x.
__global__ __launch_bounds__(NT3) void k_mix(int len, cplx* x, cplx* keep, double a, int first) {
  long i = (long)blockIdx.x * NT3 + threadIdx.x;
  if (i >= len) return;
  cplx v = x[i];
  if (!first) v = a * v + (1.0 - a) * keep[i];
  x[i] = v;
  keep[i] = v;
}

hipError_t launch_mix(int len, cplx* x, cplx* keep, double a, bool first, hipStream_t s) {
  k_mix<<<(len + NT3 - 1) / NT3, NT3, 0, s>>>(len, x, keep, a, first ? 1 : 0);
  return hipGetLastError();
}

// ------------------------------------------- Fourier-series Matsubara solve
// The method of the "Fourier series representation" (Sec. "Implementation:
// dyson", Matsubara), a fast solve of O(h_tau^2) average accuracy:
//   Sigma(i w_m) = int_0^beta Sigma^M(tau) e^{i w_m tau} dtau, integrating the
//     piecewise-cubic interpolant of the samples exactly (the cubically
//     corrected transform): on [tau_J, tau_J+1] the cubic through the grid
//     points J-1..J+2 (J..J+3 on the first interval, J-2..J+1 on the last);
//   G(i w_m) = [i w_m - x - Sigma(i w_m)]^{-1}, x = eps(0^-) - mu (the
//     algebraic Dyson equation);
//   G^M(tau) = (1/beta) sum_m e^{-i w_m tau} G~(i w_m) - c(tau) 1 with
//     G~(i w) = G(i w) - 1/(i w) (none at the bosonic w = 0), c = 1/2
//     (fermions) or 1/2 - tau/beta (bosons): the jump G^M(0+) - xi G^M(beta-)
//     = -1 removed, so that the sum converges.
// Frequencies w = q pi / beta: fermions q = 2m+1, m = -Nw..Nw-1; bosons
// q = 2m, m = -Nw..Nw; Nw = p Ntau. Phases are reduced exactly in integers:
// w_m tau_j = pi (q j mod 2 Ntau) / Ntau.
__device__ inline int mf_q(int f, int nw, int xi) { return xi == -1 ? 2 * (f - nw) + 1 : 2 * (f - nw); }

// mu_k = int_0^1 u^k e^{i th u} du, k = 0..3 (series below |th| = 1, where
// the recursion would cancel)
__device__ inline void mf_moments(double th, cplx (&mu)[4]) {
  if (fabs(th) < 1.0) {
#pragma unroll
    for (int k = 0; k < 4; k++) mu[k] = mk(0, 0);
    cplx t = mk(1, 0);  // (i th)^n / n!
    for (int n = 0; n < 24; n++) {
#pragma unroll
      for (int k = 0; k < 4; k++) mu[k] = mu[k] + (1.0 / (n + k + 1)) * t;
      t = (1.0 / (n + 1)) * (t * mk(0, th));
    }
    return;
  }
  double sn, cs;
  sincos(th, &sn, &cs);
  cplx e = mk(cs, sn), iz = mk(0, -1.0 / th);  // 1 / (i th)
  mu[0] = (e - mk(1, 0)) * iz;
#pragma unroll
  for (int k = 1; k < 4; k++) mu[k] = (e - (double)k * mu[k - 1]) * iz;
}
// int_0^1 L_i(u) e^{i th u} du for the Lagrange basis of the nodes o..o+3
__device__ inline void mf_weights(int o, const cplx (&mu)[4], cplx (&w)[4]) {
#pragma unroll
  for (int i = 0; i < 4; i++) {
    double a[4] = {1, 0, 0, 0}, den = 1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      if (j == i) continue;
      double xj = o + j;
#pragma unroll
      for (int k = 3; k >= 1; k--) a[k] = a[k - 1] - xj * a[k];
      a[0] = -xj * a[0];
      den *= (double)(i - j);
    }
    cplx v = mk(0, 0);
#pragma unroll
    for (int k = 0; k < 4; k++) v = v + (a[k] / den) * mu[k];
    w[i] = v;
  }
}
// Sigma(i w_f) for one element: thread (f, e)
__global__ __launch_bounds__(NT3) void k_mf_sigma(Prob P, int nw, int nf, cplx* W) {
  int dd = P.d * P.d, N = P.ntau;
  int idx = blockIdx.x * NT3 + threadIdx.x;
  if (idx >= nf * dd) return;
  int f = idx / dd, e = idx % dd;
  int q = mf_q(f, nw, P.sig);
  cplx mu[4], wf[4], wi[4], wl[4];
  mf_moments(M_PI * q / N, mu);
  mf_weights(0, mu, wf);
  mf_weights(-1, mu, wi);
  mf_weights(-2, mu, wl);
  const cplx* S = P.Smat;
  cplx acc = mk(0, 0);
  for (int J = 0; J < N; J++) {
    int s = min(max(J - 1, 0), N - 3), o = s - J;
    cplx v = mk(0, 0);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      cplx wv = o == 0 ? wf[i] : (o == -1 ? wi[i] : wl[i]);
      v = v + wv * gld(S + (size_t)(s + i) * dd + e);
    }
    long r = ((long)q * J) % (2L * N);
    if (r < 0) r += 2L * N;
    double sn, cs;
    sincos(M_PI * (double)r / N, &sn, &cs);
    acc = acc + mk(cs, sn) * v;
  }
  W[(size_t)f * dd + e] = (P.beta / N) * acc;
}
// G~(i w_f) = [i w - x - Sigma(i w)]^{-1} - 1/(i w): one wave per frequency
__global__ __launch_bounds__(NT3) void k_mf_solve(Prob P, int nw, int nf, cplx* W, int has_sigma) {
  __shared__ cplx A[NT3 / 64][64];
  __shared__ int piv[NT3 / 64][8];
  int d = P.d, dd = d * d, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int f = blockIdx.x * (NT3 / 64) + wave;
  if (f >= nf) return;  // (whole waves)
  int q = mf_q(f, nw, P.sig);
  double w = M_PI * q / P.beta;
  int r = lane / d, c = lane % d;
  if (lane < dd) {
    cplx v = -gld(P.eps + lane);  // eps(0^-)
    if (r == c) v = v + mk(P.mu, w);
    if (has_sigma) v = v - W[(size_t)f * dd + lane];
    A[wave][lane] = v;
  }
  wave_sync();
  wave_inverse(d, A[wave], piv[wave]);
  if (lane < dd) {
    cplx g = A[wave][lane];
    if (q != 0 && r == c) g = g + mk(0, 1.0 / w);  // - 1/(i w)
    W[(size_t)f * dd + lane] = g;
  }
}
// G^M(tau_j): one workgroup per j, thread (frequency group, element); the
// groups' sums are added in a fixed order
__global__ __launch_bounds__(NT3) void k_mf_back(Prob P, int nw, int nf, const cplx* W) {
  __shared__ cplx red[NT3];
  int dd = P.d * P.d, N = P.ntau, j = blockIdx.x, t = threadIdx.x;
  int G = NT3 / dd, e = t % dd, g = t / dd;
  cplx acc = mk(0, 0);
  if (g < G)
    for (int f = g; f < nf; f += G) {
      int q = mf_q(f, nw, P.sig);
      long r = ((long)q * j) % (2L * N);
      if (r < 0) r += 2L * N;
      double sn, cs;
      sincos(M_PI * (double)r / N, &sn, &cs);
      acc = acc + mk(cs, -sn) * W[(size_t)f * dd + e];
    }
  red[t] = acc;
  __syncthreads();
  if (t < dd) {
    cplx v = mk(0, 0);
    for (int gg = 0; gg < G; gg++) v = v + red[gg * dd + t];
    v = (1.0 / P.beta) * v;
    if (t / P.d == t % P.d) v = v - mk(P.sig == -1 ? 0.5 : 0.5 - (double)j / N, 0);
    gst(P.Gmat + (size_t)j * dd + t, v);
  }
}

size_t mats_fourier_scratch_bytes(int ntau, int d, int p) {
  return (size_t)(2 * (size_t)p * ntau + 1) * d * d * sizeof(cplx);
}

hipError_t launch_mats_fourier(const Prob& P, int p, cplx* work, hipStream_t s) {
  int nw = p * P.ntau, nf = P.sig == -1 ? 2 * nw : 2 * nw + 1, dd = P.d * P.d;
  if (P.Smat) k_mf_sigma<<<(nf * dd + NT3 - 1) / NT3, NT3, 0, s>>>(P, nw, nf, work);
  k_mf_solve<<<(nf + NT3 / 64 - 1) / (NT3 / 64), NT3, 0, s>>>(P, nw, nf, work, P.Smat ? 1 : 0);
  k_mf_back<<<P.ntau + 1, NT3, 0, s>>>(P, nw, nf, work);
  return hipGetLastError();
}

}  // namespace cntr
