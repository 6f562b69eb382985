// Device helpers shared by the kernel files: problem access, block access,
// small dense solves held in LDS.
#pragma once
#include "cntr_internal.h"

namespace cntr {

// Problems of one call: a single problem travels by value in the kernel
// arguments; batches live in a device array.
struct ProbArg {
  Prob one;
  const Prob* many;
  int count;
  __device__ inline const Prob& get(int i) const { return count == 1 ? one : many[i]; }
};

// Per-problem scratch region, and one status word per problem of the call
// (kept apart from the regions, whose layout depends on the call).
struct Scratch {
  char* base;
  size_t stride;  // bytes per problem
  size_t off_minv, off_part, off_tail, off_status;
  int* stat;      // status words, one per problem
  __device__ inline cplx* minv(int pi) const { return (cplx*)(base + pi * stride + off_minv); }
  // boundary-row source terms of the retarded boundary columns (after the
  // KMAX + 2 inverses), d x d blocks of d = dd
  __device__ inline cplx* bsrc(int pi, int dd) const { return minv(pi) + (KMAX + 2) * dd; }
  // operator of the k+1 serial boundary rows, (KMAX+1)(KMAX+2)/2 blocks
  __device__ inline cplx* zop(int pi, int dd) const { return minv(pi) + (2 * KMAX + 4) * dd; }
  __device__ inline cplx* part(int pi) const { return (cplx*)(base + pi * stride + off_part); }
  __device__ inline cplx* tail(int pi) const { return (cplx*)(base + pi * stride + off_tail); }
  __device__ inline int* status(int pi) const { return stat + pi; }
  // completion counter of the boundary-row kernel (reset to 0 by its user)
  __device__ inline int* counter(int pi) const { return (int*)(base + pi * stride + off_status + 64); }
};

__device__ inline cplx ld(const cplx* p) { return *p; }

// Loads and stores through global-address-space pointers. The contour
// pointers reach the kernels inside structures, so the compiler would emit
// flat accesses, which also count against the LDS wait counter and force
// every LDS wait to drain the outstanding HBM loads.
// (The qualifier exists only in the device pass; the host pass of the same
// source sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define CNTR_GLOBAL __attribute__((address_space(1)))
#else
#define CNTR_GLOBAL
#endif
template <class T>
__device__ inline T gld(const T* p) {
  return *(const CNTR_GLOBAL T*)p;
}
template <class T>
__device__ inline void gst(T* p, T v) {
  *(CNTR_GLOBAL T*)p = v;
}
// Complex values go through a two-double vector type: a copy of the cplx
// structure would pass through its (generic) copy constructor and lose the
// address space again.
typedef double cntr_v2d __attribute__((ext_vector_type(2)));
__device__ inline cplx gld(const cplx* p) {
  cntr_v2d t = *(const CNTR_GLOBAL cntr_v2d*)p;
  return cplx{t.x, t.y};
}
__device__ inline void gst(cplx* p, cplx v) {
  cntr_v2d t = {v.x, v.y};
  *(CNTR_GLOBAL cntr_v2d*)p = t;
}

// Completion count of the workgroups of one problem (the last to arrive
// finishes the work; no workgroup waits for another). Every wave first waits
// until its own global stores are complete in the L2 (s_waitcnt vmcnt(0):
// 0xF70 also leaves expcnt and lgkmcnt at their maxima), the workgroup meets
// at a barrier, and one thread releases them all at agent scope and counts:
// one L2 write-back per workgroup instead of one per wave. True in every
// thread of the workgroup whose count reaches `expect`, after an agent-scope
// acquire of the others' stores.
__device__ inline bool last_to_arrive(int* counter, int expect, int& flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0xF70);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    flag = atomicAdd(counter, 1) == expect;
  }
  __syncthreads();
  bool last = flag != 0;
  if (last) __threadfence();
  return last;
}

// Retarded value with the continuation t < t':  X~^R_{a,b}[r][c]
template <int D>
__device__ inline cplx ret_ext(const cplx* X, int a, int b, int r, int c) {
  if (a >= b) return gld(X + (tri(a) + b) * D * D + r * D + c);
  return -conj(gld(X + (tri(b) + a) * D * D + c * D + r));
}
// Lesser value for any order of the arguments: X^<_{a,b}[r][c]
template <int D>
__device__ inline cplx les_any(const cplx* X, int a, int b, int r, int c) {
  if (a <= b) return gld(X + (tri(b) + a) * D * D + r * D + c);
  return -conj(gld(X + (tri(a) + b) * D * D + c * D + r));
}

// The same for a block size d known only at run time.
__device__ inline cplx ret_ext_d(const cplx* X, int a, int b, int r, int c, int d) {
  if (a >= b) return gld(X + (tri(a) + b) * d * d + r * d + c);
  return -conj(gld(X + (tri(b) + a) * d * d + c * d + r));
}
__device__ inline cplx les_any_d(const cplx* X, int a, int b, int r, int c, int d) {
  if (a <= b) return gld(X + (tri(b) + a) * d * d + r * d + c);
  return -conj(gld(X + (tri(a) + b) * d * d + c * d + r));
}

// Gauss-Jordan inverse of an n x n complex matrix in LDS (in place), with
// partial pivoting, executed by the whole workgroup. piv: LDS int[n].
// Returns false (uniformly) if singular.
__device__ inline bool lds_inverse(int n, cplx* A, int* piv, double* redv, int* redi) {
  int tid = threadIdx.x, nt = blockDim.x;
  bool ok = true;
  for (int c = 0; c < n; c++) {
    if (tid == 0) {
      int p = c;
      double best = abs2(A[c * n + c]);
      for (int r = c + 1; r < n; r++) {
        double v = abs2(A[r * n + c]);
        if (v > best) {
          best = v;
          p = r;
        }
      }
      redi[0] = p;
      redv[0] = best;
      piv[c] = p;
    }
    __syncthreads();
    int p = redi[0];
    if (redv[0] == 0.0) {
      ok = false;
      __syncthreads();
      break;
    }
    if (p != c)
      for (int q = tid; q < n; q += nt) {
        cplx t = A[p * n + q];
        A[p * n + q] = A[c * n + q];
        A[c * n + q] = t;
      }
    __syncthreads();
    cplx pv = A[c * n + c];
    cplx ipv = cdiv(mk(1, 0), pv);
    // column factors and scaled pivot row, then rank-1 update
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += nt) {
      int r = idx / n, q = idx % n;
      if (r == c) continue;
      cplx f = A[r * n + c];
      if (q == c) continue;
      A[r * n + q] = A[r * n + q] - f * (A[c * n + q] * ipv);
    }
    __syncthreads();
    for (int r = tid; r < n; r += nt)
      if (r != c) A[r * n + c] = -(A[r * n + c] * ipv);
    __syncthreads();
    for (int q = tid; q < n; q += nt) A[c * n + q] = (q == c) ? ipv : A[c * n + q] * ipv;
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, in reverse order
  if (ok)
    for (int c = n - 1; c >= 0; c--) {
      int p = piv[c];
      if (p != c)
        for (int r = tid; r < n; r += nt) {
          cplx t = A[r * n + p];
          A[r * n + p] = A[r * n + c];
          A[r * n + c] = t;
        }
      __syncthreads();
    }
  return ok;
}

// Solve A X = B in LDS (A: n x n, B: n x nrhs, row-major), Gaussian
// elimination with partial pivoting by the workgroup. A, B overwritten.
__device__ inline bool lds_solve(int n, int nrhs, cplx* A, cplx* B, double* redv, int* redi) {
  int tid = threadIdx.x, nt = blockDim.x;
  for (int c = 0; c < n; c++) {
    if (tid == 0) {
      int p = c;
      double best = abs2(A[c * n + c]);
      for (int r = c + 1; r < n; r++) {
        double v = abs2(A[r * n + c]);
        if (v > best) {
          best = v;
          p = r;
        }
      }
      redi[0] = p;
      redv[0] = best;
    }
    __syncthreads();
    int p = redi[0];
    if (redv[0] == 0.0) return false;
    if (p != c) {
      for (int q = tid; q < n; q += nt) {
        cplx t = A[p * n + q];
        A[p * n + q] = A[c * n + q];
        A[c * n + q] = t;
      }
      for (int q = tid; q < nrhs; q += nt) {
        cplx t = B[p * nrhs + q];
        B[p * nrhs + q] = B[c * nrhs + q];
        B[c * nrhs + q] = t;
      }
    }
    __syncthreads();
    cplx ipv = cdiv(mk(1, 0), A[c * n + c]);
    int w = (n - c - 1);
    int cols = (n - c - 1) + nrhs;
    for (int idx = tid; idx < w * cols; idx += nt) {
      int r = c + 1 + idx / cols, q = idx % cols;
      cplx f = A[r * n + c] * ipv;
      if (q < n - c - 1) {
        int qq = c + 1 + q;
        A[r * n + qq] = A[r * n + qq] - f * A[c * n + qq];
      } else {
        int qq = q - (n - c - 1);
        B[r * nrhs + qq] = B[r * nrhs + qq] - f * B[c * nrhs + qq];
      }
    }
    __syncthreads();
  }
  // back substitution, one right-hand side column per thread group
  for (int c = n - 1; c >= 0; c--) {
    cplx ipv = cdiv(mk(1, 0), A[c * n + c]);
    for (int q = tid; q < nrhs; q += nt) B[c * nrhs + q] = B[c * nrhs + q] * ipv;
    __syncthreads();
    for (int idx = tid; idx < c * nrhs; idx += nt) {
      int r = idx / nrhs, q = idx % nrhs;
      B[r * nrhs + q] = B[r * nrhs + q] - A[r * n + c] * B[c * nrhs + q];
    }
    __syncthreads();
  }
  return true;
}

// ------------------------------------------------ single-wavefront solvers
// Executed by exactly one wavefront (64 lanes); the other waves of the
// workgroup do not take part. Synchronisation is wave-local (instruction
// order plus a compiler barrier), never a workgroup barrier.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of the largest v over the wave (ties: smallest index); every lane
// gets the same answer.
__device__ inline int wave_argmax(double v, int idx, double* vmax) {
  for (int off = 32; off > 0; off >>= 1) {
    double ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  *vmax = v;
  return idx;
}

// In-place inverse of an n x n matrix in LDS (Gauss-Jordan, partial pivoting).
// piv: LDS int[n]. Returns false if singular (the matrix is then garbage).
__device__ inline bool wave_inverse(int n, cplx* A, int* piv) {
  int lane = threadIdx.x & 63;
  bool ok = true;
  for (int c = 0; c < n; c++) {
    double best;
    int p = wave_argmax((lane >= c && lane < n) ? abs2(A[lane * n + c]) : -1.0, lane, &best);
    if (!(best > 0)) ok = false;
    if (lane == 0) piv[c] = p;
    if (p != c)
      for (int q = lane; q < n; q += 64) {
        cplx t = A[p * n + q];
        A[p * n + q] = A[c * n + q];
        A[c * n + q] = t;
      }
    wave_sync();
    cplx ipv = best > 0 ? cdiv(mk(1, 0), A[c * n + c]) : mk(0, 0);
    for (int idx = lane; idx < n * n; idx += 64) {
      int r = idx / n, q = idx % n;
      if (r == c || q == c) continue;
      A[idx] = A[idx] - A[r * n + c] * (A[c * n + q] * ipv);
    }
    wave_sync();
    for (int r = lane; r < n; r += 64)
      if (r != c) A[r * n + c] = -(A[r * n + c] * ipv);
    for (int q = lane; q < n; q += 64) A[c * n + q] = (q == c) ? ipv : A[c * n + q] * ipv;
    wave_sync();
  }
  for (int c = n - 1; c >= 0; c--) {
    int p = piv[c];
    if (p != c)
      for (int r = lane; r < n; r += 64) {
        cplx t = A[r * n + p];
        A[r * n + p] = A[r * n + c];
        A[r * n + c] = t;
      }
    wave_sync();
  }
  return ok;
}

// Solve A X = B in LDS (A: n x n, B: n x nrhs), Gaussian elimination with
// partial pivoting and back substitution; A and B are overwritten.
__device__ inline bool wave_solve(int n, int nrhs, cplx* A, cplx* B) {
  int lane = threadIdx.x & 63;
  bool ok = true;
  for (int c = 0; c < n; c++) {
    double best;
    int p = wave_argmax((lane >= c && lane < n) ? abs2(A[lane * n + c]) : -1.0, lane, &best);
    if (!(best > 0)) ok = false;
    if (p != c) {
      for (int q = lane; q < n; q += 64) {
        cplx t = A[p * n + q];
        A[p * n + q] = A[c * n + q];
        A[c * n + q] = t;
      }
      for (int q = lane; q < nrhs; q += 64) {
        cplx t = B[p * nrhs + q];
        B[p * nrhs + q] = B[c * nrhs + q];
        B[c * nrhs + q] = t;
      }
    }
    wave_sync();
    cplx ipv = best > 0 ? cdiv(mk(1, 0), A[c * n + c]) : mk(0, 0);
    int w = n - c - 1, cols = w + nrhs;
    for (int idx = lane; idx < w * cols; idx += 64) {
      int r = c + 1 + idx / cols, q = idx % cols;
      cplx f = A[r * n + c] * ipv;
      if (q < w) A[r * n + c + 1 + q] = A[r * n + c + 1 + q] - f * A[c * n + c + 1 + q];
      else B[r * nrhs + q - w] = B[r * nrhs + q - w] - f * B[c * nrhs + q - w];
    }
    wave_sync();
  }
  for (int c = n - 1; c >= 0; c--) {
    cplx ipv = cdiv(mk(1, 0), A[c * n + c]);
    for (int q = lane; q < nrhs; q += 64) B[c * nrhs + q] = B[c * nrhs + q] * ipv;
    wave_sync();
    for (int idx = lane; idx < c * nrhs; idx += 64) {
      int r = idx / nrhs, q = idx % nrhs;
      B[r * nrhs + q] = B[r * nrhs + q] - A[r * n + c] * B[c * nrhs + q];
    }
    wave_sync();
  }
  return ok;
}

// ------------------------------------------- register-resident wave solves
// Maximum of an unsigned value over the 64 lanes (DPP butterfly inside each
// row of 16 lanes, then row broadcasts; the total ends in lane 63).
__device__ inline unsigned wave_umax(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));  // row half mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));  // row mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));  // row bcast 15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));  // row bcast 31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Value of x held by lane l (l uniform over the wave).
__device__ inline double rdlane(double x, int l) {
  long long b = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), l);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline cplx rdlane(cplx x, int l) { return mk(rdlane(x.x, l), rdlane(x.y, l)); }

// Gauss-Jordan elimination with partial pivoting of an N x N system, one row
// per lane: lane r < N holds row r of A (a[0..N), zero beyond) and of the
// right-hand sides B (b). Each step picks the unused row with the largest
// |a_c| (magnitudes compared in single precision, ties to the lowest lane),
// broadcasts it with readlane and eliminates column c from every other row.
// On return the lane that pivoted column `col` holds row `col` of A^-1 B in b.
// Returns false if a pivot was zero (the result is then garbage). Executed by
// one wavefront; lanes >= N take part but never pivot.
template <int NM, int NR>
__device__ inline bool lane_gauss_jordan(int N, cplx (&a)[NM], cplx (&b)[NR], int& col) {
  int lane = threadIdx.x & 63;
  bool used = lane >= N;
  bool ok = true;
  cplx piv = mk(1, 0);
  col = -1;
#pragma unroll
  for (int c = 0; c < NM; c++) {
    if (c < N) {
      float fv = (float)abs2(a[c]);
      unsigned key = used ? 0u : ((__float_as_uint(fv) & ~63u) | (unsigned)(63 - lane));
      unsigned kmax = wave_umax(key);
      int p = 63 - (int)(kmax & 63u);
      cplx pv = rdlane(a[c], p);
      if (!(abs2(pv) > 0)) ok = false;
      cplx ipv = ok ? cdiv(mk(1, 0), pv) : mk(0, 0);
      cplx f = a[c] * ipv;
      bool me = lane == p;
      if (me) {
        used = true;
        col = c;
        piv = pv;
      }
#pragma unroll
      for (int q = c + 1; q < NM; q++) {
        cplx t = rdlane(a[q], p);
        if (!me) a[q] = a[q] - f * t;
      }
#pragma unroll
      for (int q = 0; q < NR; q++) {
        cplx t = rdlane(b[q], p);
        if (!me) b[q] = b[q] - f * t;
      }
    }
  }
  cplx ip = cdiv(mk(1, 0), piv);
#pragma unroll
  for (int q = 0; q < NR; q++) b[q] = b[q] * ip;
  return ok;
}

// Solve A X = B in LDS with the whole workgroup: Gauss-Jordan elimination
// with partial pivoting, rows left in place (the pivot row of column c is
// remembered instead of swapped, and no row is scaled until the end). Wave 0
// finds the pivot among the rows not yet used (and its reciprocal); then
// every other row loses its column-c part, lanes over the columns c+1..n-1
// and the right-hand sides, waves over the rows: two barriers per column, no
// integer division. A: n x n with leading dimension ld (padded so that the
// column reads of the pivot search spread over the LDS banks), B: n x nrhs;
// on return X is in B (row order of X). n <= 64, n - 1 + nrhs <= 64.
// s_piv: LDS int[n]; s_ipv: LDS cplx; n nrhs <= 2 x the workgroup size.
// Every thread of the workgroup calls it. Returns false (uniformly) if a
// pivot is zero.
template <int NWAVE>
__device__ inline bool wg_solve(int n, int ld, int nrhs, cplx* A, cplx* B, int* s_piv, cplx* s_ipv) {
  constexpr int RPW = 64 / NWAVE;  // rows per wave (n <= 64)
  int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool used = false;  // wave 0: row `lane` already a pivot row
  bool ok = true;
  for (int c = 0; c < n; c++) {
    if (wave == 0) {
      // largest |A[r][c]| over the unused rows: a float key with the lane in
      // its low bits, maximised by DPP steps
      double v = (lane < n && !used) ? abs2(A[lane * ld + c]) : 0.0;
      unsigned key = (lane < n && !used) ? ((__float_as_uint((float)v) & ~63u) | (unsigned)(63 - lane)) : 0u;
      int p = 63 - (int)(wave_umax(key) & 63u);
      if (lane == p) used = true;
      if (lane == 0) {
        s_piv[c] = p;
        cplx pv = A[p * ld + c];
        *s_ipv = abs2(pv) > 0 ? cdiv(mk(1, 0), pv) : mk(0, 0);
      }
    }
    __syncthreads();
    int p = s_piv[c];
    cplx ipv = *s_ipv;
    if (ipv.x == 0 && ipv.y == 0) ok = false;
    int na = n - c - 1;  // columns c+1..n-1 of A, then the right-hand sides
    if (lane < na + nrhs) {
      bool isa = lane < na;
      cplx pv = isa ? A[p * ld + c + 1 + lane] : B[p * nrhs + (lane - na)];
      // the rows of this wave: all loads first, then the updates
      cplx fr[RPW], xr[RPW];
#pragma unroll
      for (int i = 0; i < RPW; i++) {
        int r = wave + NWAVE * i;
        bool act = r < n && r != p;
        int rr = act ? r : p;
        fr[i] = A[rr * ld + c];
        xr[i] = isa ? A[rr * ld + c + 1 + lane] : B[rr * nrhs + (lane - na)];
      }
#pragma unroll
      for (int i = 0; i < RPW; i++) {
        int r = wave + NWAVE * i;
        if (r < n && r != p) {
          cplx v = xr[i] - (fr[i] * ipv) * pv;
          if (isa) A[r * ld + c + 1 + lane] = v;
          else B[r * nrhs + (lane - na)] = v;
        }
      }
    }
    __syncthreads();
  }
  // X_c = B[p_c] / A[p_c][c]: all reads, then (after a barrier) all writes;
  // n nrhs <= 2 x the workgroup size
  cplx xv[2];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    int idx = tid + u * blockDim.x;
    if (idx < n * nrhs) {
      int c = idx / nrhs, q = idx - c * nrhs;
      int p = s_piv[c];
      xv[u] = B[p * nrhs + q] * cdiv(mk(1, 0), A[p * ld + c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; u++) {
    int idx = tid + u * blockDim.x;
    if (idx < n * nrhs) B[idx] = xv[u];
  }
  __syncthreads();
  return ok;
}

// Gregory weights w(N, j), N > k, from a copy of the end weights in LDS
// (per-lane indices never reach constant or private memory in the loops).
struct WReg {
  const double* om;  // LDS, KMAX + 1 entries
  int k;
  // every thread of the workgroup calls this before a barrier
  __device__ inline void load(const KW& W, double* lds_om) {
    k = W.k;
    if (threadIdx.x <= KMAX) lds_om[threadIdx.x] = W.omega[threadIdx.x];
    om = lds_om;
  }
  __device__ inline double w(int N, int j) const {
    bool left = j <= k, right = N - j <= k;
    double wl = om[left ? j : 0], wr = om[right ? N - j : 0];
    return left ? (right ? wl + wr - 1.0 : wl) : (right ? wr : 1.0);
  }
};

}  // namespace cntr
