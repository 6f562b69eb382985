// Elementwise slice kernels: second-Born self-energy + Hartree mean field,
// polynomial extrapolation, slice distance and copy; and the general contour
// convolution C = A * f * B (Eqs. cm1, cm2, cr1, ctv1-ctv3, cles1-cles3).
#include "launch.h"

namespace cntr {

constexpr int NT2 = 256;

// element index e of slice n -> (component, block, a, c); components:
// 0 = R_{n,j} (j = 0..n), 1 = L_{j,n} (j = 0..n), 2 = T_{n,m} (m = 0..ntau)
struct SliceIdx {
  int comp, j, a, c;
};
__device__ inline SliceIdx slice_idx(long idx, int n, int ntau, int d) {
  int dd = d * d;
  long nr = (long)(n + 1) * dd;
  SliceIdx s;
  int e;
  if (idx < nr) {
    s.comp = 0;
    s.j = idx / dd;
    e = idx % dd;
  } else if (idx < 2 * nr) {
    idx -= nr;
    s.comp = 1;
    s.j = idx / dd;
    e = idx % dd;
  } else {
    idx -= 2 * nr;
    s.comp = 2;
    s.j = idx / dd;
    e = idx % dd;
  }
  s.a = e / d;
  s.c = e % d;
  return s;
}

__device__ inline cplx* slice_ptr(const Prob& P, const SliceIdx& s, int n, cplx* ret, cplx* les,
                                  cplx* tv) {
  int d = P.d, dd = d * d;
  if (s.comp == 0) return ret + (tri(n) + s.j) * dd + s.a * d + s.c;
  if (s.comp == 1) return les + (tri(n) + s.j) * dd + s.a * d + s.c;
  return tv + ((size_t)n * (P.ntau + 1) + s.j) * dd + s.a * d + s.c;
}

// ------------------------------------------------------------ Sigma 2B
// Sigma_ab(z,z') = U(z) U(z') G_ab(z,z')^2 G_ba(z',z) (Eq. sigma_hubb_2b):
//   Sigma^<_ab(j,n) = U_j U_n (L_{j,n}[a,b])^2 G^>_ba(n,j)
//   Sigma^R_ab(n,j) = Sigma^>_ab(n,j) - Sigma^<_ab(n,j)
//   Sigma^rceil_ab(n,m) = U_n U_{-1} (T_{n,m}[a,b])^2 G^lceil_ba(m,n)
//   Sigma^M_ab(m) = -xi U_{-1}^2 (M_m[a,b])^2 M_{ntau-m}[b,a]
// with G^>(t_n,t_j) = G^R + G^< (t_n >= t_j), G^<(t_n,t_j) = -[G^<(t_j,t_n)]^dag.
__global__ __launch_bounds__(NT2) void k_sigma2b(ProbArg pa, int n, double nbar) {
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  if (n > P.nt) return;
  int d = P.d, dd = d * d, ntau = P.ntau;
  const double* u = P.U;
  double xi = P.sig;
  long idx = (long)blockIdx.x * NT2 + threadIdx.x;
  if (n == -1) {
    if (idx < (long)(ntau + 1) * dd) {
      int m = idx / dd, e = idx % dd, a = e / d, c = e % d;
      cplx x = P.Gmat[(size_t)m * dd + e], y = P.Gmat[(size_t)(ntau - m) * dd + c * d + a];
      P.Smat[(size_t)m * dd + e] = (-xi * u[0] * u[0]) * (x * x * y);
    }
  } else {
    long total = (long)(2 * (n + 1) + ntau + 1) * dd;
    if (idx < total) {
      SliceIdx s = slice_idx(idx, n, ntau, d);
      int a = s.a, b = s.c, j = s.j;
      if (s.comp == 2) {
        cplx x = P.Gtv[((size_t)n * (ntau + 1) + j) * dd + a * d + b];
        cplx vt = -xi * conj(P.Gtv[((size_t)n * (ntau + 1) + ntau - j) * dd + a * d + b]);
        P.Stv[((size_t)n * (ntau + 1) + j) * dd + a * d + b] = (u[n + 1] * u[0]) * (x * x * vt);
      } else {
        double uu = u[n + 1] * u[j + 1];
        const cplx* R = P.Gret + (tri(n) + j) * dd;
        const cplx* L = P.Gles + (tri(n) + j) * dd;
        cplx Lab = L[a * d + b], Lba = L[b * d + a], Rab = R[a * d + b], Rba = R[b * d + a];
        if (s.comp == 1) {
          cplx gtr_ba_nj = Rba - conj(Lab);
          P.Sles[(tri(n) + j) * dd + a * d + b] = uu * (Lab * Lab * gtr_ba_nj);
        } else {
          cplx gtr_ab_nj = Rab - conj(Lba);
          cplx les_ab_nj = -conj(Lba);
          cplx gtr_ba_jn = Lba - conj(Rab);
          cplx sg = gtr_ab_nj * gtr_ab_nj * Lba;
          cplx sl = les_ab_nj * les_ab_nj * gtr_ba_jn;
          P.Sret[(tri(n) + j) * dd + a * d + b] = uu * (sg - sl);
        }
      }
    }
  }
  // Hartree mean field from the density matrix rho = i xi G^<(t,t)
  // (rho = -G^M(beta^-) on the Matsubara branch)
  if (P.eps_mf != nullptr && blockIdx.x == 0 && threadIdx.x < dd) {
    int e = threadIdx.x, a = e / d, c = e % d;
    const cplx* e0 = P.eps0 + (size_t)(n + 1) * dd;
    cplx v = e0[e];
    if (a == c) {
      double rho;
      if (n == -1) rho = -P.Gmat[(size_t)ntau * dd + a * d + a].x;
      else {
        cplx l = P.Gles[(tri(n) + n) * dd + a * d + a];
        rho = -xi * l.y;
      }
      v.x += u[n + 1] * (rho - nbar);
    }
    P.eps_mf[(size_t)(n + 1) * dd + e] = v;
  }
}

hipError_t launch_sigma2b(const ProbArg& pa, int n, int d, int nmax_elems, double nbar,
                          hipStream_t s) {
  dim3 g((nmax_elems + NT2 - 1) / NT2, pa.count);
  k_sigma2b<<<g, NT2, 0, s>>>(pa, n, nbar);
  return hipGetLastError();
}

// --------------------------------------------------------- extrapolation
// Eq. polyextrap: slice n+1 from slices n-k..n; left-mixing along t for every
// tau, retarded columns j <= k along t and the rest along the diagonals
// t - t' = const; lesser rows j <= k along t' and the rest along diagonals.
__global__ __launch_bounds__(NT2) void k_extrapolate(ProbArg pa, int n) {
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n1 = n + 1;
  if (n1 > P.nt) return;
  const KW& W = c_kw[P.k];
  int d = P.d, dd = d * d, ntau = P.ntau, k = P.k;
  long idx = (long)blockIdx.x * NT2 + threadIdx.x;
  long total = (long)(2 * (n1 + 1) + ntau + 1) * dd;
  if (idx >= total) return;
  SliceIdx s = slice_idx(idx, n1, ntau, d);
  int j = s.j, a = s.a, c = s.c;
  cplx acc = mk(0, 0);
  for (int l = 0; l <= k; l++) {
    cplx v;
    if (s.comp == 2) {
      v = P.Gtv[((size_t)(n - l) * (ntau + 1) + j) * dd + a * d + c];
    } else if (s.comp == 0) {
      if (j <= k) {
        int t = n - l;
        v = t >= j ? P.Gret[(tri(t) + j) * dd + a * d + c] : -conj(P.Gret[(tri(j) + t) * dd + c * d + a]);
      } else {
        int jj = n1 - j;  // diagonal offset
        v = P.Gret[(tri(n - l) + n - l - jj) * dd + a * d + c];
      }
    } else {
      if (j <= k) {
        int t = n - l;
        v = j <= t ? P.Gles[(tri(t) + j) * dd + a * d + c] : -conj(P.Gles[(tri(j) + t) * dd + c * d + a]);
      } else {
        v = P.Gles[(tri(n - l) + j - 1 - l) * dd + a * d + c];
      }
    }
    acc = acc + W.ext[l] * v;
  }
  *slice_ptr(P, s, n1, P.Gret, P.Gles, P.Gtv) = acc;
}

hipError_t launch_extrapolate(const ProbArg& pa, int n, int d, int nelems, hipStream_t s) {
  dim3 g((nelems + NT2 - 1) / NT2, pa.count);
  k_extrapolate<<<g, NT2, 0, s>>>(pa, n);
  return hipGetLastError();
}

// ------------------------------------------------------- distance / copy
__global__ __launch_bounds__(NT2) void k_distance(ProbArg pa, ProbArg pb, int n, double* out) {
  __shared__ double r0[NT2], r1[NT2];
  int pi = blockIdx.y;
  const Prob& A = pa.get(pi);
  const Prob& B = pb.get(pi);
  int d = A.d, dd = d * d, ntau = A.ntau;
  long idx = (long)blockIdx.x * NT2 + threadIdx.x;
  double s0 = 0, s1 = 0;
  if (n == -1) {
    if (idx < (long)(ntau + 1) * dd) {
      cplx x = A.Gmat[idx], y = B.Gmat[idx];
      s0 = sqrt(abs2(x - y));
      s1 = sqrt(abs2(x));
    }
  } else if (n <= A.nt) {
    long total = (long)(2 * (n + 1) + ntau + 1) * dd;
    if (idx < total) {
      SliceIdx s = slice_idx(idx, n, ntau, d);
      cplx x = *slice_ptr(A, s, n, A.Gret, A.Gles, A.Gtv);
      cplx y = *slice_ptr(B, s, n, B.Gret, B.Gles, B.Gtv);
      s0 = sqrt(abs2(x - y));
      s1 = sqrt(abs2(x));
    }
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int w = NT2 / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out[2 * pi], r0[0]);
    atomicAdd(&out[2 * pi + 1], r1[0]);
  }
}

hipError_t launch_distance(const ProbArg& pa, const ProbArg& pb, int n, int d, int nelems,
                           double* out_dev, hipStream_t s) {
  dim3 g((nelems + NT2 - 1) / NT2, pa.count);
  k_distance<<<g, NT2, 0, s>>>(pa, pb, n, out_dev);
  return hipGetLastError();
}

__global__ __launch_bounds__(NT2) void k_copy(ProbArg pd, ProbArg ps, int n) {
  int pi = blockIdx.y;
  const Prob& D = pd.get(pi);
  const Prob& S = ps.get(pi);
  int d = D.d, dd = d * d, ntau = D.ntau;
  long idx = (long)blockIdx.x * NT2 + threadIdx.x;
  if (n == -1) {
    if (idx < (long)(ntau + 1) * dd) D.Gmat[idx] = S.Gmat[idx];
    return;
  }
  if (n > D.nt) return;
  long total = (long)(2 * (n + 1) + ntau + 1) * dd;
  if (idx >= total) return;
  SliceIdx s = slice_idx(idx, n, ntau, d);
  *slice_ptr(D, s, n, D.Gret, D.Gles, D.Gtv) = *slice_ptr(S, s, n, S.Gret, S.Gles, S.Gtv);
}

// ------------------------------------------------------------ Peierls
// Vector potential as a phase factor in the hopping (Peierls substitution,
// Sec. "Example: GW for the translationally invariant Hubbard model"):
//   eps_n[a][b] = T_n[a][b] exp(i A_n Phi[a][b]),  n = -1..nt (entry n+1),
// with Phi the real phase pattern of the bonds (e.g. +1 / -1 on the two
// directions of a bond, 0 on site energies).
__global__ __launch_bounds__(NT2) void k_peierls(const cplx* T, const double* Phi, const double* A, cplx* eps,
                                                 int dd, long total) {
  long idx = (long)blockIdx.x * NT2 + threadIdx.x;
  if (idx >= total) return;
  int n1 = (int)(idx / dd), e = (int)(idx % dd);
  double sn, cs;
  sincos(A[n1] * Phi[e], &sn, &cs);
  gst(eps + idx, gld(T + idx) * mk(cs, sn));
}

// Chain rule of the substitution for a real objective J with gradient
// eps_bar = dJ/d Re eps + i dJ/d Im eps:
//   A_bar_n += Re sum_ab conj(eps_bar_n[a][b]) i Phi[a][b] eps_n[a][b].
// One wave per time entry, lanes over the d x d elements (d <= 8).
__global__ __launch_bounds__(64) void k_peierls_grad(const cplx* T, const double* Phi, const double* A,
                                                     const cplx* eps_bar, double* A_bar, int dd) {
  int n1 = blockIdx.x, e = threadIdx.x;
  double v = 0.0;
  if (e < dd) {
    long idx = (long)n1 * dd + e;
    double sn, cs;
    sincos(A[n1] * Phi[e], &sn, &cs);
    cplx ep = gld(T + idx) * mk(cs, sn);
    cplx de = mul_i(Phi[e] * ep);  // d eps / d A_n
    cplx g = gld(eps_bar + idx);
    v = g.x * de.x + g.y * de.y;  // Re(conj(g) de)
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (e == 0) A_bar[n1] += v;
}

hipError_t launch_peierls(const cplx* T, const double* Phi, const double* A, cplx* eps, int d, int nt,
                          hipStream_t s) {
  long total = (long)(nt + 2) * d * d;
  k_peierls<<<(unsigned)((total + NT2 - 1) / NT2), NT2, 0, s>>>(T, Phi, A, eps, d * d, total);
  return hipGetLastError();
}

hipError_t launch_peierls_grad(const cplx* T, const double* Phi, const double* A, const cplx* eps_bar,
                               double* A_bar, int d, int nt, hipStream_t s) {
  k_peierls_grad<<<nt + 2, 64, 0, s>>>(T, Phi, A, eps_bar, A_bar, d * d);
  return hipGetLastError();
}

// ------------------------------------------------------------ checks
__device__ inline bool finite_c(cplx v) { return isfinite(v.x) && isfinite(v.y); }

// Finite check of one time step (optional, cntr_set_checks): slice n of G
// (the step's output) and of Sigma, and eps_n; the first non-finite value of
// a problem sets its status word to CNTR_ENONFINITE.
__global__ __launch_bounds__(NT2) void k_check_finite(ProbArg pa, Scratch sc, int n0, int n1) {
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int d = P.d, dd = d * d, ntau = P.ntau;
  bool bad = false;
  for (int n = n0; n <= min(n1, P.nt); n++) {
    long total = (long)(2 * (n + 1) + ntau + 1) * dd;
    for (long idx = (long)blockIdx.x * NT2 + threadIdx.x; idx < total; idx += (long)gridDim.x * NT2) {
      SliceIdx s = slice_idx(idx, n, ntau, d);
      bad = bad || !finite_c(gld(slice_ptr(P, s, n, P.Gret, P.Gles, P.Gtv)));
      bad = bad || !finite_c(gld(slice_ptr(P, s, n, P.Sret, P.Sles, P.Stv)));
    }
    if (blockIdx.x == 0 && threadIdx.x < dd) bad = bad || !finite_c(gld(P.eps + (size_t)(n + 1) * dd + threadIdx.x));
  }
  if (bad) atomicCAS(sc.status(pi), 0, (int)CNTR_ENONFINITE);
}

hipError_t launch_check_finite(const ProbArg& pa, const Scratch& sc, int n0, int n1, int d, int ntau,
                               hipStream_t s) {
  long total = (long)(2 * (n1 + 1) + ntau + 1) * d * d;
  long nb = (total + NT2 - 1) / NT2;
  int blocks = (int)(nb < 64 ? nb : 64);
  dim3 g(blocks, pa.count);
  k_check_finite<<<g, NT2, 0, s>>>(pa, sc, n0, n1);
  return hipGetLastError();
}

// Symmetry check (optional, cntr_set_checks): the self-energy read by a
// start-up or step is a hermitian contour function, so its equal-time
// blocks Sigma^<_{n,n} and Sigma^R_{n,n} are anti-hermitian and Sigma^M(tau)
// is hermitian. One thread per block; a violation sets the problem's status
// word to CNTR_ESYMMETRY.
__global__ __launch_bounds__(NT2) void k_check_symm(ProbArg pa, Scratch sc, int n0, int n1) {
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int d = P.d, dd = d * d, ntau = P.ntau;
  int nreal = n1 >= 0 ? n1 - max(n0, 0) + 1 : 0, nmat = n0 < 0 ? ntau + 1 : 0;
  int v = blockIdx.x * NT2 + threadIdx.x;
  if (v >= 2 * nreal + nmat) return;
  const cplx* X;
  double sgn;  // +1: anti-hermitian, -1: hermitian
  if (v < 2 * nreal) {
    int n = max(n0, 0) + v / 2;
    if (n > P.nt) return;
    X = (v & 1 ? P.Sret : P.Sles) + tri(n) * dd + (size_t)n * dd;
    sgn = 1.0;
  } else {
    X = P.Smat + (size_t)(v - 2 * nreal) * dd;
    sgn = -1.0;
  }
  double dev = 0, mag = 0;
  for (int a = 0; a < d; a++)
    for (int b = 0; b < d; b++) {
      cplx x = gld(X + a * d + b), y = gld(X + b * d + a);
      cplx s = x + sgn * conj(y);
      dev = fmax(dev, fmax(fabs(s.x), fabs(s.y)));
      mag = fmax(mag, fmax(fabs(x.x), fabs(x.y)));
    }
  if (!(dev <= 1e-10 * mag)) atomicCAS(sc.status(pi), 0, (int)CNTR_ESYMMETRY);
}

hipError_t launch_check_symmetry(const ProbArg& pa, const Scratch& sc, int n0, int n1, int ntau, hipStream_t s) {
  int nreal = n1 >= 0 ? n1 - (n0 > 0 ? n0 : 0) + 1 : 0, nmat = n0 < 0 ? ntau + 1 : 0;
  dim3 g((2 * nreal + nmat + NT2 - 1) / NT2, pa.count);
  k_check_symm<<<g, NT2, 0, s>>>(pa, sc, n0, n1);
  return hipGetLastError();
}

hipError_t launch_copy(const ProbArg& pdst, const ProbArg& psrc, int n, int d, int nelems,
                       hipStream_t s) {
  dim3 g((nelems + NT2 - 1) / NT2, pdst.count);
  k_copy<<<g, NT2, 0, s>>>(pdst, psrc, n);
  return hipGetLastError();
}

// ----------------------------------------------------------- convolution
// Values outside the stored triangles of X come from its partner Xc.
__device__ inline cplx cv_ret(const Prob& X, const Prob& Xc, int a, int b, int r, int c) {
  int d = X.d, dd = d * d;
  if (a >= b) return X.Gret[(tri(a) + b) * dd + r * d + c];
  return -conj(Xc.Gret[(tri(b) + a) * dd + c * d + r]);
}
__device__ inline cplx cv_les(const Prob& X, const Prob& Xc, int a, int b, int r, int c) {
  int d = X.d, dd = d * d;
  if (a <= b) return X.Gles[(tri(b) + a) * dd + r * d + c];
  return -conj(Xc.Gles[(tri(a) + b) * dd + c * d + r]);
}
// X^A_{a,b}[r][c] = conj([Xc]~^R_{b,a}[c][r])
__device__ inline cplx cv_adv(const Prob& X, const Prob& Xc, int a, int b, int r, int c) {
  return conj(cv_ret(Xc, X, b, a, c, r));
}
// X^lceil(tau_j, t_n)[r][c] = -xi conj(Xc^rceil_{n,ntau-j}[c][r])
__device__ inline cplx cv_vt(const Prob& X, const Prob& Xc, int j, int n, int r, int c) {
  int d = X.d, dd = d * d;
  return (-(double)X.sig) * conj(Xc.Gtv[((size_t)n * (X.ntau + 1) + X.ntau - j) * dd + c * d + r]);
}

// [X f Y][a][c] for blocks given as element accessors; f may be null
template <class FA, class FB>
__device__ inline cplx triple(int d, FA Ael, const cplx* f, FB Bel, int a, int c) {
  cplx s = mk(0, 0);
  if (f == nullptr) {
    for (int q = 0; q < d; q++) cfma(s, Ael(a, q), Bel(q, c));
    return s;
  }
  for (int q = 0; q < d; q++) {
    cplx af = mk(0, 0);
    for (int p = 0; p < d; p++) cfma(af, Ael(a, p), f[p * d + q]);
    cfma(s, af, Bel(q, c));
  }
  return s;
}

__device__ inline const cplx* fat(const cplx* f, int t, int d) {
  return f == nullptr ? nullptr : f + (size_t)(t + 1) * d * d;
}

// Terms of one output element split over GC consecutive lanes (term index
// = lane mod GC), summed with shuffles in a fixed order: the sums over the
// n + Ntau terms of a slice would otherwise run serially in one thread.
constexpr int GC = 16;
__device__ cplx mat_conv_part(const Prob& P, const cplx* A, const cplx* B, const cplx* f, int m, int a, int c,
                              int g);

__device__ inline cplx conv_part(const Prob& C, const Prob& A, const Prob& Ac, const Prob& B, const Prob& Bc,
                                 int n, const SliceIdx& s, int g) {
  const cplx* f = C.f;
  const KW& W = c_kw[C.k];
  int d = C.d, dd = d * d, ntau = C.ntau, k = C.k, K1 = k + 1;
  double h = C.h, ht = C.htau;
  int a = s.a, c = s.c, m = s.j;
  cplx acc = mk(0, 0);
  if (s.comp == 0) {  // Eq. cr1, C^R(t_n, t_m)
    if (n > k && n - m > k) {
      for (int j = m + g; j <= n; j += GC)
        acc = acc + (h * greg(W, n - m, j - m)) *
                        triple(d, [&](int x, int y) { return A.Gret[(tri(n) + j) * dd + x * d + y]; },
                               fat(f, j, d), [&](int x, int y) { return B.Gret[(tri(j) + m) * dd + x * d + y]; }, a, c);
    } else if (n > k) {
      for (int j = g; j <= k; j += GC)
        acc = acc + (h * greg(W, n - m, j)) *
                        triple(d, [&](int x, int y) { return A.Gret[(tri(n) + n - j) * dd + x * d + y]; },
                               fat(f, n - j, d), [&](int x, int y) { return cv_ret(B, Bc, n - j, m, x, y); }, a, c);
    } else {
      for (int j = g; j <= k; j += GC)
        acc = acc + (h * W.I[m][n][j]) *
                        triple(d, [&](int x, int y) { return cv_ret(A, Ac, n, j, x, y); }, fat(f, j, d),
                               [&](int x, int y) { return cv_ret(B, Bc, j, m, x, y); }, a, c);
    }
  } else if (s.comp == 2) {  // Eqs. ctv1 + ctv2 + ctv3, C^rceil(t_n, tau_m)
    const cplx* fm = fat(f, -1, d);
    auto pr = [&](int la, int lb) {
      return triple(d, [&](int x, int y) { return A.Gtv[((size_t)n * (ntau + 1) + la) * dd + x * d + y]; }, fm,
                    [&](int x, int y) { return B.Gmat[(size_t)lb * dd + x * d + y]; }, a, c);
    };
    double xi = C.sig;
    if (m <= k) {
      for (int t = g; t < K1 * K1; t += GC) {
        int j = t / K1, l = t % K1;
        acc = acc + (ht * xi * W.R[m][j][l]) * pr(l, ntau - j);
      }
    } else {
      for (int l = g; l <= m; l += GC) acc = acc + (ht * xi * greg(W, m, l)) * pr(m - l, ntau - l);
    }
    if (m >= ntau - k) {
      for (int t = g; t < K1 * K1; t += GC) {
        int j = t / K1, l = t % K1;
        acc = acc + (ht * W.R[ntau - m][j][l]) * pr(ntau - l, j);
      }
    } else {
      for (int l = g; l <= ntau - m; l += GC) acc = acc + (ht * greg(W, ntau - m, l)) * pr(m + l, l);
    }
    int jmax = n > k ? n : k;
    for (int j = g; j <= jmax; j += GC) {
      double w = n > k ? greg(W, n, j) : W.s[n][j];
      acc = acc + (h * w) * triple(d, [&](int x, int y) { return cv_ret(A, Ac, n, j, x, y); }, fat(f, j, d),
                                   [&](int x, int y) { return B.Gtv[((size_t)j * (ntau + 1) + m) * dd + x * d + y]; },
                                   a, c);
    }
  } else {  // C^<(t_m, t_n): Eqs. cles1 + cles2 + cles3
    int j1 = m > k ? m : k;
    for (int j = g; j <= j1; j += GC) {
      double w = m > k ? greg(W, m, j) : W.s[m][j];
      acc = acc + (h * w) * triple(d, [&](int x, int y) { return cv_ret(A, Ac, m, j, x, y); }, fat(f, j, d),
                                   [&](int x, int y) { return cv_les(B, Bc, j, n, x, y); }, a, c);
    }
    int j2 = n > k ? n : k;
    for (int j = g; j <= j2; j += GC) {
      double w = n > k ? greg(W, n, j) : W.s[n][j];
      acc = acc + (h * w) * triple(d, [&](int x, int y) { return cv_les(A, Ac, m, j, x, y); }, fat(f, j, d),
                                   [&](int x, int y) { return cv_adv(B, Bc, j, n, x, y); }, a, c);
    }
    const cplx* fm = fat(f, -1, d);
    cplx s3 = mk(0, 0);
    for (int j = g; j <= ntau; j += GC)
      s3 = s3 + (ht * greg(W, ntau, j)) *
                    triple(d, [&](int x, int y) { return A.Gtv[((size_t)m * (ntau + 1) + j) * dd + x * d + y]; }, fm,
                           [&](int x, int y) { return cv_vt(B, Bc, j, n, x, y); }, a, c);
    acc = acc - mul_i(s3);
  }
  return acc;
}

__global__ __launch_bounds__(NT2) void k_convolution(ProbArg pc, ProbArg pa, ProbArg pac,
                                                     ProbArg pb, ProbArg pbc, int n) {
  int pi = blockIdx.y;
  const Prob& C = pc.get(pi);
  const Prob& A = pa.get(pi);
  const Prob& Ac = pac.get(pi);
  const Prob& B = pb.get(pi);
  const Prob& Bc = pbc.get(pi);
  int d = C.d, dd = d * d, ntau = C.ntau;
  long gidx = (long)blockIdx.x * NT2 + threadIdx.x;
  long idx = gidx / GC;
  int g = (int)(gidx % GC);
  if (n > C.nt) return;  // (uniform over the workgroup)
  long total = n == -1 ? (long)(ntau + 1) * dd : (long)(2 * (n + 1) + ntau + 1) * dd;
  bool valid = idx < total;
  cplx acc = mk(0, 0);
  SliceIdx s{};
  if (valid) {
    if (n == -1) {
      int m = idx / dd, e = idx % dd;
      acc = mat_conv_part(C, A.Gmat, B.Gmat, C.f, m, e / d, e % d, g);
    } else {
      s = slice_idx(idx, n, ntau, d);
      acc = conv_part(C, A, Ac, B, Bc, n, s, g);
    }
  }
  for (int off = 1; off < GC; off <<= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  if (!valid || g != 0) return;
  if (n == -1) C.Gmat[idx] = acc;
  else *slice_ptr(C, s, n, C.Gret, C.Gles, C.Gtv) = acc;
}

// --------------------------------------------------------- local Sigma
// Sigma = lam * (1/count) sum_i G_i on slice n of every component (n = -1: the
// Matsubara component): a self-energy local in the batch index, e.g. the
// k-point average G_loc of a lattice. Fixed summation order over i.
// Pointer sources: the batch (pa, count >= 1) supplies the G_i; the output is
// the Sigma of problem 0.
// One workgroup: 64 elements x 16 waves; wave w sums its sixteenth of the
// instances (sixteen loads in flight), the sixteenths are added in order.
constexpr int NSL = 1024, NSLW = NSL / 64;
__global__ __launch_bounds__(NSL) void k_sigma_local(ProbArg pa, int n, double lam) {
  constexpr int NBAT = 512;  // instances whose pointers are staged at once
  __shared__ const cplx* base[NBAT];
  __shared__ cplx qs[NSLW][64];
  const Prob& P0 = pa.get(0);
  int d = P0.d, dd = d * d, ntau = P0.ntau, cnt = pa.count;
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long idx = (long)blockIdx.x * 64 + lane;
  double w = lam / cnt;
  // component and offset of this element (identical in every instance)
  int comp;  // 0 ret, 1 les, 2 tv, 3 mat
  size_t off;
  bool valid;
  if (n == -1) {
    comp = 3;
    off = idx;
    valid = idx < (long)(ntau + 1) * dd;
  } else {
    long total = (long)(2 * (n + 1) + ntau + 1) * dd;
    valid = idx < total;
    SliceIdx sl = slice_idx(valid ? idx : 0, n, ntau, d);
    comp = sl.comp;
    off = comp == 2 ? ((size_t)n * (ntau + 1) + sl.j) * dd + sl.a * d + sl.c
                    : (tri(n) + sl.j) * dd + sl.a * d + sl.c;
  }
  cplx s = mk(0, 0);
  for (int i0 = 0; i0 < cnt; i0 += NBAT) {
    int nb = min(NBAT, cnt - i0);
    int lo = wave * nb / NSLW, hi = (wave + 1) * nb / NSLW;
    for (int c = 0; c < 4; c++) {
      // stage component c's pointers only if some element of the block needs them
      bool need = __syncthreads_or(valid && comp == c);
      if (!need) continue;
      for (int i = threadIdx.x; i < nb; i += NSL) {
        const Prob& P = pa.get(i0 + i);
        base[i] = c == 0 ? P.Gret : c == 1 ? P.Gles : c == 2 ? P.Gtv : P.Gmat;
      }
      __syncthreads();
      if (valid && comp == c) {
        int i = lo;
        for (; i + 16 <= hi; i += 16) {
          cplx v[16];
#pragma unroll
          for (int u = 0; u < 16; u++) v[u] = gld(base[i + u] + off);
#pragma unroll
          for (int u = 0; u < 16; u++) s = s + v[u];
        }
        for (; i < hi; i++) s = s + gld(base[i] + off);
      }
    }
  }
  qs[wave][lane] = s;
  __syncthreads();
  if (wave != 0 || !valid) return;
  cplx r = qs[0][lane];
  for (int q = 1; q < NSLW; q++) r = r + qs[q][lane];
  r = w * r;
  if (comp == 3) P0.Smat[off] = r;
  else if (comp == 0) P0.Sret[off] = r;
  else if (comp == 1) P0.Sles[off] = r;
  else P0.Stv[off] = r;
}

hipError_t launch_sigma_local(const ProbArg& pa, int n, int d, int nelems, double lam, hipStream_t s) {
  dim3 g((nelems + 63) / 64, 1);
  k_sigma_local<<<g, NSL, 0, s>>>(pa, n, lam);
  return hipGetLastError();
}


// ------------------------------------------------------------ observables
// Observables of slice n (per spin; Eq. Total_ener and the density matrix):
//   rho = i xi G^<(t_n, t_n)
//   out[0] = Re Tr rho                     particle number
//   out[1] = Re Tr[rho eps0_n]             one-body energy
//   out[2] = Re Tr[rho eps_mf_n]           one-body energy with the mean field
//   out[3] = 1/2 Im Tr[Sigma * G]^<(t_n, t_n)   correlation energy
//   out[4] = (out[1] + out[2]) / 2 + out[3]      Galitskii-Migdal total energy
// [Sigma * G]^<(n,n) from the three parts of Eqs. cles1-cles3 at m = n.
// One workgroup per problem: thread (element e, group g) sums the terms
// j = g, g + G, ... of every part; the groups are added in a fixed order.
__global__ __launch_bounds__(NT2) void k_observables(ProbArg pa, int n, double* out, cplx* rho_out) {
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int d = P.d, dd = d * d, ntau = P.ntau, k = P.k;
  double h = P.h, ht = P.htau, xi = P.sig;
  int tid = threadIdx.x, NG = NT2 / dd, e = tid % dd, g = tid / dd;
  int a = e / d, c = e % d;
  __shared__ cplx red[NT2];
  __shared__ cplx cl[64], rh[64];
  cplx acc = mk(0, 0);
  if (g < NG) {
    int jmax = n > k ? n : k;
    auto wt = [&](int j) { return n > k ? greg(W, n, j) : W.s[n][j]; };
    // part 1: h w(n,j) Sigma~^R_{n,j} G^<_{j,n}
    for (int j = g; j <= jmax; j += NG) {
      cplx t = mk(0, 0);
      for (int q = 0; q < d; q++)
        cfma(t, ret_ext_d(P.Sret, n, j, a, q, d), les_any_d(P.Gles, j, n, q, c, d));
      acc = acc + (h * wt(j)) * t;
    }
    // part 2: h w(n,j) Sigma^<_{n,j} G^A_{j,n},  G^A_{j,n}[q][c] = conj(G~^R_{n,j}[c][q])
    for (int j = g; j <= jmax; j += NG) {
      cplx t = mk(0, 0);
      for (int q = 0; q < d; q++)
        cfma(t, les_any_d(P.Sles, n, j, a, q, d), conj(ret_ext_d(P.Gret, n, j, c, q, d)));
      acc = acc + (h * wt(j)) * t;
    }
    // part 3: -i h_tau w(ntau,j) Sigma^rceil_{n,j} G^lceil_{j,n},
    //         G^lceil_{j,n}[q][c] = -xi conj(T_{n,ntau-j}[c][q])
    cplx s3 = mk(0, 0);
    for (int j = g; j <= ntau; j += NG) {
      cplx t = mk(0, 0);
      const cplx* sb = P.Stv + ((size_t)n * (ntau + 1) + j) * dd;
      const cplx* gb = P.Gtv + ((size_t)n * (ntau + 1) + ntau - j) * dd;
      for (int q = 0; q < d; q++) cfma(t, sb[a * d + q], -xi * conj(gb[c * d + q]));
      s3 = s3 + (ht * greg(W, ntau, j)) * t;
    }
    acc = acc - mul_i(s3);
  }
  red[tid] = acc;
  __syncthreads();
  if (tid < dd) {
    cplx sum = mk(0, 0);
    for (int gg = 0; gg < NG; gg++) sum = sum + red[gg * dd + tid];
    cl[tid] = sum;
    rh[tid] = mul_i(xi * P.Gles[(tri(n) + n) * dd + tid]);
  }
  __syncthreads();
  if (tid == 0) {
    const cplx* e0 = P.eps0 + (size_t)(n + 1) * dd;
    const cplx* em = (P.eps_mf ? P.eps_mf : P.eps0) + (size_t)(n + 1) * dd;
    double N = 0, E1 = 0, Em = 0, Ec = 0;
    for (int i = 0; i < d; i++) {
      N += rh[i * d + i].x;
      Ec += cl[i * d + i].y;
      for (int q = 0; q < d; q++) {
        E1 += (rh[i * d + q] * e0[q * d + i]).x;
        Em += (rh[i * d + q] * em[q * d + i]).x;
      }
    }
    double* o = out + (size_t)pi * 5;
    o[0] = N;
    o[1] = E1;
    o[2] = Em;
    o[3] = 0.5 * Ec;
    o[4] = 0.5 * (E1 + Em) + 0.5 * Ec;
  }
  if (rho_out && tid < dd) rho_out[(size_t)pi * dd + tid] = rh[tid];
}

hipError_t launch_observables(const ProbArg& pa, int n, double* out, cplx* rho, hipStream_t s) {
  dim3 g(1, pa.count);
  k_observables<<<g, NT2, 0, s>>>(pa, n, out, rho);
  return hipGetLastError();
}

hipError_t launch_convolution(const ProbArg& C, const ProbArg& A, const ProbArg& Acc,
                              const ProbArg& B, const ProbArg& Bcc, int n, int d, int nelems,
                              hipStream_t s) {
  dim3 g((unsigned)(((long)nelems * GC + NT2 - 1) / NT2), C.count);
  k_convolution<<<g, NT2, 0, s>>>(C, A, Acc, B, Bcc, n);
  return hipGetLastError();
}

}  // namespace cntr

namespace cntr {

// Matsubara convolution with the terms of an element split over GM = 16
// consecutive lanes (term index = lane mod 16), summed with shuffles in a
// fixed order.
constexpr int GM = GC;  // (the same lane groups as k_convolution)
__device__ cplx mat_conv_part(const Prob& P, const cplx* A, const cplx* B, const cplx* f, int m, int a,
                              int c, int g) {
  const KW& W = c_kw[P.k];
  int d = P.d, dd = d * d, k = P.k, nt = P.ntau;
  double ht = P.htau, xi = P.sig;
  const cplx* fm = fat(f, -1, d);
  cplx acc = mk(0, 0);
  auto pr = [&](int ia, int ib) {
    return triple(d, [&](int x, int y) { return A[(size_t)ia * dd + x * d + y]; }, fm,
                  [&](int x, int y) { return B[(size_t)ib * dd + x * d + y]; }, a, c);
  };
  int K1 = k + 1;
  if (m <= k) {
    for (int t = g; t < K1 * K1; t += GM) {
      int j = t / K1, l = t % K1;
      acc = acc + (ht * W.R[m][j][l]) * pr(j, l);
    }
  } else {
    for (int l = g; l <= m; l += GM) acc = acc + (ht * greg(W, m, l)) * pr(m - l, l);
  }
  if (m >= nt - k) {
    for (int t = g; t < K1 * K1; t += GM) {
      int j = t / K1, l = t % K1;
      acc = acc + (ht * xi * W.R[nt - m][j][l]) * pr(nt - j, nt - l);
    }
  } else {
    for (int l = g; l <= nt - m; l += GM) acc = acc + (ht * xi * greg(W, nt - m, l)) * pr(nt - l, m + l);
  }
  return acc;
}

__global__ __launch_bounds__(NT2) void k_mat_conv(Prob P, const cplx* A, const cplx* B, const cplx* f,
                                                  cplx* out) {
  int d = P.d, dd = d * d;
  long gidx = (long)blockIdx.x * NT2 + threadIdx.x;
  long idx = gidx / GM;
  int g = (int)(gidx % GM);
  bool valid = idx < (long)(P.ntau + 1) * dd;
  cplx acc = mk(0, 0);
  if (valid) {
    int m = idx / dd, e = idx % dd;
    acc = mat_conv_part(P, A, B, f, m, e / d, e % d, g);
  }
  for (int off = 1; off < GM; off <<= 1) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
  }
  if (valid && g == 0) out[idx] = acc;
}

hipError_t launch_mat_conv(const Prob& P, const cplx* A, const cplx* B, const cplx* f, cplx* out,
                           hipStream_t s) {
  long tot = (long)(P.ntau + 1) * P.d * P.d * GM;
  k_mat_conv<<<(unsigned)((tot + NT2 - 1) / NT2), NT2, 0, s>>>(P, A, B, f, out);
  return hipGetLastError();
}

}  // namespace cntr
