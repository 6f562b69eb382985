// Pieces of the Holstein-model DMFT with the unrenormalized Migdal impurity
// solver (Sec. "DMFT for the Holstein model") on gfx950, single band (d = 1):
//   k_phonon_free:  D0(z,z') = -i <T_C X(z) X(z')>_0 of one mode X = a + a^dag of
//                   frequency w0 at inverse temperature beta, every component in
//                   closed form (bosonic grid);
//   k_scale_slice:  C = beta C + f(t) A(t,t') f(t') on one slice (any d): the
//                   Bethe-lattice hybridization Delta = J G J (Eq. bethe_condition),
//                   the coupled propagator g D0 g of the uMig self-energy (Eq.
//                   uMig_el), and sums of slices;
//   k_holstein_mf:  the phonon displacement X(t_n) of Eq. X and the mean-field
//                   level e0 + g(t_n) X(t_n) (Eq. H_mf_Holstein).
// Time-dependent real scalars (f, g, X) hold nt + 2 entries: entry n + 1 at
// t_n, entry 0 on the Matsubara branch.
#include "launch.h"

namespace cntr {

constexpr int NTH = 256;

__device__ inline void tri_index(long idx, int& n, int& j) {
  int r = (int)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
  while ((long)tri(r + 1) <= idx) r++;
  while ((long)tri(r) > idx) r--;
  n = r;
  j = (int)(idx - (long)tri(r));
}

// D0 of X = a + a^dag with b = 1 / (1 - e^{-beta w0}) = 1 + nB:
//   R(t,t')   = -2 sin(w0 (t - t'))
//   <(t,t')   = -i [(1 + nB) e^{i w0 (t - t')} + nB e^{-i w0 (t - t')}]
//   rceil(t,tau) = -i [(1 + nB) e^{i w0 t - w0 tau} + nB e^{-i w0 t + w0 tau}]
//   M(tau)    = -[(1 + nB) e^{-w0 tau} + nB e^{w0 tau}]
// (nB e^{w0 tau} = b e^{-w0 (beta - tau)}, finite at large beta w0)
__global__ __launch_bounds__(NTH) void k_phonon_free(ProbArg pa) {
  const Prob& P = pa.get(blockIdx.y);
  const int nt = P.nt, ntau = P.ntau;
  const long nm = ntau + 1, ntr = (long)tri(nt + 1), nall = nm + 2 * ntr + (long)(nt + 1) * (ntau + 1);
  long idx = (long)blockIdx.x * NTH + threadIdx.x;
  if (idx >= nall) return;
  const double w0 = P.par, beta = P.beta, h = P.h, htau = beta / ntau;
  const double b = 1.0 / (-expm1(-beta * w0));
  if (idx < nm) {
    double tau = idx * htau;
    P.Gmat[idx] = mk(-b * (exp(-w0 * tau) + exp(-w0 * (beta - tau))), 0.0);
    return;
  }
  idx -= nm;
  if (idx < ntr) {
    int n, j;
    tri_index(idx, n, j);
    P.Gret[idx] = mk(-2.0 * sin(w0 * (n - j) * h), 0.0);
    return;
  }
  idx -= ntr;
  if (idx < ntr) {
    int n, j;
    tri_index(idx, n, j);  // L_{j,n} = D0^<(t_j, t_n)
    double s, c;
    sincos(w0 * (j - n) * h, &s, &c);
    double nb = b - 1.0;
    // -i [(1 + nB)(c + i s) + nB (c - i s)]
    double re = b * s - nb * s, im = -(b * c + nb * c);
    P.Gles[idx] = mk(re, im);
    return;
  }
  idx -= ntr;
  int n = (int)(idx / (ntau + 1)), m = (int)(idx % (ntau + 1));
  double tau = m * htau, s, c;
  sincos(w0 * n * h, &s, &c);
  double e1 = b * exp(-w0 * tau), e2 = b * exp(-w0 * (beta - tau));
  // -i [e1 (c + i s) + e2 (c - i s)]
  P.Gtv[idx] = mk(e1 * s - e2 * s, -(e1 * c + e2 * c));
}

hipError_t launch_phonon_free(const ProbArg& pa, int nt_max, int ntau, hipStream_t s) {
  long nall = (ntau + 1) + 2 * (long)tri(nt_max + 1) + (long)(nt_max + 1) * (ntau + 1);
  dim3 g((unsigned)((nall + NTH - 1) / NTH), (unsigned)pa.count);
  k_phonon_free<<<g, NTH, 0, s>>>(pa);
  return hipGetLastError();
}

// C = beta C + f(t) A(t,t') f(t') on slice n (every problem shares n, d and
// ntau); f = the C descriptor's real series U
__global__ __launch_bounds__(NTH) void k_scale_slice(ProbArg pc, ProbArg pa, int n, double beta) {
  const Prob& C = pc.get(blockIdx.y);
  const Prob& A = pa.get(blockIdx.y);
  const int d = C.d, dd = d * d, ntau = C.ntau;
  const double* f = C.U;
  long idx = (long)blockIdx.x * NTH + threadIdx.x;
  const cplx *src;
  cplx* dst;
  double fa, fb;
  long e = idx % dd, b = idx / dd;
  if (n == -1) {
    if (b > ntau) return;
    src = A.Gmat + b * dd + e;
    dst = C.Gmat + b * dd + e;
    fa = fb = f[0];
  } else if (b <= n) {  // R(n, b)
    src = A.Gret + (tri(n) + b) * dd + e;
    dst = C.Gret + (tri(n) + b) * dd + e;
    fa = f[n + 1];
    fb = f[b + 1];
  } else if (b <= 2 * n + 1) {  // L(j, n), j = b - n - 1
    long j = b - n - 1;
    src = A.Gles + (tri(n) + j) * dd + e;
    dst = C.Gles + (tri(n) + j) * dd + e;
    fa = f[j + 1];
    fb = f[n + 1];
  } else {  // T(n, m)
    long m = b - 2 * n - 2;
    if (m > ntau) return;
    src = A.Gtv + ((long)n * (ntau + 1) + m) * dd + e;
    dst = C.Gtv + ((long)n * (ntau + 1) + m) * dd + e;
    fa = f[n + 1];
    fb = f[0];
  }
  cplx v = (fa * fb) * gld(src);
  if (beta != 0.0) v = v + beta * gld(dst);
  gst(dst, v);
}

hipError_t launch_scale_slice(const ProbArg& pc, const ProbArg& pa, int n, int d, int ntau, double beta,
                              hipStream_t s) {
  long nel = (n == -1 ? (long)(ntau + 1) : (long)(2 * (n + 1) + ntau + 1)) * d * d;
  dim3 g((unsigned)((nel + NTH - 1) / NTH), (unsigned)pc.count);
  k_scale_slice<<<g, NTH, 0, s>>>(pc, pa, n, beta);
  return hipGetLastError();
}

// X(t_n) by Eq. X with the library's quadrature of order k on [0, t_n] (the
// start weights over the points 0..k for n <= k, the Gregory weights beyond),
// D0^R(t,s) = -2 sin(w0 (t - s)) and n(t_j) = 2 Im G^<(t_j,t_j); n = -1: the
// equilibrium value -2 g(0^-) n / w0 with n = -2 G^M(beta). One wave per
// problem: lane l sums the terms j = l, l + 64, ... in order, the lanes'
// sums are combined in a fixed order. Writes X (the aux series) at n + 1 and
// the level e0 + g X into eps_mf at n + 1; g is the real series U, w0 the
// parameter par.
__global__ __launch_bounds__(64) void k_holstein_mf(ProbArg pg, int n, double e0) {
  const Prob& P = pg.get(blockIdx.x);
  const double* gel = P.U;
  const double w0 = P.par;
  const int lane = threadIdx.x;
  double X;
  if (n == -1) {
    double dens = -2.0 * gld(P.Gmat + P.ntau).x;
    X = -2.0 * gel[0] * dens / w0;
  } else {
    const KW& W = c_kw[P.k];
    const double n0 = 2.0 * gld(P.Gles).y;
    const double src0 = gel[1] * n0;
    const int top = n > P.k ? n : P.k;
    double acc = 0.0;
    for (int j = lane; j <= top; j += 64) {
      double w = greg(W, n, j);
      double dens = 2.0 * gld(P.Gles + tri(j) + j).y;
      acc += w * (-2.0 * sin(w0 * (n - j) * P.h)) * (gel[j + 1] * dens - src0);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_down(acc, off);
    X = -2.0 * gel[1] * n0 / w0 + P.h * acc;
  }
  if (lane == 0) {
    int at = n + 1;
    P.aux[at] = X;
    P.eps_mf[at] = mk(e0 + gel[at] * X, 0.0);
  }
}

hipError_t launch_holstein_mf(const ProbArg& pg, int n, double e0, hipStream_t s) {
  k_holstein_mf<<<pg.count, 64, 0, s>>>(pg, n, e0);
  return hipGetLastError();
}

}  // namespace cntr
