// Free Green's function of a time-dependent single-particle Hamiltonian
// (Sec. "Implementation: Free Green's functions"). The propagator U_{n+1,n}
// is the fourth-order commutator-free exponential of Eq. cf4, with eps at the
// two intermediate times from the polynomial through the k+1 grid points
// n-k+1 .. n+1 (0 .. k near the start); U_{n,0} follows from the semigroup
// property, and every real-time and mixed block from Eq. G0_free:
//   G^R(t_n,t_j) = -i U_n U_j^dag,  G^<(t_j,t_n) = -i xi U_j rho U_n^dag,
//   G^rceil(t_n,tau) = -i xi U_n R diag(f(x) e^{x tau}) R^dag,
// with eps(0^-) - mu = R diag(x) R^dag, f(x) = 1/(e^{beta x} - xi) and
// rho = R diag(f(x)) R^dag (U_n = U_{n,0}). The exponents of Eq. cf4 carry
// the step h, and the real-time Hamiltonian is eps(t) - mu, as in the Dyson
// equations of this library (for mu = 0 the printed form).
//
// Kernels (one problem per launch; d <= 8, so a d x d block fits one wave
// with one element per lane):
//   k_cf4_steps : the step propagators, one wave per factor of Eq. cf4
//                 (Taylor series with scaling and squaring);
//   k_cf4_local : their products within chunks of CF_CH steps;
//   k_cf4_carry : the products across chunks (one wave) and, meanwhile, the
//                 eigenvectors of eps(0^-) - mu with rho;
//   k_cf4_rows  : U_n and W_n = U_n rho (one thread per block row), the
//                 mixed factors F_m = R diag(f(x) e^{x tau_m}) R^dag and G^M;
//   k_free_write: every block of G^R, G^< and G^rceil (one thread per
//                 element, operands staged in LDS; the write of the whole
//                 function bounds it).
#include "launch.h"

namespace cntr {

constexpr int CF_CH = 32;   // steps per chunk of the propagator products
constexpr int CF_NT = 256;  // threads per workgroup (4 waves)
constexpr int CF_TAYLOR = 16;

// scratch of one problem (in cplx units): local products / U (nt+1), W
// (nt+1), F (ntau+1), carries (nch), rho, R (d x d each), x (d doubles)
struct FreeScratch {
  cplx *loc, *U, *W, *F, *carry, *rho, *R;
  double* x;
};

__host__ __device__ inline size_t free_scratch_elems(int nt, int ntau, int d) {
  size_t dd = (size_t)d * d;
  int nch = (nt + CF_CH - 1) / CF_CH + 1;
  return dd * (3 * (size_t)(nt + 1) + (ntau + 1) + nch + 2) + 8;
}

// Z = X Y for d x d blocks in LDS, one element per lane (lanes >= d^2 idle);
// Z may alias X or Y.
__device__ inline void wave_prod(int d, const cplx* X, const cplx* Y, cplx* Z, int lane) {
  int dd = d * d;
  cplx z = mk(0, 0);
  if (lane < dd) {
    int a = lane / d, c = lane % d;
    for (int q = 0; q < d; q++) cfma(z, X[a * d + q], Y[q * d + c]);
  }
  wave_sync();
  if (lane < dd) Z[lane] = z;
  wave_sync();
}

// E = exp(M) for the d x d block M in LDS (M is overwritten): scaling so that
// the Frobenius norm is at most 1/2, Taylor series of degree CF_TAYLOR by
// Horner's rule (truncation below 0.5^17/17! relative), then squaring.
__device__ inline void wave_expm(int d, cplx* M, cplx* E, int lane) {
  int dd = d * d;
  double nrm = lane < dd ? abs2(M[lane]) : 0.0;
  for (int o = 32; o >= 1; o >>= 1) nrm += __shfl_xor(nrm, o);
  nrm = sqrt(nrm);
  int s = 0;
  while (nrm > 0.5 && s < 60) {
    nrm *= 0.5;
    s++;
  }
  double sc = ldexp(1.0, -s);
  bool diag = lane < dd && lane / d == lane % d;
  if (lane < dd) {
    M[lane] = sc * M[lane];
    E[lane] = diag ? mk(1, 0) : mk(0, 0);
  }
  wave_sync();
  for (int j = CF_TAYLOR; j >= 1; j--) {
    wave_prod(d, M, E, E, lane);  // E <- M E
    if (lane < dd) {
      cplx v = (1.0 / j) * E[lane];
      if (diag) v.x += 1.0;
      E[lane] = v;  // E <- 1 + M E / j
    }
    wave_sync();
  }
  for (int i = 0; i < s; i++) wave_prod(d, E, E, E, lane);
}

__device__ inline double lagrange_w(int j0, int k, int i, double t) {
  double w = 1.0;
  for (int m = 0; m <= k; m++)
    if (m != i) w *= (t - (j0 + m)) / (double)(i - m);
  return w;
}

// Step propagators S_n = U_{n+1,n}, two waves per step (2 steps per
// workgroup): the even wave of a pair forms the left factor of Eq. cf4, the
// odd wave the right one, then the even wave multiplies them into loc[n+1].
__global__ __launch_bounds__(CF_NT) void k_cf4_steps(Prob P, FreeScratch fs) {
  __shared__ cplx wk[4][2][64];
  const double SQ3 = 1.7320508075688772;
  const double a1 = (3.0 - 2.0 * SQ3) / 12.0, a2 = (3.0 + 2.0 * SQ3) / 12.0;
  const double c1 = (1.0 - 1.0 / SQ3) / 2.0, c2 = (1.0 + 1.0 / SQ3) / 2.0;
  int d = P.d, dd = d * d, k = P.k;
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, side = wave & 1;
  int n = blockIdx.x * 2 + (wave >> 1);
  bool act = n < P.nt;  // (whole waves)
  double h = P.h;
  cplx *M = wk[wave][0], *E = wk[wave][1];
  if (act) {
    int j0 = n - k + 1 > 0 ? n - k + 1 : 0;
    if (lane < dd) {
      cplx e1 = mk(0, 0), e2 = mk(0, 0);
      for (int m = 0; m <= k; m++) {
        cplx ev = gld(P.eps + (size_t)(j0 + m + 1) * dd + lane);
        e1 = e1 + lagrange_w(j0, k, m, n + c1) * ev;
        e2 = e2 + lagrange_w(j0, k, m, n + c2) * ev;
      }
      // (the Hamiltonian of the real-time branch is eps - mu, as in the Dyson
      // equations of this library)
      if (lane / d == lane % d) {
        e1.x -= P.mu;
        e2.x -= P.mu;
      }
      // exponents -i h (a1 e1 + a2 e2) (left factor) and -i h (a2 e1 + a1 e2)
      M[lane] = side == 0 ? mk(0, -h) * (a1 * e1 + a2 * e2) : mk(0, -h) * (a2 * e1 + a1 * e2);
    }
    wave_sync();
    wave_expm(d, M, E, lane);
  }
  __syncthreads();
  if (!act || side != 0) return;
  cplx* EL = wk[wave][1];
  wave_prod(d, EL, wk[wave + 1][1], EL, lane);
  if (lane < dd) gst(fs.loc + (size_t)(n + 1) * dd + lane, EL[lane]);
}

// Products within chunk blockIdx.x (one wave):
//   loc[n+1] <- S_n S_{n-1} ... S_{c CF_CH}  for n in the chunk.
__global__ __launch_bounds__(64) void k_cf4_local(Prob P, FreeScratch fs) {
  __shared__ cplx S[CF_CH][64];
  int d = P.d, dd = d * d, nt = P.nt, lane = threadIdx.x;
  int n0 = blockIdx.x * CF_CH;
  int nloc = nt - n0 < CF_CH ? nt - n0 : CF_CH;
  for (int idx = lane; idx < nloc * dd; idx += 64) S[idx / dd][idx % dd] = gld(fs.loc + (size_t)(n0 + 1) * dd + idx);
  wave_sync();
  for (int i = 1; i < nloc; i++) wave_prod(d, S[i], S[i - 1], S[i], lane);
  for (int idx = lane; idx < nloc * dd; idx += 64) gst(fs.loc + (size_t)(n0 + 1) * dd + idx, S[idx / dd][idx % dd]);
}

// Products across chunks (wave 0): carry[c] = U_{c CF_CH} (carry[0] = 1);
// meanwhile wave 1 diagonalises eps(0^-) - mu = R diag(x) R^dag and forms
// rho = R diag(f(x)) R^dag.
__global__ __launch_bounds__(128) void k_cf4_carry(Prob P, FreeScratch fs) {
  __shared__ cplx C[64], L[64], A[64], V[64];
  __shared__ double x[8];
  int d = P.d, dd = d * d, tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    int nch = (P.nt + CF_CH - 1) / CF_CH;
    if (lane < dd) C[lane] = (lane / d == lane % d) ? mk(1, 0) : mk(0, 0);
    wave_sync();
    for (int c = 0; c <= nch; c++) {
      if (lane < dd) gst(fs.carry + (size_t)c * dd + lane, C[lane]);
      if (c == nch) break;
      int last = (c + 1) * CF_CH < P.nt ? (c + 1) * CF_CH : P.nt;  // U index of the chunk's last product
      if (lane < dd) L[lane] = gld(fs.loc + (size_t)last * dd + lane);
      wave_sync();
      wave_prod(d, L, C, C, lane);
    }
  } else {
    if (lane < dd) {
      A[lane] = gld(P.eps + lane);
      if (lane / d == lane % d) A[lane].x -= P.mu;
    }
    wave_sync();
    wave_jacobi(d, A, V, x, lane);
  }
  __syncthreads();
  if (tid >= 64) return;
  double xi = P.sig, beta = P.beta;
  if (lane < dd) {
    int a = lane / d, c = lane % d;
    cplx r = mk(0, 0);
    for (int al = 0; al < d; al++) {
      double xa = x[al];
      double f = xa >= 0 ? exp(-beta * xa) / (1 - xi * exp(-beta * xa)) : 1 / (exp(beta * xa) - xi);
      r = r + f * (V[a * d + al] * conj(V[c * d + al]));
    }
    gst(fs.rho + lane, r);
    gst(fs.R + lane, V[lane]);
  }
  if (lane < d) fs.x[lane] = x[lane];
}

// Rows: U_n = loc_n carry[c(n)] (U_0 = 1) and W_n = U_n rho, one thread per
// (n, a); then F_m = R diag(f(x) e^{x tau_m}) R^dag, one thread per (m, a).
__global__ __launch_bounds__(CF_NT) void k_cf4_rows(Prob P, FreeScratch fs) {
  int d = P.d, dd = d * d, nt = P.nt, ntau = P.ntau;
  long idx = (long)blockIdx.x * CF_NT + threadIdx.x;
  long nrow = (long)(nt + 1) * d;
  if (idx < nrow) {
    int n = (int)(idx / d), a = (int)(idx % d);
    cplx u[8], w[8];
    const cplx* L = fs.loc + (size_t)n * dd + a * d;
    const cplx* C = fs.carry + (size_t)(n > 0 ? (n - 1) / CF_CH : 0) * dd;
#pragma unroll
    for (int c = 0; c < 8; c++) {
      cplx s = mk(0, 0);
      if (c < d) {
        if (n == 0) {
          s = (c == a) ? mk(1, 0) : mk(0, 0);
        } else {
          for (int q = 0; q < d; q++) cfma(s, gld(L + q), gld(C + q * d + c));
        }
      }
      u[c] = s;
    }
#pragma unroll
    for (int c = 0; c < 8; c++) {
      cplx s = mk(0, 0);
#pragma unroll
      for (int q = 0; q < 8; q++)
        if (q < d && c < d) cfma(s, u[q], gld(fs.rho + q * d + c));
      w[c] = s;
    }
#pragma unroll
    for (int c = 0; c < 8; c++)
      if (c < d) {
        gst(fs.U + (size_t)n * dd + a * d + c, u[c]);
        gst(fs.W + (size_t)n * dd + a * d + c, w[c]);
      }
    return;
  }
  idx -= nrow;
  if (idx >= (long)(ntau + 1) * d) {
    // G^M(tau_m) = -R diag(e^{-x tau}/(1 - xi e^{-beta x})) R^dag (the free
    // Matsubara function, in the overflow-free form)
    idx -= (long)(ntau + 1) * d;
    if (idx >= (long)(ntau + 1) * d) return;
    int m = (int)(idx / d), a = (int)(idx % d);
    double xi = P.sig, beta = P.beta, tau = m * P.htau;
    for (int c = 0; c < d; c++) {
      cplx s = mk(0, 0);
      for (int al = 0; al < d; al++) {
        double xa = fs.x[al];
        double g = (xa >= 0 || xi > 0) ? -exp(-xa * tau) / (1 - xi * exp(-beta * xa))
                                       : -exp(xa * (beta - tau)) / (exp(beta * xa) - xi);
        s = s + g * (gld(fs.R + a * d + al) * conj(gld(fs.R + c * d + al)));
      }
      gst(P.Gmat + (size_t)m * dd + a * d + c, s);
    }
    return;
  }
  {
    int m = (int)(idx / d), a = (int)(idx % d);
    double xi = P.sig, beta = P.beta, tau = m * P.htau;
    for (int c = 0; c < d; c++) {
      cplx s = mk(0, 0);
      for (int al = 0; al < d; al++) {
        double xa = fs.x[al];
        double g = xa >= 0 ? exp(-xa * (beta - tau)) / (1 - xi * exp(-beta * xa))
                           : exp(xa * tau) / (exp(beta * xa) - xi);
        s = s + g * (gld(fs.R + a * d + al) * conj(gld(fs.R + c * d + al)));
      }
      gst(fs.F + (size_t)m * dd + a * d + c, s);
    }
  }
}

// Blocks b0 .. b0+nb-1 of slice n = blockIdx.y, one element per thread:
// section blockIdx.z = 0: G^R(t_n, t_j) = -i U_n U_j^dag (row n, j = b);
// 1: G^<(t_j, t_n) = -i xi W_j U_n^dag (column n, j = b); 2: G^rceil(t_n,
// tau_m) = -i xi U_n F_m (m = b). The operands U_n and the nb blocks of U, W
// or F (contiguous) are staged in LDS, so each output element costs one
// coalesced 16-byte store and about one 16-byte load.
__global__ __launch_bounds__(CF_NT) void k_free_write(Prob P, FreeScratch fs) {
  __shared__ cplx X[64], Y[CF_NT];
  int d = P.d, dd = d * d, ntau = P.ntau, tid = threadIdx.x;
  int sec = blockIdx.z, n = blockIdx.y;
  int bpw = CF_NT / dd;
  int nblk = sec == 2 ? ntau + 1 : n + 1;
  int b0 = blockIdx.x * bpw;
  if (b0 >= nblk) return;
  int nb = nblk - b0 < bpw ? nblk - b0 : bpw;
  const cplx* src = sec == 0 ? fs.U : (sec == 1 ? fs.W : fs.F);
  if (tid < dd) X[tid] = gld(fs.U + (size_t)n * dd + tid);
  if (tid < nb * dd) Y[tid] = gld(src + (size_t)b0 * dd + tid);
  __syncthreads();
  if (tid >= nb * dd) return;
  int bl = tid / dd, e = tid % dd, a = e / d, c = e % d;
  const cplx* y = Y + bl * dd;
  cplx s = mk(0, 0);
  if (sec == 0) {
    for (int q = 0; q < d; q++) cfma(s, X[a * d + q], conj(y[c * d + q]));
    gst(P.Gret + (tri(n) + b0) * dd + tid, mk(s.y, -s.x));
  } else if (sec == 1) {
    for (int q = 0; q < d; q++) cfma(s, y[a * d + q], conj(X[c * d + q]));
    gst(P.Gles + (tri(n) + b0) * dd + tid, (double)P.sig * mk(s.y, -s.x));
  } else {
    for (int q = 0; q < d; q++) cfma(s, X[a * d + q], y[q * d + c]);
    gst(P.Gtv + ((size_t)n * (ntau + 1) + b0) * dd + tid, (double)P.sig * mk(s.y, -s.x));
  }
}

size_t free_green_scratch_bytes(int nt, int ntau, int d) { return free_scratch_elems(nt, ntau, d) * sizeof(cplx); }

hipError_t launch_free_green(const Prob& P, void* scratch, hipStream_t s) {
  int d = P.d, nt = P.nt, ntau = P.ntau;
  size_t dd = (size_t)d * d;
  int nch = (nt + CF_CH - 1) / CF_CH;
  FreeScratch fs;
  cplx* b = (cplx*)scratch;
  fs.loc = b;
  fs.U = fs.loc + (size_t)(nt + 1) * dd;
  fs.W = fs.U + (size_t)(nt + 1) * dd;
  fs.F = fs.W + (size_t)(nt + 1) * dd;
  fs.carry = fs.F + (size_t)(ntau + 1) * dd;
  fs.rho = fs.carry + (size_t)(nch + 1) * dd;
  fs.R = fs.rho + dd;
  fs.x = (double*)(fs.R + dd);
  if (nch > 0) {
    k_cf4_steps<<<(nt + 1) / 2, CF_NT, 0, s>>>(P, fs);
    k_cf4_local<<<nch, 64, 0, s>>>(P, fs);
  }
  k_cf4_carry<<<1, 128, 0, s>>>(P, fs);
  long rows = (long)(nt + 1 + 2 * (ntau + 1)) * d;
  k_cf4_rows<<<(unsigned)((rows + CF_NT - 1) / CF_NT), CF_NT, 0, s>>>(P, fs);
  int bpw = CF_NT / (int)dd, nbmax = (nt > ntau ? nt : ntau) + 1;
  k_free_write<<<dim3((nbmax + bpw - 1) / bpw, nt + 1, 3), CF_NT, 0, s>>>(P, fs);
  return hipGetLastError();
}

}  // namespace cntr
