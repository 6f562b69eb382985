// Discrete adjoint of the Dyson time stepper for a given self-energy:
// reverse mode of the start-up (Sec. "Dyson equation: start-up") and of the
// data-parallel time step (Sec. "Time stepping": bulk rows of R and G^< by
// the single steps of Eqs. MBCVSAMx_t / MBCVSAMx_cc_t, k+1 boundary points
// by the serial forms and the conjugate start-up, Eq. MBCVSAMx_cc_start).
//
// The forward step writes slice n as a sequence of block solves
//   A X = r(earlier blocks)   or   X A = r(earlier blocks),
// so the adjoint runs the slices backwards, n = nt .. k+1, then the start-up,
// and for every solve applies the conjugate-transposed solve to the adjoint of
// X and scatters the result into the adjoints of the blocks r reads.
// Gradients use one convention throughout: for a real objective J and a
// complex entry z = x + iy the library accumulates dJ/dx + i dJ/dy. Then
//   X = A^{-1} r : rbar = A^{-H} Xbar, Abar -= rbar X^H
//   X = r A^{-1} : rbar = Xbar A^{-H}, Abar -= X^H rbar
//   Y = c P Q    : Pbar += conj(c) Ybar Q^H, Qbar += conj(c) P^H Ybar
// and an extended block (the R continuation -[R_{b,a}]^dag, the hermitian
// partner -[L_{b,a}]^dag, G^lceil = -xi [T]^dag) sends the conjugate
// transpose of its adjoint to the stored block.
//
// Every kernel body is a host-and-device function of (thread index, thread
// count), so its index arithmetic compiles on the host as well.
#pragma once
#include "dev_common.h"
#include "launch.h"

namespace cntr {

#if defined(__HIP_DEVICE_COMPILE__)
#define ADJ_SYNC() __syncthreads()
#else
#define ADJ_SYNC() ((void)0)
#endif

// Slices lo..hi of a contour function held contiguously: the R rows, the
// L columns and the T rows of those slices; (oR, oL, oT) are the block
// offsets of slice lo's first block in the full arrays.
struct AdjWin {
  cplx *R, *L, *T;
  size_t oR, oL, oT;
};

// One problem of an adjoint sweep. Pointers are device pointers in the
// canonical layout; the adjoint arrays have the shape of the quantity, or
// are windows of it whose first block sits at the given block origin.
struct AdjProb {
  Prob p;                    // G (forward solution), Sigma, eps, grid
  cplx *aR, *aL, *aT, *aM;   // adjoint of G: seed in, dJ/dM out in aM
  cplx *sR, *sL, *sT;        // dJ/dSigma (accumulated), null: not formed
  cplx *ge;                  // dJ/deps_n at index n+1 (accumulated)
  cplx* scr;                 // scratch of this problem
  int* stat;                 // set to 1 by a kernel that meets a singular local matrix
  size_t aoR, aoL, aoT;      // block origins of aR, aL, aT (0: whole arrays)
  size_t soR, soL, soT;      // block origins of sR, sL, sT
  // second-Born mode (Sigma = Sigma_2B[G], eps = eps0 + Hartree[G])
  const double* U;           // (nt+2), index n+1
  double nbar;
  double* ub;                // dJ/dU (accumulated), (nt+2)
  AdjWin g0, s0, nu[2], gdry, sdry;
  cplx *e0, *gedry, *mdummy;
  double* conv;              // per slice: max |change| and max |value| of the last iterate
};

constexpr int ADJ_NT = 256;  // threads per workgroup of every adjoint kernel

// row s of the triangle index t = tri(s) + j, 0 <= j <= s (closed form, then
// corrected for the rounding of the square root)
__host__ __device__ inline int tri_row(size_t t) {
  int s = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (tri(s) > t) s--;
  while (tri(s + 1) <= t) s++;
  return s;
}

__host__ __device__ inline size_t oR(int a, int b) { return tri(a) + b; }  // R_{a,b}, a >= b
__host__ __device__ inline size_t oL(int a, int b) { return tri(b) + a; }  // L_{a,b}, a <= b
__host__ __device__ inline size_t oT(int n, int m, int ntau) { return (size_t)n * (ntau + 1) + m; }

// Gregory weight w_{N,j} (host-and-device copy of the time stepper's rule).
__host__ __device__ inline double adj_w(const KW& W, int N, int j) {
  int k = W.k;
  if (N <= k) return W.s[N][j];
  bool left = j <= k, right = N - j <= k;
  if (left && right) return W.omega[j] + W.omega[N - j] - 1.0;
  if (left) return W.omega[j];
  if (right) return W.omega[N - j];
  return 1.0;
}

// scratch layout of one problem, in complex units
struct AdjLayout {
  size_t mrinv, rhoB, rhoL, rhoT, rhoR, part, binv, psi, pst, ainv, cbinv, total;
  int cb, npart;
};
__host__ __device__ inline int adj_cb(int dd) { return dd >= ADJ_NT ? 1 : ADJ_NT / dd; }
__host__ __device__ inline AdjLayout adj_layout(int nt, int ntau, int d, int k) {
  AdjLayout L;
  size_t dd = (size_t)d * d;
  L.cb = adj_cb((int)dd);
  L.npart = 2 * ((nt + 1 + L.cb - 1) / L.cb) + (ntau + 1 + L.cb - 1) / L.cb + 3;
  size_t o = 0;
  L.mrinv = o; o += dd;
  L.rhoB = o; o += (size_t)(2 * k + 2) * dd;
  L.rhoL = o; o += (size_t)(nt + 1) * dd;
  L.rhoT = o; o += (size_t)(ntau + 1) * dd;
  L.rhoR = o; o += (size_t)(nt + 1) * dd;
  L.part = o; o += (size_t)L.npart * dd;
  L.binv = o; o += (size_t)k * d * k * d;
  L.psi = o; o += (size_t)k * (ntau + 1) * dd;
  L.pst = o; o += (size_t)k * (k + 1) * dd;
  L.ainv = o; o += (size_t)(k + 1) * dd;
  L.cbinv = o; o += (size_t)k * d * k * d;
  L.total = o;
  return L;
}

// ----------------------------------------------------------- element access
struct AdjView {
  const Prob& P;
  const AdjProb& A;
  const KW& W;
  int d, dd, k, nt, ntau;
  double h, ht, xi;
  AdjLayout lay;
  __host__ __device__ AdjView(const AdjProb& a, const KW& w)
      : P(a.p), A(a), W(w), d(a.p.d), dd(a.p.d * a.p.d), k(a.p.k), nt(a.p.nt), ntau(a.p.ntau),
        h(a.p.h), ht(a.p.htau), xi((double)a.p.sig), lay(adj_layout(a.p.nt, a.p.ntau, a.p.d, a.p.k)) {}
  // stored blocks
  __host__ __device__ const cplx* GR(int a, int b) const { return P.Gret + oR(a, b) * dd; }
  __host__ __device__ const cplx* GL(int a, int b) const { return P.Gles + oL(a, b) * dd; }
  __host__ __device__ const cplx* GT(int n, int m) const { return P.Gtv + oT(n, m, ntau) * dd; }
  __host__ __device__ const cplx* GM(int m) const { return P.Gmat + (size_t)m * dd; }
  __host__ __device__ const cplx* SR(int a, int b) const { return P.Sret + oR(a, b) * dd; }
  __host__ __device__ const cplx* SL(int a, int b) const { return P.Sles + oL(a, b) * dd; }
  __host__ __device__ const cplx* ST(int n, int m) const { return P.Stv + oT(n, m, ntau) * dd; }
  __host__ __device__ cplx* aR(int a, int b) const { return A.aR + (oR(a, b) - A.aoR) * dd; }
  __host__ __device__ cplx* aL(int a, int b) const { return A.aL + (oL(a, b) - A.aoL) * dd; }
  __host__ __device__ cplx* aT(int n, int m) const { return A.aT + (oT(n, m, ntau) - A.aoT) * dd; }
  __host__ __device__ cplx* aM(int m) const { return A.aM + (size_t)m * dd; }
  __host__ __device__ cplx* sR(int a, int b) const { return A.sR + (oR(a, b) - A.soR) * dd; }
  __host__ __device__ cplx* sL(int a, int b) const { return A.sL + (oL(a, b) - A.soL) * dd; }
  __host__ __device__ cplx* sT(int n, int m) const { return A.sT + (oT(n, m, ntau) - A.soT) * dd; }
  // windows
  __host__ __device__ cplx* wR(const AdjWin& w, int a, int b) const { return w.R + (oR(a, b) - w.oR) * dd; }
  __host__ __device__ cplx* wL(const AdjWin& w, int a, int b) const { return w.L + (oL(a, b) - w.oL) * dd; }
  __host__ __device__ cplx* wT(const AdjWin& w, int n, int m) const { return w.T + (oT(n, m, ntau) - w.oT) * dd; }
  __host__ __device__ cplx* ge(int n) const { return A.ge + (size_t)(n + 1) * dd; }
  __host__ __device__ cplx* scr(size_t off) const { return A.scr + off; }
  // extended elements
  __host__ __device__ cplx Rt(const cplx* X, int a, int b, int r, int c) const {
    return a >= b ? X[oR(a, b) * dd + r * d + c] : -conj(X[oR(b, a) * dd + c * d + r]);
  }
  __host__ __device__ cplx Lh(const cplx* X, int a, int b, int r, int c) const {
    return a <= b ? X[oL(a, b) * dd + r * d + c] : -conj(X[oL(b, a) * dd + c * d + r]);
  }
  // e_n - mu
  __host__ __device__ cplx eh(int n, int r, int c) const {
    cplx v = P.eps[(size_t)(n + 1) * dd + r * d + c];
    if (r == c) v.x -= P.mu;
    return v;
  }
};

// sum_q a(q) b(q), q = 0..d-1
template <class FA, class FB>
__host__ __device__ inline cplx dotq(int d, FA fa, FB fb) {
  cplx s = mk(0, 0);
  for (int q = 0; q < d; q++) cfma(s, fa(q), fb(q));
  return s;
}

// --------------------------------------------------------------- team algebra
// Gauss-Jordan inverse in place (n x n, row-major) by a team of `nth`
// threads; pivot search by thread 0. piv: n + 2 ints. Returns false if
// singular (uniform over the team).
__host__ __device__ inline bool team_inverse(int n, cplx* A, int* piv, int tid, int nth) {
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
      piv[c] = p;
      piv[n] = best > 0.0 ? 1 : 0;
    }
    ADJ_SYNC();
    if (piv[n] == 0) return false;
    int p = piv[c];
    if (p != c)
      for (int q = tid; q < n; q += nth) {
        cplx t = A[p * n + q];
        A[p * n + q] = A[c * n + q];
        A[c * n + q] = t;
      }
    ADJ_SYNC();
    cplx ipv = cdiv(mk(1, 0), A[c * n + c]);
    for (int idx = tid; idx < n * n; idx += nth) {
      int r = idx / n, q = idx % n;
      if (r == c || q == c) continue;
      A[r * n + q] = A[r * n + q] - A[r * n + c] * (A[c * n + q] * ipv);
    }
    ADJ_SYNC();
    for (int r = tid; r < n; r += nth)
      if (r != c) A[r * n + c] = -(A[r * n + c] * ipv);
    ADJ_SYNC();
    for (int q = tid; q < n; q += nth) A[c * n + q] = (q == c) ? ipv : A[c * n + q] * ipv;
    ADJ_SYNC();
  }
  for (int c = n - 1; c >= 0; c--) {
    int p = piv[c];
    if (p != c)
      for (int r = tid; r < n; r += nth) {
        cplx t = A[r * n + p];
        A[r * n + p] = A[r * n + c];
        A[r * n + c] = t;
      }
    ADJ_SYNC();
  }
  return true;
}

// ------------------------------------------------------------ les_source
// Forward value of the lesser source of row m, column n, element (r, c):
//   q = -i (C^<_2 + C^<_3)[Sigma, 1, G](m, n),
//   C^<_2 = sum_{j<=max(n,k)} h w_{n,j} Sigma^<_{m,j} G^A_{j,n},
//   C^<_3 = -i h_tau sum_j w_{ntau,j} Sigma^rceil_{m,j} G^lceil(tau_j, t_n).
__host__ __device__ inline cplx les_source_elem(const AdjView& V, int m, int n, int r, int c) {
  int d = V.d, jmax = n > V.k ? n : V.k;
  cplx c2 = mk(0, 0), c3 = mk(0, 0);
  for (int j = 0; j <= jmax; j++) {
    // G^A_{j,n}[q][c] = conj(Rt(G, n, j)[c][q])
    cplx t = dotq(d, [&](int q) { return V.Lh(V.P.Sles, m, j, r, q); },
                  [&](int q) { return conj(V.Rt(V.P.Gret, n, j, c, q)); });
    c2 = c2 + (V.h * adj_w(V.W, n, j)) * t;
  }
  for (int j = 0; j <= V.ntau; j++) {
    // G^lceil(tau_j, t_n)[q][c] = -xi conj(T_{n, ntau-j}[c][q])
    const cplx* s = V.ST(m, j);
    const cplx* g = V.GT(n, V.ntau - j);
    cplx t = dotq(d, [&](int q) { return s[r * d + q]; }, [&](int q) { return conj(g[c * d + q]); });
    c3 = c3 + (-V.xi * V.ht * adj_w(V.W, V.ntau, j)) * t;
  }
  // -i (c2 + (-i) c3) = -i c2 - c3
  return mk(c2.y, -c2.x) - c3;
}

// start_block(p, l)[r][c] = h^-1 D_{p,l} + delta_{pl} i e_p + i h s_{p,l} Sigma~^R_{p,l}
__host__ __device__ inline cplx start_block_elem(const AdjView& V, int p, int l, int r, int c) {
  cplx v = V.Rt(V.P.Sret, p, l, r, c);
  v = mul_i((V.h * V.W.s[p][l]) * v);
  if (r == c) v.x += V.W.D[p][l] / V.h;
  if (p == l) v = v + mul_i(V.eh(p, r, c));
  return v;
}

// ============================================================== K1a
// Serial part of the lesser column n (one team per problem):
//  * n > 2k: boundary rows m = n..n-k (serial steps (A)) in reverse order;
//  * k < n <= 2k: rows n..k+1 in reverse order, then the start-up rows 1..k;
//  * n <= k: the start-up rows 1..k of column n.
// Writes the row adjoints rho_m (gq of the lesser source of row m) to rhoB,
// the eps and Sigma^R adjoints of the local step matrices, and the adjoint
// updates among the rows it owns; K1b scatters the rest. Also stores M_R^{-1}
// of slice n (n > k) for the bulk kernels.
// lds: >= (2k+2) dd + 4 dd + 5 (k d)^2-sized... see adj_lcol_lds().
__host__ __device__ inline int adj_lcol_lds(int d, int k) {
  int dd = d * d, kd = k * d;
  return (2 * k + 2) * dd + 3 * dd + kd * kd + 4 * kd * d;
}

__host__ __device__ inline bool adj_lcol_team(const AdjProb& Ap, const KW& W, int n, int tid, int nth,
                                              cplx* lds, int* piv) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k;
  double h = V.h;
  bool ok = true;
  cplx* acc = lds;                      // (2k+2) blocks: adjoints of rows r0..n
  cplx* Am = acc + (2 * k + 2) * dd;    // d x d
  cplx* rho = Am + dd;                  // d x d
  cplx* tmp = rho + dd;                 // d x d
  cplx* Bb = tmp + dd;                  // (k d)^2
  cplx* yv = Bb + k * d * k * d;        // k d x d
  cplx* lam = yv + k * d * d;
  cplx* psi = lam + k * d * d;
  cplx* rr = psi + k * d * d;
  cplx* rhoB = V.scr(V.lay.rhoB);
  bool bulk = n > 2 * k;
  int r0 = bulk ? n - k : 0;  // first row held in acc
  for (int e = tid; e < (n - r0 + 1) * dd; e += nth) acc[e] = V.aL(r0 + e / dd, n)[e % dd];
  ADJ_SYNC();
  // serial steps (A), rows m = n .. mlo in reverse order
  int mlo = bulk ? n - k : k + 1;
  for (int m = n; m >= mlo && n > k; m--) {
    // A_m = h^-1 a_0 + i e_m + i h w_{m,m} Sigma^R_{m,m} (inverse prepared by
    // adj_prep_team); rho = A_m^{-H} lambda_m
    for (int e = tid; e < dd; e += nth) Am[e] = V.scr(V.lay.ainv)[(size_t)(m - mlo) * dd + e];
    ADJ_SYNC();
    const cplx* lm = acc + (m - r0) * dd;
    for (int e = tid; e < dd; e += nth) {
      int r = e / d, c = e % d;
      rho[e] = dotq(d, [&](int q) { return conj(Am[q * d + r]); }, [&](int q) { return lm[q * d + c]; });
    }
    ADJ_SYNC();
    int slot = bulk ? m - (n - k) : m - 1;
    for (int e = tid; e < dd; e += nth) rhoB[slot * dd + e] = rho[e];
    // eps_m and Sigma^R_{m,m}: Abar = -rho L_{m,n}^H
    const cplx* Lmn = V.GL(m, n);
    for (int e = tid; e < dd; e += nth) {
      int r = e / d, c = e % d;
      cplx t = dotq(d, [&](int q) { return rho[r * d + q]; }, [&](int q) { return conj(Lmn[c * d + q]); });
      V.ge(m)[e] = V.ge(m)[e] + mul_i(t);
      if (V.A.sR) V.sR(m, m)[e] = V.sR(m, m)[e] + mul_i((h * adj_w(W, m, m)) * t);
    }
    // rows j in [r0, m): history term and BDF
    for (int e = tid; e < (m - r0) * dd; e += nth) {
      int j = r0 + e / dd, r = (e % dd) / d, c = e % d;
      const cplx* s = V.SR(m, j);
      cplx t = dotq(d, [&](int q) { return conj(s[q * d + r]); }, [&](int q) { return rho[q * d + c]; });
      cplx v = mul_i((h * adj_w(W, m, j)) * t);
      int l = m - j;
      if (l <= k) v = v - (W.a[l] / h) * rho[r * d + c];
      acc[(j - r0) * dd + r * d + c] = acc[(j - r0) * dd + r * d + c] + v;
      if (V.A.sR) {
        const cplx* Lj = V.GL(j, n);
        cplx u = dotq(d, [&](int q) { return rho[r * d + q]; }, [&](int q) { return conj(Lj[c * d + q]); });
        V.sR(m, j)[r * d + c] = V.sR(m, j)[r * d + c] + mul_i((h * adj_w(W, m, j)) * u);
      }
    }
    ADJ_SYNC();
  }
  if (!bulk) {
    // start-up rows 1..k of column n (Eq. vdiff_start, y_0 = -[T_{n,0}]^dag)
    int kd = k * d;
    // r_p = q_p - B_{p,0} y_0
    for (int e = tid; e < kd * d; e += nth) {
      int p = 1 + e / dd, r = (e % dd) / d, c = e % d;
      cplx v = les_source_elem(V, p, n, r, c);
      const cplx* T0 = V.GT(n, 0);
      // y0[q][c] = -conj(T0[c][q])
      cplx t = dotq(d, [&](int q) { return start_block_elem(V, p, 0, r, q); },
                    [&](int q) { return -conj(T0[c * d + q]); });
      rr[e] = v - t;
      lam[e] = (p <= n) ? acc[p * dd + r * d + c] : mk(0, 0);
    }
    for (int e = tid; e < kd * kd; e += nth) Bb[e] = V.scr(V.lay.binv)[e];  // B^{-1}, adj_tinv_team
    ADJ_SYNC();
    for (int e = tid; e < kd * d; e += nth) {
      int R = e / d, c = e % d;
      cplx y = mk(0, 0), s = mk(0, 0);
      for (int q = 0; q < kd; q++) {
        cfma(y, Bb[R * kd + q], rr[q * d + c]);
        cfma(s, conj(Bb[q * kd + R]), lam[q * d + c]);
      }
      yv[e] = y;
      psi[e] = s;
    }
    ADJ_SYNC();
    for (int e = tid; e < kd * d; e += nth) rhoB[e] = psi[e];  // rows 1..k at slots 0..k-1
    // eps_p += i psi_p y_p^H
    for (int e = tid; e < kd * d; e += nth) {
      int p = 1 + e / dd, r = (e % dd) / d, c = e % d;
      const cplx* ps = psi + (p - 1) * dd;
      const cplx* yp = yv + (p - 1) * dd;
      cplx t = dotq(d, [&](int q) { return ps[r * d + q]; }, [&](int q) { return conj(yp[c * d + q]); });
      V.ge(p)[r * d + c] = V.ge(p)[r * d + c] + mul_i(t);
    }
    // y_0 = -[T_{n,0}]^dag: gy0 = lambda_0 - sum_p B_{p,0}^H psi_p ; Tbar_{n,0} -= gy0^H
    for (int e = tid; e < dd; e += nth) {
      int r = e / d, c = e % d;
      // (gy0^H)[r][c] = conj(gy0[c][r])
      cplx g = acc[0 * dd + c * d + r];
      for (int p = 1; p <= k; p++) {
        const cplx* ps = psi + (p - 1) * dd;
        g = g - dotq(d, [&](int q) { return conj(start_block_elem(V, p, 0, q, c)); },
                     [&](int q) { return ps[q * d + r]; });
      }
      V.aT(n, 0)[e] = V.aT(n, 0)[e] - conj(g);
    }
    // Sigma~^R_{p,l} += i h s_{p,l} psi_p y_l^H, p = 1..k, l = 0..k, on stored
    // targets (a, b), a >= b: direct from (p,l) = (a,b), continuation from (b,a).
    if (V.A.sR) {
      int nb = (k + 1) * (k + 2) / 2;
      for (int e = tid; e < nb * dd; e += nth) {
        int t = e / dd, r = (e % dd) / d, c = e % d;
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= t) a++;
        int b = t - a * (a + 1) / 2;
        auto yl = [&](int l, int rr_, int q) -> cplx {  // y_l[c'][q] element
          if (l == 0) return -conj(V.GT(n, 0)[q * d + rr_]);
          return yv[(l - 1) * dd + rr_ * d + q];
        };
        cplx v = mk(0, 0);
        if (a >= 1) {
          const cplx* ps = psi + (a - 1) * dd;
          cplx u = dotq(d, [&](int q) { return ps[r * d + q]; }, [&](int q) { return conj(yl(b, c, q)); });
          v = v + mul_i((h * W.s[a][b]) * u);
        }
        if (b >= 1 && a > b) {
          // -(i h s_{b,a} psi_b y_a^H)^H = i h s_{b,a} y_a psi_b^H
          const cplx* ps = psi + (b - 1) * dd;
          cplx u = dotq(d, [&](int q) { return yl(a, r, q); }, [&](int q) { return conj(ps[c * d + q]); });
          v = v + mul_i((h * W.s[b][a]) * u);
        }
        V.sR(a, b)[r * d + c] = V.sR(a, b)[r * d + c] + v;
      }
    }
    ADJ_SYNC();
  }
  return ok;
}

// ============================================================== K1b
// Parallel part of the lesser column: the reverse of the sources of rows
// r0..r1 (row adjoints in rhoB) and, for n > 2k, the boundary rows' history
// terms on the bulk rows j < n-k.
struct LcolGeom {
  int r0, r1, jmax, bs0;
  size_t o1, o1x, o2, o3, o4, o5, o6, total;  // element offsets of the output groups
};
__host__ __device__ inline LcolGeom lcol_geom(int n, int k, int ntau, int dd, bool sig) {
  LcolGeom G;
  bool bulk = n > 2 * k;
  G.r0 = bulk ? n - k : 1;
  G.r1 = bulk ? n : (n > k ? n : k);
  G.jmax = n > k ? n : k;
  G.bs0 = G.r0;
  size_t o = 0;
  G.o1 = o; o += (size_t)(n + 1) * dd;                                  // aR(n, j), j <= n
  G.o1x = o; o += (size_t)(n < k ? k - n : 0) * dd;                      // aR(j, n), n < j <= k
  G.o2 = o; o += (size_t)(ntau + 1) * dd;                               // aT(n, tau)
  G.o3 = o; o += sig ? (size_t)(G.r1 - G.r0 + 1) * (ntau + 1) * dd : 0;  // sT(m, j)
  G.o4 = o; o += sig ? (tri(G.jmax + 1) - tri(G.bs0)) * dd : 0;          // sL slices bs0..jmax
  G.o5 = o; o += bulk ? (size_t)(n - k) * dd : 0;                       // aL(j, n), j < n-k
  G.o6 = o; o += (bulk && sig) ? (size_t)(k + 1) * (n - k) * dd : 0;     // sR(m, j)
  G.total = o;
  return G;
}

__host__ __device__ inline void adj_lcol_elem(const AdjProb& Ap, const KW& W, int n, size_t idx) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k, ntau = V.ntau;
  double h = V.h, ht = V.ht, xi = V.xi;
  bool sig = Ap.sR != nullptr;
  LcolGeom G = lcol_geom(n, k, ntau, dd, sig);
  if (idx >= G.total) return;
  const cplx* rhoB = V.scr(V.lay.rhoB);
  bool bulk = n > 2 * k;
  auto gq = [&](int m) { return rhoB + (size_t)(bulk ? m - (n - k) : m - 1) * dd; };
  int e = (int)(idx % dd), r = e / d, c = e % d;
  if (idx < G.o1x) {
    // aR(n, j) += sum_m -i h w_{n,j} gq_m^H Lh(S, m, j)
    int j = (int)((idx - G.o1) / dd);
    cplx acc = mk(0, 0);
    for (int m = G.r0; m <= G.r1; m++) {
      const cplx* g = gq(m);
      acc = acc + dotq(d, [&](int q) { return conj(g[q * d + r]); },
                       [&](int q) { return V.Lh(V.P.Sles, m, j, q, c); });
    }
    cplx v = mul_i(-(h * adj_w(W, n, j)) * acc);
    V.aR(n, j)[e] = V.aR(n, j)[e] + v;
  } else if (idx < G.o2) {
    // j > n (start-up columns): aR(j, n) += sum_m -i h w_{n,j} Lh(S, m, j)^H gq_m
    int j = n + 1 + (int)((idx - G.o1x) / dd);
    cplx acc = mk(0, 0);
    for (int m = G.r0; m <= G.r1; m++) {
      const cplx* g = gq(m);
      acc = acc + dotq(d, [&](int q) { return conj(V.Lh(V.P.Sles, m, j, q, r)); },
                       [&](int q) { return g[q * d + c]; });
    }
    cplx v = mul_i(-(h * adj_w(W, n, j)) * acc);
    V.aR(j, n)[e] = V.aR(j, n)[e] + v;
  } else if (idx < G.o3) {
    // aT(n, tau) += sum_m xi ht w_{ntau, ntau-tau} gq_m^H Sigma^rceil_{m, ntau-tau}
    int tau = (int)((idx - G.o2) / dd), j = ntau - tau;
    cplx acc = mk(0, 0);
    for (int m = G.r0; m <= G.r1; m++) {
      const cplx* g = gq(m);
      const cplx* s = V.ST(m, j);
      acc = acc + dotq(d, [&](int q) { return conj(g[q * d + r]); }, [&](int q) { return s[q * d + c]; });
    }
    V.aT(n, tau)[e] = V.aT(n, tau)[e] + (xi * ht * adj_w(W, ntau, j)) * acc;
  } else if (idx < G.o4) {
    // sT(m, j) += xi ht w_{ntau,j} gq_m T_{n, ntau-j}
    size_t t = (idx - G.o3) / dd;
    int m = G.r0 + (int)(t / (ntau + 1)), j = (int)(t % (ntau + 1));
    const cplx* g = gq(m);
    const cplx* T = V.GT(n, ntau - j);
    cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return T[q * d + c]; });
    V.sT(m, j)[e] = V.sT(m, j)[e] + (xi * ht * adj_w(W, ntau, j)) * u;
  } else if (idx < G.o5) {
    // sL(a, b), slices b in [bs0, jmax], a <= b:
    //   a in rows:         i h w_{n,b} gq_a Rt(G, n, b)
    //   b in rows, a < b:  i h w_{n,a} Rt(G, n, a)^H gq_b^H
    size_t t = tri(G.bs0) + (idx - G.o4) / dd;
    int b = tri_row(t);
    int a = (int)(t - tri(b));
    cplx v = mk(0, 0);
    if (a >= G.r0 && a <= G.r1) {
      const cplx* g = gq(a);
      cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return V.Rt(V.P.Gret, n, b, q, c); });
      v = v + mul_i((h * adj_w(W, n, b)) * u);
    }
    if (b >= G.r0 && b <= G.r1 && a < b) {
      const cplx* g = gq(b);
      cplx u = dotq(d, [&](int q) { return conj(V.Rt(V.P.Gret, n, a, q, r)); },
                    [&](int q) { return conj(g[c * d + q]); });
      v = v + mul_i((h * adj_w(W, n, a)) * u);
    }
    V.sL(a, b)[e] = V.sL(a, b)[e] + v;
  } else if (idx < G.o6) {
    // aL(j, n), j < n-k: sum_m i h w_{m,j} S^R_{m,j}^H rho_m - sum_{m=j+l} a_l/h rho_m
    int j = (int)((idx - G.o5) / dd);
    cplx v = mk(0, 0);
    for (int m = n - k; m <= n; m++) {
      const cplx* g = gq(m);
      const cplx* s = V.SR(m, j);
      cplx u = dotq(d, [&](int q) { return conj(s[q * d + r]); }, [&](int q) { return g[q * d + c]; });
      v = v + mul_i((h * adj_w(W, m, j)) * u);
      int l = m - j;
      if (l >= 1 && l <= k) v = v - (W.a[l] / h) * g[e];
    }
    V.aL(j, n)[e] = V.aL(j, n)[e] + v;
  } else {
    // sR(m, j), m in [n-k, n], j < n-k: i h w_{m,j} rho_m L_{j,n}^H
    size_t t = (idx - G.o6) / dd;
    int m = n - k + (int)(t / (n - k)), j = (int)(t % (n - k));
    const cplx* g = gq(m);
    const cplx* L = V.GL(j, n);
    cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return conj(L[c * d + q]); });
    V.sR(m, j)[e] = V.sR(m, j)[e] + mul_i((h * adj_w(W, m, j)) * u);
  }
}

// ============================================================== Krho
// Row adjoints of the bulk solves of slice n > k:
//   lesser (n > 2k):  rhoL_m = Lbar_{m,n} M_R^{-1}           (m < n-k)
//   mixing:           rhoT_t = M_R^{-H} Tbar_{n,t}            (t = 0..ntau)
//   retarded:         rhoR_m = M_R^{-H} Rbar_{n,m}            (m < n-k)
// and per-workgroup partial sums of M_Rbar = -sum rhoL^H L - sum rhoT T^H - sum rhoR R^H.
struct RhoGeom {
  int SL, ST, SR, wl, wt, wr;
};
__host__ __device__ inline RhoGeom rho_geom(int n, int k, int ntau, int cb) {
  RhoGeom g;
  g.SL = n > 2 * k ? n - k : 0;
  g.ST = ntau + 1;
  g.SR = n - k;
  g.wl = (g.SL + cb - 1) / cb;
  g.wt = (g.ST + cb - 1) / cb;
  g.wr = (g.SR + cb - 1) / cb;
  return g;
}

// element e of block b (global block index within the segment seg)
__host__ __device__ inline cplx rho_elem(const AdjView& V, int n, int seg, int b, int r, int c) {
  int d = V.d;
  const cplx* Mi = V.scr(V.lay.mrinv);
  if (seg == 0) {
    const cplx* l = V.aL(b, n);
    return dotq(d, [&](int q) { return l[r * d + q]; }, [&](int q) { return Mi[q * d + c]; });
  }
  const cplx* l = seg == 1 ? V.aT(n, b) : V.aR(n, b);
  return dotq(d, [&](int q) { return conj(Mi[q * d + r]); }, [&](int q) { return l[q * d + c]; });
}
// contribution of block b to M_Rbar[r][c] given its rho (full block)
__host__ __device__ inline cplx mr_term(const AdjView& V, int n, int seg, int b, const cplx* rho, int r, int c) {
  int d = V.d;
  if (seg == 0) {  // -rho^H L_{b,n}
    const cplx* L = V.GL(b, n);
    return -dotq(d, [&](int q) { return conj(rho[q * d + r]); }, [&](int q) { return L[q * d + c]; });
  }
  const cplx* X = seg == 1 ? V.GT(n, b) : V.GR(n, b);  // -rho X^H
  return -dotq(d, [&](int q) { return rho[r * d + q]; }, [&](int q) { return conj(X[c * d + q]); });
}

// ============================================================== Kscatter
// Adjoints of the history blocks of slices < n, one element per thread:
//   L(a, b), a <= b < n:  lesser bulk rows (n > 2k)
//   R(a, b), b <= a < n:  lesser C^<_1 rows and retarded bulk columns
//   T(a, t), a < n:       lesser C^<_3 rows and mixing columns
struct HistGeom {
  size_t oL, oR, oT, total;
};
__host__ __device__ inline HistGeom hist_geom(int n, int k, int ntau, int dd) {
  HistGeom g;
  size_t o = 0;
  g.oL = o; o += n > 2 * k ? tri(n) * dd : 0;
  g.oR = o; o += tri(n) * dd;
  g.oT = o; o += (size_t)n * (ntau + 1) * dd;
  g.total = o;
  return g;
}

__host__ __device__ inline void adj_hist_elem(const AdjProb& Ap, const KW& W, int n, size_t idx) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k, ntau = V.ntau;
  double h = V.h, ht = V.ht, xi = V.xi;
  HistGeom G = hist_geom(n, k, ntau, dd);
  if (idx >= G.total) return;
  const cplx* rL = V.scr(V.lay.rhoL);
  const cplx* rT = V.scr(V.lay.rhoT);
  const cplx* rR = V.scr(V.lay.rhoR);
  int e = (int)(idx % dd), r = e / d, c = e % d;
  int nb = n - k;  // bulk rows / columns are < nb
  bool lb = n > 2 * k;
  if (idx < G.oR) {
    size_t t = (idx - G.oL) / dd;
    int b = tri_row(t);
    int a = (int)(t - tri(b));
    cplx v = mk(0, 0);
    if (a < nb) {
      // row m = a, l = b >= a: -i h w_{n,b} rhoL_a S^R_{n,b} (+ BDF for b >= n-k)
      const cplx* g = rL + (size_t)a * dd;
      const cplx* s = V.SR(n, b);
      cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return s[q * d + c]; });
      v = v + mul_i(-(h * adj_w(W, n, b)) * u);
      int l = n - b;
      if (l >= 1 && l <= k) v = v - (W.a[l] / h) * g[e];
    }
    if (b < nb && a < b) {
      // row m = b, l = a < b (hermitian partner): -i h w_{n,a} S^R_{n,a}^H rhoL_b^H
      const cplx* g = rL + (size_t)b * dd;
      const cplx* s = V.SR(n, a);
      cplx u = dotq(d, [&](int q) { return conj(s[q * d + r]); }, [&](int q) { return conj(g[c * d + q]); });
      v = v + mul_i(-(h * adj_w(W, n, a)) * u);
    }
    V.aL(a, b)[e] = V.aL(a, b)[e] + v;
  } else if (idx < G.oT) {
    size_t t = (idx - G.oR) / dd;
    int a = tri_row(t);
    int b = (int)(t - tri(a));
    cplx v = mk(0, 0);
    if (lb && a < nb) {
      // lesser row m = a, C^<_1 term j = b: -i h w rhoL_a S^<_{b,n}^H (w = s_{a,b} for a <= k)
      double wt = a > k ? adj_w(W, a, b) : W.s[a][b];
      const cplx* g = rL + (size_t)a * dd;
      const cplx* s = V.SL(b, n);
      cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return conj(s[c * d + q]); });
      v = v + mul_i(-(h * wt) * u);
    }
    if (lb && b < nb && b <= k && a <= k && a > b) {
      // lesser row m = b <= k, continuation Rt(G, b, a): -i h s_{b,a} S^<_{a,n} rhoL_b^H
      const cplx* g = rL + (size_t)b * dd;
      const cplx* s = V.SL(a, n);
      cplx u = dotq(d, [&](int q) { return s[r * d + q]; }, [&](int q) { return conj(g[c * d + q]); });
      v = v + mul_i(-(h * W.s[b][a]) * u);
    }
    if (b < nb) {
      // retarded column m = b: i h w_{n-b, a-b} S^R_{n,a}^H rhoR_b (+ BDF for a >= n-k)
      const cplx* g = rR + (size_t)b * dd;
      const cplx* s = V.SR(n, a);
      cplx u = dotq(d, [&](int q) { return conj(s[q * d + r]); }, [&](int q) { return g[q * d + c]; });
      v = v + mul_i((h * adj_w(W, n - b, a - b)) * u);
      int l = n - a;
      if (l >= 1 && l <= k) v = v - (W.a[l] / h) * g[e];
    }
    V.aR(a, b)[e] = V.aR(a, b)[e] + v;
  } else {
    size_t t = (idx - G.oT) / dd;
    int a = (int)(t / (ntau + 1)), tau = (int)(t % (ntau + 1));
    cplx v = mk(0, 0);
    if (lb && a < nb) {
      // lesser row m = a, C^<_3: -xi ht w_{ntau,tau} rhoL_a S^rceil_{n, ntau-tau}
      const cplx* g = rL + (size_t)a * dd;
      const cplx* s = V.ST(n, ntau - tau);
      cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return s[q * d + c]; });
      v = v + (-xi * ht * adj_w(W, ntau, tau)) * u;
    }
    {
      // mixing column tau: i h w_{n,a} S^R_{n,a}^H rhoT_tau (+ BDF for a >= n-k)
      const cplx* g = rT + (size_t)tau * dd;
      const cplx* s = V.SR(n, a);
      cplx u = dotq(d, [&](int q) { return conj(s[q * d + r]); }, [&](int q) { return g[q * d + c]; });
      v = v + mul_i((h * adj_w(W, n, a)) * u);
      int l = n - a;
      if (l >= 1 && l <= k) v = v - (W.a[l] / h) * g[e];
    }
    V.aT(a, tau)[e] = V.aT(a, tau)[e] + v;
  }
}

// ============================================================== KsigS
// Self-energy adjoints of slice n from the bulk row adjoints (reductions):
//   sR(n, j), j < n:   sum_{m<=j, m<n-k} i h w_{n-m,j-m} rhoR_m R_{j,m}^H
//                    + sum_t i h w_{n,j} rhoT_t T_{j,t}^H
//                    + sum_{m<n-k} i h w_{n,j} rhoL_m^H Lh(G, m, j)          (n > 2k)
//   sL(j, n), j <= n:  sum_m h w rhoL-terms of C^<_1                          (n > 2k)
//   sT(n, t):          sum_m -xi ht w_{ntau,ntau-t} rhoL_m^H T_{m, ntau-t}   (n > 2k)
// One output block per workgroup; term index split over lane groups.
struct SigGeom {
  int nR, nL, nT, total;
};
__host__ __device__ inline SigGeom sig_geom(int n, int k, int ntau) {
  SigGeom g;
  g.nR = n;
  g.nL = n > 2 * k ? n + 1 : 0;
  g.nT = n > 2 * k ? ntau + 1 : 0;
  g.total = g.nR + g.nL + g.nT;
  return g;
}
// Reduction terms of output block ob, over their exact ranges:
//   sR(n, j): m = 0..min(j, nb-1) (retarded), t = 0..ntau (mixing),
//             m = 0..nb-1 (lesser, n > 2k);
//   sL(j, n): m = 0..min(k, nb-1) when j <= k, then m = max(j, k+1)..nb-1;
//   sT(n, t): m = 0..nb-1.
// (nb = n - k bulk rows)
__host__ __device__ inline int sig_nterms(const AdjView& V, int n, int ob) {
  SigGeom G = sig_geom(n, V.k, V.ntau);
  int k = V.k, nb = n - k;
  if (ob < G.nR) {
    int j = ob, a = (j < nb - 1 ? j : nb - 1) + 1;
    return a + (V.ntau + 1) + (n > 2 * k ? nb : 0);
  }
  if (ob < G.nR + G.nL) {
    int j = ob - G.nR;
    int a = j <= k ? (k < nb - 1 ? k : nb - 1) + 1 : 0;
    int m0 = j > k + 1 ? j : k + 1;
    return a + (nb - m0 > 0 ? nb - m0 : 0);
  }
  return nb;
}
__host__ __device__ inline cplx sig_term(const AdjView& V, int n, int ob, int t, int r, int c) {
  SigGeom G = sig_geom(n, V.k, V.ntau);
  int d = V.d, k = V.k, ntau = V.ntau, nb = n - k;
  double h = V.h;
  const cplx* rL = V.scr(V.lay.rhoL);
  const cplx* rT = V.scr(V.lay.rhoT);
  const cplx* rR = V.scr(V.lay.rhoR);
  if (ob < G.nR) {
    int j = ob, na = (j < nb - 1 ? j : nb - 1) + 1;
    if (t < na) {
      int m = t;
      const cplx* g = rR + (size_t)m * V.dd;
      const cplx* R = V.GR(j, m);
      cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return conj(R[c * d + q]); });
      return mul_i((h * adj_w(V.W, n - m, j - m)) * u);
    }
    t -= na;
    if (t <= ntau) {
      const cplx* g = rT + (size_t)t * V.dd;
      const cplx* T = V.GT(j, t);
      cplx u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return conj(T[c * d + q]); });
      return mul_i((h * adj_w(V.W, n, j)) * u);
    }
    int m = t - (ntau + 1);
    const cplx* g = rL + (size_t)m * V.dd;
    cplx u = dotq(d, [&](int q) { return conj(g[q * d + r]); },
                  [&](int q) { return V.Lh(V.P.Gles, m, j, q, c); });
    return mul_i((h * adj_w(V.W, n, j)) * u);
  }
  if (ob < G.nR + G.nL) {
    int j = ob - G.nR;
    int na = j <= k ? (k < nb - 1 ? k : nb - 1) + 1 : 0;
    int m;
    double wt;
    if (t < na) {
      m = t;
      wt = V.W.s[m][j];  // m <= k: start weights, Rt continuation for j > m
    } else {
      m = (j > k + 1 ? j : k + 1) + (t - na);
      wt = adj_w(V.W, m, j);  // m > k, j <= m
    }
    const cplx* g = rL + (size_t)m * V.dd;
    // h w Rt(G, m, j)^H (-i rhoL_m)
    cplx u = dotq(d, [&](int q) { return conj(V.Rt(V.P.Gret, m, j, q, r)); }, [&](int q) { return g[q * d + c]; });
    return mul_i(-(h * wt) * u);
  }
  int tau = ob - G.nR - G.nL, m = t, j = ntau - tau;
  const cplx* g = rL + (size_t)m * V.dd;
  const cplx* T = V.GT(m, j);
  cplx u = dotq(d, [&](int q) { return conj(g[q * d + r]); }, [&](int q) { return T[q * d + c]; });
  return (-V.xi * V.ht * adj_w(V.W, ntau, j)) * u;
}
__host__ __device__ inline cplx* sig_out(const AdjView& V, int n, int ob) {
  SigGeom G = sig_geom(n, V.k, V.ntau);
  if (ob < G.nR) return V.sR(n, ob);
  if (ob < G.nR + G.nL) return V.sL(ob - G.nR, n);
  return V.sT(n, ob - G.nR - G.nL);
}

// ============================================================== Ktau
// Reverse of the tau source C^rceil_2 + C^rceil_3 [Sigma, 1, G](p, m) of
// row p (Eqs. ctv2, ctv3) for the column adjoints gc_m = i * src_m:
//   sT(p, a) += sum coef gc_m M_b^H,   aM(b) += sum coef Sigma^rceil_{p,a}^H gc_m
// over the terms (m, a, b, coef) of the forward rule. Outputs: ntau+1 blocks
// of sT (if formed) then ntau+1 blocks of aM (with_m = false: the Sigma^rceil
// part only, for trial steps).
// Term t of output x (the a of sT(p, a), or the b of aM(b)): sets the column
// m, the partner block y (b, or a) and coef; false past the last term.
__host__ __device__ inline int tau_nterms(int k, int nt, bool isM, int x) {
  int kk = (k + 1) * (k + 1), c;
  if (!isM) {
    c = (x <= k ? kk : 0) + (x >= nt - k ? kk : 0);
    int m0 = x > k + 1 ? x : k + 1;
    c += nt - m0 + 1 > 0 ? nt - m0 + 1 : 0;
    int m1 = x < nt - k - 1 ? x : nt - k - 1;
    c += m1 + 1 > 0 ? m1 + 1 : 0;
  } else {
    c = (x >= nt - k ? kk : 0) + (x <= k ? kk : 0);
    int m0 = nt - x > k + 1 ? nt - x : k + 1;
    c += nt - m0 + 1 > 0 ? nt - m0 + 1 : 0;
    int m1 = nt - x < nt - k - 1 ? nt - x : nt - k - 1;
    c += m1 + 1 > 0 ? m1 + 1 : 0;
  }
  return c;
}
__host__ __device__ inline bool tau_term(const KW& W, int k, int nt, double ht, double xi, bool isM, int x, int t,
                                         int& m, int& y, double& coef) {
  int kk = (k + 1) * (k + 1);
  if (!isM) {
    int a = x;
    if (a <= k) {
      if (t < kk) {
        m = t / (k + 1);
        int j = t % (k + 1);
        y = nt - j;
        coef = ht * xi * W.R[m][j][a];
        return true;
      }
      t -= kk;
    }
    int m0 = a > k + 1 ? a : k + 1, n2 = nt - m0 + 1 > 0 ? nt - m0 + 1 : 0;
    if (t < n2) {
      m = m0 + t;
      y = nt - m + a;
      coef = ht * xi * adj_w(W, m, m - a);
      return true;
    }
    t -= n2;
    if (a >= nt - k) {
      if (t < kk) {
        m = nt - k + t / (k + 1);
        int j = t % (k + 1);
        y = j;
        coef = ht * W.R[nt - m][j][nt - a];
        return true;
      }
      t -= kk;
    }
    int m1 = a < nt - k - 1 ? a : nt - k - 1;
    if (t <= m1) {
      m = t;
      y = a - m;
      coef = ht * adj_w(W, nt - m, a - m);
      return true;
    }
    return false;
  }
  int b = x;
  if (b >= nt - k) {
    if (t < kk) {
      m = t / (k + 1);
      int l = t % (k + 1);
      y = l;
      coef = ht * xi * W.R[m][nt - b][l];
      return true;
    }
    t -= kk;
  }
  int m0 = nt - b > k + 1 ? nt - b : k + 1, n2 = nt - m0 + 1 > 0 ? nt - m0 + 1 : 0;
  if (t < n2) {
    m = m0 + t;
    y = m - nt + b;
    coef = ht * xi * adj_w(W, m, nt - b);
    return true;
  }
  t -= n2;
  if (b <= k) {
    if (t < kk) {
      m = nt - k + t / (k + 1);
      int l = t % (k + 1);
      y = nt - l;
      coef = ht * W.R[nt - m][b][l];
      return true;
    }
    t -= kk;
  }
  int m1 = nt - b < nt - k - 1 ? nt - b : nt - k - 1;
  if (t <= m1) {
    m = t;
    y = m + b;
    coef = ht * adj_w(W, nt - m, b);
    return true;
  }
  return false;
}
// output block ob of a launch (sT blocks first when formed), decoded
__host__ __device__ inline bool tau_out(const AdjProb& Ap, int nt, int ob, bool with_m, bool& isM, int& x) {
  bool sig = Ap.sT != nullptr;
  int nout = ((sig ? 1 : 0) + (with_m ? 1 : 0)) * (nt + 1);
  if (ob >= nout) return false;
  isM = !sig || ob > nt;
  x = isM ? (sig ? ob - nt - 1 : ob) : ob;
  return true;
}
// contribution of term t to element (r, c) of output (isM, x)
__host__ __device__ inline cplx tau_contrib(const AdjView& V, int p, const cplx* src, bool isM, int x, int t, int r,
                                            int c) {
  int m, y;
  double coef;
  if (!tau_term(V.W, V.k, V.ntau, V.ht, V.xi, isM, x, t, m, y, coef)) return mk(0, 0);
  int d = V.d;
  const cplx* g = src + (size_t)m * V.dd;  // gc_m = i g
  cplx u;
  if (!isM) {
    const cplx* M = V.GM(y);
    u = dotq(d, [&](int q) { return g[r * d + q]; }, [&](int q) { return conj(M[c * d + q]); });
  } else {
    const cplx* S = V.ST(p, y);
    u = dotq(d, [&](int q) { return conj(S[q * d + r]); }, [&](int q) { return g[q * d + c]; });
  }
  return mul_i(coef * u);
}
__host__ __device__ inline cplx* tau_dst(const AdjView& V, int p, bool isM, int x) {
  return isM ? V.aM(x) : V.sT(p, x);
}
// element form (one thread per output element, all terms)
__host__ __device__ inline void adj_tau_elem(const AdjProb& Ap, const KW& W, int p, const cplx* src,
                                             size_t idx, bool with_m = true) {
  AdjView V(Ap, W);
  int dd = V.dd;
  bool isM;
  int x;
  if (!tau_out(Ap, V.ntau, (int)(idx / dd), with_m, isM, x)) return;
  int e = (int)(idx % dd);
  cplx v = mk(0, 0);
  int nterm = tau_nterms(V.k, V.ntau, isM, x);
  for (int t = 0; t < nterm; t++) v = v + tau_contrib(V, p, src, isM, x, t, e / V.d, e % V.d);
  cplx* o = tau_dst(V, p, isM, x);
  o[e] = o[e] + v;
}

// ============================================================== K3
// Retarded boundary of slice n (conjugate start-up, Eq. MBCVSAMx_cc_start)
// and the eps_n / Sigma^R_{n,n} adjoints from the summed M_Rbar partials.
//   Y C = -Y_0 C_0  with Y_l = R_{n,n-l},  C(l,p) = h^-1 D_{p,l} + delta_{pl} i e_{n-p}
//                                                 + i h s_{p,l} Sigma~^R_{n-l,n-p}
//   Psi = Ybar C^{-H}: C Psi^H = Ybar^H ;  Cbar(l,p) = -Y_l^H Psi_p
__host__ __device__ inline int adj_rb_lds(int d, int k) { return k * d * k * d + 3 * k * d * d + d * d + ADJ_NT; }

__host__ __device__ inline bool adj_rbound_team(const AdjProb& Ap, const KW& W, int n, int nparts, int tid,
                                                int nth, cplx* lds, int* piv) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k, kd = k * d;
  double h = V.h;
  cplx* Cb = lds;
  cplx* X = Cb + kd * kd;  // kd x d: Psi^H blocks
  cplx* gm = X + kd * d;   // d x d
  bool ok = true;
  // M_Rbar: the workgroup partials, split over thread groups (fixed order)
  const cplx* part = V.scr(V.lay.part);
  int grp = dd >= nth ? 1 : nth / dd;
  cplx* gs = gm + dd;  // grp x dd
  for (int t = tid; t < grp * dd; t += nth) {
    int gg = t / dd, e = t % dd;
    cplx s = mk(0, 0);
    for (int w = gg; w < nparts; w += grp) s = s + part[(size_t)w * dd + e];
    gs[t] = s;
  }
  ADJ_SYNC();
  for (int e = tid; e < dd; e += nth) {
    cplx s = mk(0, 0);
    for (int gg = 0; gg < grp; gg++) s = s + gs[gg * dd + e];
    gm[e] = s;
  }
  ADJ_SYNC();
  for (int e = tid; e < dd; e += nth) {
    // eps_n += -i M_Rbar ; Sigma^R_{n,n} += -i h w_{n,n} M_Rbar
    V.ge(n)[e] = V.ge(n)[e] + mul_i(-1.0 * gm[e]);
    if (V.A.sR) V.sR(n, n)[e] = V.sR(n, n)[e] + mul_i(-(h * adj_w(W, n, n)) * gm[e]);
  }
  for (int e = tid; e < kd * kd; e += nth) Cb[e] = V.scr(V.lay.cbinv)[e];  // C^{-1}, adj_prep_team
  ADJ_SYNC();
  // X = C^{-1} Ybar^H, Ybar^H block l = aR(n, n-l)^H
  for (int e = tid; e < kd * d; e += nth) {
    int R = e / d, c = e % d;
    cplx s = mk(0, 0);
    for (int q = 0; q < kd; q++) {
      int l = 1 + q / d, qq = q % d;
      cfma(s, Cb[R * kd + q], conj(V.aR(n, n - l)[c * d + qq]));
    }
    X[e] = s;
  }
  ADJ_SYNC();
  // Psi_p[r][c] = conj(X[(p-1)d + c][r])
  auto Psi = [&](int p, int rr, int cc) { return conj(X[((p - 1) * d + cc) * d + rr]); };
  auto Y = [&](int l, int rr, int cc) -> cplx {
    if (l == 0) return rr == cc ? mk(0, -1) : mk(0, 0);
    return V.GR(n, n - l)[rr * d + cc];
  };
  for (int e = tid; e < kd * d; e += nth) {
    int p = 1 + e / dd, r = (e % dd) / d, c = e % d;
    // eps_{n-p} += i Y_p^H Psi_p
    cplx u = dotq(d, [&](int q) { return conj(Y(p, q, r)); }, [&](int q) { return Psi(p, q, c); });
    V.ge(n - p)[r * d + c] = V.ge(n - p)[r * d + c] + mul_i(u);
  }
  ADJ_SYNC();
  if (V.A.sR) {
    // targets (n-l, n-p), 0 <= l <= p <= k, p >= 1:
    //   V(l,p) = i h s_{p,l} Y_l^H Psi_p  and, for 1 <= l < p, -V(p,l)^H = i h s_{l,p} Psi_l^H Y_p
    int nb = k * (k + 3) / 2;  // pairs with p >= 1, 0 <= l <= p
    for (int e = tid; e < nb * dd; e += nth) {
      int t = e / dd, r = (e % dd) / d, c = e % d;
      int p = 1;
      while (t >= p + 1) {
        t -= p + 1;
        p++;
      }
      int l = t;
      cplx u = dotq(d, [&](int q) { return conj(Y(l, q, r)); }, [&](int q) { return Psi(p, q, c); });
      cplx v = mul_i((h * W.s[p][l]) * u);
      if (l >= 1 && l < p) {
        cplx u2 = dotq(d, [&](int q) { return conj(Psi(l, q, r)); }, [&](int q) { return Y(p, q, c); });
        v = v + mul_i((h * W.s[l][p]) * u2);
      }
      V.sR(n - l, n - p)[r * d + c] = V.sR(n - l, n - p)[r * d + c] + v;
    }
  }
  ADJ_SYNC();
  return ok;
}

// ============================================================== per-slice set-up
// Inverses of the local matrices of slice n > k, which depend on Sigma and eps
// only (fixed during the sweep): M_R (bulk rows), A_m for the serial rows m
// (n-k..n, or k+1..n for n <= 2k) and the retarded-boundary matrix C.
__host__ __device__ inline int adj_prep_lds(int d, int k) { return k * d * k * d; }

__host__ __device__ inline bool adj_prep_team(const AdjProb& Ap, const KW& W, int n, int tid, int nth, cplx* lds,
                                              int* piv) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k, kd = k * d;
  double h = V.h;
  bool ok = true;
  cplx* A = lds;
  // M_R = h^-1 a_0 + i e_n + i h w_{n,n} Sigma^R_{n,n}
  for (int e = tid; e < dd; e += nth) {
    int r = e / d, c = e % d;
    cplx v = mul_i((h * adj_w(W, n, n)) * V.SR(n, n)[e]) + mul_i(V.eh(n, r, c));
    if (r == c) v.x += W.a[0] / h;
    A[e] = v;
  }
  ADJ_SYNC();
  ok = team_inverse(d, A, piv, tid, nth) && ok;
  for (int e = tid; e < dd; e += nth) V.scr(V.lay.mrinv)[e] = A[e];
  ADJ_SYNC();
  int mlo = n > 2 * k ? n - k : k + 1;
  for (int m = mlo; m <= n; m++) {
    for (int e = tid; e < dd; e += nth) {
      int r = e / d, c = e % d;
      cplx v = mul_i((h * adj_w(W, m, m)) * V.SR(m, m)[e]) + mul_i(V.eh(m, r, c));
      if (r == c) v.x += W.a[0] / h;
      A[e] = v;
    }
    ADJ_SYNC();
    ok = team_inverse(d, A, piv, tid, nth) && ok;
    for (int e = tid; e < dd; e += nth) V.scr(V.lay.ainv)[(size_t)(m - mlo) * dd + e] = A[e];
    ADJ_SYNC();
  }
  // C(l,p) = h^-1 D_{p,l} + delta_{pl} i e_{n-p} + i h s_{p,l} Sigma~^R_{n-l,n-p}, l, p = 1..k
  for (int e = tid; e < kd * kd; e += nth) {
    int R = e / kd, C = e % kd;
    int l = 1 + R / d, p = 1 + C / d, r = R % d, c = C % d;
    cplx v = mul_i((h * W.s[p][l]) * V.Rt(V.P.Sret, n - l, n - p, r, c));
    if (r == c) v.x += W.D[p][l] / h;
    if (p == l) v = v + mul_i(V.eh(n - p, r, c));
    A[e] = v;
  }
  ADJ_SYNC();
  ok = team_inverse(kd, A, piv, tid, nth) && ok;
  for (int e = tid; e < kd * kd; e += nth) V.scr(V.lay.cbinv)[e] = A[e];
  ADJ_SYNC();
  return ok;
}

// ============================================================== start-up, mixing
// B = [start_block(p, l)]_{p,l=1..k} is shared by every tau index; psi(m) =
// B^{-H} [Tbar_{p,m}]_p. tstart_inv inverts B into scratch.
__host__ __device__ inline bool adj_tinv_team(const AdjProb& Ap, const KW& W, int tid, int nth, cplx* lds,
                                              int* piv) {
  AdjView V(Ap, W);
  int d = V.d, k = V.k, kd = k * d;
  for (int e = tid; e < kd * kd; e += nth) {
    int R = e / kd, C = e % kd;
    lds[e] = start_block_elem(V, 1 + R / d, 1 + C / d, R % d, C % d);
  }
  ADJ_SYNC();
  bool ok = team_inverse(kd, lds, piv, tid, nth);
  for (int e = tid; e < kd * kd; e += nth) V.scr(V.lay.binv)[e] = lds[e];
  ADJ_SYNC();
  return ok;
}
// psi_p(m)[r][c] = sum_q conj(Binv[q][(p-1)d + r]) lambda(m)[q][c]; stored at psi + ((p-1)(ntau+1) + m) dd
__host__ __device__ inline void adj_tpsi_elem(const AdjProb& Ap, const KW& W, size_t idx) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k, kd = k * d, nt1 = V.ntau + 1;
  if (idx >= (size_t)k * nt1 * dd) return;
  int e = (int)(idx % dd), r = e / d, c = e % d;
  int t = (int)(idx / dd), p = 1 + t / nt1, m = t % nt1;
  const cplx* Bi = V.scr(V.lay.binv);
  cplx s = mk(0, 0);
  for (int q = 0; q < kd; q++) cfma(s, conj(Bi[q * kd + (p - 1) * d + r]), V.aT(1 + q / d, m)[(q % d) * d + c]);
  V.scr(V.lay.psi)[((size_t)(p - 1) * nt1 + m) * dd + e] = s;
}
// y_0 = T_{0,m} = i xi M_{ntau-m}: gy0 = Tbar_{0,m} - sum_p B_{p,0}^H psi_p(m); aM(ntau-m) += -i xi gy0
__host__ __device__ inline void adj_ty0_elem(const AdjProb& Ap, const KW& W, size_t idx) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k, nt1 = V.ntau + 1;
  if (idx >= (size_t)nt1 * dd) return;
  int e = (int)(idx % dd), r = e / d, c = e % d, m = (int)(idx / dd);
  cplx g = V.aT(0, m)[e];
  for (int p = 1; p <= k; p++) {
    const cplx* ps = V.scr(V.lay.psi) + ((size_t)(p - 1) * nt1 + m) * dd;
    g = g - dotq(d, [&](int q) { return conj(start_block_elem(V, p, 0, q, r)); }, [&](int q) { return ps[q * d + c]; });
  }
  V.aM(V.ntau - m)[e] = V.aM(V.ntau - m)[e] + mul_i(-V.xi * g);
}
// P(p, l) = sum_m psi_p(m) T_{l,m}^H, p = 1..k, l = 0..k: reduction terms
__host__ __device__ inline cplx adj_tp_term(const AdjView& V, int ob, int m, int r, int c) {
  int d = V.d, k = V.k, nt1 = V.ntau + 1;
  int p = 1 + ob / (k + 1), l = ob % (k + 1);
  const cplx* ps = V.scr(V.lay.psi) + ((size_t)(p - 1) * nt1 + m) * V.dd;
  const cplx* T = V.GT(l, m);
  return dotq(d, [&](int q) { return ps[r * d + q]; }, [&](int q) { return conj(T[c * d + q]); });
}

// ============================================================== start-up, retarded
// Finalises the mixing start-up sums (eps_p += i P(p,p); Sigma~^R_{p,l} +=
// i h s_{p,l} P(p,l)) and reverses the retarded start-up columns m = k-1..0:
//   A(p,l) = i h^-1 D_{p,l} - delta_{pl} e_p - h I_{m,p,l} Sigma~^R_{p,l},
//   sum_l A(p,l) y_l = 0 (p = m+1..k), y_l = -[R_{m,l}]^dag (l < m), y_m = -i.
__host__ __device__ inline int adj_rs_lds(int d, int k) { return k * d * k * d + 2 * k * d * d; }

__host__ __device__ inline bool adj_rstart_team(const AdjProb& Ap, const KW& W, int tid, int nth, cplx* lds,
                                                int* piv) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, k = V.k;
  double h = V.h;
  bool ok = true;
  const cplx* P = V.scr(V.lay.pst);
  auto Pb = [&](int p, int l) { return P + (size_t)((p - 1) * (k + 1) + l) * dd; };
  for (int e = tid; e < k * dd; e += nth) {
    int p = 1 + e / dd, ee = e % dd;
    V.ge(p)[ee] = V.ge(p)[ee] + mul_i(Pb(p, p)[ee]);
  }
  if (V.A.sR) {
    int nb = (k + 1) * (k + 2) / 2;
    for (int e = tid; e < nb * dd; e += nth) {
      int t = e / dd, r = (e % dd) / d, c = e % d;
      int a = 0;
      while ((a + 1) * (a + 2) / 2 <= t) a++;
      int b = t - a * (a + 1) / 2;
      cplx v = mk(0, 0);
      if (a >= 1) v = v + mul_i((h * W.s[a][b]) * Pb(a, b)[r * d + c]);
      if (b >= 1 && a > b) v = v + mul_i((h * W.s[b][a]) * conj(Pb(b, a)[c * d + r]));
      V.sR(a, b)[r * d + c] = V.sR(a, b)[r * d + c] + v;
    }
  }
  ADJ_SYNC();
  cplx* A = lds;
  cplx* lam = A + k * d * k * d;
  cplx* psi = lam + k * d * d;
  for (int m = k - 1; m >= 0; m--) {
    int nu = k - m, N = nu * d;
    auto yl = [&](int l, int rr, int cc) -> cplx {
      if (l < m) return -conj(V.GR(m, l)[cc * d + rr]);
      if (l == m) return rr == cc ? mk(0, -1) : mk(0, 0);
      return V.GR(l, m)[rr * d + cc];
    };
    auto Ael = [&](int p, int l, int rr, int cc) -> cplx {
      cplx v = (-(h * W.I[m][p][l])) * V.Rt(V.P.Sret, p, l, rr, cc);
      if (rr == cc) v = v + mk(0, W.D[p][l] / h);
      if (p == l) v = v - V.eh(p, rr, cc);
      return v;
    };
    // A^H in LDS: (A^H)[(p'..)][(l'..)] = conj(A[l'][p'])
    for (int e = tid; e < N * N; e += nth) {
      int R = e / N, C = e % N;
      A[e] = conj(Ael(m + 1 + C / d, m + 1 + R / d, C % d, R % d));
    }
    for (int e = tid; e < N * d; e += nth) {
      int p = m + 1 + e / dd, ee = e % dd;
      lam[e] = V.aR(p, m)[ee];
    }
    ADJ_SYNC();
    ok = team_inverse(N, A, piv, tid, nth) && ok;
    for (int e = tid; e < N * d; e += nth) {
      int R = e / d, c = e % d;
      cplx s = mk(0, 0);
      for (int q = 0; q < N; q++) cfma(s, A[R * N + q], lam[q * d + c]);
      psi[e] = s;
    }
    ADJ_SYNC();
    auto ps = [&](int p, int rr, int cc) { return psi[(p - m - 1) * dd + rr * d + cc]; };
    for (int e = tid; e < N * d; e += nth) {
      int p = m + 1 + e / dd, r = (e % dd) / d, c = e % d;
      // eps_p += psi_p y_p^H
      cplx u = dotq(d, [&](int q) { return ps(p, r, q); }, [&](int q) { return conj(yl(p, c, q)); });
      V.ge(p)[r * d + c] = V.ge(p)[r * d + c] + u;
    }
    // R_{m,l} (l < m) += sum_p psi_p^H A(p,l)
    for (int e = tid; e < m * dd; e += nth) {
      int l = e / dd, r = (e % dd) / d, c = e % d;
      cplx s = mk(0, 0);
      for (int p = m + 1; p <= k; p++)
        s = s + dotq(d, [&](int q) { return conj(ps(p, q, r)); }, [&](int q) { return Ael(p, l, q, c); });
      V.aR(m, l)[r * d + c] = V.aR(m, l)[r * d + c] + s;
    }
    if (V.A.sR) {
      // Sigma~^R_{p,l} += h I_{m,p,l} psi_p y_l^H, stored targets (a, b), a >= b
      int nb = (k + 1) * (k + 2) / 2;
      for (int e = tid; e < nb * dd; e += nth) {
        int t = e / dd, r = (e % dd) / d, c = e % d;
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= t) a++;
        int b = t - a * (a + 1) / 2;
        cplx v = mk(0, 0);
        if (a > m) {
          cplx u = dotq(d, [&](int q) { return ps(a, r, q); }, [&](int q) { return conj(yl(b, c, q)); });
          v = v + (h * W.I[m][a][b]) * u;
        }
        if (b > m && a > b) {
          // -(h I_{m,b,a} psi_b y_a^H)^H = -h I_{m,b,a} y_a psi_b^H
          cplx u = dotq(d, [&](int q) { return yl(a, r, q); }, [&](int q) { return conj(ps(b, c, q)); });
          v = v - (h * W.I[m][b][a]) * u;
        }
        V.sR(a, b)[r * d + c] = V.sR(a, b)[r * d + c] + v;
      }
    }
    ADJ_SYNC();
  }
  return ok;
}

// ============================================================== second-Born chain
// With Sigma = Sigma_2B[G] (elementwise in the orbital indices, per slice)
// and eps = eps0 + Hartree[G], slice s of G is a fixed point of the step that
// produces it. Its adjoint nu_s solves
//   nu_s = gbar_s + Sigma_2B'(G_s)^* (sbar_s + S_s(nu_s)) + Hartree'(G_s)^* (ebar_s + E_s(nu_s)),
// where gbar_s, sbar_s, ebar_s collect the later slices' contributions and
// S_s, E_s are the Sigma / eps adjoints that the reverse step of slice s
// itself returns for the input nu_s. The sweep iterates this map per slice
// (per start-up block of slices 0..k) on windows, then applies the reverse
// step once more, for good, with the final nu.

// element counts of slices lo..hi (R row, L column, T row per slice)
__host__ __device__ inline size_t win_elems(int lo, int hi, int ntau, int dd) {
  return (2 * (tri(hi + 1) - tri(lo)) + (size_t)(hi - lo + 1) * (ntau + 1)) * dd;
}
// decode a window element index: slice s, component (0 R, 1 L, 2 T), block j, element e
__host__ __device__ inline void win_decode(size_t idx, int lo, int hi, int ntau, int dd, int& s, int& comp,
                                           int& j, int& e) {
  s = lo;
  size_t t = idx / dd;
  e = (int)(idx % dd);
  while (s < hi) {
    size_t c = (size_t)2 * (s + 1) + ntau + 1;
    if (t < c) break;
    t -= c;
    s++;
  }
  if (t < (size_t)(s + 1)) {
    comp = 0;
    j = (int)t;
  } else if (t < (size_t)2 * (s + 1)) {
    comp = 1;
    j = (int)(t - (s + 1));
  } else {
    comp = 2;
    j = (int)(t - 2 * (s + 1));
  }
}
__host__ __device__ inline cplx* win_at(const AdjView& V, const AdjWin& w, int comp, int s, int j) {
  return comp == 0 ? V.wR(w, s, j) : (comp == 1 ? V.wL(w, j, s) : V.wT(w, s, j));
}

// Window copies of slices lo..hi:
//   mode 0: g0 <- Gbar, s0 <- Sigmabar, e0 <- eps_bar         (before the iteration)
//   mode 1: gdry <- nu[b], sdry <- s0, gedry <- e0             (before a trial step)
//   mode 2: Gbar <- nu[b]                                       (commit)
__host__ __device__ inline void adj_wcopy_elem(const AdjProb& Ap, const KW& W, int mode, int lo, int hi, int b,
                                               size_t idx) {
  AdjView V(Ap, W);
  int dd = V.dd;
  size_t nw = win_elems(lo, hi, V.ntau, dd);
  if (idx < nw) {
    int s, comp, j, e;
    win_decode(idx, lo, hi, V.ntau, dd, s, comp, j, e);
    if (mode == 0) {
      cplx* g = comp == 0 ? V.aR(s, j) : (comp == 1 ? V.aL(j, s) : V.aT(s, j));
      cplx* x = comp == 0 ? V.sR(s, j) : (comp == 1 ? V.sL(j, s) : V.sT(s, j));
      win_at(V, Ap.g0, comp, s, j)[e] = g[e];
      win_at(V, Ap.s0, comp, s, j)[e] = x[e];
    } else if (mode == 1) {
      win_at(V, Ap.gdry, comp, s, j)[e] = win_at(V, Ap.nu[b], comp, s, j)[e];
      win_at(V, Ap.sdry, comp, s, j)[e] = win_at(V, Ap.s0, comp, s, j)[e];
    } else {
      cplx* g = comp == 0 ? V.aR(s, j) : (comp == 1 ? V.aL(j, s) : V.aT(s, j));
      g[e] = win_at(V, Ap.nu[b], comp, s, j)[e];
    }
    return;
  }
  idx -= nw;
  if (mode == 2 || idx >= (size_t)(hi - lo + 1) * dd) return;
  int s = lo + (int)(idx / dd), e = (int)(idx % dd);
  if (mode == 0)
    Ap.e0[(size_t)(s - lo) * dd + e] = V.ge(s)[e];
  else
    Ap.gedry[(size_t)(s + 1) * dd + e] = Ap.e0[(size_t)(s - lo) * dd + e];
}

// nu[b] = g0 + Sigma_2B'^*(sbar) + Hartree'^*(ebar) on slices lo..hi, with
// (sbar, ebar) = (s0, e0) for src 0 and the trial step's (sdry, gedry) for src 1.
//   Sigma^<_ab(j,s) = u L_ab^2 (R_ba - conj L_ab),
//   Sigma^R_ab(s,j) = u [(R_ab - conj L_ba)^2 L_ba - conj(L_ba)^2 (L_ba - conj R_ab)],  u = U_s U_j,
//   Sigma^rceil_ab(s,m) = U_s U_{-1} T_ab(s,m)^2 (-xi conj T_ab(s, ntau-m)),
//   eps_ii(s) += U_s (Re(i xi L_ii(s,s)) - nbar).
// For w = f(z, conj z): zbar += conj(df/dz) wbar + (df/dconj z) conj(wbar).
__host__ __device__ inline void adj_sig2b_elem(const AdjProb& Ap, const KW& W, int lo, int hi, int src, int b,
                                               size_t idx) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, ntau = V.ntau;
  double xi = V.xi;
  if (idx >= win_elems(lo, hi, ntau, dd)) return;
  int s, comp, j, e;
  win_decode(idx, lo, hi, ntau, dd, s, comp, j, e);
  int p = e / d, q = e % d;
  const AdjWin& S = src == 0 ? Ap.s0 : Ap.sdry;
  auto u = [&](int t) { return Ap.U[t + 1]; };
  cplx v = win_at(V, Ap.g0, comp, s, j)[e];
  if (comp == 0) {
    double uu = u(s) * u(j);
    cplx Lqp = V.GL(j, s)[q * d + p], Rpq = V.GR(s, j)[p * d + q];
    cplx wL = V.wL(S, j, s)[q * d + p], wR = V.wR(S, s, j)[p * d + q];
    v = v + conj(uu * (Lqp * Lqp)) * wL;
    cplx A = Rpq - conj(Lqp);
    cplx fR = (2.0 * uu) * (A * Lqp), fRc = uu * (conj(Lqp) * conj(Lqp));
    v = v + conj(fR) * wR + fRc * conj(wR);
  } else if (comp == 1) {
    double uu = u(s) * u(j);
    cplx Lpq = V.GL(j, s)[p * d + q], Rqp = V.GR(s, j)[q * d + p];
    cplx wL = V.wL(S, j, s)[p * d + q], wR = V.wR(S, s, j)[q * d + p];
    cplx fl = (2.0 * uu) * (Lpq * (Rqp - conj(Lpq))), flc = -uu * (Lpq * Lpq);
    v = v + conj(fl) * wL + flc * conj(wL);
    cplx A = Rqp - conj(Lpq);
    cplx fL = uu * (A * A - conj(Lpq) * conj(Lpq));
    cplx fLc = uu * ((-2.0) * (A * Lpq) - 2.0 * (conj(Lpq) * Lpq) + 2.0 * (conj(Lpq) * conj(Rqp)));
    v = v + conj(fL) * wR + fLc * conj(wR);
    if (j == s && p == q) {
      const cplx* eb = src == 0 ? Ap.e0 + (size_t)(s - lo) * dd : Ap.gedry + (size_t)(s + 1) * dd;
      v = v + mk(0, -xi * u(s) * eb[p * d + p].x);
    }
  } else {
    int m = j;
    double uT = u(s) * u(-1);
    cplx x = V.GT(s, m)[e], y = V.GT(s, ntau - m)[e];
    cplx vt = -xi * conj(y);
    cplx w = V.wT(S, s, m)[e], w2 = V.wT(S, s, ntau - m)[e];
    v = v + conj((2.0 * uT) * (x * vt)) * w + (-xi * uT) * (y * y) * conj(w2);
  }
  win_at(V, Ap.nu[b], comp, s, j)[e] = v;
}

// max |nu[0] - nu[1]| and max |nu[1]| over slices lo..hi (team), to conv[2 slot]
__host__ __device__ inline void adj_conv_team(const AdjProb& Ap, const KW& W, int lo, int hi, int slot, int tid,
                                              int nth, double* red) {
  AdjView V(Ap, W);
  size_t nw = win_elems(lo, hi, V.ntau, V.dd);
  double dm = 0.0, vm = 0.0;
  for (size_t i = tid; i < nw; i += nth) {
    int s, comp, j, e;
    win_decode(i, lo, hi, V.ntau, V.dd, s, comp, j, e);
    if (comp == 0 && j == s) continue;  // R_{s,s} is fixed
    cplx a = win_at(V, Ap.nu[0], comp, s, j)[e], c = win_at(V, Ap.nu[1], comp, s, j)[e];
    double x = sqrt(abs2(a - c)), y = sqrt(abs2(c));
    dm = x > dm ? x : dm;
    vm = y > vm ? y : vm;
  }
  red[2 * tid] = dm;
  red[2 * tid + 1] = vm;
  ADJ_SYNC();
  if (tid == 0) {
    for (int t = 1; t < nth; t++) {
      dm = red[2 * t] > dm ? red[2 * t] : dm;
      vm = red[2 * t + 1] > vm ? red[2 * t + 1] : vm;
    }
    Ap.conv[2 * slot] = dm;
    Ap.conv[2 * slot + 1] = vm;
  }
  ADJ_SYNC();
}

// dJ/dU from the final Sigma and eps adjoints of slice s (team):
//   Ubar_j += U_s c_j, Ubar_s += U_j c_j (c_j: column j of R and L),
//   Ubar_s += U_{-1} c_T + c_H, Ubar_{-1} += U_s c_T.
__host__ __device__ inline void adj_ugrad_team(const AdjProb& Ap, const KW& W, int s, int tid, int nth,
                                               double* red) {
  AdjView V(Ap, W);
  int d = V.d, dd = V.dd, ntau = V.ntau;
  double xi = V.xi;
  auto u = [&](int t) { return Ap.U[t + 1]; };
  double accS = 0.0, accT = 0.0;
  for (int j = tid; j <= s; j += nth) {
    double c = 0.0;
    for (int e = 0; e < dd; e++) {
      int a = e / d, b = e % d;
      cplx Lab = V.GL(j, s)[a * d + b], Lba = V.GL(j, s)[b * d + a];
      cplx Rab = V.GR(s, j)[a * d + b], Rba = V.GR(s, j)[b * d + a];
      cplx wL = V.sL(j, s)[e], wR = V.sR(s, j)[e];
      cplx pl = (Lab * Lab) * (Rba - conj(Lab));
      cplx A = Rab - conj(Lba);
      cplx pr = (A * A) * Lba - (conj(Lba) * conj(Lba)) * (Lba - conj(Rab));
      c += (conj(wL) * pl).x + (conj(wR) * pr).x;
    }
    if (j < s) Ap.ub[j + 1] += u(s) * c;
    accS += u(j) * c + (j == s ? u(s) * c : 0.0);
  }
  for (int m = tid; m <= ntau; m += nth)
    for (int e = 0; e < dd; e++) {
      cplx x = V.GT(s, m)[e], y = V.GT(s, ntau - m)[e];
      cplx w = V.sT(s, m)[e];
      accT += (conj(w) * ((x * x) * (-xi * conj(y)))).x;
    }
  red[2 * tid] = accS;
  red[2 * tid + 1] = accT;
  ADJ_SYNC();
  if (tid == 0) {
    double cs = 0.0, ct = 0.0;
    for (int t = 0; t < nth; t++) {
      cs += red[2 * t];
      ct += red[2 * t + 1];
    }
    double ch = 0.0;
    for (int i = 0; i < d; i++) {
      cplx L = V.GL(s, s)[i * d + i];
      double rho = -xi * L.y;  // Re(i xi L)
      ch += V.ge(s)[i * d + i].x * (rho - Ap.nbar);
    }
    Ap.ub[s + 1] += cs + u(-1) * ct + ch;
    Ap.ub[0] += u(s) * ct;
  }
  ADJ_SYNC();
}

// ============================================================== Matsubara
// Reverse of the self-consistent Matsubara solve of the second-Born run
// (Eq. Gmat_dyson_integ: A M = g with A = 1 - B[K], K = [g * Sigma^M]^M by
// Eqs. cm1, cm2, g the free function of eps_{-1}; Sigma^M = Sigma_2B[M],
// eps_{-1} = eps0_{-1} + Hartree[M]). Its adjoint nu solves
//   nu = Mbar + Sigma_2B'^*(Sigmabar^M(nu)) + Hartree'^*(epsbar(nu)),
//   gA = A^{-H} nu,  Kbar_J = sum c gA_m M_l^H over the terms c K_J of B_{m,l},
//   gbar = gA + cm-reverse (Kbar, Sigma^M),  Sigmabar^M = cm-reverse (g, Kbar),
//   epsbar = sum_m V (Gamma_m o (V^H gbar_m V)) V^H   (Daleckii-Krein, g_m = V f_m(x) V^H),
// iterated with the damping of the forward loop.
struct MadjBuf {
  cplx *Ainv, *g, *gA, *Kb, *gb, *Sb, *nu, *nun, *eb, *V;
  double *x, *red;
};

// gA = Ainv^H nu ; N x d
__host__ __device__ inline void madj_ga_elem(int N, int d, const cplx* Ainv, const cplx* nu, cplx* gA, size_t idx) {
  if (idx >= (size_t)N * d) return;
  int r = (int)(idx / d), c = (int)(idx % d);
  cplx s = mk(0, 0);
  for (int q = 0; q < N; q++) cfma(s, conj(Ainv[(size_t)q * N + r]), nu[(size_t)q * d + c]);
  gA[idx] = s;
}

// Kbar_J[p][q] = sum c (gA_m M_col^H)[p][q] over the terms c K_J of B_{m,col}
__host__ __device__ inline void madj_kbar_elem(const Prob& P, const KW& W, const cplx* gA, cplx* Kb, size_t idx) {
  int d = P.d, dd = d * d, nt = P.ntau, k = P.k;
  if (idx >= (size_t)(nt + 1) * dd) return;
  int J = (int)(idx / dd), e = (int)(idx % dd), p = e / d, q = e % d;
  double ht = P.htau, xi = P.sig;
  cplx v = mk(0, 0);
  auto add = [&](int m, int col, double c) {
    const cplx* g = gA + (size_t)m * dd;
    const cplx* M = P.Gmat + (size_t)col * dd;
    v = v + c * dotq(d, [&](int t) { return g[p * d + t]; }, [&](int t) { return conj(M[q * d + t]); });
  };
  if (J <= k)
    for (int m = 0; m <= k; m++)
      for (int l = 0; l <= k; l++) add(m, l, ht * W.R[m][J][l]);
  for (int m = J > k + 1 ? J : k + 1; m <= nt; m++) add(m, m - J, ht * adj_w(W, m, m - J));
  if (J >= nt - k)
    for (int m = nt - k; m <= nt; m++)
      for (int l = 0; l <= k; l++) add(m, nt - l, ht * xi * W.R[nt - m][nt - J][l]);
  for (int m = 0; m <= (J < nt - k - 1 ? J : nt - k - 1); m++) add(m, m + nt - J, ht * xi * adj_w(W, nt - m, nt - J));
  Kb[idx] = v;
}

// gbar_a = gA_a + sum c Kbar_m Sigma^M_b^H, Sigmabar^M_b = sum c g_a^H Kbar_m over the
// terms c g_a Sigma^M_b of K_m (Eqs. cm1, cm2)
__host__ __device__ inline void madj_conv_elem(const Prob& P, const KW& W, const MadjBuf& B, size_t idx) {
  int d = P.d, dd = d * d, nt = P.ntau, k = P.k;
  size_t nb = (size_t)(nt + 1) * dd;
  if (idx >= 2 * nb) return;
  bool sig = idx >= nb;
  size_t i2 = sig ? idx - nb : idx;
  int X = (int)(i2 / dd), e = (int)(i2 % dd), p = e / d, q = e % d;
  double ht = P.htau, xi = P.sig;
  cplx v = sig ? mk(0, 0) : B.gA[i2];
  if (!sig) {
    int a = X;
    auto add = [&](int m, int b, double c) {
      const cplx* K = B.Kb + (size_t)m * dd;
      const cplx* S = P.Smat + (size_t)b * dd;
      v = v + c * dotq(d, [&](int t) { return K[p * d + t]; }, [&](int t) { return conj(S[q * d + t]); });
    };
    if (a <= k)
      for (int m = 0; m <= k; m++)
        for (int l = 0; l <= k; l++) add(m, l, ht * W.R[m][a][l]);
    for (int m = a > k + 1 ? a : k + 1; m <= nt; m++) add(m, m - a, ht * adj_w(W, m, m - a));
    if (a >= nt - k)
      for (int m = nt - k; m <= nt; m++)
        for (int l = 0; l <= k; l++) add(m, nt - l, ht * xi * W.R[nt - m][nt - a][l]);
    for (int m = 0; m <= (a < nt - k - 1 ? a : nt - k - 1); m++) add(m, m + nt - a, ht * xi * adj_w(W, nt - m, nt - a));
    B.gb[i2] = v;
  } else {
    int b = X;
    auto add = [&](int m, int a, double c) {
      const cplx* K = B.Kb + (size_t)m * dd;
      const cplx* g = B.g + (size_t)a * dd;
      v = v + c * dotq(d, [&](int t) { return conj(g[t * d + p]); }, [&](int t) { return K[t * d + q]; });
    };
    if (b <= k)
      for (int m = 0; m <= k; m++)
        for (int j = 0; j <= k; j++) add(m, j, ht * W.R[m][j][b]);
    for (int m = b > k + 1 ? b : k + 1; m <= nt; m++) add(m, m - b, ht * adj_w(W, m, b));
    if (b >= nt - k)
      for (int m = nt - k; m <= nt; m++)
        for (int j = 0; j <= k; j++) add(m, nt - j, ht * xi * W.R[nt - m][j][nt - b]);
    for (int m = 0; m <= (b < nt - k - 1 ? b : nt - k - 1); m++) add(m, nt - b + m, ht * xi * adj_w(W, nt - m, b - m));
    B.Sb[i2] = v;
  }
}

// f(x, tau) of the free function and its x-derivative (overflow-free forms)
__host__ __device__ inline double madj_f(double x, double tau, double beta, double xi) {
  if (x >= 0 || xi > 0) return -exp(-x * tau) / (1 - xi * exp(-beta * x));
  return -exp(x * (beta - tau)) / (exp(beta * x) - xi);
}
__host__ __device__ inline double madj_fp(double x, double tau, double beta, double xi) {
  double f = madj_f(x, tau, beta, xi);
  double q = x >= 0 ? xi * exp(-beta * x) / (1 - xi * exp(-beta * x)) : xi / (exp(beta * x) - xi);
  return f * (-tau - beta * q);
}

// eigen-decomposition of eps_{-1} - mu (thread 0 of the team)
__host__ __device__ inline void madj_eig_team(const Prob& P, const MadjBuf& B, int tid, cplx* A) {
  if (tid != 0) return;
  int d = P.d;
  for (int e = 0; e < d * d; e++) {
    A[e] = P.eps[e];
    if (e / d == e % d) A[e].x -= P.mu;
  }
  herm_jacobi(d, A, B.V, B.x);
}

// epsbar = sum_m V (Gamma_m o (V^H gbar_m V)) V^H (team; red: >= max(nth, dd) + dd complex)
__host__ __device__ inline void madj_eps_team(const Prob& P, const MadjBuf& B, int tid, int nth, cplx* red) {
  int d = P.d, dd = d * d, nt = P.ntau;
  double beta = P.beta, xi = P.sig;
  int lanes = dd >= nth ? 1 : nth / dd, slots = lanes * dd;
  for (int t = tid; t < slots; t += nth) {
    int e = t % dd, lane = t / dd, a = e / d, b = e % d;
    double xa = B.x[a], xb = B.x[b];
    bool deg = fabs(xa - xb) <= 1e-9 * (1 + fabs(xa));
    cplx y = mk(0, 0);
    for (int m = lane; m <= nt; m += lanes) {
      double tau = m * P.htau;
      double gm = deg ? madj_fp(xa, tau, beta, xi)
                      : (madj_f(xa, tau, beta, xi) - madj_f(xb, tau, beta, xi)) / (xa - xb);
      const cplx* G = B.gb + (size_t)m * dd;
      cplx u = mk(0, 0);
      for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) cfma(u, conj(B.V[i * d + a]), G[i * d + j] * B.V[j * d + b]);
      y = y + gm * u;
    }
    red[t] = y;
  }
  ADJ_SYNC();
  cplx* Y = red + slots;
  for (int e = tid; e < dd; e += nth) {
    cplx s = mk(0, 0);
    for (int l = 0; l < lanes; l++) s = s + red[l * dd + e];
    Y[e] = s;
  }
  ADJ_SYNC();
  for (int e = tid; e < dd; e += nth) {
    int pp = e / d, qq = e % d;
    cplx s = mk(0, 0);
    for (int i = 0; i < d; i++)
      for (int j = 0; j < d; j++) cfma(s, B.V[pp * d + i], Y[i * d + j] * conj(B.V[qq * d + j]));
    B.eb[e] = s;
  }
  ADJ_SYNC();
}

// nun = Mbar + Sigma_2B'^*(Sigmabar^M) + Hartree'^*(epsbar):
//   Sigma^M_ab(m) = -xi U^2 M_ab(m)^2 M_ba(nt-m),  eps_ii += U (Re(-M_ii(nt)) - nbar)
__host__ __device__ inline void madj_nu_elem(const Prob& P, const MadjBuf& B, const cplx* Mbar, double u, size_t idx) {
  int d = P.d, dd = d * d, nt = P.ntau;
  if (idx >= (size_t)(nt + 1) * dd) return;
  int m = (int)(idx / dd), e = (int)(idx % dd), a = e / d, b = e % d;
  double xi = P.sig, c2 = -xi * u * u;
  const cplx* M = P.Gmat;
  cplx x = M[(size_t)m * dd + a * d + b], y = M[(size_t)(nt - m) * dd + b * d + a];
  cplx v = Mbar[idx];
  v = v + conj((2.0 * c2) * (x * y)) * B.Sb[idx];
  v = v + conj(c2 * (y * y)) * B.Sb[(size_t)(nt - m) * dd + b * d + a];
  if (m == nt && a == b) v.x += -u * B.eb[a * d + a].x;
  B.nun[idx] = v;
}

// nu <- mix nun + (1 - mix) nu
__host__ __device__ inline void madj_mix_elem(const Prob& P, const MadjBuf& B, double mix, size_t idx) {
  if (idx >= (size_t)(P.ntau + 1) * P.d * P.d) return;
  B.nu[idx] = mix * B.nun[idx] + (1 - mix) * B.nu[idx];
}

// max |nun - nu| and max |nun| (team) into red[0], red[1]
__host__ __device__ inline void madj_change_team(const Prob& P, const MadjBuf& B, int tid, int nth) {
  size_t n = (size_t)(P.ntau + 1) * P.d * P.d;
  double dm = 0, vm = 0;
  for (size_t i = tid; i < n; i += nth) {
    double x = sqrt(abs2(B.nun[i] - B.nu[i])), y = sqrt(abs2(B.nun[i]));
    dm = x > dm ? x : dm;
    vm = y > vm ? y : vm;
  }
  B.red[2 + 2 * tid] = dm;
  B.red[3 + 2 * tid] = vm;
  ADJ_SYNC();
  if (tid == 0) {
    for (int t = 0; t < nth; t++) {
      dm = B.red[2 + 2 * t] > dm ? B.red[2 + 2 * t] : dm;
      vm = B.red[3 + 2 * t] > vm ? B.red[3 + 2 * t] : vm;
    }
    B.red[0] = dm;
    B.red[1] = vm;
  }
  ADJ_SYNC();
}

// dJ/dU_{-1} += sum Re(conj(Sigmabar^M) dSigma^M/dU) + Hartree part ; epsbar_{-1} += epsbar (team)
__host__ __device__ inline void madj_final_team(const Prob& P, const MadjBuf& B, double u, double nbar, double* ub,
                                                cplx* ge0, int tid, int nth) {
  int d = P.d, dd = d * d, nt = P.ntau;
  double xi = P.sig;
  const cplx* M = P.Gmat;
  double acc = 0;
  for (size_t i = tid; i < (size_t)(nt + 1) * dd; i += nth) {
    int m = (int)(i / dd), e = (int)(i % dd), a = e / d, b = e % d;
    cplx x = M[i], y = M[(size_t)(nt - m) * dd + b * d + a];
    acc += (conj(B.Sb[i]) * ((-2.0 * xi * u) * (x * x * y))).x;
  }
  B.red[2 + tid] = acc;
  ADJ_SYNC();
  if (tid == 0) {
    double s = 0;
    for (int t = 0; t < nth; t++) s += B.red[2 + t];
    for (int i = 0; i < d; i++) s += B.eb[i * d + i].x * (-M[(size_t)nt * dd + i * d + i].x - nbar);
    ub[0] += s;
    for (int e = 0; e < dd; e++) ge0[e] = ge0[e] + B.eb[e];
  }
  ADJ_SYNC();
}

// ============================================================== device kernels
constexpr int ADJ_LDS = 4000;  // complex entries of the team kernels' LDS (64000 B)

__device__ inline void adj_fail(const AdjProb& A) { *A.stat = 1; }

__global__ void __launch_bounds__(ADJ_NT) k_adj_lcol(const AdjProb* ap, int n) {
  __shared__ cplx lds[ADJ_LDS];
  __shared__ int piv[72];
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  if (!adj_lcol_team(A, c_kw[A.p.k], n, threadIdx.x, blockDim.x, lds, piv) && threadIdx.x == 0) adj_fail(A);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_lcol_scatter(const AdjProb* ap, int n) {
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  adj_lcol_elem(A, c_kw[A.p.k], n, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_rho(const AdjProb* ap, int n) {
  __shared__ cplx rho[ADJ_NT];
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  int dd = V.dd, cb = V.lay.cb;
  RhoGeom g = rho_geom(n, V.k, V.ntau, cb);
  int w = blockIdx.x;
  if (w >= g.wl + g.wt + g.wr) return;
  int seg = w < g.wl ? 0 : (w < g.wl + g.wt ? 1 : 2);
  int wb = seg == 0 ? w : (seg == 1 ? w - g.wl : w - g.wl - g.wt);
  int cnt = seg == 0 ? g.SL : (seg == 1 ? g.ST : g.SR);
  int b0 = wb * cb, nbk = cnt - b0 < cb ? cnt - b0 : cb;
  cplx* dst = V.scr(seg == 0 ? V.lay.rhoL : (seg == 1 ? V.lay.rhoT : V.lay.rhoR));
  int t = threadIdx.x;
  if (t < nbk * dd) {
    int b = b0 + t / dd, e = t % dd;
    cplx v = rho_elem(V, n, seg, b, e / V.d, e % V.d);
    rho[t] = v;
    dst[(size_t)b * dd + e] = v;
  }
  __syncthreads();
  if (t < dd) {
    cplx s = mk(0, 0);
    for (int bb = 0; bb < nbk; bb++) s = s + mr_term(V, n, seg, b0 + bb, rho + bb * dd, t / V.d, t % V.d);
    V.scr(V.lay.part)[(size_t)w * dd + t] = s;
  }
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_hist(const AdjProb* ap, int n) {
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  adj_hist_elem(A, c_kw[A.p.k], n, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
// one output block per workgroup: dd element rows x (ADJ_NT / dd) term lanes
template <class NT, class TERM, class OUT>
__device__ inline void team_reduce_block(int dd, NT nterms, TERM term, OUT out) {
  __shared__ cplx red[ADJ_NT];
  int lanes = dd >= ADJ_NT ? 1 : ADJ_NT / dd;
  int t = threadIdx.x, e = t % dd, lane = t / dd;
  cplx s = mk(0, 0);
  if (lane < lanes && t < lanes * dd) {
    int nt = nterms();
    int i = lane;
    // four independent terms per round keep their loads in flight together
    for (; i + 3 * lanes < nt; i += 4 * lanes) {
      cplx a0 = term(i, e), a1 = term(i + lanes, e), a2 = term(i + 2 * lanes, e), a3 = term(i + 3 * lanes, e);
      s = s + ((a0 + a1) + (a2 + a3));
    }
    for (; i < nt; i += lanes) s = s + term(i, e);
  }
  red[t] = s;
  __syncthreads();
  if (t < dd) {
    cplx acc = mk(0, 0);
    for (int l = 0; l < lanes; l++) acc = acc + red[l * dd + t];
    out(e, acc);
  }
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_sigma(const AdjProb* ap, int n) {
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  int ob = blockIdx.x;
  if (ob >= sig_geom(n, V.k, V.ntau).total) return;
  int d = V.d;
  team_reduce_block(
      V.dd, [&]() { return sig_nterms(V, n, ob); },
      [&](int i, int e) { return sig_term(V, n, ob, i, e / d, e % d); },
      [&](int e, cplx v) {
        cplx* o = sig_out(V, n, ob);
        o[e] = o[e] + v;
      });
}
// The same reductions for d <= 4 with the orbital count known at compile
// time: a thread forms whole d x d block terms (each block loaded once, the
// products unrolled), threads t, t + 256, ... take the terms of the output
// block in turn, and the 256 block sums are added in a fixed order.
template <int D>
__device__ inline void blk_ld(cplx (&b)[D * D], const cplx* p) {
#pragma unroll
  for (int e = 0; e < D * D; e++) b[e] = p[e];
}
// extended blocks: R~_{a,b} (a < b: -(R_{b,a})^dag) and L^_{a,b} (a > b: -(L_{b,a})^dag)
template <int D>
__device__ inline void blk_rt(cplx (&b)[D * D], const AdjView& V, int a, int c) {
  if (a >= c) {
    blk_ld<D>(b, V.GR(a, c));
  } else {
    const cplx* p = V.GR(c, a);
#pragma unroll
    for (int x = 0; x < D; x++)
#pragma unroll
      for (int y = 0; y < D; y++) b[x * D + y] = -conj(p[y * D + x]);
  }
}
template <int D>
__device__ inline void blk_lh(cplx (&b)[D * D], const AdjView& V, int a, int c) {
  if (a <= c) {
    blk_ld<D>(b, V.GL(a, c));
  } else {
    const cplx* p = V.GL(c, a);
#pragma unroll
    for (int x = 0; x < D; x++)
#pragma unroll
      for (int y = 0; y < D; y++) b[x * D + y] = -conj(p[y * D + x]);
  }
}
// acc += f X Y^H  and  acc += f X^H Y
template <int D>
__device__ inline void blk_abh(cplx (&acc)[D * D], cplx f, const cplx (&X)[D * D], const cplx (&Y)[D * D]) {
#pragma unroll
  for (int r = 0; r < D; r++)
#pragma unroll
    for (int c = 0; c < D; c++) {
      cplx u = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(u, X[r * D + q], conj(Y[c * D + q]));
      acc[r * D + c] = acc[r * D + c] + f * u;
    }
}
template <int D>
__device__ inline void blk_ahb(cplx (&acc)[D * D], cplx f, const cplx (&X)[D * D], const cplx (&Y)[D * D]) {
#pragma unroll
  for (int r = 0; r < D; r++)
#pragma unroll
    for (int c = 0; c < D; c++) {
      cplx u = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(u, conj(X[q * D + r]), Y[q * D + c]);
      acc[r * D + c] = acc[r * D + c] + f * u;
    }
}
// term t of output block ob (the terms of sig_term, as whole blocks)
template <int D>
__device__ inline void sig_term_blk(const AdjView& V, int n, int ob, int t, cplx (&acc)[D * D]) {
  constexpr int DD = D * D;
  SigGeom G = sig_geom(n, V.k, V.ntau);
  int k = V.k, ntau = V.ntau, nb = n - k;
  double h = V.h;
  const cplx* rL = V.scr(V.lay.rhoL);
  const cplx* rT = V.scr(V.lay.rhoT);
  const cplx* rR = V.scr(V.lay.rhoR);
  cplx X[DD], Y[DD];
  if (ob < G.nR) {
    int j = ob, na = (j < nb - 1 ? j : nb - 1) + 1;
    if (t < na) {
      int m = t;
      blk_ld<D>(X, rR + (size_t)m * DD);
      blk_ld<D>(Y, V.GR(j, m));
      blk_abh<D>(acc, mk(0, h * adj_w(V.W, n - m, j - m)), X, Y);
      return;
    }
    t -= na;
    if (t <= ntau) {
      blk_ld<D>(X, rT + (size_t)t * DD);
      blk_ld<D>(Y, V.GT(j, t));
      blk_abh<D>(acc, mk(0, h * adj_w(V.W, n, j)), X, Y);
      return;
    }
    int m = t - (ntau + 1);
    blk_ld<D>(X, rL + (size_t)m * DD);
    blk_lh<D>(Y, V, m, j);
    blk_ahb<D>(acc, mk(0, h * adj_w(V.W, n, j)), X, Y);
    return;
  }
  if (ob < G.nR + G.nL) {
    int j = ob - G.nR;
    int na = j <= k ? (k < nb - 1 ? k : nb - 1) + 1 : 0;
    int m;
    double wt;
    if (t < na) {
      m = t;
      wt = V.W.s[m][j];
    } else {
      m = (j > k + 1 ? j : k + 1) + (t - na);
      wt = adj_w(V.W, m, j);
    }
    blk_rt<D>(X, V, m, j);
    blk_ld<D>(Y, rL + (size_t)m * DD);
    blk_ahb<D>(acc, mk(0, -(h * wt)), X, Y);
    return;
  }
  int tau = ob - G.nR - G.nL, m = t, j = ntau - tau;
  blk_ld<D>(X, rL + (size_t)m * DD);
  blk_ld<D>(Y, V.GT(m, j));
  blk_ahb<D>(acc, mk(-V.xi * V.ht * adj_w(V.W, ntau, j), 0), X, Y);
}
template <int D>
__global__ void __launch_bounds__(ADJ_NT) k_adj_sigma_blk(const AdjProb* ap, int n) {
  constexpr int DD = D * D, NG = ADJ_NT / DD;
  __shared__ cplx red[DD][ADJ_NT];
  __shared__ cplx red2[NG][DD];
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  int ob = blockIdx.x;
  if (ob >= sig_geom(n, V.k, V.ntau).total) return;
  int tid = threadIdx.x;
  cplx acc[DD];
#pragma unroll
  for (int e = 0; e < DD; e++) acc[e] = mk(0, 0);
  int nt = sig_nterms(V, n, ob);
  for (int t = tid; t < nt; t += ADJ_NT) sig_term_blk<D>(V, n, ob, t, acc);
#pragma unroll
  for (int e = 0; e < DD; e++) red[e][tid] = acc[e];
  __syncthreads();
  if (tid < NG * DD) {  // group g sums the threads g, g + NG, g + 2 NG, ... element by element
    int e = tid % DD, g = tid / DD;
    cplx v = mk(0, 0);
    for (int i = g; i < ADJ_NT; i += NG) v = v + red[e][i];
    red2[g][e] = v;
  }
  __syncthreads();
  if (tid < DD) {
    cplx v = mk(0, 0);
    for (int g = 0; g < NG; g++) v = v + red2[g][tid];
    cplx* o = sig_out(V, n, ob);
    o[tid] = o[tid] + v;
  }
}
// The same reductions for d >= 5: a d x d block term does not fit a thread's
// registers, so the output block is split into four sub-blocks of
// SB = ceil(d / 2) rows and columns; thread (sub-block, lane) accumulates its
// sub-block over the terms lane, lane + 64, ... (per term it loads SB rows
// or columns of each factor: a quarter of the element-per-thread loads),
// and the 64 lane sums of each element are added in a fixed order.
// acc += f X Y^H (AHB false) or acc += f X^H Y (AHB true) on the sub-block
// at (r0, c0); X(a, b), Y(a, b) give block elements.
template <int D, int SB, bool AHB, class XA, class YA>
__device__ inline void sub_term(cplx (&acc)[SB * SB], cplx f, int r0, int c0, XA X, YA Y) {
#pragma unroll 2
  for (int q = 0; q < D; q++) {
    cplx xs[SB], ys[SB];
#pragma unroll
    for (int i = 0; i < SB; i++) {
      int r = r0 + i;
      xs[i] = r < D ? f * (AHB ? conj(X(q, r)) : X(r, q)) : mk(0, 0);
    }
#pragma unroll
    for (int j = 0; j < SB; j++) {
      int c = c0 + j;
      ys[j] = c < D ? (AHB ? Y(q, c) : conj(Y(c, q))) : mk(0, 0);
    }
#pragma unroll
    for (int i = 0; i < SB; i++)
#pragma unroll
      for (int j = 0; j < SB; j++) cfma(acc[i * SB + j], xs[i], ys[j]);
  }
}
// element accessors of a stored block and of the conjugate transpose of one
// (-(P_{b,a})^dag: the continued R~ and L^ blocks)
template <int D>
struct BlkA {
  const cplx* p;
  bool tr;
  __device__ inline cplx operator()(int a, int b) const { return tr ? -conj(p[b * D + a]) : p[a * D + b]; }
};
// term t of output block ob on the thread's sub-block (the terms of sig_term_blk)
template <int D, int SB>
__device__ inline void sig_term_sub(const AdjView& V, int n, int ob, int t, int r0, int c0, cplx (&acc)[SB * SB]) {
  constexpr int DD = D * D;
  SigGeom G = sig_geom(n, V.k, V.ntau);
  int k = V.k, ntau = V.ntau, nb = n - k;
  double h = V.h;
  const cplx* rL = V.scr(V.lay.rhoL);
  const cplx* rT = V.scr(V.lay.rhoT);
  const cplx* rR = V.scr(V.lay.rhoR);
  if (ob < G.nR) {
    int j = ob, na = (j < nb - 1 ? j : nb - 1) + 1;
    if (t < na) {
      int m = t;
      sub_term<D, SB, false>(acc, mk(0, h * adj_w(V.W, n - m, j - m)), r0, c0, BlkA<D>{rR + (size_t)m * DD, false},
                             BlkA<D>{V.GR(j, m), false});
      return;
    }
    t -= na;
    if (t <= ntau) {
      sub_term<D, SB, false>(acc, mk(0, h * adj_w(V.W, n, j)), r0, c0, BlkA<D>{rT + (size_t)t * DD, false},
                             BlkA<D>{V.GT(j, t), false});
      return;
    }
    int m = t - (ntau + 1);
    BlkA<D> Y = m <= j ? BlkA<D>{V.GL(m, j), false} : BlkA<D>{V.GL(j, m), true};
    sub_term<D, SB, true>(acc, mk(0, h * adj_w(V.W, n, j)), r0, c0, BlkA<D>{rL + (size_t)m * DD, false}, Y);
    return;
  }
  if (ob < G.nR + G.nL) {
    int j = ob - G.nR;
    int na = j <= k ? (k < nb - 1 ? k : nb - 1) + 1 : 0;
    int m;
    double wt;
    if (t < na) {
      m = t;
      wt = V.W.s[m][j];
    } else {
      m = (j > k + 1 ? j : k + 1) + (t - na);
      wt = adj_w(V.W, m, j);
    }
    BlkA<D> X = m >= j ? BlkA<D>{V.GR(m, j), false} : BlkA<D>{V.GR(j, m), true};
    sub_term<D, SB, true>(acc, mk(0, -(h * wt)), r0, c0, X, BlkA<D>{rL + (size_t)m * DD, false});
    return;
  }
  int tau = ob - G.nR - G.nL, m = t, j = ntau - tau;
  sub_term<D, SB, true>(acc, mk(-V.xi * V.ht * adj_w(V.W, ntau, j), 0), r0, c0, BlkA<D>{rL + (size_t)m * DD, false},
                        BlkA<D>{V.GT(m, j), false});
}
// the 64 lanes' sums of the four sub-blocks, added in a fixed order, onto o
template <int D, int SB, int NL>
__device__ inline void sub_flush(cplx (&acc)[SB * SB], cplx* red, cplx* o) {
  int tid = threadIdx.x, sb = tid & 3, lane = tid >> 2;
#pragma unroll
  for (int e = 0; e < SB * SB; e++) red[(sb * NL + lane) * SB * SB + e] = acc[e];
  __syncthreads();
  if (tid < D * D) {
    int r = tid / D, c = tid % D, s2 = (r / SB) * 2 + c / SB, e = (r % SB) * SB + c % SB;
    cplx v = mk(0, 0);
    for (int l = 0; l < NL; l++) v = v + red[(s2 * NL + l) * SB * SB + e];
    o[tid] = o[tid] + v;
  }
}
template <int D>
__global__ void __launch_bounds__(ADJ_NT) __attribute__((amdgpu_waves_per_eu(2))) k_adj_sigma_sub(const AdjProb* ap,
                                                                                               int n) {
  constexpr int SB = (D + 1) / 2, NL = ADJ_NT / 4;
  __shared__ cplx red[4 * NL * SB * SB];
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  int ob = blockIdx.x;
  if (ob >= sig_geom(n, V.k, V.ntau).total) return;
  int tid = threadIdx.x, sb = tid & 3, lane = tid >> 2;
  int r0 = (sb >> 1) * SB, c0 = (sb & 1) * SB;
  cplx acc[SB * SB];
#pragma unroll
  for (int e = 0; e < SB * SB; e++) acc[e] = mk(0, 0);
  int nt = sig_nterms(V, n, ob);
  for (int t = lane; t < nt; t += NL) sig_term_sub<D, SB>(V, n, ob, t, r0, c0, acc);
  sub_flush<D, SB, NL>(acc, red, sig_out(V, n, ob));
}
// tau terms (tau_contrib) on the thread's sub-block
template <int D>
__global__ void __launch_bounds__(ADJ_NT) k_adj_tau_sub(const AdjProb* ap, int p, int srcsel, int with_m) {
  constexpr int SB = (D + 1) / 2, NL = ADJ_NT / 4, DD = D * D;
  __shared__ cplx red[4 * NL * SB * SB];
  const AdjProb& A = ap[blockIdx.y];
  if (p > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  bool isM;
  int x;
  if (!tau_out(A, V.ntau, blockIdx.x, with_m != 0, isM, x)) return;
  const cplx* src = srcsel == 0 ? V.scr(V.lay.rhoT) : V.scr(V.lay.psi) + (size_t)(p - 1) * (V.ntau + 1) * DD;
  int tid = threadIdx.x, sb = tid & 3, lane = tid >> 2;
  int r0 = (sb >> 1) * SB, c0 = (sb & 1) * SB;
  cplx acc[SB * SB];
#pragma unroll
  for (int e = 0; e < SB * SB; e++) acc[e] = mk(0, 0);
  int nterm = tau_nterms(V.k, V.ntau, isM, x);
  for (int t = lane; t < nterm; t += NL) {
    int m, y;
    double coef;
    if (!tau_term(V.W, V.k, V.ntau, V.ht, V.xi, isM, x, t, m, y, coef)) continue;
    BlkA<D> g{src + (size_t)m * DD, false};
    if (!isM) sub_term<D, SB, false>(acc, mk(0, coef), r0, c0, g, BlkA<D>{V.GM(y), false});
    else sub_term<D, SB, true>(acc, mk(0, coef), r0, c0, BlkA<D>{V.ST(p, y), false}, g);
  }
  sub_flush<D, SB, NL>(acc, red, tau_dst(V, p, isM, x));
}
// one output block per workgroup, the terms split over lane groups
__global__ void __launch_bounds__(ADJ_NT) k_adj_tau(const AdjProb* ap, int p, int srcsel, int with_m) {
  const AdjProb& A = ap[blockIdx.y];
  if (p > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  bool isM;
  int x;
  if (!tau_out(A, V.ntau, blockIdx.x, with_m != 0, isM, x)) return;
  const cplx* src = srcsel == 0 ? V.scr(V.lay.rhoT) : V.scr(V.lay.psi) + (size_t)(p - 1) * (V.ntau + 1) * V.dd;
  int d = V.d;
  team_reduce_block(
      V.dd, [&]() { return tau_nterms(V.k, V.ntau, isM, x); },
      [&](int t, int e) { return tau_contrib(V, p, src, isM, x, t, e / d, e % d); },
      [&](int e, cplx v) {
        cplx* o = tau_dst(V, p, isM, x);
        o[e] = o[e] + v;
      });
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_prep(const AdjProb* ap, int n) {
  __shared__ cplx lds[ADJ_LDS];
  __shared__ int piv[72];
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  if (!adj_prep_team(A, c_kw[A.p.k], n, threadIdx.x, blockDim.x, lds, piv) && threadIdx.x == 0) adj_fail(A);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_rbound(const AdjProb* ap, int n) {
  __shared__ cplx lds[ADJ_LDS];
  __shared__ int piv[72];
  const AdjProb& A = ap[blockIdx.y];
  if (n > A.p.nt) return;
  AdjView V(A, c_kw[A.p.k]);
  RhoGeom g = rho_geom(n, V.k, V.ntau, V.lay.cb);
  if (!adj_rbound_team(A, c_kw[A.p.k], n, g.wl + g.wt + g.wr, threadIdx.x, blockDim.x, lds, piv) &&
      threadIdx.x == 0)
    adj_fail(A);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_tinv(const AdjProb* ap) {
  __shared__ cplx lds[ADJ_LDS];
  __shared__ int piv[72];
  const AdjProb& A = ap[blockIdx.y];
  if (!adj_tinv_team(A, c_kw[A.p.k], threadIdx.x, blockDim.x, lds, piv) && threadIdx.x == 0) adj_fail(A);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_tpsi(const AdjProb* ap) {
  const AdjProb& A = ap[blockIdx.y];
  adj_tpsi_elem(A, c_kw[A.p.k], (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_ty0(const AdjProb* ap) {
  const AdjProb& A = ap[blockIdx.y];
  adj_ty0_elem(A, c_kw[A.p.k], (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_tp(const AdjProb* ap) {
  const AdjProb& A = ap[blockIdx.y];
  AdjView V(A, c_kw[A.p.k]);
  int ob = blockIdx.x;
  if (ob >= V.k * (V.k + 1)) return;
  int d = V.d;
  team_reduce_block(
      V.dd, [&]() { return V.ntau + 1; }, [&](int i, int e) { return adj_tp_term(V, ob, i, e / d, e % d); },
      [&](int e, cplx v) { V.scr(V.lay.pst)[(size_t)ob * V.dd + e] = v; });
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_rstart(const AdjProb* ap) {
  __shared__ cplx lds[ADJ_LDS];
  __shared__ int piv[72];
  const AdjProb& A = ap[blockIdx.y];
  if (!adj_rstart_team(A, c_kw[A.p.k], threadIdx.x, blockDim.x, lds, piv) && threadIdx.x == 0) adj_fail(A);
}

// Start of a block of slices lo..hi: window origins of every problem, and its
// trial copy with the adjoint arrays redirected to the windows (Sigma window
// from slice wlo, the first slice the trial step's boundary terms reach).
__global__ void k_adj_setdry(AdjProb* dry, AdjProb* ap, int lo, int wlo) {
  if (threadIdx.x != 0) return;
  int i = blockIdx.y;
  int ntau = ap[i].p.ntau;
  AdjWin* ws[5] = {&ap[i].g0, &ap[i].s0, &ap[i].nu[0], &ap[i].nu[1], &ap[i].gdry};
  for (int w = 0; w < 5; w++) {
    ws[w]->oR = tri(lo);
    ws[w]->oL = tri(lo);
    ws[w]->oT = (size_t)lo * (ntau + 1);
  }
  ap[i].sdry.oR = tri(wlo);
  ap[i].sdry.oL = tri(wlo);
  ap[i].sdry.oT = (size_t)wlo * (ntau + 1);
  AdjProb a = ap[i];
  a.aR = a.gdry.R;
  a.aL = a.gdry.L;
  a.aT = a.gdry.T;
  a.aoR = tri(lo);
  a.aoL = tri(lo);
  a.aoT = (size_t)lo * (ntau + 1);
  a.sR = a.sdry.R;
  a.sL = a.sdry.L;
  a.sT = a.sdry.T;
  a.soR = tri(wlo);
  a.soL = tri(wlo);
  a.soT = (size_t)wlo * (ntau + 1);
  a.ge = a.gedry;
  a.aM = a.mdummy;
  dry[i] = a;
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_wcopy(const AdjProb* ap, int mode, int lo, int hi, int b) {
  const AdjProb& A = ap[blockIdx.y];
  if (hi > A.p.nt) return;
  adj_wcopy_elem(A, c_kw[A.p.k], mode, lo, hi, b, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_sig2b(const AdjProb* ap, int lo, int hi, int src, int b) {
  const AdjProb& A = ap[blockIdx.y];
  if (hi > A.p.nt) return;
  adj_sig2b_elem(A, c_kw[A.p.k], lo, hi, src, b, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_conv(const AdjProb* ap, int lo, int hi, int slot) {
  __shared__ double red[2 * ADJ_NT];
  const AdjProb& A = ap[blockIdx.y];
  if (hi > A.p.nt) return;
  adj_conv_team(A, c_kw[A.p.k], lo, hi, slot, threadIdx.x, blockDim.x, red);
}
__global__ void __launch_bounds__(ADJ_NT) k_adj_ugrad(const AdjProb* ap, int s) {
  __shared__ double red[2 * ADJ_NT];
  const AdjProb& A = ap[blockIdx.y];
  if (s > A.p.nt) return;
  adj_ugrad_team(A, c_kw[A.p.k], s, threadIdx.x, blockDim.x, red);
}

__global__ void __launch_bounds__(ADJ_NT) k_madj_ga(int N, int d, const cplx* Ainv, const cplx* nu, cplx* gA) {
  madj_ga_elem(N, d, Ainv, nu, gA, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_kbar(Prob P, const cplx* gA, cplx* Kb) {
  madj_kbar_elem(P, c_kw[P.k], gA, Kb, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_conv(Prob P, MadjBuf B) {
  madj_conv_elem(P, c_kw[P.k], B, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_eig(Prob P, MadjBuf B) {
  __shared__ cplx A[64];
  madj_eig_team(P, B, threadIdx.x, A);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_eps(Prob P, MadjBuf B) {
  __shared__ cplx red[ADJ_NT + 64];
  madj_eps_team(P, B, threadIdx.x, blockDim.x, red);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_nu(Prob P, MadjBuf B, const cplx* Mbar, double u) {
  madj_nu_elem(P, B, Mbar, u, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_mix(Prob P, MadjBuf B, double mix) {
  madj_mix_elem(P, B, mix, (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_change(Prob P, MadjBuf B) {
  madj_change_team(P, B, threadIdx.x, blockDim.x);
}
__global__ void __launch_bounds__(ADJ_NT) k_madj_final(Prob P, MadjBuf B, double u, double nbar, double* ub,
                                                       cplx* ge0) {
  madj_final_team(P, B, u, nbar, ub, ge0, threadIdx.x, blockDim.x);
}

// ============================================================== host sequencing
// Launches the whole backward sweep for the problems in dA (host copies in hA,
// which share d, k and ntau): slices ntmax .. k+1, then the start-up.
inline unsigned adj_blocks(size_t elems) { return (unsigned)((elems + ADJ_NT - 1) / ADJ_NT); }

struct AdjShape {
  int count, k, d, ntau, dd, ntmax;
  bool sig;
};

// set-up of slice n > k (inverses of the local matrices; once per slice)
void adj_prep_launch(const AdjProb* dA, const AdjShape& S, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_prep, dim3(1, S.count), dim3(ADJ_NT), 0, s, dA, n);
}

// tau-term kernel of the orbital count: sub-blocks for d >= 5
static void adj_tau_launch(int d, dim3 g, hipStream_t s, const AdjProb* dA, int p, int srcsel, int with_m) {
  dim3 blk(ADJ_NT);
  switch (d) {
    case 5: hipLaunchKernelGGL(k_adj_tau_sub<5>, g, blk, 0, s, dA, p, srcsel, with_m); break;
    case 6: hipLaunchKernelGGL(k_adj_tau_sub<6>, g, blk, 0, s, dA, p, srcsel, with_m); break;
    case 7: hipLaunchKernelGGL(k_adj_tau_sub<7>, g, blk, 0, s, dA, p, srcsel, with_m); break;
    case 8: hipLaunchKernelGGL(k_adj_tau_sub<8>, g, blk, 0, s, dA, p, srcsel, with_m); break;
    default: hipLaunchKernelGGL(k_adj_tau, g, blk, 0, s, dA, p, srcsel, with_m); break;
  }
}

// reverse step of slice n > k (hist: also scatter into the history of slices < n)
void adj_step_launch(const AdjProb* dA, const AdjShape& S, int n, bool hist, hipStream_t s) {
  int k = S.k, ntau = S.ntau, dd = S.dd;
  dim3 blk(ADJ_NT);
  LcolGeom lg = lcol_geom(n, k, ntau, dd, S.sig);
  RhoGeom rg = rho_geom(n, k, ntau, adj_cb(dd));
  hipLaunchKernelGGL(k_adj_lcol, dim3(1, S.count), blk, 0, s, dA, n);
  hipLaunchKernelGGL(k_adj_lcol_scatter, dim3(adj_blocks(lg.total), S.count), blk, 0, s, dA, n);
  hipLaunchKernelGGL(k_adj_rho, dim3(rg.wl + rg.wt + rg.wr, S.count), blk, 0, s, dA, n);
  if (hist) {
    HistGeom hg = hist_geom(n, k, ntau, dd);
    hipLaunchKernelGGL(k_adj_hist, dim3(adj_blocks(hg.total), S.count), blk, 0, s, dA, n);
  }
  if (S.sig) {
    dim3 gs(sig_geom(n, k, ntau).total, S.count);
    switch (S.d) {
      case 1: hipLaunchKernelGGL(k_adj_sigma_blk<1>, gs, blk, 0, s, dA, n); break;
      case 2: hipLaunchKernelGGL(k_adj_sigma_blk<2>, gs, blk, 0, s, dA, n); break;
      case 3: hipLaunchKernelGGL(k_adj_sigma_blk<3>, gs, blk, 0, s, dA, n); break;
      case 4: hipLaunchKernelGGL(k_adj_sigma_blk<4>, gs, blk, 0, s, dA, n); break;
      case 5: hipLaunchKernelGGL(k_adj_sigma_sub<5>, gs, blk, 0, s, dA, n); break;
      case 6: hipLaunchKernelGGL(k_adj_sigma_sub<6>, gs, blk, 0, s, dA, n); break;
      case 7: hipLaunchKernelGGL(k_adj_sigma_sub<7>, gs, blk, 0, s, dA, n); break;
      case 8: hipLaunchKernelGGL(k_adj_sigma_sub<8>, gs, blk, 0, s, dA, n); break;
      default: hipLaunchKernelGGL(k_adj_sigma, gs, blk, 0, s, dA, n); break;
    }
  }
  // (a trial step, hist = false, needs no M adjoint)
  int nto = (S.sig ? 1 : 0) + (hist ? 1 : 0);
  if (nto) adj_tau_launch(S.d, dim3(nto * (ntau + 1), S.count), s, dA, n, 0, hist ? 1 : 0);
  hipLaunchKernelGGL(k_adj_rbound, dim3(1, S.count), blk, 0, s, dA, n);
}

// reverse of the start-up (slices 0..k)
void adj_start_launch(const AdjProb* dA, const AdjShape& S, hipStream_t s) {
  int k = S.k, ntau = S.ntau, dd = S.dd;
  dim3 blk(ADJ_NT);
  for (int n = k; n >= 0; n--) {
    LcolGeom lg = lcol_geom(n, k, ntau, dd, S.sig);
    hipLaunchKernelGGL(k_adj_lcol, dim3(1, S.count), blk, 0, s, dA, n);
    hipLaunchKernelGGL(k_adj_lcol_scatter, dim3(adj_blocks(lg.total), S.count), blk, 0, s, dA, n);
  }
  hipLaunchKernelGGL(k_adj_tpsi, dim3(adj_blocks((size_t)k * (ntau + 1) * dd), S.count), blk, 0, s, dA);
  hipLaunchKernelGGL(k_adj_ty0, dim3(adj_blocks((size_t)(ntau + 1) * dd), S.count), blk, 0, s, dA);
  hipLaunchKernelGGL(k_adj_tp, dim3(k * (k + 1), S.count), blk, 0, s, dA);
  for (int p = 1; p <= k; p++) adj_tau_launch(S.d, dim3((S.sig ? 2 : 1) * (ntau + 1), S.count), s, dA, p, 1, 1);
  hipLaunchKernelGGL(k_adj_rstart, dim3(1, S.count), blk, 0, s, dA);
}

AdjShape adj_shape(const AdjProb* hA, int count) {
  AdjShape S;
  S.count = count;
  S.k = hA[0].p.k;
  S.d = hA[0].p.d;
  S.ntau = hA[0].p.ntau;
  S.dd = S.d * S.d;
  S.sig = hA[0].sR != nullptr;
  S.ntmax = 0;
  for (int i = 0; i < count; i++) S.ntmax = hA[i].p.nt > S.ntmax ? hA[i].p.nt : S.ntmax;
  return S;
}

// Whole backward sweep for a given self-energy: slices ntmax .. k+1, then the
// start-up (problems share d, k and ntau).
hipError_t launch_adjoint_sweep(const AdjProb* dA, const AdjProb* hA, int count, hipStream_t s) {
  AdjShape S = adj_shape(hA, count);
  // inverse of the start-up matrix (used by the columns n <= 2k and the mixing start-up)
  hipLaunchKernelGGL(k_adj_tinv, dim3(1, count), dim3(ADJ_NT), 0, s, dA);
  for (int n = S.ntmax; n > S.k; n--) {
    adj_prep_launch(dA, S, n, s);
    adj_step_launch(dA, S, n, true, s);
  }
  adj_start_launch(dA, S, s);
  return hipGetLastError();
}

// Second-Born chain: per slice (and for the start-up block 0..k) `niter`
// trial steps of the adjoint fixed point on windows, then the final step.
hipError_t launch_adjoint_2b(AdjProb* dA, AdjProb* dDry, const AdjProb* hA, int count, int niter,
                             hipStream_t s) {
  AdjShape S = adj_shape(hA, count);
  int k = S.k, ntau = S.ntau, dd = S.dd;
  dim3 blk(ADJ_NT);
  hipLaunchKernelGGL(k_adj_tinv, dim3(1, count), blk, 0, s, dA);
  auto block = [&](int lo, int hi, int wlo, bool start) {
    if (!start) adj_prep_launch(dA, S, hi, s);
    unsigned wb = adj_blocks(win_elems(lo, hi, ntau, dd) + (size_t)(hi - lo + 1) * dd);
    unsigned sb = adj_blocks(win_elems(lo, hi, ntau, dd));
    hipLaunchKernelGGL(k_adj_setdry, dim3(1, count), dim3(64), 0, s, dDry, dA, lo, wlo);
    hipLaunchKernelGGL(k_adj_wcopy, dim3(wb, count), blk, 0, s, dA, 0, lo, hi, 0);
    hipLaunchKernelGGL(k_adj_sig2b, dim3(sb, count), blk, 0, s, dA, lo, hi, 0, 0);
    for (int it = 0; it < niter; it++) {
      hipLaunchKernelGGL(k_adj_wcopy, dim3(wb, count), blk, 0, s, dA, 1, lo, hi, it % 2);
      if (start)
        adj_start_launch(dDry, S, s);
      else
        adj_step_launch(dDry, S, hi, false, s);
      hipLaunchKernelGGL(k_adj_sig2b, dim3(sb, count), blk, 0, s, dA, lo, hi, 1, (it + 1) % 2);
    }
    hipLaunchKernelGGL(k_adj_conv, dim3(1, count), blk, 0, s, dA, lo, hi, hi);
    hipLaunchKernelGGL(k_adj_wcopy, dim3(wb, count), blk, 0, s, dA, 2, lo, hi, niter % 2);
    if (start)
      adj_start_launch(dA, S, s);
    else
      adj_step_launch(dA, S, hi, true, s);
    for (int t = lo; t <= hi; t++) hipLaunchKernelGGL(k_adj_ugrad, dim3(1, count), blk, 0, s, dA, t);
  };
  for (int n = S.ntmax; n > k; n--) block(n, n, n > 2 * k ? n - k : 0, false);
  block(0, k, 0, true);
  return hipGetLastError();
}

// Matsubara part of the second-Born adjoint for one problem: A is rebuilt at
// the converged Sigma^M and inverted (Ainv, work, piv, status as for the
// forward solve); `nit` damped iterations of the adjoint fixed point, the
// last change written to B.red[0..1]; then dJ/dU_{-1} and dJ/deps0_{-1}.
hipError_t launch_adjoint_mats(const Prob& P, const MadjBuf& B, cplx* K, cplx* work, int* piv, int* status,
                               const cplx* Mbar, double u, double nbar, double* ub, cplx* ge0, int nit,
                               double mix, hipStream_t s) {
  int d = P.d, N = (P.ntau + 1) * d;
  size_t nb = (size_t)(P.ntau + 1) * d * d;
  hipError_t e;
  if ((e = launch_free_mat(P, B.g, s))) return e;
  if ((e = launch_mat_conv(P, B.g, P.Smat, nullptr, K, s))) return e;
  if ((e = launch_mat_build(P, K, B.Ainv, s))) return e;
  if ((e = launch_gj_inverse(N, B.Ainv, work, piv, status, s))) return e;
  dim3 blk(ADJ_NT);
  hipLaunchKernelGGL(k_madj_eig, dim3(1), blk, 0, s, P, B);
  if ((e = hipMemcpyAsync(B.nu, Mbar, nb * sizeof(cplx), hipMemcpyDeviceToDevice, s))) return e;
  auto rev = [&]() {
    hipLaunchKernelGGL(k_madj_ga, dim3(adj_blocks((size_t)N * d)), blk, 0, s, N, d, (const cplx*)B.Ainv,
                       (const cplx*)B.nu, B.gA);
    hipLaunchKernelGGL(k_madj_kbar, dim3(adj_blocks(nb)), blk, 0, s, P, (const cplx*)B.gA, B.Kb);
    hipLaunchKernelGGL(k_madj_conv, dim3(adj_blocks(2 * nb)), blk, 0, s, P, B);
    hipLaunchKernelGGL(k_madj_eps, dim3(1), blk, 0, s, P, B);
  };
  for (int it = 0; it < nit; it++) {
    rev();
    hipLaunchKernelGGL(k_madj_nu, dim3(adj_blocks(nb)), blk, 0, s, P, B, Mbar, u);
    if (it == nit - 1) hipLaunchKernelGGL(k_madj_change, dim3(1), blk, 0, s, P, B);
    hipLaunchKernelGGL(k_madj_mix, dim3(adj_blocks(nb)), blk, 0, s, P, B, mix);
  }
  rev();
  hipLaunchKernelGGL(k_madj_final, dim3(1), blk, 0, s, P, B, u, nbar, ub, ge0);
  return hipGetLastError();
}

}  // namespace cntr
