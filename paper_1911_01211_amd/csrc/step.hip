// Dyson time step n > k and start-up (slices 0..k) on gfx950.
//
// A time step (Sec. "Time stepping", data-parallel form) is split into
//   k_history : Gregory-weighted history sums, tiled over (output, term
//               chunk) with partial sums per chunk (deterministic order);
//               one extra workgroup per problem forms the step matrix
//               M_R = h^-1 a_0 + i e_n + i h omega_0 Sigma^R_{n,n}, inverts it,
//               and solves the k-point conjugate start-up for R_{n,n-k..n}.
//   k_reduce  : sums the partials in chunk order, adds the BDF terms and
//               applies M_R^-1 (retarded row, left-mixing row) or
//               (M_R^dag)^-1 from the right (lesser rows m < n-k).
//   k_tailpre : the long sums of the k+1 lesser boundary rows m = n-k..n
//               (sources and the history over the rows found above).
//   k_tailsolve : the k+1 serial boundary steps.
// For k < n <= 2k the lesser column is solved serially by k_column.
//
// Layout: canonical slice-major storage; a tile of consecutive outputs m
// reads consecutive blocks of one stored row, so history reads coalesce.
#include "launch.h"

namespace cntr {

constexpr int NTHR = 256;

int hist_tm(int d) { return NTHR / (d * d) > 0 ? NTHR / (d * d) : 1; }
int hist_tj(int d) { return d >= 8 ? 32 : 64; }

static int cdiv_i(int a, int b) { return (a + b - 1) / b; }

HistPlan make_plan(int n, int k, int ntau, int d) {
  HistPlan p{};
  p.n = n;
  p.TJ = hist_tj(d);
  p.TM = hist_tm(d);
  int nb = n - k;  // bulk outputs m = 0..n-k-1
  bool les_bulk = n >= 2 * k + 1;
  p.njob = NJOB;
  int mout[NJOB] = {nb, ntau + 1, ntau + 1, les_bulk ? nb : 0, les_bulk ? nb : 0, les_bulk ? nb : 0};
  int span[NJOB] = {n, n, ntau + 1, n, nb > k + 1 ? nb : k + 1, ntau + 1};
  long off = 0;
  p.wg_off[0] = 0;
  for (int j = 0; j < NJOB; j++) {
    p.mout[j] = mout[j];
    p.nch[j] = mout[j] > 0 ? cdiv_i(span[j], p.TJ) : 0;
    p.mtiles[j] = mout[j] > 0 ? cdiv_i(mout[j], p.TM) : 0;
    p.wg_off[j + 1] = p.wg_off[j] + p.nch[j] * p.mtiles[j];
    p.part_off[j] = off;
    off += (long)p.nch[j] * mout[j];
  }
  // tail: rows n-k..n; sums over j in [0,n], [0,ntau], [0,n-k-1]
  int tspan[3] = {n + 1, ntau + 1, nb};
  p.tail_mtiles = cdiv_i(k + 1, p.TM);
  p.tail_wg_off[0] = 0;
  for (int j = 0; j < 3; j++) {
    p.tail_nch[j] = les_bulk ? cdiv_i(tspan[j], p.TJ) : 0;
    p.tail_wg_off[j + 1] = p.tail_wg_off[j] + p.tail_nch[j] * p.tail_mtiles;
    p.tail_off[j] = off;
    off += (long)p.tail_nch[j] * (k + 1);
  }
  return p;
}

size_t step_scratch_bytes(int nt, int k, int ntau, int d) {
  size_t mx = 0;
  // partial storage grows with n; check the largest few n (monotone)
  for (int n = nt; n >= nt - 1 && n > k; n--) {
    HistPlan p = make_plan(n, k, ntau, d);
    size_t blocks = p.tail_off[2] + (size_t)p.tail_nch[2] * (k + 1);
    if (blocks > mx) mx = blocks;
  }
  return mx * d * d * sizeof(cplx);
}

// ----------------------------------------------------------------- helpers
template <int D>
__device__ inline cplx ehat(const Prob& P, int n, int x, int y) {
  cplx e = P.eps[(size_t)(n + 1) * D * D + x * D + y];
  if (x == y) e.x -= P.mu;
  return e;
}

// ---------------------------------------------------------------- PREP
// M_R^-1 for the step and the retarded boundary R_{n,n-l}, l = 0..k
// (conjugate start-up, Eq. MBCVSAMx_cc_start).
template <int D>
__device__ void prep_step(const Prob& P, const Scratch& sc, int pi, int n, cplx* lds) {
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  int k = P.k, tid = threadIdx.x;
  double h = P.h;
  cplx* mr = lds;                 // DD
  cplx* A = lds + DD;             // (kD)^2
  cplx* B = A + (k * D) * (k * D);  // kD x D
  __shared__ int piv[8];
  __shared__ double redv[1];
  __shared__ int redi[1];
  double w0 = greg(W, n, n);
  for (int e = tid; e < DD; e += blockDim.x) {
    int x = e / D, y = e % D;
    cplx v = mul_i(ehat<D>(P, n, x, y));
    cplx s = P.Sret[(tri(n) + n) * DD + e];
    v = v + (h * w0) * mul_i(s);
    if (x == y) v.x += W.a[0] / h;
    mr[e] = v;
  }
  __syncthreads();
  bool ok = lds_inverse(D, mr, piv, redv, redi);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int e = tid; e < DD; e += blockDim.x) sc.minv(pi)[e] = mr[e];
  // boundary system: sum_l C_{l,p}^T Y_l^T = i C_{0,p}^T  (Y_0 = -i)
  int N = k * D;
  auto Cval = [&](int l, int p, int x, int y) -> cplx {
    cplx v = (h * W.s[p][l]) * mul_i(ret_ext<D>(P.Sret, n - l, n - p, x, y));
    if (p == l) v = v + mul_i(ehat<D>(P, n - p, x, y));
    if (x == y) v.x += W.D[p][l] / h;
    return v;
  };
  for (int idx = tid; idx < N * N; idx += blockDim.x) {
    int r = idx / N, q = idx % N;
    int p = r / D + 1, a = r % D, l = q / D + 1, bb = q % D;
    A[idx] = Cval(l, p, bb, a);
  }
  for (int idx = tid; idx < N * D; idx += blockDim.x) {
    int r = idx / D, cc = idx % D;
    int p = r / D + 1, a = r % D;
    B[idx] = mul_i(Cval(0, p, cc, a));
  }
  __syncthreads();
  ok = lds_solve(N, D, A, B, redv, redi);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int idx = tid; idx < (k + 1) * DD; idx += blockDim.x) {
    int l = idx / DD, e = idx % DD, cc = e / D, bb = e % D;
    cplx v;
    if (l == 0) v = (cc == bb) ? mk(0, -1) : mk(0, 0);
    else v = B[((l - 1) * D + bb) * D + cc];
    P.Gret[(tri(n) + n - l) * DD + e] = v;
  }
}

// ------------------------------------------------------------- HISTORY
template <int D>
__global__ __launch_bounds__(NTHR) void k_history(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int TJ = D >= 8 ? 32 : 64;
  constexpr int LDSN = (2 * TJ * DD) > (DD + 40 * 40 + 40 * 8) ? (2 * TJ * DD) : (DD + 40 * 40 + 40 * 8);
  __shared__ cplx lds[LDSN];
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  int b = blockIdx.x;
  if (b >= pl.wg_off[NJOB]) {
    prep_step<D>(P, sc, pi, n, lds);
    return;
  }
  int job = 0;
  while (b >= pl.wg_off[job + 1]) job++;
  int local = b - pl.wg_off[job];
  int mt = local / pl.nch[job], ch = local % pl.nch[job];
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau;
  int tid = threadIdx.x;
  int mo = tid / DD, e = tid % DD, a = e / D, c = e % D;
  int m = mt * TM + mo;
  int mout = pl.mout[job];
  bool valid = mo < TM && m < mout;
  int j0 = ch * TJ;
  int mlo = mt * TM, mhi = min(mt * TM + TM, mout) - 1;
  if (job == 0 && j0 + TJ - 1 < mlo) return;
  if (job == 4 && j0 > max(mhi, k)) return;
  cplx* sh0 = lds;
  cplx* sh1 = lds + TJ * DD;
  // stage the operand shared by every output of the tile
  for (int idx = tid; idx < TJ * DD; idx += NTHR) {
    int jj = idx / DD, ee = idx % DD, j = j0 + jj;
    cplx v = mk(0, 0), v1 = mk(0, 0);
    switch (job) {
      case 0:
      case 1:
      case 3:
        if (j < n) v = P.Sret[(tri(n) + j) * DD + ee];
        break;
      case 2:
        if (j <= ntau) {
          v = P.Stv[((size_t)n * (ntau + 1) + j) * DD + ee];
          v1 = P.Gmat[(size_t)(ntau - j) * DD + ee];
        }
        break;
      case 4:
        if (j <= n) v = P.Sles[(tri(n) + j) * DD + ee];
        break;
      case 5:
        if (j <= ntau) v = P.Stv[((size_t)n * (ntau + 1) + ntau - j) * DD + ee];
        break;
    }
    sh0[idx] = v;
    if (job == 2) sh1[idx] = v1;
  }
  __syncthreads();
  if (!valid) return;
  cplx acc = mk(0, 0);
  double xi = P.sig;
  switch (job) {
    case 0: {  // retarded bulk: sum_j w(n-m, j-m) S^R_{n,j} R_{j,m}
      int jlo = max(m, j0), jhi = min(n - 1, j0 + TJ - 1);
      for (int j = jlo; j <= jhi; j++) {
        const cplx* sb = sh0 + (j - j0) * DD + a * D;
        const cplx* hb = P.Gret + (tri(j) + m) * DD + c;
        cplx s = mk(0, 0);
#pragma unroll
        for (int q = 0; q < D; q++) cfma(s, sb[q], hb[q * D]);
        acc = acc + greg(W, n - m, j - m) * s;
      }
    } break;
    case 1: {  // left-mixing history: sum_j w(n,j) S^R_{n,j} T_{j,m}
      int jhi = min(n - 1, j0 + TJ - 1);
      for (int j = j0; j <= jhi; j++) {
        const cplx* sb = sh0 + (j - j0) * DD + a * D;
        const cplx* hb = P.Gtv + ((size_t)j * (ntau + 1) + m) * DD + c;
        cplx s = mk(0, 0);
#pragma unroll
        for (int q = 0; q < D; q++) cfma(s, sb[q], hb[q * D]);
        acc = acc + greg(W, n, j) * s;
      }
    } break;
    case 2: {  // tau source, Gregory parts of Eqs. ctv2, ctv3
      int Jhi = min(ntau, j0 + TJ - 1);
      for (int J = j0; J <= Jhi; J++) {
        if (m > k && J <= m) {
          const cplx* sb = P.Stv + ((size_t)n * (ntau + 1) + m - J) * DD + a * D;
          const cplx* mb = sh1 + (J - j0) * DD + c;
          cplx s = mk(0, 0);
#pragma unroll
          for (int q = 0; q < D; q++) cfma(s, sb[q], mb[q * D]);
          acc = acc + (xi * greg(W, m, J)) * s;
        }
        if (m < ntau - k && J >= m) {
          const cplx* sb = sh0 + (J - j0) * DD + a * D;
          const cplx* mb = P.Gmat + (size_t)(J - m) * DD + c;
          cplx s = mk(0, 0);
#pragma unroll
          for (int q = 0; q < D; q++) cfma(s, sb[q], mb[q * D]);
          acc = acc + greg(W, ntau - m, J - m) * s;
        }
      }
    } break;
    case 3: {  // lesser history: sum_l w(n,l) L^_{m,l} (S^R_{n,l})^dag
      int lhi = min(n - 1, j0 + TJ - 1);
      for (int l = j0; l <= lhi; l++) {
        const cplx* sb = sh0 + (l - j0) * DD + c * D;
        cplx s = mk(0, 0);
        if (l >= m) {
          const cplx* hb = P.Gles + (tri(l) + m) * DD + a * D;
#pragma unroll
          for (int q = 0; q < D; q++) cfma_cb(s, hb[q], sb[q]);
        } else {
          const cplx* hb = P.Gles + (tri(m) + l) * DD + a;
#pragma unroll
          for (int q = 0; q < D; q++) cfma(s, -conj(hb[q * D]), conj(sb[q]));
        }
        acc = acc + greg(W, n, l) * s;
      }
    } break;
    case 4: {  // source C^<_1[G,1,Sigma](m,n): sum_j w(m,j) R~_{m,j} S^<_{j,n}
      int jmax = m > k ? m : k;
      int jhi = min(jmax, j0 + TJ - 1);
      for (int j = j0; j <= jhi; j++) {
        const cplx* sb = sh0 + (j - j0) * DD + c;
        cplx s = mk(0, 0);
        if (j <= m) {
          const cplx* hb = P.Gret + (tri(m) + j) * DD + a * D;
#pragma unroll
          for (int q = 0; q < D; q++) cfma(s, hb[q], sb[q * D]);
        } else {
          const cplx* hb = P.Gret + (tri(j) + m) * DD + a;
#pragma unroll
          for (int q = 0; q < D; q++) cfma(s, -conj(hb[q * D]), sb[q * D]);
        }
        double w = m > k ? greg(W, m, j) : W.s[m][j];
        acc = acc + w * s;
      }
    } break;
    case 5: {  // source C^<_3[G,1,Sigma](m,n) without -i: sum_j w T_{m,j} S^lceil_{j,n}
      int jhi = min(ntau, j0 + TJ - 1);
      for (int j = j0; j <= jhi; j++) {
        const cplx* sb = sh0 + (j - j0) * DD + c * D;
        const cplx* hb = P.Gtv + ((size_t)m * (ntau + 1) + j) * DD + a * D;
        cplx s = mk(0, 0);
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(s, hb[q], sb[q]);
        acc = acc + (-xi * greg(W, ntau, j)) * s;
      }
    } break;
  }
  sc.part(pi)[(pl.part_off[job] + (long)ch * mout + m) * DD + e] = acc;
}

// -------------------------------------------------------------- REDUCE
template <int D>
__global__ __launch_bounds__(NTHR) void k_reduce(ProbArg pa, Scratch sc, HistPlan pl, int nfam_tiles0,
                                                 int nfam_tiles1) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int TJ = D >= 8 ? 32 : 64;
  __shared__ cplx rhs[TM * DD];
  __shared__ cplx minv[DD];
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau;
  double h = P.h, ht = P.htau, xi = P.sig;
  int b = blockIdx.x, fam, mt;
  if (b < nfam_tiles0) {
    fam = 0;
    mt = b;
  } else if (b < nfam_tiles0 + nfam_tiles1) {
    fam = 1;
    mt = b - nfam_tiles0;
  } else {
    fam = 2;
    mt = b - nfam_tiles0 - nfam_tiles1;
  }
  int tid = threadIdx.x;
  int mo = tid / DD, e = tid % DD, a = e / D, c = e % D;
  int m = mt * TM + mo;
  int mout = fam == 1 ? ntau + 1 : n - k;
  bool valid = mo < TM && m < mout;
  if (tid < DD) minv[tid] = sc.minv(pi)[tid];
  const cplx* part = sc.part(pi);
  cplx r = mk(0, 0);
  if (valid) {
    if (fam == 0) {
      cplx hs = mk(0, 0);
      for (int ch = m / TJ; ch < pl.nch[0]; ch++) hs = hs + part[(pl.part_off[0] + (long)ch * mout + m) * DD + e];
      r = -(h * mul_i(hs));
      for (int l = 1; l <= k; l++) r = r - (W.a[l] / h) * P.Gret[(tri(n - l) + m) * DD + e];
    } else if (fam == 1) {
      cplx ts = mk(0, 0);
      for (int ch = 0; ch < pl.nch[2]; ch++) ts = ts + part[(pl.part_off[2] + (long)ch * mout + m) * DD + e];
      ts = ht * ts;
      if (m <= k) {  // Eq. ctv2, boundary-convolution weights
        for (int j = 0; j <= k; j++)
          for (int l = 0; l <= k; l++) {
            const cplx* sb = P.Stv + ((size_t)n * (ntau + 1) + l) * DD + a * D;
            const cplx* mb = P.Gmat + (size_t)(ntau - j) * DD + c;
            cplx s = mk(0, 0);
            for (int q = 0; q < D; q++) cfma(s, sb[q], mb[q * D]);
            ts = ts + (ht * xi * W.R[m][j][l]) * s;
          }
      }
      if (m >= ntau - k) {  // Eq. ctv3, boundary-convolution weights
        for (int j = 0; j <= k; j++)
          for (int l = 0; l <= k; l++) {
            const cplx* sb = P.Stv + ((size_t)n * (ntau + 1) + ntau - l) * DD + a * D;
            const cplx* mb = P.Gmat + (size_t)j * DD + c;
            cplx s = mk(0, 0);
            for (int q = 0; q < D; q++) cfma(s, sb[q], mb[q * D]);
            ts = ts + (ht * W.R[ntau - m][j][l]) * s;
          }
      }
      cplx hs = mk(0, 0);
      for (int ch = 0; ch < pl.nch[1]; ch++) hs = hs + part[(pl.part_off[1] + (long)ch * mout + m) * DD + e];
      r = -mul_i(ts) - h * mul_i(hs);
      for (int l = 1; l <= k; l++)
        r = r - (W.a[l] / h) * P.Gtv[((size_t)(n - l) * (ntau + 1) + m) * DD + e];
    } else {
      cplx s3 = mk(0, 0), s4 = mk(0, 0), s5 = mk(0, 0);
      for (int ch = 0; ch < pl.nch[3]; ch++) s3 = s3 + part[(pl.part_off[3] + (long)ch * mout + m) * DD + e];
      int jmax = m > k ? m : k;
      for (int ch = 0; ch <= jmax / TJ; ch++) s4 = s4 + part[(pl.part_off[4] + (long)ch * mout + m) * DD + e];
      for (int ch = 0; ch < pl.nch[5]; ch++) s5 = s5 + part[(pl.part_off[5] + (long)ch * mout + m) * DD + e];
      r = h * mul_i(s4) + ht * s5 + h * mul_i(s3);
      for (int l = 1; l <= k; l++) r = r - (W.a[l] / h) * P.Gles[(tri(n - l) + m) * DD + e];
    }
    rhs[mo * DD + e] = r;
  }
  __syncthreads();
  if (!valid) return;
  cplx out = mk(0, 0);
  if (fam < 2) {
    for (int q = 0; q < D; q++) cfma(out, minv[a * D + q], rhs[mo * DD + q * D + c]);
    if (fam == 0) P.Gret[(tri(n) + m) * DD + e] = out;
    else P.Gtv[((size_t)n * (ntau + 1) + m) * DD + e] = out;
  } else {
    // X M_L = rhs with M_L = M_R^dag:  X = rhs (M_R^-1)^dag
    for (int q = 0; q < D; q++) cfma_cb(out, rhs[mo * DD + a * D + q], minv[c * D + q]);
    P.Gles[(tri(n) + m) * DD + e] = out;
  }
}

// ------------------------------------------------------------ TAIL PRE
// Long sums of the boundary rows m = n-k..n of the lesser column n:
//   P1 = sum_{j=0}^{n} w(n,j) Sigma^<_{m,j} (R_{n,j})^dag
//   P2 = sum_{j=0}^{ntau} w(ntau,j) Sigma^rceil_{m,j} G^lceil_{j,n}
//   P3 = sum_{j=0}^{n-k-1} w(m,j) Sigma^R_{m,j} L_{j,n}
template <int D>
__global__ __launch_bounds__(NTHR) void k_tailpre(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int TJ = D >= 8 ? 32 : 64;
  __shared__ cplx sh0[TJ * DD];
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau;
  double xi = P.sig;
  int b = blockIdx.x, sub = 0;
  while (b >= pl.tail_wg_off[sub + 1]) sub++;
  int local = b - pl.tail_wg_off[sub];
  int mt = local / pl.tail_nch[sub], ch = local % pl.tail_nch[sub];
  int tid = threadIdx.x;
  int mo = tid / DD, e = tid % DD, a = e / D, c = e % D;
  int r = mt * TM + mo;  // row index 0..k
  int m = n - k + r;
  bool valid = mo < TM && r <= k;
  int j0 = ch * TJ;
  int span = sub == 0 ? n + 1 : (sub == 1 ? ntau + 1 : n - k);
  for (int idx = tid; idx < TJ * DD; idx += NTHR) {
    int jj = idx / DD, ee = idx % DD, j = j0 + jj;
    cplx v = mk(0, 0);
    if (j < span) {
      if (sub == 0) v = P.Gret[(tri(n) + j) * DD + ee];
      else if (sub == 1) v = P.Gtv[((size_t)n * (ntau + 1) + ntau - j) * DD + ee];
      else v = P.Gles[(tri(n) + j) * DD + ee];
    }
    sh0[idx] = v;
  }
  __syncthreads();
  if (!valid) return;
  cplx acc = mk(0, 0);
  int jhi = min(span - 1, j0 + TJ - 1);
  for (int j = j0; j <= jhi; j++) {
    cplx s = mk(0, 0);
    if (sub == 0) {
      const cplx* rb = sh0 + (j - j0) * DD + c * D;
#pragma unroll
      for (int q = 0; q < D; q++) cfma_cb(s, les_any<D>(P.Sles, m, j, a, q), rb[q]);
      acc = acc + greg(W, n, j) * s;
    } else if (sub == 1) {
      const cplx* tb = sh0 + (j - j0) * DD + c * D;
      const cplx* sb = P.Stv + ((size_t)m * (ntau + 1) + j) * DD + a * D;
#pragma unroll
      for (int q = 0; q < D; q++) cfma_cb(s, sb[q], tb[q]);
      acc = acc + (-xi * greg(W, ntau, j)) * s;
    } else {
      const cplx* lb = sh0 + (j - j0) * DD + c;
      const cplx* sb = P.Sret + (tri(m) + j) * DD + a * D;
#pragma unroll
      for (int q = 0; q < D; q++) cfma(s, sb[q], lb[q * D]);
      acc = acc + greg(W, m, j) * s;
    }
  }
  sc.part(pi)[(pl.tail_off[sub] + (long)ch * (k + 1) + r) * DD + e] = acc;
}

// ---------------------------------------------------------- TAIL SOLVE
// Serial boundary steps m = n-k..n of the lesser column (Eq. MBCVSAMx_t for
// y(t) = G^<(t, t_n), p = i e, k = i Sigma^R, q = -i (C^<_2 + C^<_3)[Sigma,1,G]).
template <int D>
__global__ __launch_bounds__(NTHR) void k_tailsolve(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D;
  constexpr int TJ = D >= 8 ? 32 : 64;
  __shared__ cplx ml[DD], rhs[DD];
  __shared__ int piv[8];
  __shared__ double redv[1];
  __shared__ int redi[1];
  int pi = blockIdx.x;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int k = P.k;
  double h = P.h, ht = P.htau;
  int tid = threadIdx.x;
  const cplx* part = sc.part(pi);
  for (int r = 0; r <= k; r++) {
    int m = n - k + r;
    if (tid < DD) {
      int e = tid, a = e / D, c = e % D;
      cplx p1 = mk(0, 0), p2 = mk(0, 0), p3 = mk(0, 0);
      for (int ch = 0; ch < pl.tail_nch[0]; ch++) p1 = p1 + part[(pl.tail_off[0] + (long)ch * (k + 1) + r) * DD + e];
      for (int ch = 0; ch < pl.tail_nch[1]; ch++) p2 = p2 + part[(pl.tail_off[1] + (long)ch * (k + 1) + r) * DD + e];
      for (int ch = 0; ch < pl.tail_nch[2]; ch++) p3 = p3 + part[(pl.tail_off[2] + (long)ch * (k + 1) + r) * DD + e];
      for (int j = n - k; j < m; j++) {
        cplx s = mk(0, 0);
        for (int q = 0; q < D; q++) cfma(s, P.Sret[(tri(m) + j) * DD + a * D + q], P.Gles[(tri(n) + j) * DD + q * D + c]);
        p3 = p3 + greg(W, m, j) * s;
      }
      cplx v = -(h * mul_i(p1)) - ht * p2 - h * mul_i(p3);
      for (int l = 1; l <= k; l++) v = v - (W.a[l] / h) * P.Gles[(tri(n) + m - l) * DD + e];
      rhs[e] = v;
      cplx mv = mul_i(ehat<D>(P, m, a, c)) + (h * greg(W, m, m)) * mul_i(P.Sret[(tri(m) + m) * DD + e]);
      if (a == c) mv.x += W.a[0] / h;
      ml[e] = mv;
    }
    __syncthreads();
    bool ok = lds_inverse(D, ml, piv, redv, redi);
    if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    if (tid < DD) {
      int a = tid / D, c = tid % D;
      cplx o = mk(0, 0);
      for (int q = 0; q < D; q++) cfma(o, ml[a * D + q], rhs[q * D + c]);
      P.Gles[(tri(n) + m) * DD + tid] = o;
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------- COLUMN
// Whole lesser column n by the standard Volterra start-up over rows 1..k
// (Eq. vdiff_start, y_0 = -[G^rceil(t_n,0)]^dag) followed, for n > k, by the
// serial steps of rows k+1..n. Used for the start-up slices n <= k and for
// k < n <= 2k. One workgroup per problem.
template <int D>
__global__ __launch_bounds__(NTHR) void k_column(ProbArg pa, Scratch sc, int n0) {
  constexpr int DD = D * D;
  __shared__ cplx A[(KMAX * D) * (KMAX * D)];
  __shared__ cplx B[KMAX * D * D];
  __shared__ cplx q[(2 * KMAX + 1) * DD];
  __shared__ cplx y0[DD];
  __shared__ cplx ml[DD], rhs[DD];
  __shared__ int piv[8];
  __shared__ double redv[1];
  __shared__ int redi[1];
  int pi = blockIdx.y;
  int n = n0 + blockIdx.x;  // start-up: one workgroup per column 0..k
  const Prob& P = pa.get(pi);
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau;
  double h = P.h, ht = P.htau, xi = P.sig;
  int tid = threadIdx.x;
  int rows = n > k ? n : k;
  // y_0
  for (int e = tid; e < DD; e += NTHR) {
    int a = e / D, c = e % D;
    cplx v = -conj(P.Gtv[((size_t)n * (ntau + 1) + 0) * DD + c * D + a]);
    y0[e] = v;
    P.Gles[(tri(n) + 0) * DD + e] = v;
  }
  // sources q_p = -i h C2 - h_tau C3 for p = 1..rows
  int jmx = n > k ? n : k;
  for (int idx = tid; idx < rows * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    cplx c2 = mk(0, 0), c3 = mk(0, 0);
    for (int j = 0; j <= jmx; j++) {
      cplx s = mk(0, 0);
      for (int qq = 0; qq < D; qq++) {
        cplx ga = j <= n ? conj(P.Gret[(tri(n) + j) * DD + c * D + qq]) : -P.Gret[(tri(j) + n) * DD + qq * D + c];
        cfma(s, les_any<D>(P.Sles, p, j, a, qq), ga);
      }
      c2 = c2 + greg(W, n, j) * s;
    }
    for (int j = 0; j <= ntau; j++) {
      cplx s = mk(0, 0);
      for (int qq = 0; qq < D; qq++)
        cfma_cb(s, P.Stv[((size_t)p * (ntau + 1) + j) * DD + a * D + qq],
                P.Gtv[((size_t)n * (ntau + 1) + ntau - j) * DD + c * D + qq]);
      c3 = c3 + (-xi * greg(W, ntau, j)) * s;
    }
    q[(p - 1) * DD + e] = -(h * mul_i(c2)) - ht * c3;
  }
  __syncthreads();
  // start-up system B_{p,l} y_l = q_p - B_{p,0} y_0, p,l = 1..k
  int N = k * D;
  auto Bval = [&](int p, int l, int x, int y) -> cplx {
    cplx v = (h * W.s[p][l]) * mul_i(ret_ext<D>(P.Sret, p, l, x, y));
    if (p == l) v = v + mul_i(ehat<D>(P, p, x, y));
    if (x == y) v.x += W.D[p][l] / h;
    return v;
  };
  for (int idx = tid; idx < N * N; idx += NTHR) {
    int rr = idx / N, cc = idx % N;
    A[idx] = Bval(rr / D + 1, cc / D + 1, rr % D, cc % D);
  }
  for (int idx = tid; idx < N * D; idx += NTHR) {
    int rr = idx / D, cc = idx % D, p = rr / D + 1, a = rr % D;
    cplx v = q[(p - 1) * DD + a * D + cc];
    for (int qq = 0; qq < D; qq++) v = v - Bval(p, 0, a, qq) * y0[qq * D + cc];
    B[idx] = v;
  }
  __syncthreads();
  bool ok = lds_solve(N, D, A, B, redv, redi);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    if (p <= n) P.Gles[(tri(n) + p) * DD + e] = B[((p - 1) * D + a) * D + c];
  }
  __syncthreads();
  for (int m = k + 1; m <= n; m++) {
    if (tid < DD) {
      int e = tid, a = e / D, c = e % D;
      cplx v = q[(m - 1) * DD + e];
      for (int l = 1; l <= k; l++) v = v - (W.a[l] / h) * P.Gles[(tri(n) + m - l) * DD + e];
      cplx hs = mk(0, 0);
      for (int j = 0; j < m; j++) {
        cplx s = mk(0, 0);
        for (int qq = 0; qq < D; qq++) cfma(s, P.Sret[(tri(m) + j) * DD + a * D + qq], P.Gles[(tri(n) + j) * DD + qq * D + c]);
        hs = hs + greg(W, m, j) * s;
      }
      rhs[e] = v - h * mul_i(hs);
      cplx mv = mul_i(ehat<D>(P, m, a, c)) + (h * greg(W, m, m)) * mul_i(P.Sret[(tri(m) + m) * DD + e]);
      if (a == c) mv.x += W.a[0] / h;
      ml[e] = mv;
    }
    __syncthreads();
    ok = lds_inverse(D, ml, piv, redv, redi);
    if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    if (tid < DD) {
      int a = tid / D, c = tid % D;
      cplx o = mk(0, 0);
      for (int qq = 0; qq < D; qq++) cfma(o, ml[a * D + qq], rhs[qq * D + c]);
      P.Gles[(tri(n) + m) * DD + tid] = o;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ START R
// Retarded start-up columns m = 0..k-1 (Sec. "Start", first item):
//   i h^-1 sum_l D_{p,l} y_l - e_p y_p - h sum_l I_{m,p,l} Sigma~^R_{p,l} y_l = 0.
template <int D>
__global__ __launch_bounds__(NTHR) void k_start_ret(ProbArg pa, Scratch sc) {
  constexpr int DD = D * D;
  __shared__ cplx A[(KMAX * D) * (KMAX * D)];
  __shared__ cplx B[KMAX * D * D];
  __shared__ cplx y[(KMAX + 1) * DD];
  __shared__ double redv[1];
  __shared__ int redi[1];
  int pi = blockIdx.x;
  const Prob& P = pa.get(pi);
  const KW& W = c_kw[P.k];
  int k = P.k, tid = threadIdx.x;
  double h = P.h;
  for (int m = 0; m <= k; m++) {
    for (int e = tid; e < DD; e += NTHR) P.Gret[(tri(m) + m) * DD + e] = (e / D == e % D) ? mk(0, -1) : mk(0, 0);
    if (m == k) break;
    // known y_l, l <= m
    for (int idx = tid; idx < (m + 1) * DD; idx += NTHR) {
      int l = idx / DD, e = idx % DD, a = e / D, c = e % D;
      cplx v;
      if (l == m) v = (a == c) ? mk(0, -1) : mk(0, 0);
      else v = -conj(P.Gret[(tri(m) + l) * DD + c * D + a]);
      y[l * DD + e] = v;
    }
    __syncthreads();
    auto Aval = [&](int p, int l, int x, int yy) -> cplx {
      cplx v = -(h * W.I[m][p][l]) * ret_ext<D>(P.Sret, p, l, x, yy);
      if (p == l) v = v - ehat<D>(P, p, x, yy);
      if (x == yy) v.y += W.D[p][l] / h;
      return v;
    };
    int nu = k - m, N = nu * D;
    for (int idx = tid; idx < N * N; idx += NTHR) {
      int rr = idx / N, cc = idx % N;
      A[idx] = Aval(m + 1 + rr / D, m + 1 + cc / D, rr % D, cc % D);
    }
    for (int idx = tid; idx < N * D; idx += NTHR) {
      int rr = idx / D, c = idx % D, p = m + 1 + rr / D, a = rr % D;
      cplx v = mk(0, 0);
      for (int l = 0; l <= m; l++)
        for (int qq = 0; qq < D; qq++) v = v - Aval(p, l, a, qq) * y[l * DD + qq * D + c];
      B[idx] = v;
    }
    __syncthreads();
    bool ok = lds_solve(N, D, A, B, redv, redi);
    if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    for (int idx = tid; idx < nu * DD; idx += NTHR) {
      int p = m + 1 + idx / DD, e = idx % DD, a = e / D, c = e % D;
      P.Gret[(tri(p) + m) * DD + e] = B[((p - m - 1) * D + a) * D + c];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ START TV
// Left-mixing start-up per tau index m (Sec. "Start", second item).
template <int D>
__global__ __launch_bounds__(NTHR) void k_start_tv(ProbArg pa, Scratch sc) {
  constexpr int DD = D * D;
  __shared__ cplx A[(KMAX * D) * (KMAX * D)];
  __shared__ cplx B[KMAX * D * D];
  __shared__ cplx q[KMAX * DD];
  __shared__ cplx y0[DD];
  __shared__ double redv[1];
  __shared__ int redi[1];
  int pi = blockIdx.y, m = blockIdx.x;
  const Prob& P = pa.get(pi);
  if (m > P.ntau) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  double h = P.h, ht = P.htau, xi = P.sig;
  for (int e = tid; e < DD; e += NTHR) {
    cplx v = xi * mul_i(P.Gmat[(size_t)(ntau - m) * DD + e]);
    y0[e] = v;
    P.Gtv[(size_t)m * DD + e] = v;
  }
  // q_p = -i (C^rceil_2 + C^rceil_3)[Sigma, 1, G](p, m)
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    const cplx* S = P.Stv + (size_t)p * (ntau + 1) * DD;
    cplx acc = mk(0, 0);
    auto prod = [&](int ls, int lm) {
      cplx s = mk(0, 0);
      for (int qq = 0; qq < D; qq++) cfma(s, S[(size_t)ls * DD + a * D + qq], P.Gmat[(size_t)lm * DD + qq * D + c]);
      return s;
    };
    if (m <= k) {
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) acc = acc + (ht * xi * W.R[m][j][l]) * prod(l, ntau - j);
    } else {
      for (int l = 0; l <= m; l++) acc = acc + (ht * xi * greg(W, m, l)) * prod(m - l, ntau - l);
    }
    if (m >= ntau - k) {
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) acc = acc + (ht * W.R[ntau - m][j][l]) * prod(ntau - l, j);
    } else {
      for (int l = 0; l <= ntau - m; l++) acc = acc + (ht * greg(W, ntau - m, l)) * prod(m + l, l);
    }
    q[(p - 1) * DD + e] = -mul_i(acc);
  }
  __syncthreads();
  int N = k * D;
  auto Bval = [&](int p, int l, int x, int yy) -> cplx {
    cplx v = (h * W.s[p][l]) * mul_i(ret_ext<D>(P.Sret, p, l, x, yy));
    if (p == l) v = v + mul_i(ehat<D>(P, p, x, yy));
    if (x == yy) v.x += W.D[p][l] / h;
    return v;
  };
  for (int idx = tid; idx < N * N; idx += NTHR) {
    int rr = idx / N, cc = idx % N;
    A[idx] = Bval(rr / D + 1, cc / D + 1, rr % D, cc % D);
  }
  for (int idx = tid; idx < N * D; idx += NTHR) {
    int rr = idx / D, cc = idx % D, p = rr / D + 1, a = rr % D;
    cplx v = q[(p - 1) * DD + a * D + cc];
    for (int qq = 0; qq < D; qq++) v = v - Bval(p, 0, a, qq) * y0[qq * D + cc];
    B[idx] = v;
  }
  __syncthreads();
  bool ok = lds_solve(N, D, A, B, redv, redi);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    P.Gtv[((size_t)p * (ntau + 1) + m) * DD + e] = B[((p - 1) * D + a) * D + c];
  }
}

// ------------------------------------------------------------ launches
template <int D>
static hipError_t step_d(const ProbArg& pa, const Scratch& sc, int n, hipStream_t s) {
  const Prob& P0 = pa.count == 1 ? pa.one : pa.one;  // grids are uniform within a call
  int k = P0.k, ntau = P0.ntau;
  HistPlan pl = make_plan(n, k, ntau, D);
  dim3 g1(pl.wg_off[NJOB] + 1, pa.count);
  k_history<D><<<g1, NTHR, 0, s>>>(pa, sc, pl);
  int t0 = pl.mtiles[0], t1 = cdiv_i(ntau + 1, pl.TM), t2 = pl.mtiles[3];
  dim3 g2(t0 + t1 + t2, pa.count);
  k_reduce<D><<<g2, NTHR, 0, s>>>(pa, sc, pl, t0, t1);
  if (n >= 2 * k + 1) {
    dim3 g3(pl.tail_wg_off[3], pa.count);
    k_tailpre<D><<<g3, NTHR, 0, s>>>(pa, sc, pl);
    k_tailsolve<D><<<pa.count, NTHR, 0, s>>>(pa, sc, pl);
  } else {
    dim3 g4(1, pa.count);
    k_column<D><<<g4, NTHR, 0, s>>>(pa, sc, n);
  }
  return hipGetLastError();
}

hipError_t launch_step(const ProbArg& pa, const Scratch& sc, int n, int d, hipStream_t s) {
  switch (d) {
    case 1: return step_d<1>(pa, sc, n, s);
    case 2: return step_d<2>(pa, sc, n, s);
    case 3: return step_d<3>(pa, sc, n, s);
    case 4: return step_d<4>(pa, sc, n, s);
    case 5: return step_d<5>(pa, sc, n, s);
    case 6: return step_d<6>(pa, sc, n, s);
    case 7: return step_d<7>(pa, sc, n, s);
    case 8: return step_d<8>(pa, sc, n, s);
  }
  return hipErrorInvalidValue;
}

template <int D>
static hipError_t start_d(const ProbArg& pa, const Scratch& sc, int ntau, hipStream_t s) {
  int k = pa.one.k;
  k_start_ret<D><<<pa.count, NTHR, 0, s>>>(pa, sc);
  dim3 g(ntau + 1, pa.count);
  k_start_tv<D><<<g, NTHR, 0, s>>>(pa, sc);
  dim3 g2(k + 1, pa.count);
  k_column<D><<<g2, NTHR, 0, s>>>(pa, sc, 0);
  return hipGetLastError();
}

hipError_t launch_start(const ProbArg& pa, const Scratch& sc, int d, int ntau, hipStream_t s) {
  switch (d) {
    case 1: return start_d<1>(pa, sc, ntau, s);
    case 2: return start_d<2>(pa, sc, ntau, s);
    case 3: return start_d<3>(pa, sc, ntau, s);
    case 4: return start_d<4>(pa, sc, ntau, s);
    case 5: return start_d<5>(pa, sc, ntau, s);
    case 6: return start_d<6>(pa, sc, ntau, s);
    case 7: return start_d<7>(pa, sc, ntau, s);
    case 8: return start_d<8>(pa, sc, ntau, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cntr
