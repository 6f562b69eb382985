// Dyson equation in integral form on gfx950 (Sec. "vie2: Dyson equation in
// integral form", Sec. "Implementation: vie2"):
//   (1 + F) * G = Q  (Eq. vie2),   G * (1 + F^ddagger) = Q  (Eq. vie2_cc),
// G and Q hermitian, F and Fcc = F^ddagger given.
//
// Time step n > k. The history sums are those of the Dyson step with F in
// place of Sigma: the retarded and mixing jobs of k_history read F^R, F^rceil
// and F^M, the lesser jobs read Fcc^< and, through the conjugate relations
// Fcc^A_{l,n} = (F^R_{n,l})^dag and Fcc^lceil(tau_j, t_n) = -xi
// (F^rceil_{n,ntau-j})^dag, F^R and F^rceil. So k_history runs unchanged (its
// set-up is k_v2_side's), and k_v2_reduce applies the
// second-kind local step (Eq. MBCVSAMx01_t and its conjugate):
//   G^R_{n,m}       = [1 + h w F^R_{n,n}]^-1 (Q^R_{n,m} - h C^R_{n,m}),
//   G^rceil_{n,m}   = [1 + h omega_0 F^R_{n,n}]^-1 (Q^rceil_{n,m} - C^rceil_{n,m}),
//   G^<_{m,n} [1 + h omega_0 Fcc^A_{n,n}] = Q^<_{m,n} - C^<_{m,n}   (variant B),
// with w = omega_0 for n - m > k and w = s_{n-m,0} for the rows n-m <= k,
// whose interval is shorter than k+1 points (Eq. cr1, second case; summed
// directly, as are the lesser rows m >= n-k, for which the history kernel
// has no outputs: k_v2_side sums those in chunks,
// the last reduce workgroup solves them). 1 + h omega_0 Fcc^A_{n,n} is the
// adjoint of the retarded step matrix. G^<_{n,n} needs the finished row and
// column of slice n: every reduce workgroup adds its outputs' terms into a
// partial, the last one to finish (completion count) sums them and solves.
//
// Start-up (slices 0..k): the retarded columns m = 0..k-1 from the
// (k-m) d system of Sec. "Start" (one workgroup per problem, in order of m),
// the mixing rows per tau index and the lesser columns per n from the
// start-up rule of Eq. MBCVSAMx01_start with kernel F^R (one workgroup each).
#include "launch.h"

namespace cntr {

// F~^R_{p,l}, element (x, y): stored for p >= l, else -[Fcc^R_{l,p}]^dag
template <int D>
__device__ inline cplx v2_fret(const Prob& P, int p, int l, int x, int y) {
  constexpr int DD = D * D;
  if (p >= l) return gld(P.Sret + (tri(p) + l) * DD + x * D + y);
  return -conj(gld(P.Fcret + (tri(l) + p) * DD + y * D + x));
}
// F^<_{m,j}, element (x, y): stored for m <= j, else -[Fcc^<_{j,m}]^dag
template <int D>
__device__ inline cplx v2_fles(const Prob& P, int m, int j, int x, int y) {
  constexpr int DD = D * D;
  if (m <= j) return gld(P.Fles + (tri(j) + m) * DD + x * D + y);
  return -conj(gld(P.Sles + (tri(m) + j) * DD + y * D + x));
}

// ------------------------------------------------------------- step set-up
// Inverses of the local step matrices 1 + h w F^R_{n,n} into slots r = 0..k
// of the problem's matrix scratch: w = omega_0 (slot 0: rows with n - m > k,
// the mixing row, and the lesser column through the adjoint) and
// w = s_{r,0} (slot r: the retarded row m = n - r). The first workgroup of
// k_v2_side.
template <int D>
__device__ void v2_prep(const Prob& P, const Scratch& sc, int pi, int n, cplx* lds) {
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  int k = P.k, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double h = P.h;
  int* piv = (int*)(lds + (KMAX + 1) * DD);
  // the reduce of this step starts its completion count at 0
  if (tid == 0) *sc.counter(pi) = 0;
  for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) {
    int r = idx / DD, e = idx % DD;
    double w = r == 0 ? greg(W, n, n) : W.s[r][0];
    cplx v = (h * w) * gld(P.Sret + (tri(n) + n) * DD + e);
    if (e / D == e % D) v.x += 1.0;
    lds[idx] = v;
  }
  __syncthreads();
  bool ok = true;
  for (int r = wave; r <= k; r += NTHR / 64) ok = wave_inverse(D, lds + r * DD, piv + r * D) && ok;
  if (!ok && lane == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  __syncthreads();
  for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) gst(sc.minv(pi) + idx, lds[idx]);
}

// ------------------------------------------------- lesser boundary rows
// Lesser rows m = v2_lo .. n-1 of column n, for which the history jobs have
// no outputs (m >= n-k; every m < n for n <= 2k), by the other workgroups
// of k_v2_side (they read only earlier slices). With the terms of row m
// numbered t < T1 (C1, j = t), T1 <= t < T1 + n (C2, l = t - T1) and the
// ntau+1 tau terms after them, workgroup (r, ch) sums the terms
// ch*v2_ch .. +v2_ch-1 of row v2_lo + r into one d x d partial of
//   C^<_{m,n} = h (C1 + C2) - i h_tau C3,
//   C1 = sum_j w G~^R_{m,j} Fcc^<_{j,n}                          (Eq. cles1)
//   C2 = sum_{l<n} w(n,l) G^<_{m,l} (F^R_{n,l})^dag  (Fcc^A; Eq. cles2, l = n local)
//   C3 = sum_j w(ntau,j) G^rceil_{m,j} (-xi) (F^rceil_{n,ntau-j})^dag  (Fcc^lceil; Eq. cles3)
// (NTHR / d^2 thread groups, four terms each, summed in a fixed order).
template <int D>
__device__ void v2_edge_part(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, int r, int ch,
                             cplx* lds) {
  constexpr int DD = D * D, NG = NTHR / DD > 0 ? NTHR / DD : 1;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  double h = P.h, ht = P.htau, xi = P.sig;
  int m = pl.v2_lo + r;
  int T1 = (m > k ? m : k) + 1, T2 = T1 + n, T3 = T2 + ntau + 1;
  int g = tid / DD, e = tid % DD, a = e / D, c = e % D;
  if (g < NG) {
    cplx acc = mk(0, 0);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      int t = ch * pl.v2_ch + i * NG + g;
      if (t < T1) {
        int j = t;
        double w = m > k ? greg(W, m, j) : W.s[m][j];
        cplx s = mk(0, 0);
#pragma unroll
        for (int q = 0; q < D; q++) cfma(s, ret_ext_d(P.Gret, m, j, a, q, D), gld(P.Sles + (tri(n) + j) * DD + q * D + c));
        acc = acc + (h * w) * s;
      } else if (t < T2) {
        int l = t - T1;
        cplx s = mk(0, 0);
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(s, les_any_d(P.Gles, m, l, a, q, D), gld(P.Sret + (tri(n) + l) * DD + c * D + q));
        acc = acc + (h * greg(W, n, l)) * s;
      } else if (t < T3) {
        int j = t - T2;
        const cplx* gt = P.Gtv + ((size_t)m * (ntau + 1) + j) * DD + a * D;
        const cplx* ft = P.Stv + ((size_t)n * (ntau + 1) + ntau - j) * DD + c * D;
        cplx s = mk(0, 0);
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(s, gld(gt + q), gld(ft + q));
        acc = acc - mul_i((ht * -xi * greg(W, ntau, j)) * s);
      }
    }
    lds[g * DD + e] = acc;
  }
  __syncthreads();
  if (tid < DD) {
    cplx sum = mk(0, 0);
    for (int gg = 0; gg < NG; gg++) sum = sum + lds[gg * DD + tid];
    gst(sc.part(pi) + (pl.v2_off + (long)r * pl.v2_nch + ch) * DD + tid, sum);
  }
}

// Step set-up (workgroup 0) and the boundary lesser rows' chunks (the
// others), launched before the history sums; nothing here reads slice n of G.
template <int D>
__global__ __launch_bounds__(NTHR) void k_v2_side(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D, NG = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int NP = (KMAX + 1) * DD + (KMAX + 1) * D;  // matrices and pivot ints
  __shared__ cplx lds[NP > NG * DD ? NP : NG * DD];
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  int b = blockIdx.x;
  if (b == 0) {
    v2_prep<D>(P, sc, pi, n, lds);
  } else {
    int u = b - 1;
    v2_edge_part<D>(P, sc, pi, n, pl, u / pl.v2_nch, u % pl.v2_nch, lds);
  }
}

// The boundary lesser rows from the chunk partials of k_v2_side, their C2
// terms of G^<_{n,n}, and G^<_{n,n} from the partials of every reduce
// workgroup (run by the last reduce workgroup of the problem; minv: slot 0).
template <int D>
__device__ void v2_final(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, const cplx* minv,
                         cplx* xe, cplx* xo, cplx* dg) {
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  int tid = threadIdx.x;
  double h = P.h;
  int nwg = pl.red_tiles[0] + pl.red_tiles[1] + pl.red_tiles[2] + 1;
  const cplx* dpart = sc.part(pi) + pl.v2_doff * DD;
  const cplx* epart = sc.part(pi) + pl.v2_off * DD;
  int nr = pl.v2_rows;
  // G thread groups per value sum every G-th partial of G^<_{n,n} (fixed
  // order), loaded in the same memory round as the rows' chunk partials
  constexpr int G = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int PB = D >= 2 ? 16 : 4;
  for (int vv = tid; vv < G * DD; vv += NTHR) {
    int g = vv / DD, e = vv % DD;
    dg[vv] = psum_b<PB>(dpart + (size_t)g * DD + e, (long)G * DD, g < nwg ? (nwg - g + G - 1) / G : 0);
  }
  // X_r M = Q^<_{m,n} - (sum of the chunk partials of row m)
  for (int idx = tid; idx < nr * DD; idx += NTHR) {
    int r = idx / DD, e = idx % DD, m = pl.v2_lo + r;
    cplx hs = psum_b<PB>(epart + (size_t)r * pl.v2_nch * DD + e, DD, pl.v2_nch);
    xe[idx] = gld(P.Qles + (tri(n) + m) * DD + e) - hs;
  }
  __syncthreads();
  for (int idx = tid; idx < nr * DD; idx += NTHR) {
    int r = idx / DD, e = idx % DD, a = e / D, c = e % D, m = pl.v2_lo + r;
    cplx out = mk(0, 0);
#pragma unroll
    for (int q = 0; q < D; q++) cfma_cb(out, xe[r * DD + a * D + q], minv[c * D + q]);
    gst(P.Gles + (tri(n) + m) * DD + e, out);
    xo[idx] = out;
  }
  __syncthreads();
  if (tid < DD) {
    int a2 = tid / D, c2 = tid % D;
    // their C2 terms, then the partials of every reduce workgroup in order
    cplx acc = mk(0, 0);
    for (int r = 0; r < nr; r++) {
      int l = pl.v2_lo + r;
      cplx t = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(t, xo[r * DD + q * D + a2], gld(P.Sret + (tri(n) + l) * DD + c2 * D + q));
      acc = acc - (h * greg(W, n, l)) * conj(t);
    }
    for (int g = 0; g < G && g < nwg; g++) acc = acc + dg[g * DD + tid];  // (groups g >= nwg hold no partial)
    xe[tid] = gld(P.Qles + (tri(n) + n) * DD + tid) - acc;
  }
  __syncthreads();
  if (tid < DD) {
    int a2 = tid / D, c2 = tid % D;
    cplx out = mk(0, 0);
#pragma unroll
    for (int q = 0; q < D; q++) cfma_cb(out, xe[a2 * D + q], minv[c2 * D + q]);
    gst(P.Gles + (tri(n) + n) * DD + tid, out);
  }
}

// ------------------------------------------------------------------ reduce
// Workgroups: the reduce tiles of the Dyson step (retarded rows m < n-k, the
// mixing row, lesser rows m < n-k when n > 2k), then one for the retarded
// rows m = n-k..n. Each also adds its fresh outputs to the sums of
// G^<_{n,n} (the lesser row m = n, Eq. cles1-cles3 with the new row and
// column of slice n):
//   retarded outputs  h w(n,m) G^R_{n,m} Fcc^<_{m,n}             (C1)
//   mixing outputs   -i h_tau w(ntau,m) G^rceil_{n,m} Fcc^lceil_{m,n}   (C3)
//   lesser outputs    h w(n,l) G^<_{n,l} Fcc^A_{l,n},  G^<_{n,l} = -(G^<_{l,n})^dag  (C2)
// into a d x d partial per workgroup; the last workgroup adds them up.
template <int D>
__global__ __launch_bounds__(NTHR) void k_v2_reduce(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  // partials per sequence and round: d = 1 outputs have few chunks, and
  // fewer registers let more reduce workgroups run at once
  constexpr int MSB = D >= 2 ? 16 : 4;
  constexpr int NOUT = TM * DD > (KMAX + 1) * DD ? TM * DD : (KMAX + 1) * DD;
  __shared__ cplx minv[(KMAX + 1) * DD];
  __shared__ cplx outs[NOUT];
  __shared__ cplx sol[NOUT];
  __shared__ cplx xe[2 * KMAX * DD], xo[2 * KMAX * DD];  // boundary rows: right-hand sides, solutions
  __shared__ cplx dg[NTHR];
  __shared__ int is_last;
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  double h = P.h, ht = P.htau, xi = P.sig;
  int t0 = pl.red_tiles[0], t1 = pl.red_tiles[1], t2 = pl.red_tiles[2];
  int nwg = t0 + t1 + t2 + 1;
  for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) minv[idx] = gld(sc.minv(pi) + idx);
  __syncthreads();
  cplx* dpart = sc.part(pi) + pl.v2_doff * DD;
  // one workgroup per tile, or (large batches) one per problem walking its tiles
  const int bw0 = pl.walk_tiles ? 0 : (int)blockIdx.x, bw1 = pl.walk_tiles ? nwg : bw0 + 1;
  for (int b = bw0; b < bw1; b++) {
  if (b < nwg - 1) {
    int fam, mt;
    if (b < t0) {
      fam = 0;
      mt = b;
    } else if (b < t0 + t1) {
      fam = 1;
      mt = b - t0;
    } else {
      fam = 2;
      mt = b - t0 - t1;
    }
    int mo = tid / DD, e = tid % DD, a = e / D, c = e % D;
    int m = mt * TM + mo;
    int mout = fam == 1 ? ntau + 1 : n - k;
    bool valid = mo < TM && m < mout;
    int mlo = mt * TM, nm = min(mlo + TM, mout) - mlo;
    const cplx* part = sc.part(pi);
    if (valid) {
      cplx r;
      long cs = (long)mout * DD;  // stride between the chunks of one output
      auto pp = [&](int job, int ch0) { return part + (pl.part_off[job] + (long)ch0 * mout + m) * DD + e; };
      if (fam == 0) {
        int c0 = m / pl.tj[0];
        const cplx* ps[1] = {pp(0, c0)};
        int cn[1] = {pl.nch[0] - c0};
        cplx sm[1];
        msum<1, MSB>(ps, cn, cs, sm);
        r = gld(P.Qret + (tri(n) + m) * DD + e) - h * sm[0];
      } else if (fam == 1) {
        cplx tb = (m <= k || m >= ntau - k) ? gld(part + (pl.part_off[6] + m) * DD + e) : mk(0, 0);
        const cplx* ps[2] = {pp(2, 0), pp(1, 0)};
        int cn[2] = {pl.nch[2], pl.nch[1]};
        cplx sm[2];
        msum<2, MSB>(ps, cn, cs, sm);
        r = gld(P.Qtv + ((size_t)n * (ntau + 1) + m) * DD + e) - ht * (sm[0] + tb) - h * sm[1];
      } else {
        int jmax = m > k ? m : k;
        bool split3 = pl.staged || pl.fuse_t;  // job 3 only l >= m, job 7 l < m
        int c3 = split3 ? m / pl.tj[3] : 0;
        int n7 = (split3 && m > 0) ? (m - 1) / pl.tj[7] + 1 : 0;
        const cplx* ps[4] = {pp(3, c3), split3 ? pp(7, 0) : part, pp(4, 0), pp(5, 0)};
        int cn[4] = {pl.nch[3] - c3, n7, jmax / pl.tj[4] + 1, pl.nch[5]};
        cplx sm[4];
        msum<4, MSB>(ps, cn, cs, sm);
        if (pl.fuse_t && m < k) {
          // terms j in (m, k] of C^<_1 (start-up weights), G~^R_{m,j} = -(G^R_{j,m})^dag
          cplx cr = mk(0, 0);
          for (int j = m + 1; j <= k; j++) {
            cplx t = mk(0, 0);
#pragma unroll
            for (int q = 0; q < D; q++)
              cfma_cb(t, gld(P.Sles + (tri(n) + j) * DD + q * D + c), gld(P.Gret + (tri(j) + m) * DD + q * D + a));
            cr = cr + W.s[m][j] * t;
          }
          sm[2] = sm[2] - cr;
        }
        // C^< = h (C1 + history) - i h_tau C3
        r = gld(P.Qles + (tri(n) + m) * DD + e) - h * (sm[0] + sm[1] + sm[2]) + ht * mul_i(sm[3]);
      }
      outs[mo * DD + e] = r;
    }
    __syncthreads();
    if (valid) {
      cplx out = mk(0, 0);
      if (fam < 2) {
#pragma unroll
        for (int q = 0; q < D; q++) cfma(out, minv[a * D + q], outs[mo * DD + q * D + c]);
        if (fam == 0) gst(P.Gret + (tri(n) + m) * DD + e, out);
        else gst(P.Gtv + ((size_t)n * (ntau + 1) + m) * DD + e, out);
      } else {
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(out, outs[mo * DD + a * D + q], minv[c * D + q]);
        gst(P.Gles + (tri(n) + m) * DD + e, out);
      }
      sol[mo * DD + e] = out;
    }
    __syncthreads();
    // this tile's terms of G^<_{n,n}: one output per thread group (one
    // memory round), then summed over the outputs in order
    if (valid) {
      int j = m;
      const cplx* x = sol + mo * DD;
      cplx t = mk(0, 0), v;
      if (fam == 0) {
#pragma unroll
        for (int q = 0; q < D; q++) cfma(t, x[a * D + q], gld(P.Sles + (tri(n) + j) * DD + q * D + c));
        v = (h * greg(W, n, j)) * t;
      } else if (fam == 1) {
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(t, x[a * D + q], gld(P.Stv + ((size_t)n * (ntau + 1) + ntau - j) * DD + c * D + q));
        v = -mul_i((ht * -xi * greg(W, ntau, j)) * t);
      } else {
        // G^<_{n,l} Fcc^A_{l,n} = -conj(sum_q G^<_{l,n}[q][a] F^R_{n,l}[c][q])
#pragma unroll
        for (int q = 0; q < D; q++) cfma(t, x[q * D + a], gld(P.Sret + (tri(n) + j) * DD + c * D + q));
        v = -(h * greg(W, n, j)) * conj(t);
      }
      outs[mo * DD + e] = v;
    }
    // summed over the tile's outputs by a pairwise tree (fixed order)
    constexpr int TP = TM <= 1 ? 1 : (TM <= 2 ? 2 : (TM <= 4 ? 4 : (TM <= 8 ? 8 : (TM <= 16 ? 16 : (TM <= 32 ? 32 : (TM <= 64 ? 64 : (TM <= 128 ? 128 : 256)))))));
    for (int w = TP / 2; w >= 1; w /= 2) {
      __syncthreads();
      for (int idx = tid; idx < w * DD; idx += NTHR) {
        int mm = idx / DD, e2 = idx % DD;
        if (mm + w < nm) outs[mm * DD + e2] = outs[mm * DD + e2] + outs[(mm + w) * DD + e2];
      }
    }
    __syncthreads();
    if (tid < DD) gst(dpart + (size_t)b * DD + tid, outs[tid]);
  } else {
    // retarded rows m = n - r, r = 0..k: G^R_{n,n} = Q^R_{n,n}; for r >= 1 the
    // k+1 points n-k..n with start-up weights s_{r,j} and G^R continued to
    // t < t' (Eq. cr1, second case; Eq. y_to_GR)
    for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) {
      int r = idx / DD, e = idx % DD, a = e / D, c = e % D, m = n - r;
      cplx v = gld(P.Qret + (tri(n) + m) * DD + e);
      if (r > 0) {
        cplx acc = mk(0, 0);
        for (int j = 1; j <= k; j++) {
          cplx s = mk(0, 0);
#pragma unroll
          for (int q = 0; q < D; q++)
            cfma(s, gld(P.Sret + (tri(n) + n - j) * DD + a * D + q), ret_ext_d(P.Gret, n - j, m, q, c, D));
          acc = acc + W.s[r][j] * s;
        }
        v = v - h * acc;
      }
      outs[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) {
      int r = idx / DD, e = idx % DD, a = e / D, c = e % D, m = n - r;
      cplx out = mk(0, 0);
      if (r == 0) {
        out = outs[idx];
      } else {
#pragma unroll
        for (int q = 0; q < D; q++) cfma(out, minv[r * DD + a * D + q], outs[r * DD + q * D + c]);
      }
      gst(P.Gret + (tri(n) + m) * DD + e, out);
      sol[idx] = out;
    }
    __syncthreads();
    for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) {
      int r = idx / DD, e = idx % DD, a = e / D, c = e % D, j = n - r;
      cplx t = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(t, sol[r * DD + a * D + q], gld(P.Sles + (tri(n) + j) * DD + q * D + c));
      outs[idx] = (h * greg(W, n, j)) * t;
    }
    __syncthreads();
    if (tid < DD) {
      cplx acc = mk(0, 0);
      for (int r = 0; r <= k; r++) acc = acc + outs[r * DD + tid];
      gst(dpart + (size_t)b * DD + tid, acc);
    }
  }
  __syncthreads();
  }
  // completion count (reset by k_v2_side): the last workgroup to arrive
  // finishes the column (a walking workgroup is the only one of its problem)
  if (pl.walk_tiles) __syncthreads();
  else if (!last_to_arrive(sc.counter(pi), nwg - 1, is_last)) return;
  v2_final<D>(P, sc, pi, n, pl, minv, xe, xo, dg);
}

// ---------------------------------------------------------------- start-up
// Retarded columns m = 0..k-1 (Sec. "Start", first item): y_p = G^R_{p,m},
//   y_p + h sum_{l=0..k} I_{m,p,l} F~^R_{p,l} y_l = Q^R_{p,m},  p = m+1..k,
// with y_m = Q^R_{m,m} (Eq. vie2_ini_r) and y_l = -[G^R_{m,l}]^dag, l < m.
template <int D>
__global__ __launch_bounds__(NTHR) void k_v2_start_ret(ProbArg pa, Scratch sc) {
  constexpr int DD = D * D;
  __shared__ cplx A[(KMAX * D) * (KMAX * D)];
  __shared__ cplx B[KMAX * D * D];
  __shared__ cplx y[(KMAX + 1) * DD];
  int pi = blockIdx.x;
  const Prob& P = pa.get(pi);
  const KW& W = c_kw[P.k];
  int k = P.k, tid = threadIdx.x;
  double h = P.h;
  for (int m = 0; m <= k; m++) {
    for (int e = tid; e < DD; e += NTHR) gst(P.Gret + (tri(m) + m) * DD + e, gld(P.Qret + (tri(m) + m) * DD + e));
    if (m == k) break;
    for (int idx = tid; idx < (m + 1) * DD; idx += NTHR) {
      int l = idx / DD, e = idx % DD, a = e / D, c = e % D;
      cplx v;
      if (l == m) v = gld(P.Qret + (tri(m) + m) * DD + e);
      else v = -conj(gld(P.Gret + (tri(m) + l) * DD + c * D + a));
      y[l * DD + e] = v;
    }
    __syncthreads();
    auto Aval = [&](int p, int l, int x, int yy) -> cplx {
      cplx v = (h * W.I[m][p][l]) * v2_fret<D>(P, p, l, x, yy);
      if (p == l && x == yy) v.x += 1.0;
      return v;
    };
    int nu = k - m, N = nu * D;
    for (int idx = tid; idx < N * N; idx += NTHR) {
      int rr = idx / N, cc = idx % N;
      A[idx] = Aval(m + 1 + rr / D, m + 1 + cc / D, rr % D, cc % D);
    }
    for (int idx = tid; idx < N * D; idx += NTHR) {
      int rr = idx / D, c = idx % D, p = m + 1 + rr / D, a = rr % D;
      cplx v = gld(P.Qret + (tri(p) + m) * DD + a * D + c);
      for (int l = 0; l <= m; l++)
        for (int qq = 0; qq < D; qq++) v = v - Aval(p, l, a, qq) * y[l * DD + qq * D + c];
      B[idx] = v;
    }
    __syncthreads();
    bool ok = true;
    if (tid < 64) ok = wave_solve(N, D, A, B);  // one wavefront solves
    if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    __syncthreads();
    for (int idx = tid; idx < nu * DD; idx += NTHR) {
      int p = m + 1 + idx / DD, e = idx % DD, a = e / D, c = e % D;
      gst(P.Gret + (tri(p) + m) * DD + e, B[((p - m - 1) * D + a) * D + c]);
    }
    __syncthreads();
  }
}

// Rows p = 1..k of the start-up rule with kernel F^R (Eq. MBCVSAMx01_start):
//   sum_{l=1..k} M_{p,l} y_l = q_p - M_{p,0} y_0,  M_{p,l} = delta_{pl} + h s_{p,l} F~^R_{p,l};
// q (k d x d, LDS) and y0 (d x d, LDS) given, the solution y_1..y_k left in B.
template <int D>
__device__ inline bool v2_start_solve(const Prob& P, const cplx* q, const cplx* y0, cplx* A, cplx* B) {
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  int k = P.k, tid = threadIdx.x, N = k * D;
  double h = P.h;
  auto Mval = [&](int p, int l, int x, int yy) -> cplx {
    cplx v = (h * W.s[p][l]) * v2_fret<D>(P, p, l, x, yy);
    if (p == l && x == yy) v.x += 1.0;
    return v;
  };
  for (int idx = tid; idx < N * N; idx += NTHR) {
    int rr = idx / N, cc = idx % N;
    A[idx] = Mval(rr / D + 1, cc / D + 1, rr % D, cc % D);
  }
  for (int idx = tid; idx < N * D; idx += NTHR) {
    int rr = idx / D, cc = idx % D, p = rr / D + 1, a = rr % D;
    cplx v = q[(p - 1) * DD + a * D + cc];
    for (int qq = 0; qq < D; qq++) v = v - Mval(p, 0, a, qq) * y0[qq * D + cc];
    B[idx] = v;
  }
  __syncthreads();
  bool ok = true;
  if (tid < 64) ok = wave_solve(N, D, A, B);  // one wavefront solves
  __syncthreads();
  return ok;
}

// Mixing rows 0..k at tau index m (second item): y_0 = i xi G^M(beta - tau_m)
// (Eq. vie2_ini_tv), q_p = Q^rceil_{p,m} - (C^rceil_2 + C^rceil_3)[F,1,G](p,m)
// (Eq. map_vie_tv).
template <int D>
__global__ __launch_bounds__(NTHR) void k_v2_start_tv(ProbArg pa, Scratch sc) {
  constexpr int DD = D * D;
  __shared__ cplx A[(KMAX * D) * (KMAX * D)];
  __shared__ cplx B[KMAX * D * D];
  __shared__ cplx q[KMAX * DD];
  __shared__ cplx y0[DD];
  int pi = blockIdx.y, m = blockIdx.x;
  const Prob& P = pa.get(pi);
  if (m > P.ntau) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  double ht = P.htau, xi = P.sig;
  for (int e = tid; e < DD; e += NTHR) {
    cplx v = xi * mul_i(gld(P.Gmat + (size_t)(ntau - m) * DD + e));
    y0[e] = v;
    gst(P.Gtv + (size_t)m * DD + e, v);
  }
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    const cplx* S = P.Stv + (size_t)p * (ntau + 1) * DD;
    cplx acc = mk(0, 0);
    auto prod = [&](int ls, int lm) {
      cplx s = mk(0, 0);
      for (int qq = 0; qq < D; qq++) cfma(s, gld(S + (size_t)ls * DD + a * D + qq), gld(P.Gmat + (size_t)lm * DD + qq * D + c));
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
    q[(p - 1) * DD + e] = gld(P.Qtv + ((size_t)p * (ntau + 1) + m) * DD + e) - acc;
  }
  __syncthreads();
  bool ok = v2_start_solve<D>(P, q, y0, A, B);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    gst(P.Gtv + ((size_t)p * (ntau + 1) + m) * DD + e, B[((p - 1) * D + a) * D + c]);
  }
}

// Lesser column n = 0..k (third item, after R and rceil): y_m = G^<_{m,n},
// y_0 = -[G^rceil_{n,0}]^dag (Eq. vie2_ini_les), q_p = Q^<_{p,n} -
// C^<_2[F,1,G](p,n) - C^<_3[F,1,G](p,n) (Eq. map_les_vie2); rows p <= n are kept.
template <int D>
__global__ __launch_bounds__(NTHR) void k_v2_start_les(ProbArg pa, Scratch sc) {
  constexpr int DD = D * D;
  __shared__ cplx A[(KMAX * D) * (KMAX * D)];
  __shared__ cplx B[KMAX * D * D];
  __shared__ cplx q[KMAX * DD];
  __shared__ cplx y0[DD];
  int pi = blockIdx.y, n = blockIdx.x;
  const Prob& P = pa.get(pi);
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  if (n > k) return;
  double h = P.h, ht = P.htau, xi = P.sig;
  for (int e = tid; e < DD; e += NTHR) {
    int a = e / D, c = e % D;
    cplx v = -conj(gld(P.Gtv + (size_t)n * (ntau + 1) * DD + c * D + a));
    y0[e] = v;
    gst(P.Gles + tri(n) * DD + e, v);
  }
  int jmax = n > k ? n : k;
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    cplx v = les_any_d(P.Qles, p, n, a, c, D);
    // C^<_2: int_0^{t_n} F^<(t_p, t) G^A(t, t_n), G^A_{j,n} = (G~^R_{n,j})^dag
    cplx c2 = mk(0, 0);
    for (int j = 0; j <= jmax; j++) {
      cplx t = mk(0, 0);
      for (int qq = 0; qq < D; qq++) cfma_cb(t, v2_fles<D>(P, p, j, a, qq), ret_ext_d(P.Gret, n, j, c, qq, D));
      c2 = c2 + greg(W, n, j) * t;
    }
    // C^<_3 = -i h_tau sum_j w F^rceil_{p,j} G^lceil_{j,n},
    // G^lceil_{j,n} = -xi (G^rceil_{n,ntau-j})^dag
    cplx c3 = mk(0, 0);
    for (int j = 0; j <= ntau; j++) {
      cplx t = mk(0, 0);
      for (int qq = 0; qq < D; qq++)
        cfma_cb(t, gld(P.Stv + ((size_t)p * (ntau + 1) + j) * DD + a * D + qq),
                gld(P.Gtv + ((size_t)n * (ntau + 1) + ntau - j) * DD + c * D + qq));
      c3 = c3 + (-xi * greg(W, ntau, j)) * t;
    }
    q[(p - 1) * DD + e] = v - h * c2 + ht * mul_i(c3);
  }
  __syncthreads();
  bool ok = v2_start_solve<D>(P, q, y0, A, B);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    if (p <= n) gst(P.Gles + (tri(n) + p) * DD + e, B[((p - 1) * D + a) * D + c]);
  }
}

// ---------------------------------------------------------------- launches
// k_v2_side reads only earlier slices: it runs beside the history sums on a
// stream forked from s and joined before the reduce (serially on s when the
// call may not create runtime objects or is being captured)
template <int D>
static hipError_t vie2_step_d(const ProbArg& pa, const Scratch& sc, int n, hipStream_t s, bool side_ok) {
  int k = pa.one.k, ntau = pa.one.ntau;
  HistPlan pl = make_plan(n, k, ntau, D);
  pl.vie2 = 1;
  SideStream* side = side_ok ? side_stream(s) : nullptr;
  dim3 gs(1 + pl.v2_rows * pl.v2_nch, pa.count);
  if (side) {
    (void)hipEventRecord(side->fork, s);
    (void)hipStreamWaitEvent(side->s, side->fork, 0);
    k_v2_side<D><<<gs, NTHR, 0, side->s>>>(pa, sc, pl);
    (void)hipEventRecord(side->join, side->s);
  } else {
    k_v2_side<D><<<gs, NTHR, 0, s>>>(pa, sc, pl);
  }
  k_history<D><<<dim3(pl.grid + 1, pa.count), NTHR, 0, s>>>(pa, sc, pl);
  if (side) (void)hipStreamWaitEvent(s, side->join, 0);
  int ntile = pl.red_tiles[0] + pl.red_tiles[1] + pl.red_tiles[2];
  pl.walk_tiles = pa.count >= REDUCE_WALK_MIN;
  k_v2_reduce<D><<<dim3(pl.walk_tiles ? 1 : ntile + 1, pa.count), NTHR, 0, s>>>(pa, sc, pl);
  return hipGetLastError();
}

hipError_t launch_vie2_step(const ProbArg& pa, const Scratch& sc, int n, int d, hipStream_t s, bool side_ok) {
  switch (d) {
    case 1: return vie2_step_d<1>(pa, sc, n, s, side_ok);
    case 2: return vie2_step_d<2>(pa, sc, n, s, side_ok);
    case 3: return vie2_step_d<3>(pa, sc, n, s, side_ok);
    case 4: return vie2_step_d<4>(pa, sc, n, s, side_ok);
    case 5: return vie2_step_d<5>(pa, sc, n, s, side_ok);
    case 6: return vie2_step_d<6>(pa, sc, n, s, side_ok);
    case 7: return vie2_step_d<7>(pa, sc, n, s, side_ok);
    case 8: return vie2_step_d<8>(pa, sc, n, s, side_ok);
  }
  return hipErrorInvalidValue;
}

template <int D>
static hipError_t vie2_start_d(const ProbArg& pa, const Scratch& sc, int ntau, hipStream_t s) {
  int k = pa.one.k;
  k_v2_start_ret<D><<<pa.count, NTHR, 0, s>>>(pa, sc);
  k_v2_start_tv<D><<<dim3(ntau + 1, pa.count), NTHR, 0, s>>>(pa, sc);
  k_v2_start_les<D><<<dim3(k + 1, pa.count), NTHR, 0, s>>>(pa, sc);
  return hipGetLastError();
}

hipError_t launch_vie2_start(const ProbArg& pa, const Scratch& sc, int d, int ntau, hipStream_t s) {
  switch (d) {
    case 1: return vie2_start_d<1>(pa, sc, ntau, s);
    case 2: return vie2_start_d<2>(pa, sc, ntau, s);
    case 3: return vie2_start_d<3>(pa, sc, ntau, s);
    case 4: return vie2_start_d<4>(pa, sc, ntau, s);
    case 5: return vie2_start_d<5>(pa, sc, ntau, s);
    case 6: return vie2_start_d<6>(pa, sc, ntau, s);
    case 7: return vie2_start_d<7>(pa, sc, ntau, s);
    case 8: return vie2_start_d<8>(pa, sc, ntau, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cntr
