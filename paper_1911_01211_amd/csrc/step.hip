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
//               Its workgroups also add their outputs to the long sums of
//               the k+1 lesser boundary rows m = n-k..n; the last one to
//               finish runs the k+1 short serial steps.
// For k < n <= 2k the lesser column is solved serially by k_column.
//
// Layout: canonical slice-major storage; a tile of consecutive outputs m
// reads consecutive blocks of one stored row, so history reads coalesce.
#include <map>
#include <mutex>

#include "launch.h"

namespace cntr {

constexpr int NTHR = 256;

// d <= 4: one output block per lane (64 outputs per workgroup); larger d:
// one output element per thread
int hist_tm(int d) { return d <= 4 ? 64 : (NTHR / (d * d) > 0 ? NTHR / (d * d) : 1); }
// term chunks: d = 1 blocks are single numbers, so long chunks keep the
// number of workgroups of a (large) batch moderate
constexpr int hist_tj(int d) { return d == 1 ? 256 : (d >= 8 ? 32 : 64); }
constexpr int hist_tjs(int d) { return d == 1 ? 512 : (d <= 4 ? 16 : (d >= 8 ? 16 : 32)); }
// staged path: term chunk of the history jobs and of the tau source
constexpr int STG_TJ = 32, STG_TJS = 16;
// d = 8 (FP64 MFMA path): terms per workgroup of the history jobs (staged
// shared operand: 32 KB) and of the tau source (two staged operands of 16 KB)
constexpr int MF8_TJ = 64, MF8_TAU_TJ = 16;

static int cdiv_i(int a, int b) { return (a + b - 1) / b; }

// Units of band c (terms 32c .. 32c + 31): the triangular panels have column
// tiles t <= c / 2 there, the mixing panel all of its tiles. Each group of 8
// units takes 40 workgroups.
__host__ __device__ inline int band_tri(const HistPlan& p, int c) { return min(p.bo[0], c / 2 + 1); }
__host__ __device__ inline int band_wgs(const HistPlan& p, int c) {
  return 40 * ((2 * band_tri(p, c) + p.bo[1] + 7) / 8);
}

// k_tau_shared: tiles of TSM outputs x TSP problems, chunks of TSV terms;
// the terms are split over TS_SPLIT workgroups (partial-sum chunks)
constexpr int TSM = 32, TSP = 32, TSV = 32, TS_NTAU = 512, TS_SPLIT = 4;

// Jobs: 0 retarded bulk, 1 left-mixing history, 2 tau source, 3 lesser
// history (for the staged path and d = 1 only its part l >= m), 4 source
// C^<_1, 5 source C^<_3, 6 tau-boundary corrections, 7 lesser history l < m
// (staged path and d = 1). For d = 1 the jobs 4, 5 and 7 have no workgroups
// of their own: jobs 0, 1 and 3 form them in the same pass over each stored
// panel.
constexpr bool hist_staged(int d) { return d == 2 || d == 4; }

// Term chunks of the history jobs chosen by the autotuner (cntr_set_tiles):
// per orbital count, up to TUNE_BANDS bands of slices n <= n_hi[b], each with
// its chunk; 0 bands = the built-in default. Tunable: d = 1 (one block per
// lane: chunks 32..256) and d = 8 (MFMA path: chunks 16..64).
TileTable g_tiles[9];

int tuned_tj(int d, int n) {
  const TileTable& t = g_tiles[d];
  for (int b = 0; b < t.nb; b++)
    if (n <= t.n_hi[b]) return t.tj[b];
  return t.nb > 0 ? t.tj[t.nb - 1] : 0;
}

bool tile_allowed(int d, int tj) {
  if (d == 1) return tj == 32 || tj == 64 || tj == 128 || tj == 256;
  if (d == 8) return tj == 16 || tj == 32 || tj == 64;
  return false;
}

// d = 4 one-pass units of slice n with units of 16 nsb slices
static int du_units(int n, int k, int ntau, int nsb) {
  int TS = 16 * nsb, nb = n - k;
  int ns = cdiv_i(n, TS), nt = cdiv_i(nb, DU_TT), ntt = cdiv_i(ntau + 1, DU_TT);
  int tri = 0;
  for (int c = 0; c < nt; c++) {
    int lo, cf;
    du_range(c, TS, ns, lo, cf);
    tri += ns - lo;
  }
  return (n >= 2 * k + 1 ? 2 : 1) * tri + ns * ntt;
}
// the tallest units of which there are still about six per compute unit
// (two run at once on each), so that the last ones finish close together
constexpr int DU_TARGET = 1400;

HistPlan make_plan(int n, int k, int ntau, int d, int tau_split, int du_nsb) {
  HistPlan p{};
  p.n = n;
  p.staged = hist_staged(d);
  p.TJ = hist_tj(d);
  int ttj = (d == 1 || d == 8) ? tuned_tj(d, n) : 0;
  if (d == 1 && ttj) p.TJ = ttj;
  p.TM = hist_tm(d);
  p.TJS = hist_tjs(d);
  int nb = n - k;  // bulk outputs m = 0..n-k-1
  bool les_bulk = n >= 2 * k + 1;
  p.njob = NJOB;
  int mout[NJOB] = {nb, ntau + 1, ntau + 1, les_bulk ? nb : 0, les_bulk ? nb : 0, les_bulk ? nb : 0,
                    ntau + 1, (les_bulk && (p.staged || d == 1)) ? nb : 0};
  int span[NJOB] = {n, n, ntau + 1, n, nb > k + 1 ? nb : k + 1, ntau + 1, 1, nb};
  for (int j = 0; j < NJOB; j++) {
    if (p.staged) {
      // column jobs (one term, 64 outputs per wave step) and row jobs (16
      // outputs x 4 terms per wave step)
      bool row = j == 4 || j == 5 || j == 7;
      p.tm[j] = row ? 16 : 64;
      p.tj[j] = j == 2 ? STG_TJS : STG_TJ;
    } else {
      // d = 8: tiles of 8 outputs (two per wave) on the MFMA path, except
      // the tau source
      p.tm[j] = d == 8 ? 8 : p.TM;
      p.tj[j] = d == 8 ? (j == 2 ? MF8_TAU_TJ : (ttj ? ttj : MF8_TJ)) : (j == 2 ? p.TJS : p.TJ);
    }
  }
  // d = 1: the mixing panel is read once for both of its consumers (job 1
  // forms the job-5 row sums of each 64-column tile)
  p.fuse_t = d == 1;
  if (p.fuse_t) p.tj[5] = p.tj[4] = p.tj[7] = p.TM;
  // d = 4: every panel is read once for both of its consumers; the column
  // sums come in chunks of the unit height, the row sums in chunks of DU_TT
  p.dual = d == 4;
  if (p.dual) {
    int nsb = du_nsb;
    if (nsb <= 0) {
      nsb = 1;
      for (int c : {4, 2})
        if (du_units(n, k, ntau, c) >= DU_TARGET) {
          nsb = c;
          break;
        }
    }
    p.du_nsb = nsb;
    p.tj[0] = p.tj[1] = p.tj[3] = 16 * nsb;
    p.tj[4] = p.tj[5] = p.tj[7] = DU_TT;
  }
  long off = 0;
  int wgs[NJOB];
  for (int j = 0; j < NJOB; j++) {
    p.mout[j] = mout[j];
    p.nch[j] = mout[j] > 0 ? cdiv_i(span[j], p.tj[j]) : 0;
    p.mtiles[j] = mout[j] > 0 ? cdiv_i(mout[j], p.tm[j]) : 0;
    if (j == 6) p.nch[j] = p.mtiles[j] = 1;  // one workgroup: both tau ends
    if (j == 2 && tau_split > 0) p.nch[j] = tau_split;
    bool none = (j == 2 && tau_split > 0) || ((j == 4 || j == 5 || j == 7) && p.fuse_t) ||
                (p.dual && j != 2 && j != 6);  // formed elsewhere
    wgs[j] = none ? 0 : p.nch[j] * p.mtiles[j];
    p.part_off[j] = off;
    off += (long)p.nch[j] * mout[j];
  }
  // dispatch order of the jobs' workgroups: job by job; for d = 8 the tau
  // boundary and the tau source first (short, independent of n), so that
  // they do not trail the history sums
  for (int i = 0; i < NJOB; i++) p.jorder[i] = i;
  if (d == 8) {
    const int ord8[NJOB] = {6, 2, 0, 1, 3, 4, 5, 7};
    for (int i = 0; i < NJOB; i++) p.jorder[i] = ord8[i];
  }
  p.wg_off[0] = 0;
  for (int i = 0; i < NJOB; i++) p.wg_off[i + 1] = p.wg_off[i] + wgs[p.jorder[i]];
  p.grid = p.wg_off[NJOB];
  // Band order pays once the history panels of a problem no longer fit in the
  // 256 MB last-level (Infinity) cache, so that a block's second consumer
  // would otherwise read it from HBM again.
  // Within a band the workgroups form units: one 32 x 64 tile of a panel,
  // read by its column job (one workgroup) and its row job (four workgroups
  // of 16 x 32). The five get the same index modulo 8, the XCD they are
  // dispatched to, so the second consumer finds the tile in that XCD's L2.
  // Only the tiles on or below the diagonal of the triangular panels form
  // units, so that the eight XCDs get even shares.
  double hist_bytes = 16.0 * d * d * ((double)n * (n + 1) + (double)n * (ntau + 1));
  p.banded = p.staged && !p.dual && les_bulk && hist_bytes > 160e6;
  if (p.dual) {
    int TS = 16 * p.du_nsb;
    p.du_ns = cdiv_i(n, TS);
    p.du_nt = cdiv_i(nb, DU_TT);
    p.du_ntau = cdiv_i(ntau + 1, DU_TT);
    p.du_np = les_bulk ? 2 : 1;
    p.du_full = p.du_part = 0;
    for (int c = 0; c < p.du_nt; c++) {
      int lo, cf;
      du_range(c, TS, p.du_ns, lo, cf);
      p.du_full += p.du_ns - cf;
      p.du_part += cf - lo;
    }
    p.du_total = p.du_np * (p.du_full + p.du_part) + p.du_ns * p.du_ntau;
    p.grid += p.du_total;
  }
  if (p.banded) {
    p.nband = p.nch[0];
    p.bo[0] = p.mtiles[0];  // column tiles of the retarded and lesser panels
    p.bo[1] = p.mtiles[1];  // column tiles of the mixing panel
    int w = 0;
    for (int c = 0; c < p.nband; c++) w += band_wgs(p, c);
    p.grid = w + p.nch[2] * p.mtiles[2] + 1;
  }
  // reduce tiles (retarded, mixing, lesser) and the per-tile partial sums of
  // the k+1 lesser boundary rows
  // (k_reduce: one output element per thread, NTHR / d^2 outputs per tile)
  int rtm = NTHR / (d * d) > 0 ? NTHR / (d * d) : 1;
  p.red_tiles[0] = cdiv_i(nb, rtm);
  p.red_tiles[1] = cdiv_i(ntau + 1, rtm);
  p.red_tiles[2] = les_bulk ? cdiv_i(nb, rtm) : 0;
  p.tail_off = off;
  off += (long)(p.red_tiles[0] + p.red_tiles[1] + p.red_tiles[2]) * (k + 1);
  // Dyson equation in integral form: the lesser rows without history-job
  // outputs (m >= n-k; every m < n for n <= 2k) are summed in chunks of
  // v2_ch terms by extra workgroups (row m has max(m,k)+1 + n + ntau+1
  // terms); their partials, then one partial of G^<_{n,n} per reduce
  // workgroup
  p.v2_lo = les_bulk ? nb : 0;
  p.v2_rows = n - p.v2_lo;
  p.v2_ch = 4 * rtm;
  p.v2_nch = cdiv_i((n - 1 > k ? n - 1 : k) + 1 + n + ntau + 1, p.v2_ch);
  p.v2_off = off;
  off += (long)p.v2_rows * p.v2_nch;
  p.v2_doff = off;
  off += p.red_tiles[0] + p.red_tiles[1] + p.red_tiles[2] + 1;
  p.total_blocks = off;
  return p;
}

size_t step_scratch_bytes(int nt, int k, int ntau, int d) {
  size_t mx = 0;
  // for one term chunk the partial storage grows with n: check the largest
  // few n of every band of chunks (the last slices, and the last slices of
  // each autotuned band)
  std::vector<int> ns = {nt, nt - 1};
  // (up to n = 2k the boundary lesser rows of the integral form are every
  // row, so a smaller n can need more)
  for (int n = k + 1; n <= nt && n <= 2 * k + 2; n++) ns.push_back(n);
  const TileTable& t = g_tiles[d];
  for (int b = 0; b < t.nb; b++) {
    int e = t.n_hi[b] < nt ? t.n_hi[b] : nt;
    ns.push_back(e);
    ns.push_back(e - 1);
  }
  for (int n : ns) {
    if (n <= k) continue;
    for (int ts : {0, TS_SPLIT})
      for (int nsb : {1, 2, 4}) {  // (every unit height the d = 4 path may choose)
        if (d != 4 && nsb > 1) continue;
        HistPlan p = make_plan(n, k, ntau, d, d == 1 ? ts : 0, nsb);
        size_t blocks = (size_t)p.total_blocks;
        if (blocks > mx) mx = blocks;
      }
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
__device__ __forceinline__ void prep_step(const Prob& P, const Scratch& sc, int pi, int n, cplx* lds) {
  constexpr int DD = D * D;
  constexpr int K1M = KMAX + 1;
  const KW& W = c_kw[P.k];
  int k = P.k, K1 = k + 1, tid = threadIdx.x, wave = tid / 64, lane = tid & 63;
  double h = P.h;
  int N = k * D;
  int n0 = n - k;                  // first row of the (k+1) x (k+1) window
  cplx* A = lds;                   // kD x (kD + 1) (padded rows)
  cplx* B = A + N * (N + 1);       // kD x D
  cplx* mw = B + N * D;            // 4 x DD matrices being inverted, one per wave
  cplx* sw = mw + 4 * DD;          // Sigma^R_{n0+i, n0+j}, j <= i, (k+1)^2 blocks
  cplx* ew = sw + K1M * K1M * DD;  // eps_{n0+i} - mu, k+1 blocks
  __shared__ int piv[4][8];
  // weight tables used below, staged with the operands in one memory round
  __shared__ double tS[K1M * K1M], tD[K1M * K1M], tG[K1M], ta0;
  // the boundary-row work of this step starts its completion count at 0
  if (tid == 0) *sc.counter(pi) = 0;
  if (tid < K1M * K1M) {
    tS[tid] = W.s[tid / K1M][tid % K1M];
    tD[tid] = W.D[tid / K1M][tid % K1M];
  }
  __shared__ double tGn[K1M];
  if (tid <= KMAX) tG[tid] = tid <= k ? greg(W, n0 + tid, n0 + tid) : 0.0;
  if (tid <= KMAX) tGn[tid] = tid <= k ? greg(W, n, n0 + tid) : 0.0;
  if (tid == 0) ta0 = W.a[0];
  // stage the window of Sigma^R and eps used by the solves below
#pragma unroll 4
  for (int idx = tid; idx < K1 * K1 * DD; idx += NTHR) {
    int i = idx / (K1 * DD), j = (idx / DD) % K1, e = idx % DD;
    sw[(i * K1M + j) * DD + e] = j <= i ? gld(P.Sret + (tri(n0 + i) + n0 + j) * DD + e) : mk(0, 0);
  }
  for (int idx = tid; idx < K1 * DD; idx += NTHR) {
    int i = idx / DD, e = idx % DD;
    cplx v = gld(P.eps + (size_t)(n0 + i + 1) * DD + e);
    if (e / D == e % D) v.x -= P.mu;
    ew[idx] = v;
  }
  // Sigma^<_{n0+i, n0+j}[x][y] (any order of i, j) for the boundary-row
  // source terms, d <= 4 and n >= 2k+1 only
  cplx* lw = ew + K1M * DD;
  if (D <= 4 && n >= 2 * k + 1)
#pragma unroll 4
    for (int idx = tid; idx < K1 * K1 * DD; idx += NTHR) {
      int i = idx / (K1 * DD), j = (idx / DD) % K1, e = idx % DD;
      lw[(i * K1M + j) * DD + e] = les_any<D>(P.Sles, n0 + i, n0 + j, e / D, e % D);
    }
  __syncthreads();
  // Sigma~^R_{n0+i, n0+j}[x][y] for any i, j in the window
  auto sig = [&](int i, int j, int x, int y) -> cplx {
    if (j <= i) return sw[(i * K1M + j) * DD + x * D + y];
    return -conj(sw[(j * K1M + i) * DD + y * D + x]);
  };
  // step matrix h^-1 a_0 + i e_m + i h w(m,m) Sigma^R_{m,m} of row m = n0 + i
  auto stepmat = [&](int i, int e) -> cplx {
    int x = e / D, y = e % D;
    cplx v = mul_i(ew[i * DD + e]) + (h * tG[i]) * mul_i(sw[(i * K1M + i) * DD + e]);
    if (x == y) v.x += ta0 / h;
    return v;
  };
  if constexpr (D <= 4) {
    // register-resident solves, one system per wavefront
    if (wave == 0) {
      // retarded boundary (transposed conjugate start-up): row r = (p-1)D + y
      // of  sum_l C_{l,p}^T Y_l^T = i C_{0,p}^T  with
      // C_{l,p}[x][y] = h^-1 D_{p,l} delta_xy + delta_pl i e_{n-p} + i h s_{p,l} Sigma~^R_{n-l,n-p}
      constexpr int NM = KMAX * D;
      cplx a[NM], bb[D];
      bool row = lane < N;
      int p = row ? lane / D + 1 : 1, y = lane % D;
      auto Cv = [&](int l, int x) -> cplx {
        cplx v = (h * tS[p * K1M + l]) * mul_i(sig(k - l, k - p, x, y));
        if (p == l) v = v + mul_i(ew[(k - p) * DD + x * D + y]);
        if (x == y) v.x += tD[p * K1M + l] / h;
        return v;
      };
#pragma unroll
      for (int q = 0; q < NM; q++) a[q] = (row && q < N) ? Cv(q / D + 1, q % D) : mk(0, 0);
#pragma unroll
      for (int cc = 0; cc < D; cc++) bb[cc] = row ? mul_i(Cv(0, cc)) : mk(0, 0);
      int col;
      bool ok = lane_gauss_jordan<NM, D>(N, a, bb, col);
      if (!ok && lane == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
      // unknown col = (l-1) D + c2 holds R_{n,n-l}[cc][c2] in bb[cc]
      if (row && col >= 0) {
        int l = col / D + 1, c2 = col % D;
#pragma unroll
        for (int cc = 0; cc < D; cc++) gst(P.Gret + (tri(n) + n - l) * DD + cc * D + c2, bb[cc]);
      }
      if (lane < DD) gst(P.Gret + (tri(n) + n) * DD + lane, (lane / D == lane % D) ? mk(0, -1) : mk(0, 0));
      if (n >= 2 * k + 1) {
        // source terms of the lesser boundary rows m_r = n-k+r from the
        // retarded boundary columns j = n-k..n:
        //   -i h sum_j w(n,j) Sigma^<_{m_r,j} (R_{n,j})^dag
        cplx* rb = A;  // R_{n,n-l} blocks, l = 0..k (LDS, wave 0 only)
        if (row && col >= 0) {
          int l = col / D + 1, c2 = col % D;
#pragma unroll
          for (int cc = 0; cc < D; cc++) rb[l * DD + cc * D + c2] = bb[cc];
        }
        if (lane < DD) rb[lane] = (lane / D == lane % D) ? mk(0, -1) : mk(0, 0);
        wave_sync();
        for (int v = lane; v < (k + 1) * DD; v += 64) {
          int r = v / DD, ee = v % DD, a2 = ee / D, c2 = ee % D;
          cplx pb = mk(0, 0);
          for (int jj = 0; jj <= k; jj++) {
            const cplx* sb = lw + (r * K1M + jj) * DD + a2 * D;
            const cplx* rr = rb + (k - jj) * DD + c2 * D;  // R_{n, n-k+jj}
            cplx t = mk(0, 0);
#pragma unroll
            for (int q = 0; q < D; q++) cfma_cb(t, sb[q], rr[q]);
            pb = pb + tGn[jj] * t;
          }
          sc.bsrc(pi, DD)[v] = -h * mul_i(pb);
        }
      }
    } else {
      // M_R^-1 (wave 1) and, for n >= 2k+1, the inverted step matrices of the
      // lesser boundary rows m = n-k..n (all three waves)
      for (int r = wave - 2; r <= k; r += 3) {
        if (r < 0 || n >= 2 * k + 1) {
          int i = r < 0 ? k : r;
          cplx a[D], bb[D];
#pragma unroll
          for (int q = 0; q < D; q++) {
            a[q] = lane < D ? stepmat(i, lane * D + q) : mk(0, 0);
            bb[q] = (lane == q) ? mk(1, 0) : mk(0, 0);
          }
          int col;
          bool ok = lane_gauss_jordan<D, D>(D, a, bb, col);
          if (!ok && lane == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
          cplx* dst = sc.minv(pi) + (r < 0 ? 0 : (1 + r) * DD);
          if (lane < D && col >= 0)
#pragma unroll
            for (int q = 0; q < D; q++) dst[col * D + q] = bb[q];
        }
      }
    }
    return;
  }
  // d > 4: the 8 x 8 inverses on single waves (M_R on wave 0, the lesser
  // boundary rows on waves 1..3), then the (kD) x (kD) retarded boundary
  // system on the whole workgroup
  if (wave == 0) {
    cplx* mr = mw;
    for (int e = lane; e < DD; e += 64) mr[e] = stepmat(k, e);
    wave_sync();
    bool ok = wave_inverse(D, mr, piv[0]);
    if (!ok && lane == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    for (int e = lane; e < DD; e += 64) sc.minv(pi)[e] = mr[e];
  } else if (n >= 2 * k + 1) {
    // inverses of the step matrices of the lesser boundary rows m = n-k..n;
    // waves 1..3 share the rows
    cplx* mb = mw + wave * DD;
    for (int r = wave - 1; r <= k; r += 3) {
      for (int e = lane; e < DD; e += 64) mb[e] = stepmat(r, e);
      wave_sync();
      bool okb = wave_inverse(D, mb, piv[wave]);
      if (!okb && lane == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
      for (int e = lane; e < DD; e += 64) sc.minv(pi)[(1 + r) * DD + e] = mb[e];
      wave_sync();
    }
  }
  // retarded boundary: sum_l C_{l,p}^T Y_l^T = i C_{0,p}^T  (Y_0 = -i) with
  // C_{l,p} = h^-1 D_{p,l} + delta_{pl} i e_{n-p} + i h s_{p,l} Sigma~^R_{n-l,n-p}
  auto Cval = [&](int l, int p, int x, int y) -> cplx {
    cplx v = (h * tS[p * K1M + l]) * mul_i(sig(k - l, k - p, x, y));
    if (p == l) v = v + mul_i(ew[(k - p) * DD + x * D + y]);
    if (x == y) v.x += tD[p * K1M + l] / h;
    return v;
  };
  int ld = N + 1;
  for (int idx = tid; idx < N * N; idx += NTHR) {
    int r = idx / N, q = idx % N;
    A[r * ld + q] = Cval(q / D + 1, r / D + 1, q % D, r % D);
  }
  cplx* Bw = A + N * ld;
  for (int idx = tid; idx < N * D; idx += NTHR) {
    int r = idx / D, cc = idx % D;
    Bw[idx] = mul_i(Cval(0, r / D + 1, cc, r % D));
  }
  __shared__ int s_piv[KMAX * D];
  __shared__ cplx s_ipv;
  __syncthreads();
  bool ok = wg_solve<NTHR / 64>(N, ld, D, A, Bw, s_piv, &s_ipv);
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) {
    int l = idx / DD, e = idx % DD, cc = e / D, bb = e % D;
    cplx v;
    if (l == 0) v = (cc == bb) ? mk(0, -1) : mk(0, 0);
    else v = Bw[((l - 1) * D + bb) * D + cc];
    P.Gret[(tri(n) + n - l) * DD + e] = v;
  }
}

// ------------------------------------------------------------- TAU SOURCE
// Gregory parts of Eqs. ctv2, ctv3 for a tile of tau outputs m and a chunk of
// terms J (f = 1): sum_J xi w(m,J) Sigma^rceil_{n,m-J} G^M_{ntau-J} for m > k
// and sum_J w(ntau-m, J-m) Sigma^rceil_{n,J} G^M_{J-m} for m < ntau-k. Both
// bands of operands are staged in LDS.
template <int D>
__device__ __forceinline__ void tau_source_tile(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl,
                                int mt, int ch, cplx* lds) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int TJS = D >= 8 ? 16 : 32;
  constexpr int NB = TM + TJS - 1;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  double xi = P.sig;
  int mlo = mt * TM, j0 = ch * TJS;
  int base2 = mlo - j0 - TJS + 1;  // Sigma^rceil_{n, base2 + i}
  int base3 = j0 - mlo - TM + 1;   // G^M_{base3 + i}
  cplx* sA = lds;                  // Sigma^rceil_{n,J}, J in chunk
  cplx* sB = sA + TJS * DD;        // G^M_{ntau-J}
  cplx* s2 = sB + TJS * DD;        // NB blocks
  cplx* s3 = s2 + NB * DD;         // NB blocks
  const cplx* Srow = P.Stv + (size_t)n * (ntau + 1) * DD;
  for (int idx = tid; idx < TJS * DD; idx += NTHR) {
    int J = j0 + idx / DD, ee = idx % DD;
    bool in = J <= ntau;
    sA[idx] = in ? Srow[(size_t)J * DD + ee] : mk(0, 0);
    sB[idx] = in ? P.Gmat[(size_t)(ntau - J) * DD + ee] : mk(0, 0);
  }
  for (int idx = tid; idx < NB * DD; idx += NTHR) {
    int i = idx / DD, ee = idx % DD;
    int x2 = base2 + i, x3 = base3 + i;
    s2[idx] = (x2 >= 0 && x2 <= ntau) ? Srow[(size_t)x2 * DD + ee] : mk(0, 0);
    s3[idx] = (x3 >= 0 && x3 <= ntau) ? P.Gmat[(size_t)x3 * DD + ee] : mk(0, 0);
  }
  __syncthreads();
  int mo = tid / DD, e = tid % DD, a = e / D, c = e % D;
  int m = mlo + mo;
  if (!(mo < TM && m <= ntau)) return;
  cplx acc = mk(0, 0);
  int Jhi = min(ntau, j0 + TJS - 1);
  for (int J = j0; J <= Jhi; J++) {
    if (m > k && J <= m) {
      const cplx* sb = s2 + (m - J - base2) * DD + a * D;
      const cplx* mb = sB + (J - j0) * DD + c;
      cplx s = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(s, sb[q], mb[q * D]);
      acc = acc + (xi * greg(W, m, J)) * s;
    }
    if (m < ntau - k && J >= m) {
      const cplx* sb = sA + (J - j0) * DD + a * D;
      const cplx* mb = s3 + (J - m - base3) * DD + c;
      cplx s = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(s, sb[q], mb[q * D]);
      acc = acc + greg(W, ntau - m, J - m) * s;
    }
  }
  sc.part(pi)[(pl.part_off[2] + (long)ch * (ntau + 1) + m) * DD + e] = acc;
}

// Boundary-convolution parts of Eqs. ctv2 (m <= k) and ctv3 (m >= ntau-k):
//   xi sum_{j,l} R_{m;j,l} Sigma^rceil_{n,l} G^M_{ntau-j}   and
//      sum_{j,l} R_{ntau-m;j,l} Sigma^rceil_{n,ntau-l} G^M_j
// for the 2(k+1) outputs near the two ends (one workgroup).
template <int D>
__device__ void tau_boundary(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl,
                             cplx* lds) {
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau, tid = threadIdx.x;
  double xi = P.sig;
  int K1 = k + 1;
  cplx* sLo = lds;            // Sigma^rceil_{n,0..k}
  cplx* sHi = sLo + K1 * DD;  // Sigma^rceil_{n,ntau-k..ntau}
  cplx* gLo = sHi + K1 * DD;  // G^M_{0..k}
  cplx* gHi = gLo + K1 * DD;  // G^M_{ntau-k..ntau}
  const cplx* Srow = P.Stv + (size_t)n * (ntau + 1) * DD;
  for (int idx = tid; idx < K1 * DD; idx += NTHR) {
    int i = idx / DD, ee = idx % DD;
    sLo[idx] = gld(Srow + (size_t)i * DD + ee);
    sHi[idx] = gld(Srow + (size_t)(ntau - k + i) * DD + ee);
    gLo[idx] = gld(P.Gmat + (size_t)i * DD + ee);
    gHi[idx] = gld(P.Gmat + (size_t)(ntau - k + i) * DD + ee);
  }
  __syncthreads();
  if constexpr (D == 8) {
    // the block products S^rceil_{n,l} G^M_{ntau-j} (low end) and
    // S^rceil_{n,ntau-l} G^M_j (high end) are shared by the k+1 outputs of
    // their end: each is formed once and added with the weights R of every
    // output. Thread t: end t / 128, half (t / 64) % 2 of the (j, l) pairs,
    // element t % 64; the halves are added through LDS.
    int end = tid >> 7, half = (tid >> 6) & 1, e = tid & 63, a = e / D, c = e % D;
    cplx acc[KMAX + 1];
#pragma unroll
    for (int mi = 0; mi <= KMAX; mi++) acc[mi] = mk(0, 0);
    for (int pr = half; pr < K1 * K1; pr += 2) {
      int j = pr / K1, l = pr % K1;
      const cplx* sa = end == 0 ? sLo + l * DD : sHi + (k - l) * DD;
      const cplx* gb = end == 0 ? gHi + (k - j) * DD : gLo + j * DD;
      cplx pv = mk(0, 0);
#pragma unroll
      for (int q = 0; q < D; q++) cfma(pv, sa[a * D + q], gb[q * D + c]);
#pragma unroll
      for (int mi = 0; mi <= KMAX; mi++)
        if (mi <= k) {
          double w = end == 0 ? xi * W.R[mi][j][l] : W.R[k - mi][j][l];
          acc[mi] = acc[mi] + w * pv;
        }
    }
    cplx* xr = gHi + K1 * DD;  // 2 ends x (k+1) outputs x DD
    if (half == 1)
#pragma unroll
      for (int mi = 0; mi <= KMAX; mi++)
        if (mi <= k) xr[(end * K1 + mi) * DD + e] = acc[mi];
    __syncthreads();
    if (half == 0)
#pragma unroll
      for (int mi = 0; mi <= KMAX; mi++)
        if (mi <= k) {
          int m = end == 0 ? mi : ntau - k + mi;
          sc.part(pi)[(pl.part_off[6] + m) * DD + e] = acc[mi] + xr[(end * K1 + mi) * DD + e];
        }
    return;
  }
  for (int idx = tid; idx < 2 * K1 * DD; idx += NTHR) {
    int o = idx / DD, e = idx % DD, a = e / D, c = e % D;
    cplx acc = mk(0, 0);
    int m;
    if (o < K1) {
      m = o;
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) {
          cplx s = mk(0, 0);
          for (int q = 0; q < D; q++) cfma(s, sLo[l * DD + a * D + q], gHi[(k - j) * DD + q * D + c]);
          acc = acc + (xi * W.R[m][j][l]) * s;
        }
    } else {
      m = ntau - k + (o - K1);
      for (int j = 0; j <= k; j++)
        for (int l = 0; l <= k; l++) {
          cplx s = mk(0, 0);
          for (int q = 0; q < D; q++) cfma(s, sHi[(k - l) * DD + a * D + q], gLo[j * DD + q * D + c]);
          acc = acc + W.R[ntau - m][j][l] * s;
        }
    }
    sc.part(pi)[(pl.part_off[6] + m) * DD + e] = acc;
  }
}

// ------------------------------------------- HISTORY, one block per lane
// For d <= 4 every lane owns one output block. The four waves of a workgroup
// share a tile of 64 consecutive outputs and split the chunk's terms
// (interleaved); a lane reads whole d x d history blocks (d^2 independent
// loads per term, the next term's block prefetched into registers). The
// operand shared by the tile (the Sigma row of slice n, or G^M) is staged in
// LDS; the four waves' sums are added in a fixed order through LDS.

// acc += conj(x y)
__device__ inline void cfma_cc(cplx& acc, cplx x, cplx y) {
  acc.x = fma(x.x, y.x, acc.x);
  acc.x = fma(-x.y, y.y, acc.x);
  acc.y = fma(-x.x, y.y, acc.y);
  acc.y = fma(-x.y, y.x, acc.y);
}

// pointer to read-only device memory in the global address space
using gcp = const CNTR_GLOBAL cplx*;
__device__ inline gcp G(const cplx* p) { return (gcp)p; }

template <int DD>
__device__ inline void ld_blk(cplx (&h)[DD], gcp p) {
#pragma unroll
  for (int e = 0; e < DD; e++) h[e] = p[e];
}

// acc += w S H  (S shared, in LDS)
template <int D>
__device__ inline void f_left(cplx (&acc)[D * D], double w, const cplx* S, const cplx (&H)[D * D]) {
#pragma unroll
  for (int a = 0; a < D; a++)
#pragma unroll
    for (int q = 0; q < D; q++) {
      cplx s = w * S[a * D + q];
#pragma unroll
      for (int c = 0; c < D; c++) cfma(acc[a * D + c], s, H[q * D + c]);
    }
}
// acc += w H S
template <int D>
__device__ inline void f_right(cplx (&acc)[D * D], double w, const cplx* S, const cplx (&H)[D * D]) {
#pragma unroll
  for (int q = 0; q < D; q++)
#pragma unroll
    for (int c = 0; c < D; c++) {
      cplx s = w * S[q * D + c];
#pragma unroll
      for (int a = 0; a < D; a++) cfma(acc[a * D + c], H[a * D + q], s);
    }
}
// acc += w H' S with H' = -H^dag
template <int D>
__device__ inline void f_right_t(cplx (&acc)[D * D], double w, const cplx* S, const cplx (&H)[D * D]) {
#pragma unroll
  for (int q = 0; q < D; q++)
#pragma unroll
    for (int c = 0; c < D; c++) {
      cplx s = (-w) * S[q * D + c];
#pragma unroll
      for (int a = 0; a < D; a++) cfma_cb(acc[a * D + c], s, H[q * D + a]);
    }
}
// acc += w H S^dag
template <int D>
__device__ inline void f_right_c(cplx (&acc)[D * D], double w, const cplx* S, const cplx (&H)[D * D]) {
#pragma unroll
  for (int c = 0; c < D; c++)
#pragma unroll
    for (int q = 0; q < D; q++) {
      cplx s = w * S[c * D + q];
#pragma unroll
      for (int a = 0; a < D; a++) cfma_cb(acc[a * D + c], H[a * D + q], s);
    }
}
// acc += w H' S^dag with H' = -H^dag
template <int D>
__device__ inline void f_right_tc(cplx (&acc)[D * D], double w, const cplx* S, const cplx (&H)[D * D]) {
#pragma unroll
  for (int c = 0; c < D; c++)
#pragma unroll
    for (int q = 0; q < D; q++) {
      cplx s = (-w) * S[c * D + q];
#pragma unroll
      for (int a = 0; a < D; a++) cfma_cc(acc[a * D + c], H[q * D + a], s);
    }
}

// Terms j = jb, jb+4, ... < je (uniform over the wave) of one lane.
// addr(j) gives a readable history block for every lane (clamped where the
// term does not apply), add(j, H) accumulates it (weight 0 where the term does
// not apply). Two register buffers alternate; every load is unconditional
// and the control flow uniform, so the loads of the next term stay in flight
// while the current one is multiplied.
template <int D, class Addr, class Add>
__device__ inline void term_loop(int jb, int je, Addr addr, Add add) {
  constexpr int DD = D * D;
  if (jb >= je) return;
  if constexpr (D == 1) {
    // single-number blocks: sixteen terms loaded together
    constexpr int U = 16;
    int jl = je - 1;
    for (int j = jb; j < je; j += 4 * U) {
      cplx h[U][1];
#pragma unroll
      for (int u = 0; u < U; u++) ld_blk<1>(h[u], addr(min(j + 4 * u, jl)));
#pragma unroll
      for (int u = 0; u < U; u++)
        if (j + 4 * u < je) add(j + 4 * u, h[u]);
    }
    return;
  }
  cplx ha[DD], hb[DD];
  int jl = je - 1;
  ld_blk<DD>(ha, addr(jb));
  for (int j = jb; j < je; j += 8) {
    ld_blk<DD>(hb, addr(min(j + 4, jl)));
    add(j, ha);
    if (j + 4 >= je) break;
    ld_blk<DD>(ha, addr(min(j + 8, jl)));
    add(j + 4, hb);
  }
}

// Adds the four waves' sums (fixed order) and writes the partial of each
// output of the tile. red: LDS, 3 * DD * 64 blocks.
template <int D>
__device__ inline void wave_sum_store(cplx (&acc)[D * D], cplx* red, bool valid, cplx* dst) {
  constexpr int DD = D * D;
  int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __syncthreads();
  if (wave > 0)
#pragma unroll
    for (int e = 0; e < DD; e++) red[((wave - 1) * DD + e) * 64 + lane] = acc[e];
  __syncthreads();
  if (wave == 0 && valid)
#pragma unroll
    for (int e = 0; e < DD; e++)
      gst(dst + e, ((acc[e] + red[e * 64 + lane]) + red[(DD + e) * 64 + lane]) + red[(2 * DD + e) * 64 + lane]);
}

// d = 1: both consumers of a stored panel in one pass. Each wave step loads
// one stored row j for the 64 outputs m of the tile; colf(j) is the lane's
// factor of its column sum (weight times the staged S^R_{n,j} or its
// conjugate), and rowq(j, h) gives the lane's term of the row sum of row j
// (zero where it does not apply):
//   mixing panel T (job 1 + job 5): row sums of C^<_3 without -i,
//     sum_m (-xi) w(ntau,m) T_{j,m} (S^rceil_{n,ntau-m})^*;
//   retarded panel R (job 0 + job 4): row sums of C^<_1[G,1,Sigma](j,n),
//     sum_{m<=j} w(j,m) R_{j,m} S^<_{m,n} (its terms m in (j, k] of the first
//     rows use -R_{m,j}^* and are added by k_reduce);
//   lesser panel L (job 3, stored L_{m,j}, m <= j): column sums over l >= m,
//     sum_j w(n,j) L_{m,j} (S^R_{n,j})^*; row sums over l < j (job-7
//     partials), sum_{m<j} w(n,m) (-L_{m,j}^*) (S^R_{n,m})^*.
// Eight rows are summed over the lanes at once (transposed butterfly: at
// exchange step t the lanes with bit t set keep the upper half of the live
// registers, so lane L < 8 ends with row bitrev3(L)); the sums are the
// row-job partials of column tile mt.
__device__ inline cplx shx1(cplx v, int m) { return mk(__shfl_xor(v.x, m), __shfl_xor(v.y, m)); }
// exchange step T of the transposed butterfly over W live registers pairs
template <int W, int T, int N>
__device__ inline void bfly(cplx (&q)[N], int lane) {
  bool up = (lane >> T) & 1;
#pragma unroll
  for (int i = 0; i < W; i++) {
    cplx keep = up ? q[i + W] : q[i], send = up ? q[i] : q[i + W];
    q[i] = keep + shx1(send, 1 << T);
  }
  if constexpr (W > 1) bfly<W / 2, T + 1>(q, lane);
}
template <class Addr, class ColF, class RowQ>
__device__ __forceinline__ void rows_fused(int jb, int je, int j0, int nro, cplx* dst, Addr addr, ColF colf, RowQ rowq,
                           cplx (&acc)[1]) {
  constexpr int U = 8;
  int lane = threadIdx.x & 63;
  int jl = je - 1;
  for (int j = jb; j < je; j += 4 * U) {
    cplx h[U];
#pragma unroll
    for (int u = 0; u < U; u++) h[u] = *addr(min(j + 4 * u, jl));
#pragma unroll
    for (int u = 0; u < U; u++)
      if (j + 4 * u < je) cfma(acc[0], colf(j + 4 * u), h[u]);
    if (j < nro) {  // (uniform) some row of this batch has a row output
      cplx q[U];
#pragma unroll
      for (int u = 0; u < U; u++) q[u] = (j + 4 * u < je && j + 4 * u < nro) ? rowq(j + 4 * u, h[u]) : mk(0, 0);
      bfly<U / 2, 0>(q, lane);
      q[0] = q[0] + shx1(q[0], 8);
      q[0] = q[0] + shx1(q[0], 16);
      q[0] = q[0] + shx1(q[0], 32);
      if (lane < U) {
        int b = lane, r = ((b & 1) << 2) | (b & 2) | ((b & 4) >> 2);  // bitrev3
        int row = j + 4 * r;
        if (row < je && row < nro) gst(dst + row, q[0]);
      }
    }
  }
}

template <int D>
__device__ __forceinline__ void hist_blk(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, int job,
                         int mt, int ch, cplx* lds) {
  constexpr int DD = D * D;
  constexpr int K1 = KMAX + 1;
  const KW& W = c_kw[P.k];
  __shared__ double s_om[K1];
  __shared__ double s_s[K1 * K1];
  WReg wr;
  wr.load(W, s_om);
  int k = P.k, ntau = P.ntau, tid = threadIdx.x, lane = tid & 63;
  int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
  if (tid < K1 * K1) s_s[tid] = W.s[tid / K1][tid % K1];
  int TJ = pl.TJ, mout = pl.mout[job];
  int mlo = mt * 64, mhi = min(mlo + 64, mout) - 1;
  int m = mlo + lane;
  bool valid = m < mout;
  int mc = valid ? m : mhi;  // in-range output index for address arithmetic
  int j0 = ch * TJ;
  if (job == 0 && j0 + TJ - 1 < mlo) return;
  if (job == 3 && D == 1 && pl.fuse_t && j0 + TJ - 1 < mlo) return;  // fused: stored rows l >= m only
  if (job == 4 && j0 > max(mhi, k)) return;
  gcp Gret = G(P.Gret), Gles = G(P.Gles), Gtv = G(P.Gtv);
  cplx* sh = lds;
  size_t T1 = (size_t)n * (ntau + 1);
  for (int idx = tid; idx < TJ * DD; idx += NTHR) {
    int jj = idx / DD, ee = idx % DD, j = j0 + jj;
    cplx v = mk(0, 0);
    switch (job) {
      case 0:
      case 1:
      case 3:
        if (j < n) v = gld(P.Sret + (tri(n) + j) * DD + ee);
        break;
      case 4:
        if (j <= n) v = gld(P.Sles + (tri(n) + j) * DD + ee);
        break;
      case 5:
        if (j <= ntau) v = gld(P.Stv + (T1 + ntau - j) * DD + ee);
        break;
    }
    sh[idx] = v;
  }
  __syncthreads();
  cplx acc[DD];
#pragma unroll
  for (int e = 0; e < DD; e++) acc[e] = mk(0, 0);
  int jb = j0 + wave;
  double xi = P.sig;
  size_t NT1 = ntau + 1;
  switch (job) {
    case 0: {  // retarded bulk: sum_j w(n-m, j-m) S^R_{n,j} R_{j,m}, j >= m
      int je = min(n, j0 + TJ);
      if constexpr (D == 1) {
        if (pl.fuse_t) {
          int nro = pl.mout[4];
          cplx sl = (valid && nro > 0) ? gld(P.Sles + tri(n) + mc) : mk(0, 0);  // S^<_{m,n}
          rows_fused(
              jb, je, j0, nro, sc.part(pi) + pl.part_off[4] + (long)mt * nro,
              [&](int j) { return Gret + (tri(max(j, mc)) + mc); },
              [&](int j) { return ((valid && j >= m) ? wr.w(n - m, j - m) : 0.0) * sh[j - j0]; },
              [&](int j, cplx h) {
                double w = 0.0;
                if (valid && mc <= j) w = j > k ? wr.w(j, mc) : s_s[j * K1 + mc];
                return (w * h) * sl;
              },
              acc);
          break;
        }
      }
      term_loop<D>(
          jb, je, [&](int j) { return Gret + (tri(max(j, mc)) + mc) * DD; },
          [&](int j, const cplx(&H)[DD]) {
            double w = (valid && j >= m) ? wr.w(n - m, j - m) : 0.0;
            f_left<D>(acc, w, sh + (j - j0) * DD, H);
          });
    } break;
    case 1: {  // left-mixing history: sum_j w(n,j) S^R_{n,j} T_{j,m}
      int je = min(n, j0 + TJ);
      if constexpr (D == 1) {
        if (pl.fuse_t) {
          int nro = pl.mout[5];
          cplx cst = mk(0, 0);  // per-lane factor of the row sums
          if (valid && nro > 0) cst = (-xi * wr.w(ntau, mc)) * conj(gld(P.Stv + T1 + ntau - mc));
          rows_fused(
              jb, je, j0, nro, sc.part(pi) + pl.part_off[5] + (long)mt * nro,
              [&](int j) { return Gtv + ((size_t)j * NT1 + mc); },
              [&](int j) { return (valid ? wr.w(n, j) : 0.0) * sh[j - j0]; }, [&](int j, cplx h) { return h * cst; },
              acc);
          break;
        }
      }
      term_loop<D>(
          jb, je, [&](int j) { return Gtv + ((size_t)j * NT1 + mc) * DD; },
          [&](int j, const cplx(&H)[DD]) { f_left<D>(acc, valid ? wr.w(n, j) : 0.0, sh + (j - j0) * DD, H); });
    } break;
    case 3: {  // lesser history: sum_l w(n,l) L^_{m,l} (S^R_{n,l})^dag
      int je = min(n, j0 + TJ);
      if constexpr (D == 1) {
        if (pl.fuse_t) {
          int nro = pl.mout[7];
          // per-lane factor of the row sums: -w(n,m) (S^R_{n,m})^*
          cplx fr = valid ? -(wr.w(n, mc) * conj(gld(P.Sret + tri(n) + mc))) : mk(0, 0);
          rows_fused(
              jb, je, j0, nro, sc.part(pi) + pl.part_off[7] + (long)mt * nro,
              [&](int l) { return Gles + (tri(max(l, mc)) + mc); },
              [&](int l) { return ((valid && l >= m) ? wr.w(n, l) : 0.0) * conj(sh[l - j0]); },
              [&](int l, cplx h) { return mc < l ? conj(h) * fr : mk(0, 0); }, acc);
          break;
        }
      }
      term_loop<D>(
          jb, je,
          [&](int l) { return l >= mc ? Gles + (tri(l) + mc) * DD : Gles + (tri(mc) + l) * DD; },
          [&](int l, const cplx(&H)[DD]) {
            double w = valid ? wr.w(n, l) : 0.0;
            if (l >= mc) f_right_c<D>(acc, w, sh + (l - j0) * DD, H);
            else f_right_tc<D>(acc, w, sh + (l - j0) * DD, H);
          });
    } break;
    case 4: {  // source C^<_1[G,1,Sigma](m,n): sum_j w(m,j) R~_{m,j} S^<_{j,n}, j <= max(m,k)
      int jmax = mc > k ? mc : k;
      int je = min(max(mhi, k) + 1, j0 + TJ);
      term_loop<D>(
          jb, je,
          [&](int j) {
            int jj = min(j, jmax);
            return jj <= mc ? Gret + (tri(mc) + jj) * DD : Gret + (tri(jj) + mc) * DD;
          },
          [&](int j, const cplx(&H)[DD]) {
            double w = 0.0;
            if (valid && j <= jmax) w = m > k ? wr.w(m, j) : s_s[m * K1 + j];
            if (j <= mc) f_right<D>(acc, w, sh + (j - j0) * DD, H);
            else f_right_t<D>(acc, w, sh + (j - j0) * DD, H);
          });
    } break;
    case 5: {  // source C^<_3 without -i: sum_j (-xi) w(ntau,j) T_{m,j} (S^rceil_{n,ntau-j})^dag
      int je = min(ntau + 1, j0 + TJ);
      term_loop<D>(
          jb, je, [&](int j) { return Gtv + ((size_t)mc * NT1 + j) * DD; },
          [&](int j, const cplx(&H)[DD]) {
            f_right_c<D>(acc, valid ? -xi * wr.w(ntau, j) : 0.0, sh + (j - j0) * DD, H);
          });
    } break;
  }
  wave_sum_store<D>(acc, lds, valid, sc.part(pi) + (pl.part_off[job] + (long)ch * mout + m) * DD);
}

// Tau source (Gregory parts of Eqs. ctv2, ctv3), one output block per lane:
//   sum_J xi w(m,J) Sigma^rceil_{n,m-J} G^M_{ntau-J}        (m > k, J <= m)
//   sum_J w(ntau-m, J-m) Sigma^rceil_{n,J} G^M_{J-m}        (m < ntau-k, J >= m)
// The operands indexed by J alone are staged in LDS, the banded ones are read
// per lane from the (cache-resident) Sigma row and G^M.
template <int D>
__device__ __forceinline__ void tau_blk(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, int mt, int ch,
                        cplx* lds) {
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  __shared__ double s_om[KMAX + 1];
  WReg wr;
  wr.load(W, s_om);
  int k = P.k, ntau = P.ntau, tid = threadIdx.x, lane = tid & 63;
  int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
  int TJS = pl.TJS;
  int m = mt * 64 + lane;
  bool valid = m <= ntau;
  int mc = valid ? m : ntau;
  int j0 = ch * TJS;
  const cplx* Srow = P.Stv + (size_t)n * (ntau + 1) * DD;
  gcp gS = G(Srow), gM = G(P.Gmat);
  cplx* sA = lds;             // Sigma^rceil_{n,J}
  cplx* sB = lds + TJS * DD;  // G^M_{ntau-J}
  for (int idx = tid; idx < TJS * DD; idx += NTHR) {
    int J = j0 + idx / DD, ee = idx % DD;
    bool in = J <= ntau;
    sA[idx] = in ? gld(Srow + (size_t)J * DD + ee) : mk(0, 0);
    sB[idx] = in ? gld(P.Gmat + (size_t)(ntau - J) * DD + ee) : mk(0, 0);
  }
  __syncthreads();
  cplx acc[DD];
#pragma unroll
  for (int e = 0; e < DD; e++) acc[e] = mk(0, 0);
  double xi = P.sig;
  int je = min(ntau + 1, j0 + TJS);
  int jb = j0 + wave;
  // band 1: per-lane left operand Sigma^rceil_{n,m-J}, shared right G^M_{ntau-J}
  term_loop<D>(
      jb, je, [&](int J) { return gS + (size_t)max(mc - J, 0) * DD; },
      [&](int J, const cplx(&H)[DD]) {
        double w = (valid && m > k && J <= m) ? xi * wr.w(m, J) : 0.0;
        f_right<D>(acc, w, sB + (J - j0) * DD, H);
      });
  // band 2: shared left Sigma^rceil_{n,J}, per-lane right G^M_{J-m}
  term_loop<D>(
      jb, je, [&](int J) { return gM + (size_t)max(J - mc, 0) * DD; },
      [&](int J, const cplx(&H)[DD]) {
        double w = (valid && m < ntau - k && J >= m) ? wr.w(ntau - m, J - m) : 0.0;
        f_left<D>(acc, w, sA + (J - j0) * DD, H);
      });
  wave_sum_store<D>(acc, lds, valid, sc.part(pi) + (pl.part_off[2] + (long)ch * (ntau + 1) + m) * DD);
}

// ------------------------------------------- HISTORY, staged through LDS
// d = 1, 2, 4. One wave step covers 64 history blocks. They are copied
// HBM -> LDS with direct-to-LDS loads in which every instruction reads 1 KB of
// contiguous memory (lane L loads 16 B), then each lane reads its own block
// from LDS and multiplies it from registers. The LDS copy of a step keeps one
// spare 16 B unit per 1 KB, and block b goes to lane ilane(b), so that the
// lanes' block reads are free of bank conflicts. While a lane multiplies the
// block of step s, the copy of step s + 1 is in flight.
//
// Column steps: 64 consecutive outputs m at one term j (blocks contiguous in
// one stored slice). Row steps: 16 outputs m at 4 consecutive terms (each
// output's 4 blocks contiguous in its own slice).
#if defined(__HIP_DEVICE_COMPILE__)
#define CNTR_LDS __attribute__((address_space(3)))
#else
#define CNTR_LDS
#endif

template <int D>
struct Stg {
  static constexpr int DD = D * D;
  static constexpr int NI = DD;         // copy instructions per step
  static constexpr int BPI = 64 / DD;   // blocks per instruction
  static constexpr int WBUF = NI * 65;  // 16 B units per wave buffer
  // block handled by a lane, and the lane handling a block
  __device__ static inline int blk(int lane) { return BPI * (lane % NI) + lane / NI; }
  // LDS unit of piece e of block b
  __device__ static inline int unit(int b, int e) {
    int P = b * DD + e;
    return P + P / 64;
  }
};

// The functions that stage through LDS are inlined into the kernels
// (__forceinline__): there the buffers are known LDS, and the compiler waits
// for a step's direct-to-LDS copy before its reads. Compiled as a called
// function with a generic buffer pointer, the reads became flat loads that
// were not ordered after the copies.
// Copy the 64 blocks of one step into wbuf; baddr(b) gives block b (readable).
template <int D, class BAddr>
__device__ inline void stg_copy(cplx* wbuf, BAddr baddr) {
  using S = Stg<D>;
  int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < S::NI; i++) {
    int P = i * 64 + lane, b = P / S::DD, e = P % S::DD;
    gcp src = baddr(b) + e;
    __builtin_amdgcn_global_load_lds((const CNTR_GLOBAL void*)src, (CNTR_LDS void*)(wbuf + i * 65), 16, 0, 0);
  }
}

// The steps s = 0..nsteps-1 of one wave: baddr(s, b), add(s, H).
template <int D, class BAddr, class Add>
__device__ inline void stg_loop(int nsteps, cplx* wbuf, BAddr baddr, Add add) {
  using S = Stg<D>;
  constexpr int DD = D * D;
  if (nsteps <= 0) return;
  int lane = threadIdx.x & 63, b = S::blk(lane);
  stg_copy<D>(wbuf, [&](int bb) { return baddr(0, bb); });
  for (int s = 0; s < nsteps; s++) {
    cplx H[DD];
#pragma unroll
    for (int e = 0; e < DD; e++) H[e] = wbuf[S::unit(b, e)];
    // the buffer is free once the reads are done; copy the next step
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    if (s + 1 < nsteps) stg_copy<D>(wbuf, [&](int bb) { return baddr(s + 1, bb); });
    add(s, H);
  }
}

// Adds the 4 x 64 lane sums of the workgroup (fixed order) into the partials
// of the tile's outputs. Column tiles: lane b of every wave adds to output b;
// row tiles: lanes of blocks 4o..4o+3 of every wave add to output o.
template <int D>
__device__ inline void stg_sum_store(cplx (&acc)[D * D], cplx* red, bool row, int m0, int mout,
                                     cplx* dst0) {
  using S = Stg<D>;
  constexpr int DD = D * D;
  int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < DD; e++) red[(wave * DD + e) * 64 + lane] = acc[e];
  __syncthreads();
  int nout = row ? 16 : 64, ncon = row ? 4 : 1;
  for (int v = tid; v < nout * DD; v += NTHR) {
    int o = v / DD, e = v % DD;
    int m = m0 + o;
    if (m >= mout) continue;
    cplx sum = mk(0, 0);
    for (int w = 0; w < 4; w++)
      for (int r = 0; r < ncon; r++) {
        int b = row ? 4 * o + r : o;
        int L = S::NI * (b % S::BPI) + b / S::BPI;
        sum = sum + red[(w * DD + e) * 64 + L];
      }
    gst(dst0 + (size_t)m * DD + e, sum);
  }
}

template <int D>
__device__ __forceinline__ void hist_stg(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, int job,
                         int mt, int ch, cplx* lds, cplx* sh) {
  using S = Stg<D>;
  constexpr int DD = D * D;
  constexpr int K1 = KMAX + 1;
  const KW& W = c_kw[P.k];
  __shared__ double s_om[K1];
  __shared__ double s_s[K1 * K1];
  WReg wr;
  wr.load(W, s_om);
  int k = P.k, ntau = P.ntau, tid = threadIdx.x, lane = tid & 63;
  int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < K1 * K1) s_s[tid] = W.s[tid / K1][tid % K1];
  bool row = job == 4 || job == 5 || job == 7;
  int TJ = pl.tj[job], TMj = pl.tm[job], mout = pl.mout[job];
  int m0 = mt * TMj, mhi = min(m0 + TMj, mout) - 1;
  int j0 = ch * TJ;
  if ((job == 0 || job == 3) && j0 + TJ - 1 < m0) return;  // terms j >= m only
  if (job == 4 && j0 > max(mhi, k)) return;                // terms j <= max(m, k)
  if (job == 7 && j0 >= mhi) return;                       // terms l < m
  cplx* wbuf = lds + wave * S::WBUF;
  gcp Gret = G(P.Gret), Gles = G(P.Gles), Gtv = G(P.Gtv);
  size_t T1 = (size_t)n * (ntau + 1), NT1 = ntau + 1;
  for (int idx = tid; idx < TJ * DD; idx += NTHR) {
    int jj = idx / DD, ee = idx % DD, j = j0 + jj;
    cplx v = mk(0, 0);
    switch (job) {
      case 0:
      case 1:
      case 3:
      case 7:
        if (j < n) v = gld(P.Sret + (tri(n) + j) * DD + ee);
        break;
      case 4:
        if (j <= n) v = gld(P.Sles + (tri(n) + j) * DD + ee);
        break;
      case 5:
        if (j <= ntau) v = gld(P.Stv + (T1 + ntau - j) * DD + ee);
        break;
    }
    sh[idx] = v;
  }
  __syncthreads();
  cplx acc[DD];
#pragma unroll
  for (int e = 0; e < DD; e++) acc[e] = mk(0, 0);
  double xi = P.sig;
  int b = S::blk(lane);
  // this lane's output, and for row steps its term offset
  int mo = row ? m0 + b / 4 : m0 + b, r4 = b % 4;
  bool valid = mo < mout;
  int mc = valid ? mo : mhi;
  int je;  // end of the chunk's terms (exclusive)
  switch (job) {
    case 4: je = min(max(mhi, k) + 1, j0 + TJ); break;
    case 5: je = min(ntau + 1, j0 + TJ); break;
    case 7: je = min(mhi, j0 + TJ); break;
    default: je = min(n, j0 + TJ); break;
  }
  int jl = je - 1;  // last term of the chunk (clamp for addresses)
  if (!row) {
    // column steps: term j = j0 + wave + 4 s, outputs m0 + b
    int nst = je > j0 + wave ? (je - j0 - wave + 3) / 4 : 0;
    auto jof = [&](int s) { return min(j0 + wave + 4 * s, jl); };
    auto mcl = [&](int bb) { return min(m0 + bb, mhi); };
    switch (job) {
      case 0:  // sum_j w(n-m, j-m) S^R_{n,j} R_{j,m}, j >= m
        stg_loop<D>(
            nst, wbuf, [&](int s, int bb) { int j = jof(s); return Gret + (tri(j) + min(mcl(bb), j)) * DD; },
            [&](int s, const cplx(&H)[DD]) {
              int j = j0 + wave + 4 * s;
              double w = (valid && j < je && j >= mo) ? wr.w(n - mo, j - mo) : 0.0;
              f_left<D>(acc, w, sh + (min(j, jl) - j0) * DD, H);
            });
        break;
      case 1:  // sum_j w(n,j) S^R_{n,j} T_{j,m}
        stg_loop<D>(
            nst, wbuf, [&](int s, int bb) { return Gtv + ((size_t)jof(s) * NT1 + mcl(bb)) * DD; },
            [&](int s, const cplx(&H)[DD]) {
              int j = j0 + wave + 4 * s;
              double w = (valid && j < je) ? wr.w(n, j) : 0.0;
              f_left<D>(acc, w, sh + (min(j, jl) - j0) * DD, H);
            });
        break;
      case 3:  // sum_{l >= m} w(n,l) L_{m,l} (S^R_{n,l})^dag
        stg_loop<D>(
            nst, wbuf, [&](int s, int bb) { int l = jof(s); return Gles + (tri(l) + min(mcl(bb), l)) * DD; },
            [&](int s, const cplx(&H)[DD]) {
              int l = j0 + wave + 4 * s;
              double w = (valid && l < je && l >= mo) ? wr.w(n, l) : 0.0;
              f_right_c<D>(acc, w, sh + (min(l, jl) - j0) * DD, H);
            });
        break;
    }
  } else {
    // row steps: terms jb + 0..3 with jb = j0 + 4 wave + 16 s, outputs m0 + b / 4
    int nst = je > j0 + 4 * wave ? (je - j0 - 4 * wave + 15) / 16 : 0;
    auto tof = [&](int s, int bb) { return j0 + 4 * wave + 16 * s + bb % 4; };
    auto mcl = [&](int bb) { return min(m0 + bb / 4, mhi); };
    switch (job) {
      case 4: {  // sum_j w(m,j) R~_{m,j} S^<_{j,n}, j <= max(m,k)
        int jmax = mc > k ? mc : k;
        stg_loop<D>(
            nst, wbuf,
            [&](int s, int bb) {
              int m = mcl(bb), jm = m > k ? m : k, j = min(min(tof(s, bb), jl), jm);
              return j <= m ? Gret + (tri(m) + j) * DD : Gret + (tri(j) + m) * DD;
            },
            [&](int s, const cplx(&H)[DD]) {
              int j = j0 + 4 * wave + 16 * s + r4;
              double w = 0.0;
              if (valid && j < je && j <= jmax) w = mo > k ? wr.w(mo, j) : s_s[mo * K1 + j];
              const cplx* Sb = sh + (min(j, jl) - j0) * DD;
              if (j <= mc || !(j <= jmax)) f_right<D>(acc, w, Sb, H);
              else f_right_t<D>(acc, w, Sb, H);
            });
      } break;
      case 5:  // sum_j (-xi) w(ntau,j) T_{m,j} (S^rceil_{n,ntau-j})^dag
        stg_loop<D>(
            nst, wbuf, [&](int s, int bb) { return Gtv + ((size_t)mcl(bb) * NT1 + min(tof(s, bb), jl)) * DD; },
            [&](int s, const cplx(&H)[DD]) {
              int j = j0 + 4 * wave + 16 * s + r4;
              double w = (valid && j < je) ? -xi * wr.w(ntau, j) : 0.0;
              f_right_c<D>(acc, w, sh + (min(j, jl) - j0) * DD, H);
            });
        break;
      case 7:  // sum_{l < m} w(n,l) L^_{m,l} (S^R_{n,l})^dag, L^_{m,l} = -(L_{l,m})^dag
        stg_loop<D>(
            nst, wbuf,
            [&](int s, int bb) {
              int m = mcl(bb), l = min(min(tof(s, bb), jl), max(m - 1, 0));
              return Gles + (tri(m) + l) * DD;
            },
            [&](int s, const cplx(&H)[DD]) {
              int l = j0 + 4 * wave + 16 * s + r4;
              double w = (valid && l < je && l < mo) ? wr.w(n, l) : 0.0;
              f_right_tc<D>(acc, w, sh + (min(l, jl) - j0) * DD, H);
            });
        break;
    }
  }
  stg_sum_store<D>(acc, lds, row, m0, mout, sc.part(pi) + (pl.part_off[job] + (long)ch * mout) * DD);
}

// Tau source (Gregory parts of Eqs. ctv2, ctv3), column steps over J: band 1
// xi w(m,J) Sigma^rceil_{n,m-J} G^M_{ntau-J} (m > k, J <= m) and band 2
// w(ntau-m, J-m) Sigma^rceil_{n,J} G^M_{J-m} (m < ntau-k, J >= m).
template <int D>
__device__ __forceinline__ void tau_stg(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, int mt, int ch,
                        cplx* lds, cplx* sh) {
  using S = Stg<D>;
  constexpr int DD = D * D;
  const KW& W = c_kw[P.k];
  __shared__ double s_om[KMAX + 1];
  cplx* sA = sh;                   // Sigma^rceil_{n,J}
  cplx* sB = sh + STG_TJS * DD;    // G^M_{ntau-J}
  WReg wr;
  wr.load(W, s_om);
  int k = P.k, ntau = P.ntau, tid = threadIdx.x, lane = tid & 63;
  int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int TJS = pl.tj[2];
  int m0 = mt * 64, j0 = ch * TJS;
  const cplx* Srow = P.Stv + (size_t)n * (ntau + 1) * DD;
  gcp gS = G(Srow), gM = G(P.Gmat);
  for (int idx = tid; idx < TJS * DD; idx += NTHR) {
    int J = j0 + idx / DD, ee = idx % DD;
    bool in = J <= ntau;
    sA[idx] = in ? gld(Srow + (size_t)J * DD + ee) : mk(0, 0);
    sB[idx] = in ? gld(P.Gmat + (size_t)(ntau - J) * DD + ee) : mk(0, 0);
  }
  __syncthreads();
  cplx* wbuf = lds + wave * S::WBUF;
  cplx acc[DD];
#pragma unroll
  for (int e = 0; e < DD; e++) acc[e] = mk(0, 0);
  double xi = P.sig;
  int b = S::blk(lane), m = m0 + b;
  bool valid = m <= ntau;
  int je = min(ntau + 1, j0 + TJS), jl = je - 1;
  int nst = je > j0 + wave ? (je - j0 - wave + 3) / 4 : 0;
  auto mcl = [&](int bb) { return min(m0 + bb, ntau); };
  // steps 0..nst-1: band 1 at J = j0 + wave + 4 s; steps nst..2 nst-1: band 2
  stg_loop<D>(
      2 * nst, wbuf,
      [&](int s, int bb) {
        int J = min(j0 + wave + 4 * (s < nst ? s : s - nst), jl), mm = mcl(bb);
        return s < nst ? gS + (size_t)max(mm - J, 0) * DD : gM + (size_t)max(J - mm, 0) * DD;
      },
      [&](int s, const cplx(&H)[DD]) {
        int J = j0 + wave + 4 * (s < nst ? s : s - nst);
        int Jc = min(J, jl);
        if (s < nst) {
          double w = (valid && J < je && m > k && J <= m) ? xi * wr.w(m, J) : 0.0;
          f_right<D>(acc, w, sB + (Jc - j0) * DD, H);
        } else {
          double w = (valid && J < je && m < ntau - k && J >= m) ? wr.w(ntau - m, J - m) : 0.0;
          f_left<D>(acc, w, sA + (Jc - j0) * DD, H);
        }
      });
  stg_sum_store<D>(acc, lds, false, m0, ntau + 1, sc.part(pi) + (pl.part_off[2] + (long)ch * (ntau + 1)) * DD);
}

// ------------------------------------- HISTORY, d = 4: one pass per panel
// Each stored panel feeds two sums of slice n: column sums (an output per
// position t, terms over the stored slices s) and row sums (an output per
// slice s, terms over the positions t):
//   R = G^R_{s,t} (t <= s):   column  w(n-t, s-t) S^R_{n,s} R_{s,t}           job 0
//                             row     w(s, t) R_{s,t} S^<_{t,n}               job 4
//                                     (starting weights s_{s,t} for s <= k)
//   L (block (s, t), t <= s): column  w(n, s) L_{s,t} (S^R_{n,s})^dag          job 3
//                             row     -(w(n, t) S^R_{n,t} L_{s,t})^dag, t < s  job 7
//   T = G^rceil_{s,tau}:      column  w(n, s) S^R_{n,s} T_{s,tau}             job 1
//                             row     (-xi) w(ntau, tau) T_{s,tau} (S^rceil_{n,ntau-tau})^dag
//                                                                             job 5
// (the history integrals of the retarded, left-mixing and lesser equations
// of the time step written as column and row sums of the stored panels;
// the row sums of R for s < k also take the terms t in (s, k], from the
// stored blocks (t, s)).
// A workgroup takes a unit of 16 nsb slices x DU_TT positions and walks its
// sub-tiles of 16 x 16 blocks (64 KB): while one sub-tile, staged in LDS,
// feeds both sums, the next one is loaded into registers. In a column step
// a wave takes one slice s of the sub-tile and its lane (t, p) column (or
// row) p of block (s, t); in a row step one position t and lane (s, p). The
// Sigma blocks of the sub-tile's slices and positions are staged with it;
// those of a step are the same for the whole wave (broadcast LDS reads).
// (Scalar loads would serialize: every wait on them drains all that are in
// flight.) The column sums over the unit's slices are written once per
// unit, the row sums over its positions once per sub-tile row: the partials
// of the per-job path's jobs, in column chunks of 16 nsb slices and row
// chunks of DU_TT positions.
constexpr int DU_BS = 17;              // LDS units (16 B) per staged block, one of padding
constexpr int DU_SS = 16 * DU_BS + 1;  // LDS units per staged slice
constexpr int DU_DAT = 16 * DU_SS;     // one staged sub-tile
constexpr int DU_LDS = DU_DAT + 512;   // and its 32 Sigma blocks

template <int PANEL>
__device__ __forceinline__ void hist_dual_panel(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl,
                                                int cs, int ct, cplx* lds, const double* s_om, const double* s_s) {
  constexpr int DD = 16, K1 = KMAX + 1;
  constexpr bool TRI = PANEL != 2;
  constexpr bool LEFT_COL = PANEL != 1;   // column sums S X (else X S^dag)
  constexpr bool RIGHT_ROW = PANEL != 1;  // row sums X S or X S^dag (else S X)
  constexpr int JC = PANEL == 0 ? 0 : (PANEL == 1 ? 3 : 1);
  constexpr int JR = PANEL == 0 ? 4 : (PANEL == 1 ? 7 : 5);
  const int k = P.k, ntau = P.ntau, NT1 = ntau + 1, tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int o = lane & 15, p = lane >> 4;
  const double xi = P.sig;
  const int nb = n - k, TS = 16 * pl.du_nsb, nq = 2 * pl.du_nsb;
  const int tlim = TRI ? nb : NT1;
  const int mcol = pl.mout[JC], mrow = pl.mout[JR];
  const cplx* X = PANEL == 0 ? P.Gret : (PANEL == 1 ? P.Gles : P.Gtv);
  const cplx* Fc = P.Sret + tri(n) * DD;  // S^R_{n,s}
  const cplx* Fr = PANEL == 0 ? P.Sles + tri(n) * DD : (PANEL == 1 ? P.Sret + tri(n) * DD : P.Stv + (size_t)n * NT1 * DD);
  cplx* pcol = sc.part(pi) + (pl.part_off[JC] + (long)cs * mcol) * DD;
  cplx* prow = sc.part(pi) + (pl.part_off[JR] + (long)ct * mrow) * DD;
  const int sbase = cs * TS, tbase = ct * DU_TT;
  auto gw = [&](int N, int j) -> double {
    bool left = j <= k, right = N - j <= k;
    double wl = s_om[left ? j : 0], wr = s_om[right ? N - j : 0];
    return left ? (right ? wl + wr - 1.0 : wl) : (right ? wr : 1.0);
  };
  // sub-tile q: slices sbase + 16 (q >> 1) + 0..15, positions tbase + 16 (q & 1) + 0..15
  auto valid = [&](int q) {
    int s0 = sbase + 16 * (q >> 1), t0 = tbase + 16 * (q & 1);
    return s0 < n && t0 < tlim && (!TRI || t0 <= s0 + 15);
  };
  auto next_valid = [&](int q) {
    for (q++; q < nq; q++)
      if (valid(q)) return q;
    return -1;
  };
  // wave w loads slices 4w..4w+3 of a sub-tile, each in four 1 KB pieces;
  // blocks outside the stored panel are read at a stored position (their
  // weights are zero)
  // and the Sigma blocks: 16 of the column sums (slices), 16 of the row sums
  // (positions), two values per thread
  cntr_v2d pre[16], pref[2];
  auto load = [&](int q) {
    int s0 = sbase + 16 * (q >> 1), t0 = tbase + 16 * (q & 1);
#pragma unroll
    for (int i = 0; i < 16; i++) {
      int sl = 4 * wave + (i >> 2), tl = 4 * (i & 3) + (lane >> 4), e = lane & 15;
      int s = min(s0 + sl, n - 1), t = t0 + tl;
      size_t bi = TRI ? tri(s) + min(t, s) : (size_t)s * NT1 + min(t, ntau);
      pre[i] = *(const CNTR_GLOBAL cntr_v2d*)(X + bi * DD + e);
    }
#pragma unroll
    for (int j = 0; j < 2; j++) {
      int f = 2 * tid + j, fb = f >> 4, e = f & 15;
      const cplx* src;
      if (fb < 16) {
        src = Fc + (size_t)min(s0 + fb, n - 1) * DD;
      } else {
        int tc = min(t0 + fb - 16, tlim - 1);
        src = Fr + (size_t)(PANEL == 2 ? ntau - tc : tc) * DD;
      }
      pref[j] = *(const CNTR_GLOBAL cntr_v2d*)(src + e);
    }
  };
  CNTR_LDS cntr_v2d* lv = (CNTR_LDS cntr_v2d*)lds;
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 16; i++) {
      int sl = 4 * wave + (i >> 2), tl = 4 * (i & 3) + (lane >> 4), e = lane & 15;
      lv[sl * DU_SS + tl * DU_BS + e] = pre[i];
    }
#pragma unroll
    for (int j = 0; j < 2; j++) lv[DU_DAT + 2 * tid + j] = pref[j];
  };
  auto lget = [&](int idx) {
    cntr_v2d t = lv[idx];
    return cplx{t.x, t.y};
  };
  cplx ca[4], cb[4], ra[4];  // column sums of this position half / of the other; row sums
#pragma unroll
  for (int r = 0; r < 4; r++) ca[r] = cb[r] = ra[r] = mk(0, 0);

  // One step: the lane's four values of its block and the step's Sigma block
  // are all read from LDS before any product (the reads stay in flight
  // together; a scheduling barrier keeps the compiler from interleaving them
  // with the products, which would leave one or two reads in flight).
  // column step i of the wave on sub-tile (s0, t0): slice s0 + 4 wave + i
  auto col_step = [&](int s0, int t0, int i) {
    int sl = 4 * wave + i, s = s0 + sl, t = t0 + o;
    bool ok = s < n && t < mcol && (!TRI || s >= t);
    int F = DU_DAT + sl * DD;  // staged S^R_{n,s}
    int b = sl * DU_SS + o * DU_BS;
    cplx v[4], f[16];
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = lget(LEFT_COL ? b + 4 * q + p : b + 4 * p + q);
#pragma unroll
    for (int x = 0; x < 16; x++) f[x] = lget(F + x);
    double w = 0.0;
    if (ok) w = PANEL == 0 ? gw(n - t, s - t) : gw(n, s);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = w * v[q];
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if constexpr (LEFT_COL) cfma(ca[r], f[4 * r + q], v[q]);  // ca[r] = (S X)[r][p]
        else cfma_cb(ca[r], v[q], f[4 * r + q]);                 // ca[r] = (X S^dag)[p][r]
      }
  };
  // row step i of the wave on sub-tile (s0, t0): position t0 + 4 wave + i
  auto row_step = [&](int s0, int t0, int i) {
    int tl = 4 * wave + i, t = t0 + tl, s = s0 + o;
    bool ok = s < mrow && t < tlim && (PANEL == 0 ? t <= s : (PANEL == 1 ? t < s : true));
    int E = DU_DAT + (16 + tl) * DD;  // staged Sigma block of position t
    int b = o * DU_SS + tl * DU_BS;
    // R, first rows s < k: the terms t in (s, k] take -(R_{t,s})^dag, the
    // stored block (t, s) of the same (first) sub-tile, with the starting
    // weights s_{s,t}
    bool trn = PANEL == 0 && s0 == 0 && t0 == 0 && t <= k;  // (uniform)
    bool tl_ = trn && s < t && s < mrow;
    cplx v[4], f[16];
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = lget(RIGHT_ROW ? b + 4 * p + q : b + 4 * q + p);
    if (trn) {
      int bt = tl * DU_SS + o * DU_BS;  // block (t, s): slice t, position s
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (tl_) v[q] = -conj(lget(bt + 4 * q + p));
    }
#pragma unroll
    for (int x = 0; x < 16; x++) f[x] = lget(E + x);
    double w = 0.0;
    if (ok) {
      if (PANEL == 0) w = s > k ? gw(s, t) : s_s[s * K1 + t];
      else if (PANEL == 1) w = gw(n, t);
      else w = -xi * gw(ntau, t);
    }
    if (tl_) w = s_s[s * K1 + t];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = w * v[q];
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if constexpr (PANEL == 0) cfma(ra[r], v[q], f[4 * q + r]);     // ra[r] = (X E)[p][r]
        else if constexpr (PANEL == 2) cfma_cb(ra[r], v[q], f[4 * r + q]);  // (X E^dag)[p][r]
        else cfma(ra[r], f[4 * r + q], v[q]);                         // ra[r] = (E X)[r][p]
      }
  };
  CNTR_LDS cntr_v2d* red = lv;  // the staging buffer, when free
  auto put = [&](int idx, cplx v) { red[idx] = cntr_v2d{v.x, v.y}; };
  auto get = [&](int idx) {
    cntr_v2d t = red[idx];
    return cplx{t.x, t.y};
  };
  // the four waves' row sums of slices s0..s0+15 (fixed order) to the partials
  auto row_flush = [&](int s0) {
#pragma unroll
    for (int r = 0; r < 4; r++) put((wave * 4 + r) * 64 + lane, ra[r]);
    __syncthreads();
    int oo = tid >> 4, e = tid & 15, L = (e >> 2) * 16 + oo, rr = e & 3;
    cplx sum = ((get(rr * 64 + L) + get((4 + rr) * 64 + L)) + get((8 + rr) * 64 + L)) + get((12 + rr) * 64 + L);
    if (PANEL == 1) sum = -conj(sum);
    int s = s0 + oo;
    if (s < mrow) gst(prow + (size_t)s * DD + e, sum);
    __syncthreads();
  };

  int cur = valid(0) ? 0 : next_valid(0);
  int half = cur >= 0 ? (cur & 1) : 0;  // position half of ca
  if (cur >= 0) {
    load(cur);
    store();
  }
  __syncthreads();
  while (cur >= 0) {
    int nxt = next_valid(cur);
    if (nxt >= 0) load(nxt);
    int s0 = sbase + 16 * (cur >> 1), t0 = tbase + 16 * (cur & 1);
#pragma unroll 1
    for (int i = 0; i < 4; i++) col_step(s0, t0, i);
#pragma unroll 1
    for (int i = 0; i < 4; i++) row_step(s0, t0, i);
    __syncthreads();
    if (nxt < 0 || (nxt >> 1) != (cur >> 1)) {
      row_flush(s0);
#pragma unroll
      for (int r = 0; r < 4; r++) ra[r] = mk(0, 0);
    }
    if (nxt >= 0) {
      store();
      if ((nxt & 1) != half) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          cplx t = ca[r];
          ca[r] = cb[r];
          cb[r] = t;
        }
        half = nxt & 1;
      }
    }
    __syncthreads();
    cur = nxt;
  }
  // column sums of the unit's 32 positions (the four waves' in a fixed order)
#pragma unroll
  for (int r = 0; r < 4; r++) {
    put(((wave * 2 + 0) * 4 + r) * 64 + lane, ca[r]);
    put(((wave * 2 + 1) * 4 + r) * 64 + lane, cb[r]);
  }
  __syncthreads();
#pragma unroll
  for (int h2 = 0; h2 < 2; h2++) {
    int v = tid + 256 * h2, h = v >> 8, oo = (v >> 4) & 15, e = v & 15;
    int pp = LEFT_COL ? (e & 3) : (e >> 2), rr = LEFT_COL ? (e >> 2) : (e & 3), L = pp * 16 + oo;
    cplx sum = mk(0, 0);
#pragma unroll
    for (int w = 0; w < 4; w++) sum = sum + get(((w * 2 + h) * 4 + rr) * 64 + L);
    int t = tbase + 16 * (h == 0 ? half : 1 - half) + oo;
    if (t < mcol) gst(pcol + (size_t)t * DD + e, sum);
  }
}

// unit u: the units below the diagonal of the triangular panels (R and L
// alternating), the mixing panel's, then the triangular units that meet the
// diagonal (fewer blocks), so that the short units come last
template <int D>
__device__ __forceinline__ void hist_dual(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl, int u, cplx* lds) {
  constexpr int K1 = KMAX + 1;
  __shared__ double s_om[K1];
  __shared__ double s_s[K1 * K1];
  const KW& W = c_kw[P.k];
  int tid = threadIdx.x;
  if (tid <= KMAX) s_om[tid] = W.omega[tid];
  if (tid < K1 * K1) s_s[tid] = W.s[tid / K1][tid % K1];
  // (published by the first barrier of the panel walk)
  int TS = 16 * pl.du_nsb, np = pl.du_np;
  int nfull = np * pl.du_full, ntt = pl.du_ns * pl.du_ntau;
  int panel = 2, cs = 0, ct = 0;
  auto tri_unit = [&](int v, bool full) {
    for (int c = 0; c < pl.du_nt; c++) {
      int lo, cf;
      du_range(c, TS, pl.du_ns, lo, cf);
      int a = full ? cf : lo, b = full ? pl.du_ns : cf;
      if (v < b - a) {
        ct = c;
        cs = b - 1 - v;
        return;
      }
      v -= b - a;
    }
  };
  if (u < nfull) {
    panel = np == 2 ? (u & 1) : 0;
    tri_unit(u / np, true);
  } else if (u < nfull + ntt) {
    int v = u - nfull;
    cs = pl.du_ns - 1 - v / pl.du_ntau;
    ct = v % pl.du_ntau;
  } else {
    int v = u - nfull - ntt;
    panel = np == 2 ? (v & 1) : 0;
    tri_unit(v / np, false);
  }
  if (panel == 0) hist_dual_panel<0>(P, sc, pi, n, pl, cs, ct, lds, s_om, s_s);
  else if (panel == 1) hist_dual_panel<1>(P, sc, pi, n, pl, cs, ct, lds, s_om, s_s);
  else hist_dual_panel<2>(P, sc, pi, n, pl, cs, ct, lds, s_om, s_s);
}

// ------------------------------------------- HISTORY, d = 8 on FP64 MFMA
// The d = 8 history sums are dense 8 x 8 complex block products; each is a
// real 16 x 16 x 16 product on v_mfma_f64_16x16x4f64 (four instructions)
// with the complex product embedded as
//   A = [Pr -Pi; Pi Pr] (shared operand P),  B = [Qr_0 Qr_1; Qi_0 Qi_1]
// (streamed operands of two outputs side by side), so that D rows 0..7 hold
// Re P Q_o and rows 8..15 Im P Q_o, columns 0..7 output 0 and 8..15 output 1.
// Lane l supplies A(l % 16, 4t + l / 16) and B(4t + l / 16, l % 16) of
// instruction t and holds D(l / 16 + 4r, l % 16), r = 0..3.
// Every sum has the form out_m = sum_j w(m, j) P_j Q_{j,m} (P_j shared by all
// outputs: jobs 0, 1), or out_m = sum_j w X_{m,j} Y_j (Y_j shared: jobs 3,
// 4, 5), computed as its transpose out^T = sum_j Y_j^T X_{m,j}^T.
typedef double mf_v4d __attribute__((ext_vector_type(4)));

__device__ inline void mfma8_term(mf_v4d& acc, cplx p0, cplx p1, bool bottom, cplx q0, cplx q1) {
  double a0 = bottom ? p0.y : p0.x, a1 = bottom ? p1.y : p1.x;
  double a2 = bottom ? p0.x : -p0.y, a3 = bottom ? p1.x : -p1.y;
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, q0.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, q1.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, q0.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, q1.y, acc, 0, 0, 0);
}

// Streamed block of output m and term j for the jobs above: pointer to the
// stored 8 x 8 block, read transposed (tr) and/or as -conj (nc); w = 0 when
// the term does not belong to the output (the pointer then stays in bounds).
struct Mf8Src {
  const cplx* blk;
  bool tr, nc;
  double w;
};
// Gregory weight w_{N,j} from the LDS copies of the start weights s (KP x KP)
// and the end weights omega: no memory loads of the global kind in the term
// loop, whose wait would also drain the prefetched blocks
struct Mf8W {
  const double* s;
  const double* om;
  int k;
  __device__ inline double greg(int N, int j) const {
    if (N <= k) return s[N * KP + j];
    bool left = j <= k, right = N - j <= k;
    if (left && right) return om[j] + om[N - j] - 1.0;
    if (left) return om[j];
    if (right) return om[N - j];
    return 1.0;
  }
};
template <int JOB>
__device__ inline Mf8Src mf8_src(const Prob& P, const Mf8W& W, int n, int m, bool mvalid, int j) {
  int k = P.k, ntau = P.ntau;
  Mf8Src s;
  s.tr = false;
  s.nc = false;
  if constexpr (JOB == 0) {  // R_{j,m}, j >= m, weight w(n-m, j-m)
    bool in = j >= m;
    s.blk = P.Gret + (in ? tri(j) + m : tri(m) + m) * 64;
    s.w = in ? W.greg(n - m, j - m) : 0.0;
  } else if constexpr (JOB == 1) {  // T_{j,m}, weight w(n, j)
    s.blk = P.Gtv + ((size_t)j * (ntau + 1) + m) * 64;
    s.w = W.greg(n, j);
  } else if constexpr (JOB == 3) {  // X = L^_{m,l}: L_{m,l} (l >= m) or -(L_{l,m})^dag; Q = X^T
    bool up = j >= m;
    s.blk = P.Gles + (up ? tri(j) + m : tri(m) + j) * 64;
    s.tr = up;
    s.nc = !up;
    s.w = W.greg(n, j);
  } else if constexpr (JOB == 4) {  // X = R~_{m,j}: R_{m,j} (j <= m) or -(R_{j,m})^dag; Q = X^T
    bool lo = j <= m;
    s.blk = P.Gret + (lo ? tri(m) + j : tri(j) + m) * 64;
    s.tr = lo;
    s.nc = !lo;
    s.w = j <= (m > k ? m : k) ? W.greg(m, j) : 0.0;
  } else {  // X = T_{m,j}; Q = X^T, weight -xi w(ntau, j)
    s.blk = P.Gtv + ((size_t)m * (ntau + 1) + j) * 64;
    s.tr = true;
    s.w = -(double)P.sig * W.greg(ntau, j);
  }
  if (!mvalid) s.w = 0.0;
  return s;
}

// Raw Q[kb][c], Q[kb + 4][c] of one streamed block; the weight and the sign
// of -conj are applied when the values are used, so that nothing waits for
// the load before then.
__device__ inline void mf8_load(const Mf8Src& s, int kb, int c, cplx& q0, cplx& q1) {
  int i0 = s.tr ? c * 8 + kb : kb * 8 + c;
  int i1 = s.tr ? c * 8 + kb + 4 : (kb + 4) * 8 + c;
  q0 = gld(s.blk + i0);
  q1 = gld(s.blk + i1);
}
// w q or w (-conj q)
__device__ inline cplx mf8_scale(cplx q, double w, bool nc) { return mk(nc ? -w * q.x : w * q.x, w * q.y); }

// One workgroup: 8 outputs (2 per wave) x one chunk of TJ terms of job
// 0, 1, 3, 4 or 5; the shared operand of the chunk is staged in LDS.
template <int JOB>
__device__ __forceinline__ void hist_mfma8_job(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl,
                                               int mt, int ch, cplx* lds) {
  constexpr int DD = 64, PD = 8;
  __shared__ double s_ss[KP * KP], s_om[KP];
  int k = P.k, ntau = P.ntau;
  int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int mout = pl.mout[JOB], tm = pl.tm[JOB];
  int TJ = pl.tj[JOB];  // <= MF8_TJ (the staging buffer)
  int j0 = ch * TJ;
  int mlo = mt * tm, mhi = min(mlo + tm, mout) - 1;
  if (JOB == 0 && j0 + TJ - 1 < mlo) return;
  if (JOB == 4 && j0 > max(mhi, k)) return;
  if (tid < KP * KP) s_ss[tid] = c_kw[k].s[tid / KP][tid % KP];
  if (tid < KP) s_om[tid] = c_kw[k].omega[tid];
  Mf8W W{s_ss, s_om, k};
  for (int idx = tid; idx < TJ * DD; idx += NTHR) {
    int jj = idx / DD, ee = idx % DD, j = j0 + jj;
    cplx v = mk(0, 0);
    if constexpr (JOB == 0 || JOB == 1 || JOB == 3) {
      if (j < n) v = gld(P.Sret + (tri(n) + j) * DD + ee);
    } else if constexpr (JOB == 4) {
      if (j <= n) v = gld(P.Sles + (tri(n) + j) * DD + ee);
    } else {
      if (j <= ntau) v = gld(P.Stv + ((size_t)n * (ntau + 1) + ntau - j) * DD + ee);
    }
    lds[idx] = v;
  }
  __syncthreads();
  int m0 = mlo + 2 * wv;
  if (m0 > mhi) return;
  int c16 = lane & 15, o = c16 >> 3, c = c16 & 7, kb = lane >> 4, r8 = lane & 7;
  bool bottom = (lane & 15) >= 8;
  int m = m0 + o;
  bool mvalid = m <= mhi;
  int mc = mvalid ? m : m0;  // clamped output of the lane
  // term range of the chunk (uniform over the wave)
  int jlo = j0, jhi;
  if constexpr (JOB == 0) {
    jlo = max(j0, m0);
    jhi = min(n - 1, j0 + TJ - 1);
  } else if constexpr (JOB == 1 || JOB == 3) {
    jhi = min(n - 1, j0 + TJ - 1);
  } else if constexpr (JOB == 4) {
    jhi = min(max(min(m0 + 1, mhi), k), j0 + TJ - 1);
  } else {
    jhi = min(ntau, j0 + TJ - 1);
  }
  // shared operand P_j of the lane: S (jobs 0, 1), conj(S) (3, 5), S^T (4)
  constexpr bool PT = JOB == 4, PC = JOB == 3 || JOB == 5;
  int pi0 = PT ? kb * 8 + r8 : r8 * 8 + kb;
  int pi1 = PT ? (kb + 4) * 8 + r8 : r8 * 8 + kb + 4;
  mf_v4d acc = {0.0, 0.0, 0.0, 0.0};
  if (jlo <= jhi) {
    cplx qa[PD], qb[PD];
    double wa[PD];
    bool na[PD];
#pragma unroll
    for (int u = 0; u < PD; u++) {
      Mf8Src sv = mf8_src<JOB>(P, W, n, mc, mvalid && jlo + u <= jhi, min(jlo + u, jhi));
      mf8_load(sv, kb, c, qa[u], qb[u]);
      wa[u] = sv.w;
      na[u] = sv.nc;
    }
    for (int jb = jlo; jb <= jhi; jb += PD) {
#pragma unroll
      for (int u = 0; u < PD; u++) {
        int j = jb + u;
        cplx q0 = mf8_scale(qa[u], wa[u], na[u]), q1 = mf8_scale(qb[u], wa[u], na[u]);
        int jn = j + PD;
        Mf8Src sv = mf8_src<JOB>(P, W, n, mc, mvalid && jn <= jhi, min(jn, jhi));
        mf8_load(sv, kb, c, qa[u], qb[u]);
        wa[u] = sv.w;
        na[u] = sv.nc;
        if (j <= jhi) {
          const cplx* sb = lds + (j - j0) * DD;
          cplx p0 = sb[pi0], p1 = sb[pi1];
          if (PC) {
            p0 = conj(p0);
            p1 = conj(p1);
          }
          mfma8_term(acc, p0, p1, bottom, q0, q1);
        }
      }
    }
  }
  if (!mvalid) return;
  // lane holds out'[kb][c] = (acc0, acc2) and out'[kb + 4][c] = (acc1, acc3)
  constexpr bool TRANS = JOB >= 3;
  cplx* dst = sc.part(pi) + (pl.part_off[JOB] + (long)ch * mout + m) * DD;
  int e0 = TRANS ? c * 8 + kb : kb * 8 + c;
  int e1 = TRANS ? c * 8 + kb + 4 : (kb + 4) * 8 + c;
  gst(dst + e0, mk(acc[0], acc[2]));
  gst(dst + e1, mk(acc[1], acc[3]));
}

// Tau source of d = 8 on MFMA (Gregory parts of Eqs. ctv2, ctv3), outputs
// m = 0..ntau, terms J of the chunk:
//   part B (m < ntau - k, J >= m): w(ntau-m, J-m) S^rceil_{n,J} G^M_{J-m}
//                                  (shared S^rceil_{n,J}: out accumulates)
//   part A (m > k, J <= m): xi w(m, J) S^rceil_{n,m-J} G^M_{ntau-J}
//                            (shared G^M_{ntau-J}: out^T accumulates)
// The two are added through LDS at the end. Every (chunk, output) of a
// valid output is written (zeros where no term applies).
__device__ __forceinline__ void tau_mfma8(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl,
                                          int mt, int ch, cplx* lds) {
  constexpr int DD = 64, PD = 8, TJ = MF8_TAU_TJ;
  __shared__ double s_ss[KP * KP], s_om[KP];
  int k = P.k, ntau = P.ntau;
  double xi = P.sig;
  int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int mout = ntau + 1, tm = pl.tm[2];
  int j0 = ch * TJ;
  int mlo = mt * tm, mhi = min(mlo + tm, mout) - 1;
  if (tid < KP * KP) s_ss[tid] = c_kw[k].s[tid / KP][tid % KP];
  if (tid < KP) s_om[tid] = c_kw[k].omega[tid];
  Mf8W W{s_ss, s_om, k};
  cplx* sS = lds;            // S^rceil_{n,J}, J in the chunk
  cplx* sM = lds + TJ * DD;  // G^M_{ntau-J}
  for (int idx = tid; idx < TJ * DD; idx += NTHR) {
    int J = j0 + idx / DD, ee = idx % DD;
    bool in = J <= ntau;
    sS[idx] = in ? gld(P.Stv + ((size_t)n * (ntau + 1) + J) * DD + ee) : mk(0, 0);
    sM[idx] = in ? gld(P.Gmat + (size_t)(ntau - J) * DD + ee) : mk(0, 0);
  }
  __syncthreads();
  int m0 = mlo + 2 * wv;
  if (m0 > mhi) return;
  int c16 = lane & 15, o = c16 >> 3, c = c16 & 7, kb = lane >> 4, r8 = lane & 7;
  bool bottom = (lane & 15) >= 8;
  int m = m0 + o;
  bool mvalid = m <= mhi;
  int mc = mvalid ? m : m0;
  int m1 = min(m0 + 1, mhi);
  int Jend = min(ntau, j0 + TJ - 1);
  mf_v4d accB = {0.0, 0.0, 0.0, 0.0}, accA = {0.0, 0.0, 0.0, 0.0};
  // part B: J in [max(j0, m0), Jend]; P = S_J (direct), Q = G^M_{J-m} (direct)
  {
    int jlo = max(j0, m0), jhi = Jend;
    auto src = [&](int J, bool ok, const cplx*& blk, double& w) {
      bool in = ok && mvalid && J >= mc && mc < ntau - k;
      blk = P.Gmat + (size_t)(in ? J - mc : 0) * DD;
      w = in ? W.greg(ntau - mc, J - mc) : 0.0;
    };
    if (jlo <= jhi) {
      cplx qa[PD], qb[PD];
      double wa[PD];
#pragma unroll
      for (int u = 0; u < PD; u++) {
        const cplx* blk;
        src(min(jlo + u, jhi), jlo + u <= jhi, blk, wa[u]);
        qa[u] = gld(blk + kb * 8 + c);
        qb[u] = gld(blk + (kb + 4) * 8 + c);
      }
      for (int jb = jlo; jb <= jhi; jb += PD) {
#pragma unroll
        for (int u = 0; u < PD; u++) {
          int J = jb + u;
          cplx q0 = wa[u] * qa[u], q1 = wa[u] * qb[u];
          const cplx* blk;
          src(min(J + PD, jhi), J + PD <= jhi, blk, wa[u]);
          qa[u] = gld(blk + kb * 8 + c);
          qb[u] = gld(blk + (kb + 4) * 8 + c);
          if (J <= jhi) {
            const cplx* sb = sS + (J - j0) * DD;
            mfma8_term(accB, sb[r8 * 8 + kb], sb[r8 * 8 + kb + 4], bottom, q0, q1);
          }
        }
      }
    }
  }
  // part A: J in [j0, min(Jend, m1)]; P = (G^M_{ntau-J})^T, Q = (S^rceil_{n,m-J})^T
  {
    int jlo = j0, jhi = min(Jend, m1);
    auto src = [&](int J, bool ok, const cplx*& blk, double& w) {
      bool in = ok && mvalid && J <= mc && mc > k;
      blk = P.Stv + ((size_t)n * (ntau + 1) + (in ? mc - J : 0)) * DD;
      w = in ? xi * W.greg(mc, J) : 0.0;
    };
    if (jlo <= jhi) {
      cplx qa[PD], qb[PD];
      double wa[PD];
#pragma unroll
      for (int u = 0; u < PD; u++) {
        const cplx* blk;
        src(min(jlo + u, jhi), jlo + u <= jhi, blk, wa[u]);
        qa[u] = gld(blk + c * 8 + kb);
        qb[u] = gld(blk + c * 8 + kb + 4);
      }
      for (int jb = jlo; jb <= jhi; jb += PD) {
#pragma unroll
        for (int u = 0; u < PD; u++) {
          int J = jb + u;
          cplx q0 = wa[u] * qa[u], q1 = wa[u] * qb[u];
          const cplx* blk;
          src(min(J + PD, jhi), J + PD <= jhi, blk, wa[u]);
          qa[u] = gld(blk + c * 8 + kb);
          qb[u] = gld(blk + c * 8 + kb + 4);
          if (J <= jhi) {
            const cplx* sb = sM + (J - j0) * DD;
            mfma8_term(accA, sb[kb * 8 + r8], sb[(kb + 4) * 8 + r8], bottom, q0, q1);
          }
        }
      }
    }
  }
  // out = accB + (accA)^T: the transposed part through this wave's LDS tile
  cplx* xt = lds + 2 * TJ * DD + wv * 2 * DD;
  xt[o * DD + c * 8 + kb] = mk(accA[0], accA[2]);
  xt[o * DD + c * 8 + kb + 4] = mk(accA[1], accA[3]);
  wave_sync();
  cplx t0 = xt[o * DD + kb * 8 + c], t1 = xt[o * DD + (kb + 4) * 8 + c];
  if (!mvalid) return;
  cplx* dst = sc.part(pi) + (pl.part_off[2] + (long)ch * mout + m) * DD;
  gst(dst + kb * 8 + c, mk(accB[0], accB[2]) + t0);
  gst(dst + (kb + 4) * 8 + c, mk(accB[1], accB[3]) + t1);
}

__device__ __forceinline__ void hist_mfma8(const Prob& P, const Scratch& sc, int pi, int n, const HistPlan& pl,
                                           int job, int mt, int ch, cplx* lds) {
  switch (job) {
    case 0: hist_mfma8_job<0>(P, sc, pi, n, pl, mt, ch, lds); break;
    case 1: hist_mfma8_job<1>(P, sc, pi, n, pl, mt, ch, lds); break;
    case 3: hist_mfma8_job<3>(P, sc, pi, n, pl, mt, ch, lds); break;
    case 4: hist_mfma8_job<4>(P, sc, pi, n, pl, mt, ch, lds); break;
    case 5: hist_mfma8_job<5>(P, sc, pi, n, pl, mt, ch, lds); break;
  }
}

// ------------------------------------------------------------- HISTORY
template <int D>
__global__ __launch_bounds__(NTHR) void k_history(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int TJ = D >= 8 ? 32 : 64;
  constexpr int PREPN = (KMAX * D) * (KMAX * D + 1) + KMAX * D * D + 4 * DD + (KMAX + 1) * (KMAX + 1) * DD +
                        (KMAX + 1) * DD + (D <= 4 ? (KMAX + 1) * (KMAX + 1) * DD : 0);
  constexpr int TSN = 2 * (D >= 8 ? 16 : 32) * DD + 2 * (TM + (D >= 8 ? 16 : 32) - 1) * DD;
  constexpr int LDSA = (2 * TJ * DD) > PREPN ? (2 * TJ * DD) : PREPN;
  constexpr int LDSB = LDSA > TSN ? LDSA : TSN;
  constexpr int LDSR0 = D <= 4 ? 3 * DD * 64 : 0;  // wave sums of the block-per-lane path
  constexpr bool STG = hist_staged(D);
  constexpr int LDSB1 = hist_tj(D) * DD > 2 * hist_tjs(D) * DD ? hist_tj(D) * DD : 2 * hist_tjs(D) * DD;
  constexpr int LDSR1 = D <= 4 && LDSB1 > LDSR0 ? LDSB1 : LDSR0;  // operands of the block-per-lane path
  constexpr int LDSR = STG ? 4 * Stg<D>::WBUF : LDSR1;              // staged path buffers
  constexpr int LDS8 = MF8_TJ * DD > 2 * MF8_TAU_TJ * DD + 8 * DD ? MF8_TJ * DD : 2 * MF8_TAU_TJ * DD + 8 * DD;
  constexpr int LDSS = PREPN > LDSR ? PREPN : LDSR;
  constexpr int LDSN = D == 8 ? LDS8 : (STG ? (D == 4 && DU_LDS > LDSS ? DU_LDS : LDSS) : (LDSB > LDSR ? LDSB : LDSR));
  __shared__ cplx lds[LDSN];
  // shared operand of a staged chunk (a separate array: its reads never wait
  // for the copies in flight into lds)
  __shared__ cplx shop[STG && D != 4 ? STG_TJ * DD : 1];
  // (d = 4: the tau jobs' shared operands go to the one-pass kernel's Sigma area)
  cplx* shp = D == 4 ? lds + DU_DAT : shop;
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  // workgroup 0 sets up the step (dispatched first, it overlaps the sums)
  int b = blockIdx.x - 1;
  if (b < 0) {
    // (d = 8: the set-up has a kernel of its own, k_prep, launched before)
    // (the integral form sets its step up in k_v2_side)
    if constexpr (D != 8)
      if (!pl.vie2) prep_step<D>(P, sc, pi, n, lds);
    return;
  }
  if constexpr (D == 4) {  // (one-pass units after the tau jobs)
    if (b >= pl.wg_off[NJOB]) {
      hist_dual<D>(P, sc, pi, n, pl, b - pl.wg_off[NJOB], lds);
      return;
    }
  }
  int job = 0, mt, ch;
  if (pl.banded) {
    // tau source and tau boundary first (short, latency-bound), then the bands
    int ntw = pl.nch[2] * pl.mtiles[2];
    if (b < ntw) {
      job = 2;
      mt = b / pl.nch[2];
      ch = b % pl.nch[2];
    } else if (b == ntw) {
      job = 6;
      mt = ch = 0;
    } else {
      b -= ntw + 1;
      // band c, unit u (8 units per group of 40 workgroups), slot s: 0 the
      // column job, 1..4 the row job's quarters of the unit's tile
      int c = 0, w;
      while (c < pl.nband - 1 && b >= (w = band_wgs(pl, c))) {
        b -= w;
        c++;
      }
      int g = b % 40, s = g / 8, u = (b / 40) * 8 + g % 8, nr = band_tri(pl, c);
      if (u >= 2 * nr + pl.bo[1]) return;
      int pn = u < nr ? 0 : (u < nr + pl.bo[1] ? 1 : 2);
      int t = pn == 0 ? u : (pn == 1 ? u - nr : u - nr - pl.bo[1]);
      if (s == 0) {
        job = pn == 0 ? 0 : (pn == 1 ? 1 : 3);
        mt = t;
        ch = c;
      } else {
        job = pn == 0 ? 4 : (pn == 1 ? 5 : 7);
        mt = 2 * c + ((s - 1) >> 1);
        ch = 2 * t + ((s - 1) & 1);
      }
      if (mt >= pl.mtiles[job] || ch >= pl.nch[job]) return;
    }
  } else {
    int i = 0;
    while (b >= pl.wg_off[i + 1]) i++;
    job = pl.jorder[i];
    int local = b - pl.wg_off[i];
    mt = local / pl.nch[job];
    ch = local % pl.nch[job];
  }
  if (job == 6) {
    tau_boundary<D>(P, sc, pi, n, pl, lds);
    return;
  }
  if constexpr (STG) {
    if (job == 2) tau_stg<D>(P, sc, pi, n, pl, mt, ch, lds, shp);
    else if constexpr (D != 4) hist_stg<D>(P, sc, pi, n, pl, job, mt, ch, lds, shop);
    return;
  } else if constexpr (D <= 4) {
    if (job == 2) {
      if (!pl.tau_shared) tau_blk<D>(P, sc, pi, n, pl, mt, ch, lds);  // else k_tau_shared
    } else {
      hist_blk<D>(P, sc, pi, n, pl, job, mt, ch, lds);
    }
    return;
  }
  if constexpr (D == 8) {
    if (job == 2) tau_mfma8(P, sc, pi, n, pl, mt, ch, lds);
    else hist_mfma8(P, sc, pi, n, pl, job, mt, ch, lds);
    return;
  } else {
  if (job == 2) {
    tau_source_tile<D>(P, sc, pi, n, pl, mt, ch, lds);
    return;
  }
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
}

// Set-up of a time step in a kernel of its own (d = 8: the 40 x 40 register
// solve would otherwise set the register and LDS budget of every history
// workgroup).
template <int D>
__global__ __launch_bounds__(NTHR) void k_prep(ProbArg pa, Scratch sc, int n) {
  constexpr int DD = D * D;
  constexpr int PREPN = (KMAX * D) * (KMAX * D + 1) + KMAX * D * D + 4 * DD + (KMAX + 1) * (KMAX + 1) * DD +
                        (KMAX + 1) * DD + (D <= 4 ? (KMAX + 1) * (KMAX + 1) * DD : 0);
  __shared__ cplx lds[PREPN];
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  if (n > P.nt) return;
  prep_step<D>(P, sc, pi, n, lds);
}

// -------------------------------------------------------------- REDUCE
// Sums the history partials of each output in chunk order, adds the BDF
// terms and applies M_R^-1 (retarded and left-mixing rows) or (M_R^dag)^-1
// from the right (lesser rows m < n-k). For n > 2k each workgroup then adds
// its fresh outputs to the long sums of the k+1 lesser boundary rows
// m_r = n-k+r, which take the serial form (Eq. MBCVSAMx_t for
// y(t) = G^<(t, t_n), p = i e, k = i Sigma^R, q = -i (C^<_2 + C^<_3)[Sigma,1,G]):
//   retarded tile : -i h    sum_j w(n,j)     Sigma^<_{m_r,j} (R_{n,j})^dag
//   mixing tile   : -h_tau  sum_j w(ntau,j)  Sigma^rceil_{m_r,j} G^lceil_{j,n},
//                   G^lceil_{j,n} = -xi (T_{n,ntau-j})^dag
//   lesser tile   : -i h    sum_j w(m_r,j)   Sigma^R_{m_r,j} L_{j,n}
// and the last workgroup to finish (completion counter, no waiting) sums the
// per-workgroup partials and adds the terms of the boundary rows themselves.
// The k+1 serial steps are linear in those sources: one more workgroup forms
// their block lower-triangular solution operator Z (from the inverses of the
// step set-up) while the tiles run, so the last workgroup applies Z in one
// parallel product instead of k+1 dependent steps.
// Sum of cnt values p[i * stride] (in a fixed order), B loads in flight.
template <int B>
__device__ inline cplx psum_b(const cplx* p, long stride, int cnt) {
  static_assert((B & (B - 1)) == 0, "pairwise sum over a power of two");
  cplx s[B];
#pragma unroll
  for (int u = 0; u < B; u++) s[u] = mk(0, 0);
  int i = 0;
  for (; i + B <= cnt; i += B) {
    cplx v[B];
#pragma unroll
    for (int u = 0; u < B; u++) v[u] = gld(p + (long)(i + u) * stride);
#pragma unroll
    for (int u = 0; u < B; u++) s[u] = s[u] + v[u];
  }
  {
    cplx v[B];
#pragma unroll
    for (int u = 0; u < B; u++) v[u] = i + u < cnt ? gld(p + (long)(i + u) * stride) : mk(0, 0);
#pragma unroll
    for (int u = 0; u < B; u++) s[u] = s[u] + v[u];
  }
#pragma unroll
  for (int w = B / 2; w >= 1; w /= 2)
#pragma unroll
    for (int u = 0; u < w; u++) s[u] = s[u] + s[u + w];
  return s[0];
}

// Sums of NS sequences p[s][i * stride], i < cnt[s], in rounds of B terms of
// every sequence loaded together: a round's loads are all in flight at once,
// so the sums take ceil(max cnt / B) memory rounds (not one per sequence and
// tail). Fixed summation order.
template <int NS, int B>
__device__ inline void msum(const cplx* const (&p)[NS], const int (&cnt)[NS], long stride, cplx (&out)[NS]) {
  static_assert((B & (B - 1)) == 0, "pairwise sum over a power of two");
  int mx = 0;
#pragma unroll
  for (int q = 0; q < NS; q++) {
    out[q] = mk(0, 0);
    mx = cnt[q] > mx ? cnt[q] : mx;
  }
  for (int i0 = 0; i0 < mx; i0 += B) {
    cplx v[NS][B];
#pragma unroll
    for (int q = 0; q < NS; q++)
#pragma unroll
      for (int u = 0; u < B; u++) v[q][u] = i0 + u < cnt[q] ? gld(p[q] + (long)(i0 + u) * stride) : mk(0, 0);
#pragma unroll
    for (int q = 0; q < NS; q++) {
#pragma unroll
      for (int w = B / 2; w >= 1; w /= 2)
#pragma unroll
        for (int u = 0; u < w; u++) v[q][u] = v[q][u] + v[q][u + w];
      out[q] = out[q] + v[q][0];
    }
  }
}

// BDF part -h^-1 sum_{l=1..k} a_l X_{n-l} of one element; x(l) gives the
// address of X_{n-l} (all loads issued together).
// (bdf_load issues the loads; bdf_add combines them later, so that other
// loads can be issued in between.)
template <class F>
__device__ inline void bdf_load(int k, F x, cplx (&v)[KMAX]) {
#pragma unroll
  for (int l = 1; l <= KMAX; l++) v[l - 1] = l <= k ? gld(x(l)) : mk(0, 0);
}
__device__ inline cplx bdf_add(const KW& W, int k, double h, const cplx (&v)[KMAX]) {
  cplx r = mk(0, 0);
#pragma unroll
  for (int l = 1; l <= KMAX; l++)
    if (l <= k) r = r - (W.a[l] / h) * v[l - 1];
  return r;
}

template <int D>
__global__ __launch_bounds__(NTHR) void k_reduce(ProbArg pa, Scratch sc, HistPlan pl) {
  constexpr int DD = D * D;
  constexpr int TM = NTHR / DD > 0 ? NTHR / DD : 1;
  constexpr int NVMAX = (KMAX + 1) * DD;
  constexpr int NSTAGE = NVMAX > NTHR ? NVMAX : NTHR;
  // partial sums loaded per sequence in one round (one workgroup per compute
  // unit for d >= 2, so registers are plentiful)
  constexpr int MSB = D == 4 ? 8 : (D >= 2 ? 16 : 8);
  __shared__ cplx outs[TM * DD];
  __shared__ cplx minv[DD];
  __shared__ cplx pre[NVMAX];
  __shared__ cplx stage[NSTAGE];
  __shared__ cplx sigs[(KMAX + 1) * TM * DD];
  __shared__ double twt[(KMAX + 1) * TM];  // quadrature weights of the tile terms
  __shared__ cplx ser[(KMAX * (KMAX + 1) / 2 + 2 * KMAX + 1) * DD];
  __shared__ double s_om[KMAX + 1], s_ss[(KMAX + 1) * (KMAX + 1)];  // Gregory end weights
  __shared__ double s_ah[KMAX + 1];                                // a_l / h (BDF)
  __shared__ double s_gw[(KMAX + 1) * (KMAX + 1)];                 // weights of the boundary rows
  __shared__ int is_last;
  int pi = blockIdx.y;
  const Prob& P = pa.get(pi);
  int n = pl.n;
  if (n > P.nt) return;
  const KW& W = c_kw[P.k];
  int k = P.k, ntau = P.ntau;
  double h = P.h, ht = P.htau, xi = P.sig;
  int t0 = pl.red_tiles[0], t1 = pl.red_tiles[1], t2 = pl.red_tiles[2];
  int nwg = t0 + t1 + t2;
  int NV = (k + 1) * DD;
  cplx* tpart = sc.part(pi) + pl.tail_off * DD;
  // Large batches: one workgroup per problem walks all its tiles and then
  // runs the boundary rows itself (no completion count across workgroups).
  bool walk = pl.walk_tiles;
  int tid = threadIdx.x;
  constexpr int K1M = KMAX + 1;
  if (tid <= KMAX) s_om[tid] = W.omega[tid];
  if (tid >= 1 && tid <= k) s_ah[tid] = W.a[tid] / h;
  if (tid < K1M * K1M) s_ss[tid] = W.s[tid / K1M][tid % K1M];
  // Gregory weight w(N, j) from the LDS tables (per-lane indices)
  auto gw = [&](int N, int j) -> double {
    if (N <= k) return s_ss[N * K1M + j];
    bool left = j <= k, right = N - j <= k;
    if (left && right) return s_om[j] + s_om[N - j] - 1.0;
    if (left) return s_om[j];
    if (right) return s_om[N - j];
    return 1.0;
  };
  auto bdf = [&](const cplx(&v)[KMAX]) {
    cplx r = mk(0, 0);
#pragma unroll
    for (int l = 1; l <= KMAX; l++)
      if (l <= k) r = r - s_ah[l] * v[l - 1];
    return r;
  };
  // Without the walk, workgroup nwg (present when n >= 2k+1) forms the
  // operator of the boundary rows instead of a tile; the walking workgroup
  // forms it after its tiles.
  int b_end = walk ? nwg : min((int)blockIdx.x + 1, nwg);
  for (int b = walk ? 0 : (int)blockIdx.x; b < b_end; b++) {
  __syncthreads();  // the LDS buffers of the previous tile are free
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
  if (tid < DD) minv[tid] = sc.minv(pi)[tid];
  const cplx* part = sc.part(pi);
  int mlo = mt * TM, mhi = min(mlo + TM, mout) - 1, nm = mhi - mlo + 1;
  // self-energy blocks of the boundary rows paired with this tile (used after
  // the outputs are formed; loaded now into registers, in the same memory
  // round as the partial sums, and stored to LDS afterwards)
  constexpr int NSG = KMAX + 1;  // (k+1) nm d^2 <= (KMAX+1) NTHR
  cplx sgv[NSG];
  bool bnd = n >= 2 * k + 1;
#pragma unroll
  for (int u = 0; u < NSG; u++) {
    int idx = tid + u * NTHR;
    sgv[u] = mk(0, 0);
    if (bnd && idx < (k + 1) * nm * DD) {
      int r = idx / (nm * DD), rem = idx % (nm * DD), mm = mlo + rem / DD, ee = rem % DD;
      int mr = n - k + r;
      if (fam == 0) sgv[u] = gld(P.Sles + (tri(mr) + mm) * DD + ee);  // Sigma^<_{mm,mr}, mm < mr
      else if (fam == 1) sgv[u] = gld(P.Stv + ((size_t)mr * (ntau + 1) + ntau - mm) * DD + ee);
      else sgv[u] = gld(P.Sret + (tri(mr) + mm) * DD + ee);
    }
  }
  if (valid) {
    cplx r = mk(0, 0);
    long cs = (long)mout * DD;  // stride between the chunks of one output
    auto pp = [&](int job, int ch0) { return part + (pl.part_off[job] + (long)ch0 * mout + m) * DD + e; };
    // every load of this output (partials, BDF history) in one round
    if (fam == 0) {
      int c0 = m / pl.tj[0];
      cplx bv[KMAX];
      bdf_load(k, [&](int l) { return P.Gret + (tri(n - l) + m) * DD + e; }, bv);
      const cplx* ps[1] = {pp(0, c0)};
      int cn[1] = {pl.nch[0] - c0};
      cplx sm[1];
      msum<1, MSB>(ps, cn, cs, sm);
      r = bdf(bv) - h * mul_i(sm[0]);
    } else if (fam == 1) {
      cplx bv[KMAX];
      bdf_load(k, [&](int l) { return P.Gtv + ((size_t)(n - l) * (ntau + 1) + m) * DD + e; }, bv);
      cplx tb = (m <= k || m >= ntau - k) ? gld(part + (pl.part_off[6] + m) * DD + e) : mk(0, 0);
      const cplx* ps[2] = {pp(2, 0), pp(1, 0)};
      int cn[2] = {pl.nch[2], pl.nch[1]};
      cplx sm[2];
      msum<2, MSB>(ps, cn, cs, sm);
      cplx ts = ht * (sm[0] + tb);
      r = bdf(bv) - mul_i(ts) - h * mul_i(sm[1]);
    } else {
      int jmax = m > k ? m : k;
      cplx bv[KMAX];
      bdf_load(k, [&](int l) { return P.Gles + (tri(n - l) + m) * DD + e; }, bv);
      // lesser history: one job over all l, or (staged) l >= m and l < m
      bool split3 = pl.staged || pl.fuse_t;  // job 3 only l >= m, job 7 l < m
      int c3 = split3 ? m / pl.tj[3] : 0;
      int n7 = (split3 && m > 0) ? (m - 1) / pl.tj[7] + 1 : 0;
      const cplx* ps[4] = {pp(3, c3), split3 ? pp(7, 0) : part, pp(4, 0), pp(5, 0)};
      int cn[4] = {pl.nch[3] - c3, n7, jmax / pl.tj[4] + 1, pl.nch[5]};
      cplx sm[4];
      msum<4, MSB>(ps, cn, cs, sm);
      if (pl.fuse_t && m < k) {
        // terms j in (m, k] of C^<_1 (start-up weights), R~_{m,j} = -(R_{j,m})^dag
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
      cplx s3 = sm[0] + sm[1];
      r = bdf(bv) + h * mul_i(sm[2]) + ht * sm[3] + h * mul_i(s3);
    }
    outs[mo * DD + e] = r;
  }
  if (bnd) {
#pragma unroll
    for (int u = 0; u < NSG; u++)
      if (tid + u * NTHR < (k + 1) * nm * DD) sigs[tid + u * NTHR] = sgv[u];
    for (int idx = tid; idx < (k + 1) * nm; idx += NTHR) {
      int r = idx / nm, mm = mlo + idx % nm;
      double w;
      if (fam == 0) w = gw(n, mm);
      else if (fam == 1) w = -xi * gw(ntau, ntau - mm);
      else w = gw(n - k + r, mm);
      twt[idx] = w;
    }
  }
  __syncthreads();
  cplx out = mk(0, 0);
  if (valid) {
    if (fam < 2) {
      for (int q = 0; q < D; q++) cfma(out, minv[a * D + q], outs[mo * DD + q * D + c]);
      if (fam == 0) gst(P.Gret + (tri(n) + m) * DD + e, out);
      else gst(P.Gtv + ((size_t)n * (ntau + 1) + m) * DD + e, out);
    } else {
      // X M_L = rhs with M_L = M_R^dag:  X = rhs (M_R^-1)^dag
      for (int q = 0; q < D; q++) cfma_cb(out, outs[mo * DD + a * D + q], minv[c * D + q]);
      gst(P.Gles + (tri(n) + m) * DD + e, out);
    }
  }
  if (n >= 2 * k + 1) {  // (else the column is finished serially by k_column)
  __syncthreads();
  if (valid) outs[mo * DD + e] = out;
  __syncthreads();
  // contribution of this tile to the boundary rows
  // G2 thread groups per value split the tile's outputs; the groups' sums
  // are added in a fixed order
  int G2 = NV >= NTHR ? 1 : NTHR / NV;
  for (int vv = tid; vv < G2 * NV; vv += NTHR) {
    int g2 = vv / NV, v = vv % NV;
    int r = v / DD, ee = v % DD, a2 = ee / D, c2 = ee % D;
    int mr = n - k + r;
    cplx acc = mk(0, 0);
    for (int mm = mlo + g2; mm <= mhi; mm += G2) {
      const cplx* ob = outs + (mm - mlo) * DD;
      const cplx* sb = sigs + (r * nm + mm - mlo) * DD;
      cplx s = mk(0, 0);
      if (fam == 0) {  // Sigma^<_{mr,mm} = -[Sigma^<_{mm,mr}]^dag
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(s, -conj(sb[q * D + a2]), ob[c2 * D + q]);
        acc = acc + twt[r * nm + mm - mlo] * s;
      } else if (fam == 1) {
#pragma unroll
        for (int q = 0; q < D; q++) cfma_cb(s, sb[a2 * D + q], ob[c2 * D + q]);
        acc = acc + twt[r * nm + mm - mlo] * s;
      } else {
#pragma unroll
        for (int q = 0; q < D; q++) cfma(s, sb[a2 * D + q], ob[q * D + c2]);
        acc = acc + twt[r * nm + mm - mlo] * s;
      }
    }
    stage[vv] = acc;
  }
  __syncthreads();
  for (int v = tid; v < NV; v += NTHR) {
    cplx sum = mk(0, 0);
    for (int g2 = 0; g2 < G2; g2++) sum = sum + stage[g2 * NV + v];
    cplx coef = fam == 1 ? mk(-ht, 0) : mk(0, -h);
    tpart[(size_t)b * NV + v] = coef * sum;
  }
  }  // n >= 2k+1
  }  // tiles
  if (n < 2 * k + 1) return;
  int npk = k * (k + 1) / 2;
  cplx* s_r = ser;  // Sigma^R_{m_r, n-k+jj}, jj < r, packed at r(r-1)/2 + jj
  cplx* s_l = s_r + npk * DD;  // L_{n-2k..n-k-1, n} (BDF of the first rows)
  cplx* s_b = s_l + k * DD;    // inverted boundary step matrices
  int nz = (k + 1) * (k + 2) / 2;  // blocks of the operator Z, packed at r(r+1)/2 + c
  cplx* zl = sigs;                 // Z in LDS
  static_assert((KMAX + 1) * (KMAX + 2) / 2 * DD <= (KMAX + 1) * TM * DD, "operator exceeds its LDS");
  if (walk || (int)blockIdx.x == nwg) {
    // The k+1 serial rows read X_r = B_r (b_r - sum_{jj<r} C_{r,jj} X_jj), with
    // B_r the inverted step matrix of row m_r, C_{r,jj} = (a_{r-jj}/h) 1 +
    // i h w(m_r, n-k+jj) Sigma^R_{m_r, n-k+jj}, and b_r their sources. Their
    // solution X = Z b with the block lower-triangular Z formed here, by
    // forward substitution over the block rows, while the tiles run:
    //   Z_{r,c} = B_r (delta_rc 1 - sum_{c <= jj < r} C_{r,jj} Z_{jj,c}).
    for (int idx = tid; idx < npk * DD; idx += NTHR) {
      int pr = idx / DD, ee = idx % DD, r = 1;
      while (r * (r + 1) / 2 <= pr) r++;
      int jj = pr - r * (r - 1) / 2;
      s_r[idx] = gld(P.Sret + (tri(n - k + r) + n - k + jj) * DD + ee);
    }
    for (int idx = tid; idx < (k + 1) * DD; idx += NTHR) s_b[idx] = gld(sc.minv(pi) + DD + idx);
    for (int v = tid; v < (k + 1) * (k + 1); v += NTHR) {
      int r = v / (k + 1), jj = v % (k + 1);
      s_gw[r * K1M + jj] = jj < r ? gw(n - k + r, n - k + jj) : 0.0;
    }
    __syncthreads();
    for (int r = 0; r <= k; r++) {
      for (int v = tid; v < (r + 1) * DD; v += NTHR) {
        int c = v / DD, e = v % DD, a2 = e / D, c2 = e % D;
        cplx t = (c == r && a2 == c2) ? mk(1, 0) : mk(0, 0);
        for (int jj = c; jj < r; jj++) {
          const cplx* zb = zl + (jj * (jj + 1) / 2 + c) * DD;
          const cplx* sb = s_r + (r * (r - 1) / 2 + jj) * DD + a2 * D;
          cplx sz = mk(0, 0);
          for (int q = 0; q < D; q++) cfma(sz, sb[q], zb[q * D + c2]);
          t = t - s_ah[r - jj] * zb[e] - mul_i((h * s_gw[r * K1M + jj]) * sz);
        }
        stage[v] = t;
      }
      __syncthreads();
      for (int v = tid; v < (r + 1) * DD; v += NTHR) {
        int c = v / DD, e = v % DD, a2 = e / D, c2 = e % D;
        cplx o = mk(0, 0);
        for (int q = 0; q < D; q++) cfma(o, s_b[r * DD + a2 * D + q], stage[c * DD + q * D + c2]);
        zl[(r * (r + 1) / 2 + c) * DD + e] = o;
      }
      __syncthreads();
    }
    if (!walk)
      for (int idx = tid; idx < nz * DD; idx += NTHR) gst(sc.zop(pi, DD) + idx, zl[idx]);
  }
  if (walk) {
    __syncthreads();  // this workgroup's own partials
  } else {
    // completion count (the tiles and the operator workgroup)
    if (!last_to_arrive(sc.counter(pi), nwg, is_last)) return;
  }
  // last workgroup. The operator Z and the earlier rows are loaded first
  // (into registers), then the partials of all workgroups are summed (G
  // groups per value); the loads of both overlap.
  constexpr int NSL = (KMAX * DD + NTHR - 1) / NTHR;
  constexpr int NSZ = ((KMAX + 1) * (KMAX + 2) / 2 * DD + NTHR - 1) / NTHR;
  cplx vl[NSL], vz[NSZ];
#pragma unroll
  for (int u = 0; u < NSZ; u++) {
    int idx = tid + u * NTHR;
    if (!walk && idx < nz * DD) vz[u] = gld(sc.zop(pi, DD) + idx);
  }
#pragma unroll
  for (int u = 0; u < NSL; u++) {
    int idx = tid + u * NTHR;
    if (idx < k * DD) vl[u] = gld(P.Gles + (tri(n) + n - 2 * k + idx / DD) * DD + idx % DD);
  }
  // (the retarded boundary sources of d <= 4 are loaded in the same round)
  constexpr int NSB = (NVMAX + NTHR - 1) / NTHR;
  cplx vb[NSB];
#pragma unroll
  for (int u = 0; u < NSB; u++) {
    int idx = tid + u * NTHR;
    if (D <= 4 && idx < NV) vb[u] = gld(sc.bsrc(pi, DD) + idx);
  }
  int G = NV >= NTHR ? 1 : NTHR / NV;
  for (int vv = tid; vv < G * NV; vv += NTHR) {
    int g = vv / NV, v = vv % NV;
    // workgroups g, g+G, g+2G, ... of value v (32 loads in flight: fewer
    // memory rounds over the tiles)
    stage[vv] = psum_b<32>(tpart + (size_t)g * NV + v, (long)G * NV, g < nwg ? (nwg - g + G - 1) / G : 0);
  }
#pragma unroll
  for (int u = 0; u < NSB; u++)
    if (D <= 4 && tid + u * NTHR < NV) pre[tid + u * NTHR] = vb[u];
#pragma unroll
  for (int u = 0; u < NSZ; u++)
    if (!walk && tid + u * NTHR < nz * DD) zl[tid + u * NTHR] = vz[u];
#pragma unroll
  for (int u = 0; u < NSL; u++)
    if (tid + u * NTHR < k * DD) s_l[tid + u * NTHR] = vl[u];
  __syncthreads();
  for (int v = tid; v < NV; v += NTHR) {
    int r = v / DD, ee = v % DD, a2 = ee / D, c2 = ee % D;
    int mr = n - k + r;
    cplx s = mk(0, 0);
    for (int g = 0; g < G; g++) s = s + stage[g * NV + v];
    if constexpr (D <= 4) {
      // the retarded boundary columns j = n-k..n were summed by the step set-up
      pre[v] = s + pre[v];
    } else {
      cplx pb = mk(0, 0);
#pragma unroll
      for (int jj = 0; jj <= KMAX; jj++) {
        if (jj <= k) {
          int j = n - k + jj;
          cplx t = mk(0, 0);
#pragma unroll
          for (int q = 0; q < D; q++)
            cfma_cb(t, les_any<D>(P.Sles, mr, j, a2, q), gld(P.Gret + (tri(n) + j) * DD + c2 * D + q));
          pb = pb + greg(W, n, j) * t;
        }
      }
      pre[v] = s - h * mul_i(pb);
    }
  }
  __syncthreads();
  // sources b_r: pre_r less the BDF terms of the rows before n-k; then X = Z b
  for (int v = tid; v < NV; v += NTHR) {
    int r = v / DD, ee = v % DD;
    cplx b = pre[v];
    for (int l = r + 1; l <= k; l++) b = b - s_ah[l] * s_l[(k + r - l) * DD + ee];
    stage[v] = b;
  }
  __syncthreads();
  cplx* const gles_b = P.Gles + (tri(n) + n - k) * DD;
  for (int v = tid; v < NV; v += NTHR) {
    int r = v / DD, ee = v % DD, a2 = ee / D, c2 = ee % D;
    cplx o = mk(0, 0);
    for (int c = 0; c <= r; c++) {
      const cplx* zb = zl + (r * (r + 1) / 2 + c) * DD + a2 * D;
      for (int q = 0; q < D; q++) cfma(o, zb[q], stage[c * DD + q * D + c2]);
    }
    gst(gles_b + v, o);
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
  bool ok = true;
  if (tid < 64) ok = wave_solve(N, D, A, B);  // one wavefront solves
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  __syncthreads();
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
    if (tid < 64) ok = wave_inverse(D, ml, piv);
    if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    __syncthreads();
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
    bool ok = true;
    if (tid < 64) ok = wave_solve(N, D, A, B);  // one wavefront solves
    if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
    __syncthreads();
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
  bool ok = true;
  if (tid < 64) ok = wave_solve(N, D, A, B);  // one wavefront solves
  if (!ok && tid == 0) atomicExch(sc.status(pi), CNTR_ESINGULAR);
  __syncthreads();
  for (int idx = tid; idx < k * DD; idx += NTHR) {
    int p = idx / DD + 1, e = idx % DD, a = e / D, c = e % D;
    P.Gtv[((size_t)p * (ntau + 1) + m) * DD + e] = B[((p - 1) * D + a) * D + c];
  }
}

// ------------------------------------------------------------ profiling
ProfState g_prof;

static hipEvent_t prof_event() {
  if (g_prof.used < g_prof.pool.size()) return g_prof.pool[g_prof.used++];
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  g_prof.pool.push_back(e);
  g_prof.used++;
  return e;
}

// algorithmic block multiply-adds of the history kernel at slice n
static double hist_block_macs(int n, int k, int ntau) {
  double macs = 0;
  for (int m = 0; m < n - k; m++) macs += n - m;          // retarded bulk
  macs += (double)n * (ntau + 1);                          // left-mixing history
  for (int m = 0; m <= ntau; m++) {                        // tau source (Gregory parts)
    if (m > k) macs += m + 1;
    if (m < ntau - k) macs += ntau - m + 1;
  }
  if (n >= 2 * k + 1)
    for (int m = 0; m < n - k; m++) macs += n + (m > k ? m : k) + 1 + ntau + 1;  // lesser bulk
  return macs;
}

// ----------------------------------- TAU SOURCE OF A SHARED SIGMA (d = 1)
// Batches whose problems share Sigma (k-points with a local self-energy):
// the tau source of every problem at once, out[m][p] = sum_v A[m][v]
// G^M_p[v], with one operator built from the slice's Sigma^rceil_{n,.}:
//   A[m][v] = xi w(m, ntau-v) Sigma^rceil_{n,m-ntau+v}   (m > k, ntau-v <= m)
//           + w(ntau-m, v) Sigma^rceil_{n,m+v}            (m < ntau-k, m+v <= ntau),
// the Gregory parts of Eqs. ctv2 and ctv3 with J = ntau - v and J = m + v.
// A workgroup computes 32 outputs m x 32 problems (2 x 2 per thread) over
// chunks of 32 v in LDS (the next chunk of G^M in flight while one is
// multiplied). The terms are split over TS_SPLIT workgroups; split z writes
// chunk z of the tau-source partials.
__global__ __launch_bounds__(NTHR) void k_tau_shared(ProbArg pa, Scratch sc, HistPlan pl) {
  __shared__ cplx s_row[TS_NTAU];
  __shared__ cplx sa[TSM][TSV + 1];
  __shared__ cplx sx[TSV][TSP + 1];
  __shared__ double s_om[KMAX + 1];
  __shared__ const cplx* s_gm[TSP];
  const Prob& P0 = pa.get(0);
  int n = pl.n, ntau = P0.ntau, k = P0.k, tid = threadIdx.x;
  int m0 = blockIdx.x * TSM, p0 = blockIdx.y * TSP;
  // this workgroup's share of the terms v (whole chunks of TSV)
  int nchunk = (ntau + TSV) / TSV, per = (nchunk + TS_SPLIT - 1) / TS_SPLIT;
  int vbeg = blockIdx.z * per * TSV, vend = min(ntau + 1, (int)(blockIdx.z + 1) * per * TSV);
  const KW& W = c_kw[k];
  WReg wr;
  wr.load(W, s_om);
  double xi = P0.sig;
  const cplx* Srow = P0.Stv + (size_t)n * (ntau + 1);
  for (int j = tid; j <= ntau; j += NTHR) s_row[j] = gld(Srow + j);
  if (tid < TSP) s_gm[tid] = pa.get(min(p0 + tid, pa.count - 1)).Gmat;
  __syncthreads();
  int tm = tid / 16, tp = tid % 16;
  cplx acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] = mk(0, 0);
  constexpr int NX = TSV * TSP / NTHR;  // G^M values per thread and chunk
  cplx xn[NX];
  auto load_x = [&](int v0) {
#pragma unroll
    for (int u = 0; u < NX; u++) {
      int i = tid + u * NTHR, vv = i / TSP, pp = i % TSP, v = v0 + vv;
      xn[u] = v <= ntau ? gld(s_gm[pp] + v) : mk(0, 0);
    }
  };
  if (vbeg < vend) load_x(vbeg);
  for (int v0 = vbeg; v0 < vend; v0 += TSV) {
    // operator tile A[m0 .. m0+31][v0 .. v0+31]
    for (int i = tid; i < TSM * TSV; i += NTHR) {
      int mm = i / TSV, vv = i % TSV, m = m0 + mm, v = v0 + vv;
      cplx a = mk(0, 0);
      if (m <= ntau && v <= ntau) {
        int J = ntau - v;
        if (m > k && J <= m) a = a + (xi * wr.w(m, J)) * s_row[m - J];
        if (m < ntau - k && m + v <= ntau) a = a + wr.w(ntau - m, v) * s_row[m + v];
      }
      sa[mm][vv] = a;
    }
#pragma unroll
    for (int u = 0; u < NX; u++) {
      int i = tid + u * NTHR;
      sx[i / TSP][i % TSP] = xn[u];
    }
    __syncthreads();
    if (v0 + TSV < vend) load_x(v0 + TSV);
#pragma unroll 8
    for (int vv = 0; vv < TSV; vv++) {
      cplx a0 = sa[2 * tm][vv], a1 = sa[2 * tm + 1][vv];
      cplx x0 = sx[vv][2 * tp], x1 = sx[vv][2 * tp + 1];
      cfma(acc[0][0], a0, x0);
      cfma(acc[0][1], a0, x1);
      cfma(acc[1][0], a1, x0);
      cfma(acc[1][1], a1, x1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) {
      int m = m0 + 2 * tm + i, p = p0 + 2 * tp + j;
      if (m <= ntau && p < pa.count && n <= pa.get(p).nt)
        gst(sc.part(p) + pl.part_off[2] + (size_t)blockIdx.z * (ntau + 1) + m, acc[i][j]);
    }
}

// ------------------------------------------------------------ side streams
// One side stream (default priority, non-blocking) and a fork / join event
// pair per (device, stream) of the caller, created on first use and kept
// until the process ends.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
static SideStream* side_stream(hipStream_t main) {
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, SideStream> tab;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  SideStream& x = tab[{dev, main}];
  if (!x.s) {
    if (hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) != hipSuccess) {
      x.s = nullptr;
      return nullptr;
    }
    if (hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&x.join, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(x.s);
      x = SideStream{};
      return nullptr;
    }
  }
  return &x;
}

// ------------------------------------------------------------ launches
template <int D>
static hipError_t step_d(const ProbArg& pa, const Scratch& sc, int n, hipStream_t s, bool shared_sigma,
                         bool record) {
  const Prob& P0 = pa.one;  // d, k and ntau are uniform within a call
  int k = P0.k, ntau = P0.ntau;
  HistPlan pl = make_plan(n, k, ntau, D);
  // one operator for the whole batch: d = 1, Sigma shared, enough problems
  // for the product to pay
  if (D == 1 && shared_sigma && pa.count >= TSP && ntau + 1 <= TS_NTAU) {
    pl = make_plan(n, k, ntau, D, TS_SPLIT);
    pl.tau_shared = 1;
    dim3 gt((ntau + TSM) / TSM, (pa.count + TSP - 1) / TSP, TS_SPLIT);
    k_tau_shared<<<gt, NTHR, 0, s>>>(pa, sc, pl);
  }
  dim3 g1(pl.grid + 1, pa.count);
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  bool rec = record && g_prof.on && g_prof.seen++ % g_prof.every == 0;
  if (rec) {
    e0 = prof_event();
    e1 = prof_event();
    e2 = prof_event();
    if (e0) (void)hipEventRecord(e0, s);
  }
  // d = 8: the set-up kernel runs beside the history sums, on a side stream
  // forked from s and joined before the reduction (serially on s when the
  // caller creates no runtime objects or captures a graph)
  SideStream* side = nullptr;
  if constexpr (D == 8) {
    side = record ? side_stream(s) : nullptr;
    if (side) {
      (void)hipEventRecord(side->fork, s);
      (void)hipStreamWaitEvent(side->s, side->fork, 0);
      k_prep<D><<<dim3(1, pa.count), NTHR, 0, side->s>>>(pa, sc, n);
      (void)hipEventRecord(side->join, side->s);
    } else {
      k_prep<D><<<dim3(1, pa.count), NTHR, 0, s>>>(pa, sc, n);
    }
  }
  k_history<D><<<g1, NTHR, 0, s>>>(pa, sc, pl);
  if (side) (void)hipStreamWaitEvent(s, side->join, 0);
  if (rec && e1) {
    (void)hipEventRecord(e1, s);
    double dd = (double)D * D;
    double blocks = (double)n * (n + 1) / 2 + (double)n * (ntau + 1) + (n >= 2 * k + 1 ? (double)n * (n + 1) / 2 : 0);
    g_prof.rec.push_back({e0, e1, e2, 16.0 * dd * blocks * pa.count,
                          8.0 * dd * D * hist_block_macs(n, k, ntau) * pa.count});
  }
  pl.walk_tiles = pa.count >= REDUCE_WALK_MIN;
  // (one more workgroup forms the boundary-row operator when there are rows)
  int ntile = pl.red_tiles[0] + pl.red_tiles[1] + pl.red_tiles[2];
  dim3 g2(pl.walk_tiles ? 1 : ntile + (pl.red_tiles[2] > 0 ? 1 : 0), pa.count);
  k_reduce<D><<<g2, NTHR, 0, s>>>(pa, sc, pl);
  if (n < 2 * k + 1) {
    dim3 g4(1, pa.count);
    k_column<D><<<g4, NTHR, 0, s>>>(pa, sc, n);
  }
  if (rec && e2) (void)hipEventRecord(e2, s);
  return hipGetLastError();
}

hipError_t launch_step(const ProbArg& pa, const Scratch& sc, int n, int d, hipStream_t s, bool shared_sigma,
                       bool record) {
  switch (d) {
    case 1: return step_d<1>(pa, sc, n, s, shared_sigma, record);
    case 2: return step_d<2>(pa, sc, n, s, shared_sigma, record);
    case 3: return step_d<3>(pa, sc, n, s, shared_sigma, record);
    case 4: return step_d<4>(pa, sc, n, s, shared_sigma, record);
    case 5: return step_d<5>(pa, sc, n, s, shared_sigma, record);
    case 6: return step_d<6>(pa, sc, n, s, shared_sigma, record);
    case 7: return step_d<7>(pa, sc, n, s, shared_sigma, record);
    case 8: return step_d<8>(pa, sc, n, s, shared_sigma, record);
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
