// Momentum-convolution self-energies of the k-space GW example (Sec.
// "Example: GW for the translationally invariant Hubbard model") on gfx950,
// for Nk momenta (indices mod Nk), element by element in the orbitals:
//   polarization  Pi_k    = -(1/Nk) sum_q Bubble1(G_{k+q}, G_q)    (Eq. Pol)
//   self-energy   Sigma_k =  (1/Nk) sum_q Bubble2(G_{k-q}, dW_q)   (Eq. Sigmak)
// with Bubble1: C(t,t') = i A(t,t') B(t',t), C_ij from A_ij and B_ji, and
// Bubble2: C(t,t') = i A(t,t') B(t,t') (Eqs. def_bubble1, def_bubble2), on
// the stored components of one time slice (tstp = -1: Matsubara). The same
// product without a momentum sum (C_i = i A_i B_i for independent instances)
// is k_bubble2_local at the end of the file.
//
// A workgroup takes a tile of TJ consecutive stored elements of one
// component (flat index over (time or tau index, orbital pair), contiguous in
// memory for every momentum) and KC consecutive output momenta k. The terms q
// run in chunks of QC: per chunk the first factor's values over the window of
// momenta k + q (or k - q) and the second factor's over q are staged in LDS,
// sixteen lanes loading sixteen consecutive elements of one momentum, so a
// wave's load touches four momenta's pages rather than sixty-four. Each
// thread owns R consecutive outputs k of one element and keeps the first
// factor's R window values in registers, shifting in one value per term; the
// terms of each output are accumulated with fused multiply-adds in order
// q = 0 .. Nk-1 (the second product of a two-term rule in a sum of its own,
// added at the end).
#include "launch.h"

namespace cntr {

constexpr int NKB = 256;           // threads per workgroup
constexpr int KB_TJ = 16;          // elements per tile
constexpr int KB_R = 4;            // outputs per thread
constexpr int KB_KC = KB_R * (NKB / KB_TJ);  // output momenta per workgroup (64)
constexpr int KB_QC = 32;          // terms per staged chunk
constexpr int KB_XW = KB_KC + KB_QC;         // window of first-factor momenta

// Langreth rules on element (comp, j, a, c) of slice n (the Matsubara rules
// from X^M(tau) = -i X(-i tau, 0), the form in which X^rceil(0, tau) =
// i xi X^M(beta - tau)). Bubble1 with
// A = G_{k+q}, B = G_q:
//   R (n, m):  i A^R(n,m)[a][c] B^<(m,n)[c][a] + i A^<(n,m)[a][c] B^A(m,n)[c][a],
//              B^A(m,n)[c][a] = conj(B^R(n,m)[a][c])
//   < (m, n):  i A^<(m,n)[a][c] B^>(n,m)[c][a],  B^> = B^R + B^<
//   rceil:     i A^rceil(n,m)[a][c] B^lceil(m,n)[c][a],  B^lceil(m,n) = -xi conj(B^rceil(n,ntau-m))
//   M (m):     -xi A^M(m)[a][c] B^M(ntau-m)[c][a]
// Bubble2 with A = G_{k-q}, B = dW_q, element [a][c] of each factor:
//   R:   i [A^R B^R + A^<(n,m) B^R + A^R B^<(n,m)]
//   <:   i A^< B^<;  rceil: i A^rceil B^rceil;  M: -A^M B^M
// A lesser value below the stored triangle, X^<(n,m) with m < n, is
// -conj(L_{m,n}) transposed; at m = n the stored L_{n,n} itself is used (a
// computed G^<(t,t) is anti-hermitian only up to the solver's error).

// Base pointers of one momentum's components: a = ret, b = les (components
// R and <), a = tv (rceil) or a = mat (M).
struct KPtr {
  cplx *a, *b;
};

// The momenta's base pointers, read once per workgroup from the descriptor
// array (global loads: a flat load of a descriptor field would be ordered
// behind LDS stores) into an LDS table tab[0..nk) (a) and tab[nk..2nk) (b).
template <int COMP>
__device__ inline void kb_ptab(cplx** tab, const Prob* arr, int nk, int tid) {
  for (int p = tid; p < nk; p += NKB) {
    const Prob* P = arr + p;
    if (COMP == 3) {
      tab[p] = gld(&P->Gmat);
    } else if (COMP == 2) {
      tab[p] = gld(&P->Gtv);
    } else {
      tab[p] = gld(&P->Gret);
      tab[nk + p] = gld(&P->Gles);
    }
  }
}
template <int COMP>
__device__ inline KPtr kptr(cplx* const* tab, int nk, int p) {
  return KPtr{tab[p], COMP <= 1 ? tab[nk + p] : nullptr};
}

// X^<(t_n, t_m)[a][c] for m <= n from the stored lesser column n: below the
// diagonal -conj(L_{m,n}[c][a]), at m = n the stored value
__device__ inline cplx les_below(const cplx* les, int d, int n, int m, int a, int c) {
  bool diag = m == n;
  cplx v = gld(les + (tri(n) + m) * d * d + (diag ? a * d + c : c * d + a));
  return diag ? v : mk(-v.x, v.y);
}

// The staged operands of one element: the term of output k and term q is
// xa(k +- q) ya(q) [+ xb(k +- q) yb(q)], the leading factor i, the sign xi
// of Bubble1's mixing and Matsubara rules and the conjugations folded in here.
//   Bubble1  R:  xa = A^R,  xb = A^<(n,m);  ya = B^<(m,n)^T,  yb = conj(B^R)   [B^A(m,n)^T]
//            <:  xa = A^<;  ya = (B^R + B^<(n,m))^T
//            rceil: xa = A^rceil;  ya = -xi conj(B^rceil(n, ntau-m))
//            M:  xa = A^M;  ya = -xi B^M(ntau-m)^T
//   Bubble2  R:  xa = A^R + A^<(n,m),  xb = A^R;  ya = B^R,  yb = B^<(n,m)
//            <, rceil:  xa = A,  ya = B  (same component);  M:  xa = A^M,  ya = -B^M
template <int MODE, int COMP>
__device__ inline void kb_first(const KPtr& P, int d, int ntau, int n, int j, int a, int c, cplx& xa, cplx& xb) {
  int dd = d * d;
  if (COMP == 3) {
    xa = gld(P.a + (size_t)j * dd + a * d + c);
  } else if (COMP == 2) {
    xa = gld(P.a + ((size_t)n * (ntau + 1) + j) * dd + a * d + c);
  } else if (COMP == 1) {
    xa = gld(P.b + (tri(n) + j) * dd + a * d + c);
  } else {
    cplx r = gld(P.a + (tri(n) + j) * dd + a * d + c);
    cplx l = les_below(P.b, d, n, j, a, c);
    if (MODE == 1) {
      xa = r;
      xb = l;
    } else {
      xa = r + l;
      xb = r;
    }
  }
}

template <int MODE, int COMP>
__device__ inline void kb_second(const KPtr& P, int d, int ntau, int n, int j, int a, int c, double xi, cplx& ya,
                                 cplx& yb) {
  int dd = d * d;
  if (MODE == 2) {
    if (COMP == 3) ya = -gld(P.a + (size_t)j * dd + a * d + c);
    else if (COMP == 2) ya = gld(P.a + ((size_t)n * (ntau + 1) + j) * dd + a * d + c);
    else if (COMP == 1) ya = gld(P.b + (tri(n) + j) * dd + a * d + c);
    else {
      ya = gld(P.a + (tri(n) + j) * dd + a * d + c);
      yb = les_below(P.b, d, n, j, a, c);
    }
    return;
  }
  if (COMP == 3) {
    ya = (-xi) * gld(P.a + (size_t)(ntau - j) * dd + c * d + a);
  } else if (COMP == 2) {
    ya = (-xi) * conj(gld(P.a + ((size_t)n * (ntau + 1) + ntau - j) * dd + a * d + c));
  } else if (COMP == 1) {
    ya = gld(P.a + (tri(n) + j) * dd + c * d + a) + les_below(P.b, d, n, j, c, a);
  } else {
    ya = gld(P.b + (tri(n) + j) * dd + c * d + a);
    yb = conj(gld(P.a + (tri(n) + j) * dd + a * d + c));
  }
}

__device__ inline int kmod(int v, int nk) {
  v %= nk;
  return v < 0 ? v + nk : v;
}

// The QC terms of a staged chunk for the thread's R outputs, unrolled at
// compile time (the window shifts are register renames). Terms past the last
// momentum are staged with a zero second factor and add exact zeros. The
// second product of a two-term rule goes to its own sum (accb), added to the
// first at the end.
template <int MODE, bool TWO>
__device__ inline void kb_chunk(const cplx (*xs)[KB_XW][KB_TJ], const cplx (*ys)[KB_QC][KB_TJ], int kl, int jj,
                                cplx* acc, cplx* accb) {
  // first-factor window of the thread's R outputs at the chunk's first term
  cplx xa[KB_R], xb[KB_R];
#pragma unroll
  for (int r = 0; r < KB_R; r++) {
    int w = MODE == 1 ? kl + r : kl + r + KB_QC - 1;
    xa[r] = xs[0][w][jj];
    if (TWO) xb[r] = xs[1][w][jj];
  }
#pragma unroll
  for (int qq = 0; qq < KB_QC; qq++) {
    cplx ya = ys[0][qq][jj];
    cplx yb = TWO ? ys[1][qq][jj] : mk(0, 0);
#pragma unroll
    for (int r = 0; r < KB_R; r++) {
      cfma(acc[r], xa[r], ya);
      if (TWO) cfma(accb[r], xb[r], yb);
    }
    if (qq + 1 < KB_QC) {
      if (MODE == 1) {  // window k + q moves up by one
#pragma unroll
        for (int r = 0; r < KB_R - 1; r++) {
          xa[r] = xa[r + 1];
          if (TWO) xb[r] = xb[r + 1];
        }
        int w = kl + KB_R + qq;
        xa[KB_R - 1] = xs[0][w][jj];
        if (TWO) xb[KB_R - 1] = xs[1][w][jj];
      } else {  // window k - q moves down by one
#pragma unroll
        for (int r = KB_R - 1; r > 0; r--) {
          xa[r] = xa[r - 1];
          if (TWO) xb[r] = xb[r - 1];
        }
        int w = kl + KB_QC - 2 - qq;
        xa[0] = xs[0][w][jj];
        if (TWO) xb[0] = xs[1][w][jj];
      }
    }
  }
}

constexpr int KB_NX = KB_XW * KB_TJ / NKB;  // staged first-factor values per thread (6)
constexpr int KB_NY = KB_QC * KB_TJ / NKB;  // staged second-factor values per thread (2)
static_assert(KB_NX * NKB == KB_XW * KB_TJ && KB_NY * NKB == KB_QC * KB_TJ, "staging split");

// one chunk's staged values, held in registers between the loads and the
// LDS stores (the next chunk's loads are in flight while the current one is
// summed)
struct KStage {
  cplx xa[KB_NX], xb[KB_NX], ya[KB_NY], yb[KB_NY];
};

// Loads of one chunk without branches: every base pointer first, then every
// value; an element past the component's end reads the last element and is
// staged as zero, a term past the last momentum reads momentum 0 and is
// staged as zero.
template <int MODE, int COMP>
__device__ inline void kb_load(KStage& S, cplx* const* first, cplx* const* second, int nk, int d, int ntau, int n,
                               int cnt, int idx0, int k0, int q0, double xi, int tid) {
  const int dd = d * d;
  const int xb0 = MODE == 1 ? k0 + q0 : k0 - q0 - (KB_QC - 1);
  KPtr px[KB_NX], py[KB_NY];
#pragma unroll
  for (int u = 0; u < KB_NX; u++) px[u] = kptr<COMP>(first, nk, kmod(xb0 + (tid + u * NKB) / KB_TJ, nk));
#pragma unroll
  for (int u = 0; u < KB_NY; u++) {
    int q = q0 + (tid + u * NKB) / KB_TJ;
    py[u] = kptr<COMP>(second, nk, q < nk ? q : 0);
  }
#pragma unroll
  for (int u = 0; u < KB_NX; u++) {
    int idx = idx0 + (tid + u * NKB) % KB_TJ;
    bool ok = idx < cnt;
    idx = ok ? idx : cnt - 1;
    int j = idx / dd, e = idx - j * dd;
    cplx va, vb = mk(0, 0);
    kb_first<MODE, COMP>(px[u], d, ntau, n, j, e / d, e % d, va, vb);
    S.xa[u] = ok ? va : mk(0, 0);
    S.xb[u] = ok ? vb : mk(0, 0);
  }
#pragma unroll
  for (int u = 0; u < KB_NY; u++) {
    int i = tid + u * NKB, idx = idx0 + i % KB_TJ;
    bool ok = idx < cnt && q0 + i / KB_TJ < nk;
    idx = idx < cnt ? idx : cnt - 1;
    int j = idx / dd, e = idx - j * dd;
    cplx va, vb = mk(0, 0);
    kb_second<MODE, COMP>(py[u], d, ntau, n, j, e / d, e % d, xi, va, vb);
    S.ya[u] = ok ? va : mk(0, 0);
    S.yb[u] = ok ? vb : mk(0, 0);
  }
}

template <bool TWO>
__device__ inline void kb_store(const KStage& S, cplx (*xs)[KB_XW][KB_TJ], cplx (*ys)[KB_QC][KB_TJ], int tid) {
#pragma unroll
  for (int u = 0; u < KB_NX; u++) {
    int i = tid + u * NKB;
    xs[0][i / KB_TJ][i % KB_TJ] = S.xa[u];
    if (TWO) xs[1][i / KB_TJ][i % KB_TJ] = S.xb[u];
  }
#pragma unroll
  for (int u = 0; u < KB_NY; u++) {
    int i = tid + u * NKB;
    ys[0][i / KB_TJ][i % KB_TJ] = S.ya[u];
    if (TWO) ys[1][i / KB_TJ][i % KB_TJ] = S.yb[u];
  }
}

template <int MODE, int COMP>
__device__ inline void kb_body(cplx (*xs)[KB_XW][KB_TJ], cplx (*ys)[KB_QC][KB_TJ], cplx** tab, const Prob* first,
                               const Prob* second, const Prob* out, int nk, int d, int ntau, int n, int cnt, int tile,
                               double xi, double alpha) {
  constexpr bool TWO = COMP == 0;
  const int tid = threadIdx.x, dd = d * d;
  const int k0 = blockIdx.y * KB_KC, idx0 = tile * KB_TJ;
  const int jj = tid % KB_TJ, kl = (tid / KB_TJ) * KB_R;
  cplx** tf = tab;
  cplx** ts = MODE == 1 ? tab : tab + 2 * nk;
  kb_ptab<COMP>(tf, first, nk, tid);
  if (MODE == 2) kb_ptab<COMP>(ts, second, nk, tid);
  __syncthreads();
  cplx acc[KB_R], accb[KB_R];
#pragma unroll
  for (int r = 0; r < KB_R; r++) acc[r] = accb[r] = mk(0, 0);
  KStage S;
  kb_load<MODE, COMP>(S, tf, ts, nk, d, ntau, n, cnt, idx0, k0, 0, xi, tid);
  for (int q0 = 0; q0 < nk; q0 += KB_QC) {
    kb_store<TWO>(S, xs, ys, tid);
    __syncthreads();
    if (q0 + KB_QC < nk) kb_load<MODE, COMP>(S, tf, ts, nk, d, ntau, n, cnt, idx0, k0, q0 + KB_QC, xi, tid);
    kb_chunk<MODE, TWO>(xs, ys, kl, jj, acc, accb);
    __syncthreads();
  }
  const int idx = idx0 + jj;
  if (idx >= cnt) return;
  const int j = idx / dd, e = idx - j * dd;
  const double scale = alpha * (MODE == 1 ? -1.0 : 1.0) / nk;
#pragma unroll
  for (int r = 0; r < KB_R; r++) {
    int k = k0 + kl + r;
    if (k >= nk) break;
    const Prob* O = out + k;
    cplx a = TWO ? acc[r] + accb[r] : acc[r];
    cplx v = COMP == 3 ? a : mul_i(a);
    cplx* dst;
    if (COMP == 3) dst = gld(&O->Gmat) + (size_t)j * dd + e;
    else if (COMP == 0) dst = gld(&O->Gret) + (tri(n) + j) * dd + e;
    else if (COMP == 1) dst = gld(&O->Gles) + (tri(n) + j) * dd + e;
    else dst = gld(&O->Gtv) + ((size_t)n * (ntau + 1) + j) * dd + e;
    gst(dst, scale * v);
  }
}

// grid: x = element tiles of the slice's components in order (R, <, rceil;
// or M), y = chunks of KC output momenta. first/second/out: the descriptor
// arrays of the two factors and of the output (nk each, sharing one grid).
template <int MODE>
__global__ __launch_bounds__(NKB) void k_kbubble(const Prob* first, const Prob* second, const Prob* out, int nk,
                                                 int d, int ntau, int sig, int n, int tiles_r, int tiles_t,
                                                 double alpha) {
  __shared__ cplx xs[2][KB_XW][KB_TJ];
  __shared__ cplx ys[2][KB_QC][KB_TJ];
  extern __shared__ cplx* kb_tab[];  // base pointers: 2 nk (Bubble1) or 4 nk (Bubble2)
  const int dd = d * d;
  const double xi = sig >= 0 ? 1.0 : -1.0;
  int tile = blockIdx.x;
  if (n == -1) {
    kb_body<MODE, 3>(xs, ys, kb_tab, first, second, out, nk, d, ntau, n, (ntau + 1) * dd, tile, xi, alpha);
  } else if (tile < tiles_r) {
    kb_body<MODE, 0>(xs, ys, kb_tab, first, second, out, nk, d, ntau, n, (n + 1) * dd, tile, xi, alpha);
  } else if (tile < 2 * tiles_r) {
    kb_body<MODE, 1>(xs, ys, kb_tab, first, second, out, nk, d, ntau, n, (n + 1) * dd, tile - tiles_r, xi, alpha);
  } else if (tile - 2 * tiles_r < tiles_t) {
    kb_body<MODE, 2>(xs, ys, kb_tab, first, second, out, nk, d, ntau, n, (ntau + 1) * dd, tile - 2 * tiles_r, xi, alpha);
  }
}

// C_i = alpha i A_i B_i element by element for independent instances (the
// local Bubble2, no momentum sum): one thread per stored element of slice n,
// grid y = instance
__global__ __launch_bounds__(NKB) void k_bubble2_local(ProbArg pa, ProbArg pb, ProbArg pc, int n, double alpha) {
  const Prob& A = pa.get(blockIdx.y);
  const Prob& B = pb.get(blockIdx.y);
  const Prob& C = pc.get(blockIdx.y);
  const int d = C.d, dd = d * d, ntau = C.ntau;
  const long idx = (long)blockIdx.x * NKB + threadIdx.x;
  const long bl = idx / dd;
  const int e = (int)(idx % dd), a = e / d, c = e % d;
  if (n == -1) {
    if (bl > ntau) return;
    size_t o = (size_t)bl * dd + e;
    gst(C.Gmat + o, (-alpha) * (gld(A.Gmat + o) * gld(B.Gmat + o)));
    return;
  }
  cplx v;
  cplx* dst;
  if (bl <= n) {  // R(n, m), m = bl
    int m = (int)bl;
    size_t o = (tri(n) + m) * dd + e;
    cplx ra = gld(A.Gret + o), rb = gld(B.Gret + o);
    cplx la = les_below(A.Gles, d, n, m, a, c), lb = les_below(B.Gles, d, n, m, a, c);
    v = mul_i((ra + la) * rb + ra * lb);
    dst = C.Gret + o;
  } else if (bl <= 2 * (long)n + 1) {  // L(m, n)
    size_t o = (tri(n) + (bl - n - 1)) * dd + e;
    v = mul_i(gld(A.Gles + o) * gld(B.Gles + o));
    dst = C.Gles + o;
  } else {  // T(n, m)
    long m = bl - 2 * (long)n - 2;
    if (m > ntau) return;
    size_t o = ((size_t)n * (ntau + 1) + m) * dd + e;
    v = mul_i(gld(A.Gtv + o) * gld(B.Gtv + o));
    dst = C.Gtv + o;
  }
  gst(dst, alpha * v);
}

hipError_t launch_bubble2_local(const ProbArg& pa, const ProbArg& pb, const ProbArg& pc, int n, int d, int ntau,
                                double alpha, hipStream_t s) {
  long nel = (n == -1 ? (long)(ntau + 1) : (long)(2 * (n + 1) + ntau + 1)) * d * d;
  dim3 g((unsigned)((nel + NKB - 1) / NKB), (unsigned)pc.count);
  k_bubble2_local<<<g, NKB, 0, s>>>(pa, pb, pc, n, alpha);
  return hipGetLastError();
}

hipError_t launch_kbubble(int mode, const Prob* pg, const Prob* pw, const Prob* po, int nk, int d, int ntau,
                          int sig, int n, double alpha, hipStream_t s) {
  int dd = d * d;
  int tiles_r = n == -1 ? 0 : ((n + 1) * dd + KB_TJ - 1) / KB_TJ;
  int tiles_t = ((ntau + 1) * dd + KB_TJ - 1) / KB_TJ;
  int tiles = n == -1 ? tiles_t : 2 * tiles_r + tiles_t;
  dim3 g((unsigned)tiles, (unsigned)((nk + KB_KC - 1) / KB_KC));
  size_t tab = (size_t)(mode == 1 ? 2 : 4) * nk * sizeof(cplx*);
  if (mode == 1) k_kbubble<1><<<g, NKB, tab, s>>>(pg, pg, po, nk, d, ntau, sig, n, tiles_r, tiles_t, alpha);
  else k_kbubble<2><<<g, NKB, tab, s>>>(pg, pw, po, nk, d, ntau, sig, n, tiles_r, tiles_t, alpha);
  return hipGetLastError();
}

}  // namespace cntr
