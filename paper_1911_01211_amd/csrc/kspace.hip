// Momentum-convolution self-energies of the k-space GW example (Sec.
// "Example: GW for the translationally invariant Hubbard model") on gfx950,
// for Nk momenta (indices mod Nk), element by element in the orbitals:
//   polarization  Pi_k    = -(1/Nk) sum_q Bubble1(G_{k+q}, G_q)    (Eq. Pol)
//   self-energy   Sigma_k =  (1/Nk) sum_q Bubble2(G_{k-q}, dW_q)   (Eq. Sigmak)
// with Bubble1: C(t,t') = i A(t,t') B(t',t), C_ij from A_ij and B_ji, and
// Bubble2: C(t,t') = i A(t,t') B(t,t') (Eqs. def_bubble1, def_bubble2), on
// the stored components of one time slice (tstp = -1: Matsubara).
//
// One workgroup per stored element of the slice (component, time or tau
// index, orbital pair): its threads stage, for every momentum p, the two or
// four values of G_p (and dW_p) that the element's Langreth rule needs into
// LDS, then each thread forms the momentum sums of its outputs k from LDS
// (term q in order, no reassociation) and writes alpha times Pi_k or Sigma_k.
#include "launch.h"

namespace cntr {

constexpr int NKB = 256;  // threads per workgroup

// Bubble1 on element (comp, j, a, c) of slice n with A = G_{k+q}, B = G_q:
//   R (n, m):  i A^R_{n,m}[a][c] B^<(m,n)[c][a] + i A^<(n,m)[a][c] B^A(m,n)[c][a],
//              B^A(m,n)[c][a] = conj(R_{n,m}[a][c]);
//              planes: 0 = R_{n,m}[a][c], 1 = L_{m,n}[c][a], 2 = A^<(n,m)[a][c]
//   < (m, n):  i A^<_{m,n}[a][c] B^>(n,m)[c][a],  B^> = R + B^<;
//              planes: 0 = L_{m,n}[a][c], 1 = R_{n,m}[c][a], 2 = B^<(n,m)[c][a]
//   rceil:     i A^rceil_{n,m}[a][c] B^lceil(m,n)[c][a],  B^lceil = -xi conj(T_{n,ntau-m}[a][c]);
//              planes: 0 = T_{n,m}[a][c], 1 = T_{n,ntau-m}[a][c]
//   M (m):     A^M_m[a][c] xi B^M_{ntau-m}[c][a];  planes: 0 = M_m[a][c], 1 = M_{ntau-m}[c][a]
// Bubble2 with A = G_{k-q}, B = dW_q:
//   R:   i [A^R B^R + A^<(n,m) B^R + A^R B^<(n,m)];
//        planes of each factor: R_{n,m}[a][c], X^<(n,m)[a][c]
//   <:   i A^<_{m,n} B^<_{m,n};  rceil: i A^rceil B^rceil;  M: A^M B^M  (element [a][c] of each)
// A lesser value below the stored triangle, X^<(n,m) with m < n, is
// -conj(L_{m,n}) transposed; at m = n the stored L_{n,n} itself is used (a
// computed G^<(t,t) is anti-hermitian only up to the solver's error).

// X^<(t_n, t_m)[a][c] for m <= n from the stored lesser column n
__device__ inline cplx les_below(const Prob& P, int n, int m, int a, int c) {
  int d = P.d, dd = d * d;
  if (m == n) return gld(P.Gles + (tri(n) + m) * dd + a * d + c);
  cplx v = gld(P.Gles + (tri(n) + m) * dd + c * d + a);
  return mk(-v.x, v.y);
}

__device__ inline cplx kval(const Prob& P, int mode, int comp, int n, int j, int a, int c, int plane) {
  int d = P.d, dd = d * d, ntau = P.ntau;
  if (comp == 3) {  // Matsubara
    if (mode == 1 && plane == 1) return gld(P.Gmat + (size_t)(ntau - j) * dd + c * d + a);
    return gld(P.Gmat + (size_t)j * dd + a * d + c);
  }
  if (comp == 2) {  // rceil
    int m = (mode == 1 && plane == 1) ? ntau - j : j;
    return gld(P.Gtv + ((size_t)n * (ntau + 1) + m) * dd + a * d + c);
  }
  if (comp == 0) {  // R row n, position m = j
    if (plane == 0) return gld(P.Gret + (tri(n) + j) * dd + a * d + c);
    if (mode == 1 && plane == 1) return gld(P.Gles + (tri(n) + j) * dd + c * d + a);
    return les_below(P, n, j, a, c);
  }
  // lesser column n, row m = j
  if (mode == 1) {
    if (plane == 0) return gld(P.Gles + (tri(n) + j) * dd + a * d + c);
    if (plane == 1) return gld(P.Gret + (tri(n) + j) * dd + c * d + a);
    return les_below(P, n, j, c, a);
  }
  return gld(P.Gles + (tri(n) + j) * dd + a * d + c);
}

template <int MODE>
__global__ __launch_bounds__(NKB) void k_kbubble(ProbArg pg, ProbArg pw, ProbArg po, int n, long nelem, double alpha) {
  constexpr int NKMAX = 1024;
  __shared__ cplx lv[4][NKMAX];
  const Prob& P0 = po.get(0);
  int nk = pg.count, d = P0.d, dd = d * d, ntau = P0.ntau, tid = threadIdx.x;
  long idx = blockIdx.x;
  if (idx >= nelem) return;
  // the element: component, time or tau index, orbital pair
  int comp, j, e;
  if (n == -1) {
    comp = 3;
    j = (int)(idx / dd);
    e = (int)(idx % dd);
  } else {
    long nr = (long)(n + 1) * dd;
    if (idx < nr) {
      comp = 0;
    } else if (idx < 2 * nr) {
      comp = 1;
      idx -= nr;
    } else {
      comp = 2;
      idx -= 2 * nr;
    }
    j = (int)(idx / dd);
    e = (int)(idx % dd);
  }
  int a = e / d, c = e % d;
  // statistics of G (the second factor of Bubble1)
  double xiG = pg.get(0).sig >= 0 ? 1.0 : -1.0;
  // the G planes (Bubble1: both factors; Bubble2: the first) and dW's planes
  for (int p = tid; p < nk; p += NKB) {
    const Prob& G = pg.get(p);
    lv[0][p] = kval(G, MODE, comp, n, j, a, c, 0);
    if (MODE == 1 || comp == 0) lv[1][p] = kval(G, MODE, comp, n, j, a, c, 1);
    if (MODE == 1 && comp <= 1) lv[2][p] = kval(G, MODE, comp, n, j, a, c, 2);
    if (MODE == 2) {
      const Prob& Wq = pw.get(p);
      lv[2][p] = kval(Wq, MODE, comp, n, j, a, c, 0);
      if (comp == 0) lv[3][p] = kval(Wq, MODE, comp, n, j, a, c, 1);
    }
  }
  __syncthreads();
  double scale = alpha * (MODE == 1 ? -1.0 : 1.0) / nk;
  for (int k = tid; k < nk; k += NKB) {
    cplx acc = mk(0, 0);
    int pa = k;  // momentum of the first factor: k + q (MODE 1) or k - q (MODE 2)
    for (int q = 0; q < nk; q++) {
      cplx t;
      if (MODE == 1) {
        cplx x0 = lv[0][pa], y0 = lv[0][q];
        if (comp == 0) {
          cplx x2 = lv[2][pa], y1 = lv[1][q];
          // i [A^R B^< + A^< B^A]
          t = mul_i(x0 * y1 + x2 * conj(y0));
        } else if (comp == 1) {
          cplx y1 = lv[1][q], y2 = lv[2][q];
          t = mul_i(x0 * (y1 + y2));
        } else if (comp == 2) {
          cplx y1 = lv[1][q];
          t = mul_i(x0 * ((-xiG) * conj(y1)));
        } else {
          cplx y1 = lv[1][q];
          t = xiG * (x0 * y1);
        }
        pa = pa + 1 == nk ? 0 : pa + 1;
      } else {
        cplx x0 = lv[0][pa], y0 = lv[2][q];
        if (comp == 0) {
          cplx x1 = lv[1][pa], y1 = lv[3][q];
          // i [A^R B^R + A^<(n,m) B^R + A^R B^<(n,m)]
          t = mul_i(x0 * y0 + x1 * y0 + x0 * y1);
        } else if (comp == 3) {
          t = x0 * y0;
        } else {
          t = mul_i(x0 * y0);
        }
        pa = pa == 0 ? nk - 1 : pa - 1;
      }
      acc = acc + t;
    }
    const Prob& O = po.get(k);
    cplx* dst;
    if (comp == 3) dst = O.Gmat + (size_t)j * dd + e;
    else if (comp == 0) dst = O.Gret + (tri(n) + j) * dd + e;
    else if (comp == 1) dst = O.Gles + (tri(n) + j) * dd + e;
    else dst = O.Gtv + ((size_t)n * (ntau + 1) + j) * dd + e;
    gst(dst, scale * acc);
  }
}

hipError_t launch_kbubble(int mode, const ProbArg& pg, const ProbArg& pw, const ProbArg& po, int n, int d,
                          int ntau, double alpha, hipStream_t s) {
  long nelem = n == -1 ? (long)(ntau + 1) * d * d : (long)(2 * (n + 1) + ntau + 1) * d * d;
  dim3 g((unsigned)nelem);
  if (mode == 1) k_kbubble<1><<<g, NKB, 0, s>>>(pg, pw, po, n, nelem, alpha);
  else k_kbubble<2><<<g, NKB, 0, s>>>(pg, pw, po, n, nelem, alpha);
  return hipGetLastError();
}

}  // namespace cntr
