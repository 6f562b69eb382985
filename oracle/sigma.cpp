// Second-Born self-energy, Hartree mean field, density matrix, polynomial
// extrapolation and the distance norm. Test infrastructure only.
#include <cmath>

#include "oracle.hpp"

namespace oracle {

// Eq. sigma_hubb_2b for the spin-symmetric case: elementwise in the orbital
// indices (a, b),  Sigma_ab(z, z') = U(z) U(z') G_ab(z, z')^2 G_ba(z', z).
// Reading: every Keldysh component is derived directly from this contour
// identity (the printed Matsubara bubble rules carry signs that cancel here):
//   Sigma^<_ab(t_j,t_n)  = U_j U_n (G^<_ab(j,n))^2 G^>_ba(n,j)
//   Sigma^R_ab(t_n,t_j)  = Sigma^>_ab(n,j) - Sigma^<_ab(n,j)   (Eq. Cretmod)
//   Sigma^rceil_ab(n,m)  = U_n U_{-1} (G^rceil_ab(n,m))^2 G^lceil_ba(m,n)
//   Sigma^M_ab(m)        = -xi U_{-1}^2 (G^M_ab(m))^2 G^M_ba(ntau-m)
// with G^>(t_n,t_j) = G^R + G^< for t_n >= t_j, G^<(t_n,t_j) = -[G^<(t_j,t_n)]^dag,
// G^lceil(tau_m,t_n) = -xi [G^rceil(t_n, beta - tau_m)]^dag.
void sigma_2b(int n, const HM& G, const double* U, const HM& S) {
  const Grid& g = G.g;
  int d = g.d, ntau = g.ntau;
  double xi = g.sig;
  auto u = [&](int t) { return U[t + 1]; };
  if (n == -1) {
    for (int m = 0; m <= ntau; m++)
      for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) {
          cd x = G.M(m)[a * d + b], y = G.M(ntau - m)[b * d + a];
          S.M(m)[a * d + b] = -xi * u(-1) * u(-1) * x * x * y;
        }
    return;
  }
  for (int j = 0; j <= n; j++) {
    double uu = u(n) * u(j);
    const cd *R = G.R(n, j), *L = G.L(j, n);
    for (int a = 0; a < d; a++)
      for (int b = 0; b < d; b++) {
        cd Lab = L[a * d + b], Lba = L[b * d + a];
        cd Rab = R[a * d + b], Rba = R[b * d + a];
        // G^>_ba(n, j) = R_ba - conj(L_ab);  G^<_ab(n, j) = -conj(L_ba)
        cd gtr_ba_nj = Rba - std::conj(Lab);
        S.L(j, n)[a * d + b] = uu * Lab * Lab * gtr_ba_nj;
        cd gtr_ab_nj = Rab - std::conj(Lba);
        cd les_ab_nj = -std::conj(Lba);
        cd gtr_ba_jn = Lba - std::conj(Rab);  // G^>_ba(j, n) = -conj(G^>_ab(n, j))
        cd sg = uu * gtr_ab_nj * gtr_ab_nj * Lba;
        cd sl = uu * les_ab_nj * les_ab_nj * gtr_ba_jn;
        S.R(n, j)[a * d + b] = sg - sl;
      }
  }
  for (int m = 0; m <= ntau; m++)
    for (int a = 0; a < d; a++)
      for (int b = 0; b < d; b++) {
        cd x = G.T(n, m)[a * d + b];
        cd vt = -xi * std::conj(G.T(n, ntau - m)[a * d + b]);
        S.T(n, m)[a * d + b] = u(n) * u(-1) * x * x * vt;
      }
}

// rho = <c^dag c>: rho_n = i xi G^<(t_n, t_n) for n >= 0 and
// rho = -G^M(beta^-) on the Matsubara branch.
void density_matrix(int n, const HM& G, cd* rho) {
  int d = G.g.d;
  double xi = G.g.sig;
  for (int i = 0; i < d * d; i++)
    rho[i] = n == -1 ? -G.M(G.g.ntau)[i] : I1 * xi * G.L(n, n)[i];
}

// Mean field of the Hubbard chain with the chemical-potential shift -U nbar:
// eps_mf = eps0 + U (n_i - nbar) delta_ij  (Fock term zero by spin symmetry).
void hartree(int n, const HM& G, const double* U, const cd* eps0, cd* eps_mf, double nbar) {
  int d = G.g.d;
  Mat rho = zeros(d);
  density_matrix(n, G, rho.data());
  const cd* e0 = eps0 + (size_t)(n + 1) * d * d;
  cd* em = eps_mf + (size_t)(n + 1) * d * d;
  for (int i = 0; i < d * d; i++) em[i] = e0[i];
  for (int i = 0; i < d; i++) em[i * d + i] += U[n + 1] * (rho[i * d + i].real() - nbar);
}

// Eq. polyextrap: y_{n+1} = sum_l C_l y_{n-l}, with C from the interpolating
// polynomial through the k+1 latest points evaluated one step ahead
// (App. "Extrapolation of contour functions").
void extrapolate_timestep(int n, const HM& G) {
  const Grid& g = G.g;
  int d = g.d, k = g.k, ntau = g.ntau;
  const Weights& W = weights(k);
  std::vector<double> C(k + 1);
  for (int l = 0; l <= k; l++) {
    // node i = k - l carries y_{n-l}; evaluate at x = k+1
    int i = k - l;
    double acc = 0.0, xp = 1.0;
    for (int a = 0; a <= k; a++) {
      acc += W.p(a, i) * xp;
      xp *= (k + 1);
    }
    C[l] = acc;
  }
  size_t bs = (size_t)d * d;
  int n1 = n + 1;
  for (int m = 0; m <= ntau; m++) {
    cd* o = G.T(n1, m);
    for (size_t i = 0; i < bs; i++) o[i] = 0.0;
    for (int l = 0; l <= k; l++)
      for (size_t i = 0; i < bs; i++) o[i] += C[l] * G.T(n - l, m)[i];
  }
  // retarded: columns j = 0..k along t, then the diagonals t - t' = j h
  for (int j = 0; j <= k; j++) {
    cd* o = G.R(n1, j);
    for (size_t i = 0; i < bs; i++) o[i] = 0.0;
    for (int l = 0; l <= k; l++) {
      Mat y = Rt(G, n - l, j);
      for (size_t i = 0; i < bs; i++) o[i] += C[l] * y[i];
    }
  }
  for (int j = 0; j <= n - k; j++) {
    cd* o = G.R(n1, n1 - j);
    for (size_t i = 0; i < bs; i++) o[i] = 0.0;
    for (int l = 0; l <= k; l++)
      for (size_t i = 0; i < bs; i++) o[i] += C[l] * G.R(n - l, n - l - j)[i];
  }
  // lesser: rows j = 0..k along t', then the diagonals
  for (int j = 0; j <= k; j++) {
    cd* o = G.L(j, n1);
    for (size_t i = 0; i < bs; i++) o[i] = 0.0;
    for (int l = 0; l <= k; l++) {
      Mat y = Lh(G, j, n - l);
      for (size_t i = 0; i < bs; i++) o[i] += C[l] * y[i];
    }
  }
  for (int j = k + 1; j <= n1; j++) {
    cd* o = G.L(j, n1);
    for (size_t i = 0; i < bs; i++) o[i] = 0.0;
    for (int l = 0; l <= k; l++)
      for (size_t i = 0; i < bs; i++) o[i] += C[l] * G.L(j - 1 - l, n - l)[i];
  }
}

// Eq. distancenorm (a sum of absolute values per component).
double distance_norm2(int n, const HM& A, const HM& B) {
  const Grid& g = A.g;
  size_t bs = (size_t)g.d * g.d;
  double s = 0.0;
  if (n == -1) {
    for (int m = 0; m <= g.ntau; m++)
      for (size_t i = 0; i < bs; i++) s += std::abs(A.M(m)[i] - B.M(m)[i]);
    return s;
  }
  for (int m = 0; m <= g.ntau; m++)
    for (size_t i = 0; i < bs; i++) s += std::abs(A.T(n, m)[i] - B.T(n, m)[i]);
  for (int j = 0; j <= n; j++)
    for (size_t i = 0; i < bs; i++) {
      s += std::abs(A.R(n, j)[i] - B.R(n, j)[i]);
      s += std::abs(A.L(j, n)[i] - B.L(j, n)[i]);
    }
  return s;
}

double slice_norm(int n, const HM& A) {
  const Grid& g = A.g;
  size_t bs = (size_t)g.d * g.d;
  double s = 0.0;
  if (n == -1) {
    for (int m = 0; m <= g.ntau; m++)
      for (size_t i = 0; i < bs; i++) s += std::abs(A.M(m)[i]);
    return s;
  }
  for (int m = 0; m <= g.ntau; m++)
    for (size_t i = 0; i < bs; i++) s += std::abs(A.T(n, m)[i]);
  for (int j = 0; j <= n; j++)
    for (size_t i = 0; i < bs; i++) s += std::abs(A.R(n, j)[i]) + std::abs(A.L(j, n)[i]);
  return s;
}

void copy_timestep(int n, const HM& dst, const HM& src) {
  const Grid& g = src.g;
  size_t bs = (size_t)g.d * g.d;
  if (n == -1) {
    std::copy(src.M(0), src.M(0) + (g.ntau + 1) * bs, dst.M(0));
    return;
  }
  std::copy(src.T(n, 0), src.T(n, 0) + (g.ntau + 1) * bs, dst.T(n, 0));
  std::copy(src.R(n, 0), src.R(n, 0) + (n + 1) * bs, dst.R(n, 0));
  std::copy(src.L(0, n), src.L(0, n) + (n + 1) * bs, dst.L(0, n));
}

}  // namespace oracle
