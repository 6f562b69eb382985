// Plain CPU oracle for the Kadanoff-Baym (Dyson) time stepper of
// NESSi / libcntr (arXiv:1911.01211).
//
// TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
// baseline leg of the benchmark may load or call this code. The GPU
// library does not include, link or call anything in this directory, and
// this directory shares no code with it.
//
// Every routine is a direct, unoptimised transcription of the discrete
// scheme of Part II of the paper (polynomial, BDF, Gregory and boundary
// convolution weights; the Volterra start-up and time-stepping rules; the
// discrete contour convolutions; the Dyson start-up and time steps).
// Arithmetic is std::complex<double>; weights are exact rationals rounded
// once to double. Readings of ambiguous passages are marked "Reading:".
#pragma once
#include <complex>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace oracle {

using cd = std::complex<double>;
static const cd I1(0.0, 1.0);

// ---------------------------------------------------------------- weights
// Sec. "Basic integration and differentiation rules": P (Eq. integrator_P),
// D (Eq. integrator_D), I (Eq. integrator_I), BDF a (Eq. integrator_bd,
// Tab. integrator_bd), Gregory w (Eq. integrator_greg, Tab. gregory) and the
// boundary-convolution weights R (Eq. integrator_R).
struct Weights {
  int k = 0;
  std::vector<double> P;      // [a][l], (k+1)^2
  std::vector<double> D;      // [m][l], (k+1)^2
  std::vector<double> Iw;     // [m][n][l], (k+1)^3
  std::vector<double> bdf;    // a_l, k+1
  std::vector<double> start;  // s_{n,j} = I_{0,n,j}, (k+1)^2
  std::vector<double> omega;  // end weights omega_j, k+1
  std::vector<double> R;      // [m][r][s], (k+1)^3
  std::vector<double> wlow;   // w_{n,j} for n <= 2k, [(2k+1)][(2k+1)]
  // Gregory weight w^{(k)}_{n,j}; valid for 0<=j<=max(n,k).
  double w(int n, int j) const;
  double p(int a, int l) const { return P[a * (k + 1) + l]; }
  double d(int m, int l) const { return D[m * (k + 1) + l]; }
  double i(int m, int n, int l) const { return Iw[(m * (k + 1) + n) * (k + 1) + l]; }
  double s(int n, int j) const { return start[n * (k + 1) + j]; }
  double r(int m, int a, int b) const { return R[(m * (k + 1) + a) * (k + 1) + b]; }
};
const Weights& weights(int k);  // k in 1..5 (also 0..6 for the tables)

// Gregory weights from the classical end-correction construction, as exact
// rationals (numerator, denominator). Exposed for the exactness tests.
void gregory_rational(int k, int n, int j, int64_t* num, int64_t* den);

// -------------------------------------------------------------- data view
// Canonical storage of a hermitian contour function (Eq. storage_herm):
//   mat[m]            C^M_m,         m = 0..ntau
//   ret[n(n+1)/2+j]   C^R_{n,j},     j = 0..n
//   les[n(n+1)/2+j]   C^<_{j,n},     j = 0..n
//   tv [n(ntau+1)+m]  C^rceil_{n,m}, m = 0..ntau
// each entry a row-major d x d complex block. The view does not own memory.
struct Grid {
  int nt, ntau, d, sig, k;
  double beta, h, mu;
  double htau() const { return beta / ntau; }
};

struct HM {
  Grid g;
  cd *mat, *ret, *les, *tv;
  int d() const { return g.d; }
  size_t bs() const { return (size_t)g.d * g.d; }
  cd* M(int m) const { return mat + (size_t)m * bs(); }
  cd* R(int n, int j) const { return ret + ((size_t)n * (n + 1) / 2 + j) * bs(); }
  cd* L(int j, int n) const { return les + ((size_t)n * (n + 1) / 2 + j) * bs(); }
  cd* T(int n, int m) const { return tv + ((size_t)n * (g.ntau + 1) + m) * bs(); }
};

// Single-time contour function f_n, n=-1..nt, stored at index n+1 (d x d).
struct Fn {
  int d;
  const cd* p;
  const cd* at(int n) const { return p + (size_t)(n + 1) * d * d; }
};

// ---------------------------------------------------------- small algebra
using Mat = std::vector<cd>;  // row-major d x d
Mat zeros(int d);
Mat eye(int d);
Mat dag(const Mat& A, int d);
Mat dag(const cd* A, int d);
void gemm_acc(cd* C, const cd* A, const cd* B, int d, cd alpha);  // C += a A B
// Solve A X = B for X (A: n x n, B: n x nrhs, both row-major; overwritten).
// Gaussian elimination with partial pivoting. Returns false if singular.
bool solve(int n, int nrhs, cd* A, cd* B);
// Hermitian eigen-decomposition by cyclic Jacobi rotations: A = V diag(w) V^dag
void eigh(int d, const cd* A, double* w, cd* V);

// ---------------------------------------------------------- contour tools
// Extensions outside the stored triangles (hermitian symmetry, Eq. hermconjg
// and the continuation of the retarded component beyond t<t').
Mat Rt(const HM& G, int a, int b);   // G^R_{a,b} for any a,b (b>a extended)
Mat Lh(const HM& G, int a, int b);   // G^<_{a,b} for any a,b
Mat Adv(const HM& G, int a, int b);  // G^A_{a,b} = (G~^R_{b,a})^dag
Mat Vt(const HM& G, int j, int n);   // G^lceil(tau_j, t_n) = -xi (T_{n,ntau-j})^dag
// The same for a function X that is not hermitian, with Xc = X^ddagger
// supplying the values outside X's stored triangles.
Mat RtX(const HM& X, const HM& Xc, int a, int b);   // X~^R_{a,b}
Mat LhX(const HM& X, const HM& Xc, int a, int b);   // X^<_{a,b}
Mat AdvX(const HM& X, const HM& Xc, int a, int b);  // X^A_{a,b} = ([Xc]~^R_{b,a})^dag
Mat VtX(const HM& X, const HM& Xc, int j, int n);   // X^lceil(tau_j, t_n)

// ------------------------------------------------------------ convolution
// Sec. "Numerical details: convolution integrals": T[C]_n of C = A*f*B.
// A, Acc (= A^ddagger), B, Bcc given; f at n=-1..nt (nullptr means f = 1).
void convolution_timestep(int n, const HM& C, const HM& A, const HM& Acc, const HM& B,
                          const HM& Bcc, const Fn* f);
// Individual pieces, used by the solvers.
Mat cm12(int m, const HM& A, const HM& B, const cd* f_m1);  // C^M_1 + C^M_2
Mat ctv23(int n, int m, const HM& A, const HM& B, const cd* f_m1);  // C^rceil_2+3
// [A*B]^<(t_n,t_n) for hermitian A, B (f = 1): used for correlation energies.
Mat conv_les_diag(int n, const HM& A, const HM& B);

// ------------------------------------------------------------------ dyson
// Matsubara: exact solution of the discrete integral form
// G = g + [K*G]^M, K = [g*Sigma]^M (Eq. Gmat_dyson_integ) by a dense solve.
bool dyson_mat(const HM& G, const HM& Sig, const cd* eps_m1);
// Free Matsubara function g_m for the hermitian d x d matrix eps - mu.
void free_mat(const Grid& g, const cd* eps, cd* out);
// Start-up: slices 0..k (Sec. "Start").
bool dyson_start(const HM& G, const HM& Sig, const Fn& eps);
// Time step n > k. variant 'B': data-parallel form (bulk by the
// non-conjugate/conjugate single steps, k+1 boundary points serial);
// variant 'A': fully serial form.
bool dyson_timestep(int n, const HM& G, const HM& Sig, const Fn& eps, char variant);

// ------------------------------------------------------------------- vie2
// Dyson equation in integral form, (1 + F) * G = Q with F^ddagger = Fcc
// (Sec. "vie2: Dyson equation in integral form", Sec. "Implementation: vie2").
// Matsubara: dense solve of the discrete Eq. vie2_langreth_m.
bool vie2_mat(const HM& G, const HM& F, const HM& Q);
// Start-up: slices 0..k (Sec. "Start" of the vie2 implementation).
bool vie2_start(const HM& G, const HM& F, const HM& Fcc, const HM& Q);
// Time step n > k: retarded and left-mixing rows by Eq. MBCVSAMx01_t, the
// lesser column by the conjugate equation (variant B) for every row m <= n.
bool vie2_timestep(int n, const HM& G, const HM& F, const HM& Fcc, const HM& Q);

// --------------------------------------------------------- self-energies
// Second-Born self-energy (Eq. sigma_hubb_2b, spin-symmetric) on slice n
// from G slice n; U at n=-1..nt stored at index n+1.
void sigma_2b(int n, const HM& G, const double* U, const HM& Sig);
// Hartree mean field eps_mf_n = eps0_n + diag(U_n (n_i - nbar)).
void hartree(int n, const HM& G, const double* U, const cd* eps0, cd* eps_mf, double nbar);
// Density matrix rho_n (n=-1: from the Matsubara component).
void density_matrix(int n, const HM& G, cd* rho);

// ------------------------------------------------------------- utilities
void extrapolate_timestep(int n, const HM& G);      // T[G]_{n} -> T[G]_{n+1}
double distance_norm2(int n, const HM& A, const HM& B);
double slice_norm(int n, const HM& A);
void copy_timestep(int n, const HM& dst, const HM& src);

}  // namespace oracle
