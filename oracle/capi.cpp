// C entry points of the oracle for the Python test harness (ctypes) and the
// self-consistent drivers of the example programs (Sec. "Hubbard chain":
// Matsubara loop, bootstrapping loop, predictor-corrector time stepping).
// Test infrastructure only.
#include <chrono>
#include <cstring>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.hpp"

using namespace oracle;

extern "C" {

struct oracle_grid {
  int32_t nt, ntau, d, sig, k;
  double beta, h, mu;
};

static HM view(const oracle_grid* g, void* mat, void* ret, void* les, void* tv) {
  HM v;
  v.g = Grid{g->nt, g->ntau, g->d, g->sig, g->k, g->beta, g->h, g->mu};
  v.mat = (cd*)mat;
  v.ret = (cd*)ret;
  v.les = (cd*)les;
  v.tv = (cd*)tv;
  return v;
}

#define HMARGS(X) void *X##_mat, void *X##_ret, void *X##_les, void *X##_tv
#define HMV(g, X) view(g, X##_mat, X##_ret, X##_les, X##_tv)

int oracle_weights(int k, double* P, double* D, double* Iw, double* bdf, double* start,
                   double* omega, double* R) {
  if (k < 0 || k > 6) return -1;
  const Weights& W = weights(k);
  std::memcpy(P, W.P.data(), W.P.size() * sizeof(double));
  std::memcpy(D, W.D.data(), W.D.size() * sizeof(double));
  std::memcpy(Iw, W.Iw.data(), W.Iw.size() * sizeof(double));
  std::memcpy(bdf, W.bdf.data(), W.bdf.size() * sizeof(double));
  std::memcpy(start, W.start.data(), W.start.size() * sizeof(double));
  std::memcpy(omega, W.omega.data(), W.omega.size() * sizeof(double));
  std::memcpy(R, W.R.data(), W.R.size() * sizeof(double));
  return 0;
}

double oracle_gregory(int k, int n, int j) { return weights(k).w(n, j); }

void oracle_gregory_rational(int k, int n, int j, int64_t* num, int64_t* den) {
  gregory_rational(k, n, j, num, den);
}

int oracle_solve(int n, int nrhs, void* A, void* B) { return solve(n, nrhs, (cd*)A, (cd*)B) ? 0 : -4; }

void oracle_eigh(int d, const void* A, double* w, void* V) { eigh(d, (const cd*)A, w, (cd*)V); }

void oracle_free_mat(const oracle_grid* g, const void* eps, void* out) {
  Grid gg{g->nt, g->ntau, g->d, g->sig, g->k, g->beta, g->h, g->mu};
  free_mat(gg, (const cd*)eps, (cd*)out);
}

void oracle_convolution_timestep(int n, const oracle_grid* g, HMARGS(C), HMARGS(A), HMARGS(Acc),
                                 HMARGS(B), HMARGS(Bcc), const void* f) {
  Fn fn{g->d, (const cd*)f};
  convolution_timestep(n, HMV(g, C), HMV(g, A), HMV(g, Acc), HMV(g, B), HMV(g, Bcc),
                       f ? &fn : nullptr);
}

void oracle_conv_les_diag(int n, const oracle_grid* g, HMARGS(A), HMARGS(B), void* out) {
  Mat c = conv_les_diag(n, HMV(g, A), HMV(g, B));
  std::memcpy(out, c.data(), c.size() * sizeof(cd));
}

int oracle_dyson_mat(const oracle_grid* g, HMARGS(G), HMARGS(S), const void* eps_m1) {
  return dyson_mat(HMV(g, G), HMV(g, S), (const cd*)eps_m1) ? 0 : -4;
}

int oracle_dyson_start(const oracle_grid* g, HMARGS(G), HMARGS(S), const void* eps) {
  Fn e{g->d, (const cd*)eps};
  return dyson_start(HMV(g, G), HMV(g, S), e) ? 0 : -4;
}

int oracle_dyson_timestep(int n, const oracle_grid* g, HMARGS(G), HMARGS(S), const void* eps,
                          int variant) {
  Fn e{g->d, (const cd*)eps};
  return dyson_timestep(n, HMV(g, G), HMV(g, S), e, (char)variant) ? 0 : -4;
}

int oracle_vie2_mat(const oracle_grid* g, HMARGS(G), HMARGS(F), HMARGS(Q)) {
  return vie2_mat(HMV(g, G), HMV(g, F), HMV(g, Q)) ? 0 : -4;
}

int oracle_vie2_start(const oracle_grid* g, HMARGS(G), HMARGS(F), HMARGS(Fcc), HMARGS(Q)) {
  return vie2_start(HMV(g, G), HMV(g, F), HMV(g, Fcc), HMV(g, Q)) ? 0 : -4;
}

int oracle_vie2_timestep(int n, const oracle_grid* g, HMARGS(G), HMARGS(F), HMARGS(Fcc), HMARGS(Q)) {
  return vie2_timestep(n, HMV(g, G), HMV(g, F), HMV(g, Fcc), HMV(g, Q)) ? 0 : -4;
}

void oracle_sigma_2b(int n, const oracle_grid* g, HMARGS(G), const double* U, HMARGS(S)) {
  sigma_2b(n, HMV(g, G), U, HMV(g, S));
}

void oracle_hartree(int n, const oracle_grid* g, HMARGS(G), const double* U, const void* eps0,
                    void* eps_mf, double nbar) {
  hartree(n, HMV(g, G), U, (const cd*)eps0, (cd*)eps_mf, nbar);
}

void oracle_density_matrix(int n, const oracle_grid* g, HMARGS(G), void* rho) {
  density_matrix(n, HMV(g, G), (cd*)rho);
}

void oracle_extrapolate(int n, const oracle_grid* g, HMARGS(G)) { extrapolate_timestep(n, HMV(g, G)); }

double oracle_distance(int n, const oracle_grid* g, HMARGS(A), HMARGS(B)) {
  return distance_norm2(n, HMV(g, A), HMV(g, B));
}

// Self-consistent second-Born + Hartree propagation of a Hubbard cluster.
// Matsubara loop until rel. distance < mats_tol (or mats_maxit); bootstrap
// loop over slices 0..k until rel. distance < boot_tol and at least 3
// iterations (or boot_maxit); then for n = k+1..nt_stop: predictor
// (extrapolation) and ncorr corrector iterations {Hartree, Sigma_2B, step}
// (stopping early when corr_tol > 0 and the rel. distance is below it).
// stats[0..5] = mats iterations, boot iterations, total corrector
// iterations, last mats error, last boot error, max last corrector error.
int oracle_solve_2b(const oracle_grid* g, HMARGS(G), HMARGS(S), HMARGS(Gold), const void* eps0,
                    const double* U, void* eps_mf, double nbar, int mats_maxit, double mats_tol,
                    double mats_mix, int boot_maxit, double boot_tol, int ncorr, double corr_tol,
                    int nt_stop, int variant, double* stats) {
  HM G = HMV(g, G), S = HMV(g, S), Go = HMV(g, Gold);
  const cd* e0 = (const cd*)eps0;
  cd* emf = (cd*)eps_mf;
  Fn emf_fn{g->d, emf};
  int k = g->k;
  bool ok = true;
  free_mat(G.g, e0, G.mat);
  int it;
  double err = 0.0;
  size_t bs = (size_t)g->d * g->d, nm = (g->ntau + 1) * bs;
  std::vector<cd> s_in(nm), e_in(bs);
  for (it = 0; it < mats_maxit; it++) {
    hartree(-1, G, U, e0, emf, nbar);
    sigma_2b(-1, G, U, S);
    // Reading: the plain Sigma <-> G iteration of the Matsubara loop has an
    // oscillating unstable mode for strong coupling; linear mixing of the
    // input (Sigma^M, eps_mf_{-1}) with the previous input keeps the same
    // fixed point and converges.
    if (it > 0)
      for (size_t i = 0; i < nm; i++) S.mat[i] = mats_mix * S.mat[i] + (1.0 - mats_mix) * s_in[i];
    if (it > 0)
      for (size_t i = 0; i < bs; i++) emf[i] = mats_mix * emf[i] + (1.0 - mats_mix) * e_in[i];
    std::copy(S.mat, S.mat + nm, s_in.begin());
    std::copy(emf, emf + bs, e_in.begin());
    copy_timestep(-1, Go, G);
    ok = dyson_mat(G, S, emf) && ok;
    err = distance_norm2(-1, G, Go) / slice_norm(-1, G);
    if (err < mats_tol) {
      it++;
      break;
    }
  }
  stats[0] = it;
  stats[3] = err;
  for (it = 0; it < boot_maxit; it++) {
    for (int n = 0; n <= k; n++) hartree(n, G, U, e0, emf, nbar);
    for (int n = 0; n <= k; n++) sigma_2b(n, G, U, S);
    for (int n = 0; n <= k; n++) copy_timestep(n, Go, G);
    ok = dyson_start(G, S, emf_fn) && ok;
    double num = 0.0, den = 0.0;
    for (int n = 0; n <= k; n++) {
      num += distance_norm2(n, G, Go);
      den += slice_norm(n, G);
    }
    err = num / den;
    if (err < boot_tol && it > 2) {
      it++;
      break;
    }
  }
  stats[1] = it;
  stats[4] = err;
  double total = 0.0, maxerr = 0.0;
  for (int n = k + 1; n <= nt_stop; n++) {
    extrapolate_timestep(n - 1, G);
    for (it = 0; it < ncorr; it++) {
      hartree(n, G, U, e0, emf, nbar);
      sigma_2b(n, G, U, S);
      copy_timestep(n, Go, G);
      ok = dyson_timestep(n, G, S, emf_fn, (char)variant) && ok;
      err = distance_norm2(n, G, Go) / slice_norm(n, G);
      total += 1;
      if (corr_tol > 0 && err < corr_tol) break;
    }
    if (err > maxerr) maxerr = err;
  }
  // final mean field and self-energy consistent with the last G
  for (int n = k + 1; n <= nt_stop; n++) {
    hartree(n, G, U, e0, emf, nbar);
    sigma_2b(n, G, U, S);
  }
  stats[2] = total;
  stats[5] = maxerr;
  return ok ? 0 : -4;
}

// Fixed self-energy: Matsubara, start-up and steps k+1..nt_stop.
int oracle_solve_fixed(const oracle_grid* g, HMARGS(G), HMARGS(S), const void* eps, int nt_stop,
                       int variant, double* seconds) {
  HM G = HMV(g, G), S = HMV(g, S);
  Fn e{g->d, (const cd*)eps};
  auto t0 = std::chrono::steady_clock::now();
  bool ok = dyson_mat(G, S, e.at(-1));
  auto t1 = std::chrono::steady_clock::now();
  ok = dyson_start(G, S, e) && ok;
  auto t2 = std::chrono::steady_clock::now();
  for (int n = g->k + 1; n <= nt_stop; n++) ok = dyson_timestep(n, G, S, e, (char)variant) && ok;
  auto t3 = std::chrono::steady_clock::now();
  if (seconds) {
    seconds[0] = std::chrono::duration<double>(t1 - t0).count();
    seconds[1] = std::chrono::duration<double>(t2 - t1).count();
    seconds[2] = std::chrono::duration<double>(t3 - t2).count();
  }
  return ok ? 0 : -4;
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
