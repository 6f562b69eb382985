/* cntr.h -- C ABI of the MI355X (gfx950) Kadanoff-Baym / Dyson time stepper.
 *
 * The library solves the Dyson equation of nonequilibrium Green's functions
 * on the L-shaped Kadanoff-Baym contour, following NESSi / libcntr
 * (arXiv:1911.01211, Part II): Matsubara solve, start-up, k-th order time
 * stepping with BDF derivatives and Gregory quadrature for the history
 * convolutions, the contour convolution, and the second-Born self-energy.
 *
 * Conventions (all entry points)
 *  - Complex numbers are complex128, interleaved (re, im), the storage of
 *    torch.complex128 / numpy.complex128 / C99 double _Complex.
 *  - Contour functions are given by four DEVICE pointers in the canonical
 *    storage of the paper (Eq. storage_herm), each entry a row-major d x d
 *    block:
 *        mat : [ntau+1]                 C^M_m = C^M(m h_tau)
 *        ret : [(nt+1)(nt+2)/2]         C^R_{n,j} at n(n+1)/2 + j, j <= n
 *        les : [(nt+1)(nt+2)/2]         C^<_{j,n} at n(n+1)/2 + j, j <= n
 *        tv  : [(nt+1)(ntau+1)]         C^rceil_{n,m} at n(ntau+1) + m
 *    Time slice n (Sec. "Numerical representation of NEGFs") is the row
 *    R_{n,0..n}, the column L_{0..n,n} and the row T_{n,0..ntau}; slice -1 is
 *    the Matsubara component.
 *  - Single-time functions (eps, eps_mf) are DEVICE arrays of (nt+2) d x d
 *    blocks; entry n+1 holds time n, entry 0 holds the equilibrium value
 *    f(0^-) of the imaginary branch. U is a DEVICE array of nt+2 doubles
 *    with the same indexing.
 *  - sig = -1 for fermions, +1 for bosons; k (1..5) is the order of the
 *    scheme; h is the time step, beta the inverse temperature, h_tau =
 *    beta/ntau, mu the chemical potential (the contour evolves with eps-mu).
 *  - Every call takes `count` instances: host arrays of `count` grids and
 *    contour descriptors (the pointers inside are device pointers). count = 1
 *    is the plain per-instance path.
 *  - Ownership: the caller allocates and frees every array passed in; the
 *    library keeps no pointer after a call returns. Internal scratch memory
 *    and the weight tables are owned by the library (released by
 *    cntr_finalize).
 *  - Streams: `stream` is a hipStream_t (NULL = default stream). Work is
 *    enqueued asynchronously; host-side validation fails before anything is
 *    enqueued. Conditions detected on the device (a singular step matrix)
 *    are reported by cntr_sync on the same stream.
 *  - Errors: every call returns a cntr_status; nothing aborts or exits.
 *    cntr_last_error() returns a message for the last failure of the
 *    calling thread.
 */
#ifndef CNTR_H
#define CNTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CNTR_OK = 0,
  CNTR_EINVAL = -1,     /* k not in 1..5, d < 1 or d > 8, ntau < 2k+2, nt < k, sig not +-1, h/beta <= 0 */
  CNTR_ESHAPE = -2,     /* inconsistent instances or NULL pointers */
  CNTR_EORDER = -3,     /* tstp out of range, or (order checks on) inputs of tstp not complete (Tab. dyson) */
  CNTR_ESINGULAR = -4,  /* singular step or start-up matrix (device) */
  CNTR_ENONFINITE = -5, /* non-finite value detected */
  CNTR_EHIP = -6,       /* HIP runtime error */
  CNTR_ENOMEM = -7,     /* device allocation failed */
  CNTR_ENOCONV = -8,    /* iteration did not reach its tolerance */
  CNTR_ESYMMETRY = -9   /* (symmetry checks on) a self-energy violates hermitian symmetry */
} cntr_status;

typedef struct {
  int32_t nt, ntau, d, sig, k;
  double beta, h, mu;
} cntr_grid;

typedef struct {
  void *mat, *ret, *les, *tv; /* device pointers, canonical layout */
} cntr_gf;

/* ------------------------------------------------------------------ A1 --
 * Matsubara component T[G]_{-1} (Sec. "Matsubara", Eq. Gmat_dyson_integ):
 * the exact solution of the discrete integral equation
 *     G^M = g + [K * G]^M,  K = [g * Sigma]^M,
 * with g the free Matsubara function of eps_{-1} - mu and the convolutions
 * discretised by Eqs. cm1/cm2 (Gregory weights, boundary-convolution
 * weights near the ends). Inputs: Sigma[i].mat, eps[i] (entry 0 used).
 * Output: G[i].mat. The linear system is solved on the device to a relative
 * residual below `tol` (<= 0: 1e-14) within `max_iter` refinement sweeps
 * (<= 0: 200); otherwise CNTR_ENOCONV. This call synchronizes `stream`. */
cntr_status cntr_init_matsubara(int32_t count, const cntr_grid* grids, const cntr_gf* G,
                                const cntr_gf* Sigma, const void* const* eps, double tol,
                                int32_t max_iter, void* stream);

/* Fourier-series Matsubara solve (Sec. "Implementation: dyson", Matsubara,
 * "Fourier series representation"; the paper's fast initial guess): with
 * x = eps(0^-) - mu and frequencies w = (2m+1) pi/beta, m = -Nw..Nw-1
 * (fermions) or 2 m pi/beta, m = -Nw..Nw (bosons), Nw = oversample * ntau,
 *   Sigma(i w) = integral of the piecewise-cubic interpolant of Sigma^M
 *                times e^{i w tau} over [0, beta] (on each interval the cubic
 *                through the grid points J-1..J+2, one-sided at the ends),
 *   G(i w)     = [i w - x - Sigma(i w)]^{-1},
 *   G^M(tau_j) = (1/beta) sum_w e^{-i w tau_j} [G(i w) - 1/(i w)] - c(tau_j) 1,
 *                c = 1/2 (fermions), 1/2 - tau/beta (bosons; no 1/(i w) at w = 0).
 * Average error O(h_tau^2), largest (at tau = 0, beta) O(1/Nw) against the
 * continuous solution; cntr_init_matsubara solves the discrete equation
 * exactly. Inputs: grids[i] (ntau >= 3, beta, mu, sig), Sigma[i].mat (DEVICE;
 * Sigma == NULL: Sigma = 0), eps[i] (DEVICE, entry 0 = eps(0^-)), oversample
 * in 1..64 (the paper's default is 10). Output: G[i].mat (overwritten; the
 * other components untouched). Uses the stream's scratch ((2 Nw + 1) d^2
 * complex values), asynchronous. Errors: CNTR_EINVAL (ntau < 3, oversample
 * out of range), CNTR_ESHAPE (null pointers). */
cntr_status cntr_matsubara_fourier(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                                   const void* const* eps, int32_t oversample, void* stream);

/* ---------------------------------------------------------------- A2-A7 --
 * Dyson equation (Eq. dyson, Sec. "Implementation: dyson").
 *  tstp <= k : start-up, computes slices 0..k from T[G]_{-1}, Sigma slices
 *              -1..k and eps (Sec. "Start", Tab. dyson row dyson_start).
 *  tstp  > k : time step, computes slice tstp from slices -1..tstp-1 of G,
 *              Sigma slices tstp-k..tstp and eps (Sec. "Time stepping"):
 *              retarded row by single Volterra steps per column plus a
 *              k-point conjugate start-up at the diagonal, left-mixing row by
 *              one Volterra step per tau index, lesser column by single
 *              conjugate steps per row and k+1 serial boundary steps (for
 *              tstp <= 2k the whole column is done serially).
 * Instances with nt < tstp are skipped. eps[i] is the (mean-field)
 * single-particle Hamiltonian. Writes slice(s) of G[i] only. */
cntr_status cntr_dyson_step(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                            const cntr_gf* Sigma, const void* const* eps, void* stream);

/* Allocation-free variant of cntr_dyson_step, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments, kernels and results as
 * cntr_dyson_step; it calls no hipMalloc/hipFree and creates no runtime
 * objects (no profiler events). Its scratch (partial sums, step inverses,
 * status words, batch descriptors) is a static device array of
 * 64 MiB + 41 KiB held by every GPU the library runs on until the process
 * ends; the descriptors of a batch (count > 1) are written by a small kernel
 * whose arguments carry them, so nothing refers to host memory after the
 * call. Limits: count <= 256, and the step regions of all problems (the step
 * at the largest nt of the call; about 42 MB for nt = 1000, ntau = 400,
 * d = 4) must fit in 64 MiB, else CNTR_ENOMEM with nothing enqueued. Every
 * call on one GPU shares that GPU's array and leaves its contents for the
 * next: calls that overlap on one GPU (two streams, two threads) race.
 * Device-detected failures are reported by cntr_sync. */
cntr_status cntr_dyson_step_noalloc(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                                    const cntr_gf* Sigma, const void* const* eps, void* stream);

/* ------------------------------------------------------------------ F1 --
 * Dyson equation in integral form (Sec. "vie2: Dyson equation in integral
 * form", Tab. vie2; implementation Sec. "Implementation: vie2"):
 *   (1 + F) * G = Q  (Eq. vie2),  equivalently  G * (1 + F^ddagger) = Q,
 * for G and Q hermitian (Eq. ,masbX,. holds for the usual inputs, e.g.
 * F = -G0 * Sigma, F^ddagger = -Sigma * G0, Q = G0). F[i] is not hermitian:
 * Fcc[i] is its hermitian conjugate F^ddagger, which supplies the values
 * outside F's stored triangles (and vice versa). Layouts as for G; every
 * pointer is DEVICE memory, owned by the caller.
 *
 * cntr_vie2_matsubara: G^M + [F * G]^M = Q^M (Eq. vie2_langreth_m), the
 * convolution by Eqs. cm1 + cm2, as one dense (ntau+1) d system: an explicit
 * inverse (Gauss-Jordan, partial pivoting) and residual refinement to the
 * relative tolerance tol (<= 0: 1e-14) in at most max_iter rounds (<= 0:
 * 200). Reads F[i].mat and Q[i].mat, writes G[i].mat. Synchronizes the
 * stream (norm readbacks), so it may not be captured. Errors: CNTR_ESHAPE
 * (null pointers), CNTR_ESINGULAR, CNTR_ENOCONV, CNTR_ENOMEM.
 *
 * cntr_vie2_step:
 *  tstp <= k : start-up, slices 0..k (Tab. vie2 row vie2_start): retarded
 *              columns from the (k-m) d systems of Sec. "Start" with
 *              G^R_{m,m} = Q^R_{m,m}; mixing rows per tau index and lesser
 *              columns per n from the second-kind start-up rule
 *              (Eq. MBCVSAMx01_start, kernel F^R). Reads slices -1..k of G
 *              (G^M), F, Fcc and Q.
 *  tstp  > k : time step (row vie2_timestep): slice tstp from slices
 *              -1..tstp-1 of G, slices 0..tstp of F and Fcc, slice tstp of Q.
 *              Retarded row and mixing row by one step of Eq. MBCVSAMx01_t
 *              per column / tau index, the lesser column by one step of the
 *              conjugate equation per row (variant B; every row m < tstp is
 *              independent), then G^<_{tstp,tstp}.
 * Instances with nt < tstp are skipped; writes slice(s) of G[i] only.
 * Asynchronous on `stream`; uses the stream's step scratch (the size of the
 * Dyson step's). A singular local step matrix is reported by cntr_sync
 * (CNTR_ESINGULAR). Errors: CNTR_ESHAPE (null pointers, mixed d/k/ntau),
 * CNTR_EORDER (tstp outside 0..nt, or, with order checks on, slices missing). */
cntr_status cntr_vie2_matsubara(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* F,
                                const cntr_gf* Q, double tol, int32_t max_iter, void* stream);
cntr_status cntr_vie2_step(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* F,
                           const cntr_gf* Fcc, const cntr_gf* Q, void* stream);

/* ------------------------------------------------------------------ F2 --
 * Momentum-convolution self-energies of the k-space GW example (Sec.
 * "Example: GW for the translationally invariant Hubbard model", Eqs. Pol
 * and Sigmak), for a lattice of nk momenta k = 0..nk-1 (k + q, k - q taken
 * mod nk), element by element in the orbital indices:
 *   cntr_polarization_k: Pi_k(t,t')    = -(i/nk) sum_q G_{k+q}(t,t') G_q(t',t)
 *                        (Pi_{k,ij} from G_{k+q,ij} and G_{q,ji}),
 *   cntr_sigma_gw_k:     Sigma_k(t,t') =  (i/nk) sum_q G_{k-q}(t,t') dW_q(t,t')
 *                        (Sigma_{k,ij} from G_{k-q,ij} and dW_{q,ij}),
 * on the stored components of time slice tstp (tstp = -1: the Matsubara
 * component), by the Langreth rules of the two contour products (Eqs.
 * def_bubble1, def_bubble2; the Matsubara component from X^M(tau) =
 * -i X(-i tau, 0), the form in which X^rceil(0, tau) = i xi X^M(beta - tau):
 * Bubble1^M = -xi A^M(tau) B^M(beta - tau)^T, Bubble2^M = -A^M B^M), times
 * the real factor alpha (e.g. -U for the
 * kernel F = -U Pi of the screened interaction's integral equation, as the
 * paper's example multiplies Pol by U). G, dW hermitian (a lesser value
 * below the stored triangle is -[X^<(t',t)]^dagger; the stored X^<(t,t) is
 * used as it is); grids[0..nk-1] one grid
 * (d, k, ntau, nt, statistics of G). G[k], dW[k], Pi[k], Sigma[k]: DEVICE
 * contour functions of momentum k, owned by the caller; writes slice tstp
 * of Pi / Sigma only. Asynchronous on `stream`. Errors: CNTR_EINVAL
 * (nk > 1024, bad grid), CNTR_ESHAPE (null pointers, grids that differ),
 * CNTR_EORDER (tstp outside -1..nt). */
cntr_status cntr_polarization_k(int32_t tstp, int32_t nk, const cntr_grid* grids, const cntr_gf* G,
                                const cntr_gf* Pi, double alpha, void* stream);
cntr_status cntr_sigma_gw_k(int32_t tstp, int32_t nk, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* dW,
                            const cntr_gf* Sigma, double alpha, void* stream);

/* The same contour product for independent instances (no momentum sum):
 * C_i(t,t') = alpha i A_i(t,t') B_i(t,t') element by element (Eq.
 * def_bubble2; Matsubara: C^M = -alpha A^M B^M), on the stored components
 * of slice tstp, for count <= 65535
 * instances sharing d and ntau (e.g. the uMig self-energy i g g D0 G of each
 * impurity of a Holstein batch, Eq. uMig_el). A, B hermitian DEVICE contour
 * functions, C written on slice tstp only; asynchronous. Errors:
 * CNTR_ESHAPE (null pointers), CNTR_EORDER (tstp outside -1..nt). */
cntr_status cntr_bubble2_local(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* A,
                               const cntr_gf* B, const cntr_gf* C, double alpha, void* stream);

/* ------------------------------------------------------------------ F4 --
 * Pieces of the Holstein-model DMFT with the unrenormalized Migdal impurity
 * solver (Sec. "DMFT for the Holstein model"; the Bethe-lattice loop itself
 * is host code over these calls, cntr_sigma_gw_k and cntr_dyson_step).
 *
 * cntr_phonon_free: the free phonon propagator D0(z,z') = -i <T_C X(z) X(z')>_0
 *   of one mode X = a + a^dagger of frequency w0[i] > 0 at the grid's inverse
 *   temperature, into every component of D[i] (all slices 0..nt and the
 *   Matsubara branch): D0^R(t,t') = -2 sin(w0 (t - t')), D0^< and the mixing
 *   component from the Bose factor nB = 1/(e^{beta w0} - 1), D0^M(tau) =
 *   -[(1 + nB) e^{-w0 tau} + nB e^{w0 tau}]. grids: bosonic (sig = +1), d = 1;
 *   w0: HOST array of count values. Errors: CNTR_ESHAPE (d != 1, sig != +1,
 *   null pointers), CNTR_EINVAL (w0 <= 0).
 *
 * cntr_scale_slice: C = beta C + f(t) A(t,t') f(t') on slice tstp (tstp = -1:
 *   the Matsubara component, both times on the vertical branch, f(0^-)): the
 *   Bethe-lattice hybridization Delta = J G J (Eq. bethe_condition), the
 *   coupled propagator g D0 g of the uMig self-energy (Eq. uMig_el), and
 *   Delta + Sigma (f = 1, beta = 1). f[i]: DEVICE array of nt+2 real values,
 *   entry 0 on the Matsubara branch, entry n+1 at t_n. C may be A. With
 *   beta = 0 C is not read. Any d. Errors: CNTR_ESHAPE, CNTR_EORDER (tstp
 *   outside -1..nt).
 *
 * cntr_holstein_mf: the phonon displacement of Eq. X,
 *   X(t_n) = -2 g(0) n(0)/w0 + int_0^{t_n} D0^R(t_n,s) [g(s) n(s) - g(0) n(0)] ds,
 *   n(t) = 2 Im G^<(t,t) (both spins), by the library's quadrature of order k
 *   (start weights over slices 0..k for tstp <= k, Gregory weights beyond), and
 *   the mean-field level e0 + g(t_n) X(t_n) (Eq. H_mf_Holstein); tstp = -1:
 *   the equilibrium X(0^-) = -2 g(0^-) n / w0 with n = -2 G^M(beta^-). Writes
 *   X[i][tstp+1] and eps[i][tstp+1] (one complex value, the d = 1 level of
 *   the Dyson calls). g[i], X[i]: DEVICE arrays of nt+2 reals (same indexing
 *   as f above); eps[i]: DEVICE array of nt+2 complex values; w0: HOST array.
 *   Reads slices 0..max(tstp, k) of G. Errors: CNTR_ESHAPE (d != 1, null
 *   pointers), CNTR_EINVAL (w0 <= 0), CNTR_EORDER (tstp outside -1..nt). */
cntr_status cntr_phonon_free(int32_t count, const cntr_grid* grids, const cntr_gf* D, const double* w0,
                             void* stream);
cntr_status cntr_scale_slice(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* C,
                             const cntr_gf* A, const void* const* f, double beta, void* stream);
cntr_status cntr_holstein_mf(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             const void* const* g, const double* w0, double e0, void* const* X, void* const* eps,
                             void* stream);

/* ------------------------------------------------------------------ A8 --
 * Contour convolution C = A * f * B on time slice tstp (Eq. convolution,
 * Tab. convolution; discretised by Eqs. cm1, cm2, cr1, ctv1-ctv3,
 * cles1-cles3). A and B need not be hermitian: Acc and Bcc are their
 * hermitian conjugates A^ddagger, B^ddagger, used for values outside the
 * stored triangles (pass A and B again for hermitian inputs). f[i] is a
 * single-time function or NULL for f = 1 (f may itself be NULL). tstp = -1
 * computes the Matsubara component. tstp <= k reads slices 0..k of the
 * inputs; tstp > k reads slices 0..tstp. Writes slice tstp of C[i]. */
cntr_status cntr_convolution(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* C,
                             const cntr_gf* A, const cntr_gf* Acc, const cntr_gf* B,
                             const cntr_gf* Bcc, const void* const* f, void* stream);

/* ------------------------------------------------------------------ A9 --
 * Second-Born self-energy of the spin-symmetric Hubbard model on slice tstp
 * (Eq. sigma_hubb_2b): Sigma_ab(z,z') = U(z) U(z') G_ab(z,z')^2 G_ba(z',z),
 * elementwise in the orbital indices, every Keldysh component derived from
 * the contour product (Sigma^R = Sigma^> - Sigma^<, Eq. Cretmod); tstp = -1
 * gives the Matsubara component. When eps_mf is non-NULL the Hartree mean
 * field eps_mf_tstp = eps0_tstp + diag(U_tstp (n_i - nbar)) is also written
 * (Sec. "Hubbard chain"; n_i from the density matrix of slice tstp). Reads
 * slice tstp of G[i]; writes slice tstp of Sigma[i] (and eps_mf[i]). */
cntr_status cntr_sigma_2b(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                          const double* const* U, const cntr_gf* Sigma, const void* const* eps0,
                          void* const* eps_mf, double nbar, void* stream);

/* ----------------------------------------------------------------- A11 --
 * Batch-local self-energy on slice tstp (tstp = -1: Matsubara):
 *   Sigma = lam * (1/count) * sum_i G[i]
 * on every component, e.g. a lattice self-energy proportional to the local
 * Green's function G_loc = (1/N_k) sum_k G_k (the per-k Dyson problems of the
 * parallel k-point scheme, Sec. on MPI parallelisation, coupled only through
 * a local self-energy). All grids must agree. Sigma is ONE contour function
 * (the same one is then passed as the self-energy of every instance to
 * cntr_dyson_step). Reads slice tstp of every G[i]; writes slice tstp of
 * Sigma. */
cntr_status cntr_sigma_local(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             const cntr_gf* Sigma, double lam, void* stream);

/* ----------------------------------------------------------------- A13 --
 * Observables of slice tstp >= 0, per spin (density matrix and Eq.
 * Total_ener, the Galitskii-Migdal energy):
 *   rho = i xi G^<(t, t)                              (d x d)
 *   obs[5*i + 0] = Re Tr rho                          particle number
 *   obs[5*i + 1] = Re Tr[rho eps0(t)]                 one-body energy
 *   obs[5*i + 2] = Re Tr[rho eps_mf(t)]               (eps0 when eps_mf is NULL)
 *   obs[5*i + 3] = 1/2 Im Tr[Sigma * G]^<(t, t)       correlation energy
 *   obs[5*i + 4] = (obs[1] + obs[2]) / 2 + obs[3]     total energy
 * The convolution [Sigma * G]^<(t_n, t_n) uses the Gregory weights of the
 * time step (start weights for tstp <= k). eps0 / eps_mf: arrays of DEVICE
 * pointers as in cntr_sigma_2b (eps_mf may be NULL). obs: DEVICE array of
 * 5*count doubles; rho: DEVICE array of count d x d blocks, or NULL. Reads
 * slice tstp of G and Sigma. */
#define CNTR_NOBS 5
cntr_status cntr_observables(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             const cntr_gf* Sigma, const void* const* eps0, const void* const* eps_mf,
                             double* obs, void* rho, void* stream);

/* ------------------------------------------------------------------ F3 --
 * Free Green's function of a time-dependent single-particle Hamiltonian
 * (Sec. "Implementation: Free Green's functions", Eqs. cf4 and G0_free):
 *   G^M       the free Matsubara function of eps(0^-) - mu (as cntr_init_matsubara's g),
 *   G^R(t_n,t_j)      = -i U_n U_j^dag,
 *   G^<(t_j,t_n)      = -i xi U_j rho U_n^dag,
 *   G^rceil(t_n,tau)  = -i xi U_n R diag(f(x) e^{x tau}) R^dag,
 * with U_n = U_{n,0} from the fourth-order commutator-free exponential
 * U_{n+1,n} = exp[-i h (a1 e1 + a2 e2)] exp[-i h (a2 e1 + a1 e2)], e1,2 = eps - mu at
 * t_n + c1,2 h from the polynomial through the grid points n-k+1 .. n+1
 * (0 .. k while n < k-1); eps(0^-) - mu = R diag(x) R^dag, f(x) = 1/(e^{beta x} - xi),
 * rho = R diag(f(x)) R^dag. Inputs: eps[i] (DEVICE, (nt+2) d x d, entry 0 =
 * eps(0^-), entry n+1 = eps(t_n)), grids[i] (beta, mu, sig = xi, h, k). Output:
 * every component of G[i] for slices 0..nt (overwritten). Needs nt >= k, else
 * CNTR_EINVAL. Uses the stream's scratch (grown as needed); asynchronous. */
cntr_status cntr_green_from_H(int32_t count, const cntr_grid* grids, const cntr_gf* G, const void* const* eps,
                              void* stream);

/* ----------------------------------------------------------------- A12 --
 * Peierls substitution: the vector potential as a phase factor in the
 * hopping (Sec. "Example: GW for the translationally invariant Hubbard
 * model"), the differentiable drive of the adjoint workload:
 *   eps_n[a][b] = T_n[a][b] exp(i A_n Phi[a][b]),   n = -1..nt,
 * T[i]: DEVICE (nt+2) d x d complex blocks (the bare levels, index n+1),
 * Phi[i]: DEVICE d x d doubles (the phase pattern, e.g. +1 on a bond's
 * i+1 <- i element, -1 on its conjugate, 0 on site energies),
 * A[i]: DEVICE nt+2 doubles (index n+1; entry 0 is A(0^-)),
 * eps[i]: DEVICE output of (nt+2) d x d blocks. Asynchronous. */
cntr_status cntr_peierls(int32_t count, const cntr_grid* grids, const void* const* T, const double* const* Phi,
                         const double* const* A, void* const* eps, void* stream);
/* Its chain rule for a real objective J with eps_bar = dJ/dRe eps + i dJ/dIm
 * eps (the gradient convention of cntr_adjoint_sweep):
 *   A_bar[i][n+1] += Re sum_ab conj(eps_bar_n[a][b]) i Phi[a][b] eps_n[a][b]
 * (eps recomputed from T, Phi, A). A_bar[i]: DEVICE nt+2 doubles (+=). d <= 8. */
cntr_status cntr_peierls_grad(int32_t count, const cntr_grid* grids, const void* const* T,
                              const double* const* Phi, const double* const* A, const void* const* eps_bar,
                              double* const* A_bar, void* stream);

/* --------------------------------------------------------------- A10, A13 --/* --------------------------------------------------------------- A10, A13 --
 * Polynomial predictor T[G]_tstp -> T[G]_{tstp+1} (Eq. polyextrap, App.
 * "Extrapolation of contour functions"); needs tstp >= k. */
cntr_status cntr_extrapolate(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             void* stream);

/* Distance of two slices (Eq. distancenorm: sum of |A - B| over the slice)
 * and the norm of A's slice, written to out[2*i], out[2*i+1] (HOST array of
 * 2*count doubles). Synchronizes `stream`. */
cntr_status cntr_distance(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* A,
                          const cntr_gf* B, double* out, void* stream);

/* Copy slice tstp of src into dst (same grids). */
cntr_status cntr_copy_slice(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* dst,
                            const cntr_gf* src, void* stream);

/* Self-consistent second-Born + Hartree propagation (Sec. "Hubbard chain":
 * Matsubara loop, bootstrapping over slices 0..k, then predictor-corrector
 * time steps k+1..nt_stop) run by the library on `stream`:
 *   Matsubara : {Hartree, Sigma_2B, Matsubara solve} until the relative
 *               distance is below mats_tol (at most mats_maxit); the new
 *               input (Sigma^M, eps_mf_{-1}) is mixed with the previous one,
 *               x <- mats_mix x + (1 - mats_mix) x_prev, 0 < mats_mix <= 1
 *               (1 = plain iteration), which leaves the fixed point unchanged,
 *   bootstrap : {Hartree, Sigma_2B on 0..k, start-up} until below boot_tol
 *               and at least 3 iterations (at most boot_maxit),
 *   steps     : extrapolation, then `ncorr` corrector iterations
 *               {Hartree, Sigma_2B, time step} per slice.
 * G, Sigma, eps_mf are outputs (Sigma and eps_mf consistent with the final
 * G). Gscratch is a caller-owned contour function of the same grid used for
 * the convergence checks. stats (HOST, may be NULL) receives: Matsubara
 * iterations, bootstrap iterations, last Matsubara error, last bootstrap
 * error. */
cntr_status cntr_solve_2b(const cntr_grid* grid, const cntr_gf* G, const cntr_gf* Sigma,
                          const cntr_gf* Gscratch, const void* eps0, const double* U,
                          void* eps_mf, double nbar, int32_t mats_maxit, double mats_tol,
                          double mats_mix, int32_t boot_maxit, double boot_tol, int32_t ncorr,
                          int32_t nt_stop, double* stats, void* stream);

/* ----------------------------------------------------------------- A12 --
 * Discrete adjoint (reverse mode) of the Dyson solution: the start-up of
 * slices 0..k and the data-parallel time steps k+1..nt, exactly as
 * cntr_dyson_step computes them (Sec. "Dyson equation: start-up" and "Time
 * stepping"; the adjoint itself is not in the paper). The Matsubara
 * component M is held fixed; for a real objective J(G) the call returns the
 * gradients of J, with the convention dJ/dx + i dJ/dy for a complex entry
 * z = x + i y (so dJ = Re sum conj(grad) dz).
 *
 * Given self-energy (U == NULL): G(eps, Sigma, M) solves slices 0..nt;
 *   eps_bar += dJ/deps_n, Sigmabar += dJ/dSigma (if not NULL), Gbar.mat += dJ/dM.
 * Second-Born mode (U != NULL): Sigma = Sigma_2B[G; U] (as cntr_sigma_2b) and
 *   eps = eps0 + Hartree[G; U, nbar] on every slice -1..nt; G, Sigma and eps
 *   are the converged self-consistent solution (cntr_solve_2b; eps is its
 *   eps_mf), including the Matsubara component. Each slice's adjoint is the
 *   fixed point of the reverse step composed with the adjoints of Sigma_2B
 *   and Hartree, iterated `niter` times per slice (the start-up block of
 *   slices 0..k together); the Matsubara solve (Eq. Gmat_dyson_integ, its
 *   operator rebuilt and inverted at the converged Sigma^M) is reversed
 *   likewise, with 150 damped iterations (weight 1/2, as the forward loop).
 *   eps_bar += dJ/deps0_n and U_bar += dJ/dU_n for n = -1..nt (eps0_{-1}
 *   through a hermitian eigen-decomposition: its gradient is exact along
 *   hermitian directions). Gbar.mat returns dJ/dM with M held fixed (the
 *   seed of the equilibrium part). Sigmabar is required (work space; returns
 *   the total dJ/dSigma of slices 0..nt), U_bar is required.
 *
 *   G        : the converged solution (slices -1..nt) of the same grid.
 *   Sigma    : the self-energy the solution was computed with.
 *   eps      : the levels of the solution (eps_mf in the second-Born mode).
 *   U, nbar  : per problem DEVICE array of nt+2 doubles (as cntr_sigma_2b),
 *              and the Hartree shift, or U = NULL.
 *   Gbar     : in: dJ/dG of the objective's explicit dependence on slices
 *              0..nt (ret, les, tv) and on M (mat); out: mat += every
 *              slice's contribution (the total dJ/dM); ret, les and tv are
 *              consumed as work space (on return: intermediate adjoints).
 *   Sigmabar : accumulators (+=) of dJ/dSigma, slices 0..nt (mat untouched).
 *   eps_bar  : accumulators (+=) of (nt+2) blocks, entry n+1 for time n
 *              (entry 0, time -1, only in the second-Born mode).
 *   U_bar    : per problem DEVICE array of nt+2 doubles (+=), index n+1.
 *   niter    : fixed-point iterations per slice (<= 0: 10; each contracts the
 *              error by ~60x at the 2B chain's coupling).
 *   tol      : second-Born mode, tol > 0: CNTR_ENOCONV (after the sweep, whose
 *              outputs are then unreliable) when the largest relative change of
 *              a slice (or Matsubara) adjoint in its last iteration exceeds tol;
 *              tol <= 0: no check.
 *   conv     : HOST double or NULL: that largest relative change (second-Born
 *              mode).
 * Instances may have different nt (each is swept from its own nt). Every
 * pointer except conv is a DEVICE pointer, owned by the caller. Synchronizes
 * `stream`; CNTR_ESINGULAR if a local step or start-up matrix is singular. */
cntr_status cntr_adjoint_sweep(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                               const void* const* eps, const double* const* U, double nbar,
                               const cntr_gf* Gbar, const cntr_gf* Sigmabar, void* const* eps_bar,
                               double* const* U_bar, int32_t niter, double tol, double* conv, void* stream);

/* ----------------------------------------------------------------- A11 --
 * The same self-consistent second-Born + Hartree propagation for `count`
 * independent problems that share d, k and ntau (nt, beta, h, mu, eps0 and U
 * may differ): each problem's Matsubara loop runs on its own (it has its own
 * dense solve); the bootstrap and the time steps advance every problem in one
 * launch per kernel, each problem up to its own nt (problems whose nt is
 * reached drop out of the later launches). Loop controls as cntr_solve_2b;
 * the bootstrap tolerance applies to the largest relative distance of the
 * batch. Arrays of `count` descriptors / DEVICE pointers; stats (HOST, may be
 * NULL): largest Matsubara iteration count, bootstrap iterations, largest
 * last Matsubara error, last bootstrap error. Synchronizes `stream`. */
cntr_status cntr_solve_2b_batch(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                                const cntr_gf* Gscratch, const void* const* eps0, const double* const* U,
                                void* const* eps_mf, double nbar, int32_t mats_maxit, double mats_tol,
                                double mats_mix, int32_t boot_maxit, double boot_tol, int32_t ncorr,
                                double* stats, void* stream);

/* ----------------------------------------------------------------- A11 --
 * The same self-consistent propagation for problems of different orbital
 * counts (d, and k or ntau, may differ between problems). The problems are
 * grouped by (d, k, ntau); each group is solved as by cntr_solve_2b_batch on
 * a stream of its own (forked from `stream`, default priority, kept by the
 * library), and slice n of every group is enqueued in turn, so that the
 * groups' kernels run side by side on the device; `stream` waits for all
 * groups at the end. At most 16 groups. Arguments, loop controls and stats as
 * cntr_solve_2b_batch (stats: largest over the groups). Synchronizes `stream`
 * during the Matsubara and bootstrap loops. */
cntr_status cntr_solve_2b_uneven(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                                 const cntr_gf* Gscratch, const void* const* eps0, const double* const* U,
                                 void* const* eps_mf, double nbar, int32_t mats_maxit, double mats_tol,
                                 double mats_mix, int32_t boot_maxit, double boot_tol, int32_t ncorr,
                                 double* stats, void* stream);

/* ------------------------------------------------------------ profiling --/* ------------------------------------------------------------ profiling --
 * Device-time accounting of the time step, measured with HIP events
 * recorded on the stream each kernel is launched on. Between
 * cntr_profile_begin and cntr_profile_end every time step (n > k) records
 * events around its history-sum kernel and around the whole step. The
 * algorithmic counts per history launch at slice n are
 *   bytes = 16 d^2 [ n(n+1) + n (ntau+1) ]   (every stored R, <, rceil
 *           history block of slices 0..n-1 once; lesser part only for n > 2k)
 *   flops = 8 d^3 x (number of d x d block multiply-adds of the sums).
 * cntr_profile_end synchronizes the device. */
typedef struct {
  double hist_ms;       /* summed device time of the history-sum kernel */
  int64_t hist_launches;
  double hist_bytes;    /* summed algorithmic bytes of those launches */
  double hist_flops;    /* summed algorithmic flops of those launches */
  double step_ms;       /* summed device time of whole time steps */
  int64_t steps;
} cntr_profile;
cntr_status cntr_profile_begin(void);
/* The same, recording only every `every`-th time step (the 1st, the
 * (every+1)-th, ...), so that the events add little to the timed work; the
 * sums then cover the recorded steps only. every >= 1, else CNTR_EINVAL. */
cntr_status cntr_profile_begin_every(int32_t every);
cntr_status cntr_profile_end(cntr_profile* out);

/* --------------------------------------------------------------- graphs --
 * Capture of launch sequences into a HIP graph and its replay: the step
 * sequences of launch-bound runs (short grids, many problems) become one
 * graph launch. Between cntr_graph_begin(s) and cntr_graph_end(s, &g) the
 * calls that only enqueue work on s are recorded instead of executed:
 * cntr_dyson_step(_noalloc), cntr_sigma_2b, cntr_sigma_local,
 * cntr_extrapolate, cntr_copy_slice, cntr_convolution, cntr_observables,
 * cntr_green_from_H, cntr_peierls(_grad). Batch descriptors are then written
 * by kernels whose arguments carry them, and nothing is allocated: a call
 * whose scratch is not yet large enough returns CNTR_EINVAL (make the same
 * call once before capturing). Calls that synchronize (cntr_init_matsubara,
 * cntr_distance, cntr_solve_2b(_batch), cntr_adjoint_sweep, cntr_sync)
 * return CNTR_EINVAL during capture. s must not be the default (NULL)
 * stream. The graph refers to the device arrays and to the stream's scratch
 * as they were at capture time: keep them alive and do not make calls with
 * larger problems on that stream (which would reallocate its scratch) while
 * the graph is in use. cntr_graph_launch replays the graph on any stream. */
typedef struct cntr_graph_s* cntr_graph;
cntr_status cntr_graph_begin(void* stream);
cntr_status cntr_graph_end(void* stream, cntr_graph* out);
cntr_status cntr_graph_launch(cntr_graph graph, void* stream);
cntr_status cntr_graph_destroy(cntr_graph graph);

/* ---------------------------------------------------------------- tiles --
 * Term chunks of the history sums picked by an autotuner (the Python module
 * paper_1911_01211_amd.autotune times the candidates on the device and keeps
 * a cache): for problems of orbital count d, time steps at slices
 * n <= n_hi[0] use chunk tj[0], n <= n_hi[1] tj[1], ..., later slices the
 * last chunk. nbands = 0 restores the built-in chunk. Tunable: d = 1 (tj in
 * 32, 64, 128, 256; built-in 256) and d = 8 (16, 32, 64; built-in 64);
 * else CNTR_EINVAL. At most 8 bands, edges increasing. Process-wide; the
 * results change only in the summation order of the history sums. */
cntr_status cntr_set_tiles(int32_t d, int32_t nbands, const int32_t* n_hi, const int32_t* tj);

/* --------------------------------------------------------------- checks --/* --------------------------------------------------------------- checks --/* --------------------------------------------------------------- checks --
 * Optional checks of the preconditions of the Dyson equation (Tab. dyson:
 * the step at tstp needs slices -1..tstp-1 of G) and of the values, in the
 * spirit of the library's debug mode (Sec. "Compilation of libcntr"). Off by
 * default; process-wide.
 *  CNTR_CHECK_ORDER  : the library records, per instance (keyed by the
 *     device pointer G.ret), the last completed slice: cntr_init_matsubara
 *     sets it to -1, the start-up to k, a step at tstp to max(last, tstp),
 *     cntr_solve_2b(_batch) to the last slice computed. cntr_dyson_step(_noalloc)
 *     then returns CNTR_EORDER, with nothing enqueued, for an instance that
 *     is unknown or whose last completed slice is below tstp - 1 (below -1
 *     for the start-up). Instances filled by other means are declared with
 *     cntr_mark_slices. Records persist until cntr_mark_slices(.., -2),
 *     cntr_set_checks without the flag, or cntr_finalize; an allocation
 *     freed and reused for another instance keeps its record.
 *  CNTR_CHECK_FINITE : after every start-up or step a device check of the
 *     slices it wrote, the self-energy slices of the same index and eps;
 *     a non-finite value sets the problem's status word, reported as
 *     CNTR_ENONFINITE by cntr_sync. Costs one read of those slices.
 *  CNTR_CHECK_SYMMETRY : with every start-up or step a device check that the
 *     self-energy it reads is a hermitian contour function (Sec. "Contour
 *     Green's functions", the hermitian symmetry the Dyson solver assumes):
 *     the equal-time blocks Sigma^<_{n,n} and Sigma^R_{n,n} anti-hermitian at
 *     every slice the call reads (0..k for the start-up, tstp for a step),
 *     and for the start-up Sigma^M(tau) hermitian at every tau; a block
 *     with max|X + X^dag| > 1e-10 max|X| sets the problem's status word,
 *     reported as CNTR_ESYMMETRY by cntr_sync. */
#define CNTR_CHECK_ORDER 1
#define CNTR_CHECK_FINITE 2
#define CNTR_CHECK_SYMMETRY 4
cntr_status cntr_set_checks(int32_t flags);
/* Declare slices -1..last of `count` instances complete (last = -2 removes
 * the records). Host only; count >= 1, G non-NULL. */
cntr_status cntr_mark_slices(int32_t count, const cntr_gf* G, int32_t last);

/* ------------------------------------------------------------- plumbing -- */
/* Wait for `stream`; report a failure recorded by kernels since the last
 * check (CNTR_ESINGULAR, or CNTR_ENONFINITE with the finite check on; every
 * problem of the last step call on the stream is scanned) or a HIP error. */
cntr_status cntr_sync(void* stream);
/* Message for the last failing call of this thread ("" if none). */
const char* cntr_last_error(void);
/* Release library-owned device memory (scratch). Safe to call any time no
 * work is in flight; the library re-initialises on the next call. */
cntr_status cntr_finalize(void);
/* Library version string. */
const char* cntr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CNTR_H */
