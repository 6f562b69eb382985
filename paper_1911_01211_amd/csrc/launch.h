// Host-side launch interface between the C ABI layer (api.cpp) and the
// kernel files. All functions enqueue on `s` and return a hipError_t.
#pragma once
#include <vector>

#include "dev_common.h"

namespace cntr {

constexpr int NJOB = 8;  // history jobs of one time step

// Work plan of one time step n (identical for every problem of the call).
struct HistPlan {
  int n;
  int njob;
  int staged;       // history blocks staged through LDS (d = 1, 2, 4)
  int TJ, TM, TJS;  // term chunk, outputs per tile, tau-source chunk
  int tj[NJOB];     // term chunk of each job
  int tm[NJOB];     // outputs per tile of each job
  int mout[NJOB];
  int nch[NJOB];
  int mtiles[NJOB];
  int jorder[NJOB];      // job of each dispatch position
  int wg_off[NJOB + 1];  // first workgroup of each dispatch position
  // staged path: workgroups ordered by bands of stored slices, so that the
  // two consumers of a history block (jobs 0/4, 1/5, 3/7) run close together
  int banded;         // workgroups in band order (else job by job)
  int nband, wpb;     // bands (wpb unused)
  int bo[7];          // column tiles of the triangular panels and of the mixing panel
  int grid;           // history workgroups (without the set-up workgroup)
  long part_off[NJOB];  // in blocks
  // reduce tiles of the retarded, mixing and lesser rows; partial sums of
  // the lesser boundary rows, one set per reduce tile
  int red_tiles[3];
  int walk_tiles;     // one reduce workgroup per problem (REDUCE_WALK_MIN problems or more)
  int tau_shared;     // d = 1 batch sharing Sigma: tau source by k_tau_shared
  int fuse_t;         // d = 1: job 1 also forms the job-5 row sums (no job-5 workgroups)
  long tail_off;      // in blocks
  long total_blocks;  // scratch blocks of the step
  // d = 4: each stored panel (R, L, T) feeds its column and its row sums in
  // one pass (workgroup units of 16 du_nsb slices x DU_TT positions, after
  // the tau jobs' workgroups)
  int dual;
  int du_nsb;            // sub-tile rows of 16 slices per unit (1, 2, 4)
  int du_ns;             // slice chunks (all panels)
  int du_nt, du_ntau;    // position chunks of the triangular panels / of T
  int du_np;             // triangular panels with units: 1 (R), 2 (R, L)
  int du_full, du_part;  // units per triangular panel below the diagonal / meeting it
  int du_total;          // units per problem
  // Dyson equation in integral form: no Dyson set-up in the history kernel;
  // v2_rows x v2_nch workgroups of k_v2_side sum the lesser rows v2_lo.. in
  // chunks of v2_ch terms
  int vie2;
  int v2_lo, v2_rows, v2_ch, v2_nch;
  long v2_off, v2_doff;  // partials of those rows, and of G^<_{n,n} (in blocks)
};

// d = 4 one-pass units: positions per unit and the chunk bounds of the units
// of position chunk c of a triangular panel: slice chunks [lo, ns) meet the
// stored triangle s >= t; those from cf on lie entirely below the diagonal.
constexpr int DU_TT = 32;
// Reductions of the time step and of the integral-form step: from this many
// problems in one call on (one per compute unit), one workgroup per problem
// walks all of its tiles (the batch alone fills the chip, and there is no
// completion count); smaller batches get one workgroup per tile, since a
// walking batch would leave compute units idle while each walks its tiles
// (152 at d = 4 and slice 1000). Measured on the batched legs: 256 and 512
// problems of d = 1 run 23-30 % faster walking, 16 to 64 problems 3-10 %
// faster with a workgroup per tile.
constexpr int REDUCE_WALK_MIN = 256;
__host__ __device__ inline void du_range(int c, int TS, int ns, int& lo, int& cf) {
  lo = (c * DU_TT) / TS;
  cf = (c * DU_TT + DU_TT - 1 + TS - 1) / TS;
  if (lo > ns) lo = ns;
  if (cf > ns) cf = ns;
}

// event-based device timing of time steps (cntr_profile_begin/end)
struct ProfRec {
  hipEvent_t before, after_hist, after_step;
  double bytes, flops;
};
struct ProfState {
  bool on = false;
  int every = 1;   // record every every-th time step
  long seen = 0;   // time steps since cntr_profile_begin
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRec> rec;
};
extern ProfState g_prof;


// autotuned term chunks of the history jobs, per orbital count (see make_plan)
constexpr int TUNE_BANDS = 8;
struct TileTable {
  int nb = 0;
  int n_hi[TUNE_BANDS];
  int tj[TUNE_BANDS];
};
extern TileTable g_tiles[9];
bool tile_allowed(int d, int tj);

int hist_tm(int d);
// tau_split > 0: the tau source comes from k_tau_shared in tau_split chunks
// (no history workgroups for it)
// du_nsb > 0 fixes the unit height of the d = 4 one-pass path (else chosen
// from the number of units)
HistPlan make_plan(int n, int k, int ntau, int d, int tau_split = 0, int du_nsb = 0);
// scratch bytes (per problem) for the step at the largest n = nt
size_t step_scratch_bytes(int nt, int k, int ntau, int d);

// shared_sigma: every problem of the call has the same Sigma (pointer) and
// statistics; for d = 1 batches the tau source is then one product of the
// shared (Nτ+1) x (Nτ+1) operator with the problems' G^M
// record: the profiler may record events around the step (off for callers
// that must not create runtime objects)
hipError_t launch_step(const ProbArg& pa, const Scratch& sc, int n, int d, hipStream_t s,
                       bool shared_sigma = false, bool record = true);
hipError_t launch_start(const ProbArg& pa, const Scratch& sc, int d, int ntau, hipStream_t s);
// non-finite values in slices n0..n1 of G and Sigma or in eps_n0..n1 set the
// problem's status word to CNTR_ENONFINITE
hipError_t launch_check_finite(const ProbArg& pa, const Scratch& sc, int n0, int n1, int d, int ntau,
                               hipStream_t s);
// self-energy symmetry of slices n0..n1 (n0 = -1: also Sigma^M) sets the
// problem's status word to CNTR_ESYMMETRY
hipError_t launch_check_symmetry(const ProbArg& pa, const Scratch& sc, int n0, int n1, int ntau, hipStream_t s);
hipError_t launch_sigma2b(const ProbArg& pa, int n, int d, int nmax_elems, double nbar,
                          hipStream_t s);
hipError_t launch_extrapolate(const ProbArg& pa, int n, int d, int nelems, hipStream_t s);
hipError_t launch_distance(const ProbArg& pa, const ProbArg& pb, int n, int d, int nelems,
                           double* out_dev, hipStream_t s);
hipError_t launch_copy(const ProbArg& pdst, const ProbArg& psrc, int n, int d, int nelems,
                       hipStream_t s);
// f is taken from C's problem descriptor (Prob::f)
hipError_t launch_convolution(const ProbArg& C, const ProbArg& A, const ProbArg& Acc,
                              const ProbArg& B, const ProbArg& Bcc, int n, int d, int nelems,
                              hipStream_t s);

hipError_t launch_observables(const ProbArg& pa, int n, double* out, cplx* rho, hipStream_t s);
// Peierls phase of the hopping and its chain rule (entries n = -1..nt)
hipError_t launch_peierls(const cplx* T, const double* Phi, const double* A, cplx* eps, int d, int nt,
                          hipStream_t s);
hipError_t launch_peierls_grad(const cplx* T, const double* Phi, const double* A, const cplx* eps_bar,
                               double* A_bar, int d, int nt, hipStream_t s);
hipError_t launch_sigma_local(const ProbArg& pa, int n, int d, int nelems, double lam, hipStream_t s);

// Dyson equation in integral form, (1 + F) * G = Q: start-up (slices 0..k)
// and time step n > k (problem descriptors as described at Prob)
hipError_t launch_vie2_start(const ProbArg& pa, const Scratch& sc, int d, int ntau, hipStream_t s);
// side_ok: the step may run its side kernel on a forked stream
hipError_t launch_vie2_step(const ProbArg& pa, const Scratch& sc, int n, int d, hipStream_t s, bool side_ok = true);

// momentum-convolution bubbles of the k-space GW example: mode 1 the
// polarization of pg into po, mode 2 the self-energy of (pg, pw) into po;
// pg, pw, po: device descriptor arrays of nk momenta (<= 1024) sharing one
// grid (d, ntau, the statistics sig of G); the result times alpha
hipError_t launch_kbubble(int mode, const Prob* pg, const Prob* pw, const Prob* po, int nk, int d, int ntau,
                          int sig, int n, double alpha, hipStream_t s);
// C_i = alpha i A_i B_i (local Bubble2) on slice n for every instance
hipError_t launch_bubble2_local(const ProbArg& pa, const ProbArg& pb, const ProbArg& pc, int n, int d, int ntau,
                                double alpha, hipStream_t s);

// Holstein DMFT pieces (d = 1 for the phonon propagator and the displacement):
// the free propagator of X = a + a^dag into every component (w0 = P.par,
// bosonic grids); C = beta C + f A f on slice n (f = C's series U); the
// displacement X(t_n) (into P.aux) and the level e0 + g X (into P.eps_mf),
// g = P.U, w0 = P.par
hipError_t launch_phonon_free(const ProbArg& pa, int nt_max, int ntau, hipStream_t s);
hipError_t launch_scale_slice(const ProbArg& pc, const ProbArg& pa, int n, int d, int ntau, double beta,
                              hipStream_t s);
hipError_t launch_holstein_mf(const ProbArg& pg, int n, double e0, hipStream_t s);

// Matsubara pieces (per problem, one problem per call)
hipError_t launch_free_mat(const Prob& P, cplx* g, hipStream_t s);
// free Green's function of eps(t) into every component of P's G (scratch of
// free_green_scratch_bytes)
size_t free_green_scratch_bytes(int nt, int ntau, int d);
hipError_t launch_free_green(const Prob& P, void* scratch, hipStream_t s);
hipError_t launch_mat_conv(const Prob& P, const cplx* A, const cplx* B, const cplx* f,
                           cplx* out, hipStream_t s);
// sgn = -1: A = 1 - B[K] (Dyson, K = [g * Sigma]^M); sgn = +1: A = 1 + B[K]
hipError_t launch_mat_build(const Prob& P, const cplx* K, cplx* Amat, hipStream_t s, double sgn = -1.0);
// Fourier-series solve of the Matsubara equation into P.Gmat (P.Smat null: Sigma = 0),
// oversampling p (work: mats_fourier_scratch_bytes)
size_t mats_fourier_scratch_bytes(int ntau, int d, int p);
hipError_t launch_mats_fourier(const Prob& P, int p, cplx* work, hipStream_t s);
hipError_t launch_gj_inverse(int N, cplx* Amat, cplx* work, int* piv, int* status,
                             hipStream_t s);
// complex elements of the work buffer of launch_gj_inverse
size_t gj_work_elems(int N);
// The blocked inverse of B matrices of one size N <= GJ_BATCH_MAX_N side by
// side in one launch sequence (matrices N*N apart, work regions
// gj_work_elems(N) apart, pivots N apart, one status word each).
constexpr int GJ_BATCH_MAX_N = 2048;
hipError_t launch_gj_inverse_batch(int N, int B, cplx* A, cplx* work, int* piv, int* status, hipStream_t s);
// y = X v  (X: N x N, v, y: N x nrhs); y = b - X v when b != nullptr;
// zero2[0..1] = 0 when zero2 != nullptr (accumulators of a following norm)
hipError_t launch_matvec(int N, int nrhs, const cplx* X, const cplx* v, const cplx* b, cplx* y,
                         hipStream_t s, double* zero2 = nullptr);
hipError_t launch_mix(int len, cplx* x, cplx* keep, double a, bool first, hipStream_t s);
hipError_t launch_axpy_norm(int len, cplx* x, const cplx* dx, const cplx* r, const cplx* g,
                            double* norms, hipStream_t s);

}  // namespace cntr
