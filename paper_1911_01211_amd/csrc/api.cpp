// C ABI of the HIP Dyson time stepper: argument validation, library state
// (weight tables, per-stream scratch), and the host-side sequencing of the
// Matsubara solve and the self-consistent second-Born propagation.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"

namespace cntr {

__constant__ KW c_kw[KMAX + 1];

namespace {

thread_local std::string g_err;
std::mutex g_mu;
bool g_weights_ready[64] = {false};

// optional checks (cntr_set_checks): the last completed slice of every
// instance seen, keyed by its retarded-component pointer
int g_checks = 0;
std::map<const void*, int> g_last;

// Each stream's scratch starts with STAT_WORDS status words (one per problem
// of a call; a kernel that detects a failure writes its code there, cntr_sync
// reports and clears them), followed by the data region of the calls.
constexpr int STAT_WORDS = 65536;
constexpr size_t STAT_HEAD = STAT_WORDS * sizeof(int);
struct StreamScratch {
  char* buf = nullptr;
  size_t bytes = 0;  // of the data region
  int nstat = 0;     // status words written since the last cntr_sync (problems of the largest call)
  char* data() const { return buf + STAT_HEAD; }
  int* stat() const { return (int*)buf; }
  Prob* probs = nullptr;  // device copies of batched descriptors (5 sets)
  size_t nprob = 0;
  double* red = nullptr;  // reduction outputs
  size_t nred = 0;
  void* host = nullptr;   // pinned bounce buffer of the small read-backs
  // device copies of recently used descriptor arrays, found by content: a
  // repeated batch needs no upload (an upload from pageable memory holds the
  // host until the stream has drained, which would leave the GPU idle
  // between calls)
  struct Desc {
    std::vector<Prob> host;
    uint64_t hash = 0;
    Prob* dev = nullptr;
    size_t cap = 0;
    uint64_t used = 0;
  };
  std::vector<Desc> descs;
  uint64_t tick = 0;
};
constexpr size_t DESC_CACHE = 48;
constexpr size_t READBACK_MAX = 4096;
std::map<std::pair<int, hipStream_t>, StreamScratch> g_scratch;

// True while `s` is being captured into a graph: then nothing may allocate,
// synchronize or read host memory at replay time.
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

// descriptors of a batch travel in kernel arguments (no host buffer that a
// graph replay would have to read), NA_CHUNK per launch
constexpr int NA_CHUNK = 16;
struct ProbChunk {
  Prob p[NA_CHUNK];
  int count;
};
__global__ void k_put_probs(ProbChunk c, Prob* dst) {
  int i = threadIdx.x;
  if (i < c.count) dst[i] = c.p[i];
}

// Descriptors of count problems to dst, through kernel arguments.
hipError_t put_probs(const Prob* v, int count, Prob* dst, hipStream_t s) {
  for (int i0 = 0; i0 < count; i0 += NA_CHUNK) {
    ProbChunk c;
    c.count = count - i0 < NA_CHUNK ? count - i0 : NA_CHUNK;
    for (int i = 0; i < c.count; i++) c.p[i] = v[i0 + i];
    k_put_probs<<<1, 64, 0, s>>>(c, dst + i0);
  }
  return hipGetLastError();
}

cntr_status fail(cntr_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

cntr_status hip_fail(hipError_t e, const char* where) {
  return fail(CNTR_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

cntr_status ensure_weights() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev < 64 && g_weights_ready[dev]) return CNTR_OK;
  KW host[KMAX + 1];
  std::memset(host, 0, sizeof(host));
  for (int k = 1; k <= KMAX; k++) make_weights(k, &host[k]);
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_kw), host, sizeof(host), 0, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "weight upload");
  if (dev < 64) g_weights_ready[dev] = true;
  return CNTR_OK;
}

StreamScratch* scratch_for(hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  return &g_scratch[{dev, s}];
}

// Small device-to-host read-back on stream s (waits for the stream): through
// a pinned buffer, so that the copy is a plain DMA of the stream.
cntr_status readback(hipStream_t s, void* dst, const void* src, size_t bytes, const char* what) {
  if (bytes > READBACK_MAX) return fail(CNTR_EINVAL, std::string(what) + ": read-back too large");
  StreamScratch* sc = scratch_for(s);
  if (!sc->host && hipHostMalloc(&sc->host, READBACK_MAX, hipHostMallocDefault) != hipSuccess) {
    sc->host = nullptr;
    return fail(CNTR_ENOMEM, "pinned read-back buffer");
  }
  hipError_t e = hipMemcpyAsync(sc->host, src, bytes, hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return hip_fail(e, what);
  std::memcpy(dst, sc->host, bytes);
  return CNTR_OK;
}

cntr_status grow(hipStream_t s, StreamScratch* sc, size_t bytes, size_t nprob, size_t nred) {
  if ((bytes > sc->bytes || nprob > sc->nprob || nred > sc->nred) && capturing(s))
    return fail(CNTR_EINVAL, "the call would allocate scratch during graph capture: make the same call once "
                             "before capturing");
  if (bytes > sc->bytes) {
    if (sc->buf) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(sc->buf);
    }
    sc->buf = nullptr;
    size_t nb = bytes + bytes / 4;
    if (hipMalloc(&sc->buf, nb + STAT_HEAD) != hipSuccess) {
      sc->bytes = 0;
      return fail(CNTR_ENOMEM, "scratch allocation failed");
    }
    sc->bytes = nb;
    sc->nstat = 0;
    if (hipMemsetAsync(sc->buf, 0, nb + STAT_HEAD, s) != hipSuccess) return fail(CNTR_EHIP, "scratch clear");
  }
  if (nprob > sc->nprob) {
    if (sc->probs) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(sc->probs);
    }
    sc->probs = nullptr;
    if (hipMalloc(&sc->probs, nprob * sizeof(Prob)) != hipSuccess) {
      sc->nprob = 0;
      return fail(CNTR_ENOMEM, "descriptor allocation failed");
    }
    sc->nprob = nprob;
  }
  if (nred > sc->nred) {
    if (sc->red) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(sc->red);
    }
    sc->red = nullptr;
    if (hipMalloc(&sc->red, nred * sizeof(double)) != hipSuccess) {
      sc->nred = 0;
      return fail(CNTR_ENOMEM, "reduction buffer allocation failed");
    }
    sc->nred = nred;
  }
  return CNTR_OK;
}

cntr_status check_grid(const cntr_grid& g, const char* what) {
  char buf[256];
  if (g.k < 1 || g.k > KMAX) {
    snprintf(buf, sizeof buf, "%s: order k=%d outside 1..%d", what, g.k, KMAX);
    return fail(CNTR_EINVAL, buf);
  }
  if (g.d < 1 || g.d > 8) {
    snprintf(buf, sizeof buf, "%s: orbital dimension d=%d outside 1..8", what, g.d);
    return fail(CNTR_EINVAL, buf);
  }
  if (g.ntau < 2 * g.k + 2) {
    snprintf(buf, sizeof buf, "%s: ntau=%d < 2k+2=%d", what, g.ntau, 2 * g.k + 2);
    return fail(CNTR_EINVAL, buf);
  }
  if (g.nt < g.k) {
    snprintf(buf, sizeof buf, "%s: nt=%d < k=%d", what, g.nt, g.k);
    return fail(CNTR_EINVAL, buf);
  }
  if (g.sig != 1 && g.sig != -1) return fail(CNTR_EINVAL, std::string(what) + ": sig must be +1 or -1");
  if (!(g.h > 0) || !(g.beta > 0) || !std::isfinite(g.mu))
    return fail(CNTR_EINVAL, std::string(what) + ": h and beta must be positive, mu finite");
  return CNTR_OK;
}

cntr_status check_batch(int count, const cntr_grid* grids, const char* what) {
  if (count < 1 || grids == nullptr) return fail(CNTR_ESHAPE, std::string(what) + ": empty batch");
  for (int i = 0; i < count; i++) {
    cntr_status st = check_grid(grids[i], what);
    if (st != CNTR_OK) return st;
    if (grids[i].d != grids[0].d || grids[i].k != grids[0].k || grids[i].ntau != grids[0].ntau)
      return fail(CNTR_ESHAPE, std::string(what) + ": instances of one call must share d, k and ntau");
  }
  return CNTR_OK;
}

bool gf_ok(const cntr_gf* g, int count) {
  if (!g) return false;
  for (int i = 0; i < count; i++)
    if (!g[i].mat || !g[i].ret || !g[i].les || !g[i].tv) return false;
  return true;
}

Prob make_prob(const cntr_grid& g, const cntr_gf* G, const cntr_gf* S, const void* eps) {
  Prob p{};
  p.nt = g.nt;
  p.ntau = g.ntau;
  p.d = g.d;
  p.sig = g.sig;
  p.k = g.k;
  p.beta = g.beta;
  p.h = g.h;
  p.mu = g.mu;
  p.htau = g.beta / g.ntau;
  if (G) {
    p.Gmat = (cplx*)G->mat;
    p.Gret = (cplx*)G->ret;
    p.Gles = (cplx*)G->les;
    p.Gtv = (cplx*)G->tv;
  }
  if (S) {
    p.Smat = (cplx*)S->mat;
    p.Sret = (cplx*)S->ret;
    p.Sles = (cplx*)S->les;
    p.Stv = (cplx*)S->tv;
  }
  p.eps = (const cplx*)eps;
  return p;
}

// ProbArg for `count` descriptors; batches are copied to device slot `slot`.
static uint64_t desc_hash(const std::vector<Prob>& v) {
  const unsigned char* b = (const unsigned char*)v.data();
  size_t n = v.size() * sizeof(Prob), nw = n / 8;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < nw; i++) {
    uint64_t w;
    std::memcpy(&w, b + 8 * i, 8);
    h = (h ^ w) * 1099511628211ull;
  }
  for (size_t i = 8 * nw; i < n; i++) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

cntr_status make_arg(hipStream_t s, StreamScratch* sc, const std::vector<Prob>& v, int slot,
                     ProbArg* out) {
  out->one = v[0];
  out->count = (int)v.size();
  out->many = nullptr;
  if (v.size() > 1 && !capturing(s)) {
    size_t bytes = v.size() * sizeof(Prob);
    uint64_t h = desc_hash(v);
    for (auto& e : sc->descs)
      if (e.hash == h && e.host.size() == v.size() && std::memcmp(e.host.data(), v.data(), bytes) == 0) {
        e.used = ++sc->tick;
        out->many = e.dev;
        return CNTR_OK;
      }
    StreamScratch::Desc* e = nullptr;
    if (sc->descs.size() < DESC_CACHE) {
      sc->descs.emplace_back();
      e = &sc->descs.back();
    } else {
      e = &sc->descs[0];
      for (auto& x : sc->descs)
        if (x.used < e->used) e = &x;
    }
    if (e->cap < v.size()) {
      if (e->dev) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(e->dev);
      }
      e->dev = nullptr;
      e->cap = 0;
      if (hipMalloc(&e->dev, bytes) != hipSuccess) {
        e->host.clear();
        e->hash = 0;
        return fail(CNTR_ENOMEM, "descriptor allocation failed");
      }
      e->cap = v.size();
    }
    // (a reused copy is overwritten in stream order, after the kernels that
    // read it)
    hipError_t err = hipMemcpyAsync(e->dev, v.data(), bytes, hipMemcpyHostToDevice, s);
    if (err != hipSuccess) {
      e->host.clear();
      e->hash = 0;
      return hip_fail(err, "descriptor upload");
    }
    e->host = v;
    e->hash = h;
    e->used = ++sc->tick;
    out->many = e->dev;
    return CNTR_OK;
  }
  if (v.size() > 1) {
    Prob* dst = sc->probs + slot * (sc->nprob / 5);
    hipError_t e = capturing(s) ? put_probs(v.data(), (int)v.size(), dst, s)
                                : hipMemcpyAsync(dst, v.data(), v.size() * sizeof(Prob), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    out->many = dst;
  }
  return CNTR_OK;
}

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

struct StepScratch {
  Scratch sc;
  size_t per;
};

// the step layout depends on the grid shape and the tile table; every step
// call needs it, so it is computed once per shape (and table version)
static int g_tiles_gen = 0;
StepScratch step_layout_uncached(const cntr_grid& g);
StepScratch step_layout(const cntr_grid& g) {
  static std::mutex mu;
  static std::map<std::array<int, 5>, StepScratch> memo;
  std::array<int, 5> key;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    key = {g.nt, g.k, g.ntau, g.d, g_tiles_gen};
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  if (memo.size() > 256) memo.clear();
  StepScratch r = step_layout_uncached(g);
  memo[key] = r;
  return r;
}

StepScratch step_layout_uncached(const cntr_grid& g) {
  StepScratch r{};
  size_t dd = (size_t)g.d * g.d;
  r.sc.off_status = 0;
  r.sc.off_minv = 256;
  // step inverses (KMAX + 2 blocks), the boundary-row source terms (KMAX + 1,
  // one spare) and the boundary-row operator ((KMAX + 1)(KMAX + 2) / 2)
  r.sc.off_part = 256 + round256((2 * KMAX + 4 + (KMAX + 1) * (KMAX + 2) / 2) * dd * sizeof(cplx));
  r.sc.off_tail = r.sc.off_part;
  r.per = r.sc.off_part + round256(step_scratch_bytes(g.nt, g.k, g.ntau, g.d));
  r.sc.stride = r.per;
  return r;
}

long slice_elems(const cntr_grid& g, int n) {
  long dd = (long)g.d * g.d;
  if (n < 0) return (g.ntau + 1) * dd;
  return (2L * (n + 1) + g.ntau + 1) * dd;
}

// ------------------------------------------------------- order checks
// With CNTR_CHECK_ORDER: the step at tstp needs slices -1..tstp-1 of every
// instance (Tab. dyson); the start-up needs the Matsubara component.
cntr_status order_check(int tstp, int k, int count, const cntr_gf* G, const char* what) {
  if (!(g_checks & CNTR_CHECK_ORDER)) return CNTR_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < count; i++) {
    auto it = g_last.find(G[i].ret);
    int need = tstp <= k ? -1 : tstp - 1;
    if (it == g_last.end() || it->second < need) {
      char buf[256];
      snprintf(buf, sizeof buf, "%s: instance %d has slices up to %d, slice %d needs slices -1..%d", what, i,
               it == g_last.end() ? -2 : it->second, tstp, need);
      return fail(CNTR_EORDER, buf);
    }
  }
  return CNTR_OK;
}
// records slices -1..last as complete (only when order checks are on; an
// instance is entered by the Matsubara solve or cntr_mark_slices)
void order_mark(int count, const cntr_gf* G, int last, bool create) {
  if (!(g_checks & CNTR_CHECK_ORDER)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < count; i++) {
    auto it = g_last.find(G[i].ret);
    if (it != g_last.end()) {
      if (create || last > it->second) it->second = last;
    } else if (create) {
      g_last[G[i].ret] = last;
    }
  }
}

// ------------------------------------------------- Matsubara solve state
struct MatsState {
  int N = 0, d = 0;
  cplx *g = nullptr, *K = nullptr, *A = nullptr, *Ainv = nullptr, *r = nullptr, *dx = nullptr,
       *work = nullptr, *smix = nullptr, *emix = nullptr;
  int* piv = nullptr;
  int* status = nullptr;
  double* norms = nullptr;
  bool have_inv = false;
  cntr_status alloc(int ntau, int dd) {
    d = dd;
    N = (ntau + 1) * dd;
    size_t bs = (size_t)(ntau + 1) * dd * dd * sizeof(cplx);
    size_t nn = (size_t)N * N * sizeof(cplx);
    size_t vec = (size_t)N * dd * sizeof(cplx);
    if (hipMalloc(&g, bs) || hipMalloc(&K, bs) || hipMalloc(&A, nn) || hipMalloc(&Ainv, nn) ||
        hipMalloc(&r, vec) || hipMalloc(&dx, vec) || hipMalloc(&work, gj_work_elems(N) * sizeof(cplx)) ||
        hipMalloc(&piv, N * sizeof(int)) || hipMalloc(&status, sizeof(int)) ||
        hipMalloc(&norms, 2 * sizeof(double)) || hipMalloc(&smix, bs) ||
        hipMalloc(&emix, (size_t)dd * dd * sizeof(cplx))) {
      release();
      return fail(CNTR_ENOMEM, "Matsubara workspace allocation failed");
    }
    return CNTR_OK;
  }
  void release() {
    for (void* p : {(void*)g, (void*)K, (void*)A, (void*)Ainv, (void*)r, (void*)dx, (void*)work,
                    (void*)piv, (void*)status, (void*)norms, (void*)smix, (void*)emix})
      if (p) (void)hipFree(p);
    g = K = A = Ainv = r = dx = work = smix = emix = nullptr;
    piv = status = nullptr;
    norms = nullptr;
    have_inv = false;
  }
  ~MatsState() { release(); }
};

cntr_status mats_refine(MatsState& st, const Prob& P, bool use_guess, double tol, int max_iter,
                        hipStream_t s, int* iters);

// Operators, right-hand sides and inverses of B Matsubara problems of one
// size side by side, for one batched inverse launch sequence.
struct MatsGroup {
  int N = 0, B = 0;
  size_t ws = 0, gs = 0;
  cplx *g = nullptr, *A = nullptr, *Ainv = nullptr, *work = nullptr;
  int *piv = nullptr, *status = nullptr;
  cntr_status alloc(int ntau, int dd, int b) {
    N = (ntau + 1) * dd;
    B = b;
    ws = gj_work_elems(N);
    gs = (size_t)(ntau + 1) * dd * dd;
    size_t nn = (size_t)N * N;
    if (hipMalloc(&g, B * gs * sizeof(cplx)) || hipMalloc(&A, B * nn * sizeof(cplx)) ||
        hipMalloc(&Ainv, B * nn * sizeof(cplx)) || hipMalloc(&work, B * ws * sizeof(cplx)) ||
        hipMalloc(&piv, (size_t)B * N * sizeof(int)) || hipMalloc(&status, (size_t)B * sizeof(int))) {
      release();
      return fail(CNTR_ENOMEM, "Matsubara batch workspace allocation failed");
    }
    return CNTR_OK;
  }
  void release() {
    for (void* p : {(void*)g, (void*)A, (void*)Ainv, (void*)work, (void*)piv, (void*)status})
      if (p) (void)hipFree(p);
    g = A = Ainv = work = nullptr;
    piv = status = nullptr;
  }
  ~MatsGroup() { release(); }
};

// A MatsState that borrows the memory of a group and of a state (frees nothing)
struct MatsView : MatsState {
  ~MatsView() {
    g = K = A = Ainv = r = dx = work = smix = emix = nullptr;
    piv = status = nullptr;
    norms = nullptr;
  }
};

// Matsubara solves of count problems of one size: build(i, A, g) enqueues
// problem i's operator into A and its right-hand side into g and returns its
// descriptor. The operators of a group (at most 256, at most 2 GiB of
// matrices) are inverted by one batched launch sequence, then each problem
// is refined with its own inverse (the inverse and the refinement of a
// single solve, so the results are those of the one-problem path).
template <class Build>
static cntr_status mats_solve_batch(int count, MatsState& ms, int ntau, Build build, double tol, int max_iter,
                                    hipStream_t s) {
  int N = ms.N, d = ms.d;
  size_t nn = (size_t)N * N;
  size_t fit = ((size_t)2 << 30) / (2 * nn * sizeof(cplx));
  int gmax = (int)std::max<size_t>(1, std::min<size_t>(256, fit));
  for (int i0 = 0; i0 < count; i0 += gmax) {
    int B = std::min(gmax, count - i0);
    MatsGroup grp;
    cntr_status st = grp.alloc(ntau, d, B);
    if (st) return st;
    std::vector<Prob> P(B);
    hipError_t e = hipSuccess;
    for (int b = 0; b < B && e == hipSuccess; b++) e = build(i0 + b, grp.A + b * nn, grp.g + b * grp.gs, &P[b]);
    if (e != hipSuccess) return hip_fail(e, "Matsubara operators");
    if ((e = hipMemcpyAsync(grp.Ainv, grp.A, B * nn * sizeof(cplx), hipMemcpyDeviceToDevice, s)) ||
        (e = hipMemsetAsync(grp.status, 0, (size_t)B * sizeof(int), s)) ||
        (e = launch_gj_inverse_batch(N, B, grp.Ainv, grp.work, grp.piv, grp.status, s)))
      return hip_fail(e, "batched inverse");
    std::vector<int> stat(B);
    if ((st = readback(s, stat.data(), grp.status, (size_t)B * sizeof(int), "inverse status"))) return st;
    for (int b = 0; b < B; b++)
      if (stat[b] != 0) return fail(CNTR_ESINGULAR, "singular Matsubara operator");
    for (int b = 0; b < B; b++) {
      MatsView v;
      v.N = N;
      v.d = d;
      v.g = grp.g + b * grp.gs;
      v.K = ms.K;
      v.A = grp.A + b * nn;
      v.Ainv = grp.Ainv + b * nn;
      v.r = ms.r;
      v.dx = ms.dx;
      v.work = grp.work + b * grp.ws;
      v.piv = grp.piv + (size_t)b * N;
      v.status = grp.status + b;
      v.norms = ms.norms;
      v.have_inv = true;
      if ((st = mats_refine(v, P[b], false, tol, max_iter, s, nullptr))) return st;
    }
  }
  return CNTR_OK;
}

// Solve the discrete Matsubara equation for P (eps = eps_{-1} at entry 0,
// Sigma^M in P.Smat) into P.Gmat. The current P.Gmat is the initial guess
// when use_guess; the inverse of an earlier operator is reused when present.
// The refinement of mats_solve for an operator in st.A and a right-hand side
// in st.g (the current P.Gmat is the initial guess when use_guess, else st.g).
cntr_status mats_refine(MatsState& st, const Prob& P, bool use_guess, double tol, int max_iter,
                        hipStream_t s, int* iters);

cntr_status mats_solve(MatsState& st, const Prob& P, bool use_guess, double tol, int max_iter,
                       hipStream_t s, int* iters) {
  hipError_t e;
  if ((e = launch_free_mat(P, st.g, s))) return hip_fail(e, "free Matsubara function");
  if ((e = launch_mat_conv(P, st.g, P.Smat, nullptr, st.K, s))) return hip_fail(e, "[g*Sigma]^M");
  if ((e = launch_mat_build(P, st.K, st.A, s))) return hip_fail(e, "Matsubara operator");
  return mats_refine(st, P, use_guess, tol, max_iter, s, iters);
}

cntr_status mats_refine(MatsState& st, const Prob& P, bool use_guess, double tol, int max_iter,
                        hipStream_t s, int* iters) {
  hipError_t e;
  int N = st.N, d = st.d;
  size_t vec = (size_t)N * d * sizeof(cplx);
  if (!use_guess && (e = hipMemcpyAsync(P.Gmat, st.g, vec, hipMemcpyDeviceToDevice, s)))
    return hip_fail(e, "initial guess");
  double prev = -1;
  int since_inv = 0;
  for (int it = 0; it < max_iter; it++) {
    if ((e = launch_matvec(N, d, st.A, P.Gmat, st.g, st.r, s, st.norms))) return hip_fail(e, "residual");
    if ((e = launch_axpy_norm(N * d, P.Gmat, nullptr, st.r, st.g, st.norms, s))) return hip_fail(e, "norm");
    double nrm[2];
    cntr_status rs = readback(s, nrm, st.norms, sizeof nrm, "norm readback");
    if (rs) return rs;
    double rel = std::sqrt(nrm[0] / (nrm[1] > 0 ? nrm[1] : 1.0));
    if (!std::isfinite(rel)) return fail(CNTR_ENONFINITE, "non-finite Matsubara residual");
    if (iters) *iters = it;
    if (rel <= tol) return CNTR_OK;
    // the inverse is formed when first needed, and refreshed when the
    // refinement stops contracting
    if (st.have_inv && since_inv >= 2 && prev > 0 && rel > 0.25 * prev) st.have_inv = false;
    if (!st.have_inv) {
      if ((e = hipMemsetAsync(st.status, 0, sizeof(int), s))) return hip_fail(e, "status clear");
      if ((e = hipMemcpyAsync(st.Ainv, st.A, (size_t)N * N * sizeof(cplx), hipMemcpyDeviceToDevice, s)))
        return hip_fail(e, "operator copy");
      if ((e = launch_gj_inverse(N, st.Ainv, st.work, st.piv, st.status, s))) return hip_fail(e, "inverse");
      int stat = 0;
      if ((rs = readback(s, &stat, st.status, sizeof(int), "inverse status"))) return rs;
      if (stat != 0) return fail(CNTR_ESINGULAR, "singular Matsubara operator");
      st.have_inv = true;
      since_inv = 0;
      prev = -1;
    }
    prev = rel;
    since_inv++;
    if ((e = launch_matvec(N, d, st.Ainv, st.r, nullptr, st.dx, s, st.norms))) return hip_fail(e, "correction");
    if ((e = launch_axpy_norm(N * d, P.Gmat, st.dx, st.r, st.g, st.norms, s))) return hip_fail(e, "update");
  }
  return fail(CNTR_ENOCONV, "Matsubara refinement did not reach its tolerance");
}

// Matsubara loop of the second-Born run of one problem (P, with its scratch
// copy in po): {Hartree + Sigma_2B on slice -1, mixing of that input with the
// previous one, Matsubara solve} until the relative distance of G^M is below
// tol (at most maxit). G^M starts as the free function of eps0_{-1}.
cntr_status mats_loop_2b(const cntr_grid& g, const Prob& P, const ProbArg& pa, const ProbArg& po,
                         StreamScratch* sc, double nbar, int maxit, double tol, double mix, hipStream_t s,
                         int* iters, double* err_out) {
  int d = g.d;
  hipError_t e;
  cntr_status st;
  MatsState ms;
  if ((st = ms.alloc(g.ntau, d))) return st;
  Prob P0 = P;
  P0.eps = P.eps0;
  int it = 0;
  double err = 0, dist[2];
  if ((e = launch_free_mat(P0, P.Gmat, s))) {
    ms.release();
    return hip_fail(e, "initial G^M");
  }
  for (it = 0; it < maxit; it++) {
    if ((e = launch_sigma2b(pa, -1, d, (int)slice_elems(g, -1), nbar, s)) ||
        (e = launch_mix((g.ntau + 1) * d * d, P.Smat, ms.smix, mix, it == 0, s)) ||
        (e = launch_mix(d * d, P.eps_mf, ms.emix, mix, it == 0, s)) ||
        (e = launch_copy(po, pa, -1, d, (int)slice_elems(g, -1), s))) {
      ms.release();
      return hip_fail(e, "Matsubara loop");
    }
    // inexact inner solves: the refinement stops three orders of magnitude
    // below the last outer distance (at most 1e-8, at least 1e-15); the
    // fixpoint and the final accuracy are those of exact inner solves
    double itol = std::min(1e-8, std::max(1e-15, 1e-3 * (it == 0 ? 1.0 : err)));
    if ((st = mats_solve(ms, P, true, itol, 200, s, nullptr))) {
      ms.release();
      return st;
    }
    e = hipMemsetAsync(sc->red, 0, 2 * sizeof(double), s);
    if (!e) e = launch_distance(pa, po, -1, d, (int)slice_elems(g, -1), sc->red, s);
    if (e) {
      ms.release();
      return hip_fail(e, "distance");
    }
    if ((st = readback(s, dist, sc->red, 2 * sizeof(double), "distance"))) {
      ms.release();
      return st;
    }
    err = dist[0] / dist[1];
    if (err < tol) {
      it++;
      break;
    }
  }
  ms.release();
  *iters = it;
  *err_out = err;
  return CNTR_OK;
}

// ------------------------------------------------- allocation-free step
// Scratch of cntr_dyson_step_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends. In host code `scratch` names a host-side
// stand-in, so every host use goes through the device address obtained once
// per device with hipGetSymbolAddress (g_na_ptr). Layout: descriptor slots of
// NA_MAX_PROBS problems, then the per-problem step regions (status word and
// completion counter at the start of each region, as in the stream scratch).
constexpr size_t NA_STEP_BYTES = (size_t)64 << 20;
constexpr int NA_MAX_PROBS = 256;
constexpr size_t NA_DESC_BYTES = (NA_MAX_PROBS * sizeof(Prob) + 255) / 256 * 256;
constexpr size_t NA_STAT_BYTES = NA_MAX_PROBS * sizeof(int);
__device__ __align__(256) char scratch[NA_DESC_BYTES + NA_STAT_BYTES + NA_STEP_BYTES];

char* g_na_ptr[64] = {nullptr};
int g_na_nstat[64] = {0};  // status words written since the last cntr_sync

__global__ void k_zero_words(int* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Device address of `scratch` on the current device (set up on first use:
// symbol address, status words cleared by a kernel).
cntr_status noalloc_setup(hipStream_t s, char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(CNTR_EINVAL, "cntr_dyson_step_noalloc: device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_na_ptr[dev]) {
    char* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    k_zero_words<<<1024, 256, 0, s>>>((int*)ptr, sizeof(scratch) / sizeof(int));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "scratch clear");
    g_na_ptr[dev] = ptr;
  }
  *out = g_na_ptr[dev];
  return CNTR_OK;
}

// first failure code among the status words of the allocation-free calls on
// the current device since the last check (0 when none); clears them
cntr_status noalloc_status(int* code) {
  *code = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return CNTR_OK;
  char* ptr;
  int cnt;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    ptr = g_na_ptr[dev];
    cnt = g_na_nstat[dev];
    g_na_nstat[dev] = 0;
  }
  if (!ptr || cnt == 0) return CNTR_OK;
  int codes[NA_MAX_PROBS];
  hipError_t e = hipMemcpy(codes, ptr + NA_DESC_BYTES, cnt * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "status readback");
  for (int i = 0; i < cnt && !*code; i++) *code = codes[i];
  if (*code != 0) {
    for (int i = 0; i < cnt; i++) codes[i] = 0;
    (void)hipMemcpy(ptr + NA_DESC_BYTES, codes, cnt * sizeof(int), hipMemcpyHostToDevice);
  }
  return CNTR_OK;
}

}  // namespace
}  // namespace cntr

using namespace cntr;

extern "C" {

const char* cntr_version(void) { return "cntr-gfx950 0.1"; }

cntr_status cntr_profile_begin(void) { return cntr_profile_begin_every(1); }

cntr_status cntr_profile_begin_every(int32_t every) {
  if (every < 1) return fail(CNTR_EINVAL, "cntr_profile_begin_every: every < 1");
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof.on = true;
  g_prof.every = every;
  g_prof.seen = 0;
  g_prof.used = 0;
  g_prof.rec.clear();
  return CNTR_OK;
}

cntr_status cntr_profile_end(cntr_profile* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof.on = false;
  cntr_profile p{};
  for (const ProfRec& r : g_prof.rec) {
    hipError_t e = hipEventSynchronize(r.after_step);
    if (e != hipSuccess) return hip_fail(e, "profile event");
    float a = 0, b = 0;
    if (hipEventElapsedTime(&a, r.before, r.after_hist) != hipSuccess ||
        hipEventElapsedTime(&b, r.before, r.after_step) != hipSuccess)
      return fail(CNTR_EHIP, "profile elapsed time");
    p.hist_ms += a;
    p.step_ms += b;
    p.hist_launches++;
    p.steps++;
    p.hist_bytes += r.bytes;
    p.hist_flops += r.flops;
  }
  g_prof.rec.clear();
  g_prof.used = 0;
  if (out) *out = p;
  return CNTR_OK;
}

const char* cntr_last_error(void) { return g_err.c_str(); }

struct cntr_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

cntr_status cntr_graph_begin(void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (s == nullptr) return fail(CNTR_EINVAL, "cntr_graph_begin: the default stream cannot be captured");
  if (capturing(s)) return fail(CNTR_EINVAL, "cntr_graph_begin: stream already capturing");
  cntr_status st = ensure_weights();
  if (st) return st;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "cntr_graph_begin");
  return CNTR_OK;
}

cntr_status cntr_graph_end(void* stream, cntr_graph* out) {
  hipStream_t s = (hipStream_t)stream;
  if (!out) return fail(CNTR_ESHAPE, "cntr_graph_end: null output");
  *out = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || !g) return hip_fail(e, "cntr_graph_end: capture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "cntr_graph_end: instantiate");
  }
  cntr_graph h = new cntr_graph_s;
  h->graph = g;
  h->exec = x;
  *out = h;
  return CNTR_OK;
}

cntr_status cntr_graph_launch(cntr_graph g, void* stream) {
  if (!g || !g->exec) return fail(CNTR_ESHAPE, "cntr_graph_launch: null graph");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "cntr_graph_launch");
  return CNTR_OK;
}

cntr_status cntr_graph_destroy(cntr_graph g) {
  if (!g) return CNTR_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return CNTR_OK;
}

cntr_status cntr_set_tiles(int32_t d, int32_t nbands, const int32_t* n_hi, const int32_t* tj) {
  if (d < 1 || d > 8) return fail(CNTR_EINVAL, "cntr_set_tiles: d outside 1..8");
  if (nbands < 0 || nbands > TUNE_BANDS) return fail(CNTR_EINVAL, "cntr_set_tiles: 0..8 bands");
  if (nbands > 0 && (!n_hi || !tj)) return fail(CNTR_ESHAPE, "cntr_set_tiles: null pointer");
  for (int b = 0; b < nbands; b++) {
    if (!tile_allowed(d, tj[b])) return fail(CNTR_EINVAL, "cntr_set_tiles: chunk not available for this d");
    if (b > 0 && n_hi[b] <= n_hi[b - 1]) return fail(CNTR_EINVAL, "cntr_set_tiles: band edges must increase");
  }
  std::lock_guard<std::mutex> lk(g_mu);
  TileTable t;
  t.nb = nbands;
  for (int b = 0; b < nbands; b++) {
    t.n_hi[b] = n_hi[b];
    t.tj[b] = tj[b];
  }
  g_tiles[d] = t;
  g_tiles_gen++;
  return CNTR_OK;
}

cntr_status cntr_set_checks(int32_t flags) {
  if (flags & ~(CNTR_CHECK_ORDER | CNTR_CHECK_FINITE | CNTR_CHECK_SYMMETRY))
    return fail(CNTR_EINVAL, "cntr_set_checks: unknown flag");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!(flags & CNTR_CHECK_ORDER)) g_last.clear();
  g_checks = flags;
  return CNTR_OK;
}

cntr_status cntr_mark_slices(int32_t count, const cntr_gf* G, int32_t last) {
  if (count < 1 || !G) return fail(CNTR_ESHAPE, "cntr_mark_slices: empty batch");
  if (last < -2) return fail(CNTR_EINVAL, "cntr_mark_slices: last < -2");
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < count; i++) {
    if (!G[i].ret) return fail(CNTR_ESHAPE, "cntr_mark_slices: null pointer");
    if (last == -2) g_last.erase(G[i].ret);
    else g_last[G[i].ret] = last;
  }
  return CNTR_OK;
}

cntr_status cntr_finalize(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_scratch) {
    if (kv.second.buf) (void)hipFree(kv.second.buf);
    if (kv.second.probs) (void)hipFree(kv.second.probs);
    if (kv.second.red) (void)hipFree(kv.second.red);
    if (kv.second.host) (void)hipHostFree(kv.second.host);
    for (auto& e : kv.second.descs)
      if (e.dev) (void)hipFree(e.dev);
  }
  g_scratch.clear();
  g_last.clear();
  for (hipEvent_t e : g_prof.pool) (void)hipEventDestroy(e);
  g_prof.pool.clear();
  g_prof.rec.clear();
  g_prof.used = 0;
  return CNTR_OK;
}

// text of a device status word (problem i, or -1: not known)
static std::string status_text(int code, int i) {
  std::string what = code == CNTR_ENONFINITE    ? "non-finite value in a time step"
                     : code == CNTR_ESYMMETRY ? "self-energy violates hermitian symmetry"
                                              : "singular step matrix detected on the device";
  return i >= 0 ? what + " (problem " + std::to_string(i) + ")" : what;
}

cntr_status cntr_sync(void* stream) {
  if (capturing((hipStream_t)stream)) return fail(CNTR_EINVAL, "cntr_sync: synchronizes the stream, not allowed during graph capture");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  int code = 0;
  cntr_status st = noalloc_status(&code);
  if (st) return st;
  if (code != 0)
    return fail((cntr_status)code, status_text(code, -1));
  StreamScratch* sc = scratch_for(s);
  if (!sc->buf || sc->nstat == 0) return CNTR_OK;
  // the status words of the problems of the calls since the last check
  int cnt = sc->nstat;
  std::vector<int> codes(cnt, 0);
  e = hipMemcpy(codes.data(), sc->stat(), cnt * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "status readback");
  sc->nstat = 0;
  for (int i = 0; i < cnt; i++)
    if (codes[i] != 0) {
      code = codes[i];
      std::vector<int> zero(cnt, 0);
      (void)hipMemcpy(sc->stat(), zero.data(), cnt * sizeof(int), hipMemcpyHostToDevice);
      return fail((cntr_status)code, status_text(code, i));
    }
  return CNTR_OK;
}

cntr_status cntr_dyson_step(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                            const cntr_gf* Sigma, const void* const* eps, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_dyson_step");
  if (st) return st;
  if (count > STAT_WORDS) return fail(CNTR_ESHAPE, "cntr_dyson_step: more than 65536 problems");
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !eps) return fail(CNTR_ESHAPE, "cntr_dyson_step: null pointer");
  int k = grids[0].k, d = grids[0].d, ntau = grids[0].ntau;
  int ntmax = 0;
  for (int i = 0; i < count; i++) {
    if (!eps[i]) return fail(CNTR_ESHAPE, "cntr_dyson_step: null eps");
    if (grids[i].nt > ntmax) ntmax = grids[i].nt;
  }
  if (tstp < 0 || tstp > ntmax) return fail(CNTR_EORDER, "cntr_dyson_step: tstp outside 0..nt");
  if ((st = order_check(tstp, k, count, G, "cntr_dyson_step"))) return st;
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  cntr_grid gmax = grids[0];
  gmax.nt = ntmax < k + 1 ? k + 1 : ntmax;
  StepScratch lay = step_layout(gmax);
  if ((st = grow(s, sc, lay.per * count, 5 * (size_t)count, 2 * (size_t)count))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) v[i] = make_prob(grids[i], &G[i], &Sigma[i], eps[i]);
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  Scratch scr = lay.sc;
  scr.base = sc->data();
  scr.stat = sc->stat();
  sc->nstat = std::max(sc->nstat, (int)count);
  bool shared = true;  // one Sigma (statistics, grid) for every problem
  for (int i = 1; i < count; i++)
    shared = shared && v[i].Stv == v[0].Stv && v[i].sig == v[0].sig && grids[i].nt == grids[0].nt;
  hipError_t e = tstp <= k ? launch_start(pa, scr, d, ntau, s)
                           : launch_step(pa, scr, tstp, d, s, shared, !capturing(s));
  if (e == hipSuccess && (g_checks & CNTR_CHECK_FINITE))
    e = launch_check_finite(pa, scr, tstp <= k ? 0 : tstp, tstp <= k ? k : tstp, d, ntau, s);
  if (e == hipSuccess && (g_checks & CNTR_CHECK_SYMMETRY))
    e = launch_check_symmetry(pa, scr, tstp <= k ? -1 : tstp, tstp <= k ? k : tstp, ntau, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_dyson_step launch");
  order_mark(count, G, tstp <= k ? k : tstp, false);
  return CNTR_OK;
}

cntr_status cntr_dyson_step_noalloc(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                                    const cntr_gf* Sigma, const void* const* eps, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_dyson_step_noalloc");
  if (st) return st;
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !eps)
    return fail(CNTR_ESHAPE, "cntr_dyson_step_noalloc: null pointer");
  if (count > NA_MAX_PROBS) return fail(CNTR_ENOMEM, "cntr_dyson_step_noalloc: more than 256 problems");
  int k = grids[0].k, d = grids[0].d, ntau = grids[0].ntau;
  int ntmax = 0;
  for (int i = 0; i < count; i++) {
    if (!eps[i]) return fail(CNTR_ESHAPE, "cntr_dyson_step_noalloc: null eps");
    if (grids[i].nt > ntmax) ntmax = grids[i].nt;
  }
  if (tstp < 0 || tstp > ntmax) return fail(CNTR_EORDER, "cntr_dyson_step_noalloc: tstp outside 0..nt");
  if ((st = order_check(tstp, k, count, G, "cntr_dyson_step_noalloc"))) return st;
  // the scratch this call needs: the regions of the step at the largest nt
  cntr_grid gmax = grids[0];
  gmax.nt = ntmax < k + 1 ? k + 1 : ntmax;
  StepScratch lay = step_layout(gmax);
  if (lay.per * (size_t)count > NA_STEP_BYTES) {
    char buf[200];
    snprintf(buf, sizeof buf, "cntr_dyson_step_noalloc: needs %zu bytes of scratch, the static array holds %zu",
             lay.per * (size_t)count, NA_STEP_BYTES);
    return fail(CNTR_ENOMEM, buf);
  }
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ptr = nullptr;
  if ((st = noalloc_setup(s, &ptr))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) v[i] = make_prob(grids[i], &G[i], &Sigma[i], eps[i]);
  ProbArg pa;
  pa.one = v[0];
  pa.count = count;
  pa.many = nullptr;
  if (count > 1) {
    Prob* dst = (Prob*)ptr;
    hipError_t e = put_probs(v.data(), count, dst, s);
    if (e != hipSuccess) return hip_fail(e, "cntr_dyson_step_noalloc descriptors");
    pa.many = dst;
  }
  Scratch scr = lay.sc;
  scr.base = ptr + NA_DESC_BYTES + NA_STAT_BYTES;
  scr.stat = (int*)(ptr + NA_DESC_BYTES);
  {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    g_na_nstat[dev] = std::max(g_na_nstat[dev], (int)count);
  }
  bool shared = true;
  for (int i = 1; i < count; i++)
    shared = shared && v[i].Stv == v[0].Stv && v[i].sig == v[0].sig && grids[i].nt == grids[0].nt;
  hipError_t e = tstp <= k ? launch_start(pa, scr, d, ntau, s) : launch_step(pa, scr, tstp, d, s, shared, false);
  if (e == hipSuccess && (g_checks & CNTR_CHECK_FINITE))
    e = launch_check_finite(pa, scr, tstp <= k ? 0 : tstp, tstp <= k ? k : tstp, d, ntau, s);
  if (e == hipSuccess && (g_checks & CNTR_CHECK_SYMMETRY))
    e = launch_check_symmetry(pa, scr, tstp <= k ? -1 : tstp, tstp <= k ? k : tstp, ntau, s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "cntr_dyson_step_noalloc launch");
  order_mark(count, G, tstp <= k ? k : tstp, false);
  return CNTR_OK;
}

cntr_status cntr_init_matsubara(int32_t count, const cntr_grid* grids, const cntr_gf* G,
                                const cntr_gf* Sigma, const void* const* eps, double tol,
                                int32_t max_iter, void* stream) {
  if (capturing((hipStream_t)stream)) return fail(CNTR_EINVAL, "cntr_init_matsubara: synchronizes the stream, not allowed during graph capture");
  cntr_status st = check_batch(count, grids, "cntr_init_matsubara");
  if (st) return st;
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !eps) return fail(CNTR_ESHAPE, "cntr_init_matsubara: null pointer");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  if (tol <= 0) tol = 1e-14;
  if (max_iter <= 0) max_iter = 200;
  for (int i = 0; i < count; i++)
    if (!eps[i]) return fail(CNTR_ESHAPE, "cntr_init_matsubara: null eps");
  MatsState ms;
  if ((st = ms.alloc(grids[0].ntau, grids[0].d))) return st;
  if (count > 1 && ms.N <= GJ_BATCH_MAX_N) {
    auto build = [&](int i, cplx* A, cplx* g, Prob* P) -> hipError_t {
      *P = make_prob(grids[i], &G[i], &Sigma[i], eps[i]);
      hipError_t e;
      if ((e = launch_free_mat(*P, g, s)) || (e = launch_mat_conv(*P, g, P->Smat, nullptr, ms.K, s)) ||
          (e = launch_mat_build(*P, ms.K, A, s)))
        return e;
      return hipSuccess;
    };
    if ((st = mats_solve_batch(count, ms, grids[0].ntau, build, tol, max_iter, s))) return st;
  } else {
    for (int i = 0; i < count; i++) {
      Prob P = make_prob(grids[i], &G[i], &Sigma[i], eps[i]);
      ms.have_inv = false;
      if ((st = mats_solve(ms, P, false, tol, max_iter, s, nullptr))) return st;
    }
  }
  order_mark(count, G, -1, true);
  return CNTR_OK;
}

// ------------------------------------------ Dyson equation in integral form
// Problem descriptor of (1 + F) * G = Q (the layout described at Prob).
static Prob vie2_prob(const cntr_grid& g, const cntr_gf* G, const cntr_gf* F, const cntr_gf* Fcc, const cntr_gf* Q) {
  Prob p = make_prob(g, G, nullptr, nullptr);
  p.Smat = (cplx*)F->mat;
  p.Sret = (cplx*)F->ret;
  p.Stv = (cplx*)F->tv;
  p.Fles = (const cplx*)F->les;
  if (Fcc) {
    p.Sles = (cplx*)Fcc->les;
    p.Fcret = (const cplx*)Fcc->ret;
  }
  p.Qmat = (const cplx*)Q->mat;
  p.Qret = (const cplx*)Q->ret;
  p.Qles = (const cplx*)Q->les;
  p.Qtv = (const cplx*)Q->tv;
  return p;
}

cntr_status cntr_vie2_matsubara(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* F,
                                const cntr_gf* Q, double tol, int32_t max_iter, void* stream) {
  if (capturing((hipStream_t)stream))
    return fail(CNTR_EINVAL, "cntr_vie2_matsubara: synchronizes the stream, not allowed during graph capture");
  cntr_status st = check_batch(count, grids, "cntr_vie2_matsubara");
  if (st) return st;
  if (!gf_ok(G, count) || !gf_ok(F, count) || !gf_ok(Q, count))
    return fail(CNTR_ESHAPE, "cntr_vie2_matsubara: null pointer");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  if (tol <= 0) tol = 1e-14;
  if (max_iter <= 0) max_iter = 200;
  MatsState ms;
  if ((st = ms.alloc(grids[0].ntau, grids[0].d))) return st;
  size_t vec = (size_t)ms.N * ms.d * sizeof(cplx);
  if (count > 1 && ms.N <= GJ_BATCH_MAX_N) {
    // G_m + [F * G]^M(m) = Q_m (Eq. vie2_langreth_m) as one dense system each
    auto build = [&](int i, cplx* A, cplx* g, Prob* P) -> hipError_t {
      *P = vie2_prob(grids[i], &G[i], &F[i], nullptr, &Q[i]);
      hipError_t e;
      if ((e = launch_mat_build(*P, P->Smat, A, s, +1.0))) return e;
      return hipMemcpyAsync(g, P->Qmat, vec, hipMemcpyDeviceToDevice, s);
    };
    if ((st = mats_solve_batch(count, ms, grids[0].ntau, build, tol, max_iter, s))) return st;
  } else {
    for (int i = 0; i < count; i++) {
      Prob P = vie2_prob(grids[i], &G[i], &F[i], nullptr, &Q[i]);
      hipError_t e;
      // G_m + [F * G]^M(m) = Q_m (Eq. vie2_langreth_m) as one dense system
      if ((e = launch_mat_build(P, P.Smat, ms.A, s, +1.0))) return hip_fail(e, "vie2 Matsubara operator");
      if ((e = hipMemcpyAsync(ms.g, P.Qmat, vec, hipMemcpyDeviceToDevice, s))) return hip_fail(e, "vie2 source");
      ms.have_inv = false;
      if ((st = mats_refine(ms, P, false, tol, max_iter, s, nullptr))) return st;
    }
  }
  order_mark(count, G, -1, true);
  return CNTR_OK;
}

cntr_status cntr_vie2_step(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* F,
                           const cntr_gf* Fcc, const cntr_gf* Q, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_vie2_step");
  if (st) return st;
  if (count > STAT_WORDS) return fail(CNTR_ESHAPE, "cntr_vie2_step: more than 65536 problems");
  if (!gf_ok(G, count) || !gf_ok(F, count) || !gf_ok(Fcc, count) || !gf_ok(Q, count))
    return fail(CNTR_ESHAPE, "cntr_vie2_step: null pointer");
  int k = grids[0].k, d = grids[0].d, ntau = grids[0].ntau;
  int ntmax = 0;
  for (int i = 0; i < count; i++)
    if (grids[i].nt > ntmax) ntmax = grids[i].nt;
  if (tstp < 0 || tstp > ntmax) return fail(CNTR_EORDER, "cntr_vie2_step: tstp outside 0..nt");
  if ((st = order_check(tstp, k, count, G, "cntr_vie2_step"))) return st;
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  cntr_grid gmax = grids[0];
  gmax.nt = ntmax < k + 1 ? k + 1 : ntmax;
  StepScratch lay = step_layout(gmax);
  if ((st = grow(s, sc, lay.per * count, 5 * (size_t)count, 2 * (size_t)count))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) v[i] = vie2_prob(grids[i], &G[i], &F[i], &Fcc[i], &Q[i]);
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  Scratch scr = lay.sc;
  scr.base = sc->data();
  scr.stat = sc->stat();
  sc->nstat = std::max(sc->nstat, (int)count);
  hipError_t e = tstp <= k ? launch_vie2_start(pa, scr, d, ntau, s) : launch_vie2_step(pa, scr, tstp, d, s, !capturing(s));
  if (e != hipSuccess) return hip_fail(e, "cntr_vie2_step launch");
  order_mark(count, G, tstp <= k ? k : tstp, false);
  return CNTR_OK;
}

// ------------------------------------------ momentum-convolution bubbles
static cntr_status kspace_call(int mode, int32_t tstp, int32_t nk, const cntr_grid* grids, const cntr_gf* G,
                               const cntr_gf* dW, const cntr_gf* Out, double alpha, void* stream, const char* what) {
  cntr_status st = check_batch(nk, grids, what);
  if (st) return st;
  if (nk > 1024) return fail(CNTR_EINVAL, std::string(what) + ": more than 1024 momenta");
  if (!gf_ok(G, nk) || !gf_ok(Out, nk) || (mode == 2 && !gf_ok(dW, nk)))
    return fail(CNTR_ESHAPE, std::string(what) + ": null pointer");
  for (int i = 1; i < nk; i++)
    if (grids[i].nt != grids[0].nt || grids[i].ntau != grids[0].ntau || grids[i].d != grids[0].d ||
        grids[i].sig != grids[0].sig)
      return fail(CNTR_ESHAPE, std::string(what) + ": the momenta must share one grid");
  if (tstp < -1 || tstp > grids[0].nt) return fail(CNTR_EORDER, std::string(what) + ": tstp outside -1..nt");
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  // the kernels always read the descriptor arrays: one momentum is uploaded
  // as a pair (the second entry unused)
  size_t nup = nk < 2 ? 2 : (size_t)nk;
  if ((st = grow(s, sc, 256, 5 * nup, 2))) return st;
  std::vector<Prob> vg(nup), vw(nup), vo(nup);
  for (size_t i = 0; i < nup; i++) {
    size_t u = i < (size_t)nk ? i : 0;
    vg[i] = make_prob(grids[u], &G[u], nullptr, nullptr);
    vo[i] = make_prob(grids[u], &Out[u], nullptr, nullptr);
    vw[i] = mode == 2 ? make_prob(grids[u], &dW[u], nullptr, nullptr) : vg[i];
  }
  ProbArg pg, pw, po;
  if ((st = make_arg(s, sc, vg, 0, &pg)) || (st = make_arg(s, sc, vw, 1, &pw)) || (st = make_arg(s, sc, vo, 2, &po)))
    return st;
  hipError_t e = launch_kbubble(mode, pg.many, pw.many, po.many, nk, grids[0].d, grids[0].ntau, grids[0].sig, tstp,
                                alpha, s);
  if (e != hipSuccess) return hip_fail(e, (std::string(what) + " launch").c_str());
  return CNTR_OK;
}

cntr_status cntr_polarization_k(int32_t tstp, int32_t nk, const cntr_grid* grids, const cntr_gf* G,
                                const cntr_gf* Pi, double alpha, void* stream) {
  return kspace_call(1, tstp, nk, grids, G, nullptr, Pi, alpha, stream, "cntr_polarization_k");
}

cntr_status cntr_sigma_gw_k(int32_t tstp, int32_t nk, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* dW,
                            const cntr_gf* Sigma, double alpha, void* stream) {
  return kspace_call(2, tstp, nk, grids, G, dW, Sigma, alpha, stream, "cntr_sigma_gw_k");
}

cntr_status cntr_bubble2_local(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* A,
                               const cntr_gf* B, const cntr_gf* C, double alpha, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_bubble2_local");
  if (st) return st;
  if (count > 65535) return fail(CNTR_EINVAL, "cntr_bubble2_local: more than 65535 instances");
  if (!gf_ok(A, count) || !gf_ok(B, count) || !gf_ok(C, count))
    return fail(CNTR_ESHAPE, "cntr_bubble2_local: null pointer");
  for (int i = 0; i < count; i++)
    if (tstp < -1 || tstp > grids[i].nt) return fail(CNTR_EORDER, "cntr_bubble2_local: tstp outside -1..nt");
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> va(count), vb(count), vc(count);
  for (int i = 0; i < count; i++) {
    va[i] = make_prob(grids[i], &A[i], nullptr, nullptr);
    vb[i] = make_prob(grids[i], &B[i], nullptr, nullptr);
    vc[i] = make_prob(grids[i], &C[i], nullptr, nullptr);
  }
  ProbArg pa, pb, pc;
  if ((st = make_arg(s, sc, va, 0, &pa)) || (st = make_arg(s, sc, vb, 1, &pb)) || (st = make_arg(s, sc, vc, 2, &pc)))
    return st;
  hipError_t e = launch_bubble2_local(pa, pb, pc, tstp, grids[0].d, grids[0].ntau, alpha, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_bubble2_local launch");
  return CNTR_OK;
}

// ------------------------------------------------- Holstein DMFT pieces
cntr_status cntr_phonon_free(int32_t count, const cntr_grid* grids, const cntr_gf* D, const double* w0,
                             void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_phonon_free");
  if (st) return st;
  if (!gf_ok(D, count) || !w0) return fail(CNTR_ESHAPE, "cntr_phonon_free: null pointer");
  int ntmax = 0;
  for (int i = 0; i < count; i++) {
    if (grids[i].d != 1 || grids[i].sig != 1)
      return fail(CNTR_ESHAPE, "cntr_phonon_free: one bosonic mode per problem (d = 1, sig = +1)");
    if (!(w0[i] > 0) || !std::isfinite(w0[i])) return fail(CNTR_EINVAL, "cntr_phonon_free: w0 must be > 0");
    ntmax = std::max(ntmax, (int)grids[i].nt);
  }
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) {
    v[i] = make_prob(grids[i], &D[i], nullptr, nullptr);
    v[i].par = w0[i];
  }
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  hipError_t e = launch_phonon_free(pa, ntmax, grids[0].ntau, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_phonon_free launch");
  return CNTR_OK;
}

cntr_status cntr_scale_slice(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* C,
                             const cntr_gf* A, const void* const* f, double beta, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_scale_slice");
  if (st) return st;
  if (!gf_ok(C, count) || !gf_ok(A, count) || !f) return fail(CNTR_ESHAPE, "cntr_scale_slice: null pointer");
  for (int i = 0; i < count; i++) {
    if (!f[i]) return fail(CNTR_ESHAPE, "cntr_scale_slice: null f");
    if (tstp < -1 || tstp > grids[i].nt) return fail(CNTR_EORDER, "cntr_scale_slice: tstp outside -1..nt");
  }
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> vc(count), va(count);
  for (int i = 0; i < count; i++) {
    vc[i] = make_prob(grids[i], &C[i], nullptr, nullptr);
    vc[i].U = (const double*)f[i];
    va[i] = make_prob(grids[i], &A[i], nullptr, nullptr);
  }
  ProbArg pc, pa;
  if ((st = make_arg(s, sc, vc, 0, &pc)) || (st = make_arg(s, sc, va, 1, &pa))) return st;
  hipError_t e = launch_scale_slice(pc, pa, tstp, grids[0].d, grids[0].ntau, beta, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_scale_slice launch");
  return CNTR_OK;
}

cntr_status cntr_holstein_mf(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             const void* const* g, const double* w0, double e0, void* const* X, void* const* eps,
                             void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_holstein_mf");
  if (st) return st;
  if (!gf_ok(G, count) || !g || !w0 || !X || !eps) return fail(CNTR_ESHAPE, "cntr_holstein_mf: null pointer");
  for (int i = 0; i < count; i++) {
    if (grids[i].d != 1) return fail(CNTR_ESHAPE, "cntr_holstein_mf: single band (d = 1)");
    if (!g[i] || !X[i] || !eps[i]) return fail(CNTR_ESHAPE, "cntr_holstein_mf: null series");
    if (!(w0[i] > 0) || !std::isfinite(w0[i])) return fail(CNTR_EINVAL, "cntr_holstein_mf: w0 must be > 0");
    if (tstp < -1 || tstp > grids[i].nt || grids[i].k > grids[i].nt)
      return fail(CNTR_EORDER, "cntr_holstein_mf: tstp outside -1..nt (or k > nt)");
  }
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) {
    v[i] = make_prob(grids[i], &G[i], nullptr, nullptr);
    v[i].U = (const double*)g[i];
    v[i].par = w0[i];
    v[i].aux = (double*)X[i];
    v[i].eps_mf = (cplx*)eps[i];
  }
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  hipError_t e = launch_holstein_mf(pa, tstp, e0, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_holstein_mf launch");
  return CNTR_OK;
}

cntr_status cntr_convolution(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* C,
                             const cntr_gf* A, const cntr_gf* Acc, const cntr_gf* B,
                             const cntr_gf* Bcc, const void* const* f, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_convolution");
  if (st) return st;
  if (!gf_ok(C, count) || !gf_ok(A, count) || !gf_ok(Acc, count) || !gf_ok(B, count) || !gf_ok(Bcc, count))
    return fail(CNTR_ESHAPE, "cntr_convolution: null pointer");
  int ntmax = 0;
  for (int i = 0; i < count; i++) ntmax = grids[i].nt > ntmax ? grids[i].nt : ntmax;
  if (tstp < -1 || tstp > ntmax) return fail(CNTR_EORDER, "cntr_convolution: tstp outside -1..nt");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> vc(count), va(count), vac(count), vb(count), vbc(count);
  for (int i = 0; i < count; i++) {
    vc[i] = make_prob(grids[i], &C[i], nullptr, nullptr);
    vc[i].f = f ? (const cplx*)f[i] : nullptr;
    va[i] = make_prob(grids[i], &A[i], nullptr, nullptr);
    vac[i] = make_prob(grids[i], &Acc[i], nullptr, nullptr);
    vb[i] = make_prob(grids[i], &B[i], nullptr, nullptr);
    vbc[i] = make_prob(grids[i], &Bcc[i], nullptr, nullptr);
  }
  ProbArg pc, pa, pac, pb, pbc;
  if ((st = make_arg(s, sc, vc, 0, &pc)) || (st = make_arg(s, sc, va, 1, &pa)) ||
      (st = make_arg(s, sc, vac, 2, &pac)) || (st = make_arg(s, sc, vb, 3, &pb)) ||
      (st = make_arg(s, sc, vbc, 4, &pbc)))
    return st;
  cntr_grid gm = grids[0];
  gm.nt = tstp < 0 ? 0 : tstp;
  hipError_t e = launch_convolution(pc, pa, pac, pb, pbc, tstp, grids[0].d, (int)slice_elems(gm, tstp), s);
  if (e != hipSuccess) return hip_fail(e, "cntr_convolution launch");
  return CNTR_OK;
}

cntr_status cntr_sigma_2b(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                          const double* const* U, const cntr_gf* Sigma, const void* const* eps0,
                          void* const* eps_mf, double nbar, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_sigma_2b");
  if (st) return st;
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !U) return fail(CNTR_ESHAPE, "cntr_sigma_2b: null pointer");
  if (eps_mf && !eps0) return fail(CNTR_ESHAPE, "cntr_sigma_2b: eps_mf requires eps0");
  int ntmax = 0;
  for (int i = 0; i < count; i++) {
    if (!U[i]) return fail(CNTR_ESHAPE, "cntr_sigma_2b: null U");
    ntmax = grids[i].nt > ntmax ? grids[i].nt : ntmax;
  }
  if (tstp < -1 || tstp > ntmax) return fail(CNTR_EORDER, "cntr_sigma_2b: tstp outside -1..nt");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) {
    v[i] = make_prob(grids[i], &G[i], &Sigma[i], nullptr);
    v[i].U = U[i];
    v[i].eps0 = eps0 ? (const cplx*)eps0[i] : nullptr;
    v[i].eps_mf = eps_mf ? (cplx*)eps_mf[i] : nullptr;
    if (eps_mf && eps_mf[i] && !eps0[i]) return fail(CNTR_ESHAPE, "cntr_sigma_2b: null eps0");
  }
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  cntr_grid gm = grids[0];
  hipError_t e = launch_sigma2b(pa, tstp, gm.d, (int)slice_elems(gm, tstp), nbar, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_sigma_2b launch");
  return CNTR_OK;
}

cntr_status cntr_sigma_local(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             const cntr_gf* Sigma, double lam, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_sigma_local");
  if (st) return st;
  if (!gf_ok(G, count) || !gf_ok(Sigma, 1)) return fail(CNTR_ESHAPE, "cntr_sigma_local: null pointer");
  for (int i = 1; i < count; i++)
    if (grids[i].nt != grids[0].nt || grids[i].ntau != grids[0].ntau)
      return fail(CNTR_ESHAPE, "cntr_sigma_local: all grids must agree");
  if (tstp < -1 || tstp > grids[0].nt) return fail(CNTR_EORDER, "cntr_sigma_local: tstp outside -1..nt");
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) v[i] = make_prob(grids[i], &G[i], i == 0 ? Sigma : nullptr, nullptr);
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  hipError_t e = launch_sigma_local(pa, tstp, grids[0].d, (int)slice_elems(grids[0], tstp), lam, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_sigma_local launch");
  return CNTR_OK;
}

cntr_status cntr_observables(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             const cntr_gf* Sigma, const void* const* eps0, const void* const* eps_mf,
                             double* obs, void* rho, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_observables");
  if (st) return st;
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !eps0 || !obs)
    return fail(CNTR_ESHAPE, "cntr_observables: null pointer");
  int ntmax = 0;
  for (int i = 0; i < count; i++) {
    if (!eps0[i]) return fail(CNTR_ESHAPE, "cntr_observables: null eps0");
    ntmax = grids[i].nt > ntmax ? grids[i].nt : ntmax;
  }
  if (tstp < 0 || tstp > ntmax) return fail(CNTR_EORDER, "cntr_observables: tstp outside 0..nt");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) {
    v[i] = make_prob(grids[i], &G[i], &Sigma[i], nullptr);
    v[i].eps0 = (const cplx*)eps0[i];
    v[i].eps_mf = eps_mf ? (cplx*)eps_mf[i] : nullptr;
  }
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  hipError_t e = launch_observables(pa, tstp, obs, (cplx*)rho, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_observables launch");
  return CNTR_OK;
}

cntr_status cntr_adjoint_sweep(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                               const void* const* eps, const double* const* U, double nbar,
                               const cntr_gf* Gbar, const cntr_gf* Sigmabar, void* const* eps_bar,
                               double* const* U_bar, int32_t niter, double tol, double* conv, void* stream) {
  if (capturing((hipStream_t)stream)) return fail(CNTR_EINVAL, "cntr_adjoint_sweep: synchronizes the stream, not allowed during graph capture");
  cntr_status st = check_batch(count, grids, "cntr_adjoint_sweep");
  if (st) return st;
  if (count > 65535) return fail(CNTR_ESHAPE, "cntr_adjoint_sweep: at most 65535 problems per call");
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !gf_ok(Gbar, count) || !eps || !eps_bar)
    return fail(CNTR_ESHAPE, "cntr_adjoint_sweep: null pointer");
  bool twob = U != nullptr;
  if (twob && (!Sigmabar || !U_bar))
    return fail(CNTR_ESHAPE, "cntr_adjoint_sweep: the second-Born mode needs Sigmabar and U_bar");
  for (int i = 0; i < count; i++) {
    if (!eps[i] || !eps_bar[i]) return fail(CNTR_ESHAPE, "cntr_adjoint_sweep: null eps or eps_bar");
    if (Sigmabar && (!Sigmabar[i].ret || !Sigmabar[i].les || !Sigmabar[i].tv))
      return fail(CNTR_ESHAPE, "cntr_adjoint_sweep: Sigmabar needs ret, les and tv");
    if (twob && (!U[i] || !U_bar[i])) return fail(CNTR_ESHAPE, "cntr_adjoint_sweep: null U or U_bar");
  }
  if (niter <= 0) niter = 10;
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  int ntmax = 0, k = grids[0].k, d = grids[0].d, ntau = grids[0].ntau;
  for (int i = 0; i < count; i++) ntmax = grids[i].nt > ntmax ? grids[i].nt : ntmax;
  size_t dd = (size_t)d * d;
  AdjLayout lay = adj_layout(ntmax, ntau, d, k);
  // second-Born work windows (blocks): slice windows of slices [n, n] or [0, k],
  // Sigma windows of slices [n-k, n] or [0, n <= 2k]
  size_t wr = std::max<size_t>(ntmax + 1, tri(k + 1)), wt = (size_t)(k + 1) * (ntau + 1);
  size_t sr = std::max<size_t>((size_t)(k + 1) * (ntmax + 1), tri(2 * k + 1)), stt = (size_t)(2 * k + 1) * (ntau + 1);
  size_t wblk = 2 * wr + wt, sblk = 2 * sr + stt;
  size_t work = twob ? round256((5 * wblk + sblk + (k + 1) + (ntmax + 2) + (ntau + 1)) * dd * sizeof(cplx)) +
                           round256(2 * (ntmax + 2) * sizeof(double))
                     : 0;
  size_t per = round256(lay.total * sizeof(cplx)) + work;
  size_t head = round256(count * sizeof(int)) + 2 * round256(count * sizeof(AdjProb));
  if ((st = grow(s, sc, head + per * count, 5, 2))) return st;
  int* dstat = (int*)sc->data();
  AdjProb* dA = (AdjProb*)(sc->data() + round256(count * sizeof(int)));
  AdjProb* dDry = (AdjProb*)((char*)dA + round256(count * sizeof(AdjProb)));
  std::vector<AdjProb> hA(count);
  for (int i = 0; i < count; i++) {
    AdjProb& a = hA[i];
    a = AdjProb{};
    a.p = make_prob(grids[i], &G[i], &Sigma[i], eps[i]);
    a.aR = (cplx*)Gbar[i].ret;
    a.aL = (cplx*)Gbar[i].les;
    a.aT = (cplx*)Gbar[i].tv;
    a.aM = (cplx*)Gbar[i].mat;
    a.sR = Sigmabar ? (cplx*)Sigmabar[i].ret : nullptr;
    a.sL = Sigmabar ? (cplx*)Sigmabar[i].les : nullptr;
    a.sT = Sigmabar ? (cplx*)Sigmabar[i].tv : nullptr;
    a.ge = (cplx*)eps_bar[i];
    char* base = sc->data() + head + per * i;
    a.scr = (cplx*)base;
    a.stat = dstat + i;
    if (twob) {
      a.U = U[i];
      a.nbar = nbar;
      a.ub = U_bar[i];
      cplx* w = (cplx*)(base + round256(lay.total * sizeof(cplx)));
      auto win = [&](AdjWin& x, size_t r, size_t t) {
        x.R = w;
        x.L = w + r * dd;
        x.T = w + 2 * r * dd;
        w += (2 * r + t) * dd;
      };
      win(a.g0, wr, wt);
      win(a.s0, wr, wt);
      win(a.nu[0], wr, wt);
      win(a.nu[1], wr, wt);
      win(a.gdry, wr, wt);
      win(a.sdry, sr, stt);
      a.e0 = w;
      w += (k + 1) * dd;
      a.gedry = w;
      w += (ntmax + 2) * dd;
      a.mdummy = w;
      w += (ntau + 1) * dd;
      a.conv = (double*)((char*)a.scr + round256(lay.total * sizeof(cplx)) +
                         round256((5 * wblk + sblk + (k + 1) + (ntmax + 2) + (ntau + 1)) * dd * sizeof(cplx)));
    }
  }
  hipError_t e = hipMemsetAsync(dstat, 0, count * sizeof(int), s);
  if (e == hipSuccess) e = hipMemcpyAsync(dA, hA.data(), count * sizeof(AdjProb), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = twob ? launch_adjoint_2b(dA, dDry, hA.data(), count, niter, s) : launch_adjoint_sweep(dA, hA.data(), count, s);
  // equilibrium part (second-Born mode): the Matsubara solve's adjoint, per problem
  double mats_change = 0.0;
  if (twob && e == hipSuccess) {
    MatsState ms;
    if ((st = ms.alloc(ntau, d))) return st;
    size_t nb = (size_t)(ntau + 1) * dd;
    int N = (ntau + 1) * d;
    MadjBuf B{};
    cplx* mb = nullptr;
    double* md = nullptr;
    size_t ncx = 7 * nb + 2 * dd;
    if (hipMalloc(&mb, ncx * sizeof(cplx)) != hipSuccess || hipMalloc(&md, (d + 1024) * sizeof(double)) != hipSuccess) {
      if (mb) (void)hipFree(mb);
      ms.release();
      return fail(CNTR_ENOMEM, "cntr_adjoint_sweep: Matsubara adjoint workspace");
    }
    B.Ainv = ms.Ainv;
    B.g = mb;
    B.gA = mb + nb;
    B.Kb = mb + 2 * nb;
    B.gb = mb + 3 * nb;
    B.Sb = mb + 4 * nb;
    B.nu = mb + 5 * nb;
    B.nun = mb + 6 * nb;
    B.eb = mb + 7 * nb;
    B.V = mb + 7 * nb + dd;
    B.x = md;
    B.red = md + d;
    for (int i = 0; i < count && e == hipSuccess; i++) {
      double u = 0.0, red[2] = {0, 0};
      int stat = 0;
      e = hipMemcpyAsync(&u, U[i], sizeof(double), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemsetAsync(ms.status, 0, sizeof(int), s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess)
        e = launch_adjoint_mats(hA[i].p, B, ms.K, ms.work, ms.piv, ms.status, (const cplx*)Gbar[i].mat, u, nbar,
                                U_bar[i], (cplx*)eps_bar[i], 150, 0.5, s);
      if (e == hipSuccess) e = hipMemcpyAsync(red, B.red, sizeof red, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(&stat, ms.status, sizeof(int), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess && stat) {
        (void)hipFree(mb);
        (void)hipFree(md);
        ms.release();
        return fail(CNTR_ESINGULAR, "cntr_adjoint_sweep: singular Matsubara operator");
      }
      double r = red[1] > 0 ? red[0] / red[1] : red[0];
      mats_change = r > mats_change ? r : mats_change;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(mb);
    (void)hipFree(md);
    ms.release();
  }
  std::vector<int> hs(count, 0);
  std::vector<std::vector<double>> hc;
  if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), dstat, count * sizeof(int), hipMemcpyDeviceToHost, s);
  if (twob && (conv || tol > 0))
    for (int i = 0; i < count && e == hipSuccess; i++) {
      hc.emplace_back(2 * (grids[i].nt + 2));
      e = hipMemcpyAsync(hc.back().data(), hA[i].conv, hc.back().size() * sizeof(double), hipMemcpyDeviceToHost, s);
    }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "cntr_adjoint_sweep");
  for (int i = 0; i < count; i++)
    if (hs[i]) return fail(CNTR_ESINGULAR, "cntr_adjoint_sweep: singular local matrix in problem " + std::to_string(i));
  if (twob && (conv || tol > 0)) {
    // slots: slice n for the steps (n > k), slot k for the start-up block
    double worst = 0.0;
    for (int i = 0; i < count; i++)
      for (int n = k; n <= grids[i].nt; n++) {
        double ch = hc[i][2 * n], v = hc[i][2 * n + 1];
        double r = v > 0 ? ch / v : ch;
        worst = r > worst ? r : worst;
      }
    worst = worst > mats_change ? worst : mats_change;
    if (conv) *conv = worst;
    if (tol > 0 && !(worst <= tol)) {
      char buf[160];
      snprintf(buf, sizeof buf, "cntr_adjoint_sweep: last fixed-point change %.3e above tol %.3e", worst, tol);
      return fail(CNTR_ENOCONV, buf);
    }
  }
  return CNTR_OK;
}

cntr_status cntr_green_from_H(int32_t count, const cntr_grid* grids, const cntr_gf* G, const void* const* eps,
                              void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_green_from_H");
  if (st) return st;
  if (!gf_ok(G, count) || !eps) return fail(CNTR_ESHAPE, "cntr_green_from_H: null pointer");
  size_t need = 256;
  for (int i = 0; i < count; i++) {
    if (!eps[i]) return fail(CNTR_ESHAPE, "cntr_green_from_H: null eps");
    if (grids[i].nt < grids[i].k) return fail(CNTR_EINVAL, "cntr_green_from_H: nt < k");
    need = std::max(need, free_green_scratch_bytes(grids[i].nt, grids[i].ntau, grids[i].d));
  }
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, need, 0, 0))) return st;
  for (int i = 0; i < count; i++) {
    Prob P = make_prob(grids[i], &G[i], nullptr, eps[i]);
    hipError_t e = launch_free_green(P, sc->data(), s);
    if (e != hipSuccess) return hip_fail(e, "cntr_green_from_H");
  }
  return CNTR_OK;
}

cntr_status cntr_matsubara_fourier(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                                   const void* const* eps, int32_t oversample, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_matsubara_fourier");
  if (st) return st;
  if (!gf_ok(G, count) || !eps) return fail(CNTR_ESHAPE, "cntr_matsubara_fourier: null pointer");
  if (oversample < 1 || oversample > 64) return fail(CNTR_EINVAL, "cntr_matsubara_fourier: oversampling outside 1..64");
  size_t need = 256;
  for (int i = 0; i < count; i++) {
    if (!eps[i]) return fail(CNTR_ESHAPE, "cntr_matsubara_fourier: null eps");
    if (grids[i].ntau < 3) return fail(CNTR_EINVAL, "cntr_matsubara_fourier: ntau < 3");
    if (Sigma && !Sigma[i].mat) return fail(CNTR_ESHAPE, "cntr_matsubara_fourier: null Sigma^M");
    need = std::max(need, mats_fourier_scratch_bytes(grids[i].ntau, grids[i].d, oversample));
  }
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, need, 0, 0))) return st;
  for (int i = 0; i < count; i++) {
    Prob P = make_prob(grids[i], &G[i], Sigma ? &Sigma[i] : nullptr, eps[i]);
    hipError_t e = launch_mats_fourier(P, oversample, (cplx*)sc->data(), s);
    if (e != hipSuccess) return hip_fail(e, "cntr_matsubara_fourier");
  }
  return CNTR_OK;
}

cntr_status cntr_peierls(int32_t count, const cntr_grid* grids, const void* const* T, const double* const* Phi,
                         const double* const* A, void* const* eps, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_peierls");
  if (st) return st;
  if (!T || !Phi || !A || !eps) return fail(CNTR_ESHAPE, "cntr_peierls: null pointer");
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < count; i++) {
    if (!T[i] || !Phi[i] || !A[i] || !eps[i]) return fail(CNTR_ESHAPE, "cntr_peierls: null pointer");
    hipError_t e = launch_peierls((const cplx*)T[i], Phi[i], A[i], (cplx*)eps[i], grids[i].d, grids[i].nt, s);
    if (e != hipSuccess) return hip_fail(e, "cntr_peierls launch");
  }
  return CNTR_OK;
}

cntr_status cntr_peierls_grad(int32_t count, const cntr_grid* grids, const void* const* T,
                              const double* const* Phi, const double* const* A, const void* const* eps_bar,
                              double* const* A_bar, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_peierls_grad");
  if (st) return st;
  if (!T || !Phi || !A || !eps_bar || !A_bar) return fail(CNTR_ESHAPE, "cntr_peierls_grad: null pointer");
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < count; i++) {
    if (!T[i] || !Phi[i] || !A[i] || !eps_bar[i] || !A_bar[i])
      return fail(CNTR_ESHAPE, "cntr_peierls_grad: null pointer");
    hipError_t e = launch_peierls_grad((const cplx*)T[i], Phi[i], A[i], (const cplx*)eps_bar[i], A_bar[i],
                                       grids[i].d, grids[i].nt, s);
    if (e != hipSuccess) return hip_fail(e, "cntr_peierls_grad launch");
  }
  return CNTR_OK;
}

cntr_status cntr_extrapolate(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* G,
                             void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_extrapolate");
  if (st) return st;
  if (!gf_ok(G, count)) return fail(CNTR_ESHAPE, "cntr_extrapolate: null pointer");
  int ntmax = 0;
  for (int i = 0; i < count; i++) ntmax = grids[i].nt > ntmax ? grids[i].nt : ntmax;
  if (tstp < grids[0].k || tstp + 1 > ntmax) return fail(CNTR_EORDER, "cntr_extrapolate: need k <= tstp < nt");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> v(count);
  for (int i = 0; i < count; i++) v[i] = make_prob(grids[i], &G[i], nullptr, nullptr);
  ProbArg pa;
  if ((st = make_arg(s, sc, v, 0, &pa))) return st;
  hipError_t e = launch_extrapolate(pa, tstp, grids[0].d, (int)slice_elems(grids[0], tstp + 1), s);
  if (e != hipSuccess) return hip_fail(e, "cntr_extrapolate launch");
  return CNTR_OK;
}

cntr_status cntr_copy_slice(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* dst,
                            const cntr_gf* src, void* stream) {
  cntr_status st = check_batch(count, grids, "cntr_copy_slice");
  if (st) return st;
  if (!gf_ok(dst, count) || !gf_ok(src, count)) return fail(CNTR_ESHAPE, "cntr_copy_slice: null pointer");
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2))) return st;
  std::vector<Prob> vd(count), vs(count);
  for (int i = 0; i < count; i++) {
    vd[i] = make_prob(grids[i], &dst[i], nullptr, nullptr);
    vs[i] = make_prob(grids[i], &src[i], nullptr, nullptr);
  }
  ProbArg pd, ps;
  if ((st = make_arg(s, sc, vd, 0, &pd)) || (st = make_arg(s, sc, vs, 1, &ps))) return st;
  hipError_t e = launch_copy(pd, ps, tstp, grids[0].d, (int)slice_elems(grids[0], tstp), s);
  if (e != hipSuccess) return hip_fail(e, "cntr_copy_slice launch");
  return CNTR_OK;
}

cntr_status cntr_distance(int32_t tstp, int32_t count, const cntr_grid* grids, const cntr_gf* A,
                          const cntr_gf* B, double* out, void* stream) {
  if (capturing((hipStream_t)stream)) return fail(CNTR_EINVAL, "cntr_distance: synchronizes the stream, not allowed during graph capture");
  cntr_status st = check_batch(count, grids, "cntr_distance");
  if (st) return st;
  if (!gf_ok(A, count) || !gf_ok(B, count) || !out) return fail(CNTR_ESHAPE, "cntr_distance: null pointer");
  hipStream_t s = (hipStream_t)stream;
  StreamScratch* sc = scratch_for(s);
  if ((st = grow(s, sc, 256, 5 * (size_t)count, 2 * (size_t)count))) return st;
  std::vector<Prob> va(count), vb(count);
  for (int i = 0; i < count; i++) {
    va[i] = make_prob(grids[i], &A[i], nullptr, nullptr);
    vb[i] = make_prob(grids[i], &B[i], nullptr, nullptr);
  }
  ProbArg pa, pb;
  if ((st = make_arg(s, sc, va, 0, &pa)) || (st = make_arg(s, sc, vb, 1, &pb))) return st;
  hipError_t e = hipMemsetAsync(sc->red, 0, 2 * count * sizeof(double), s);
  if (e == hipSuccess) e = launch_distance(pa, pb, tstp, grids[0].d, (int)slice_elems(grids[0], tstp), sc->red, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, sc->red, 2 * count * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "cntr_distance");
  return CNTR_OK;
}

cntr_status cntr_solve_2b(const cntr_grid* grid, const cntr_gf* G, const cntr_gf* Sigma,
                          const cntr_gf* Gscratch, const void* eps0, const double* U,
                          void* eps_mf, double nbar, int32_t mats_maxit, double mats_tol,
                          double mats_mix, int32_t boot_maxit, double boot_tol, int32_t ncorr,
                          int32_t nt_stop, double* stats, void* stream) {
  if (capturing((hipStream_t)stream)) return fail(CNTR_EINVAL, "cntr_solve_2b: synchronizes the stream, not allowed during graph capture");
  if (!grid) return fail(CNTR_ESHAPE, "cntr_solve_2b: null grid");
  cntr_status st = check_grid(*grid, "cntr_solve_2b");
  if (st) return st;
  if (!gf_ok(G, 1) || !gf_ok(Sigma, 1) || !gf_ok(Gscratch, 1) || !eps0 || !U || !eps_mf)
    return fail(CNTR_ESHAPE, "cntr_solve_2b: null pointer");
  if (nt_stop < grid->k || nt_stop > grid->nt) return fail(CNTR_EORDER, "cntr_solve_2b: nt_stop outside k..nt");
  if ((st = ensure_weights())) return st;
  hipStream_t s = (hipStream_t)stream;
  const cntr_grid& g = *grid;
  int k = g.k, d = g.d;
  StreamScratch* sc = scratch_for(s);
  cntr_grid gmax = g;
  if (gmax.nt < k + 1) gmax.nt = k + 1;
  StepScratch lay = step_layout(gmax);
  if ((st = grow(s, sc, lay.per, 5, 2))) return st;
  Scratch scr = lay.sc;
  scr.base = sc->data();
  scr.stat = sc->stat();
  sc->nstat = std::max(sc->nstat, 1);
  Prob P = make_prob(g, G, Sigma, eps_mf);
  P.U = U;
  P.eps0 = (const cplx*)eps0;
  P.eps_mf = (cplx*)eps_mf;
  Prob Po = make_prob(g, Gscratch, nullptr, nullptr);
  ProbArg pa{P, nullptr, 1}, po{Po, nullptr, 1};
  hipError_t e;
  double dist[2];
  // distance summed over the slices n0..n1 (one read-back)
  auto distance = [&](int n0, int n1, double* out) -> cntr_status {
    hipError_t ee = hipMemsetAsync(sc->red, 0, 2 * sizeof(double), s);
    for (int n = n0; n <= n1 && !ee; n++) ee = launch_distance(pa, po, n, d, (int)slice_elems(g, n), sc->red, s);
    if (ee) return hip_fail(ee, "distance");
    return readback(s, out, sc->red, 2 * sizeof(double), "distance");
  };
  // Matsubara self-consistency. Initial G^M: free function of eps0_{-1}.
  if (!(mats_mix > 0 && mats_mix <= 1)) return fail(CNTR_EINVAL, "cntr_solve_2b: mats_mix outside (0,1]");
  int it = 0;
  double err = 0;
  if ((st = mats_loop_2b(g, P, pa, po, sc, nbar, mats_maxit, mats_tol, mats_mix, s, &it, &err))) return st;
  if (stats) {
    stats[0] = it;
    stats[2] = err;
  }
  // bootstrap over slices 0..k
  for (it = 0; it < boot_maxit; it++) {
    for (int n = 0; n <= k; n++)
      if ((e = launch_sigma2b(pa, n, d, (int)slice_elems(g, n), nbar, s))) return hip_fail(e, "Sigma start");
    for (int n = 0; n <= k; n++)
      if ((e = launch_copy(po, pa, n, d, (int)slice_elems(g, n), s))) return hip_fail(e, "copy");
    if ((e = launch_start(pa, scr, d, g.ntau, s))) return hip_fail(e, "start-up");
    if ((st = distance(0, k, dist))) return st;
    err = dist[0] / dist[1];
    if (err < boot_tol && it > 2) {
      it++;
      break;
    }
  }
  if (stats) {
    stats[1] = it;
    stats[3] = err;
  }
  // predictor-corrector time steps
  for (int n = k + 1; n <= nt_stop; n++) {
    if ((e = launch_extrapolate(pa, n - 1, d, (int)slice_elems(g, n), s))) return hip_fail(e, "extrapolate");
    for (int c = 0; c < ncorr; c++) {
      if ((e = launch_sigma2b(pa, n, d, (int)slice_elems(g, n), nbar, s))) return hip_fail(e, "Sigma");
      if ((e = launch_step(pa, scr, n, d, s))) return hip_fail(e, "step");
    }
  }
  for (int n = k + 1; n <= nt_stop; n++)
    if ((e = launch_sigma2b(pa, n, d, (int)slice_elems(g, n), nbar, s))) return hip_fail(e, "Sigma");
  order_mark(1, G, nt_stop, true);
  return CNTR_OK;
}


}  // extern "C"

namespace cntr {
namespace {

// Problems of one orbital count (and k, ntau) of a second-Born batch: the
// descriptors and scratch of their stream, and the phases of the solve.
struct Group2B {
  std::vector<int> idx;
  std::vector<Prob> v, vo;
  cntr_grid gmax{};
  int k = 0, d = 0, ntmax = 0;
  hipStream_t s = nullptr;
  StreamScratch* sc = nullptr;
  Scratch scr{};
  ProbArg pa{}, po{};
};

cntr_status group_setup(Group2B& g, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                        const cntr_gf* Gscratch, const void* const* eps0, const double* const* U,
                        void* const* eps_mf, hipStream_t s) {
  int count = (int)g.idx.size();
  g.s = s;
  g.k = grids[g.idx[0]].k;
  g.d = grids[g.idx[0]].d;
  g.ntmax = 0;
  for (int i : g.idx) g.ntmax = std::max(g.ntmax, (int)grids[i].nt);
  g.gmax = grids[g.idx[0]];
  g.gmax.nt = g.ntmax < g.k + 1 ? g.k + 1 : g.ntmax;
  g.sc = scratch_for(s);
  StepScratch lay = step_layout(g.gmax);
  cntr_status st = grow(s, g.sc, lay.per * count, 5 * (size_t)count, 2 * (size_t)count);
  if (st) return st;
  g.scr = lay.sc;
  g.scr.base = g.sc->data();
  g.scr.stat = g.sc->stat();
  g.sc->nstat = std::max(g.sc->nstat, count);
  g.v.resize(count);
  g.vo.resize(count);
  for (int q = 0; q < count; q++) {
    int i = g.idx[q];
    g.v[q] = make_prob(grids[i], &G[i], &Sigma[i], eps_mf[i]);
    g.v[q].U = U[i];
    g.v[q].eps0 = (const cplx*)eps0[i];
    g.v[q].eps_mf = (cplx*)eps_mf[i];
    g.vo[q] = make_prob(grids[i], &Gscratch[i], nullptr, nullptr);
  }
  if ((st = make_arg(s, g.sc, g.v, 0, &g.pa)) || (st = make_arg(s, g.sc, g.vo, 1, &g.po))) return st;
  return CNTR_OK;
}

// Matsubara loops one problem at a time (each has its own dense solve)
cntr_status group_mats(Group2B& g, const cntr_grid* grids, double nbar, int mats_maxit, double mats_tol,
                       double mats_mix, int* itmax, double* errmax) {
  for (size_t q = 0; q < g.idx.size(); q++) {
    ProbArg p1{g.v[q], nullptr, 1}, o1{g.vo[q], nullptr, 1};
    int it = 0;
    double err = 0;
    cntr_status st = mats_loop_2b(grids[g.idx[q]], g.v[q], p1, o1, g.sc, nbar, mats_maxit, mats_tol, mats_mix, g.s,
                                  &it, &err);
    if (st) return st;
    *itmax = std::max(*itmax, it);
    *errmax = std::max(*errmax, err);
  }
  return CNTR_OK;
}

// bootstrap of slices 0..k, one launch per kernel for the group; the
// tolerance applies to the largest relative distance of the group
cntr_status group_boot(Group2B& g, double nbar, int boot_maxit, double boot_tol, int* iters, double* err_out) {
  int count = (int)g.idx.size(), k = g.k, d = g.d;
  hipStream_t s = g.s;
  hipError_t e;
  std::vector<double> dist(2 * (size_t)count);
  int it;
  double err = 0;
  for (it = 0; it < boot_maxit; it++) {
    for (int n = 0; n <= k; n++)
      if ((e = launch_sigma2b(g.pa, n, d, (int)slice_elems(g.gmax, n), nbar, s))) return hip_fail(e, "Sigma start");
    for (int n = 0; n <= k; n++)
      if ((e = launch_copy(g.po, g.pa, n, d, (int)slice_elems(g.gmax, n), s))) return hip_fail(e, "copy");
    if ((e = launch_start(g.pa, g.scr, d, g.gmax.ntau, s))) return hip_fail(e, "start-up");
    std::vector<double> num(count, 0.0), den(count, 0.0);
    for (int n = 0; n <= k; n++) {
      e = hipMemsetAsync(g.sc->red, 0, 2 * (size_t)count * sizeof(double), s);
      if (!e) e = launch_distance(g.pa, g.po, n, d, (int)slice_elems(g.gmax, n), g.sc->red, s);
      if (!e) e = hipMemcpyAsync(dist.data(), g.sc->red, 2 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s);
      if (!e) e = hipStreamSynchronize(s);
      if (e) return hip_fail(e, "distance");
      for (int i = 0; i < count; i++) {
        num[i] += dist[2 * i];
        den[i] += dist[2 * i + 1];
      }
    }
    err = 0;
    for (int i = 0; i < count; i++) err = std::max(err, num[i] / den[i]);
    if (err < boot_tol && it > 2) {
      it++;
      break;
    }
  }
  *iters = it;
  *err_out = err;
  return CNTR_OK;
}

// predictor and ncorr corrector iterations of slice n for the problems of
// the group still running (enqueued on the group's stream, no waiting)
cntr_status group_step(Group2B& g, int n, int ncorr, double nbar) {
  if (n > g.ntmax) return CNTR_OK;
  hipError_t e;
  int d = g.d;
  if ((e = launch_extrapolate(g.pa, n - 1, d, (int)slice_elems(g.gmax, n), g.s))) return hip_fail(e, "extrapolate");
  for (int c = 0; c < ncorr; c++) {
    if ((e = launch_sigma2b(g.pa, n, d, (int)slice_elems(g.gmax, n), nbar, g.s))) return hip_fail(e, "Sigma");
    if ((e = launch_step(g.pa, g.scr, n, d, g.s))) return hip_fail(e, "step");
  }
  if ((e = launch_sigma2b(g.pa, n, d, (int)slice_elems(g.gmax, n), nbar, g.s))) return hip_fail(e, "Sigma");
  return CNTR_OK;
}

// one stream per orbital-count group beside the caller's (default priority)
hipStream_t group_stream(hipStream_t main, int slot) {
  static std::map<std::tuple<int, hipStream_t, int>, hipStream_t> tab;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t& x = tab[{dev, main, slot}];
  if (!x && hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) x = nullptr;
  return x;
}

cntr_status check_2b_args(int count, const cntr_gf* G, const cntr_gf* Sigma, const cntr_gf* Gscratch,
                          const void* const* eps0, const double* const* U, void* const* eps_mf, double mats_mix,
                          const char* what) {
  if (!gf_ok(G, count) || !gf_ok(Sigma, count) || !gf_ok(Gscratch, count) || !eps0 || !U || !eps_mf)
    return fail(CNTR_ESHAPE, std::string(what) + ": null pointer");
  for (int i = 0; i < count; i++)
    if (!eps0[i] || !U[i] || !eps_mf[i]) return fail(CNTR_ESHAPE, std::string(what) + ": null eps0, U or eps_mf");
  if (!(mats_mix > 0 && mats_mix <= 1)) return fail(CNTR_EINVAL, std::string(what) + ": mats_mix outside (0,1]");
  if (count > STAT_WORDS) return fail(CNTR_ESHAPE, std::string(what) + ": more than 65536 problems");
  return CNTR_OK;
}

}  // namespace
}  // namespace cntr

extern "C" {

cntr_status cntr_solve_2b_batch(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                                const cntr_gf* Gscratch, const void* const* eps0, const double* const* U,
                                void* const* eps_mf, double nbar, int32_t mats_maxit, double mats_tol,
                                double mats_mix, int32_t boot_maxit, double boot_tol, int32_t ncorr,
                                double* stats, void* stream) {
  if (capturing((hipStream_t)stream))
    return fail(CNTR_EINVAL, "cntr_solve_2b_batch: synchronizes the stream, not allowed during graph capture");
  cntr_status st = check_batch(count, grids, "cntr_solve_2b_batch");
  if (st) return st;
  if ((st = check_2b_args(count, G, Sigma, Gscratch, eps0, U, eps_mf, mats_mix, "cntr_solve_2b_batch"))) return st;
  if ((st = ensure_weights())) return st;
  Group2B g;
  for (int i = 0; i < count; i++) g.idx.push_back(i);
  if ((st = group_setup(g, grids, G, Sigma, Gscratch, eps0, U, eps_mf, (hipStream_t)stream))) return st;
  int itmax = 0, bit = 0;
  double errmax = 0, berr = 0;
  if ((st = group_mats(g, grids, nbar, mats_maxit, mats_tol, mats_mix, &itmax, &errmax))) return st;
  if (stats) {
    stats[0] = itmax;
    stats[2] = errmax;
  }
  if ((st = group_boot(g, nbar, boot_maxit, boot_tol, &bit, &berr))) return st;
  if (stats) {
    stats[1] = bit;
    stats[3] = berr;
  }
  for (int n = g.k + 1; n <= g.ntmax; n++)
    if ((st = group_step(g, n, ncorr, nbar))) return st;
  for (int i = 0; i < count; i++) order_mark(1, &G[i], grids[i].nt, true);
  return CNTR_OK;
}

cntr_status cntr_solve_2b_uneven(int32_t count, const cntr_grid* grids, const cntr_gf* G, const cntr_gf* Sigma,
                                 const cntr_gf* Gscratch, const void* const* eps0, const double* const* U,
                                 void* const* eps_mf, double nbar, int32_t mats_maxit, double mats_tol,
                                 double mats_mix, int32_t boot_maxit, double boot_tol, int32_t ncorr,
                                 double* stats, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (capturing(s))
    return fail(CNTR_EINVAL, "cntr_solve_2b_uneven: synchronizes the stream, not allowed during graph capture");
  if (count < 1 || !grids) return fail(CNTR_ESHAPE, "cntr_solve_2b_uneven: empty batch");
  cntr_status st;
  for (int i = 0; i < count; i++)
    if ((st = check_grid(grids[i], "cntr_solve_2b_uneven"))) return st;
  if ((st = check_2b_args(count, G, Sigma, Gscratch, eps0, U, eps_mf, mats_mix, "cntr_solve_2b_uneven"))) return st;
  if ((st = ensure_weights())) return st;
  // groups of equal (d, k, ntau), in order of first appearance
  std::vector<Group2B> gs;
  for (int i = 0; i < count; i++) {
    size_t q = 0;
    for (; q < gs.size(); q++) {
      const cntr_grid& a = grids[gs[q].idx[0]];
      if (a.d == grids[i].d && a.k == grids[i].k && a.ntau == grids[i].ntau) break;
    }
    if (q == gs.size()) gs.emplace_back();
    gs[q].idx.push_back(i);
  }
  if (gs.size() > 16) return fail(CNTR_ESHAPE, "cntr_solve_2b_uneven: more than 16 groups of (d, k, ntau)");
  // every group on a stream of its own, forked from s
  hipEvent_t fork = nullptr;
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(fork, s);
  if (e != hipSuccess) return hip_fail(e, "cntr_solve_2b_uneven: fork");
  for (size_t q = 0; q < gs.size(); q++) {
    hipStream_t gsq = group_stream(s, (int)q);
    if (!gsq) {
      (void)hipEventDestroy(fork);
      return fail(CNTR_EHIP, "cntr_solve_2b_uneven: group stream");
    }
    if ((e = hipStreamWaitEvent(gsq, fork, 0))) return hip_fail(e, "cntr_solve_2b_uneven: fork wait");
    if ((st = group_setup(gs[q], grids, G, Sigma, Gscratch, eps0, U, eps_mf, gsq))) return st;
  }
  (void)hipEventDestroy(fork);
  int itmax = 0, bmax = 0;
  double errmax = 0, bemax = 0;
  for (auto& g : gs)
    if ((st = group_mats(g, grids, nbar, mats_maxit, mats_tol, mats_mix, &itmax, &errmax))) return st;
  for (auto& g : gs) {
    int bit = 0;
    double berr = 0;
    if ((st = group_boot(g, nbar, boot_maxit, boot_tol, &bit, &berr))) return st;
    bmax = std::max(bmax, bit);
    bemax = std::max(bemax, berr);
  }
  if (stats) {
    stats[0] = itmax;
    stats[1] = bmax;
    stats[2] = errmax;
    stats[3] = bemax;
  }
  // time steps: slice n of every group in turn, each group on its stream, so
  // that the groups' kernels run side by side
  int ntmax = 0, k = gs[0].k;
  for (auto& g : gs) {
    ntmax = std::max(ntmax, g.ntmax);
    k = std::min(k, g.k);
  }
  for (int n = k + 1; n <= ntmax; n++)
    for (auto& g : gs)
      if (n > g.k && (st = group_step(g, n, ncorr, nbar))) return st;
  // join: s waits for every group
  for (auto& g : gs) {
    hipEvent_t j = nullptr;
    e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(j, g.s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, j, 0);
    if (j) (void)hipEventDestroy(j);
    if (e != hipSuccess) return hip_fail(e, "cntr_solve_2b_uneven: join");
  }
  for (int i = 0; i < count; i++) order_mark(1, &G[i], grids[i].nt, true);
  return CNTR_OK;
}

}  // extern "C"
