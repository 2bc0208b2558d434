// C ABI of the PMINRES solver (see include/bltt.h): handle lifecycle, table
// upload, the FP64 MINRES loop and the FP32-inside-FP64 refinement loop.
//
// Method: preconditioned MINRES (Paige-Saunders, in the Elman-Silvester-Wathen
// form) on Y A u = Y f with P_alpha = |C_alpha| (Li, Lin, Hon, Wu, arXiv
// 2307.07749, Sections 2-3 and 5.1).  Every vector operation runs in the HIP
// kernels of this library; the host only sequences launches and reads back the
// FP64 scalar state once per iteration.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <functional>
#include <vector>

#include "bltt.h"
#include "host_tables.hpp"
#include "launchers.hpp"
#include "plan_cache.hpp"

using namespace bltt;

// ---------------------------------------------------------------------------
// Device scratch of bltt_modes_lanczos_noalloc, one copy per GPU (a static
// device array is instantiated on every device the library runs on and holds
// it until the process ends).  Layout in doubles: per-workgroup partial sums,
// the first stage of their reduction, the step's coefficients, the scalar
// state the reduction writes.  Host code uses the address hipGetSymbolAddress
// returns for the current device, never the array's name.
// ---------------------------------------------------------------------------
namespace scr {
constexpr int64_t PARTS = 16384;    // partial sums of one launch, at most
constexpr int64_t RED_HALF = 32;    // first reduction stage: 2 * RED_HALF doubles
constexpr int64_t RED = PARTS;
constexpr int64_t COEF = RED + 2 * RED_HALF;
constexpr int64_t STATE = COEF + 8;
constexpr int64_t LEN = STATE + (int64_t)((sizeof(SolverState) + 7) / 8);
}  // namespace scr

static __device__ __align__(256) double scratch[scr::LEN];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// this device's copy of `scratch` (dev must be the current device); resolved
// once per device
int scratch_init(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= MAX_DEVICES) return BLTT_EHIP;
  if (g_scratch_ptr[dev]) return BLTT_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return BLTT_EHIP;
  }
  g_scratch_ptr[dev] = static_cast<double*>(p);
  return BLTT_OK;
}

double* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev >= 0 && dev < MAX_DEVICES ? g_scratch_ptr[dev] : nullptr;
}

}  // namespace

namespace {

template <typename T>
struct DeviceTables {
  cx<T>* tw_time = nullptr;
  cx<T>* tw_dst[3] = {nullptr, nullptr, nullptr};
  T* dinv = nullptr;
  T* d2 = nullptr;
  cx<T>* sigma = nullptr;
  cx<T>* rho = nullptr;
  T* mu = nullptr;
  cx<T>* tw_mv = nullptr;  // length 2N
  cx<T>* phat = nullptr;
  cx<T>* chat = nullptr;   // circulant / skew-circulant spectra of p (sine basis)
  cx<T>* shat = nullptr;
  cx<T>* omega = nullptr;  // e^{i pi n/N}
  bool ready = false;
};

template <typename T>
struct Workspace {
  T* Q = nullptr;  // matvec output / transform scratch
  T* V[3] = {nullptr, nullptr, nullptr};
  T* Z[2] = {nullptr, nullptr};
  T* W[2] = {nullptr, nullptr};
  T* X = nullptr;  // inner solution (FP32 refinement sweeps)
  bool ready = false;
  bool dirs = false;  // W (and X) allocated
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

hipError_t g_config_err = hipSuccess;

// layout of bltt_handle::step_dev
constexpr int STEP_COEF = 0, STEP_SCALE = 4, STEP_Y = 8, STEP_LEN = STEP_Y + ZB_MAX;

// Executable graphs of one form of the sine-basis MINRES loop, one per
// iteration position (the buffers an iteration touches repeat with the
// rotation of the Lanczos and direction vectors; a stored-basis sweep writes a
// new pool vector at every position).  pubs: the mirror publications one
// replay makes.  X and hist: the iterate and history buffers the nodes write;
// a call with other ones rebuilds the graphs.
struct IterGraphs {
  static constexpr int CAP = ZB_MAX > 7 ? ZB_MAX : 7;
  hipGraphExec_t exec[CAP] = {};
  int32_t pubs[CAP] = {};
  const void* X = nullptr;
  const double* hist = nullptr;
  void reset() {
    for (hipGraphExec_t& e : exec) {
      if (e) (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
    X = nullptr;
    hist = nullptr;
  }
};

}  // namespace

struct bltt_handle {
  uint32_t magic = HANDLE_MAGIC;  // first member (bltt_destroy tells handle types apart)
  hipStream_t stream = nullptr;
  int device = 0;  // device current at setup (its scratch copy serves the no-alloc entry point)
  int dim = 0;
  int m[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int64_t N = 0, M = 0, n = 0;
  double alpha = 1.0;
  bltt_options opt{};
  double c0 = 0.0;
  std::vector<double> p, q;
  int ptaps = 0, qtaps = 0;
  // variable coefficient (Section 5.2): L_{a,h} from face coefficients in the
  // operator, the mean-coefficient system abar L_h in the preconditioner
  bool var = false;
  double abar = 1.0;
  double* face_dev[3] = {nullptr, nullptr, nullptr};
  DeviceTables<float> t32;
  DeviceTables<double> t64;
  Workspace<float> w32;
  Workspace<double> w64;
  double* R64 = nullptr;
  double* F64 = nullptr;       // sine basis: (I_N x U) f
  double* partials = nullptr;
  int64_t partials_cap = 0;
  double* red_scratch = nullptr;  // first stage of long reductions (2 * red_half)
  int64_t max_blocks = 1024;      // workgroups of the persistent sine-basis kernels
  int64_t red_half = 0;
  double* partials_aux = nullptr;  // time pass: spatial part of the next <q, z>
  int64_t np_aux = 0;
  SolverState* state = nullptr;
  SolverState* state_host = nullptr;
  // host-mapped pinned copy of the state that every scalar kernel publishes
  // (mirror: host address, mirror_dev: its device address); seq_host counts
  // the publications enqueued, so the host waits for mirror->seq to reach it
  SolverState* mirror = nullptr;
  SolverState* mirror_dev = nullptr;
  int32_t seq_host = 0;
  // one HIP graph per iteration position of the sine-basis MINRES loop,
  // captured on cap_stream (the caller's stream may be the null stream, which
  // cannot be captured) and launched on stream
  hipStream_t cap_stream = nullptr;
  IterGraphs graphs[3];  // FP64 direction form, FP32 direction form, FP32 stored basis
  double* hist_dev = nullptr;
  int64_t hist_cap = 0;
  double* coef_one = nullptr;
  // step entry points: coefficients and refinement weights copied from the host
  // (STEP_COEF: 4 Lanczos coefficients, STEP_SCALE: 1 scale, STEP_Y: ZB_MAX weights)
  double* step_dev = nullptr;
  // stored-basis sweeps (mixed, sine basis): Z_0..Z_{K-1} and the
  // coefficient arrays of the directions and of the iterate
  float* zpool[ZB_MAX] = {};
  int zb_K = 0;
  double* zb_dev = nullptr;  // 3*ZB_MAX doubles: om (2K), y (K)
  double setup_ms = 0.0;
  std::string plan_cache;  // autotuner plan file ("" = none)
  // plans of the FP32 sine-basis kernels: radix plans of the time pass and of
  // the N-point matvec, workgroups of the persistent time pass (tuned at setup)
  int plan_time = 0, plan_cs = 0;
  int64_t time_blocks = 0;  // 0: max_blocks
  int64_t cs_blocks = 0;    // FP32 N-point matvec workgroups, 0: one per tile
  double* rsc_dev = nullptr;  // 1/scale of the FP32 residual the refinement hands to its next sweep
  int plan_source = BLTT_PLAN_SOURCE_DEFAULT;
  std::vector<void*> allocs;
  // per-kernel timing (bltt_profile_enable)
  struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

#define HIPCHK(...)                        \
  do {                                     \
    hipError_t e_ = (__VA_ARGS__);         \
    if (e_ != hipSuccess) return BLTT_EHIP; \
  } while (0)

namespace {

hipEvent_t prof_event(bltt_handle* h) {
  if (h->pool_used == h->pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->pool.push_back(e);
  }
  return h->pool[h->pool_used++];
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
  ProfScope(bltt_handle* h_, int cls_, double bytes_) : h(h_), cls(cls_), bytes(bytes_) {
    if (h->prof) {
      a = prof_event(h);
      if (a) (void)hipEventRecord(a, h->stream);
    }
  }
  ~ProfScope() {
    if (h->prof && a) {
      hipEvent_t b = prof_event(h);
      if (b) {
        (void)hipEventRecord(b, h->stream);
        h->recs.push_back({cls, a, b, bytes});
      }
    }
  }
  bltt_handle* h;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
};

template <typename T>
int dalloc(bltt_handle* h, T** ptr, size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, count * sizeof(T) + 64) != hipSuccess) {
    (void)hipGetLastError();
    return BLTT_ENOMEM;
  }
  h->allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return BLTT_OK;
}

template <typename T, typename S>
int upload(bltt_handle* h, T** dst, const std::vector<S>& src) {
  std::vector<T> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
  int rc = dalloc(h, dst, tmp.size());
  if (rc) return rc;
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return BLTT_OK;
}

template <typename T>
int upload_c(bltt_handle* h, cx<T>** dst, const std::vector<host::cd>& src) {
  std::vector<cx<T>> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = mkc<T>((T)src[i].real(), (T)src[i].imag());
  int rc = dalloc(h, dst, tmp.size());
  if (rc) return rc;
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(cx<T>), hipMemcpyHostToDevice));
  return BLTT_OK;
}

template <typename T>
DeviceTables<T>& tables(bltt_handle* h);
template <>
DeviceTables<float>& tables<float>(bltt_handle* h) { return h->t32; }
template <>
DeviceTables<double>& tables<double>(bltt_handle* h) { return h->t64; }
template <typename T>
Workspace<T>& workspace(bltt_handle* h);
template <>
Workspace<float>& workspace<float>(bltt_handle* h) { return h->w32; }
template <>
Workspace<double>& workspace<double>(bltt_handle* h) { return h->w64; }

bool short_p(const bltt_handle* h) { return h->ptaps <= 8; }

// workgroups and radix plan of the time pass, radix plan of the N-point matvec
// for precision T (the tuned ones apply to FP32; FP64 runs the defaults)
template <typename T>
int64_t time_blocks(const bltt_handle* h) {
  return sizeof(T) == 4 && h->time_blocks > 0 ? h->time_blocks : h->max_blocks;
}
template <typename T>
int time_plan(const bltt_handle* h) { return sizeof(T) == 4 ? h->plan_time : 0; }
template <typename T>
int cs_plan(const bltt_handle* h) { return sizeof(T) == 4 ? h->plan_cs : 0; }
template <typename T>
int64_t cs_blocks(const bltt_handle* h) { return sizeof(T) == 4 ? h->cs_blocks : 0; }

// alpha of the preconditioner that precision T applies (ALPHA_MIN_FP32)
template <typename T>
double prec_alpha(const bltt_handle* h) {
  return sizeof(T) == 4 ? std::max(h->alpha, ALPHA_MIN_FP32) : h->alpha;
}

template <typename T>
int build_tables(bltt_handle* h) {
  DeviceTables<T>& t = tables<T>(h);
  if (t.ready) return BLTT_OK;
  int rc;
  if ((rc = upload_c<T>(h, &t.tw_time, host::twiddles((int)h->N)))) return rc;
  for (int d = 0; d < h->dim; ++d)
    if ((rc = upload_c<T>(h, &t.tw_dst[d], host::twiddles(2 * (h->m[d] + 1))))) return rc;
  const double alpha = prec_alpha<T>(h);
  if ((rc = upload<T>(h, &t.dinv, host::alpha_pow(h->N, alpha, -1.0)))) return rc;
  if ((rc = upload<T>(h, &t.d2, host::alpha_pow(h->N, alpha, 2.0)))) return rc;
  if ((rc = upload_c<T>(h, &t.sigma, host::alpha_spectrum(h->p, alpha)))) return rc;
  if ((rc = upload_c<T>(h, &t.rho, host::alpha_spectrum(h->q, alpha)))) return rc;
  {
    // Laplacian eigenvalue of each sine mode, of abar L_h for a variable coefficient
    std::vector<double> mu = host::lap_eigs(h->dim, h->m, h->h);
    for (double& v : mu) v *= h->abar;
    if ((rc = upload<T>(h, &t.mu, mu))) return rc;
  }
  if (!short_p(h)) {
    if ((rc = upload_c<T>(h, &t.tw_mv, host::twiddles((int)(2 * h->N))))) return rc;
    if ((rc = upload_c<T>(h, &t.phat, host::matvec_spectrum(h->p)))) return rc;
    if ((rc = upload_c<T>(h, &t.chat, host::circulant_spectrum(h->p, false)))) return rc;
    if ((rc = upload_c<T>(h, &t.shat, host::circulant_spectrum(h->p, true)))) return rc;
    if ((rc = upload_c<T>(h, &t.omega, host::half_roots(h->N)))) return rc;
  }
  t.ready = true;
  return BLTT_OK;
}

// Krylov workspace of one precision; dirs: also the explicit direction
// vectors W (and the FP32 inner solution X), which the stored-basis sweeps
// and the step entry points do not need
template <typename T>
int build_workspace(bltt_handle* h, bool dirs) {
  Workspace<T>& w = workspace<T>(h);
  int rc;
  const size_t n = (size_t)h->n;
  if (!w.ready) {
    if ((rc = dalloc(h, &w.Q, n))) return rc;
    for (int i = 0; i < 3; ++i)
      if ((rc = dalloc(h, &w.V[i], n))) return rc;
    for (int i = 0; i < 2; ++i)
      if ((rc = dalloc(h, &w.Z[i], n))) return rc;
    w.ready = true;
  }
  if (dirs && !w.dirs) {
    for (int i = 0; i < 2; ++i)
      if ((rc = dalloc(h, &w.W[i], n))) return rc;
    if (sizeof(T) == 4)
      if ((rc = dalloc(h, &w.X, n))) return rc;
    w.dirs = true;
  }
  return BLTT_OK;
}

// Pool of stored Z vectors for the FP32 sweeps: K = 16 (ZB_MAX at most), fewer
// when device memory is short (at least 4).  Z[0], Z[1] of the workspace are
// the first two.
constexpr int ZB_DEFAULT = 16;
int build_zpool(bltt_handle* h) {
  if (h->zb_K) return BLTT_OK;
  int rc;
  Workspace<float>& w = h->w32;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return BLTT_EHIP;
  const double per = (double)h->n * sizeof(float) + 64;
  int K = ZB_DEFAULT;
  const int fit = (int)std::min<double>(ZB_MAX, 2.0 + 0.6 * (double)free_b / per);
  if (fit < K) K = fit;
  if (K < 4) return BLTT_ENOMEM;
  h->zpool[0] = w.Z[0];
  h->zpool[1] = w.Z[1];
  for (int i = 2; i < K; ++i)
    if ((rc = dalloc(h, &h->zpool[i], (size_t)h->n))) return rc;
  if ((rc = dalloc(h, &h->zb_dev, (size_t)(3 * ZB_MAX)))) return rc;
  h->zb_K = K;
  return BLTT_OK;
}

Grid make_grid(const bltt_handle* h) {
  Grid g;
  g.dim = h->dim;
  for (int d = 0; d < 3; ++d) {
    g.m[d] = h->m[d];
    g.inv_h2[d] = d < h->dim ? 1.0 / (h->h[d] * h->h[d]) : 0.0;
    g.face[d] = h->face_dev[d];
  }
  return g;
}

template <typename T>
int64_t partials_needed(const bltt_handle* h) {
  int64_t need = ew_blocks(h->n);
  if (short_p(h)) {
    const int64_t gx = (h->M + TPB_EW - 1) / TPB_EW;
    const int64_t gy = ((h->N + 1) / 2 + 7) / 8;
    need = std::max(need, gx * gy);
  } else {
    need = std::max({need, mv_blocks<T>(false, (int)(2 * h->N), h->M), mv_blocks<T>(true, (int)(2 * h->N), h->M)});
  }
  need = std::max(need, fft_blocks<T, FK_DSTX>(2 * (h->m[0] + 1), h->n / h->m[0]));
  need = std::max(need, h->n / h->m[0]);  // one partial per x-line (residual stencil pass)
  need = std::max(need, fft_blocks<T, FK_TIME>((int)h->N, h->M));
  need = std::max(need, fft_tiles<T, FK_SPEC>((int)h->N, h->M));  // sine-basis kernels
  need = std::max(need, ((h->M + TR_TILE - 1) / TR_TILE) * ((h->N + TR_TILE - 1) / TR_TILE));  // transpose + norm
  return need;
}

template <typename T>
VupdStencil<T> vupd_stencil(bltt_handle* h, const T* z) {
  VupdStencil<T> st;
  st.z = z;
  for (int k = 0; k < 4; ++k) st.q[k] = (T)(k < h->qtaps ? h->q[(size_t)k] : 0.0);
  st.qtaps = h->qtaps;
  st.grid = make_grid(h);
  st.N = (int)h->N;
  st.R = h->M / h->m[0];
  return st;
}

template <typename T>
MatvecTables<T> mv_tables(bltt_handle* h) {
  DeviceTables<T>& t = tables<T>(h);
  MatvecTables<T> tb;
  tb.tw = t.tw_mv;
  tb.phat = t.phat;
  tb.mu = t.mu;
  for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < h->qtaps ? h->q[(size_t)k] : 0.0);
  tb.qtaps = h->qtaps;
  tb.grid = make_grid(h);
  tb.mx = (int)h->m[0];
  return tb;
}

template <typename T>
MatvecCSTables<T> cs_tables(bltt_handle* h) {
  DeviceTables<T>& t = tables<T>(h);
  MatvecCSTables<T> tb;
  tb.tw = t.tw_time;
  tb.chat = t.chat;
  tb.shat = t.shat;
  tb.omega = t.omega;
  tb.mu = t.mu;
  for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < h->qtaps ? h->q[(size_t)k] : 0.0);
  tb.qtaps = h->qtaps;
  tb.mx = (int)h->m[0];
  return tb;
}

// q = Y A z (MV_DOT, partial sums of <q, z>) or out = Y (fin - A z) (MV_RESID,
// partial sums of the squared norm).  term selects the spatial part:
// TERM_STENCIL the full physical-space operator, TERM_NONE only Y (p * z)
// (inside the physical-space MINRES the spatial term is added by the x-line
// pass of the preconditioner and its share of <q, z> comes from the preceding
// time pass), TERM_SPEC the sine-coordinate operator (mu_i on mode i).
template <typename T>
int matvec(bltt_handle* h, int mode, int term, const T* z, T* out, const T* fin, int64_t* np) {
  DeviceTables<T>& t = tables<T>(h);
  if (short_p(h)) {
    ShortTables<T> tb;
    for (int k = 0; k < 8; ++k) tb.p[k] = (T)(k < h->ptaps ? h->p[(size_t)k] : 0.0);
    tb.ptaps = h->ptaps;
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < h->qtaps ? h->q[(size_t)k] : 0.0);
    tb.qtaps = h->qtaps;
    tb.grid = make_grid(h);
    tb.N = (int)h->N;
    tb.chunk = 8;
    tb.term = term;
    tb.mu = t.mu;
    ProfScope ps(h, mode == MV_DOT ? BLTT_K_MATVEC : BLTT_K_RESID64, (mode == MV_DOT ? 2.0 : 3.0) * h->n * sizeof(T));
    HIPCHK(launch_matvec_short<T>(mode, z, out, fin, h->M, tb, h->partials, np, h->stream));
  } else {
    MatvecTables<T> tb;
    tb.tw = t.tw_mv;
    tb.phat = t.phat;
    tb.mu = t.mu;
    for (int k = 0; k < 4; ++k) tb.q[k] = (T)(k < h->qtaps ? h->q[(size_t)k] : 0.0);
    tb.qtaps = h->qtaps;
    tb.grid = make_grid(h);
    IterUpd up{};
    if (term == TERM_SPEC && sizeof(T) == 4) {
      // FP32: N-point circulant + skew-circulant form (one wavefront per line pair)
      ProfScope ps(h, mode == MV_DOT ? BLTT_K_MATVEC : BLTT_K_RESID64, (mode == MV_DOT ? 2.0 : 3.0) * h->n * sizeof(T));
      HIPCHK(launch_matvec_cs<T>((int)h->N, mode, const_cast<T*>(z), out, fin, h->M, cs_tables<T>(h), up,
                                 h->partials, cs_blocks<T>(h), np, h->stream, cs_plan<T>(h)));
      return BLTT_OK;
    }
    if (mode == MV_RESID && term == TERM_STENCIL && !h->var) {
      // r = Y (f - p * u) on time lines, then the spatial term and ||r||^2 on x-lines
      const int64_t nlx = h->n / h->m[0];
      {
        ProfScope ps(h, BLTT_K_RESID64, 3.0 * h->n * sizeof(T));
        HIPCHK(launch_matvec_fft<T>((int)(2 * h->N), MV_RESID, TERM_NONE, const_cast<T*>(z), out, fin, h->M, tb, up,
                                    h->partials,
                                    h->stream));
      }
      ProfScope ps(h, BLTT_K_RESID64, 3.0 * h->n * sizeof(T));
      HIPCHK(launch_resid_stencil<T>(out, vupd_stencil<T>(h, z), nlx, h->partials, np, h->stream));
    } else {
      ProfScope ps(h, mode == MV_DOT ? BLTT_K_MATVEC : BLTT_K_RESID64, (mode == MV_DOT ? 2.0 : 3.0) * h->n * sizeof(T));
      HIPCHK(launch_matvec_fft<T>((int)(2 * h->N), mode, term, const_cast<T*>(z), out, fin, h->M, tb, up, h->partials,
                                  h->stream));
      *np = mv_blocks<T>(term == TERM_SPEC, (int)(2 * h->N), h->M);
    }
  }
  return BLTT_OK;
}

template <typename T>
DstTables<T> dst_tables(bltt_handle* h, int d) {
  DstTables<T> tb;
  tb.tw = tables<T>(h).tw_dst[d];
  tb.m = h->m[d];
  tb.nrm = (T)(1.0 / std::sqrt(2.0 * (h->m[d] + 1)));
  return tb;
}

// strided sine transforms along dimensions 1..dim-1 (in place on x)
template <typename T>
int space_strided(bltt_handle* h, T* x, bool reverse) {
  for (int k = 1; k < h->dim; ++k) {
    const int d = reverse ? h->dim - k : k;
    int64_t S = 1;
    for (int e = 0; e < d; ++e) S *= h->m[e];
    const int64_t nlines = h->n / h->m[d];
    ProfScope ps(h, BLTT_K_DST_STRIDED, 2.0 * h->n * sizeof(T));
    HIPCHK(launch_dst_strided<T>(2 * (h->m[d] + 1), x, nlines, S, dst_tables<T>(h, d), h->stream));
  }
  return BLTT_OK;
}

template <typename T>
TimeTables<T> time_tables(bltt_handle* h, bool aux) {
  TimeTables<T> tt;
  DeviceTables<T>& t = tables<T>(h);
  tt.tw = t.tw_time;
  tt.dinv = t.dinv;
  tt.d2 = t.d2;
  tt.sigma = t.sigma;
  tt.rho = t.rho;
  tt.mu = t.mu;
  tt.log2_alpha_over_N = (T)(std::log2(prec_alpha<T>(h)) / (double)h->N);
  for (int k = 0; k < 4; ++k) tt.q[k] = (T)(k < h->qtaps ? h->q[(size_t)k] : 0.0);
  tt.qtaps = h->qtaps;
  tt.aux = aux ? h->partials_aux : nullptr;
  tt.mx = (int)h->m[0];
  return tt;
}

// zout = P^{-1} vhat with vhat = coef[0] in + coef[1] v1 + coef[2] v2 (written to
// vout when non-null); tmp is scratch and may equal `in`; partial sums of
// <vdot, zout> are left in h->partials (count in *np).
// zstencil: z_j whose spatial matvec term joins the Lanczos update (nullptr:
// none).  aux: when true the time pass also leaves the spatial part of the
// next <q, z> in h->partials_aux.
template <typename T>
int precond(bltt_handle* h, const T* in, const T* v1, const T* v2, T* vout, const double* coef, T* tmp,
            const T* vdot, T* zout, int64_t* np, const T* zstencil = nullptr, bool aux = false) {
  int rc;
  const int Lx = 2 * (h->m[0] + 1);
  const int64_t nlx = h->n / h->m[0];
  {
    const double streams = 2.0 + (v1 ? 1 : 0) + (v2 ? 1 : 0) + (vout ? 1 : 0) + (zstencil ? 1 : 0);
    ProfScope ps(h, BLTT_K_DST_X_VUPD, streams * h->n * sizeof(T));
    HIPCHK(launch_dst_x<T>(Lx, KIND_VUPD, in, v1, v2, vout, nullptr, tmp, nlx, dst_tables<T>(h, 0), coef, nullptr,
                           vupd_stencil<T>(h, zstencil), h->stream));
  }
  if ((rc = space_strided<T>(h, tmp, false))) return rc;
  const TimeTables<T> tt = time_tables<T>(h, aux);
  if (aux) h->np_aux = fft_blocks<T, FK_TIME>((int)h->N, h->M);
  {
    ProfScope ps(h, BLTT_K_TIME, 2.0 * h->n * sizeof(T));
    HIPCHK(launch_time_prec<T>((int)h->N, tmp, h->M, tt, h->stream));
  }
  if ((rc = space_strided<T>(h, tmp, true))) return rc;
  {
    ProfScope ps(h, BLTT_K_DST_X_DOT, 3.0 * h->n * sizeof(T));
    HIPCHK(launch_dst_x<T>(Lx, KIND_DOT, tmp, nullptr, nullptr, nullptr, vdot, zout, nlx, dst_tables<T>(h, 0), coef,
                           h->partials, vupd_stencil<T>(h, nullptr), h->stream));
  }
  *np = fft_blocks<T, FK_DSTX>(Lx, nlx);
  return BLTT_OK;
}

// Every phase the host reads afterwards publishes the state to the host
// mirror; the delta phase, read by the device only, does not.
int scalar(bltt_handle* h, int phase, int64_t np, double* hist, bool with_aux = false, bool zbasis = false) {
  ProfScope ps(h, BLTT_K_OTHER, 8.0 * np);
  const bool publish = phase != SC_DELTA;
  ZBasis zb;
  zb.om = zbasis ? h->zb_dev : nullptr;
  zb.y = zbasis ? h->zb_dev + 2 * h->zb_K : nullptr;
  zb.K = zbasis ? h->zb_K : 0;
  HIPCHK(launch_scalar(phase, h->state, h->partials, np, with_aux ? h->partials_aux : nullptr,
                       with_aux ? h->np_aux : 0, hist, h->red_scratch, h->red_half, zb, h->stream,
                       publish ? h->mirror_dev : nullptr));
  if (publish) h->seq_host += 1;
  return BLTT_OK;
}

// The state after the last scalar kernel enqueued: wait until its publication
// reaches the host mirror (polling, with the stream queried now and then so a
// finished stream whose mirror did not move is an error rather than a hang),
// then copy it to state_host.  Work enqueued after that scalar kernel may
// still be running.
int read_state(bltt_handle* h) {
  const int32_t want = h->seq_host;
  for (uint32_t spin = 0;; ++spin) {
    if (__atomic_load_n(&h->mirror->seq, __ATOMIC_ACQUIRE) == want) break;
    if ((spin & 255u) == 255u) {
      const hipError_t q = hipStreamQuery(h->stream);
      if (q == hipSuccess) {
        if (__atomic_load_n(&h->mirror->seq, __ATOMIC_ACQUIRE) == want) break;
        return BLTT_EHIP;
      }
      if (q != hipErrorNotReady) return BLTT_EHIP;
    }
  }
  std::memcpy(h->state_host, (const void*)h->mirror, sizeof(SolverState));
  return BLTT_OK;
}

// Record what step() enqueues on h->stream into *exec (step runs with
// h->stream set to the handle's capture stream), then launch it on the
// caller's stream.  The publications step() counted into seq_host are the
// graph's; *pubs keeps their number for later replays.
template <class Step>
int capture_and_launch(bltt_handle* h, Step&& step, hipGraphExec_t* exec, int32_t* pubs) {
  if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  const hipStream_t user = h->stream;
  const int32_t seq0 = h->seq_host;
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  h->stream = h->cap_stream;
  const int rc = step();
  h->stream = user;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
  hipError_t ei = hipErrorUnknown;
  if (!rc && e == hipSuccess && graph) ei = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (rc || ei != hipSuccess) {
    *exec = nullptr;
    h->seq_host = seq0;
    return rc ? rc : BLTT_EHIP;
  }
  *pubs = h->seq_host - seq0;
  HIPCHK(hipGraphLaunch(*exec, h->stream));
  return BLTT_OK;
}

int ensure_hist(bltt_handle* h, int64_t need) {
  if (h->hist_cap >= need) return BLTT_OK;
  double* p = nullptr;
  int rc = dalloc(h, &p, (size_t)need);
  if (rc) return rc;
  h->hist_dev = p;
  h->hist_cap = need;
  return BLTT_OK;
}

struct CoreResult {
  int iters = 0;
  int status = 0;  // BLTT_OK / BLTT_NOCONV / error
  double relres = -1.0;
};

// MINRES on K x = b, b already in ws.V[0]; X must be zero on entry.
// Stops when |eta_j|/eta_0 <= eta_tol, confirmed (when f_dev != nullptr, FP64
// only) by the explicit residual ||Y(f - A x)|| <= tol * bnorm.
template <typename T, typename TX>
int minres_core(bltt_handle* h, TX* X, int maxit, double eta_tol, const double* f_dev, double tol, double bnorm,
                double* hist_host, CoreResult* res) {
  Workspace<T>& ws = workspace<T>(h);
  hipStream_t s = h->stream;
  int rc;
  int64_t np = 0;
  T* Vc = ws.V[0];
  T* Vp = ws.V[1];
  T* Vn = ws.V[2];
  T* Zc = ws.Z[0];
  T* Zn = ws.Z[1];
  T* Wa = ws.W[0];
  T* Wb = ws.W[1];
  {
    ProfScope ps(h, BLTT_K_OTHER, 2.0 * h->n * sizeof(T));
    HIPCHK(launch_fill<T>(Wa, h->n, T(0), s));
    HIPCHK(launch_fill<T>(Wb, h->n, T(0), s));
  }
  if ((rc = ensure_hist(h, (int64_t)maxit + 2))) return rc;
  // Constant coefficient: the time-line matvec leaves out the stencil, which
  // the x-line pass of the Lanczos update adds, and the stencil's share of
  // delta comes from the previous time pass in sine coordinates.  A variable
  // coefficient is not sine-diagonal: the matvec carries the whole operator.
  const bool split = !h->var;
  // z_1 = P^{-1} b, beta_1 = sqrt(<b, z_1>)
  if ((rc = precond<T>(h, Vc, nullptr, nullptr, nullptr, h->coef_one, ws.Q, Vc, Zc, &np, nullptr, split))) return rc;
  if ((rc = scalar(h, SC_START, np, h->hist_dev))) return rc;
  if ((rc = read_state(h))) return rc;
  if (h->state_host->status == -3) return BLTT_ENAN;
  if (h->state_host->status == -4) return BLTT_EBREAKDOWN;
  const double* coef_v = h->state->coef_v;
  const double* coef_w = h->state->coef_w;
  res->status = BLTT_NOCONV;
  int j = 0;
  for (j = 1; j <= maxit; ++j) {
    if ((rc = matvec<T>(h, MV_DOT, split ? TERM_NONE : TERM_STENCIL, Zc, ws.Q, nullptr, &np))) return rc;
    if ((rc = scalar(h, SC_DELTA, np, nullptr, split))) return rc;
    if ((rc = precond<T>(h, ws.Q, Vc, j > 1 ? Vp : nullptr, Vn, coef_v, ws.Q, Vn, Zn, &np, split ? Zc : nullptr, split)))
      return rc;
    if ((rc = scalar(h, SC_BETA, np, h->hist_dev))) return rc;
    {
      ProfScope ps(h, BLTT_K_WX, (4.0 * sizeof(T) + 2.0 * sizeof(TX)) * h->n);
      HIPCHK(launch_wx<T, TX>(Zc, Wa, Wb, X, h->n, coef_w, s));
    }
    {
      T* t = Vp;
      Vp = Vc;
      Vc = Vn;
      Vn = t;
      std::swap(Zc, Zn);
      std::swap(Wa, Wb);
    }
    if ((rc = read_state(h))) return rc;
    const SolverState& st = *h->state_host;
    if (st.status == -3) return BLTT_ENAN;
    if (st.status == -4) return BLTT_EBREAKDOWN;
    const double eta_rel = std::fabs(st.eta) / st.eta0;
    if (eta_rel <= eta_tol || st.status == 1) {
      if (f_dev) {
        if constexpr (sizeof(TX) == 8 && sizeof(T) == 8) {
          if ((rc = matvec<double>(h, MV_RESID, TERM_STENCIL, (const double*)X, (double*)ws.Q, f_dev, &np))) return rc;
          if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
          if ((rc = read_state(h))) return rc;
          res->relres = std::sqrt(h->state_host->norm2) / bnorm;
          if (!(res->relres == res->relres)) return BLTT_ENAN;
          if (res->relres <= tol || st.status == 1) {
            res->status = BLTT_OK;
            break;
          }
        }
      } else {
        res->status = BLTT_OK;
        break;
      }
    }
  }
  res->iters = j > maxit ? maxit : j;
  if (hist_host) {
    HIPCHK(hipMemcpyAsync(hist_host, h->hist_dev, sizeof(double) * (size_t)(res->iters + 1), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return BLTT_OK;
}

// MINRES in sine coordinates (every block p_k I + q_k L_h is diagonalised by
// the sine transform, Remark 1): per iteration one time-line matvec with the
// mu_i term, one Lanczos-update + time-pass kernel, one direction/iterate
// update.  The right-hand side is cq * bsrc with cq = bcoef[0] (bsrc may be
// FP64 for an FP32 sweep); it is copied into V[0] as the first Lanczos vector
// unless bsrc already is V[0]; brev: the right-hand side is Y bsrc (bsrc read
// with its time lines reversed).  X must be zero on entry.  fhat (FP64 only):
// the transformed f for the explicit residual check, as in minres_core.
//
// zbasis (FP32 only): keep every Z_j in the stored pool instead of forming the
// directions W and the iterate X; the sweep's iterate is sum_i y[i] Z_i with the
// coefficients the scalar kernel carries (the caller adds it with
// launch_combine over res->iters vectors).  A sweep then ends after at most
// K - 1 iterations (the pool size); in the refinement loop that is a restart.
template <typename T, typename TX, typename TB>
int minres_spec(bltt_handle* h, TX* X, int maxit, double eta_tol, const double* fhat, double tol, double bnorm,
                double* hist_host, CoreResult* res, const TB* bsrc, const double* bcoef, bool zbasis = false,
                bool brev = false) {
  Workspace<T>& ws = workspace<T>(h);
  hipStream_t s = h->stream;
  int rc;
  int64_t np = 0;
  if (zbasis && (sizeof(T) != 4 || h->zb_K < 4)) return BLTT_EINVAL;
  T* Vc = ws.V[0];
  T* Vp = ws.V[1];
  T* Vn = ws.V[2];
  T* Zc = ws.Z[0];
  T* Zn = ws.Z[1];
  T* Wa = ws.W[0];
  T* Wb = ws.W[1];
  const double n = (double)h->n;
  if (zbasis) {
    Zc = reinterpret_cast<T*>(h->zpool[0]);
    Zn = reinterpret_cast<T*>(h->zpool[1]);
    maxit = std::min(maxit, h->zb_K - 1);
  } else {
    ProfScope ps(h, BLTT_K_OTHER, 2.0 * n * sizeof(T));
    HIPCHK(launch_fill<T>(Wa, h->n, T(0), s));
    HIPCHK(launch_fill<T>(Wb, h->n, T(0), s));
  }
  if ((rc = ensure_hist(h, (int64_t)maxit + 2))) return rc;
  const TimeTables<T> tt = time_tables<T>(h, false);
  const int L = (int)h->N;
  int64_t npt = 0;
  // v_1 = b, z_1 = P^{-1} b, beta_1 = sqrt(<b, z_1>)
  {
    const bool copy = (const void*)bsrc != (const void*)Vc;
    ProfScope ps(h, BLTT_K_TIME_START, n * (sizeof(TB) + (copy ? 2.0 : 1.0) * sizeof(T)));
    HIPCHK(launch_time_upd<T, TB>(L, false, h->opt.precond == BLTT_PRECOND_ABAC, bsrc, nullptr, nullptr,
                                  copy ? Vc : nullptr, Zc, h->M, tt, bcoef, h->partials, time_blocks<T>(h), &npt, s,
                                  brev, time_plan<T>(h)));
  }
  if ((rc = scalar(h, SC_START, npt, h->hist_dev, false, zbasis))) return rc;
  if ((rc = read_state(h))) return rc;
  if (h->state_host->status == -3) return BLTT_ENAN;
  if (h->state_host->status == -4) return BLTT_EBREAKDOWN;
  const double* coef_v = h->state->coef_v;
  const double* coef_w = h->state->coef_w;
  res->status = BLTT_NOCONV;
  // graph replay unless profiling (which times every kernel) or asked not to
  IterGraphs* g = nullptr;
  if (!h->prof && !h->opt.eager) {
    g = &h->graphs[zbasis ? 2 : (sizeof(T) == 8 ? 0 : 1)];
    if (g->X != (const void*)X || g->hist != h->hist_dev) {
      g->reset();
      g->X = X;
      g->hist = h->hist_dev;
    }
  }
  int j = 0;
  for (j = 1; j <= maxit; ++j) {
    auto step = [&]() -> int {
      const hipStream_t cs = h->stream;
      int src;
      if ((src = matvec<T>(h, MV_DOT, TERM_SPEC, Zc, ws.Q, nullptr, &np))) return src;
      if ((src = scalar(h, SC_DELTA, np, nullptr))) return src;
      {
        // at j = 1 there is no v_0: V2 = V1 with a zero coefficient
        ProfScope ps(h, BLTT_K_TIME, (j > 1 ? 5.0 : 4.0) * n * sizeof(T));
        HIPCHK(launch_time_upd<T, T>(L, true, h->opt.precond == BLTT_PRECOND_ABAC, ws.Q, Vc, j > 1 ? Vp : Vc, Vn,
                                     Zn, h->M, tt, coef_v, h->partials, time_blocks<T>(h), &npt, cs, false,
                                     time_plan<T>(h)));
      }
      if ((src = scalar(h, SC_BETA, npt, h->hist_dev, false, zbasis))) return src;
      if (!zbasis) {
        ProfScope ps(h, BLTT_K_WX, (4.0 * sizeof(T) + 2.0 * sizeof(TX)) * n);
        HIPCHK(launch_wx<T, TX>(Zc, Wa, Wb, X, h->n, coef_w, cs));
      }
      return BLTT_OK;
    };
    if (g) {
      // FP64/FP32 direction form: j = 1, then the period-6 rotation (V by 3,
      // Z and W by 2); stored basis: one position per pool vector
      const int key = zbasis ? j : (j == 1 ? 0 : 1 + (j - 2) % 6);
      if (!g->exec[key]) {
        if ((rc = capture_and_launch(h, step, &g->exec[key], &g->pubs[key]))) return rc;
      } else {
        h->seq_host += g->pubs[key];
        HIPCHK(hipGraphLaunch(g->exec[key], s));
      }
    } else if ((rc = step())) {
      return rc;
    }
    {
      T* t = Vp;
      Vp = Vc;
      Vc = Vn;
      Vn = t;
      if (zbasis) {
        Zc = Zn;
        Zn = j + 1 < h->zb_K ? reinterpret_cast<T*>(h->zpool[j + 1]) : nullptr;
      } else {
        std::swap(Zc, Zn);
        std::swap(Wa, Wb);
      }
    }
    if ((rc = read_state(h))) return rc;
    const SolverState& st = *h->state_host;
    if (st.status == -3) return BLTT_ENAN;
    if (st.status == -4) return BLTT_EBREAKDOWN;
    const double eta_rel = std::fabs(st.eta) / st.eta0;
    if (eta_rel <= eta_tol || st.status == 1) {
      if (fhat) {
        if constexpr (sizeof(TX) == 8 && sizeof(T) == 8) {
          if ((rc = matvec<double>(h, MV_RESID, TERM_SPEC, (const double*)X, (double*)ws.Q, fhat, &np))) return rc;
          if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
          if ((rc = read_state(h))) return rc;
          res->relres = std::sqrt(h->state_host->norm2) / bnorm;
          if (!(res->relres == res->relres)) return BLTT_ENAN;
          if (res->relres <= tol || st.status == 1) {
            res->status = BLTT_OK;
            break;
          }
        }
      } else {
        res->status = BLTT_OK;
        break;
      }
    }
  }
  res->iters = j > maxit ? maxit : j;
  if (hist_host) {
    HIPCHK(hipMemcpyAsync(hist_host, h->hist_dev, sizeof(double) * (size_t)(res->iters + 1), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return BLTT_OK;
}

// [a, a + na) and [b, b + nb) share a byte
bool overlaps(const void* a, int64_t na, const void* b, int64_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}
bool overlaps(const void* a, const void* b, int64_t bytes) { return overlaps(a, bytes, b, bytes); }

int check_power(int64_t v, int64_t lo, int64_t hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// Stopping tolerance of one FP32 sweep on |eta|/eta_0: the inner tolerance,
// loosened to a tenth of what the outer tolerance still asks for
// (0.1 tol / relres, relres the current relative residual), so the last sweep
// does not solve far past the target while the solution error, which the
// conditioning makes a multiple of the residual, keeps a decade of margin.
// The explicit FP64 residual that follows decides convergence either way.
constexpr double SWEEP_MARGIN = 0.1;
double sweep_tol(const bltt_handle* h, double tol, double relres) {
  return relres > 0.0 ? std::max(h->opt.inner_tol, SWEEP_MARGIN * tol / relres) : h->opt.inner_tol;
}

// strided sine transforms along dimensions 1..dim-1 on a mode-major vector
// (element (i, n) at i*N + n: the lines of dimension d have stride N * m_0 * ... * m_{d-1})
int space_strided_mm(bltt_handle* h, double* x, bool reverse) {
  for (int k = 1; k < h->dim; ++k) {
    const int d = reverse ? h->dim - k : k;
    int64_t S = h->N;
    for (int e = 0; e < d; ++e) S *= h->m[e];
    const int64_t nlines = h->n / h->m[d];
    ProfScope ps(h, BLTT_K_DST_STRIDED, 16.0 * h->n);
    HIPCHK(launch_dst_strided<double>(2 * (h->m[d] + 1), x, nlines, S, dst_tables<double>(h, d), h->stream));
  }
  return BLTT_OK;
}

// fhat = (I x U) f: f time-major (caller's), fhat mode-major; partial sums of
// ||f||^2 = ||fhat||^2 left in h->partials (count in *np)
int sine_forward(bltt_handle* h, const double* f, double* fhat, int64_t* np) {
  {
    ProfScope ps(h, BLTT_K_DST_X_VUPD, 16.0 * h->n);
    HIPCHK(launch_dst_xt<double>(2 * (h->m[0] + 1), 0, f, fhat, h->N, h->M, dst_tables<double>(h, 0), h->partials,
                                 np, h->stream));
  }
  return space_strided_mm(h, fhat, false);
}

// u = (I x U) uhat: uhat mode-major (overwritten), u time-major
int sine_backward(bltt_handle* h, double* uhat, double* u) {
  int rc;
  if ((rc = space_strided_mm(h, uhat, true))) return rc;
  ProfScope ps(h, BLTT_K_DST_X_VUPD, 16.0 * h->n);
  HIPCHK(launch_dst_xt<double>(2 * (h->m[0] + 1), 1, uhat, u, h->N, h->M, dst_tables<double>(h, 0), nullptr,
                               nullptr, h->stream));
  return BLTT_OK;
}

// Kernel plans of the FP32 sine-basis iteration.  Forced by opt.fft_plan, read
// from the plan cache, or timed here on the handle's own buffers (filled with a
// constant first; the values computed are discarded): the time pass in every
// radix plan (where fft_plan_alt(N)) and with 2, 4 or 8 workgroups per compute
// unit, the N-point matvec in every radix plan.  Each variant runs once to
// warm up (its first launch loads its code) and three times timed; the
// variant with the smallest of its timed runs wins.
int tune_fp32_plans(bltt_handle* h, int cus) {
  const int L = (int)h->N;
  const bool alt = fft_plan_alt(L);
  if (h->opt.fft_plan != BLTT_PLAN_AUTO) {
    h->plan_time = h->plan_cs = (h->opt.fft_plan == BLTT_PLAN_ALT && alt) ? 1 : 0;
    h->plan_source = BLTT_PLAN_SOURCE_FORCED;
    return BLTT_OK;
  }
  const std::string key = "bltt/1 " + plans::device_tag() + " fp32-sine N=" + std::to_string(h->N) +
                          " M=" + std::to_string(h->M) + " shortp=" + std::to_string(short_p(h) ? 1 : 0);
  std::string val;
  if (plans::lookup(h->plan_cache, key, &val)) {
    auto f = plans::fields(val);
    const int pt = (int)f["time_plan"], pc = (int)f["cs_plan"];
    const long bpc = f["blocks_per_cu"], cpc = f["cs_blocks_per_cu"];  // absent: 0, one tile per workgroup
    if ((pt == 0 || (pt == 1 && alt)) && (pc == 0 || (pc == 1 && alt)) && bpc >= 1 && bpc <= 64 && cpc >= 0 &&
        cpc <= 64) {
      h->plan_time = pt;
      h->plan_cs = pc;
      h->time_blocks = bpc * (int64_t)cus;
      h->cs_blocks = cpc * (int64_t)cus;
      h->plan_source = BLTT_PLAN_SOURCE_CACHE;
      return BLTT_OK;
    }
  }
  Workspace<float>& w = h->w32;
  hipStream_t s = h->stream;
  const int64_t n = h->n;
  HIPCHK(launch_fill<float>(w.Q, n, 0.5f, s));
  for (int i = 0; i < 3; ++i) HIPCHK(launch_fill<float>(w.V[i], n, 0.25f, s));
  HIPCHK(launch_fill<float>(w.Z[0], n, 0.5f, s));
  hipEvent_t a = nullptr, z = nullptr;
  HIPCHK(hipEventCreate(&a));
  if (hipEventCreate(&z) != hipSuccess) {
    (void)hipEventDestroy(a);
    return BLTT_EHIP;
  }
  int rc = BLTT_OK;
  // Every candidate launch is timed once per round, the candidates in turn,
  // over 8 rounds (the first a warm-up); each keeps its best time.  Taking the
  // candidates in turn rather than one after another keeps clock and thermal
  // drift during the tuning from favouring whichever ran last.
  struct Cand {
    std::function<hipError_t()> launch;
    int plan;
    int64_t blocks;
    float best;
  };
  auto tournament = [&](std::vector<Cand>& cands) -> int {
    for (int rep = 0; rep < 8; ++rep) {
      for (Cand& c : cands) {
        if (hipEventRecord(a, s) != hipSuccess || c.launch() != hipSuccess || hipEventRecord(z, s) != hipSuccess ||
            hipEventSynchronize(z) != hipSuccess)
          return BLTT_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, a, z) != hipSuccess) return BLTT_EHIP;
        if (rep > 0 && ms < c.best) c.best = ms;
      }
    }
    return BLTT_OK;
  };
  const TimeTables<float> tt = time_tables<float>(h, false);
  const int64_t tiles = fft_tiles<float, FK_SPEC>(L, h->M);
  int bt_plan = 0;
  int64_t bt_blocks = h->max_blocks;
  {
    std::vector<Cand> cands;
    for (int plan = 0; plan <= (alt ? 1 : 0); ++plan)
      for (int per : {2, 4, 8}) {
        const int64_t blocks = per * (int64_t)cus;
        if (per > 2 && (per / 2) * (int64_t)cus >= tiles) continue;  // same launch as the smaller count
        cands.push_back({[&, plan, blocks]() {
                           int64_t np = 0;
                           return launch_time_upd<float, float>(L, true, true, w.Q, w.V[0], w.V[1], w.V[2], w.Z[0],
                                                                h->M, tt, h->coef_one, h->partials, blocks, &np, s,
                                                                false, plan);
                         },
                         plan, blocks, 1e30f});
      }
    rc = tournament(cands);
    float best = 1e30f;
    for (const Cand& c : cands)
      if (c.best < best) {
        best = c.best;
        bt_plan = c.plan;
        bt_blocks = c.blocks;
      }
  }
  // the N-point matvec: radix plan, and one tile per workgroup (blocks 0) or
  // 2, 4, 8 persistent workgroups per CU
  int bc_plan = 0;
  int64_t bc_blocks = 0;
  if (rc == BLTT_OK && !short_p(h)) {
    std::vector<Cand> cands;
    for (int plan = 0; plan <= (alt ? 1 : 0); ++plan)
      for (int per : {0, 2, 4, 8}) {
        const int64_t blocks = per * (int64_t)cus;
        if (per > 0 && blocks >= tiles) continue;  // the same launch as one tile per workgroup
        cands.push_back({[&, plan, blocks]() {
                           int64_t np = 0;
                           return launch_matvec_cs<float>(L, MV_DOT, w.Z[0], w.Q, nullptr, h->M, cs_tables<float>(h),
                                                          IterUpd{}, h->partials, blocks, &np, s, plan);
                         },
                         plan, blocks, 1e30f});
      }
    rc = tournament(cands);
    float best = 1e30f;
    for (const Cand& c : cands)
      if (c.best < best) {
        best = c.best;
        bc_plan = c.plan;
        bc_blocks = c.blocks;
      }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  if (rc) return rc;
  h->plan_time = bt_plan;
  h->plan_cs = bc_plan;
  h->time_blocks = bt_blocks;
  h->cs_blocks = bc_blocks;
  h->plan_source = BLTT_PLAN_SOURCE_TIMED;
  plans::store(h->plan_cache, key,
               "time_plan=" + std::to_string(bt_plan) + " cs_plan=" + std::to_string(bc_plan) +
                   " blocks_per_cu=" + std::to_string(bt_blocks / cus) +
                   " cs_blocks_per_cu=" + std::to_string(bc_blocks / cus));
  return BLTT_OK;
}

}  // namespace

extern "C" {

const char* bltt_version(void) { return "bltt-mi355x 0.2"; }

int bltt_plan_info(const bltt_handle* h, int32_t* time_plan, int32_t* cs_plan, int64_t* time_blocks,
                   int64_t* cs_blocks, int32_t* source) {
  if (!h) return BLTT_EINVAL;
  if (time_plan) *time_plan = h->plan_time;
  if (cs_plan) *cs_plan = h->plan_cs;
  if (time_blocks) *time_blocks = h->time_blocks > 0 ? h->time_blocks : h->max_blocks;
  if (cs_blocks) *cs_blocks = h->cs_blocks;
  if (source) *source = h->plan_source;
  return BLTT_OK;
}

const char* bltt_strerror(int code) {
  switch (code) {
    case BLTT_OK: return "ok";
    case BLTT_NOCONV: return "iteration limit reached before the tolerance";
    case BLTT_EINVAL: return "invalid argument";
    case BLTT_EASSUMPTION: return "blocks violate Assumption 1(ii): preconditioner may be singular";
    case BLTT_ENAN: return "non-finite value in input or iteration";
    case BLTT_EBREAKDOWN: return "preconditioner not positive definite in floating point";
    case BLTT_ENOMEM: return "device allocation failed";
    case BLTT_EHIP: return "HIP runtime error";
    case BLTT_EUNSUPPORTED: return "size or block structure not supported";
  }
  return "unknown status";
}

void bltt_destroy(void* handle) {
  if (!handle) return;
  const uint32_t magic = *static_cast<const uint32_t*>(handle);
  if (magic == BATCH_MAGIC) {
    bltt_destroy_batched(static_cast<bltt_batch*>(handle));
    return;
  }
  if (magic != HANDLE_MAGIC) return;
  bltt_handle* h = static_cast<bltt_handle*>(handle);
  h->magic = 0;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (void* p : h->allocs) (void)hipFree(p);
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  if (h->state_host) (void)hipHostFree(h->state_host);
  if (h->mirror) (void)hipHostFree((void*)h->mirror);
  for (IterGraphs& g : h->graphs) g.reset();
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
}

}  // extern "C"

namespace {

int setup_impl(const bltt_blocks* blk, const double* const* face, double abar, int64_t N, int64_t M, double alpha,
               const bltt_options* opt, void* stream, bltt_handle** out) {
  const double t0 = now_ms();
  if (!blk || !out || !blk->p || !blk->q) return BLTT_EINVAL;
  if (blk->dim < 1 || blk->dim > 3 || N < 1 || M < 1) return BLTT_EINVAL;
  if (!(alpha > 0.0 && alpha <= 1.0)) return BLTT_EINVAL;
  int64_t Mp = 1;
  for (int d = 0; d < blk->dim; ++d) {
    if (blk->m[d] < 1 || !(blk->h[d] > 0.0) || !std::isfinite(blk->h[d])) return BLTT_EINVAL;
    Mp *= blk->m[d];
  }
  if (Mp != M) return BLTT_EINVAL;
  for (int64_t k = 0; k < N; ++k)
    if (!std::isfinite(blk->p[k]) || !std::isfinite(blk->q[k])) return BLTT_EINVAL;
  if (opt) {
    if (opt->precision != BLTT_FP64 && opt->precision != BLTT_MIXED) return BLTT_EINVAL;
    if (opt->basis != BLTT_BASIS_SINE && opt->basis != BLTT_BASIS_PHYSICAL) return BLTT_EINVAL;
    if (opt->precond != BLTT_PRECOND_ABAC && opt->precond != BLTT_PRECOND_NONE) return BLTT_EINVAL;
    if (opt->initial_guess != 0 && opt->initial_guess != 1) return BLTT_EINVAL;
    if (opt->fft_plan < BLTT_PLAN_AUTO || opt->fft_plan > BLTT_PLAN_ALT) return BLTT_EINVAL;
    if (opt->eager != 0 && opt->eager != 1) return BLTT_EINVAL;
    // the unpreconditioned comparator runs the FP64 sine-basis path
    if (opt->precond == BLTT_PRECOND_NONE && (opt->precision != BLTT_FP64 || opt->basis != BLTT_BASIS_SINE))
      return BLTT_EUNSUPPORTED;
  }
  // N = 1 (one block, Section 3): P_alpha = |A_(0)| = A_(0), solved per sine
  // mode; the variable-coefficient and unpreconditioned variants need N >= 2
  if (N == 1) {
    if (face || (opt && opt->precond == BLTT_PRECOND_NONE)) return BLTT_EUNSUPPORTED;
  } else if (!check_power(N, 2, 2048)) {
    return BLTT_EUNSUPPORTED;
  }
  for (int d = 0; d < blk->dim; ++d)
    if (!check_power(2 * ((int64_t)blk->m[d] + 1), 4, 2048)) return BLTT_EUNSUPPORTED;
  int qtaps = 0, ptaps = 0;
  for (int64_t k = 0; k < N; ++k) {
    if (blk->q[k] != 0.0) qtaps = (int)k + 1;
    if (blk->p[k] != 0.0) ptaps = (int)k + 1;
  }
  if (qtaps > 4) return BLTT_EUNSUPPORTED;
  if (ptaps == 0 && qtaps == 0) return BLTT_EASSUMPTION;
  std::vector<double> face_host[3];
  if (face) {
    // a > 0 at every face, abar > 0; the operator is not sine-diagonal, so the
    // physical basis runs, with the preconditioner of the mean-coefficient system
    if (!(abar > 0.0) || !std::isfinite(abar)) return BLTT_EINVAL;
    if (opt && opt->precond == BLTT_PRECOND_NONE) return BLTT_EUNSUPPORTED;
    for (int d = 0; d < blk->dim; ++d) {
      if (!face[d]) return BLTT_EINVAL;
      int64_t cnt = 1;
      for (int e = 0; e < blk->dim; ++e) cnt *= blk->m[e] + (e == d ? 1 : 0);
      face_host[d].assign(face[d], face[d] + cnt);
      for (double v : face_host[d])
        if (!(v > 0.0) || !std::isfinite(v)) return BLTT_EINVAL;
    }
  }

  bltt_handle* h = new (std::nothrow) bltt_handle();
  if (!h) return BLTT_ENOMEM;
  h->stream = (hipStream_t)stream;
  h->dim = blk->dim;
  for (int d = 0; d < 3; ++d) {
    h->m[d] = d < blk->dim ? blk->m[d] : 1;
    h->h[d] = d < blk->dim ? blk->h[d] : 1.0;
  }
  h->N = N;
  h->M = M;
  h->n = N * M;
  h->alpha = alpha;
  h->p.assign(blk->p, blk->p + N);
  h->q.assign(blk->q, blk->q + N);
  h->ptaps = ptaps;
  h->qtaps = qtaps;
  h->opt.precision = BLTT_FP64;
  h->opt.inner_tol = 1e-4;
  h->opt.max_refine = 20;
  h->opt.check_factor = 10.0;
  h->opt.basis = BLTT_BASIS_SINE;
  h->opt.precond = BLTT_PRECOND_ABAC;
  if (opt) {
    h->opt.precision = opt->precision;
    h->opt.basis = opt->basis;
    h->opt.precond = opt->precond;
    if (opt->inner_tol > 0.0) h->opt.inner_tol = opt->inner_tol;
    if (opt->max_refine > 0) h->opt.max_refine = opt->max_refine;
    if (opt->check_factor >= 1.0) h->opt.check_factor = opt->check_factor;
    h->opt.initial_guess = opt->initial_guess;
    h->opt.fft_plan = opt->fft_plan;
    h->opt.eager = opt->eager;
    if (opt->plan_cache) h->plan_cache = opt->plan_cache;
  }
  h->opt.plan_cache = nullptr;  // the handle keeps its own copy of the path
  if (N == 1) h->opt.basis = BLTT_BASIS_SINE;  // the single-step solve runs in sine coordinates
  if (face) {
    h->var = true;
    h->abar = abar;
    h->opt.basis = BLTT_BASIS_PHYSICAL;
  }
  // Assumption 1(ii) (Proposition 1), for the system the preconditioner is built from
  double mu_min = 0.0, mu_max = 0.0;
  for (int d = 0; d < h->dim; ++d) {
    const std::vector<double> e = host::lap_eigs_1d(h->m[d], h->h[d]);
    mu_min += h->abar * e.front();
    mu_max += h->abar * e.back();
  }
  h->c0 = host::assumption_margin(h->p, h->q, mu_min, mu_max);
  if (!(h->c0 > 0.0)) {
    delete h;
    return BLTT_EASSUMPTION;
  }

  g_config_err = configure_kernels_once();
  {
    // persistent kernels: two workgroups per compute unit resident, two rounds
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
      delete h;
      return BLTT_EHIP;
    }
    h->max_blocks = 4 * (int64_t)cus;
    h->device = dev;
    if (scratch_init(dev) != BLTT_OK) {
      delete h;
      return BLTT_EHIP;
    }
  }
  if (g_config_err != hipSuccess) {
    delete h;
    return BLTT_EHIP;
  }

  int rc = BLTT_OK;
  auto fail = [&](int code) {
    bltt_destroy(h);
    return code;
  };
  h->partials_cap = std::max(partials_needed<float>(h), partials_needed<double>(h));
  if ((rc = dalloc(h, &h->partials, (size_t)h->partials_cap))) return fail(rc);
  h->red_half = h->partials_cap / RED_CHUNK + 2;
  if ((rc = dalloc(h, &h->red_scratch, (size_t)(2 * h->red_half)))) return fail(rc);
  if ((rc = dalloc(h, &h->partials_aux,
                   (size_t)std::max(fft_blocks<float, FK_TIME>((int)h->N, h->M),
                                    fft_blocks<double, FK_TIME>((int)h->N, h->M)))))
    return fail(rc);
  if ((rc = dalloc(h, &h->state, 1))) return fail(rc);
  if (hipHostMalloc((void**)&h->state_host, sizeof(SolverState), hipHostMallocDefault) != hipSuccess)
    return fail(BLTT_ENOMEM);
  std::memset(h->state_host, 0, sizeof(SolverState));
  if (hipMemcpy(h->state, h->state_host, sizeof(SolverState), hipMemcpyHostToDevice) != hipSuccess)
    return fail(BLTT_EHIP);
  if (hipHostMalloc((void**)&h->mirror, sizeof(SolverState), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess)
    return fail(BLTT_ENOMEM);
  std::memset((void*)h->mirror, 0, sizeof(SolverState));
  if (hipHostGetDevicePointer((void**)&h->mirror_dev, (void*)h->mirror, 0) != hipSuccess) return fail(BLTT_EHIP);
  {
    std::vector<double> one = {1.0, 0.0, 0.0, 0.0};
    if ((rc = upload<double>(h, &h->coef_one, one))) return fail(rc);
    if ((rc = dalloc(h, &h->step_dev, (size_t)STEP_LEN))) return fail(rc);
    if ((rc = dalloc(h, &h->rsc_dev, 1))) return fail(rc);
  }
  for (int d = 0; d < h->dim; ++d)
    if (h->var && (rc = upload<double>(h, &h->face_dev[d], face_host[d]))) return fail(rc);
  if ((rc = build_tables<double>(h))) return fail(rc);
  const bool sine = h->opt.basis == BLTT_BASIS_SINE;
  if (h->opt.precision == BLTT_MIXED) {
    if ((rc = build_tables<float>(h))) return fail(rc);
    if ((rc = build_workspace<float>(h, !sine))) return fail(rc);
    if ((rc = dalloc(h, &h->R64, (size_t)h->n))) return fail(rc);
  } else {
    if ((rc = build_workspace<double>(h, true))) return fail(rc);
  }
  if (sine) {
    if ((rc = dalloc(h, &h->F64, (size_t)h->n))) return fail(rc);
    if (h->opt.precision == BLTT_MIXED)
      if ((rc = build_zpool(h))) return fail(rc);
  }
  if (sine && h->opt.precision == BLTT_MIXED && h->opt.precond == BLTT_PRECOND_ABAC && !h->var && N > 1)
    if ((rc = tune_fp32_plans(h, (int)(h->max_blocks / 4)))) return fail(rc);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(BLTT_EHIP);
  h->setup_ms = now_ms() - t0;
  *out = h;
  return BLTT_OK;
}

}  // namespace

extern "C" {

int bltt_setup(const bltt_blocks* blk, int64_t N, int64_t M, double alpha, const bltt_options* opt, void* stream,
               bltt_handle** out) {
  return setup_impl(blk, nullptr, 1.0, N, M, alpha, opt, stream, out);
}

int bltt_setup_varcoef(const bltt_blocks* blk, const double* const* face, double abar, int64_t N, int64_t M,
                       double alpha, const bltt_options* opt, void* stream, bltt_handle** out) {
  if (!face) return BLTT_EINVAL;
  return setup_impl(blk, face, abar, N, M, alpha, opt, stream, out);
}

int bltt_pminres(bltt_handle* h, const double* f_dev, double tol, int32_t maxit, double* u_dev, int32_t* iters,
                 double* hist, bltt_info* info) {
  const double t0 = now_ms();
  if (!h || !f_dev || !u_dev || !(tol > 0.0) || maxit < 1) return BLTT_EINVAL;
  if (overlaps(f_dev, u_dev, h->n * (int64_t)sizeof(double))) return BLTT_EINVAL;
  hipStream_t s = h->stream;
  int rc;
  int64_t np = 0;
  const bool guess = h->opt.initial_guess != 0;
  if (h->opt.basis != BLTT_BASIS_SINE && !guess) {
    ProfScope ps(h, BLTT_K_OTHER, 8.0 * h->n);
    HIPCHK(launch_fill<double>(u_dev, h->n, 0.0, s));
  }
  int total_iters = 0, outer = 0;
  double relres = 0.0;
  int status = BLTT_OK;

  if (h->opt.basis == BLTT_BASIS_SINE) {
    // fhat = (I x U) f once, stored mode-major (each mode's time line
    // contiguous) in u_dev; the iteration and the FP64 residuals run on the
    // mode-decoupled system in that layout, with uhat in F64; u = (I x U) uhat
    // once at the end (U = U^T = U^{-1}), over fhat.  ||fhat||^2 = ||Y fhat||^2
    // comes from the first pass; b = Y fhat is never stored: the first Lanczos
    // start reads fhat reversed.
    double* fhat = u_dev;
    double* uhat = h->F64;
    // an initial guess u0 enters as uhat = (I x U) u0, before fhat takes its buffer
    if (guess && (rc = sine_forward(h, u_dev, uhat, &np))) return rc;
    if ((rc = sine_forward(h, f_dev, fhat, &np))) return rc;
    if (!guess && (h->opt.precision == BLTT_FP64 || short_p(h))) {
      // the FP64 path and the direct-form residual read uhat from the start;
      // the fused FFT residual of the mixed path writes it on the first sweep
      ProfScope ps(h, BLTT_K_OTHER, 8.0 * h->n);
      HIPCHK(launch_fill<double>(uhat, h->n, 0.0, s));
    }
    if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
    if ((rc = read_state(h))) return rc;
    const double bn2 = h->state_host->norm2;
    if (!std::isfinite(bn2)) return BLTT_ENAN;
    const double bnorm = std::sqrt(bn2);
    if (hist) hist[0] = 1.0;
    if (bn2 == 0.0) {
      relres = 0.0;
      HIPCHK(launch_fill<double>(uhat, h->n, 0.0, s));
    } else if (h->N == 1) {
      // One block: P_alpha = |A_(0)| = A_(0) (the alpha-circulant of a single
      // block has no wrap, and A_(0) is SPD), so P^{-1} Y A = I and MINRES
      // reaches u = A_(0)^{-1} f in its first iteration, whatever the
      // precision; that iterate is formed directly, mode by mode, in FP64.
      const double* mu = tables<double>(h).mu;
      double r0 = 1.0;
      if (guess) {
        HIPCHK(launch_single_step(fhat, uhat, h->M, mu, h->p[0], h->q[0], 0, h->partials, &np, s));
        if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
        if ((rc = read_state(h))) return rc;
        r0 = std::sqrt(h->state_host->norm2) / bnorm;
        if (!std::isfinite(r0)) return BLTT_ENAN;
      }
      if (guess && r0 <= tol) {
        relres = r0;
      } else {
        HIPCHK(launch_single_step(fhat, uhat, h->M, mu, h->p[0], h->q[0], 1, h->partials, &np, s));
        if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
        if ((rc = read_state(h))) return rc;
        relres = std::sqrt(h->state_host->norm2) / bnorm;
        if (!std::isfinite(relres)) return BLTT_ENAN;
        total_iters = 1;
        if (hist) hist[1] = relres;
      }
      outer = 1;
      status = relres <= tol ? BLTT_OK : BLTT_NOCONV;
    } else if (h->opt.precision == BLTT_FP64) {
      CoreResult cr;
      double r0 = 1.0;
      if (guess) {
        // MINRES from uhat: the Lanczos process starts from r0 = Y(fhat - T uhat)
        if ((rc = matvec<double>(h, MV_RESID, TERM_SPEC, uhat, h->w64.V[0], fhat, &np))) return rc;
        if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
        if ((rc = read_state(h))) return rc;
        r0 = std::sqrt(h->state_host->norm2) / bnorm;
        if (!std::isfinite(r0)) return BLTT_ENAN;
      }
      if (guess && r0 <= tol) {
        cr.iters = 0;
        cr.status = BLTT_OK;
        cr.relres = r0;
      } else if (guess) {
        rc = minres_spec<double, double, double>(h, uhat, maxit, h->opt.check_factor * tol / r0, fhat, tol, bnorm,
                                                 hist, &cr, h->w64.V[0], h->coef_one, false, false);
        if (rc) return rc;
      } else {
        rc = minres_spec<double, double, double>(h, uhat, maxit, h->opt.check_factor * tol, fhat, tol, bnorm, hist,
                                                 &cr, fhat, h->coef_one, false, true);
        if (rc) return rc;
      }
      total_iters = cr.iters;
      outer = 1;
      status = cr.status;
      relres = cr.relres;
      if (relres < 0.0) {
        if ((rc = matvec<double>(h, MV_RESID, TERM_SPEC, uhat, h->w64.Q, fhat, &np))) return rc;
        if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
        if ((rc = read_state(h))) return rc;
        relres = std::sqrt(h->state_host->norm2) / bnorm;
      }
    } else {
      // FP64 refinement around FP32 MINRES sweeps on r / ||r|| (state->rinv).
      // With dense p the residual pass hands the next sweep its right-hand
      // side as FP32, r / ||fhat|| (read once; its norm is summed in FP64 before
      // the rounding, and the rounding, 6e-8 relative, is far inside the
      // sweep's own tolerance); that sweep then runs on it unscaled and its
      // update is multiplied by ||fhat|| (rsc_dev).
      double rnorm = bnorm;
      status = BLTT_NOCONV;
      int hist_pos = 0;
      std::vector<double> hbuf;
      bool r32 = false;  // the current residual is in w32.V[0] as FP32, times 1/||fhat||
      HIPCHK(hipMemcpyAsync(h->rsc_dev, &bnorm, sizeof(double), hipMemcpyHostToDevice, s));
      if (guess) {
        // refinement from uhat: the first sweep solves for the residual of the guess
        if ((rc = matvec<double>(h, MV_RESID, TERM_SPEC, uhat, h->R64, fhat, &np))) return rc;
        if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
        if ((rc = read_state(h))) return rc;
        rnorm = std::sqrt(h->state_host->norm2);
        if (!std::isfinite(rnorm)) return BLTT_ENAN;
      }
      while (true) {
        relres = rnorm / bnorm;
        if (relres <= tol) {
          status = BLTT_OK;
          break;
        }
        if (outer >= h->opt.max_refine || total_iters >= maxit) break;
        CoreResult cr;
        const int left = maxit - total_iters;
        hbuf.assign((size_t)left + 2, 0.0);
        // r = b = Y fhat on the first sweep (read from fhat reversed), then the residual
        const bool from_b = outer == 0 && !guess;
        const bool rhs32 = r32;  // this sweep's right-hand side is r / ||fhat|| in FP32
        if (rhs32)
          rc = minres_spec<float, float, float>(h, nullptr, left, sweep_tol(h, tol, relres), nullptr, 0.0, 1.0,
                                                hbuf.data(), &cr, h->w32.V[0], h->coef_one, true, false);
        else
          rc = minres_spec<float, float, double>(h, nullptr, left, sweep_tol(h, tol, relres), nullptr, 0.0, 1.0,
                                                 hbuf.data(), &cr, from_b ? fhat : h->R64, &h->state->rinv, true,
                                                 from_b);
        if (rc) return rc;
        if (hist)
          for (int k = 1; k <= cr.iters; ++k) hist[hist_pos + k] = hbuf[(size_t)k];
        hist_pos += cr.iters;
        total_iters += cr.iters;
        outer += 1;
        // uhat += ||r|| sum_i y_i Z_i, then r = Y(fhat - A uhat) in FP64 (one
        // pass for dense p; the first sweep's uhat starts at zero and is not read)
        const double* ycoef = h->zb_dev + 2 * h->zb_K;
        if (short_p(h)) {
          ZList<float> zl;
          for (int i = 0; i < ZB_MAX; ++i) zl.z[i] = i < cr.iters ? h->zpool[i] : nullptr;
          zl.k = cr.iters;
          {
            ProfScope ps(h, BLTT_K_WX, (16.0 + 4.0 * cr.iters) * h->n);
            HIPCHK(launch_combine<float>(uhat, zl, ycoef, &h->state->rscale, h->n, s));
          }
          if ((rc = matvec<double>(h, MV_RESID, TERM_SPEC, uhat, h->R64, fhat, &np))) return rc;
        } else {
          IterUpd up{};
          for (int i = 0; i < ZB_MAX; ++i) up.z[i] = i < cr.iters ? h->zpool[i] : nullptr;
          up.k = cr.iters;
          up.y = ycoef;
          up.s = rhs32 ? h->rsc_dev : &h->state->rscale;
          up.u_zero = outer == 1 && !guess ? 1 : 0;
          up.r32 = h->w32.V[0];
          up.r32_scale = 1.0 / bnorm;
          ProfScope ps(h, BLTT_K_RESID64, (28.0 + 4.0 * cr.iters - (up.u_zero ? 8.0 : 0.0)) * h->n);
          HIPCHK(launch_matvec_fft<double>((int)(2 * h->N), MV_RESID, TERM_SPEC, uhat, h->R64, fhat, h->M,
                                           mv_tables<double>(h), up, h->partials, s));
          np = mv_blocks<double>(true, (int)(2 * h->N), h->M);
          r32 = true;
        }
        if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
        if ((rc = read_state(h))) return rc;
        rnorm = std::sqrt(h->state_host->norm2);
        if (!std::isfinite(rnorm)) return BLTT_ENAN;
      }
    }
    if ((rc = sine_backward(h, uhat, u_dev))) return rc;
  } else if (h->opt.precision == BLTT_FP64) {
    Workspace<double>& ws = h->w64;
    // b = Y f into V[0]
    {
      ProfScope ps(h, BLTT_K_OTHER, 16.0 * h->n);
      HIPCHK(launch_rhs<double>(f_dev, ws.V[0], h->N, h->M, 1.0, h->partials, &np, s));
    }
    if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
    if ((rc = read_state(h))) return rc;
    const double bn2 = h->state_host->norm2;
    if (!std::isfinite(bn2)) return BLTT_ENAN;
    if (bn2 == 0.0) {
      if (guess) HIPCHK(launch_fill<double>(u_dev, h->n, 0.0, s));
      if (iters) *iters = 0;
      if (hist) hist[0] = 1.0;
      if (info) {
        info->iters_inner = 0;
        info->iters_outer = 0;
        info->true_relres = 0.0;
        info->setup_ms = h->setup_ms;
        info->solve_ms = now_ms() - t0;
        info->c0 = h->c0;
      }
      HIPCHK(hipStreamSynchronize(s));
      return BLTT_OK;
    }
    const double bnorm = std::sqrt(bn2);
    CoreResult cr;
    double r0 = 1.0;
    if (guess) {
      // MINRES from u_dev: V[0] = r0 = Y(f - A u0)
      if ((rc = matvec<double>(h, MV_RESID, TERM_STENCIL, u_dev, ws.V[0], f_dev, &np))) return rc;
      if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
      if ((rc = read_state(h))) return rc;
      r0 = std::sqrt(h->state_host->norm2) / bnorm;
      if (!std::isfinite(r0)) return BLTT_ENAN;
    }
    if (guess && r0 <= tol) {
      cr.iters = 0;
      cr.status = BLTT_OK;
      cr.relres = r0;
      if (hist) hist[0] = 1.0;
    } else {
      rc = minres_core<double, double>(h, u_dev, maxit, h->opt.check_factor * tol / r0, f_dev, tol, bnorm, hist,
                                       &cr);
      if (rc) return rc;
    }
    total_iters = cr.iters;
    outer = 1;
    status = cr.status;
    relres = cr.relres;
    if (relres < 0.0) {
      if ((rc = matvec<double>(h, MV_RESID, TERM_STENCIL, u_dev, ws.Q, f_dev, &np))) return rc;
      if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
      if ((rc = read_state(h))) return rc;
      relres = std::sqrt(h->state_host->norm2) / bnorm;
    }
  } else {
    // FP64 refinement around FP32 MINRES sweeps
    Workspace<float>& ws = h->w32;
    {
      ProfScope ps(h, BLTT_K_OTHER, 16.0 * h->n);
      HIPCHK(launch_rhs<double>(f_dev, h->R64, h->N, h->M, 1.0, h->partials, &np, s));
    }
    if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
    if ((rc = read_state(h))) return rc;
    const double bn2 = h->state_host->norm2;
    if (!std::isfinite(bn2)) return BLTT_ENAN;
    const double bnorm = std::sqrt(bn2);
    double rnorm = bnorm;
    status = BLTT_NOCONV;
    if (bn2 == 0.0) {
      status = BLTT_OK;
      relres = 0.0;
      HIPCHK(launch_fill<double>(u_dev, h->n, 0.0, s));
    } else if (guess) {
      if ((rc = matvec<double>(h, MV_RESID, TERM_STENCIL, u_dev, h->R64, f_dev, &np))) return rc;
      if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
      if ((rc = read_state(h))) return rc;
      rnorm = std::sqrt(h->state_host->norm2);
      if (!std::isfinite(rnorm)) return BLTT_ENAN;
    }
    if (hist) hist[0] = 1.0;
    int hist_pos = 0;
    std::vector<double> hbuf;
    while (status != BLTT_OK) {
      relres = rnorm / bnorm;
      if (relres <= tol) {
        status = BLTT_OK;
        break;
      }
      if (outer >= h->opt.max_refine || total_iters >= maxit) break;
      // inner right-hand side r / ||r|| in FP32 (state->rscale = ||r||)
      {
        ProfScope ps(h, BLTT_K_OTHER, 16.0 * h->n);
        HIPCHK(launch_scale_cast<double, float>(h->R64, ws.V[0], h->n, &h->state->rscale, 1, s));
        HIPCHK(launch_fill<float>(ws.X, h->n, 0.0f, s));
      }
      CoreResult cr;
      const int left = maxit - total_iters;
      hbuf.assign((size_t)left + 2, 0.0);
      rc = minres_core<float, float>(h, ws.X, left, sweep_tol(h, tol, relres), nullptr, 0.0, 1.0, hbuf.data(), &cr);
      if (rc) return rc;
      if (hist) {
        for (int k = 1; k <= cr.iters; ++k) hist[hist_pos + k] = hbuf[(size_t)k];
      }
      hist_pos += cr.iters;
      total_iters += cr.iters;
      outer += 1;
      // u += ||r|| d, then r = Y(f - A u) in FP64
      {
        ProfScope ps(h, BLTT_K_OTHER, 20.0 * h->n);
        HIPCHK(launch_axpy64<float>(u_dev, ws.X, h->n, &h->state->rscale, s));
      }
      if ((rc = matvec<double>(h, MV_RESID, TERM_STENCIL, u_dev, h->R64, f_dev, &np))) return rc;
      if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
      if ((rc = read_state(h))) return rc;
      rnorm = std::sqrt(h->state_host->norm2);
      if (!std::isfinite(rnorm)) return BLTT_ENAN;
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = total_iters;
  if (info) {
    info->iters_inner = total_iters;
    info->iters_outer = outer;
    info->true_relres = relres;
    info->setup_ms = h->setup_ms;
    info->solve_ms = now_ms() - t0;
    info->c0 = h->c0;
  }
  return status;
}

static int step_prepare(bltt_handle* h, int32_t precision) {
  int rc;
  if (precision == BLTT_FP64) {
    if ((rc = build_tables<double>(h))) return rc;
    return build_workspace<double>(h, false);
  }
  if (precision == BLTT_FP32) {
    if ((rc = build_tables<float>(h))) return rc;
    return build_workspace<float>(h, false);
  }
  return BLTT_EINVAL;
}

int bltt_apply_sym(bltt_handle* h, int32_t precision, const void* x_dev, void* y_dev) {
  if (!h || !x_dev || !y_dev) return BLTT_EINVAL;
  if (h->N == 1) return BLTT_EUNSUPPORTED;
  const int64_t bytes = h->n * (precision == BLTT_FP64 ? 8 : 4);
  if (overlaps(x_dev, y_dev, bytes)) return BLTT_EINVAL;
  int rc = step_prepare(h, precision);
  if (rc) return rc;
  int64_t np = 0;
  if (precision == BLTT_FP64)
    rc = matvec<double>(h, MV_DOT, TERM_STENCIL, (const double*)x_dev, (double*)y_dev, nullptr, &np);
  else
    rc = matvec<float>(h, MV_DOT, TERM_STENCIL, (const float*)x_dev, (float*)y_dev, nullptr, &np);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  return BLTT_OK;
}

int bltt_apply_precond(bltt_handle* h, int32_t precision, const void* x_dev, void* y_dev) {
  if (!h || !x_dev || !y_dev) return BLTT_EINVAL;
  if (h->N == 1) return BLTT_EUNSUPPORTED;
  const int64_t bytes = h->n * (precision == BLTT_FP64 ? 8 : 4);
  if (overlaps(x_dev, y_dev, bytes)) return BLTT_EINVAL;
  int rc = step_prepare(h, precision);
  if (rc) return rc;
  int64_t np = 0;
  if (precision == BLTT_FP64)
    rc = precond<double>(h, (const double*)x_dev, nullptr, nullptr, nullptr, h->coef_one, h->w64.Q,
                         (const double*)x_dev, (double*)y_dev, &np);
  else
    rc = precond<float>(h, (const float*)x_dev, nullptr, nullptr, nullptr, h->coef_one, h->w32.Q,
                        (const float*)x_dev, (float*)y_dev, &np);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  return BLTT_OK;
}

int bltt_apply_space(bltt_handle* h, int32_t precision, const void* x_dev, void* y_dev) {
  if (!h || !x_dev || !y_dev) return BLTT_EINVAL;
  const int64_t bytes = h->n * (precision == BLTT_FP64 ? 8 : 4);
  if (overlaps(x_dev, y_dev, bytes)) return BLTT_EINVAL;
  int rc = step_prepare(h, precision);
  if (rc) return rc;
  const int Lx = 2 * (h->m[0] + 1);
  const int64_t nlx = h->n / h->m[0];
  if (precision == BLTT_FP64) {
    HIPCHK(launch_dst_x<double>(Lx, KIND_VUPD, (const double*)x_dev, nullptr, nullptr, nullptr, nullptr,
                                (double*)y_dev, nlx, dst_tables<double>(h, 0), h->coef_one, nullptr,
                                vupd_stencil<double>(h, nullptr), h->stream));
    if ((rc = space_strided<double>(h, (double*)y_dev, false))) return rc;
  } else {
    HIPCHK(launch_dst_x<float>(Lx, KIND_VUPD, (const float*)x_dev, nullptr, nullptr, nullptr, nullptr,
                               (float*)y_dev, nlx, dst_tables<float>(h, 0), h->coef_one, nullptr,
                               vupd_stencil<float>(h, nullptr), h->stream));
    if ((rc = space_strided<float>(h, (float*)y_dev, false))) return rc;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return BLTT_OK;
}

// ---------------------------------------------------------------------------
// Sine-coordinate step entry points: the kernels of the default (sine-basis)
// solve, one application each, on mode-major vectors (element (i, n) at
// i*N + n).  Reductions go through h->partials and the scalar kernel.
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

template <typename T>
int step_tables(bltt_handle* h) {
  return build_tables<T>(h);
}

int step_tables_for(bltt_handle* h, int32_t precision) {
  if (precision == BLTT_FP64) return step_tables<double>(h);
  if (precision == BLTT_FP32) return step_tables<float>(h);
  if (precision == BLTT_MIXED) {
    int rc = step_tables<double>(h);
    return rc ? rc : step_tables<float>(h);
  }
  return BLTT_EINVAL;
}

// reduce the np partial sums left in h->partials; *out receives the sum
int reduce_to_host(bltt_handle* h, int64_t np, double* out) {
  int rc;
  if ((rc = scalar(h, SC_NORM, np, nullptr))) return rc;
  if ((rc = read_state(h))) return rc;
  if (out) *out = h->state_host->norm2;
  return BLTT_OK;
}

int upload_step(bltt_handle* h, int at, const double* src, int count) {
  HIPCHK(hipMemcpyAsync(h->step_dev + at, src, sizeof(double) * (size_t)count, hipMemcpyHostToDevice, h->stream));
  return BLTT_OK;
}

template <typename T, typename TQ>
int modes_lanczos_impl(bltt_handle* h, const void* q, const void* v1, const void* v2, const double* coef,
                       void* vout, void* zout, double* dot) {
  const bool full = v1 || v2;
  double c[4] = {coef ? coef[0] : 1.0, coef && v1 ? coef[1] : 0.0, coef && v2 ? coef[2] : 0.0, 0.0};
  const T* V1 = (const T*)(v1 ? v1 : v2);
  const T* V2 = (const T*)(v2 ? v2 : V1);
  int rc;
  if ((rc = upload_step(h, STEP_COEF, c, 4))) return rc;
  int64_t np = 0;
  {
    ProfScope ps(h, BLTT_K_TIME, (double)h->n * (sizeof(TQ) + sizeof(T) * (1.0 + (vout ? 1 : 0) + (v1 ? 1 : 0) +
                                                                               (v2 ? 1 : 0))));
    HIPCHK(launch_time_upd<T, TQ>((int)h->N, full, h->opt.precond == BLTT_PRECOND_ABAC, (const TQ*)q, V1, V2,
                                  (T*)vout, (T*)zout, h->M, time_tables<T>(h, false), h->step_dev + STEP_COEF,
                                  h->partials, time_blocks<T>(h), &np, h->stream, false, time_plan<T>(h)));
  }
  return reduce_to_host(h, np, dot);
}

}  // namespace

extern "C" {

int bltt_modes_forward(bltt_handle* h, const double* x_dev, double* xhat_dev, double* norm2) {
  if (!h || !x_dev || !xhat_dev) return BLTT_EINVAL;
  if (overlaps(x_dev, xhat_dev, h->n * (int64_t)sizeof(double))) return BLTT_EINVAL;
  int rc = step_tables<double>(h);
  if (rc) return rc;
  int64_t np = 0;
  if ((rc = sine_forward(h, x_dev, xhat_dev, &np))) return rc;
  return reduce_to_host(h, np, norm2);
}

int bltt_modes_backward(bltt_handle* h, double* xhat_dev, double* x_dev) {
  if (!h || !x_dev || !xhat_dev) return BLTT_EINVAL;
  if (overlaps(x_dev, xhat_dev, h->n * (int64_t)sizeof(double))) return BLTT_EINVAL;
  int rc = step_tables<double>(h);
  if (rc) return rc;
  if ((rc = sine_backward(h, xhat_dev, x_dev))) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  return BLTT_OK;
}

int bltt_modes_sym(bltt_handle* h, int32_t precision, const void* z_dev, void* q_dev, double* dot) {
  if (!h || !z_dev || !q_dev) return BLTT_EINVAL;
  if (precision != BLTT_FP64 && precision != BLTT_FP32) return BLTT_EINVAL;
  if (h->var || h->N == 1) return BLTT_EUNSUPPORTED;
  const int64_t bytes = h->n * (precision == BLTT_FP64 ? 8 : 4);
  if (overlaps(z_dev, q_dev, bytes)) return BLTT_EINVAL;
  int rc = step_tables_for(h, precision);
  if (rc) return rc;
  int64_t np = 0;
  if (precision == BLTT_FP64)
    rc = matvec<double>(h, MV_DOT, TERM_SPEC, (const double*)z_dev, (double*)q_dev, nullptr, &np);
  else
    rc = matvec<float>(h, MV_DOT, TERM_SPEC, (const float*)z_dev, (float*)q_dev, nullptr, &np);
  if (rc) return rc;
  return reduce_to_host(h, np, dot);
}

}  // extern "C"

namespace {

// argument checks shared by bltt_modes_lanczos and its no-alloc variant
int lanczos_args(const bltt_handle* h, int32_t precision, const void* q_dev, const void* v1_dev, const void* v2_dev,
                 const void* vout_dev, const void* zout_dev) {
  if (!h || !q_dev || !zout_dev) return BLTT_EINVAL;
  if (h->var || h->N == 1) return BLTT_EUNSUPPORTED;
  if (precision != BLTT_FP64 && precision != BLTT_FP32 && precision != BLTT_MIXED) return BLTT_EINVAL;
  if (precision == BLTT_MIXED && (v1_dev || v2_dev)) return BLTT_EINVAL;
  if (h->opt.precond != BLTT_PRECOND_ABAC && precision != BLTT_FP64) return BLTT_EUNSUPPORTED;
  const int64_t bt = h->n * (precision == BLTT_FP64 ? 8 : 4);
  const int64_t bq = h->n * (precision == BLTT_FP32 ? 4 : 8);
  // outputs overlap no input and not each other
  const void* ins[3] = {q_dev, v1_dev, v2_dev};
  const int64_t inb[3] = {bq, bt, bt};
  for (int i = 0; i < 3; ++i) {
    if (!ins[i]) continue;
    if (overlaps(ins[i], inb[i], zout_dev, bt)) return BLTT_EINVAL;
    if (vout_dev && overlaps(ins[i], inb[i], vout_dev, bt)) return BLTT_EINVAL;
  }
  if (vout_dev && overlaps(vout_dev, zout_dev, bt)) return BLTT_EINVAL;
  return BLTT_OK;
}

// the launch of bltt_modes_lanczos_noalloc: coefficients, partial sums,
// reduction and scalar state in this device's scratch
template <typename T, typename TQ>
int lanczos_noalloc_impl(bltt_handle* h, double* scr_dev, const void* q, const void* v1, const void* v2,
                         const double* coef, void* vout, void* zout, double* dot) {
  const bool full = v1 || v2;
  const double c[4] = {coef ? coef[0] : 1.0, coef && v1 ? coef[1] : 0.0, coef && v2 ? coef[2] : 0.0, 0.0};
  const T* V1 = (const T*)(v1 ? v1 : v2);
  const T* V2 = (const T*)(v2 ? v2 : V1);
  HIPCHK(hipMemcpyAsync(scr_dev + scr::COEF, c, sizeof(c), hipMemcpyHostToDevice, h->stream));
  int64_t np = 0;
  HIPCHK(launch_time_upd<T, TQ>((int)h->N, full, h->opt.precond == BLTT_PRECOND_ABAC, (const TQ*)q, V1, V2, (T*)vout,
                                (T*)zout, h->M, time_tables<T>(h, false), scr_dev + scr::COEF, scr_dev,
                                time_blocks<T>(h), &np, h->stream, false, time_plan<T>(h)));
  SolverState* st = reinterpret_cast<SolverState*>(scr_dev + scr::STATE);
  HIPCHK(launch_scalar(SC_NORM, st, scr_dev, np, nullptr, 0, nullptr, scr_dev + scr::RED, scr::RED_HALF, ZBasis{},
                       h->stream));
  HIPCHK(hipMemcpyAsync(&h->state_host->norm2, &st->norm2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (dot) *dot = h->state_host->norm2;
  return BLTT_OK;
}

}  // namespace

extern "C" {

int bltt_modes_lanczos_noalloc(bltt_handle* h, int32_t precision, const void* q_dev, const void* v1_dev,
                               const void* v2_dev, const double* coef, void* vout_dev, void* zout_dev,
                               double* dot) {
  int rc = lanczos_args(h, precision, q_dev, v1_dev, v2_dev, vout_dev, zout_dev);
  if (rc) return rc;
  // the tables must exist already: building them would allocate
  const bool ready = precision == BLTT_FP64 ? h->t64.ready
                                            : (precision == BLTT_FP32 ? h->t32.ready : h->t32.ready && h->t64.ready);
  if (!ready) return BLTT_EINVAL;
  const int64_t np = precision == BLTT_FP64 ? upd_blocks<double>((int)h->N, h->M, time_blocks<double>(h))
                                            : upd_blocks<float>((int)h->N, h->M, time_blocks<float>(h));
  if (np > scr::PARTS) return BLTT_EUNSUPPORTED;
  double* scr_dev = scratch_ptr(h->device);
  if (!scr_dev) return BLTT_EHIP;
  if (precision == BLTT_FP64)
    return lanczos_noalloc_impl<double, double>(h, scr_dev, q_dev, v1_dev, v2_dev, coef, vout_dev, zout_dev, dot);
  if (precision == BLTT_FP32)
    return lanczos_noalloc_impl<float, float>(h, scr_dev, q_dev, v1_dev, v2_dev, coef, vout_dev, zout_dev, dot);
  return lanczos_noalloc_impl<float, double>(h, scr_dev, q_dev, nullptr, nullptr, coef, vout_dev, zout_dev, dot);
}

int bltt_modes_lanczos(bltt_handle* h, int32_t precision, const void* q_dev, const void* v1_dev,
                       const void* v2_dev, const double* coef, void* vout_dev, void* zout_dev, double* dot) {
  int rc = lanczos_args(h, precision, q_dev, v1_dev, v2_dev, vout_dev, zout_dev);
  if (rc) return rc;
  rc = step_tables_for(h, precision);
  if (rc) return rc;
  if (precision == BLTT_FP64)
    return modes_lanczos_impl<double, double>(h, q_dev, v1_dev, v2_dev, coef, vout_dev, zout_dev, dot);
  if (precision == BLTT_FP32)
    return modes_lanczos_impl<float, float>(h, q_dev, v1_dev, v2_dev, coef, vout_dev, zout_dev, dot);
  return modes_lanczos_impl<float, double>(h, q_dev, nullptr, nullptr, coef, vout_dev, zout_dev, dot);
}

int bltt_modes_resid(bltt_handle* h, const double* fhat_dev, double* u_dev, double* r_dev,
                     const float* const* z_dev, const double* y, int32_t k, double scale, double* norm2) {
  if (!h || !fhat_dev || !u_dev || !r_dev) return BLTT_EINVAL;
  if (h->var || h->N == 1) return BLTT_EUNSUPPORTED;
  if (k < 0 || k > ZB_MAX || (k > 0 && (!z_dev || !y))) return BLTT_EINVAL;
  const int64_t b8 = h->n * 8;
  if (overlaps(fhat_dev, r_dev, b8) || overlaps(u_dev, r_dev, b8) || overlaps(u_dev, fhat_dev, b8))
    return BLTT_EINVAL;
  for (int i = 0; i < k; ++i) {
    if (!z_dev[i]) return BLTT_EINVAL;
    if (overlaps(z_dev[i], h->n * 4, u_dev, b8) || overlaps(z_dev[i], h->n * 4, r_dev, b8)) return BLTT_EINVAL;
  }
  int rc = step_tables<double>(h);
  if (rc) return rc;
  int64_t np = 0;
  if (k > 0) {
    if ((rc = upload_step(h, STEP_Y, y, k))) return rc;
    if ((rc = upload_step(h, STEP_SCALE, &scale, 1))) return rc;
  }
  if (k > 0 && short_p(h)) {
    ZList<float> zl;
    for (int i = 0; i < ZB_MAX; ++i) zl.z[i] = i < k ? z_dev[i] : nullptr;
    zl.k = k;
    ProfScope ps(h, BLTT_K_WX, (16.0 + 4.0 * k) * h->n);
    HIPCHK(launch_combine<float>(u_dev, zl, h->step_dev + STEP_Y, h->step_dev + STEP_SCALE, h->n, h->stream));
  }
  if (k > 0 && !short_p(h)) {
    IterUpd up{};
    for (int i = 0; i < ZB_MAX; ++i) up.z[i] = i < k ? z_dev[i] : nullptr;
    up.k = k;
    up.y = h->step_dev + STEP_Y;
    up.s = h->step_dev + STEP_SCALE;
    up.u_zero = 0;
    ProfScope ps(h, BLTT_K_RESID64, (32.0 + 4.0 * k) * h->n);
    HIPCHK(launch_matvec_fft<double>((int)(2 * h->N), MV_RESID, TERM_SPEC, u_dev, r_dev, fhat_dev, h->M,
                                     mv_tables<double>(h), up, h->partials, h->stream));
    np = mv_blocks<double>(true, (int)(2 * h->N), h->M);
  } else {
    if ((rc = matvec<double>(h, MV_RESID, TERM_SPEC, u_dev, r_dev, fhat_dev, &np))) return rc;
  }
  return reduce_to_host(h, np, norm2);
}

int bltt_profile_enable(bltt_handle* h, int32_t enable) {
  if (!h) return BLTT_EINVAL;
  if (enable) {
    HIPCHK(hipStreamSynchronize(h->stream));
    h->recs.clear();
    h->pool_used = 0;
  }
  h->prof = enable != 0;
  return BLTT_OK;
}

int bltt_profile_read(bltt_handle* h, int32_t kernel_class, int64_t* launches, double* total_ms, double* bytes) {
  if (!h || kernel_class < 0 || kernel_class >= BLTT_K_COUNT) return BLTT_EINVAL;
  HIPCHK(hipStreamSynchronize(h->stream));
  int64_t cnt = 0;
  double ms = 0.0, by = 0.0;
  for (const auto& r : h->recs) {
    if (r.cls != kernel_class) continue;
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ++cnt;
    ms += t;
    by += r.bytes;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  return BLTT_OK;
}

}  // extern "C"
