// Host-side launchers of the hot-path kernels (one definition per kernel
// translation unit, explicitly instantiated for float and double).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bltt_kernels.hpp"

namespace bltt {

// Smallest alpha of the FP32 preconditioner (the mixed path's sweeps and the
// FP32 step entry points): an FP32 time pass scales its lines by up to
// 1/alpha around its transforms, so its rounding grows like eps_32/alpha.
// Below 1e-4 the mixed path's sweeps converge more slowly (8 iterations at
// 1e-5, 12 at 1e-6 against 6) and not at all at 1e-8; they use
// P_alpha' with alpha' = max(alpha, 1e-4), an SPD preconditioner of the same
// system.  The FP64 residual and the FP64 path use alpha itself.
constexpr double ALPHA_MIN_FP32 = 1e-4;

// First member of every handle type, so that one destroy call serves them all
constexpr uint32_t HANDLE_MAGIC = 0x424c5448u;  // single system
constexpr uint32_t BATCH_MAGIC = 0x424c5442u;   // batch

// Device-side context: thread/block indices and the workgroup barrier.
struct DevCtx {
  int tid, bid, bid_y, nbx;
  __device__ void sync() { __syncthreads(); }
  // wavefront-scope barrier: orders this wavefront's LDS accesses (the LDS
  // executes one wavefront's instructions in order)
  __device__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};
__device__ inline DevCtx make_ctx() {
  DevCtx c;
  c.tid = (int)threadIdx.x;
  c.bid = (int)blockIdx.x;
  c.bid_y = (int)blockIdx.y;
  c.nbx = (int)gridDim.x;
  return c;
}

inline int64_t ew_blocks(int64_t n) {
  const int64_t b = (n + TPB_EW - 1) / TPB_EW;
  return b < 1 ? 1 : (b > 16384 ? 16384 : b);
}

template <typename T>
hipError_t launch_time_prec(int L, T* x, int64_t M, const TimeTables<T>& tb, hipStream_t s);

// workgroups (= partial sums) of one launch_time_upd: FP32 runs persistently
// on at most max_blocks workgroups, FP64 one workgroup per tile
template <typename T>
inline int64_t upd_blocks(int L, int64_t M, int64_t max_blocks) {
  const int64_t tiles = fft_tiles<T, FK_SPEC>(L, M);
  return upd_persistent<T>() ? std::max<int64_t>(1, std::min(tiles, max_blocks)) : tiles;
}

// sine coordinates: vhat = cq Q (+ cv V1 + cvp V2 when full) -> Vout (optional),
// Zout = P^{-1} vhat (time pass), per-workgroup partial sums of <vhat, Zout>
// (persistent: at most max_blocks workgroups, *nparts receives the partial count)
// prec false: no preconditioner (Zout = vhat; FP64 only)
// qrev (start only): read Q with its time lines reversed, i.e. vhat = cq Y Q
// plan: radix plan of the FP32 transforms (0, or 1 where fft_plan_alt(L); FP64 runs plan 0)
template <typename T, typename TQ>
hipError_t launch_time_upd(int L, bool full, bool prec, const TQ* Q, const T* V1, const T* V2, T* Vout, T* Zout, int64_t M,
                           const TimeTables<T>& tb, const double* coef, double* partials, int64_t max_blocks,
                           int64_t* nparts, hipStream_t s, bool qrev = false, int plan = 0);

// up: refinement update of the iterate z (MV_RESID with TERM_SPEC only; k = 0 for none)
template <typename T>
hipError_t launch_matvec_fft(int L, int mode, int term, T* z, T* out, const T* fin, int64_t M,
                             const MatvecTables<T>& tb, const IterUpd& up, double* partials, hipStream_t s);

// sine coordinates, mode-major: Y (p * z + mu (q * z)) with N-point transforms
// (MV_DOT: out, partial sums of <out, z>; MV_RESID: out = Y (fin - A u) after
// u <- u + s sum y_i Z_i when up.k > 0, partial sums of ||out||^2)
template <typename T>
hipError_t launch_matvec_cs(int L, int mode, T* z, T* out, const T* fin, int64_t M, const MatvecCSTables<T>& tb,
                            const IterUpd& up, double* partials, int64_t max_blocks, int64_t* nparts,
                            hipStream_t s, int plan = 0);

template <typename T>
hipError_t launch_matvec_short(int mode, const T* z, T* out, const T* fin, int64_t M,
                               const ShortTables<T>& tb, double* partials, int64_t* nparts, hipStream_t s);

template <typename T>
hipError_t launch_dst_x(int L, int kind, const T* in, const T* v1, const T* v2, T* vout, const T* vdot, T* out,
                        int64_t nlines, const DstTables<T>& tb, const double* coef, double* partials,
                        const VupdStencil<T>& sten, hipStream_t s);

// x-line sine transform fused with the layout move: dir 0 time-major in ->
// mode-major out (+ partial sums of ||in||^2 when partials is non-null, count
// in *nparts); dir 1 mode-major in -> time-major out.  FP64.
template <typename T>
hipError_t launch_dst_xt(int L, int dir, const T* in, T* out, int64_t N, int64_t M, const DstTables<T>& tb,
                         double* partials, int64_t* nparts, hipStream_t s);
template <typename T>
hipError_t launch_dst_strided(int L, T* x, int64_t nlines, int64_t S, const DstTables<T>& tb, hipStream_t s);
// launch_dst_xt for S systems of one shape (n = N M elements each) in one
// launch; each side is a device array of per-system pointers (p) or a base
// with stride n (b), the other null.  No norm partial sums.  FP64.
template <typename T>
hipError_t launch_bt_dst_xt(int L, int dir, const T* const* in_p, const T* in_b, T* const* out_p, T* out_b,
                            int64_t n, int64_t N, int64_t M, int S, const DstTables<T>& tb, hipStream_t s);

// kernel attribute setup (dynamic LDS above 64 KiB): configure_kernels_once
// runs it once per process
hipError_t configure_kernels();
hipError_t configure_kernels_once();

// streaming and scalar kernels
template <typename T>
hipError_t launch_resid_stencil(T* r, const VupdStencil<T>& st, int64_t nlines, double* partials, int64_t* nparts,
                                hipStream_t s);
template <typename TO>
hipError_t launch_rhs(const double* f, TO* b, int64_t N, int64_t M, double scale, double* partials,
                      int64_t* nparts, hipStream_t s);
template <typename T, typename TX>
hipError_t launch_wx(const T* Z, T* Wa, const T* Wb, TX* X, int64_t n, const double* coef, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* x, int64_t n, T val, hipStream_t s);
template <typename TI, typename TO>
hipError_t launch_scale_cast(const TI* x, TO* y, int64_t n, const double* sptr, int invert, hipStream_t s);
template <typename TD>
hipError_t launch_axpy64(double* u, const TD* d, int64_t n, const double* sptr, hipStream_t s);
// scratch: 2*scratch_half doubles for the first reduction stage of long
// partial-sum arrays (at most scratch_half workgroups of RED_CHUNK each)
// mirror: null, or a host-mapped pinned SolverState the kernel publishes the
// state to (st->seq counts the publications; the host polls mirror->seq)
// one time step (N = 1): uhat = fhat / (p0 + q0 mu) when solve, then the
// partial sums of ||fhat - (p0 + q0 mu) uhat||^2
hipError_t launch_single_step(const double* fhat, double* uhat, int64_t M, const double* mu, double p0, double q0,
                              int solve, double* partials, int64_t* nparts, hipStream_t s);
hipError_t launch_scalar(int phase, SolverState* st, const double* partials, int64_t np, const double* aux,
                         int64_t naux, double* hist, double* scratch, int64_t scratch_half, ZBasis zb,
                         hipStream_t s, SolverState* mirror = nullptr);
// u += (*sptr) * sum_i y[i] Z_i over the zl.k stored vectors
template <typename T>
hipError_t launch_combine(double* u, const ZList<T>& zl, const double* y, const double* sptr, int64_t n,
                          hipStream_t s);

// ---------------------------------------------------------------------------
// batched sine-basis kernels (kern_batch.hip): S systems of one shape, vectors
// back to back (system s at s*n), per-instance tables
// ---------------------------------------------------------------------------
enum { BT_START = 0, BT_UPD = 1, BT_MATVEC = 2, BT_START32 = 3 };

// BT_START: Z = P^{-1} (rinv_s Q) with Q the FP64 residual, Vout = rinv_s Q;
// BT_START32: Z = P^{-1} Q with Q the FP32 residual r/||fhat_s|| a residual
// pass left (Vout null: Q itself is v_1); BT_UPD: Vout = coef_v (Q, V1, V2),
// Z = P^{-1} Vout; BT_MATVEC: Qout = Y T Z.
// plan: radix plan of the transforms (0, or 1 where fft_plan_alt(L))
hipError_t launch_bt(int which, int L, int tpb, int plan, const void* Q, const float* V1, const float* V2,
                     float* Vout, float* Z, float* Qout, const BatchVec& bv, const BatchTabs& bt, double* partials,
                     hipStream_t s);
int64_t bt_tiles(int L, int tpb, int64_t M);
// r32 non-null (with bv.bscale): the residual goes to r32 as FP32 r/||fhat_s||
// and the update is scaled by ||fhat_s||; null: R in FP64, scaled by ||r_s||
hipError_t launch_bt_resid(int L2, double* const* u, double* R, const double* Fh, const BatchVec& bv,
                           const BatchTabs& bt, const ZPool& pool, const double* zb, int K, int u_zero,
                           double* partials, int64_t* T2, float* r32, hipStream_t s);
hipError_t launch_bt_scalar(int phase, const BatchVec& bv, const double* partials, int64_t T, double* hist,
                            int64_t hist_stride, double* zb, int K, double inner_tol, int cap, hipStream_t s);
hipError_t launch_bt_rhs(const double* f, double* b, int64_t N, const BatchVec& bv, double* partials, int64_t* BPS,
                         hipStream_t s);
}  // namespace bltt
