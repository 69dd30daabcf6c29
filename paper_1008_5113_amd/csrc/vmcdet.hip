// vmcdet: kernels and the C-ABI entry points (see include/vmcdet.h).
//
// Every walker is processed by one workgroup of NT threads; a launch covers a
// list of walkers (one workgroup each).  The persistent path (vmc_run_steps)
// keeps each workgroup on its walker for all requested steps, so refactors and
// reorders of one walker never stall the others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "vmc_step.hpp"

using namespace vmc;

namespace {

constexpr int MODE_BUILD = 1;
constexpr int MODE_REORDER = 2;
constexpr int MODE_ILUTP = 4;

__device__ inline Smem setup_smem(char* smem, const Walker& W, const DevParams& P, int ktb) {
  LdsLayout L = lds_layout(W.n, ktb, P);
  return make_smem(smem, L);
}

template <int PREC>
__global__ void __launch_bounds__(NT) k_setup(const Walker* __restrict__ walkers, WalkerState* states,
                                              DevParams P, const int* list, int mode) {
  extern __shared__ __align__(16) char smem[];
  const int w = list ? list[blockIdx.x] : (int)blockIdx.x;
  const Walker& W = walkers[w];
  Smem S = setup_smem(smem, W, P, PREC == VMC_PREC_FP64 ? 8 : 4);
  S.ph = states[w].ph;
  S.ilu_retries = &states[w].ilu_retries;
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  __syncthreads();
  int st = WST_OK;
  // a rebuild or refactor starts the walker afresh: earlier errors are
  // re-detected if they persist
  if (threadIdx.x == 0) states[w].status = WST_OK;
  if (mode & MODE_REORDER)
    wg_reorder(W, S, (void*)W.V, (size_t)(P.maxit + 1) * W.n * (PREC == VMC_PREC_FP64 ? 8 : 4));
  if (mode & (MODE_BUILD | MODE_REORDER)) st |= wg_build_all_rows(W, S);
  PhaseClock pc;
  pc.start();
  if (st == WST_OK && (mode & MODE_ILUTP)) {
    st = wg_ilutp(W, P, S);
    pc.stop(S, PH_REFACTOR);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    WalkerState* ws = states + w;
    if (mode & MODE_ILUTP) {
      ws->m = 0;
      ws->upd_entries = 0.0;
      ws->st_refactors += 1;
      if (mode & MODE_REORDER) ws->st_reorders += 1;
    }
    ws->pend_valid = 0;
    if (st != WST_OK) ws->status |= st;
  }
}

// One trial move of each listed walker (list null: walker = block index).
// ratio_out (may be null) receives the ratios, out the step records.
template <int PREC>
__global__ void __launch_bounds__(NT, 4) k_ratio(const Walker* __restrict__ walkers, WalkerState* states,
                                              DevParams P, const int* list, const int* particles,
                                              const double* newpos, vmc_step_record* out, double* ratio_out) {
  extern __shared__ __align__(16) char smem[];
  const int w = list ? list[blockIdx.x] : (int)blockIdx.x;
  const Walker& W = walkers[w];
  WalkerState* ws = states + w;
  Smem S = setup_smem(smem, W, P, PREC == VMC_PREC_FP64 ? 8 : 4);
  S.ph = states[w].ph;
  S.ilu_retries = &states[w].ilu_retries;
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  __syncthreads();
  if (ws->status != WST_OK) {
    if (threadIdx.x == 0) {
      out[blockIdx.x].flags = -1;
      if (ratio_out) ratio_out[blockIdx.x] = 0.0;
      ws->pend_valid = 0;
    }
    return;
  }
  const long long g = ws->g;
  double u[4];
  step_draws(W.seed, g, u);
  int p;
  double rnew[3];
  if (particles) {
    p = particles[blockIdx.x];
    rnew[0] = newpos[3 * blockIdx.x];
    rnew[1] = newpos[3 * blockIdx.x + 1];
    rnew[2] = newpos[3 * blockIdx.x + 2];
  } else {
    p = (int)(g % W.n);
    for (int c = 0; c < 3; ++c) rnew[c] = propose_axis(W.pos[3 * p + c], u[c], P.step, W.box[c]);
  }
  wg_det_ratio<PREC>(W, ws, P, S, p, rnew, u[3]);
  if (threadIdx.x == 0) {
    if ((P.test_knobs & VMC_TEST_ZERO_RATIO) && ws->pend_valid) ws->pend_ratio = 0.0;
    fill_record(out[blockIdx.x], ws, w, ws->pend_ratio, ws->pend_flags);
    if (ratio_out) ratio_out[blockIdx.x] = ws->pend_ratio;
  }
}

// Commit or discard the pending move of each listed walker (list null:
// walker = block index).  err_out[k] (may be null) receives CERR_* bits: no
// pending move, or a forced acceptance of a zero or non-finite ratio, which
// is refused with the move left pending.  With sticky set the bits also go to
// the walker's call_err, for vmc_sync to report.
template <int PREC>
__global__ void __launch_bounds__(NT) k_accept(const Walker* __restrict__ walkers, WalkerState* states,
                                               DevParams P, const int* list, const unsigned char* decide,
                                               unsigned char* accepted_out, int* err_out, int sticky) {
  extern __shared__ __align__(16) char smem[];
  const int w = list ? list[blockIdx.x] : (int)blockIdx.x;
  const Walker& W = walkers[w];
  WalkerState* ws = states + w;
  Smem S = setup_smem(smem, W, P, PREC == VMC_PREC_FP64 ? 8 : 4);
  S.ph = states[w].ph;
  S.ilu_retries = &states[w].ilu_retries;
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  __syncthreads();
  int err = 0;
  if (!ws->pend_valid) err = CERR_NOPENDING;
  else if (decide && decide[blockIdx.x] && !ratio_acceptable(ws->pend_ratio)) err = CERR_ZERO_RATIO;
  if (err) {
    if (threadIdx.x == 0) {
      if (err_out) err_out[blockIdx.x] = err;
      if (accepted_out) accepted_out[blockIdx.x] = 0;
      if (sticky) ws->call_err |= err;
    }
    return;
  }
  int acc;
  if (decide) acc = decide[blockIdx.x] ? 1 : 0;
  else acc = (ws->pend_ratio * ws->pend_ratio > ws->pend_uacc && ratio_acceptable(ws->pend_ratio)) ? 1 : 0;
  wg_accept<PREC>(W, ws, P, S, acc, w, nullptr);
  if (threadIdx.x == 0) {
    if (accepted_out) accepted_out[blockIdx.x] = (unsigned char)acc;
    if (err_out) err_out[blockIdx.x] = 0;
  }
}

// Persistent fused path: `steps` Metropolis steps of one walker per workgroup.
template <int PREC>
__global__ void __launch_bounds__(NT, 4) k_run(const Walker* __restrict__ walkers, WalkerState* states,
                                            DevParams P, int steps, vmc_step_record* log, long long log_cap,
                                            const int* order) {
  extern __shared__ __align__(16) char smem[];
  // workgroup -> walker: the autotuner's longest-first order, else identity
  const int w = order ? order[blockIdx.x] : (int)blockIdx.x;
  const Walker& W = walkers[w];
  WalkerState* ws = states + w;
  Smem S = setup_smem(smem, W, P, PREC == VMC_PREC_FP64 ? 8 : 4);
  S.ph = states[w].ph;
  S.ilu_retries = &states[w].ilu_retries;
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  __syncthreads();
  PhaseClock pstep;
  pstep.start();
  for (int s = 0; s < steps; ++s) {
    if (ws->status != WST_OK) break;
    const long long g = ws->g;
    double u[4];
    step_draws(W.seed, g, u);
    const int p = (int)(g % W.n);
    double rnew[3];
    for (int c = 0; c < 3; ++c) rnew[c] = propose_axis(W.pos[3 * p + c], u[c], P.step, W.box[c]);
    wg_det_ratio<PREC>(W, ws, P, S, p, rnew, u[3]);
    if (!ws->pend_valid) break;
    const int acc = (ws->pend_ratio * ws->pend_ratio > u[3] && ratio_acceptable(ws->pend_ratio)) ? 1 : 0;
    const long long slot = (long long)w * steps + s;
    vmc_step_record* rec = (log && slot < log_cap) ? log + slot : nullptr;
    wg_accept<PREC>(W, ws, P, S, acc, w, rec);
  }
  pstep.stop(S, PH_STEP);
}

// Kinetic-energy terms of particles [p0, p1) (clamped to n) of the listed
// walkers at their current positions: e_out[k * estride] = (sum of the terms)
// / n, and the terms themselves at terms + toff[k] when terms is not null.  A
// walker with a pending move or an error is skipped with err_out[k] != 0.
template <int PREC>
__global__ void __launch_bounds__(NT, 4) k_energy(const Walker* __restrict__ walkers, WalkerState* states,
                                               DevParams P, const int* list, int p0, int p1, double* e_out,
                                               int estride, double* terms, const long long* toff,
                                               int* err_out) {
  extern __shared__ __align__(16) char smem[];
  const int w = list[blockIdx.x];
  const Walker& W = walkers[w];
  WalkerState* ws = states + w;
  Smem S = setup_smem(smem, W, P, PREC == VMC_PREC_FP64 ? 8 : 4);
  S.ph = states[w].ph;
  S.ilu_retries = &states[w].ilu_retries;
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  __syncthreads();
  if (ws->status != WST_OK || ws->pend_valid) {
    if (threadIdx.x == 0) {
      err_out[blockIdx.x] = ws->pend_valid ? 2 : 1;
      e_out[(size_t)blockIdx.x * estride] = 0.0;
    }
    return;
  }
  const int hi = min(p1, W.n), lo = min(p0, hi);
  const double sum = wg_energy<PREC>(W, ws, P, S, lo, hi, terms ? terms + toff[blockIdx.x] : nullptr);
  if (threadIdx.x == 0) {
    e_out[(size_t)blockIdx.x * estride] = sum / W.n;
    err_out[blockIdx.x] = ws->status != WST_OK ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// The standard algorithm (Section 1), as a comparison path: the explicit
// inverse, read for the ratio and updated by Sherman-Morrison on an accepted
// move.  Walker w's inverse is stored particle-major in original labels:
// bmat[w][p * n + j] = (A^{-1})_{jp} for particle p and site j, so column p of
// the inverse is one contiguous row.
// ---------------------------------------------------------------------------

// Row stride of a stored inverse (16-byte aligned rows) and the LDS carve of
// the standard-algorithm step kernel.
__host__ __device__ inline size_t sm_ld(int n) { return align_up((size_t)n, 2); }
struct SmLds {
  size_t col, nv, ov, nc, oc, sd, si, total;
};
__host__ __device__ inline SmLds sm_lds(int n, int cap) {
  SmLds L;
  size_t o = 0;
  L.col = o; o += align_up((size_t)n * 8, 16);
  L.nv = o;  o += align_up((size_t)cap * 8, 16);
  L.ov = o;  o += align_up((size_t)cap * 8, 16);
  L.nc = o;  o += align_up((size_t)cap * 4, 16);
  L.oc = o;  o += align_up((size_t)cap * 4, 16);
  L.sd = o;  o += 64;
  L.si = o;  o += 32;
  L.total = o;
  return L;
}

// Columns p0..p1-1 of A^{-1}: A z = e_{rpos[p]} by the preconditioned solver
// with its tolerance replaced by tol, z mapped back to site labels.
template <int PREC>
__global__ void __launch_bounds__(NT, 4) k_inverse_cols(const Walker* __restrict__ walkers, WalkerState* states,
                                                     DevParams P, double* const* bmat, int p0, int p1,
                                                     double tol, int* nonconv) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x;
  const Walker& W = walkers[w];
  WalkerState* ws = states + w;
  P.rtol = tol;
  P.refine_tol = tol;
  Smem S = setup_smem(smem, W, P, PREC == VMC_PREC_FP64 ? 8 : 4);
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  __syncthreads();
  if (ws->status != WST_OK || ws->pend_valid) {
    if (threadIdx.x == 0) nonconv[w] = -1;
    return;
  }
  const int n = W.n;
  const size_t ld = sm_ld(n);
  double* B = bmat[w];
  int bad = 0;
  for (int p = p0; p < min(p1, n); ++p) {
    const StepSolve o = wg_solve<PREC>(W, ws->m, P, S, W.rpos[p], 0, true);
    bad += o.conv ? 0 : 1;
    for (int c = vmc_tid(); c < n; c += NT) B[(size_t)p * ld + W.colsite[c]] = W.zvec[c];
    __syncthreads();
  }
  if (threadIdx.x == 0) nonconv[w] = bad;
}

// `steps` Metropolis steps of every walker by the standard algorithm:
// ratio = a'^T A^{-1} e_p; on accept A^{-1} <- A^{-1} - (A^{-1} e_p)(u^T A^{-1}) / ratio
// with u = a' - a_p.  The proposal, the draws and the decision are those of
// the sparse path.  Row m of the update is one wave's: it forms
// (u^T A^{-1})_m from the row's entries at the two rows' sites, then streams
// the row.  LDS: column p of the old inverse and the two Slater rows.
__global__ void __launch_bounds__(NT) k_sm_run(const Walker* __restrict__ walkers, WalkerState* states,
                                               DevParams P, double* const* bmat, int steps,
                                               vmc_step_record* log, long long log_cap) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x;
  const Walker& W = walkers[w];
  WalkerState* ws = states + w;
  const int n = W.n, cap = W.W;
  const size_t ld = sm_ld(n);
  const SmLds L = sm_lds(n, cap);
  double* col = (double*)(smem + L.col);
  double* nv = (double*)(smem + L.nv);
  double* ov = (double*)(smem + L.ov);
  int* nc = (int*)(smem + L.nc);
  int* oc = (int*)(smem + L.oc);
  double* sd = (double*)(smem + L.sd);  // [0] ratio
  int* si = (int*)(smem + L.si);        // [0] new count, [1] old count
  double* B = bmat[w];
  const int lane = lane_id(), wid = wave_id();
  for (int s = 0; s < steps; ++s) {
    if (ws->status != WST_OK) break;
    const long long g = ws->g;
    double u[4];
    step_draws(W.seed, g, u);
    const int p = (int)(g % n);
    double rnew[3], rold[3];
    for (int c = 0; c < 3; ++c) {
      rold[c] = W.pos[3 * p + c];
      rnew[c] = propose_axis(rold[c], u[c], P.step, W.box[c]);
    }
    // new row (wave 0) and old row (wave 1), by site
    if (wid == 0) {
      const int cnt = wave_row<int, 0>(W, rnew[0], rnew[1], rnew[2], nullptr, nc, nv, nullptr, cap);
      if (lane == 0) si[0] = cnt;
    } else if (wid == 1) {
      const int cnt = wave_row<int, 0>(W, rold[0], rold[1], rold[2], nullptr, oc, ov, nullptr, cap);
      if (lane == 0) si[1] = cnt;
    }
    __syncthreads();
    const int cn = si[0], co = si[1];
    if (cn > cap || co > cap) {
      if (threadIdx.x == 0) ws->status |= WST_CAPACITY;
      break;
    }
    // ratio = a'^T (A^{-1} e_p) (wave 0), broadcast through LDS
    if (wid == 0) {
      double acc = 0.0;
      for (int e = lane; e < cn; e += 64) acc += nv[e] * B[(size_t)p * ld + nc[e]];
      acc = wave_sum(acc);
      if (lane == 0) sd[0] = acc;
    }
    __syncthreads();
    const double ratio = sd[0];
    const int acc = (ratio * ratio > u[3] && isfinite(ratio) && ratio != 0.0) ? 1 : 0;
    if (acc) {
      for (int j = vmc_tid(); j < n; j += NT) col[j] = B[(size_t)p * ld + j];
      __syncthreads();
      const double inv = 1.0 / ratio;
      for (int m = wid; m < n; m += NWAVE) {
        double* row = B + (size_t)m * ld;
        double t = 0.0;
        for (int e = lane; e < cn; e += 64) t += nv[e] * row[nc[e]];
        for (int e = lane; e < co; e += 64) t -= ov[e] * row[oc[e]];
        const double f = wave_sum(t) * inv;
        int j = 2 * lane;
        for (; j + 384 + 1 < n; j += 512) {
          double2 x0 = *(const double2*)(row + j);
          double2 x1 = *(const double2*)(row + j + 128);
          double2 x2 = *(const double2*)(row + j + 256);
          double2 x3 = *(const double2*)(row + j + 384);
          x0.x -= f * col[j];       x0.y -= f * col[j + 1];
          x1.x -= f * col[j + 128]; x1.y -= f * col[j + 129];
          x2.x -= f * col[j + 256]; x2.y -= f * col[j + 257];
          x3.x -= f * col[j + 384]; x3.y -= f * col[j + 385];
          *(double2*)(row + j) = x0;
          *(double2*)(row + j + 128) = x1;
          *(double2*)(row + j + 256) = x2;
          *(double2*)(row + j + 384) = x3;
        }
        for (; j < n; j += 128) {
          row[j] -= f * col[j];
          if (j + 1 < n) row[j + 1] -= f * col[j + 1];
        }
      }
      if (threadIdx.x == 0) {
        W.pos[3 * p] = rnew[0];
        W.pos[3 * p + 1] = rnew[1];
        W.pos[3 * p + 2] = rnew[2];
      }
    }
    if (threadIdx.x == 0) {
      const long long slot = (long long)w * steps + s;
      if (log && slot < log_cap) {
        vmc_step_record& r = log[slot];
        r.step = g;
        r.walker = w;
        r.particle = p;
        r.new_pos[0] = rnew[0];
        r.new_pos[1] = rnew[1];
        r.new_pos[2] = rnew[2];
        r.ratio = ratio;
        r.log_abs_ratio = ::log(fabs(ratio));
        r.u_acc = u[3];
        r.N = 0.0;
        r.resid = 0.0;
        r.iters = 0;
        r.flags = (acc ? VMC_FLAG_ACCEPTED : 0) | VMC_FLAG_CONVERGED;
        r.refinements = 0;
        r.inner_solves = 0;
      }
      ws->g = g + 1;
      ws->st_steps += 1;
      if (acc) ws->st_acc += 1;
    }
    __threadfence();
    __syncthreads();
  }
}

// Diagnostic: one phase of the solve, repeated `reps` times per walker on the
// walker's current matrix and factors (no state change except ILUTP).
template <int PREC>
__global__ void __launch_bounds__(NT, 4) k_phase(const Walker* __restrict__ walkers, WalkerState* states,
                                                 DevParams P, int phase, int reps) {
  extern __shared__ __align__(16) char smem[];
  using KT = typename std::conditional<PREC == VMC_PREC_FP64, double, float>::type;
  const int w = blockIdx.x;
  const Walker& W = walkers[w];
  Smem S = setup_smem(smem, W, P, sizeof(KT));
  if (threadIdx.x < 32) S.ic[threadIdx.x] = 0;
  const int n = W.n;
  KT* xs = (KT*)S.A;
  KT* D = xs + align_up((size_t)n, 4);
  KT* st = (KT*)S.stmp;
  for (int e = threadIdx.x; e < DTILE; e += NT) D[e] = (KT)0;
  for (int r = threadIdx.x; r < n; r += NT) xs[r] = (KT)(1.0 / (1.0 + r));
  __syncthreads();
  const int m = states[w].m;
  for (int it = 0; it < reps; ++it) {
    switch (phase) {
      case 0: wg_spmv<KT>(W, Fac<KT>::aval(W), xs, (KT*)W.wv); break;
      case 1: wg_lsolve<KT>(W, Fac<KT>::lval(W), nullptr, it % n, xs, D, st); break;
      case 2: wg_usolve<KT>(W, Fac<KT>::usval(W), Fac<KT>::dinv(W), xs, D, st); break;
      case 3: wg_updates<KT>(W, m, P.m_max, xs, S); break;
      case 4: {
        const size_t stage = (size_t)((char*)S.red - S.A);
        (void)wg_resid64(W, W.zvec, it % n, W.rvec, S, stage);
        for (int e = threadIdx.x; e < DTILE; e += NT) D[e] = (KT)0;
        break;
      }
      case 5: (void)wg_ilutp(W, P, S); break;
      default: break;
    }
    __syncthreads();
  }
  if (phase == 5 && reps > 0 && threadIdx.x == 0) {
    // a refactor: the stored updates belong to the old factors
    states[w].m = 0;
    states[w].upd_entries = 0.0;
    states[w].st_refactors += reps;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
std::string g_create_error;

struct Ctx {
  hipStream_t stream = nullptr;
  vmc_params prm;
  DevParams dp;
  int nw = 0;
  int maxn = 0;
  int all_same_n = 1;
  std::vector<Walker> hw;
  std::vector<void*> arenas;
  Walker* dW = nullptr;
  WalkerState* dS = nullptr;
  size_t lds = 0;
  // argument staging
  int* d_list = nullptr;
  int* d_part = nullptr;
  double* d_pos = nullptr;
  vmc_step_record* d_rec = nullptr;
  unsigned char* d_dec = nullptr;
  unsigned char* d_acc = nullptr;
  int* d_err = nullptr;
  int* d_all = nullptr;
  // workgroup -> walker order of the persistent launch (set by the autotuner)
  int* d_order = nullptr;
  bool use_order = false;
  // graph of the persistent launch and the arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  int g_steps = -1;
  void* g_log = nullptr;
  long long g_cap = -1;
  bool g_order = false;
  // standard algorithm: one stored inverse per walker, and the device table of them
  std::vector<void*> sm_bufs;
  double** d_smB = nullptr;        // the inverse table and flags in use
  int* d_nonconv = nullptr;
  double** smB_own = nullptr;      // the ones vmc_sm_prepare allocated
  int* nonconv_own = nullptr;
  bool sm_static = false;          // the inverses in use live in the static scratch
  int sm_dev = -1;                 // the device whose scratch holds them
  int max_cap = 0;
  // the stored inverses belong to the walkers' current matrices: set by
  // vmc_sm_prepare, kept by vmc_sm_run_steps, cleared by every other call that
  // may move a walker, rebuild its rows or reorder them
  bool sm_current = false;
  // per walker: positions moved by vmc_sm_run_steps since its rows (A) or its
  // factors were last rebuilt, so the sparse path would use stale matrices
  std::vector<char> rows_stale, fac_stale;
  std::string err;
};

#define HIPCHK(ctx, expr)                                                   \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);       \
      return VMC_EHIP;                                                      \
    }                                                                       \
  } while (0)

int lattice_bound(double radius, double a) {
  const int K = (int)std::ceil(radius / a);
  int cnt = 0;
  for (int x = -K; x <= K; ++x)
    for (int y = -K; y <= K; ++y)
      for (int z = -K; z <= K; ++z)
        if ((double)(x * x + y * y + z * z) * a * a <= radius * radius) ++cnt;
  return cnt;
}

template <int PREC>
vmc_status launch_setup(Ctx* c, const int* dlist, int count, int mode) {
  hipLaunchKernelGGL(k_setup<PREC>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, dlist, mode);
  HIPCHK(c, hipGetLastError());
  return VMC_OK;
}

vmc_status stage_list(Ctx* c, const int32_t* walkers, int32_t count, int** dlist) {
  if (count < 0 || count > c->nw) { c->err = "bad walker count"; return VMC_EINVAL; }
  if (walkers == nullptr) { *dlist = c->d_all; return VMC_OK; }
  std::vector<char> seen(c->nw, 0);
  for (int k = 0; k < count; ++k) {
    if (walkers[k] < 0 || walkers[k] >= c->nw) { c->err = "walker index out of range"; return VMC_EINVAL; }
    // one workgroup per listed walker: a walker listed twice would be worked on twice at once
    if (seen[walkers[k]]++) { c->err = "walker " + std::to_string(walkers[k]) + " listed twice"; return VMC_EINVAL; }
  }
  HIPCHK(c, hipMemcpyAsync(c->d_list, walkers, sizeof(int) * count, hipMemcpyHostToDevice, c->stream));
  *dlist = c->d_list;
  return VMC_OK;
}

vmc_status check_sparse(Ctx* c, const int32_t* walkers, int32_t count) {
  for (int k = 0; k < count; ++k) {
    const int w = walkers ? walkers[k] : k;
    if (c->rows_stale[w] || c->fac_stale[w]) {
      c->err = "walker " + std::to_string(w) +
               ": moved by vmc_sm_run_steps; rebuild its rows and factors (vmc_build_slater, then vmc_ilutp, or "
               "vmc_ilutp with reorder) first";
      return VMC_ESTATE;
    }
  }
  return VMC_OK;
}

vmc_status walker_errors(Ctx* c) {
  // the walker states come back a few at a time through a stack buffer, so
  // the check allocates nothing
  constexpr int CH = 8;
  WalkerState hs[CH];
  for (int w0 = 0; w0 < c->nw; w0 += CH) {
    const int cnt = std::min(CH, c->nw - w0);
    HIPCHK(c, hipMemcpyAsync(hs, c->dS + w0, sizeof(WalkerState) * cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < cnt; ++k) {
      const int w = w0 + k;
      if (hs[k].status & WST_CAPACITY) { c->err = "walker " + std::to_string(w) + ": capacity exceeded"; return VMC_ECAPACITY; }
      if (hs[k].status & WST_SINGULAR) { c->err = "walker " + std::to_string(w) + ": singular pivot"; return VMC_ESINGULAR; }
      if (hs[k].status & WST_NOCONV) {
        c->err = "walker " + std::to_string(w) + ": GMRES did not converge even after reorder and refactor";
        return VMC_ENOCONV;
      }
    }
  }
  return VMC_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of vmc_sm_prepare_static: one array per GPU the library runs
// on, held until the process ends.  A call lays out in it the inverse table
// (one pointer per walker), the not-converged flags and then every walker's
// inverse (sm_ld(n) x n doubles), each part 256-byte aligned.  Host code uses
// the device address hipGetSymbolAddress gives for the current device, never
// the array's name.  The last context to fill a GPU's scratch owns it.
constexpr size_t SM_STATIC_BYTES = (size_t)64 << 20;
constexpr int SM_STATIC_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SM_STATIC_BYTES];
static char* g_scratch_ptr[SM_STATIC_DEVICES];
static const Ctx* g_scratch_owner[SM_STATIC_DEVICES];

size_t sm_static_offset(const Ctx* c, int walker) {
  size_t o = align_up((size_t)c->nw * sizeof(double*), 256) + align_up((size_t)c->nw * 4, 256);
  for (int w = 0; w < walker; ++w) o += align_up(sm_ld(c->hw[w].n) * (size_t)c->hw[w].n * 8, 256);
  return o;
}

bool sm_static_owned(const Ctx* c) {
  return c->sm_dev >= 0 && c->sm_dev < SM_STATIC_DEVICES && g_scratch_owner[c->sm_dev] == c;
}

const void* sm_static_inverse(const Ctx* c, int walker) {
  if (!sm_static_owned(c)) return nullptr;
  return g_scratch_ptr[c->sm_dev] + sm_static_offset(c, walker);
}

void sm_static_release(const Ctx* c) {
  if (c->sm_static && sm_static_owned(c)) g_scratch_owner[c->sm_dev] = nullptr;
}

// The inverse table of a static layout (the same offsets as sm_static_offset).
__global__ void k_sm_table(const Walker* __restrict__ walkers, int nw, char* base) {
  if (threadIdx.x != 0) return;
  double** tab = (double**)base;
  size_t o = align_up((size_t)nw * sizeof(double*), 256) + align_up((size_t)nw * 4, 256);
  for (int w = 0; w < nw; ++w) {
    tab[w] = (double*)(base + o);
    const int n = walkers[w].n;
    o += align_up(sm_ld(n) * (size_t)n * 8, 256);
  }
}

// Caller errors recorded by device-pointer calls since the last check; clears them.
vmc_status call_errors(Ctx* c) {
  std::vector<WalkerState> hs(c->nw);
  HIPCHK(c, hipMemcpyAsync(hs.data(), c->dS, sizeof(WalkerState) * c->nw, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  vmc_status first = VMC_OK;
  bool any = false;
  for (int w = 0; w < c->nw; ++w) {
    if (!hs[w].call_err) continue;
    any = true;
    if (first == VMC_OK) {
      if (hs[w].call_err & CERR_NOPENDING) {
        c->err = "walker " + std::to_string(w) + ": accept without a pending ratio";
        first = VMC_ESTATE;
      } else {
        c->err = "walker " + std::to_string(w) + ": forced acceptance of a zero or non-finite ratio refused";
        first = VMC_ESINGULAR;
      }
    }
    hs[w].call_err = 0;
  }
  if (any) {
    // only the call_err words change; nothing runs on the stream meanwhile
    for (int w = 0; w < c->nw; ++w)
      HIPCHK(c, hipMemcpyAsync((char*)(c->dS + w) + offsetof(WalkerState, call_err), &hs[w].call_err, sizeof(int),
                               hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return first;
}

}  // namespace

extern "C" {

vmc_status vmc_default_params(vmc_params* p) {
  if (!p) return VMC_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->precision = VMC_PREC_FP64;
  p->gmres_maxit = 40;
  p->gmres_rtol = 1e-10;
  p->droptol = 1e-4;
  p->permtol = 0.1;
  p->lfil = -1;
  p->m_max = 32;
  p->n_thresh = 100.0;
  p->iter_factor = 4.0;
  p->iter_min_solves = 10;
  p->inner_rtol = 1e-6;
  p->refine_tol = 1e-10;
  p->refine_maxit = 4;
  p->step = 0.25;
  p->row_cap = 0;
  p->force_reorder_every = 0;
  p->refactor_cost = 0.0;
  return VMC_OK;
}

vmc_status vmc_create(void** ctx_out, const vmc_params* p, int32_t n_walkers, const vmc_walker_init* wi,
                      void* hip_stream) {
  if (!ctx_out || !p || !wi || n_walkers <= 0) { g_create_error = "invalid arguments"; return VMC_EINVAL; }
  *ctx_out = nullptr;
  if (p->precision != VMC_PREC_FP64 && p->precision != VMC_PREC_MIXED) { g_create_error = "bad precision"; return VMC_EINVAL; }
  if (p->gmres_maxit < 1 || p->gmres_maxit > MAXIT) { g_create_error = "gmres_maxit out of range"; return VMC_EINVAL; }
  if (p->m_max < 1 || p->m_max > MMAX_CAP) { g_create_error = "m_max out of range"; return VMC_EINVAL; }
  Ctx* c = new Ctx();
  c->stream = (hipStream_t)hip_stream;
  c->prm = *p;
  c->nw = n_walkers;
  DevParams& d = c->dp;
  d.precision = p->precision;
  d.maxit = p->gmres_maxit;
  d.rtol = p->gmres_rtol;
  d.droptol = p->droptol;
  d.permtol = p->permtol;
  d.lfil = p->lfil;
  d.m_max = p->m_max;
  d.n_thresh = p->n_thresh;
  d.iter_factor = p->iter_factor;
  d.iter_min_solves = p->iter_min_solves;
  d.inner_rtol = p->inner_rtol;
  d.refine_tol = p->refine_tol;
  d.refine_maxit = p->refine_maxit;
  d.step = p->step;
  d.force_reorder_every = p->force_reorder_every;
  if (p->ilu_drop_norm != 0 && p->ilu_drop_norm != 1) {
    delete c;
    g_create_error = "ilu_drop_norm must be 0 or 1";
    return VMC_EINVAL;
  }
  d.ilu_drop_norm = p->ilu_drop_norm;
  d.test_knobs = p->test_knobs;
  d.plain_stop = p->plain_stop != 0;
  auto hshift_of = [](int hs) {
    int lg = 0;
    while ((1 << lg) < hs) ++lg;
    return 32 - lg;
  };
  d.ilu = IluCfg{ILU_R, ILU_DEF_HS, 0, ILU_DEF_NZ, ILU_DEF_C, ILU_DEF_L};
  d.ilu_fast = IluCfg{ILU_FAST_R, ILU_FAST_HS, 0, ILU_FAST_NZ, ILU_FAST_C, ILU_FAST_L};
  if (p->ilu_work_cap > 0) {
    if (p->ilu_work_cap > 8192) {
      delete c;
      g_create_error = "ilu_work_cap out of range";
      return VMC_EINVAL;
    }
    const int cap = (p->ilu_work_cap + 63) / 64 * 64;
    d.ilu.nz = std::max(cap, ILU_DEF_NZ);
    d.ilu.c = std::max(cap, ILU_DEF_C);
    d.ilu.l = std::max(cap, ILU_DEF_L);
    d.ilu.hs = ILU_DEF_HS;
    while (d.ilu.hs < 2 * d.ilu.nz) d.ilu.hs *= 2;
    d.ilu_fast.r = 0;  // a given capacity is the one used
  }
  if (p->test_knobs & VMC_TEST_ILU_FAST_SMALL) {
    d.ilu_fast.nz = 64;
    d.ilu_fast.c = 64;
    d.ilu_fast.l = 16;
  }
  d.ilu.hshift = hshift_of(d.ilu.hs);
  d.ilu_fast.hshift = hshift_of(d.ilu_fast.hs);

  const int ktb = p->precision == VMC_PREC_FP64 ? 8 : 4;
  auto fail = [&](vmc_status s, const std::string& msg) {
    g_create_error = msg;
    for (void* a : c->arenas) (void)hipFree(a);
    for (void* q : {(void*)c->dW, (void*)c->dS, (void*)c->d_list, (void*)c->d_all, (void*)c->d_part, (void*)c->d_pos,
                    (void*)c->d_rec, (void*)c->d_dec, (void*)c->d_acc, (void*)c->d_err, (void*)c->d_order})
      if (q) (void)hipFree(q);
    delete c;
    return s;
  };
  c->hw.resize(n_walkers);
  c->rows_stale.assign(n_walkers, 0);
  c->fac_stale.assign(n_walkers, 0);
  for (int w = 0; w < n_walkers; ++w) {
    const vmc_walker_init& in = wi[w];
    const int n = in.n;
    if (n < 1 || n > 16384 || !in.sites || !in.sigma || !in.pos0 || in.a <= 0.0 || in.cutoff <= 0.0)
      return fail(VMC_EINVAL, "walker " + std::to_string(w) + ": invalid init");
    const int nb = in.n_basis == 0 ? 1 : in.n_basis;
    if (nb < 1 || nb > 4 || in.lattice[0] < 1 || in.lattice[1] < 1 || in.lattice[2] < 1 ||
        (long long)nb * in.lattice[0] * in.lattice[1] * in.lattice[2] != n)
      return fail(VMC_EINVAL, "walker " + std::to_string(w) + ": lattice and basis do not match n");
    for (int b = 0; b < nb && in.n_basis > 0; ++b)
      for (int k = 0; k < 3; ++k)
        if (!(in.basis[b][k] >= 0.0 && in.basis[b][k] < 1.0))
          return fail(VMC_EINVAL, "walker " + std::to_string(w) + ": basis offsets must lie in [0, 1)");
    if (w > 0 && n != wi[0].n) c->all_same_n = 0;
    c->maxn = std::max(c->maxn, n);
    Walker& W = c->hw[w];
    std::memset(&W, 0, sizeof(W));
    W.n = n;
    for (int k = 0; k < 3; ++k) {
      W.lat[k] = in.lattice[k];
      W.box[k] = in.lattice[k] * in.a;
    }
    W.a = in.a;
    W.nb = nb;
    for (int k = 0; k < 3; ++k) {
      double mx = 0.0;
      for (int b = 0; b < nb && in.n_basis > 0; ++b) mx = std::max(mx, in.basis[b][k]);
      W.bmax[k] = mx * in.a;
    }
    W.margin = in.site_margin;
    W.cutoff = in.cutoff;
    W.kind = in.orbital_kind;
    W.p_scale = in.p_scale;
    W.p_sigma = in.p_sigma;
    W.seed = in.seed;
    // every site of the cell repeats on a simple-cubic lattice of spacing a
    int Wc = p->row_cap > 0 ? p->row_cap
                            : nb * lattice_bound(in.cutoff + in.site_margin + 0.8660254037844387 * in.a, in.a);
    Wc = std::min(Wc, n);
    Wc = (Wc + 15) / 16 * 16;  // 64-byte aligned rows (whole cache lines, vector loads)
    W.W = Wc;
    c->max_cap = std::max(c->max_cap, Wc);
    W.F = std::min(n, Wc + (Wc + 1) / 2 + 2);
    W.UC = 2 * Wc;
    const int km = p->gmres_maxit;
    const int mm = p->m_max;
    // arena layout
    std::vector<std::pair<void**, size_t>> parts;
    size_t off = 0;
    auto add = [&](size_t bytes) {
      size_t o = off;
      off = align_up(off + bytes, 256);
      return o;
    };
    const size_t nn = (size_t)n;
    size_t o_sites = add(nn * 3 * 8), o_sigma = add(nn * 8), o_pos = add(nn * 3 * 8);
    size_t o_rowperm = add(nn * 4), o_rpos = add(nn * 4), o_cpos = add(nn * 4), o_colsite = add(nn * 4);
    size_t o_reo_row = add(nn * 4), o_reo_col = add(nn * 4);
    const size_t na = a_rows_padded(n);  // A's rows, padded to whole slices
    size_t o_alen = add(nn * 4), o_acol = add(na * Wc * 2), o_aval = add(na * Wc * 8), o_aval32 = add(na * Wc * 4);
    const size_t F = W.F;
    size_t o_llen = add(nn * 4), o_lcol = add(nn * F * 4), o_lval = add(nn * F * 8);
    size_t o_ulen = add(nn * 4), o_ucol = add(nn * F * 4), o_uval = add(nn * F * 8), o_udiag = add(nn * 8);
    size_t o_udinv = add(nn * 8), o_udinv32 = add(nn * 4);
    size_t o_lp = add((nn + 1) * 4), o_lc = add(nn * F * 2), o_lv64 = add(nn * F * 8), o_lv32 = add(nn * F * 4);
    size_t o_up = add((nn + 1) * 4), o_uc = add(nn * F * 2), o_uv64 = add(nn * F * 8), o_uv32 = add(nn * F * 4);
    size_t o_q = add(nn * 4);
    size_t o_Z64 = p->precision == VMC_PREC_FP64 ? add((size_t)mm * nn * 8) : 0;
    size_t o_Z32 = p->precision == VMC_PREC_MIXED ? add((size_t)mm * nn * 4) : 0;
    size_t o_uplen = add((size_t)mm * 4), o_upcol = add((size_t)mm * W.UC * 4), o_upval = add((size_t)mm * W.UC * 8),
           o_upval32 = add((size_t)mm * W.UC * 4), o_T = add((size_t)mm * mm * 8);
    size_t o_V = add((size_t)(km + 1) * nn * ktb), o_Xp = add((size_t)km * nn * ktb), o_wv = add(nn * ktb);
    size_t o_z = add(nn * 8), o_r = add(nn * 8);
    size_t o_newcol = add((size_t)Wc * 4), o_newval = add((size_t)Wc * 8), o_pucol = add((size_t)W.UC * 4),
           o_puval = add((size_t)W.UC * 8);
    void* arena = nullptr;
    {
      const hipError_t e = hipMalloc(&arena, off);
      if (e != hipSuccess)
        return fail(VMC_ENOMEM, "walker " + std::to_string(w) + ": device allocation of " + std::to_string(off) +
                                    " bytes failed: " + hipGetErrorString(e));
    }
    c->arenas.push_back(arena);
    if (hipMemset(arena, 0, off) != hipSuccess) return fail(VMC_EHIP, "memset failed");
    char* b = (char*)arena;
    W.sites = (decltype(W.sites))(b + o_sites);
    W.sigma = (decltype(W.sigma))(b + o_sigma);
    W.pos = (decltype(W.pos))(b + o_pos);
    W.rowperm = (decltype(W.rowperm))(b + o_rowperm);
    W.rpos = (decltype(W.rpos))(b + o_rpos);
    W.cpos = (decltype(W.cpos))(b + o_cpos);
    W.colsite = (decltype(W.colsite))(b + o_colsite);
    W.reo_row = (decltype(W.reo_row))(b + o_reo_row);
    W.reo_col = (decltype(W.reo_col))(b + o_reo_col);
    W.a_len = (decltype(W.a_len))(b + o_alen);
    W.a_col = (decltype(W.a_col))(b + o_acol);
    W.a_val = (decltype(W.a_val))(b + o_aval);
    W.a_val32 = (decltype(W.a_val32))(b + o_aval32);
    W.l_len = (decltype(W.l_len))(b + o_llen);
    W.l_col = (decltype(W.l_col))(b + o_lcol);
    W.l_val = (decltype(W.l_val))(b + o_lval);
    W.u_len = (decltype(W.u_len))(b + o_ulen);
    W.u_col = (decltype(W.u_col))(b + o_ucol);
    W.u_val = (decltype(W.u_val))(b + o_uval);
    W.u_diag = (decltype(W.u_diag))(b + o_udiag);
    W.u_dinv = (decltype(W.u_dinv))(b + o_udinv);
    W.u_dinv32 = (decltype(W.u_dinv32))(b + o_udinv32);
    W.lp = (decltype(W.lp))(b + o_lp);
    W.lc = (decltype(W.lc))(b + o_lc);
    W.lv64 = (decltype(W.lv64))(b + o_lv64);
    W.lv32 = (decltype(W.lv32))(b + o_lv32);
    W.up = (decltype(W.up))(b + o_up);
    W.uc = (decltype(W.uc))(b + o_uc);
    W.uv64 = (decltype(W.uv64))(b + o_uv64);
    W.uv32 = (decltype(W.uv32))(b + o_uv32);
    W.ilu_q = (decltype(W.ilu_q))(b + o_q);
    W.Z64 = p->precision == VMC_PREC_FP64 ? (decltype(W.Z64))(b + o_Z64) : nullptr;
    W.Z32 = p->precision == VMC_PREC_MIXED ? (decltype(W.Z32))(b + o_Z32) : nullptr;
    W.up_len = (decltype(W.up_len))(b + o_uplen);
    W.up_col = (decltype(W.up_col))(b + o_upcol);
    W.up_val = (decltype(W.up_val))(b + o_upval);
    W.up_val32 = (decltype(W.up_val32))(b + o_upval32);
    W.T = (decltype(W.T))(b + o_T);
    W.V = (decltype(W.V))(b + o_V);
    W.Xp = (decltype(W.Xp))(b + o_Xp);
    W.wv = (decltype(W.wv))(b + o_wv);
    W.zvec = (decltype(W.zvec))(b + o_z);
    W.rvec = (decltype(W.rvec))(b + o_r);
    W.new_col = (decltype(W.new_col))(b + o_newcol);
    W.new_val = (decltype(W.new_val))(b + o_newval);
    W.pu_col = (decltype(W.pu_col))(b + o_pucol);
    W.pu_val = (decltype(W.pu_val))(b + o_puval);
    // host-side initial data
    std::vector<int> ident(n);
    for (int k = 0; k < n; ++k) ident[k] = k;
    bool ok = true;
    ok &= hipMemcpy((void*)W.sites, in.sites, nn * 3 * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy((void*)W.sigma, in.sigma, nn * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy((void*)W.pos, in.pos0, nn * 3 * 8, hipMemcpyHostToDevice) == hipSuccess;
    for (void* dst : {(void*)W.rowperm, (void*)W.rpos, (void*)W.cpos, (void*)W.colsite, (void*)W.reo_row,
                      (void*)W.reo_col, (void*)W.ilu_q})
      ok &= hipMemcpy(dst, ident.data(), nn * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return fail(VMC_EHIP, "initial copy failed");
  }
  if (hipMalloc(&c->dW, sizeof(Walker) * n_walkers) != hipSuccess ||
      hipMalloc(&c->dS, sizeof(WalkerState) * n_walkers) != hipSuccess)
    return fail(VMC_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(hipGetLastError()));
  if (hipMemcpy(c->dW, c->hw.data(), sizeof(Walker) * n_walkers, hipMemcpyHostToDevice) != hipSuccess)
    return fail(VMC_EHIP, "initial copy failed");
  {
    std::vector<WalkerState> hs(n_walkers);
    std::memset(hs.data(), 0, sizeof(WalkerState) * n_walkers);
    for (auto& s : hs) s.refactor_cost = p->refactor_cost;
    if (hipMemcpy(c->dS, hs.data(), sizeof(WalkerState) * n_walkers, hipMemcpyHostToDevice) != hipSuccess)
      return fail(VMC_EHIP, "initial copy failed");
  }
  // staging buffers
  std::vector<int> all(n_walkers);
  for (int k = 0; k < n_walkers; ++k) all[k] = k;
  bool ok = hipMalloc(&c->d_list, sizeof(int) * n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_all, sizeof(int) * n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_part, sizeof(int) * n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_pos, sizeof(double) * 3 * n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_rec, sizeof(vmc_step_record) * n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_dec, n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_acc, n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_err, sizeof(int) * n_walkers) == hipSuccess;
  ok &= hipMalloc(&c->d_order, sizeof(int) * n_walkers) == hipSuccess;
  if (!ok) return fail(VMC_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(hipGetLastError()));
  if (hipMemcpy(c->d_all, all.data(), sizeof(int) * n_walkers, hipMemcpyHostToDevice) != hipSuccess)
    return fail(VMC_EHIP, "initial copy failed");

  int dev = 0, maxlds = 0, cu_lds = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  (void)hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  if (cu_lds <= 0) cu_lds = maxlds;
  // as many concurrently factored ILUTP rows as the LDS holds (results do not
  // depend on it): first the full configuration alone, then the fast one with
  // as many rows as keep the workgroups per CU that the full one allows
  const IluCfg fast = c->dp.ilu_fast;
  c->dp.ilu_fast.r = 0;
  LdsLayout L = lds_layout(c->maxn, ktb, c->dp);
  while (c->dp.ilu.r > 1 && maxlds > 0 && (int)L.total > maxlds) {
    c->dp.ilu.r -= 1;
    L = lds_layout(c->maxn, ktb, c->dp);
  }
  const auto per_cu = [&](size_t bytes) { return cu_lds > 0 ? (size_t)cu_lds / bytes : 1; };
  for (int r = fast.r; r > c->dp.ilu.r; --r) {
    DevParams t = c->dp;
    t.ilu_fast = fast;
    t.ilu_fast.r = r;
    const LdsLayout Lf = lds_layout(c->maxn, ktb, t);
    if ((maxlds <= 0 || (int)Lf.total <= maxlds) && per_cu(Lf.total) >= per_cu(L.total)) {
      c->dp.ilu_fast = t.ilu_fast;
      L = Lf;
      break;
    }
  }
  c->lds = L.total;
  if (maxlds > 0 && (int)c->lds > maxlds) {
    return fail(VMC_EINVAL, "n too large: needs " + std::to_string(c->lds) + " bytes of LDS per workgroup, device has " +
                                std::to_string(maxlds));
  }
  if (p->precision == VMC_PREC_FP64) {
    (void)hipFuncSetAttribute((const void*)k_setup<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_ratio<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_accept<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_run<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_energy<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_inverse_cols<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
  } else {
    (void)hipFuncSetAttribute((const void*)k_setup<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_ratio<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_accept<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_run<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_energy<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    (void)hipFuncSetAttribute((const void*)k_inverse_cols<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(VMC_EHIP, "device synchronize failed");
  *ctx_out = c;
  return VMC_OK;
}

vmc_status vmc_build_slater(void* ctx, const int32_t* walkers, int32_t count) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return VMC_EINVAL;
  c->sm_current = false;
  if (!walkers) count = c->nw;
  int* dl = nullptr;
  vmc_status s = stage_list(c, walkers, count, &dl);
  if (s) return s;
  if (count == 0) return VMC_OK;
  s = c->dp.precision == VMC_PREC_FP64 ? launch_setup<VMC_PREC_FP64>(c, dl, count, MODE_BUILD)
                                       : launch_setup<VMC_PREC_MIXED>(c, dl, count, MODE_BUILD);
  if (s) return s;
  s = walker_errors(c);
  if (s) return s;
  for (int k = 0; k < count; ++k) c->rows_stale[walkers ? walkers[k] : k] = 0;
  return VMC_OK;
}

vmc_status vmc_ilutp(void* ctx, const int32_t* walkers, int32_t count, int32_t reorder) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return VMC_EINVAL;
  c->sm_current = false;
  if (!walkers) count = c->nw;
  int* dl = nullptr;
  vmc_status s = stage_list(c, walkers, count, &dl);
  if (s) return s;
  if (count == 0) return VMC_OK;
  const int mode = MODE_ILUTP | (reorder ? MODE_REORDER : 0);
  s = c->dp.precision == VMC_PREC_FP64 ? launch_setup<VMC_PREC_FP64>(c, dl, count, mode)
                                       : launch_setup<VMC_PREC_MIXED>(c, dl, count, mode);
  if (s) return s;
  s = walker_errors(c);
  if (s) return s;
  for (int k = 0; k < count; ++k) {
    const int w = walkers ? walkers[k] : k;
    if (reorder) c->rows_stale[w] = 0;  // the reorder rebuilds every row in the new order
    if (!c->rows_stale[w]) c->fac_stale[w] = 0;
  }
  return VMC_OK;
}

vmc_status vmc_det_ratio(void* ctx, const int32_t* walkers, int32_t count, const int32_t* particle,
                         const double* new_pos, double* ratio_out, vmc_step_record* info_out) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !ratio_out || count < 0) return VMC_EINVAL;
  c->sm_current = false;
  if ((particle == nullptr) != (new_pos == nullptr)) { c->err = "particle and new_pos go together"; return VMC_EINVAL; }
  const bool dev = c->prm.device_ptrs != 0;
  if (dev) {
    // device arrays, every walker, no synchronisation
    if (walkers) { c->err = "device-pointer mode takes every walker (walkers must be NULL)"; return VMC_EINVAL; }
    if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
    if (c->dp.precision == VMC_PREC_FP64)
      hipLaunchKernelGGL(k_ratio<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                         (const int*)nullptr, particle, new_pos, info_out ? info_out : c->d_rec, ratio_out);
    else
      hipLaunchKernelGGL(k_ratio<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                         (const int*)nullptr, particle, new_pos, info_out ? info_out : c->d_rec, ratio_out);
    HIPCHK(c, hipGetLastError());
    return VMC_OK;
  }
  if (!walkers) count = c->nw;
  int* dl = nullptr;
  vmc_status s = stage_list(c, walkers, count, &dl);
  if (s) return s;
  if (count == 0) return VMC_OK;
  s = check_sparse(c, walkers, count);
  if (s) return s;
  if (particle) {
    for (int k = 0; k < count; ++k) {
      const int w = walkers ? walkers[k] : k;
      const Walker& W = c->hw[w];
      if (particle[k] < 0 || particle[k] >= W.n) { c->err = "particle out of range"; return VMC_EINVAL; }
      for (int a = 0; a < 3; ++a) {
        const double x = new_pos[3 * k + a];
        if (!(x >= 0.0 && x < W.box[a])) { c->err = "new_pos outside the box"; return VMC_EINVAL; }
      }
    }
    HIPCHK(c, hipMemcpyAsync(c->d_part, particle, sizeof(int) * count, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_pos, new_pos, sizeof(double) * 3 * count, hipMemcpyHostToDevice, c->stream));
  }
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_ratio<VMC_PREC_FP64>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, dl,
                       particle ? c->d_part : nullptr, particle ? c->d_pos : nullptr, c->d_rec, (double*)nullptr);
  else
    hipLaunchKernelGGL(k_ratio<VMC_PREC_MIXED>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, dl,
                       particle ? c->d_part : nullptr, particle ? c->d_pos : nullptr, c->d_rec, (double*)nullptr);
  HIPCHK(c, hipGetLastError());
  std::vector<vmc_step_record> rec(count);
  HIPCHK(c, hipMemcpyAsync(rec.data(), c->d_rec, sizeof(vmc_step_record) * count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < count; ++k) {
    ratio_out[k] = rec[k].ratio;
    if (info_out) info_out[k] = rec[k];
  }
  return walker_errors(c);
}

vmc_status vmc_accept(void* ctx, const int32_t* walkers, int32_t count, const uint8_t* accept,
                      uint8_t* accepted_out) {
  Ctx* c = (Ctx*)ctx;
  if (!c || count < 0) return VMC_EINVAL;
  c->sm_current = false;
  const bool dev = c->prm.device_ptrs != 0;
  if (dev) {
    if (walkers) { c->err = "device-pointer mode takes every walker (walkers must be NULL)"; return VMC_EINVAL; }
    if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
    if (c->dp.precision == VMC_PREC_FP64)
      hipLaunchKernelGGL(k_accept<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                         (const int*)nullptr, accept, accepted_out, (int*)nullptr, 1);
    else
      hipLaunchKernelGGL(k_accept<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                         (const int*)nullptr, accept, accepted_out, (int*)nullptr, 1);
    HIPCHK(c, hipGetLastError());
    return VMC_OK;
  }
  if (!walkers) count = c->nw;
  int* dl = nullptr;
  vmc_status s = stage_list(c, walkers, count, &dl);
  if (s) return s;
  if (count == 0) return VMC_OK;
  s = check_sparse(c, walkers, count);
  if (s) return s;
  if (accept) HIPCHK(c, hipMemcpyAsync(c->d_dec, accept, count, hipMemcpyHostToDevice, c->stream));
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_accept<VMC_PREC_FP64>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, dl,
                       accept ? c->d_dec : nullptr, c->d_acc, c->d_err, 0);
  else
    hipLaunchKernelGGL(k_accept<VMC_PREC_MIXED>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, dl,
                       accept ? c->d_dec : nullptr, c->d_acc, c->d_err, 0);
  HIPCHK(c, hipGetLastError());
  std::vector<unsigned char> acc(count);
  std::vector<int> err(count);
  HIPCHK(c, hipMemcpyAsync(acc.data(), c->d_acc, count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(err.data(), c->d_err, sizeof(int) * count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (accepted_out) std::memcpy(accepted_out, acc.data(), count);
  vmc_status first = VMC_OK;
  for (int k = 0; k < count && first == VMC_OK; ++k) {
    const int w = walkers ? walkers[k] : k;
    if (err[k] & CERR_NOPENDING) {
      c->err = "walker " + std::to_string(w) + ": accept without a pending ratio";
      first = VMC_ESTATE;
    } else if (err[k] & CERR_ZERO_RATIO) {
      c->err = "walker " + std::to_string(w) + ": forced acceptance of a zero or non-finite ratio refused";
      first = VMC_ESINGULAR;
    }
  }
  if (first != VMC_OK) return first;
  return walker_errors(c);
}

static void launch_run_on(Ctx* c, int steps, vmc_step_record* dev_log, long long cap, hipStream_t stream) {
  c->sm_current = false;
  const int* order = c->use_order ? c->d_order : nullptr;
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_run<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, stream, c->dW, c->dS, c->dp, steps,
                       dev_log, cap, order);
  else
    hipLaunchKernelGGL(k_run<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, stream, c->dW, c->dS, c->dp, steps,
                       dev_log, cap, order);
}
static void launch_run(Ctx* c, int steps, vmc_step_record* dev_log, long long cap) {
  launch_run_on(c, steps, dev_log, cap, c->stream);
}

vmc_status vmc_run_steps(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap) {
  Ctx* c = (Ctx*)ctx;
  if (!c || steps < 0) return VMC_EINVAL;
  if (steps == 0) return VMC_OK;
  if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
  launch_run(c, steps, dev_log, (long long)(dev_log ? log_cap : 0));
  HIPCHK(c, hipGetLastError());
  return VMC_OK;
}

vmc_status vmc_run_steps_graph(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap) {
  Ctx* c = (Ctx*)ctx;
  if (!c || steps < 0) return VMC_EINVAL;
  if (steps == 0) return VMC_OK;
  if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
  c->sm_current = false;
  const long long cap = dev_log ? log_cap : 0;
  if (!c->gexec || c->g_steps != steps || c->g_log != (void*)dev_log || c->g_cap != cap ||
      c->g_order != c->use_order) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    // the launch is recorded on a private stream (capture is not possible on
    // the null stream, and recording runs nothing); the graph then runs on
    // the context's stream
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    launch_run_on(c, steps, dev_log, cap, c->cap_stream);
    const hipError_t le = hipGetLastError();
    const hipError_t ee = hipStreamEndCapture(c->cap_stream, &c->graph);
    HIPCHK(c, le);
    HIPCHK(c, ee);
    HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->g_steps = steps;
    c->g_log = (void*)dev_log;
    c->g_cap = cap;
    c->g_order = c->use_order;
  }
  HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  return VMC_OK;
}

vmc_status vmc_run_sweeps(void* ctx, int32_t sweeps, vmc_step_record* dev_log, int64_t log_cap) {
  Ctx* c = (Ctx*)ctx;
  if (!c || sweeps < 0) return VMC_EINVAL;
  if (!c->all_same_n) { c->err = "vmc_run_sweeps needs walkers of equal n; use vmc_run_steps"; return VMC_EINVAL; }
  const long long steps = (long long)sweeps * c->hw[0].n;
  if (steps > 0x7fffffffLL) { c->err = "too many steps"; return VMC_EINVAL; }
  return vmc_run_steps_graph(ctx, (int32_t)steps, dev_log, log_cap);
}

// Solver parameters of the kinetic-energy solves: the ratio solves' unless
// energy_tol is set.
static DevParams energy_params(const Ctx* c) {
  DevParams d = c->dp;
  if (c->prm.energy_tol > 0.0) {
    d.rtol = c->prm.energy_tol;
    d.refine_tol = c->prm.energy_tol;
  }
  return d;
}

// k_energy over all walkers, writing walker w's energy to e_out[w * estride].
static void launch_energy_all(Ctx* c, double* e_out, int estride) {
  const DevParams d = energy_params(c);
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_energy<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, d,
                       c->d_all, 0, 1 << 30, e_out, estride, (double*)nullptr, (const long long*)nullptr, c->d_err);
  else
    hipLaunchKernelGGL(k_energy<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, d,
                       c->d_all, 0, 1 << 30, e_out, estride, (double*)nullptr, (const long long*)nullptr, c->d_err);
}

// Steps up to each sweep end run as ordinary persistent launches; the energy
// of every walker is then one more launch.  (Fusing both into one kernel
// doubles the kernel's code, past what the step code tolerates.)
vmc_status vmc_run_steps_energy(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap,
                                double* dev_energy, int32_t energy_cap) {
  Ctx* c = (Ctx*)ctx;
  if (!c || steps < 0 || energy_cap < 0 || (energy_cap > 0 && !dev_energy)) return VMC_EINVAL;
  if (steps == 0) return VMC_OK;
  if (!c->all_same_n) { c->err = "vmc_run_steps_energy needs walkers of equal n"; return VMC_EINVAL; }
  if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
  std::vector<WalkerState> hs(c->nw);
  HIPCHK(c, hipMemcpyAsync(hs.data(), c->dS, sizeof(WalkerState) * c->nw, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int w = 1; w < c->nw; ++w)
    if (hs[w].g != hs[0].g) { c->err = "vmc_run_steps_energy needs walkers at the same step"; return VMC_EINVAL; }
  const long long n = c->hw[0].n;
  long long g = hs[0].g;
  const long long cap = dev_log ? log_cap : 0;
  const size_t rec = sizeof(vmc_step_record);
  struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
  } tmp;
  if (cap > 0 && hipMalloc(&tmp.p, rec * (size_t)c->nw * (size_t)std::min<long long>(n, steps)) != hipSuccess) {
    c->err = "device allocation failed";
    return VMC_ENOMEM;
  }
  long long done = 0;
  int k = 0;
  while (done < steps) {
    const long long chunk = std::min<long long>(steps - done, n - g % n);
    launch_run(c, (int)chunk, cap > 0 ? (vmc_step_record*)tmp.p : nullptr, cap > 0 ? (long long)c->nw * chunk : 0);
    HIPCHK(c, hipGetLastError());
    if (cap > 0) {
      // walker w's records of this chunk go to dev_log[w * steps + done ...], within log_cap
      for (int w = 0; w < c->nw; ++w) {
        const long long first = (long long)w * steps + done;
        const long long cnt = std::min<long long>(chunk, cap - first);
        if (cnt <= 0) break;
        HIPCHK(c, hipMemcpyAsync(dev_log + first, (char*)tmp.p + rec * (size_t)w * chunk, rec * (size_t)cnt,
                                 hipMemcpyDeviceToDevice, c->stream));
      }
    }
    done += chunk;
    g += chunk;
    if (g % n == 0 && k < energy_cap) {
      launch_energy_all(c, dev_energy + k, energy_cap);
      HIPCHK(c, hipGetLastError());
    }
    if (g % n == 0) ++k;
  }
  return VMC_OK;
}

vmc_status vmc_kinetic_energy(void* ctx, const int32_t* walkers, int32_t count, int32_t p_begin, int32_t p_end,
                              double* energy_out, double* terms_out) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !energy_out || p_begin < 0 || p_end < p_begin) return VMC_EINVAL;
  if (!walkers) count = c->nw;
  int* dl = nullptr;
  vmc_status s = stage_list(c, walkers, count, &dl);
  if (s) return s;
  if (count == 0) return VMC_OK;
  s = check_sparse(c, walkers, count);
  if (s) return s;
  std::vector<long long> toff(count);
  long long tot = 0;
  for (int k = 0; k < count; ++k) {
    const int n = c->hw[walkers ? walkers[k] : k].n;
    const int hi = std::min(p_end, n), lo = std::min(p_begin, hi);
    toff[k] = tot;
    tot += hi - lo;
  }
  struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
  } be, bt, bo, br;
  if (hipMalloc(&be.p, sizeof(double) * count) != hipSuccess ||
      hipMalloc(&bo.p, sizeof(long long) * count) != hipSuccess ||
      hipMalloc(&br.p, sizeof(int) * count) != hipSuccess ||
      (terms_out && tot > 0 && hipMalloc(&bt.p, sizeof(double) * tot) != hipSuccess)) {
    c->err = "device allocation failed";
    return VMC_ENOMEM;
  }
  HIPCHK(c, hipMemcpyAsync(bo.p, toff.data(), sizeof(long long) * count, hipMemcpyHostToDevice, c->stream));
  double* dt = (double*)bt.p;
  const DevParams dpe = energy_params(c);
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_energy<VMC_PREC_FP64>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, dpe, dl,
                       p_begin, p_end, (double*)be.p, 1, dt, (const long long*)bo.p, (int*)br.p);
  else
    hipLaunchKernelGGL(k_energy<VMC_PREC_MIXED>, dim3(count), dim3(NT), c->lds, c->stream, c->dW, c->dS, dpe, dl,
                       p_begin, p_end, (double*)be.p, 1, dt, (const long long*)bo.p, (int*)br.p);
  HIPCHK(c, hipGetLastError());
  std::vector<int> err(count);
  HIPCHK(c, hipMemcpyAsync(energy_out, be.p, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(err.data(), br.p, sizeof(int) * count, hipMemcpyDeviceToHost, c->stream));
  if (dt) HIPCHK(c, hipMemcpyAsync(terms_out, dt, sizeof(double) * tot, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < count; ++k)
    if (err[k] == 2) { c->err = "kinetic energy requested with a pending move"; return VMC_ESTATE; }
  return walker_errors(c);
}

vmc_status vmc_sm_prepare(void* ctx, double tol) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !(tol > 0.0)) return VMC_EINVAL;
  if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
  if (!c->smB_own) {
    std::vector<double*> ptrs(c->nw);
    for (int w = 0; w < c->nw; ++w) {
      void* b = nullptr;
      const size_t bytes = sm_ld(c->hw[w].n) * (size_t)c->hw[w].n * 8;
      const hipError_t e = hipMalloc(&b, bytes);
      if (e != hipSuccess) {
        for (void* q : c->sm_bufs) (void)hipFree(q);
        c->sm_bufs.clear();
        c->err = "walker " + std::to_string(w) + ": allocation of the " + std::to_string(bytes) +
                 "-byte inverse failed: " + hipGetErrorString(e);
        return VMC_ENOMEM;
      }
      c->sm_bufs.push_back(b);
      ptrs[w] = (double*)b;
    }
    // the table and the flags are set together, so a failed call leaves neither
    void* tab = nullptr;
    void* flags = nullptr;
    if (hipMalloc(&tab, sizeof(double*) * c->nw) != hipSuccess || hipMalloc(&flags, sizeof(int) * c->nw) != hipSuccess) {
      if (tab) (void)hipFree(tab);
      for (void* q : c->sm_bufs) (void)hipFree(q);
      c->sm_bufs.clear();
      c->err = "device allocation failed";
      return VMC_ENOMEM;
    }
    c->smB_own = (double**)tab;
    c->nonconv_own = (int*)flags;
    HIPCHK(c, hipMemcpyAsync(c->smB_own, ptrs.data(), sizeof(double*) * c->nw, hipMemcpyHostToDevice, c->stream));
  }
  sm_static_release(c);
  c->d_smB = c->smB_own;
  c->d_nonconv = c->nonconv_own;
  c->sm_static = false;
  c->sm_current = false;
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_inverse_cols<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                       (double* const*)c->d_smB, 0, c->maxn, tol, c->d_nonconv);
  else
    hipLaunchKernelGGL(k_inverse_cols<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                       (double* const*)c->d_smB, 0, c->maxn, tol, c->d_nonconv);
  HIPCHK(c, hipGetLastError());
  std::vector<int> bad(c->nw);
  HIPCHK(c, hipMemcpyAsync(bad.data(), c->d_nonconv, sizeof(int) * c->nw, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int w = 0; w < c->nw; ++w) {
    if (bad[w] < 0) { c->err = "walker " + std::to_string(w) + ": pending move or error"; return VMC_ESTATE; }
    if (bad[w] > 0) {
      c->err = "walker " + std::to_string(w) + ": " + std::to_string(bad[w]) + " inverse columns missed the tolerance";
      return VMC_ENOCONV;
    }
  }
  const vmc_status st = walker_errors(c);
  c->sm_current = (st == VMC_OK);
  return st;
}

vmc_status vmc_sm_prepare_static(void* ctx, double tol) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !(tol > 0.0)) return VMC_EINVAL;
  if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= SM_STATIC_DEVICES) {
    c->err = "vmc_sm_prepare_static: device index beyond the static scratch table";
    return VMC_EINVAL;
  }
  const size_t need = sm_static_offset(c, c->nw);
  if (need > SM_STATIC_BYTES) {
    c->err = "vmc_sm_prepare_static: the inverses need " + std::to_string(need) + " bytes, the static scratch holds " +
             std::to_string(SM_STATIC_BYTES);
    return VMC_EINVAL;
  }
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (char*)ptr;
  }
  char* base = g_scratch_ptr[dev];
  int* flags = (int*)(base + align_up((size_t)c->nw * sizeof(double*), 256));
  c->sm_current = false;
  // this context takes the scratch: another one that held it can no longer
  // run on its inverses (vmc_sm_run_steps and vmc_sm_get_inverse refuse)
  g_scratch_owner[dev] = c;
  c->sm_dev = dev;
  c->sm_static = true;
  c->d_smB = (double**)base;
  c->d_nonconv = flags;
  hipLaunchKernelGGL(k_sm_table, dim3(1), dim3(64), 0, c->stream, c->dW, c->nw, base);
  HIPCHK(c, hipGetLastError());
  if (c->dp.precision == VMC_PREC_FP64)
    hipLaunchKernelGGL(k_inverse_cols<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                       (double* const*)c->d_smB, 0, c->maxn, tol, c->d_nonconv);
  else
    hipLaunchKernelGGL(k_inverse_cols<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp,
                       (double* const*)c->d_smB, 0, c->maxn, tol, c->d_nonconv);
  HIPCHK(c, hipGetLastError());
  int bad[256];
  for (int w0 = 0; w0 < c->nw; w0 += 256) {
    const int cnt = std::min(256, c->nw - w0);
    HIPCHK(c, hipMemcpyAsync(bad, flags + w0, sizeof(int) * cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < cnt; ++k) {
      if (bad[k] < 0) { c->err = "walker " + std::to_string(w0 + k) + ": pending move or error"; return VMC_ESTATE; }
      if (bad[k] > 0) {
        c->err = "walker " + std::to_string(w0 + k) + ": " + std::to_string(bad[k]) +
                 " inverse columns missed the tolerance";
        return VMC_ENOCONV;
      }
    }
  }
  const vmc_status st = walker_errors(c);
  c->sm_current = (st == VMC_OK);
  return st;
}

vmc_status vmc_sm_run_steps(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap) {
  Ctx* c = (Ctx*)ctx;
  if (!c || steps < 0) return VMC_EINVAL;
  if (!c->d_smB) { c->err = "vmc_sm_run_steps before vmc_sm_prepare"; return VMC_ESTATE; }
  if (c->sm_static && !sm_static_owned(c)) {
    c->err = "the static inverses now belong to another context (vmc_sm_prepare_static)";
    return VMC_ESTATE;
  }
  if (!c->sm_current) {
    c->err = "the stored inverses are stale: the walkers have changed since vmc_sm_prepare";
    return VMC_ESTATE;
  }
  if (steps == 0) return VMC_OK;
  const size_t lds = sm_lds(c->maxn, c->max_cap).total;
  (void)hipFuncSetAttribute((const void*)k_sm_run, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_sm_run, dim3(c->nw), dim3(NT), lds, c->stream, c->dW, c->dS, c->dp, (double* const*)c->d_smB,
                     steps, dev_log, (long long)(dev_log ? log_cap : 0));
  HIPCHK(c, hipGetLastError());
  c->rows_stale.assign(c->nw, 1);
  c->fac_stale.assign(c->nw, 1);
  return VMC_OK;
}

vmc_status vmc_sm_get_inverse(void* ctx, int32_t walker, double* host_out) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !host_out || walker < 0 || walker >= c->nw) return VMC_EINVAL;
  if (!c->d_smB) { c->err = "no stored inverse (call vmc_sm_prepare)"; return VMC_ESTATE; }
  const int n = c->hw[walker].n;
  const void* src = c->sm_static ? sm_static_inverse(c, walker) : (const void*)c->sm_bufs[walker];
  if (!src) { c->err = "the static inverses now belong to another context (vmc_sm_prepare_static)"; return VMC_ESTATE; }
  HIPCHK(c, hipMemcpy2DAsync(host_out, (size_t)n * 8, src, sm_ld(n) * 8, (size_t)n * 8, n,
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return VMC_OK;
}

// Cost-balance autotuner (Section 3.2: a new ILUTP once applying the stored
// updates has cost as much as computing it), plus the longest-first launch
// order of the walkers.  Per walker size n the thresholds are medians, so a
// cache line per n reproduces them.
vmc_status vmc_autotune(void* ctx, const char* cache_path, int32_t trial_steps, vmc_tune_info* info) {
  Ctx* c = (Ctx*)ctx;
  if (!c || trial_steps < 0) return VMC_EINVAL;
  const int nw = c->nw;
  vmc_tune_info ti;
  std::memset(&ti, 0, sizeof(ti));
  std::map<int, double> cached;
  if (cache_path) {
    std::ifstream f(cache_path);
    int n;
    double v;
    while (f >> n >> v)
      if (n > 0 && v > 0.0) cached[n] = v;
  }
  bool have_all = !cached.empty();
  for (int w = 0; w < nw && have_all; ++w) have_all = cached.count(c->hw[w].n) > 0;
  std::vector<double> cost(nw, 0.0), step_ticks(nw, 0.0);
  if (have_all) {
    for (int w = 0; w < nw; ++w) {
      cost[w] = cached[c->hw[w].n];
      step_ticks[w] = (double)c->hw[w].n * c->hw[w].W;  // model: bigger rows, longer steps
    }
    ti.from_cache = 1;
  } else {
    if (trial_steps < 1) {
      c->err = "vmc_autotune: no cached thresholds for these walker sizes and trial_steps < 1";
      return VMC_EINVAL;
    }
    std::vector<vmc_stats> s0(nw), s1(nw), s2(nw);
    vmc_status st = vmc_get_stats(ctx, s0.data());
    if (st) return st;
    st = vmc_ilutp(ctx, nullptr, 0, 0);
    if (st) return st;
    st = vmc_get_stats(ctx, s1.data());
    if (st) return st;
    st = vmc_run_steps(ctx, trial_steps, nullptr, 0);
    if (st) return st;
    st = vmc_sync(ctx);
    if (st) return st;
    st = vmc_get_stats(ctx, s2.data());
    if (st) return st;
    // per walker size: median ILUTP ticks and median ticks per applied entry
    std::map<int, std::vector<double>> ilu_by_n, ent_by_n;
    for (int w = 0; w < nw; ++w) {
      const int n = c->hw[w].n;
      ilu_by_n[n].push_back((double)(s1[w].phase_ticks[PH_REFACTOR] - s0[w].phase_ticks[PH_REFACTOR]));
      const double ent = s2[w].update_entries - s1[w].update_entries;
      const double upd = (double)(s2[w].phase_ticks[PH_UPDATES] - s1[w].phase_ticks[PH_UPDATES]);
      if (ent > 0.0) ent_by_n[n].push_back(upd / ent);
      step_ticks[w] = (double)(s2[w].phase_ticks[PH_STEP] - s1[w].phase_ticks[PH_STEP]) / trial_steps;
    }
    auto median = [](std::vector<double> v) {
      std::sort(v.begin(), v.end());
      return v.empty() ? 0.0 : v[v.size() / 2];
    };
    std::map<int, double> per_n;
    std::vector<double> all_ent;
    for (auto& kv : ent_by_n) all_ent.insert(all_ent.end(), kv.second.begin(), kv.second.end());
    const double ent_all = median(all_ent);
    double ilu_sum = 0.0;
    for (auto& kv : ilu_by_n) {
      const double ilu = median(kv.second);
      const double te = ent_by_n.count(kv.first) ? median(ent_by_n[kv.first]) : ent_all;
      per_n[kv.first] = (ilu > 0.0 && te > 0.0) ? ilu / te : 0.0;
      for (double x : kv.second) ilu_sum += x;
    }
    for (int w = 0; w < nw; ++w) cost[w] = per_n[c->hw[w].n];
    ti.ilutp_us_mean = ilu_sum / nw / 100.0;          // 100 MHz wall clock
    ti.update_ns_per_entry = ent_all * 10.0;
    ti.trial_steps = trial_steps;
    if (cache_path) {
      std::ofstream f(cache_path);
      f.precision(17);
      for (auto& kv : per_n)
        if (kv.second > 0.0) f << kv.first << " " << kv.second << "\n";
    }
  }
  // thresholds into the walker states
  std::vector<WalkerState> hs(nw);
  HIPCHK(c, hipMemcpyAsync(hs.data(), c->dS, sizeof(WalkerState) * nw, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double csum = 0.0;
  for (int w = 0; w < nw; ++w) {
    hs[w].refactor_cost = cost[w];
    csum += cost[w];
  }
  HIPCHK(c, hipMemcpyAsync(c->dS, hs.data(), sizeof(WalkerState) * nw, hipMemcpyHostToDevice, c->stream));
  // longest step first, so the walkers that finish last start first
  std::vector<int> order(nw);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return step_ticks[a] > step_ticks[b]; });
  HIPCHK(c, hipMemcpyAsync(c->d_order, order.data(), sizeof(int) * nw, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->use_order = nw > 1;
  ti.refactor_cost_mean = csum / nw;
  if (!ti.from_cache) {
    double mn = 1e300, mx = 0.0;
    for (double t : step_ticks) {
      mn = std::min(mn, t);
      mx = std::max(mx, t);
    }
    ti.step_us_min = mn / 100.0;
    ti.step_us_max = mx / 100.0;
  }
  if (info) *info = ti;
  return VMC_OK;
}

vmc_status vmc_phase_bench(void* ctx, int32_t phase, int32_t reps) {
  Ctx* c = (Ctx*)ctx;
  if (!c || phase < 0 || phase > 5 || reps < 0) return VMC_EINVAL;
  if (vmc_status s = check_sparse(c, nullptr, c->nw)) return s;
  c->sm_current = false;
  if (c->dp.precision == VMC_PREC_FP64) {
    (void)hipFuncSetAttribute((const void*)k_phase<VMC_PREC_FP64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    hipLaunchKernelGGL(k_phase<VMC_PREC_FP64>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, phase, reps);
  } else {
    (void)hipFuncSetAttribute((const void*)k_phase<VMC_PREC_MIXED>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds);
    hipLaunchKernelGGL(k_phase<VMC_PREC_MIXED>, dim3(c->nw), dim3(NT), c->lds, c->stream, c->dW, c->dS, c->dp, phase, reps);
  }
  HIPCHK(c, hipGetLastError());
  return VMC_OK;
}

vmc_status vmc_sync(void* ctx) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return VMC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const vmc_status ce = call_errors(c);
  const vmc_status we = walker_errors(c);
  return we != VMC_OK ? we : ce;
}

vmc_status vmc_get_dims(void* ctx, int32_t walker, int32_t* n, int32_t* row_cap, int32_t* fact_cap) {
  Ctx* c = (Ctx*)ctx;
  if (!c || walker < 0 || walker >= c->nw) return VMC_EINVAL;
  if (n) *n = c->hw[walker].n;
  if (row_cap) *row_cap = c->hw[walker].W;
  if (fact_cap) *fact_cap = c->hw[walker].F;
  return VMC_OK;
}

vmc_status vmc_get_state(void* ctx, int32_t walker, const vmc_state_view* v) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !v || walker < 0 || walker >= c->nw) return VMC_EINVAL;
  const Walker& W = c->hw[walker];
  const size_t n = W.n;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!dst) return hipSuccess;
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  };
  HIPCHK(c, cp(v->pos, (const void*)W.pos, n * 3 * 8));
  HIPCHK(c, cp(v->row_particle, (const void*)W.rowperm, n * 4));
  HIPCHK(c, cp(v->col_site, (const void*)W.colsite, n * 4));
  HIPCHK(c, cp(v->reorder_row, (const void*)W.reo_row, n * 4));
  HIPCHK(c, cp(v->reorder_col, (const void*)W.reo_col, n * 4));
  HIPCHK(c, cp(v->a_len, (const void*)W.a_len, n * 4));
  {
    // A is stored in slices of 64 rows (aidx) with 16-bit column positions;
    // exported row-major, n x W, columns as int32
    const size_t na = a_rows_padded(n);
    if (v->a_col) {
      std::vector<unsigned short> tmp(na * (size_t)W.W);
      HIPCHK(c, cp(tmp.data(), (const void*)W.a_col, na * W.W * 2));
      for (int i = 0; i < n; ++i)
        for (int e = 0; e < W.W; ++e) v->a_col[(size_t)i * W.W + e] = tmp[aidx(W.W, i, e)];
    }
    if (v->a_val) {
      std::vector<double> tmp(na * (size_t)W.W);
      HIPCHK(c, cp(tmp.data(), (const void*)W.a_val, na * W.W * 8));
      for (int i = 0; i < n; ++i)
        for (int e = 0; e < W.W; ++e) v->a_val[(size_t)i * W.W + e] = tmp[aidx(W.W, i, e)];
    }
  }
  HIPCHK(c, cp(v->l_len, (const void*)W.l_len, n * 4));
  HIPCHK(c, cp(v->l_col, (const void*)W.l_col, n * W.F * 4));
  HIPCHK(c, cp(v->l_val, (const void*)W.l_val, n * W.F * 8));
  HIPCHK(c, cp(v->u_len, (const void*)W.u_len, n * 4));
  HIPCHK(c, cp(v->u_col, (const void*)W.u_col, n * W.F * 4));
  HIPCHK(c, cp(v->u_val, (const void*)W.u_val, n * W.F * 8));
  HIPCHK(c, cp(v->u_diag, (const void*)W.u_diag, n * 8));
  HIPCHK(c, cp(v->ilu_perm, (const void*)W.ilu_q, n * 4));
  if (v->step || v->n_updates) {
    WalkerState s;
    HIPCHK(c, hipMemcpy(&s, c->dS + walker, sizeof(s), hipMemcpyDeviceToHost));
    if (v->step) *v->step = s.g;
    if (v->n_updates) *v->n_updates = s.m;
  }
  return VMC_OK;
}

vmc_status vmc_get_stats(void* ctx, vmc_stats* out) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !out) return VMC_EINVAL;
  std::vector<WalkerState> hs(c->nw);
  HIPCHK(c, hipMemcpyAsync(hs.data(), c->dS, sizeof(WalkerState) * c->nw, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int w = 0; w < c->nw; ++w) {
    const WalkerState& s = hs[w];
    vmc_stats& o = out[w];
    std::memset(&o, 0, sizeof(o));
    o.steps = s.st_steps;
    o.accepted = s.st_acc;
    o.solves = s.st_solves;
    o.iters = s.st_iters;
    o.reorders = s.st_reorders;
    o.refactors = s.st_refactors;
    o.nonconverged = s.st_nonconv;
    o.inner_solves = s.st_inner;
    o.refine_passes = s.st_refine;
    o.update_sum = s.st_msum;
    for (int k = 0; k < PH_COUNT && k < 12; ++k) o.phase_ticks[k] = (int64_t)s.ph[k];
    o.max_N = s.st_maxN;
    o.sum_N = s.st_sumN;
    o.update_entries = s.st_upd_entries;
    o.refactor_cost = s.refactor_cost;
    o.ilu_retries = (int32_t)s.ilu_retries;
    o.status = (s.status & WST_CAPACITY)   ? VMC_ECAPACITY
               : (s.status & WST_SINGULAR) ? VMC_ESINGULAR
               : (s.status & WST_NOCONV)   ? VMC_ENOCONV
                                           : VMC_OK;
  }
  return VMC_OK;
}

const char* vmc_last_error(void* ctx) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

vmc_status vmc_destroy(void* ctx) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return VMC_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  for (void* a : c->arenas) (void)hipFree(a);
  (void)hipFree(c->dW);
  (void)hipFree(c->dS);
  (void)hipFree(c->d_list);
  (void)hipFree(c->d_all);
  (void)hipFree(c->d_part);
  (void)hipFree(c->d_pos);
  (void)hipFree(c->d_rec);
  (void)hipFree(c->d_dec);
  (void)hipFree(c->d_acc);
  (void)hipFree(c->d_err);
  (void)hipFree(c->d_order);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* b : c->sm_bufs) (void)hipFree(b);
  if (c->smB_own) (void)hipFree(c->smB_own);
  if (c->nonconv_own) (void)hipFree(c->nonconv_own);
  sm_static_release(c);
  delete c;
  return VMC_OK;
}

}  // extern "C"
