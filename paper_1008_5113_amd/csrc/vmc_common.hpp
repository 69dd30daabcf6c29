// Device helpers: LDS layout, reductions, Philox, geometry and row evaluation.
#pragma once

#include "vmc_internal.hpp"

namespace vmc {

// Phase-level device functions (inlined into the fused kernels).
#define VMC_PHASE __device__ __attribute__((always_inline)) inline

// ---------------------------------------------------------------------------
// Shared-memory layout.  Region A is a union of the phase-private buffers
// (Krylov/triangular-solve vectors, the ILUTP work row, the reorder
// permutations); region B holds reduction slots and GMRES scalars.
// ---------------------------------------------------------------------------
struct LdsLayout {
  size_t regionA, red, hb, cs, sn, gg, rp, yb, ux, gb, cb, sc, ic, stmp, total;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ILUTP: rows are factored concurrently, one wave each, every wave with a
// hashed sparse work row, a candidate table and its multipliers.  The
// capacities are runtime values (DevParams::ilu, ilu_fast).  The full
// configuration (ILU_R rows, the ILU_DEF_* tables) suits matrices whose rows
// stay within a few hundred entries during elimination; the fast one keeps
// twice the rows in flight in about the same LDS with tables that hold the
// rows of the usual workloads, and hands the rows around one that overflows
// them to the full one.
constexpr int ILU_R = 4;
constexpr int ILU_DEF_HS = 1024;  // hash slots per wave (power of two)
constexpr int ILU_DEF_NZ = 512;   // work-row entries per wave
constexpr int ILU_DEF_C = 192;    // elimination candidates per row
constexpr int ILU_DEF_L = 160;    // multipliers per row before the fill limit
constexpr int ILU_FAST_R = 8;
constexpr int ILU_FAST_HS = 512;
constexpr int ILU_FAST_NZ = 256;
constexpr int ILU_FAST_C = 128;
constexpr int ILU_FAST_L = 96;
constexpr int ILU_FALLBACK_ROWS = 64;  // rows the full configuration takes after an overflow

__host__ __device__ inline size_t ilu_wave_bytes(int hs, int nz, int c, int l) {
  return align_up((size_t)hs * 4, 16) + align_up((size_t)nz * 2, 16) + (size_t)nz * 8 +
         align_up((size_t)c * 2, 16) * 3 + (size_t)c * 8 + align_up((size_t)l * 2, 16) + (size_t)l * 8;
}

__host__ __device__ inline size_t ilu_wave_bytes(const IluCfg& C) {
  return ilu_wave_bytes(C.hs, C.nz, C.c, C.l);
}

__host__ __device__ inline size_t ilutp_lds_bytes(int n, const DevParams& P) {
  size_t b = 0;
  b += align_up((size_t)n * 2, 16);  // pinv
  b += align_up((size_t)n * 2, 16);  // q
  const size_t full = (size_t)P.ilu.r * ilu_wave_bytes(P.ilu);
  const size_t fast = (size_t)P.ilu_fast.r * ilu_wave_bytes(P.ilu_fast);
  const size_t waves = full > fast ? full : fast;
  const size_t tmp = (size_t)n * 4;  // column relabelling after the factorisation
  b += waves > tmp ? waves : tmp;
  return b;
}

// Region A (phase union): the solve phase holds the triangular-solve vector,
// the in-block coefficient tile, the GMRES scalars and the update
// coefficients; the ILUTP and reorder phases reuse the same bytes.  Region B
// (reduction slots and broadcast scalars) is live in every phase.
__host__ __device__ inline LdsLayout lds_layout(int n, int ktb, const DevParams& P) {
  const int maxit = P.maxit, mmax = P.m_max;
  LdsLayout L;
  size_t o = align_up((size_t)n, 4) * ktb + align_up((size_t)DTILE * ktb, 16);  // xs, D
  L.hb = o; o += (size_t)(maxit + 2) * 8;
  L.cs = o; o += (size_t)(maxit + 1) * 8;
  L.sn = o; o += (size_t)(maxit + 1) * 8;
  L.gg = o; o += (size_t)(maxit + 2) * 8;
  L.rp = o; o += (size_t)maxit * (maxit + 1) / 2 * 8 + 8;
  L.yb = o; o += (size_t)(maxit + 1) * 8;
  L.ux = o; o += (size_t)(maxit + 1) * 8;
  L.gb = o; o += (size_t)(mmax + 1) * 8;
  L.cb = o; o += (size_t)(mmax + 1) * 8;
  size_t a = o;
  const size_t ilu = ilutp_lds_bytes(n, P);
  const size_t reo = align_up((size_t)n * 2, 16) * 2;
  if (ilu > a) a = ilu;
  if (reo > a) a = reo;
  o = align_up(a, 16);
  L.regionA = 0;
  // reduction slots: the Gram-Schmidt dot products (NWAVE per basis vector,
  // plus the stability term) and, in the factor packing, one int per thread
  const size_t red_dots = (size_t)NWAVE * (maxit + 2) * 8;
  const size_t red_scan = (size_t)NT * 4;
  L.red = o; o += red_dots > red_scan ? red_dots : red_scan;
  L.sc = o; o += 32 * 8;
  L.ic = o; o += 32 * 4;
  L.stmp = o; o += BLK * 8;
  L.total = align_up(o, 16);
  return L;
}

struct Smem {
  char* A;
  double* red;
  double* hb;
  double* cs;
  double* sn;
  double* gg;
  double* rp;
  double* yb;
  double* ux;
  double* gb;
  double* cb;
  double* sc;
  int* ic;
  void* stmp;
  unsigned long long* ph;
  unsigned long long* ilu_retries;  // the walker's counter of ILUTP second attempts (or null)
};

__device__ inline Smem make_smem(char* base, const LdsLayout& L) {
  Smem s;
  s.A = base + L.regionA;
  s.red = (double*)(base + L.red);
  s.hb = (double*)(base + L.hb);
  s.cs = (double*)(base + L.cs);
  s.sn = (double*)(base + L.sn);
  s.gg = (double*)(base + L.gg);
  s.rp = (double*)(base + L.rp);
  s.yb = (double*)(base + L.yb);
  s.ux = (double*)(base + L.ux);
  s.gb = (double*)(base + L.gb);
  s.cb = (double*)(base + L.cb);
  s.sc = (double*)(base + L.sc);
  s.ic = (int*)(base + L.ic);
  s.stmp = (void*)(base + L.stmp);
  s.ph = nullptr;
  s.ilu_retries = nullptr;
  return s;
}

// Phase timer: thread 0 adds the wall-clock ticks between two points.
struct PhaseClock {
  unsigned long long t;
  __device__ inline void start() { t = wall_clock64(); }
  __device__ inline void stop(const Smem& S, int ph) {
    if (S.ph && threadIdx.x == 0) {
      const unsigned long long now = wall_clock64();
      S.ph[ph] += now - t;
      t = now;
    }
  }
};

// ---------------------------------------------------------------------------
// Reductions (deterministic: fixed butterfly order, identical in every lane)
// ---------------------------------------------------------------------------
// Thread index as a value the optimizer cannot see through.  Index arithmetic
// derived from it is then recomputed inside each phase instead of being hoisted
// out of the step and Krylov loops and held in registers across every phase.
__device__ inline int vmc_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
__device__ inline int lane_id() { return vmc_tid() & 63; }
__device__ inline int wave_id() { return vmc_tid() >> 6; }

// DPP lane moves (VALU, no LDS traffic).  quad_perm xor 1 / xor 2 and the
// row mirrors stay inside a 16-lane row; row_shl:4 reads lane+4 of the row.
constexpr int DPP_QXOR1 = 0xB1;       // quad_perm:[1,0,3,2]
constexpr int DPP_QXOR2 = 0x4E;       // quad_perm:[2,3,0,1]
constexpr int DPP_HMIRROR = 0x141;    // row_half_mirror
constexpr int DPP_MIRROR = 0x140;     // row_mirror
constexpr int DPP_SHL4 = 0x104;       // row_shl:4

template <int CTRL>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ inline double dpp_t(double v) { return dpp_d<CTRL>(v); }
template <int CTRL> __device__ inline float dpp_t(float v) { return dpp_f<CTRL>(v); }
template <int CTRL> __device__ inline int dpp_t(int v) { return dpp_i<CTRL>(v); }

__device__ inline double readlane_d(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}
__device__ inline float readlane_f(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ inline int readlane_i(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ inline double readlane_t(double v, int k) { return readlane_d(v, k); }
__device__ inline float readlane_t(float v, int k) { return readlane_f(v, k); }
__device__ inline int readlane_t(int v, int k) { return readlane_i(v, k); }

// Marks a point where every lane's preceding memory reads must come before
// any lane's following writes (one lane updating what all lanes just read).
// A wave executes in lockstep, so on the device this only keeps the compiler
// from moving memory operations across it.
__device__ inline void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Sum over the 64 lanes; every lane gets the same value (fixed order).
template <typename T>
__device__ inline T wave_sum_t(T v) {
  v += dpp_t<DPP_QXOR1>(v);
  v += dpp_t<DPP_QXOR2>(v);
  v += dpp_t<DPP_HMIRROR>(v);
  v += dpp_t<DPP_MIRROR>(v);
  return (readlane_t(v, 0) + readlane_t(v, 16)) + (readlane_t(v, 32) + readlane_t(v, 48));
}
__device__ inline double wave_sum(double v) { return wave_sum_t(v); }
__device__ inline float wave_sumf(float v) { return wave_sum_t(v); }
__device__ inline int wave_sumi(int v) { return wave_sum_t(v); }
__device__ inline int wave_mini(int v) {
  v = min(v, dpp_i<DPP_QXOR1>(v));
  v = min(v, dpp_i<DPP_QXOR2>(v));
  v = min(v, dpp_i<DPP_HMIRROR>(v));
  v = min(v, dpp_i<DPP_MIRROR>(v));
  return min(min(readlane_i(v, 0), readlane_i(v, 16)), min(readlane_i(v, 32), readlane_i(v, 48)));
}
__device__ inline double wave_maxd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// Sum over groups of 8 consecutive lanes; the total is valid in lanes 8k.
template <typename T>
__device__ inline T sum8(T v) {
  v += dpp_t<DPP_QXOR1>(v);
  v += dpp_t<DPP_QXOR2>(v);
  v += dpp_t<DPP_SHL4>(v);
  return v;
}
// Sum over groups of 4 consecutive lanes; valid in every lane of the group.
template <typename T>
__device__ inline T sum4(T v) {
  v += dpp_t<DPP_QXOR1>(v);
  v += dpp_t<DPP_QXOR2>(v);
  return v;
}

// Sum over the workgroup; every thread gets the same value.
__device__ inline double wg_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) s += red[w];
  return s;
}

// Lexicographic (value, index) minimum over the workgroup.
__device__ inline void wg_argmin(double& v, int& idx, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double ov = __shfl_xor(v, o, 64);
    int oi = __shfl_xor(idx, o, 64);
    if (ov < v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  __syncthreads();
  if (lane_id() == 0) { red[wave_id()] = v; ((int*)(red + NWAVE))[wave_id()] = idx; }
  __syncthreads();
  v = red[0];
  idx = ((int*)(red + NWAVE))[0];
  for (int w = 1; w < NWAVE; ++w) {
    double ov = red[w];
    int oi = ((int*)(red + NWAVE))[w];
    if (ov < v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the step draws.
// Key (seed, 0), counter (g, 0, 0, 0); outputs 0..2 move the particle, output
// 3 is the acceptance draw.
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(unsigned long long c[4], unsigned long long k0,
                                     unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    unsigned long long hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    unsigned long long hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    unsigned long long n0 = hi1 ^ c[1] ^ k0;
    unsigned long long n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// (top 52 bits + 1/2) * 2^-52: exact in binary64, strictly inside (0,1).
__device__ inline double u01(unsigned long long x) {
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

__device__ inline void step_draws(unsigned long long seed, long long g, double u[4]) {
  unsigned long long c[4] = {(unsigned long long)g, 0ull, 0ull, 0ull};
  philox4x64_10(c, seed, 0ull);
  for (int k = 0; k < 4; ++k) u[k] = u01(c[k]);
}

// ---------------------------------------------------------------------------
// Geometry.  Contraction into FMA is disabled so the sparsity pattern and the
// proposal are the same bits as any IEEE evaluation of the same expressions.
// ---------------------------------------------------------------------------
__device__ inline double min_image(double d, double L) {
#pragma clang fp contract(off)
  double half = 0.5 * L;
  if (d > half) d = d - L;
  else if (d < -half) d = d + L;
  return d;
}

__device__ inline double propose_axis(double r, double u, double h, double L) {
#pragma clang fp contract(off)
  double t = 2.0 * u - 1.0;
  double dx = h * t;
  double x = r + dx;
  if (x >= L) x = x - L;
  else if (x < 0.0) x = x + L;
  return x;
}

struct RowHit {
  double d2, dx;
};

__device__ inline double dist2_xyz(double rx, double ry, double rz, const double* Z, const double* box,
                                   double* dx_out) {
#pragma clang fp contract(off)
  double dx = min_image(rx - Z[0], box[0]);
  double dy = min_image(ry - Z[1], box[1]);
  double dz = min_image(rz - Z[2], box[2]);
  double xx = dx * dx;
  double yy = dy * dy;
  double zz = dz * dz;
  double s = xx + yy;
  *dx_out = dx;
  return s + zz;
}

__device__ inline double orbital_value(const Walker& W, double d2, double dx, double sig) {
#pragma clang fp contract(off)
  double den = 2.0 * sig * sig;
  double v = exp(-d2 / den);
  if (W.kind == VMC_ORB_GAUSS_PX) {
    double den2 = 2.0 * W.p_sigma * W.p_sigma;
    v = v + W.p_scale * dx * exp(-d2 / den2);
  }
  return v;
}

// Candidate lattice range along one axis: all nominal sites whose unwrapped
// coordinate lies within cutoff + margin of x, widened by one; the whole axis
// when that covers it.
__device__ inline void axis_range(double x, double R, double a, int L, int& lo, int& cnt) {
  int l = (int)floor((x - R) / a);
  int h = (int)floor((x + R) / a) + 1;
  cnt = h - l + 1;
  lo = l;
  if (cnt >= L) { lo = 0; cnt = L; }
}

__device__ inline int wrap_index(int i, int L) {
  int r = i % L;
  return r < 0 ? r + L : r;
}

// -(1/2) lap phi_j at a point where phi_j is given by orbital_value: with
// c = 1/sigma^2, -(1/2) lap exp(-c|d|^2/2) = (3c - c^2|d|^2)/2 * exp(-c|d|^2/2);
// the p-like term s d_x exp(-e|d|^2/2) gives s d_x (5e - e^2|d|^2)/2 * exp(..).
// Its ratio with Psi is the kinetic-energy term of eq. (energyEq).
__device__ inline double orbital_kinetic(const Walker& W, double d2, double dx, double sig) {
  const double c = 1.0 / (sig * sig);
  double v = 0.5 * (3.0 * c - c * c * d2) * exp(-0.5 * c * d2);
  if (W.kind == VMC_ORB_GAUSS_PX) {
    const double e = 1.0 / (W.p_sigma * W.p_sigma);
    v += W.p_scale * dx * 0.5 * (5.0 * e - e * e * d2) * exp(-0.5 * e * d2);
  }
  return v;
}

// Evaluate one Slater row phi_j(r) (KIN = 0) or its kinetic row
// -(1/2) lap phi_j(r) (KIN = 1) over the sites within the cutoff (one wave).
// Candidates: every site of the cells whose corner lies within
// cutoff + margin of r, the range stretched down by the largest in-cell site
// offset.  Entries are written in candidate order to out_col/out_val as
// column positions cmap[site] (site ids when cmap is null), entry o at
// out[o * stride].  Returns the entry count (may exceed cap; entries past cap
// are not written).
template <typename CT, int KIN = 0>
__device__ inline int wave_row(const Walker& W, double rx, double ry, double rz, const int* cmap,
                               CT* out_col, double* out_val, float* out_val32, int cap, int stride = 1) {
  const int lane = lane_id();
  const double R = W.cutoff + W.margin;
  const int nb = W.nb;
  int lox, cx, loy, cy, loz, cz;
  axis_range(rx - W.bmax[0], R, W.a, W.lat[0], lox, cx);
  axis_range(ry - W.bmax[1], R, W.a, W.lat[1], loy, cy);
  axis_range(rz - W.bmax[2], R, W.a, W.lat[2], loz, cz);
  const int total = cx * cy * cz * nb;
  const double rc2 = W.cutoff * W.cutoff;
  int count = 0;
  for (int t0 = 0; t0 < total; t0 += 64) {
    int t = t0 + lane;
    bool hit = false;
    int site = 0;
    double val = 0.0;
    if (t < total) {
      const int b = t % nb;
      const int cell = t / nb;
      int tx = cell % cx;
      int ty = (cell / cx) % cy;
      int tz = cell / (cx * cy);
      int ix = wrap_index(lox + tx, W.lat[0]);
      int iy = wrap_index(loy + ty, W.lat[1]);
      int iz = wrap_index(loz + tz, W.lat[2]);
      site = b + nb * (ix + W.lat[0] * (iy + W.lat[1] * iz));
      double dx;
      double d2 = dist2_xyz(rx, ry, rz, W.sites + 3 * (size_t)site, W.box, &dx);
      if (d2 <= rc2) {
        hit = true;
        val = KIN ? orbital_kinetic(W, d2, dx, W.sigma[site]) : orbital_value(W, d2, dx, W.sigma[site]);
      }
    }
    unsigned long long mask = __ballot(hit);
    int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (hit) {
      int o = count + before;
      if (o < cap) {
        const size_t so = (size_t)o * stride;
        out_col[so] = (CT)(cmap ? cmap[site] : site);
        out_val[so] = val;
        if (out_val32) out_val32[so] = (float)val;
      }
    }
    count += __popcll(mask);
  }
  return count;
}

}  // namespace vmc
