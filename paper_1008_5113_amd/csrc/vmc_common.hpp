// Device helpers: LDS layout, reductions, Philox, geometry and row evaluation.
#pragma once

#include "vmc_internal.hpp"

namespace vmc {

// ---------------------------------------------------------------------------
// Shared-memory layout.  Region A is a union of the phase-private buffers
// (Krylov/triangular-solve vectors, the ILUTP work row, the reorder
// permutations); region B holds reduction slots and GMRES scalars.
// ---------------------------------------------------------------------------
struct LdsLayout {
  size_t regionA, red, hb, cs, sn, gg, rp, yb, gb, cb, sc, ic, stmp, total;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline size_t ilutp_lds_bytes(int n) {
  size_t b = 0;
  b += align_up((size_t)n * 8, 16);        // wv
  b += align_up((size_t)n, 16);            // present flags
  b += align_up((size_t)n * 2, 16);        // pinv
  b += align_up((size_t)n * 2, 16);        // q
  b += align_up((size_t)NZMAX * 2, 16);    // work-row column list
  b += align_up((size_t)LMAX * 2, 16);     // multiplier positions
  b += align_up((size_t)LMAX * 8, 16);     // multiplier values
  return b;
}

__host__ __device__ inline LdsLayout lds_layout(int n, int ktb, int maxit, int mmax) {
  LdsLayout L;
  size_t solve = align_up((size_t)n, 4) * ktb + (size_t)BLK * BLK * ktb;
  size_t ilu = ilutp_lds_bytes(n);
  size_t reo = align_up((size_t)n * 2, 16) * 2;
  size_t a = solve;
  if (ilu > a) a = ilu;
  if (reo > a) a = reo;
  size_t o = align_up(a, 16);
  L.regionA = 0;
  L.red = o; o += (size_t)NWAVE * (MAXIT + 2) * 8;
  L.hb = o; o += (MAXIT + 2) * 8;
  L.cs = o; o += (MAXIT + 1) * 8;
  L.sn = o; o += (MAXIT + 1) * 8;
  L.gg = o; o += (MAXIT + 2) * 8;
  L.rp = o; o += (size_t)maxit * (maxit + 1) / 2 * 8 + 8;
  L.yb = o; o += (MAXIT + 1) * 8;
  L.gb = o; o += (size_t)(mmax + 1) * 8;
  L.cb = o; o += (size_t)(mmax + 1) * 8;
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
  double* gb;
  double* cb;
  double* sc;
  int* ic;
  void* stmp;
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
  s.gb = (double*)(base + L.gb);
  s.cb = (double*)(base + L.cb);
  s.sc = (double*)(base + L.sc);
  s.ic = (int*)(base + L.ic);
  s.stmp = (void*)(base + L.stmp);
  return s;
}

// ---------------------------------------------------------------------------
// Reductions (deterministic: fixed butterfly order, identical in every lane)
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline int wave_id() { return threadIdx.x >> 6; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_sumi(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_mini(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_maxd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// sum over groups of 8 consecutive lanes
template <typename T>
__device__ inline T sum8(T v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
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

// Evaluate one Slater row phi_j(r) over sites within the cutoff (one wave).
// Entries are written in candidate order to out_col/out_val (global) as column
// positions cmap[site].  Returns the entry count (may exceed cap; entries past
// cap are not written).
__device__ inline int wave_row(const Walker& W, double rx, double ry, double rz, const int* cmap,
                               int* out_col, double* out_val, float* out_val32, int cap) {
  const int lane = lane_id();
  const double R = W.cutoff + W.margin;
  int lox, cx, loy, cy, loz, cz;
  axis_range(rx, R, W.a, W.lat[0], lox, cx);
  axis_range(ry, R, W.a, W.lat[1], loy, cy);
  axis_range(rz, R, W.a, W.lat[2], loz, cz);
  const int total = cx * cy * cz;
  const double rc2 = W.cutoff * W.cutoff;
  int count = 0;
  for (int t0 = 0; t0 < total; t0 += 64) {
    int t = t0 + lane;
    bool hit = false;
    int site = 0;
    double val = 0.0;
    if (t < total) {
      int tx = t % cx;
      int ty = (t / cx) % cy;
      int tz = t / (cx * cy);
      int ix = wrap_index(lox + tx, W.lat[0]);
      int iy = wrap_index(loy + ty, W.lat[1]);
      int iz = wrap_index(loz + tz, W.lat[2]);
      site = ix + W.lat[0] * (iy + W.lat[1] * iz);
      double dx;
      double d2 = dist2_xyz(rx, ry, rz, W.sites + 3 * (size_t)site, W.box, &dx);
      if (d2 <= rc2) {
        hit = true;
        val = orbital_value(W, d2, dx, W.sigma[site]);
      }
    }
    unsigned long long mask = __ballot(hit);
    int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (hit) {
      int o = count + before;
      if (o < cap) {
        out_col[o] = cmap[site];
        out_val[o] = val;
        if (out_val32) out_val32[o] = (float)val;
      }
    }
    count += __popcll(mask);
  }
  return count;
}

}  // namespace vmc
