// Preconditioner application, SpMV and right-preconditioned full GMRES
// (workgroup-level device code, templated on the Krylov precision KT).
#pragma once

#include "vmc_common.hpp"

namespace vmc {

template <typename KT> struct Fac;
template <> struct Fac<double> {
  __device__ static const double* lval(const Walker& W) { return W.l_val; }
  __device__ static const double* usval(const Walker& W) { return W.us_val; }
  __device__ static const double* dinv(const Walker& W) { return W.u_dinv; }
  __device__ static const double* aval(const Walker& W) { return W.a_val; }
  __device__ static const double* Z(const Walker& W) { return W.Z64; }
  __device__ static const double* upval(const Walker& W) { return W.up_val; }
};
template <> struct Fac<float> {
  __device__ static const float* lval(const Walker& W) { return W.l_val32; }
  __device__ static const float* usval(const Walker& W) { return W.us_val32; }
  __device__ static const float* dinv(const Walker& W) { return W.u_dinv32; }
  __device__ static const float* aval(const Walker& W) { return W.a_val32; }
  __device__ static const float* Z(const Walker& W) { return W.Z32; }
  __device__ static const float* upval(const Walker& W) { return W.up_val32; }
};

__device__ inline float readlane_k(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ inline double readlane_k(double v, int k) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

constexpr int PF = 8;  // entries per thread held in registers per block (8 threads per row)

// One 64-row block of a triangular factor, as seen by one of the 8 threads of a row.
template <typename KT>
struct RowChunk {
  int len;
  int col[PF];
  KT val[PF];
};

template <typename KT>
__device__ inline void load_chunk(RowChunk<KT>& ch, int r, int n, int len, const int* cols,
                                  const KT* vals, int F, int sub) {
  ch.len = (r < n) ? len : 0;
#pragma unroll
  for (int t = 0; t < PF; ++t) {
    const int e = sub + 8 * t;
    if (e < ch.len) {
      ch.col[t] = cols[(size_t)r * F + e];
      ch.val[t] = vals[(size_t)r * F + e];
    }
  }
}

// In-block substitution by wave 0: lane r holds the block right-hand side of
// row r; D (LDS, column-major 64x64) holds the in-block coefficients and is
// cleared as it is read.  Forward (unit lower) or backward (unit upper).
template <typename KT, bool FORWARD>
__device__ inline KT block_chain(KT a, KT* D) {
  const int lane = lane_id();
  if (FORWARD) {
#pragma unroll 16
    for (int k = 0; k < BLK; ++k) {
      const KT dk = D[k * BLK + lane];
      D[k * BLK + lane] = (KT)0;
      const KT xk = readlane_k(a, k);
      a -= dk * xk;
    }
  } else {
#pragma unroll 16
    for (int k = BLK - 1; k >= 0; --k) {
      const KT dk = D[k * BLK + lane];
      D[k * BLK + lane] = (KT)0;
      const KT xk = readlane_k(a, k);
      a -= dk * xk;
    }
  }
  return a;
}

// Forward solve L x = b with unit lower L (rows by position, capacity F).
// b = rhs (global) or, when rhs == nullptr, the unit vector e_unit.
// Blocks of 64 rows: 8 threads per row gather the contributions of columns in
// earlier blocks from x (LDS) and scatter in-block coefficients into D; wave 0
// then runs the in-block chain.  Row data of the next block is loaded into
// registers while the current block is processed.
template <typename KT>
__device__ inline void wg_lsolve(const Walker& W, const KT* lval, const KT* rhs, int unit, KT* xs,
                                 KT* D, KT* st) {
  const int n = W.n, F = W.F;
  const int rr = threadIdx.x >> 3, sub = threadIdx.x & 7;
  const int nb = (n + BLK - 1) / BLK;
  RowChunk<KT> cur, nxt;
  KT crhs = 0, nrhs = 0;
  int nlen2 = 0;
  {
    const int r = rr;
    load_chunk(cur, r, n, r < n ? W.l_len[r] : 0, W.l_col, lval, F, sub);
    crhs = (r < n) ? (rhs ? rhs[r] : (KT)(r == unit ? 1 : 0)) : (KT)0;
    const int r1 = BLK + rr;
    nlen2 = (r1 < n) ? W.l_len[r1] : 0;
  }
  for (int b = 0; b < nb; ++b) {
    const int r0 = b * BLK;
    const int r = r0 + rr;
    // prefetch block b+1 (its lengths were loaded one block earlier) and lengths of b+2
    if (b + 1 < nb) {
      const int r1 = r + BLK;
      load_chunk(nxt, r1, n, nlen2, W.l_col, lval, F, sub);
      nrhs = (r1 < n) ? (rhs ? rhs[r1] : (KT)(r1 == unit ? 1 : 0)) : (KT)0;
      const int r2 = r + 2 * BLK;
      nlen2 = (r2 < n) ? W.l_len[r2] : 0;
    }
    KT acc = 0;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = sub + 8 * t;
      if (e < cur.len) {
        const int c = cur.col[t];
        if (c < r0) acc += cur.val[t] * xs[c];
        else D[(c - r0) * BLK + rr] = cur.val[t];
      }
    }
    for (int e = sub + 8 * PF; e < cur.len; e += 8) {
      const int c = W.l_col[(size_t)r * F + e];
      const KT v = lval[(size_t)r * F + e];
      if (c < r0) acc += v * xs[c];
      else D[(c - r0) * BLK + rr] = v;
    }
    acc = sum8(acc);
    if (sub == 0) st[rr] = crhs - acc;
    __syncthreads();
    if (wave_id() == 0) {
      KT a = st[lane_id()];
      a = block_chain<KT, true>(a, D);
      if (r0 + lane_id() < n) xs[r0 + lane_id()] = a;
    }
    __syncthreads();
    cur = nxt;
    crhs = nrhs;
  }
}

// Backward solve with U, stored as D^{-1}U (unit upper, off-diagonal) and
// D^{-1}; in place on xs.
template <typename KT>
__device__ inline void wg_usolve(const Walker& W, const KT* usval, const KT* dinv, KT* xs, KT* D,
                                 KT* st) {
  const int n = W.n, F = W.F;
  const int rr = threadIdx.x >> 3, sub = threadIdx.x & 7;
  const int nb = (n + BLK - 1) / BLK;
  RowChunk<KT> cur, nxt;
  KT cd = 0, nd = 0;
  int nlen2 = 0;
  {
    const int r = (nb - 1) * BLK + rr;
    load_chunk(cur, r, n, r < n ? W.u_len[r] : 0, W.u_col, usval, F, sub);
    cd = (r < n) ? dinv[r] : (KT)0;
    const int r1 = r - BLK;
    nlen2 = (r1 >= 0 && r1 < n) ? W.u_len[r1] : 0;
  }
  for (int b = nb - 1; b >= 0; --b) {
    const int r0 = b * BLK;
    const int r = r0 + rr;
    if (b > 0) {
      const int r1 = r - BLK;
      load_chunk(nxt, r1, n, nlen2, W.u_col, usval, F, sub);
      nd = (r1 < n) ? dinv[r1] : (KT)0;
      const int r2 = r - 2 * BLK;
      nlen2 = (r2 >= 0 && r2 < n) ? W.u_len[r2] : 0;
    }
    const int rend = r0 + BLK;
    KT acc = 0;
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int e = sub + 8 * t;
      if (e < cur.len) {
        const int c = cur.col[t];
        if (c >= rend) acc += cur.val[t] * xs[c];
        else D[(c - r0) * BLK + rr] = cur.val[t];
      }
    }
    for (int e = sub + 8 * PF; e < cur.len; e += 8) {
      const int c = W.u_col[(size_t)r * F + e];
      const KT v = usval[(size_t)r * F + e];
      if (c >= rend) acc += v * xs[c];
      else D[(c - r0) * BLK + rr] = v;
    }
    acc = sum8(acc);
    if (sub == 0) st[rr] = (r < n) ? xs[r] * cd - acc : (KT)0;
    __syncthreads();
    if (wave_id() == 0) {
      KT a = st[lane_id()];
      a = block_chain<KT, false>(a, D);
      if (r0 + lane_id() < n) xs[r0 + lane_id()] = a;
    }
    __syncthreads();
    cur = nxt;
    cd = nd;
  }
}

// x <- (I - zhat_{m-1} u_{m-1}^T) ... (I - zhat_0 u_0^T) x, in the compact form
// c = G g with g_s = u_s^T x and G = (I + T)^{-1}, T_{st} = u_s^T zhat_t (t < s).
template <typename KT>
__device__ inline void wg_updates(const Walker& W, int m, int mmax, KT* xs, Smem& S) {
  if (m <= 0) return;
  const int n = W.n;
  const KT* upv = Fac<KT>::upval(W);
  for (int s = wave_id(); s < m; s += NWAVE) {
    const int len = W.up_len[s];
    KT acc = 0;
    for (int e = lane_id(); e < len; e += 64)
      acc += upv[(size_t)s * W.UC + e] * xs[W.up_col[(size_t)s * W.UC + e]];
    const double sacc = wave_sum((double)acc);
    if (lane_id() == 0) S.gb[s] = sacc;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < m; s += NT) {
    double c = 0.0;
    for (int t = 0; t <= s; ++t) c += W.T[(size_t)s * mmax + t] * S.gb[t];
    S.cb[s] = c;
  }
  __syncthreads();
  const KT* Z = Fac<KT>::Z(W);
  for (int r = threadIdx.x; r < n; r += NT) {
    KT v = xs[r];
    for (int s = 0; s < m; ++s) v -= Z[(size_t)s * n + r] * (KT)S.cb[s];
    xs[r] = v;
  }
  __syncthreads();
}

// y = M v:  x = L^{-1} v, x = U^{-1} x, then the rank-one factors (all in the
// column-position numbering, which already contains the ILUTP permutation).
template <typename KT>
__device__ inline void wg_precond(const Walker& W, int m, int mmax, const KT* vin, int unit, KT* xs,
                                  Smem& S) {
  KT* D = xs + align_up((size_t)W.n, 4);
  KT* st = (KT*)S.stmp;
  wg_lsolve<KT>(W, Fac<KT>::lval(W), vin, unit, xs, D, st);
  wg_usolve<KT>(W, Fac<KT>::usval(W), Fac<KT>::dinv(W), xs, D, st);
  wg_updates<KT>(W, m, mmax, xs, S);
}

// w = A x with x in LDS; 8 threads per row.
template <typename KT>
__device__ inline void wg_spmv(const Walker& W, const KT* aval, const KT* xs, KT* w) {
  const int n = W.n, Wc = W.W;
  const int rr = threadIdx.x >> 3, sub = threadIdx.x & 7;
  for (int base = 0; base < n; base += BLK) {
    const int r = base + rr;
    KT acc = 0;
    if (r < n) {
      const int len = W.a_len[r];
      const int* ac = W.a_col + (size_t)r * Wc;
      const KT* av = aval + (size_t)r * Wc;
      for (int e = sub; e < len; e += 8) acc += av[e] * xs[ac[e]];
    }
    acc = sum8(acc);
    if (sub == 0 && r < n) w[r] = acc;
  }
}

// r = e_unit - A z in FP64 (z global); returns ||r||_2.
__device__ inline double wg_resid64(const Walker& W, const double* z, int unit, double* rv, Smem& S) {
  const int n = W.n, Wc = W.W;
  const int rr = threadIdx.x >> 3, sub = threadIdx.x & 7;
  double nl = 0.0;
  for (int base = 0; base < n; base += BLK) {
    const int r = base + rr;
    double acc = 0.0;
    if (r < n) {
      const int len = W.a_len[r];
      const int* ac = W.a_col + (size_t)r * Wc;
      const double* av = W.a_val + (size_t)r * Wc;
      for (int e = sub; e < len; e += 8) acc += av[e] * z[ac[e]];
    }
    acc = sum8(acc);
    if (sub == 0 && r < n) {
      const double x = (r == unit ? 1.0 : 0.0) - acc;
      rv[r] = x;
      nl += x * x;
    }
  }
  __syncthreads();
  return sqrt(wg_sum(nl, S.red));
}

// h[i] = sum_r w[r] V_i[r] for i < cnt (FP64 reduction), written to out[] (LDS).
template <typename KT>
__device__ inline void wg_dots(const KT* w, const KT* V, int n, int cnt, double* out, Smem& S) {
  __syncthreads();
  for (int i = 0; i < cnt; ++i) {
    KT acc = 0;
    const KT* vi = V + (size_t)i * n;
    for (int r = threadIdx.x; r < n; r += NT) acc += w[r] * vi[r];
    const double s = wave_sum((double)acc);
    if (lane_id() == 0) S.red[i * NWAVE + wave_id()] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += NT) {
    double s = 0.0;
    for (int k = 0; k < NWAVE; ++k) s += S.red[i * NWAVE + k];
    out[i] = s;
  }
  __syncthreads();
}

struct SolveOut {
  int iters;
  int conv;
  double N;
  double res;
};

// Right-preconditioned full GMRES on A M x~ = b, z = M x~ (Section 3.2), with
// x0 = 0, Arnoldi by classical Gram-Schmidt applied twice, Givens rotations,
// and the effective stability N = max_j ||v_j - A M v_j|| (eq.
// (stabilityVecEq)).  b = e_unit (rhs64 == nullptr) or rhs64 / beta.  The
// solution is accumulated in FP64: z (+)= scale * sum_j y_j (M v_j).
template <typename KT>
__device__ inline SolveOut wg_gmres(const Walker& W, int m, const DevParams& P, Smem& S, int unit,
                                    const double* rhs64, double beta, double tol, int maxit, double* z,
                                    double scale, bool zinit) {
  const int n = W.n;
  KT* V = (KT*)W.V;
  KT* Xp = (KT*)W.Xp;
  KT* w = (KT*)W.wv;
  KT* xs = (KT*)S.A;
  const KT* aval = Fac<KT>::aval(W);
  const bool unit_rhs = (rhs64 == nullptr);
  {
    KT* D = xs + align_up((size_t)n, 4);
    for (int e = threadIdx.x; e < BLK * BLK; e += NT) D[e] = (KT)0;
  }
  for (int r = threadIdx.x; r < n; r += NT)
    V[r] = unit_rhs ? (KT)(r == unit ? 1 : 0) : (KT)(rhs64[r] / beta);
  if (threadIdx.x == 0) S.gg[0] = 1.0;
  __syncthreads();
  double N = 0.0;
  int k = 0;
  int conv = 0;
  double res = 1.0;
  for (int j = 0; j < maxit; ++j) {
    const KT* vj = V + (size_t)j * n;
    wg_precond<KT>(W, m, P.m_max, (j == 0 && unit_rhs) ? nullptr : vj, unit, xs, S);
    KT* xp = Xp + (size_t)j * n;
    for (int r = threadIdx.x; r < n; r += NT) xp[r] = xs[r];
    wg_spmv<KT>(W, aval, xs, w);
    __syncthreads();
    // effective stability: ||v_j - A M v_j||
    double nl = 0.0;
    for (int r = threadIdx.x; r < n; r += NT) {
      const double d = (double)vj[r] - (double)w[r];
      nl += d * d;
    }
    const double Nj = sqrt(wg_sum(nl, S.red));
    N = fmax(N, Nj);
    // classical Gram-Schmidt, twice
    double* h = S.hb;
    wg_dots<KT>(w, V, n, j + 1, h, S);
    for (int r = threadIdx.x; r < n; r += NT) {
      KT x = w[r];
      for (int i = 0; i <= j; ++i) x -= (KT)h[i] * V[(size_t)i * n + r];
      w[r] = x;
    }
    __syncthreads();
    double* h2 = S.yb;
    wg_dots<KT>(w, V, n, j + 1, h2, S);
    double nw = 0.0;
    for (int r = threadIdx.x; r < n; r += NT) {
      KT x = w[r];
      for (int i = 0; i <= j; ++i) x -= (KT)h2[i] * V[(size_t)i * n + r];
      w[r] = x;
      nw += (double)x * (double)x;
    }
    const double hn = sqrt(wg_sum(nw, S.red));
    KT* vn = V + (size_t)(j + 1) * n;
    const KT inv = (hn > 0.0) ? (KT)(1.0 / hn) : (KT)0;
    for (int r = threadIdx.x; r < n; r += NT) vn[r] = w[r] * inv;
    if (threadIdx.x == 0) {
      double* col = S.hb;
      for (int i = 0; i <= j; ++i) col[i] += h2[i];
      col[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double t = S.cs[i] * col[i] + S.sn[i] * col[i + 1];
        col[i + 1] = -S.sn[i] * col[i] + S.cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = hypot(col[j], col[j + 1]);
      double c = 1.0, s = 0.0;
      if (den > 0.0) { c = col[j] / den; s = col[j + 1] / den; }
      S.cs[j] = c;
      S.sn[j] = s;
      col[j] = den;
      S.gg[j + 1] = -s * S.gg[j];
      S.gg[j] = c * S.gg[j];
      double* Rc = S.rp + (size_t)j * (j + 1) / 2;
      for (int i = 0; i <= j; ++i) Rc[i] = col[i];
      const double rj = fabs(S.gg[j + 1]);
      S.sc[0] = rj;
      S.ic[2] = (rj <= tol || den == 0.0) ? 1 : 0;
      S.ic[3] = (den == 0.0) ? 1 : 0;
    }
    __syncthreads();
    res = S.sc[0];
    conv = S.ic[2];
    const int broke = S.ic[3];
    k = broke ? j : j + 1;
    if (conv) break;
  }
  // y = R^{-1} g, z (+)= scale * sum y_i Xp_i
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s = S.gg[i];
      for (int l = i + 1; l < k; ++l) s -= S.rp[(size_t)l * (l + 1) / 2 + i] * S.yb[l];
      S.yb[i] = s / S.rp[(size_t)i * (i + 1) / 2 + i];
    }
    for (int i = 0; i < k; ++i) S.yb[i] *= scale;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += NT) {
    double acc = zinit ? 0.0 : z[r];
    for (int i = 0; i < k; ++i) acc += S.yb[i] * (double)Xp[(size_t)i * n + r];
    z[r] = acc;
  }
  __syncthreads();
  SolveOut o;
  o.iters = k;
  o.conv = conv;
  o.N = N;
  o.res = res * beta;
  return o;
}

// ratio = 1 + u^T z (FP64), u = pending update (column positions).
__device__ inline double wg_ratio(const Walker& W, int ulen, const double* z, Smem& S) {
  double acc = 0.0;
  for (int e = threadIdx.x; e < ulen; e += NT) acc += W.pu_val[e] * z[W.pu_col[e]];
  return 1.0 + wg_sum(acc, S.red);
}

}  // namespace vmc
