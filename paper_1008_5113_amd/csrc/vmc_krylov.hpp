// Preconditioner application, SpMV and right-preconditioned full GMRES
// (workgroup-level device code, templated on the Krylov precision KT).
#pragma once

#include "vmc_common.hpp"

namespace vmc {

template <typename KT> struct Fac;
template <> struct Fac<double> {
  __device__ static const double* lval(const Walker& W) { return W.lv64; }
  __device__ static const double* usval(const Walker& W) { return W.uv64; }
  __device__ static const double* dinv(const Walker& W) { return W.u_dinv; }
  __device__ static const double* aval(const Walker& W) { return W.a_val; }
  __device__ static const double* Z(const Walker& W) { return W.Z64; }
  __device__ static const double* upval(const Walker& W) { return W.up_val; }
};
template <> struct Fac<float> {
  __device__ static const float* lval(const Walker& W) { return W.lv32; }
  __device__ static const float* usval(const Walker& W) { return W.uv32; }
  __device__ static const float* dinv(const Walker& W) { return W.u_dinv32; }
  __device__ static const float* aval(const Walker& W) { return W.a_val32; }
  __device__ static const float* Z(const Walker& W) { return W.Z32; }
  __device__ static const float* upval(const Walker& W) { return W.up_val32; }
};


// In-block substitution by wave 0: lane r holds the block right-hand side of
// row r; D (LDS, column-major 64x64) holds the in-block coefficients.  Step k
// broadcasts x_k from lane k (v_readlane) and every lane subtracts its
// coefficient times x_k.  The coefficients are read in batches of 16 that are
// issued one batch ahead of use, so LDS latency stays off the dependency chain.
template <typename KT, bool FORWARD>
VMC_PHASE KT block_chain(KT a, const KT* D) {
  constexpr int B = sizeof(KT) == 8 ? 8 : 16;  // coefficients per batch (register budget)
  const int lane = lane_id();
  KT d0[B], d1[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int k = FORWARD ? j : BLK - 1 - j;
    d0[j] = D[k * DSTR + lane];
  }
#pragma unroll
  for (int q = 0; q < BLK / B; ++q) {
    if (q + 1 < BLK / B) {
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const int k = FORWARD ? B * (q + 1) + j : BLK - 1 - (B * (q + 1) + j);
        d1[j] = D[k * DSTR + lane];
      }
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int k = FORWARD ? B * q + j : BLK - 1 - (B * q + j);
      const KT xk = readlane_t(a, k);
      a -= d0[j] * xk;
    }
#pragma unroll
    for (int j = 0; j < B; ++j) d0[j] = d1[j];
  }
  return a;
}

constexpr int PF = 4;  // entries per thread per row (8 threads per row)

__device__ inline bool is_far(bool forward, int c, int r0) {
  return forward ? (c < r0) : (c >= r0 + BLK);
}

// Triangular solve by 64-row blocks on the compact CSR factors.  8 threads
// per row hold up to PF entries each in registers; rows longer than 8*PF
// finish in a strided tail loop, which runs before the block's prefetch is
// issued.  A block's row data is loaded two blocks ahead of its use and its row
// pointers three blocks ahead.  The loads are branch-free (indices clamped to a
// valid entry, selects applied at the use), and the block loop is unrolled by
// three over a block count padded to a multiple of three, so the register sets
// keep fixed roles and every path issues the same loads: no load is waited for
// before its block comes up.
template <typename KT>
struct RowChunk {
  int ok;       // row exists
  int len;
  int start;
  int col[PF];
  KT val[PF];
  KT aux;       // right-hand side (L) or inverse diagonal (U) as loaded
};

template <typename KT, bool FORWARD>
VMC_PHASE void wg_trisolve_rows(const Walker& W, const int* ptr, const unsigned short* cols,
                                const KT* vals, const KT* aux, int unit, KT* xs, KT* D, KT* st) {
  const int n = W.n;
  const int rr = vmc_tid() >> 3, sub = vmc_tid() & 7;
  const int nb = (n + BLK - 1) / BLK;
  auto row_of = [&](int t) { return (t >= 0 && t < nb) ? (FORWARD ? t : nb - 1 - t) * BLK + rr : -1; };
  // Row pointers travel in three register sets with fixed roles: block t
  // loads the pointers of block t+3 before it loads the rows of block t+2
  // (whose pointers block t-1 loaded), so a pointer load is always older
  // than the row loads issued after it and waiting for it leaves those in
  // flight.
  struct RowPtr {
    int a, b, ok;
  };
  auto load_ptr = [&](RowPtr& P, int t) {
    const int r = row_of(t);
    P.ok = (r >= 0 && r < n);
    const int rc = P.ok ? r : 0;
    P.a = ptr[rc];
    P.b = ptr[rc + 1];
  };
  auto load_chunk = [&](RowChunk<KT>& ch, const RowPtr& P, int t) {
    const int r = row_of(t);
    const int pa = P.a;
    const bool pok = P.ok;
    ch.ok = pok;
    ch.len = pok ? P.b - pa : 0;
    ch.start = pa;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = sub + 8 * k;
      const int idx = (e < ch.len) ? pa + e : 0;
      ch.col[k] = cols[idx];
      ch.val[k] = vals[idx];
    }
    if (aux) ch.aux = aux[pok ? r : 0];
  };
  auto block = [&](int t, const RowChunk<KT>& cur, RowChunk<KT>& ahead, RowPtr& pnew, const RowPtr& pold) {
    const bool live = t < nb;  // the padding blocks only issue loads
    const int r0 = (FORWARD ? t : nb - 1 - t) * BLK;
    const int r = r0 + rr;
    KT acc = 0;
    int dpos[PF];
    const bool tail = cur.len > 8 * PF;
    if (live) {
      // branch-free: every entry issues one gather (far entries; others read
      // xs[0], whose value is discarded by a select: it may hold anything) and
      // one tile write (in-block entries; others hit the spare row), so all of
      // a thread's LDS accesses are in flight at once
      int gi[PF];
      bool gf[PF];
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int e = sub + 8 * k;
        const int c = cur.col[k];
        const bool valid = e < cur.len;
        const bool far = is_far(FORWARD, c, r0);
        gf[k] = valid && far;
        gi[k] = gf[k] ? c : 0;
        dpos[k] = (valid && !far) ? (c - r0) * DSTR + rr : BLK * DSTR + lane_id();
        D[dpos[k]] = cur.val[k];
      }
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const KT xk = xs[gi[k]];
        acc += gf[k] ? cur.val[k] * xk : (KT)0;
      }
      if (tail) {
        for (int e = sub + 8 * PF; e < cur.len; e += 8) {
          const int c = cols[cur.start + e];
          const KT v = vals[cur.start + e];
          if (is_far(FORWARD, c, r0)) acc += v * xs[c];
          else D[(c - r0) * DSTR + rr] = v;
        }
      }
    }
    load_ptr(pnew, t + 3);
    load_chunk(ahead, pold, t + 2);
    if (!live) return;
    acc = sum8(acc);
    if (sub == 0) {
      KT b;
      if (FORWARD) b = !cur.ok ? (KT)0 : (aux ? cur.aux : (KT)(r == unit ? 1 : 0));
      else b = cur.ok ? xs[r] * cur.aux : (KT)0;
      st[rr] = b - acc;
    }
    __syncthreads();
    if (wave_id() == 0) {
      // the chain is the block's critical path: let this wave issue first
      __builtin_amdgcn_s_setprio(3);
      KT a = st[lane_id()];
      a = block_chain<KT, FORWARD>(a, D);
      __builtin_amdgcn_s_setprio(0);
      if (r0 + lane_id() < n) xs[r0 + lane_id()] = a;
    }
    __syncthreads();
    if (tail) {
      // clear the row's whole tile row instead of re-reading its columns
      for (int cc = sub; cc < BLK; cc += 8) D[cc * DSTR + rr] = (KT)0;
    } else {
#pragma unroll
      for (int k = 0; k < PF; ++k) D[dpos[k]] = (KT)0;
    }
  };
  // forward substitution of a unit vector e_unit: every row above the unit's
  // block solves to zero, so the sweep starts at that block
  const int t0 = (FORWARD && !aux && unit >= 0 && unit < n) ? unit / BLK : 0;
  if (t0 > 0) {
    for (int r = vmc_tid(); r < t0 * BLK; r += NT) xs[r] = (KT)0;
    __syncthreads();
  }
  RowChunk<KT> X0, X1, X2;
  RowPtr Q0, Q1, Q2;
  load_ptr(Q0, t0);
  load_chunk(X0, Q0, t0);
  load_ptr(Q1, t0 + 1);
  load_chunk(X1, Q1, t0 + 1);
  load_ptr(Q2, t0 + 2);
  const int nb3 = t0 + (nb - t0 + 2) / 3 * 3;
  for (int t = t0; t < nb3; t += 3) {
    // block t uses rows X[t%3], loads rows t+2 into X[(t+2)%3] with pointers
    // Q[(t+2)%3] and loads pointers t+3 into Q[t%3]
    block(t, X0, X2, Q0, Q2);
    block(t + 1, X1, X0, Q1, Q0);
    block(t + 2, X2, X1, Q2, Q1);
  }
}

template <typename KT>
VMC_PHASE void wg_lsolve(const Walker& W, const KT* lval, const KT* rhs, int unit, KT* xs,
                                 KT* D, KT* st) {
  wg_trisolve_rows<KT, true>(W, W.lp, W.lc, lval, rhs, unit, xs, D, st);
}

template <typename KT>
VMC_PHASE void wg_usolve(const Walker& W, const KT* usval, const KT* dinv, KT* xs, KT* D,
                                 KT* st) {
  wg_trisolve_rows<KT, false>(W, W.up, W.uc, usval, dinv, -1, xs, D, st);
}

// x <- (I - zhat_{m-1} u_{m-1}^T) ... (I - zhat_0 u_0^T) x, in the compact form
// c = G g with g_s = u_s^T x and G = (I + T)^{-1}, T_{st} = u_s^T zhat_t (t < s).
// g: 4 threads per update vector; c: one thread per update; the x update
// reads four stored vectors per pass with every thread's rows in registers.
template <typename KT>
VMC_PHASE void wg_updates(const Walker& W, int m, int mmax, KT* xs, Smem& S) {
  if (m <= 0) return;
  const int n = W.n;
  const KT* upv = Fac<KT>::upval(W);
  constexpr int TPS = 8;  // threads per stored update in the two small products
  // g_s = u_s^T x (u_s sparse): every thread issues four loads at a time,
  // branch-free (indices clamped to a valid entry, products masked)
  for (int s0 = 0; s0 < m; s0 += NT / TPS) {
    const int s = s0 + (vmc_tid() >> 3), part = vmc_tid() & (TPS - 1);
    const int sc = s < m ? s : 0;
    const int len = s < m ? W.up_len[sc] : 0;
    const int* uc = W.up_col + (size_t)sc * W.UC;
    const KT* uv = upv + (size_t)sc * W.UC;
    KT acc = 0;
    for (int e0 = part; e0 < len; e0 += 4 * TPS) {
      int cc[4];
      KT vv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * TPS;
        const int ec = e < len ? e : 0;
        cc[q] = uc[ec];
        vv[q] = uv[ec];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const KT xv = xs[cc[q]];
        acc += (e0 + q * TPS < len) ? vv[q] * xv : (KT)0;
      }
    }
    acc = sum8(acc);
    if (s < m && part == 0) S.gb[s] = (double)acc;
  }
  __syncthreads();
  // c = G g with G = (I + T)^{-1} lower triangular (FP64)
  for (int s0 = 0; s0 < m; s0 += NT / TPS) {
    const int s = s0 + (vmc_tid() >> 3), part = vmc_tid() & (TPS - 1);
    const int sc = s < m ? s : 0;
    const double* Gs = W.T + (size_t)sc * mmax;
    const int tl = s < m ? s + 1 : 0;
    double c = 0.0;
    for (int t0 = part; t0 < tl; t0 += 4 * TPS) {
      double gv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = t0 + q * TPS;
        gv[q] = Gs[t < tl ? t : 0];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = t0 + q * TPS;
        c += (t < tl) ? gv[q] * S.gb[t < tl ? t : 0] : 0.0;
      }
    }
    c = sum8(c);
    if (s < m && part == 0) S.cb[s] = c;
  }
  __syncthreads();
  // x -= Z c: every thread keeps RPT rows in registers and streams four
  // stored vectors at a time with unconditional (clamped) loads
  const KT* Z = Fac<KT>::Z(W);
  constexpr int RPT = 4;
  for (int rb = 0; rb < n; rb += NT * RPT) {
    KT xr[RPT];
    int rc[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = rb + k * NT + vmc_tid();
      rc[k] = r < n ? r : 0;
      xr[k] = xs[rc[k]];
    }
    int s = 0;
    for (; s + 4 <= m; s += 4) {
      const KT c0 = (KT)S.cb[s], c1 = (KT)S.cb[s + 1], c2 = (KT)S.cb[s + 2], c3 = (KT)S.cb[s + 3];
      const KT* z0 = Z + (size_t)s * n;
      KT a0[RPT], a1[RPT], a2[RPT], a3[RPT];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        a0[k] = z0[rc[k]];
        a1[k] = z0[n + rc[k]];
        a2[k] = z0[2 * (size_t)n + rc[k]];
        a3[k] = z0[3 * (size_t)n + rc[k]];
      }
#pragma unroll
      for (int k = 0; k < RPT; ++k) xr[k] -= a0[k] * c0 + a1[k] * c1 + a2[k] * c2 + a3[k] * c3;
    }
    for (; s < m; ++s) {
      const KT c0 = (KT)S.cb[s];
      const KT* z0 = Z + (size_t)s * n;
#pragma unroll
      for (int k = 0; k < RPT; ++k) xr[k] -= z0[rc[k]] * c0;
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = rb + k * NT + vmc_tid();
      if (r < n) xs[r] = xr[k];
    }
  }
  __syncthreads();
}

// y = M v:  x = L^{-1} v, x = U^{-1} x, then the rank-one factors (all in the
// column-position numbering, which already contains the ILUTP permutation).
template <typename KT>
VMC_PHASE void wg_precond(const Walker& W, int m, int mmax, const KT* vin, int unit, KT* xs,
                                  Smem& S) {
  KT* D = xs + align_up((size_t)W.n, 4);
  KT* st = (KT*)S.stmp;
  PhaseClock pc;
  pc.start();
  wg_lsolve<KT>(W, Fac<KT>::lval(W), vin, unit, xs, D, st);
  pc.stop(S, PH_LSOLVE);
  wg_usolve<KT>(W, Fac<KT>::usval(W), Fac<KT>::dinv(W), xs, D, st);
  pc.stop(S, PH_USOLVE);
  wg_updates<KT>(W, m, mmax, xs, S);
  pc.stop(S, PH_UPDATES);
}

// w = A x (x in LDS or global).  A is stored in slices of 64 rows with entry
// e of the slice's rows contiguous (aidx), so one wave takes a slice with one
// lane per row and every load of columns or values is a full contiguous line.
// A wave walks its slice to the longest row length in it, U entries at a time,
// with the next U entries in flight while the current ones are consumed;
// entries at or past a lane's own row length are masked at the use (their
// loads stay within the slice's row capacity).  When `resid` is set, writes
// e_unit - A x instead and returns the partial sum of squares.
template <typename VT, typename XT, typename AT, typename OT>
VMC_PHASE double wg_rows_apply(const Walker& W, const VT* aval, const XT* x, OT* out, int unit,
                               bool resid) {
  constexpr int U = 8;
  const int n = W.n, Wc = W.W, lane = lane_id();
  const int nsl = (n + ASL - 1) / ASL;
  double sq = 0.0;
  for (int s = wave_id(); s < nsl; s += NWAVE) {
    const int r = s * ASL + lane;
    const int len = r < n ? W.a_len[r] : 0;
    const int wl = -wave_mini(-len);
    const size_t base = (size_t)s * Wc * ASL + lane;
    const unsigned short* ac = W.a_col + base;
    const VT* av = aval + base;
    int cA[U], cB[U];
    VT vA[U], vB[U];
    auto issue = [&](int* c, VT* v, int e0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = (size_t)min(e0 + u, Wc - 1) * ASL;
        c[u] = ac[e];
        v[u] = av[e];
      }
    };
    AT acc = 0;
    auto consume = [&](const int* c, const VT* v, int e0) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + u < len) acc += (AT)v[u] * (AT)x[c[u]];
    };
    issue(cA, vA, 0);
#pragma unroll
    for (int u = 0; u < U; ++u) { cB[u] = 0; vB[u] = (VT)0; }
    for (int e0 = 0; e0 < wl; e0 += 2 * U) {
      if (e0 + U < wl) issue(cB, vB, e0 + U);
      consume(cA, vA, e0);
      if (e0 + 2 * U < wl) issue(cA, vA, e0 + 2 * U);
      consume(cB, vB, e0 + U);
    }
    if (r < n) {
      if (resid) {
        const double y = (r == unit ? 1.0 : 0.0) - (double)acc;
        out[r] = (OT)y;
        sq += y * y;
      } else {
        out[r] = (OT)acc;
      }
    }
  }
  return sq;
}

// w = A x with x in LDS.
template <typename KT>
VMC_PHASE void wg_spmv(const Walker& W, const KT* aval, const KT* xs, KT* w) {
  wg_rows_apply<KT, KT, KT, KT>(W, aval, xs, w, -1, false);
}

// r = e_unit - A z in FP64; returns ||r||_2.  z is staged in LDS when the
// stage_bytes at S.A can hold it, otherwise gathered from global memory.
VMC_PHASE double wg_resid64(const Walker& W, const double* z, int unit, double* rv, Smem& S,
                                    size_t stage_bytes) {
  const int n = W.n;
  double sq;
  if ((size_t)n * 8 <= stage_bytes) {
    double* zs = (double*)S.A;
    for (int r = vmc_tid(); r < n; r += NT) zs[r] = z[r];
    __syncthreads();
    sq = wg_rows_apply<double, double, double, double>(W, W.a_val, zs, rv, unit, true);
  } else {
    sq = wg_rows_apply<double, double, double, double>(W, W.a_val, z, rv, unit, true);
  }
  __syncthreads();
  return sqrt(wg_sum(sq, S.red));
}
// h[i] = sum_r w[r] V_i[r] for i < cnt (FP64 reduction), written to out[] (LDS).
// Up to four dot products share one pass over w.  With vdiff set, the same
// first pass also accumulates ||vdiff - w||^2 (FP64) into out[cnt].
template <typename KT>
VMC_PHASE void wg_dots(const KT* w, const KT* V, int n, int cnt, double* out, Smem& S,
                       const KT* vdiff = nullptr) {
  __syncthreads();
  for (int i0 = 0; i0 < cnt; i0 += 4) {
    const int c = min(4, cnt - i0);
    const bool withd = vdiff && i0 == 0;
    KT acc[4] = {(KT)0, (KT)0, (KT)0, (KT)0};
    double dn = 0.0;
    for (int r = vmc_tid(); r < n; r += NT) {
      const KT wr = w[r];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < c) acc[q] += wr * V[(size_t)(i0 + q) * n + r];
      if (withd) {
        const double d = (double)vdiff[r] - (double)wr;
        dn += d * d;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < c) {
        const double sq = wave_sum((double)acc[q]);
        if (lane_id() == 0) S.red[(i0 + q) * NWAVE + wave_id()] = sq;
      }
    }
    if (withd) {
      const double sq = wave_sum(dn);
      if (lane_id() == 0) S.red[cnt * NWAVE + wave_id()] = sq;
    }
  }
  __syncthreads();
  const int tot = cnt + (vdiff ? 1 : 0);
  for (int i = vmc_tid(); i < tot; i += NT) {
    double sq = 0.0;
    for (int k = 0; k < NWAVE; ++k) sq += S.red[i * NWAVE + k];
    out[i] = sq;
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
// The solve counts as converged once the residual estimate is at most tol
// (relative to beta).  With rel_ulen >= 0 it iterates further, until the
// estimate is at most tol * min(1, |1 + u^T z_j|), with u the pending update
// vector (rel_ulen entries) and z_j the current iterate, whose ratio comes from
// the dots u^T (M v_i) kept per basis vector, so that a small ratio keeps its
// relative accuracy; missing only that target by maxit still counts as
// converged.  A breakdown with a singular rotated column (A M singular on the
// Krylov space) ends the solve unconverged.
template <typename KT>
VMC_PHASE SolveOut wg_gmres(const Walker& W, int m, const DevParams& P, Smem& S, int unit,
                                    const double* rhs64, double beta, double tol, int maxit, double* z,
                                    double scale, bool zinit, int rel_ulen = -1) {
  const int n = W.n;
  KT* V = (KT*)W.V;
  KT* Xp = (KT*)W.Xp;
  KT* w = (KT*)W.wv;
  KT* xs = (KT*)S.A;
  const KT* aval = Fac<KT>::aval(W);
  const bool unit_rhs = (rhs64 == nullptr);
  {
    KT* D = xs + align_up((size_t)n, 4);
    for (int e = vmc_tid(); e < DTILE; e += NT) D[e] = (KT)0;
  }
  for (int r = vmc_tid(); r < n; r += NT)
    V[r] = unit_rhs ? (KT)(r == unit ? 1 : 0) : (KT)(rhs64[r] / beta);
  if (vmc_tid() == 0) S.gg[0] = 1.0;
  __syncthreads();
  double N = 0.0;
  int k = 0;
  int conv = 0;   // at tol
  int done = 0;   // at the iteration's target (tol, or the ratio-relative one)
  double res = 1.0;
  for (int j = 0; j < maxit; ++j) {
    const KT* vj = V + (size_t)j * n;
    wg_precond<KT>(W, m, P.m_max, (j == 0 && unit_rhs) ? nullptr : vj, unit, xs, S);
    KT* xp = Xp + (size_t)j * n;
    PhaseClock pc;
    pc.start();
    if (rel_ulen >= 0 && wave_id() == 0) {
      // u^T (M v_j) for the ratio of the current iterate (u sparse, FP64)
      double acc = 0.0;
      for (int e = lane_id(); e < rel_ulen; e += 64) acc += W.pu_val[e] * (double)xs[W.pu_col[e]];
      acc = wave_sum(acc);
      if (lane_id() == 0) S.ux[j] = acc;
    }
    for (int r = vmc_tid(); r < n; r += NT) xp[r] = xs[r];
    wg_spmv<KT>(W, aval, xs, w);
    __syncthreads();
    pc.stop(S, PH_SPMV);
    // classical Gram-Schmidt, twice; the first pass also gives the effective
    // stability term ||v_j - A M v_j||
    double* h = S.hb;
    wg_dots<KT>(w, V, n, j + 1, h, S, vj);
    N = fmax(N, sqrt(h[j + 1]));
    for (int r = vmc_tid(); r < n; r += NT) {
      KT x = w[r];
      for (int i = 0; i <= j; ++i) x -= (KT)h[i] * V[(size_t)i * n + r];
      w[r] = x;
    }
    __syncthreads();
    double* h2 = S.yb;
    wg_dots<KT>(w, V, n, j + 1, h2, S);
    double nw = 0.0;
    for (int r = vmc_tid(); r < n; r += NT) {
      KT x = w[r];
      for (int i = 0; i <= j; ++i) x -= (KT)h2[i] * V[(size_t)i * n + r];
      w[r] = x;
      nw += (double)x * (double)x;
    }
    const double hn = sqrt(wg_sum(nw, S.red));
    KT* vn = V + (size_t)(j + 1) * n;
    const KT inv = (hn > 0.0) ? (KT)(1.0 / hn) : (KT)0;
    for (int r = vmc_tid(); r < n; r += NT) vn[r] = w[r] * inv;
    if (vmc_tid() == 0) {
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
      double rj = fabs(S.gg[j + 1]);
      int cv = rj <= tol;
      int dn = cv;
      if (den == 0.0) {
        // singular rotated column: the residual is still |g_j|, and the
        // least-squares problem has no solution in this space
        rj = fabs(S.gg[j]);
        cv = dn = 0;
      } else if (cv && rel_ulen >= 0) {
        // ratio of the current iterate: y = R^{-1} g (k = j + 1), 1 + sum y_i u^T M v_i
        double* y = S.yb;  // free here: the second Gram-Schmidt pass has been added in
        double ratio = 1.0;
        for (int i = j; i >= 0; --i) {
          double t = S.gg[i];
          for (int l = i + 1; l <= j; ++l) t -= S.rp[(size_t)l * (l + 1) / 2 + i] * y[l];
          y[i] = t / S.rp[(size_t)i * (i + 1) / 2 + i];
          ratio += y[i] * S.ux[i];
        }
        dn = rj <= tol * fmin(1.0, fabs(ratio));
      }
      S.sc[0] = rj;
      S.ic[2] = cv;
      S.ic[3] = (den == 0.0) ? 1 : 0;
      S.ic[9] = dn;
    }
    __syncthreads();
    pc.stop(S, PH_ORTHO);
    res = S.sc[0];
    conv = S.ic[2];
    done = S.ic[9];
    const int broke = S.ic[3];
    k = broke ? j : j + 1;
    if (done || broke) break;
  }
  // y = R^{-1} g, z (+)= scale * sum y_i Xp_i
  PhaseClock pz;
  pz.start();
  if (vmc_tid() == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s = S.gg[i];
      for (int l = i + 1; l < k; ++l) s -= S.rp[(size_t)l * (l + 1) / 2 + i] * S.yb[l];
      S.yb[i] = s / S.rp[(size_t)i * (i + 1) / 2 + i];
    }
    for (int i = 0; i < k; ++i) S.yb[i] *= scale;
  }
  __syncthreads();
  for (int r = vmc_tid(); r < n; r += NT) {
    double acc = zinit ? 0.0 : z[r];
    for (int i = 0; i < k; ++i) acc += S.yb[i] * (double)Xp[(size_t)i * n + r];
    z[r] = acc;
  }
  __syncthreads();
  pz.stop(S, PH_SOLUTION);
  SolveOut o;
  o.iters = k;
  o.conv = conv;
  o.N = N;
  o.res = res * beta;
  return o;
}

// ratio = 1 + u^T z (FP64), u = pending update (column positions).
VMC_PHASE double wg_ratio(const Walker& W, int ulen, const double* z, Smem& S, double base = 1.0) {
  double acc = 0.0;
  for (int e = vmc_tid(); e < ulen; e += NT) acc += W.pu_val[e] * z[W.pu_col[e]];
  return base + wg_sum(acc, S.red);
}

}  // namespace vmc
