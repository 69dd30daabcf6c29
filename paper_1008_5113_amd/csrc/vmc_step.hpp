// One Metropolis step of one walker (workgroup-level): proposal, new row and
// u, determinant ratio, reorder triggers, decision, row replacement and
// preconditioner update.
#pragma once

#include "vmc_krylov.hpp"
#include "vmc_setup.hpp"

namespace vmc {

// New row of particle p at rnew (column positions) and u = new row - old row
// (eq. (matrixUpdateU)), written to the walker's pending buffers.  Returns
// WST_*; the row position and the lengths come back through S.ic[4..6].
VMC_PHASE int wg_prepare(const Walker& W, Smem& S, int p, const double* rnew) {
  PhaseClock pc;
  pc.start();
  const int i = W.rpos[p];
  // LDS staging of the old and the new row (the solve region is free here)
  int* oc = (int*)S.A;
  double* ov = (double*)(S.A + align_up((size_t)W.W * 4, 16));
  int* nc = (int*)(S.A + align_up((size_t)W.W * 4, 16) + (size_t)W.W * 8);
  double* nv = (double*)((char*)nc + align_up((size_t)W.W * 4, 16));
  const int lo = W.a_len[i];
  for (int e = vmc_tid(); e < lo; e += NT) {
    oc[e] = W.a_col[aidx(W.W, i, e)];
    ov[e] = W.a_val[aidx(W.W, i, e)];
  }
  if (wave_id() == 0) {
    const int lane = lane_id();
    int st = WST_OK;
    const int cnt = wave_row(W, rnew[0], rnew[1], rnew[2], W.cpos, nc, nv, nullptr, W.W);
    if (cnt > W.W) st = WST_CAPACITY;
    if (lane == 0) {
      S.ic[4] = i;
      S.ic[5] = cnt;
      S.ic[7] = st;
    }
  }
  __syncthreads();
  const int cnt = S.ic[5];
  int st = S.ic[7];
  int ul = 0;
  if (st == WST_OK) {
    // u = new row - old row over the union of the two patterns (eq. (matrixUpdateU))
    for (int e = vmc_tid(); e < cnt; e += NT) {
      const int c = nc[e];
      double vo = 0.0;
      for (int f = 0; f < lo; ++f)
        if (oc[f] == c) { vo = ov[f]; break; }
      W.pu_col[e] = c;
      W.pu_val[e] = nv[e] - vo;
      W.new_col[e] = c;
      W.new_val[e] = nv[e];
    }
    if (wave_id() == 0) {
      const int lane = lane_id();
      ul = cnt;
      for (int e0 = 0; e0 < lo; e0 += 64) {
        const int e = e0 + lane;
        bool miss = false;
        int c = 0;
        if (e < lo) {
          c = oc[e];
          miss = true;
          for (int f = 0; f < cnt; ++f)
            if (nc[f] == c) { miss = false; break; }
        }
        const unsigned long long mask = __ballot(miss);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (miss) {
          W.pu_col[ul + before] = c;
          W.pu_val[ul + before] = -ov[e];
        }
        ul += __popcll(mask);
      }
      if (lane == 0) S.ic[6] = ul;
    }
  }
  __threadfence_block();
  __syncthreads();
  pc.stop(S, PH_PREPARE);
  return st;
}

struct StepSolve {
  double ratio;
  int iters_first;  // iterations of the first (inner) solve
  int iters_total;
  int conv_first;
  int conv;
  double N;
  double res;
  int inner;
  int passes;
};

// ratio = 1 + u^T z with A z = e_i (eq. (detRatioEq)).  With kin set, the
// pending vector holds a whole replacement row (a kinetic row) and the result
// is its dot product with z alone; the mixed refinement then stops on the
// residual norm without the ratio scale.
template <int PREC>
VMC_PHASE StepSolve wg_solve(const Walker& W, int m, const DevParams& P, Smem& S, int i, int ulen,
                             bool kin = false, int maxit = -1) {
  StepSolve o;
  const double base = kin ? 0.0 : 1.0;
  if (maxit < 1) maxit = P.maxit;
  if (PREC == VMC_PREC_FP64) {
    // a ratio solve iterates to rtol * min(1, |ratio|) and counts as
    // converged at rtol; a kinetic term (base 0) stops at rtol
    SolveOut g = wg_gmres<double>(W, m, P, S, i, nullptr, 1.0, P.rtol, maxit, W.zvec, 1.0, true,
                                  (kin || P.plain_stop) ? -1 : ulen);
    o.ratio = wg_ratio(W, ulen, W.zvec, S, base);
    o.iters_first = o.iters_total = g.iters;
    o.conv_first = o.conv = g.conv;
    o.N = g.N;
    o.res = g.res;
    o.inner = 1;
    o.passes = 0;
  } else {
    // FP32 inner solves, FP64 residual, ratio and monitor (iterative refinement)
    SolveOut g = wg_gmres<float>(W, m, P, S, i, nullptr, 1.0, P.inner_rtol, maxit, W.zvec, 1.0, true);
    o.iters_first = g.iters;
    o.iters_total = g.iters;
    o.conv_first = g.conv;
    o.N = g.N;
    o.inner = 1;
    o.conv = 0;
    int pass = 0;
    while (true) {
      PhaseClock pc;
      pc.start();
      // between the solves nothing in region A is live (the new row has been
      // handed over in global memory), so all of it may stage z
      const size_t stage = (size_t)((char*)S.red - S.A);
      const double rn = wg_resid64(W, W.zvec, i, W.rvec, S, stage);
      o.ratio = wg_ratio(W, ulen, W.zvec, S, base);
      pc.stop(S, PH_RESID);
      o.res = rn;
      const double target = P.refine_tol * ((kin || P.plain_stop) ? 1.0 : fmin(1.0, fabs(o.ratio)));
      if (rn <= target) {
        o.conv = 1;
        break;
      }
      // out of passes short of the ratio-relative target: converged if the
      // residual meets refine_tol itself
      if (pass >= P.refine_maxit || !(rn > 0.0)) {
        o.conv = rn <= P.refine_tol ? 1 : 0;
        break;
      }
      ++pass;
      // the correction only has to bring the residual under the target (with
      // a factor 2 of margin for its FP32 estimate), not a full inner_rtol
      // reduction; the next FP64 residual checks what it reached
      const double ctol = fmax(P.inner_rtol, 0.5 * target / rn);
      SolveOut c = wg_gmres<float>(W, m, P, S, -1, W.rvec, rn, ctol, P.maxit, W.zvec, rn, false);
      o.N = fmax(o.N, c.N);
      o.iters_total += c.iters;
      ++o.inner;
    }
    o.passes = pass;
  }
  return o;
}

// Geometric reorder, rebuild of A in the new order, ILUTP (Section 3.1/3.2).
template <int PREC>
VMC_PHASE int wg_reorder_refactor(const Walker& W, const DevParams& P, Smem& S) {
  PhaseClock pc;
  pc.start();
  // the Krylov basis is free between solves: the reorder's cell lists
  wg_reorder(W, S, (void*)W.V, (size_t)(P.maxit + 1) * W.n * (PREC == VMC_PREC_FP64 ? 8 : 4));
  int st = wg_build_all_rows(W, S);
  pc.stop(S, PH_REORDER);
  if (st != WST_OK) return st;
  st = wg_ilutp(W, P, S);
  pc.stop(S, PH_REFACTOR);
  return st;
}

// Append the rank-one factor of an accepted move (eq. (mkp1)): zhat = z/ratio,
// u; G = (I + T)^{-1} gains a row.
template <int PREC>
VMC_PHASE void wg_append_update(const Walker& W, const DevParams& P, Smem& S, int s, double ratio,
                                        int ulen) {
  const int n = W.n, mm = P.m_max;
  const double inv = 1.0 / ratio;
  for (int r = vmc_tid(); r < n; r += NT) {
    const double zh = W.zvec[r] * inv;
    if (PREC == VMC_PREC_FP64) W.Z64[(size_t)s * n + r] = zh;
    else W.Z32[(size_t)s * n + r] = (float)zh;
  }
  for (int e = vmc_tid(); e < ulen; e += NT) {
    W.up_col[(size_t)s * W.UC + e] = W.pu_col[e];
    W.up_val[(size_t)s * W.UC + e] = W.pu_val[e];
    W.up_val32[(size_t)s * W.UC + e] = (float)W.pu_val[e];
  }
  if (vmc_tid() == 0) W.up_len[s] = ulen;
  __threadfence_block();
  __syncthreads();
  // t_l = u_s^T zhat_l, l < s, in the precision the apply uses
  for (int l = wave_id(); l < s; l += NWAVE) {
    double acc = 0.0;
    for (int e = lane_id(); e < ulen; e += 64) {
      const int c = W.up_col[(size_t)s * W.UC + e];
      if (PREC == VMC_PREC_FP64) acc += W.up_val[(size_t)s * W.UC + e] * W.Z64[(size_t)l * n + c];
      else acc += (double)(W.up_val32[(size_t)s * W.UC + e] * W.Z32[(size_t)l * n + c]);
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) S.gb[l] = acc;
  }
  __syncthreads();
  // G[s][t] = -sum_{l=t}^{s-1} t_l G[l][t];  G[s][s] = 1
  for (int t = vmc_tid(); t <= s; t += NT) {
    double v = 1.0;
    if (t < s) {
      double acc = 0.0;
      for (int l = t; l < s; ++l) acc += S.gb[l] * W.T[(size_t)l * mm + t];
      v = -acc;
    }
    W.T[(size_t)s * mm + t] = v;
  }
  __threadfence_block();
  __syncthreads();
}

// Ratio of a trial move (particle p to rnew), with the reorder triggers of
// Section 4: N > n_thresh, first solve not converged, or iterations >=
// iter_factor * running average.  Leaves the pending state in the walker.
template <int PREC>
VMC_PHASE void wg_det_ratio(const Walker& W, WalkerState* ws, const DevParams& P, Smem& S, int p,
                                    const double* rnew, double u_acc) {
  if (vmc_tid() == 0) S.ic[8] = 0;
  __syncthreads();
  int flags = 0;
  int st = wg_prepare(W, S, p, rnew);
  int i = S.ic[4];
  int ulen = S.ic[6];
  StepSolve o;
  o.ratio = 0.0;
  o.iters_first = o.iters_total = 0;
  o.conv = o.conv_first = 0;
  o.N = 0.0;
  o.res = 0.0;
  o.inner = o.passes = 0;
  if (st == WST_OK) {
    const int m = ws->m;
    o = wg_solve<PREC>(W, m, P, S, i, ulen, false, (P.test_knobs & VMC_TEST_FIRST_SOLVE_ONE_ITER) ? 1 : -1);
    const long long g = ws->g;
    const double avg = ws->avg_iters;
    const long long navg = ws->avg_count;
    // the reorder triggers of Section 4; a refinement that misses its
    // tolerance counts as not converged
    int why = 0;
    if (o.N > P.n_thresh) why |= VMC_FLAG_TRIG_N;
    if (!o.conv_first || !o.conv) why |= VMC_FLAG_TRIG_NOCONV;
    if (navg >= P.iter_min_solves && (double)o.iters_first >= P.iter_factor * avg) why |= VMC_FLAG_TRIG_ITERS;
    if (P.force_reorder_every > 0 && ((g + 1) % P.force_reorder_every) == 0) why |= VMC_FLAG_TRIG_FORCED;
    const bool trig = why != 0;
    __syncthreads();
    if (vmc_tid() == 0) {
      ws->avg_count = navg + 1;
      ws->avg_iters = avg + ((double)o.iters_first - avg) / (double)(navg + 1);
      ws->st_solves += 1;
      ws->st_inner += o.inner;
      ws->st_refine += o.passes;
      ws->st_msum += (long long)m * o.inner;
      // one preconditioner application per GMRES iteration, each streaming
      // the m stored update vectors
      const double ent = (double)m * W.n * o.iters_total;
      ws->upd_entries += ent;
      ws->st_upd_entries += ent;
    }
    if (trig) {
      flags |= VMC_FLAG_REORDERED | why;
      st = wg_reorder_refactor<PREC>(W, P, S);
      if (vmc_tid() == 0) {
        ws->m = 0;
        ws->upd_entries = 0.0;
        ws->st_reorders += 1;
        ws->st_refactors += 1;
      }
      __threadfence_block();
      __syncthreads();
      if (st == WST_OK) st = wg_prepare(W, S, p, rnew);
      if (st == WST_OK) {
        i = S.ic[4];
        ulen = S.ic[6];
        o = wg_solve<PREC>(W, 0, P, S, i, ulen);
        if (vmc_tid() == 0) {
          ws->st_solves += 1;
          ws->st_inner += o.inner;
          ws->st_refine += o.passes;
        }
        // still not converged with a fresh ordering and factorisation: the
        // walker stops with VMC_ENOCONV
        if (!o.conv) {
          st |= WST_NOCONV;
          flags |= VMC_FLAG_NOCONV;
        }
      }
    }
  }
  if (o.conv) flags |= VMC_FLAG_CONVERGED;
  if (st & WST_SINGULAR) flags |= VMC_FLAG_SINGULAR;
  if (st & WST_CAPACITY) flags |= VMC_FLAG_CAPACITY;
  __syncthreads();
  if (vmc_tid() == 0) {
    ws->pend_valid = (st == WST_OK) ? 1 : 0;
    ws->pend_p = p;
    ws->pend_i = i;
    ws->pend_newlen = S.ic[5];
    ws->pend_ulen = ulen;
    ws->pend_flags = flags;
    ws->pend_iters = o.iters_total;
    ws->pend_passes = o.passes;
    ws->pend_inner = o.inner;
    ws->pend_newpos[0] = rnew[0];
    ws->pend_newpos[1] = rnew[1];
    ws->pend_newpos[2] = rnew[2];
    ws->pend_ratio = o.ratio;
    ws->pend_uacc = u_acc;
    ws->pend_N = o.N;
    ws->pend_resid = o.res;
    ws->st_iters += o.iters_total;
    ws->st_sumN += o.N;
    if (o.N > ws->st_maxN) ws->st_maxN = o.N;
    if (!o.conv) ws->st_nonconv += 1;
    if (st != WST_OK) ws->status |= st;
  }
  __threadfence_block();
  __syncthreads();
}

// The step record of the pending move (walker state after wg_det_ratio).
__device__ inline void fill_record(vmc_step_record& r, const WalkerState* ws, int widx, double ratio, int flags) {
  r.step = ws->g;
  r.walker = widx;
  r.particle = ws->pend_p;
  r.new_pos[0] = ws->pend_newpos[0];
  r.new_pos[1] = ws->pend_newpos[1];
  r.new_pos[2] = ws->pend_newpos[2];
  r.ratio = ratio;
  r.log_abs_ratio = log(fabs(ratio));
  r.u_acc = ws->pend_uacc;
  r.N = ws->pend_N;
  r.resid = ws->pend_resid;
  r.iters = ws->pend_iters;
  r.flags = flags;
  r.refinements = ws->pend_passes;
  r.inner_solves = ws->pend_inner;
}

// A move may be committed only with a finite nonzero ratio: otherwise the new
// Slater matrix is singular and zhat = z / ratio undefined.
__device__ inline bool ratio_acceptable(double ratio) { return isfinite(ratio) && ratio != 0.0; }

// Commit (accept != 0) or discard the pending move; advance the step counter.
template <int PREC>
VMC_PHASE void wg_accept(const Walker& W, WalkerState* ws, const DevParams& P, Smem& S, int accept,
                                 int widx, vmc_step_record* rec) {
  const int p = ws->pend_p, i = ws->pend_i;
  const int newlen = ws->pend_newlen, ulen = ws->pend_ulen;
  const double ratio = ws->pend_ratio;
  int flags = ws->pend_flags;
  int st = WST_OK;
  PhaseClock pc;
  pc.start();
  if (accept) {
    flags |= VMC_FLAG_ACCEPTED;
    for (int e = vmc_tid(); e < newlen; e += NT) {
      const size_t o = aidx(W.W, i, e);
      W.a_col[o] = (unsigned short)W.new_col[e];
      const double v = W.new_val[e];
      W.a_val[o] = v;
      W.a_val32[o] = (float)v;
    }
    if (vmc_tid() == 0) {
      W.a_len[i] = newlen;
      W.pos[3 * p] = ws->pend_newpos[0];
      W.pos[3 * p + 1] = ws->pend_newpos[1];
      W.pos[3 * p + 2] = ws->pend_newpos[2];
    }
    __threadfence_block();
    __syncthreads();
    const int m = ws->m;
    // refactor when the update list is full, or (cost balance, Section 3.2)
    // once applying the stored updates has cost as much as a new ILUTP
    const bool balance = ws->refactor_cost > 0.0 && ws->upd_entries >= ws->refactor_cost;
    if (m + 1 >= P.m_max || balance) {
      pc.stop(S, PH_ACCEPT);
      st = wg_ilutp(W, P, S);
      pc.stop(S, PH_REFACTOR);
      flags |= VMC_FLAG_REFACTORED;
      if (vmc_tid() == 0) {
        ws->m = 0;
        ws->upd_entries = 0.0;
        ws->st_refactors += 1;
      }
    } else {
      wg_append_update<PREC>(W, P, S, m, ratio, ulen);
      if (vmc_tid() == 0) ws->m = m + 1;
    }
  }
  pc.stop(S, PH_ACCEPT);
  __syncthreads();
  if (vmc_tid() == 0) {
    if (rec) {
      fill_record(*rec, ws, widx, ratio, flags | ((st & WST_SINGULAR) ? VMC_FLAG_SINGULAR : 0));
    }
    ws->g += 1;
    ws->st_steps += 1;
    if (accept) ws->st_acc += 1;
    ws->pend_valid = 0;
    if (st != WST_OK) ws->status |= st;
  }
  __threadfence_block();
  __syncthreads();
}

// Kinetic row of particle p at its current position, -(1/2) lap phi_j(r_p)
// over the sites within the cutoff, in the pending-vector buffers.  The row
// position comes back in S.ic[4], the length in S.ic[5].
VMC_PHASE int wg_kinetic_row(const Walker& W, Smem& S, int p) {
  if (wave_id() == 0) {
    const double* r = W.pos + 3 * (size_t)p;
    const int cnt = wave_row<int, 1>(W, r[0], r[1], r[2], W.cpos, W.pu_col, W.pu_val, nullptr, W.W);
    if (lane_id() == 0) {
      S.ic[4] = W.rpos[p];
      S.ic[5] = cnt;
      S.ic[7] = cnt > W.W ? WST_CAPACITY : WST_OK;
    }
  }
  __threadfence_block();
  __syncthreads();
  return S.ic[7];
}

// Kinetic-energy terms of particles p0..p1-1 (Section 2.3 and eq. (energyEq)):
// t_p = -(1/2) lap_p Psi / Psi = lkin_p^T A^{-1} e_{i(p)}, the determinant
// ratio of A with row i(p) replaced by the kinetic row.  Every term is one
// more solve A z = e_i through the same preconditioned GMRES (with its mixed
// refinement) and the same reorder triggers as a determinant ratio.  Writes
// t_p to terms[p - p0] when terms is not null and returns their sum, added in
// particle order.
template <int PREC>
VMC_PHASE double wg_energy(const Walker& W, WalkerState* ws, const DevParams& P, Smem& S, int p0, int p1,
                           double* terms) {
  double sum = 0.0;
  for (int p = p0; p < p1; ++p) {
    int st = wg_kinetic_row(W, S, p);
    double t = 0.0;
    if (st == WST_OK) {
      const int m = ws->m;
      StepSolve o = wg_solve<PREC>(W, m, P, S, S.ic[4], S.ic[5], true);
      const double avg = ws->avg_iters;
      const bool trig = (o.N > P.n_thresh) || !o.conv_first ||
                        (ws->avg_count >= P.iter_min_solves && (double)o.iters_first >= P.iter_factor * avg);
      __syncthreads();
      if (vmc_tid() == 0) {
        ws->st_solves += 1;
        ws->st_inner += o.inner;
        ws->st_refine += o.passes;
        ws->st_iters += o.iters_total;
        ws->st_msum += (long long)m * o.inner;
        const double ent = (double)m * W.n * o.iters_total;
        ws->upd_entries += ent;
        ws->st_upd_entries += ent;
      }
      if (trig) {
        st = wg_reorder_refactor<PREC>(W, P, S);
        if (vmc_tid() == 0) {
          ws->m = 0;
          ws->upd_entries = 0.0;
          ws->st_reorders += 1;
          ws->st_refactors += 1;
        }
        __threadfence_block();
        __syncthreads();
        if (st == WST_OK) st = wg_kinetic_row(W, S, p);
        if (st == WST_OK) {
          o = wg_solve<PREC>(W, 0, P, S, S.ic[4], S.ic[5], true);
          if (vmc_tid() == 0) {
            ws->st_solves += 1;
            ws->st_inner += o.inner;
            ws->st_refine += o.passes;
            ws->st_iters += o.iters_total;
          }
        }
      }
      if (!o.conv && vmc_tid() == 0) ws->st_nonconv += 1;
      t = o.ratio;
    }
    if (st != WST_OK) {
      if (vmc_tid() == 0) ws->status |= st;
      __syncthreads();
      break;
    }
    sum += t;
    if (terms && vmc_tid() == 0) terms[p - p0] = t;
    __syncthreads();
  }
  __threadfence_block();
  __syncthreads();
  return sum;
}

}  // namespace vmc
