// Slater-matrix build, geometric reorder and ILUTP (workgroup-level device code).
#pragma once

#include "vmc_common.hpp"

namespace vmc {

// Evaluate every row of A (row position i holds particle rowperm[i]; column
// position of site s is cpos[s]).  One wave per row.  Returns WST_* bits.
__device__ inline int wg_build_all_rows(const Walker& W, Smem& S) {
  const int n = W.n;
  int bad = 0;
  for (int i = wave_id(); i < n; i += NWAVE) {
    const int p = W.rowperm[i];
    const double rx = W.pos[3 * p], ry = W.pos[3 * p + 1], rz = W.pos[3 * p + 2];
    int cnt = wave_row(W, rx, ry, rz, W.cpos, W.a_col + (size_t)i * W.W, W.a_val + (size_t)i * W.W,
                       W.a_val32 + (size_t)i * W.W, W.W);
    if (lane_id() == 0) W.a_len[i] = cnt < W.W ? cnt : W.W;
    if (cnt > W.W) bad = 1;
  }
  __syncthreads();
  if (lane_id() == 0 && bad) S.ic[0] = 1;
  // combine the capacity flag across waves
  __syncthreads();
  int flag = S.ic[0];
  __syncthreads();
  if (threadIdx.x == 0) S.ic[0] = 0;
  __syncthreads();
  return flag ? WST_CAPACITY : WST_OK;
}

// Geometric greedy reorder of particles and orbitals (Section 3.1): for each
// position i, bring the orbital closest to the particle at i to column i; if
// it already is there, bring the particle closest to that orbital to row i.
// Starts from the identity labelling; squared minimum-image distances; ties to
// the first position.  Writes rowperm/rpos and colsite/cpos (reorder order)
// and reo_row/reo_col.
__device__ inline void wg_reorder(const Walker& W, Smem& S) {
  const int n = W.n;
  short* rp = (short*)S.A;
  short* cp = rp + align_up((size_t)n, 8);
  for (int k = threadIdx.x; k < n; k += NT) { rp[k] = (short)k; cp[k] = (short)k; }
  __syncthreads();
  for (int i = 0; i < n - 1; ++i) {
    const int pi = rp[i];
    const double rx = W.pos[3 * pi], ry = W.pos[3 * pi + 1], rz = W.pos[3 * pi + 2];
    double best = INFINITY;
    int bj = 0x7fffffff;
    for (int j = i + threadIdx.x; j < n; j += NT) {
      double dx;
      double d2 = dist2_xyz(rx, ry, rz, W.sites + 3 * (size_t)cp[j], W.box, &dx);
      if (d2 < best) { best = d2; bj = j; }
    }
    wg_argmin(best, bj, S.red);
    if (bj != i) {
      __syncthreads();
      if (threadIdx.x == 0) { short t = cp[i]; cp[i] = cp[bj]; cp[bj] = t; }
      __syncthreads();
      continue;
    }
    const double* Zi = W.sites + 3 * (size_t)cp[i];
    best = INFINITY;
    int bk = 0x7fffffff;
    for (int k = i + threadIdx.x; k < n; k += NT) {
      const int pk = rp[k];
      double dx;
      double d2 = dist2_xyz(W.pos[3 * pk], W.pos[3 * pk + 1], W.pos[3 * pk + 2], Zi, W.box, &dx);
      if (d2 < best) { best = d2; bk = k; }
    }
    wg_argmin(best, bk, S.red);
    __syncthreads();
    if (bk != i && threadIdx.x == 0) { short t = rp[i]; rp[i] = rp[bk]; rp[bk] = t; }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < n; k += NT) {
    const int p = rp[k], s = cp[k];
    W.reo_row[k] = p;
    W.reo_col[k] = s;
    W.rowperm[k] = p;
    W.rpos[p] = k;
    W.colsite[k] = s;
    W.cpos[s] = k;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// ILUTP, row-wise (Saad's threshold ILU with column pivoting), run by wave 0.
// A's current column numbering is the label space; the result is folded into
// the column numbering: afterwards column position k holds label q[k] and A,
// cpos/colsite are renumbered, so A (renumbered) ~ L U.
// ---------------------------------------------------------------------------
__device__ inline int ilutp_row_cap_extra(const Walker& W, const DevParams& P, Smem& S) {
  // p = ceil(nnz(A) / (2n)) unless given
  if (P.lfil >= 0) return P.lfil;
  int s = 0;
  for (int i = threadIdx.x; i < W.n; i += NT) s += W.a_len[i];
  double tot = wg_sum((double)s, S.red);
  return (int)ceil(tot / (2.0 * W.n));
}

__device__ inline int wg_ilutp(const Walker& W, const DevParams& P, Smem& S) {
  const int n = W.n;
  const int F = W.F;
  const int pfill = ilutp_row_cap_extra(W, P, S);
  char* base = S.A;
  double* wv = (double*)base;               base += align_up((size_t)n * 8, 16);
  unsigned char* present = (unsigned char*)base; base += align_up((size_t)n, 16);
  short* pinv = (short*)base;               base += align_up((size_t)n * 2, 16);
  short* q = (short*)base;                  base += align_up((size_t)n * 2, 16);
  short* nzc = (short*)base;                base += align_up((size_t)NZMAX * 2, 16);
  short* lk = (short*)base;                 base += align_up((size_t)LMAX * 2, 16);
  double* lv = (double*)base;

  for (int k = threadIdx.x; k < n; k += NT) {
    wv[k] = 0.0;
    present[k] = 0;
    pinv[k] = (short)k;
    q[k] = (short)k;
  }
  __syncthreads();

  int status = WST_OK;
  if (wave_id() == 0) {
    const int lane = lane_id();
    const double droptol = P.droptol, permtol = P.permtol;
    for (int i = 0; i < n && status == WST_OK; ++i) {
      // 1. load row i
      const int len = W.a_len[i];
      double nrm = 0.0;
      int nl0 = 0, nu0 = 0;
      for (int e = lane; e < len; e += 64) {
        const int c = W.a_col[(size_t)i * W.W + e];
        const double v = W.a_val[(size_t)i * W.W + e];
        wv[c] = v;
        present[c] = 1;
        nzc[e] = (short)c;
        nrm += v * v;
        const int k = pinv[c];
        nl0 += (k < i);
        nu0 += (k > i);
      }
      nrm = wave_sum(nrm);
      nl0 = wave_sumi(nl0);
      nu0 = wave_sumi(nu0);
      const double tau = droptol * sqrt(nrm);
      int nz = len;
      int lcount = 0;
      int kcur = -1;
      // 2. eliminate in increasing position order
      while (true) {
        int best = 0x7fffffff;
        for (int e = lane; e < nz; e += 64) {
          const int k = pinv[nzc[e]];
          if (k > kcur && k < i && k < best) best = k;
        }
        best = wave_mini(best);
        if (best == 0x7fffffff) break;
        kcur = best;
        const int c = q[best];
        const double lik = wv[c] / W.u_diag[best];
        if (fabs(lik) < tau) continue;
        if (lcount < LMAX) {
          if (lane == 0) { lk[lcount] = (short)best; lv[lcount] = lik; }
        } else {
          status = WST_CAPACITY;
          break;
        }
        ++lcount;
        const int ul = W.u_len[best];
        const int* ucol = W.u_col + (size_t)best * F;
        const double* uval = W.u_val + (size_t)best * F;
        for (int e0 = 0; e0 < ul; e0 += 64) {
          const int e = e0 + lane;
          bool isnew = false;
          int c2 = 0;
          double v2 = 0.0;
          if (e < ul) {
            c2 = ucol[e];
            v2 = uval[e];
            if (present[c2]) {
              wv[c2] -= lik * v2;
            } else {
              isnew = true;
            }
          }
          unsigned long long mask = __ballot(isnew);
          const int before = __popcll(mask & ((1ull << lane) - 1ull));
          if (isnew) {
            const int o = nz + before;
            wv[c2] = -lik * v2;
            present[c2] = 1;
            if (o < NZMAX) nzc[o] = (short)c2;
          }
          nz += __popcll(mask);
        }
        if (nz > NZMAX) { status = WST_CAPACITY; break; }
      }
      if (status != WST_OK) break;

      // 3./4. U part: threshold drop (never the current diagonal column), fill limit
      const int cd = q[i];
      const int ucap = nu0 + pfill;
      const int lcap = nl0 + pfill;
      // count off-diagonal candidates
      int ucnt = 0;
      for (int e = lane; e < nz; e += 64) {
        const int c = nzc[e];
        if (c != cd && pinv[c] >= i && fabs(wv[c]) >= tau) ++ucnt;
      }
      ucnt = wave_sumi(ucnt);
      // rank threshold: an off-diagonal candidate is kept when fewer than ucap
      // candidates precede it in (|v| desc, position asc) order
      double vmax = -1.0;
      int cmax_pos = 0x7fffffff;
      const double vd = present[cd] ? wv[cd] : 0.0;
      if (present[cd]) { vmax = fabs(vd); cmax_pos = i; }
      int uwrite = 0;
      int* out_col = W.u_col + (size_t)i * F;
      double* out_val = W.u_val + (size_t)i * F;
      for (int e0 = 0; e0 < nz; e0 += 64) {
        const int e = e0 + lane;
        bool keep = false;
        int c = 0;
        double v = 0.0;
        if (e < nz) {
          c = nzc[e];
          v = wv[c];
          if (c != cd && pinv[c] >= i && fabs(v) >= tau) {
            keep = true;
            if (ucnt > ucap) {
              const double av = fabs(v);
              const int kp = pinv[c];
              int rank = 0;
              for (int f = 0; f < nz; ++f) {
                const int c3 = nzc[f];
                if (c3 == cd || pinv[c3] < i) continue;
                const double a3 = fabs(wv[c3]);
                if (a3 < tau) continue;
                if (a3 > av || (a3 == av && pinv[c3] < kp)) ++rank;
              }
              keep = rank < ucap;
            }
          }
        }
        unsigned long long mask = __ballot(keep);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) {
          const int o = uwrite + before;
          if (o < F) { out_col[o] = c; out_val[o] = v; }
          const double av = fabs(v);
          const int kp = pinv[c];
          if (av > vmax || (av == vmax && kp < cmax_pos)) { vmax = av; cmax_pos = kp; }
        }
        uwrite += __popcll(mask);
      }
      // wave argmax of (|v| desc, position asc)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(vmax, o, 64);
        const int op = __shfl_xor(cmax_pos, o, 64);
        if (ov > vmax || (ov == vmax && op < cmax_pos)) { vmax = ov; cmax_pos = op; }
      }
      if (uwrite > F - 1) { status = WST_CAPACITY; break; }
      if (!(vmax > 0.0)) { status = WST_SINGULAR; break; }
      // 5. pivot: swap the diagonal column with the largest entry's column
      int newdiag = cd;
      double dval = vd;
      if (permtol * vmax > fabs(vd) && cmax_pos != i) {
        const int cm = q[cmax_pos];
        newdiag = cm;
        dval = wv[cm];
        if (lane == 0) {
          q[i] = (short)cm;
          q[cmax_pos] = (short)cd;
          pinv[cm] = (short)i;
          pinv[cd] = (short)cmax_pos;
        }
        // the new diagonal leaves the off-diagonal list; the old diagonal joins it
        // (present entries only)
        int slot = -1;
        for (int e = lane; e < uwrite; e += 64)
          if (out_col[e] == cm) slot = e;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) slot = max(slot, __shfl_xor(slot, o, 64));
        if (present[cd]) {
          if (lane == 0) { out_col[slot] = cd; out_val[slot] = vd; }
        } else {
          // move the last entry into the hole
          if (lane == 0) {
            out_col[slot] = out_col[uwrite - 1];
            out_val[slot] = out_val[uwrite - 1];
          }
          --uwrite;
        }
      }
      if (dval == 0.0) { status = WST_SINGULAR; break; }
      // 4. L part: keep the lcap largest multipliers
      int lwrite = 0;
      int* lcol = W.l_col + (size_t)i * F;
      double* lval = W.l_val + (size_t)i * F;
      for (int e0 = 0; e0 < lcount; e0 += 64) {
        const int e = e0 + lane;
        bool keep = false;
        if (e < lcount) {
          keep = true;
          if (lcount > lcap) {
            const double av = fabs(lv[e]);
            const int kp = lk[e];
            int rank = 0;
            for (int f = 0; f < lcount; ++f) {
              const double a3 = fabs(lv[f]);
              if (a3 > av || (a3 == av && lk[f] < kp)) ++rank;
            }
            keep = rank < lcap;
          }
        }
        unsigned long long mask = __ballot(keep);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) {
          const int o = lwrite + before;
          if (o < F) { lcol[o] = lk[e]; lval[o] = lv[e]; }
        }
        lwrite += __popcll(mask);
      }
      if (lwrite > F) { status = WST_CAPACITY; break; }
      if (lane == 0) {
        W.u_len[i] = uwrite;
        W.u_diag[i] = dval;
        W.l_len[i] = lwrite;
      }
      // 6. clear the work row
      for (int e = lane; e < nz && e < NZMAX; e += 64) {
        const int c = nzc[e];
        wv[c] = 0.0;
        present[c] = 0;
      }
      (void)newdiag;
      __threadfence_block();
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) S.ic[1] = status;
  __syncthreads();
  status = S.ic[1];
  __syncthreads();
  if (status != WST_OK) return status;

  // Fold Q into the column numbering: label c -> position pinv[c].
  for (int i = threadIdx.x; i < n; i += NT) {
    const int ul = W.u_len[i];
    int* uc = W.u_col + (size_t)i * F;
    double* uv = W.u_val + (size_t)i * F;
    const double d = W.u_diag[i];
    const double dinv = 1.0 / d;
    W.u_dinv[i] = dinv;
    W.u_dinv32[i] = (float)dinv;
    for (int e = 0; e < ul; ++e) {
      uc[e] = pinv[uc[e]];
      const double s = uv[e] * dinv;
      W.us_val[(size_t)i * F + e] = s;
      W.us_val32[(size_t)i * F + e] = (float)s;
    }
    const int ll = W.l_len[i];
    for (int e = 0; e < ll; ++e) W.l_val32[(size_t)i * F + e] = (float)W.l_val[(size_t)i * F + e];
    const int al = W.a_len[i];
    int* ac = W.a_col + (size_t)i * W.W;
    for (int e = 0; e < al; ++e) ac[e] = pinv[ac[e]];
    W.ilu_q[i] = q[i];
  }
  // colsite_new[k] = colsite_old[q[k]]; cpos[s] = pinv[cpos[s]]
  __syncthreads();
  int* tmp = (int*)wv;  // reuse the work row (n ints fit in n doubles)
  for (int k = threadIdx.x; k < n; k += NT) tmp[k] = W.colsite[q[k]];
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += NT) {
    W.colsite[k] = tmp[k];
    W.cpos[tmp[k]] = k;
  }
  __syncthreads();
  return WST_OK;
}

}  // namespace vmc
