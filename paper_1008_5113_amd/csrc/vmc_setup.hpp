// Slater-matrix build, geometric reorder and ILUTP (workgroup-level device code).
#pragma once

#include "vmc_common.hpp"

namespace vmc {

// Evaluate every row of A (row position i holds particle rowperm[i]; column
// position of site s is cpos[s]).  One wave per row.  Returns WST_* bits.
VMC_PHASE int wg_build_all_rows(const Walker& W, Smem& S) {
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
  if (vmc_tid() == 0) S.ic[0] = 0;
  __syncthreads();
  return flag ? WST_CAPACITY : WST_OK;
}

// Geometric greedy reorder of particles and orbitals (Section 3.1): for each
// position i, bring the orbital closest to the particle at i to column i; if
// it already is there, bring the particle closest to that orbital to row i.
// Starts from the identity labelling; squared minimum-image distances; ties to
// the first position.  Writes rowperm/rpos and colsite/cpos (reorder order)
// and reo_row/reo_col.
VMC_PHASE void wg_reorder(const Walker& W, Smem& S) {
  const int n = W.n;
  short* rp = (short*)S.A;
  short* cp = rp + align_up((size_t)n, 8);
  for (int k = vmc_tid(); k < n; k += NT) { rp[k] = (short)k; cp[k] = (short)k; }
  __syncthreads();
  for (int i = 0; i < n - 1; ++i) {
    const int pi = rp[i];
    const double rx = W.pos[3 * pi], ry = W.pos[3 * pi + 1], rz = W.pos[3 * pi + 2];
    double best = INFINITY;
    int bj = 0x7fffffff;
    for (int j = i + vmc_tid(); j < n; j += NT) {
      double dx;
      double d2 = dist2_xyz(rx, ry, rz, W.sites + 3 * (size_t)cp[j], W.box, &dx);
      if (d2 < best) { best = d2; bj = j; }
    }
    wg_argmin(best, bj, S.red);
    if (bj != i) {
      __syncthreads();
      if (vmc_tid() == 0) { short t = cp[i]; cp[i] = cp[bj]; cp[bj] = t; }
      __syncthreads();
      continue;
    }
    const double* Zi = W.sites + 3 * (size_t)cp[i];
    best = INFINITY;
    int bk = 0x7fffffff;
    for (int k = i + vmc_tid(); k < n; k += NT) {
      const int pk = rp[k];
      double dx;
      double d2 = dist2_xyz(W.pos[3 * pk], W.pos[3 * pk + 1], W.pos[3 * pk + 2], Zi, W.box, &dx);
      if (d2 < best) { best = d2; bk = k; }
    }
    wg_argmin(best, bk, S.red);
    __syncthreads();
    if (bk != i && vmc_tid() == 0) { short t = rp[i]; rp[i] = rp[bk]; rp[bk] = t; }
    __syncthreads();
  }
  for (int k = vmc_tid(); k < n; k += NT) {
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

// Exclusive prefix sum over n row lengths into ptr[0..n] (ptr[n] = total),
// each thread owning a contiguous run of rows.
VMC_PHASE void wg_exclusive_scan(const int* len, int* ptr, int n, Smem& S) {
  int* sc = (int*)S.red;  // NT ints
  const int chunk = (n + NT - 1) / NT;
  const int b0 = vmc_tid() * chunk;
  const int b1 = min(n, b0 + chunk);
  int loc = 0;
  for (int r = b0; r < b1; ++r) loc += len[r];
  __syncthreads();
  sc[vmc_tid()] = loc;
  __syncthreads();
  if (vmc_tid() == 0) {
    int run = 0;
    for (int t = 0; t < NT; ++t) {
      const int v = sc[t];
      sc[t] = run;
      run += v;
    }
    ptr[n] = run;
  }
  __syncthreads();
  int run = sc[vmc_tid()];
  for (int r = b0; r < b1; ++r) {
    ptr[r] = run;
    run += len[r];
  }
  __syncthreads();
}

// Compact CSR copies of L and of D^{-1}U for the triangular solves.
VMC_PHASE void wg_pack_factors(const Walker& W, Smem& S) {
  const int n = W.n, F = W.F;
  wg_exclusive_scan(W.l_len, W.lp, n, S);
  wg_exclusive_scan(W.u_len, W.up, n, S);
  __threadfence_block();
  __syncthreads();
  for (int r = vmc_tid(); r < n; r += NT) {
    int o = W.lp[r];
    const int ll = W.l_len[r];
    for (int e = 0; e < ll; ++e) {
      W.lc[o + e] = (unsigned short)W.l_col[(size_t)r * F + e];
      const double v = W.l_val[(size_t)r * F + e];
      W.lv64[o + e] = v;
      W.lv32[o + e] = (float)v;
    }
    o = W.up[r];
    const int ul = W.u_len[r];
    const double dinv = W.u_dinv[r];
    for (int e = 0; e < ul; ++e) {
      W.uc[o + e] = (unsigned short)W.u_col[(size_t)r * F + e];
      const double v = W.u_val[(size_t)r * F + e] * dinv;
      W.uv64[o + e] = v;
      W.uv32[o + e] = (float)v;
    }
  }
  __threadfence_block();
  __syncthreads();
}

// ---------------------------------------------------------------------------
// ILUTP, row-wise (Saad's threshold ILU with column pivoting), run by wave 0.
// A's current column numbering is the label space; the result is folded into
// the column numbering: afterwards column position k holds label q[k] and A,
// cpos/colsite are renumbered, so A (renumbered) ~ L U.
// ---------------------------------------------------------------------------
VMC_PHASE int ilutp_row_cap_extra(const Walker& W, const DevParams& P, Smem& S) {
  // p = ceil(nnz(A) / (2n)) unless given
  if (P.lfil >= 0) return P.lfil;
  int s = 0;
  for (int i = vmc_tid(); i < W.n; i += NT) s += W.a_len[i];
  double tot = wg_sum((double)s, S.red);
  return (int)ceil(tot / (2.0 * W.n));
}

// Fetch the diagonal, length and (when it fits) the entries of U row k for
// every candidate that has not been fetched yet, into the LDS staging area.
// One batch of independent loads instead of one dependent load per candidate.
struct IluCand {
  short* pos;    // candidate position k (CAND_DONE once eliminated)
  double* diag;  // u_kk
  short* off;    // staging offset; -1 not fetched; -2 fetched but read from global
  short* len;    // off-diagonal length of U row k
  short* scol;   // staged columns (labels)
  double* sval;  // staged values
};

constexpr int ST_UNFETCHED = -1;
constexpr int CAND_DONE = 32767;
constexpr int ST_GLOBAL = -2;
constexpr int STAGE_UNR = 8;

VMC_PHASE void ilu_fetch_pending(const Walker& W, IluCand& C, int ncand, int& stoff) {
  const int lane = lane_id();
  const int F = W.F;
  for (int s0 = 0; s0 < ncand; s0 += 64) {
    const int s = s0 + lane;
    bool need = false;
    int k = 0, len = 0;
    if (s < ncand && C.off[s] == ST_UNFETCHED) {
      need = true;
      k = C.pos[s];
      C.diag[s] = W.u_diag[k];
      len = W.u_len[k];
      C.len[s] = (short)len;
    }
    // exclusive prefix sum of the lengths of needed slots
    int pre = need ? len : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(pre, o, 64);
      if (lane >= o) pre += t;
    }
    const int total = __shfl(pre, 63, 64);
    pre -= need ? len : 0;
    int off = ST_GLOBAL;
    if (need && stoff + pre + len <= SCAP) off = stoff + pre;
    if (need) C.off[s] = (short)off;
    const bool stage = need && off >= 0;
    // copy the rows: each lane its own row, STAGE_UNR entries per pass
    for (int base = 0;; base += STAGE_UNR) {
      const bool more = stage && base < len;
      if (!__ballot(more)) break;
      int cc[STAGE_UNR];
      double vv[STAGE_UNR];
#pragma unroll
      for (int t = 0; t < STAGE_UNR; ++t) {
        const int e = base + t;
        if (more && e < len) {
          cc[t] = W.u_col[(size_t)k * F + e];
          vv[t] = W.u_val[(size_t)k * F + e];
        }
      }
#pragma unroll
      for (int t = 0; t < STAGE_UNR; ++t) {
        const int e = base + t;
        if (more && e < len) {
          C.scol[off + e] = (short)cc[t];
          C.sval[off + e] = vv[t];
        }
      }
    }
    if (stoff + total <= SCAP) stoff += total;
    else stoff = SCAP;  // later fetches read from global
  }
}

VMC_PHASE int wg_ilutp(const Walker& W, const DevParams& P, Smem& S) {
  const int n = W.n;
  const int F = W.F;
  const int pfill = ilutp_row_cap_extra(W, P, S);
  char* base = S.A;
  double* wv = (double*)base;               base += align_up((size_t)n * 8, 16);
  unsigned* pbits = (unsigned*)base;        base += align_up((size_t)(n + 31) / 32 * 4, 16);
  short* pinv = (short*)base;               base += align_up((size_t)n * 2, 16);
  short* q = (short*)base;                  base += align_up((size_t)n * 2, 16);
  short* nzc = (short*)base;                base += align_up((size_t)NZMAX * 2, 16);
  short* lk = (short*)base;                 base += align_up((size_t)LMAX * 2, 16);
  double* lv = (double*)base;               base += align_up((size_t)LMAX * 8, 16);
  const int cmax = ilu_cmax(n);
  IluCand C;
  C.diag = (double*)base;                   base += (size_t)cmax * 8;
  C.pos = (short*)base;                     base += align_up((size_t)cmax * 2, 16);
  C.off = (short*)base;                     base += align_up((size_t)cmax * 2, 16);
  C.len = (short*)base;                     base += align_up((size_t)cmax * 2, 16);
  C.scol = (short*)base;                    base += align_up((size_t)SCAP * 2, 16);
  C.sval = (double*)base;

  for (int k = vmc_tid(); k < n; k += NT) {
    wv[k] = 0.0;
    pinv[k] = (short)k;
    q[k] = (short)k;
  }
  for (int k = vmc_tid(); k < (n + 31) / 32; k += NT) pbits[k] = 0u;
  __syncthreads();

  int status = WST_OK;
  if (wave_id() == 0) {
    const int lane = lane_id();
    const double droptol = P.droptol, permtol = P.permtol;
    for (int i = 0; i < n && status == WST_OK; ++i) {
      // 1. load row i; its entries left of the diagonal are the first candidates
      const int len = W.a_len[i];
      double nrm = 0.0;
      int nl0 = 0, nu0 = 0;
      int ncand = 0;
      for (int e0 = 0; e0 < len; e0 += 64) {
        const int e = e0 + lane;
        bool cand = false;
        int k = 0;
        if (e < len) {
          const int c = W.a_col[(size_t)i * W.W + e];
          const double v = W.a_val[(size_t)i * W.W + e];
          wv[c] = v;
          atomicOr(&pbits[c >> 5], 1u << (c & 31));
          nzc[e] = (short)c;
          nrm += v * v;
          k = pinv[c];
          nl0 += (k < i);
          nu0 += (k > i);
          cand = k < i;
        }
        const unsigned long long mask = __ballot(cand);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (cand && ncand + before < cmax) {
          C.pos[ncand + before] = (short)k;
          C.off[ncand + before] = ST_UNFETCHED;
        }
        ncand += __popcll(mask);
      }
      if (ncand > cmax) { status = WST_CAPACITY; break; }
      nrm = wave_sum(nrm);
      nl0 = wave_sumi(nl0);
      nu0 = wave_sumi(nu0);
      const double tau = droptol * sqrt(nrm);
      int nz = len;
      int lcount = 0;
      int stoff = 0;
      // 2. eliminate in increasing position order
      while (true) {
        int best = CAND_DONE, bslot = -1;
        for (int s = lane; s < ncand; s += 64) {
          const int p = C.pos[s];
          if (p < best) { best = p; bslot = s; }
        }
        {
          // positions are distinct, so exactly one lane holds the minimum
          const int bmin = wave_mini(best);
          if (bmin == CAND_DONE) break;
          const unsigned long long who = __ballot(best == bmin);
          bslot = readlane_i(bslot, __ffsll((long long)who) - 1);
          best = bmin;
        }
        if (C.off[bslot] == ST_UNFETCHED) ilu_fetch_pending(W, C, ncand, stoff);
        const int c = q[best];
        const double lik = wv[c] / C.diag[bslot];
        if (lane == 0) C.pos[bslot] = (short)CAND_DONE;
        if (fabs(lik) < tau) continue;
        if (lcount >= LMAX) { status = WST_CAPACITY; break; }
        if (lane == 0) { lk[lcount] = (short)best; lv[lcount] = lik; }
        ++lcount;
        const int ul = C.len[bslot];
        const int uoff = C.off[bslot];
        for (int e0 = 0; e0 < ul; e0 += 64) {
          const int e = e0 + lane;
          bool isnew = false, newcand = false;
          int c2 = 0, k2 = 0;
          double v2 = 0.0;
          if (e < ul) {
            if (uoff >= 0) {
              c2 = C.scol[uoff + e];
              v2 = C.sval[uoff + e];
            } else {
              c2 = W.u_col[(size_t)best * F + e];
              v2 = W.u_val[(size_t)best * F + e];
            }
            const unsigned bit = 1u << (c2 & 31);
            const unsigned old = atomicOr(&pbits[c2 >> 5], bit);
            if (old & bit) {
              wv[c2] -= lik * v2;
            } else {
              wv[c2] = -lik * v2;
              isnew = true;
              k2 = pinv[c2];
              newcand = k2 < i;
            }
          }
          unsigned long long mask = __ballot(isnew);
          int before = __popcll(mask & ((1ull << lane) - 1ull));
          if (isnew && nz + before < NZMAX) nzc[nz + before] = (short)c2;
          nz += __popcll(mask);
          mask = __ballot(newcand);
          before = __popcll(mask & ((1ull << lane) - 1ull));
          if (newcand && ncand + before < cmax) {
            C.pos[ncand + before] = (short)k2;
            C.off[ncand + before] = ST_UNFETCHED;
          }
          ncand += __popcll(mask);
        }
        if (nz > NZMAX || ncand > cmax) { status = WST_CAPACITY; break; }
      }
      if (status != WST_OK) break;

      // 3./4. U part: threshold drop (never the current diagonal column), fill limit
      const int cd = q[i];
      const bool cd_present = (pbits[cd >> 5] >> (cd & 31)) & 1u;
      const int ucap = nu0 + pfill;
      const int lcap = nl0 + pfill;
      int ucnt = 0;
      for (int e = lane; e < nz; e += 64) {
        const int c = nzc[e];
        if (c != cd && pinv[c] >= i && fabs(wv[c]) >= tau) ++ucnt;
      }
      ucnt = wave_sumi(ucnt);
      double vmax = -1.0;
      int cmax_pos = 0x7fffffff;
      const double vd = cd_present ? wv[cd] : 0.0;
      if (cd_present) { vmax = fabs(vd); cmax_pos = i; }
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
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(vmax, o, 64);
        const int op = __shfl_xor(cmax_pos, o, 64);
        if (ov > vmax || (ov == vmax && op < cmax_pos)) { vmax = ov; cmax_pos = op; }
      }
      if (uwrite > F - 1) { status = WST_CAPACITY; break; }
      if (!(vmax > 0.0)) { status = WST_SINGULAR; break; }
      // 5. pivot: swap the diagonal column with the largest entry's column
      double dval = vd;
      if (permtol * vmax > fabs(vd) && cmax_pos != i) {
        const int cm = q[cmax_pos];
        dval = wv[cm];
        if (lane == 0) {
          q[i] = (short)cm;
          q[cmax_pos] = (short)cd;
          pinv[cm] = (short)i;
          pinv[cd] = (short)cmax_pos;
        }
        // the new diagonal leaves the off-diagonal list; the old diagonal joins it
        int slot = -1;
        for (int e = lane; e < uwrite; e += 64)
          if (out_col[e] == cm) slot = e;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) slot = max(slot, __shfl_xor(slot, o, 64));
        if (cd_present) {
          if (lane == 0) { out_col[slot] = cd; out_val[slot] = vd; }
        } else {
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
      for (int e = lane; e < nz; e += 64) {
        const int c = nzc[e];
        wv[c] = 0.0;
        pbits[c >> 5] = 0u;
      }
      __threadfence_block();
    }
  }
  __syncthreads();
  if (vmc_tid() == 0) S.ic[1] = status;
  __syncthreads();
  status = S.ic[1];
  __syncthreads();
  if (status != WST_OK) return status;

  // Fold Q into the column numbering: label c -> position pinv[c].
  for (int i = vmc_tid(); i < n; i += NT) {
    const int ul = W.u_len[i];
    int* uc = W.u_col + (size_t)i * F;
    const double d = W.u_diag[i];
    const double dinv = 1.0 / d;
    W.u_dinv[i] = dinv;
    W.u_dinv32[i] = (float)dinv;
    for (int e = 0; e < ul; ++e) uc[e] = pinv[uc[e]];
    const int al = W.a_len[i];
    int* ac = W.a_col + (size_t)i * W.W;
    for (int e = 0; e < al; ++e) ac[e] = pinv[ac[e]];
    W.ilu_q[i] = q[i];
  }
  __threadfence_block();
  __syncthreads();
  wg_pack_factors(W, S);
  // colsite_new[k] = colsite_old[q[k]]; cpos[s] = pinv[cpos[s]]
  __syncthreads();
  int* tmp = (int*)wv;  // reuse the work row (n ints fit in n doubles)
  for (int k = vmc_tid(); k < n; k += NT) tmp[k] = W.colsite[q[k]];
  __syncthreads();
  for (int k = vmc_tid(); k < n; k += NT) {
    W.colsite[k] = tmp[k];
    W.cpos[tmp[k]] = k;
  }
  __syncthreads();
  return WST_OK;
}

}  // namespace vmc
