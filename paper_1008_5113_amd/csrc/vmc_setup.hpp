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
    const size_t a0 = aidx(W.W, i, 0);
    int cnt = wave_row(W, rx, ry, rz, W.cpos, W.a_col + a0, W.a_val + a0, W.a_val32 + a0, W.W, ASL);
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
// The pass renumbers the matrix from its current order: the previous
// reorder's result (reo_row/reo_col, without the factorisation's column
// pivots; the identity after creation).  Squared minimum-image distances; ties
// to the first position.  Writes rowperm/rpos and colsite/cpos (reorder order)
// and reo_row/reo_col.
// Two lexicographic minima (smaller value, then smaller index: the rule of
// wg_argmin) reduced over the workgroup together, with one barrier.  buf
// holds 2 * NWAVE doubles and 2 * NWAVE ints; a caller that reduces again
// before a barrier of its own alternates between two such buffers.
VMC_PHASE void wg_argmin2(double& v1, int& i1, double& v2, int& i2, double* buf) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double a = __shfl_xor(v1, o, 64);
    const int ai = __shfl_xor(i1, o, 64);
    if (a < v1 || (a == v1 && ai < i1)) { v1 = a; i1 = ai; }
    const double b = __shfl_xor(v2, o, 64);
    const int bi = __shfl_xor(i2, o, 64);
    if (b < v2 || (b == v2 && bi < i2)) { v2 = b; i2 = bi; }
  }
  int* ib = (int*)(buf + 2 * NWAVE);
  if (lane_id() == 0) {
    buf[wave_id()] = v1;
    buf[NWAVE + wave_id()] = v2;
    ib[wave_id()] = i1;
    ib[NWAVE + wave_id()] = i2;
  }
  __syncthreads();
  v1 = buf[0];
  i1 = ib[0];
  v2 = buf[NWAVE];
  i2 = ib[NWAVE];
  for (int w = 1; w < NWAVE; ++w) {
    const double a = buf[w];
    const int ai = ib[w];
    if (a < v1 || (a == v1 && ai < i1)) { v1 = a; i1 = ai; }
    const double b = buf[NWAVE + w];
    const int bi = ib[NWAVE + w];
    if (b < v2 || (b == v2 && bi < i2)) { v2 = b; i2 = bi; }
  }
}

VMC_PHASE void wg_exclusive_scan(const int* len, int* ptr, int n, Smem& S);

// Lattice cell of a point in [0, L) (a point at L rounds into the last cell).
__device__ inline int lattice_cell(const Walker& W, double x, double y, double z) {
  const int ix = min(max((int)floor(x / W.a), 0), W.lat[0] - 1);
  const int iy = min(max((int)floor(y / W.a), 0), W.lat[1] - 1);
  const int iz = min(max((int)floor(z / W.a), 0), W.lat[2] - 1);
  return ix + W.lat[0] * (iy + W.lat[1] * iz);
}

// Lexicographic (distance, position) minimum update.
__device__ inline void lex_min(double d, int p, double& bd, int& bp) {
  if (d < bd || (d == bd && p < bp)) { bd = d; bp = p; }
}

// scratch (global, scratch_bytes long, free during the reorder) holds the
// particles' cell lists when it is large enough, and the LDS region then also
// holds both inverse permutations: each step first searches the lattice cells
// within one lattice spacing of the particle (orbitals) and of the orbital
// (particles), and only when a search finds nothing closer than that radius
// falls back to the scan of every free position.  The minimum over (distance,
// position) pairs is the same either way: every free site or particle within
// the radius lies in the cells searched, and any other is farther.  The cell
// search keeps a step's cost flat in n (Section 3.1 notes that an O(n)
// reorder is possible for sparse Slater matrices); while few positions are
// free, the scan is cheaper and is used instead.
VMC_PHASE void wg_reorder(const Walker& W, Smem& S, void* scratch, size_t scratch_bytes) {
  constexpr int RU = 2;
  const int n = W.n;
  const size_t an = align_up((size_t)n, 8);
  short* rp = (short*)S.A;
  short* cp = rp + an;
  short* rposl = cp + an;
  short* cposl = rposl + an;
  const int L0 = W.lat[0], L1 = W.lat[1], L2 = W.lat[2], nb = W.nb;
  const int ncell = L0 * L1 * L2;
  const bool cells = (size_t)((char*)S.red - S.A) >= 4 * an * sizeof(short) && ncell * nb == n &&
                     scratch != nullptr && scratch_bytes >= ((size_t)2 * ncell + 1 + n) * sizeof(int);
  int* ccount = (int*)scratch;
  int* cstart = ccount + ncell;
  int* citem = cstart + ncell + 1;
  for (int k = vmc_tid(); k < n; k += NT) {
    rp[k] = (short)W.reo_row[k];
    cp[k] = (short)W.reo_col[k];
  }
  __syncthreads();
  if (cells) {
    for (int k = vmc_tid(); k < n; k += NT) {
      rposl[rp[k]] = (short)k;
      cposl[cp[k]] = (short)k;
    }
    for (int c = vmc_tid(); c < ncell; c += NT) ccount[c] = 0;
    __threadfence_block();
    __syncthreads();
    for (int p = vmc_tid(); p < n; p += NT)
      atomicAdd(&ccount[lattice_cell(W, W.pos[3 * p], W.pos[3 * p + 1], W.pos[3 * p + 2])], 1);
    __threadfence_block();
    __syncthreads();
    wg_exclusive_scan(ccount, cstart, ncell, S);
    for (int c = vmc_tid(); c < ncell; c += NT) ccount[c] = 0;
    __threadfence_block();
    __syncthreads();
    for (int p = vmc_tid(); p < n; p += NT) {
      const int c = lattice_cell(W, W.pos[3 * p], W.pos[3 * p + 1], W.pos[3 * p + 2]);
      citem[cstart[c] + atomicAdd(&ccount[c], 1)] = p;
    }
    __threadfence_block();
    __syncthreads();
  }
  const double RL = W.a;
  // below RL^2 by far more than the rounding of a squared distance
  const double cert = 0.999 * RL * RL;
  int rb = 0;
  for (int i = 0; i < n - 1; ++i) {
    const int pi = rp[i];
    const double rx = W.pos[3 * pi], ry = W.pos[3 * pi + 1], rz = W.pos[3 * pi + 2];
    const double* Zi = W.sites + 3 * (size_t)cp[i];
    double bo = INFINITY, bq = INFINITY;
    int jo = 0x7fffffff, kq = 0x7fffffff;
    bool local = false;
    // the scan costs one gather round per RU * NT free positions, the cell
    // search about three (measured): cells only while many are free
    if (cells && n - i > 6 * NT) {
      // free orbitals in the cells around the particle (the row builder's
      // enumeration, for radius RL)
      int lox, cx, loy, cy, loz, cz;
      axis_range(rx - W.bmax[0], RL + W.margin, W.a, L0, lox, cx);
      axis_range(ry - W.bmax[1], RL + W.margin, W.a, L1, loy, cy);
      axis_range(rz - W.bmax[2], RL + W.margin, W.a, L2, loz, cz);
      const int tot = cx * cy * cz * nb;
      for (int t = vmc_tid(); t < tot; t += NT) {
        const int b = t % nb, cell = t / nb;
        const int ix = wrap_index(lox + cell % cx, L0);
        const int iy = wrap_index(loy + (cell / cx) % cy, L1);
        const int iz = wrap_index(loz + cell / (cx * cy), L2);
        const int site = b + nb * (ix + L0 * (iy + L1 * iz));
        const int ps = cposl[site];
        if (ps >= i) {
          double dx;
          lex_min(dist2_xyz(rx, ry, rz, W.sites + 3 * (size_t)site, W.box, &dx), ps, bo, jo);
        }
      }
      // free particles in the cells around the orbital at i
      axis_range(Zi[0], RL, W.a, L0, lox, cx);
      axis_range(Zi[1], RL, W.a, L1, loy, cy);
      axis_range(Zi[2], RL, W.a, L2, loz, cz);
      const int ptot = cx * cy * cz;
      for (int t = vmc_tid(); t < ptot; t += NT) {
        const int ix = wrap_index(lox + t % cx, L0);
        const int iy = wrap_index(loy + (t / cx) % cy, L1);
        const int iz = wrap_index(loz + t / (cx * cy), L2);
        const int c = ix + L0 * (iy + L1 * iz);
        for (int e = cstart[c]; e < cstart[c + 1]; ++e) {
          const int p = citem[e];
          const int pp = rposl[p];
          if (pp >= i) {
            double dx;
            lex_min(dist2_xyz(W.pos[3 * p], W.pos[3 * p + 1], W.pos[3 * p + 2], Zi, W.box, &dx), pp, bq, kq);
          }
        }
      }
      wg_argmin2(bo, jo, bq, kq, S.red + (rb++ & 1) * 4 * NWAVE);
      local = bo < cert && (jo != i || bq < cert);
    }
    if (!local) {
      // Both searches of position i scan positions i..n-1 in one pass: the
      // closest orbital to the particle at i and, for the case that this
      // orbital already is at i, the closest particle to the orbital at i
      // (nothing moves between the two searches, so the second one's answer
      // is the one the sequential order would find).
      bo = bq = INFINITY;
      jo = kq = 0x7fffffff;
      // RU positions per thread at a time: their coordinates are gathered
      // before any is compared, so the loads overlap; the comparisons then
      // run in ascending position, as a plain strided loop would
      for (int t0 = i + vmc_tid(); t0 < n; t0 += RU * NT) {
        double cs[RU][3], cr[RU][3];
#pragma unroll
        for (int q = 0; q < RU; ++q) {
          const int t = t0 + q * NT;
          const int tc = t < n ? t : i;
          const double* Z = W.sites + 3 * (size_t)cp[tc];
          const double* R = W.pos + 3 * (size_t)rp[tc];
          cs[q][0] = Z[0];
          cs[q][1] = Z[1];
          cs[q][2] = Z[2];
          cr[q][0] = R[0];
          cr[q][1] = R[1];
          cr[q][2] = R[2];
        }
#pragma unroll
        for (int q = 0; q < RU; ++q) {
          const int t = t0 + q * NT;
          double dx;
          const double d1 = dist2_xyz(rx, ry, rz, cs[q], W.box, &dx);
          if (t < n && d1 < bo) { bo = d1; jo = t; }
          const double d2 = dist2_xyz(cr[q][0], cr[q][1], cr[q][2], Zi, W.box, &dx);
          if (t < n && d2 < bq) { bq = d2; kq = t; }
        }
      }
      wg_argmin2(bo, jo, bq, kq, S.red + (rb++ & 1) * 4 * NWAVE);
    }
    // every thread's search is done once the reduction's barrier is passed,
    // so thread 0 may swap right away; the decision is the same everywhere
    if (jo != i) {
      if (vmc_tid() == 0) {
        const short a = cp[i], b = cp[jo];
        cp[i] = b;
        cp[jo] = a;
        if (cells) {
          cposl[b] = (short)i;
          cposl[a] = (short)jo;
        }
      }
      __syncthreads();
    } else if (kq != i) {
      if (vmc_tid() == 0) {
        const short a = rp[i], b = rp[kq];
        rp[i] = b;
        rp[kq] = a;
        if (cells) {
          rposl[b] = (short)i;
          rposl[a] = (short)kq;
        }
      }
      __syncthreads();
    }
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

// Rows are factored concurrently by ILU_R waves (row i by wave i mod ILU_R),
// each with its own sparse work row.  The row algorithm is exactly the serial
// one; only the waiting differs:
// - rows finish in order, and FIN (LDS) counts the finished rows.  Positions
//   below FIN hold their final column labels, because a pivot of row j only
//   swaps positions >= j;
// - a row eliminates, in increasing order, the candidates whose positions are
//   already final.  When it runs out, it waits for FIN to advance and scans
//   the newly final positions for labels present in its work row;
// - the drop, fill-limit and pivot decisions of row i run once all rows
//   before i have finished, on the same data the serial algorithm would see.
constexpr int CAND_DONE = 32767;
constexpr int IC_FIN = 24;
constexpr int IC_FAIL = 25;
// Row-loop status only: a work table of the configuration overflowed (or the
// wave stopped waiting because another one failed).  It never leaves wg_ilutp.
constexpr int WST_ILU_TABLE = 8;
constexpr int SPIN_CAP = 1 << 22;  // bound on every wait; exceeding it is an error

__device__ inline int lds_acquire(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One wave's work row and candidate table.
struct IluWave {
  int* hent;      // hash: (label << 16) | slot, -1 empty
  short* slab;    // slot -> label
  double* sval;   // slot -> value
  short* cpos;    // candidate position (CAND_DONE once eliminated)
  short* cslot;   // work-row slot of the candidate's label
  short* clen;    // length of U row cpos
  double* cdiag;  // u_kk of row cpos
  short* lk;      // kept multipliers: positions
  double* lv;     //                   values
  int hmask, hshift;
};

__device__ inline IluWave ilu_wave_carve(char* base, const IluCfg& C) {
  IluWave R;
  R.hent = (int*)base;     base += align_up((size_t)C.hs * 4, 16);
  R.slab = (short*)base;   base += align_up((size_t)C.nz * 2, 16);
  R.sval = (double*)base;  base += (size_t)C.nz * 8;
  R.cpos = (short*)base;   base += align_up((size_t)C.c * 2, 16);
  R.cslot = (short*)base;  base += align_up((size_t)C.c * 2, 16);
  R.clen = (short*)base;   base += align_up((size_t)C.c * 2, 16);
  R.cdiag = (double*)base; base += (size_t)C.c * 8;
  R.lk = (short*)base;     base += align_up((size_t)C.l * 2, 16);
  R.lv = (double*)base;
  R.hmask = C.hs - 1;
  R.hshift = C.hshift;
  return R;
}

__device__ inline int ilu_hash(const IluWave& R, int c) {
  return (int)(((unsigned)c * 2654435761u) >> R.hshift);
}

// Slot of label c in the work row, or -1.
__device__ inline int ilu_find(const IluWave& R, int c) {
  int h = ilu_hash(R, c);
  while (true) {
    const int e = R.hent[h];
    if (e == -1) return -1;
    if ((e >> 16) == c) return e & 0xFFFF;
    h = (h + 1) & R.hmask;
  }
}

__device__ inline void ilu_insert(const IluWave& R, int c, int slot) {
  int h = ilu_hash(R, c);
  while (atomicCAS(&R.hent[h], -1, (c << 16) | slot) != -1) h = (h + 1) & R.hmask;
}

// Drop the eliminated candidates from the table (their order is irrelevant:
// the next candidate is always the smallest position).
__device__ inline int ilu_compact(IluWave& R, int ncand) {
  const int lane = lane_id();
  int w = 0;
  for (int s0 = 0; s0 < ncand; s0 += 64) {
    const int s = s0 + lane;
    int p = CAND_DONE, c = 0, l = 0;
    double d = 0.0;
    if (s < ncand) {
      p = R.cpos[s];
      c = R.cslot[s];
      l = R.clen[s];
      d = R.cdiag[s];
    }
    const bool live = p != CAND_DONE;
    const unsigned long long mask = __ballot(live);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (live) {
      const int t = w + before;
      R.cpos[t] = (short)p;
      R.cslot[t] = (short)c;
      R.clen[t] = (short)l;
      R.cdiag[t] = d;
    }
    w += __popcll(mask);
  }
  return w;
}

// Append the lanes flagged `add` as candidates (position p, its label at
// work-row slot sl), with the diagonal and length of U row p.  Returns the new
// count; a count above cap means the table overflowed.
__device__ inline int ilu_add_cands(const Walker& W, IluWave& R, int ncand, bool add, int p, int sl, int cap) {
  const int lane = lane_id();
  const unsigned long long mask = __ballot(add);
  if (ncand + (int)__popcll(mask) > cap) ncand = ilu_compact(R, ncand);
  const int before = __popcll(mask & ((1ull << lane) - 1ull));
  if (add && ncand + before < cap) {
    const int s = ncand + before;
    R.cpos[s] = (short)p;
    R.cslot[s] = (short)sl;
    R.cdiag[s] = W.u_diag[p];
    R.clen[s] = (short)W.u_len[p];
  }
  wave_sync();  // the new entries are in the table before any lane scans it
  return ncand + __popcll(mask);
}

// The row loop with configuration C over rows [start, end): the factors of
// those rows into L/U (label space), their pivots into q/pinv (which start as
// the identity when start is 0).  Rows finish in order; afterwards S.ic[IC_FIN]
// is the first row not finished.  Returns the OR of the rows' WST_* bits.
VMC_PHASE int ilu_rows(const Walker& W, const DevParams& P, Smem& S, const IluCfg& C, int pfill, short* pinv,
                       short* q, char* base, int start, int end) {
  const int n = W.n;
  const int F = W.F;
  const int wid = wave_id();
  const int nrow = C.r, cap_nz = C.nz, cap_c = C.c, cap_l = C.l;
  IluWave R = ilu_wave_carve(base + (size_t)(wid < nrow ? wid : 0) * ilu_wave_bytes(C), C);

  if (start == 0)
    for (int k = vmc_tid(); k < n; k += NT) {
      pinv[k] = (short)k;
      q[k] = (short)k;
    }
  if (wid < nrow)
    for (int h = lane_id(); h <= R.hmask; h += 64) R.hent[h] = -1;
  if (vmc_tid() == 0) {
    S.ic[IC_FIN] = start;
    S.ic[IC_FAIL] = 0;
  }
  __syncthreads();

  if (wid < nrow) {
    const int lane = lane_id();
    const double droptol = P.droptol, permtol = P.permtol;
    const bool mean_scale = P.ilu_drop_norm == 1;
    int status = WST_OK;
    for (int i = start + wid; i < end; i += nrow) {
      if (lds_acquire(&S.ic[IC_FAIL])) break;
      int known = min(lds_acquire(&S.ic[IC_FIN]), i);  // positions < known are final
      // 1. load row i into the work row; entries at final positions left of
      //    the diagonal are the first candidates
      const int len = W.a_len[i];
      if (len > cap_nz) { status = WST_ILU_TABLE; break; }
      double nrm = 0.0;
      int ncand = 0;
      for (int e0 = 0; e0 < len; e0 += 64) {
        const int e = e0 + lane;
        bool cand = false;
        int c = 0, k = 0;
        if (e < len) {
          c = W.a_col[aidx(W.W, i, e)];
          const double v = W.a_val[aidx(W.W, i, e)];
          R.slab[e] = (short)c;
          R.sval[e] = v;
          ilu_insert(R, c, e);
          nrm += mean_scale ? fabs(v) : v * v;
          k = pinv[c];
          cand = k < known;
        }
        ncand = ilu_add_cands(W, R, ncand, cand, k, e, cap_c);
      }
      if (ncand > cap_c) { status = WST_ILU_TABLE; break; }
      nrm = wave_sum(nrm);
      // drop scale: the row's 2-norm, or its mean magnitude (SPARSKIT's ILUTP)
      const double tau = droptol * (mean_scale ? nrm / (double)len : sqrt(nrm));
      int nz = len;
      int lcount = 0;
      bool lfull = false;  // multipliers were kept beyond the table
      // 2. eliminate in increasing position order
      while (true) {
        // each lane keeps the fields of its smallest candidate, so the
        // winner's come back by readlane instead of further LDS round trips
        int best = CAND_DONE, bslot = -1, bsk = 0, bul = 0;
        double bdiag = 1.0;
        for (int s = lane; s < ncand; s += 64) {
          const int p = R.cpos[s];
          const int sl = R.cslot[s];
          const int cl = R.clen[s];
          const double dg = R.cdiag[s];
          if (p < best) { best = p; bslot = s; bsk = sl; bul = cl; bdiag = dg; }
        }
        const int bmin = wave_mini(best);
        if (bmin == CAND_DONE) {
          if (known >= i) break;
          // wait for more rows to finish, then scan the newly final positions
          int f = known, spins = 0;
          while (true) {
            f = lds_acquire(&S.ic[IC_FIN]);
            if (f > known) break;
            if (lds_acquire(&S.ic[IC_FAIL]) || ++spins > SPIN_CAP) { status = WST_ILU_TABLE; break; }
          }
          if (status != WST_OK) break;
          f = min(f, i);
          for (int p0 = known; p0 < f; p0 += 64) {
            const int p = p0 + lane;
            bool add = false;
            int sl = 0;
            if (p < f) {
              sl = ilu_find(R, q[p]);
              add = sl >= 0;
            }
            ncand = ilu_add_cands(W, R, ncand, add, p, sl, cap_c);
          }
          if (ncand > cap_c) { status = WST_ILU_TABLE; break; }
          known = f;
          continue;
        }
        {
          // positions are distinct, so exactly one lane holds the minimum
          const unsigned long long who = __ballot(best == bmin);
          const int wl = __ffsll((long long)who) - 1;
          bslot = readlane_i(bslot, wl);
          bsk = readlane_i(bsk, wl);
          bul = readlane_i(bul, wl);
          bdiag = readlane_t(bdiag, wl);
          best = bmin;
        }
        const int sk = bsk;
        const double lik = R.sval[sk] / bdiag;
        const int ul = bul;
        wave_sync();  // the candidate's entries are read before any lane updates the row
        if (lane == 0) R.cpos[bslot] = (short)CAND_DONE;
        if (fabs(lik) < tau) continue;
        if (lcount < cap_l) {
          if (lane == 0) { R.lk[lcount] = (short)best; R.lv[lcount] = lik; }
          ++lcount;
        } else {
          // A full table keeps the cap_l multipliers that rank first (larger
          // magnitude, then smaller position).  The row stores only its
          // nL0 + p first, so none of those is lost while cap_l >= nL0 + p,
          // which the L part checks.  The new multiplier replaces the table's
          // last-ranked one if it ranks before it.
          double wa = 1e308;
          int wp = -1, wi = -1;
          for (int f = lane; f < cap_l; f += 64) {
            const double a3 = fabs(R.lv[f]);
            const int p3 = R.lk[f];
            if (a3 < wa || (a3 == wa && p3 > wp)) { wa = a3; wp = p3; wi = f; }
          }
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            const double oa = __shfl_xor(wa, o, 64);
            const int op = __shfl_xor(wp, o, 64);
            const int oi = __shfl_xor(wi, o, 64);
            if (oa < wa || (oa == wa && op > wp)) { wa = oa; wp = op; wi = oi; }
          }
          const double al = fabs(lik);
          wave_sync();  // every lane has read the table before lane 0 replaces an entry
          if (lane == 0 && (al > wa || (al == wa && best < wp))) {
            R.lk[wi] = (short)best;
            R.lv[wi] = lik;
          }
          lfull = true;
        }
        for (int e0 = 0; e0 < ul; e0 += 64) {
          const int e = e0 + lane;
          bool isnew = false, cand = false;
          int c2 = 0, k2 = 0;
          double v2 = 0.0;
          if (e < ul) {
            c2 = W.u_col[(size_t)best * F + e];
            v2 = W.u_val[(size_t)best * F + e];
            // the columns of one U row are distinct: no two lanes share a label
            const int s2 = ilu_find(R, c2);
            if (s2 >= 0) R.sval[s2] -= lik * v2;
            else isnew = true;
          }
          const unsigned long long mask = __ballot(isnew);
          const int before = __popcll(mask & ((1ull << lane) - 1ull));
          int s2 = 0;
          if (isnew && nz + before < cap_nz) {
            s2 = nz + before;
            R.slab[s2] = (short)c2;
            R.sval[s2] = -lik * v2;
            ilu_insert(R, c2, s2);
            k2 = pinv[c2];
            cand = k2 < known;
          }
          nz += __popcll(mask);
          if (nz > cap_nz) break;
          ncand = ilu_add_cands(W, R, ncand, cand, k2, s2, cap_c);
        }
        if (nz > cap_nz || ncand > cap_c) { status = WST_ILU_TABLE; break; }
      }
      if (status != WST_OK) break;

      // 3. U part (rows < i have all finished: positions are final).  Drop
      //    below tau (never the current diagonal column), keep the nU0 + p
      //    largest, where nU0/nL0 count the row's original entries right/left
      //    of the diagonal.
      int nl0 = 0, nu0 = 0;
      for (int e = lane; e < len; e += 64) {
        const int k = pinv[R.slab[e]];
        nl0 += (k < i);
        nu0 += (k > i);
      }
      nl0 = wave_sumi(nl0);
      nu0 = wave_sumi(nu0);
      const int cd = q[i];
      const int sd = ilu_find(R, cd);
      const bool cd_present = sd >= 0;
      const int ucap = nu0 + pfill;
      const int lcap = nl0 + pfill;
      int ucnt = 0;
      for (int e = lane; e < nz; e += 64) {
        const int c = R.slab[e];
        if (c != cd && pinv[c] >= i && fabs(R.sval[e]) >= tau) ++ucnt;
      }
      ucnt = wave_sumi(ucnt);
      double vmax = -1.0, vmaxv = 0.0;
      int cmax_pos = 0x7fffffff;
      const double vd = cd_present ? R.sval[sd] : 0.0;
      if (cd_present) { vmax = fabs(vd); vmaxv = vd; cmax_pos = i; }
      int uwrite = 0;
      int* out_col = W.u_col + (size_t)i * F;
      double* out_val = W.u_val + (size_t)i * F;
      for (int e0 = 0; e0 < nz; e0 += 64) {
        const int e = e0 + lane;
        bool keep = false;
        int c = 0;
        double v = 0.0;
        if (e < nz) {
          c = R.slab[e];
          v = R.sval[e];
          if (c != cd && pinv[c] >= i && fabs(v) >= tau) {
            keep = true;
            if (ucnt > ucap) {
              const double av = fabs(v);
              const int kp = pinv[c];
              int rank = 0;
              for (int f = 0; f < nz; ++f) {
                const int c3 = R.slab[f];
                if (c3 == cd || pinv[c3] < i) continue;
                const double a3 = fabs(R.sval[f]);
                if (a3 < tau) continue;
                if (a3 > av || (a3 == av && pinv[c3] < kp)) ++rank;
              }
              keep = rank < ucap;
            }
          }
        }
        const unsigned long long mask = __ballot(keep);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) {
          const int o = uwrite + before;
          if (o < F) { out_col[o] = c; out_val[o] = v; }
          const double av = fabs(v);
          const int kp = pinv[c];
          if (av > vmax || (av == vmax && kp < cmax_pos)) { vmax = av; vmaxv = v; cmax_pos = kp; }
        }
        uwrite += __popcll(mask);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(vmax, o, 64);
        const double ovv = __shfl_xor(vmaxv, o, 64);
        const int op = __shfl_xor(cmax_pos, o, 64);
        if (ov > vmax || (ov == vmax && op < cmax_pos)) { vmax = ov; vmaxv = ovv; cmax_pos = op; }
      }
      if (uwrite > F - 1) { status = WST_CAPACITY; break; }
      if (!(vmax > 0.0)) { status = WST_SINGULAR; break; }
      // 4. pivot: swap the diagonal column with the largest entry's column
      double dval = vd;
      if (permtol * vmax > fabs(vd) && cmax_pos != i) {
        const int cm = q[cmax_pos];
        dval = vmaxv;
        wave_sync();  // every lane reads the new diagonal's label before lane 0 swaps it
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
      // 5. L part: keep the lcap largest multipliers
      if (lfull && lcap > cap_l) { status = WST_ILU_TABLE; break; }
      int lwrite = 0;
      int* lcol = W.l_col + (size_t)i * F;
      double* lval = W.l_val + (size_t)i * F;
      for (int e0 = 0; e0 < lcount; e0 += 64) {
        const int e = e0 + lane;
        bool keep = false;
        if (e < lcount) {
          keep = true;
          if (lcount > lcap) {
            const double av = fabs(R.lv[e]);
            const int kp = R.lk[e];
            int rank = 0;
            for (int f = 0; f < lcount; ++f) {
              const double a3 = fabs(R.lv[f]);
              if (a3 > av || (a3 == av && R.lk[f] < kp)) ++rank;
            }
            keep = rank < lcap;
          }
        }
        const unsigned long long mask = __ballot(keep);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) {
          const int o = lwrite + before;
          if (o < F) { lcol[o] = R.lk[e]; lval[o] = R.lv[e]; }
        }
        lwrite += __popcll(mask);
      }
      if (lwrite > F) { status = WST_CAPACITY; break; }
      if (lane == 0) {
        W.u_len[i] = uwrite;
        W.u_diag[i] = dval;
        W.l_len[i] = lwrite;
      }
      // 6. clear the work row, then publish row i as finished
      for (int h = lane; h <= R.hmask; h += 64) R.hent[h] = -1;
      __threadfence_block();
      if (lane == 0) lds_release(&S.ic[IC_FIN], i + 1);
    }
    if (status != WST_OK && lane == 0) atomicOr(&S.ic[IC_FAIL], status);
  }
  __syncthreads();
  const int status = S.ic[IC_FAIL];
  __syncthreads();
  return status;
}

VMC_PHASE int wg_ilutp(const Walker& W, const DevParams& P, Smem& S) {
  const int n = W.n;
  const int F = W.F;
  const int pfill = ilutp_row_cap_extra(W, P, S);
  char* base = S.A;
  short* pinv = (short*)base;               base += align_up((size_t)n * 2, 16);
  short* q = (short*)base;                  base += align_up((size_t)n * 2, 16);
  // The fast configuration runs until a row overflows its tables.  Rows finish
  // in order and a row changes q/pinv, L or U only when it finishes, so the
  // rows before the first unfinished one are final: the full configuration
  // takes over there for ILU_FALLBACK_ROWS rows (a window that holds every row
  // that was in flight), then the fast one resumes.  The arithmetic of every
  // row is the same in both, so the factors are too.
  int status = WST_OK;
  if (P.ilu_fast.r > 0) {
    int start = 0;
    while (true) {
      status = ilu_rows(W, P, S, P.ilu_fast, pfill, pinv, q, base, start, n);
      if (status != WST_ILU_TABLE) break;
      const int fin = S.ic[IC_FIN];
      __syncthreads();
      if (S.ilu_retries && vmc_tid() == 0) *S.ilu_retries += 1;
      const int stop = min(n, fin + ILU_FALLBACK_ROWS);
      status = ilu_rows(W, P, S, P.ilu, pfill, pinv, q, base, fin, stop);
      if (status != WST_OK || stop == n) break;
      start = stop;
    }
  } else {
    status = ilu_rows(W, P, S, P.ilu, pfill, pinv, q, base, 0, n);
  }
  if (status & WST_ILU_TABLE) status = (status & ~WST_ILU_TABLE) | WST_CAPACITY;
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
    unsigned short* ac = W.a_col + aidx(W.W, i, 0);
    for (int e = 0; e < al; ++e) ac[(size_t)e * ASL] = (unsigned short)pinv[ac[(size_t)e * ASL]];
    W.ilu_q[i] = q[i];
  }
  __threadfence_block();
  __syncthreads();
  wg_pack_factors(W, S);
  // colsite_new[k] = colsite_old[q[k]]; cpos[s] = pinv[cpos[s]]
  __syncthreads();
  int* tmp = (int*)base;  // the work rows' bytes (they hold at least n ints)
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
