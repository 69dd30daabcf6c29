// Internal types of the vmcdet library (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vmcdet.h"

namespace vmc {

// Pointer members of the walker table point to device global memory.  The
// device compilation pass says so explicitly (address space 1), so loads
// through them become global_load instructions, which only wait on the vector
// memory counter, instead of FLAT loads, which also hold the LDS counter and
// would make every LDS wait and barrier drain the prefetched loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define GAS __attribute__((address_space(1)))
#else
#define GAS
#endif

constexpr int NT = 512;        // threads per walker workgroup
constexpr int NWAVE = NT / 64;
constexpr int BLK = 64;        // rows per triangular-solve block (one lane per row)
// In-block coefficient tile of the triangular solves: column-major with a
// column stride of BLK + 1 (the 8 threads of a row scatter into 8 different
// banks), plus one spare row that masked-off scatters write to.
constexpr int DSTR = BLK + 1;
constexpr int DTILE = BLK * DSTR + BLK;
constexpr int MAXIT = 64;      // largest supported GMRES iteration count

constexpr int MMAX_CAP = 256;  // largest supported m_max

// In-kernel phase timers (wall-clock ticks, accumulated by thread 0).
enum Phase {
  PH_PREPARE = 0, PH_LSOLVE, PH_USOLVE, PH_UPDATES, PH_SPMV, PH_ORTHO, PH_SOLUTION, PH_RESID,
  PH_ACCEPT, PH_REFACTOR, PH_REORDER, PH_STEP, PH_COUNT
};

// Walker-level error codes stored on the device (mapped to vmc_status on the host).
constexpr int WST_OK = 0;
constexpr int WST_CAPACITY = 1;
constexpr int WST_SINGULAR = 2;
constexpr int WST_NOCONV = 4;

// Caller errors of the per-move calls in device-pointer mode (reported and
// cleared by vmc_sync; they do not stop the walker).
constexpr int CERR_NOPENDING = 1;   // accept without a pending ratio
constexpr int CERR_ZERO_RATIO = 2;  // forced acceptance of a zero or non-finite ratio

// One ILUTP configuration: r rows factored concurrently (one wave each), each
// wave with hs hash slots, a work row of nz entries, c candidates and l
// multipliers; hshift = 32 - log2(hs).
struct IluCfg {
  int r, hs, hshift, nz, c, l;
};

struct DevParams {
  int precision;
  int maxit;
  double rtol;
  double droptol, permtol;
  int lfil;
  int m_max;
  double n_thresh, iter_factor;
  int iter_min_solves;
  double inner_rtol, refine_tol;
  int refine_maxit;
  double step;
  int force_reorder_every;
  // ILUTP configurations: a factorisation runs with ilu_fast (more rows in
  // flight, smaller tables; r = 0: none) and is redone with ilu when a row
  // overflows those tables.  Both give the same factors.
  IluCfg ilu, ilu_fast;
  int ilu_drop_norm;          // 0: tau = droptol*||a_i||_2; 1: droptol*||a_i||_1/nnz(a_i)
  int test_knobs;             // VMC_TEST_* bits
  int plain_stop;             // ratio solves stop at their tolerance (no ratio-relative target)
};

// Everything the device needs about one walker.  Arrays are per walker; the
// Slater matrix is stored by row position with capacity W per row, the ILU
// factors with capacity F per row.  Column indices of A, L, U, the update
// vectors and all Krylov vectors live in the same column numbering (the
// current "column positions"), so the preconditioner's column permutation is
// folded into that numbering at every factorisation.
struct Walker {
  // sizes
  int n, W, F, UC;            // n, Slater row cap, factor row cap, update-vector cap
  int lat[3];
  int kind;
  int nb;                     // sites per lattice cell
  double box[3], a, margin, cutoff, p_scale, p_sigma;
  double bmax[3];             // largest in-cell site offset per axis (length)
  unsigned long long seed;

  // system (by site id) and positions (by particle id)
  const double GAS* sites;        // n*3
  const double GAS* sigma;        // n
  double GAS* pos;                // n*3

  // orderings
  int GAS* rowperm;               // row position -> particle
  int GAS* rpos;                  // particle -> row position
  int GAS* cpos;                  // site -> column position
  int GAS* colsite;               // column position -> site
  int GAS* reo_row;               // last geometric reorder (particle per position)
  int GAS* reo_col;               // last geometric reorder (site per position)

  // Slater matrix
  int GAS* a_len;
  // A in slices of 64 rows: entry e of row i at aidx(W, i, e) (see there)
  unsigned short GAS* a_col;
  double GAS* a_val;
  float GAS* a_val32;

  // ILU factors (column positions); U stored off-diagonal, scaled copies for the solve
  int GAS* l_len;
  int GAS* l_col;
  double GAS* l_val;
  int GAS* u_len;
  int GAS* u_col;
  double GAS* u_val;              // unscaled off-diagonal U
  double GAS* u_diag;
  double GAS* u_dinv;
  float GAS* u_dinv32;
  // compact CSR copies for the triangular solves, rebuilt after every
  // factorisation; 16-bit column positions
  int GAS* lp;                    // n+1
  unsigned short GAS* lc;
  double GAS* lv64;
  float GAS* lv32;
  int GAS* up;                    // n+1
  unsigned short GAS* uc;
  double GAS* uv64;               // D^{-1} U off-diagonal
  float GAS* uv32;
  int GAS* ilu_q;                 // last ILUTP column permutation (labels before it)

  // rank-one updates M <- (I - zhat u^T) M, oldest first
  double GAS* Z64;                // m_max * n
  float GAS* Z32;
  int GAS* up_len;                // m_max
  int GAS* up_col;                // m_max * UC
  double GAS* up_val;
  float GAS* up_val32;
  double GAS* T;                  // m_max * m_max: T[s*m_max+t] = u_s^T zhat_t (t < s)

  // Krylov workspace (typed by the solve precision)
  void GAS* V;                    // (maxit+1) * n
  void GAS* Xp;                   // maxit * n : preconditioned basis vectors
  void GAS* wv;                   // n
  double GAS* zvec;               // n : solution z (FP64 accumulation)
  double GAS* rvec;               // n : FP64 residual (mixed)

  // pending move
  int GAS* new_col;               // W
  double GAS* new_val;            // W
  int GAS* pu_col;                // UC
  double GAS* pu_val;             // UC
};

// Slot of entry e of row i of A: rows are grouped in slices of 64, and a
// slice stores entry e of its 64 rows together (rows of a slice at
// consecutive addresses), so a wave reading one entry of each of 64 rows
// reads one contiguous run.  A slice holds W entries per row.
constexpr int ASL = 64;
__host__ __device__ inline size_t aidx(int W, int i, int e) {
  return ((size_t)(i / ASL) * (size_t)W + (size_t)e) * ASL + (size_t)(i % ASL);
}
__host__ __device__ inline size_t a_rows_padded(int n) { return ((size_t)n + ASL - 1) / ASL * ASL; }

// Mutable per-walker scalars, kept apart from the (read-mostly) pointer table.
struct WalkerState {
  long long g;                // steps taken (Philox counter)
  int m;                      // stored updates
  int status;                 // WST_* bits
  int pend_valid, pend_p, pend_i, pend_newlen, pend_ulen, pend_flags, pend_iters;
  int pend_passes, pend_inner;
  int call_err;               // CERR_* bits of device-pointer calls since the last vmc_sync
  double pend_newpos[3];
  double pend_ratio, pend_uacc, pend_N, pend_resid;
  double avg_iters;           // running mean of first-solve iteration counts
  long long avg_count;
  // counters
  long long st_steps, st_acc, st_solves, st_iters, st_reorders, st_refactors, st_nonconv;
  long long st_inner, st_refine, st_msum;
  double st_maxN, st_sumN;
  // cost balance (Section 3.2): stored-update entries streamed by the
  // preconditioner applications since the last factorisation, and the
  // threshold at which a new factorisation is cheaper than going on
  double upd_entries;
  double refactor_cost;
  double st_upd_entries;
  unsigned long long ph[PH_COUNT];
  unsigned long long ilu_retries;  // ILUTP fallbacks to the full configuration
};

}  // namespace vmc
