/*
 * vmcdet — determinant ratios of consecutive sparse Slater matrices for
 * Variational Monte Carlo on insulators, on AMD MI355X (gfx950).
 *
 * Method: Ahuja, Clark, de Sturler, Ceperley, Kim, "Improved Scaling for
 * Quantum Monte Carlo on Insulators" (arXiv 1008.5113).  Each Metropolis step
 * moves one particle i; the Slater matrix changes by one row,
 * A' = A + e_i u^T (eqs. (MatrixUpdate_1), (matrixUpdate2)), and the move is
 * accepted with probability |det A'/det A|^2 = |1 + u^T A^{-1} e_i|^2
 * (eq. (detRatioEq)).  The library obtains z = A^{-1} e_i with
 * right-preconditioned full GMRES (Section 3.2, eq. (precondSystem)), an ILUTP
 * preconditioner A Q ~ L U (eq. (ilu)) that is kept across steps by the
 * rank-one updates M_{k+1} = (I - zhat u^T) M_k (eqs. (finalMk0), (mkp1),
 * (finalMkm)), the geometric particle/orbital reordering (Section 3.1) and
 * the effective-stability monitor N (eq. (stabilityVecEq)) with the reorder
 * triggers of Section 4.
 *
 * Conventions
 * - Every entry point returns a vmc_status: 0 on success, a negative code on
 *   failure (see VMC_E*); vmc_last_error() returns a message for the context.
 *   No C++ exception crosses this interface.
 * - A context owns all device memory it allocates; host arrays passed in are
 *   copied and stay owned by the caller.
 * - Work is issued on the HIP stream given to vmc_create (NULL = default
 *   stream).  Calls that write host outputs synchronise that stream before
 *   returning; vmc_run_steps with a device log pointer is asynchronous.
 * - A context is not thread-safe; one context per stream.
 * - Walker lists (int32 indices into the context's walkers) may not repeat a
 *   walker: VMC_EINVAL.  NULL means every walker (count ignored).
 * - Walker w's state: particle positions, the Slater matrix stored by row
 *   positions (a permutation of particles) and column positions (a
 *   permutation of orbitals), the current ILUTP factors and the list of
 *   rank-one updates.  Ratios are independent of the permutations because a
 *   simultaneous row and column permutation cancels in det A'/det A.
 */
#ifndef VMCDET_H
#define VMCDET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vmc_status;

#define VMC_OK 0
#define VMC_EINVAL (-1)     /* invalid argument (sizes, NULL pointers, ranges) */
#define VMC_ENOMEM (-2)     /* device or host allocation failed */
#define VMC_EHIP (-3)       /* HIP runtime error; message in vmc_last_error */
#define VMC_ENOCONV (-4)    /* GMRES did not converge even after reorder + refactor */
#define VMC_ESINGULAR (-5)  /* zero pivot in ILUTP that reordering did not remove */
#define VMC_ECAPACITY (-6)  /* a Slater row or an ILUTP work row exceeded its capacity */
#define VMC_ESTATE (-7)     /* call out of order (e.g. accept without a pending ratio) */

#define VMC_PREC_FP64 0     /* FP64 everywhere */
#define VMC_PREC_MIXED 1    /* FP32 SpMV/factors/Krylov, FP64 residual, ratio, monitor */

#define VMC_ORB_GAUSS 0     /* phi_j(r) = exp(-|d|^2 / (2 sigma_j^2)) */
#define VMC_ORB_GAUSS_PX 1  /* + p_scale * d_x * exp(-|d|^2 / (2 p_sigma^2)) */

/* Step-record flag bits */
#define VMC_FLAG_ACCEPTED 1
#define VMC_FLAG_REORDERED 2     /* a trigger fired: reorder + refactor + re-solve */
#define VMC_FLAG_REFACTORED 4    /* periodic refactor after m_max stored updates */
#define VMC_FLAG_CONVERGED 8     /* the final solve met its tolerance */
#define VMC_FLAG_SINGULAR 16
#define VMC_FLAG_CAPACITY 32
/* Which reorder trigger of Section 4 fired (set together with VMC_FLAG_REORDERED) */
#define VMC_FLAG_TRIG_N 64         /* effective stability N above n_thresh */
#define VMC_FLAG_TRIG_NOCONV 128   /* the solve missed its tolerance within gmres_maxit
                                      (mixed: the first inner solve, or the refinement) */
#define VMC_FLAG_TRIG_ITERS 256    /* iterations >= iter_factor * running average */
#define VMC_FLAG_TRIG_FORCED 512   /* force_reorder_every test knob */
#define VMC_FLAG_NOCONV 1024       /* not converged even after reorder + refactor: the walker
                                      stops with VMC_ENOCONV */

/* Solver and chain parameters.  Zero-initialise and call vmc_default_params. */
typedef struct vmc_params {
  int32_t precision;        /* VMC_PREC_FP64 or VMC_PREC_MIXED */
  int32_t gmres_maxit;      /* full GMRES, no restart (Section 4: 40); <= 64 */
  double gmres_rtol;        /* FP64 path: stop when ||r|| <= rtol * ||b|| */
  double droptol;           /* ILUTP relative drop tolerance (see ilu_drop_norm) */
  double permtol;           /* ILUTP: swap columns when permtol*|max| > |diag| */
  int32_t lfil;             /* extra fill per L row and per U row; < 0: ceil(nnz/(2n)) */
  int32_t m_max;            /* stored rank-one updates before a refactor (>= 1) */
  double n_thresh;          /* reorder when the effective stability N exceeds this */
  double iter_factor;       /* reorder when iterations >= factor * running average */
  int32_t iter_min_solves;  /* solves before the iteration average is used */
  double inner_rtol;        /* mixed: tolerance of the first FP32 solve; a correction
                               solve stops at max(inner_rtol, half the reduction the
                               refinement target still needs) */
  double refine_tol;        /* mixed: converged when ||e_i - A z|| <= tol; refines on to
                               tol * min(1, |ratio|) within refine_maxit passes */
  int32_t refine_maxit;     /* mixed: maximum refinement passes */
  double step;              /* proposal half-width h (uniform cube) */
  int32_t row_cap;          /* nonzeros per stored Slater row; <= 0: automatic */
  int32_t force_reorder_every; /* test knob: trigger every k-th step (0 = off) */
  int32_t plain_stop;       /* nonzero: a ratio solve stops once converged (residual at
                               its tolerance, Section 4's criterion) instead of going on
                               to the tolerance times min(1, |ratio|) (vmc_det_ratio) */
  double refactor_cost;     /* cost-balance refactor (Section 3.2): refactor once the
                               stored-update vector entries streamed by preconditioner
                               applications since the last factorisation reach this value
                               (the expected cost of a new ILUTP in the same units); <= 0:
                               refactor only after m_max updates.  vmc_autotune measures it
                               per walker. */
  int32_t ilu_work_cap;     /* ILUTP work-row capacity (entries of one row during its
                               elimination, candidates, multipliers before the fill
                               limit); <= 0: 512 entries, 192 candidates, 160 multipliers,
                               four rows in flight, used where the factorisation's usual
                               tables (eight rows in flight, 256 entries, 128 candidates,
                               96 multipliers) overflow: from the first unfinished row, for
                               64 rows, after which the usual tables resume (the factors
                               are the same either way).  Larger values fit
                               matrices with more fill (e.g. the paper's b.c.c. k = 1
                               orbitals at droptol 0.01 need about 9 K^2) and are used
                               alone; fewer rows are then factored concurrently so the LDS
                               fits.  At most 8192.  The multiplier table keeps the
                               largest multipliers once full, which loses none of the
                               nL0 + p a row stores while that many fit.  Rows beyond
                               these capacities give VMC_ECAPACITY. */
  int32_t ilu_drop_norm;    /* ILUTP drop scale of row i: 0 = droptol * ||a_i||_2; 1 =
                               droptol * ||a_i||_1 / nnz(a_i), the mean magnitude that
                               SPARSKIT's ILUTP (the paper's preconditioner, Section 4) uses */
  double energy_tol;        /* residual at which the kinetic-energy solves stop (the FP64
                               path's GMRES rtol and the mixed path's refinement tolerance);
                               <= 0: the tolerances of the ratio solves.  A term then errs by
                               at most ||A^{-T} lkin_p|| * energy_tol */
  int32_t device_ptrs;      /* nonzero: the array arguments of vmc_det_ratio and vmc_accept
                               (particle, new_pos, ratio_out, info_out, accept, accepted_out)
                               are device pointers, the walker list must be NULL (all
                               walkers, count ignored), and both calls return without
                               synchronising; walker errors then surface at vmc_sync */
  int32_t test_knobs;       /* test knobs (0 = off), bits VMC_TEST_*: they force conditions
                               that the error and trigger paths need, from the host */
} vmc_params;

/* vmc_params.test_knobs bits */
#define VMC_TEST_ZERO_RATIO 1      /* vmc_det_ratio reports, and leaves pending, a ratio of
                                      exactly 0 for every move (exercises the refusal of a
                                      forced acceptance) */
#define VMC_TEST_FIRST_SOLVE_ONE_ITER 2  /* the first solve of every step stops after one
                                      GMRES iteration, so it misses its tolerance and the
                                      not-converged reorder trigger fires; the solve after the
                                      reorder runs normally */
#define VMC_TEST_ILU_FAST_SMALL 4  /* the ILUTP's usual tables shrink to 64 entries, so rows
                                      that hold more during their elimination overflow them and
                                      the factorisation falls back to the larger tables again
                                      and again (vmc_stats.ilu_retries counts the fallbacks) */

/* One walker: its physical system (orbital centres and shapes) and start. */
typedef struct vmc_walker_init {
  int32_t n;                /* particles = orbitals, 1 <= n <= 16384; n = n_basis*Lx*Ly*Lz */
  int32_t lattice[3];       /* cell counts per axis (Lx, Ly, Lz); box = lattice * a */
  double a;                 /* cell side */
  double site_margin;       /* max per-axis distance of a site from its nominal position */
  const double* sites;      /* host, n*3, orbital centres in [0, box); site
                               j = b + n_basis*(ix + Lx*(iy + Ly*iz)) sits nominally at
                               ((ix, iy, iz) + basis[b]) * a */
  const double* sigma;      /* host, n, Gaussian width of each orbital */
  int32_t orbital_kind;     /* VMC_ORB_* */
  double p_scale;
  double p_sigma;
  double cutoff;            /* orbital j vanishes where the minimum-image distance > cutoff */
  const double* pos0;       /* host, n*3, initial positions in [0, box) */
  uint64_t seed;            /* Philox key word 0 for this walker's draws */
  int32_t n_basis;          /* sites per cell, 0..4; 0 is read as 1 with basis[0] = 0
                               (simple cubic).  The paper's lattice is b.c.c. (Section 2.1,
                               Section 4): two sites, offsets (0,0,0) and (1/2,1/2,1/2) */
  int32_t pad0;
  double basis[4][3];       /* fractional offsets of the cell's sites, each in [0, 1) */
} vmc_walker_init;

/* Per-step outcome, also used as the record of the step log. */
typedef struct vmc_step_record {
  int64_t step;             /* the walker's step index g (Philox counter) */
  int32_t walker;
  int32_t particle;         /* particle id moved */
  double new_pos[3];
  double ratio;             /* det A'/det A = 1 + u^T z, FP64 (eq. (detRatioEq)) */
  double log_abs_ratio;     /* ln|ratio| in FP64; -inf for a zero ratio */
  double u_acc;             /* acceptance draw in (0,1) */
  double N;                 /* effective stability of the (last) solve */
  double resid;             /* final residual norm ||e_i - A z||_2 (mixed: computed in FP64;
                               FP64 path: the GMRES recurrence estimate) */
  int32_t iters;            /* GMRES iterations of the final solve (all inner solves, mixed) */
  int32_t flags;            /* VMC_FLAG_* */
  int32_t refinements;      /* mixed: FP64 refinement passes of the final solve; 0 in FP64 */
  int32_t inner_solves;     /* GMRES solves behind the final ratio (1 + refinements) */
} vmc_step_record;

/* Host copies of a walker's state (any pointer may be NULL to skip). */
typedef struct vmc_state_view {
  double* pos;              /* n*3, by particle id */
  int32_t* row_particle;    /* n: particle at each row position */
  int32_t* col_site;        /* n: orbital (site id) at each column position */
  int32_t* reorder_row;     /* n: last geometric reorder, particle per position */
  int32_t* reorder_col;     /* n: last geometric reorder, site per position */
  int32_t* a_len;           /* n: nonzeros per Slater row (by row position) */
  int32_t* a_col;           /* n*row_cap: column positions */
  double* a_val;            /* n*row_cap */
  int32_t* l_len;           /* n */
  int32_t* l_col;           /* n*fact_cap: column positions (< row) */
  double* l_val;            /* n*fact_cap: multipliers l_ik */
  int32_t* u_len;           /* n: off-diagonal count */
  int32_t* u_col;           /* n*fact_cap: column positions (> row) */
  double* u_val;            /* n*fact_cap: u_ik */
  double* u_diag;           /* n */
  int32_t* ilu_perm;        /* n: column permutation q of the last ILUTP, relative to the
                               column numbering A had when it was factored */
  int64_t* step;            /* 1: steps taken */
  int32_t* n_updates;       /* 1: stored rank-one updates */
} vmc_state_view;

/* Per-walker counters. */
typedef struct vmc_stats {
  int64_t steps, accepted, solves, iters, reorders, refactors, nonconverged;
  int64_t inner_solves, refine_passes;
  int64_t update_sum;       /* sum over inner solves of the stored updates applied */
  int64_t phase_ticks[12];  /* device wall-clock ticks per phase: prepare, L solve, U solve,
                               updates, SpMV, orthogonalisation, solution, FP64 residual,
                               accept, refactor, reorder, whole persistent launch */
  double max_N, sum_N;
  double update_entries;    /* stored-update vector entries streamed by all preconditioner
                               applications (sum over solves of m * n * iterations) */
  double refactor_cost;     /* the walker's current cost-balance threshold (<= 0: off) */
  int32_t status;           /* VMC_OK or the first error the walker hit */
  int32_t ilu_retries;      /* ILUTP fallbacks: windows of rows that overflowed the usual
                               tables and were factored with the larger ones */
} vmc_stats;

/* What vmc_autotune measured or loaded. */
typedef struct vmc_tune_info {
  double ilutp_us_mean;      /* one ILUTP factorisation, mean over walkers (microseconds) */
  double update_ns_per_entry;/* applying stored updates: time per vector entry (median) */
  double refactor_cost_mean; /* resulting cost-balance thresholds, mean over walkers */
  double step_us_min, step_us_max; /* trial step time per walker, extremes */
  int32_t from_cache;        /* 1: thresholds came from cache_path, nothing was measured */
  int32_t trial_steps;       /* steps every walker took during the measurement */
} vmc_tune_info;

/* Fill p with the defaults (Section 4 settings where the paper gives them). */
vmc_status vmc_default_params(vmc_params* p);

/* Create a context for n_walkers walkers; copies all host arrays.  hip_stream
   is a hipStream_t (NULL for the default stream).  One workgroup works on one
   walker with its vectors staged in LDS, so the largest n must fit one
   workgroup's LDS: on a 160 KiB device n = 16384 fits in mixed precision and
   FP64 stops near n = 14700 (less with a larger m_max); a larger n returns
   VMC_EINVAL with the bytes needed in vmc_last_error(NULL).  VMC_ENOMEM when
   a walker's device arena cannot be allocated.  On any error nothing stays
   allocated and no context is returned. */
vmc_status vmc_create(void** ctx_out, const vmc_params* p, int32_t n_walkers,
                      const vmc_walker_init* walkers, void* hip_stream);

/* Evaluate every Slater row from the current positions (Section 2.1,
   eq. (SlaterMatrix)): a_{ij} = phi_j(r_i) for minimum-image distances within
   the cutoff.  walkers = NULL means all. */
vmc_status vmc_build_slater(void* ctx, const int32_t* walkers, int32_t count);

/* Compute a new preconditioner: with reorder != 0, first the geometric
   particle/orbital reordering (Section 3.1) and a rebuild of the Slater matrix
   in that order; then ILUTP (Section 3.2, eq. (ilu); Section 4 settings) and
   clearing of the rank-one update list.  walkers = NULL means all. */
vmc_status vmc_ilutp(void* ctx, const int32_t* walkers, int32_t count, int32_t reorder);

/* Determinant ratio of a trial move for each listed walker (eq. (detRatioEq)):
   ratio = 1 + u^T z with A z = e_i by preconditioned GMRES, with the reorder
   triggers of Section 4 (N > n_thresh, the solve missing its tolerance within
   gmres_maxit, or iterations >= iter_factor * running average: reorder,
   refactor and solve again).  A solve is converged when its residual is at
   most its tolerance (gmres_rtol; mixed: ||e_i - A z|| <= refine_tol in FP64);
   it goes on, within gmres_maxit (mixed: refine_maxit passes), until the
   residual is at most the tolerance times min(1, |ratio|), the ratio estimated
   from the current iterate, so that small ratios keep their relative accuracy.
   particle / new_pos (count and count*3) give the move; NULL draws it from the
   walker's Philox stream (particle = step mod n).  ratio_out (count) and
   info_out (count, may be NULL) receive the results; the move stays pending
   until vmc_accept.  Host arrays unless vmc_params.device_ptrs (see there).
   A walker whose solve still misses its tolerance after the reorder and
   refactor stops: its status becomes VMC_ENOCONV (returned here, and by
   vmc_sync and the vmc_run_* paths through vmc_sync), its record carries
   VMC_FLAG_NOCONV and no move is pending.  vmc_build_slater or vmc_ilutp on the
   walker clears that status. */
vmc_status vmc_det_ratio(void* ctx, const int32_t* walkers, int32_t count,
                         const int32_t* particle, const double* new_pos,
                         double* ratio_out, vmc_step_record* info_out);

/* Commit or discard each pending move.  accept (host, count) forces the
   decision; NULL applies the Metropolis rule ratio^2 > u_acc with the
   walker's draw (Section 2.2).  On acceptance the row is replaced and the
   preconditioner updated (eq. (mkp1)); after m_max updates it is refactored.
   accepted_out (host, count, may be NULL) receives the decisions.  A forced
   acceptance of a move whose pending ratio is 0 or not finite (the new Slater
   matrix would be singular and the update z/ratio undefined) is refused with
   VMC_ESINGULAR: that walker's move stays pending, so the caller can still
   reject it; the other listed walkers are processed normally.  The Metropolis
   rule never accepts such a move. */
vmc_status vmc_accept(void* ctx, const int32_t* walkers, int32_t count,
                      const uint8_t* accept, uint8_t* accepted_out);

/* Persistent fused path: every walker takes `steps` Metropolis steps (propose,
   row, ratio, decision, update, refactor/reorder as triggered) in one launch,
   each walker on its own workgroup.  dev_log (device memory, may be NULL)
   receives record [w * steps + s] if log_cap allows.  Asynchronous. */
vmc_status vmc_run_steps(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap);

/* vmc_run_steps with steps = sweeps * n of each walker (a sweep moves every
   particle once), issued as a replay of the captured graph of that launch
   (vmc_run_steps_graph); requires all walkers to share n.  Asynchronous. */
vmc_status vmc_run_sweeps(void* ctx, int32_t sweeps, vmc_step_record* dev_log, int64_t log_cap);

/* vmc_run_steps replayed from a HIP graph: the first call with a given
   (steps, dev_log, log_cap) records the persistent launch into a graph (on a
   private stream of the context, so a context on the null stream works too);
   that call and later calls with the same arguments launch the graph on the
   context's stream (a different argument set records a new one).  Same
   results as vmc_run_steps.  Asynchronous. */
vmc_status vmc_run_steps_graph(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap);

/* Kinetic energy (Section 2.3, Local Energy; Section 4, eq. (energyEq)), with
   hbar = m = 1.  For particle p, replacing row i(p) of the Slater matrix by the
   kinetic row -(1/2) lap phi_j(r_p) gives the term
     t_p = -(1/2) lap_p Psi / Psi = lkin_p^T A^{-1} e_{i(p)},
   obtained by one more solve A z = e_{i(p)} with the same preconditioned GMRES
   (mixed refinement included) and the same reorder triggers as a ratio; the
   energy per particle is E = (1/n) sum_p t_p.  Terms are computed for the
   particle ids p_begin <= p < p_end (clamped to each walker's n) of the listed
   walkers (walkers NULL: all, count ignored), at their current positions.
   energy_out (host, count): (sum of the computed terms) / n, i.e. E when the
   range covers every particle.  terms_out (host, may be NULL): the terms, walker
   after walker in list order, each walker's in particle order.  A walker with a
   pending ratio (vmc_det_ratio without vmc_accept) gives VMC_ESTATE.  A solve may
   reorder and refactor the walker, as a step does.  Synchronous. */
vmc_status vmc_kinetic_energy(void* ctx, const int32_t* walkers, int32_t count, int32_t p_begin, int32_t p_end,
                              double* energy_out, double* terms_out);

/* vmc_run_steps that also samples the kinetic energy per particle E at the end
   of every sweep (whenever the step count becomes a multiple of n), as
   Section 4 does.  All walkers must share n and their step count.  The k-th
   sample of this call goes to dev_energy[w * energy_cap + k] (device memory,
   n_walkers * energy_cap doubles) while k < energy_cap; dev_log as for
   vmc_run_steps.  Reads the step counts from the device first (one
   synchronisation), then runs asynchronously. */
vmc_status vmc_run_steps_energy(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap,
                                double* dev_energy, int32_t energy_cap);

/* The standard algorithm (Section 1), as a comparison path: the explicit
   inverse of every walker's Slater matrix, read for each ratio and updated by
   Sherman-Morrison on each accepted move, so an accepted step rewrites n^2
   values.
   vmc_sm_prepare allocates one n x n FP64 inverse per walker (8 n^2 bytes,
   owned by the context) and fills it column by column with the
   preconditioned solver at relative tolerance tol (e.g. 1e-13) from the
   walkers' current state.  VMC_ENOCONV if a column misses tol, VMC_ESTATE with
   a pending move.  Synchronous.
   vmc_sm_run_steps then takes `steps` steps of every walker by the standard
   algorithm: the same proposals, draws and decision rule as vmc_run_steps
   (ratio = a'^T A^{-1} e_p), records in dev_log as vmc_run_steps writes them
   (iters 0, N 0).  VMC_ESTATE before vmc_sm_prepare, or when any other call
   that may move a walker or rebuild its rows (vmc_build_slater, vmc_ilutp,
   vmc_det_ratio, vmc_accept, the vmc_run_* calls, vmc_phase_bench) came after
   the last vmc_sm_prepare.  It moves the particles but leaves the sparse state
   (A, the factors, the update list) behind: until vmc_build_slater and then
   vmc_ilutp (or vmc_ilutp with reorder) have rebuilt a walker, the sparse-path
   calls on it (vmc_det_ratio, vmc_accept, vmc_kinetic_energy, the vmc_run_*
   calls, vmc_sm_prepare, vmc_phase_bench) return VMC_ESTATE.  Asynchronous.
   vmc_sm_get_inverse copies walker w's inverse to host_out (n*n doubles,
   host_out[p*n + j] = (A^{-1})_{jp}, particle p, site j).  Synchronous. */
vmc_status vmc_sm_prepare(void* ctx, double tol);
/* vmc_sm_prepare for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same inverses, computed by the same kernels, but stored in a static
   device array of 64 MiB that the library holds on each GPU it runs on until
   the process ends, instead of buffers the context allocates.  It calls no
   hipMalloc, hipFree or other allocating routine (an error message may
   allocate host memory).  The inverses, their pointer table and the
   not-converged flags must fit 64 MiB: sum over walkers of
   n2 * n * 8 bytes (n2 = n rounded up to even), each rounded up to 256,
   plus 256-byte-rounded 8 * walkers and 4 * walkers; larger requests return VMC_EINVAL and leave
   the context as it was.  One array per GPU: the last context to call this
   on a GPU owns it, and the contexts that held it before get VMC_ESTATE from
   vmc_sm_run_steps and vmc_sm_get_inverse until they prepare again.  Calls
   on one GPU that overlap race.  vmc_sm_prepare afterwards goes back to the
   context's own buffers.  Synchronous. */
vmc_status vmc_sm_prepare_static(void* ctx, double tol);
vmc_status vmc_sm_run_steps(void* ctx, int32_t steps, vmc_step_record* dev_log, int64_t log_cap);
vmc_status vmc_sm_get_inverse(void* ctx, int32_t walker, double* host_out);

/* Autotuner for the batch (Section 3.2 cost balance, and the walker-to-
   workgroup map).  With a readable cache_path holding a threshold for every
   walker size n in the context, loads those; otherwise measures on the device:
   - one ILUTP factorisation of every walker (it counts as a refactor and
     clears the update lists), timed per walker;
   - trial_steps ordinary steps of every walker (they advance the chains),
     from which the time per applied stored-update entry and the step time of
     every walker are read;
   and sets each walker's refactor_cost = ILUTP time / time per entry: a walker
   refactors once its update applications have cost as much as a new
   factorisation.  Walkers are then launched longest-step first.  Writes
   cache_path (one line per n) when given and measured.  Synchronous.
   info (host, may be NULL) receives the figures. */
vmc_status vmc_autotune(void* ctx, const char* cache_path, int32_t trial_steps, vmc_tune_info* info);

/* Diagnostic micro-benchmark: every walker's workgroup runs one phase of the
   solve `reps` times on its current matrix and factors, in one launch:
   0 SpMV (solve precision), 1 forward solve with L, 2 backward solve with U,
   3 rank-one update application, 4 FP64 residual e_i - A z, 5 ILUTP.
   Phases 0-4 leave the walker state unchanged; 5 refactors (and clears the
   update list, as any refactor does).  Asynchronous. */
vmc_status vmc_phase_bench(void* ctx, int32_t phase, int32_t reps);

/* Wait for all work issued on the context's stream; returns the first walker
   error (if any) as a status. */
vmc_status vmc_sync(void* ctx);

/* Sizes of walker w: n, stored Slater row capacity, factor row capacity. */
vmc_status vmc_get_dims(void* ctx, int32_t walker, int32_t* n, int32_t* row_cap,
                        int32_t* fact_cap);

/* Copy walker w's state to host buffers (synchronises). */
vmc_status vmc_get_state(void* ctx, int32_t walker, const vmc_state_view* view);

/* Copy per-walker counters to stats_out[n_walkers] (synchronises). */
vmc_status vmc_get_stats(void* ctx, vmc_stats* stats_out);

/* Last error message of the context (or of the last failed vmc_create when ctx is NULL). */
const char* vmc_last_error(void* ctx);

/* Free the context and all its device memory. */
vmc_status vmc_destroy(void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* VMCDET_H */
