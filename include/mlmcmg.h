/*
 * mlmcmg -- MI355X (gfx950) multilevel Monte Carlo multigrid hot path.
 *
 * C ABI of the HIP library libmlmcmg.so.  It computes the per-sample work of
 * multilevel Monte Carlo as stated in arXiv 1607.03252 (Gmeiner, Drzisga,
 * Ruede, Scheichl, Wohlmuth):
 *   - the model problem -div(k(x,omega) grad u) = f on D = (0,1)^3 with
 *     u = 0 on the boundary (Section 3, eq. modweak);
 *   - a lognormal coefficient k = exp(Z) with exponential covariance
 *     (Section 3.2, eq. def:expcov), here the separable covariance
 *     sigma^2 prod_d exp(-|x_d - y_d|/lambda) truncated to its 4x4x4
 *     Karhunen-Loeve block, driven by Philox4x32-10 numbers;
 *   - the level differences Y_l = Q_l - Q_{l-1} computed from two solves on
 *     one shared omega, Y_0 = Q_0 (Section 2.2, eq. MLMC_defn, Algorithm 1,
 *     steps 1.a.i-ii), with Q = integral of u over D;
 *   - multigrid V(nu1,nu2) cycles with red-black Gauss-Seidel smoothing
 *     (the paper's solver is multigrid with pre/post smoothing, Section 7.1).
 *
 * Discretisation: an n x n x n vertex grid, n = 2^m + 1 (m >= 1), h = 1/(n-1),
 * vertex (i,j,k) at (ih, jh, kh) stored at index (i*n + j)*n + k (k fastest).
 * 7-point finite differences, face coefficient 2 k_p k_q / (k_p + k_q).
 * MLMC level l uses n_l = (n0 - 1) 2^l + 1.
 *
 * Conventions for every call:
 *   - "device" pointers are HIP device memory (e.g. torch CUDA tensors),
 *     "host" pointers are ordinary CPU memory; the caller owns both.
 *   - The plan owns its workspace and frees it in mg_plan_destroy.
 *   - Calls are blocking unless stated: on return the plan's stream has been
 *     synchronised and every output is written.
 *   - Plans are not thread-safe; use one plan per host thread.
 *   - Errors are returned as status codes (MG_*); mg_last_error gives text.
 *     No C++ exception crosses this interface.
 */
#ifndef MLMCMG_H
#define MLMCMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_plan_s* mg_plan;

enum {
  MG_OK = 0,
  MG_EINVAL = -1,   /* bad argument (size, pointer, parameter) */
  MG_ENOMEM = -2,   /* device allocation failed or HBM budget exceeded */
  MG_ENOCONV = -3,  /* at least one solve missed tol within max_cycles */
  MG_EHIP = -4,     /* a HIP runtime call failed */
  MG_EBUSY = -5,    /* serving queue full */
  MG_ENOTIMPL = -6  /* option not supported by this build */
};

enum { MG_FP64 = 0, MG_MIXED = 1 };

typedef struct {
  int n0;             /* vertices per axis of MLMC level 0, 2^m + 1, m >= 1     */
  int max_level;      /* L >= 0: finest MLMC level, n_L = (n0-1) 2^L + 1       */
  int nu1, nu2;       /* pre- and post-smoothing sweeps (>= 0, sum >= 1)       */
  int max_cycles;     /* cycle cap per solve (>= 1)                            */
  double tol;         /* relative residual ||b - Au|| / ||b|| to stop at (> 0) */
  int precision;      /* MG_FP64 or MG_MIXED (FP32 inner cycles)               */
  double sigma2;      /* variance sigma^2 of log k (>= 0)                      */
  double corr_len;    /* correlation length lambda (> 0)                       */
  int kl_per_axis;    /* 1D modes per axis; this build supports 4 (4^3 terms)  */
  size_t hbm_budget;  /* bytes a batch workspace may hold; 0 = no limit (a     */
                      /* server's lanes share it; 8 GiB for a server if 0)   */
  void* stream;       /* hipStream_t to run on; NULL = the null stream         */
} mg_plan_desc;

/* Fill *d with the defaults: n0 = 33, max_level = 0, V(2,2), 50 cycles,
 * tol = 1e-8, MG_FP64, sigma2 = 1, lambda = 0.1, 4 modes, no budget, NULL. */
void mg_plan_desc_default(mg_plan_desc* d);

/* Create a plan: the fixed data of one MLMC run (Section 2.2, Algorithm 1:
 * the hierarchy of levels h_l = 2^-l h_0 on which samples Y_l are drawn; the
 * problem of Section 3, eq. modweak, with f = 1; the lognormal coefficient
 * of Section 3.2, eq. def:expcov, with the plan's sigma^2 and lambda).
 * Validates *desc and precomputes the 1D KL eigenpairs and their tables at
 * the vertices of every grid of levels 0..max_level.  *out (host) receives
 * the handle, which the caller releases with mg_plan_destroy.  Returns MG_OK,
 * MG_EINVAL (bad field, or a finest grid above 1025^3), MG_ENOTIMPL
 * (kl_per_axis != 4), MG_ENOMEM or MG_EHIP; *out is NULL on failure. */
int mg_plan_create(const mg_plan_desc* desc, mg_plan* out);
int mg_plan_destroy(mg_plan plan);

/* Copy the description the plan was created with into *out (host). */
int mg_plan_get_desc(mg_plan plan, mg_plan_desc* out);

/* Switch the stream later calls run on (e.g. torch's current stream). */
int mg_plan_set_stream(mg_plan plan, void* stream);

/* One multigrid solve of -div(k grad u) = f (Section 3, eq. modweak) on an
 * n^3 grid, n = 2^m + 1.  Device pointers, n^3 doubles each, z fastest:
 *   k: vertex values of the coefficient (> 0, boundary included);
 *   f: right-hand side at vertices (boundary entries ignored);
 *   u: in = initial guess, out = solution; its boundary entries are set to 0.
 * Runs V(nu1,nu2) cycles (the plan's) until ||b - Au||_2/||b||_2 <= tol
 * (tol <= 0: the plan's tol), or, when fixed_cycles > 0, exactly fixed_cycles
 * cycles.  cycles/relres (host, may be NULL) receive the cycle count and the
 * last relative residual.  MG_ENOCONV if max_cycles passed without reaching
 * tol (u then holds the last iterate); MG_EINVAL for n not of the form
 * 2^m + 1 with 3 <= n <= 1025, a NULL k, f or u, or fixed_cycles < 0. */
int mg_solve(mg_plan plan, int n, const double* k, const double* f, double* u,
             double tol, int fixed_cycles, int* cycles, double* relres);

/* Allocation-free variant of mg_solve, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, results and status
 * codes as mg_solve (the same kernels, bit for bit), with these limits:
 *   - the whole workspace (hierarchy, solve state, descriptor lists) lives
 *     in a static device array of 96 MiB that the library holds on every GPU
 *     it runs on until the process ends; no device or pinned host memory is
 *     allocated or freed by the call;
 *   - n <= 129 (the 129^3 hierarchy, FP64 or mixed precision, fits); larger
 *     n returns MG_EINVAL;
 *   - every call on one GPU uses the same array, which keeps the last call's
 *     contents (each call clears what it needs).  Calls that overlapped on
 *     one GPU would race: the library serialises them within a process (a
 *     lock per device), and each call blocks until its solve is done. */
int mg_solve_noalloc(mg_plan plan, int n, const double* k, const double* f, double* u,
                     double tol, int fixed_cycles, int* cycles, double* relres);

/* n_samples MLMC samples of Y_level (Algorithm 1, steps 1.a.i-ii): for each
 * seed s the normals xi(s, level) define omega; the solve on n_level and (for
 * level > 0) the solve on n_{level-1} use the same omega, with f = 1 and a
 * zero initial guess.  seeds: host uint64[n_samples].  Outputs (device,
 * n_samples entries; Qf/Qc/cycles_out may be NULL):
 *   Y_out: Q(u_level) - Q(u_{level-1}) (Y_0 = Q_0);  Qf_out, Qc_out: the two
 *   QoIs (Qc = 0 at level 0);  cycles_out: int[2*n_samples], fine and coarse
 *   cycle counts, -1 where a solve missed tol.
 * fixed_cycles > 0 runs exactly that many cycles per solve (parity mode).
 * Returns MG_ENOCONV if any solve missed tol (the others are complete), and
 * MG_EINVAL, with no device work, for n_samples < 1, a level outside
 * [0, max_level], a NULL seeds or Y_out, or fixed_cycles < 0. */
int mlmc_sample_batch(mg_plan plan, int level, const uint64_t* seeds, int n_samples,
                      double* Y_out, double* Qf_out, double* Qc_out, int* cycles_out,
                      int fixed_cycles);

/* Samples of several levels in one batch (levels: host int[n_samples], each
 * in [0, max_level]; other arguments as mlmc_sample_batch).  Sample i is
 * Y_{levels[i]} of seed seeds[i]; every grid of every sample that has the same
 * size is advanced by the same launches (the V-cycles of smaller grids nest in
 * those of larger ones), so a mix of levels runs as one batch.  Results equal
 * those of mlmc_sample_batch on each level alone, bit for bit.  MG_EINVAL
 * as mlmc_sample_batch, and for any levels[i] outside [0, max_level]. */
int mlmc_sample_mixed(mg_plan plan, const int* levels, const uint64_t* seeds, int n_samples,
                      double* Y_out, double* Qf_out, double* Qc_out, int* cycles_out,
                      int fixed_cycles);

/* Execution options (no effect on results beyond rounding order unless
 * stated):
 *   "smoother": 0 = fused single-pass red-black sweep (default; grids
 *               whose arrays reach 2 GiB, e.g. 1025^3 in FP64, use the
 *               colour sweeps), 1 = two-pass in-place colour sweeps (same
 *               iterates);
 *   "graph":    1 = capture the cycles of mlmc_sample_batch into HIP graphs
 *               (default), 0 = launch eagerly;
 *   "transfer": 0 = residual and full weighting in one pass (default; a
 *               launch with few grids splits each tile's plane march into
 *               pieces of coarse planes), 1 = separate residual and
 *               restriction kernels (same results, bit for bit);
 *   "small_vcycle": 17 (default), 9 or 5 = from the largest grid of at most
 *               this size down, each V-cycle runs in one launch with the
 *               grids held in LDS; 0 = one launch per level and step
 *               (same results, bit for bit);
 *   "norm":     1 (default) = the residual norm of an iterate is summed in
 *               the sweeps around it (black points in the cycle's last sweep,
 *               red points in the next cycle's first) and the solve is judged
 *               after that first sweep; 0 = a residual pass after each cycle
 *               (same stopping cycle and results; the reported relative
 *               residual differs by summation order only).
 * Options that change what the samples compute (mlmc_sample_batch and
 * mlmc_sample_mixed; the server supports only the defaults):
 *   "qoi":      0 (default) = Q = integral of u over D; 1 = u at
 *               x* = (1/4, 1/4, 1/4); 2 = the flux of -k grad u in the +x_2
 *               direction across the plane x_2 = 1/4 (|Gamma| = 1), the mean
 *               of the discrete face fluxes on either side of that vertex
 *               plane (Section 3's two other QoIs; 1 and 2 need n0 = 4m + 1);
 *   "solver":   0 (default) = V(nu1,nu2) cycles from zero until tol;
 *               1 = full multigrid (nested iteration, Section 7.1): the 3^3
 *               grid solved exactly, then on every finer grid the trilinear
 *               interpolation of the coarser result and "fmg_cycles"
 *               V(nu1,nu2) cycles against that grid's own problem; FMG-2V(4,4)
 *               is nu1 = nu2 = 4 in the plan and fmg_cycles = 2.  The coarse
 *               solve of Y_l is the fine schedule's n_(l-1) stage.  FP64 only
 *               (MG_ENOTIMPL on a mixed-precision plan); cycles_out reports
 *               fmg_cycles; fixed_cycles is ignored;
 *   "fmg_cycles": V-cycles per grid of the full multigrid schedule (1..64,
 *               default 2).
 *   "kl":       1 = the FP64 smoother and residual-restriction launches on
 *               the top grids of KL-field samples (constant right-hand side,
 *               up to 257^3) evaluate the coefficient wh = exp(-Z)/2 from the
 *               sample's normals and the 1D modes instead of reading it, in
 *               the operations of the field kernel that stores it: identical
 *               results with 16 instead of 24 bytes per node and sweep, but
 *               slower on MI355X, where these kernels are bound by FP64
 *               issue rather than by bytes; 0 (default) = read wh.
 *   "inner_cycles": mixed precision (MG_MIXED plans): FP32 V(nu1,nu2) cycles
 *               per FP64 defect-correction step (1..8, default 1).  With c
 *               inner cycles a step applies, in exact arithmetic, the same
 *               correction as c FP64 V-cycles (the cycle is linear in the
 *               error), so the FP64 defect and correction passes are paid once
 *               per c cycles; convergence is still judged by the FP64 residual
 *               after each step, and cycles_out counts V-cycles (steps x c):
 *               a multiple of c, so fixed_cycles and max_cycles are in effect
 *               rounded up to multiples of c.  Ignored by FP64 plans.
 *   "operator": 0 (default) = 7-point finite differences with harmonic-mean
 *               face coefficients; 1 = the paper's P1 finite elements
 *               (Section 3.1) on the Kuhn tetrahedra of the vertex grid (every
 *               cell split into the six tetrahedra x_a >= x_b >= x_c), each
 *               tetrahedron's coefficient the mean of its four vertex values
 *               (the four-node quadrature), rediscretised on every level with
 *               injected k.  This operator couples axis neighbours only, with
 *               the coupling of an edge the sum of the four-vertex means of
 *               its six tetrahedra over 6, so the same red-black V-cycle
 *               applies (two-pass colour sweeps, separate residual and
 *               restriction; no LDS cycle).  FP64, V-cycles to tol, integral
 *               or point QoI (MG_ENOTIMPL otherwise); also used by mg_solve. 
 *   "field":    0 (default) = the 4x4x4 separable KL field; 1 = the paper's
 *               SPDE sampler (Section 3.2, eq. spde): (kappa^2 - Laplace) Z = W
 *               on the box (-1,2)^3 with natural Neumann boundary, lumped-mass
 *               P1 elements on the Kuhn tetrahedra of the box grid at the
 *               sample grid's spacing (3(n-1)+1 vertices per axis), the white
 *               noise load sqrt(M_pp) xi_p from Philox4x32-10 with counter
 *               (j, level, 1, 0) (normals 2j, 2j+1), V(2,2) cycles to relative
 *               residual 1e-10 over all box vertices, and
 *               k = exp(sigma sqrt(8 pi kappa) Z) at D's vertices with
 *               kappa = 1/lambda (the Whittle variance 1/(8 pi kappa)
 *               rescaled to sigma^2).  The coarse solve of Y_l takes the same
 *               noise on the coarse box grid (load P^T b / 2) and a box solve
 *               of its own.  Not with "solver" = 1 or the server (MG_ENOTIMPL);
 *               mlmc_field then serves n = n_level (fine) and n_(level-1)
 *               (coarse) of a level <= max_level.
 * Returns MG_EINVAL for an unknown name or value. */
int mg_plan_set_option(mg_plan plan, const char* name, long long value);

/* Tile shape of the fused smoother on grids of size n: tj rows (j) by tk
 * columns (k) per workgroup, the planes split into `chunks` pieces (0 = chosen
 * per launch from the number of grids: the march is split until the launch
 * fills the machine once at the shape's occupancy, 512 workgroups, or 256
 * for the 16x64 tile of which one fits a CU, at least four planes per
 * piece).  Only the
 * compiled shapes whose tj, tk divide n-1 are accepted (MG_EINVAL otherwise).
 * A server captures the shapes in force at its first step. */
int mg_set_tile(mg_plan plan, int n, int tj, int tk, int chunks);
int mg_get_tile(mg_plan plan, int n, int* tj, int* tk, int* chunks);
/* The same for one kind of sweep only: fused_correction = 1 is the first
 * post-smoothing sweep, which also adds the coarse-grid correction (it uses
 * more registers, so its best shape can differ); 0 is every other sweep.
 * mg_set_tile sets both, mg_get_tile reads kind 0. */
int mg_set_tile_for(mg_plan plan, int n, int fused_correction, int tj, int tk, int chunks);
int mg_get_tile_for(mg_plan plan, int n, int fused_correction, int* tj, int* tk, int* chunks);

/* Autotuner: runs one batch of n_samples samples of `level` (seeds
 * 0x5eed0000 + i), then times every compiled tile shape with chunk counts
 * 0 (automatic), 1, 2, 4 of both kinds of smoothing sweep on each grid size
 * of that batch above the LDS V-cycle's sizes (reps launches each, HIP
 * events) and picks the fastest per size and kind (a fixed chunk count that
 * launches what the automatic one launches with every grid active is kept
 * as automatic).  The picks are kept only if whole batches (reps each,
 * alternated with the shapes in force before tuning, best of two rounds)
 * run more than 1% faster with them; otherwise the plan keeps its previous
 * shapes. */
int mg_autotune(mg_plan plan, int level, int n_samples, int reps);

/* Serving: continuous batching of MLMC sample requests --------------------
 *
 * A request asks for one sample Y_level(seed) (Algorithm 1, steps 1.a.i-ii,
 * as mlmc_sample_batch with one seed).  Resident samples live in lanes: a
 * lane holds a fixed number of sample slots of one level (one workspace,
 * its own stream and graphs; its grids stay in HBM while the lane lives).
 * All lanes share the plan's HBM budget.  Lanes are opened when requests of
 * their level find no free slot and the budget has room, and evicted when
 * empty and their bytes are needed by another level, so memory left idle by
 * one level admits requests of another.  Lanes progress independently: when
 * a lane's launch has finished, its finished samples leave, queued requests
 * of its level are admitted into the freed slots (fields and coefficient
 * hierarchies generated on the device), and the lane is launched again while
 * the other lanes' work is still on the device.  A sample's results do not
 * depend on what else is resident: they equal those of mlmc_sample_batch for
 * that seed and level, bit for bit.  (The paper's dynamic strategies, which
 * hand a new sample to whichever processor group has finished one, are the
 * prior art; Section 5.3.)
 */

/* Device bytes of one resident sample slot of `level` (fine and coarse
 * hierarchies, FP32 twins in mixed precision, state).  *bytes: host. */
int mg_sample_footprint(mg_plan plan, int level, size_t* bytes);

/* Admission scheduler (host only, no device work; the server uses it).
 * Level l is served in lanes of lane_slots[l] slots costing lane_bytes[l]
 * bytes each; all lanes together stay within `budget` bytes.  Requests wait
 * in one queue in arrival order.  mg_sched_admit walks the queue from its
 * head; a request
 *  - takes the lowest free slot of the lowest-numbered idle lane of its
 *    level that is not draining; if its level's free slots are all in lanes
 *    marked in flight, it waits for them;
 *  - otherwise opens a lane of its level, evicting empty idle lanes when the
 *    budget is short (the smallest one that covers the shortfall, else the
 *    largest first until it is covered);
 *  - if no lane can be opened and its level has no lane, it reserves the
 *    memory: until it is admitted no other request opens a lane, and lanes of
 *    other levels covering the shortfall (empty idle ones, then the fewest
 *    resident samples first) drain: they take no new samples, so they empty
 *    and are evicted for it.
 * Once a request waits, later requests of its level wait for the rest of
 * that walk.  So requests of one level are admitted in arrival order, the
 * lanes' bytes never exceed the budget, and every request is admitted once
 * enough resident samples have finished.  Lanes opened and evicted are reported as
 * events, which the executor applies before using the tickets of that pass. */
typedef struct mg_sched_s* mg_sched;
typedef struct {
  long long tag;     /* caller's request id */
  uint64_t seed;
  int level;
  int slot;          /* assigned slot */
  int lane;          /* lane holding that slot */
  double t_arrival;  /* caller's arrival time, seconds */
} mg_ticket;
enum { MG_LANE_OPEN = 1, MG_LANE_CLOSE = 2 };
typedef struct {
  int kind;    /* MG_LANE_OPEN or MG_LANE_CLOSE */
  int lane;    /* lane id (ids are never reused) */
  int level;
  int first;   /* the lane's slots are first .. first + nslots - 1 */
  int nslots;
  size_t bytes;
} mg_lane_event;
/* lane_slots, lane_bytes: host arrays of n_levels; lane_slots[l] in [0, 4096]
 * (0: level l is not served), lane_bytes[l] > 0 where lane_slots[l] > 0;
 * budget > 0 bytes; queue_capacity >= 1. */
int mg_sched_create(int n_levels, const int* lane_slots, const size_t* lane_bytes, size_t budget,
                    int queue_capacity, mg_sched* out);
int mg_sched_destroy(mg_sched s);
/* MG_EINVAL for a level outside [0, n_levels), MG_ENOMEM when a lane of that
 * level exceeds the budget or the level is not served, MG_EBUSY when the
 * queue is full. */
int mg_sched_submit(mg_sched s, int level, uint64_t seed, long long tag, double t_arrival);
/* Writes up to max_out admitted tickets to out (host) and their number to *n_out. */
int mg_sched_admit(mg_sched s, mg_ticket* out, int max_out, int* n_out);
/* Takes up to max_out pending lane events (oldest first) into out (host). */
int mg_sched_events(mg_sched s, mg_lane_event* out, int max_out, int* n_out);
/* Marks a lane as running on the device (nonzero: it neither admits nor is
 * evicted) or idle.  MG_EINVAL for an unknown lane. */
int mg_sched_set_inflight(mg_sched s, int lane, int inflight);
/* MG_EINVAL if the slot is not busy. */
int mg_sched_release(mg_sched s, int slot);
int mg_sched_counts(mg_sched s, int* queued, int* busy);
/* Bytes of the open lanes, their maximum so far, and how many are open. */
int mg_sched_memory(mg_sched s, size_t* used, size_t* peak, int* lanes);

typedef struct mg_server_s* mg_server;
typedef struct {
  long long tag;
  uint64_t seed;
  int level;
  int status;              /* MG_OK, or MG_ENOCONV if a solve missed tol   */
  double Y, Qf, Qc;        /* as mlmc_sample_batch                          */
  int cycles_fine, cycles_coarse;
  double t_arrival;        /* as submitted                                  */
  double t_admit, t_done;  /* server clock (mg_serve_now), seconds          */
} mg_result;

/* Create a server on a plan (levels 0..max_level of the plan).  Its budget is
 * the plan's hbm_budget, or 8 GiB if that is 0.  lane_slots: host
 * int[max_level + 1], slots per lane of each level (each >= 0, 0: level not
 * served), or NULL to size each level's lanes to at most an eighth of the
 * budget (clamped to [1, 256] slots).  A lane's bytes are its workspace
 * (mg_sample_footprint per slot plus descriptor lists) and its staging
 * buffers.  Nothing is allocated until requests arrive.  MG_ENOMEM if one
 * lane of a served level exceeds the budget.  The plan must outlive the
 * server; calls on the plan and on its servers must not overlap. */
int mg_serve_create(mg_plan plan, const int* lane_slots, int queue_capacity, mg_server* out);
int mg_serve_destroy(mg_server s);
/* Queue one request.  t_arrival < 0: stamped with mg_serve_now().  Errors as
 * mg_sched_submit. */
int mg_serve_submit(mg_server s, int level, uint64_t seed, long long tag, double t_arrival);
/* One scheduling step: harvest every lane whose last launch has finished,
 * admit queued requests (opening and evicting lanes as the scheduler
 * decides), launch `cycles` V-cycles (>= 1; graph-captured) on every idle
 * lane that holds samples, and wait until at least one lane has finished if
 * none had.  Returns the samples that finished (up to max_out per call; the
 * rest come with the next call).  out: host mg_result[max_out]; *n_out: how
 * many were written.  With nothing queued or resident it returns at once.
 * MG_EHIP or MG_ENOMEM (a device allocation failed while opening a lane,
 * e.g. a budget above the device's free memory) leave the server unusable:
 * later steps return MG_EINVAL; destroy it. */
int mg_serve_step(mg_server s, int cycles, mg_result* out, int max_out, int* n_out);
/* Seconds since the server was created (steady clock). */
double mg_serve_now(mg_server s);
int mg_serve_counts(mg_server s, int* queued, int* resident, long long* completed);
/* Slots per lane of a level (after NULL sizing), or -1. */
int mg_serve_slots(mg_server s, int level);
/* Device bytes of the open lanes (each lane counted at its stated bytes,
 * which bound what it allocates: creating a lane that allocates more fails
 * with MG_EHIP), their maximum so far, the budget, the number of open lanes,
 * how many lanes were opened and evicted so far, and the host seconds spent
 * opening and evicting them.  Any pointer may be NULL. */
int mg_serve_memory(mg_server s, size_t* used, size_t* peak, size_t* budget, int* lanes,
                    long long* opened, long long* evicted, double* lane_seconds);

/* Test and parity exports ------------------------------------------------- */

/* Philox4x32-10 words of samples on the device: words_out (device) receives
 * uint32[n_samples][128]; block j of sample s uses counter (j, level, 0, 0)
 * and key (seed lo, seed hi).  normals_out (device, may be NULL) receives
 * double[n_samples][64]: U_m = (M_m + 1) 2^-53 with
 * M_m = (w[2m] >> 5) 2^26 + (w[2m+1] >> 6), then Box-Muller pairs. */
int mlmc_philox(mg_plan plan, const uint64_t* seeds, int n_samples, int level,
                uint32_t* words_out, double* normals_out);

/* Host Philox4x32-10 words of one sample (Salmon, Moraes, Dror, Shaw,
 * SC'11): block j = 0..31 uses counter (j, level, 0, 0) and key (seed lo,
 * seed hi); out (host, caller-owned, 128 entries) receives the four words of
 * block j at out[4j..4j+3].  These words define omega of sample (seed,
 * level) (Section 2.2: one omega shared by the two solves of Y_l, independent
 * draws across levels).  No device work.  MG_EINVAL for out == NULL or
 * level < 0. */
int mlmc_philox_words(uint64_t seed, int level, uint32_t out[128]);

/* The exponential with which the kernels form the KL coefficient
 * k = exp(Z) and wh = exp(-Z)/2 (Section 3: the lognormal field), evaluated
 * on the host by the same code and table: Tang's table-driven method
 * (32-entry 2^(j/32) table, degree-6 polynomial), relative error below 2
 * units in the last place, x clamped to [-700, 700].  For tests; no device
 * work. */
double mlmc_exp(double x);

/* Coefficient k = exp(Z(seed, level)) (Section 3.2, eq. def:expcov: the
 * lognormal field, here its 4x4x4 separable KL truncation, sampled from the
 * normals of omega(seed, level)) at the n^3 vertices of an n grid (any
 * n = 2^m + 1 up to 1025, z fastest), computed by the same kernel the
 * samples use.  k_out: device, caller-owned, n^3 doubles.  Blocking.
 * MG_EINVAL for a bad n, level < 0 or k_out == NULL. */
int mlmc_field(mg_plan plan, int n, uint64_t seed, int level, double* k_out);

/* Host-side MLMC level statistics (Section 2.3: sample mean and s_l^2 with
 * divisor N).  A shifted, compensated accumulator; add takes device or host
 * arrays according to on_device. */
typedef struct {
  long long n;
  double shift, s1, c1, s2, c2;
} mlmc_level_acc;
void mlmc_acc_init(mlmc_level_acc* a);
int mlmc_acc_add(mlmc_level_acc* a, const double* y, int count, int on_device);
/* mean = shift + S1/N, var = S2/N - (S1/N)^2 (N = count so far). */
void mlmc_acc_result(const mlmc_level_acc* a, double* mean, double* var);

/* Adaptive MLMC (Section 2.3, Algorithm 2) --------------------------------
 *
 * Step 1: L = 1, N_0 = N_1 = N_Init.  Step 2: for every level l <= L the
 * missing samples of Y_l (sample i of level l has seed seed0 + i, computed
 * with mlmc_sample_mixed, every level in the same batches of at most
 * max_batch samples), then the level mean, s_l^2 (divisor N) and the cost
 * C_l.  Step 3: N_l from eq. (quasioptimal_Nl) with eps_s^2 = theta eps^2
 * (eq. def:eps), never below the samples already taken; if
 * |Yhat_L| > (8^alpha - 1) eps_b with eps_b^2 = (1 - theta) eps^2 (the bias
 * estimate of eq. bias_estimate) and L < the plan's max_level, L -> L + 1
 * with N_L = N_Init.  Step 4: repeat from step 2 until neither any N_l nor L
 * changed (or max_iter rounds).  Step 5: Q = sum of the level means.
 * C_l is the mean work of one sample of Y_l in node-cycles (grid vertices
 * times V-cycles of each of its solves); only cost ratios enter step 3.
 * The plan's description fixes n0, the field, the solver and max_level
 * (>= 1, at most MLMC_MAX_LEVELS - 1). */
#define MLMC_MAX_LEVELS 11
#define MLMC_MAX_TRACE 64
typedef struct {
  double eps;       /* target root mean square error (> 0)                       */
  double theta;     /* share of eps^2 given to the sampling error, in (0, 1)     */
  double alpha;     /* bias rate: |E[Q_l - Q]| ~ M_l^-alpha, M_l ~ 8^l M_0 (> 0) */
  int n_init;       /* N_Init (>= 2)                                             */
  int max_iter;     /* rounds of steps 2-4 at most (>= 1)                        */
  int max_batch;    /* samples per device batch (>= 1)                           */
  uint64_t seed0;   /* sample i of every level uses seed seed0 + i               */
} mlmc_adaptive_desc;

typedef struct {
  int status;                         /* MG_OK                                    */
  int L;                              /* finest level used                        */
  int iterations;                     /* rounds of steps 2-4                      */
  int bias_ok;                        /* 1 if the bias estimate is <= eps_b       */
  long long N[MLMC_MAX_LEVELS];       /* samples per level (levels 0..L)          */
  double mean[MLMC_MAX_LEVELS];       /* Yhat_l                                   */
  double var[MLMC_MAX_LEVELS];        /* s_l^2, divisor N_l                       */
  double cost[MLMC_MAX_LEVELS];       /* C_l in node-cycles per sample            */
  double Q;                           /* sum of the level means (compensated)     */
  double sampling_rms;                /* sqrt(sum_l s_l^2 / N_l)                   */
  double bias_estimate;               /* |Yhat_L| / (8^alpha - 1)                 */
  int trace_len;                      /* rounds recorded below (<= MLMC_MAX_TRACE) */
  int trace_L[MLMC_MAX_TRACE];        /* L after step 3 of each round             */
  long long trace_N[MLMC_MAX_TRACE][MLMC_MAX_LEVELS];  /* N_l after step 3       */
} mlmc_adaptive_result;

/* Defaults: eps = 1e-3, theta = 0.5, alpha = 2/3, N_Init = 32, 64 rounds,
 * batches of 256, seed0 = 0. */
void mlmc_adaptive_desc_default(mlmc_adaptive_desc* d);
/* Run Algorithm 2 on the plan.  *desc and *result are host memory (result
 * caller-owned, fully overwritten).  Blocking.  Returns MG_OK, MG_EINVAL (bad
 * description, or a plan with max_level < 1), MG_ENOCONV (a solve missed
 * its tolerance; the run stops there), MG_ENOMEM or MG_EHIP. */
int mlmc_adaptive(mg_plan plan, const mlmc_adaptive_desc* desc, mlmc_adaptive_result* result);

/* Kernel timing: when enabled, the plan records HIP events around every
 * smoothing sweep on the finest grids of a batch (the top grids of each
 * stage under FMG; both colour passes of a finite-element sweep; both
 * colour passes of a sweep on the SPDE sampler's finest box grid), on the
 * plan's stream, and runs its cycles eagerly.  mg_profile_read returns the
 * number of such launches and their summed duration in milliseconds since
 * the last reset. */
int mg_profile_enable(mg_plan plan, int on);
int mg_profile_read(mg_plan plan, long long* launches, double* total_ms, double* nodes_per_launch);
/* The timed sweeps one by one (since the last mg_profile_enable), in launch
 * order: cycle[i] is the V-cycle of its batch or box solve it belongs to
 * (1-based; each batch restarts the count), kind[i] the sweep (0 plain,
 * 1 with the coarse-grid correction, 2 with the residual norm of its
 * output's black points, 3 with the residual norm of its input's red
 * points, 4 finite-element colour passes, 5 SPDE box colour passes),
 * grid_n[i] the vertices per axis of its grids, ms[i] its duration.  Host
 * arrays of max_out entries; *n_out receives the number of records (which
 * may exceed max_out; only max_out are written). */
int mg_profile_records(mg_plan plan, int max_out, int* cycle, int* kind, int* grid_n, double* ms,
                       int* n_out);

const char* mg_last_error(mg_plan plan);

#ifdef __cplusplus
}
#endif
#endif
