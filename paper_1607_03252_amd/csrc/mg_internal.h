// Internal interfaces of libmlmcmg: device descriptors and kernel launchers.
//
// Storage: an n^3 vertex grid, z (k) fastest, boundary vertices included,
// n <= 1025 so every offset fits in 32 bits.  The coefficient is kept as
// wh = 1/(2k) per vertex, so the harmonic-mean face coefficient
// 2 k_p k_q / (k_p + k_q) is the single reciprocal 1/(wh_p + wh_q).
// Right-hand sides are h^2-scaled: b' = h^2 f, so every level's operator is
// (A'u)_p = D_p u_p - sum_q c_pq u_q with D_p = sum_q c_pq.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4x32 bijection on counter c under key (k0, k1), in place.  One definition
// for the device kernel and the host export: the high word of each 32x32-bit
// product is taken from the 64-bit product (the device compiler maps it to
// its multiply-high instruction).
__host__ __device__ __forceinline__ void philox_block(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// One grid of one solve at one multigrid level, in precision T.
template <typename T>
struct GridDescT {
  T* u[2];          // iterate: the smoother reads u[buf] and writes u[1-buf]
  const T* wh;      // 1/(2k) at all n^3 vertices
  const T* fc;      // P1 finite-element operator only: the couplings of every
                    // vertex to its +i, +j and +k neighbours, three n^3 arrays
                    // one after the other (nullptr for the FD operator)
  T* b;             // h^2-scaled right-hand side: b[i*bstride + j*n + k] (bstride 0:
                    // one n^2 plane holding a constant right-hand side)
  T* r;             // residual scratch, n^3 (nullptr on 3^3)
  T* uc[2];         // the coarser grid's iterate buffers (nullptr on 3^3)
  T* bc;            // the coarser grid's right-hand side
  double bconst;    // value of a constant right-hand side (h^2 for f = 1)
  int solve;        // owning solve: index into per-solve arrays
  int n;            // vertices per axis
  int poff;         // offset of this grid's reduction partials (top grids only)
  int spoff;        // top grids: offset of the in-sweep residual-norm partials
                    // (SolveState::spart); -1 otherwise
  int bstride;      // n*n for a full right-hand side array, 0 for a constant plane
  // The KL coefficient evaluated in the kernel instead of read from wh (FP64
  // smoother and transfer launches with kl = true): the solve's 64 normals,
  // the 64 mode weights, and the 1D modes at this grid's vertex coordinates
  // (klphi[a*n + i]).  The kernels form wh = exp(-Z)/2 in the operations of
  // the field kernel that wrote wh, so they see the same values.  nullptr:
  // the grid's coefficient is not such a field.
  const double* kln;
  const double* klcoef;
  const double* klphi;
};
using GridDesc = GridDescT<double>;
using GridDesc32 = GridDescT<float>;

// One grid of size 17, 9 or 5 and its coarser grids down to 3^3 (lv[0] is
// the largest), for the small-grid V-cycle kernel.
template <typename T>
struct SmallChain {
  GridDescT<T> lv[4];
};

// Per-solve device state of a batch.
struct SolveState {
  int* active;      // 1 while the solve still cycles
  int* cycles;      // cycles done when it stopped, -1 if it missed tol
  double* relres;   // last relative residual
  double* bnorm;    // ||b'||_2 (1 when b' = 0)
  double* q;        // QoI of the solve's top grid
  double* partials; // reduction partials
  int* ran;         // V-cycles credited to the solve so far: the judgement of
                    // each outer step adds that step's cycles
  int* qpend;       // 1 from admission until the QoI of a stopped solve is taken
  double* spart;    // per solve 2 x kSweepParts + 2: in-sweep residual-norm
                    // partials (black points of the output of a cycle's last
                    // sweep, red points of the input of the next cycle's first
                    // sweep), then the two partial counts
};

// Workgroups per grid that a sweep computing the residual norm may use (the
// capacity of SolveState::spart per solve).
constexpr int kSweepParts = 1024;

// RED_QOI_PENDING: the QoI of solves that have stopped (active 0) but whose
// QoI is still pending (qpend 1); it clears qpend.  RED_COUNT (finalise
// only): a fixed schedule's step without a residual, see launch_finalize2.
enum ReduceMode {
  RED_BNORM = 0,
  RED_RESID = 1,
  RED_QOI = 2,
  RED_QOI_PENDING = 3,
  RED_R2 = 4,
  RED_COUNT = 5
};
// QoI kinds (Section 3): the integral of u, u(1/4,1/4,1/4), the flux across x_2 = 1/4
enum QoiKind { QOI_INTEGRAL = 0, QOI_POINT = 1, QOI_FLUX = 2 };

// Point kernels cover the interior (or, for the "full" kernels, every vertex)
// with 256-thread blocks of 4 rows (j) x 64 columns (k) of one plane i.
__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ inline long ceil_div_l(long a, long b) { return (a + b - 1) / b; }
__host__ __device__ inline int point_blocks(int m) { return m * ceil_div(m, 4) * ceil_div(m, 64); }
// Column-marching kernels (residual, reductions): one 256-thread block per
// 4 x 64 interior columns; reductions keep one partial per block.
__host__ __device__ inline int reduce_blocks(int n) {
  return ceil_div(n - 2, 4) * ceil_div(n - 2, 64);
}

// Tile shape of the fused smoother: TJ rows (j) x TK columns (k), streamed
// over planes i in `chunks` pieces.
struct SweepShape {
  int tj, tk, chunks;
};
// Shapes with compiled kernels for grid size n (TJ, TK divide n-1).
int sweep_shapes(int n, SweepShape* out, int max_out);
// fused_correction: the sweep that also adds the coarse correction;
// single: FP32 sweeps (the inner cycles of mixed precision)
SweepShape default_sweep_shape(int n, bool fused_correction = false, bool single = false);
// Whether the fused smoother can run on grids of size n with elements of
// elem bytes: it addresses a whole grid array with 32-bit byte offsets, so the
// array must stay below 2 GiB (larger grids use the two-pass colour sweeps).
bool sweep_fits(int n, size_t elem);

// exp as the kernels form the KL coefficient (table-driven, below 2 ulp),
// evaluated on the host
double kl_exp_host(double x);

// ---- launchers (all asynchronous on `st`) --------------------------------
// Normals of `count` samples; the counter's level word is d_levels[s] when
// d_levels is given, else `level`.
void launch_philox(const uint64_t* d_seeds, int count, int level, uint32_t* d_words,
                   double* d_normals, hipStream_t st, const int* d_levels = nullptr);
// wh (mode 0) or k (mode 1) of the KL field on `count` grids of size n.
void launch_field(int n, int count, double* const* d_out, const int* d_xi_index,
                  const double* d_normals, const double* d_phi, const double* d_coef,
                  int mode, hipStream_t st);
void launch_inject(int n_fine, int count, const double* const* d_fine, double* const* d_coarse,
                   hipStream_t st);
// float copies of `count` arrays of n^3 doubles
void launch_to_float(int n, int count, const double* const* d_src, float* const* d_dst,
                     hipStream_t st);
// wh = 1/(2k), b = h^2 f and a zero boundary for u, for a caller's problem.
void launch_prepare_problem(int n, const double* k, const double* f, double* wh, double* b,
                            double* u, hipStream_t st);

// Fill `count` doubles with `value`.
void launch_fill(double* p, long count, double value, hipStream_t st);

// Multigrid steps on a device list of `count` grids of size n.
// The fused smoother: one red-black sweep from u[buf] into u[1-buf]; with
// cbuf_prolong >= 0 the input is first corrected by the trilinear
// interpolation of the coarse iterate uc[cbuf_prolong].  With spart (FP64,
// no correction) it also writes, for every grid with spoff >= 0, one partial
// per workgroup to spart[spoff + wg]: the sum of squared residuals at the red
// points of its input (norm 1) or at the black points of its output (norm 2).
// const_b: every grid of the list has a constant right-hand side plane
// (bstride 0).  kl: every grid has a KL coefficient (kln != nullptr), which
// the FP64 sweep then evaluates instead of reading wh where the list also has
// a constant right-hand side and n <= kKLMaxN (the results are the same
// either way).  Returns the workgroups per grid.
template <typename T>
int launch_sweep(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                 int cbuf_prolong, SweepShape shape, hipStream_t st, T* spart = nullptr,
                 int norm = 0, bool const_b = false, bool kl = false);
// Largest grid on which the kernels evaluate the KL coefficient themselves
// (its 1D mode table is staged in LDS).
constexpr int kKLMaxN = 257;
// Workgroups per grid of launch_sweep for `count` grids of size n.
int sweep_blocks(int n, int count, SweepShape shape);
template <typename T>
void launch_rbgs_colour(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                        int colour, int buf, hipStream_t st);
template <typename T>
void launch_residual(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                     hipStream_t st);
template <typename T>
void launch_restrict(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                     hipStream_t st);
// Residual of u[buf] and full weighting into bc, in one pass (r is not stored);
// each tile's plane march is split into resrestrict_chunks(n, count) pieces.
int resrestrict_chunks(int n, int count);
template <typename T>
void launch_resrestrict(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                        int buf, hipStream_t st, bool const_b = false, bool kl = false);
template <typename T>
void launch_coarsest(const GridDescT<T>* d_list, int count, const int* d_active, hipStream_t st);
template <typename T>
void launch_prolong(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                    int cbuf, hipStream_t st);
template <typename T>
void launch_copy_buf(const GridDescT<T>* d_list, int count, int n, const int* d_active, int from,
                     hipStream_t st);
// u[0] = 0 on every vertex of the listed grids (u[1] needs no clearing: the
// first sweep of a level writes all its interior points before any read).
template <typename T>
void launch_zero_u(const GridDescT<T>* d_list, int count, int n, hipStream_t st);

// The rest of a V(nu1,nu2) cycle from grids of size ns (17, 9 or 5) down,
// one workgroup per chain, in LDS; the iterate stays in u[0].
template <typename T>
void launch_vsmall(const SmallChain<T>* d_chains, int count, int ns, const int* d_active, int nu1,
                   int nu2, hipStream_t st);

// Reductions on the top grids of solves.
// d_pend: the solves' qpend flags (RED_QOI_PENDING only).
void launch_reduce(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                   int mode, double* d_partials, hipStream_t st, const int* d_pend = nullptr);
// Mixed precision: r = b' - A'u in FP64 on the top grids, stored rounded to
// FP32 as the inner right-hand side d_list32[g].b (whose u[0] is zeroed),
// plus the partial sums of r^2.
void launch_defect(const GridDesc* d_list, const GridDesc32* d_list32, int count, int n,
                   const int* d_active, double* d_partials, hipStream_t st);
// Mixed precision: u[0] += (double) e32 on the top grids.
void launch_correct(const GridDesc* d_list, const GridDesc32* d_list32, int count, int n,
                    const int* d_active, int buf32, hipStream_t st);
// Finalise per solve.  RED_RESID runs once per outer step for every active
// solve: it credits the step's `step` cycles to the solve (ran += step) and
// judges the iterate after ran - lag cycles (an iterate before the first
// cycle is never judged); fixed_cycles > 0 selects fixed-count mode.
// RED_RESID with sweep_parts > 0 sums the in-sweep partials instead of the
// reduction's: spart[spoff + q] and
// spart[spoff + kSweepParts + q] for the counts the sweeps stored at
// spart[spoff + 2 kSweepParts] and [... + 1] (sweep_parts_red is unused).
// RED_COUNT credits the step to every active solve and stops it once it has
// run fixed_cycles, reading no partials (a schedule that needs no residual).
void launch_finalize2(const GridDesc* d_list, int count, SolveState s, int mode, int step,
                      int lag, int fixed_cycles, int max_cycles, double tol, hipStream_t st,
                      int sweep_parts = 0, int sweep_parts_red = 0);
// active = 1, cycles = 0, ran = 0, qpend = qpend.
void launch_init_state2(SolveState s, int ns, hipStream_t st, int qpend = 0);
// Start the listed solves now: active = 1, cycles = 0, ran = 0, qpend = 1.
void launch_admit(const int* d_solves, int count, SolveState s, hipStream_t st);
void launch_ydiff(const double* d_q, const int* d_fine_idx, const int* d_coarse_idx, int count,
                  double* d_y, double* d_qf, double* d_qc, const int* d_cycles, int* d_cycles_out,
                  hipStream_t st);

// Point or flux QoI (QOI_POINT, QOI_FLUX) of the listed top grids (u[0])
// into d_q[solve]; one workgroup per grid.
void launch_qoi_pf(const GridDesc* d_list, int count, int mode, double* d_q, hipStream_t st);
// Y = Q_f - Q_c per sample from two per-solve QoI arrays (d_qc may be null:
// level 0), with fixed cycle counts cyc_f, cyc_c; sample t is written at
// output position d_pos[t].
void launch_ydiff2(const double* d_qf, const double* d_qc, int count, const int* d_pos,
                   double* d_y, double* d_qf_out, double* d_qc_out, int cyc_f, int cyc_c,
                   int* d_cycles_out, hipStream_t st);

// P1 finite elements (FP64): the axis couplings fc of `count` grids of size
// n from their wh (k = 1/(2 wh)); d_wh[g] and d_fc[g] per grid.
void launch_fe_faces(int n, int count, const double* const* d_wh, double* const* d_fc,
                     hipStream_t st);
// In-place Gauss-Seidel on one colour, residual into r, and the 3^3 solve,
// with the operator given by the grids' fc.
void launch_fe_colour(const GridDesc* d_list, int count, int n, const int* d_active, int colour,
                      hipStream_t st);
void launch_fe_residual(const GridDesc* d_list, int count, int n, const int* d_active,
                        hipStream_t st);
void launch_fe_coarsest(const GridDesc* d_list, int count, const int* d_active, hipStream_t st);

// ---- SPDE field sampler: (kappa^2 - Laplace) Z = W on the box (-1,2)^3 ----
// One grid of one SPDE solve: the box grid at spacing h (nt = 3(n-1)+1
// vertices per axis on the finest level), every vertex an unknown (natural
// Neumann boundary), z fastest like the solver's grids.
struct SpdeGrid {
  double* z;      // iterate
  double* b;      // scaled load (restricted residual on coarse levels)
  double* r;      // residual scratch
  double* zc;     // the next coarser level's z (nullptr on the coarsest)
  double* bc;     // the next coarser level's b
  double k2h2;    // kappa^2 h^2 of this level
  int nt;         // vertices per axis
  int solve;      // index into the active / cycle arrays
};
// load b_p = sqrt(h m_p) xi_p of `count` grids from the white noise of
// (seeds[g], levels[g]): Philox counter (j, level, 1, 0), normals 2j, 2j+1
void launch_spde_noise(const SpdeGrid* d_list, int count, int nt, const uint64_t* d_seeds,
                       const int* d_levels, double h, hipStream_t st);
void launch_spde_colour(const SpdeGrid* d_list, int count, int nt, const int* d_active, int colour,
                        hipStream_t st);
void launch_spde_residual(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                          hipStream_t st);
// bc = P^T r / 2 on the next coarser level (and zc = 0); with from_b, of b
// instead of r (the load of the same noise on a coarser box grid)
void launch_spde_restrict(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                          bool from_b, hipStream_t st);
void launch_spde_prolong(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                         hipStream_t st);
// 32 red-black sweeps on an odd-interval coarsest grid (one workgroup per grid)
void launch_spde_coarsest(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                          hipStream_t st);
// per-grid partial sums of r^2 (which = 0) or b^2 (which = 1): spde_blocks(nt) per grid
int spde_blocks(int nt);
void launch_spde_sumsq(const SpdeGrid* d_list, int count, int nt, const int* d_active, int which,
                       double* d_partials, hipStream_t st);
// judge after a cycle: relres = sqrt(sum r^2) / bnorm; with bnorm_mode, store
// bnorm = sqrt(sum b^2) instead
void launch_spde_judge(const SpdeGrid* d_list, int count, int nt, int* d_active, int* d_cycles,
                       double* d_bnorm, const double* d_partials, int cycle, double tol,
                       int max_cycles, int bnorm_mode, hipStream_t st);
// wh = exp(-s z) / 2 (mode 0) or k = exp(s z) (mode 1) at the n^3 vertices
// of D (box index i + n - 1)
void launch_spde_field(const SpdeGrid* d_list, int count, int n, double s, double* const* d_wh,
                       int mode, hipStream_t st);

}  // namespace mg
