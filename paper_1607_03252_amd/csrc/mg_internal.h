// Internal interfaces of libmlmcmg: device descriptors and kernel launchers.
//
// Storage: an n^3 vertex grid, z (k) fastest, boundary vertices included.
// The coefficient is kept as wh = 1/(2k) per vertex, so the harmonic-mean face
// coefficient 2 k_p k_q / (k_p + k_q) is the single reciprocal 1/(wh_p + wh_q).
// Right-hand sides are h^2-scaled: b' = h^2 f, so every level's operator is
// (A'u)_p = D_p u_p - sum_q c_pq u_q with D_p = sum_q c_pq.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

// One grid of one solve at one multigrid level.
struct GridDesc {
  double* u[2];       // iterate; u[1] is the second buffer of the out-of-place smoother
  const double* wh;   // 1/(2k) at all n^3 vertices
  double* b;          // h^2-scaled right-hand side, or nullptr for the constant bconst
  double* r;          // residual scratch, n^3 (nullptr on the coarsest grid)
  double* uc;         // u[0] of the next coarser grid of the same solve (nullptr on 3^3)
  double* bc;         // b of the next coarser grid
  float* u32;         // single-precision twins (mixed precision inner cycles)
  const float* wh32;
  float* b32;
  float* r32;
  float* uc32;
  float* bc32;
  double bconst;      // used when b == nullptr
  int solve;          // owning solve: index into per-solve arrays
  int n;              // vertices per axis
  int poff;           // offset of this grid's reduction partials (top grids only)
  int pad_;
};

// Per-solve device state of a batch.
struct SolveState {
  int* active;        // 1 while the solve still cycles
  int* cycles;        // cycles done when it stopped, -1 if it missed tol
  double* relres;     // last relative residual
  double* bnorm;      // ||b'||_2 (1 when b' = 0)
  double* q;          // QoI of the solve's top grid
  double* partials;   // reduction partials
};

enum ReduceMode { RED_BNORM = 0, RED_RESID = 1, RED_QOI = 2 };

// Reduction partial count of one grid of size n (256-thread blocks over the
// interior vertices).
__host__ __device__ inline int reduce_blocks(int n) {
  const long m = n - 2;
  return (int)((m * m * m + 255) / 256);
}

// ---- launchers (all asynchronous on `st`) --------------------------------
// Random numbers and fields.
void launch_philox(const uint64_t* d_seeds, int count, int level, uint32_t* d_words,
                   double* d_normals, hipStream_t st);
// wh (mode 0) or k (mode 1) of the field sum_abc coef[abc] xi_s[abc] phi_a phi_b phi_c
// on `count` grids of size n.  out[g] = destination of grid g, xi_index[g] = its
// sample's row of d_normals.
void launch_field(int n, int count, double* const* d_out, const int* d_xi_index,
                  const double* d_normals, const double* d_phi, const double* d_coef,
                  int mode, hipStream_t st);
void launch_inject(int n_fine, int count, const double* const* d_fine, double* const* d_coarse,
                   hipStream_t st);
// wh = 1/(2k) and b = h^2 f for a caller-supplied problem.
void launch_prepare_problem(int n, const double* k, const double* f, double* wh, double* b,
                            double* u, hipStream_t st);

// Multigrid steps on a list of `count` grids of size n (device list).
void launch_rbgs_colour(const GridDesc* d_list, int count, int n, const int* d_active,
                        int colour, int buf, hipStream_t st);
void launch_residual(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                     hipStream_t st);
void launch_restrict(const GridDesc* d_list, int count, int n, const int* d_active,
                     hipStream_t st);
void launch_coarsest(const GridDesc* d_list, int count, const int* d_active, hipStream_t st);
void launch_prolong(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                    hipStream_t st);
// u[0] (and u[1] if present) = 0 on every vertex of the listed grids.
void launch_zero_u(const GridDesc* d_list, int count, int n, hipStream_t st);
void launch_copy_buf(const GridDesc* d_list, int count, int n, const int* d_active, int from,
                     hipStream_t st);

// Reductions on the top grids of solves (list of `count` grids of size n).
void launch_reduce(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                   int mode, double* d_partials, hipStream_t st);
// Finalise per solve: modes as ReduceMode.  `cycle` is the cycle just done,
// `fixed_cycles` > 0 selects fixed-count mode.
void launch_finalize(const GridDesc* d_list, int count, int n, SolveState s, int mode,
                     int cycle, int fixed_cycles, int max_cycles, double tol, hipStream_t st);
void launch_count_active(const int* d_active, int nsolves, int* d_count, hipStream_t st);
void launch_ydiff(const double* d_q, const int* d_fine_idx, const int* d_coarse_idx, int count,
                  double* d_y, double* d_qf, double* d_qc, const int* d_cycles, int* d_cycles_out,
                  hipStream_t st);

}  // namespace mg
