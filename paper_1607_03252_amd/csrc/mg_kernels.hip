// Device kernels of libmlmcmg (gfx950, wave64).
//
// Every multigrid kernel takes a device list of GridDesc of one grid size and
// runs blockIdx.y over the list, so one launch advances every sample of a
// batch that has a grid of that size (sample parallelism inside one launch).
// A per-solve `active` flag freezes solves that have converged.
#include "mg_internal.h"

namespace mg {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ size_t vidx(int n, int i, int j, int k) {
  return ((size_t)i * (size_t)n + (size_t)j) * (size_t)n + (size_t)k;
}

// Harmonic-mean face coefficients of vertex p and the stencil sums
// D = sum_q c_pq, S = sum_q c_pq u_q, neighbours in the order i-1, i+1,
// j-1, j+1, k-1, k+1.  u is zero on boundary vertices.
__device__ __forceinline__ void stencil(const double* __restrict__ u,
                                        const double* __restrict__ wh, size_t p,
                                        size_t sj, size_t si, double& D, double& S) {
  const double w = wh[p];
  const double c0 = 1.0 / (w + wh[p - si]);
  const double c1 = 1.0 / (w + wh[p + si]);
  const double c2 = 1.0 / (w + wh[p - sj]);
  const double c3 = 1.0 / (w + wh[p + sj]);
  const double c4 = 1.0 / (w + wh[p - 1]);
  const double c5 = 1.0 / (w + wh[p + 1]);
  D = c0 + c1 + c2 + c3 + c4 + c5;
  S = c0 * u[p - si] + c1 * u[p + si] + c2 * u[p - sj] + c3 * u[p + sj] + c4 * u[p - 1] +
      c5 * u[p + 1];
}

__device__ __forceinline__ double block_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (ws[0] + ws[1]) + (ws[2] + ws[3]);
  return t;
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ----------------------
__device__ __forceinline__ void philox_block(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// One 64-thread block per sample: 32 Philox blocks -> 128 words -> 64
// uniforms on (0,1] with 53 random bits -> 32 Box-Muller pairs.
__global__ void __launch_bounds__(64) k_philox(const uint64_t* __restrict__ seeds, int level,
                                               uint32_t* __restrict__ words,
                                               double* __restrict__ normals) {
  __shared__ uint32_t w[128];
  __shared__ double U[64];
  const int s = blockIdx.x, t = threadIdx.x;
  const uint64_t seed = seeds[s];
  if (t < 32) {
    uint32_t c[4] = {(uint32_t)t, (uint32_t)level, 0u, 0u};
    philox_block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int q = 0; q < 4; ++q) w[4 * t + q] = c[q];
  }
  __syncthreads();
  if (words)
    for (int q = t; q < 128; q += 64) words[(size_t)s * 128 + q] = w[q];
  const uint64_t M = ((uint64_t)(w[2 * t] >> 5) << 26) | (uint64_t)(w[2 * t + 1] >> 6);
  U[t] = (double)(M + 1) * 0x1p-53;
  __syncthreads();
  if (normals && t < 32) {
    const double R = sqrt(-2.0 * log(U[2 * t]));
    const double a = 6.283185307179586 * U[2 * t + 1];
    normals[(size_t)s * 64 + 2 * t] = R * cos(a);
    normals[(size_t)s * 64 + 2 * t + 1] = R * sin(a);
  }
}

// Field on `count` grids of size n: Z = sum_{a,b,c} coef[abc] xi[abc]
// phi_a(x_i) phi_b(y_j) phi_c(z_k), summed as nested 1D contractions over a,
// then b, then c.  mode 0 stores wh = exp(-Z)/2, mode 1 stores k = exp(Z).
__global__ void __launch_bounds__(kBlock) k_field(int n, double* const* __restrict__ out,
                                                  const int* __restrict__ xi_index,
                                                  const double* __restrict__ normals,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ coef, int mode) {
  __shared__ double C[64];
  const int g = blockIdx.y;
  if (threadIdx.x < 64)
    C[threadIdx.x] = coef[threadIdx.x] * normals[(size_t)xi_index[g] * 64 + threadIdx.x];
  __syncthreads();
  const size_t N = (size_t)n * n * n;
  const size_t v = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= N) return;
  const int k = (int)(v % n), j = (int)((v / n) % n), i = (int)(v / ((size_t)n * n));
  double px[4], py[4], pz[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    px[a] = phi[a * n + i];
    py[a] = phi[a * n + j];
    pz[a] = phi[a * n + k];
  }
  double Z = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double g2 = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double g1 = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) g1 += C[16 * a + 4 * b + c] * px[a];
      g2 += g1 * py[b];
    }
    Z += g2 * pz[c];
  }
  out[g][v] = mode == 0 ? 0.5 * exp(-Z) : exp(Z);
}

__global__ void __launch_bounds__(kBlock) k_inject(int nf, const double* const* __restrict__ fine,
                                                   double* const* __restrict__ coarse) {
  const int nc = (nf - 1) / 2 + 1;
  const size_t Nc = (size_t)nc * nc * nc;
  const size_t v = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= Nc) return;
  const int K = (int)(v % nc), J = (int)((v / nc) % nc), I = (int)(v / ((size_t)nc * nc));
  coarse[blockIdx.y][v] = fine[blockIdx.y][vidx(nf, 2 * I, 2 * J, 2 * K)];
}

__global__ void __launch_bounds__(kBlock) k_prepare(int n, const double* __restrict__ k,
                                                    const double* __restrict__ f,
                                                    double* __restrict__ wh,
                                                    double* __restrict__ b,
                                                    double* __restrict__ u) {
  const size_t N = (size_t)n * n * n;
  const size_t v = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= N) return;
  const int kk = (int)(v % n), j = (int)((v / n) % n), i = (int)(v / ((size_t)n * n));
  const bool bnd = i == 0 || j == 0 || kk == 0 || i == n - 1 || j == n - 1 || kk == n - 1;
  const double h = 1.0 / (double)(n - 1);
  wh[v] = 0.5 / k[v];
  b[v] = bnd ? 0.0 : h * h * f[v];
  if (bnd) u[v] = 0.0;
}

// ---- smoothing, residual, transfer ------------------------------------------

// Gauss-Seidel update of the interior vertices of one colour ((i+j+k) even =
// red, odd = black): u_p <- (b'_p + sum_q c_pq u_q) / D_p, in place.
__global__ void __launch_bounds__(kBlock) k_rbgs_colour(const GridDesc* __restrict__ list,
                                                        const int* __restrict__ active,
                                                        int colour, int buf) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n, m = n - 2, W = (n - 1) / 2;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long)m * m * W) return;
  const int row = (int)(t / W), kh = (int)(t - (long)row * W);
  const int i = 1 + row / m, j = 1 + row % m;
  const int k = 1 + 2 * kh + ((colour + i + j + 1) & 1);
  if (k > n - 2) return;
  const size_t sj = (size_t)n, si = (size_t)n * n;
  const size_t p = vidx(n, i, j, k);
  double* u = d.u[buf];
  double D, S;
  stencil(u, d.wh, p, sj, si, D, S);
  const double bp = d.b ? d.b[p] : d.bconst;
  u[p] = (bp + S) / D;
}

__global__ void __launch_bounds__(kBlock) k_residual(const GridDesc* __restrict__ list,
                                                     const int* __restrict__ active, int buf) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n, m = n - 2;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long)m * m * m) return;
  const int k = 1 + (int)(t % m), j = 1 + (int)((t / m) % m), i = 1 + (int)(t / ((long)m * m));
  const size_t p = vidx(n, i, j, k);
  const double* u = d.u[buf];
  double D, S;
  stencil(u, d.wh, p, (size_t)n, (size_t)n * n, D, S);
  const double bp = d.b ? d.b[p] : d.bconst;
  d.r[p] = bp - (D * u[p] - S);
}

// Full weighting of the residual to the coarse right-hand side, h^2 scaling
// included: b'_c(I) = 4 * sum_d 2^{-|d|_1}/8 r'(2I+d); also starts the coarse
// cycle from a zero iterate.
__global__ void __launch_bounds__(kBlock) k_restrict(const GridDesc* __restrict__ list,
                                                     const int* __restrict__ active) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n, nc = (n - 1) / 2 + 1, mc = nc - 2;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long)mc * mc * mc) return;
  const int K = 1 + (int)(t % mc), J = 1 + (int)((t / mc) % mc), I = 1 + (int)(t / ((long)mc * mc));
  const double* r = d.r;
  double s = 0.0;
  for (int di = -1; di <= 1; ++di) {
    const double wi = di == 0 ? 1.0 : 0.5;
    for (int dj = -1; dj <= 1; ++dj) {
      const double wj = dj == 0 ? wi : 0.5 * wi;
      const size_t row = vidx(n, 2 * I + di, 2 * J + dj, 2 * K);
      s += wj * (r[row] + 0.5 * (r[row - 1] + r[row + 1]));
    }
  }
  const size_t pc = vidx(nc, I, J, K);
  d.bc[pc] = 0.5 * s;
  d.uc[pc] = 0.0;
}

// 3^3 grid: one unknown, solved exactly.
__global__ void k_coarsest(const GridDesc* __restrict__ list, int count,
                           const int* __restrict__ active) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const GridDesc d = list[g];
  if (!active[d.solve]) return;
  const size_t p = 13;
  const double w = d.wh[p];
  const double D = 1.0 / (w + d.wh[p - 9]) + 1.0 / (w + d.wh[p + 9]) + 1.0 / (w + d.wh[p - 3]) +
                   1.0 / (w + d.wh[p + 3]) + 1.0 / (w + d.wh[p - 1]) + 1.0 / (w + d.wh[p + 1]);
  const double bp = d.b ? d.b[p] : d.bconst;
  d.u[0][p] = bp / D;
}

// u_f += P e_c with trilinear P; coarse boundary values are stored as zero.
__global__ void __launch_bounds__(kBlock) k_prolong(const GridDesc* __restrict__ list,
                                                    const int* __restrict__ active, int buf) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n, m = n - 2, nc = (n - 1) / 2 + 1;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long)m * m * m) return;
  const int k = 1 + (int)(t % m), j = 1 + (int)((t / m) % m), i = 1 + (int)(t / ((long)m * m));
  const double* e = d.uc;
  const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
  const int ni = (i & 1) + 1, nj = (j & 1) + 1, nk = (k & 1) + 1;
  const double wi = (i & 1) ? 0.5 : 1.0, wj = (j & 1) ? 0.5 : 1.0, wk = (k & 1) ? 0.5 : 1.0;
  double s = 0.0;
  for (int a = 0; a < ni; ++a)
    for (int b = 0; b < nj; ++b) {
      const size_t row = vidx(nc, i0 + a, j0 + b, k0);
      double z = e[row];
      if (nk == 2) z = z + e[row + 1];
      s += wi * wj * wk * z;
    }
  d.u[buf][vidx(n, i, j, k)] += s;
}

__global__ void __launch_bounds__(kBlock) k_zero_u(const GridDesc* __restrict__ list) {
  const GridDesc d = list[blockIdx.y];
  const int n = d.n;
  const size_t N = (size_t)n * n * n;
  const size_t v = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= N) return;
  d.u[0][v] = 0.0;
  if (d.u[1]) d.u[1][v] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_copy_buf(const GridDesc* __restrict__ list,
                                                     const int* __restrict__ active, int from) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n;
  const size_t N = (size_t)n * n * n;
  const size_t v = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= N) return;
  d.u[1 - from][v] = d.u[from][v];
}

// ---- reductions ---------------------------------------------------------------
// Per-block partial sums over interior vertices of: b'^2 (RED_BNORM),
// (b' - A'u)^2 (RED_RESID) or u (RED_QOI).  Fixed block decomposition per
// grid size, so the result of a solve never depends on the rest of the batch.
__global__ void __launch_bounds__(kBlock) k_reduce(const GridDesc* __restrict__ list,
                                                   const int* __restrict__ active, int buf,
                                                   int mode, double* __restrict__ partials) {
  const GridDesc d = list[blockIdx.y];
  if (mode == RED_RESID && !active[d.solve]) return;
  const int n = d.n, m = n - 2;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  double v = 0.0;
  if (t < (long)m * m * m) {
    const int k = 1 + (int)(t % m), j = 1 + (int)((t / m) % m), i = 1 + (int)(t / ((long)m * m));
    const size_t p = vidx(n, i, j, k);
    const double* u = d.u[buf];
    const double bp = d.b ? d.b[p] : d.bconst;
    if (mode == RED_BNORM) {
      v = bp * bp;
    } else if (mode == RED_RESID) {
      double D, S;
      stencil(u, d.wh, p, (size_t)n, (size_t)n * n, D, S);
      const double r = bp - (D * u[p] - S);
      v = r * r;
    } else {
      v = u[p];
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[d.poff + blockIdx.x] = v;
}

__global__ void __launch_bounds__(kBlock) k_finalize(const GridDesc* __restrict__ list,
                                                     SolveState s, int mode, int cycle,
                                                     int fixed_cycles, int max_cycles,
                                                     double tol) {
  const GridDesc d = list[blockIdx.x];
  const int sv = d.solve;
  if (mode == RED_RESID && !s.active[sv]) return;
  const int P = reduce_blocks(d.n);
  double v = 0.0;
  for (int q = threadIdx.x; q < P; q += kBlock) v += s.partials[d.poff + q];
  v = block_sum(v);
  if (threadIdx.x != 0) return;
  if (mode == RED_BNORM) {
    const double nb = sqrt(v);
    s.bnorm[sv] = nb > 0.0 ? nb : 1.0;
  } else if (mode == RED_RESID) {
    const double rho = sqrt(v) / s.bnorm[sv];
    s.relres[sv] = rho;
    if (fixed_cycles > 0) {
      if (cycle >= fixed_cycles) {
        s.active[sv] = 0;
        s.cycles[sv] = cycle;
      }
    } else if (rho <= tol) {
      s.active[sv] = 0;
      s.cycles[sv] = cycle;
    } else if (cycle >= max_cycles) {
      s.active[sv] = 0;
      s.cycles[sv] = -1;
    }
  } else {
    const double h = 1.0 / (double)(d.n - 1);
    s.q[sv] = h * h * h * v;
  }
}

__global__ void __launch_bounds__(kBlock) k_count_active(const int* __restrict__ active, int ns,
                                                         int* __restrict__ count) {
  double c = 0.0;
  for (int q = threadIdx.x; q < ns; q += kBlock) c += (double)active[q];
  c = block_sum(c);
  if (threadIdx.x == 0) *count = (int)c;
}

__global__ void k_ydiff(const double* __restrict__ q, const int* __restrict__ fi,
                        const int* __restrict__ ci, int count, double* __restrict__ y,
                        double* __restrict__ qf, double* __restrict__ qc,
                        const int* __restrict__ cyc, int* __restrict__ cyc_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const double a = q[fi[t]];
  const double b = ci[t] >= 0 ? q[ci[t]] : 0.0;
  y[t] = a - b;
  if (qf) qf[t] = a;
  if (qc) qc[t] = b;
  if (cyc_out) {
    cyc_out[2 * t] = cyc[fi[t]];
    cyc_out[2 * t + 1] = ci[t] >= 0 ? cyc[ci[t]] : 0;
  }
}

__global__ void k_init_state(int* __restrict__ active, int* __restrict__ cycles, int ns) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  active[t] = 1;
  cycles[t] = 0;
}

inline unsigned blocks_for(long work) { return (unsigned)((work + kBlock - 1) / kBlock); }

}  // namespace


// ---- launchers ------------------------------------------------------------------
void launch_philox(const uint64_t* d_seeds, int count, int level, uint32_t* d_words,
                   double* d_normals, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_philox, dim3(count), dim3(64), 0, st, d_seeds, level, d_words, d_normals);
}

void launch_field(int n, int count, double* const* d_out, const int* d_xi_index,
                  const double* d_normals, const double* d_phi, const double* d_coef, int mode,
                  hipStream_t st) {
  if (count <= 0) return;
  const long N = (long)n * n * n;
  hipLaunchKernelGGL(k_field, dim3(blocks_for(N), count), dim3(kBlock), 0, st, n, d_out,
                     d_xi_index, d_normals, d_phi, d_coef, mode);
}

void launch_inject(int nf, int count, const double* const* d_fine, double* const* d_coarse,
                   hipStream_t st) {
  if (count <= 0) return;
  const long nc = (nf - 1) / 2 + 1;
  hipLaunchKernelGGL(k_inject, dim3(blocks_for(nc * nc * nc), count), dim3(kBlock), 0, st, nf,
                     d_fine, d_coarse);
}

void launch_prepare_problem(int n, const double* k, const double* f, double* wh, double* b,
                            double* u, hipStream_t st) {
  const long N = (long)n * n * n;
  hipLaunchKernelGGL(k_prepare, dim3(blocks_for(N)), dim3(kBlock), 0, st, n, k, f, wh, b, u);
}

void launch_rbgs_colour(const GridDesc* d_list, int count, int n, const int* d_active, int colour,
                        int buf, hipStream_t st) {
  if (count <= 0) return;
  const long m = n - 2, W = (n - 1) / 2;
  hipLaunchKernelGGL(k_rbgs_colour, dim3(blocks_for(m * m * W), count), dim3(kBlock), 0, st,
                     d_list, d_active, colour, buf);
}

void launch_residual(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                     hipStream_t st) {
  if (count <= 0) return;
  const long m = n - 2;
  hipLaunchKernelGGL(k_residual, dim3(blocks_for(m * m * m), count), dim3(kBlock), 0, st, d_list,
                     d_active, buf);
}

void launch_restrict(const GridDesc* d_list, int count, int n, const int* d_active,
                     hipStream_t st) {
  if (count <= 0) return;
  const long mc = (n - 1) / 2 - 1;
  hipLaunchKernelGGL(k_restrict, dim3(blocks_for(mc * mc * mc), count), dim3(kBlock), 0, st,
                     d_list, d_active);
}

void launch_coarsest(const GridDesc* d_list, int count, const int* d_active, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_coarsest, dim3((count + 63) / 64), dim3(64), 0, st, d_list, count,
                     d_active);
}

void launch_prolong(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                    hipStream_t st) {
  if (count <= 0) return;
  const long m = n - 2;
  hipLaunchKernelGGL(k_prolong, dim3(blocks_for(m * m * m), count), dim3(kBlock), 0, st, d_list,
                     d_active, buf);
}

void launch_zero_u(const GridDesc* d_list, int count, int n, hipStream_t st) {
  if (count <= 0) return;
  const long N = (long)n * n * n;
  hipLaunchKernelGGL(k_zero_u, dim3(blocks_for(N), count), dim3(kBlock), 0, st, d_list);
}

void launch_copy_buf(const GridDesc* d_list, int count, int n, const int* d_active, int from,
                     hipStream_t st) {
  if (count <= 0) return;
  const long N = (long)n * n * n;
  hipLaunchKernelGGL(k_copy_buf, dim3(blocks_for(N), count), dim3(kBlock), 0, st, d_list,
                     d_active, from);
}

void launch_reduce(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                   int mode, double* d_partials, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_reduce, dim3(reduce_blocks(n), count), dim3(kBlock), 0, st, d_list,
                     d_active, buf, mode, d_partials);
}

void launch_finalize(const GridDesc* d_list, int count, int n, SolveState s, int mode, int cycle,
                     int fixed_cycles, int max_cycles, double tol, hipStream_t st) {
  (void)n;
  if (count <= 0) return;
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(kBlock), 0, st, d_list, s, mode, cycle,
                     fixed_cycles, max_cycles, tol);
}

void launch_init_state(int* active, int* cycles, int ns, hipStream_t st) {
  hipLaunchKernelGGL(k_init_state, dim3((ns + 255) / 256), dim3(256), 0, st, active, cycles, ns);
}

void launch_count_active(const int* d_active, int nsolves, int* d_count, hipStream_t st) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(kBlock), 0, st, d_active, nsolves, d_count);
}

void launch_ydiff(const double* d_q, const int* d_fi, const int* d_ci, int count, double* d_y,
                  double* d_qf, double* d_qc, const int* d_cycles, int* d_cycles_out,
                  hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ydiff, dim3((count + 255) / 256), dim3(256), 0, st, d_q, d_fi, d_ci, count,
                     d_y, d_qf, d_qc, d_cycles, d_cycles_out);
}

}  // namespace mg
