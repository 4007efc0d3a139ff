// Device kernels of libmlmcmg (gfx950, wave64).
//
// Every multigrid kernel takes a device list of grid descriptors of one grid
// size and runs blockIdx.y over the list, so one launch advances every sample
// of a batch that has a grid of that size.  A per-solve `active` flag freezes
// solves that have converged.  Kernels are templated on the arithmetic type
// (double for the FP64 path, float for the inner cycles of mixed precision).
//
// The smoother (k_sweep) is one red-black Gauss-Seidel sweep in a single
// pass over memory: a workgroup owns a TJ x TK tile of (j,k) columns and
// streams the planes i.  At plane step i it updates the red points of plane i
// on the tile plus a one-point ring (the ring's red values are recomputed, not
// written, because the neighbouring tiles own them), then the black points of
// plane i-1, which need exactly those red values.  Planes of u, wh and the new
// red values live in small LDS ring buffers.  The sweep reads u[buf] and
// writes u[1-buf], so tiles never see a neighbour's half-updated values.
#include "mg_internal.h"

namespace mg {

namespace {

constexpr int kBlock = 256;

// Reciprocals: the hardware estimate refined by Newton-Raphson steps
// y <- y + y (1 - x y) (two for double, one for float).
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ double rcp<double>(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  float y = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, y, 1.0f);
  return __builtin_fmaf(y, e, y);
}

__device__ __forceinline__ int vidx(int n, int i, int j, int k) { return (i * n + j) * n + k; }

// Interior point of block `bid` of a grid with m = n-2 interior points per
// axis: blocks cover (plane i, 4 rows j, 64 columns k).
struct Pt {
  int i, j, k;
  bool ok;
};
__device__ __forceinline__ Pt interior_point(int m, int bid) {
  const int nkc = ceil_div(m, 64), njc = ceil_div(m, 4);
  const int kc = bid % nkc;
  const int t = bid / nkc;
  const int jc = t % njc;
  const int i = t / njc;
  const int k = kc * 64 + (threadIdx.x & 63), j = jc * 4 + (threadIdx.x >> 6);
  return {1 + i, 1 + j, 1 + k, j < m && k < m};
}
// Same over every vertex (boundary included) of an n grid.
__device__ __forceinline__ Pt full_point(int n, int bid) {
  Pt p = interior_point(n, bid);
  return {p.i - 1, p.j - 1, p.k - 1, p.ok};
}

// Harmonic-mean face coefficients of vertex p and the stencil sums
// D = sum_q c_pq, S = sum_q c_pq u_q (neighbours i-1, i+1, j-1, j+1, k-1, k+1).
template <typename T>
__device__ __forceinline__ void stencil(const T* __restrict__ u, const T* __restrict__ wh, int p,
                                        int sj, int si, T& D, T& S) {
  const T w = wh[p];
  const T c0 = rcp<T>(w + wh[p - si]);
  const T c1 = rcp<T>(w + wh[p + si]);
  const T c2 = rcp<T>(w + wh[p - sj]);
  const T c3 = rcp<T>(w + wh[p + sj]);
  const T c4 = rcp<T>(w + wh[p - 1]);
  const T c5 = rcp<T>(w + wh[p + 1]);
  D = ((c0 + c1) + (c2 + c3)) + (c4 + c5);
  S = c0 * u[p - si] + c1 * u[p + si] + c2 * u[p - sj] + c3 * u[p + sj] + c4 * u[p - 1] +
      c5 * u[p + 1];
}

// Deterministic block sum (wave64 shuffles, then the 4 waves in fixed order).
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

// Trilinear interpolation of the coarse array e (size nc, zero on its
// boundary) at fine interior vertex (i, j, k).
template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ e, int nc, int i, int j, int k) {
  const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
  const int ni = (i & 1) + 1, nj = (j & 1) + 1;
  const bool ko = (k & 1) != 0;
  const T wij = (T)(((i & 1) ? 0.5 : 1.0) * ((j & 1) ? 0.5 : 1.0) * (ko ? 0.5 : 1.0));
  T s = 0;
  for (int a = 0; a < ni; ++a)
    for (int b = 0; b < nj; ++b) {
      const int row = vidx(nc, i0 + a, j0 + b, k0);
      T z = e[row];
      if (ko) z += e[row + 1];
      s += z;
    }
  return wij * s;
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
// phi_a(x_i) phi_b(y_j) phi_c(z_k), as nested 1D contractions over a, then b,
// then c.  mode 0 stores wh = exp(-Z)/2, mode 1 stores k = exp(Z).
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
  const Pt p = full_point(n, blockIdx.x);
  if (!p.ok) return;
  double px[4], py[4], pz[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    px[a] = phi[a * n + p.i];
    py[a] = phi[a * n + p.j];
    pz[a] = phi[a * n + p.k];
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
  out[g][vidx(n, p.i, p.j, p.k)] = mode == 0 ? 0.5 * exp(-Z) : exp(Z);
}

__global__ void __launch_bounds__(kBlock) k_inject(int nf, const double* const* __restrict__ fine,
                                                   double* const* __restrict__ coarse) {
  const int nc = (nf - 1) / 2 + 1;
  const Pt p = full_point(nc, blockIdx.x);
  if (!p.ok) return;
  coarse[blockIdx.y][vidx(nc, p.i, p.j, p.k)] =
      fine[blockIdx.y][vidx(nf, 2 * p.i, 2 * p.j, 2 * p.k)];
}

__global__ void __launch_bounds__(kBlock) k_to_float(int n, const double* const* __restrict__ src,
                                                     float* const* __restrict__ dst) {
  const Pt p = full_point(n, blockIdx.x);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  dst[blockIdx.y][v] = (float)src[blockIdx.y][v];
}

__global__ void __launch_bounds__(kBlock) k_prepare(int n, const double* __restrict__ k,
                                                    const double* __restrict__ f,
                                                    double* __restrict__ wh,
                                                    double* __restrict__ b,
                                                    double* __restrict__ u) {
  const Pt p = full_point(n, blockIdx.x);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  const bool bnd = p.i == 0 || p.j == 0 || p.k == 0 || p.i == n - 1 || p.j == n - 1 || p.k == n - 1;
  const double h = 1.0 / (double)(n - 1);
  wh[v] = 0.5 / k[v];
  b[v] = bnd ? 0.0 : h * h * f[v];
  if (bnd) u[v] = 0.0;
}

// ---- the fused red-black smoother --------------------------------------------
template <typename T, int TJ, int TK>
__global__ void __launch_bounds__(kBlock) k_sweep(const GridDescT<T>* __restrict__ list,
                                                  const int* __restrict__ active, int buf,
                                                  int cbuf, int tiles_k, int tiles_jk,
                                                  int chunk_len) {
  constexpr int W2 = TK + 4, H2 = TJ + 4, A2 = W2 * H2;  // tile + 2-point ring
  constexpr int W1 = TK + 2, H1 = TJ + 2, A1 = W1 * H1;  // tile + 1-point ring
  __shared__ T sU[3][A2];  // u[buf] planes (ring of 3)
  __shared__ T sW[5][A2];  // wh planes (ring of 5)
  __shared__ T sR[3][A1];  // new red values (ring of 3)

  const GridDescT<T> d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n, sn2 = n * n;
  const int ch = blockIdx.x / tiles_jk, tile = blockIdx.x - ch * tiles_jk;
  const int tj = tile / tiles_k, tk = tile - tj * tiles_k;
  const int j0 = 1 + tj * TJ, k0 = 1 + tk * TK;
  const int ia = 1 + ch * chunk_len;
  const int ib = min(n - 2, ia + chunk_len - 1);
  const T* __restrict__ uin = (buf ? d.u[1] : d.u[0]);
  T* __restrict__ uout = (buf ? d.u[0] : d.u[1]);
  const T* __restrict__ wh = d.wh;
  const T* __restrict__ bb = d.b;
  const T bconst = (T)d.bconst;
  const T* __restrict__ ec = cbuf < 0 ? nullptr : (cbuf ? d.uc[1] : d.uc[0]);
  const int nc = (n - 1) / 2 + 1;

  auto load_plane = [&](int i) {
    T* du = sU[i % 3];
    T* dw = sW[i % 5];
    for (int q = threadIdx.x; q < A2; q += kBlock) {
      const int r = q / W2, c = q - r * W2;
      const int j = j0 - 2 + r, k = k0 - 2 + c;
      T uv = 0, wv = 0;
      if (j >= 0 && j < n && k >= 0 && k < n) {
        const int g = i * sn2 + j * n + k;
        uv = uin[g];
        wv = wh[g];
        if (ec && i > 0 && i < n - 1 && j > 0 && j < n - 1 && k > 0 && k < n - 1)
          uv += prolong_at<T>(ec, nc, i, j, k);
      }
      du[q] = uv;
      dw[q] = wv;
    }
  };

  // red points of plane i on the tile and its 1-point ring -> sR[i % 3]
  auto red = [&](int i) {
    T* R = sR[i % 3];
    if (i >= n - 1) {
      for (int q = threadIdx.x; q < A1; q += kBlock) R[q] = 0;
      return;
    }
    const T* U0 = sU[(i + 2) % 3];
    const T* U1 = sU[i % 3];
    const T* U2 = sU[(i + 1) % 3];
    const T* Wm = sW[(i + 4) % 5];
    const T* W0 = sW[i % 5];
    const T* Wp = sW[(i + 1) % 5];
    constexpr int HR = W1 / 2;
    for (int q = threadIdx.x; q < H1 * HR; q += kBlock) {
      const int r = q / HR, c2 = q - r * HR;
      const int j = j0 - 1 + r;
      const int c = 2 * c2 + ((i + j + k0 - 1) & 1);  // (i + j + k) even
      const int k = k0 - 1 + c;
      T val = 0;
      if (j >= 1 && j <= n - 2 && k >= 1 && k <= n - 2) {
        const int q2 = (r + 1) * W2 + (c + 1);
        const T w = W0[q2];
        const T a0 = rcp<T>(w + Wm[q2]), a1 = rcp<T>(w + Wp[q2]);
        const T a2 = rcp<T>(w + W0[q2 - W2]), a3 = rcp<T>(w + W0[q2 + W2]);
        const T a4 = rcp<T>(w + W0[q2 - 1]), a5 = rcp<T>(w + W0[q2 + 1]);
        const T D = ((a0 + a1) + (a2 + a3)) + (a4 + a5);
        const T S = a0 * U0[q2] + a1 * U2[q2] + a2 * U1[q2 - W2] + a3 * U1[q2 + W2] +
                    a4 * U1[q2 - 1] + a5 * U1[q2 + 1];
        const T bp = bb ? bb[i * sn2 + j * n + k] : bconst;
        val = (bp + S) * rcp<T>(D);
      }
      R[r * W1 + c] = val;
    }
  };

  // black points of plane p on the tile, then both colours of the tile out
  auto black = [&](int p) {
    const T* Rm = sR[(p + 2) % 3];
    const T* R0 = sR[p % 3];
    const T* Rp = sR[(p + 1) % 3];
    const T* Wm = sW[(p + 4) % 5];
    const T* W0 = sW[p % 5];
    const T* Wp = sW[(p + 1) % 5];
    constexpr int HP = TK / 2;
    for (int q = threadIdx.x; q < TJ * HP; q += kBlock) {
      const int r = q / HP, c2 = q - r * HP;
      const int j = j0 + r;
      if (j > n - 2) continue;
      const int kA = k0 + 2 * c2;  // pair (kA, kA+1): one red, one black
      const bool redA = ((p + j + kA) & 1) == 0;
      const int kb = redA ? kA + 1 : kA;
      const int kr = redA ? kA : kA + 1;
      const T vr = R0[(r + 1) * W1 + (kr - k0 + 1)];
      T vb = 0;
      if (kb <= n - 2) {
        const int q1 = (r + 1) * W1 + (kb - k0 + 1);
        const int q2 = (r + 2) * W2 + (kb - k0 + 2);
        const T w = W0[q2];
        const T a0 = rcp<T>(w + Wm[q2]), a1 = rcp<T>(w + Wp[q2]);
        const T a2 = rcp<T>(w + W0[q2 - W2]), a3 = rcp<T>(w + W0[q2 + W2]);
        const T a4 = rcp<T>(w + W0[q2 - 1]), a5 = rcp<T>(w + W0[q2 + 1]);
        const T D = ((a0 + a1) + (a2 + a3)) + (a4 + a5);
        const T S = a0 * Rm[q1] + a1 * Rp[q1] + a2 * R0[q1 - W1] + a3 * R0[q1 + W1] +
                    a4 * R0[q1 - 1] + a5 * R0[q1 + 1];
        const T bp = bb ? bb[p * sn2 + j * n + kb] : bconst;
        vb = (bp + S) * rcp<T>(D);
      }
      const int g = p * sn2 + j * n + kA;
      uout[g] = redA ? vr : vb;
      if (kA + 1 <= n - 2) uout[g + 1] = redA ? vb : vr;
    }
  };

  const int istart = ia > 1 ? ia - 1 : 1;
  const int iend = min(ib + 1, n - 1);
  load_plane(istart - 1);
  load_plane(istart);
  if (istart == 1)
    for (int q = threadIdx.x; q < A1; q += kBlock) sR[0][q] = 0;  // plane 0 is boundary
  for (int i = istart; i <= iend; ++i) {
    if (i + 1 <= n - 1) load_plane(i + 1);
    __syncthreads();
    red(i);
    __syncthreads();
    if (i - 1 >= ia && i - 1 <= ib) black(i - 1);
  }
}

// ---- point kernels: colour sweep, residual, transfer -------------------------

// In-place Gauss-Seidel update of one colour ((i+j+k) even = red): the
// two-pass alternative to k_sweep.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rbgs_colour(const GridDescT<T>* __restrict__ list,
                                                        const int* __restrict__ active,
                                                        int colour, int buf) {
  const GridDescT<T> d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = interior_point(n - 2, blockIdx.x);
  if (!p.ok || ((p.i + p.j + p.k) & 1) != colour) return;
  const int v = vidx(n, p.i, p.j, p.k);
  T* u = (buf ? d.u[1] : d.u[0]);
  T D, S;
  stencil<T>(u, d.wh, v, n, n * n, D, S);
  const T bp = d.b ? d.b[v] : (T)d.bconst;
  u[v] = (bp + S) * rcp<T>(D);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_residual(const GridDescT<T>* __restrict__ list,
                                                     const int* __restrict__ active, int buf) {
  const GridDescT<T> d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = interior_point(n - 2, blockIdx.x);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  const T* u = (buf ? d.u[1] : d.u[0]);
  T D, S;
  stencil<T>(u, d.wh, v, n, n * n, D, S);
  const T bp = d.b ? d.b[v] : (T)d.bconst;
  d.r[v] = bp - (D * u[v] - S);
}

// Full weighting of the residual to the coarse right-hand side, h^2 scaling
// included: b'_c(I) = 4 * sum_d 2^{-|d|_1}/8 r'(2I+d); also starts the coarse
// cycle from a zero iterate in uc[0].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(const GridDescT<T>* __restrict__ list,
                                                     const int* __restrict__ active) {
  const GridDescT<T> d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n, nc = (n - 1) / 2 + 1;
  const Pt p = interior_point(nc - 2, blockIdx.x);
  if (!p.ok) return;
  const T* r = d.r;
  T s = 0;
  for (int di = -1; di <= 1; ++di) {
    const T wi = di == 0 ? (T)1 : (T)0.5;
    for (int dj = -1; dj <= 1; ++dj) {
      const T wj = dj == 0 ? wi : (T)0.5 * wi;
      const int row = vidx(n, 2 * p.i + di, 2 * p.j + dj, 2 * p.k);
      s += wj * (r[row] + (T)0.5 * (r[row - 1] + r[row + 1]));
    }
  }
  const int pc = vidx(nc, p.i, p.j, p.k);
  d.bc[pc] = (T)0.5 * s;
  d.uc[0][pc] = 0;
}

// 3^3 grid: one unknown, solved exactly into u[0].
template <typename T>
__global__ void k_coarsest(const GridDescT<T>* __restrict__ list, int count,
                           const int* __restrict__ active) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const GridDescT<T> d = list[g];
  if (!active[d.solve]) return;
  const int p = 13;
  const T w = d.wh[p];
  const T D = ((rcp<T>(w + d.wh[p - 9]) + rcp<T>(w + d.wh[p + 9])) +
               (rcp<T>(w + d.wh[p - 3]) + rcp<T>(w + d.wh[p + 3]))) +
              (rcp<T>(w + d.wh[p - 1]) + rcp<T>(w + d.wh[p + 1]));
  const T bp = d.b ? d.b[p] : (T)d.bconst;
  d.u[0][p] = bp * rcp<T>(D);
}

// u[buf] += P uc[cbuf] (trilinear).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong(const GridDescT<T>* __restrict__ list,
                                                    const int* __restrict__ active, int buf,
                                                    int cbuf) {
  const GridDescT<T> d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = interior_point(n - 2, blockIdx.x);
  if (!p.ok) return;
  (buf ? d.u[1] : d.u[0])[vidx(n, p.i, p.j, p.k)] += prolong_at<T>((cbuf ? d.uc[1] : d.uc[0]), (n - 1) / 2 + 1, p.i, p.j, p.k);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_zero_u(const GridDescT<T>* __restrict__ list) {
  const GridDescT<T> d = list[blockIdx.y];
  const int n = d.n;
  const Pt p = full_point(n, blockIdx.x);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  d.u[0][v] = 0;
  if (d.u[1]) d.u[1][v] = 0;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy_buf(const GridDescT<T>* __restrict__ list,
                                                     const int* __restrict__ active, int from) {
  const GridDescT<T> d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = full_point(n, blockIdx.x);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  if (from) d.u[0][v] = d.u[1][v];
  else d.u[1][v] = d.u[0][v];
}

// ---- reductions ---------------------------------------------------------------
// Per-block partial sums over interior vertices of: b'^2 (RED_BNORM),
// (b' - A'u)^2 (RED_RESID) or u (RED_QOI).  The block decomposition depends
// only on the grid size, so a solve's sums never depend on the rest of the batch.
__global__ void __launch_bounds__(kBlock) k_reduce(const GridDesc* __restrict__ list,
                                                   const int* __restrict__ active, int buf,
                                                   int mode, double* __restrict__ partials) {
  const GridDesc d = list[blockIdx.y];
  if (mode == RED_RESID && !active[d.solve]) return;
  const int n = d.n;
  const Pt p = interior_point(n - 2, blockIdx.x);
  double v = 0.0;
  if (p.ok) {
    const int q = vidx(n, p.i, p.j, p.k);
    const double* u = (buf ? d.u[1] : d.u[0]);
    const double bp = d.b ? d.b[q] : d.bconst;
    if (mode == RED_BNORM) {
      v = bp * bp;
    } else if (mode == RED_RESID) {
      double D, S;
      stencil<double>(u, d.wh, q, n, n * n, D, S);
      const double r = bp - (D * u[q] - S);
      v = r * r;
    } else {
      v = u[q];
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[d.poff + blockIdx.x] = v;
}

// Mixed precision outer step: r = b' - A'u (FP64) -> inner rhs (FP32), inner
// iterate zeroed, partial sums of r^2.
__global__ void __launch_bounds__(kBlock) k_defect(const GridDesc* __restrict__ list,
                                                   const GridDesc32* __restrict__ list32,
                                                   const int* __restrict__ active,
                                                   double* __restrict__ partials) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const GridDesc32 e = list32[blockIdx.y];
  const int n = d.n;
  const Pt p = interior_point(n - 2, blockIdx.x);
  double v = 0.0;
  if (p.ok) {
    const int q = vidx(n, p.i, p.j, p.k);
    const double* u = d.u[0];
    const double bp = d.b ? d.b[q] : d.bconst;
    double D, S;
    stencil<double>(u, d.wh, q, n, n * n, D, S);
    const double r = bp - (D * u[q] - S);
    v = r * r;
    e.b[q] = (float)r;
    e.u[0][q] = 0.0f;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partials[d.poff + blockIdx.x] = v;
}

__global__ void __launch_bounds__(kBlock) k_correct(const GridDesc* __restrict__ list,
                                                    const GridDesc32* __restrict__ list32,
                                                    const int* __restrict__ active, int buf32) {
  const GridDesc d = list[blockIdx.y];
  if (!active[d.solve]) return;
  const GridDesc32 e = list32[blockIdx.y];
  const int n = d.n;
  const Pt p = interior_point(n - 2, blockIdx.x);
  if (!p.ok) return;
  const int q = vidx(n, p.i, p.j, p.k);
  d.u[0][q] += (double)(buf32 ? e.u[1] : e.u[0])[q];
}

// Per-solve finalisation of the reductions.  For RED_RESID the cycle being
// judged is *cycle_ctr - lag (lag 1 when the residual belongs to the iterate
// of the previous outer step).
__global__ void __launch_bounds__(kBlock) k_finalize(const GridDesc* __restrict__ list,
                                                     SolveState s, int mode,
                                                     const int* __restrict__ cycle_ctr, int lag,
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
    const int cycle = *cycle_ctr - lag;
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

__global__ void k_init_state(int* __restrict__ active, int* __restrict__ cycles,
                             int* __restrict__ cycle_ctr, int ns) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *cycle_ctr = 0;
  if (t >= ns) return;
  active[t] = 1;
  cycles[t] = 0;
}

__global__ void k_tick(int* __restrict__ ctr) {
  if (threadIdx.x == 0) *ctr += 1;
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

inline dim3 interior_grid(int n, int count) { return dim3(point_blocks(n - 2), count); }
inline dim3 full_grid(int n, int count) { return dim3(point_blocks(n), count); }

template <typename T, int TJ, int TK>
void sweep_launch(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                  int cbuf, int chunks, hipStream_t st) {
  const int tiles_k = (n - 1) / TK, tiles_j = (n - 1) / TJ;
  const int tiles = tiles_k * tiles_j;
  const int chunk_len = ceil_div(n - 2, chunks);
  const int nch = ceil_div(n - 2, chunk_len);
  hipLaunchKernelGGL((k_sweep<T, TJ, TK>), dim3(tiles * nch, count), dim3(kBlock), 0, st, d_list,
                     d_active, buf, cbuf, tiles_k, tiles, chunk_len);
}

}  // namespace

// ---- tile shapes ------------------------------------------------------------
static const SweepShape kShapes[] = {
    {4, 64, 1}, {16, 32, 1}, {8, 32, 1}, {4, 32, 1}, {16, 16, 1}, {8, 16, 1},
    {4, 16, 1}, {8, 8, 1},   {4, 8, 1},  {4, 4, 1},  {2, 2, 1},
};

int sweep_shapes(int n, SweepShape* out, int max_out) {
  int c = 0;
  for (const SweepShape& s : kShapes)
    if (s.tj <= n - 1 && s.tk <= n - 1 && (n - 1) % s.tj == 0 && (n - 1) % s.tk == 0 && c < max_out)
      out[c++] = s;
  return c;
}

SweepShape default_sweep_shape(int n) {
  if (n - 1 >= 64) return {4, 64, 1};
  if (n - 1 >= 32) return {8, 32, 1};
  if (n - 1 >= 16) return {8, 16, 1};
  if (n - 1 >= 8) return {8, 8, 1};
  if (n - 1 >= 4) return {4, 4, 1};
  return {2, 2, 1};
}

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
  hipLaunchKernelGGL(k_field, full_grid(n, count), dim3(kBlock), 0, st, n, d_out, d_xi_index,
                     d_normals, d_phi, d_coef, mode);
}

void launch_inject(int nf, int count, const double* const* d_fine, double* const* d_coarse,
                   hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_inject, full_grid((nf - 1) / 2 + 1, count), dim3(kBlock), 0, st, nf,
                     d_fine, d_coarse);
}

void launch_to_float(int n, int count, const double* const* d_src, float* const* d_dst,
                     hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_to_float, full_grid(n, count), dim3(kBlock), 0, st, n, d_src, d_dst);
}

void launch_prepare_problem(int n, const double* k, const double* f, double* wh, double* b,
                            double* u, hipStream_t st) {
  hipLaunchKernelGGL(k_prepare, full_grid(n, 1), dim3(kBlock), 0, st, n, k, f, wh, b, u);
}

template <typename T>
void launch_sweep(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                  int cbuf, SweepShape s, hipStream_t st) {
  if (count <= 0) return;
  const int c = s.chunks < 1 ? 1 : s.chunks;
#define MG_SWEEP_CASE(TJ_, TK_)                                                     \
  if (s.tj == TJ_ && s.tk == TK_) {                                                 \
    sweep_launch<T, TJ_, TK_>(d_list, count, n, d_active, buf, cbuf, c, st);        \
    return;                                                                         \
  }
  MG_SWEEP_CASE(4, 64)
  MG_SWEEP_CASE(16, 32)
  MG_SWEEP_CASE(8, 32)
  MG_SWEEP_CASE(4, 32)
  MG_SWEEP_CASE(16, 16)
  MG_SWEEP_CASE(8, 16)
  MG_SWEEP_CASE(4, 16)
  MG_SWEEP_CASE(8, 8)
  MG_SWEEP_CASE(4, 8)
  MG_SWEEP_CASE(4, 4)
  MG_SWEEP_CASE(2, 2)
#undef MG_SWEEP_CASE
}

template <typename T>
void launch_rbgs_colour(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                        int colour, int buf, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_rbgs_colour<T>), interior_grid(n, count), dim3(kBlock), 0, st, d_list,
                     d_active, colour, buf);
}

template <typename T>
void launch_residual(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                     hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_residual<T>), interior_grid(n, count), dim3(kBlock), 0, st, d_list,
                     d_active, buf);
}

template <typename T>
void launch_restrict(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                     hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_restrict<T>), interior_grid((n - 1) / 2 + 1, count), dim3(kBlock), 0, st,
                     d_list, d_active);
}

template <typename T>
void launch_coarsest(const GridDescT<T>* d_list, int count, const int* d_active, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_coarsest<T>), dim3((count + 63) / 64), dim3(64), 0, st, d_list, count,
                     d_active);
}

template <typename T>
void launch_prolong(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                    int cbuf, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_prolong<T>), interior_grid(n, count), dim3(kBlock), 0, st, d_list,
                     d_active, buf, cbuf);
}

template <typename T>
void launch_zero_u(const GridDescT<T>* d_list, int count, int n, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_zero_u<T>), full_grid(n, count), dim3(kBlock), 0, st, d_list);
}

template <typename T>
void launch_copy_buf(const GridDescT<T>* d_list, int count, int n, const int* d_active, int from,
                     hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_copy_buf<T>), full_grid(n, count), dim3(kBlock), 0, st, d_list, d_active,
                     from);
}

#define MG_INSTANTIATE(T)                                                                       \
  template void launch_sweep<T>(const GridDescT<T>*, int, int, const int*, int, int, SweepShape, \
                                hipStream_t);                                                   \
  template void launch_rbgs_colour<T>(const GridDescT<T>*, int, int, const int*, int, int,      \
                                      hipStream_t);                                             \
  template void launch_residual<T>(const GridDescT<T>*, int, int, const int*, int, hipStream_t); \
  template void launch_restrict<T>(const GridDescT<T>*, int, int, const int*, hipStream_t);      \
  template void launch_coarsest<T>(const GridDescT<T>*, int, const int*, hipStream_t);           \
  template void launch_prolong<T>(const GridDescT<T>*, int, int, const int*, int, int,           \
                                  hipStream_t);                                                 \
  template void launch_zero_u<T>(const GridDescT<T>*, int, int, hipStream_t);                    \
  template void launch_copy_buf<T>(const GridDescT<T>*, int, int, const int*, int, hipStream_t);
MG_INSTANTIATE(double)
MG_INSTANTIATE(float)
#undef MG_INSTANTIATE

void launch_reduce(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                   int mode, double* d_partials, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_reduce, interior_grid(n, count), dim3(kBlock), 0, st, d_list, d_active,
                     buf, mode, d_partials);
}

void launch_defect(const GridDesc* d_list, const GridDesc32* d_list32, int count, int n,
                   const int* d_active, double* d_partials, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_defect, interior_grid(n, count), dim3(kBlock), 0, st, d_list, d_list32,
                     d_active, d_partials);
}

void launch_correct(const GridDesc* d_list, const GridDesc32* d_list32, int count, int n,
                    const int* d_active, int buf32, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_correct, interior_grid(n, count), dim3(kBlock), 0, st, d_list, d_list32,
                     d_active, buf32);
}

void launch_finalize2(const GridDesc* d_list, int count, SolveState s, int mode,
                      const int* cycle_ctr, int lag, int fixed_cycles, int max_cycles, double tol,
                      hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(kBlock), 0, st, d_list, s, mode, cycle_ctr, lag,
                     fixed_cycles, max_cycles, tol);
}

void launch_init_state2(int* active, int* cycles, int* cycle_ctr, int ns, hipStream_t st) {
  hipLaunchKernelGGL(k_init_state, dim3((ns + 255) / 256), dim3(256), 0, st, active, cycles,
                     cycle_ctr, ns);
}

void launch_tick(int* ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, ctr);
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
