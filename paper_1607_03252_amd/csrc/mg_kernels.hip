// Device kernels of libmlmcmg (gfx950, wave64).
//
// Every multigrid kernel takes a device list of grid descriptors of one grid
// size and spreads (grid, block) units over its workgroups (xcd_unit), so one
// launch advances every sample of a batch that has a grid of that size.  A per-solve `active` flag freezes
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
#include <algorithm>
#include <type_traits>

#include "mg_internal.h"

namespace mg {

namespace {

constexpr int kBlock = 256;

// Reciprocals: the hardware estimate y refined.  The FP64 estimate is good
// to about 2^-25, so with e = 1 - x y the third-order step
// y (1 + e + e^2) = 1/x (1 - e^3) leaves a truncation of 2^-75 and the result
// is within half a unit in the last place bar rounding (three FMAs: the same
// accuracy as two Newton-Raphson steps, one FMA fewer on a path whose
// sweeps are bound by FP64 issue).  FP32 (the inner cycles of mixed
// precision, whose corrections the FP64 defect of the next outer step
// checks): the hardware estimate as it is, within about one unit in the
// last place.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ double rcp<double>(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, __builtin_fma(e, e, e), y);
}
template <>
__device__ __forceinline__ float rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

__device__ __forceinline__ int vidx(int n, int i, int j, int k) { return (i * n + j) * n + k; }

// Grid buffers reach the kernels as generic pointers inside descriptors, so
// plain dereferences compile to flat memory instructions, which count
// against both vmcnt and lgkmcnt: every wait for LDS data would also drain
// the in-flight global loads and stores.  These views put them in the global
// address space so the compiler emits global_* instructions instead.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gview(T* p) {
  return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<const T> gview(const T* p) {
  return (gptr<const T>)p;
}

// Raw buffer access: a descriptor (uniform base, range in bytes) and 32-bit
// per-lane byte offsets.  Loads past the range read 0 and stores past it are
// dropped, which lets a kernel express "outside the grid" by an offset.
constexpr uint32_t kOut = 0x7ffffff0u;  // an offset past any range used here
// s_waitcnt immediate (gfx9 encoding) that waits for every vector memory
// operation and for nothing else: vmcnt 0, expcnt 7, lgkmcnt 15.
constexpr int kWaitVmem0 = 0x0F70;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, T v);
template <>
__device__ __forceinline__ void bstore<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  typedef unsigned int v2u __attribute__((__vector_size__(8)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, off, 0, 0);
}
template <>
__device__ __forceinline__ void bstore<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}

// Two consecutive elements in one load (16 bytes for double): offsets need
// only the alignment of one element (8 bytes, a multiple of the dword).
template <typename T>
struct Two {
  T lo, hi;
};
template <typename T>
__device__ __forceinline__ Two<T> bload2(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ Two<double> bload2<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(Two<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <>
__device__ __forceinline__ Two<float> bload2<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(Two<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

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

// Workgroup -> (grid g, block blk of that grid).  Workgroups are dealt to
// the 8 XCDs round-robin; this gives each XCD one contiguous range of the
// count * per units, so the neighbouring tiles of a grid (whose halos
// overlap) run under the same L2.
__device__ __forceinline__ bool xcd_unit(int count, int per, int& g, int& blk) {
  const int total = count * per;
  const int Q = (total + 7) >> 3;
  const int L = blockIdx.x;
  const int u = (L & 7) * Q + (L >> 3);
  g = u / per;
  blk = u - g * per;
  return u < total;
}

// Right-hand side at vertex (i, j, k): a full array or a constant plane.
template <typename T>
__device__ __forceinline__ T b_at(const GridDescT<T>& d, int i, int j, int k) {
  return gview<T>(d.b)[i * d.bstride + j * d.n + k];
}

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c);
template <>
__device__ __forceinline__ double fmaT<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// The 7-point stencil at one vertex: w = 1/(2k) there, w0..w5 and u0..u5 the
// neighbours' values in the order i-1, i+1, j-1, j+1, k-1, k+1.  Face
// coefficients c_q = 1/(w + w_q) (the harmonic mean 2 k k_q/(k + k_q)),
// D = sum_q c_q and S = sum_q c_q u_q.  Every kernel evaluates the operator
// through this one function (explicit FMAs, the rest rounded as written; the
// library is compiled without contraction), so every code path that applies
// the same update to the same data gets the same bits.
template <typename T>
struct St {
  T D, S;
};
// D and S from the six face coefficients a0..a5 (same order).
template <typename T>
__device__ __forceinline__ St<T> stencil_faces(T a0, T a1, T a2, T a3, T a4, T a5, T u0, T u1,
                                               T u2, T u3, T u4, T u5) {
  St<T> s;
  s.D = ((a0 + a1) + (a2 + a3)) + (a4 + a5);
  T S = a0 * u0;
  S = fmaT<T>(a1, u1, S);
  S = fmaT<T>(a2, u2, S);
  S = fmaT<T>(a3, u3, S);
  S = fmaT<T>(a4, u4, S);
  s.S = fmaT<T>(a5, u5, S);
  return s;
}
template <typename T>
__device__ __forceinline__ St<T> stencil6(T w, T w0, T w1, T w2, T w3, T w4, T w5, T u0, T u1,
                                          T u2, T u3, T u4, T u5) {
  return stencil_faces<T>(rcp<T>(w + w0), rcp<T>(w + w1), rcp<T>(w + w2), rcp<T>(w + w3),
                          rcp<T>(w + w4), rcp<T>(w + w5), u0, u1, u2, u3, u4, u5);
}
// Gauss-Seidel value (b' + S)/D and residual b' - (D u - S).
template <typename T>
__device__ __forceinline__ T gs_value(St<T> s, T b) {
  return (b + s.S) * rcp<T>(s.D);
}
template <typename T>
__device__ __forceinline__ T res_value(St<T> s, T b, T u) {
  return b - fmaT<T>(s.D, u, -s.S);
}
// The stencil at vertex p of arrays with plane stride si and row stride sj.
template <typename T, typename PU, typename PW>
__device__ __forceinline__ St<T> stencil_at(PU u, PW wh, int p, int sj, int si) {
  return stencil6<T>(wh[p], wh[p - si], wh[p + si], wh[p - sj], wh[p + sj], wh[p - 1], wh[p + 1],
                     u[p - si], u[p + si], u[p - sj], u[p + sj], u[p - 1], u[p + 1]);
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
// boundary) at fine interior vertex (i, j, k): the 8 surrounding coarse values
// with per-axis weights (1, 0) on even and (1/2, 1/2) on odd fine indices.
// Branch-free, and the one formula both the fused sweep and k_prolong use.
template <typename T, typename P>
__device__ __forceinline__ void prolong_load(P e, int nc, int i, int j, int k, T (&v)[8]) {
  const int base = ((i >> 1) * nc + (j >> 1)) * nc + (k >> 1), pl = nc * nc;
  v[0] = e[base];
  v[1] = e[base + 1];
  v[2] = e[base + nc];
  v[3] = e[base + nc + 1];
  v[4] = e[base + pl];
  v[5] = e[base + pl + 1];
  v[6] = e[base + pl + nc];
  v[7] = e[base + pl + nc + 1];
}
template <typename T>
__device__ __forceinline__ T prolong_combine(int i, int j, int k, const T (&v)[8]) {
  const T wi1 = (i & 1) ? (T)0.5 : (T)0, wi0 = (i & 1) ? (T)0.5 : (T)1;
  const T wj1 = (j & 1) ? (T)0.5 : (T)0, wj0 = (j & 1) ? (T)0.5 : (T)1;
  const T wk1 = (k & 1) ? (T)0.5 : (T)0, wk0 = (k & 1) ? (T)0.5 : (T)1;
  return wi0 * (wj0 * (wk0 * v[0] + wk1 * v[1]) + wj1 * (wk0 * v[2] + wk1 * v[3])) +
         wi1 * (wj0 * (wk0 * v[4] + wk1 * v[5]) + wj1 * (wk0 * v[6] + wk1 * v[7]));
}
template <typename T, typename P>
__device__ __forceinline__ T prolong_at(P e, int nc, int i, int j, int k) {
  T v[8];
  prolong_load<T>(e, nc, i, j, k, v);
  return prolong_combine<T>(i, j, k, v);
}

// ---- Philox4x32-10: philox_block (mg_internal.h) ----------------------------

// One 64-thread block per sample: 32 Philox blocks -> 128 words -> 64
// uniforms on (0,1] with 53 random bits -> 32 Box-Muller pairs.
__global__ void __launch_bounds__(64) k_philox(const uint64_t* __restrict__ seeds, int level,
                                               const int* __restrict__ levels,
                                               uint32_t* __restrict__ words,
                                               double* __restrict__ normals) {
  __shared__ uint32_t w[128];
  __shared__ double U[64];
  const int s = blockIdx.x, t = threadIdx.x;
  const uint64_t seed = seeds[s];
  if (levels) level = levels[s];
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

// The KL field at a vertex, in one fixed order of operations shared by every
// kernel that forms it, so that the stored coefficient and one recomputed
// inside a smoother are the same bits:
//   P[4a + c] = sum_b C[16a + 4b + c] phi_b(y)    (b ascending)
//   H[a]      = sum_c P[4a + c] phi_c(z)          (c ascending)
//   Z         = sum_a phi_a(x) H[a]               (a ascending)
// with C[abc] = coef[abc] * xi[abc]; wh = exp(-Z)/2 and k = exp(Z).
__device__ __forceinline__ void kl_rows(const double* C, const double (&py)[4], double (&P)[16]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double v = C[16 * a + c] * py[0];
      v = __builtin_fma(C[16 * a + 4 + c], py[1], v);
      v = __builtin_fma(C[16 * a + 8 + c], py[2], v);
      P[4 * a + c] = __builtin_fma(C[16 * a + 12 + c], py[3], v);
    }
}
__device__ __forceinline__ void kl_cols(const double (&P)[16], const double (&pz)[4],
                                        double (&H)[4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double v = P[4 * a] * pz[0];
    v = __builtin_fma(P[4 * a + 1], pz[1], v);
    v = __builtin_fma(P[4 * a + 2], pz[2], v);
    H[a] = __builtin_fma(P[4 * a + 3], pz[3], v);
  }
}
// px: phi_0..3 at the plane's coordinate
__device__ __forceinline__ double kl_z(const double (&H)[4], const double* px) {
  double z = H[0] * px[0];
  z = __builtin_fma(H[1], px[1], z);
  z = __builtin_fma(H[2], px[2], z);
  return __builtin_fma(H[3], px[3], z);
}

// exp by the table-driven method of P. T. P. Tang (ACM TOMS 15(2), 1989):
// x = (32 m + j) ln2/32 + r with |r| <= ln2/64, exp(x) = 2^m 2^(j/32) exp(r),
// exp(r) - 1 from its degree-6 Taylor polynomial (truncation below 4e-18),
// ln2/32 split so that (32 m + j) times the leading part is exact.  tab[j] is
// 2^(j/32) rounded to double (kExp2Tab, staged in LDS by the kernels).
// Relative error below 2 units in the last place for |x| <= 700 (x is
// clamped to that range).  Every kernel that forms the KL coefficient uses
// this function, so the stored and the recomputed coefficient are the same bits.
__host__ __device__ __forceinline__ double kl_exp(double x, const double* tab) {
  constexpr double kInvL = 0x1.71547652b82fep+5;  // 32 / ln2
  constexpr double kLhi = 0x1.62e42fefa0000p-6;   // ln2/32, leading 37 bits
  constexpr double kLlo = 0x1.cf79abc9e3b3ap-45;  // ln2/32 - kLhi
  x = fmin(fmax(x, -700.0), 700.0);
  const double kf = rint(x * kInvL);
  const int kq = (int)kf;
  const int j = kq & 31, m = kq >> 5;  // kq = 32 m + j (arithmetic shift)
  double r = __builtin_fma(-kf, kLhi, x);
  r = __builtin_fma(-kf, kLlo, r);
  double p = __builtin_fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = __builtin_fma(r, p, 1.0 / 24.0);
  p = __builtin_fma(r, p, 1.0 / 6.0);
  p = __builtin_fma(r, p, 0.5);
  p = __builtin_fma(r * r, p, r);  // exp(r) - 1
  const double tj = tab[j];
  return ldexp(__builtin_fma(tj, p, tj), m);
}
#define MG_EXP2_TAB { \
    0x1.0000000000000p+0, 0x1.059b0d3158574p+0, 0x1.0b5586cf9890fp+0, 0x1.11301d0125b51p+0, \
    0x1.172b83c7d517bp+0, 0x1.1d4873168b9aap+0, 0x1.2387a6e756238p+0, 0x1.29e9df51fdee1p+0, \
    0x1.306fe0a31b715p+0, 0x1.371a7373aa9cbp+0, 0x1.3dea64c123422p+0, 0x1.44e086061892dp+0, \
    0x1.4bfdad5362a27p+0, 0x1.5342b569d4f82p+0, 0x1.5ab07dd485429p+0, 0x1.6247eb03a5585p+0, \
    0x1.6a09e667f3bcdp+0, 0x1.71f75e8ec5f74p+0, 0x1.7a11473eb0187p+0, 0x1.82589994cce13p+0, \
    0x1.8ace5422aa0dbp+0, 0x1.93737b0cdc5e5p+0, 0x1.9c49182a3f090p+0, 0x1.a5503b23e255dp+0, \
    0x1.ae89f995ad3adp+0, 0x1.b7f76f2fb5e47p+0, 0x1.c199bdd85529cp+0, 0x1.cb720dcef9069p+0, \
    0x1.d5818dcfba487p+0, 0x1.dfc97337b9b5fp+0, 0x1.ea4afa2a490dap+0, 0x1.f50765b6e4540p+0}
__device__ const double kExp2Tab[32] = MG_EXP2_TAB;
static const double kExp2TabHost[32] = MG_EXP2_TAB;
#undef MG_EXP2_TAB
// LDS layout of the KL data of a launch (doubles): the mode table
// [0, 4n) as tab[4m + a] = phi_a(x_m), the weights [4n, 4n + 64), the exp
// table [4n + 64, 4n + 96).
__host__ __device__ constexpr int kl_lds_doubles(int n) { return 4 * n + 96; }
__device__ __forceinline__ double kl_wh(double z, const double* etab) {
  return 0.5 * kl_exp(-z, etab);
}

// Field on `count` grids of size n (mode 0: wh = exp(-Z)/2, mode 1:
// k = exp(Z)).  A thread owns one column (j, k) of a grid: it forms the
// column parts H once and marches the planes i, its stores coalesced with
// the neighbouring columns'.
constexpr int kFieldMaxN = 1025;
__global__ void __launch_bounds__(kBlock) k_field(int n, double* const* __restrict__ out,
                                                  const int* __restrict__ xi_index,
                                                  const double* __restrict__ normals,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ coef, int mode,
                                                  int count, int per) {
  __shared__ double C[64], E[32];
  int g, blk;
  if (!xcd_unit(count, per, g, blk)) return;
  const int t = threadIdx.x;
  if (t < 64) C[t] = coef[t] * normals[(size_t)xi_index[g] * 64 + t];
  if (t < 32) E[t] = kExp2Tab[t];
  __syncthreads();
  const int q = blk * kBlock + t;
  if (q >= n * n) return;
  const int j = q / n, k = q - (q / n) * n;
  double py[4], pz[4], P[16], H[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    py[a] = phi[a * n + j];
    pz[a] = phi[a * n + k];
  }
  kl_rows(C, py, P);
  kl_cols(P, pz, H);
  double* o = out[g] + q;
  const size_t np = (size_t)n * n;
  for (int i = 0; i < n; ++i) {
    const double px[4] = {phi[i], phi[n + i], phi[2 * n + i], phi[3 * n + i]};
    const double z = kl_z(H, px);
    o[(size_t)i * np] = mode == 0 ? kl_wh(z, E) : kl_exp(z, E);
  }
}

__global__ void __launch_bounds__(kBlock) k_inject(int nf, const double* const* __restrict__ fine,
                                                   double* const* __restrict__ coarse, int count,
                                                   int per) {
  const int nc = (nf - 1) / 2 + 1;
  int g, blk;
  if (!xcd_unit(count, per, g, blk)) return;
  const Pt p = full_point(nc, blk);
  if (!p.ok) return;
  coarse[g][vidx(nc, p.i, p.j, p.k)] = fine[g][vidx(nf, 2 * p.i, 2 * p.j, 2 * p.k)];
}

__global__ void __launch_bounds__(kBlock) k_to_float(int n, const double* const* __restrict__ src,
                                                     float* const* __restrict__ dst, int count,
                                                     int per) {
  int g, blk;
  if (!xcd_unit(count, per, g, blk)) return;
  const Pt p = full_point(n, blk);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  dst[g][v] = (float)src[g][v];
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
// One pass computes a whole red-black sweep u_in -> u_out.  A workgroup owns
// a TJ x TK column tile and marches the planes i; on plane i it updates the
// red points of the tile plus a one-point ring (from u_in), and the black
// points of plane i-1 (from the new red values of planes i-2, i-1, i).
//
// Each thread owns a pair of k-adjacent columns of the tile plus a two-point
// ring (T2 = (TJ+4) x (TK+4) positions).  The pair is indexed by role, not
// position: role 0 is the column that is red on planes istart, istart+2, ...
// so on every plane all threads agree which role is red.  Every face of the
// grid joins one red and one black point: the red update computes its six
// face coefficients, and the black update reuses them (the two vertical
// ones from the same thread's registers, the four in-plane ones through LDS),
// so a black point needs no reciprocal but 1/D.  A red update reads no old
// value of its own and a black update reads no old values at all, so only
// the black position of each pair is needed from u_in (the input-residual
// sweep also needs the red one).
//
// Registers hold, per plane, in rings of four indexed by plane offset from
// istart (the march is unrolled by four, so no value moves): the black
// u_in, wh and b of both positions of the pair (one 16-byte load each where
// the register budget allows, else one load per role), the new red value and
// the red point's +i face.
// The loads of plane i+3 are issued at the end of plane i.  LDS holds, per
// plane parity: u_in and wh of black positions (for red neighbours), the new
// red values and the +j / +k faces (for black points), so each plane needs a
// single barrier.  Position q of the tile is stored at LDS index
// (q & 1) * PAIRS + (q >> 1): even and odd positions of a row lie apart, so the
// lanes of a row touch consecutive words although each owns two positions
// (indexing by q directly makes every access a two-way bank conflict).
template <int TJ, int TK>
struct SweepGeom {
  static constexpr int W2 = TK + 4, H2 = TJ + 4, A2 = W2 * H2;
  static constexpr int PAIRS = H2 * (W2 / 2);
  static constexpr int THREADS = ((PAIRS + 63) / 64) * 64;
  // LDS index of tile position q (A2 is even: W2 is)
  static __device__ __forceinline__ int lidx(int q) { return (q & 1) * PAIRS + (q >> 1); }
  static constexpr int DJ = W2 / 2;  // LDS index step of one row
};

// NM: the sweep also sums squared residuals over its tile, for grids with
// spoff >= 0, one partial per workgroup into spart[spoff + workgroup]:
//   NM = 1: the red points of its input iterate: the red update forms their
//           D and S from the input values already; their own input values
//           come with the black ones (one load of both positions of a pair);
//   NM = 2: the black points of its output iterate: a black update's D and S
//           are those of the residual of the new black value.
// Red points depend only on black values and vice versa, so the residual of
// an iterate is the NM = 2 sums of the sweep that produced it plus the NM = 1
// sums of the next sweep, both evaluated exactly as the residual kernels do.
// CB: every grid of the launch has a constant right-hand side (bstride 0):
// its two values per thread are loaded once instead of per plane.
// KL (FP64): the coefficient wh is evaluated from the grid's KL data instead
// of read (kl_rows/kl_cols once per column, kl_z and exp per plane, the 1D
// mode table staged in dynamic LDS), in the operations of the field kernel,
// so the sweep's results are the same bits; the sweep then reads only u.
//
// Work: the launch has nwg workgroups (a multiple of 8) for the list's count
// grids.  Every wave counts the active grids of the list by ballots; with
// nact of them active, each active grid's tiles are split into C pieces of
// its plane march (chunks > 0: C = chunks; else as many as the workgroups
// allow, at least four planes per piece), so a launch in which most solves
// have stopped still spreads its work over the machine.  Workgroups are
// numbered XCD-contiguously (neighbouring tiles share an L2).
template <typename T, int TJ, int TK, bool PRO, int NM, bool CB, bool KL>
__device__ __forceinline__ void sweep_tile(const GridDescT<T>* __restrict__ list,
                                           const int* __restrict__ active, int buf, int cbuf,
                                           int tiles_k, int tiles_jk, int chunks, int count,
                                           int nwg, T* __restrict__ spart) {
  using Geo = SweepGeom<TJ, TK>;
  constexpr int W2 = Geo::W2, A2 = Geo::A2, HW = W2 / 2;
  __shared__ T sU[2][A2];   // u_in of black positions, plane parity
  __shared__ T sW[2][A2];   // wh of black positions
  __shared__ T sR[2][A2];   // new red values
  __shared__ T sFj[2][A2];  // face between x and x + W2 (x red or black)
  __shared__ T sFk[2][A2];  // face between x and x + 1

  const int nl = list[0].n;
  const int wl = threadIdx.x & 63;
  // active masks of the first 128 grids kept for the search below
  const bool on0 = wl < count && active[list[wl].solve];
  const bool on1 = 64 + wl < count && active[list[64 + wl].solve];
  const unsigned long long m0 = __ballot(on0), m1 = __ballot(on1);
  int nact = __popcll(m0) + __popcll(m1);
  for (int b = 128; b < count; b += 64) {
    const bool on = b + wl < count && active[list[b + wl].solve];
    nact += __popcll(__ballot(on));
  }
  if (nact == 0) return;
  // (at most kSweepParts workgroups per grid: the residual sums keep one
  // partial per workgroup)
  const int C = chunks > 0 ? chunks
                           : max(1, min(min(nwg / (nact * tiles_jk), (nl - 2) / 4),
                                        kSweepParts / tiles_jk));
  const int chunk_len = ceil_div(nl - 2, C);
  const int per = tiles_jk * ceil_div(nl - 2, chunk_len);  // workgroups per active grid
  const int w = (int)(blockIdx.x & 7) * (nwg >> 3) + (int)(blockIdx.x >> 3);
  if (w >= nact * per) return;
  int a = w / per;
  const int blk = w - a * per;
  int gi = 0;
  // the a-th active grid: its bit among the masks
  auto nth = [&](unsigned long long m, int r) {
    const bool hit = ((m >> wl) & 1ull) && __popcll(m & ((1ull << wl) - 1ull)) == r;
    return __ffsll(__ballot(hit)) - 1;
  };
  if (a < __popcll(m0)) {
    gi = nth(m0, a);
  } else if ((a -= __popcll(m0)) < __popcll(m1)) {
    gi = 64 + nth(m1, a);
  } else {
    a -= __popcll(m1);
    for (int b = 128; b < count; b += 64) {
      const bool on = b + wl < count && active[list[b + wl].solve];
      const unsigned long long m = __ballot(on);
      if (a < __popcll(m)) {
        gi = b + nth(m, a);
        break;
      }
      a -= __popcll(m);
    }
  }
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n, sn2 = n * n, bs = d.bstride;
  const int ch = blk / tiles_jk, tile = blk - ch * tiles_jk;
  const int tj = tile / tiles_k, tk = tile - tj * tiles_k;
  const int j0 = 1 + tj * TJ, k0 = 1 + tk * TK;
  const int ia = 1 + ch * chunk_len;
  const int ib = min(n - 2, ia + chunk_len - 1);
  const int istart = ia > 1 ? ia - 1 : 1;
  const int iend = min(ib + 1, n - 1);
  const gptr<const T> ec = gview<T>(PRO ? (cbuf ? d.uc[1] : d.uc[0]) : d.u[0]);
  const int nc = (n - 1) / 2 + 1;

  // this thread's pair: T2 row r, positions 2*c2 and 2*c2 + 1
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const bool live = t < Geo::PAIRS;
  const int r = live ? t / HW : 0, c2 = live ? t - (t / HW) * HW : 0;
  const int j = j0 - 2 + r;
  const int kA = k0 - 2 + 2 * c2;
  const int sw = (istart + j + kA) & 1;  // role rho sits at position 2*c2 + (rho ^ sw)
  int kc[2], qr[2], col[2];
  bool in[2], intr[2], t1[2], tl[2];
  const bool intJ = j >= 1 && j <= n - 2;
#pragma unroll
  for (int rho = 0; rho < 2; ++rho) {
    const int x = 2 * c2 + (rho ^ sw);  // position in the T2 row
    kc[rho] = kA + (rho ^ sw);
    qr[rho] = r * W2 + x;
    col[rho] = min(max(kc[rho], 0), n - 1);
    in[rho] = live && j >= 0 && j < n && kc[rho] >= 0 && kc[rho] < n;
    intr[rho] = intJ && kc[rho] >= 1 && kc[rho] <= n - 2;
    t1[rho] = live && r >= 1 && r <= TJ + 2 && x >= 1 && x <= TK + 2;
    tl[rho] = live && r >= 2 && r < TJ + 2 && x >= 2 && x < TK + 2 && intr[rho];
  }
  const int jc = min(max(j, 0), n - 1);
  const int jI = min(max(j, 1), n - 2);
  // KL: the mode table (sPhi[4m + a] = phi_a at plane m) and the weights in
  // LDS, then the column parts of this thread's two positions (a position
  // outside the grid gets wh = 0, as a read past a buffer's range does)
  static_assert(!KL || std::is_same<T, double>::value, "the KL sweep is FP64");
  extern __shared__ double kl_lds[];
  double KH[KL ? 2 : 1][4];
  bool kin[2] = {false, false};
  const double* etab = kl_lds + 4 * n + 64;
  if constexpr (KL) {
    double* sC = kl_lds + 4 * n;
    for (int q = t; q < 4 * n; q += Geo::THREADS) kl_lds[q] = d.klphi[(q & 3) * n + (q >> 2)];
    if (t < 64) sC[t] = d.klcoef[t] * d.kln[t];
    if (t < 32) sC[64 + t] = kExp2Tab[t];
    __syncthreads();
    double py[4], P[16];
#pragma unroll
    for (int b = 0; b < 4; ++b) py[b] = kl_lds[4 * jc + b];
    kl_rows(sC, py, P);
#pragma unroll
    for (int pos = 0; pos < 2; ++pos) {
      const int kk = min(max(kA + pos, 0), n - 1);
      double pz[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) pz[c] = kl_lds[4 * kk + c];
      kl_cols(P, pz, KH[pos]);
      kin[pos] = live && j >= 0 && j < n && kA + pos >= 0 && kA + pos < n;
    }
  }
  // LDS indexes, per role: own position (lq), and for the stencil reads of a
  // ring-1 position (the others read around a safe interior position whose
  // results are not used) the position itself (lc; its j-neighbours are
  // lc -+ one row) and its k-neighbours (lm and lm + 1: q - 1 and q + 1 have the
  // same parity and q >> 1 apart by one)
  int lq[2], lc[2], lm[2], lp[2];
#pragma unroll
  for (int rho = 0; rho < 2; ++rho) {
    const int qq = t1[rho] ? qr[rho] : W2 + 1;
    lq[rho] = Geo::lidx(qr[rho]);
    lc[rho] = Geo::lidx(qq);
    lm[rho] = Geo::lidx(qq - 1);
    lp[rho] = lm[rho] + 1;
  }

  // rings indexed by plane offset from istart: UB, W, B, NR mod 4, FIP (the
  // red point's +i face, read two planes later) and PA mod 2
  T UB[4], W[4][2], B[CB ? 1 : 4][2], NR[4], FIP[2];
  // right-hand side at this thread's positions on the plane in ring slot sl
  // With PW, W and (a full right-hand side) B hold a pair's two positions in
  // position order (one load each), else in role order (one load per role);
  // these pick role rho's value.  Tiles of which one workgroup fits a CU
  // (ONE: 16x64, three waves per SIMD, up to 168 registers) load pairs in
  // every variant, and the input-residual sweep its u_in pairs too (at 257^3
  // that sweep took 1368 instead of 1541 us); on the smaller tiles the
  // variants held to four waves per SIMD keep the role loads (the selects'
  // registers do not fit that budget, and the sweep with the coarse
  // correction measured slower with pairs).
  constexpr bool ONE = !KL && 10 * A2 * (int)sizeof(double) > 80 * 1024;
  constexpr bool PW = ONE || (NM == 0 && !PRO) || (NM == 1 && !CB);
  auto bv = [&](int sl, int rho) -> T {
    if constexpr (CB) return B[0][rho];
    else if constexpr (PW) return (rho ^ sw) ? B[sl][1] : B[sl][0];
    else return B[sl][rho];
  };
  auto w_role = [&](int sl, int rho) -> T {
    if constexpr (PW) return (rho ^ sw) ? W[sl][1] : W[sl][0];
    else return W[sl][rho];
  };
  // plane m = istart + rel: black role (rel + 1) & 1
  // byte offsets within a plane of this thread's two columns (past the plane
  // for positions outside the grid, which then read 0), and of its outputs
  // (past the plane for positions outside the tile or the interior)
  const uint32_t pbytes = (uint32_t)(sn2 * sizeof(T));
  uint32_t offi[2], offo[2];
#pragma unroll
  for (int rho = 0; rho < 2; ++rho) {
    offi[rho] = in[rho] ? (uint32_t)((jc * n + col[rho]) * sizeof(T)) : kOut;
    // outputs: the tile's interior points, and the boundary columns k = 0 and
    // k = n-1 of its rows (rewritten with their value 0, so that no cache
    // line of the output is left partly written: partial lines cost the
    // memory system a read-modify-write)
    const bool tb = t1[rho] && r >= 2 && r < TJ + 2 && intJ && (kc[rho] == 0 || kc[rho] == n - 1);
    offo[rho] = (tl[rho] || tb) ? (uint32_t)((j * n + kc[rho]) * sizeof(T)) : kOut;
  }
  const uint32_t gbytes = (uint32_t)n * pbytes;
  const auto rw0 = rsrc(d.wh, gbytes), rb0 = rsrc(d.b, bs ? gbytes : pbytes);
  const auto ru0 = rsrc(buf ? d.u[1] : d.u[0], gbytes);
  const T* const uout = buf ? d.u[0] : d.u[1];
  // wh (and a full right-hand side) of both positions of the pair come in one
  // 16-byte load, kept in position order and picked by role where used; with
  // NM = 1 and a full right-hand side u_in too (the black value feeds the red
  // update, the red one the residual of the input).  The pair starts at an
  // odd k; a pair reaching out of the grid on the left (k = -1) reads the
  // last values of the previous row there (where the outside used to read
  // zero: those positions feed only results that are masked or dropped, and
  // u there is a boundary zero either way), and the pair (-1, 0) of row 0 is
  // not loaded (both positions are boundary or outside).
  constexpr bool PL = NM == 1 && (!CB || ONE);  // (see below)
  T UP[PL ? 4 : 1][2];
  const bool pin = live && j >= 0 && j < n && kA <= n - 2 && (kA >= 0 || j >= 1);
  const uint32_t offp = pin ? (uint32_t)((j * n + kA) * (int)sizeof(T)) : kOut;
  // this slot's (plane istart + rel, rel = sl mod 4) u_in of role rho
  auto u_role = [&](int sl, int rho) -> T { return (rho ^ sw) ? UP[sl][1] : UP[sl][0]; };
  auto load = [&](int rel, int sl) {
    // planes past the grid are past the range and read 0
    const int m = istart + rel;
    const uint32_t so = (uint32_t)m * pbytes, sob = bs ? so : 0u;
    const int rb = (rel + 1) & 1;
    if constexpr (KL) {
      // wh of both positions on plane m (0 off the grid)
      const double* px = kl_lds + 4 * min(max(m, 0), n - 1);
      const bool pin = m >= 0 && m <= n - 1;
      T wv[2];
#pragma unroll
      for (int pos = 0; pos < 2; ++pos) {
        const double w = kl_wh(kl_z(KH[pos], px), etab);
        wv[pos] = (kin[pos] && pin) ? w : 0.0;
      }
      if constexpr (PW) {
        W[sl][0] = wv[0];
        W[sl][1] = wv[1];
      } else {
        W[sl][0] = sw ? wv[1] : wv[0];
        W[sl][1] = sw ? wv[0] : wv[1];
      }
    }
    if constexpr (PW) {
      if constexpr (!KL) {
        const Two<T> wv = bload2<T>(rw0, offp + so);
        W[sl][0] = wv.lo;
        W[sl][1] = wv.hi;
      }
      if constexpr (!CB) {
        const Two<T> bb = bload2<T>(rb0, offp + sob);
        B[sl][0] = bb.lo;
        B[sl][1] = bb.hi;
      }
    } else {
#pragma unroll
      for (int rho = 0; rho < 2; ++rho) {
        if constexpr (!KL) W[sl][rho] = bload<T>(rw0, offi[rho] + so);
        if (!CB) B[CB ? 0 : sl][rho] = bload<T>(rb0, offi[rho] + sob);
      }
    }
    if constexpr (PL) {
      const Two<T> v = bload2<T>(ru0, offp + so);
      UP[sl][0] = v.lo;
      UP[sl][1] = v.hi;
    } else {
      UB[sl] = bload<T>(ru0, (rb ? offi[1] : offi[0]) + so);
    }
  };
  // u_in of the black role on the plane in slot sl
  auto ubv = [&](int sl) -> T {
    if constexpr (PL) return u_role(sl, (sl + 1) & 1);
    else return UB[sl];
  };
  // NM = 1 with a constant right-hand side (held to the plain sweep's
  // registers, which the pair ring does not fit): the red role's input
  // value loaded on its own, two planes ahead, in slot rel & 1
  T UR[2];
  auto load_red = [&](int rel) {
    UR[rel & 1] = bload<T>(ru0, (rel & 1 ? offi[1] : offi[0]) + (uint32_t)(istart + rel) * pbytes);
  };

  // Coarse correction (PRO): the coarse iterate's planes under the tile are
  // staged in LDS (four slots by plane index mod 4), one value per thread,
  // loaded two planes ahead; the correction of a fine plane is formed from
  // LDS one plane before its values are first used.  A coarse value goes to
  // LDS two fine planes after its load is issued (two staging registers by
  // plane parity), so it has as long to arrive as the fine plane loads.
  constexpr int CJM = PRO ? TJ / 2 + 4 : 1, CKM = PRO ? TK / 2 + 4 : 1;
  __shared__ T sC[PRO ? 4 : 1][CJM * CKM];
  const int cj0 = max(j0 - 2, 1) >> 1, ck0 = max(k0 - 2, 1) >> 1;
  const int CK = (min(k0 + TK + 1, n - 2) >> 1) + 2 - ck0;
  const int CJ = (min(j0 + TJ + 1, n - 2) >> 1) + 2 - cj0;
  const bool cown = PRO && t < CJ * CK;
  const int crow = cown ? t / CK : 0, ccol = cown ? t - (t / CK) * CK : 0;
  T cstage[2] = {0, 0}, PA[2] = {0, 0};
  auto c_issue = [&](int C, int sl) {
    const int Cc = min(max(C, 0), nc - 1);
    cstage[sl] = ec[(Cc * nc + min(cj0 + crow, nc - 1)) * nc + min(ck0 + ccol, nc - 1)];
  };
  auto c_store = [&](int C, int sl) {
    if (cown) sC[C & 3][crow * CKM + ccol] = cstage[sl];
  };
  // Correction at fine (m, j, kk), zero off the interior, evaluated as the
  // trilinear interpolation is written (prolong_combine): the (j, k) part on
  // the coarse planes (m >> 1) and (m >> 1) + 1, then the i part.  The (j, k)
  // part on the upper plane is the lower one of plane m + 2, the next plane
  // of the same role: it is returned in P1 and passed back as P0 then.
  // The weights 1 and 1/2 are taken as index choices: an even position
  // pairs a coarse value with itself, so the sum of two values halved
  // (exactly, by a power of two) gives the bits of the weighted form, with
  // four operations instead of nine per (j, k) part.
  auto pjk = [&](int I, int kk) -> T {
    const int ki = min(max(kk, 1), n - 2);
    const T* c = sC[I & 3];
    const int o = ((jI >> 1) - cj0) * CKM + (ki >> 1) - ck0;
    const int dk = ki & 1, dj = (jI & 1) ? CKM : 0;
    return (T)0.25 * ((c[o] + c[o + dk]) + (c[o + dj] + c[o + dj + dk]));
  };
  auto pa_from = [&](int m, int kk, bool intk, T P0, T& P1) -> T {
    const int mi = min(max(m, 1), n - 2);
    P1 = pjk((mi >> 1) + 1, kk);
    const T pa = (T)0.5 * (P0 + ((mi & 1) ? P1 : P0));
    return (m >= 1 && m <= n - 2 && intk) ? pa : (T)0;
  };
  auto pa_of = [&](int m, int kk, bool intk, T& P1) -> T {
    return pa_from(m, kk, intk, pjk(min(max(m, 1), n - 2) >> 1, kk), P1);
  };
  T PJ[2] = {0, 0};  // per role: the (j, k) part for its next plane

  // prologue: planes istart-1 .. istart+2, the +i face of the red point below
  // plane istart (the black points of plane istart use it), plane istart to LDS
  if (CB) {
    B[0][0] = bload<T>(rb0, offi[0]);
    B[0][1] = bload<T>(rb0, offi[1]);
  }
  if (NM == 1 && !PL) {
    load_red(0);
    load_red(1);
  }
  load(-1, 3);
  load(0, 0);
  load(1, 1);
  load(2, 2);
  T acc = 0;  // NM: this thread's sum of squared residuals
  if (PRO) {
    const int clo = max((istart - 1) >> 1, 0), chi = ((istart + 2) >> 1) + 1;
    for (int C = clo; C <= chi; ++C) {
      c_issue(C, 0);
      c_store(C, 0);
    }
    c_issue(((istart + 3) >> 1) + 1, 0);  // stored at the end of plane istart
    c_issue(((istart + 4) >> 1) + 1, 1);  // and of plane istart + 1
    __syncthreads();
    // black roles: plane istart-1 -> 0, istart -> 1, istart+1 -> 0
    T P1;
    UB[3] += pa_of(istart - 1, kc[0], intr[0], P1);
    UB[0] += pa_of(istart, kc[1], intr[1], PJ[1]);     // role 1 again on plane istart + 2
    PA[1] = pa_of(istart + 1, kc[0], intr[0], PJ[0]);  // role 0 again on plane istart + 3
  }
  NR[3] = 0;
  NR[2] = 0;
  FIP[1] = rcp<T>(w_role(3, 1) + w_role(0, 1));  // plane istart-1 is red in role 1
  FIP[0] = 0;
  if (live) {
    sU[0][lq[1]] = ubv(0);
    sW[0][lq[1]] = w_role(0, 1);
  }
  __syncthreads();
  // All prologue loads are waited for once here.  The compiler sets the
  // memory waits at the head of the march for the loads pending on both ways
  // into it: without this wait the prologue's issue order would set them,
  // and every group of four planes would wait for almost all of its loads
  // in flight instead of those it uses.
  __builtin_amdgcn_s_waitcnt(kWaitVmem0);

  // one plane, K = (i - istart) mod 4 at compile time
  auto plane = [&](auto kk, int i) {
    constexpr int K = decltype(kk)::value;
    constexpr int RHO = K & 1;                 // red role on plane i
    constexpr int S0 = K, SM = (K + 3) & 3, SP = (K + 1) & 3, SM2 = (K + 2) & 3;
    constexpr int PB = K & 1, PBM = (K + 1) & 1;  // LDS buffers of planes i and i-1
    const int qc = lc[RHO], qm = lm[RHO], qp = lp[RHO];
    constexpr int DJ = Geo::DJ;  // LDS index step of one row
    if (PRO) {
      UB[SP] += PA[(K + 1) & 1];                                 // plane i+1 (black role RHO)
      PA[K & 1] = pa_from(i + 2, kc[1 - RHO], intr[1 - RHO], PJ[1 - RHO], PJ[1 - RHO]);  // i+2
    }
    // red point of plane i
    const T wc = w_role(S0, RHO);
    const T* Wl = sW[PB];
    const T* Ul = sU[PB];
    const T fim = rcp<T>(wc + w_role(SM, RHO)), fip = rcp<T>(wc + w_role(SP, RHO));
    const T fjm = rcp<T>(wc + Wl[qc - DJ]), fjp = rcp<T>(wc + Wl[qc + DJ]);
    const T fkm = rcp<T>(wc + Wl[qm]), fkp = rcp<T>(wc + Wl[qp]);
    const St<T> sr = stencil_faces<T>(fim, fip, fjm, fjp, fkm, fkp, ubv(SM), ubv(SP), Ul[qc - DJ],
                                      Ul[qc + DJ], Ul[qm], Ul[qp]);
    const T vr = gs_value<T>(sr, bv(S0, RHO));
    NR[S0] = (t1[RHO] && intr[RHO] && i <= n - 2) ? vr : (T)0;
    if (NM == 1) {
      const T rr = res_value<T>(sr, bv(S0, RHO), PL ? u_role(S0, RHO) : UR[K & 1]);
      acc += (tl[RHO] && i >= ia && i <= ib) ? rr * rr : (T)0;
    }
    // black point of plane p = i - 1 (the column that is red on plane i)
    // (planes outside this chunk, including the ones the last unrolled step
    // may run past the end, are computed and their stores dropped: the
    // output descriptor then has an empty range; no branch keeps the memory
    // counters' bookkeeping exact)
    const int p = i - 1;
    {
      const bool outp = p >= ia && p <= ib;
      const T* Rl = sR[PBM];
      const T* Fj = sFj[PBM];
      const T* Fk = sFk[PBM];
      const St<T> sb = stencil_faces<T>(FIP[K & 1], fim, Fj[qc - DJ], Fj[qc], Fk[qm], Fk[qc],
                                        NR[SM2], NR[S0], Rl[qc - DJ], Rl[qc + DJ], Rl[qm],
                                        Rl[qp]);
      const T vb = gs_value<T>(sb, bv(SM, RHO));
      if (NM == 2) {
        const T rb = res_value<T>(sb, bv(SM, RHO), vb);
        acc += (tl[RHO] && outp) ? rb * rb : (T)0;
      }
      const uint32_t sop = (uint32_t)p * pbytes;
      const auto ro = rsrc(uout, outp ? gbytes : 0u);
      bstore<T>(ro, offo[RHO] + sop, intr[RHO] ? vb : (T)0);
      bstore<T>(ro, offo[1 - RHO] + sop, NR[SM]);
    }
    FIP[K & 1] = fip;  // after the black point above read plane i-2's
    // publish plane i's red values and faces, and plane i+1's black u_in and
    // wh (the buffers read in this plane are the other parity)
    if (t1[RHO]) {
      sR[PB][qc] = NR[S0];
      sFj[PB][qc - DJ] = fjm;
      sFj[PB][qc] = fjp;
      sFk[PB][qm] = fkm;
      sFk[PB][qc] = fkp;
    }
    if (live) {
      sU[PBM][lq[RHO]] = ubv(SP);
      sW[PBM][lq[RHO]] = w_role(SP, RHO);
    }
    // loads of plane i+3 (into the ring slot plane i-1 leaves); the next
    // coarse plane to LDS every second plane
    if (NM == 1 && !PL) load_red(i - istart + 2);
    load(i - istart + 3, SM);
    if (PRO) {
      // coarse plane ((i+3)>>1)+1 to LDS (a second store of the same plane
      // rewrites identical values), the one for plane i+2 into its register
      c_store(((i + 3) >> 1) + 1, K & 1);
      c_issue(((i + 5) >> 1) + 1, K & 1);
    }
    __syncthreads();
  };

  // whole groups of four planes (up to three past iend: loads there read
  // zeros or clamped planes, stores are dropped, LDS values are not used)
  for (int i = istart; i <= iend; i += 4) {
    plane(std::integral_constant<int, 0>{}, i);
    plane(std::integral_constant<int, 1>{}, i + 1);
    plane(std::integral_constant<int, 2>{}, i + 2);
    plane(std::integral_constant<int, 3>{}, i + 3);
  }
  if (NM) {
    // workgroup sum in a fixed order: within waves by shuffles, then the
    // wave totals in wave order
    constexpr int NW = Geo::THREADS / 64;
    __shared__ T ws[NM ? NW : 1];
    T v = acc;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    // (lane from the lane counter and wave index from a scalar register: the
    // thread index then need not stay live through the march)
    const int lane = __lane_id();
    if (lane == 0) ws[wave] = v;
    __syncthreads();
    if (wave == 0 && lane == 0 && d.spoff >= 0) {
      T sum = 0;
      for (int w = 0; w < NW; ++w) sum += ws[w];
      spart[d.spoff + blk] = sum;
      // the number of partials of this grid, for the judgement that sums them
      if (blk == 0) spart[d.spoff + (NM == 2 ? 2 * kSweepParts : kSweepParts + 1)] = (T)per;
    }
  }
}

// (KL: held to three waves per SIMD, the occupancy its LDS allows on the
// larger tiles)
template <typename T, int TJ, int TK, bool PRO, bool CB, bool KL>
__global__ void __launch_bounds__((SweepGeom<TJ, TK>::THREADS))
    __attribute__((amdgpu_waves_per_eu(KL ? 3 : 1)))
    k_sweep(const GridDescT<T>* __restrict__ list, const int* __restrict__ active, int buf,
            int cbuf, int tiles_k, int tiles_jk, int chunks, int count, int nwg) {
  sweep_tile<T, TJ, TK, PRO, 0, CB, KL>(list, active, buf, cbuf, tiles_k, tiles_jk, chunks,
                                        count, nwg, nullptr);
}

// The sweep with the black residuals of its output, held to the plain
// sweep's register budget (four waves per SIMD) so that it runs with the
// plain sweep's shape and occupancy.
template <typename T, int TJ, int TK, bool CB, bool KL>
__global__ void __launch_bounds__((SweepGeom<TJ, TK>::THREADS))
    __attribute__((amdgpu_waves_per_eu(KL ? 3 : 4)))
    k_sweep_res_out(const GridDescT<T>* __restrict__ list, const int* __restrict__ active,
                    int buf, int tiles_k, int tiles_jk, int chunks, int count, int nwg,
                    T* __restrict__ spart) {
  sweep_tile<T, TJ, TK, false, 2, CB, KL>(list, active, buf, -1, tiles_k, tiles_jk, chunks,
                                          count, nwg, spart);
}

// The sweep with the red residuals of its input keeps the input values of
// the red role in registers as well.  With a constant right-hand side (no
// right-hand-side ring) it fits the plain sweep's budget and shapes; with a
// full one it takes the budget and shapes of the sweep with the coarse
// correction.
template <typename T, int TJ, int TK, bool KL>
__global__ void __launch_bounds__((SweepGeom<TJ, TK>::THREADS))
    __attribute__((amdgpu_waves_per_eu(KL ? 3 : 4)))
    k_sweep_res_in_cb(const GridDescT<T>* __restrict__ list, const int* __restrict__ active,
                      int buf, int tiles_k, int tiles_jk, int chunks, int count, int nwg,
                      T* __restrict__ spart) {
  sweep_tile<T, TJ, TK, false, 1, true, KL>(list, active, buf, -1, tiles_k, tiles_jk, chunks,
                                            count, nwg, spart);
}
template <typename T, int TJ, int TK, bool KL>
__global__ void __launch_bounds__((SweepGeom<TJ, TK>::THREADS))
    __attribute__((amdgpu_waves_per_eu(KL ? 3 : 1)))
    k_sweep_res_in(const GridDescT<T>* __restrict__ list, const int* __restrict__ active,
                   int buf, int tiles_k, int tiles_jk, int chunks, int count, int nwg,
                   T* __restrict__ spart) {
  sweep_tile<T, TJ, TK, false, 1, false, KL>(list, active, buf, -1, tiles_k, tiles_jk, chunks,
                                             count, nwg, spart);
}

// ---- point kernels: colour sweep, residual, transfer -------------------------

// In-place Gauss-Seidel update of one colour ((i+j+k) even = red): the
// two-pass alternative to k_sweep.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rbgs_colour(const GridDescT<T>* __restrict__ list,
                                                        const int* __restrict__ active,
                                                        int colour, int buf, int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = interior_point(n - 2, blk);
  if (!p.ok || ((p.i + p.j + p.k) & 1) != colour) return;
  const int v = vidx(n, p.i, p.j, p.k);
  const gptr<T> u = gview<T>(buf ? d.u[1] : d.u[0]);
  const St<T> st = stencil_at<T>(u, gview<T>(d.wh), v, n, n * n);
  u[v] = gs_value<T>(st, b_at<T>(d, p.i, p.j, p.k));
}

// Column marching: a 256-thread block owns 4 rows (j) x 64 columns (k) of
// interior columns and walks the planes i, keeping u and wh of its own column
// at i-1, i, i+1 in registers; the in-plane neighbours come through the cache.
struct Col {
  int j, k;
  bool ok;
};
__device__ __forceinline__ Col column_of(int m, int bid) {
  const int nkc = ceil_div(m, 64);
  const int kc = bid % nkc, jc = bid / nkc;
  const int k = kc * 64 + (threadIdx.x & 63), j = jc * 4 + (threadIdx.x >> 6);
  return {1 + j, 1 + k, j < m && k < m};
}

// Column data of one plane m for the residual at (m, j, k): the four
// in-plane neighbours of u and wh, b', and the centre u, wh of plane m + 1.
template <typename T>
struct ColSlot {
  T u4[4], w4[4], b, uc, wc;
};
// Loads of column slots through per-plane buffer descriptors: a plane outside
// the grid (or, for b', outside the interior) reads zeros, so a march can run
// past its last plane without branches.
template <typename T>
struct ColLoader {
  const T* u;
  const T* wh;
  const T* b;
  int n, sn2, bs;
  uint32_t pbytes, oc, o4[4];
  __device__ __forceinline__ ColLoader(const GridDescT<T>& d, const T* u_, int j, int k)
      : u(u_), wh(d.wh), b(d.b), n(d.n), sn2(d.n * d.n), bs(d.bstride) {
    pbytes = (uint32_t)(sn2 * sizeof(T));
    oc = (uint32_t)((j * n + k) * sizeof(T));
    o4[0] = oc - (uint32_t)(n * sizeof(T));
    o4[1] = oc + (uint32_t)(n * sizeof(T));
    o4[2] = oc - (uint32_t)sizeof(T);
    o4[3] = oc + (uint32_t)sizeof(T);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane(const T* base, int m, bool ok) const {
    return rsrc(base + (size_t)(ok ? m : 0) * sn2, ok ? pbytes : 0u);
  }
  __device__ __forceinline__ void load(int m, ColSlot<T>& s) const {
    const bool ok0 = m <= n - 1, ok1 = m + 1 <= n - 1, okb = m <= n - 2;
    const auto ru = plane(u, m, ok0), rw = plane(wh, m, ok0);
    const auto ru1 = plane(u, m + 1, ok1), rw1 = plane(wh, m + 1, ok1);
    const auto rb = rsrc(b + (size_t)(okb ? m : 0) * bs, okb ? pbytes : 0u);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s.u4[q] = bload<T>(ru, o4[q]);
      s.w4[q] = bload<T>(rw, o4[q]);
    }
    s.b = bload<T>(rb, oc);
    s.uc = bload<T>(ru1, oc);
    s.wc = bload<T>(rw1, oc);
  }
};

// Walks the interior planes of column (c.j, c.k), calling f(i, r) with the
// residual r = b' - A'u at (i, c.j, c.k) for i = 1 .. n-2, then with r = 0 for
// up to two planes past n-2 (callers drop those: stores through an
// empty-range descriptor, sums of zeros).  Three planes of loads are in
// flight (a ring of three slots, the march unrolled by three, no branch).
template <typename T, typename F>
__device__ __forceinline__ void march_residual(const GridDescT<T>& d, const T* u_, Col c, F&& f) {
  const int n = d.n;
  const ColLoader<T> L(d, u_, c.ok ? c.j : 1, c.ok ? c.k : 1);
  ColSlot<T> S[3];
  L.load(1, S[0]);
  L.load(2, S[1]);
  L.load(3, S[2]);
  const auto r0 = L.plane(u_, 1, true), w0r = L.plane(d.wh, 1, true), wm0 = L.plane(d.wh, 0, true);
  T um = 0, u0 = bload<T>(r0, L.oc), w0 = bload<T>(w0r, L.oc);
  // the face to the plane below is the previous plane's face to the plane above
  T fim = rcp<T>(w0 + bload<T>(wm0, L.oc));
  auto step = [&](auto kk, int i) {
    constexpr int K = decltype(kk)::value;
    ColSlot<T>& sl = S[K];
    const T up = sl.uc, wp = sl.wc;
    const T fip = rcp<T>(w0 + wp);
    const St<T> st = stencil_faces<T>(fim, fip, rcp<T>(w0 + sl.w4[0]), rcp<T>(w0 + sl.w4[1]),
                                      rcp<T>(w0 + sl.w4[2]), rcp<T>(w0 + sl.w4[3]), um, up,
                                      sl.u4[0], sl.u4[1], sl.u4[2], sl.u4[3]);
    const T r = res_value<T>(st, sl.b, u0);
    f(i, (c.ok && i <= n - 2) ? r : (T)0);
    um = u0;
    u0 = up;
    w0 = wp;
    fim = fip;
    L.load(i + 3, sl);
    // keep each plane's loads where they are (issued two planes before use)
    __builtin_amdgcn_sched_barrier(0);
  };
  for (int i = 1; i <= n - 2; i += 3) {
    step(std::integral_constant<int, 0>{}, i);
    step(std::integral_constant<int, 1>{}, i + 1);
    step(std::integral_constant<int, 2>{}, i + 2);
  }
}

// The residual over a tile of 4 rows x 64 columns (one column per thread of
// a 256-thread block, the column decomposition of column_of), marched over the
// planes with each plane's u and wh of the tile and its one-point ring in LDS:
// a thread loads only its own column (and 136 threads one ring position), the
// in-plane neighbours come from LDS.  Calls f(i, r) for i = 1 .. n-2 with
// r = b' - A'u at (i, c.j, c.k) (0 where c is not interior), then with r = 0
// for up to three planes past n-2.  Loads run two planes ahead (rings of
// four slots, the march unrolled by four, no branch); one barrier per plane.
// The stencil operands and their order are those of march_residual, so the
// values are identical.
template <typename T, typename F>
__device__ __forceinline__ void tile_residual(const GridDescT<T>& d, const T* u_, int blk, F&& f) {
  constexpr int TJ = 4, TK = 64, W = TK + 2, H = TJ + 2, A = W * H;
  __shared__ T LU[2][A], LW[2][A];
  const int n = d.n, sn2 = n * n, m = n - 2;
  const int nkc = ceil_div(m, TK);
  const int kc = blk % nkc, jc = blk / nkc;
  const int t = threadIdx.x;
  const int r = t >> 6, cc = t & 63;
  const int j = 1 + jc * TJ + r, k = 1 + kc * TK + cc;
  const bool interior = j <= n - 2 && k <= n - 2;
  const bool ingrid = j <= n - 1 && k <= n - 1;
  const int q = (r + 1) * W + cc + 1;
  // ring position of this thread (t < 136): rows above/below, columns left/right
  int hr, hc;
  if (t < 64) { hr = 0; hc = t + 1; }
  else if (t < 128) { hr = H - 1; hc = t - 63; }
  else if (t < 132) { hr = t - 127; hc = 0; }
  else { hr = t - 131; hc = W - 1; }
  const bool halo = t < 136;
  const int hj = jc * TJ + hr, hk = kc * TK + hc;  // grid coordinates (row j0-1+hr)
  const bool hgrid = halo && hj >= 0 && hj <= n - 1 && hk >= 0 && hk <= n - 1;
  const int hq = hr * W + hc;
  const uint32_t pbytes = (uint32_t)(sn2 * sizeof(T));
  const uint32_t oo = ingrid ? (uint32_t)((j * n + k) * sizeof(T)) : kOut;
  const uint32_t oh = hgrid ? (uint32_t)((hj * n + hk) * sizeof(T)) : kOut;
  auto plane = [&](const T* base, int pm, bool ok) {
    return rsrc(base + (size_t)(ok ? pm : 0) * sn2, ok ? pbytes : 0u);
  };
  T OU[4], OW[4], OB[4], HU[4], HW[4];
  // plane pm into ring slot (pm - 1) & 3
  auto load = [&](int pm, int sl) {
    const bool ok = pm <= n - 1, okb = pm <= n - 2;
    const auto ru = plane(u_, pm, ok), rw = plane(d.wh, pm, ok);
    const auto rb = rsrc(d.b + (size_t)(okb ? pm : 0) * d.bstride, okb ? pbytes : 0u);
    OU[sl] = bload<T>(ru, oo);
    OW[sl] = bload<T>(rw, oo);
    OB[sl] = bload<T>(rb, oo);
    HU[sl] = bload<T>(ru, oh);
    HW[sl] = bload<T>(rw, oh);
  };
  load(0, 3);
  load(1, 0);
  load(2, 1);
  load(3, 2);
  LU[1][q] = OU[0];
  LW[1][q] = OW[0];
  if (halo) {
    LU[1][hq] = HU[0];
    LW[1][hq] = HW[0];
  }
  __syncthreads();
  T fim = rcp<T>(OW[0] + OW[3]);
  auto step = [&](auto kk, int i) {
    constexpr int K = decltype(kk)::value;
    constexpr int S0 = K, SM = (K + 3) & 3, SP = (K + 1) & 3;
    constexpr int PB = (K + 1) & 1, PN = K & 1;  // LDS buffers of planes i and i+1
    const T w = OW[S0];
    const T fip = rcp<T>(w + OW[SP]);
    const T* Lu = LU[PB];
    const T* Lw = LW[PB];
    const St<T> st = stencil_faces<T>(fim, fip, rcp<T>(w + Lw[q - W]), rcp<T>(w + Lw[q + W]),
                                      rcp<T>(w + Lw[q - 1]), rcp<T>(w + Lw[q + 1]), OU[SM],
                                      OU[SP], Lu[q - W], Lu[q + W], Lu[q - 1], Lu[q + 1]);
    const T rv = res_value<T>(st, OB[S0], OU[S0]);
    f(i, (interior && i <= n - 2) ? rv : (T)0);
    fim = fip;
    // plane i+1 to LDS, loads of plane i+3 into the slot plane i-1 leaves
    LU[PN][q] = OU[SP];
    LW[PN][q] = OW[SP];
    if (halo) {
      LU[PN][hq] = HU[SP];
      LW[PN][hq] = HW[SP];
    }
    load(i + 3, SM);
    __syncthreads();
  };
  for (int i = 1; i <= n - 2; i += 4) {
    step(std::integral_constant<int, 0>{}, i);
    step(std::integral_constant<int, 1>{}, i + 1);
    step(std::integral_constant<int, 2>{}, i + 2);
    step(std::integral_constant<int, 3>{}, i + 3);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_residual(const GridDescT<T>* __restrict__ list,
                                                     const int* __restrict__ active, int buf,
                                                     int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const Col c = column_of(d.n - 2, blk);
  if (!c.ok) return;
  const int n = d.n, sn2 = n * n;
  const uint32_t oc = (uint32_t)((c.j * n + c.k) * sizeof(T)), pbytes = (uint32_t)(sn2 * sizeof(T));
  march_residual<T>(d, buf ? d.u[1] : d.u[0], c, [&](int i, T v) {
    const bool ok = i <= n - 2;
    bstore<T>(rsrc(d.r + (size_t)(ok ? i : 0) * sn2, ok ? pbytes : 0u), oc, v);
  });
}

// Full weighting of the residual to the coarse right-hand side, h^2 scaling
// included: b'_c(I) = 4 * sum_d 2^{-|d|_1}/8 r'(2I+d); also starts the coarse
// cycle from a zero iterate in uc[0].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(const GridDescT<T>* __restrict__ list,
                                                     const int* __restrict__ active, int count,
                                                     int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n, nc = (n - 1) / 2 + 1;
  const Pt p = interior_point(nc - 2, blk);
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

// Residual and full weighting in one pass: a workgroup owns RJ x RK coarse
// columns and the (2RJ+1) x (2RK+1) fine columns under them; every fine
// thread marches its column computing r = b' - A'u (as the residual kernel),
// puts each plane's residuals in LDS, and the coarse threads add that
// plane's share of the 27-point weights to their running sums, plane by plane
// in increasing order (the order of the separate restriction).  r never goes
// to memory; the coarse iterate uc[0] is zeroed as by the restriction.
template <int RJ, int RK>
struct RRGeom {
  static constexpr int FJ = 2 * RJ + 1, FK = 2 * RK + 1, FT = FJ * FK;
  static constexpr int THREADS = ((FT + 63) / 64) * 64;
};

// CB: every grid has a constant right-hand side plane (loaded once).  Grid
// arrays are addressed as in the sweep: one descriptor per array, the
// plane's offset added to the per-lane offsets.  KL (FP64): wh evaluated from
// the grid's KL data as in the sweep (the mode table in dynamic LDS).
// chunks: pieces of the coarse planes per tile (a launch with few grids
// splits each tile's march so that it still has many workgroups); a piece
// of coarse planes Ia..Ib marches the fine planes 2Ia-1..2Ib+1 and stores
// only its own coarse planes, each summed over its fine planes in the same
// order as by a whole march.
template <typename T, int RJ, int RK, bool CB, bool KL>
__global__ void __launch_bounds__((RRGeom<RJ, RK>::THREADS))
    k_resrestrict(const GridDescT<T>* __restrict__ list, const int* __restrict__ active, int buf,
                  int tiles_k, int tiles, int chunks, int count, int per) {
  using G = RRGeom<RJ, RK>;
  // fine tile FJ x FK with a one-point ring in LDS (u, wh per plane parity)
  constexpr int FJ = G::FJ, FK = G::FK, W = FK + 2, H = FJ + 2, A = W * H;
  constexpr int NH = 2 * FK + 2 * FJ;  // ring positions (corners are not needed)
  __shared__ T LU[2][A], LW[2][A];
  __shared__ T R[2][G::FT];
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n, sn2 = n * n, nc = (n - 1) / 2 + 1;
  const int ch = blk / tiles, tile = blk - ch * tiles;
  const int tj = tile / tiles_k, tk = tile - tj * tiles_k;
  const int J0 = 1 + tj * RJ, K0 = 1 + tk * RK;
  // this piece's coarse planes and the fine planes it marches
  const int clen = ceil_div(nc - 2, chunks);
  const int Ia = 1 + ch * clen, Ib = min(nc - 2, Ia + clen - 1);
  const int i0 = 2 * Ia - 1, i1 = 2 * Ib + 1;
  const int jb = 2 * J0 - 1, kb = 2 * K0 - 1;  // fine origin of the tile
  const int t = threadIdx.x;
  // this thread's fine column
  const bool fl = t < G::FT;
  const int fj = fl ? t / FK : 0, fk = fl ? t - (t / FK) * FK : 0;
  const int j = jb + fj, k = kb + fk;
  const bool fin = fl && j <= n - 2 && k <= n - 2;
  const bool fgrid = fl && j <= n - 1 && k <= n - 1;
  const int q = (fj + 1) * W + fk + 1;
  // ring position (t < NH): rows above/below the tile, then columns left/right
  int hr = 0, hc = 0;
  if (t < FK) { hr = 0; hc = t + 1; }
  else if (t < 2 * FK) { hr = H - 1; hc = t - FK + 1; }
  else if (t < 2 * FK + FJ) { hr = t - 2 * FK + 1; hc = 0; }
  else if (t < NH) { hr = t - 2 * FK - FJ + 1; hc = W - 1; }
  const bool halo = t < NH;
  const int hj = jb - 1 + hr, hk = kb - 1 + hc;
  const bool hgrid = halo && hj >= 0 && hj <= n - 1 && hk >= 0 && hk <= n - 1;
  const int hq = hr * W + hc;
  // this thread's coarse column
  const bool cl = t < RJ * RK;  // coarse threads: the first waves
  const int cj = cl ? t / RK : 0, ck = cl ? t - (t / RK) * RK : 0;
  const int J = J0 + cj, K = K0 + ck;
  const bool cin = cl && J <= nc - 2 && K <= nc - 2;
  const int o = (2 * cj + 1) * FK + 2 * ck + 1;  // R index of fine (2J, 2K)
  const uint32_t pbytes = (uint32_t)(sn2 * sizeof(T));
  const uint32_t cbytes = (uint32_t)(nc * nc * sizeof(T));
  const uint32_t oo = fgrid ? (uint32_t)((j * n + k) * sizeof(T)) : kOut;
  const uint32_t oh = hgrid ? (uint32_t)((hj * n + hk) * sizeof(T)) : kOut;
  // coarse outputs: interior points, and the boundary columns K = 0 (a second
  // store by the threads of column K0 = 1) and K = nc-1 of interior rows,
  // rewritten with 0 so that no cache line is left partly written
  const bool cbr = cl && J <= nc - 2 && K == nc - 1;
  const uint32_t oco = (cin || cbr) ? (uint32_t)((J * nc + K) * sizeof(T)) : kOut;
  const uint32_t oc0 = (cl && K == 1 && J <= nc - 2) ? (uint32_t)(J * nc * sizeof(T)) : kOut;
  // (planes past the grid are past the range and read 0; the residual of
  // the boundary planes is not used)
  const uint32_t gbytes = (uint32_t)n * pbytes;
  const auto ru = rsrc(buf ? d.u[1] : d.u[0], gbytes), rw = rsrc(d.wh, gbytes);
  const auto rb = rsrc(d.b, d.bstride ? gbytes : pbytes);
  T OU[4], OW[4], OB[CB ? 1 : 4], HU[4], HW[4];
  if (CB) OB[0] = bload<T>(rb, oo);
  // KL: mode table and weights in LDS, the column parts of the own column
  // (wh = 0 off the grid, as a read past the range gives); the ring columns
  // still read wh (values a neighbouring workgroup streams: cache hits)
  static_assert(!KL || std::is_same<T, double>::value, "the KL transfer is FP64");
  extern __shared__ double kl_lds[];
  double KO[KL ? 4 : 1];
  const double* etab = kl_lds + 4 * n + 64;
  if constexpr (KL) {
    double* sC = kl_lds + 4 * n;
    for (int qq = t; qq < 4 * n; qq += G::THREADS) kl_lds[qq] = d.klphi[(qq & 3) * n + (qq >> 2)];
    if (t < 64) sC[t] = d.klcoef[t] * d.kln[t];
    if (t < 32) sC[64 + t] = kExp2Tab[t];
    __syncthreads();
    auto column = [&](int jj, int kk, double (&H)[4]) {
      const int jy = min(max(jj, 0), n - 1), kz = min(max(kk, 0), n - 1);
      double py[4], pz[4], P[16];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        py[b] = kl_lds[4 * jy + b];
        pz[b] = kl_lds[4 * kz + b];
      }
      kl_rows(sC, py, P);
      kl_cols(P, pz, H);
    };
    column(j, k, KO);
  }
  auto load = [&](int pm, int sl) {
    const uint32_t so = (uint32_t)pm * pbytes;
    OU[sl] = bload<T>(ru, oo + so);
    if constexpr (KL) {
      const double* px = kl_lds + 4 * min(pm, n - 1);
      const double wo = kl_wh(kl_z(KO, px), etab);
      OW[sl] = (fgrid && pm <= n - 1) ? wo : 0.0;
    } else {
      OW[sl] = bload<T>(rw, oo + so);
    }
    HW[sl] = bload<T>(rw, oh + so);
    if (!CB) OB[sl] = bload<T>(rb, oo + (d.bstride ? so : 0u));  // (a constant plane: stride 0)
    HU[sl] = bload<T>(ru, oh + so);
  };
  auto prologue = [&]() {
    load(i0 - 1, 3);
    load(i0, 0);
    load(i0 + 1, 1);
    load(i0 + 2, 2);
    if (fl) {
      LU[1][q] = OU[0];
      LW[1][q] = OW[0];
    }
    if (halo) {
      LU[1][hq] = HU[0];
      LW[1][hq] = HW[0];
    }
  };
  T fim = 0;
  T s = 0;
  // the residual of plane i into R (fine threads), the next plane to LDS
  auto fine = [&](auto kk, int i) {
    constexpr int KS = decltype(kk)::value;
    constexpr int S0 = KS, SM = (KS + 3) & 3, SP = (KS + 1) & 3;
    constexpr int PB = (KS + 1) & 1, PN = KS & 1;  // buffers of planes i and i+1
    const int qs = fl ? q : W + 1;
    const T w = OW[S0];
    const T fip = rcp<T>(w + OW[SP]);
    const T* Lu = LU[PB];
    const T* Lw = LW[PB];
    const St<T> st = stencil_faces<T>(fim, fip, rcp<T>(w + Lw[qs - W]), rcp<T>(w + Lw[qs + W]),
                                      rcp<T>(w + Lw[qs - 1]), rcp<T>(w + Lw[qs + 1]), OU[SM],
                                      OU[SP], Lu[qs - W], Lu[qs + W], Lu[qs - 1], Lu[qs + 1]);
    const T rv = res_value<T>(st, OB[CB ? 0 : S0], OU[S0]);
    fim = fip;
    if (fl) {
      R[PB][t] = (fin && i <= n - 2) ? rv : (T)0;
      LU[PN][q] = OU[SP];
      LW[PN][q] = OW[SP];
    }
    if (halo) {
      LU[PN][hq] = HU[SP];
      LW[PN][hq] = HW[SP];
    }
    load(i + 3, SM);
  };
  // plane i's share of the 27-point weights (coarse threads), in increasing
  // plane order; an odd plane closes coarse plane (i-1)/2 (stored if
  // interior) and opens (i+1)/2
  auto coarse = [&](auto kk, int i) {
    constexpr int KS = decltype(kk)::value;
    constexpr int PB = (KS + 1) & 1;
    if (cl) {
      const T* Rp = R[PB];
      const bool odd = (i & 1) != 0;
      const T wi = odd ? (T)0.5 : (T)1;
      T tm[3];
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const T wj = dj == 0 ? wi : (T)0.5 * wi;
        const int row = o + dj * FK;
        tm[dj + 1] = wj * (Rp[row] + (T)0.5 * (Rp[row - 1] + Rp[row + 1]));
      }
      T s1 = s;
      s1 += tm[0];
      s1 += tm[1];
      s1 += tm[2];
      const int I = (i - 1) >> 1;
      const bool st_ok = odd && I >= Ia && I <= Ib;
      const uint32_t cso = (uint32_t)I * cbytes, cg = st_ok ? (uint32_t)nc * cbytes : 0u;
      const auto rbc = rsrc(d.bc, cg), ruc = rsrc(d.uc[0], cg);
      bstore<T>(rbc, oco + cso, cin ? (T)0.5 * s1 : (T)0);
      bstore<T>(ruc, oco + cso, (T)0);
      bstore<T>(rbc, oc0 + cso, (T)0);
      bstore<T>(ruc, oc0 + cso, (T)0);
      T s0 = 0;
      s0 += tm[0];
      s0 += tm[1];
      s0 += tm[2];
      s = odd ? s0 : s1;
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  prologue();
  fim = rcp<T>(OW[0] + OW[3]);
  __syncthreads();
  // prologue loads waited for once (as in the smoother: the waits at the
  // head of the march then follow the loop's own load order)
  __builtin_amdgcn_s_waitcnt(kWaitVmem0);
  for (int i = i0; i <= i1; i += 4) {
    fine(I0{}, i);
    __syncthreads();
    coarse(I0{}, i);
    fine(I1{}, i + 1);
    __syncthreads();
    coarse(I1{}, i + 1);
    fine(I2{}, i + 2);
    __syncthreads();
    coarse(I2{}, i + 2);
    fine(I3{}, i + 3);
    __syncthreads();
    coarse(I3{}, i + 3);
  }
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
  const St<T> st = stencil6<T>(w, d.wh[p - 9], d.wh[p + 9], d.wh[p - 3], d.wh[p + 3],
                               d.wh[p - 1], d.wh[p + 1], (T)0, (T)0, (T)0, (T)0, (T)0, (T)0);
  d.u[0][p] = gs_value<T>(st, b_at<T>(d, 1, 1, 1));
}

// u[buf] += P uc[cbuf] (trilinear).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong(const GridDescT<T>* __restrict__ list,
                                                    const int* __restrict__ active, int buf,
                                                    int cbuf, int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = interior_point(n - 2, blk);
  if (!p.ok) return;
  gview<T>(buf ? d.u[1] : d.u[0])[vidx(n, p.i, p.j, p.k)] +=
      prolong_at<T>(gview<T>(cbuf ? d.uc[1] : d.uc[0]), (n - 1) / 2 + 1, p.i, p.j, p.k);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_zero_u(const GridDescT<T>* __restrict__ list,
                                                   int count, int per) {
  // each plane as a flat range, 8 values per thread through a buffer
  // descriptor (positions past the plane are dropped); u[1] needs no
  // clearing: a level's first sweep writes all its interior points before any
  // read, and its boundary stays zero from allocation
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  const int n = d.n, sn2 = n * n;
  const int bpp = ceil_div(sn2, kBlock * 8);  // blocks per plane (offsets stay 32-bit)
  const int pl = blk / bpp, ch = blk - pl * bpp;
  const auto r = rsrc(d.u[0] + (size_t)pl * sn2, (uint32_t)(sn2 * sizeof(T)));
  const uint32_t base = ((uint32_t)ch * kBlock * 8u + threadIdx.x) * (uint32_t)sizeof(T);
#pragma unroll
  for (int e = 0; e < 8; ++e) bstore<T>(r, base + (uint32_t)(e * kBlock * sizeof(T)), (T)0);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy_buf(const GridDescT<T>* __restrict__ list,
                                                     const int* __restrict__ active, int from,
                                                     int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDescT<T> d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = full_point(n, blk);
  if (!p.ok) return;
  const int v = vidx(n, p.i, p.j, p.k);
  if (from) d.u[0][v] = d.u[1][v];
  else d.u[1][v] = d.u[0][v];
}

// ---- the small-grid V-cycle in LDS ---------------------------------------------
// One workgroup runs the whole remaining V-cycle of one grid of size NS
// (17, 9 or 5) and its coarser grids down to 3^3: every level's u, wh, b and
// r live in LDS (b of the top level is read from memory), so the cycle costs
// one launch instead of several per level.  Each step is the same update as
// the per-level kernels: red then black passes, residual, full weighting,
// exact 3^3 solve, trilinear correction.
constexpr int kSmallThreads = 1024;

template <int NS>
struct SmallGeo {
  static constexpr int J = NS == 17 ? 3 : NS == 9 ? 2 : 1;  // index of the 3^3 level
  __host__ __device__ static constexpr int n(int j) { return (NS - 1) / (1 << j) + 1; }
  __host__ __device__ static constexpr int vol(int j) { return n(j) * n(j) * n(j); }
  // level j holds u, wh, b (not on level 0: its b is read from memory) and
  // r (not on the coarsest level), in that order
  __host__ __device__ static constexpr int base(int j) {
    int o = 0;
    for (int q = 0; q < j; ++q) o += vol(q) * (2 + (q > 0 ? 1 : 0) + (q < J ? 1 : 0));
    return o;
  }
  __host__ __device__ static constexpr int off_u(int j) { return base(j); }
  __host__ __device__ static constexpr int off_w(int j) { return base(j) + vol(j); }
  __host__ __device__ static constexpr int off_b(int j) { return base(j) + 2 * vol(j); }
  __host__ __device__ static constexpr int off_r(int j) { return base(j) + (j > 0 ? 3 : 2) * vol(j); }
  static constexpr int total = base(J + 1);
};

template <int L>
using IC = std::integral_constant<int, L>;

// Item q of a pass over a level with m interior points per axis, dealt to the
// threads as q = t + r * kSmallThreads: the point (i, jj, k) of a colour pass
// of colour c (k > m: no point) and of a pass over every interior point.
template <int m>
__device__ __forceinline__ void vs_colour_point(int c, int q, int& i, int& jj, int& k) {
  constexpr int hk = (m + 1) / 2;
  i = q / (m * hk) + 1;
  const int rr = q % (m * hk);
  jj = rr / hk + 1;
  k = 2 - ((c + i + jj) & 1) + 2 * (rr % hk);
}
template <int m>
__device__ __forceinline__ void vs_point(int q, int& i, int& jj, int& k) {
  i = q / (m * m) + 1;
  const int rr = q % (m * m);
  jj = rr / m + 1;
  k = rr % m + 1;
}

template <typename T, int NS>
__global__ void __launch_bounds__(kSmallThreads) k_vsmall(const SmallChain<T>* __restrict__ chains,
                                                          const int* __restrict__ active,
                                                          int nu1, int nu2) {
  using Geo = SmallGeo<NS>;
  constexpr int J = Geo::J;
  __shared__ T lds[Geo::total];
  const SmallChain<T>& ch = chains[blockIdx.x];
  const GridDescT<T> top = ch.lv[0];
  if (!active[top.solve]) return;
  const int t = threadIdx.x;

  // The top level's right-hand side stays in memory (LDS holds u, wh and r of
  // every level): the values of this thread's points in the top level's
  // colour passes and residual pass are read once, here, into registers.
  constexpr int kM0 = NS - 2, kColQ = kM0 * kM0 * ((kM0 + 1) / 2), kResQ = kM0 * kM0 * kM0;
  constexpr int kColR = (kColQ + kSmallThreads - 1) / kSmallThreads;
  constexpr int kResR = (kResQ + kSmallThreads - 1) / kSmallThreads;
  T b0c[2][kColR], b0r[kResR];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int r = 0; r < kColR; ++r) {
      const int q = t + r * kSmallThreads;
      int i, jj, k;
      vs_colour_point<kM0>(c, q, i, jj, k);
      b0c[c][r] = 0;
      if (q < kColQ && k <= kM0) b0c[c][r] = b_at<T>(top, i, jj, k);
    }
  }
#pragma unroll
  for (int r = 0; r < kResR; ++r) {
    const int q = t + r * kSmallThreads;
    int i, jj, k;
    vs_point<kM0>(q, i, jj, k);
    b0r[r] = 0;
    if (q < kResQ) b0r[r] = b_at<T>(top, i, jj, k);
  }
  // load wh of every level and u of the top level; coarse u and every r = 0
  for (int j = 0; j <= J; ++j) {
    const int v = Geo::vol(j);
    const gptr<const T> w = gview<T>(ch.lv[j].wh);
    for (int q = t; q < v; q += kSmallThreads) {
      lds[Geo::off_w(j) + q] = w[q];
      lds[Geo::off_u(j) + q] = j == 0 ? gview<T>(top.u[0])[q] : (T)0;
      if (j < J) lds[Geo::off_r(j) + q] = 0;
    }
  }
  __syncthreads();

  // (every level's size is a compile-time constant below, so the index
  // arithmetic needs no division)
  // one colour pass on level L (in place), over the points of that colour only
  auto colour = [&](auto lvl, auto cc) {
    constexpr int Lv = decltype(lvl)::value, c = decltype(cc)::value;
    constexpr int n = Geo::n(Lv), m = n - 2, NQ = m * m * ((m + 1) / 2);
    T* u = lds + Geo::off_u(Lv);
    const T* w = lds + Geo::off_w(Lv);
#pragma unroll
    for (int r = 0; r < (NQ + kSmallThreads - 1) / kSmallThreads; ++r) {
      const int q = t + r * kSmallThreads;
      int i, jj, k;
      vs_colour_point<m>(c, q, i, jj, k);
      if (q < NQ && k <= m) {
        const int p = (i * n + jj) * n + k;
        T bv;
        if constexpr (Lv == 0) bv = b0c[c][r];
        else bv = lds[Geo::off_b(Lv) + p];
        u[p] = gs_value<T>(stencil_at<T>(u, w, p, n, n * n), bv);
      }
    }
    __syncthreads();
  };
  auto down = [&](auto lvl) {
    constexpr int Lv = decltype(lvl)::value, n = Geo::n(Lv), m = n - 2, NQ = m * m * m;
    for (int s = 0; s < nu1; ++s) {
      colour(lvl, IC<0>{});
      colour(lvl, IC<1>{});
    }
    // residual of this level, then full weighting into b of the next
    const T* u = lds + Geo::off_u(Lv);
    const T* w = lds + Geo::off_w(Lv);
    T* r = lds + Geo::off_r(Lv);
#pragma unroll
    for (int ri = 0; ri < (NQ + kSmallThreads - 1) / kSmallThreads; ++ri) {
      const int q = t + ri * kSmallThreads;
      int i, jj, k;
      vs_point<m>(q, i, jj, k);
      if (q < NQ) {
        const int p = (i * n + jj) * n + k;
        T bv;
        if constexpr (Lv == 0) bv = b0r[ri];
        else bv = lds[Geo::off_b(Lv) + p];
        r[p] = res_value<T>(stencil_at<T>(u, w, p, n, n * n), bv, u[p]);
      }
    }
    __syncthreads();
    constexpr int nc = Geo::n(Lv + 1), mc = nc - 2;
    T* bc = lds + Geo::off_b(Lv + 1);
    for (int q = t; q < mc * mc * mc; q += kSmallThreads) {
      const int I = q / (mc * mc) + 1, rr = q % (mc * mc), Jj = rr / mc + 1, K = rr % mc + 1;
      T acc = 0;
      for (int di = -1; di <= 1; ++di) {
        const T wi = di == 0 ? (T)1 : (T)0.5;
        for (int dj = -1; dj <= 1; ++dj) {
          const T wj = dj == 0 ? wi : (T)0.5 * wi;
          const int row = ((2 * I + di) * n + 2 * Jj + dj) * n + 2 * K;
          acc += wj * (r[row] + (T)0.5 * (r[row - 1] + r[row + 1]));
        }
      }
      bc[(I * nc + Jj) * nc + K] = (T)0.5 * acc;
    }
    __syncthreads();
  };
  auto up = [&](auto lvl) {
    constexpr int Lv = decltype(lvl)::value, n = Geo::n(Lv), m = n - 2, nc = Geo::n(Lv + 1);
    T* u = lds + Geo::off_u(Lv);
    const T* e = lds + Geo::off_u(Lv + 1);
    for (int q = t; q < m * m * m; q += kSmallThreads) {
      const int i = q / (m * m) + 1, rr = q % (m * m), jj = rr / m + 1, k = rr % m + 1;
      u[(i * n + jj) * n + k] += prolong_at<T>(e, nc, i, jj, k);
    }
    __syncthreads();
    for (int s = 0; s < nu2; ++s) {
      colour(lvl, IC<0>{});
      colour(lvl, IC<1>{});
    }
  };

  down(IC<0>{});
  if constexpr (J > 1) down(IC<1>{});
  if constexpr (J > 2) down(IC<2>{});
  // the 3^3 level: one unknown, solved exactly
  if (t == 0) {
    const T* w = lds + Geo::off_w(J);
    const St<T> st = stencil6<T>(w[13], w[4], w[22], w[10], w[16], w[12], w[14], (T)0, (T)0,
                                 (T)0, (T)0, (T)0, (T)0);
    lds[Geo::off_u(J) + 13] = gs_value<T>(st, lds[Geo::off_b(J) + 13]);
  }
  __syncthreads();
  if constexpr (J > 2) up(IC<2>{});
  if constexpr (J > 1) up(IC<1>{});
  up(IC<0>{});
  // the top level's iterate back to u[0]
  const gptr<T> uo = gview<T>(top.u[0]);
  constexpr int n = NS, m = n - 2;
  for (int q = t; q < m * m * m; q += kSmallThreads) {
    const int i = q / (m * m) + 1, rr = q % (m * m), jj = rr / m + 1, k = rr % m + 1;
    const int p = (i * n + jj) * n + k;
    uo[p] = lds[Geo::off_u(0) + p];
  }
}

// ---- reductions ---------------------------------------------------------------
// Per-block partial sums over interior vertices of: b'^2 (RED_BNORM),
// (b' - A'u)^2 (RED_RESID) or u (RED_QOI), blocks as in column marching.
// The decomposition depends only on the grid size, so a solve's sums never
// depend on the rest of the batch.
__global__ void __launch_bounds__(kBlock) k_reduce(const GridDesc* __restrict__ list,
                                                   const int* __restrict__ active, int buf,
                                                   int mode, double* __restrict__ partials,
                                                   const int* __restrict__ pend, int count,
                                                   int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDesc d = list[gi];
  if ((mode == RED_RESID || mode == RED_R2) && !active[d.solve]) return;
  if (mode == RED_QOI_PENDING && (!pend[d.solve] || active[d.solve])) return;
  const int n = d.n, sn2 = n * n;
  const Col c = column_of(n - 2, blk);
  const double* u = buf ? d.u[1] : d.u[0];
  double acc = 0.0;
  if (mode == RED_RESID) {
    tile_residual<double>(d, u, blk, [&](int, double r) { acc += r * r; });
  } else if (c.ok) {
    {
      int p = sn2 + c.j * n + c.k;
      for (int i = 1; i <= n - 2; ++i, p += sn2) {
        if (mode == RED_BNORM) {
          const double bp = b_at<double>(d, i, c.j, c.k);
          acc += bp * bp;
        } else if (mode == RED_R2) {
          acc += d.r[p] * d.r[p];
        } else {
          acc += u[p];
        }
      }
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[d.poff + blk] = acc;
}

// Mixed precision outer step: r = b' - A'u (FP64) -> inner rhs (FP32), inner
// iterate zeroed, partial sums of r^2.
__global__ void __launch_bounds__(kBlock) k_defect(const GridDesc* __restrict__ list,
                                                   const GridDesc32* __restrict__ list32,
                                                   const int* __restrict__ active,
                                                   double* __restrict__ partials, int count,
                                                   int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDesc d = list[gi];
  if (!active[d.solve]) return;
  const GridDesc32 e = list32[gi];
  const Col c = column_of(d.n - 2, blk);
  double acc = 0.0;
  const int n = d.n, sn2 = n * n;
  const uint32_t oc = (uint32_t)((c.j * n + c.k) * sizeof(float));
  const uint32_t pbytes = (uint32_t)(sn2 * sizeof(float));
  const uint32_t ocx = c.ok ? oc : kOut;
  tile_residual<double>(d, d.u[0], blk, [&](int i, double r) {
    acc += r * r;
    const bool ok = i <= n - 2;
    bstore<float>(rsrc(e.b + (size_t)(ok ? i : 0) * sn2, ok ? pbytes : 0u), ocx, (float)r);
    bstore<float>(rsrc(e.u[0] + (size_t)(ok ? i : 0) * sn2, ok ? pbytes : 0u), ocx, 0.0f);
  });
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[d.poff + blk] = acc;
}

__global__ void __launch_bounds__(kBlock) k_correct(const GridDesc* __restrict__ list,
                                                    const GridDesc32* __restrict__ list32,
                                                    const int* __restrict__ active, int buf32,
                                                    int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDesc d = list[gi];
  if (!active[d.solve]) return;
  const GridDesc32 e = list32[gi];
  const int n = d.n;
  const Pt p = interior_point(n - 2, blk);
  if (!p.ok) return;
  const int q = vidx(n, p.i, p.j, p.k);
  d.u[0][q] += (double)(buf32 ? e.u[1] : e.u[0])[q];
}

// Per-solve finalisation of the reductions.  RED_RESID runs once per outer
// step of each active solve: it credits the step's cycles to the solve and
// judges the iterate after ran - lag cycles (lag 1 when the residual belongs
// to the iterate of the previous outer step).
__global__ void __launch_bounds__(kBlock) k_finalize(const GridDesc* __restrict__ list,
                                                     SolveState s, int mode, int step,
                                                     int lag, int fixed_cycles, int max_cycles,
                                                     double tol, int sweep_parts,
                                                     int sweep_parts_red) {
  const GridDesc d = list[blockIdx.x];
  const int sv = d.solve;
  if (mode == RED_COUNT) {
    if (threadIdx.x != 0 || !s.active[sv]) return;
    const int ran = s.ran[sv] + step;
    s.ran[sv] = ran;
    if (ran >= fixed_cycles) {
      s.active[sv] = 0;
      s.cycles[sv] = ran;
    }
    return;
  }
  if (mode == RED_RESID && !s.active[sv]) return;
  if (mode == RED_QOI_PENDING && (!s.qpend[sv] || s.active[sv])) return;
  const bool sw = mode == RED_RESID && sweep_parts > 0;
  const double* src = sw ? s.spart + d.spoff : s.partials + d.poff;
  // in-sweep sums: the counts the two sweeps recorded after their partials
  const int P = sw ? (int)src[2 * kSweepParts] : reduce_blocks(d.n);
  double v = 0.0;
  for (int q = threadIdx.x; q < P; q += kBlock) v += src[q];
  if (sw) {
    const int P2 = (int)src[2 * kSweepParts + 1];
    for (int q = threadIdx.x; q < P2; q += kBlock) v += src[kSweepParts + q];
  }
  v = block_sum(v);
  if (threadIdx.x != 0) return;
  if (mode == RED_BNORM) {
    const double nb = sqrt(v);
    s.bnorm[sv] = nb > 0.0 ? nb : 1.0;
  } else if (mode == RED_RESID) {
    // (once per outer step of an active solve: credit the step's cycles)
    const int ran = s.ran[sv] + step;
    s.ran[sv] = ran;
    const int cycle = ran - lag;
    const double rho = sqrt(v) / s.bnorm[sv];
    s.relres[sv] = rho;
    if (cycle < 1) return;  // the initial iterate: convergence is judged after cycles
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
    if (mode == RED_QOI_PENDING) s.qpend[sv] = 0;
  }
}

__global__ void k_init_state(SolveState s, int ns, int qpend) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  s.active[t] = 1;
  s.cycles[t] = 0;
  s.ran[t] = 0;
  s.qpend[t] = qpend;
}

__global__ void k_admit(const int* __restrict__ solves, int count, SolveState s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int sv = solves[t];
  s.active[sv] = 1;
  s.cycles[sv] = 0;
  s.ran[sv] = 0;
  s.qpend[sv] = 1;
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

__global__ void k_fill(double* __restrict__ p, long count, double value) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

inline dim3 xcd_grid(int count, int per) { return dim3(8 * ceil_div(count * per, 8)); }

// Workgroups of a sweep launch: with automatic plane pieces (chunks 0) at
// least one round of the machine at the shape's occupancy (the kernel
// spreads them over the grids still active): 512 for tiles of which two
// workgroups fit a CU, 256 for the 16x64 tile, whose FP64 LDS leaves room
// for one; otherwise the count x tiles x pieces of the fixed split.
constexpr int sweep_min_units(int tj, int tk) {
  return 10 * (tj + 4) * (tk + 4) * (int)sizeof(double) > 80 * 1024 ? 256 : 512;
}
template <typename T, int TJ, int TK, bool CB, bool KL>
int sweep_launch_kl(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                    int cbuf, int chunks, hipStream_t st, T* spart, int norm) {
  const int tiles_k = (n - 1) / TK, tiles_j = (n - 1) / TJ;
  const int tiles = tiles_k * tiles_j;
  int units;
  if (chunks > 0) {
    const int chunk_len = ceil_div(n - 2, chunks);
    units = count * tiles * ceil_div(n - 2, chunk_len);
  } else {
    units = std::max(count * tiles, sweep_min_units(TJ, TK));
  }
  const int nwg = 8 * ceil_div(units, 8);
  const int per = nwg;  // (returned: an upper bound of the workgroups per grid)
  const dim3 grid(nwg), block(SweepGeom<TJ, TK>::THREADS);
  // KL: the mode table and the weights in dynamic LDS
  const size_t lds = KL ? sizeof(double) * (size_t)kl_lds_doubles(n) : 0;
  if (cbuf >= 0) {
    hipLaunchKernelGGL((k_sweep<T, TJ, TK, true, CB, KL>), grid, block, lds, st, d_list, d_active,
                       buf, cbuf, tiles_k, tiles, chunks, count, nwg);
  } else if (spart && norm == 1) {
    if constexpr (std::is_same<T, double>::value) {
      if constexpr (CB)
        hipLaunchKernelGGL((k_sweep_res_in_cb<T, TJ, TK, KL>), grid, block, lds, st, d_list,
                           d_active, buf, tiles_k, tiles, chunks, count, nwg, spart);
      else
        hipLaunchKernelGGL((k_sweep_res_in<T, TJ, TK, KL>), grid, block, lds, st, d_list,
                           d_active, buf, tiles_k, tiles, chunks, count, nwg, spart);
    }
  } else if (spart && norm == 2) {
    if constexpr (std::is_same<T, double>::value)
      hipLaunchKernelGGL((k_sweep_res_out<T, TJ, TK, CB, KL>), grid, block, lds, st, d_list,
                         d_active, buf, tiles_k, tiles, chunks, count, nwg, spart);
  } else {
    hipLaunchKernelGGL((k_sweep<T, TJ, TK, false, CB, KL>), grid, block, lds, st, d_list,
                       d_active, buf, cbuf, tiles_k, tiles, chunks, count, nwg);
  }
  return per;
}

// KL launches for FP64 grids with a constant right-hand side (the top grids
// of samples; with a full right-hand side the KL sweeps exceed the register
// budget of three waves per SIMD), on the shapes the larger grids use
template <typename T, int TJ, int TK, bool CB>
int sweep_launch(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                 int cbuf, int chunks, hipStream_t st, T* spart, int norm, bool kl) {
  if constexpr (std::is_same<T, double>::value && TJ * TK >= 256 && CB)
    if (kl && n <= kKLMaxN)
      return sweep_launch_kl<T, TJ, TK, CB, true>(d_list, count, n, d_active, buf, cbuf, chunks,
                                                  st, spart, norm);
  return sweep_launch_kl<T, TJ, TK, CB, false>(d_list, count, n, d_active, buf, cbuf, chunks, st,
                                               spart, norm);
}

}  // namespace

// the coefficient's exponential on the host (the kernels' code and table)
double kl_exp_host(double x) { return kl_exp(x, kExp2TabHost); }

// ---- tile shapes ------------------------------------------------------------
static const SweepShape kShapes[] = {
    {16, 64, 1}, {8, 64, 1},  {4, 64, 1}, {16, 32, 1}, {8, 32, 1}, {4, 32, 1}, {16, 16, 1},
    {8, 16, 1},  {4, 16, 1}, {8, 8, 1},   {4, 8, 1},  {4, 4, 1},  {2, 2, 1},
};

int sweep_shapes(int n, SweepShape* out, int max_out) {
  int c = 0;
  for (const SweepShape& s : kShapes)
    if (s.tj <= n - 1 && s.tk <= n - 1 && (n - 1) % s.tj == 0 && (n - 1) % s.tk == 0 && c < max_out)
      out[c++] = s;
  return c;
}

bool sweep_fits(int n, size_t elem) {
  // offsets up to kOut + (n + 6) planes must not wrap, and the array must end
  // below kOut so that kOut-based offsets stay out of range
  const uint64_t g = (uint64_t)n * n * n * elem, plane = (uint64_t)n * n * elem;
  return g < kOut && (uint64_t)kOut + (uint64_t)(n + 6) * plane < (1ull << 32);
}

SweepShape default_sweep_shape(int n, bool fused_correction, bool single) {
  // measured best on MI355X: 65^3 and 33^3 for a batch of 64 MLMC level pairs
  // (64 grids of 65^3, 128 of 33^3); 257^3 and 129^3 for batches of 16 and 48
  // grids; FP32 (the inner cycles of mixed precision) for 16 grids of 257^3
  // (the plane split is automatic where one piece per tile measured best
  // for those batches, so that small launches still get split).  From 65^3
  // up the 16x64 tile: its LDS leaves room for one workgroup (eleven waves)
  // per CU, and its rows of 68 values make fewer, longer runs of addresses
  // per plane than the two 16x32 workgroups it replaces; the sweeps are
  // bound by how well the memory serves that pattern (13% faster at 257^3)
  if (single) {
    if (n >= 257) return {16, 64, 0};
    if (n == 129) return {8, 64, 0};
    if (n == 65) return {16, 32, 0};
    if (n == 33) return fused_correction ? SweepShape{16, 32, 0} : SweepShape{16, 16, 0};
  } else {
    if (n >= 65) return {16, 64, 0};
    if (n == 33) return fused_correction ? SweepShape{8, 32, 0} : SweepShape{16, 16, 0};
  }
  if (n - 1 >= 16) return {8, 16, 0};
  if (n - 1 >= 8) return {8, 8, 0};
  if (n - 1 >= 4) return {4, 4, 0};
  return {2, 2, 0};
}

// ---- launchers ------------------------------------------------------------------
void launch_philox(const uint64_t* d_seeds, int count, int level, uint32_t* d_words,
                   double* d_normals, hipStream_t st, const int* d_levels) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_philox, dim3(count), dim3(64), 0, st, d_seeds, level, d_levels, d_words,
                     d_normals);
}

void launch_field(int n, int count, double* const* d_out, const int* d_xi_index,
                  const double* d_normals, const double* d_phi, const double* d_coef, int mode,
                  hipStream_t st) {
  if (count <= 0) return;
  if (n > kFieldMaxN) return;  // plans stop at 1025 vertices per axis
  const int per = ceil_div(n * n, kBlock);
  hipLaunchKernelGGL(k_field, xcd_grid(count, per), dim3(kBlock), 0, st, n, d_out, d_xi_index,
                     d_normals, d_phi, d_coef, mode, count, per);
}

void launch_inject(int nf, int count, const double* const* d_fine, double* const* d_coarse,
                   hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks((nf - 1) / 2 + 1);
  hipLaunchKernelGGL(k_inject, xcd_grid(count, per), dim3(kBlock), 0, st, nf, d_fine, d_coarse,
                     count, per);
}

void launch_to_float(int n, int count, const double* const* d_src, float* const* d_dst,
                     hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks(n);
  hipLaunchKernelGGL(k_to_float, xcd_grid(count, per), dim3(kBlock), 0, st, n, d_src, d_dst, count,
                     per);
}

void launch_fill(double* p, long count, double value, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, value);
}

void launch_prepare_problem(int n, const double* k, const double* f, double* wh, double* b,
                            double* u, hipStream_t st) {
  hipLaunchKernelGGL(k_prepare, dim3(point_blocks(n)), dim3(kBlock), 0, st, n, k, f, wh, b, u);
}

// Plane pieces of a sweep launch: the shape's, or automatic: split the plane
// march until the launch fills one round of the machine at the shape's
// occupancy (512 workgroups, two per CU, or 256 for the 16x64 tile; small
// batches and small grids are latency-bound by the sequential march),
// keeping at least four planes per piece.
// (automatic: as the kernel splits a launch of this many active grids)
static int sweep_chunks(int n, int count, SweepShape s) {
  if (s.chunks >= 1) return s.chunks;
  const int tiles = ((n - 1) / s.tj) * ((n - 1) / s.tk);
  const int nwg = 8 * ceil_div(std::max(count * tiles, sweep_min_units(s.tj, s.tk)), 8);
  return std::max(1, std::min(std::min(nwg / std::max(1, count * tiles), (n - 2) / 4),
                              kSweepParts / tiles));
}

int sweep_blocks(int n, int count, SweepShape s) {
  const int chunk_len = ceil_div(n - 2, sweep_chunks(n, count, s));
  return ((n - 1) / s.tj) * ((n - 1) / s.tk) * ceil_div(n - 2, chunk_len);
}

template <typename T>
int launch_sweep(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                 int cbuf, SweepShape s, hipStream_t st, T* spart, int norm, bool const_b,
                 bool kl) {
  if (count <= 0) return 0;
  const int c = s.chunks;  // 0: chosen in the kernel from the active grids
#define MG_SWEEP_CASE(TJ_, TK_)                                                              \
  if (s.tj == TJ_ && s.tk == TK_)                                                            \
    return const_b ? sweep_launch<T, TJ_, TK_, true>(d_list, count, n, d_active, buf, cbuf, c, \
                                                     st, spart, norm, kl)                   \
                   : sweep_launch<T, TJ_, TK_, false>(d_list, count, n, d_active, buf, cbuf,  \
                                                      c, st, spart, norm, kl);
  MG_SWEEP_CASE(16, 64)
  MG_SWEEP_CASE(8, 64)
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
  return 0;
}

template <typename T>
void launch_rbgs_colour(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                        int colour, int buf, hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks(n - 2);
  hipLaunchKernelGGL((k_rbgs_colour<T>), xcd_grid(count, per), dim3(kBlock), 0, st, d_list,
                     d_active, colour, buf, count, per);
}

template <typename T>
void launch_residual(const GridDescT<T>* d_list, int count, int n, const int* d_active, int buf,
                     hipStream_t st) {
  if (count <= 0) return;
  const int per = reduce_blocks(n);
  hipLaunchKernelGGL((k_residual<T>), xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     buf, count, per);
}

// coarse tile shapes of the one-pass transfer (grids from 65^3 up, smaller)
constexpr int kRRJ1 = 4, kRRK1 = 32, kRRJ2 = 8, kRRK2 = 16;
static int rr_tiles(int n) {
  const int m = (n - 1) / 2 - 1;
  return n >= 65 ? ceil_div(m, kRRJ1) * ceil_div(m, kRRK1) : ceil_div(m, kRRJ2) * ceil_div(m, kRRK2);
}
// pieces per tile: enough workgroups for two per CU, down to one coarse
// plane per piece for launches over few grids
int resrestrict_chunks(int n, int count) {
  const int m = (n - 1) / 2 - 1;
  return std::max(1, std::min(m, ceil_div(512, std::max(1, count) * rr_tiles(n))));
}

template <typename T>
void launch_resrestrict(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                        int buf, hipStream_t st, bool const_b, bool kl) {
  if (count <= 0) return;
  const int m = (n - 1) / 2 - 1;  // coarse interior points per axis
  const int ch = resrestrict_chunks(n, count), tiles = rr_tiles(n), per = tiles * ch;
  auto go = [&](auto cb, auto klc) {
    constexpr bool CB = decltype(cb)::value, KL = decltype(klc)::value;
    const size_t lds = KL ? sizeof(double) * (size_t)kl_lds_doubles(n) : 0;
    if (n >= 65) {
      const int tk = ceil_div(m, kRRK1);
      hipLaunchKernelGGL((k_resrestrict<T, kRRJ1, kRRK1, CB, KL>), xcd_grid(count, per),
                         dim3(RRGeom<kRRJ1, kRRK1>::THREADS), lds, st, d_list, d_active, buf, tk,
                         tiles, ch, count, per);
    } else {
      const int tk = ceil_div(m, kRRK2);
      hipLaunchKernelGGL((k_resrestrict<T, kRRJ2, kRRK2, CB, KL>), xcd_grid(count, per),
                         dim3(RRGeom<kRRJ2, kRRK2>::THREADS), lds, st, d_list, d_active, buf, tk,
                         tiles, ch, count, per);
    }
  };
  // KL launches for FP64 grids with a constant right-hand side (as the sweep)
  if constexpr (std::is_same<T, double>::value) {
    if (kl && const_b && n <= kKLMaxN) {
      go(std::true_type{}, std::true_type{});
      return;
    }
  }
  if (const_b)
    go(std::true_type{}, std::false_type{});
  else
    go(std::false_type{}, std::false_type{});
}

template <typename T>
void launch_restrict(const GridDescT<T>* d_list, int count, int n, const int* d_active,
                     hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks((n - 1) / 2 - 1);
  hipLaunchKernelGGL((k_restrict<T>), xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     count, per);
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
  const int per = point_blocks(n - 2);
  hipLaunchKernelGGL((k_prolong<T>), xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     buf, cbuf, count, per);
}

template <typename T>
void launch_zero_u(const GridDescT<T>* d_list, int count, int n, hipStream_t st) {
  if (count <= 0) return;
  const int per = n * ceil_div(n * n, kBlock * 8);
  hipLaunchKernelGGL((k_zero_u<T>), xcd_grid(count, per), dim3(kBlock), 0, st, d_list, count, per);
}

template <typename T>
void launch_copy_buf(const GridDescT<T>* d_list, int count, int n, const int* d_active, int from,
                     hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks(n);
  hipLaunchKernelGGL((k_copy_buf<T>), xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     from, count, per);
}

#define MG_INSTANTIATE(T)                                                                       \
  template int launch_sweep<T>(const GridDescT<T>*, int, int, const int*, int, int, SweepShape,  \
                               hipStream_t, T*, int, bool, bool);                               \
  template void launch_rbgs_colour<T>(const GridDescT<T>*, int, int, const int*, int, int,      \
                                      hipStream_t);                                             \
  template void launch_residual<T>(const GridDescT<T>*, int, int, const int*, int, hipStream_t); \
  template void launch_restrict<T>(const GridDescT<T>*, int, int, const int*, hipStream_t);      \
  template void launch_resrestrict<T>(const GridDescT<T>*, int, int, const int*, int, hipStream_t, \
                                      bool, bool);                                                \
  template void launch_coarsest<T>(const GridDescT<T>*, int, const int*, hipStream_t);           \
  template void launch_prolong<T>(const GridDescT<T>*, int, int, const int*, int, int,           \
                                  hipStream_t);                                                 \
  template void launch_zero_u<T>(const GridDescT<T>*, int, int, hipStream_t);                    \
  template void launch_copy_buf<T>(const GridDescT<T>*, int, int, const int*, int, hipStream_t);
MG_INSTANTIATE(double)
MG_INSTANTIATE(float)
#undef MG_INSTANTIATE

template <typename T>
void launch_vsmall(const SmallChain<T>* d_chains, int count, int ns, const int* d_active, int nu1,
                   int nu2, hipStream_t st) {
  if (count <= 0) return;
  if (ns == 17)
    hipLaunchKernelGGL((k_vsmall<T, 17>), dim3(count), dim3(kSmallThreads), 0, st, d_chains,
                       d_active, nu1, nu2);
  else if (ns == 9)
    hipLaunchKernelGGL((k_vsmall<T, 9>), dim3(count), dim3(kSmallThreads), 0, st, d_chains,
                       d_active, nu1, nu2);
  else if (ns == 5)
    hipLaunchKernelGGL((k_vsmall<T, 5>), dim3(count), dim3(kSmallThreads), 0, st, d_chains,
                       d_active, nu1, nu2);
}
template void launch_vsmall<double>(const SmallChain<double>*, int, int, const int*, int, int,
                                    hipStream_t);
template void launch_vsmall<float>(const SmallChain<float>*, int, int, const int*, int, int,
                                   hipStream_t);

void launch_reduce(const GridDesc* d_list, int count, int n, const int* d_active, int buf,
                   int mode, double* d_partials, hipStream_t st, const int* d_pend) {
  if (count <= 0) return;
  const int per = reduce_blocks(n);
  hipLaunchKernelGGL(k_reduce, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active, buf,
                     mode, d_partials, d_pend, count, per);
}

void launch_defect(const GridDesc* d_list, const GridDesc32* d_list32, int count, int n,
                   const int* d_active, double* d_partials, hipStream_t st) {
  if (count <= 0) return;
  const int per = reduce_blocks(n);
  hipLaunchKernelGGL(k_defect, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_list32,
                     d_active, d_partials, count, per);
}

void launch_correct(const GridDesc* d_list, const GridDesc32* d_list32, int count, int n,
                    const int* d_active, int buf32, hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks(n - 2);
  hipLaunchKernelGGL(k_correct, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_list32,
                     d_active, buf32, count, per);
}

void launch_finalize2(const GridDesc* d_list, int count, SolveState s, int mode, int step,
                      int lag, int fixed_cycles, int max_cycles, double tol, hipStream_t st,
                      int sweep_parts, int sweep_parts_red) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(kBlock), 0, st, d_list, s, mode, step, lag,
                     fixed_cycles, max_cycles, tol, sweep_parts, sweep_parts_red);
}

void launch_init_state2(SolveState s, int ns, hipStream_t st, int qpend) {
  hipLaunchKernelGGL(k_init_state, dim3((ns + 255) / 256), dim3(256), 0, st, s, ns, qpend);
}

void launch_admit(const int* d_solves, int count, SolveState s, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_admit, dim3((count + 255) / 256), dim3(256), 0, st, d_solves, count, s);
}

// QoIs of Section 3 besides the integral, on the top grids (u[0]), one
// workgroup per grid.  Mode QOI_POINT: u at the vertex x* = (1/4, 1/4, 1/4),
// index (n-1)/4 on every axis.  Mode QOI_FLUX: the flux of -k grad u in +x_2
// (the j direction) across the vertex plane j* = (n-1)/4, as the mean of the
// face planes j* -+ 1/2, each h * sum over interior (i, k) of
// c (u_a - u_(a+1)) with the operator's face coefficient c = 1/(wh_a + wh_(a+1)).
// Boundary values of u are stored zeros.  Each thread sums a fixed stride of
// the (i, k) points, then a fixed tree over the workgroup: the result does
// not depend on the rest of the batch.
__global__ void __launch_bounds__(kBlock) k_qoi_pf(const GridDesc* __restrict__ list, int mode,
                                                   double* __restrict__ q) {
  const GridDesc d = list[blockIdx.x];
  const int n = d.n, c = (n - 1) / 4, m = n - 2;
  if (mode == QOI_POINT) {
    if (threadIdx.x == 0) q[d.solve] = d.u[0][((size_t)c * n + c) * n + c];
    return;
  }
  const double h = 1.0 / (double)(n - 1);
  double sm = 0.0, sp = 0.0;
  for (int e = threadIdx.x; e < m * m; e += kBlock) {
    const int i = 1 + e / m, k = 1 + e - (e / m) * m;
    const size_t p1 = ((size_t)i * n + c) * n + k, p0 = p1 - n, p2 = p1 + n;
    const double u0 = d.u[0][p0], u1 = d.u[0][p1], u2 = d.u[0][p2];
    const double w0 = d.wh[p0], w1 = d.wh[p1], w2 = d.wh[p2];
    sm += (u0 - u1) / (w0 + w1);
    sp += (u1 - u2) / (w1 + w2);
  }
  sm = block_sum(sm);
  sp = block_sum(sp);
  if (threadIdx.x == 0) q[d.solve] = 0.5 * (h * sm + h * sp);
}

// ---- P1 finite elements on the Kuhn tetrahedra (Section 3.1) -----------------
// The P1 operator of the vertex grid's Kuhn triangulation (each cell split
// into the six tetrahedra x_a >= x_b >= x_c, one per ordering of the axes),
// each tetrahedron's coefficient the mean of its four vertex values, couples
// axis neighbours only: in a Kuhn tetrahedron the barycentric gradients are
// orthogonal across its diagonal edges.  An axis edge p -- p + e_d lies in six
// of the tetrahedra; its coupling, scaled by 1/h like the FD form, is the sum
// of their four-vertex means over 6:
//   c_d(p) = [6 (k_p + k_(p+e_d)) + 2 (k_(p+e_d+e_a) + k_(p+e_d+e_b)
//            + k_(p+e_d+e_a+e_b) + k_(p-e_a) + k_(p-e_b) + k_(p-e_a-e_b))] / 24
// with a, b the other two axes.  The stencil of an interior vertex then has
// the FD form with these six faces (red-black colouring stays exact).
__global__ void __launch_bounds__(kBlock) k_fe_faces(int n, const double* const* __restrict__ wh_l,
                                                     double* const* __restrict__ fc_l, int count,
                                                     int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const Pt p = full_point(n, blk);
  if (!p.ok) return;
  const int i = p.i, j = p.j, k = p.k;
  const double* w = wh_l[gi];
  double* fc = fc_l[gi];
  const int sn2 = n * n;
  const size_t N = (size_t)sn2 * n;
  const int v = (i * n + j) * n + k;
  const int step[3] = {sn2, n, 1};
  const int c[3] = {i, j, k};
  auto kv = [&](int q) { return 0.5 / w[q]; };
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    const int a = dd == 0 ? 1 : 0, b = dd == 2 ? 1 : 2;
    const bool ok = c[dd] <= n - 2 && c[a] >= 1 && c[a] <= n - 2 && c[b] >= 1 && c[b] <= n - 2;
    double val = 0.0;
    if (ok) {
      const int sd = step[dd], sa = step[a], sb = step[b];
      const double s6 = kv(v) + kv(v + sd);
      const double s2 = ((kv(v + sd + sa) + kv(v + sd + sb)) + kv(v + sd + sa + sb)) +
                        ((kv(v - sa) + kv(v - sb)) + kv(v - sa - sb));
      val = (6.0 * s6 + 2.0 * s2) / 24.0;
    }
    fc[dd * N + v] = val;
  }
}

// The six faces of interior vertex v from fc (at v and at v - e_d).
__device__ __forceinline__ St<double> fe_stencil_at(const double* fc, const double* u, int v, int n,
                                                    size_t N) {
  const int sj = n, si = n * n;
  return stencil_faces<double>(fc[v - si], fc[v], fc[N + v - sj], fc[N + v], fc[2 * N + v - 1],
                               fc[2 * N + v], u[v - si], u[v + si], u[v - sj], u[v + sj],
                               u[v - 1], u[v + 1]);
}

// Point kernels over flat vertex indices v = (i n + j) n + k: consecutive
// lanes on consecutive addresses, rows and planes run on without gaps.  On a
// grid with an odd n, i + j + k and v have the same parity (n and n^2 are
// odd), so the vertices of colour c are exactly v = 2t + c: a colour pass
// gives every thread one vertex of its colour.
__device__ __forceinline__ Pt flat_point(int v, int nt) {
  const int n2 = nt * nt;
  Pt p;
  p.i = v / n2;
  const int r = v - p.i * n2;
  p.j = r / nt;
  p.k = r - p.j * nt;
  p.ok = v < n2 * nt;
  return p;
}
__device__ __forceinline__ bool interior(int n, const Pt& p) {
  return p.i >= 1 && p.j >= 1 && p.k >= 1 && p.i <= n - 2 && p.j <= n - 2 && p.k <= n - 2;
}

__global__ void __launch_bounds__(kBlock) k_fe_colour(const GridDesc* __restrict__ list,
                                                      const int* __restrict__ active, int colour,
                                                      int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDesc d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n;
  const int t = blk * kBlock + (int)threadIdx.x;
  const Pt p = flat_point((n & 1) ? 2 * t + colour : t, n);
  if (!p.ok || !interior(n, p) || ((p.i + p.j + p.k) & 1) != colour) return;
  const int v = vidx(n, p.i, p.j, p.k);
  double* u = d.u[0];
  const St<double> st = fe_stencil_at(d.fc, u, v, n, (size_t)n * n * n);
  u[v] = gs_value<double>(st, b_at<double>(d, p.i, p.j, p.k));
}

__global__ void __launch_bounds__(kBlock) k_fe_residual(const GridDesc* __restrict__ list,
                                                        const int* __restrict__ active, int count,
                                                        int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const GridDesc d = list[gi];
  if (!active[d.solve]) return;
  const int n = d.n;
  const Pt p = flat_point(blk * kBlock + (int)threadIdx.x, n);
  if (!p.ok || !interior(n, p)) return;
  const int v = vidx(n, p.i, p.j, p.k);
  const St<double> st = fe_stencil_at(d.fc, d.u[0], v, n, (size_t)n * n * n);
  d.r[v] = res_value<double>(st, b_at<double>(d, p.i, p.j, p.k), d.u[0][v]);
}

__global__ void k_fe_coarsest(const GridDesc* __restrict__ list, int count,
                              const int* __restrict__ active) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  const GridDesc d = list[g];
  if (!active[d.solve]) return;
  const double zero[27] = {};
  const St<double> st = fe_stencil_at(d.fc, zero, 13, 3, 27);
  d.u[0][13] = gs_value<double>(st, b_at<double>(d, 1, 1, 1));
}

void launch_fe_faces(int n, int count, const double* const* d_wh, double* const* d_fc,
                     hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks(n);
  hipLaunchKernelGGL(k_fe_faces, xcd_grid(count, per), dim3(kBlock), 0, st, n, d_wh, d_fc, count,
                     per);
}

void launch_fe_colour(const GridDesc* d_list, int count, int n, const int* d_active, int colour,
                      hipStream_t st) {
  if (count <= 0) return;
  const long N = (long)n * n * n;
  const int per = (int)ceil_div_l((n & 1) ? (N + 1) / 2 : N, kBlock);
  hipLaunchKernelGGL(k_fe_colour, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     colour, count, per);
}

void launch_fe_residual(const GridDesc* d_list, int count, int n, const int* d_active,
                        hipStream_t st) {
  if (count <= 0) return;
  const int per = (int)ceil_div_l((long)n * n * n, kBlock);
  hipLaunchKernelGGL(k_fe_residual, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     count, per);
}

void launch_fe_coarsest(const GridDesc* d_list, int count, const int* d_active, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fe_coarsest, dim3((count + 63) / 64), dim3(64), 0, st, d_list, count,
                     d_active);
}

// ---- SPDE field sampler (Section 3.2, eq. spde) --------------------------------
// (kappa^2 - Laplace) Z = W on the box (-1,2)^3, natural Neumann boundary,
// lumped-mass P1 elements on the Kuhn tetrahedra of the box grid, scaled by
// 1/h: (K' + kappa^2 h^2 diag(m)) Z = sqrt(h m) xi.  With unit coefficient the
// element couplings count tetrahedra: an axis edge p -- p + e_d lies in the
// four cells p - s_a e_a - s_b e_b (s_a, s_b in {0, 1}; a, b the other axes),
// which hold 2 Kuhn tetrahedra containing it when s_a == s_b and 1 otherwise,
// each adding 1/6; a cell outside the box adds nothing.  The lumped mass of p
// (in units of h^3) is 1/24 times, over the cells at p, 6 where p is the
// cell's (0,0,0) or (1,1,1) corner (all six tetrahedra) and 2 at the other
// corners.
__device__ __forceinline__ bool spde_cell(int nt, int a, int b, int c) {
  return a >= 0 && b >= 0 && c >= 0 && a <= nt - 2 && b <= nt - 2 && c <= nt - 2;
}
__device__ __forceinline__ double spde_mass(int nt, int i, int j, int k) {
  int w = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int di = q >> 2, dj = (q >> 1) & 1, dk = q & 1;
    if (spde_cell(nt, i - di, j - dj, k - dk)) w += (di == dj && dj == dk) ? 6 : 2;
  }
  return (double)w / 24.0;
}
// coupling of p = (i, j, k) to p + e_d (0 if that edge leaves the box)
__device__ __forceinline__ double spde_coupling(int nt, int i, int j, int k, int d) {
  const int p[3] = {i, j, k};
  if (p[d] < 0 || p[d] > nt - 2) return 0.0;
  const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
  int w = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int sa = q >> 1, sb = q & 1;
    int c[3] = {i, j, k};
    c[a] -= sa;
    c[b] -= sb;
    if (spde_cell(nt, c[0], c[1], c[2])) w += sa == sb ? 2 : 1;
  }
  return (double)w / 6.0;
}
// D + kappa^2 h^2 m and S = sum of couplings times neighbour values at p.
// Off the box's boundary planes every coupling is 1 (4 cells, 6 tetrahedra)
// and the mass 1, so there D = 6 and S is the plain neighbour sum, formed in
// the order the general sum takes (a unit-coupling FMA is the addition), so
// both paths give the same bits.
__device__ __forceinline__ bool spde_interior(int nt, int i, int j, int k) {
  return i >= 1 && j >= 1 && k >= 1 && i <= nt - 2 && j <= nt - 2 && k <= nt - 2;
}
__device__ __forceinline__ St<double> spde_stencil(const double* z, int nt, int i, int j, int k) {
  const int si = nt * nt, sj = nt, v = (i * nt + j) * nt + k;
  if (spde_interior(nt, i, j, k)) {
    St<double> s;
    s.D = 6.0;
    double S = z[v - si];
    S += z[v + si];
    S += z[v - sj];
    S += z[v + sj];
    S += z[v - 1];
    s.S = S + z[v + 1];
    return s;
  }
  const double a0 = i >= 1 ? spde_coupling(nt, i - 1, j, k, 0) : 0.0;
  const double a1 = spde_coupling(nt, i, j, k, 0);
  const double a2 = j >= 1 ? spde_coupling(nt, i, j - 1, k, 1) : 0.0;
  const double a3 = spde_coupling(nt, i, j, k, 1);
  const double a4 = k >= 1 ? spde_coupling(nt, i, j, k - 1, 2) : 0.0;
  const double a5 = spde_coupling(nt, i, j, k, 2);
  // neighbours outside the box have coupling 0: read p itself there
  return stencil_faces<double>(a0, a1, a2, a3, a4, a5, z[i >= 1 ? v - si : v],
                               z[i <= nt - 2 ? v + si : v], z[j >= 1 ? v - sj : v],
                               z[j <= nt - 2 ? v + sj : v], z[k >= 1 ? v - 1 : v],
                               z[k <= nt - 2 ? v + 1 : v]);
}

__global__ void __launch_bounds__(kBlock) k_spde_noise(const SpdeGrid* __restrict__ list,
                                                       const uint64_t* __restrict__ seeds,
                                                       const int* __restrict__ levels, int nt,
                                                       double h, int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const long N = (long)nt * nt * nt;
  const long jb = (long)blk * kBlock + threadIdx.x;
  if (2 * jb >= N) return;
  const SpdeGrid g = list[gi];
  const uint64_t seed = seeds[gi];
  uint32_t c[4] = {(uint32_t)jb, (uint32_t)levels[gi], 1u, 0u};
  philox_block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t M0 = ((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6);
  const uint64_t M1 = ((uint64_t)(c[2] >> 5) << 26) | (uint64_t)(c[3] >> 6);
  const double U0 = (double)(M0 + 1) * 0x1p-53, U1 = (double)(M1 + 1) * 0x1p-53;
  const double R = sqrt(-2.0 * log(U0)), ang = 6.283185307179586 * U1;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const long p = 2 * jb + e;
    if (p >= N) break;
    const int k = (int)(p % nt), j = (int)((p / nt) % nt), i = (int)(p / ((long)nt * nt));
    const double xi = e == 0 ? R * cos(ang) : R * sin(ang);
    g.b[p] = sqrt(h * spde_mass(nt, i, j, k)) * xi;
  }
}

// (the box kernels map threads by flat_point, as the finite-element passes)
__global__ void __launch_bounds__(kBlock) k_spde_colour(const SpdeGrid* __restrict__ list,
                                                        const int* __restrict__ active, int colour,
                                                        int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const SpdeGrid g = list[gi];
  if (!active[g.solve]) return;
  const int nt = g.nt;
  const int t = blk * kBlock + (int)threadIdx.x;
  const bool odd = nt & 1;
  const Pt p = flat_point(odd ? 2 * t + colour : t, nt);
  if (!p.ok || ((p.i + p.j + p.k) & 1) != colour) return;
  const int v = (p.i * nt + p.j) * nt + p.k;
  const St<double> st = spde_stencil(g.z, nt, p.i, p.j, p.k);
  const double m = spde_interior(nt, p.i, p.j, p.k) ? 1.0 : spde_mass(nt, p.i, p.j, p.k);
  g.z[v] = (g.b[v] + st.S) / (st.D + g.k2h2 * m);
}

__global__ void __launch_bounds__(kBlock) k_spde_residual(const SpdeGrid* __restrict__ list,
                                                          const int* __restrict__ active,
                                                          int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const SpdeGrid g = list[gi];
  if (!active[g.solve]) return;
  const int nt = g.nt;
  const Pt p = flat_point(blk * kBlock + (int)threadIdx.x, nt);
  if (!p.ok) return;
  const int v = (p.i * nt + p.j) * nt + p.k;
  const St<double> st = spde_stencil(g.z, nt, p.i, p.j, p.k);
  const double m = spde_interior(nt, p.i, p.j, p.k) ? 1.0 : spde_mass(nt, p.i, p.j, p.k);
  const double diag = st.D + g.k2h2 * m;
  g.r[v] = g.b[v] - (diag * g.z[v] - st.S);
}

// over the coarse vertices: bc = P^T src / 2 (src = r, or b with from_b), zc = 0
__global__ void __launch_bounds__(kBlock) k_spde_restrict(const SpdeGrid* __restrict__ list,
                                                          const int* __restrict__ active,
                                                          int from_b, int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const SpdeGrid g = list[gi];
  if (!active[g.solve]) return;
  const int nt = g.nt, ntc = (nt - 1) / 2 + 1;
  const Pt p = flat_point(blk * kBlock + (int)threadIdx.x, ntc);
  if (!p.ok) return;
  const double* src = from_b ? g.b : g.r;
  double sum = 0.0;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj)
      for (int dk = -1; dk <= 1; ++dk) {
        const int i = 2 * p.i + di, j = 2 * p.j + dj, k = 2 * p.k + dk;
        if (i < 0 || j < 0 || k < 0 || i >= nt || j >= nt || k >= nt) continue;
        const double w = (di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * (dk ? 0.5 : 1.0);
        sum += w * src[(i * nt + j) * nt + k];
      }
  const int vc = (p.i * ntc + p.j) * ntc + p.k;
  g.bc[vc] = 0.5 * sum;
  g.zc[vc] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_spde_prolong(const SpdeGrid* __restrict__ list,
                                                         const int* __restrict__ active, int count,
                                                         int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const SpdeGrid g = list[gi];
  if (!active[g.solve]) return;
  const int nt = g.nt, ntc = (nt - 1) / 2 + 1;
  const Pt p = flat_point(blk * kBlock + (int)threadIdx.x, nt);
  if (!p.ok) return;
  // the coarse vertices at the corners of the fine vertex's coarse cell
  // face (one to eight of them, weight 2^-(odd coordinates) each), summed in
  // the order a, b, c; the loops are unrolled over the eight corners with
  // the absent ones skipped, so the sum takes the same operations
  const int oi = p.i & 1, oj = p.j & 1, ok = p.k & 1;
  const double w = (oi ? 0.5 : 1.0) * (oj ? 0.5 : 1.0) * (ok ? 0.5 : 1.0);
  const double* zc = g.zc + ((p.i >> 1) * ntc + (p.j >> 1)) * ntc + (p.k >> 1);
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q >> 2, b = (q >> 1) & 1, c = q & 1;
    if (a <= oi && b <= oj && c <= ok) sum += w * zc[(a * ntc + b) * ntc + c];
  }
  g.z[(p.i * nt + p.j) * nt + p.k] += sum;
}

// the coarsest grid (64 vertices for these boxes): 32 red-black sweeps in LDS
__global__ void __launch_bounds__(64) k_spde_coarsest(const SpdeGrid* __restrict__ list,
                                                      const int* __restrict__ active) {
  const SpdeGrid g = list[blockIdx.x];
  if (!active[g.solve]) return;
  const int nt = g.nt, N = nt * nt * nt, t = threadIdx.x;
  __shared__ double z[64];
  const bool own = t < N;
  if (own) z[t] = g.z[t];
  __syncthreads();
  const int i = t / (nt * nt), j = (t / nt) % nt, k = t % nt;
  for (int s = 0; s < 32; ++s)
    for (int colour = 0; colour < 2; ++colour) {
      if (own && ((i + j + k) & 1) == colour) {
        const St<double> st = spde_stencil(z, nt, i, j, k);
        z[t] = (g.b[t] + st.S) / (st.D + g.k2h2 * spde_mass(nt, i, j, k));
      }
      __syncthreads();
    }
  if (own) g.z[t] = z[t];
}

int spde_blocks(int nt) {
  const long N = (long)nt * nt * nt;
  return (int)std::min<long>(256, std::max<long>(1, (N + 4095) / 4096));
}

// a fixed contiguous range of the grid per workgroup, fixed order inside
__global__ void __launch_bounds__(kBlock) k_spde_sumsq(const SpdeGrid* __restrict__ list,
                                                       const int* __restrict__ active, int which,
                                                       double* __restrict__ partials, int count,
                                                       int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const SpdeGrid g = list[gi];
  if (!active[g.solve]) return;
  const long N = (long)g.nt * g.nt * g.nt;
  const long chunk = (N + per - 1) / per;
  const long lo = (long)blk * chunk, hi = std::min<long>(N, lo + chunk);
  const double* x = which ? g.b : g.r;
  double acc = 0.0;
  for (long p = lo + threadIdx.x; p < hi; p += kBlock) acc += x[p] * x[p];
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[(size_t)gi * per + blk] = acc;
}

__global__ void __launch_bounds__(kBlock) k_spde_judge(const SpdeGrid* __restrict__ list,
                                                       int* __restrict__ active,
                                                       int* __restrict__ cycles,
                                                       double* __restrict__ bnorm,
                                                       const double* __restrict__ partials,
                                                       int per, int cycle, double tol,
                                                       int max_cycles, int bnorm_mode) {
  const int gi = blockIdx.x;
  const int sv = list[gi].solve;
  if (!active[sv]) return;
  double v = 0.0;
  for (int q = threadIdx.x; q < per; q += kBlock) v += partials[(size_t)gi * per + q];
  v = block_sum(v);
  if (threadIdx.x != 0) return;
  if (bnorm_mode) {
    bnorm[sv] = v > 0.0 ? sqrt(v) : 1.0;
    return;
  }
  const double rho = sqrt(v) / bnorm[sv];
  if (rho <= tol) {
    active[sv] = 0;
    cycles[sv] = cycle;
  } else if (cycle >= max_cycles) {
    active[sv] = 0;
    cycles[sv] = -1;
  }
}

__global__ void __launch_bounds__(kBlock) k_spde_field(const SpdeGrid* __restrict__ list, int n,
                                                       double s, double* const* __restrict__ whl,
                                                       int mode, int count, int per) {
  int gi, blk;
  if (!xcd_unit(count, per, gi, blk)) return;
  const Pt p = full_point(n, blk);
  if (!p.ok) return;
  const SpdeGrid g = list[gi];
  const int nt = g.nt, o = n - 1;
  const double z = g.z[((p.i + o) * nt + p.j + o) * nt + p.k + o];
  whl[gi][(p.i * n + p.j) * n + p.k] = mode ? exp(s * z) : 0.5 * exp(-s * z);
}

void launch_spde_noise(const SpdeGrid* d_list, int count, int nt, const uint64_t* d_seeds,
                       const int* d_levels, double h, hipStream_t st) {
  if (count <= 0) return;
  const long N = (long)nt * nt * nt;
  const int per = (int)(((N + 1) / 2 + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_spde_noise, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_seeds,
                     d_levels, nt, h, count, per);
}
void launch_spde_colour(const SpdeGrid* d_list, int count, int nt, const int* d_active, int colour,
                        hipStream_t st) {
  if (count <= 0) return;
  const long N = (long)nt * nt * nt;
  const int per = (int)ceil_div_l((nt & 1) ? (N + 1) / 2 : N, kBlock);
  hipLaunchKernelGGL(k_spde_colour, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     colour, count, per);
}
void launch_spde_residual(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                          hipStream_t st) {
  if (count <= 0) return;
  const int per = (int)ceil_div_l((long)nt * nt * nt, kBlock);
  hipLaunchKernelGGL(k_spde_residual, xcd_grid(count, per), dim3(kBlock), 0, st, d_list,
                     d_active, count, per);
}
void launch_spde_restrict(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                          bool from_b, hipStream_t st) {
  if (count <= 0) return;
  const long ntc = (nt - 1) / 2 + 1;
  const int per = (int)ceil_div_l(ntc * ntc * ntc, kBlock);
  hipLaunchKernelGGL(k_spde_restrict, xcd_grid(count, per), dim3(kBlock), 0, st, d_list,
                     d_active, from_b ? 1 : 0, count, per);
}
void launch_spde_prolong(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                         hipStream_t st) {
  if (count <= 0) return;
  const int per = (int)ceil_div_l((long)nt * nt * nt, kBlock);
  hipLaunchKernelGGL(k_spde_prolong, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     count, per);
}
void launch_spde_coarsest(const SpdeGrid* d_list, int count, int nt, const int* d_active,
                          hipStream_t st) {
  if (count <= 0 || nt * nt * nt > 64) return;
  hipLaunchKernelGGL(k_spde_coarsest, dim3(count), dim3(64), 0, st, d_list, d_active);
}
void launch_spde_sumsq(const SpdeGrid* d_list, int count, int nt, const int* d_active, int which,
                       double* d_partials, hipStream_t st) {
  if (count <= 0) return;
  const int per = spde_blocks(nt);
  hipLaunchKernelGGL(k_spde_sumsq, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, d_active,
                     which, d_partials, count, per);
}
void launch_spde_judge(const SpdeGrid* d_list, int count, int nt, int* d_active, int* d_cycles,
                       double* d_bnorm, const double* d_partials, int cycle, double tol,
                       int max_cycles, int bnorm_mode, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_spde_judge, dim3(count), dim3(kBlock), 0, st, d_list, d_active, d_cycles,
                     d_bnorm, d_partials, spde_blocks(nt), cycle, tol, max_cycles, bnorm_mode);
}
void launch_spde_field(const SpdeGrid* d_list, int count, int n, double s, double* const* d_wh,
                       int mode, hipStream_t st) {
  if (count <= 0) return;
  const int per = point_blocks(n);
  hipLaunchKernelGGL(k_spde_field, xcd_grid(count, per), dim3(kBlock), 0, st, d_list, n, s, d_wh,
                     mode, count, per);
}

// Y = Q_f - Q_c from two batches' per-solve QoIs (solve t of each is sample
// t; qc == nullptr: level 0), with the cycle counts of both solves, written
// at output position pos[t].
__global__ void k_ydiff2(const double* __restrict__ qf, const double* __restrict__ qc,
                         const int* __restrict__ pos, int count, double* __restrict__ y,
                         double* __restrict__ qfo, double* __restrict__ qco, int cyc_f, int cyc_c,
                         int* __restrict__ cyc_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const double a = qf[t], b = qc ? qc[t] : 0.0;
  const int o = pos[t];
  y[o] = a - b;
  if (qfo) qfo[o] = a;
  if (qco) qco[o] = b;
  if (cyc_out) {
    cyc_out[2 * o] = cyc_f;
    cyc_out[2 * o + 1] = qc ? cyc_c : 0;
  }
}

void launch_qoi_pf(const GridDesc* d_list, int count, int mode, double* d_q, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_qoi_pf, dim3(count), dim3(kBlock), 0, st, d_list, mode, d_q);
}

void launch_ydiff2(const double* d_qf, const double* d_qc, int count, const int* d_pos,
                   double* d_y, double* d_qf_out, double* d_qc_out, int cyc_f, int cyc_c,
                   int* d_cycles_out, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ydiff2, dim3((count + 255) / 256), dim3(256), 0, st, d_qf, d_qc, d_pos,
                     count, d_y, d_qf_out, d_qc_out, cyc_f, cyc_c, d_cycles_out);
}

void launch_ydiff(const double* d_q, const int* d_fi, const int* d_ci, int count, double* d_y,
                  double* d_qf, double* d_qc, const int* d_cycles, int* d_cycles_out,
                  hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_ydiff, dim3((count + 255) / 256), dim3(256), 0, st, d_q, d_fi, d_ci, count,
                     d_y, d_qf, d_qc, d_cycles, d_cycles_out);
}

}  // namespace mg
