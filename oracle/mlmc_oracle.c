/*
 * Plain FP64 CPU oracle for the per-sample hot path of multilevel Monte
 * Carlo, arXiv 1607.03252 (Gmeiner, Drzisga, Ruede, Scheichl, Wohlmuth).
 *
 * TEST INFRASTRUCTURE ONLY: slow and obviously correct, loaded only by the
 * test suite, the smoke check and the benchmark's CPU-baseline leg.  Built
 * with gcc -O2 -ffp-contract=off (no fast-math, no FMA contraction).
 *
 * What each function follows:
 *   - MLMC sample Y_l = Q_l - Q_{l-1} on one shared omega, Y_0 = Q_0:
 *     Section 2.2, eq. (MLMC_defn) and Algorithm 1 (steps 1.a.i-ii).
 *   - Model problem -div(k grad u) = f on D = (0,1)^3, u = 0 on the
 *     boundary, f deterministic (f = 1 in Section 7): Section 3, eq. (modweak).
 *   - k = exp(Z), Z Gaussian with exponential covariance sigma^2, lambda;
 *     Karhunen-Loeve expansion named as one way to sample Z: Section 3.2,
 *     eq. (def:expcov).  Here the separable (product of 1D exponentials)
 *     covariance truncated to the 4x4x4 block of 1D modes.
 *   - Multigrid V-cycles with pre- and post-smoothing: Section 7.1 (the
 *     paper uses FMG-2V(4,4)); here V(nu1,nu2) with red-black Gauss-Seidel
 *     to a relative residual tolerance.
 *   - Level statistics with divisor N: Section 2.3 (the estimator s_l^2).
 *
 * Readings where the paper is silent (all also listed in the design notes):
 * 7-point finite differences with harmonic-mean face coefficients, scaled by
 * h^2; coarse operators rediscretised with injected k; coarsest grid 3^3;
 * Philox4x32-10 with key = seed and counter = (block, level, 0, 0);
 * QoI = integral of u (trapezoidal, = h^3 * sum over interior vertices).
 */
#include "mlmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(n, i, j, k) ((((size_t)(i)) * (size_t)(n) + (size_t)(j)) * (size_t)(n) + (size_t)(k))

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers.                                             */
/* Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11):      */
/* multipliers 0xD2511F53, 0xCD9E8D57; key increments (Weyl) 0x9E3779B9,     */
/* 0xBB67AE85; ten rounds, the key bumped between rounds.                    */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One omega per (seed, level): the two solves of a sample Y_l share it
 * (Section 2.2), different levels draw independent numbers (Section 2.2,
 * "independent samples across all levels"). */
void or_philox_words(uint64_t seed, uint32_t level, uint32_t out[128]) {
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  for (uint32_t j = 0; j < 32; ++j) {
    uint32_t ctr[4] = {j, level, 0u, 0u};
    or_philox4x32_10(ctr, key, out + 4 * j);
  }
}

void or_uniform_ints(uint64_t seed, uint32_t level, uint64_t out[64]) {
  uint32_t w[128];
  or_philox_words(seed, level, w);
  for (int m = 0; m < 64; ++m) {
    uint64_t hi = (uint64_t)(w[2 * m] >> 5);     /* 27 bits */
    uint64_t lo = (uint64_t)(w[2 * m + 1] >> 6); /* 26 bits */
    out[m] = hi * 67108864ull + lo;              /* hi * 2^26 + lo < 2^53 */
  }
}

void or_gaussians(uint64_t seed, uint32_t level, double xi[64]) {
  uint64_t M[64];
  double U[64];
  or_uniform_ints(seed, level, M);
  for (int m = 0; m < 64; ++m) U[m] = ((double)M[m] + 1.0) * 0x1p-53; /* (0,1] exact */
  const double two_pi = 6.283185307179586;
  for (int p = 0; p < 32; ++p) {
    double R = sqrt(-2.0 * log(U[2 * p]));
    double a = two_pi * U[2 * p + 1];
    xi[2 * p] = R * cos(a);
    xi[2 * p + 1] = R * sin(a);
  }
}

/* ------------------------------------------------------------------------ */
/* 1D Karhunen-Loeve pairs of C(s,t) = exp(-|s-t|/lambda) on [0,1].          */
/* Differentiating the integral eigen-equation twice gives phi'' = -w^2 phi  */
/* with theta = 2 lambda/(1 + lambda^2 w^2) and the Robin conditions         */
/* phi'(0) = phi(0)/lambda, phi'(1) = -phi(1)/lambda, hence                  */
/* phi = sin(w s) + lambda w cos(w s) and the transcendental equation        */
/* g(w) = (lambda^2 w^2 - 1) sin w - 2 lambda w cos w = 0, one root in each  */
/* interval (m pi, (m+1) pi).                                                 */
/* ------------------------------------------------------------------------ */
static double kl_g(double lambda, double w) {
  return (lambda * lambda * w * w - 1.0) * sin(w) - 2.0 * lambda * w * cos(w);
}

int or_kl_1d(double lambda, int nterms, double *omega, double *theta, double *norm) {
  if (!(lambda > 0.0) || nterms < 1) return OR_EINVAL;
  const double pi = 3.141592653589793;
  for (int m = 0; m < nterms; ++m) {
    double lo = m * pi, hi = (m + 1) * pi;
    /* sign of g just right of m*pi is -(-1)^m (also for m = 0, where g ~ -(1+2 lambda) w) */
    double slo = (m % 2 == 0) ? -1.0 : 1.0;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      double gm = kl_g(lambda, mid);
      if (gm == 0.0) { lo = hi = mid; break; }
      if ((gm < 0.0) == (slo < 0.0)) lo = mid; else hi = mid;
    }
    double w = 0.5 * (lo + hi);
    omega[m] = w;
    theta[m] = 2.0 * lambda / (1.0 + lambda * lambda * w * w);
    /* N = int_0^1 (sin ws + lambda w cos ws)^2 ds in closed form */
    double s2w = sin(2.0 * w), sw = sin(w);
    norm[m] = 0.5 - s2w / (4.0 * w) + lambda * lambda * w * w * (0.5 + s2w / (4.0 * w)) +
              lambda * sw * sw;
  }
  return OR_OK;
}

double or_kl_phi(double lambda, double omega, double norm, double s) {
  return (sin(omega * s) + lambda * omega * cos(omega * s)) / sqrt(norm);
}

/* Z(x,y,z) = sigma * sum_{a,b,c<4} sqrt(theta_a theta_b theta_c) xi_{16a+4b+c}
 *            phi_a(x) phi_b(y) phi_c(z),   k = exp(Z) at every vertex. */
int or_field(int n, double sigma2, double lambda, const double xi[64], double *k) {
  if (n < 3 || !(sigma2 >= 0.0) || !(lambda > 0.0)) return OR_EINVAL;
  double om[4], th[4], nm[4];
  int st = or_kl_1d(lambda, 4, om, th, nm);
  if (st) return st;
  double *phi = (double *)malloc(sizeof(double) * 4 * (size_t)n);
  if (!phi) return OR_EINVAL;
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < n; ++i) phi[a * n + i] = or_kl_phi(lambda, om[a], nm[a], (double)i / (double)(n - 1));
  double coef[64];
  double sigma = sqrt(sigma2);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c)
        coef[16 * a + 4 * b + c] = sigma * sqrt(th[a] * th[b] * th[c]) * xi[16 * a + 4 * b + c];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int kk = 0; kk < n; ++kk) {
        double Z = 0.0;
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
              Z += coef[16 * a + 4 * b + c] * phi[a * n + i] * phi[b * n + j] * phi[c * n + kk];
        k[IDX(n, i, j, kk)] = exp(Z);
      }
  free(phi);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Operator: 7-point finite differences with harmonic-mean face              */
/* coefficients c_pq = 2 k_p k_q / (k_p + k_q), scaled by h^2:               */
/* (A'u)_p = D_p u_p - sum_q c_pq u_q, D_p = sum_q c_pq, u = 0 on boundary.  */
/* Neighbour order: i-1, i+1, j-1, j+1, k-1, k+1.                            */
/* ------------------------------------------------------------------------ */
static double hmean(double a, double b) { return 2.0 * a * b / (a + b); }

static void neighbours(int n, int i, int j, int kk, size_t q[6]) {
  q[0] = IDX(n, i - 1, j, kk);
  q[1] = IDX(n, i + 1, j, kk);
  q[2] = IDX(n, i, j - 1, kk);
  q[3] = IDX(n, i, j + 1, kk);
  q[4] = IDX(n, i, j, kk - 1);
  q[5] = IDX(n, i, j, kk + 1);
}

static int on_boundary(int n, size_t q) {
  int kk = (int)(q % (size_t)n);
  int j = (int)((q / (size_t)n) % (size_t)n);
  int i = (int)(q / ((size_t)n * (size_t)n));
  return i == 0 || j == 0 || kk == 0 || i == n - 1 || j == n - 1 || kk == n - 1;
}

/* value of u at vertex q, with the Dirichlet value 0 on the boundary */
static double uval(int n, const double *u, size_t q) { return on_boundary(n, q) ? 0.0 : u[q]; }

int or_apply(int n, const double *k, const double *u, double *out) {
  if (n < 3) return OR_EINVAL;
  size_t N = (size_t)n * n * n;
  for (size_t p = 0; p < N; ++p) out[p] = 0.0;
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        size_t p = IDX(n, i, j, kk), q[6];
        neighbours(n, i, j, kk, q);
        double D = 0.0, s = 0.0;
        for (int t = 0; t < 6; ++t) {
          double c = hmean(k[p], k[q[t]]);
          D += c;
          s += c * uval(n, u, q[t]);
        }
        out[p] = D * u[p] - s;
      }
  return OR_OK;
}

int or_residual(int n, const double *k, const double *b, const double *u, double *r) {
  int st = or_apply(n, k, u, r);
  if (st) return st;
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        size_t p = IDX(n, i, j, kk);
        r[p] = b[p] - r[p];
      }
  return OR_OK;
}

/* Gauss-Seidel point update u_p <- (b'_p + sum_q c_pq u_q) / D_p over the
 * interior vertices of one colour ((i+j+k) even = red, odd = black). */
static void gs_colour(int n, const double *k, const double *b, double *u, int colour) {
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        if (((i + j + kk) & 1) != colour) continue;
        size_t p = IDX(n, i, j, kk), q[6];
        neighbours(n, i, j, kk, q);
        double D = 0.0, s = 0.0;
        for (int t = 0; t < 6; ++t) {
          double c = hmean(k[p], k[q[t]]);
          D += c;
          s += c * uval(n, u, q[t]);
        }
        u[p] = (b[p] + s) / D;
      }
}

int or_rbgs_sweep(int n, const double *k, const double *b, double *u) {
  if (n < 3) return OR_EINVAL;
  gs_colour(n, k, b, u, 0);
  gs_colour(n, k, b, u, 1);
  return OR_OK;
}

/* Full weighting: b'_c(I) = 4 * sum_{d in {-1,0,1}^3} 2^{-|d|_1} / 8 * r'(2I+d).
 * The factor 4 = h_c^2 / h^2 converts the h^2-scaled fine residual into the
 * h_c^2-scaled coarse right-hand side. */
int or_restrict(int n, const double *r, double *bc) {
  if (n < 5 || ((n - 1) & 1)) return OR_EINVAL;
  int nc = (n - 1) / 2 + 1;
  size_t Nc = (size_t)nc * nc * nc;
  for (size_t p = 0; p < Nc; ++p) bc[p] = 0.0;
  for (int I = 1; I < nc - 1; ++I)
    for (int J = 1; J < nc - 1; ++J)
      for (int K = 1; K < nc - 1; ++K) {
        double s = 0.0;
        for (int di = -1; di <= 1; ++di)
          for (int dj = -1; dj <= 1; ++dj)
            for (int dk = -1; dk <= 1; ++dk) {
              int l1 = abs(di) + abs(dj) + abs(dk);
              double w = ldexp(1.0, -l1) / 8.0;
              s += w * r[IDX(n, 2 * I + di, 2 * J + dj, 2 * K + dk)];
            }
        bc[IDX(nc, I, J, K)] = 4.0 * s;
      }
  return OR_OK;
}

/* Trilinear interpolation: per axis, an even fine index 2I takes coarse I
 * with weight 1, an odd one 2I+1 takes I and I+1 with weight 1/2 each; the
 * coarse correction is 0 on the boundary. */
int or_prolong_add(int nc, const double *ec, double *uf) {
  if (nc < 3) return OR_EINVAL;
  int n = 2 * (nc - 1) + 1;
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        int ci[2], cj[2], ck[2];
        double wi[2], wj[2], wk[2];
        int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (kk & 1) ? 2 : 1;
        ci[0] = i / 2; ci[1] = i / 2 + 1; wi[0] = wi[1] = (ni == 2) ? 0.5 : 1.0;
        cj[0] = j / 2; cj[1] = j / 2 + 1; wj[0] = wj[1] = (nj == 2) ? 0.5 : 1.0;
        ck[0] = kk / 2; ck[1] = kk / 2 + 1; wk[0] = wk[1] = (nk == 2) ? 0.5 : 1.0;
        double s = 0.0;
        for (int a = 0; a < ni; ++a)
          for (int b = 0; b < nj; ++b)
            for (int c = 0; c < nk; ++c) {
              size_t q = IDX(nc, ci[a], cj[b], ck[c]);
              double e = on_boundary(nc, q) ? 0.0 : ec[q];
              s += wi[a] * wj[b] * wk[c] * e;
            }
        uf[IDX(n, i, j, kk)] += s;
      }
  return OR_OK;
}

int or_inject(int n, const double *kf, double *kc) {
  if (n < 5 || ((n - 1) & 1)) return OR_EINVAL;
  int nc = (n - 1) / 2 + 1;
  for (int I = 0; I < nc; ++I)
    for (int J = 0; J < nc; ++J)
      for (int K = 0; K < nc; ++K) kc[IDX(nc, I, J, K)] = kf[IDX(n, 2 * I, 2 * J, 2 * K)];
  return OR_OK;
}

static int valid_n(int n) {
  if (n < 3) return 0;
  int m = n - 1;
  return (m & (m - 1)) == 0;
}

/* V-cycle on level with n vertices: nu1 sweeps, residual, restriction, a
 * recursive cycle on the coarse grid from a zero guess, prolongation and
 * correction, nu2 sweeps.  On 3^3 the single unknown is solved exactly. */
static int vcycle_rec(int n, const double *k, const double *b, double *u, int nu1, int nu2) {
  if (n == 3) {
    size_t p = IDX(3, 1, 1, 1), q[6];
    neighbours(3, 1, 1, 1, q);
    double D = 0.0;
    for (int t = 0; t < 6; ++t) D += hmean(k[p], k[q[t]]);
    u[p] = b[p] / D;
    return OR_OK;
  }
  size_t N = (size_t)n * n * n;
  int nc = (n - 1) / 2 + 1;
  size_t Nc = (size_t)nc * nc * nc;
  double *r = (double *)malloc(sizeof(double) * N);
  double *kc = (double *)malloc(sizeof(double) * Nc);
  double *bc = (double *)malloc(sizeof(double) * Nc);
  double *ec = (double *)calloc(Nc, sizeof(double));
  if (!r || !kc || !bc || !ec) { free(r); free(kc); free(bc); free(ec); return OR_EINVAL; }
  for (int s = 0; s < nu1; ++s) or_rbgs_sweep(n, k, b, u);
  or_residual(n, k, b, u, r);
  or_restrict(n, r, bc);
  or_inject(n, k, kc);
  vcycle_rec(nc, kc, bc, ec, nu1, nu2);
  or_prolong_add(nc, ec, u);
  for (int s = 0; s < nu2; ++s) or_rbgs_sweep(n, k, b, u);
  free(r); free(kc); free(bc); free(ec);
  return OR_OK;
}

int or_vcycle(int n, const double *k, const double *b, double *u, int nu1, int nu2) {
  if (!valid_n(n) || nu1 < 0 || nu2 < 0) return OR_EINVAL;
  return vcycle_rec(n, k, b, u, nu1, nu2);
}

/* Neumaier's compensated summation. */
double or_sum(const double *x, long n) {
  double s = 0.0, c = 0.0;
  for (long i = 0; i < n; ++i) {
    double t = s + x[i];
    if (fabs(s) >= fabs(x[i])) c += (s - t) + x[i];
    else c += (x[i] - t) + s;
    s = t;
  }
  return s + c;
}

double or_norm2(int n, const double *v) {
  double s = 0.0, c = 0.0;
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        double x = v[IDX(n, i, j, kk)];
        double y = x * x;
        double t = s + y;
        if (fabs(s) >= fabs(y)) c += (s - t) + y;
        else c += (y - t) + s;
        s = t;
      }
  return sqrt(s + c);
}

/* Cycle until ||b' - A'u||_2 / ||b'||_2 <= tol (checked after every full
 * cycle) or, with fixed_cycles > 0, for exactly fixed_cycles cycles.  With
 * ||b'|| = 0 the absolute residual norm is used instead. */
int or_solve(int n, const double *k, const double *b, double *u, int nu1, int nu2,
             double tol, int max_cycles, int fixed_cycles,
             int *cycles, double *relres, double *hist) {
  if (!valid_n(n) || nu1 < 0 || nu2 < 0) return OR_EINVAL;
  if (fixed_cycles <= 0 && (max_cycles < 1 || !(tol > 0.0))) return OR_EINVAL;
  size_t N = (size_t)n * n * n;
  double *r = (double *)malloc(sizeof(double) * N);
  if (!r) return OR_EINVAL;
  /* Dirichlet boundary values of u are 0 */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int kk = 0; kk < n; ++kk)
        if (i == 0 || j == 0 || kk == 0 || i == n - 1 || j == n - 1 || kk == n - 1) u[IDX(n, i, j, kk)] = 0.0;
  double bn = or_norm2(n, b);
  double scale = bn > 0.0 ? bn : 1.0;
  int limit = fixed_cycles > 0 ? fixed_cycles : max_cycles;
  int m = 0, status = OR_ENOCONV;
  double rho = 0.0;
  for (m = 1; m <= limit; ++m) {
    vcycle_rec(n, k, b, u, nu1, nu2);
    or_residual(n, k, b, u, r);
    rho = or_norm2(n, r) / scale;
    if (hist) hist[m - 1] = rho;
    if (fixed_cycles > 0) {
      if (m == fixed_cycles) { status = OR_OK; break; }
    } else if (rho <= tol) {
      status = OR_OK;
      break;
    }
  }
  if (m > limit) m = limit;
  if (cycles) *cycles = m;
  if (relres) *relres = rho;
  free(r);
  return status;
}

/* QoI: the integral of u over D; u vanishes on the boundary, so the
 * trapezoidal rule reduces to h^3 times the sum over interior vertices. */
double or_qoi(int n, const double *u) {
  double s = 0.0, c = 0.0;
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        double x = u[IDX(n, i, j, kk)];
        double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
      }
  double h = 1.0 / (double)(n - 1);
  return h * h * h * (s + c);
}

/* Point QoI of Section 3: Q(u) = u(x*) at x* = (1/4, 1/4, 1/4), the vertex
 * ((n-1)/4, (n-1)/4, (n-1)/4) for n = 4m + 1 (the paper's point in its
 * Section 7.1 experiments). */
double or_point_qoi(int n, const double *u) {
  if (n < 5 || ((n - 1) % 4) != 0) return 0.0;
  int c = (n - 1) / 4;
  return u[IDX(n, c, c, c)];
}

/* Flux QoI of Section 3 across Gamma = {x_2 = 1/4} (the plane of the
 * Section 7.2 experiments), as the flux of -k grad u in the +x_2 direction
 * with |Gamma| = 1.  x_2 is the j index; the plane is the vertex plane
 * j* = (n-1)/4.  The discrete flux through the face plane between vertex
 * planes a and a+1 is h^2 sum over interior (i,k) of c * (u(a) - u(a+1)) / h
 * with the operator's face coefficient c; the flux through Gamma is the mean
 * of the face planes j* - 1/2 and j* + 1/2 (second order). */
double or_flux_qoi(int n, const double *k, const double *u) {
  if (n < 5 || ((n - 1) % 4) != 0) return 0.0;
  int js = (n - 1) / 4;
  double h = 1.0 / (double)(n - 1);
  double F[2];
  for (int side = 0; side < 2; ++side) {
    int a = js - 1 + side; /* face between planes a and a + 1 */
    double s = 0.0, c = 0.0;
    for (int i = 1; i < n - 1; ++i)
      for (int kk = 1; kk < n - 1; ++kk) {
        size_t p = IDX(n, i, a, kk), q = IDX(n, i, a + 1, kk);
        double x = hmean(k[p], k[q]) * (uval(n, u, p) - uval(n, u, q));
        double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
      }
    F[side] = h * (s + c);
  }
  return 0.5 * (F[0] + F[1]);
}

/* Full multigrid (nested iteration, the FMG-nu V(nu1,nu2) schedule of
 * Section 7.1): on every grid of the hierarchy the problem itself is
 * discretised (coefficient and f injected, b' = h_j^2 f); the 3^3 grid is
 * solved exactly; each finer grid starts from the trilinear interpolation of
 * the coarser grid's result and runs ncycles V(nu1,nu2) cycles.  u (n^3)
 * receives the finest grid's result; f is an n^3 array of vertex values. */
int or_fmg(int n, const double *k, const double *f, double *u, int nu1, int nu2, int ncycles) {
  if (!valid_n(n) || nu1 < 0 || nu2 < 0 || ncycles < 1) return OR_EINVAL;
  int nl = 0, ns[32];
  for (int m = n; ; m = (m - 1) / 2 + 1) {
    ns[nl++] = m;
    if (m == 3) break;
  }
  double *K[32], *B[32], *U[32];
  for (int j = 0; j < nl; ++j) {
    size_t N = (size_t)ns[j] * ns[j] * ns[j];
    K[j] = (double *)malloc(sizeof(double) * N);
    B[j] = (double *)malloc(sizeof(double) * N);
    U[j] = (double *)calloc(N, sizeof(double));
  }
  /* coefficients and f injected level by level; b' = h_j^2 f */
  memcpy(K[0], k, sizeof(double) * (size_t)n * n * n);
  memcpy(B[0], f, sizeof(double) * (size_t)n * n * n);
  for (int j = 1; j < nl; ++j) {
    or_inject(ns[j - 1], K[j - 1], K[j]);
    or_inject(ns[j - 1], B[j - 1], B[j]);
  }
  for (int j = 0; j < nl; ++j) {
    size_t N = (size_t)ns[j] * ns[j] * ns[j];
    double h = 1.0 / (double)(ns[j] - 1);
    for (size_t p = 0; p < N; ++p) B[j][p] *= h * h;
  }
  /* coarsest: the single unknown exactly */
  vcycle_rec(3, K[nl - 1], B[nl - 1], U[nl - 1], nu1, nu2);
  for (int j = nl - 2; j >= 0; --j) {
    or_prolong_add(ns[j + 1], U[j + 1], U[j]); /* U[j] = 0 + P U[j+1] */
    for (int c = 0; c < ncycles; ++c) vcycle_rec(ns[j], K[j], B[j], U[j], nu1, nu2);
  }
  memcpy(u, U[0], sizeof(double) * (size_t)n * n * n);
  for (int j = 0; j < nl; ++j) { free(K[j]); free(B[j]); free(U[j]); }
  return OR_OK;
}

/* Solve one grid for one sample: field, right-hand side h^2 * f with f = 1,
 * zero initial guess, V-cycles, QoI. */
static int solve_q(int n, double sigma2, double lambda, const double xi[64], int nu1, int nu2,
                   double tol, int max_cycles, int fixed_cycles, double *Q, int *cycles) {
  size_t N = (size_t)n * n * n;
  double *k = (double *)malloc(sizeof(double) * N);
  double *b = (double *)malloc(sizeof(double) * N);
  double *u = (double *)calloc(N, sizeof(double));
  if (!k || !b || !u) { free(k); free(b); free(u); return OR_EINVAL; }
  int st = or_field(n, sigma2, lambda, xi, k);
  double h = 1.0 / (double)(n - 1);
  for (size_t p = 0; p < N; ++p) b[p] = h * h * 1.0;
  if (!st) st = or_solve(n, k, b, u, nu1, nu2, tol, max_cycles, fixed_cycles, cycles, NULL, NULL);
  *Q = or_qoi(n, u);
  free(k); free(b); free(u);
  return st;
}

int or_mlmc_sample(int n0, int level, uint64_t seed, double sigma2, double lambda,
                   int nu1, int nu2, double tol, int max_cycles, int fixed_cycles,
                   double *Y, double *Qf, double *Qc, int cycles[2]) {
  if (!valid_n(n0) || level < 0 || level > 12) return OR_EINVAL;
  double xi[64];
  or_gaussians(seed, (uint32_t)level, xi);
  int nf = (n0 - 1) * (1 << level) + 1;
  double qf = 0.0, qc = 0.0;
  int cf = 0, cc = 0;
  int st = solve_q(nf, sigma2, lambda, xi, nu1, nu2, tol, max_cycles, fixed_cycles, &qf, &cf);
  int st2 = OR_OK;
  if (level > 0) {
    int nc = (n0 - 1) * (1 << (level - 1)) + 1;
    st2 = solve_q(nc, sigma2, lambda, xi, nu1, nu2, tol, max_cycles, fixed_cycles, &qc, &cc);
  }
  if (Qf) *Qf = qf;
  if (Qc) *Qc = qc;
  if (Y) *Y = qf - qc;
  if (cycles) { cycles[0] = cf; cycles[1] = cc; }
  return st ? st : st2;
}

/* One sample with a chosen solver and QoI: solver 0 = V(nu1,nu2) cycles to
 * tol (or fixed_cycles) from zero, 1 = FMG with fmg_cycles V(nu1,nu2) cycles
 * per grid; qoi 0 = integral of u, 1 = u(1/4,1/4,1/4), 2 = flux across
 * x_2 = 1/4.  Both solves of a pair use the same normals xi(seed, level).
 * cycles[] receives the V-cycles run on the top grid of each solve. */
static int solve_q_ex(int n, double sigma2, double lambda, const double xi[64], int nu1, int nu2,
                      int solver, int fmg_cycles, int qoi, double tol, int max_cycles,
                      int fixed_cycles, double *Q, int *cycles) {
  size_t N = (size_t)n * n * n;
  double *k = (double *)malloc(sizeof(double) * N);
  double *b = (double *)malloc(sizeof(double) * N);
  double *u = (double *)calloc(N, sizeof(double));
  if (!k || !b || !u) { free(k); free(b); free(u); return OR_EINVAL; }
  int st = or_field(n, sigma2, lambda, xi, k);
  double h = 1.0 / (double)(n - 1);
  if (!st && solver == 1) {
    for (size_t p = 0; p < N; ++p) b[p] = 1.0; /* f = 1 */
    st = or_fmg(n, k, b, u, nu1, nu2, fmg_cycles);
    *cycles = fmg_cycles;
  } else if (!st) {
    for (size_t p = 0; p < N; ++p) b[p] = h * h * 1.0;
    st = or_solve(n, k, b, u, nu1, nu2, tol, max_cycles, fixed_cycles, cycles, NULL, NULL);
  }
  *Q = qoi == 1 ? or_point_qoi(n, u) : qoi == 2 ? or_flux_qoi(n, k, u) : or_qoi(n, u);
  free(k); free(b); free(u);
  return st;
}

int or_mlmc_sample_ex(int n0, int level, uint64_t seed, double sigma2, double lambda,
                      int nu1, int nu2, int solver, int fmg_cycles, int qoi, double tol,
                      int max_cycles, int fixed_cycles, double *Y, double *Qf, double *Qc,
                      int cycles[2]) {
  if (!valid_n(n0) || level < 0 || level > 12 || solver < 0 || solver > 1 || qoi < 0 || qoi > 2)
    return OR_EINVAL;
  int nf = (n0 - 1) * (1 << level) + 1;
  int nc = level > 0 ? (n0 - 1) * (1 << (level - 1)) + 1 : 0;
  if (qoi > 0 && ((nf - 1) % 4 != 0 || nf < 5 || (level > 0 && ((nc - 1) % 4 != 0 || nc < 5))))
    return OR_EINVAL;
  double xi[64];
  or_gaussians(seed, (uint32_t)level, xi);
  double qf = 0.0, qc = 0.0;
  int cf = 0, cc = 0;
  int st = solve_q_ex(nf, sigma2, lambda, xi, nu1, nu2, solver, fmg_cycles, qoi, tol, max_cycles,
                      fixed_cycles, &qf, &cf);
  int st2 = OR_OK;
  if (level > 0)
    st2 = solve_q_ex(nc, sigma2, lambda, xi, nu1, nu2, solver, fmg_cycles, qoi, tol, max_cycles,
                     fixed_cycles, &qc, &cc);
  if (Qf) *Qf = qf;
  if (Qc) *Qc = qc;
  if (Y) *Y = qf - qc;
  if (cycles) { cycles[0] = cf; cycles[1] = cc; }
  return st ? st : st2;
}

/* ------------------------------------------------------------------------ */
/* P1 finite elements (Section 3.1): the system matrix assembled element by  */
/* element, A_ij = sum over tetrahedra of grad(phi_i).grad(phi_j) |tau| times */
/* the mean of k at the tetrahedron's four vertices (the four-node           */
/* quadrature).  Mesh (reading of "uniformly refined simplicial meshes" on a  */
/* vertex grid): every cell [i,i+1]x[j,j+1]x[k,k+1] split into the 6 Kuhn     */
/* tetrahedra v0 = corner, v1 = v0 + e_a, v2 = v1 + e_b, v3 = v2 + e_c, one   */
/* for each ordering (a, b, c) of the axes.  Scaled by 1/h, so that with      */
/* F_i = int f phi_i = h^3 f the system reads A' u = h^2 f as the FD one.     */
/* ------------------------------------------------------------------------ */
static const int kuhn_perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

/* The scaled element matrix of one tetrahedron with integer vertex offsets
 * v[4][3] (in units of h) and coefficient kbar: Ke[m][q] = kbar |tau|/h *
 * grad(lambda_m).grad(lambda_q), the barycentric gradients from the inverse
 * of the edge matrix E = [v1-v0, v2-v0, v3-v0]. */
static void p1_element(const int v[4][3], double kbar, double Ke[4][4]) {
  double E[3][3], adj[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) E[r][c] = (double)(v[c + 1][r] - v[0][r]);
  double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
               E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
               E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
  /* inverse = adjugate / det; lambda_{m+1}(x) = row m of E^-1 applied to x - v0 */
  adj[0][0] = E[1][1] * E[2][2] - E[1][2] * E[2][1];
  adj[0][1] = E[0][2] * E[2][1] - E[0][1] * E[2][2];
  adj[0][2] = E[0][1] * E[1][2] - E[0][2] * E[1][1];
  adj[1][0] = E[1][2] * E[2][0] - E[1][0] * E[2][2];
  adj[1][1] = E[0][0] * E[2][2] - E[0][2] * E[2][0];
  adj[1][2] = E[0][2] * E[1][0] - E[0][0] * E[1][2];
  adj[2][0] = E[1][0] * E[2][1] - E[1][1] * E[2][0];
  adj[2][1] = E[0][1] * E[2][0] - E[0][0] * E[2][1];
  adj[2][2] = E[0][0] * E[1][1] - E[0][1] * E[1][0];
  double g[4][3];
  for (int m = 0; m < 3; ++m)
    for (int c = 0; c < 3; ++c) g[m + 1][c] = adj[m][c] / det;
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  double vol = fabs(det) / 6.0; /* |tau| / h^3 */
  for (int m = 0; m < 4; ++m)
    for (int q = 0; q < 4; ++q)
      Ke[m][q] = kbar * vol * (g[m][0] * g[q][0] + g[m][1] * g[q][1] + g[m][2] * g[q][2]);
}

/* The scaled P1 operator as a 27-point stencil per vertex: S[27 p + t] is the
 * coupling of vertex p to its neighbour p + (di, dj, dk), t = (di+1)*9 +
 * (dj+1)*3 + (dk+1), summed over every tetrahedron of every cell (rows of
 * boundary vertices are assembled too; they are not used). */
int or_fe_stencil(int n, const double *k, double *S) {
  if (n < 3) return OR_EINVAL;
  size_t N = (size_t)n * n * n;
  memset(S, 0, sizeof(double) * 27 * N);
  for (int i = 0; i < n - 1; ++i)
    for (int j = 0; j < n - 1; ++j)
      for (int kk = 0; kk < n - 1; ++kk)
        for (int t = 0; t < 6; ++t) {
          int v[4][3] = {{i, j, kk}};
          for (int s2 = 1; s2 < 4; ++s2) {
            for (int c = 0; c < 3; ++c) v[s2][c] = v[s2 - 1][c];
            v[s2][kuhn_perm[t][s2 - 1]] += 1;
          }
          double kbar = 0.0;
          for (int m = 0; m < 4; ++m) kbar += k[IDX(n, v[m][0], v[m][1], v[m][2])];
          kbar *= 0.25;
          double Ke[4][4];
          p1_element(v, kbar, Ke);
          for (int m = 0; m < 4; ++m)
            for (int q = 0; q < 4; ++q) {
              int di = v[q][0] - v[m][0], dj = v[q][1] - v[m][1], dk = v[q][2] - v[m][2];
              S[27 * IDX(n, v[m][0], v[m][1], v[m][2]) + (di + 1) * 9 + (dj + 1) * 3 + (dk + 1)] +=
                  Ke[m][q];
            }
        }
  return OR_OK;
}

/* (A'u)_p over interior rows with u = 0 on the boundary. */
static void fe_apply_s(int n, const double *S, const double *u, double *out) {
  size_t N = (size_t)n * n * n;
  for (size_t p = 0; p < N; ++p) out[p] = 0.0;
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        size_t p = IDX(n, i, j, kk);
        double s = 0.0;
        for (int t = 0; t < 27; ++t) {
          size_t q = IDX(n, i + t / 9 - 1, j + (t / 3) % 3 - 1, kk + t % 3 - 1);
          s += S[27 * p + t] * uval(n, u, q);
        }
        out[p] = s;
      }
}

int or_fe_apply(int n, const double *k, const double *u, double *out) {
  if (n < 3) return OR_EINVAL;
  size_t N = (size_t)n * n * n;
  double *S = (double *)malloc(sizeof(double) * 27 * N);
  if (!S) return OR_EINVAL;
  or_fe_stencil(n, k, S);
  fe_apply_s(n, S, u, out);
  free(S);
  return OR_OK;
}

/* Gauss-Seidel on one colour ((i+j+k) even = red) with the full 27-point
 * row: u_p = (b_p - sum_{q != p} S_pq u_q) / S_pp. */
static void fe_gs_colour(int n, const double *S, const double *b, double *u, int colour) {
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        if (((i + j + kk) & 1) != colour) continue;
        size_t p = IDX(n, i, j, kk);
        double s = 0.0;
        for (int t = 0; t < 27; ++t) {
          if (t == 13) continue;
          size_t q = IDX(n, i + t / 9 - 1, j + (t / 3) % 3 - 1, kk + t % 3 - 1);
          s += S[27 * p + t] * uval(n, u, q);
        }
        u[p] = (b[p] - s) / S[27 * p + 13];
      }
}

static void fe_residual_s(int n, const double *S, const double *b, const double *u, double *r) {
  fe_apply_s(n, S, u, r);
  for (int i = 1; i < n - 1; ++i)
    for (int j = 1; j < n - 1; ++j)
      for (int kk = 1; kk < n - 1; ++kk) {
        size_t p = IDX(n, i, j, kk);
        r[p] = b[p] - r[p];
      }
}

/* V(nu1,nu2) with the P1 operator rediscretised on every level (k injected). */
static int fe_vcycle_rec(int n, const double *k, const double *b, double *u, int nu1, int nu2) {
  size_t N = (size_t)n * n * n;
  double *S = (double *)malloc(sizeof(double) * 27 * N);
  if (!S) return OR_EINVAL;
  or_fe_stencil(n, k, S);
  if (n == 3) {
    size_t p = IDX(3, 1, 1, 1);
    u[p] = b[p] / S[27 * p + 13];
    free(S);
    return OR_OK;
  }
  int nc = (n - 1) / 2 + 1;
  size_t Nc = (size_t)nc * nc * nc;
  double *r = (double *)malloc(sizeof(double) * N);
  double *kc = (double *)malloc(sizeof(double) * Nc);
  double *bc = (double *)malloc(sizeof(double) * Nc);
  double *ec = (double *)calloc(Nc, sizeof(double));
  for (int s2 = 0; s2 < nu1; ++s2) { fe_gs_colour(n, S, b, u, 0); fe_gs_colour(n, S, b, u, 1); }
  fe_residual_s(n, S, b, u, r);
  or_restrict(n, r, bc);
  or_inject(n, k, kc);
  fe_vcycle_rec(nc, kc, bc, ec, nu1, nu2);
  or_prolong_add(nc, ec, u);
  for (int s2 = 0; s2 < nu2; ++s2) { fe_gs_colour(n, S, b, u, 0); fe_gs_colour(n, S, b, u, 1); }
  free(S); free(r); free(kc); free(bc); free(ec);
  return OR_OK;
}

/* Solve the P1 system as or_solve does the FD one (same stopping rule). */
int or_fe_solve(int n, const double *k, const double *b, double *u, int nu1, int nu2,
                double tol, int max_cycles, int fixed_cycles, int *cycles, double *relres) {
  if (!valid_n(n) || nu1 < 0 || nu2 < 0) return OR_EINVAL;
  if (fixed_cycles <= 0 && (max_cycles < 1 || !(tol > 0.0))) return OR_EINVAL;
  size_t N = (size_t)n * n * n;
  double *r = (double *)malloc(sizeof(double) * N);
  double *S = (double *)malloc(sizeof(double) * 27 * N);
  if (!r || !S) { free(r); free(S); return OR_EINVAL; }
  or_fe_stencil(n, k, S);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int kk = 0; kk < n; ++kk)
        if (i == 0 || j == 0 || kk == 0 || i == n - 1 || j == n - 1 || kk == n - 1) u[IDX(n, i, j, kk)] = 0.0;
  double bn = or_norm2(n, b);
  double scale = bn > 0.0 ? bn : 1.0;
  int limit = fixed_cycles > 0 ? fixed_cycles : max_cycles;
  int m = 0, status = OR_ENOCONV;
  double rho = 0.0;
  for (m = 1; m <= limit; ++m) {
    fe_vcycle_rec(n, k, b, u, nu1, nu2);
    fe_residual_s(n, S, b, u, r);
    rho = or_norm2(n, r) / scale;
    if (fixed_cycles > 0) {
      if (m == fixed_cycles) { status = OR_OK; break; }
    } else if (rho <= tol) {
      status = OR_OK;
      break;
    }
  }
  if (m > limit) m = limit;
  if (cycles) *cycles = m;
  if (relres) *relres = rho;
  free(r); free(S);
  return status;
}

/* One MLMC sample with the P1 operator (V-cycles to tol; qoi 0 = integral,
 * 1 = point value). */
int or_mlmc_sample_fe(int n0, int level, uint64_t seed, double sigma2, double lambda, int nu1,
                      int nu2, int qoi, double tol, int max_cycles, int fixed_cycles, double *Y,
                      double *Qf, double *Qc, int cycles[2]) {
  if (!valid_n(n0) || level < 0 || level > 12 || qoi < 0 || qoi > 1) return OR_EINVAL;
  double xi[64];
  or_gaussians(seed, (uint32_t)level, xi);
  double q[2] = {0.0, 0.0};
  int cyc[2] = {0, 0}, st = OR_OK;
  for (int s2 = 0; s2 < (level > 0 ? 2 : 1); ++s2) {
    int n = (n0 - 1) * (1 << (level - s2)) + 1;
    if (qoi == 1 && ((n - 1) % 4 != 0 || n < 5)) return OR_EINVAL;
    size_t N = (size_t)n * n * n;
    double *k = (double *)malloc(sizeof(double) * N);
    double *b = (double *)malloc(sizeof(double) * N);
    double *u = (double *)calloc(N, sizeof(double));
    int st2 = or_field(n, sigma2, lambda, xi, k);
    double h = 1.0 / (double)(n - 1);
    for (size_t p = 0; p < N; ++p) b[p] = h * h;
    if (!st2) st2 = or_fe_solve(n, k, b, u, nu1, nu2, tol, max_cycles, fixed_cycles, &cyc[s2], NULL);
    q[s2] = qoi == 1 ? or_point_qoi(n, u) : or_qoi(n, u);
    if (st2 && !st) st = st2;
    free(k); free(b); free(u);
  }
  if (Qf) *Qf = q[0];
  if (Qc) *Qc = q[1];
  if (Y) *Y = q[0] - q[1];
  if (cycles) { cycles[0] = cyc[0]; cycles[1] = cyc[1]; }
  return st;
}

/* ------------------------------------------------------------------------ */
/* SPDE sampler of the lognormal field (Section 3.2, eq. spde):              */
/* (kappa^2 - Laplace) Z = W on the box (-1,2)^3 with natural (homogeneous  */
/* Neumann) boundary conditions, P1 elements on the Kuhn tetrahedra of the   */
/* extended vertex grid (spacing h = 1/(n-1) of the n grid on D, nt =        */
/* 3(n-1)+1 vertices per axis, D's vertex i at nt-index i + n - 1), with the */
/* mass matrix lumped (its row sums).  White noise: the load <W, phi_p> has  */
/* variance M_pp, so b_p = sqrt(M_pp) xi_p.  Divided by h like the FD form:  */
/*   (K' + kappa^2 h^2 diag(m)) Z = sqrt(h m_p) xi_p,  m_p = M_pp / h^3.     */
/* Whittle: Z has covariance exp(-kappa r) / (8 pi kappa); reading: kappa =  */
/* 1/lambda and k = exp(sigma sqrt(8 pi kappa) Z).                          */
/* ------------------------------------------------------------------------ */

/* Normals of the white noise of sample (seed, level): count values, block j of
 * Philox4x32-10 with counter (j, level, 1, 0) and key (seed lo, seed hi)
 * giving normals 2j and 2j+1 (53-bit uniforms from word pairs, Box-Muller). */
void or_white_noise(uint64_t seed, uint32_t level, long count, double *xi) {
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  const double two_pi = 6.283185307179586;
  for (long j = 0; 2 * j < count; ++j) {
    uint32_t ctr[4] = {(uint32_t)j, level, 1u, 0u}, w[4];
    or_philox4x32_10(ctr, key, w);
    double U0 = ((double)((uint64_t)(w[0] >> 5) * 67108864ull + (uint64_t)(w[1] >> 6)) + 1.0) * 0x1p-53;
    double U1 = ((double)((uint64_t)(w[2] >> 5) * 67108864ull + (uint64_t)(w[3] >> 6)) + 1.0) * 0x1p-53;
    double R = sqrt(-2.0 * log(U0)), a = two_pi * U1;
    xi[2 * j] = R * cos(a);
    if (2 * j + 1 < count) xi[2 * j + 1] = R * sin(a);
  }
}

/* Stiffness (unit coefficient, 27 couplings per vertex, every vertex of the
 * box) and lumped mass m_p = sum over tetrahedra at p of |tau|/4 / h^3, both
 * by element-wise assembly (the same elements as or_fe_stencil). */
int or_spde_operator(int nt, double *S, double *m) {
  if (nt < 2) return OR_EINVAL;
  size_t N = (size_t)nt * nt * nt;
  memset(S, 0, sizeof(double) * 27 * N);
  memset(m, 0, sizeof(double) * N);
  for (int i = 0; i < nt - 1; ++i)
    for (int j = 0; j < nt - 1; ++j)
      for (int kk = 0; kk < nt - 1; ++kk)
        for (int t = 0; t < 6; ++t) {
          int v[4][3] = {{i, j, kk}};
          for (int s2 = 1; s2 < 4; ++s2) {
            for (int c = 0; c < 3; ++c) v[s2][c] = v[s2 - 1][c];
            v[s2][kuhn_perm[t][s2 - 1]] += 1;
          }
          double Ke[4][4];
          p1_element(v, 1.0, Ke);
          for (int a = 0; a < 4; ++a) {
            size_t pa = IDX(nt, v[a][0], v[a][1], v[a][2]);
            m[pa] += (1.0 / 6.0) / 4.0;
            for (int q = 0; q < 4; ++q) {
              int di = v[q][0] - v[a][0], dj = v[q][1] - v[a][1], dk = v[q][2] - v[a][2];
              S[27 * pa + (di + 1) * 9 + (dj + 1) * 3 + (dk + 1)] += Ke[a][q];
            }
          }
        }
  return OR_OK;
}

/* value of z at nt-index (i,j,k), 0 outside the box */
static double zval(int nt, const double *z, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= nt || j >= nt || k >= nt) return 0.0;
  return z[IDX(nt, i, j, k)];
}

/* Red-black Gauss-Seidel over every vertex of the box (one colour). */
static void spde_gs_colour(int nt, const double *S, const double *m, double k2h2, const double *b,
                           double *z, int colour) {
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j)
      for (int kk = 0; kk < nt; ++kk) {
        if (((i + j + kk) & 1) != colour) continue;
        size_t p = IDX(nt, i, j, kk);
        double s = 0.0;
        for (int t = 0; t < 27; ++t)
          if (t != 13) s += S[27 * p + t] * zval(nt, z, i + t / 9 - 1, j + (t / 3) % 3 - 1, kk + t % 3 - 1);
        z[p] = (b[p] - s) / (S[27 * p + 13] + k2h2 * m[p]);
      }
}

static void spde_residual(int nt, const double *S, const double *m, double k2h2, const double *b,
                          const double *z, double *r) {
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j)
      for (int kk = 0; kk < nt; ++kk) {
        size_t p = IDX(nt, i, j, kk);
        double s = k2h2 * m[p] * z[p];
        for (int t = 0; t < 27; ++t)
          s += S[27 * p + t] * zval(nt, z, i + t / 9 - 1, j + (t / 3) % 3 - 1, kk + t % 3 - 1);
        r[p] = b[p] - s;
      }
}

/* Coarse right-hand side from a fine one: b_c = (1/2) P^T b_f with P the
 * trilinear interpolation (the 1/2 is h / h_c of the scaled form); fine
 * points outside the box do not exist. */
int or_spde_restrict(int nt, const double *r, double *bc) {
  if (nt < 3 || ((nt - 1) & 1)) return OR_EINVAL;
  int ntc = (nt - 1) / 2 + 1;
  for (int I = 0; I < ntc; ++I)
    for (int J = 0; J < ntc; ++J)
      for (int K = 0; K < ntc; ++K) {
        double s = 0.0;
        for (int di = -1; di <= 1; ++di)
          for (int dj = -1; dj <= 1; ++dj)
            for (int dk = -1; dk <= 1; ++dk) {
              int l1 = abs(di) + abs(dj) + abs(dk);
              s += ldexp(1.0, -l1) * zval(nt, r, 2 * I + di, 2 * J + dj, 2 * K + dk);
            }
        bc[IDX(ntc, I, J, K)] = 0.5 * s;
      }
  return OR_OK;
}

/* z_f += P z_c over every fine vertex (trilinear, coarse boundary included). */
int or_spde_prolong_add(int ntc, const double *zc, double *zf) {
  int nt = 2 * (ntc - 1) + 1;
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j)
      for (int kk = 0; kk < nt; ++kk) {
        double s = 0.0;
        for (int a = 0; a <= (i & 1); ++a)
          for (int b2 = 0; b2 <= (j & 1); ++b2)
            for (int c = 0; c <= (kk & 1); ++c) {
              double w = ((i & 1) ? 0.5 : 1.0) * ((j & 1) ? 0.5 : 1.0) * ((kk & 1) ? 0.5 : 1.0);
              s += w * zc[IDX(ntc, i / 2 + a, j / 2 + b2, kk / 2 + c)];
            }
        zf[IDX(nt, i, j, kk)] += s;
      }
  return OR_OK;
}

/* V(nu1,nu2) cycle on the box grid nt at spacing h; the coarsest grid (an odd
 * number of intervals, 4^3 for these boxes) gets 32 red-black sweeps. */
static int spde_vcycle(int nt, double h, double kappa, const double *b, double *z, int nu1, int nu2) {
  size_t N = (size_t)nt * nt * nt;
  double *S = (double *)malloc(sizeof(double) * 27 * N), *m = (double *)malloc(sizeof(double) * N);
  or_spde_operator(nt, S, m);
  double k2h2 = kappa * kappa * h * h;
  if ((nt - 1) & 1) {
    for (int s2 = 0; s2 < 32; ++s2) {
      spde_gs_colour(nt, S, m, k2h2, b, z, 0);
      spde_gs_colour(nt, S, m, k2h2, b, z, 1);
    }
    free(S); free(m);
    return OR_OK;
  }
  int ntc = (nt - 1) / 2 + 1;
  size_t Nc = (size_t)ntc * ntc * ntc;
  double *r = (double *)malloc(sizeof(double) * N);
  double *bc = (double *)malloc(sizeof(double) * Nc), *ec = (double *)calloc(Nc, sizeof(double));
  for (int s2 = 0; s2 < nu1; ++s2) {
    spde_gs_colour(nt, S, m, k2h2, b, z, 0);
    spde_gs_colour(nt, S, m, k2h2, b, z, 1);
  }
  spde_residual(nt, S, m, k2h2, b, z, r);
  or_spde_restrict(nt, r, bc);
  spde_vcycle(ntc, 2.0 * h, kappa, bc, ec, nu1, nu2);
  or_spde_prolong_add(ntc, ec, z);
  for (int s2 = 0; s2 < nu2; ++s2) {
    spde_gs_colour(nt, S, m, k2h2, b, z, 0);
    spde_gs_colour(nt, S, m, k2h2, b, z, 1);
  }
  free(S); free(m); free(r); free(bc); free(ec);
  return OR_OK;
}

static double norm2_all(long N, const double *v) {
  double s = 0.0, c = 0.0;
  for (long p = 0; p < N; ++p) {
    double y = v[p] * v[p], t = s + y;
    if (fabs(s) >= fabs(y)) c += (s - t) + y;
    else c += (y - t) + s;
    s = t;
  }
  return sqrt(s + c);
}

/* Solve the scaled SPDE system from z = 0 with V(nu1,nu2) cycles until
 * ||b - A z|| / ||b|| <= tol over all vertices (or max_cycles). */
int or_spde_solve(int nt, double h, double kappa, const double *b, double *z, int nu1, int nu2,
                  double tol, int max_cycles, int *cycles, double *relres) {
  size_t N = (size_t)nt * nt * nt;
  double *S = (double *)malloc(sizeof(double) * 27 * N), *m = (double *)malloc(sizeof(double) * N);
  double *r = (double *)malloc(sizeof(double) * N);
  or_spde_operator(nt, S, m);
  memset(z, 0, sizeof(double) * N);
  double bn = norm2_all((long)N, b), rho = 1.0;
  int c = 0, st = OR_ENOCONV;
  for (c = 1; c <= max_cycles; ++c) {
    spde_vcycle(nt, h, kappa, b, z, nu1, nu2);
    spde_residual(nt, S, m, kappa * kappa * h * h, b, z, r);
    rho = norm2_all((long)N, r) / (bn > 0.0 ? bn : 1.0);
    if (rho <= tol) { st = OR_OK; break; }
  }
  if (c > max_cycles) c = max_cycles;
  if (cycles) *cycles = c;
  if (relres) *relres = rho;
  free(S); free(m); free(r);
  return st;
}

/* The scaled white-noise load on the box grid of an n grid. */
int or_spde_rhs(int n, const double *xi, double *b) {
  int nt = 3 * (n - 1) + 1;
  size_t N = (size_t)nt * nt * nt;
  double *S = (double *)malloc(sizeof(double) * 27 * N), *m = (double *)malloc(sizeof(double) * N);
  or_spde_operator(nt, S, m);
  double h = 1.0 / (double)(n - 1);
  for (size_t p = 0; p < N; ++p) b[p] = sqrt(h * m[p]) * xi[p];
  free(S); free(m);
  return OR_OK;
}

/* k = exp(sigma sqrt(8 pi kappa) Z) at the n^3 vertices of D from a box
 * solution z (nt = 3(n-1)+1). */
int or_spde_to_k(int n, double sigma2, double lambda, const double *z, double *k) {
  int nt = 3 * (n - 1) + 1, o = n - 1;
  double kappa = 1.0 / lambda, sc = sqrt(sigma2) * sqrt(8.0 * 3.141592653589793 * kappa);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int kk = 0; kk < n; ++kk) k[IDX(n, i, j, kk)] = exp(sc * z[IDX(nt, i + o, j + o, kk + o)]);
  return OR_OK;
}

/* One MLMC sample with the SPDE field: the fine field from the white noise of
 * (seed, level) on the fine box grid, the coarse field (level > 0) from the
 * same noise, b_c = (1/2) P^T b_f, on the coarse box grid; each SPDE solve to
 * spde_tol with V(2,2); the PDE solves as or_mlmc_sample (FD, V(nu1,nu2) to
 * tol, integral QoI).  spde_cycles[2] (optional) receives the SPDE cycles. */
int or_mlmc_sample_spde(int n0, int level, uint64_t seed, double sigma2, double lambda, int nu1,
                        int nu2, double tol, int max_cycles, double spde_tol, double *Y,
                        double *Qf, double *Qc, int cycles[2], int spde_cycles[2]) {
  if (!valid_n(n0) || level < 0 || level > 10) return OR_EINVAL;
  int n[2] = {(n0 - 1) * (1 << level) + 1, level > 0 ? (n0 - 1) * (1 << (level - 1)) + 1 : 0};
  int nt = 3 * (n[0] - 1) + 1;
  size_t Nt = (size_t)nt * nt * nt;
  double *xi = (double *)malloc(sizeof(double) * Nt), *bf = (double *)malloc(sizeof(double) * Nt);
  or_white_noise(seed, (uint32_t)level, (long)Nt, xi);
  or_spde_rhs(n[0], xi, bf);
  free(xi);
  double q[2] = {0.0, 0.0};
  int cyc[2] = {0, 0}, sc[2] = {0, 0}, st = OR_OK;
  double *b = bf;
  for (int s2 = 0; s2 < (level > 0 ? 2 : 1); ++s2) {
    int ns = n[s2], nts = 3 * (ns - 1) + 1;
    size_t Ns = (size_t)nts * nts * nts, N = (size_t)ns * ns * ns;
    if (s2 == 1) {
      double *bc = (double *)malloc(sizeof(double) * Ns);
      or_spde_restrict(nt, bf, bc);
      b = bc;
    }
    double *z = (double *)malloc(sizeof(double) * Ns);
    double h = 1.0 / (double)(ns - 1);
    int st1 = or_spde_solve(nts, h, 1.0 / lambda, b, z, 2, 2, spde_tol, 50, &sc[s2], NULL);
    double *k = (double *)malloc(sizeof(double) * N), *bb = (double *)malloc(sizeof(double) * N);
    double *u = (double *)calloc(N, sizeof(double));
    or_spde_to_k(ns, sigma2, lambda, z, k);
    for (size_t p = 0; p < N; ++p) bb[p] = h * h;
    int st2 = or_solve(ns, k, bb, u, nu1, nu2, tol, max_cycles, 0, &cyc[s2], NULL, NULL);
    q[s2] = or_qoi(ns, u);
    if (!st) st = st1 ? st1 : st2;
    free(z); free(k); free(bb); free(u);
    if (s2 == 1) free(b);
  }
  free(bf);
  if (Qf) *Qf = q[0];
  if (Qc) *Qc = q[1];
  if (Y) *Y = q[0] - q[1];
  if (cycles) { cycles[0] = cyc[0]; cycles[1] = cyc[1]; }
  if (spde_cycles) { spde_cycles[0] = sc[0]; spde_cycles[1] = sc[1]; }
  return st;
}

/* ------------------------------------------------------------------------ */
/* Level accumulator: shift K = first Y; compensated sums of (Y-K) and       */
/* (Y-K)^2; mean = K + S1/N, s^2 = S2/N - (S1/N)^2 (divisor N as in the      */
/* paper's estimator of V[Y_l]).                                            */
/* ------------------------------------------------------------------------ */
void or_acc_init(or_level_acc *a) { memset(a, 0, sizeof(*a)); }

static void neumaier_add(double *s, double *c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
  else *c += (x - t) + *s;
  *s = t;
}

void or_acc_add(or_level_acc *a, double y) {
  if (a->n == 0) a->shift = y;
  double d = y - a->shift;
  neumaier_add(&a->s1, &a->c1, d);
  neumaier_add(&a->s2, &a->c2, d * d);
  a->n += 1;
}

void or_acc_result(const or_level_acc *a, double *mean, double *var) {
  if (a->n == 0) { *mean = 0.0; *var = 0.0; return; }
  double N = (double)a->n;
  double m1 = (a->s1 + a->c1) / N;
  *mean = a->shift + m1;
  *var = (a->s2 + a->c2) / N - m1 * m1;
}
