/*
 * Plain FP64 CPU oracle for the per-sample hot path of multilevel Monte
 * Carlo (Gmeiner, Drzisga, Ruede, Scheichl, Wohlmuth, "Scheduling massively
 * parallel multigrid for multilevel Monte Carlo methods", arXiv 1607.03252).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library under paper_1607_03252_amd/) shares no code with it.
 *
 * Storage convention: an n x n x n vertex grid on [0,1]^3, n = 2^m + 1,
 * h = 1/(n-1), vertex (i,j,k) at (i h, j h, k h), stored at (i*n + j)*n + k
 * (k, the z index, fastest).  Boundary vertices carry the homogeneous
 * Dirichlet value 0 for u and are ignored for b.
 *
 * All functions return 0 on success and a negative code on bad arguments.
 */
#ifndef MLMC_ORACLE_H
#define MLMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOCONV = -3 };

/* Philox4x32-10 block: ctr[4], key[2] -> out[4]. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The 128 words of sample (seed, level): block j uses ctr = (j, level, 0, 0). */
void or_philox_words(uint64_t seed, uint32_t level, uint32_t out[128]);
/* 64 integers M_m in [0, 2^53) built from the words. */
void or_uniform_ints(uint64_t seed, uint32_t level, uint64_t out[64]);
/* 64 standard normals xi_m (Box-Muller on U = (M+1) 2^-53). */
void or_gaussians(uint64_t seed, uint32_t level, double xi[64]);

/* 1D KL eigenpairs of exp(-|s-t|/lambda) on [0,1]: roots omega[m] and
 * eigenvalues theta[m] for m = 0..nterms-1, normalisation constants norm[m]. */
int or_kl_1d(double lambda, int nterms, double *omega, double *theta, double *norm);
/* phi_m(s) for one mode. */
double or_kl_phi(double lambda, double omega, double norm, double s);
/* k = exp(Z) at all n^3 vertices for the given 64 normals (4x4x4 block). */
int or_field(int n, double sigma2, double lambda, const double xi[64], double *k);

/* A' u = h^2 A u on interior vertices (boundary of out set to 0). */
int or_apply(int n, const double *k, const double *u, double *out);
/* r' = b' - A' u on interior vertices, 0 on the boundary. */
int or_residual(int n, const double *k, const double *b, const double *u, double *r);
/* One red-black Gauss-Seidel sweep (red then black), in place. */
int or_rbgs_sweep(int n, const double *k, const double *b, double *u);
/* Full-weighting restriction of an h^2-scaled fine residual to an
 * h_c^2-scaled coarse right-hand side (includes the factor 4). */
int or_restrict(int n_fine, const double *r, double *bc);
/* u_fine += P e_coarse (trilinear). */
int or_prolong_add(int n_coarse, const double *ec, double *uf);
/* Coarse vertex coefficient by injection k_c(I) = k_f(2I). */
int or_inject(int n_fine, const double *kf, double *kc);
/* One V(nu1,nu2) cycle on the hierarchy rooted at n (scratch allocated inside). */
int or_vcycle(int n, const double *k, const double *b, double *u, int nu1, int nu2);
/* Euclidean norm over interior vertices (compensated sum of squares). */
double or_norm2(int n, const double *v);
/* Solve A'u = b' from the given u.  fixed_cycles > 0 runs exactly that many
 * cycles; otherwise stops at the first cycle with relres <= tol.
 * hist (optional, length >= max_cycles) receives relres after each cycle. */
int or_solve(int n, const double *k, const double *b, double *u, int nu1, int nu2,
             double tol, int max_cycles, int fixed_cycles,
             int *cycles, double *relres, double *hist);
/* Q = h^3 * sum of u over interior vertices (compensated). */
double or_qoi(int n, const double *u);

/* Point QoI u(1/4, 1/4, 1/4) (n = 4m + 1). */
double or_point_qoi(int n, const double *u);
/* Flux of -k grad u in +x_2 across the plane x_2 = 1/4 (n = 4m + 1). */
double or_flux_qoi(int n, const double *k, const double *u);
/* Full multigrid: exact 3^3 solve, then on each finer grid trilinear
 * interpolation of the coarser result and ncycles V(nu1,nu2) cycles. */
int or_fmg(int n, const double *k, const double *f, double *u, int nu1, int nu2, int ncycles);

/* One MLMC sample Y_level = Q(n_level) - Q(n_level-1) (Y_0 = Q(n_0)), with
 * n_level = (n0-1) 2^level + 1, f = 1, u0 = 0, both solves from the same
 * normals xi(seed, level).  Qc = 0 and cycles[1] = 0 for level 0. */
int or_mlmc_sample(int n0, int level, uint64_t seed, double sigma2, double lambda,
                   int nu1, int nu2, double tol, int max_cycles, int fixed_cycles,
                   double *Y, double *Qf, double *Qc, int cycles[2]);

/* As or_mlmc_sample with a solver (0 = V-cycles to tol, 1 = FMG with
 * fmg_cycles V(nu1,nu2) cycles per grid) and a QoI (0 = integral of u,
 * 1 = u(1/4,1/4,1/4), 2 = flux across x_2 = 1/4). */
int or_mlmc_sample_ex(int n0, int level, uint64_t seed, double sigma2, double lambda,
                      int nu1, int nu2, int solver, int fmg_cycles, int qoi, double tol,
                      int max_cycles, int fixed_cycles, double *Y, double *Qf, double *Qc,
                      int cycles[2]);

/* P1 finite elements on the Kuhn triangulation of the vertex grid, the
 * tetrahedron's coefficient the mean of its four vertex values, scaled by 1/h
 * (so A'u = h^2 f as in the FD form).  S: 27 couplings per vertex,
 * S[27 p + (di+1)*9 + (dj+1)*3 + (dk+1)]. */
int or_fe_stencil(int n, const double *k, double *S);
int or_fe_apply(int n, const double *k, const double *u, double *out);
int or_fe_solve(int n, const double *k, const double *b, double *u, int nu1, int nu2,
                double tol, int max_cycles, int fixed_cycles, int *cycles, double *relres);
int or_mlmc_sample_fe(int n0, int level, uint64_t seed, double sigma2, double lambda, int nu1,
                      int nu2, int qoi, double tol, int max_cycles, int fixed_cycles, double *Y,
                      double *Qf, double *Qc, int cycles[2]);

/* SPDE sampler (Section 3.2): white noise, the box operator (stiffness
 * S[27 p + t] and lumped mass m_p), restriction b_c = P^T b_f / 2 and
 * prolongation on box grids, the V-cycle solve, the scaled load, the field
 * on D, and an MLMC sample with the SPDE field. */
void or_white_noise(uint64_t seed, uint32_t level, long count, double *xi);
int or_spde_operator(int nt, double *S, double *m);
int or_spde_restrict(int nt, const double *r, double *bc);
int or_spde_prolong_add(int ntc, const double *zc, double *zf);
int or_spde_solve(int nt, double h, double kappa, const double *b, double *z, int nu1, int nu2,
                  double tol, int max_cycles, int *cycles, double *relres);
int or_spde_rhs(int n, const double *xi, double *b);
int or_spde_to_k(int n, double sigma2, double lambda, const double *z, double *k);
int or_mlmc_sample_spde(int n0, int level, uint64_t seed, double sigma2, double lambda, int nu1,
                        int nu2, double tol, int max_cycles, double spde_tol, double *Y,
                        double *Qf, double *Qc, int cycles[2], int spde_cycles[2]);

/* Compensated (Neumaier) summation of a vector. */
double or_sum(const double *x, long n);

/* Shifted, compensated level accumulator. */
typedef struct {
  long   n;
  double shift;
  double s1, c1, s2, c2;
} or_level_acc;
void or_acc_init(or_level_acc *a);
void or_acc_add(or_level_acc *a, double y);
/* mean = shift + S1/N ; var = S2/N - (S1/N)^2 (divisor N). */
void or_acc_result(const or_level_acc *a, double *mean, double *var);

#ifdef __cplusplus
}
#endif
#endif
