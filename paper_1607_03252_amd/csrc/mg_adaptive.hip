// Adaptive multilevel Monte Carlo (Section 2.3, Algorithm 2) over the batched
// sample path: each round computes the missing samples of every level with
// mlmc_sample_mixed (all levels in the same batches), updates the level
// statistics, the sample numbers of eq. (quasioptimal_Nl) and the finest
// level by the bias estimate of eq. (bias_estimate).
//
// Readings: N_l never drops below the samples already taken (new N_l =
// max(N_l, ceil(eq. quasioptimal_Nl))); the bias test uses |Yhat_L|; C_l is
// the mean work of a sample of Y_l in node-cycles (vertices of each grid
// times its V-cycles), measured from the samples' cycle counts; only ratios
// of the C_l enter eq. (quasioptimal_Nl), and for these bandwidth-bound
// solves the work is proportional to the run time.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mlmcmg.h"

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

void mlmc_adaptive_desc_default(mlmc_adaptive_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->eps = 1e-3;
  d->theta = 0.5;
  d->alpha = 2.0 / 3.0;
  d->n_init = 32;
  d->max_iter = 64;
  d->max_batch = 256;
  d->seed0 = 0;
}

int mlmc_adaptive(mg_plan plan, const mlmc_adaptive_desc* d, mlmc_adaptive_result* r) {
  if (!plan || !d || !r) return MG_EINVAL;
  if (!(d->eps > 0.0) || !(d->theta > 0.0 && d->theta < 1.0) || !(d->alpha > 0.0) ||
      d->n_init < 2 || d->max_iter < 1 || d->max_batch < 1)
    return MG_EINVAL;
  mg_plan_desc pd;
  if (mg_plan_get_desc(plan, &pd) != MG_OK) return MG_EINVAL;
  if (pd.max_level < 1 || pd.max_level >= MLMC_MAX_LEVELS) return MG_EINVAL;
  std::memset(r, 0, sizeof(*r));

  const double eps_s2 = d->theta * d->eps * d->eps;
  const double eps_b = std::sqrt((1.0 - d->theta) * d->eps * d->eps);
  const double bias_factor = std::pow(8.0, d->alpha) - 1.0;
  const int B = d->max_batch;
  DevBuf dY, dC;
  if (hipMalloc(&dY.p, sizeof(double) * B) != hipSuccess ||
      hipMalloc(&dC.p, sizeof(int) * 2 * B) != hipSuccess)
    return MG_ENOMEM;
  std::vector<double> hY(B);
  std::vector<int> hC(2 * B);

  int L = 1;
  std::vector<long long> N = {d->n_init, d->n_init};
  std::vector<mlmc_level_acc> acc;
  std::vector<double> work;
  std::vector<long long> done;
  auto n_of = [&](int l) { return (double)((pd.n0 - 1) * (1 << l) + 1); };

  int it = 0;
  for (;;) {
    ++it;
    while ((int)acc.size() < L + 1) {
      mlmc_level_acc a;
      mlmc_acc_init(&a);
      acc.push_back(a);
      work.push_back(0.0);
      done.push_back(0);
    }
    // step 2a: the missing samples of every level, level by level in seed order
    std::vector<int> lv;
    std::vector<uint64_t> sd;
    for (int l = 0; l <= L; ++l)
      for (long long i = done[l]; i < N[l]; ++i) {
        lv.push_back(l);
        sd.push_back(d->seed0 + (uint64_t)i);
      }
    for (size_t c0 = 0; c0 < lv.size(); c0 += (size_t)B) {
      const int m = (int)std::min<size_t>((size_t)B, lv.size() - c0);
      const int st = mlmc_sample_mixed(plan, lv.data() + c0, sd.data() + c0, m, (double*)dY.p,
                                       nullptr, nullptr, (int*)dC.p, 0);
      if (st != MG_OK) return st;
      if (hipMemcpy(hY.data(), dY.p, sizeof(double) * m, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(hC.data(), dC.p, sizeof(int) * 2 * m, hipMemcpyDeviceToHost) != hipSuccess)
        return MG_EHIP;
      for (int q = 0; q < m; ++q) {
        const int l = lv[c0 + q];
        mlmc_acc_add(&acc[l], &hY[q], 1, 0);
        double w = n_of(l) * n_of(l) * n_of(l) * (double)hC[2 * q];
        if (l > 0) w += n_of(l - 1) * n_of(l - 1) * n_of(l - 1) * (double)hC[2 * q + 1];
        work[l] += w;
        done[l] += 1;
      }
    }
    // step 2b: level means, s_l^2 (divisor N) and costs
    std::vector<double> mean(L + 1), var(L + 1), cost(L + 1);
    for (int l = 0; l <= L; ++l) {
      mlmc_acc_result(&acc[l], &mean[l], &var[l]);
      cost[l] = work[l] / (double)done[l];
    }
    // step 3: eq. (quasioptimal_Nl) and the bias test of eq. (bias_estimate)
    double tot = 0.0;
    for (int l = 0; l <= L; ++l) tot += std::sqrt(var[l] * cost[l]);
    bool changed = false;
    for (int l = 0; l <= L; ++l) {
      const long long q =
          var[l] > 0.0 ? (long long)std::ceil(tot * std::sqrt(var[l] / cost[l]) / eps_s2) : 0;
      if (q > N[l]) {
        N[l] = q;
        changed = true;
      }
    }
    if (std::fabs(mean[L]) > bias_factor * eps_b && L < pd.max_level) {
      ++L;
      N.push_back(d->n_init);
      changed = true;
    }
    if (r->trace_len < MLMC_MAX_TRACE) {
      r->trace_L[r->trace_len] = L;
      for (int l = 0; l <= L; ++l) r->trace_N[r->trace_len][l] = N[l];
      r->trace_len += 1;
    }
    // step 4
    if (!changed || it >= d->max_iter) break;
  }
  // step 5
  r->L = L;
  r->iterations = it;
  double q = 0.0, c = 0.0, s = 0.0;
  for (int l = 0; l <= L; ++l) {
    double m, v;
    mlmc_acc_result(&acc[l], &m, &v);
    r->N[l] = N[l];
    r->mean[l] = m;
    r->var[l] = v;
    r->cost[l] = work[l] / (double)done[l];
    // Neumaier sum of the level means
    const double t = q + m;
    c += std::fabs(q) >= std::fabs(m) ? (q - t) + m : (m - t) + q;
    q = t;
    s += v / (double)N[l];
  }
  r->Q = q + c;
  r->sampling_rms = std::sqrt(s);
  r->bias_estimate = std::fabs(r->mean[L]) / bias_factor;
  r->bias_ok = r->bias_estimate <= eps_b;
  r->status = MG_OK;
  return MG_OK;
}

}  // extern "C"
