// Plan, batch workspace, batched V-cycle driver and the C ABI of libmlmcmg.
//
// A batch is a set of solves (one per grid of an MLMC sample: the level-l
// solve and, for l > 0, the level-(l-1) solve of the same omega).  Every
// multigrid level of every solve gets its own buffers; all grids of one size
// form one device list, so each step of the V-cycle is one launch for the
// whole batch.  Grids of different top sizes nest: a solve with a smaller top
// grid starts its cycle when the larger ones reach its size (the cycles are
// aligned at the coarsest grid), so every launch sees grids of one size only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mlmcmg.h"
#include "mg_internal.h"
#include "mg_kl.h"

namespace mg {

struct HipError {
  hipError_t e;
  const char* what;
};

#define CK(x)                                   \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) throw HipError{e_, #x}; \
  } while (0)

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Level {
  int n = 0;
  double* u[2] = {nullptr, nullptr};
  double* wh = nullptr;
  double* b = nullptr;
  double* r = nullptr;
};

struct BatchSpec {
  std::vector<int> top_n;   // top grid size of each solve
  std::vector<int> share;   // solve whose levels 1.. supply this solve's wh (or -1)
  bool const_b_top = true;  // top right-hand side is the constant h^2 (f = 1)
  bool ext_u_top = false;   // top u is caller memory (mg_solve)
  std::string key() const {
    std::string s = const_b_top ? "c" : "v";
    s += ext_u_top ? "e" : "i";
    for (size_t i = 0; i < top_n.size(); ++i) s += ":" + std::to_string(top_n[i]) + "/" + std::to_string(share[i]);
    return s;
  }
};

struct Batch {
  BatchSpec spec;
  int ns = 0;
  std::vector<std::vector<Level>> lev;  // [solve][mg level]
  std::vector<int> sizes;               // distinct grid sizes, descending (ends with 3)
  std::vector<std::vector<GridDesc>> h_lists;
  std::vector<GridDesc*> d_lists;
  std::vector<int> top_sizes;           // distinct top sizes
  std::vector<std::vector<GridDesc>> h_top;
  std::vector<GridDesc*> d_top;
  SolveState ss{};
  int* d_count = nullptr;
  int* h_count = nullptr;               // pinned
  // MLMC sample plumbing
  int nsamples = 0;
  uint64_t* d_seeds = nullptr;
  double* d_normals = nullptr;
  int* d_fi = nullptr;
  int* d_ci = nullptr;
  double** d_field_out = nullptr;       // top wh of the solves that own a field
  int* d_xi_index = nullptr;
  int field_count = 0;
  int field_n = 0;
  // coefficient injection, per fine size (descending): pointer lists of the
  // grids that own their wh and of their coarse children
  std::vector<double**> d_inj_src, d_inj_dst;
  std::vector<int> inj_n, inj_count;
  void* mem = nullptr;
  size_t bytes = 0;
  std::vector<void*> extra;  // small device allocations owned by the batch
  void* dalloc(size_t bytes) {
    void* p = nullptr;
    CK(hipMalloc(&p, bytes));
    extra.push_back(p);
    return p;
  }
  ~Batch() {
    for (void* p : extra) (void)hipFree(p);
    if (mem) (void)hipFree(mem);
    if (h_count) (void)hipHostFree(h_count);
  }
};

static std::vector<int> hierarchy(int n) {
  std::vector<int> v;
  for (int m = n; m >= 3; m = (m - 1) / 2 + 1) {
    v.push_back(m);
    if (m == 3) break;
  }
  return v;
}

static bool valid_n(int n) {
  if (n < 3) return false;
  const int m = n - 1;
  return (m & (m - 1)) == 0;
}

}  // namespace mg

using namespace mg;

struct mg_plan_s {
  mg_plan_desc desc{};
  hipStream_t stream = nullptr;
  std::string err;
  double omega[4]{}, theta[4]{}, scale[4]{};
  double* d_coef = nullptr;
  std::map<int, double*> d_phi;
  std::unique_ptr<Batch> batch;
  std::string batch_key;
  // profiling of the finest-grid smoothing launches
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  long long prof_launches = 0;
  double prof_ms = 0.0;
  double prof_nodes = 0.0;
  // mg_solve workspace for the caller's problem
  double* s_wh = nullptr;
  double* s_b = nullptr;
  int s_n = 0;

  ~mg_plan_s() {
    batch.reset();
    for (auto& kv : d_phi) (void)hipFree(kv.second);
    if (d_coef) (void)hipFree(d_coef);
    if (s_wh) (void)hipFree(s_wh);
    if (s_b) (void)hipFree(s_b);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace mg {

static const double* phi_table(mg_plan_s* P, int n) {
  auto it = P->d_phi.find(n);
  if (it != P->d_phi.end()) return it->second;
  std::vector<double> t(4 * (size_t)n);
  kl_phi_table(P->desc.corr_len, 4, P->omega, P->scale, n, t.data());
  double* d = nullptr;
  CK(hipMalloc(&d, t.size() * sizeof(double)));
  CK(hipMemcpy(d, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
  P->d_phi[n] = d;
  return d;
}

// Allocate and describe a batch.  One device allocation holds every buffer.
static std::unique_ptr<Batch> build_batch(mg_plan_s* P, const BatchSpec& spec) {
  auto B = std::make_unique<Batch>();
  B->spec = spec;
  const int ns = (int)spec.top_n.size();
  B->ns = ns;
  B->lev.resize(ns);
  // pass 1: sizes
  size_t total = 0;
  auto add = [&](size_t bytes) { total += align256(bytes); };
  for (int s = 0; s < ns; ++s) {
    const auto h = hierarchy(spec.top_n[s]);
    for (size_t j = 0; j < h.size(); ++j) {
      const size_t N = (size_t)h[j] * h[j] * h[j] * sizeof(double);
      if (!(j == 0 && spec.ext_u_top)) add(N);        // u0
      if (spec.share[s] < 0) add(N);                  // wh
      if (!(j == 0 && spec.const_b_top)) add(N);      // b
      if (h[j] > 3) add(N);                           // r
    }
  }
  int npart = 0;
  for (int s = 0; s < ns; ++s) npart += reduce_blocks(spec.top_n[s]);
  add(sizeof(int) * ns * 2);      // active, cycles
  add(sizeof(double) * ns * 3);   // relres, bnorm, q
  add(sizeof(double) * npart);
  add(sizeof(int));               // count
  if (P->desc.hbm_budget && total > P->desc.hbm_budget) return nullptr;
  CK(hipMalloc(&B->mem, total));
  CK(hipMemsetAsync(B->mem, 0, total, P->stream));
  B->bytes = total;
  char* cur = (char*)B->mem;
  auto take = [&](size_t bytes) {
    void* p = cur;
    cur += align256(bytes);
    return p;
  };
  // pass 2: carve (solves whose wh is shared must come after their parent)
  for (int s = 0; s < ns; ++s) {
    const auto h = hierarchy(spec.top_n[s]);
    B->lev[s].resize(h.size());
    for (size_t j = 0; j < h.size(); ++j) {
      Level& L = B->lev[s][j];
      L.n = h[j];
      const size_t N = (size_t)h[j] * h[j] * h[j] * sizeof(double);
      if (!(j == 0 && spec.ext_u_top)) L.u[0] = (double*)take(N);
      if (spec.share[s] < 0) L.wh = (double*)take(N);
      else L.wh = B->lev[spec.share[s]][j + 1].wh;
      if (!(j == 0 && spec.const_b_top)) L.b = (double*)take(N);
      if (h[j] > 3) L.r = (double*)take(N);
    }
  }
  B->ss.active = (int*)take(sizeof(int) * ns * 2);
  B->ss.cycles = B->ss.active + ns;
  double* dd = (double*)take(sizeof(double) * ns * 3);
  B->ss.relres = dd;
  B->ss.bnorm = dd + ns;
  B->ss.q = dd + 2 * ns;
  B->ss.partials = (double*)take(sizeof(double) * npart);
  B->d_count = (int*)take(sizeof(int));
  CK(hipHostMalloc((void**)&B->h_count, sizeof(int), hipHostMallocDefault));
  // lists per size
  int nmax = 0;
  for (int n : spec.top_n) nmax = std::max(nmax, n);
  B->sizes = hierarchy(nmax);
  B->h_lists.assign(B->sizes.size(), {});
  for (int s = 0; s < ns; ++s) {
    for (auto& L : B->lev[s]) {
      const size_t si = std::find(B->sizes.begin(), B->sizes.end(), L.n) - B->sizes.begin();
      B->h_lists[si].push_back(GridDesc{});
    }
  }
  // top groups
  for (int s = 0; s < ns; ++s)
    if (std::find(B->top_sizes.begin(), B->top_sizes.end(), spec.top_n[s]) == B->top_sizes.end())
      B->top_sizes.push_back(spec.top_n[s]);
  std::sort(B->top_sizes.begin(), B->top_sizes.end(), std::greater<int>());
  B->h_top.assign(B->top_sizes.size(), {});
  return B;
}

// (Re)write the device descriptor lists from the current buffers.
static void upload_lists(mg_plan_s* P, Batch* B) {
  const auto& spec = B->spec;
  for (auto& v : B->h_lists) v.clear();
  for (auto& v : B->h_top) v.clear();
  int poff = 0;
  std::vector<int> poffs(B->ns);
  for (int s = 0; s < B->ns; ++s) {
    poffs[s] = poff;
    poff += reduce_blocks(spec.top_n[s]);
  }
  for (int s = 0; s < B->ns; ++s) {
    auto& lv = B->lev[s];
    for (size_t j = 0; j < lv.size(); ++j) {
      const Level& L = lv[j];
      GridDesc d{};
      d.u[0] = L.u[0];
      d.u[1] = L.u[1];
      d.wh = L.wh;
      d.b = L.b;
      d.r = L.r;
      if (j + 1 < lv.size()) {
        d.uc = lv[j + 1].u[0];
        d.bc = lv[j + 1].b;
      }
      const double h = 1.0 / (double)(L.n - 1);
      d.bconst = h * h;  // f = 1
      d.solve = s;
      d.n = L.n;
      d.poff = (j == 0) ? poffs[s] : 0;
      const size_t si = std::find(B->sizes.begin(), B->sizes.end(), L.n) - B->sizes.begin();
      B->h_lists[si].push_back(d);
      if (j == 0) {
        const size_t ti =
            std::find(B->top_sizes.begin(), B->top_sizes.end(), L.n) - B->top_sizes.begin();
        B->h_top[ti].push_back(d);
      }
    }
  }
  // one device block for all lists (kept inside the batch allocation would
  // complicate sizing; a separate small allocation is made once)
  size_t cnt = 0;
  for (auto& v : B->h_lists) cnt += v.size();
  for (auto& v : B->h_top) cnt += v.size();
  if (B->d_lists.empty()) {
    GridDesc* base = (GridDesc*)B->dalloc(sizeof(GridDesc) * cnt);
    size_t off = 0;
    for (auto& v : B->h_lists) { B->d_lists.push_back(base + off); off += v.size(); }
    for (auto& v : B->h_top) { B->d_top.push_back(base + off); off += v.size(); }
    // injection lists: every grid that owns its wh feeds its coarse child
    for (size_t si = 0; si + 1 < B->sizes.size(); ++si) {
      std::vector<double*> src, dst;
      for (int s = 0; s < B->ns; ++s) {
        if (spec.share[s] >= 0) continue;
        const auto& lv = B->lev[s];
        for (size_t j = 0; j + 1 < lv.size(); ++j)
          if (lv[j].n == B->sizes[si]) {
            src.push_back(lv[j].wh);
            dst.push_back(lv[j + 1].wh);
          }
      }
      if (src.empty()) continue;
      double** ds = (double**)B->dalloc(sizeof(double*) * src.size());
      double** dd = (double**)B->dalloc(sizeof(double*) * dst.size());
      CK(hipMemcpy(ds, src.data(), sizeof(double*) * src.size(), hipMemcpyHostToDevice));
      CK(hipMemcpy(dd, dst.data(), sizeof(double*) * dst.size(), hipMemcpyHostToDevice));
      B->d_inj_src.push_back(ds);
      B->d_inj_dst.push_back(dd);
      B->inj_n.push_back(B->sizes[si]);
      B->inj_count.push_back((int)src.size());
    }
  }
  for (size_t i = 0; i < B->h_lists.size(); ++i)
    CK(hipMemcpyAsync(B->d_lists[i], B->h_lists[i].data(), sizeof(GridDesc) * B->h_lists[i].size(),
                      hipMemcpyHostToDevice, P->stream));
  for (size_t i = 0; i < B->h_top.size(); ++i)
    CK(hipMemcpyAsync(B->d_top[i], B->h_top[i].data(), sizeof(GridDesc) * B->h_top[i].size(),
                      hipMemcpyHostToDevice, P->stream));
  CK(hipStreamSynchronize(P->stream));
}

// Coarse-grid coefficients by injection, finest size first.
static void inject_all(mg_plan_s* P, Batch* B) {
  for (size_t j = 0; j < B->inj_n.size(); ++j)
    launch_inject(B->inj_n[j], B->inj_count[j], (const double* const*)B->d_inj_src[j],
                  B->d_inj_dst[j], P->stream);
}

static hipEvent_t next_event(mg_plan_s* P) {
  if (P->ev_used == P->ev_pool.size()) {
    hipEvent_t e;
    CK(hipEventCreate(&e));
    P->ev_pool.push_back(e);
  }
  return P->ev_pool[P->ev_used++];
}

static void collect_profile(mg_plan_s* P) {
  if (P->ev_used == 0) return;
  CK(hipStreamSynchronize(P->stream));
  for (size_t i = 0; i + 1 < P->ev_used; i += 2) {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, P->ev_pool[i], P->ev_pool[i + 1]));
    P->prof_ms += ms;
    P->prof_launches += 1;
  }
  P->ev_used = 0;
}

static void smooth(mg_plan_s* P, Batch* B, size_t si, int sweeps) {
  const int n = B->sizes[si];
  const int cnt = (int)B->h_lists[si].size();
  const bool timed = P->prof && si == 0;
  for (int s = 0; s < sweeps; ++s) {
    for (int colour = 0; colour < 2; ++colour) {
      if (timed) {
        if (P->ev_used + 2 > 4096) collect_profile(P);
        CK(hipEventRecord(next_event(P), P->stream));
      }
      launch_rbgs_colour(B->d_lists[si], cnt, n, B->ss.active, colour, 0, P->stream);
      if (timed) {
        CK(hipEventRecord(next_event(P), P->stream));
        P->prof_nodes = (double)cnt * (double)(n - 2) * (n - 2) * (n - 2);
      }
    }
  }
}

// One V(nu1,nu2) cycle for every active solve of the batch.
static void run_cycle(mg_plan_s* P, Batch* B) {
  const int nu1 = P->desc.nu1, nu2 = P->desc.nu2;
  const size_t L = B->sizes.size();
  hipStream_t st = P->stream;
  for (size_t si = 0; si < L; ++si) {
    const int n = B->sizes[si];
    const int cnt = (int)B->h_lists[si].size();
    if (n == 3) {
      launch_coarsest(B->d_lists[si], cnt, B->ss.active, st);
      continue;
    }
    smooth(P, B, si, nu1);
    launch_residual(B->d_lists[si], cnt, n, B->ss.active, 0, st);
    launch_restrict(B->d_lists[si], cnt, n, B->ss.active, st);
  }
  for (size_t si = L - 1; si-- > 0;) {
    const int n = B->sizes[si];
    const int cnt = (int)B->h_lists[si].size();
    launch_prolong(B->d_lists[si], cnt, n, B->ss.active, 0, st);
    smooth(P, B, si, nu2);
  }
}

static void reduce_tops(mg_plan_s* P, Batch* B, int mode, int cycle, int fixed, double tol) {
  for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
    const int n = B->top_sizes[ti];
    const int cnt = (int)B->h_top[ti].size();
    launch_reduce(B->d_top[ti], cnt, n, B->ss.active, 0, mode, B->ss.partials, P->stream);
    launch_finalize(B->d_top[ti], cnt, n, B->ss, mode, cycle, fixed, P->desc.max_cycles, tol,
                    P->stream);
  }
}

void launch_init_state(int* active, int* cycles, int ns, hipStream_t st);

// Cycle all solves of the batch until each has converged (or run exactly
// fixed_cycles).  Returns true when every solve met tol.
static bool run_solves(mg_plan_s* P, Batch* B, double tol, int fixed_cycles) {
  hipStream_t st = P->stream;
  launch_init_state(B->ss.active, B->ss.cycles, B->ns, st);
  reduce_tops(P, B, RED_BNORM, 0, fixed_cycles, tol);
  const int limit = fixed_cycles > 0 ? fixed_cycles : P->desc.max_cycles;
  for (int m = 1; m <= limit; ++m) {
    run_cycle(P, B);
    reduce_tops(P, B, RED_RESID, m, fixed_cycles, tol);
    launch_count_active(B->ss.active, B->ns, B->d_count, st);
    CK(hipMemcpyAsync(B->h_count, B->d_count, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (*B->h_count == 0) break;
  }
  std::vector<int> cyc(B->ns);
  CK(hipMemcpyAsync(cyc.data(), B->ss.cycles, sizeof(int) * B->ns, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  for (int c : cyc)
    if (c <= 0) return false;
  return true;
}

static Batch* get_batch(mg_plan_s* P, const BatchSpec& spec, int* status) {
  const std::string key = spec.key();
  if (!P->batch || P->batch_key != key) {
    P->batch.reset();
    P->batch_key.clear();
    auto B = build_batch(P, spec);
    if (!B) {
      *status = MG_ENOMEM;
      P->err = "batch workspace exceeds the plan's HBM budget";
      return nullptr;
    }
    P->batch = std::move(B);
    P->batch_key = key;
  }
  return P->batch.get();
}

}  // namespace mg

// ============================== C ABI ==========================================

#define API_BEGIN try {
#define API_END(P)                                                                    \
  }                                                                                   \
  catch (const mg::HipError& he) {                                                    \
    if (P) P->err = std::string(he.what) + ": " + hipGetErrorString(he.e);            \
    return MG_EHIP;                                                                   \
  }                                                                                   \
  catch (const std::bad_alloc&) {                                                     \
    if (P) P->err = "host allocation failed";                                         \
    return MG_ENOMEM;                                                                 \
  }                                                                                   \
  catch (...) {                                                                       \
    if (P) P->err = "unexpected error";                                               \
    return MG_EHIP;                                                                   \
  }

extern "C" {

void mg_plan_desc_default(mg_plan_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->n0 = 33;
  d->max_level = 0;
  d->nu1 = 2;
  d->nu2 = 2;
  d->max_cycles = 50;
  d->tol = 1e-8;
  d->precision = MG_FP64;
  d->sigma2 = 1.0;
  d->corr_len = 0.1;
  d->kl_per_axis = 4;
  d->hbm_budget = 0;
  d->stream = nullptr;
}

int mg_plan_create(const mg_plan_desc* desc, mg_plan* out) {
  if (!desc || !out) return MG_EINVAL;
  *out = nullptr;
  if (!valid_n(desc->n0) || desc->max_level < 0 || desc->max_level > 10 || desc->nu1 < 0 ||
      desc->nu2 < 0 || desc->nu1 + desc->nu2 < 1 || desc->max_cycles < 1 || !(desc->tol > 0.0) ||
      !(desc->sigma2 >= 0.0) || !(desc->corr_len > 0.0) ||
      (desc->precision != MG_FP64 && desc->precision != MG_MIXED))
    return MG_EINVAL;
  if (desc->kl_per_axis != 4) return MG_ENOTIMPL;
  if ((long long)(desc->n0 - 1) * (1ll << desc->max_level) + 1 > 2049) return MG_EINVAL;
  mg_plan_s* P = new (std::nothrow) mg_plan_s();
  if (!P) return MG_ENOMEM;
  P->desc = *desc;
  P->stream = (hipStream_t)desc->stream;
  try {
    if (!kl_1d_modes(desc->corr_len, 4, P->omega, P->theta, P->scale)) {
      delete P;
      return MG_EINVAL;
    }
    double coef[64];
    const double sigma = std::sqrt(desc->sigma2);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c)
          coef[16 * a + 4 * b + c] = sigma * std::sqrt(P->theta[a] * P->theta[b] * P->theta[c]);
    CK(hipMalloc(&P->d_coef, sizeof(coef)));
    CK(hipMemcpy(P->d_coef, coef, sizeof(coef), hipMemcpyHostToDevice));
    for (int l = 0; l <= desc->max_level; ++l) phi_table(P, (desc->n0 - 1) * (1 << l) + 1);
  } catch (const HipError& he) {
    delete P;
    return MG_EHIP;
  }
  *out = P;
  return MG_OK;
}

int mg_plan_destroy(mg_plan P) {
  if (!P) return MG_EINVAL;
  (void)hipStreamSynchronize(P->stream);
  delete P;
  return MG_OK;
}

int mg_plan_set_stream(mg_plan P, void* stream) {
  if (!P) return MG_EINVAL;
  P->stream = (hipStream_t)stream;
  return MG_OK;
}

const char* mg_last_error(mg_plan P) { return P ? P->err.c_str() : "null plan"; }

int mg_solve(mg_plan P, int n, const double* k, const double* f, double* u, double tol,
             int fixed_cycles, int* cycles, double* relres) {
  if (!P) return MG_EINVAL;
  if (!valid_n(n) || !k || !f || !u || fixed_cycles < 0) {
    P->err = "mg_solve: n must be 2^m+1 (m>=1) and k, f, u non-null";
    return MG_EINVAL;
  }
  if (n > 1025) {
    P->err = "mg_solve: n > 1025 is not supported";
    return MG_EINVAL;
  }
  API_BEGIN
  const double t = tol > 0.0 ? tol : P->desc.tol;
  BatchSpec spec;
  spec.top_n = {n};
  spec.share = {-1};
  spec.const_b_top = false;
  spec.ext_u_top = true;
  int status = MG_OK;
  Batch* B = get_batch(P, spec, &status);
  if (!B) return status;
  // the caller's u is the top iterate; wh and b of the top grid live in the batch
  B->lev[0][0].u[0] = u;
  upload_lists(P, B);
  const Level& T = B->lev[0][0];
  launch_prepare_problem(n, k, f, T.wh, T.b, u, P->stream);
  inject_all(P, B);
  const bool ok = run_solves(P, B, t, fixed_cycles);
  int cyc = 0;
  double rel = 0.0;
  CK(hipMemcpy(&cyc, B->ss.cycles, sizeof(int), hipMemcpyDeviceToHost));
  CK(hipMemcpy(&rel, B->ss.relres, sizeof(double), hipMemcpyDeviceToHost));
  if (cycles) *cycles = cyc > 0 ? cyc : P->desc.max_cycles;
  if (relres) *relres = rel;
  if (!ok) {
    P->err = "mg_solve: tolerance not reached within max_cycles";
    return MG_ENOCONV;
  }
  return MG_OK;
  API_END(P)
}

int mlmc_sample_batch(mg_plan P, int level, const uint64_t* seeds, int n_samples, double* Y_out,
                      double* Qf_out, double* Qc_out, int* cycles_out, int fixed_cycles) {
  if (!P) return MG_EINVAL;
  if (level < 0 || level > P->desc.max_level || !seeds || n_samples < 1 || !Y_out ||
      fixed_cycles < 0) {
    P->err = "mlmc_sample_batch: level must be in [0, max_level], seeds/Y_out non-null, n >= 1";
    return MG_EINVAL;
  }
  API_BEGIN
  const int nf = (P->desc.n0 - 1) * (1 << level) + 1;
  const int nc = level > 0 ? (P->desc.n0 - 1) * (1 << (level - 1)) + 1 : 0;
  BatchSpec spec;
  for (int i = 0; i < n_samples; ++i) {
    spec.top_n.push_back(nf);
    spec.share.push_back(-1);
    if (level > 0) {
      spec.top_n.push_back(nc);
      spec.share.push_back((int)spec.top_n.size() - 2);
    }
  }
  spec.const_b_top = true;
  spec.ext_u_top = false;
  int status = MG_OK;
  const bool fresh = !P->batch || P->batch_key != spec.key();
  Batch* B = get_batch(P, spec, &status);
  if (!B) return status;
  hipStream_t st = P->stream;
  if (fresh || B->nsamples != n_samples) {
    upload_lists(P, B);
    B->nsamples = n_samples;
    const int per = level > 0 ? 2 : 1;
    B->d_seeds = (uint64_t*)B->dalloc(sizeof(uint64_t) * n_samples);
    B->d_normals = (double*)B->dalloc(sizeof(double) * 64 * n_samples);
    std::vector<int> fi(n_samples), ci(n_samples), xi(n_samples);
    std::vector<double*> fo(n_samples);
    for (int i = 0; i < n_samples; ++i) {
      fi[i] = per * i;
      ci[i] = level > 0 ? per * i + 1 : -1;
      xi[i] = i;
      fo[i] = B->lev[per * i][0].wh;
    }
    B->d_fi = (int*)B->dalloc(sizeof(int) * n_samples);
    B->d_ci = (int*)B->dalloc(sizeof(int) * n_samples);
    B->d_xi_index = (int*)B->dalloc(sizeof(int) * n_samples);
    B->d_field_out = (double**)B->dalloc(sizeof(double*) * n_samples);
    CK(hipMemcpy(B->d_fi, fi.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_ci, ci.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_xi_index, xi.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_field_out, fo.data(), sizeof(double*) * n_samples, hipMemcpyHostToDevice));
    B->field_count = n_samples;
    B->field_n = nf;
  }
  CK(hipMemcpyAsync(B->d_seeds, seeds, sizeof(uint64_t) * n_samples, hipMemcpyHostToDevice, st));
  launch_philox(B->d_seeds, n_samples, level, nullptr, B->d_normals, st);
  launch_field(nf, n_samples, B->d_field_out, B->d_xi_index, B->d_normals, phi_table(P, nf),
               P->d_coef, 0, st);
  inject_all(P, B);
  // every sample starts from the zero iterate (the workspace may hold the last batch)
  for (size_t ti = 0; ti < B->top_sizes.size(); ++ti)
    launch_zero_u(B->d_top[ti], (int)B->h_top[ti].size(), B->top_sizes[ti], st);
  const bool ok = run_solves(P, B, P->desc.tol, fixed_cycles);
  reduce_tops(P, B, RED_QOI, 0, 0, 0.0);
  launch_ydiff(B->ss.q, B->d_fi, B->d_ci, n_samples, Y_out, Qf_out, Qc_out, B->ss.cycles,
               cycles_out, st);
  CK(hipStreamSynchronize(st));
  if (P->prof) collect_profile(P);
  if (!ok) {
    P->err = "mlmc_sample_batch: some solve missed tol within max_cycles";
    return MG_ENOCONV;
  }
  return MG_OK;
  API_END(P)
}

int mlmc_philox(mg_plan P, const uint64_t* seeds, int n_samples, int level, uint32_t* words_out,
                double* normals_out) {
  if (!P) return MG_EINVAL;
  if (!seeds || n_samples < 1 || level < 0 || (!words_out && !normals_out)) return MG_EINVAL;
  API_BEGIN
  uint64_t* d = nullptr;
  CK(hipMalloc(&d, sizeof(uint64_t) * n_samples));
  CK(hipMemcpyAsync(d, seeds, sizeof(uint64_t) * n_samples, hipMemcpyHostToDevice, P->stream));
  launch_philox(d, n_samples, level, words_out, normals_out, P->stream);
  CK(hipStreamSynchronize(P->stream));
  CK(hipFree(d));
  return MG_OK;
  API_END(P)
}

int mlmc_field(mg_plan P, int n, uint64_t seed, int level, double* k_out) {
  if (!P) return MG_EINVAL;
  if (!valid_n(n) || n > 1025 || level < 0 || !k_out) return MG_EINVAL;
  API_BEGIN
  uint64_t* d_seed = nullptr;
  double* d_norm = nullptr;
  double** d_out = nullptr;
  int* d_xi = nullptr;
  CK(hipMalloc(&d_seed, sizeof(uint64_t)));
  CK(hipMalloc(&d_norm, sizeof(double) * 64));
  CK(hipMalloc(&d_out, sizeof(double*)));
  CK(hipMalloc(&d_xi, sizeof(int)));
  const int zero = 0;
  CK(hipMemcpyAsync(d_seed, &seed, sizeof(uint64_t), hipMemcpyHostToDevice, P->stream));
  CK(hipMemcpyAsync(d_out, &k_out, sizeof(double*), hipMemcpyHostToDevice, P->stream));
  CK(hipMemcpyAsync(d_xi, &zero, sizeof(int), hipMemcpyHostToDevice, P->stream));
  launch_philox(d_seed, 1, level, nullptr, d_norm, P->stream);
  launch_field(n, 1, d_out, d_xi, d_norm, phi_table(P, n), P->d_coef, 1, P->stream);
  CK(hipStreamSynchronize(P->stream));
  CK(hipFree(d_seed));
  CK(hipFree(d_norm));
  CK(hipFree(d_out));
  CK(hipFree(d_xi));
  return MG_OK;
  API_END(P)
}

void mlmc_acc_init(mlmc_level_acc* a) {
  if (a) std::memset(a, 0, sizeof(*a));
}

static void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

int mlmc_acc_add(mlmc_level_acc* a, const double* y, int count, int on_device) {
  if (!a || !y || count < 0) return MG_EINVAL;
  std::vector<double> h;
  const double* src = y;
  if (on_device) {
    h.resize(count);
    if (hipMemcpy(h.data(), y, sizeof(double) * count, hipMemcpyDeviceToHost) != hipSuccess)
      return MG_EHIP;
    src = h.data();
  }
  for (int i = 0; i < count; ++i) {
    if (a->n == 0) a->shift = src[i];
    const double d = src[i] - a->shift;
    neumaier(a->s1, a->c1, d);
    neumaier(a->s2, a->c2, d * d);
    a->n += 1;
  }
  return MG_OK;
}

void mlmc_acc_result(const mlmc_level_acc* a, double* mean, double* var) {
  if (!a || !mean || !var) return;
  if (a->n == 0) {
    *mean = 0.0;
    *var = 0.0;
    return;
  }
  const double N = (double)a->n;
  const double m1 = (a->s1 + a->c1) / N;
  *mean = a->shift + m1;
  *var = (a->s2 + a->c2) / N - m1 * m1;
}

int mg_profile_enable(mg_plan P, int on) {
  if (!P) return MG_EINVAL;
  P->prof = on != 0;
  P->prof_launches = 0;
  P->prof_ms = 0.0;
  P->ev_used = 0;
  return MG_OK;
}

int mg_profile_read(mg_plan P, long long* launches, double* total_ms, double* nodes_per_launch) {
  if (!P) return MG_EINVAL;
  API_BEGIN
  collect_profile(P);
  if (launches) *launches = P->prof_launches;
  if (total_ms) *total_ms = P->prof_ms;
  if (nodes_per_launch) *nodes_per_launch = P->prof_nodes;
  return MG_OK;
  API_END(P)
}

}  // extern "C"
