// Plan, batch workspace, batched V-cycle driver and the C ABI of libmlmcmg.
//
// A batch is a set of solves (for an MLMC sample: the level-l solve and, for
// l > 0, the level-(l-1) solve of the same omega, Algorithm 1 step 1.a).
// Every multigrid level of every solve owns its buffers; all grids of one
// size form one device list, so each step of the V-cycle is one launch for the
// whole batch.  Grids of different top sizes nest: a solve with a smaller top
// grid starts its cycle when the larger ones reach its size (the cycles are
// aligned at the coarsest grid), so a launch only ever sees grids of one size.
//
// Work runs on a private stream of the plan (so it can be captured into HIP
// graphs); it is ordered after the caller's stream at the start of each call
// and every call synchronises before returning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mlmcmg.h"
#include "mg_internal.h"
#include "mg_kl.h"
#include "mg_sched.h"

namespace mg {

struct HipError {
  hipError_t e;
  const char* what;
};

#define CK(x)                                     \
  do {                                            \
    hipError_t e_ = (x);                          \
    if (e_ != hipSuccess) throw HipError{e_, #x}; \
  } while (0)

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename T>
struct LevelT {
  int n = 0;
  T* u[2] = {nullptr, nullptr};
  T* wh = nullptr;
  T* b = nullptr;
  T* r = nullptr;
  T* fc = nullptr;  // P1 finite elements: the axis couplings (3 n^3)
};

struct BatchSpec {
  std::vector<int> top_n;   // top grid size of each solve
  std::vector<int> share;   // solve whose levels 1.. supply this solve's wh (or -1)
  bool const_b_top = true;  // top right-hand side is the constant h^2 (f = 1)
  bool ext_u_top = false;   // top u is caller memory (mg_solve)
  bool mixed = false;       // FP32 inner cycles inside FP64 defect correction
  bool fe = false;          // P1 finite-element operator (FP64)
  std::string key() const {
    std::string s = fe ? "f" : "";
    s += const_b_top ? "c" : "v";
    s += ext_u_top ? "e" : "i";
    s += mixed ? "m" : "d";
    for (size_t i = 0; i < top_n.size(); ++i)
      s += ":" + std::to_string(top_n[i]) + "/" + std::to_string(share[i]);
    return s;
  }
};

template <typename T>
struct Lists {
  std::vector<std::vector<GridDescT<T>>> h;  // per size index
  // whether every grid of h[si] has a constant right-hand side plane
  bool const_b(size_t si) const {
    for (const auto& g : h[si])
      if (g.bstride != 0) return false;
    return !h[si].empty();
  }
  // whether every grid of h[si] carries its KL coefficient data
  bool kl(size_t si) const {
    for (const auto& g : h[si])
      if (!g.kln) return false;
    return !h[si].empty();
  }
  std::vector<GridDescT<T>*> d;
  std::vector<std::vector<GridDescT<T>>> htop;  // per top size index
  std::vector<GridDescT<T>*> dtop;
  // small-grid V-cycle: every solve's chain is rooted at its largest grid of
  // at most the threshold size; one group per root size, descending;
  // chain_si is the size index of the largest root (-1: no chains)
  int chain_si = -1;
  struct Group {
    int ns;
    std::vector<SmallChain<T>> h;
    SmallChain<T>* d = nullptr;
  };
  std::vector<Group> chains;
};

struct Batch {
  BatchSpec spec;
  hipStream_t st = nullptr;  // stream the batch's cycles run on
  int ns = 0;
  std::vector<std::vector<LevelT<double>>> lev;    // [solve][mg level]
  std::vector<std::vector<LevelT<float>>> lev32;   // mixed precision only
  std::vector<int> sizes;                          // distinct grid sizes, descending
  std::vector<int> top_sizes;                      // distinct top sizes, descending
  Lists<double> L64;
  Lists<float> L32;
  SolveState ss{};
  int* h_state = nullptr;  // pinned: active then cycles of every solve (2 ns)
  // MLMC sample plumbing
  int nsamples = 0;
  uint64_t* d_seeds = nullptr;
  uint64_t* h_seeds = nullptr;  // pinned staging of the seeds (an asynchronous upload)
  double* d_normals = nullptr;
  int* d_levels = nullptr;
  int* d_fi = nullptr;
  int* d_ci = nullptr;
  struct FieldGroup {
    int n, count;
    double** d_out;  // top wh of the fine solve of each sample of this level
    int* d_xi;       // their rows of d_normals
  };
  std::vector<FieldGroup> fields;
  // per solve: the normals of its KL field (its grids' descriptors then carry
  // the KL data), or nullptr; empty when the batch has no KL samples
  std::vector<const double*> kl_normals;
  // coefficient injection per fine size, and FP32 conversion per size
  std::vector<double**> d_inj_src, d_inj_dst;
  std::vector<int> inj_n, inj_count;
  std::vector<double**> d_cvt_src;
  std::vector<float**> d_cvt_dst;
  std::vector<int> cvt_n, cvt_count;
  // P1 finite elements: per size, the wh and fc arrays of the grids that own them
  std::vector<double**> d_fe_wh, d_fe_fc;
  std::vector<int> fe_n, fe_count;
  bool uploaded = false;
  std::vector<double*> const_plane;  // per size index: n^2 values h^2
  // graphs of c consecutive cycles
  std::map<int, hipGraphExec_t> graphs;
  int last_cycles = 0;
  bool bnorm_ready = false;  // ||b'|| of every solve computed (constant top rhs)
  // a fixed schedule whose residuals nobody reads (full multigrid stages):
  // steps are counted, no residual norm is formed
  bool count_only = false;
  void* mem = nullptr;
  size_t bytes = 0;
  std::vector<void*> extra;
  size_t extra_bytes = 0;  // what the extra allocations hold (256-byte units)
  // a batch built over caller-provided device memory (the allocation-free
  // solve): mem and every later dalloc are carved from it, nothing is freed
  char* arena = nullptr;
  size_t arena_cap = 0, arena_off = 0;
  void* dalloc(size_t bytes) {
    if (arena) {
      const size_t a = align256(bytes);
      if (arena_off + a > arena_cap) throw HipError{hipErrorOutOfMemory, "static workspace full"};
      void* p = arena + arena_off;
      arena_off += a;
      return p;
    }
    void* p = nullptr;
    CK(hipMalloc(&p, bytes));
    extra.push_back(p);
    extra_bytes += align256(bytes);
    return p;
  }
  // full multigrid stage: the top descriptors with uc = the previous stage's
  // top iterates (link_src: that stage's batch)
  GridDesc* d_link = nullptr;
  const Batch* link_src = nullptr;
  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~Batch() {
    drop_graphs();
    for (void* p : extra) (void)hipFree(p);
    if (mem && !arena) (void)hipFree(mem);
    if (h_state && !arena) (void)hipHostFree(h_state);
    if (h_seeds) (void)hipHostFree(h_seeds);
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

namespace mg {
struct SpdeWork;
}

struct mg_plan_s {
  mg_plan_desc desc{};
  hipStream_t caller = nullptr;  // stream the caller's data is ordered on
  hipStream_t work = nullptr;    // the plan's own stream (default priority)
  hipEvent_t order_ev = nullptr;
  std::string err;
  double omega[4]{}, theta[4]{}, scale[4]{};
  double* d_coef = nullptr;
  std::map<int, double*> d_phi;
  std::unique_ptr<Batch> batch;
  std::string batch_key;
  // options
  int smoother = 0;      // 0: fused single-pass sweep, 1: two-pass colour sweeps
  int use_graph = 1;     // capture cycles into HIP graphs (mlmc_sample_batch)
  int small_ns = 17;     // grids of this size and below: the LDS V-cycle (0: off)
  int transfer = 0;      // 0: fused residual + restriction, 1: separate kernels
  int norm_sweep = 1;    // 1: a cycle's first sweep also takes the residual norm of
                         // the previous iterate (convergence judged one cycle late)
  int qoi_kind = QOI_INTEGRAL;  // the samples' QoI (Section 3)
  int solver = 0;        // 0: V-cycles to tol, 1: full multigrid (fixed schedule)
  int fmg_cycles = 2;    // V-cycles per grid of the full multigrid schedule
  int op_fe = 0;         // 1: the P1 finite-element operator instead of FD
  int inner_cycles = 1;  // mixed precision: FP32 V-cycles per FP64 defect-correction step
  int kl_inline = 0;     // 1: FP64 sweeps and transfers of KL-field samples evaluate the
                         // coefficient instead of reading it (same values; slower on
                         // MI355X: the sweeps are bound by FP64 issue, not by bytes)
  int field_spde = 0;    // 1: coefficient fields from the SPDE sampler instead of KL
  // SPDE sampler workspaces keyed by (finest box size, solves)
  std::map<std::pair<int, int>, std::unique_ptr<mg::SpdeWork>> spde;
  // full multigrid: one batch per grid size of the schedule (n -> batch)
  std::map<int, std::unique_ptr<Batch>> fmg;
  std::map<int, SweepShape> shape;      // tile shape per grid size
  std::map<int, SweepShape> shape_pro;  // same, sweeps with the fused coarse correction
  // profiling of the finest-grid smoothing launches
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  long long prof_launches = 0;
  double prof_ms = 0.0;
  double prof_nodes = 0.0;
  // per timed launch: the cycle of its batch (1-based), its sweep kind, the
  // grid size and its duration; ev_meta holds the (cycle, kind, n) of each
  // pending event pair
  struct ProfRec {
    int cycle, kind, n;
    double ms;
  };
  std::vector<ProfRec> prof_recs;
  std::vector<ProfRec> ev_meta;
  int prof_cycle = 0;
  // allocation-free solve: this device's static workspace and a small pinned
  // host buffer for the per-solve state read back after each cycle (both
  // set up at plan creation)
  void* scratch = nullptr;
  int scratch_dev = 0;
  int* h_small = nullptr;

  ~mg_plan_s();
};

namespace mg {

// The sweep shape for n, for a launch over count grids (0: unknown).  A
// launch over so few grids that the kernel's automatic split, which stops at
// pieces of four planes, would leave it under 512 workgroups takes pieces of
// two planes instead (one 33^3 grid: 28 -> 64 workgroups per sweep, the
// single-sample latency 718 -> 659 us; the results are the same for any split).
static SweepShape shape_for(mg_plan_s* P, int n, bool pro = false, int count = 0) {
  const auto& m = pro ? P->shape_pro : P->shape;
  auto it = m.find(n);
  if (it != m.end()) return it->second;
  SweepShape s = default_sweep_shape(n, pro, P->desc.precision == MG_MIXED);
  if (count > 0 && s.chunks == 0 && n >= 9) {
    const int tiles = ((n - 1) / s.tj) * ((n - 1) / s.tk);
    if ((long)count * tiles * ((n - 2) / 4) < 512) s.chunks = (n - 1) / 2;
  }
  return s;
}

// Order the plan's stream after everything queued so far on the caller's.
static void order_after_caller(mg_plan_s* P) {
  CK(hipEventRecord(P->order_ev, P->caller));
  CK(hipStreamWaitEvent(P->work, P->order_ev, 0));
}

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

// Allocate a batch.  One device allocation holds every grid buffer.  With
// size_only, only the bytes that allocation would take are computed.
static std::unique_ptr<Batch> build_batch(mg_plan_s* P, const BatchSpec& spec,
                                          size_t* size_only = nullptr, char* arena = nullptr,
                                          size_t arena_cap = 0) {
  auto B = std::make_unique<Batch>();
  B->spec = spec;
  B->st = P->work;
  const int ns = (int)spec.top_n.size();
  B->ns = ns;
  B->lev.resize(ns);
  if (spec.mixed) B->lev32.resize(ns);
  size_t total = 0;
  char* cur = nullptr;
  // pass 0 sizes the allocation, pass 1 carves it
  for (int pass = 0; pass < 2; ++pass) {
    auto take = [&](size_t bytes) -> void* {
      if (pass == 0) {
        total += align256(bytes);
        return nullptr;
      }
      void* p = cur;
      cur += align256(bytes);
      return p;
    };
    for (int s = 0; s < ns; ++s) {
      const auto h = hierarchy(spec.top_n[s]);
      B->lev[s].assign(h.size(), LevelT<double>{});
      if (spec.mixed) B->lev32[s].assign(h.size(), LevelT<float>{});
      for (size_t j = 0; j < h.size(); ++j) {
        const size_t N = (size_t)h[j] * h[j] * h[j];
        auto& L = B->lev[s][j];
        L.n = h[j];
        const bool top = j == 0;
        if (spec.share[s] < 0) L.wh = (double*)take(N * 8);
        else if (pass == 1) L.wh = B->lev[spec.share[s]][j + 1].wh;
        if (spec.fe) {
          if (spec.share[s] < 0) L.fc = (double*)take(3 * N * 8);
          else if (pass == 1) L.fc = B->lev[spec.share[s]][j + 1].fc;
        }
        if (!spec.mixed) {
          if (!(top && spec.ext_u_top)) L.u[0] = (double*)take(N * 8);
          L.u[1] = (double*)take(N * 8);
          if (!(top && spec.const_b_top)) L.b = (double*)take(N * 8);
          if (h[j] > 3) L.r = (double*)take(N * 8);
        } else {
          if (top && !spec.ext_u_top) L.u[0] = (double*)take(N * 8);
          if (top && !spec.const_b_top) L.b = (double*)take(N * 8);
          auto& F = B->lev32[s][j];
          F.n = h[j];
          F.u[0] = (float*)take(N * 4);
          F.u[1] = (float*)take(N * 4);
          if (spec.share[s] < 0) F.wh = (float*)take(N * 4);
          else if (pass == 1) F.wh = B->lev32[spec.share[s]][j + 1].wh;
          F.b = (float*)take(N * 4);
          if (h[j] > 3) F.r = (float*)take(N * 4);
        }
      }
    }
    int npart = 0;
    for (int s = 0; s < ns; ++s) npart += reduce_blocks(spec.top_n[s]);
    int* ai = (int*)take(sizeof(int) * (ns * 4 + 1));
    double* dd = (double*)take(sizeof(double) * ns * 3);
    double* pp = (double*)take(sizeof(double) * npart);
    double* sp = (double*)take(sizeof(double) * ns * (2 * kSweepParts + 2));
    if (pass == 0) {
      if (size_only) {
        *size_only = total;
        return nullptr;
      }
      if (arena) {
        if (total > arena_cap) return nullptr;
        B->arena = arena;
        B->arena_cap = arena_cap;
        B->arena_off = total;
        B->mem = arena;
        // the static workspace keeps the last call's contents: clear it with
        // a fill kernel (no memset node, no allocation)
        launch_fill((double*)arena, (long)(total / sizeof(double)), 0.0, P->work);
      } else {
        if (P->desc.hbm_budget && total > P->desc.hbm_budget) return nullptr;
        CK(hipMalloc(&B->mem, total));
        // zero boundaries and state once; later kernels only write interiors
        CK(hipMemsetAsync(B->mem, 0, total, P->work));
      }
      B->bytes = total;
      cur = (char*)B->mem;
    } else {
      B->ss.active = ai;
      B->ss.cycles = ai + ns;  // (right after active: the host reads both in one copy)
      B->ss.ran = ai + 2 * ns;
      B->ss.qpend = ai + 3 * ns;
      B->ss.relres = dd;
      B->ss.bnorm = dd + ns;
      B->ss.q = dd + 2 * ns;
      B->ss.partials = pp;
      B->ss.spart = sp;
    }
  }
  if (arena) B->h_state = P->h_small;  // one solve: two ints
  else CK(hipHostMalloc((void**)&B->h_state, sizeof(int) * 2 * ns, hipHostMallocDefault));
  int nmax = 0;
  for (int n : spec.top_n) nmax = std::max(nmax, n);
  B->sizes = hierarchy(nmax);
  for (int s = 0; s < ns; ++s)
    if (std::find(B->top_sizes.begin(), B->top_sizes.end(), spec.top_n[s]) == B->top_sizes.end())
      B->top_sizes.push_back(spec.top_n[s]);
  std::sort(B->top_sizes.begin(), B->top_sizes.end(), std::greater<int>());
  return B;
}

static size_t size_index(const std::vector<int>& v, int n) {
  return std::find(v.begin(), v.end(), n) - v.begin();
}

template <typename T>
static GridDescT<T> make_desc(const std::vector<LevelT<T>>& lv, size_t j, int solve, int poff,
                             T* const_plane) {
  const LevelT<T>& L = lv[j];
  GridDescT<T> d{};
  d.u[0] = L.u[0];
  d.u[1] = L.u[1];
  d.wh = L.wh;
  d.fc = L.fc;
  d.b = L.b ? L.b : const_plane;  // constant right-hand side: one plane, stride 0
  d.bstride = L.b ? L.n * L.n : 0;
  d.r = L.r;
  if (j + 1 < lv.size()) {
    d.uc[0] = lv[j + 1].u[0];
    d.uc[1] = lv[j + 1].u[1];
    d.bc = lv[j + 1].b;
  }
  const double h = 1.0 / (double)(L.n - 1);
  d.bconst = h * h;  // f = 1
  d.solve = solve;
  d.n = L.n;
  d.poff = poff;
  d.spoff = j == 0 ? solve * (2 * kSweepParts + 2) : -1;
  return d;
}

template <typename T>
static void upload(Batch* B, Lists<T>& Ls, hipStream_t st) {
  for (auto& g : Ls.chains) {
    if (g.h.empty()) continue;
    if (!g.d) g.d = (SmallChain<T>*)B->dalloc(sizeof(SmallChain<T>) * g.h.size());
    CK(hipMemcpyAsync(g.d, g.h.data(), sizeof(SmallChain<T>) * g.h.size(),
                      hipMemcpyHostToDevice, st));
  }
  size_t cnt = 0;
  for (auto& v : Ls.h) cnt += v.size();
  for (auto& v : Ls.htop) cnt += v.size();
  if (Ls.d.empty()) {
    GridDescT<T>* base = (GridDescT<T>*)B->dalloc(sizeof(GridDescT<T>) * std::max<size_t>(cnt, 1));
    size_t off = 0;
    for (auto& v : Ls.h) { Ls.d.push_back(base + off); off += v.size(); }
    for (auto& v : Ls.htop) { Ls.dtop.push_back(base + off); off += v.size(); }
  }
  for (size_t i = 0; i < Ls.h.size(); ++i)
    if (!Ls.h[i].empty())
      CK(hipMemcpyAsync(Ls.d[i], Ls.h[i].data(), sizeof(GridDescT<T>) * Ls.h[i].size(),
                        hipMemcpyHostToDevice, st));
  for (size_t i = 0; i < Ls.htop.size(); ++i)
    if (!Ls.htop[i].empty())
      CK(hipMemcpyAsync(Ls.dtop[i], Ls.htop[i].data(), sizeof(GridDescT<T>) * Ls.htop[i].size(),
                        hipMemcpyHostToDevice, st));
}

// (Re)write the device descriptor lists from the current buffers.
static void upload_lists(mg_plan_s* P, Batch* B) {
  const auto& spec = B->spec;
  if (B->const_plane.empty()) {
    // h^2 (f = 1) on one n^2 plane per grid size, read with plane stride 0
    for (int n : B->sizes) {
      double* pl = (double*)B->dalloc(sizeof(double) * n * n);
      const double h = 1.0 / (double)(n - 1);
      launch_fill(pl, (long)n * n, h * h, P->work);
      B->const_plane.push_back(pl);
    }
  }
  B->L64.h.assign(B->sizes.size(), {});
  B->L64.htop.assign(B->top_sizes.size(), {});
  B->L32.h.assign(spec.mixed ? B->sizes.size() : 0, {});
  B->L32.htop.assign(spec.mixed ? B->top_sizes.size() : 0, {});
  // the small-grid V-cycle takes over from each solve's largest grid of at
  // most P->small_ns (and at least 5) vertices per axis; a batch with a 3^3
  // top grid keeps the per-level path
  bool small_ok = P->small_ns >= 5 && !spec.fe;
  for (int s = 0; s < B->ns; ++s)
    if (spec.top_n[s] < 5) small_ok = false;
  int chain_si = -1;
  if (small_ok)
    for (size_t si = 0; si < B->sizes.size(); ++si)
      if (B->sizes[si] <= P->small_ns) {
        chain_si = (int)si;
        break;
      }
  B->L64.chain_si = B->L32.chain_si = chain_si;
  if (B->L64.chains.empty() && chain_si >= 0)
    for (size_t si = chain_si; si < B->sizes.size() && B->sizes[si] >= 5; ++si) {
      B->L64.chains.push_back({B->sizes[si], {}, nullptr});
      if (spec.mixed) B->L32.chains.push_back({B->sizes[si], {}, nullptr});
    }
  for (auto& g : B->L64.chains) g.h.clear();
  for (auto& g : B->L32.chains) g.h.clear();
  int poff = 0;
  for (int s = 0; s < B->ns; ++s) {
    const auto& lv = B->lev[s];
    for (size_t j = 0; j < lv.size(); ++j) {
      const size_t si = size_index(B->sizes, lv[j].n);
      GridDesc d = make_desc(lv, j, s, j == 0 ? poff : 0, B->const_plane[si]);
      if (!B->kl_normals.empty() && B->kl_normals[s]) {
        // every grid of a KL solve: the coarse grids' wh is the injection of
        // the finest one's, i.e. the same field at their own vertices
        d.kln = B->kl_normals[s];
        d.klcoef = P->d_coef;
        d.klphi = phi_table(P, lv[j].n);
      }
      B->L64.h[si].push_back(d);
      if (spec.mixed)
        B->L32.h[si].push_back(make_desc<float>(B->lev32[s], j, s, j == 0 ? poff : 0, nullptr));
      // the root of this solve's chain: its first grid at or below the threshold
      const bool root = chain_si >= 0 && lv[j].n <= P->small_ns &&
                        (j == 0 || lv[j - 1].n > P->small_ns);
      if (root) {
        SmallChain<double> c{};
        SmallChain<float> c32{};
        for (size_t q = j; q < lv.size() && q - j < 4; ++q) {
          const size_t sq = size_index(B->sizes, lv[q].n);
          c.lv[q - j] = make_desc(lv, q, s, q == 0 ? poff : 0, B->const_plane[sq]);
          if (spec.mixed) c32.lv[q - j] = make_desc<float>(B->lev32[s], q, s, q == 0 ? poff : 0, nullptr);
        }
        const size_t gi = si - (size_t)chain_si;
        B->L64.chains[gi].h.push_back(c);
        if (spec.mixed) B->L32.chains[gi].h.push_back(c32);
      }
      if (j == 0) {
        const size_t ti = size_index(B->top_sizes, lv[j].n);
        B->L64.htop[ti].push_back(d);
        if (spec.mixed) B->L32.htop[ti].push_back(make_desc<float>(B->lev32[s], j, s, poff, nullptr));
      }
    }
    poff += reduce_blocks(spec.top_n[s]);
  }
  upload(B, B->L64, P->work);
  if (spec.mixed) upload(B, B->L32, P->work);
  if (!B->uploaded) {
    // coefficient injection (every grid that owns its wh feeds its coarse child)
    // and, for mixed precision, the FP32 copies of every owned wh
    for (size_t si = 0; si < B->sizes.size(); ++si) {
      std::vector<double*> src, dst, csrc;
      std::vector<float*> cdst;
      for (int s = 0; s < B->ns; ++s) {
        if (spec.share[s] >= 0) continue;
        const auto& lv = B->lev[s];
        for (size_t j = 0; j < lv.size(); ++j) {
          if (lv[j].n != B->sizes[si]) continue;
          if (j + 1 < lv.size()) {
            src.push_back(lv[j].wh);
            dst.push_back(lv[j + 1].wh);
          }
          if (spec.mixed) {
            csrc.push_back(lv[j].wh);
            cdst.push_back(B->lev32[s][j].wh);
          }
        }
      }
      if (!src.empty()) {
        double** ds = (double**)B->dalloc(sizeof(double*) * src.size());
        double** dd = (double**)B->dalloc(sizeof(double*) * dst.size());
        CK(hipMemcpyAsync(ds, src.data(), sizeof(double*) * src.size(), hipMemcpyHostToDevice, P->work));
        CK(hipMemcpyAsync(dd, dst.data(), sizeof(double*) * dst.size(), hipMemcpyHostToDevice, P->work));
        B->d_inj_src.push_back(ds);
        B->d_inj_dst.push_back(dd);
        B->inj_n.push_back(B->sizes[si]);
        B->inj_count.push_back((int)src.size());
      }
      if (spec.fe) {
        std::vector<double*> fw, ff;
        for (int s = 0; s < B->ns; ++s) {
          if (spec.share[s] >= 0) continue;
          for (const auto& L : B->lev[s])
            if (L.n == B->sizes[si]) {
              fw.push_back(L.wh);
              ff.push_back(L.fc);
            }
        }
        if (!fw.empty()) {
          double** dw = (double**)B->dalloc(sizeof(double*) * fw.size());
          double** df = (double**)B->dalloc(sizeof(double*) * ff.size());
          CK(hipMemcpyAsync(dw, fw.data(), sizeof(double*) * fw.size(), hipMemcpyHostToDevice, P->work));
          CK(hipMemcpyAsync(df, ff.data(), sizeof(double*) * ff.size(), hipMemcpyHostToDevice, P->work));
          B->d_fe_wh.push_back(dw);
          B->d_fe_fc.push_back(df);
          B->fe_n.push_back(B->sizes[si]);
          B->fe_count.push_back((int)fw.size());
        }
      }
      if (!csrc.empty()) {
        double** ds = (double**)B->dalloc(sizeof(double*) * csrc.size());
        float** dd = (float**)B->dalloc(sizeof(float*) * cdst.size());
        CK(hipMemcpyAsync(ds, csrc.data(), sizeof(double*) * csrc.size(), hipMemcpyHostToDevice, P->work));
        CK(hipMemcpyAsync(dd, cdst.data(), sizeof(float*) * cdst.size(), hipMemcpyHostToDevice, P->work));
        B->d_cvt_src.push_back(ds);
        B->d_cvt_dst.push_back(dd);
        B->cvt_n.push_back(B->sizes[si]);
        B->cvt_count.push_back((int)csrc.size());
      }
    }
    B->uploaded = true;
  }
  CK(hipStreamSynchronize(P->work));
}

// Coarse-grid coefficients by injection (finest size first), then the FP32
// copies for mixed precision.
static void prepare_coefficients(mg_plan_s* P, Batch* B) {
  for (size_t j = 0; j < B->inj_n.size(); ++j)
    launch_inject(B->inj_n[j], B->inj_count[j], (const double* const*)B->d_inj_src[j],
                  B->d_inj_dst[j], P->work);
  for (size_t j = 0; j < B->cvt_n.size(); ++j)
    launch_to_float(B->cvt_n[j], B->cvt_count[j], (const double* const*)B->d_cvt_src[j],
                    B->d_cvt_dst[j], P->work);
  // P1 finite elements: every level's couplings from its (injected) coefficient
  for (size_t j = 0; j < B->fe_n.size(); ++j)
    launch_fe_faces(B->fe_n[j], B->fe_count[j], (const double* const*)B->d_fe_wh[j],
                    B->d_fe_fc[j], P->work);
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
  CK(hipStreamSynchronize(P->work));
  for (size_t i = 0; i + 1 < P->ev_used; i += 2) {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, P->ev_pool[i], P->ev_pool[i + 1]));
    P->prof_ms += ms;
    P->prof_launches += 1;
    auto m = P->ev_meta[i / 2];
    m.ms = (double)ms;
    P->prof_recs.push_back(m);
  }
  P->ev_used = 0;
  P->ev_meta.clear();
}

// Timed region of one sweep of another operator (kind 4: the finite-element
// colour passes, 5: the SPDE box colour passes) on the grids of size n.
static void prof_begin(mg_plan_s* P, int kind, int n, int cycle, hipStream_t st) {
  if (P->ev_used + 4 > 8192) collect_profile(P);
  P->ev_meta.push_back({cycle, kind, n, 0.0});
  CK(hipEventRecord(next_event(P), st));
}
static void prof_end(mg_plan_s* P, hipStream_t st) { CK(hipEventRecord(next_event(P), st)); }

// One red-black sweep on the grids of size index si; returns the new buffer.
template <typename T>
static int smooth_once(mg_plan_s* P, Batch* B, Lists<T>& Ls, size_t si, int buf, int cbuf,
                       bool timed, T* spart = nullptr, int norm = 0) {
  const int n = B->sizes[si];
  const int cnt = (int)Ls.h[si].size();
  hipStream_t st = B->st;
  if (timed) {
    if (P->ev_used + 4 > 8192) collect_profile(P);
    // kind: 0 plain sweep, 1 with the coarse correction, 2 with the black
    // residuals of its output, 3 with the red residuals of its input
    const int kind = cbuf >= 0 ? 1 : (spart ? (norm == 2 ? 2 : 3) : 0);
    P->ev_meta.push_back({P->prof_cycle, kind, n, 0.0});
    CK(hipEventRecord(next_event(P), st));
  }
  int out = buf;
  if (P->smoother == 0 && sweep_fits(n, sizeof(T))) {
    // (with a full right-hand side, the sweep with the input's red residuals
    // takes the register budget and shape of the sweep with the coarse
    // correction)
    const bool cb = Ls.const_b(si);
    launch_sweep<T>(Ls.d[si], cnt, n, B->ss.active, buf, cbuf,
                    shape_for(P, n, cbuf >= 0 || (spart && norm == 1 && !cb), cnt), st, spart,
                    norm, cb,
                    P->kl_inline && Ls.kl(si));
    out = 1 - buf;
  } else {
    if (cbuf >= 0) launch_prolong<T>(Ls.d[si], cnt, n, B->ss.active, buf, cbuf, st);
    launch_rbgs_colour<T>(Ls.d[si], cnt, n, B->ss.active, 0, buf, st);
    launch_rbgs_colour<T>(Ls.d[si], cnt, n, B->ss.active, 1, buf, st);
  }
  if (timed) {
    CK(hipEventRecord(next_event(P), st));
    P->prof_nodes = (double)cnt * (double)(n - 2) * (n - 2) * (n - 2);
  }
  return out;
}


// Partials per grid when the top grids of size index si take their
// convergence norm from the sweeps (the black residuals from a cycle's last
// sweep, the red ones from the next cycle's first sweep, which runs in the
// shape of the sweep with the coarse correction unless the right-hand side is
// constant: *red gets its count), else 0 (a reduction after the cycle).
// Decided on the full lists L64 (the same for every cycle of a batch); the
// counts are those of the given lists.
static int lagged_parts(mg_plan_s* P, Batch* B, size_t si, int* red = nullptr,
                        const Lists<double>* Lp = nullptr) {
  const Lists<double>& L = Lp ? *Lp : B->L64;
  const int n = B->sizes[si];
  if (B->count_only || B->spec.mixed || B->spec.fe || !P->norm_sweep || P->smoother != 0 || P->desc.nu1 < 1 ||
      P->desc.nu2 < 2 || n < 5)
    return 0;
  if (B->L64.chain_si >= 0 && si >= (size_t)B->L64.chain_si) return 0;  // LDS V-cycle sizes
  if (std::find(B->top_sizes.begin(), B->top_sizes.end(), n) == B->top_sizes.end()) return 0;
  if (!sweep_fits(n, sizeof(double))) return 0;
  // at most kSweepParts workgroups per grid (a launch whose automatic split
  // finds one grid active gives it the most plane pieces)
  const int cnt = std::max<int>(1, (int)L.h[si].size());
  if (std::max(sweep_blocks(n, 1, shape_for(P, n, false, cnt)),
               sweep_blocks(n, 1, shape_for(P, n, true, cnt))) > kSweepParts)
    return 0;
  if (red) *red = sweep_blocks(n, cnt, shape_for(P, n, !L.const_b(si), cnt));
  return sweep_blocks(n, cnt, shape_for(P, n, false, cnt));
}

// One V(nu1,nu2) cycle with the P1 finite-element operator: two-pass
// red-black Gauss-Seidel in place in buffer 0, residual and full weighting as
// two kernels, trilinear correction, exact 3^3 solve.
static void run_cycle_fe(mg_plan_s* P, Batch* B, Lists<double>& Ls) {
  const int nu1 = P->desc.nu1, nu2 = P->desc.nu2;
  const size_t L = B->sizes.size();
  hipStream_t st = B->st;
  for (size_t si = 0; si < L; ++si) {
    const int n = B->sizes[si];
    const int cnt = (int)Ls.h[si].size();
    if (n == 3) {
      launch_fe_coarsest(Ls.d[si], cnt, B->ss.active, st);
      continue;
    }
    for (int s = 0; s < nu1; ++s) {
      if (P->prof && si == 0) prof_begin(P, 4, n, P->prof_cycle, st);
      launch_fe_colour(Ls.d[si], cnt, n, B->ss.active, 0, st);
      launch_fe_colour(Ls.d[si], cnt, n, B->ss.active, 1, st);
      if (P->prof && si == 0) prof_end(P, st);
    }
    launch_fe_residual(Ls.d[si], cnt, n, B->ss.active, st);
    launch_restrict<double>(Ls.d[si], cnt, n, B->ss.active, st);
  }
  for (size_t si = L - 1; si-- > 0;) {
    const int n = B->sizes[si];
    const int cnt = (int)Ls.h[si].size();
    launch_prolong<double>(Ls.d[si], cnt, n, B->ss.active, 0, 0, st);
    for (int s = 0; s < nu2; ++s) {
      if (P->prof && si == 0) prof_begin(P, 4, n, P->prof_cycle, st);
      launch_fe_colour(Ls.d[si], cnt, n, B->ss.active, 0, st);
      launch_fe_colour(Ls.d[si], cnt, n, B->ss.active, 1, st);
      if (P->prof && si == 0) prof_end(P, st);
    }
  }
}

// One V(nu1,nu2) cycle on every active solve.  Each level starts in buffer 0
// (the iterate of a top grid, the zero guess of a coarse one); returns the
// buffer that holds the top grids' iterates afterwards.  With norms (the FP64
// cycles), on a size whose top grids qualify (lagged_parts) the last sweep
// sums the squared residuals at the black points of the iterate it makes, the
// next cycle's first sweep those at the red points of the same iterate, and
// the solves are judged right after that sweep (the iterate of the previous
// cycle: lag 1).
template <typename T>
static int run_cycle(mg_plan_s* P, Batch* B, Lists<T>& Ls, bool norms = false, double tol = 0.0,
                     int fixed = 0) {
  const int nu1 = P->desc.nu1, nu2 = P->desc.nu2;
  const size_t L = B->sizes.size();
  hipStream_t st = B->st;
  std::vector<int> cur(L, 0);
  // sizes from `small` down run in the LDS V-cycle kernel
  const size_t small = Ls.chain_si >= 0 ? (size_t)Ls.chain_si : L;
  for (size_t si = 0; si < small; ++si) {
    const int n = B->sizes[si];
    const int cnt = (int)Ls.h[si].size();
    if (n == 3) {
      launch_coarsest<T>(Ls.d[si], cnt, B->ss.active, st);
      continue;
    }
    int lpr = 0, lp = 0;
    if constexpr (std::is_same<T, double>::value)
      if (norms) lp = lagged_parts(P, B, si, &lpr, &Ls);
    for (int s = 0; s < nu1; ++s) {
      cur[si] = smooth_once<T>(P, B, Ls, si, cur[si], -1, P->prof && si == 0,
                               s == 0 && lp > 0 ? (T*)B->ss.spart + kSweepParts : nullptr, 1);
      if constexpr (std::is_same<T, double>::value) {
        if (s == 0 && lp > 0) {
          // judge the incoming iterates now: a solve that stops keeps it in
          // buffer 0 (this sweep wrote buffer 1; nothing after it runs for it)
          const size_t ti = size_index(B->top_sizes, n);
          launch_finalize2(Ls.dtop[ti], (int)Ls.htop[ti].size(), B->ss, RED_RESID, 1, 1,
                           fixed, P->desc.max_cycles, tol, st, lp, lpr);
        }
      }
    }
    // the one-pass transfer (same results as the separate kernels; it splits
    // its plane marches when a launch has few grids, and addresses whole
    // grids with 32-bit offsets, as the fused sweep)
    if (P->transfer == 0 && sweep_fits(n, sizeof(T))) {
      launch_resrestrict<T>(Ls.d[si], cnt, n, B->ss.active, cur[si], st, Ls.const_b(si),
                            P->kl_inline && Ls.kl(si));
    } else {
      launch_residual<T>(Ls.d[si], cnt, n, B->ss.active, cur[si], st);
      launch_restrict<T>(Ls.d[si], cnt, n, B->ss.active, st);
    }
  }
  size_t up = L - 1;  // the levels above this one are corrected and post-smoothed
  if (small < L) {
    for (const auto& g : Ls.chains)
      launch_vsmall<T>(g.d, (int)g.h.size(), g.ns, B->ss.active, nu1, nu2, st);
    cur[small] = 0;
    up = small;
  }
  for (size_t si = up; si-- > 0;) {
    const int n = B->sizes[si];
    const int cnt = (int)Ls.h[si].size();
    const int cbuf = cur[si + 1];
    if (nu2 == 0) {
      launch_prolong<T>(Ls.d[si], cnt, n, B->ss.active, cur[si], cbuf, st);
      continue;
    }
    int lp = 0;
    if constexpr (std::is_same<T, double>::value)
      if (norms) lp = lagged_parts(P, B, si, nullptr, &Ls);
    cur[si] = smooth_once<T>(P, B, Ls, si, cur[si], cbuf, P->prof && si == 0);
    for (int s = 1; s < nu2; ++s)
      cur[si] = smooth_once<T>(P, B, Ls, si, cur[si], -1, P->prof && si == 0,
                               s == nu2 - 1 && lp > 0 ? (T*)B->ss.spart : nullptr, 2);
  }
  return cur[0];
}

// One outer iteration for every active solve (recorded into graphs as is).
static void cycle_step(mg_plan_s* P, Batch* B, double tol, int fixed) {
  hipStream_t st = B->st;
  Lists<double>& L = B->L64;
  if (P->prof) ++P->prof_cycle;  // (eager while profiling: one call per cycle)
  // V-cycles per step, credited to each active solve by its judgement: a
  // mixed-precision step applies inner_cycles
  const int per_step = B->spec.mixed ? P->inner_cycles : 1;
  if (B->spec.fe) {
    run_cycle_fe(P, B, L);
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
      const int n = B->top_sizes[ti], cnt = (int)L.htop[ti].size();
      launch_fe_residual(L.dtop[ti], cnt, n, B->ss.active, st);
      launch_reduce(L.dtop[ti], cnt, n, B->ss.active, 0, RED_R2, B->ss.partials, st);
      launch_finalize2(L.dtop[ti], cnt, B->ss, RED_RESID, 1, 0, fixed,
                       P->desc.max_cycles, tol, st);
    }
  } else if (!B->spec.mixed) {
    const int out = run_cycle<double>(P, B, L, true, tol, fixed);
    if (out != 0)  // odd sweep count: bring the top iterates back to buffer 0
      for (size_t ti = 0; ti < B->top_sizes.size(); ++ti)
        launch_copy_buf<double>(L.dtop[ti], (int)L.htop[ti].size(), B->top_sizes[ti],
                                B->ss.active, 1, st);
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
      const int n = B->top_sizes[ti], cnt = (int)L.htop[ti].size();
      if (lagged_parts(P, B, size_index(B->sizes, n)) > 0) continue;  // judged in the sweep
      if (B->count_only) {
        launch_finalize2(L.dtop[ti], cnt, B->ss, RED_COUNT, 1, 0, fixed, P->desc.max_cycles, tol,
                         st);
        continue;
      }
      launch_reduce(L.dtop[ti], cnt, n, B->ss.active, 0, RED_RESID, B->ss.partials, st);
      launch_finalize2(L.dtop[ti], cnt, B->ss, RED_RESID, 1, 0, fixed,
                       P->desc.max_cycles, tol, st);
    }
  } else {
    // defect of the current iterate (this also decides convergence of the
    // previous outer step), one FP32 V-cycle, FP64 update
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
      const int n = B->top_sizes[ti], cnt = (int)B->L64.htop[ti].size();
      launch_defect(B->L64.dtop[ti], B->L32.dtop[ti], cnt, n, B->ss.active, B->ss.partials, st);
      launch_finalize2(B->L64.dtop[ti], cnt, B->ss, RED_RESID, per_step, per_step, fixed,
                       P->desc.max_cycles, tol, st);
    }
    // inner_cycles FP32 V-cycles on A e = r from e = 0; the next one starts
    // from the last one's e (in buffer 0)
    int out = 0;
    for (int c = 0; c < P->inner_cycles; ++c) {
      if (out != 0)
        for (size_t ti = 0; ti < B->top_sizes.size(); ++ti)
          launch_copy_buf<float>(B->L32.dtop[ti], (int)B->L32.htop[ti].size(), B->top_sizes[ti],
                                 B->ss.active, 1, st);
      out = run_cycle<float>(P, B, B->L32);
    }
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti)
      launch_correct(B->L64.dtop[ti], B->L32.dtop[ti], (int)B->L64.htop[ti].size(),
                     B->top_sizes[ti], B->ss.active, out, st);
  }
}

static hipGraphExec_t graph_for(mg_plan_s* P, Batch* B, int c, double tol, int fixed) {
  auto it = B->graphs.find(c);
  if (it != B->graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  CK(hipStreamBeginCapture(B->st, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < c; ++i) cycle_step(P, B, tol, fixed);
  CK(hipStreamEndCapture(B->st, &g));
  hipGraphExec_t ex = nullptr;
  CK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  CK(hipGraphDestroy(g));
  B->graphs[c] = ex;
  return ex;
}

// Cycle every solve of the batch until each has converged (or run exactly
// fixed_cycles).  Returns true when every solve met tol.
// post: enqueued after every launch of cycles, before the host waits (work
// that is valid once the last launch is done, e.g. the QoI of stopped solves);
// qpend: the initial QoI-pending flag of every solve.
static bool run_solves(mg_plan_s* P, Batch* B, double tol, int fixed, bool graphs,
                       const std::function<void()>& post = nullptr, int qpend = 0) {
  hipStream_t st = B->st;
  P->prof_cycle = 0;
  launch_init_state2(B->ss, B->ns, st, qpend);
  // ||b'|| per solve (a constant top right-hand side gives the same norms for
  // every batch of this workspace)
  if (!(B->spec.const_b_top && B->bnorm_ready)) {
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
      const int n = B->top_sizes[ti], cnt = (int)B->L64.htop[ti].size();
      launch_reduce(B->L64.dtop[ti], cnt, n, B->ss.active, 0, RED_BNORM, B->ss.partials, st);
      launch_finalize2(B->L64.dtop[ti], cnt, B->ss, RED_BNORM, 0, 0, fixed,
                       P->desc.max_cycles, tol, st);
    }
    B->bnorm_ready = B->spec.const_b_top;
  }
  // mixed precision, and top grids judged in the next cycle's first sweep,
  // decide convergence one step late: one extra step
  int extra = B->spec.mixed ? 1 : 0;
  for (int n : B->top_sizes)
    if (lagged_parts(P, B, size_index(B->sizes, n)) > 0) extra = 1;
  // (in steps of cycle_step: a mixed-precision step is inner_cycles V-cycles)
  const int per_step = B->spec.mixed ? P->inner_cycles : 1;
  const int limit = ceil_div(fixed > 0 ? fixed : P->desc.max_cycles, per_step) + extra;
  const bool use_graphs = graphs && P->use_graph && !P->prof;
  const int* cyc = B->h_state + B->ns;
  int done = 0, maxc = 0, left = B->ns;
  while (done < limit) {
    int c = 1;
    if (use_graphs) {
      // the first launch covers the steps the last batch needed (a step in
      // which every solve has stopped costs only launches that exit at once;
      // a missing one costs a round trip to the host)
      const int guess = fixed > 0 ? ceil_div(fixed, per_step) + extra : B->last_cycles;
      c = done == 0 ? std::max(1, std::min(limit, guess)) : 1;
      CK(hipGraphLaunch(graph_for(P, B, c, tol, fixed), st));
    } else {
      cycle_step(P, B, tol, fixed);
    }
    done += c;
    if (post) post();
    // the active flags and cycle counts of every solve in one copy
    CK(hipMemcpyAsync(B->h_state, B->ss.active, sizeof(int) * 2 * B->ns, hipMemcpyDeviceToHost,
                      st));
    CK(hipStreamSynchronize(st));
    left = 0;
    for (int q = 0; q < B->ns; ++q) left += B->h_state[q] != 0;
    if (left == 0) break;
  }
  bool ok = left == 0;
  for (int q = 0; q < B->ns; ++q) {
    if (cyc[q] < 0) ok = false;
    maxc = std::max(maxc, cyc[q]);
  }
  B->last_cycles = ceil_div(maxc, per_step) + extra;
  return ok;
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

static int level_n(mg_plan_s* P, int level) { return (P->desc.n0 - 1) * (1 << level) + 1; }

// Solves of a batch of samples: sample i owns solve fi[i] on n_{l_i} and, for
// l_i > 0, solve fi[i] + 1 on n_{l_i - 1}, which shares the fine solve's
// coefficients from its second multigrid level down.
static BatchSpec mlmc_spec(mg_plan_s* P, const std::vector<int>& levels) {
  BatchSpec spec;
  for (int l : levels) {
    spec.top_n.push_back(level_n(P, l));
    spec.share.push_back(-1);
    if (l > 0) {
      spec.top_n.push_back(level_n(P, l - 1));
      // the coarse solve's coefficient is the fine one's injection (KL), or a
      // field of its own (SPDE: a coarse box solve of the same noise)
      spec.share.push_back(P->field_spde ? -1 : (int)spec.top_n.size() - 2);
    }
  }
  spec.const_b_top = true;
  spec.ext_u_top = false;
  spec.mixed = P->desc.precision == MG_MIXED;
  spec.fe = P->op_fe != 0;
  return spec;
}

// Fields, coefficient hierarchy and zero iterates for a batch of samples.
static int spde_fields(mg_plan_s* P, int level, const uint64_t* seeds, int S,
                       const std::vector<double*>& outs_f, const std::vector<double*>& outs_c,
                       int mode);

static int setup_samples(mg_plan_s* P, Batch* B, const std::vector<int>& levels,
                         const uint64_t* seeds) {
  hipStream_t st = P->work;
  const int n_samples = (int)levels.size();
  if (B->nsamples != n_samples) {
    B->nsamples = n_samples;
    B->d_seeds = (uint64_t*)B->dalloc(sizeof(uint64_t) * n_samples);
    if (B->h_seeds) CK(hipHostFree(B->h_seeds));
    CK(hipHostMalloc((void**)&B->h_seeds, sizeof(uint64_t) * n_samples, hipHostMallocDefault));
    B->d_levels = (int*)B->dalloc(sizeof(int) * n_samples);
    B->d_normals = (double*)B->dalloc(sizeof(double) * 64 * n_samples);
    std::vector<int> fi(n_samples), ci(n_samples);
    std::map<int, std::pair<std::vector<double*>, std::vector<int>>> groups;
    const bool kl = !P->field_spde && !B->spec.fe;
    B->kl_normals.assign(kl ? B->ns : 0, nullptr);
    int s = 0;
    for (int i = 0; i < n_samples; ++i) {
      fi[i] = s;
      ci[i] = levels[i] > 0 ? s + 1 : -1;
      groups[levels[i]].first.push_back(B->lev[s][0].wh);
      groups[levels[i]].second.push_back(i);
      if (kl) {
        // both solves of a pair take the sample's normals
        B->kl_normals[s] = B->d_normals + 64 * (size_t)i;
        if (levels[i] > 0) B->kl_normals[s + 1] = B->kl_normals[s];
      }
      s += levels[i] > 0 ? 2 : 1;
    }
    upload_lists(P, B);
    B->d_fi = (int*)B->dalloc(sizeof(int) * n_samples);
    B->d_ci = (int*)B->dalloc(sizeof(int) * n_samples);
    CK(hipMemcpy(B->d_fi, fi.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_ci, ci.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_levels, levels.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice));
    for (auto& kv : groups) {
      Batch::FieldGroup g;
      g.n = level_n(P, kv.first);
      g.count = (int)kv.second.first.size();
      g.d_out = (double**)B->dalloc(sizeof(double*) * g.count);
      g.d_xi = (int*)B->dalloc(sizeof(int) * g.count);
      CK(hipMemcpy(g.d_out, kv.second.first.data(), sizeof(double*) * g.count, hipMemcpyHostToDevice));
      CK(hipMemcpy(g.d_xi, kv.second.second.data(), sizeof(int) * g.count, hipMemcpyHostToDevice));
      B->fields.push_back(g);
    }
  }
  // (the previous batch's upload from the staging buffer finished before that
  // batch returned)
  std::memcpy(B->h_seeds, seeds, sizeof(uint64_t) * n_samples);
  CK(hipMemcpyAsync(B->d_seeds, B->h_seeds, sizeof(uint64_t) * n_samples, hipMemcpyHostToDevice,
                    st));
  if (P->field_spde) {
    // the SPDE sampler, level by level (fine and coarse box solves)
    std::map<int, std::vector<int>> groups;
    for (int i = 0; i < n_samples; ++i) groups[levels[i]].push_back(i);
    std::vector<int> fi(n_samples);
    for (int i = 0, s = 0; i < n_samples; ++i) {
      fi[i] = s;
      s += levels[i] > 0 ? 2 : 1;
    }
    for (const auto& kv : groups) {
      std::vector<double*> outs_f, outs_c;
      std::vector<uint64_t> sd;
      for (int i : kv.second) {
        outs_f.push_back(B->lev[fi[i]][0].wh);
        if (kv.first > 0) outs_c.push_back(B->lev[fi[i] + 1][0].wh);
        sd.push_back(seeds[i]);
      }
      const int stt = spde_fields(P, kv.first, sd.data(), (int)sd.size(), outs_f, outs_c, 0);
      if (stt != MG_OK) return stt;
    }
  } else {
    launch_philox(B->d_seeds, n_samples, 0, nullptr, B->d_normals, st, B->d_levels);
    for (const auto& g : B->fields)
      launch_field(g.n, g.count, g.d_out, g.d_xi, B->d_normals, phi_table(P, g.n), P->d_coef, 0,
                   st);
  }
  prepare_coefficients(P, B);
  // every sample starts from the zero iterate (the workspace may hold the last batch)
  for (size_t ti = 0; ti < B->top_sizes.size(); ++ti)
    launch_zero_u<double>(B->L64.dtop[ti], (int)B->L64.htop[ti].size(), B->top_sizes[ti], st);
  return MG_OK;
}

// Samples of (possibly different) levels in one batch: one launch per grid
// size and V-cycle step covers every sample that has a grid of that size.
static int run_samples(mg_plan_s* P, const std::vector<int>& levels, const uint64_t* seeds,
                       double* Y_out, double* Qf_out, double* Qc_out, int* cycles_out,
                       int fixed_cycles) {
  int status = MG_OK;
  order_after_caller(P);
  Batch* B = get_batch(P, mlmc_spec(P, levels), &status);
  if (!B) return status;
  hipStream_t st = P->work;
  const int n_samples = (int)levels.size();
  {
    const int stt = setup_samples(P, B, levels, seeds);
    if (stt != MG_OK) {
      P->err = "an SPDE field solve missed its tolerance";
      return stt;
    }
  }
  if (fixed_cycles > 0) B->drop_graphs();  // graphs bake in the stopping mode
  // the QoI and Y are enqueued after every launch of cycles: once the solves
  // have stopped, the host's wait for the last launch covers them too.  Each
  // solve's QoI is taken once, after the launch in which it stopped (its
  // iterate does not change afterwards); Y is formed again each time.
  auto qoi = [&](int mode) {
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
      const int n = B->top_sizes[ti], cnt = (int)B->L64.htop[ti].size();
      launch_reduce(B->L64.dtop[ti], cnt, n, B->ss.active, 0, mode, B->ss.partials, st,
                    B->ss.qpend);
      launch_finalize2(B->L64.dtop[ti], cnt, B->ss, mode, 0, 0, 0, 0, 0.0, st);
    }
    launch_ydiff(B->ss.q, B->d_fi, B->d_ci, n_samples, Y_out, Qf_out, Qc_out, B->ss.cycles,
                 cycles_out, st);
  };
  bool ok;
  if (P->qoi_kind == QOI_INTEGRAL) {
    ok = run_solves(P, B, P->desc.tol, fixed_cycles, fixed_cycles == 0,
                    [&]() { qoi(RED_QOI_PENDING); }, 1);
    if (!ok) {
      // solves that missed tol never stopped: their QoI from the last iterate
      qoi(RED_QOI);
      CK(hipStreamSynchronize(st));
    }
  } else {
    // the point value or the plane flux, once every solve has stopped (the
    // top iterates are in buffer 0)
    ok = run_solves(P, B, P->desc.tol, fixed_cycles, fixed_cycles == 0);
    for (size_t ti = 0; ti < B->top_sizes.size(); ++ti)
      launch_qoi_pf(B->L64.dtop[ti], (int)B->L64.htop[ti].size(), P->qoi_kind, B->ss.q, st);
    launch_ydiff(B->ss.q, B->d_fi, B->d_ci, n_samples, Y_out, Qf_out, Qc_out, B->ss.cycles,
                 cycles_out, st);
    CK(hipStreamSynchronize(st));
  }
  if (P->prof) collect_profile(P);
  if (!ok) {
    P->err = "some solve missed tol within max_cycles";
    return MG_ENOCONV;
  }
  return MG_OK;
}


// ---- full multigrid samples (Section 7.1's FMG-nu V(nu1,nu2) schedule) -----------
//
// Nested iteration on every solve of a sample: the 3^3 grid solved exactly,
// then on each finer grid size the trilinear interpolation of the coarser
// grid's result as initial guess and fmg_cycles V(nu1,nu2) cycles against
// that grid's own problem (f = 1: b' = h^2).  One batch per grid size holds
// the samples' grids of that size with their coefficient hierarchies (the
// field evaluated at that size's vertices: the same formula at the same
// dyadic points as injection).  The schedule of the fine solve of Y_l passes
// through the coarse solve's whole schedule, so both QoIs of a sample come
// from one pass: Q_f from the n_l stage, Q_c from the n_(l-1) stage.

static Batch* fmg_stage(mg_plan_s* P, int n, int S) {
  auto& slot = P->fmg[n];
  if (!slot || slot->ns != S) {
    slot.reset();
    BatchSpec spec;
    spec.top_n.assign(S, n);
    spec.share.assign(S, -1);
    spec.const_b_top = true;
    spec.ext_u_top = false;
    spec.mixed = false;
    auto B = build_batch(P, spec);
    if (!B) return nullptr;
    B->count_only = true;  // stages run fixed cycles; no residual is reported
    B->nsamples = S;
    B->d_seeds = (uint64_t*)B->dalloc(sizeof(uint64_t) * S);
    B->d_levels = (int*)B->dalloc(sizeof(int) * S);
    B->d_normals = (double*)B->dalloc(sizeof(double) * 64 * S);
    if (!P->field_spde && !P->op_fe) {
      B->kl_normals.resize(S);
      for (int i = 0; i < S; ++i) B->kl_normals[i] = B->d_normals + 64 * (size_t)i;
    }
    upload_lists(P, B.get());
    B->d_fi = (int*)B->dalloc(sizeof(int) * S);  // output position of each sample
    Batch::FieldGroup g;
    g.n = n;
    g.count = S;
    g.d_out = (double**)B->dalloc(sizeof(double*) * S);
    g.d_xi = (int*)B->dalloc(sizeof(int) * S);
    std::vector<double*> outs(S);
    std::vector<int> xi(S);
    for (int i = 0; i < S; ++i) {
      outs[i] = B->lev[i][0].wh;
      xi[i] = i;
    }
    CK(hipMemcpy(g.d_out, outs.data(), sizeof(double*) * S, hipMemcpyHostToDevice));
    CK(hipMemcpy(g.d_xi, xi.data(), sizeof(int) * S, hipMemcpyHostToDevice));
    B->fields.push_back(g);
    slot = std::move(B);
  }
  return slot.get();
}

// The top descriptors of `fine` with uc[0] = the top iterate of the same
// sample in `coarse` (the previous stage), for the interpolation.
static GridDesc* fmg_link(Batch* fine, Batch* coarse) {
  if (fine->link_src == coarse && fine->d_link) return fine->d_link;
  const int S = fine->ns;
  std::vector<GridDesc> h = fine->L64.htop[0];
  for (int i = 0; i < S; ++i) {
    h[i].uc[0] = coarse->lev[i][0].u[0];
    h[i].uc[1] = coarse->lev[i][0].u[0];
  }
  if (!fine->d_link) fine->d_link = (GridDesc*)fine->dalloc(sizeof(GridDesc) * S);
  CK(hipMemcpy(fine->d_link, h.data(), sizeof(GridDesc) * S, hipMemcpyHostToDevice));
  fine->link_src = coarse;
  return fine->d_link;
}

// Samples of one level by full multigrid; out_pos[i]: the output position of
// sample i.  Every stage runs a fixed schedule, so no solve can miss a tol.
static int run_fmg_level(mg_plan_s* P, int level, const uint64_t* seeds,
                         const std::vector<int>& out_pos, double* Y_out, double* Qf_out,
                         double* Qc_out, int* cycles_out) {
  hipStream_t st = P->work;
  const int S = (int)out_pos.size();
  const int nL = level_n(P, level);
  std::vector<int> sizes = hierarchy(nL);
  std::reverse(sizes.begin(), sizes.end());  // 3, 5, ..., n_level
  Batch* prev = nullptr;
  Batch* fine = nullptr;
  Batch* coarse = nullptr;
  std::vector<int> lv(S, level);
  for (int n : sizes) {
    Batch* B = fmg_stage(P, n, S);
    if (!B) {
      P->err = "full multigrid stages exceed the plan's HBM budget";
      return MG_ENOMEM;
    }
    // the samples' normals (omega of (seed, level)) and the field at this size
    CK(hipMemcpy(B->d_seeds, seeds, sizeof(uint64_t) * S, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_levels, lv.data(), sizeof(int) * S, hipMemcpyHostToDevice));
    CK(hipMemcpy(B->d_fi, out_pos.data(), sizeof(int) * S, hipMemcpyHostToDevice));
    launch_philox(B->d_seeds, S, 0, nullptr, B->d_normals, st, B->d_levels);
    for (const auto& g : B->fields)
      launch_field(g.n, g.count, g.d_out, g.d_xi, B->d_normals, phi_table(P, g.n), P->d_coef, 0,
                   st);
    prepare_coefficients(P, B);
    launch_zero_u<double>(B->L64.dtop[0], S, n, st);
    if (prev) {
      GridDesc* d_link = fmg_link(B, prev);
      launch_init_state2(B->ss, S, st);  // active flags for the interpolation
      launch_prolong<double>(d_link, S, n, B->ss.active, 0, 0, st);
    }
    // the 3^3 grid: one exact solve; above: the fixed V-cycles
    run_solves(P, B, P->desc.tol, n == 3 ? 1 : P->fmg_cycles, false);
    if (n == nL) fine = B;
    if (level > 0 && n == level_n(P, level - 1)) coarse = B;
    prev = B;
  }
  for (Batch* B : {fine, coarse}) {
    if (!B) continue;
    if (P->qoi_kind == QOI_INTEGRAL) {
      launch_reduce(B->L64.dtop[0], S, B->top_sizes[0], B->ss.active, 0, RED_QOI, B->ss.partials,
                    st);
      launch_finalize2(B->L64.dtop[0], S, B->ss, RED_QOI, 0, 0, 0, 0, 0.0, st);
    } else {
      launch_qoi_pf(B->L64.dtop[0], S, P->qoi_kind, B->ss.q, st);
    }
  }
  launch_ydiff2(fine->ss.q, coarse ? coarse->ss.q : nullptr, S, fine->d_fi, Y_out, Qf_out,
                Qc_out, P->fmg_cycles, P->fmg_cycles, cycles_out, st);
  CK(hipStreamSynchronize(st));
  return MG_OK;
}

static int run_samples_fmg(mg_plan_s* P, const std::vector<int>& levels, const uint64_t* seeds,
                           double* Y_out, double* Qf_out, double* Qc_out, int* cycles_out) {
  if (P->desc.precision != MG_FP64) {
    P->err = "full multigrid runs in FP64 only";
    return MG_ENOTIMPL;
  }
  order_after_caller(P);
  std::map<int, std::vector<int>> groups;
  for (int i = 0; i < (int)levels.size(); ++i) groups[levels[i]].push_back(i);
  for (auto& kv : groups) {
    std::vector<uint64_t> sd;
    for (int i : kv.second) sd.push_back(seeds[i]);
    const int st = run_fmg_level(P, kv.first, sd.data(), kv.second, Y_out, Qf_out, Qc_out,
                                 cycles_out);
    if (st != MG_OK) return st;
  }
  return MG_OK;
}

// ---- SPDE field sampler (Section 3.2, eq. spde) ------------------------------------
//
// The fields of a batch's samples from (kappa^2 - Laplace) Z = W on the box
// (-1,2)^3: per sample the white-noise load on the fine box grid, a V(2,2)
// solve to relative residual 1e-10 over every box vertex (natural Neumann
// boundary), k = exp(sigma sqrt(8 pi kappa) Z) at D's vertices (kappa =
// 1/lambda); the coarse solve of Y_l takes the same noise on the coarse box
// grid (its load P^T b / 2) and its own box solve.
constexpr double kSpdeTol = 1e-10;
constexpr int kSpdeMaxCycles = 50;

struct SpdeWork {
  int S = 0;
  std::vector<int> nts;                  // box sizes per level, descending (.. 4)
  std::vector<std::vector<SpdeGrid>> h;  // per level: S descriptors
  std::vector<SpdeGrid*> d;              // their device copies
  void* mem = nullptr;
  int* d_active = nullptr;
  int* d_cycles = nullptr;
  double* d_bnorm = nullptr;
  double* d_part = nullptr;
  int* h_active = nullptr;               // pinned
  uint64_t* d_seeds = nullptr;
  int* d_levels = nullptr;
  double** d_out = nullptr;              // field targets of the S solves
  SpdeGrid* d_link = nullptr;            // top descriptors with bc/zc of another box size
  ~SpdeWork() {
    if (mem) (void)hipFree(mem);
    if (h_active) (void)hipHostFree(h_active);
  }
};

static SpdeWork* spde_work(mg_plan_s* P, int nt, int S, double h) {
  auto& slot = P->spde[{nt, S}];
  if (slot) return slot.get();
  auto W = std::make_unique<SpdeWork>();
  W->S = S;
  for (int m = nt;; m = (m - 1) / 2 + 1) {
    W->nts.push_back(m);
    if ((m - 1) & 1) break;  // an odd number of intervals: the coarsest box grid
  }
  const int L = (int)W->nts.size();
  size_t total = 0;
  for (int m : W->nts) total += align256(3 * sizeof(double) * (size_t)m * m * m) * (size_t)S;
  const int part = spde_blocks(nt);
  const size_t extra = align256(sizeof(int) * 2 * S) + align256(sizeof(double) * S) +
                       align256(sizeof(double) * (size_t)S * part) + align256(sizeof(uint64_t) * S) +
                       align256(sizeof(int) * S) + align256(sizeof(double*) * S) +
                       align256(sizeof(SpdeGrid) * S) * (size_t)(L + 1);
  CK(hipMalloc(&W->mem, total + extra));
  char* cur = (char*)W->mem;
  auto take = [&](size_t b) {
    void* p = cur;
    cur += align256(b);
    return p;
  };
  W->h.assign(L, std::vector<SpdeGrid>(S));
  double hl = h;
  const double kappa = 1.0 / P->desc.corr_len;
  for (int l = 0; l < L; ++l, hl *= 2.0) {
    const size_t N = (size_t)W->nts[l] * W->nts[l] * W->nts[l];
    for (int g = 0; g < S; ++g) {
      SpdeGrid& G = W->h[l][g];
      double* a = (double*)take(3 * sizeof(double) * N);
      G.z = a;
      G.b = a + N;
      G.r = a + 2 * N;
      G.nt = W->nts[l];
      G.k2h2 = kappa * kappa * hl * hl;
      G.solve = g;
    }
  }
  for (int l = 0; l + 1 < L; ++l)
    for (int g = 0; g < S; ++g) {
      W->h[l][g].zc = W->h[l + 1][g].z;
      W->h[l][g].bc = W->h[l + 1][g].b;
    }
  W->d_active = (int*)take(sizeof(int) * 2 * S);
  W->d_cycles = W->d_active + S;
  W->d_bnorm = (double*)take(sizeof(double) * S);
  W->d_part = (double*)take(sizeof(double) * (size_t)S * part);
  W->d_seeds = (uint64_t*)take(sizeof(uint64_t) * S);
  W->d_levels = (int*)take(sizeof(int) * S);
  W->d_out = (double**)take(sizeof(double*) * S);
  for (int l = 0; l < L; ++l) {
    W->d.push_back((SpdeGrid*)take(sizeof(SpdeGrid) * S));
    CK(hipMemcpy(W->d[l], W->h[l].data(), sizeof(SpdeGrid) * S, hipMemcpyHostToDevice));
  }
  W->d_link = (SpdeGrid*)take(sizeof(SpdeGrid) * S);
  CK(hipHostMalloc((void**)&W->h_active, sizeof(int) * S, hipHostMallocDefault));
  slot = std::move(W);
  return slot.get();
}

// Solve every grid of W from z = 0 (its top b set); returns false if a solve
// missed kSpdeTol.
static bool spde_solve(mg_plan_s* P, SpdeWork* W) {
  hipStream_t st = P->work;
  const int S = W->S, L = (int)W->nts.size(), nt = W->nts[0];
  CK(hipMemsetD32Async(W->d_active, 1, S, st));
  for (int g = 0; g < S; ++g)
    launch_fill(W->h[0][g].z, (long)nt * nt * nt, 0.0, st);
  launch_spde_sumsq(W->d[0], S, nt, W->d_active, 1, W->d_part, st);
  launch_spde_judge(W->d[0], S, nt, W->d_active, W->d_cycles, W->d_bnorm, W->d_part, 0, 0.0, 0, 1,
                    st);
  int left = S;
  for (int c = 1; c <= kSpdeMaxCycles && left > 0; ++c) {
    for (int l = 0; l + 1 < L; ++l) {
      for (int s2 = 0; s2 < 2; ++s2) {
        if (P->prof && l == 0) prof_begin(P, 5, nt, c, st);
        launch_spde_colour(W->d[l], S, W->nts[l], W->d_active, 0, st);
        launch_spde_colour(W->d[l], S, W->nts[l], W->d_active, 1, st);
        if (P->prof && l == 0) prof_end(P, st);
      }
      launch_spde_residual(W->d[l], S, W->nts[l], W->d_active, st);
      launch_spde_restrict(W->d[l], S, W->nts[l], W->d_active, false, st);
    }
    launch_spde_coarsest(W->d[L - 1], S, W->nts[L - 1], W->d_active, st);
    for (int l = L - 1; l-- > 0;) {
      launch_spde_prolong(W->d[l], S, W->nts[l], W->d_active, st);
      for (int s2 = 0; s2 < 2; ++s2) {
        if (P->prof && l == 0) prof_begin(P, 5, nt, c, st);
        launch_spde_colour(W->d[l], S, W->nts[l], W->d_active, 0, st);
        launch_spde_colour(W->d[l], S, W->nts[l], W->d_active, 1, st);
        if (P->prof && l == 0) prof_end(P, st);
      }
    }
    launch_spde_residual(W->d[0], S, nt, W->d_active, st);
    launch_spde_sumsq(W->d[0], S, nt, W->d_active, 0, W->d_part, st);
    launch_spde_judge(W->d[0], S, nt, W->d_active, W->d_cycles, W->d_bnorm, W->d_part, c,
                      kSpdeTol, kSpdeMaxCycles, 0, st);
    CK(hipMemcpyAsync(W->h_active, W->d_active, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    left = 0;
    for (int g = 0; g < S; ++g) left += W->h_active[g] != 0;
  }
  std::vector<int> cyc(S);
  CK(hipMemcpy(cyc.data(), W->d_cycles, sizeof(int) * S, hipMemcpyDeviceToHost));
  for (int c : cyc)
    if (c < 0) return false;
  return true;
}

// Fields of S samples of one MLMC level: fine into outs_f (n_f grids), for
// level > 0 coarse into outs_c (n_c grids); mode 0 writes wh, 1 writes k.
static int spde_fields(mg_plan_s* P, int level, const uint64_t* seeds, int S,
                       const std::vector<double*>& outs_f, const std::vector<double*>& outs_c,
                       int mode) {
  hipStream_t st = P->work;
  const int nf = level_n(P, level), ntf = 3 * (nf - 1) + 1;
  const double kappa = 1.0 / P->desc.corr_len;
  const double sc = std::sqrt(P->desc.sigma2) * std::sqrt(8.0 * 3.141592653589793 * kappa);
  SpdeWork* Wf = spde_work(P, ntf, S, 1.0 / (double)(nf - 1));
  const std::vector<int> lv(S, level);
  CK(hipMemcpy(Wf->d_seeds, seeds, sizeof(uint64_t) * S, hipMemcpyHostToDevice));
  CK(hipMemcpy(Wf->d_levels, lv.data(), sizeof(int) * S, hipMemcpyHostToDevice));
  launch_spde_noise(Wf->d[0], S, ntf, Wf->d_seeds, Wf->d_levels, 1.0 / (double)(nf - 1), st);
  if (!outs_f.empty()) {
    if (!spde_solve(P, Wf)) return MG_ENOCONV;
    CK(hipMemcpy(Wf->d_out, outs_f.data(), sizeof(double*) * S, hipMemcpyHostToDevice));
    launch_spde_field(Wf->d[0], S, nf, sc, Wf->d_out, mode, st);
  }
  if (level > 0 && !outs_c.empty()) {
    const int nc = level_n(P, level - 1), ntc = 3 * (nc - 1) + 1;
    SpdeWork* Wc = spde_work(P, ntc, S, 1.0 / (double)(nc - 1));
    // the same noise on the coarse box grid: b_c = P^T b_f / 2
    std::vector<SpdeGrid> link = Wf->h[0];
    for (int g = 0; g < S; ++g) {
      link[g].bc = Wc->h[0][g].b;
      link[g].zc = Wc->h[0][g].z;
    }
    CK(hipMemcpy(Wf->d_link, link.data(), sizeof(SpdeGrid) * S, hipMemcpyHostToDevice));
    CK(hipMemsetD32Async(Wf->d_active, 1, S, st));
    launch_spde_restrict(Wf->d_link, S, ntf, Wf->d_active, true, st);
    if (!spde_solve(P, Wc)) return MG_ENOCONV;
    CK(hipMemcpy(Wc->d_out, outs_c.data(), sizeof(double*) * S, hipMemcpyHostToDevice));
    launch_spde_field(Wc->d[0], S, nc, sc, Wc->d_out, mode, st);
  }
  CK(hipStreamSynchronize(st));
  return MG_OK;
}

// ---- serving: continuous batching over resident sample slots --------------------
//
// A lane is a batch of k sample slots of one MLMC level with its own stream,
// graphs and staging buffers; the scheduler opens and evicts lanes under the
// server's HBM budget.  Lanes progress independently: a lane whose launch
// has finished is harvested (finished samples leave, their slots free up),
// admits queued requests of its level into free slots and is launched
// again, while the other lanes' work is still on the device.  So a small
// sample never waits for the cycles of larger ones.

struct Lane {
  int id = -1, level = 0, first = 0, nslots = 0;
  std::unique_ptr<Batch> B;
  hipStream_t st = nullptr;
  std::vector<int> fi, ci;                   // per local slot: fine and coarse solve
  std::vector<std::pair<int, int>> top_pos;  // per solve: (top size index, list index)
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  size_t stage_bytes = 0;
  double* d_normals = nullptr;
  int* h_state = nullptr;  // active, cycles, start, qpend of every solve
  double* h_q = nullptr;
  hipEvent_t done = nullptr;
  bool inflight = false;
  int resident = 0;
  std::map<int, hipGraphExec_t> graphs;
  ~Lane() {
    if (st) (void)hipStreamSynchronize(st);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    B.reset();
    if (d_stage) (void)hipFree(d_stage);
    if (d_normals) (void)hipFree(d_normals);
    if (h_stage) (void)hipHostFree(h_stage);
    if (h_state) (void)hipHostFree(h_state);
    if (h_q) (void)hipHostFree(h_q);
    if (done) (void)hipEventDestroy(done);
    if (st) (void)hipStreamDestroy(st);
  }
};

}  // namespace mg

struct mg_server_s {
  mg_plan_s* P = nullptr;
  std::map<int, std::unique_ptr<mg::Lane>> lanes;  // open lanes by scheduler id
  std::unique_ptr<mg::Scheduler> sched;
  std::vector<int> lane_slots;
  long long opened = 0, evicted = 0;
  double lane_seconds = 0.0;  // host time spent opening and evicting lanes
  bool failed = false;  // a step threw: lanes and scheduler may disagree
  struct Slot {
    bool busy = false;
    long long tag = 0;
    uint64_t seed = 0;
    double t_arrival = 0, t_admit = 0;
  };
  std::vector<Slot> slot;  // by slot number (grows with the scheduler's slot space)
  int resident = 0;
  long long completed = 0;
  std::deque<mg_result> done;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace mg {

// Appends arrays to a lane's pinned staging buffer; device addresses mirror it.
struct Packer {
  Lane* ln;
  size_t used = 0;
  template <typename T>
  T* put(const std::vector<T>& v) {
    used = (used + 255) & ~(size_t)255;
    if (used + v.size() * sizeof(T) > ln->stage_bytes)
      throw HipError{hipErrorOutOfMemory, "serve staging"};
    std::memcpy(ln->h_stage + used, v.data(), v.size() * sizeof(T));
    T* d = (T*)(ln->d_stage + used);
    used += v.size() * sizeof(T);
    return d;
  }
};

static size_t sample_bytes(mg_plan_s* P, int level) {
  size_t b = 0;
  build_batch(P, mlmc_spec(P, std::vector<int>{level}), &b);
  return b;
}

static size_t lane_stage_bytes(int nslots) { return (size_t)nslots * 1536 + 65536; }

// Device bytes of a lane of k slots of `level`: the batch workspace, what
// upload_lists adds to it (constant right-hand-side planes, descriptor
// lists; the small-grid chain lists counted for every grid size, so this
// bounds them), the staging buffer and the normals.
static size_t lane_bytes(mg_plan_s* P, int level, int k) {
  const BatchSpec spec = mlmc_spec(P, std::vector<int>(k, level));
  size_t b = 0;
  build_batch(P, spec, &b);
  std::set<int> sizes;
  size_t grids = 0;
  const size_t ns = spec.top_n.size();
  for (int n : spec.top_n) {
    const auto h = hierarchy(n);
    grids += h.size();
    sizes.insert(h.begin(), h.end());
  }
  const size_t nm = spec.mixed ? 2 : 1;
  const size_t desc = std::max(sizeof(GridDesc), sizeof(GridDesc32));
  const size_t chain = std::max(sizeof(SmallChain<double>), sizeof(SmallChain<float>));
  b += nm * align256(desc * (grids + ns));
  for (int n : sizes) {
    b += align256(sizeof(double) * (size_t)n * n);
    b += nm * align256(chain * ns);
    b += 2 * align256(sizeof(double*) * ns);
    if (spec.mixed) b += 2 * align256(sizeof(double*) * ns);
  }
  return b + align256(lane_stage_bytes(k)) + align256(sizeof(double) * 64 * k);
}

// A lane's workspace, lists and buffers; `bytes` is what the scheduler counts
// for it, which what it allocates must not exceed.
static std::unique_ptr<Lane> make_lane(mg_plan_s* P, int level, int first, int nslots,
                                       size_t bytes) {
  auto ln = std::make_unique<Lane>();
  ln->level = level;
  ln->first = first;
  ln->nslots = nslots;
  CK(hipStreamCreateWithFlags(&ln->st, hipStreamNonBlocking));
  CK(hipEventCreateWithFlags(&ln->done, hipEventDisableTiming));
  ln->B = build_batch(P, mlmc_spec(P, std::vector<int>(nslots, level)));
  if (!ln->B) return nullptr;
  Batch* B = ln->B.get();
  upload_lists(P, B);  // on the plan's stream, synchronised
  B->st = ln->st;
  for (int s = 0, sv = 0; s < nslots; ++s) {
    ln->fi.push_back(sv);
    ln->ci.push_back(level > 0 ? sv + 1 : -1);
    sv += level > 0 ? 2 : 1;
  }
  ln->top_pos.assign(B->ns, {-1, -1});
  for (size_t ti = 0; ti < B->L64.htop.size(); ++ti)
    for (size_t i = 0; i < B->L64.htop[ti].size(); ++i)
      ln->top_pos[B->L64.htop[ti][i].solve] = {(int)ti, (int)i};
  ln->stage_bytes = lane_stage_bytes(nslots);
  CK(hipHostMalloc((void**)&ln->h_stage, ln->stage_bytes, hipHostMallocDefault));
  CK(hipMalloc((void**)&ln->d_stage, ln->stage_bytes));
  CK(hipMalloc((void**)&ln->d_normals, sizeof(double) * 64 * nslots));
  CK(hipHostMalloc((void**)&ln->h_state, sizeof(int) * 4 * B->ns, hipHostMallocDefault));
  CK(hipHostMalloc((void**)&ln->h_q, sizeof(double) * B->ns, hipHostMallocDefault));
  const size_t got = B->bytes + B->extra_bytes + align256(ln->stage_bytes) +
                     align256(sizeof(double) * 64 * nslots);
  if (got > bytes) throw HipError{hipErrorOutOfMemory, "serving lane larger than its stated bytes"};
  // ||b'|| of every solve (constant right-hand side, fixed for the lane's
  // life); the workspace starts zeroed: no solve active, counter 0
  for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
    const int n = B->top_sizes[ti], cnt = (int)B->L64.htop[ti].size();
    launch_reduce(B->L64.dtop[ti], cnt, n, B->ss.active, 0, RED_BNORM, B->ss.partials, ln->st);
    launch_finalize2(B->L64.dtop[ti], cnt, B->ss, RED_BNORM, 0, 0, 0,
                     P->desc.max_cycles, P->desc.tol, ln->st);
  }
  CK(hipStreamSynchronize(ln->st));
  return ln;
}

// Fields, coefficient hierarchies, zero iterates and solve state of the
// samples just admitted into a lane's slots (tickets carry global slots).
static void serve_admit(mg_plan_s* P, Lane* ln, const std::vector<Ticket>& tk) {
  Batch* B = ln->B.get();
  hipStream_t st = ln->st;
  const int m = (int)tk.size();
  Packer pk{ln};
  std::vector<uint64_t> seeds(m);
  std::vector<int> levels(m, ln->level), admit, xi(m);
  std::vector<double*> out(m);
  for (int j = 0; j < m; ++j) {
    const int s = tk[j].slot - ln->first;
    seeds[j] = tk[j].seed;
    xi[j] = j;
    out[j] = B->lev[ln->fi[s]][0].wh;
    admit.push_back(ln->fi[s]);
    if (ln->ci[s] >= 0) admit.push_back(ln->ci[s]);
  }
  uint64_t* d_seeds = pk.put(seeds);
  int* d_levels = pk.put(levels);
  int* d_admit = pk.put(admit);
  double** d_out = pk.put(out);
  int* d_xi = pk.put(xi);
  // injection down each new fine hierarchy (finest size first) and FP32 copies
  struct Lst { int n, count; double** src; double** dst; float** fdst; };
  std::vector<Lst> inj, cvt;
  for (size_t si = 0; si < B->sizes.size(); ++si) {
    std::vector<double*> src, dst, csrc;
    std::vector<float*> cdst;
    for (int j = 0; j < m; ++j) {
      const int fs = ln->fi[tk[j].slot - ln->first];
      const auto& lv = B->lev[fs];
      for (size_t q = 0; q < lv.size(); ++q) {
        if (lv[q].n != B->sizes[si]) continue;
        if (q + 1 < lv.size()) {
          src.push_back(lv[q].wh);
          dst.push_back(lv[q + 1].wh);
        }
        if (B->spec.mixed) {
          csrc.push_back(lv[q].wh);
          cdst.push_back(B->lev32[fs][q].wh);
        }
      }
    }
    if (!src.empty()) inj.push_back(Lst{B->sizes[si], (int)src.size(), pk.put(src), pk.put(dst), nullptr});
    if (!csrc.empty()) cvt.push_back(Lst{B->sizes[si], (int)csrc.size(), pk.put(csrc), nullptr, pk.put(cdst)});
  }
  // top-grid descriptors of the new solves, per top size
  std::vector<std::pair<int, GridDesc*>> zero;
  for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
    std::vector<GridDesc> v;
    for (int sv : admit)
      if (ln->top_pos[sv].first == (int)ti) v.push_back(B->L64.htop[ti][ln->top_pos[sv].second]);
    if (!v.empty()) zero.push_back({(int)v.size(), pk.put(v)});
    else zero.push_back({0, nullptr});
  }
  CK(hipMemcpyAsync(ln->d_stage, ln->h_stage, pk.used, hipMemcpyHostToDevice, st));
  launch_philox(d_seeds, m, 0, nullptr, ln->d_normals, st, d_levels);
  launch_field(level_n(P, ln->level), m, d_out, d_xi, ln->d_normals, phi_table(P, level_n(P, ln->level)),
               P->d_coef, 0, st);
  for (const auto& l : inj) launch_inject(l.n, l.count, (const double* const*)l.src, l.dst, st);
  for (const auto& l : cvt) launch_to_float(l.n, l.count, (const double* const*)l.src, l.fdst, st);
  for (size_t ti = 0; ti < zero.size(); ++ti)
    if (zero[ti].first) launch_zero_u<double>(zero[ti].second, zero[ti].first, B->top_sizes[ti], st);
  launch_admit(d_admit, (int)admit.size(), B->ss, st);
}

// c cycles of every resident solve of a lane, then the QoI of the solves
// that stopped.
static void serve_cycles(mg_plan_s* P, Lane* ln, int c) {
  Batch* B = ln->B.get();
  for (int i = 0; i < c; ++i) cycle_step(P, B, P->desc.tol, 0);
  for (size_t ti = 0; ti < B->top_sizes.size(); ++ti) {
    const int n = B->top_sizes[ti], cnt = (int)B->L64.htop[ti].size();
    launch_reduce(B->L64.dtop[ti], cnt, n, B->ss.active, 0, RED_QOI_PENDING, B->ss.partials,
                  ln->st, B->ss.qpend);
    launch_finalize2(B->L64.dtop[ti], cnt, B->ss, RED_QOI_PENDING, 0, 0, 0, 0, 0.0,
                     ln->st);
  }
}

// Launch c cycles of a lane and the copy of its state back to the host.
static void lane_launch(mg_plan_s* P, Lane* ln, int c) {
  Batch* B = ln->B.get();
  if (!P->use_graph || P->prof) {
    serve_cycles(P, ln, c);
  } else {
    auto it = ln->graphs.find(c);
    if (it == ln->graphs.end()) {
      hipGraph_t g = nullptr;
      CK(hipStreamBeginCapture(ln->st, hipStreamCaptureModeThreadLocal));
      serve_cycles(P, ln, c);
      CK(hipStreamEndCapture(ln->st, &g));
      hipGraphExec_t ex = nullptr;
      CK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      CK(hipGraphDestroy(g));
      it = ln->graphs.emplace(c, ex).first;
    }
    CK(hipGraphLaunch(it->second, ln->st));
  }
  const int ns = B->ns;
  CK(hipMemcpyAsync(ln->h_state, B->ss.active, sizeof(int) * 4 * ns, hipMemcpyDeviceToHost, ln->st));
  CK(hipMemcpyAsync(ln->h_q, B->ss.q, sizeof(double) * ns, hipMemcpyDeviceToHost, ln->st));
  CK(hipEventRecord(ln->done, ln->st));
  ln->inflight = true;
}

// Finished samples of a lane whose launch has completed.
static void lane_harvest(mg_server_s* S, Lane* ln) {
  ln->inflight = false;
  S->sched->set_inflight(ln->id, false);
  const double t = S->now();
  const int ns = ln->B->ns;
  const int* cyc = ln->h_state + ns;
  const int* pend = ln->h_state + 3 * ns;
  for (int s = 0; s < ln->nslots; ++s) {
    auto& sl = S->slot[ln->first + s];
    if (!sl.busy) continue;
    const int f = ln->fi[s], g = ln->ci[s];
    if (pend[f] || (g >= 0 && pend[g])) continue;
    mg_result r{};
    r.tag = sl.tag;
    r.seed = sl.seed;
    r.level = ln->level;
    r.Qf = ln->h_q[f];
    r.Qc = g >= 0 ? ln->h_q[g] : 0.0;
    r.Y = r.Qf - r.Qc;
    r.cycles_fine = cyc[f];
    r.cycles_coarse = g >= 0 ? cyc[g] : 0;
    r.status = (r.cycles_fine < 0 || r.cycles_coarse < 0) ? MG_ENOCONV : MG_OK;
    r.t_arrival = sl.t_arrival;
    r.t_admit = sl.t_admit;
    r.t_done = t;
    S->done.push_back(r);
    sl.busy = false;
    --ln->resident;
    --S->resident;
    ++S->completed;
    S->sched->release(ln->first + s);
  }
}

// Harvest finished lanes, admit queued requests (opening and evicting lanes
// as the scheduler decides), launch every idle lane that holds samples.
// Waits until at least one lane has finished when nothing else can progress.
static void serve_step(mg_server_s* S, int c) {
  mg_plan_s* P = S->P;
  bool harvested = false;
  for (;;) {
    for (auto& kv : S->lanes) {
      Lane* ln = kv.second.get();
      if (!ln->inflight) continue;
      const hipError_t q = hipEventQuery(ln->done);
      if (q == hipSuccess) {
        lane_harvest(S, ln);
        harvested = true;
      } else if (q != hipErrorNotReady) {
        throw HipError{q, "hipEventQuery"};
      }
    }
    // admission (the scheduler admits only into lanes not in flight: an
    // in-flight lane's staging buffer is busy)
    std::vector<Ticket> tk(std::max(1, S->sched->queued()));
    tk.resize(S->sched->admit(tk.data(), (int)tk.size()));
    LaneEvent ev[64];
    for (int ne; (ne = S->sched->take_events(ev, 64)) > 0;) {
      const double t_ev = S->now();
      for (int i = 0; i < ne; ++i) {
        if (ev[i].kind == LaneEvent::kClose) {
          S->lanes.erase(ev[i].lane);  // idle and empty; its destructor frees it
          ++S->evicted;
          continue;
        }
        auto ln = make_lane(P, ev[i].level, ev[i].first, ev[i].nslots, ev[i].bytes);
        if (!ln) throw HipError{hipErrorOutOfMemory, "serving lane"};
        ln->id = ev[i].lane;
        S->lanes.emplace(ev[i].lane, std::move(ln));
        if ((int)S->slot.size() < ev[i].first + ev[i].nslots)
          S->slot.resize(ev[i].first + ev[i].nslots);
        ++S->opened;
      }
      S->lane_seconds += S->now() - t_ev;
    }
    std::map<int, std::vector<Ticket>> per;
    const double t = S->now();
    for (const Ticket& x : tk) {
      auto& sl = S->slot[x.slot];
      sl.busy = true;
      sl.tag = x.tag;
      sl.seed = x.seed;
      sl.t_arrival = x.t_arrival;
      sl.t_admit = t;
      ++S->resident;
      per[x.lane].push_back(x);
    }
    for (auto& kv : per) {
      Lane* ln = S->lanes.at(kv.first).get();
      ln->resident += (int)kv.second.size();
      serve_admit(P, ln, kv.second);
    }
    for (auto& kv : S->lanes) {
      Lane* ln = kv.second.get();
      if (ln->inflight || ln->resident == 0) continue;
      lane_launch(P, ln, c);
      S->sched->set_inflight(ln->id, true);
    }
    if (harvested || S->resident == 0) return;
    // nothing finished yet: wait for the first lane to finish
    bool any = false;
    for (auto& kv : S->lanes) any = any || kv.second->inflight;
    if (!any) return;
    std::this_thread::yield();
  }
}

}  // namespace mg

// ---- allocation-free solve: a static device workspace ----------------------------
//
// mg_solve_noalloc runs the solve of mg_solve with its whole workspace (the
// multigrid hierarchy, the solve state and the descriptor lists) carved from
// one file-scope device array instead of device allocations.  Each GPU the
// library runs on holds its own copy of the array until the process ends.
// In host code the array's name is only a stand-in: its device address on
// the current GPU comes from hipGetSymbolAddress, taken once per device (at
// plan creation, with that device current) and kept in scratch_ptr.
namespace mg {
constexpr size_t kScratchBytes = (size_t)96 << 20;  // the 129^3 hierarchy (FP64 or mixed) + lists
constexpr int kScratchMaxN = 129;
constexpr int kScratchDevices = 64;
}  // namespace mg

static __device__ __align__(256) char scratch[mg::kScratchBytes];

namespace mg {
static std::mutex scratch_mu;                  // guards scratch_ptr
static void* scratch_ptr[kScratchDevices];     // device address of `scratch` per device
static std::mutex scratch_use[kScratchDevices];  // one allocation-free solve per device at a time

// The device address of the static workspace on the current device (resolved
// once per device); nullptr if HIP cannot resolve it.
static void* scratch_for_current_device(int* dev_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return nullptr;
  *dev_out = dev;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    scratch_ptr[dev] = p;
  }
  return scratch_ptr[dev];
}

// The solve of mg_solve on a batch of one solve whose top u is the caller's.
static int solve_one(mg_plan_s* P, Batch* B, int n, const double* k, const double* f, double* u,
                     double t, int fixed_cycles, int* cycles, double* relres) {
  B->lev[0][0].u[0] = u;  // the caller's u is the top iterate
  B->drop_graphs();
  upload_lists(P, B);
  const LevelT<double>& T = B->lev[0][0];
  launch_prepare_problem(n, k, f, T.wh, T.b, u, P->work);
  prepare_coefficients(P, B);
  const bool ok = run_solves(P, B, t, fixed_cycles, false);
  int cyc = 0;
  double rel = 0.0;
  CK(hipMemcpy(&cyc, B->ss.cycles, sizeof(int), hipMemcpyDeviceToHost));
  CK(hipMemcpy(&rel, B->ss.relres, sizeof(double), hipMemcpyDeviceToHost));
  if (cycles) *cycles = cyc >= 0 ? cyc : P->desc.max_cycles;
  if (relres) *relres = rel;
  if (!ok) {
    P->err = "mg_solve: tolerance not reached within max_cycles";
    return MG_ENOCONV;
  }
  return MG_OK;
}

static BatchSpec solve_spec(mg_plan_s* P, int n) {
  BatchSpec spec;
  spec.top_n = {n};
  spec.share = {-1};
  spec.const_b_top = false;
  spec.ext_u_top = true;
  spec.mixed = P->desc.precision == MG_MIXED;
  spec.fe = P->op_fe != 0;
  return spec;
}
}  // namespace mg

mg_plan_s::~mg_plan_s() {
  batch.reset();
  fmg.clear();
  spde.clear();
  if (h_small) (void)hipHostFree(h_small);
  for (auto& kv : d_phi) (void)hipFree(kv.second);
  if (d_coef) (void)hipFree(d_coef);
  for (auto e : ev_pool) (void)hipEventDestroy(e);
  if (order_ev) (void)hipEventDestroy(order_ev);
  if (work) (void)hipStreamDestroy(work);
}

// ============================== C ABI ==========================================

#define API_BEGIN try {
#define API_END(P)                                                         \
  }                                                                        \
  catch (const mg::HipError& he) {                                         \
    if (P) P->err = std::string(he.what) + ": " + hipGetErrorString(he.e); \
    return MG_EHIP;                                                        \
  }                                                                        \
  catch (const std::bad_alloc&) {                                          \
    if (P) P->err = "host allocation failed";                              \
    return MG_ENOMEM;                                                      \
  }                                                                        \
  catch (...) {                                                            \
    if (P) P->err = "unexpected error";                                    \
    return MG_EHIP;                                                        \
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
  if ((long long)(desc->n0 - 1) * (1ll << desc->max_level) + 1 > 1025) return MG_EINVAL;
  mg_plan_s* P = new (std::nothrow) mg_plan_s();
  if (!P) return MG_ENOMEM;
  P->desc = *desc;
  P->caller = (hipStream_t)desc->stream;
  try {
    if (!kl_1d_modes(desc->corr_len, 4, P->omega, P->theta, P->scale)) {
      delete P;
      return MG_EINVAL;
    }
    CK(hipStreamCreateWithFlags(&P->work, hipStreamNonBlocking));
    CK(hipEventCreateWithFlags(&P->order_ev, hipEventDisableTiming));
    P->scratch = scratch_for_current_device(&P->scratch_dev);
    if (!P->scratch) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
    CK(hipHostMalloc((void**)&P->h_small, 256, hipHostMallocDefault));
    double coef[64];
    const double sigma = std::sqrt(desc->sigma2);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c)
          coef[16 * a + 4 * b + c] = sigma * std::sqrt(P->theta[a] * P->theta[b] * P->theta[c]);
    CK(hipMalloc(&P->d_coef, sizeof(coef)));
    CK(hipMemcpy(P->d_coef, coef, sizeof(coef), hipMemcpyHostToDevice));
    for (int l = 0; l <= desc->max_level; ++l) phi_table(P, (desc->n0 - 1) * (1 << l) + 1);
  } catch (const HipError&) {
    delete P;
    return MG_EHIP;
  }
  *out = P;
  return MG_OK;
}

int mg_plan_destroy(mg_plan P) {
  if (!P) return MG_EINVAL;
  (void)hipStreamSynchronize(P->work);
  delete P;
  return MG_OK;
}

int mg_plan_get_desc(mg_plan P, mg_plan_desc* out) {
  if (!P || !out) return MG_EINVAL;
  *out = P->desc;
  return MG_OK;
}

int mg_plan_set_stream(mg_plan P, void* stream) {
  if (!P) return MG_EINVAL;
  P->caller = (hipStream_t)stream;
  return MG_OK;
}

int mg_plan_set_option(mg_plan P, const char* name, long long value) {
  if (!P || !name) return MG_EINVAL;
  const std::string k = name;
  if (k == "smoother") {
    if (value != 0 && value != 1) return MG_EINVAL;
    P->smoother = (int)value;
  } else if (k == "graph") {
    P->use_graph = value != 0;
  } else if (k == "transfer") {
    if (value != 0 && value != 1) return MG_EINVAL;
    P->transfer = (int)value;
  } else if (k == "norm") {
    if (value != 0 && value != 1) return MG_EINVAL;
    P->norm_sweep = (int)value;
  } else if (k == "qoi") {
    if (value < QOI_INTEGRAL || value > QOI_FLUX) return MG_EINVAL;
    if (value != QOI_INTEGRAL && ((P->desc.n0 - 1) % 4 != 0)) {
      P->err = "point and flux QoIs need n0 = 4m + 1 (the point and plane are vertices)";
      return MG_EINVAL;
    }
    if (value == QOI_FLUX && P->op_fe) {
      P->err = "the flux QoI uses the FD face coefficients";
      return MG_ENOTIMPL;
    }
    P->qoi_kind = (int)value;
  } else if (k == "solver") {
    if (value != 0 && value != 1) return MG_EINVAL;
    if (value == 1 && (P->desc.precision != MG_FP64 || P->op_fe || P->field_spde)) {
      P->err = "full multigrid runs in FP64 with the FD operator and the KL field";
      return MG_ENOTIMPL;
    }
    P->solver = (int)value;
  } else if (k == "operator") {
    if (value != 0 && value != 1) return MG_EINVAL;
    if (value == 1 && (P->desc.precision != MG_FP64 || P->solver != 0 || P->qoi_kind == QOI_FLUX)) {
      P->err = "the P1 operator runs in FP64 with V-cycles to tol and the integral or point QoI";
      return MG_ENOTIMPL;
    }
    P->op_fe = (int)value;
    P->batch.reset();  // the workspace layout differs
    P->batch_key.clear();
  } else if (k == "field") {
    if (value != 0 && value != 1) return MG_EINVAL;
    if (value == 1 && P->solver != 0) {
      P->err = "full multigrid samples use the KL field";
      return MG_ENOTIMPL;
    }
    P->field_spde = (int)value;
    P->batch.reset();  // coarse solves own their coefficient with the SPDE field
    P->batch_key.clear();
  } else if (k == "kl") {
    if (value != 0 && value != 1) return MG_EINVAL;
    P->kl_inline = (int)value;
  } else if (k == "inner_cycles") {
    if (value < 1 || value > 8) return MG_EINVAL;
    P->inner_cycles = (int)value;
  } else if (k == "fmg_cycles") {
    if (value < 1 || value > 64) return MG_EINVAL;
    P->fmg_cycles = (int)value;
  } else if (k == "small_vcycle") {
    if (value != 0 && value != 5 && value != 9 && value != 17) return MG_EINVAL;
    P->small_ns = (int)value;
    P->batch.reset();  // its lists are rebuilt for the new split
    P->batch_key.clear();
  } else {
    P->err = "unknown option " + k;
    return MG_EINVAL;
  }
  if (P->batch) P->batch->drop_graphs();
  for (auto& kv : P->fmg) kv.second->drop_graphs();
  return MG_OK;
}

int mg_set_tile_for(mg_plan P, int n, int fused_correction, int tj, int tk, int chunks) {
  if (!P) return MG_EINVAL;
  SweepShape shapes[32];
  const int c = sweep_shapes(n, shapes, 32);
  for (int i = 0; i < c; ++i)
    if (shapes[i].tj == tj && shapes[i].tk == tk && chunks >= 0 && chunks <= n - 2) {
      (fused_correction ? P->shape_pro : P->shape)[n] = SweepShape{tj, tk, chunks};
      if (P->batch) P->batch->drop_graphs();
      return MG_OK;
    }
  P->err = "mg_set_tile: no compiled tile shape for this grid size";
  return MG_EINVAL;
}

int mg_set_tile(mg_plan P, int n, int tj, int tk, int chunks) {
  const int st = mg_set_tile_for(P, n, 0, tj, tk, chunks);
  return st == MG_OK ? mg_set_tile_for(P, n, 1, tj, tk, chunks) : st;
}

int mg_get_tile_for(mg_plan P, int n, int fused_correction, int* tj, int* tk, int* chunks) {
  if (!P || !tj || !tk || !chunks) return MG_EINVAL;
  const SweepShape s = shape_for(P, n, fused_correction != 0);
  *tj = s.tj;
  *tk = s.tk;
  *chunks = s.chunks;
  return MG_OK;
}

int mg_get_tile(mg_plan P, int n, int* tj, int* tk, int* chunks) {
  return mg_get_tile_for(P, n, 0, tj, tk, chunks);
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
  int status = MG_OK;
  order_after_caller(P);
  Batch* B = get_batch(P, solve_spec(P, n), &status);
  if (!B) return status;
  const int st = solve_one(P, B, n, k, f, u, t, fixed_cycles, cycles, relres);
  if (P->prof) collect_profile(P);
  return st;
  API_END(P)
}

int mg_solve_noalloc(mg_plan P, int n, const double* k, const double* f, double* u, double tol,
                     int fixed_cycles, int* cycles, double* relres) {
  if (!P) return MG_EINVAL;
  if (!valid_n(n) || !k || !f || !u || fixed_cycles < 0) {
    P->err = "mg_solve_noalloc: n must be 2^m+1 (m>=1) and k, f, u non-null";
    return MG_EINVAL;
  }
  if (n > kScratchMaxN) {
    P->err = "mg_solve_noalloc: n above 129 exceeds the static workspace (96 MiB)";
    return MG_EINVAL;
  }
  API_BEGIN
  if (!P->scratch || !P->h_small) {
    P->err = "mg_solve_noalloc: no static workspace on this plan's device";
    return MG_EHIP;
  }
  const BatchSpec spec = solve_spec(P, n);
  size_t need = 0;
  build_batch(P, spec, &need);  // bytes only, no allocation
  if (need > kScratchBytes - ((size_t)1 << 20)) {  // (1 MiB kept for the lists)
    P->err = "mg_solve_noalloc: the hierarchy exceeds the static workspace";
    return MG_EINVAL;
  }
  const double t = tol > 0.0 ? tol : P->desc.tol;
  // every call on this device shares the array: one at a time in this process
  std::lock_guard<std::mutex> g(scratch_use[P->scratch_dev]);
  const bool prof = P->prof;  // no timing events in this path
  P->prof = false;
  order_after_caller(P);
  std::unique_ptr<Batch> B = build_batch(P, spec, nullptr, (char*)P->scratch, kScratchBytes);
  int st = MG_EINVAL;
  if (B) {
    B->st = P->work;
    try {
      st = solve_one(P, B.get(), n, k, f, u, t, fixed_cycles, cycles, relres);
    } catch (...) {
      P->prof = prof;
      throw;
    }
  } else {
    P->err = "mg_solve_noalloc: the hierarchy exceeds the static workspace";
  }
  P->prof = prof;
  return st;
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
  const std::vector<int> levels(n_samples, level);
  if (P->solver == 1) return run_samples_fmg(P, levels, seeds, Y_out, Qf_out, Qc_out, cycles_out);
  return run_samples(P, levels, seeds, Y_out, Qf_out, Qc_out, cycles_out, fixed_cycles);
  API_END(P)
}

int mlmc_sample_mixed(mg_plan P, const int* levels, const uint64_t* seeds, int n_samples,
                      double* Y_out, double* Qf_out, double* Qc_out, int* cycles_out,
                      int fixed_cycles) {
  if (!P) return MG_EINVAL;
  if (!levels || !seeds || n_samples < 1 || !Y_out || fixed_cycles < 0) {
    P->err = "mlmc_sample_mixed: levels/seeds/Y_out non-null, n >= 1";
    return MG_EINVAL;
  }
  for (int i = 0; i < n_samples; ++i)
    if (levels[i] < 0 || levels[i] > P->desc.max_level) {
      P->err = "mlmc_sample_mixed: every level must be in [0, max_level]";
      return MG_EINVAL;
    }
  API_BEGIN
  const std::vector<int> lv(levels, levels + n_samples);
  if (P->solver == 1) return run_samples_fmg(P, lv, seeds, Y_out, Qf_out, Qc_out, cycles_out);
  return run_samples(P, lv, seeds, Y_out, Qf_out, Qc_out, cycles_out, fixed_cycles);
  API_END(P)
}

int mg_autotune(mg_plan P, int level, int n_samples, int reps) {
  if (!P) return MG_EINVAL;
  if (level < 0 || level > P->desc.max_level || n_samples < 1) return MG_EINVAL;
  API_BEGIN
  std::vector<uint64_t> seeds(n_samples);
  for (int i = 0; i < n_samples; ++i) seeds[i] = 0x5eed0000ull + i;
  double* d_y = nullptr;
  CK(hipMalloc(&d_y, sizeof(double) * n_samples));
  const int st = mlmc_sample_batch(P, level, seeds.data(), n_samples, d_y, nullptr, nullptr,
                                   nullptr, 0);
  CK(hipFree(d_y));
  if (st != MG_OK && st != MG_ENOCONV) return st;
  Batch* B = P->batch.get();
  const bool mixed = B->spec.mixed;
  // the shapes in force before tuning: a pick must beat them on whole batches
  const std::map<int, SweepShape> before = P->shape, before_pro = P->shape_pro;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  reps = std::max(1, reps);
  for (size_t si = 0; si < B->sizes.size(); ++si) {
    const int n = B->sizes[si];
    if (n < 5 || n <= P->small_ns) continue;  // small grids run in the LDS V-cycle
    if (!sweep_fits(n, mixed ? sizeof(float) : sizeof(double))) continue;  // colour sweeps
    SweepShape shapes[32];
    const int c = sweep_shapes(n, shapes, 32);
    // the plain sweep and the one with the fused coarse correction are tuned
    // separately (their register use, hence occupancy, differs)
    for (int pro = 0; pro < 2; ++pro) {
      double best = 1e30;
      SweepShape pick = default_sweep_shape(n, pro != 0, mixed);
      for (int i = 0; i < c; ++i)
        for (int chunks : {0, 1, 2, 4}) {
          if (chunks > 1 && (n - 2) / chunks < 4) continue;
          if (n >= 33 && shapes[i].tj * shapes[i].tk < 64) continue;  // tiny tiles on big grids
          SweepShape s = shapes[i];
          s.chunks = chunks;
          // every solve active while timing; the next batch reinitialises the workspace
          launch_init_state2(B->ss, B->ns, P->work);
          const int cb = pro ? 0 : -1;
          auto one = [&]() {
            if (mixed)
              launch_sweep<float>(B->L32.d[si], (int)B->L32.h[si].size(), n, B->ss.active, 0, cb,
                                  s, P->work, nullptr, 0, B->L32.const_b(si));
            else
              launch_sweep<double>(B->L64.d[si], (int)B->L64.h[si].size(), n, B->ss.active, 0,
                                   cb, s, P->work, nullptr, 0, B->L64.const_b(si),
                                   P->kl_inline && B->L64.kl(si));
          };
          one();
          CK(hipEventRecord(e0, P->work));
          for (int r = 0; r < reps; ++r) one();
          CK(hipEventRecord(e1, P->work));
          CK(hipEventSynchronize(e1));
          float ms = 0.f;
          CK(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best) {
            best = ms;
            pick = s;
          }
        }
      // a fixed split that launches what the automatic one launches with
      // every grid active is kept as the automatic split: the same launch
      // then, and the marches still spread out once most solves have stopped
      const int cnt = mixed ? (int)B->L32.h[si].size() : (int)B->L64.h[si].size();
      if (pick.chunks > 0 &&
          sweep_blocks(n, cnt, pick) == sweep_blocks(n, cnt, SweepShape{pick.tj, pick.tk, 0}))
        pick.chunks = 0;
      (pro ? P->shape_pro : P->shape)[n] = pick;
    }
  }
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  B->drop_graphs();
  // whole batches (graphs, every sweep kind, the real stopping) with the
  // picks and with the shapes before tuning, alternately, best of two each
  const std::map<int, SweepShape> picked = P->shape, picked_pro = P->shape_pro;
  CK(hipMalloc(&d_y, sizeof(double) * n_samples));
  auto batch_ms = [&]() {
    B->drop_graphs();
    (void)mlmc_sample_batch(P, level, seeds.data(), n_samples, d_y, nullptr, nullptr, nullptr, 0);
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps; ++r)
      (void)mlmc_sample_batch(P, level, seeds.data(), n_samples, d_y, nullptr, nullptr, nullptr,
                              0);
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  double t_pick = 1e300, t_before = 1e300;
  for (int round = 0; round < 2; ++round) {
    P->shape = picked;
    P->shape_pro = picked_pro;
    t_pick = std::min(t_pick, batch_ms());
    P->shape = before;
    P->shape_pro = before_pro;
    t_before = std::min(t_before, batch_ms());
  }
  CK(hipFree(d_y));
  // a pick must be faster by more than the 1% that whole-batch timings
  // vary by from run to run, or the shapes in force stay
  if (t_pick < 0.99 * t_before) {
    P->shape = picked;
    P->shape_pro = picked_pro;
  }
  B = P->batch.get();
  if (B) B->drop_graphs();
  return MG_OK;
  API_END(P)
}

int mlmc_philox(mg_plan P, const uint64_t* seeds, int n_samples, int level, uint32_t* words_out,
                double* normals_out) {
  if (!P) return MG_EINVAL;
  if (!seeds || n_samples < 1 || level < 0 || (!words_out && !normals_out)) return MG_EINVAL;
  API_BEGIN
  order_after_caller(P);
  uint64_t* d = nullptr;
  CK(hipMalloc(&d, sizeof(uint64_t) * n_samples));
  CK(hipMemcpyAsync(d, seeds, sizeof(uint64_t) * n_samples, hipMemcpyHostToDevice, P->work));
  launch_philox(d, n_samples, level, words_out, normals_out, P->work);
  CK(hipStreamSynchronize(P->work));
  CK(hipFree(d));
  return MG_OK;
  API_END(P)
}

int mlmc_philox_words(uint64_t seed, int level, uint32_t* out) {
  if (!out || level < 0) return MG_EINVAL;
  for (uint32_t j = 0; j < 32; ++j) {
    uint32_t c[4] = {j, (uint32_t)level, 0u, 0u};
    philox_block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int q = 0; q < 4; ++q) out[4 * j + q] = c[q];
  }
  return MG_OK;
}

double mlmc_exp(double x) { return mg::kl_exp_host(x); }

int mlmc_field(mg_plan P, int n, uint64_t seed, int level, double* k_out) {
  if (!P) return MG_EINVAL;
  if (!valid_n(n) || n > 1025 || level < 0 || !k_out) return MG_EINVAL;
  API_BEGIN
  order_after_caller(P);
  if (P->field_spde) {
    if (level > P->desc.max_level) {
      P->err = "mlmc_field: the SPDE field needs level <= max_level";
      return MG_EINVAL;
    }
    int st;
    if (n == level_n(P, level))
      st = spde_fields(P, level, &seed, 1, {k_out}, {}, 1);
    else if (level > 0 && n == level_n(P, level - 1))
      st = spde_fields(P, level, &seed, 1, {}, {k_out}, 1);
    else {
      P->err = "mlmc_field: with the SPDE field n must be n_level or n_(level-1)";
      return MG_EINVAL;
    }
    if (st != MG_OK) P->err = "mlmc_field: the SPDE solve missed its tolerance";
    return st;
  }
  uint64_t* d_seed = nullptr;
  double* d_norm = nullptr;
  double** d_out = nullptr;
  int* d_xi = nullptr;
  CK(hipMalloc(&d_seed, sizeof(uint64_t)));
  CK(hipMalloc(&d_norm, sizeof(double) * 64));
  CK(hipMalloc(&d_out, sizeof(double*)));
  CK(hipMalloc(&d_xi, sizeof(int)));
  const int zero = 0;
  CK(hipMemcpyAsync(d_seed, &seed, sizeof(uint64_t), hipMemcpyHostToDevice, P->work));
  CK(hipMemcpyAsync(d_out, &k_out, sizeof(double*), hipMemcpyHostToDevice, P->work));
  CK(hipMemcpyAsync(d_xi, &zero, sizeof(int), hipMemcpyHostToDevice, P->work));
  launch_philox(d_seed, 1, level, nullptr, d_norm, P->work);
  launch_field(n, 1, d_out, d_xi, d_norm, phi_table(P, n), P->d_coef, 1, P->work);
  CK(hipStreamSynchronize(P->work));
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
  P->prof_recs.clear();
  P->ev_meta.clear();
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

int mg_profile_records(mg_plan P, int max_out, int* cycle, int* kind, int* grid_n, double* ms,
                       int* n_out) {
  if (!P || !n_out || max_out < 0 || (max_out > 0 && (!cycle || !kind || !grid_n || !ms)))
    return MG_EINVAL;
  API_BEGIN
  collect_profile(P);
  const int n = (int)std::min<size_t>((size_t)max_out, P->prof_recs.size());
  for (int i = 0; i < n; ++i) {
    cycle[i] = P->prof_recs[i].cycle;
    kind[i] = P->prof_recs[i].kind;
    grid_n[i] = P->prof_recs[i].n;
    ms[i] = P->prof_recs[i].ms;
  }
  *n_out = (int)P->prof_recs.size();
  return MG_OK;
  API_END(P)
}

int mg_sample_footprint(mg_plan P, int level, size_t* bytes) {
  if (!P || !bytes || level < 0 || level > P->desc.max_level) return MG_EINVAL;
  API_BEGIN
  *bytes = sample_bytes(P, level);
  return MG_OK;
  API_END(P)
}

int mg_serve_create(mg_plan P, const int* lane_slots, int queue_capacity, mg_server* out) {
  if (!P || !out) return MG_EINVAL;
  *out = nullptr;
  if (queue_capacity < 1) {
    P->err = "mg_serve_create: queue_capacity must be >= 1";
    return MG_EINVAL;
  }
  if (P->solver != 0 || P->qoi_kind != QOI_INTEGRAL || P->op_fe || P->field_spde) {
    P->err = "mg_serve_create: the server runs FD V-cycles to tol with the KL field and the "
             "integral QoI";
    return MG_ENOTIMPL;
  }
  API_BEGIN
  const int L = P->desc.max_level;
  const size_t budget = P->desc.hbm_budget ? P->desc.hbm_budget : ((size_t)8 << 30);
  std::vector<int> k(L + 1);
  std::vector<size_t> bytes(L + 1, 0);
  bool any = false;
  for (int l = 0; l <= L; ++l) {
    if (lane_slots) {
      k[l] = lane_slots[l];
      if (k[l] < 0 || k[l] > Scheduler::kMaxLaneSlots) {
        P->err = "mg_serve_create: slots per lane outside [0, 4096]";
        return MG_EINVAL;
      }
    } else {
      // at most an eighth of the budget per lane, 1..256 slots
      const size_t c = budget / 8 / sample_bytes(P, l);
      k[l] = (int)std::max<size_t>(1, std::min<size_t>(256, c));
      while (k[l] > 1 && lane_bytes(P, l, k[l]) > budget / 8) --k[l];
    }
    if (k[l] == 0) continue;
    bytes[l] = lane_bytes(P, l, k[l]);
    if (bytes[l] > budget) {
      P->err = "mg_serve_create: a lane of level " + std::to_string(l) + " (" +
               std::to_string(bytes[l]) + " bytes) exceeds the HBM budget";
      return MG_ENOMEM;
    }
    any = true;
  }
  if (!any) {
    P->err = "mg_serve_create: no level has slots";
    return MG_EINVAL;
  }
  auto S = std::make_unique<mg_server_s>();
  S->P = P;
  S->lane_slots = k;
  S->sched = std::make_unique<Scheduler>(k, bytes, budget, queue_capacity);
  S->t0 = std::chrono::steady_clock::now();
  *out = S.release();
  return MG_OK;
  API_END(P)
}

int mg_serve_destroy(mg_server S) {
  if (!S) return MG_EINVAL;
  delete S;  // each lane synchronises its stream before freeing
  return MG_OK;
}

int mg_serve_submit(mg_server S, int level, uint64_t seed, long long tag, double t_arrival) {
  if (!S) return MG_EINVAL;
  const int st = S->sched->submit(level, seed, tag, t_arrival < 0 ? S->now() : t_arrival);
  if (st == MG_EINVAL) S->P->err = "mg_serve_submit: level outside [0, max_level]";
  if (st == MG_EBUSY) S->P->err = "mg_serve_submit: queue full";
  if (st == MG_ENOMEM) S->P->err = "mg_serve_submit: the level is not served (no slots)";
  return st;
}

int mg_serve_step(mg_server S, int cycles, mg_result* out, int max_out, int* n_out) {
  if (!S || !n_out || cycles < 1 || max_out < 0 || (max_out > 0 && !out)) return MG_EINVAL;
  mg_plan P = S->P;
  *n_out = 0;
  if (S->failed) {
    P->err = "mg_serve_step: an earlier step failed; destroy the server";
    return MG_EINVAL;
  }
  API_BEGIN
  if (S->resident > 0 || S->sched->queued() > 0) {
    try {
      serve_step(S, cycles);
    } catch (...) {
      S->failed = true;
      throw;
    }
  }
  int n = 0;
  while (n < max_out && !S->done.empty()) {
    out[n++] = S->done.front();
    S->done.pop_front();
  }
  *n_out = n;
  return MG_OK;
  API_END(P)
}

double mg_serve_now(mg_server S) { return S ? S->now() : 0.0; }

int mg_serve_counts(mg_server S, int* queued, int* resident, long long* completed) {
  if (!S) return MG_EINVAL;
  if (queued) *queued = S->sched->queued();
  if (resident) *resident = S->resident;
  if (completed) *completed = S->completed;
  return MG_OK;
}

int mg_serve_slots(mg_server S, int level) {
  if (!S || level < 0 || level >= S->sched->levels()) return -1;
  return S->sched->lane_slots(level);
}

int mg_serve_memory(mg_server S, size_t* used, size_t* peak, size_t* budget, int* lanes,
                    long long* opened, long long* evicted, double* lane_seconds) {
  if (!S) return MG_EINVAL;
  if (used) *used = S->sched->used();
  if (peak) *peak = S->sched->peak();
  if (budget) *budget = S->sched->budget();
  if (lanes) *lanes = (int)S->lanes.size();
  if (opened) *opened = S->opened;
  if (evicted) *evicted = S->evicted;
  if (lane_seconds) *lane_seconds = S->lane_seconds;
  return MG_OK;
}

}  // extern "C"
