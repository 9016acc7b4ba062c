// Batched stepping: several bound solvers, of any dimension, degree, size,
// precision and launch plan, advance together, one LSRK step (Sec. 5.4) per
// call, as ONE hipGraph replay. Per RK stage, the active solves whose stage
// kernel has a work-list form (stage_list_kernel, stage_k3_list_kernel) are
// grouped by kernel variant and launch shape, and each group is ONE launch
// over a work list of (solve, tile) items (work_list.h): each item is one
// workgroup running the same stage body, with the same parameters, as the
// solve's own launch, so a solve's result is bitwise the same alone and in
// the mix. The remaining solves (Gauss-Legendre, mapped cells, the
// Vlasov-Poisson field, or a variant whose work-list form the compiler gives
// fewer waves per SIMD or more scratch than its own launch) keep their own
// stage launches in the same graph. The stages follow each other on one
// stream; no launch waits on another solve's data.
//
// The kernel parameters and work lists of a captured step are built and
// checked on the host, uploaded before the capture, and never written again:
// they belong to the cached graph and are freed only after its last replay.
// Graphs are cached for the two alternating solution-buffer parities; a
// change of the active set, a time step, a parity pattern or a solver's
// plan, field or memory leads to a new capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "hd_internal.h"
#include "work_list.h"

namespace {

constexpr int kMaxBatch = 1024;
constexpr size_t kDevAlign = 256;

using hd::rt::fail;

size_t align_dev(size_t x) { return (x + kDevAlign - 1) / kDevAlign * kDevAlign; }

// What a captured step depends on.
struct StepKey {
  std::vector<int> active, par;
  std::vector<double> dt;
  std::vector<uint64_t> version;
  bool operator==(const StepKey &o) const {
    return active == o.active && par == o.par && dt == o.dt && version == o.version;
  }
};

struct Cached {
  StepKey key;
  hipGraphExec_t exec = nullptr;
  uint64_t used = 0;
  // Device memory the graph's work-list launches read (parameters, lists).
  void *dev = nullptr;
  // Recorded after each replay: the exec and its memory are released only
  // after it.
  hipEvent_t done = nullptr;
  bool pending = false;
  int list_launches = 0, solve_launches = 0;
};

// Destroy a cached step graph and free its memory once its last replay has
// finished.
void release(Cached &c) {
  if (c.pending && c.done) (void)hipEventSynchronize(c.done);
  c.pending = false;
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  c.exec = nullptr;
  if (c.dev) (void)hipFree(c.dev);
  c.dev = nullptr;
}

// Whether the work-list form of a variant keeps its own launch's resources:
// at least as many workgroups per CU at this launch shape and no more
// scratch per lane. Cached per (entry pair, shape).
bool list_form_keeps_resources(const void *single, const void *list, unsigned block, size_t shmem) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, const void *, unsigned, size_t>, bool> memo;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(single, list, block, shmem);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  bool ok = false;
  hipFuncAttributes a{}, b{};
  int occ_a = 0, occ_b = 0;
  if (shmem > 65536) {
    if (hd::rt::allow_large_lds(single) != hipSuccess || hd::rt::allow_large_lds(list) != hipSuccess) {
      memo[key] = false;
      return false;
    }
  }
  if (hipFuncGetAttributes(&a, single) == hipSuccess && hipFuncGetAttributes(&b, list) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_a, single, (int)block, shmem) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_b, list, (int)block, shmem) == hipSuccess)
    ok = occ_b >= occ_a && occ_b > 0 && b.localSizeBytes <= a.localSizeBytes;
  memo[key] = ok;
  return ok;
}

// One work-list launch of a captured step.
struct GroupLaunch {
  int stage = 0;
  int prec = 0;
  const void *fn = nullptr;
  unsigned block = 0;
  size_t shmem = 0;
  std::vector<unsigned char> prm;  // the slots' StageParams, packed
  std::vector<uint32_t> tiles, item0;
  size_t off_prm = 0, off_item0 = 0;  // in the graph's device memory
};

struct StageStep {
  std::vector<int> own;  // solves launched on their own at this stage
  std::vector<GroupLaunch> groups;
};

}  // namespace

struct hd_batch {
  std::vector<hd_solver *> solvers;
  hipStream_t cap = nullptr;
  Cached cache[2];
  uint64_t clock = 0;
};

namespace {

template <typename P>
hd_status plan_solve_stage(hd_solver *s, int par, int stage, double dt, int prec,
                           std::map<std::tuple<const void *, unsigned, size_t, int>, size_t> *index,
                           StageStep *ss, int solve) {
  hd::StageParams<P> prm;
  hd::LaunchShape ls{};
  int role = 0;
  hd::rt::fill_stage<P>(s, s->u(par), nullptr, s->u(1 - par), 1, stage, dt, &prm, &ls, &role);
  const void *single = hd::rt::stage_entry(s, role, 0);
  const void *list = hd::rt::stage_entry(s, role, 1);
  if (!single) return fail(HD_ERR_HIP, "no compiled stage kernel for a batched solver's plan");
  if (ls.grid == 0) return HD_OK;
  if (!list || !list_form_keeps_resources(single, list, ls.block, ls.shmem)) {
    ss->own.push_back(solve);
    return HD_OK;
  }
  const auto key = std::make_tuple(list, ls.block, ls.shmem, prec);
  auto it = index->find(key);
  // A launch holds fewer than 2^32 work-items: a group that would outgrow
  // that continues in a new launch.
  const auto items_of = [](const GroupLaunch &g) {
    uint64_t at = 0;
    for (uint32_t t : g.tiles) at += ((uint64_t)t + hd::kListAlign - 1) / hd::kListAlign * hd::kListAlign;
    return at;
  };
  const uint64_t mine = ((uint64_t)ls.grid + hd::kListAlign - 1) / hd::kListAlign * hd::kListAlign;
  if (it != index->end() &&
      (items_of(ss->groups[it->second]) + mine) * ls.block >= (uint64_t(1) << 32)) {
    index->erase(it);
    it = index->end();
  }
  if ((uint64_t)mine * ls.block >= (uint64_t(1) << 32)) {
    ss->own.push_back(solve);  // its own launch reports the limit
    return HD_OK;
  }
  if (it == index->end()) {
    it = index->emplace(key, ss->groups.size()).first;
    GroupLaunch g;
    g.stage = stage;
    g.prec = prec;
    g.fn = list;
    g.block = ls.block;
    g.shmem = ls.shmem;
    ss->groups.push_back(std::move(g));
  }
  GroupLaunch &g = ss->groups[it->second];
  const unsigned char *b = reinterpret_cast<const unsigned char *>(&prm);
  g.prm.insert(g.prm.end(), b, b + sizeof(prm));
  g.tiles.push_back(ls.grid);
  return HD_OK;
}

template <typename P>
hd_status launch_group(const GroupLaunch &g, char *dev, hipStream_t st) {
  hd::ListParams<P> lp;
  lp.prm = (hd::ConstStageParams<P> *)(uintptr_t)(dev + g.off_prm);
  lp.item0 = reinterpret_cast<const uint32_t *>(dev + g.off_item0);
  lp.nslots = (int)g.tiles.size();
  lp.nitems = g.item0.back();
  void *args[] = {&lp};
  hipError_t e = hipLaunchKernel(g.fn, dim3(lp.nitems), dim3(g.block), args, g.shmem, st);
  if (e != hipSuccess) return fail(HD_ERR_HIP, std::string("work-list launch: ") + hipGetErrorString(e));
  return HD_OK;
}

hd_status capture(hd_batch *b, const StepKey &key, Cached *c) {
  const int n = (int)b->solvers.size();
  // Host plan of the five stages (no device call but attribute queries).
  std::vector<StageStep> steps(5);
  for (int stage = 0; stage < 5; ++stage) {
    std::map<std::tuple<const void *, unsigned, size_t, int>, size_t> index;
    for (int i = 0; i < n; ++i) {
      if (!key.active[i]) continue;
      hd_solver *s = b->solvers[i];
      const int par = key.par[i] ^ (stage & 1);
      if (!hd::rt::list_capable(s)) {
        steps[stage].own.push_back(i);
        continue;
      }
      const hd_status r = s->prec == HD_FP32_OP_FP64_ACC
                              ? plan_solve_stage<float>(s, par, stage, key.dt[i], s->prec, &index,
                                                        &steps[stage], i)
                              : plan_solve_stage<double>(s, par, stage, key.dt[i], s->prec, &index,
                                                         &steps[stage], i);
      if (r != HD_OK) return r;
    }
  }
  // Work lists, checked, and one device allocation for all of them.
  size_t bytes = 0;
  int nlist = 0, nown = 0;
  for (StageStep &ss : steps) {
    nown += (int)ss.own.size();
    for (GroupLaunch &g : ss.groups) {
      std::string why;
      if (!hd::build_work_list(g.tiles, &g.item0, &why) || !hd::check_work_list(g.tiles, g.item0, &why))
        return fail(HD_ERR_UNSUPPORTED, "batch work list: " + why);
      g.off_prm = bytes;
      bytes = align_dev(bytes + g.prm.size());
      g.off_item0 = bytes;
      bytes = align_dev(bytes + g.item0.size() * sizeof(uint32_t));
      ++nlist;
      if (g.shmem > 65536) {
        const hipError_t e = hd::rt::allow_large_lds(g.fn);
        if (e != hipSuccess)
          return fail(HD_ERR_HIP, std::string("raising the LDS limit: ") + hipGetErrorString(e));
      }
    }
  }
  if (bytes) {
    std::vector<unsigned char> host(bytes, 0);
    for (StageStep &ss : steps)
      for (GroupLaunch &g : ss.groups) {
        std::copy(g.prm.begin(), g.prm.end(), host.begin() + g.off_prm);
        std::memcpy(host.data() + g.off_item0, g.item0.data(), g.item0.size() * sizeof(uint32_t));
      }
    HD_HIP(hipMalloc(&c->dev, bytes));
    HD_HIP(hipMemcpy(c->dev, host.data(), bytes, hipMemcpyHostToDevice));
  }
  // The step: stage after stage on one stream.
  hipGraph_t graph = nullptr;
  HD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hd_status r = HD_OK;
  for (int stage = 0; stage < 5 && r == HD_OK; ++stage) {
    for (int i : steps[stage].own) {
      r = hd::rt::enqueue_stage_of(b->solvers[i], key.par[i] ^ (stage & 1), stage, key.dt[i], b->cap);
      if (r != HD_OK) break;
    }
    for (const GroupLaunch &g : steps[stage].groups) {
      if (r != HD_OK) break;
      r = g.prec == HD_FP32_OP_FP64_ACC ? launch_group<float>(g, static_cast<char *>(c->dev), b->cap)
                                        : launch_group<double>(g, static_cast<char *>(c->dev), b->cap);
    }
  }
  hipError_t ce = hipStreamEndCapture(b->cap, &graph);
  if (r != HD_OK || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (r != HD_OK) return r;
    return fail(HD_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(ce));
  }
  hipError_t ie = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    c->exec = nullptr;
    return fail(HD_ERR_HIP, std::string("batch graph instantiate: ") + hipGetErrorString(ie));
  }
  c->list_launches = nlist;
  c->solve_launches = nown;
  return HD_OK;
}

void destroy_batch(hd_batch *b) {
  if (!b) return;
  for (Cached &c : b->cache) {
    release(c);
    if (c.done) (void)hipEventDestroy(c.done);
  }
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

hd_status init_batch(hd_batch *b) {
  HD_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  for (Cached &c : b->cache) HD_HIP(hipEventCreateWithFlags(&c.done, hipEventDisableTiming));
  return HD_OK;
}

}  // namespace

extern "C" {

hd_status hd_batch_create(hd_solver *const *solvers, int n, hd_batch **out) {
  if (!out || (!solvers && n)) return fail(HD_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (n < 1 || n > kMaxBatch) return fail(HD_ERR_INVALID, "batch size must be 1..1024");
  for (int i = 0; i < n; ++i) {
    hd_solver *s = solvers[i];
    if (!s || !s->bound()) return fail(HD_ERR_INVALID, "every batched solver must be bound (hd_bind)");
    for (int j = 0; j < i; ++j)
      if (solvers[j] == s) return fail(HD_ERR_INVALID, "a solver appears twice in the batch");
  }
  hd_batch *b = new (std::nothrow) hd_batch();
  if (!b) return fail(HD_ERR_OOM, "host allocation failed");
  b->solvers.assign(solvers, solvers + n);
  hd_status r = init_batch(b);
  if (r != HD_OK) {
    destroy_batch(b);
    return r;
  }
  *out = b;
  return HD_OK;
}

hd_status hd_batch_destroy(hd_batch *b) {
  destroy_batch(b);
  return HD_OK;
}

hd_status hd_batch_step(hd_batch *b, const double *dt, const int *active, hd_stream stream) {
  if (!b || !dt) return fail(HD_ERR_INVALID, "NULL argument");
  const int n = (int)b->solvers.size();
  StepKey key;
  key.active.resize(n);
  key.par.assign(n, 0);
  key.dt.assign(n, 0.0);
  key.version.assign(n, 0);
  bool any = false;
  for (int i = 0; i < n; ++i) {
    key.active[i] = active ? (active[i] != 0) : 1;
    if (!key.active[i]) continue;
    any = true;
    if (!(dt[i] == dt[i] && dt[i] > -1e300 && dt[i] < 1e300))
      return fail(HD_ERR_INVALID, "dt must be finite");
    if (!b->solvers[i]->bound()) return fail(HD_ERR_INVALID, "a batched solver lost its memory");
    key.par[i] = b->solvers[i]->cur;
    key.dt[i] = dt[i];
    key.version[i] = b->solvers[i]->version;
  }
  if (!any) return HD_OK;
  Cached *hit = nullptr;
  for (Cached &c : b->cache)
    if (c.exec && c.key == key) hit = &c;
  if (!hit) {
    // Replace the least recently used of the two cached steps.
    hit = b->cache[0].used <= b->cache[1].used ? &b->cache[0] : &b->cache[1];
    release(*hit);
    hd_status r = capture(b, key, hit);
    if (r != HD_OK) {
      release(*hit);
      return r;
    }
    hit->key = key;
  }
  hit->used = ++b->clock;
  HD_HIP(hipGraphLaunch(hit->exec, (hipStream_t)stream));
  HD_HIP(hipEventRecord(hit->done, (hipStream_t)stream));
  hit->pending = true;
  for (int i = 0; i < n; ++i)
    if (key.active[i]) b->solvers[i]->cur ^= 1;  // five stages: the other buffer
  return HD_OK;
}

hd_status hd_batch_launch_counts(const hd_batch *b, int *list_launches, int *solve_launches) {
  if (!b || !list_launches || !solve_launches) return fail(HD_ERR_INVALID, "NULL argument");
  const Cached *last = nullptr;
  for (const Cached &c : b->cache)
    if (c.exec && (!last || c.used > last->used)) last = &c;
  *list_launches = last ? last->list_launches : 0;
  *solve_launches = last ? last->solve_launches : 0;
  return HD_OK;
}

}  // extern "C"
