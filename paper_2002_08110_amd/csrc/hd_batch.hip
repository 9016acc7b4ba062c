// Batched stepping: several bound solvers, of any dimension, degree, size,
// precision and launch plan, advance together, one LSRK step per call. The
// step of all active solves is ONE hipGraph replay: each solve's five fused
// stage launches (the same kernels, with the same parameters, as the solve
// stepped alone, so results agree bitwise) form a chain, and the chains are
// spread over up to eight independent branches balanced by bytes moved, so
// small solves overlap with each other and with the tails of large ones.
// Graphs are captured on demand and cached for the two alternating
// solution-buffer parities; a change of the active set, a time step, a
// parity pattern or a solver's plan, field or memory leads to a new capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "hd_internal.h"

namespace {

constexpr int kMaxBatch = 1024;
constexpr int kMaxBranches = 8;

using hd::rt::fail;

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
  // Recorded after each replay: the exec is destroyed only after it.
  hipEvent_t done = nullptr;
  bool pending = false;
};

// Destroy a cached step graph once its last replay has finished.
void release(Cached &c) {
  if (c.pending && c.done) hipEventSynchronize(c.done);
  c.pending = false;
  if (c.exec) hipGraphExecDestroy(c.exec);
  c.exec = nullptr;
}

}  // namespace

struct hd_batch {
  std::vector<hd_solver *> solvers;
  hipStream_t cap = nullptr;
  hipStream_t side[kMaxBranches] = {};
  hipEvent_t ev[kMaxBranches + 1] = {};
  Cached cache[2];
  uint64_t clock = 0;
};

namespace {

// Bytes a solve moves per stage (FP64 u in and out, du in and out).
double stage_bytes(const hd_solver *s) {
  return (double)s->ndofs * (16.0 + 2.0 * (double)s->psize());
}

hd_status capture(hd_batch *b, const StepKey &key, hipGraphExec_t *out) {
  const int n = (int)b->solvers.size();
  std::vector<int> act;
  for (int i = 0; i < n; ++i)
    if (key.active[i]) act.push_back(i);
  const int nb = std::min<int>((int)act.size(), kMaxBranches);
  // Largest first onto the least loaded branch.
  std::sort(act.begin(), act.end(), [&](int x, int y) {
    return stage_bytes(b->solvers[x]) > stage_bytes(b->solvers[y]);
  });
  std::vector<double> load(nb, 0.0);
  std::vector<std::vector<int>> branch(nb);
  for (int i : act) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    branch[k].push_back(i);
    load[k] += stage_bytes(b->solvers[i]);
  }
  hipGraph_t graph = nullptr;
  HD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hd_status r = HD_OK;
  hipError_t e = hipEventRecord(b->ev[kMaxBranches], b->cap);
  for (int k = 0; k < nb && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->ev[kMaxBranches], 0);
  for (int k = 0; k < nb && e == hipSuccess && r == HD_OK; ++k)
    for (int i : branch[k]) {
      r = hd::rt::enqueue_step(b->solvers[i], key.par[i], key.dt[i], b->side[k]);
      if (r != HD_OK) break;
    }
  for (int k = 0; k < nb && e == hipSuccess; ++k) {
    e = hipEventRecord(b->ev[k], b->side[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->ev[k], 0);
  }
  hipError_t ce = hipStreamEndCapture(b->cap, &graph);
  if (r != HD_OK || e != hipSuccess || ce != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    if (r != HD_OK) return r;
    return fail(HD_ERR_HIP, std::string("batch graph capture: ") +
                                hipGetErrorString(e != hipSuccess ? e : ce));
  }
  hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    *out = nullptr;
    return fail(HD_ERR_HIP, std::string("batch graph instantiate: ") + hipGetErrorString(ie));
  }
  return HD_OK;
}

void destroy_batch(hd_batch *b) {
  if (!b) return;
  for (Cached &c : b->cache) {
    release(c);
    if (c.done) hipEventDestroy(c.done);
  }
  for (hipEvent_t e : b->ev)
    if (e) hipEventDestroy(e);
  for (hipStream_t s : b->side)
    if (s) hipStreamDestroy(s);
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
}

hd_status init_batch(hd_batch *b) {
  HD_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  for (hipStream_t &s : b->side) HD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  for (hipEvent_t &e : b->ev) HD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
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
    hd_status r = capture(b, key, &hit->exec);
    if (r != HD_OK) return r;
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

}  // extern "C"
