// Batched stepping: several bound solvers, of any dimension, degree and
// size (one precision per batch), advance together. Each RK stage of all
// active solves is ONE persistent launch: its workgroups walk a device-side
// work list of (solve, cell tile) items and run the stage body of that
// solve's (d, k) variant. A whole RK step - five stage launches and a tiny
// kernel that flips each solve's solution-buffer parity - is one hipGraph,
// captured once; the time steps, the active set and the work list live in
// device memory and are refreshed by plain copies, so the graph never needs
// to be captured again. Stage boundaries are kernel boundaries: no
// workgroup waits on another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hd_internal.h"
#include "stage_k3.h"
#include "stage_kernel.h"

namespace hd {
namespace {

constexpr int kMaxBatch = 1024;
constexpr int kBatchThreads = 256;
constexpr size_t kBatchCellLds = 40 * 1024;  // LDS budget of a generic variant's tile

constexpr int split_dx(int d) { return d == 2 ? 1 : (d == 3 ? 2 : (d == 4 ? 2 : 3)); }

// The launch variant of (D, N, P) inside the batched kernel; one source of
// truth for the device dispatch and the host work-list sizes.
template <int D, int N, typename P>
struct BatchVariant {
  static constexpr int DX = split_dx(D);
  static constexpr int DV = D - DX;
  static constexpr bool K3 = D == 6 && N == 4;
  static constexpr int RD = (N <= 3 && DV >= 2) ? 2 : 1;
  static constexpr int T = ipow(N, D - RD);
  static constexpr bool LDS =
      !K3 && T <= kBatchThreads &&
      (size_t)(kBatchThreads / T) * ipow(N, D) * sizeof(P) <= kBatchCellLds;
  static constexpr int CPW = LDS ? kBatchThreads / T : 1;
  static constexpr size_t SHMEM =
      K3 ? k3_lds_bytes<P>() : (LDS ? (size_t)CPW * ipow(N, D) * sizeof(P) : 0);
};

struct VariantInfo {
  int k3, lds, cpw, threads_per_cell;
  size_t shmem;
};

template <int D, int N, typename P>
VariantInfo info_of() {
  using V = BatchVariant<D, N, P>;
  return VariantInfo{V::K3 ? 1 : 0, V::LDS ? 1 : 0, V::CPW, V::T, V::SHMEM};
}

template <typename P>
VariantInfo variant_info(int d, int n) {
#define HD_BV_CASE(DD, NN) \
  if (d == DD && n == NN) return info_of<DD, NN, P>();
#define HD_BV_ROW(DD) HD_BV_CASE(DD, 2) HD_BV_CASE(DD, 3) HD_BV_CASE(DD, 4) HD_BV_CASE(DD, 5) HD_BV_CASE(DD, 6)
  HD_BV_ROW(2) HD_BV_ROW(3) HD_BV_ROW(4) HD_BV_ROW(5) HD_BV_ROW(6)
  return VariantInfo{0, 0, 1, 0, 0};
}

template <int D, int N, typename P>
__device__ __forceinline__ void run_one(const StageParams<P> &prm, unsigned tile,
                                        unsigned char *smem, bool reuse) {
  using V = BatchVariant<D, N, P>;
  if constexpr (V::K3)
    stage_k3_body<P, sizeof(P) == 4 ? (kOptStream | kOptKeepU64) : kOptStream>(prm, tile, smem,
                                                                              reuse);
  else
    stage_body<D, N, V::DX, V::RD, P, V::LDS>(prm, tile, reinterpret_cast<P *>(smem), reuse);
}

template <typename P>
__device__ __forceinline__ void run_variant(int variant, const StageParams<P> &prm, unsigned tile,
                                            unsigned char *smem, bool reuse) {
  switch (variant) {
#define HD_RV_CASE(DD, NN) \
  case (DD - 2) * 5 + (NN - 2): run_one<DD, NN, P>(prm, tile, smem, reuse); break;
#define HD_RV_ROW(DD) HD_RV_CASE(DD, 2) HD_RV_CASE(DD, 3) HD_RV_CASE(DD, 4) HD_RV_CASE(DD, 5) HD_RV_CASE(DD, 6)
    HD_RV_ROW(2) HD_RV_ROW(3) HD_RV_ROW(4) HD_RV_ROW(5) HD_RV_ROW(6)
    default: break;
  }
}

// One solve's kernel parameters for every (stage, solution-buffer parity).
template <typename P>
struct BatchEntry {
  StageParams<P> prm[5][2];
  int variant;
  int pad[3];
};

// The work list: active solves, their first work item, and each solve's
// current solution buffer (indexed by solve).
struct BatchList {
  int nact;
  unsigned nitems;
  int act[kMaxBatch];
  unsigned item0[kMaxBatch + 1];
  int cur[kMaxBatch];
};

// Register budget: the largest variant (6D degree 3) bounds every variant's
// occupancy; 2 waves per SIMD in FP64, 3 in FP32.
template <typename P>
constexpr int batch_waves_per_eu() {
  return sizeof(P) == 8 ? 2 : 3;
}

template <typename P>
__global__ void __launch_bounds__(kBatchThreads)
    __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<P>(), batch_waves_per_eu<P>())))
    batch_stage_kernel(const BatchEntry<P> *__restrict__ entries, const BatchList *__restrict__ list,
                       int stage) {
  extern __shared__ unsigned char smem[];
  const int nact = list->nact;
  const unsigned nitems = list->nitems;
  bool reuse = false;
  for (unsigned item = blockIdx.x; item < nitems; item += gridDim.x) {
    int lo = 0, hi = nact;  // item0[lo] <= item < item0[lo + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (list->item0[mid] <= item) lo = mid;
      else hi = mid;
    }
    // (readfirstlane: the values are uniform across the workgroup; saying so
    // keeps the solve's parameters in scalar registers.)
    const int sid = __builtin_amdgcn_readfirstlane(list->act[lo]);
    const unsigned tile = __builtin_amdgcn_readfirstlane(item - list->item0[lo]);
    const int par = __builtin_amdgcn_readfirstlane((list->cur[sid] + stage) & 1);
    run_variant<P>(__builtin_amdgcn_readfirstlane(entries[sid].variant), entries[sid].prm[stage][par],
                   tile, smem, reuse);
    reuse = true;
  }
}

// After the fifth stage every active solve's solution sits in the other buffer.
__global__ void batch_flip_kernel(BatchList *list) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < list->nact) list->cur[list->act[i]] ^= 1;
}

}  // namespace
}  // namespace hd

struct hd_batch {
  std::vector<hd_solver *> solvers;
  int prec = 0;
  std::vector<hd::VariantInfo> info;
  std::vector<unsigned> tiles;
  void *entries_dev = nullptr;  // BatchEntry<P>[n]
  hd::BatchList *list_dev = nullptr;
  std::vector<unsigned char> entries_host;
  hd::BatchList *list_host = nullptr;
  size_t entry_bytes = 0, shmem = 0;
  int grid = 0;
  std::vector<double> dt;       // time step each entry was filled with
  std::vector<int> active;      // active set of the uploaded list
  std::vector<int> dev_cur;     // solution parities as the device holds them
  bool list_valid = false;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

using hd::rt::fail;

template <typename P>
void fill_entry(hd_batch *b, int i, double dt) {
  hd_solver *s = b->solvers[i];
  auto *e = reinterpret_cast<hd::BatchEntry<P> *>(b->entries_host.data() + i * b->entry_bytes);
  const hd::VariantInfo &vi = b->info[i];
  for (int st = 0; st < 5; ++st)
    for (int par = 0; par < 2; ++par) {
      hd::StageParams<P> &prm = e->prm[st][par];
      hd::rt::fill_params<P>(s, &prm, vi.k3 ? 1 : 0);
      prm.cells_per_wg = (unsigned)vi.cpw;
      prm.xcd_remap = 0;
      prm.nblocks = b->tiles[i];
      prm.u_in = s->u(par);
      prm.u_out = s->u(1 - par);
      prm.du = reinterpret_cast<P *>(s->du());
      prm.mode = 1;
      prm.read_du = st > 0;
      prm.write_du = st < 4;
      prm.rk_a = (P)hd::rt::kRkA[st];
      prm.rk_b = hd::rt::kRkB[st];
      prm.dt = (P)dt;
    }
  e->variant = (s->d - 2) * 5 + (s->n - 2);
}

template <typename P>
hd_status create_typed(hd_batch *b) {
  b->entry_bytes = sizeof(hd::BatchEntry<P>);
  const int n = (int)b->solvers.size();
  b->info.resize(n);
  b->tiles.resize(n);
  size_t shmem = 0;
  for (int i = 0; i < n; ++i) {
    hd_solver *s = b->solvers[i];
    b->info[i] = hd::variant_info<P>(s->d, s->n);
    const hd::VariantInfo &vi = b->info[i];
    if (vi.threads_per_cell == 0) return fail(HD_ERR_UNSUPPORTED, "no batched variant for this d, k");
    uint64_t tiles;
    if (vi.k3) tiles = (uint64_t)s->ncells;
    else if (vi.lds) tiles = ((uint64_t)s->ncells + vi.cpw - 1) / vi.cpw;
    else tiles = ((uint64_t)s->ncells * vi.threads_per_cell + hd::kBatchThreads - 1) / hd::kBatchThreads;
    if (tiles >= (1ull << 32)) return fail(HD_ERR_UNSUPPORTED, "solve too large for the batch list");
    b->tiles[i] = (unsigned)tiles;
    shmem = std::max(shmem, vi.shmem);
  }
  b->shmem = shmem;
  b->entries_host.assign(b->entry_bytes * n, 0);
  b->dt.assign(n, 0.0);
  b->dev_cur.assign(n, -1);
  for (int i = 0; i < n; ++i) fill_entry<P>(b, i, 0.0);
  HD_HIP(hipMalloc(&b->entries_dev, b->entry_bytes * n));
  HD_HIP(hipMalloc(&b->list_dev, sizeof(hd::BatchList)));
  HD_HIP(hipHostMalloc(&b->list_host, sizeof(hd::BatchList)));
  std::memset(b->list_host, 0, sizeof(hd::BatchList));
  HD_HIP(hipMemcpy(b->entries_dev, b->entries_host.data(), b->entry_bytes * n, hipMemcpyHostToDevice));
  HD_HIP(hipMemcpy(b->list_dev, b->list_host, sizeof(hd::BatchList), hipMemcpyHostToDevice));
  auto fn = hd::batch_stage_kernel<P>;
  if (shmem > 65536)
    HD_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  int per_cu = 0, dev = 0, cus = 0;
  HD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, hd::kBatchThreads, shmem));
  HD_HIP(hipGetDevice(&dev));
  HD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  b->grid = std::max(1, per_cu) * std::max(1, cus);
  // Capture one RK step.
  HD_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const auto *ent = reinterpret_cast<const hd::BatchEntry<P> *>(b->entries_dev);
  for (int st = 0; st < 5; ++st)
    hipLaunchKernelGGL(fn, dim3(b->grid), dim3(hd::kBatchThreads), shmem, b->cap, ent, b->list_dev, st);
  hipLaunchKernelGGL(hd::batch_flip_kernel, dim3((hd::kMaxBatch + 255) / 256), dim3(256), 0, b->cap,
                     b->list_dev);
  hipError_t le = hipGetLastError();
  hipError_t ce = hipStreamEndCapture(b->cap, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return fail(HD_ERR_HIP, std::string("batch graph capture: ") +
                                hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(HD_ERR_HIP, std::string("batch graph instantiate: ") + hipGetErrorString(ie));
  return HD_OK;
}

void destroy_batch(hd_batch *b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->entries_dev) hipFree(b->entries_dev);
  if (b->list_dev) hipFree(b->list_dev);
  if (b->list_host) hipHostFree(b->list_host);
  delete b;
}

}  // namespace

extern "C" {

hd_status hd_batch_create(hd_solver *const *solvers, int n, hd_batch **out) {
  if (!out || (!solvers && n)) return fail(HD_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (n < 1 || n > hd::kMaxBatch) return fail(HD_ERR_INVALID, "batch size must be 1..1024");
  hd_batch *b = new (std::nothrow) hd_batch();
  if (!b) return fail(HD_ERR_OOM, "host allocation failed");
  for (int i = 0; i < n; ++i) {
    hd_solver *s = solvers[i];
    if (!s || !s->ws) {
      destroy_batch(b);
      return fail(HD_ERR_INVALID, "every batched solver must be bound (hd_bind)");
    }
    for (int j = 0; j < i; ++j)
      if (solvers[j] == s) {
        destroy_batch(b);
        return fail(HD_ERR_INVALID, "a solver appears twice in the batch");
      }
    if (i > 0 && s->prec != solvers[0]->prec) {
      destroy_batch(b);
      return fail(HD_ERR_INVALID, "all batched solvers must have the same precision");
    }
    b->solvers.push_back(s);
  }
  b->prec = solvers[0]->prec;
  hd_status r = b->prec == HD_FP32 ? create_typed<float>(b) : create_typed<double>(b);
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
  hipStream_t st = (hipStream_t)stream;
  std::vector<int> act(n);
  for (int i = 0; i < n; ++i) {
    act[i] = active ? (active[i] != 0) : 1;
    if (act[i] && !(dt[i] == dt[i] && dt[i] > -1e300 && dt[i] < 1e300))
      return fail(HD_ERR_INVALID, "dt must be finite");
  }
  // Refresh the entries whose time step changed.
  bool any = false;
  for (int i = 0; i < n; ++i) {
    if (!act[i] || dt[i] == b->dt[i]) continue;
    if (b->prec == HD_FP32) fill_entry<float>(b, i, dt[i]);
    else fill_entry<double>(b, i, dt[i]);
    b->dt[i] = dt[i];
    HD_HIP(hipMemcpyAsync(static_cast<char *>(b->entries_dev) + i * b->entry_bytes,
                          b->entries_host.data() + i * b->entry_bytes, b->entry_bytes,
                          hipMemcpyHostToDevice, st));
  }
  // Refresh the work list and the solution parities.
  bool list_dirty = !b->list_valid || act != b->active;
  for (int i = 0; i < n; ++i)
    if (b->dev_cur[i] != b->solvers[i]->cur) list_dirty = true;  // stepped outside the batch
  if (list_dirty) {
    HD_HIP(hipStreamSynchronize(st));  // the pinned staging copy may still be in flight
    hd::BatchList *L = b->list_host;
    L->nact = 0;
    unsigned items = 0;
    for (int i = 0; i < n; ++i) {
      L->cur[i] = b->solvers[i]->cur;
      if (!act[i]) continue;
      L->act[L->nact] = i;
      L->item0[L->nact] = items;
      items += b->tiles[i];
      ++L->nact;
    }
    L->item0[L->nact] = items;
    L->nitems = items;
    HD_HIP(hipMemcpyAsync(b->list_dev, L, sizeof(hd::BatchList), hipMemcpyHostToDevice, st));
    b->active = act;
    for (int i = 0; i < n; ++i) b->dev_cur[i] = L->cur[i];
    b->list_valid = true;
  }
  for (int i = 0; i < n; ++i) any = any || act[i];
  if (!any) return HD_OK;
  HD_HIP(hipGraphLaunch(b->gexec, st));
  // The graph's last kernel flips the device parities of the active solves.
  for (int i = 0; i < n; ++i)
    if (act[i]) {
      b->solvers[i]->cur ^= 1;
      b->dev_cur[i] ^= 1;
    }
  return HD_OK;
}

}  // extern "C"
