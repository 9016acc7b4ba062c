// Runs the library's stage kernels on the host (one host thread per GPU
// thread, workgroups one after another) under AddressSanitizer and
// UndefinedBehaviorSanitizer: every global access must stay inside its
// buffer and every LDS access inside the launch's dynamic LDS. Built by
// tests/test_kernel_emulation_cpu.py with one kernel variant chosen at
// compile time (EMU_D, EMU_N, EMU_DX, EMU_RD, EMU_P, EMU_LDS, EMU_SD,
// EMU_OPT, EMU_LD; EMU_SPLIT: the two dimension-split passes instead).
//
// Usage: emu_stage DIR  with DIR/spec.txt holding
//   cells (d values)  lo (d)  hi (d)  field_kind  a (d) or esign
//   cells_per_wg wg_size xcd_remap  mode stage dt rk_a rk_b
// and DIR/u.bin (FP64 state), DIR/du.bin (increment, operator precision),
// DIR/E.bin (E table, operator precision; phase-space field only). Runs the
// kernel's own launch and its work-list form (two slots: the solve and a
// copy with its own buffers), checks that all three results are bitwise
// equal, and writes DIR/out_u.bin and DIR/out_du.bin (stage mode) or
// DIR/out.bin (operator mode).
#include "hip/hip_runtime.h"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sanitizer/asan_interface.h>
#include <string>
#include <thread>
#include <vector>

#include "hd_internal.h"
#include "stage_k3.h"
#include "stage_split.h"
#include "work_list.h"

thread_local emu_dim3 threadIdx, blockIdx;
emu_dim3 blockDim, gridDim;

namespace hd {
alignas(256) unsigned char smem_raw[160 * 1024];
}

namespace {

// A reusable barrier over the threads of one workgroup (or wave); a thread
// that returns from the kernel leaves it. Waiting threads yield the CPU
// (there are far more of them than cores).
struct Barrier {
  std::mutex mu;
  int expected = 0, arrived = 0;
  std::atomic<uint64_t> gen{0};
  void arrive_and_wait() {
    uint64_t g;
    {
      std::lock_guard<std::mutex> lk(mu);
      g = gen.load();
      if (++arrived == expected) {
        arrived = 0;
        gen.store(g + 1);
        return;
      }
    }
    const auto t0 = std::chrono::steady_clock::now();
    while (gen.load() == g) {
      std::this_thread::yield();
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) {
        std::fprintf(stderr, "barrier timeout (divergent barrier or cross-lane move)\n");
        std::abort();
      }
    }
  }
  void leave() {
    std::lock_guard<std::mutex> lk(mu);
    --expected;
    if (arrived == expected && arrived > 0) {
      arrived = 0;
      gen.store(gen.load() + 1);
    }
  }
};
Barrier *g_bar = nullptr;

// Per wave of a workgroup: a barrier over its threads and an exchange
// buffer for cross-lane moves.
struct Wave {
  Barrier bar;
  int buf[64];
  bool live[64];
};
std::vector<Wave> *g_waves = nullptr;

// The workgroups of a grid, one after another, each on `block` host
// threads that stay alive across workgroups (a gate between workgroups
// resets the LDS and the barriers).
template <typename F>
void run_grid(unsigned grid, unsigned block, size_t shmem, F kernel) {
  gridDim.x = grid;
  blockDim.x = block;
  Barrier bar, gate;
  gate.expected = (int)block;
  const unsigned nw = (block + 63) / 64;
  std::vector<Wave> waves(nw);
  std::mutex gmu;
  int at_gate = 0;
  auto fresh_block = [&] {
    // Fresh LDS contents (NaN pattern), poisoned beyond the launch's bytes.
    ASAN_UNPOISON_MEMORY_REGION(hd::smem_raw, sizeof(hd::smem_raw));
    std::memset(hd::smem_raw, 0xff, sizeof(hd::smem_raw));
    ASAN_POISON_MEMORY_REGION(hd::smem_raw + shmem, sizeof(hd::smem_raw) - shmem);
    bar.expected = (int)block;
    bar.arrived = 0;
    for (unsigned w = 0; w < nw; ++w) {
      waves[w].bar.expected = (int)std::min(64u, block - 64 * w);
      waves[w].bar.arrived = 0;
      for (int l = 0; l < 64; ++l) waves[w].live[l] = 64 * w + l < block;
    }
  };
  fresh_block();
  g_bar = &bar;
  g_waves = &waves;
  std::vector<std::thread> th;
  th.reserve(block);
  for (unsigned t = 0; t < block; ++t)
    th.emplace_back([&, t] {
      threadIdx.x = t;
      for (unsigned b = 0; b < grid; ++b) {
        blockIdx.x = b;
        kernel();
        {
          Wave &wv = waves[t / 64];
          std::lock_guard<std::mutex> lk(wv.bar.mu);
          wv.live[t % 64] = false;
        }
        waves[t / 64].bar.leave();
        bar.leave();
        {
          // The last thread of this workgroup prepares the next one.
          std::lock_guard<std::mutex> lk(gmu);
          if (++at_gate == (int)block) {
            at_gate = 0;
            fresh_block();
          }
        }
        gate.arrive_and_wait();
      }
    });
  for (auto &x : th) x.join();
  ASAN_UNPOISON_MEMORY_REGION(hd::smem_raw, sizeof(hd::smem_raw));
}

template <typename T>
std::vector<T> read_bin(const std::string &path, size_t n) {
  std::vector<T> v(n);
  std::ifstream f(path, std::ios::binary);
  if (!f.read(reinterpret_cast<char *>(v.data()), n * sizeof(T))) {
    std::fprintf(stderr, "cannot read %s\n", path.c_str());
    std::exit(2);
  }
  return v;
}

template <typename T>
void write_bin(const std::string &path, const T *p, size_t n) {
  std::ofstream f(path, std::ios::binary);
  f.write(reinterpret_cast<const char *>(p), n * sizeof(T));
}

}  // namespace

void emu_syncthreads() { g_bar->arrive_and_wait(); }

// DPP move within a 64-lane wave: quad_perm (ctrl 0x00-0xff: lane p reads
// lane 4*(p/4) + sel_(p%4)) and row_ror:n (0x121-0x12f: lane p of a 16-lane
// row reads lane (p - n) mod 16 of that row). A source lane that has left
// the kernel is an error.
int emu_mov_dpp(int v, int ctrl) {
  const unsigned t = threadIdx.x, lane = t % 64;
  Wave &wv = (*g_waves)[t / 64];
  wv.buf[lane] = v;
  wv.bar.arrive_and_wait();
  unsigned src;
  if (ctrl >= 0 && ctrl <= 0xff) {
    src = (lane & ~3u) | ((unsigned)(ctrl >> (2 * (lane & 3))) & 3u);
  } else if (ctrl >= 0x121 && ctrl <= 0x12f) {
    const unsigned n = (unsigned)ctrl & 15u;
    src = (lane & ~15u) | ((lane - n) & 15u);
  } else {
    std::fprintf(stderr, "unsupported DPP control 0x%x\n", ctrl);
    std::abort();
  }
  if (!wv.live[src]) {
    std::fprintf(stderr, "DPP move reads lane %u, which has left the kernel\n", src);
    std::abort();
  }
  const int r = wv.buf[src];
  wv.bar.arrive_and_wait();
  return r;
}

#ifdef EMU_SPLIT
// The dimension-split passes (plan kernel 2): pass x, then pass v, on one
// set of buffers, with the library's launch shapes.
template <typename P, int D, int N, int DX>
int run_split(hd_solver &s, const std::string &dir, int mode, int stage, double dt, double rk_a,
              double rk_b, int xcd, size_t nE) {
  using S = hd::SplitShape<D, N, DX, sizeof(P)>;
  const size_t nd = (size_t)s.ndofs;
  const std::vector<double> u = read_bin<double>(dir + "/u.bin", nd);
  std::vector<P> du = read_bin<P>(dir + "/du.bin", nd);
  std::vector<P> E(std::max<size_t>(nE, 1), P(0));
  if (s.field_kind == 1) E = read_bin<P>(dir + "/E.bin", nE);
  std::vector<double> uo(nd, -7.0);
  std::vector<P> out(nd, P(-7));
  hd::StageParams<P> prm;
  hd::rt::fill_params<P>(&s, &prm, 0);
  prm.xcd_remap = xcd;
  prm.E = E.data();
  prm.u_in = u.data();
  prm.mode = mode;
  prm.du = du.data();
  if (mode == 0) {
    prm.out = out.data();
  } else {
    prm.u_out = uo.data();
    prm.read_du = stage > 0;
    prm.write_du = stage < 4;
    prm.rk_a = (P)rk_a;
    prm.rk_b = rk_b;
    prm.dt = (P)dt;
  }
  const uint64_t rows = (uint64_t)s.ncells * S::NVB;
  const unsigned gx = (unsigned)((rows + S::R - 1) / S::R);
  const unsigned gv = (unsigned)(s.ncells * S::NCH);
  const size_t lx = hd::split_x_lds_bytes<D, N, DX, P>(), lv = hd::split_v_lds_bytes<D, N, DX, P>();
  prm.nblocks = gx;
  const hd::StageParams<P> px = prm;
  run_grid(gx, S::TX, lx, [&] { hd::stage_split_x_kernel<D, N, DX, P, EMU_OPT>(px); });
  prm.nblocks = gv;
  const hd::StageParams<P> pv = prm;
  run_grid(gv, S::TV, lv, [&] { hd::stage_split_v_kernel<D, N, DX, P, EMU_OPT>(pv); });
  if (mode == 0) {
    write_bin(dir + "/out.bin", out.data(), nd);
  } else {
    write_bin(dir + "/out_u.bin", uo.data(), nd);
    write_bin(dir + "/out_du.bin", du.data(), nd);
  }
  std::printf("split: pass x grid %u lds %zu, pass v grid %u lds %zu\n", gx, lx, gv, lv);
  return 0;
}
#endif

int main(int argc, char **argv) {
  using P = EMU_P;
  constexpr int D = EMU_D, N = EMU_N, DX = EMU_DX, RD = EMU_RD, SD = EMU_SD, LD = EMU_LD;
  constexpr bool LDS = EMU_LDS;
  if (argc < 2) return 2;
  const std::string dir = argv[1];
  std::ifstream spec(dir + "/spec.txt");
  hd_solver s;
  s.d = D;
  s.dx = DX;
  s.dv = D - DX;
  s.k = N - 1;
  s.n = N;
  s.prec = sizeof(P) == 4 ? HD_FP32_OP_FP64_ACC : HD_FP64;
  s.mesh.dim_x = DX;
  s.mesh.dim_v = D - DX;
  for (int j = 0; j < D; ++j) spec >> s.mesh.cells[j];
  for (int j = 0; j < D; ++j) spec >> s.mesh.lo[j];
  for (int j = 0; j < D; ++j) spec >> s.mesh.hi[j];
  spec >> s.field_kind;
  if (s.field_kind == 0)
    for (int j = 0; j < D; ++j) spec >> s.a_const[j];
  else
    spec >> s.esign;
  int cpw, wg, xcd, mode, stage;
  double dt, rk_a, rk_b;
  spec >> cpw >> wg >> xcd >> mode >> stage >> dt >> rk_a >> rk_b;
  if (!spec) return 2;
  s.nd = 1;
  s.ncells = 1;
  for (int j = 0; j < D; ++j) {
    s.nd *= N;
    s.ncells *= s.mesh.cells[j];
    s.h[j] = (s.mesh.hi[j] - s.mesh.lo[j]) / s.mesh.cells[j];
  }
  s.ndofs = s.nd * s.ncells;
  if (!hd::make_tables(N - 1, &s.tab)) return 2;
  s.plan.lds = LDS;
  s.plan.cells_per_wg = cpw;
  s.plan.wg_size = wg;
  s.plan.xcd_remap = xcd;
  s.plan.reg_dims = RD;
  s.plan.split_dims = SD;
  s.plan.loop_dims = LD;
  s.plan.options = EMU_OPT;
  s.plan.kernel = 0;
  const size_t nd = (size_t)s.ndofs;
  int64_t nxnodes = 1;
  for (int j = 0; j < DX; ++j) nxnodes *= s.mesh.cells[j] * N;
  const size_t nE = (size_t)(nxnodes * DX);

#ifdef EMU_K3
  // The 6D degree-3 kernel: one cell per 256-thread workgroup.
  constexpr bool K3 = true;
#else
  constexpr bool K3 = false;
#endif
  s.plan.kernel = K3 ? 1 : 0;
#ifdef EMU_SPLIT
  s.plan.kernel = 2;
  return run_split<P, D, N, DX>(s, dir, mode, stage, dt, rk_a, rk_b, xcd, nE);
#endif
  // Launch shape of the generic kernel under this plan (as the library's).
  int64_t T = 1, per_cell = 1;
  for (int j = 0; j < D - RD - SD - LD; ++j) T *= N;
  for (int j = 0; j < SD; ++j) per_cell *= N;
  unsigned grid, block;
  size_t shmem;
  if (K3) {
    grid = (unsigned)s.ncells;
    block = 256;
    shmem = 4096 * sizeof(P);
  } else if (LDS) {
    const int64_t units = s.ncells * per_cell;
    grid = (unsigned)((units + cpw - 1) / cpw);
    block = (unsigned)(cpw * T);
    shmem = (size_t)(cpw * (s.nd / per_cell)) * sizeof(P);
  } else {
    grid = (unsigned)((s.ncells * T + wg - 1) / wg);
    block = (unsigned)wg;
    shmem = 0;
  }

  const std::vector<double> u = read_bin<double>(dir + "/u.bin", nd);
  const std::vector<P> du0 = read_bin<P>(dir + "/du.bin", nd);
  std::vector<P> E;
  if (s.field_kind == 1) E = read_bin<P>(dir + "/E.bin", nE);
  else if (K3) {
    // The 6D degree-3 kernel reads a constant a_v from the E table.
    E.resize(nE);
    for (size_t i = 0; i < nE; ++i) E[i] = (P)s.a_const[DX + (int)(i % DX)];
  }
  // Stage variant of the 6D degree-3 kernel and its cell order (as the
  // library chooses them): first stage, late increment (FP32 after the
  // first stage, FP64 last stage) or general; the FP64 first and late
  // variants take one slab of cells per XCD.
  const bool f32 = sizeof(P) == 4;
  const int role = mode != 1 ? 0 : (stage == 0 ? 1 : (f32 || stage == 4 ? 2 : 0));
  if (K3 && !f32 && role != 0) xcd = 1;

  struct Bufs {
    std::vector<double> u, uo;
    std::vector<P> du, out, E;
  };
  auto make = [&]() {
    Bufs b;
    b.u = u;
    b.uo.assign(nd, -7.0);
    b.du = du0;
    b.out.assign(nd, P(-7));
    b.E = E;
    if (b.E.empty()) b.E.assign(std::max<size_t>(nE, 1), P(0));
    return b;
  };
  auto params = [&](Bufs &b) {
    // A constant field passes its a_v in the E table (the kernel reads
    // prm.a_const for the generic variant; the table is unused then).
    hd::StageParams<P> prm;
    hd::rt::fill_params<P>(&s, &prm, K3 ? 1 : 0);
    prm.xcd_remap = xcd;
    prm.E = b.E.data();
    prm.nblocks = grid;
    prm.u_in = b.u.data();
    prm.mode = mode;
    prm.du = b.du.data();  // as the library passes it, also to operator applications
    if (mode == 0) {
      prm.out = b.out.data();
    } else {
      prm.u_out = b.uo.data();
      prm.du = b.du.data();
      prm.read_du = stage > 0;
      prm.write_du = stage < 4;
      prm.rk_a = (P)rk_a;
      prm.rk_b = rk_b;
      prm.dt = (P)dt;
    }
    return prm;
  };

  // The kernel's own launch.
  Bufs own = make();
  const hd::StageParams<P> prm_own = params(own);
  run_grid(grid, block, shmem, [&] {
#ifdef EMU_K3
    if (role == 1) hd::stage_k3_kernel<P, EMU_OPT, hd::kK3First>(prm_own);
    else if (role == 2) hd::stage_k3_kernel<P, EMU_OPT, hd::kK3Last>(prm_own);
    else hd::stage_k3_kernel<P, EMU_OPT, hd::kK3General>(prm_own);
#else
    hd::stage_kernel<D, N, DX, RD, P, LDS, SD, EMU_OPT, LD>(prm_own);
#endif
  });

  // The work-list form: the solve and a copy with its own buffers.
  Bufs a = make(), b = make();
  std::vector<hd::StageParams<P>> prms = {params(a), params(b)};
  std::vector<uint32_t> item0;
  std::string why;
  if (!hd::build_work_list({grid, grid}, &item0, &why) || !hd::check_work_list({grid, grid}, item0, &why)) {
    std::fprintf(stderr, "work list: %s\n", why.c_str());
    return 1;
  }
  hd::ListParams<P> lp;
  lp.prm = (hd::ConstStageParams<P> *)prms.data();
  lp.item0 = item0.data();
  lp.nslots = 2;
  lp.nitems = item0.back();
  run_grid(lp.nitems, block, shmem, [&] {
#ifdef EMU_K3
    if (role == 1) hd::stage_k3_list_kernel<P, EMU_OPT, hd::kK3First>(lp);
    else if (role == 2) hd::stage_k3_list_kernel<P, EMU_OPT, hd::kK3Last>(lp);
    else hd::stage_k3_list_kernel<P, EMU_OPT, hd::kK3General>(lp);
#else
    hd::stage_list_kernel<D, N, DX, RD, P, LDS, SD, EMU_OPT, LD>(lp);
#endif
  });

  auto same = [&](const Bufs &x, const Bufs &y) {
    if (mode == 0) return std::memcmp(x.out.data(), y.out.data(), nd * sizeof(P)) == 0;
    return std::memcmp(x.uo.data(), y.uo.data(), nd * sizeof(double)) == 0 &&
           std::memcmp(x.du.data(), y.du.data(), nd * sizeof(P)) == 0;
  };
  const bool ok_a = same(own, a), ok_b = same(own, b);
  if (mode == 0) {
    write_bin(dir + "/out.bin", own.out.data(), nd);
  } else {
    write_bin(dir + "/out_u.bin", own.uo.data(), nd);
    write_bin(dir + "/out_du.bin", own.du.data(), nd);
  }
  std::printf("grid %u block %u shmem %zu work-list items %u: list slot 0 %s, slot 1 %s\n", grid,
              block, shmem, lp.nitems, ok_a ? "equal" : "DIFFERS", ok_b ? "equal" : "DIFFERS");
  return ok_a && ok_b ? 0 : 1;
}
