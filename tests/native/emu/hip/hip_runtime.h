// Host stand-in for the HIP device environment the stage kernels use, so
// that tests can compile the kernel sources for the CPU and run them under
// AddressSanitizer (tests/native/emu_stage.cpp). Test harness only: the
// library itself is always built with hipcc for gfx950.
//
// A workgroup runs as blockDim.x host threads; __syncthreads is a barrier
// over them. Workgroups run one after another, so the dynamic LDS
// (hd::smem_raw) is one host array, poisoned beyond the launch's size.
// readfirstlane is given its uniform-value meaning; cross-lane moves (DPP
// quad permutations and row rotations) exchange values between the host
// threads of one 64-lane wave.
#pragma once

#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define amdgpu_waves_per_eu(...)
#define __shared__
#define __align__(n) __attribute__((aligned(n)))

struct emu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};
extern thread_local emu_dim3 threadIdx, blockIdx;
extern emu_dim3 blockDim, gridDim;

void emu_syncthreads();
int emu_mov_dpp(int v, int ctrl);
#define __syncthreads() emu_syncthreads()
#define __builtin_amdgcn_mov_dpp(v, ctrl, row_mask, bank_mask, bound_ctrl) emu_mov_dpp((v), (ctrl))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_readfirstlane(x) (x)
inline int atomicOr(int *p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }

typedef void *hipStream_t;
typedef void *hipGraphExec_t;
typedef void *hipEvent_t;
typedef int hipError_t;
struct double2 {
  double x, y;
};
