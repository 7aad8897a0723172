// mi_kernels.hip -- kernel entry points and their launchers.
#include <algorithm>

#include "mi_device.hpp"
#include "mi_internal.hpp"

namespace mi {

#define MI_DECLARE_SMEM(C, sm)                                               \
  __shared__ __attribute__((aligned(16))) uint8_t ring0_[C::STAGE];         \
  __shared__ __attribute__((aligned(16))) uint8_t ring1_[C::STAGE];         \
  __shared__ __attribute__((aligned(16))) uint8_t ring2_[C::STAGE];         \
  __shared__ __attribute__((aligned(16))) uint8_t ring3_[C::STAGE];         \
  __shared__ __attribute__((aligned(16))) int32_t cols_[2 * C::BT + 4];     \
  __shared__ __attribute__((aligned(16))) float rcp_[4 * C::BT];            \
  __shared__ __attribute__((aligned(16))) float mir_[C::BT == 256 ? C::NWAVES * 16 * 36 : 4]; \
  const Smem<C> sm{{ring0_, ring1_, ring2_, ring3_}, cols_, rcp_, C::BT == 256 ? mir_ : nullptr}

// Plain launch of one dataset: one workgroup per (tile, K split) unit.
// Workgroup u runs on XCD u % 8.  XCD x owns the tile ranks
// [x * tpx, (x + 1) * tpx) of the Morton order table (a compact block of the
// triangle) for every split, and sweeps the splits in order, so the units
// resident on one XCD at a time read the same rows of a few shared column
// panels, which its L2 then serves.  Orders without that sharing (splits
// spread over XCDs, or each workgroup streaming its own share of all tiles)
// measured 1.2-1.7x slower on the 1,000,000 x 4,096 workload, whose input
// does not fit the last-level cache.  Padding units of the grid exit at once.
template <class C, int IN>
__global__ __launch_bounds__(C::NT) void k_plain(ProbDev P) {
  MI_DECLARE_SMEM(C, sm);
  const int u = blockIdx.x;
  const int xcd = u & 7, local = u >> 3;
  const int tpx = P.tiles_per_xcd;
  const int s = local / tpx;
  const int t = xcd * tpx + (local - s * tpx);
  if (t >= P.ntiles || s >= P.splits) return;  // uniform
  const int k0 = s * P.kchunk;
  run_unit<C, IN>(P, t, k0, min(P.m, k0 + P.kchunk), sm);
}

// Persistent workgroups pull units of many datasets from a device queue.  IN:
// the input layout of every dataset of the launch (bytes: int8 Gram, FP4: FP4
// Gram); a batch with both runs one launch of each.  Two waves per SIMD are
// requested explicitly: left alone, the compiler gives the 128-wide FP4
// variant 211 VGPRs + 64 AGPRs and a single wave per SIMD.
template <class C, int IN>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_persistent(const ProbDev* __restrict__ probs,
                                                      const UnitRef* __restrict__ units, int nunits,
                                                      int* __restrict__ head) {
  MI_DECLARE_SMEM(C, sm);
  __shared__ int s_u;
  for (;;) {
    if (threadIdx.x == 0) s_u = atomicAdd(head, 1);
    __syncthreads();
    const int u = __builtin_amdgcn_readfirstlane(s_u);  // uniform: scalar loads of the unit and its dataset
    __syncthreads();
    if (u >= nunits) break;  // uniform: every wave leaves together
    const UnitRef ur = units[u];
    const ProbDev P = probs[ur.prob];
    const int k0 = ur.split * P.kchunk;
    run_unit<C, IN>(P, ur.tile, k0, min(P.m, k0 + P.kchunk), sm);
    __syncthreads();
  }
}

__global__ void k_fill_i32(int* p, int v, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

template <class C>
static hipError_t launch_plain_c(const ProbDev& P, hipStream_t st) {
  const int64_t grid = 8LL * P.tiles_per_xcd * P.splits;
  if (P.packed == kInFp4)
    hipLaunchKernelGGL((k_plain<C, kInFp4>), dim3((unsigned)grid), dim3(C::NT), 0, st, P);
  else if (P.packed == kInBitsFp4)
    hipLaunchKernelGGL((k_plain<C, kInBitsFp4>), dim3((unsigned)grid), dim3(C::NT), 0, st, P);
  else if (P.packed == kInBits)
    hipLaunchKernelGGL((k_plain<C, kInBits>), dim3((unsigned)grid), dim3(C::NT), 0, st, P);
  else
    hipLaunchKernelGGL((k_plain<C, kInBytes>), dim3((unsigned)grid), dim3(C::NT), 0, st, P);
  return hipGetLastError();
}

hipError_t launch_plain(int cfg, const ProbDev& P, hipStream_t st) {
  if (P.ntiles <= 0 || P.splits <= 0) return hipSuccess;
  return cfg == 1 ? launch_plain_c<Cfg256>(P, st) : launch_plain_c<Cfg128>(P, st);
}

hipError_t launch_persistent(int cfg, bool fp4, const ProbDev* probs, const UnitRef* units, int nunits, int* head,
                             int grid, hipStream_t st) {
  if (nunits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, head, 0, 1);
  if (cfg == 1 && fp4)
    hipLaunchKernelGGL((k_persistent<Cfg256, kInFp4>), dim3(grid), dim3(Cfg256::NT), 0, st, probs, units, nunits, head);
  else if (cfg == 1)
    hipLaunchKernelGGL((k_persistent<Cfg256, kInBytes>), dim3(grid), dim3(Cfg256::NT), 0, st, probs, units, nunits, head);
  else if (fp4)
    hipLaunchKernelGGL((k_persistent<Cfg128, kInFp4>), dim3(grid), dim3(Cfg128::NT), 0, st, probs, units, nunits, head);
  else
    hipLaunchKernelGGL((k_persistent<Cfg128, kInBytes>), dim3(grid), dim3(Cfg128::NT), 0, st, probs, units, nunits, head);
  return hipGetLastError();
}

// bytes / 4 int32 zeros at p (bytes a multiple of 4), grid-strided.
__global__ __launch_bounds__(256) void k_zero_i32(int* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t count = (int64_t)(bytes / 4);
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)blocks), dim3(256), 0, st, (int*)p, count);
  return hipGetLastError();
}

hipError_t fill_i32(int* p, int v, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

int cfg_tile(int cfg) { return cfg == 1 ? Cfg256::BT : Cfg128::BT; }
int cfg_threads(int cfg) { return cfg == 1 ? Cfg256::NT : Cfg128::NT; }

int occupancy(int cfg) {
  int blocks = 0;
  hipError_t e = cfg == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<Cfg256, kInBytes>, Cfg256::NT, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<Cfg128, kInBytes>, Cfg128::NT, 0);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

int persistent_occupancy(int cfg, bool fp4) {
  int blocks = 0;
  hipError_t e;
  if (cfg == 1)
    e = fp4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<Cfg256, kInFp4>, Cfg256::NT, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<Cfg256, kInBytes>, Cfg256::NT, 0);
  else
    e = fp4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<Cfg128, kInFp4>, Cfg128::NT, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<Cfg128, kInBytes>, Cfg128::NT, 0);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

}  // namespace mi
