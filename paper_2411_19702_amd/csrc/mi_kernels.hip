// mi_kernels.hip -- kernel entry points and their launchers.
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
  const Smem<C> sm{{ring0_, ring1_, ring2_, ring3_}, cols_, rcp_}

// Plain launch of one dataset: one workgroup per (tile, K split) unit.
// Workgroup u runs on XCD u % 8.  XCD x owns the tile ranks
// [x * tpx, (x + 1) * tpx) of the Morton order table (a compact block of the
// triangle) for every split, and sweeps the splits in order, so the units
// resident on one XCD at a time read the same rows of a few shared column
// panels, which its L2 then serves.  Orders without that sharing (splits
// spread over XCDs, or each workgroup streaming its own share of all tiles)
// measured 1.2-1.7x slower on the 1,000,000 x 4,096 workload, whose input
// does not fit the last-level cache.  Padding units of the grid exit at once.
template <class C>
__global__ __launch_bounds__(C::NT) void k_plain(ProbDev P) {
  MI_DECLARE_SMEM(C, sm);
  const int u = blockIdx.x;
  const int xcd = u & 7, local = u >> 3;
  const int tpx = P.tiles_per_xcd;
  const int s = local / tpx;
  const int t = xcd * tpx + (local - s * tpx);
  if (t >= P.ntiles || s >= P.splits) return;  // uniform
  const int k0 = s * P.kchunk;
  run_unit<C>(P, t, k0, min(P.m, k0 + P.kchunk), sm);
}

// Persistent workgroups pull units of many datasets from a device queue.
template <class C>
__global__ __launch_bounds__(C::NT) void k_persistent(const ProbDev* __restrict__ probs,
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
    run_unit<C>(P, ur.tile, k0, min(P.m, k0 + P.kchunk), sm);
    __syncthreads();
  }
}

__global__ void k_fill_i32(int* p, int v, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// flag |= (some byte of X[:, :n] is not 0/1)
__global__ void k_validate(const uint8_t* __restrict__ X, int64_t m, int64_t n, int64_t ldx, int* flag) {
  int bad = 0;
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const uint8_t* r = X + row * ldx;
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) bad |= (r[c] > 1);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Y[r][c] = X[r][c] for c < n, 0 for n <= c < ldy: a 16-byte aligned copy with
// pitch ldy (a multiple of 16) for layouts the DMA path cannot read directly.
__global__ void k_repack(const uint8_t* __restrict__ X, int64_t m, int64_t n, int64_t ldx, uint8_t* __restrict__ Y,
                         int64_t ldy) {
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const uint8_t* src = X + row * ldx;
    uint32_t* dst = reinterpret_cast<uint32_t*>(Y + row * ldy);
    for (int64_t w = threadIdx.x; w < ldy / 4; w += blockDim.x) {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t c = 4 * w + b;
        if (c < n) v |= (uint32_t)src[c] << (8 * b);
      }
      dst[w] = v;
    }
  }
}

template <class C>
static hipError_t launch_plain_c(const ProbDev& P, hipStream_t st) {
  const int64_t grid = 8LL * P.tiles_per_xcd * P.splits;
  hipLaunchKernelGGL(k_plain<C>, dim3((unsigned)grid), dim3(C::NT), 0, st, P);
  return hipGetLastError();
}

hipError_t launch_plain(int cfg, const ProbDev& P, hipStream_t st) {
  if (P.ntiles <= 0 || P.splits <= 0) return hipSuccess;
  return cfg == 1 ? launch_plain_c<Cfg256>(P, st) : launch_plain_c<Cfg128>(P, st);
}

hipError_t launch_persistent(int cfg, const ProbDev* probs, const UnitRef* units, int nunits, int* head, int grid,
                             hipStream_t st) {
  if (nunits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, head, 0, 1);
  if (cfg == 1)
    hipLaunchKernelGGL(k_persistent<Cfg256>, dim3(grid), dim3(Cfg256::NT), 0, st, probs, units, nunits, head);
  else
    hipLaunchKernelGGL(k_persistent<Cfg128>, dim3(grid), dim3(Cfg128::NT), 0, st, probs, units, nunits, head);
  return hipGetLastError();
}

hipError_t launch_validate(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flag, 0, 1);
  const int64_t blocks = m < 4096 ? m : 4096;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, flag);
  return hipGetLastError();
}

hipError_t launch_repack(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Y, int64_t ldy,
                         hipStream_t st) {
  const int64_t blocks = m < 8192 ? m : 8192;
  hipLaunchKernelGGL(k_repack, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, Y, ldy);
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
  hipError_t e = cfg == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<Cfg256>, Cfg256::NT, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<Cfg128>, Cfg128::NT, 0);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

int persistent_occupancy(int cfg) {
  int blocks = 0;
  hipError_t e = cfg == 1
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<Cfg256>, Cfg256::NT, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<Cfg128>, Cfg128::NT, 0);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

}  // namespace mi
