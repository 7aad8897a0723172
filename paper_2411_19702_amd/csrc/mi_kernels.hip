// mi_kernels.hip -- kernel entry points and their launchers.
#include "mi_device.hpp"
#include "mi_internal.hpp"

namespace mi {

// One workgroup per (tile, split) unit; unit u = split * ntiles + tile so that
// workgroups that run together share a K range (their panels overlap in L2).
template <int BT, bool ALIGNED>
__global__ __launch_bounds__(NTHREADS) void k_plain(ProbDev P) {
  __shared__ __attribute__((aligned(16))) uint8_t smem[TileGeom<BT>::LDS_BYTES];
  const int u = blockIdx.x;
  run_unit<BT, ALIGNED>(P, u % P.ntiles, u / P.ntiles, smem);
}

// Persistent workgroups pull units of many datasets from a device queue.
template <int BT>
__global__ __launch_bounds__(NTHREADS) void k_persistent(const ProbDev* __restrict__ probs,
                                                         const UnitRef* __restrict__ units, int nunits,
                                                         int* __restrict__ head) {
  __shared__ __attribute__((aligned(16))) uint8_t smem[TileGeom<BT>::LDS_BYTES];
  __shared__ int s_u;
  for (;;) {
    if (threadIdx.x == 0) s_u = atomicAdd(head, 1);
    __syncthreads();
    const int u = s_u;
    __syncthreads();
    if (u >= nunits) break;  // uniform: every wave leaves together
    const UnitRef ur = units[u];
    const ProbDev P = probs[ur.prob];
    if (P.aligned)
      run_unit<BT, true>(P, ur.tile, ur.split, smem);
    else
      run_unit<BT, false>(P, ur.tile, ur.split, smem);
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

template <int BT>
static hipError_t launch_plain_bt(const ProbDev& P, int units, hipStream_t st) {
  if (P.aligned)
    hipLaunchKernelGGL((k_plain<BT, true>), dim3(units), dim3(NTHREADS), 0, st, P);
  else
    hipLaunchKernelGGL((k_plain<BT, false>), dim3(units), dim3(NTHREADS), 0, st, P);
  return hipGetLastError();
}

hipError_t launch_plain(int bt, const ProbDev& P, hipStream_t st) {
  const int units = P.ntiles * P.splits;
  if (units <= 0) return hipSuccess;
  return bt == 256 ? launch_plain_bt<256>(P, units, st) : launch_plain_bt<128>(P, units, st);
}

hipError_t launch_persistent(int bt, const ProbDev* probs, const UnitRef* units, int nunits, int* head, int grid,
                             hipStream_t st) {
  if (nunits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, head, 0, 1);
  if (bt == 256)
    hipLaunchKernelGGL(k_persistent<256>, dim3(grid), dim3(NTHREADS), 0, st, probs, units, nunits, head);
  else
    hipLaunchKernelGGL(k_persistent<128>, dim3(grid), dim3(NTHREADS), 0, st, probs, units, nunits, head);
  return hipGetLastError();
}

hipError_t launch_validate(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flag, 0, 1);
  const int64_t blocks = m < 4096 ? m : 4096;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, flag);
  return hipGetLastError();
}

hipError_t fill_i32(int* p, int v, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

int occupancy(int bt) {
  int blocks = 0;
  hipError_t e;
  if (bt == 256)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<256, true>, NTHREADS, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<128, true>, NTHREADS, 0);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

int persistent_occupancy(int bt) {
  int blocks = 0;
  hipError_t e;
  if (bt == 256)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<256>, NTHREADS, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<128>, NTHREADS, 0);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

}  // namespace mi
