// mi_sparse.hip -- sparse-input path of the all-pairs MI (for inputs where
// nearly every entry is 0).
//
// The method's only matrix product is the Gram n11 = X^T X (Section 2 step 2,
// Section 3.1).  For a very sparse X it is cheaper as a sum over rows of the
// pairs of columns that are both 1 in that row: a row with k ones adds 1 to
// k (k - 1) / 2 counts, so the work is about m (n p)^2 / 2 instead of
// m n^2 / 2 for density p (the paper's sparse variant wins at the highest
// sparsity, Section 4.2 / Fig. 3).  Steps, all on the caller's stream:
//   1. count pass: ones per row and per column (the column sums c);
//   2. exclusive scan of the row counts -> row offsets (three small
//      kernels: chunk sums, a one-block scan of the sums, chunk scans);
//   3. fill pass: the column indices of every row's ones, ascending;
//   4. pair pass: one wave per row adds 1 to n11[a][b] for every a < b of
//      its ones (int32 atomics, exact);
//   5. epilogue over 64 x 64 output tiles: derived cells and MI with the
//      same per-pair arithmetic as the fused kernel (bitwise the same
//      values), tile and mirror written coalesced, optional counts, column
//      sums and sparse pair list.
// The total number of ones is read back once (to size the index list), so
// the call synchronises its stream once.  The automatic choice first counts
// the ones of a sample of rows (one short kernel and a 16-byte read-back);
// only when the sample leaves the choice open does it run the full count
// before deciding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "mi_device.hpp"
#include "mi_host.hpp"
#include "mi_internal.hpp"

namespace mi {

namespace {

constexpr int kHistCols = 16384;  // column sums in LDS up to this many columns
constexpr int64_t kSampleRows = 4096;  // rows sampled by the automatic choice

// Ones in the 16-byte chunk [c, c + 16) of a row (bytes past n count 0): the
// bytes are 0/1, so a dword's ones are its popcount.
__device__ __forceinline__ void chunk_bytes(const uint8_t* row, int64_t c, int32_t n, bool vec, uint8_t (&b)[16]) {
  if (vec && c + 16 <= n) {
    const uint4 v = *reinterpret_cast<const uint4*>(row + c);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) b[k] = (uint8_t)((w[k >> 2] >> (8 * (k & 3))) & 0xFF);
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) b[k] = (c + k < n) ? row[c + k] : (uint8_t)0;
  }
}

// 1. Ones per row (int64, for the scan) and per column, and the number of
//    pairs of ones summed over rows (the pair pass's work).  One wave per
//    row; lane l reads the 16-byte chunks l, l + 64, ...
__global__ __launch_bounds__(256) void k_sp_count(const uint8_t* __restrict__ X, int64_t m, int32_t n, int64_t ldx,
                                                  bool vec, int64_t* __restrict__ row_nnz,
                                                  int32_t* __restrict__ colsum,
                                                  unsigned long long* __restrict__ pair_total) {
  __shared__ int32_t hist[kHistCols];
  __shared__ unsigned long long block_pairs;
  const bool lds = n <= kHistCols;
  if (lds)
    for (int c = threadIdx.x; c < n; c += 256) hist[c] = 0;
  if (threadIdx.x == 0) block_pairs = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < m; r += waves) {
    const uint8_t* row = X + r * ldx;
    int cnt = 0;
    for (int64_t c = 16 * (int64_t)lane; c < n; c += 16 * 64) {
      uint8_t b[16];
      chunk_bytes(row, c, n, vec, b);
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (b[k]) {
          ++cnt;
          if (lds)
            atomicAdd(&hist[c + k], 1);
          else
            atomicAdd(&colsum[c + k], 1);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane == 0) {
      row_nnz[r] = cnt;
      atomicAdd(&block_pairs, (unsigned long long)cnt * (unsigned long long)(cnt > 0 ? cnt - 1 : 0) / 2ull);
    }
  }
  __syncthreads();
  if (lds)
    for (int c = threadIdx.x; c < n; c += 256)
      if (hist[c]) atomicAdd(&colsum[c], hist[c]);
  if (threadIdx.x == 0 && block_pairs) atomicAdd(pair_total, block_pairs);
}

// 3. Column indices of every row's ones, ascending, at the row's offset.
__global__ __launch_bounds__(256) void k_sp_fill(const uint8_t* __restrict__ X, int64_t m, int32_t n, int64_t ldx,
                                                 bool vec, const int64_t* __restrict__ row_ptr,
                                                 int32_t* __restrict__ cols) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < m; r += waves) {
    const uint8_t* row = X + r * ldx;
    int64_t base = row_ptr[r];
    for (int64_t c0 = 0; c0 < n; c0 += 16 * 64) {  // uniform: one 1 KB slice of the row per pass
      const int64_t c = c0 + 16 * lane;
      uint8_t b[16];
      int cnt = 0;
      if (c < n) {
        chunk_bytes(row, c, n, vec, b);
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt += b[k] ? 1 : 0;
      }
      // exclusive prefix of the lane counts
      int incl = cnt;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      const int total = __shfl(incl, 63);
      int64_t pos = base + (incl - cnt);
      if (cnt) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (b[k]) cols[pos++] = (int32_t)(c + k);
      }
      base += total;
    }
  }
}

// 4. Pairs of ones per row -> 1-1 counts (upper triangle, a < b).  One wave
//    per row: the wave walks a, the lanes walk b.
__global__ __launch_bounds__(256) void k_sp_pairs(const int64_t* __restrict__ row_ptr, int64_t m, int32_t n,
                                                  const int32_t* __restrict__ cols, int32_t* __restrict__ acc) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < m; r += waves) {
    const int64_t b0 = row_ptr[r], k = row_ptr[r + 1] - b0;
    for (int64_t a = 0; a + 1 < k; ++a) {
      const int64_t ca = cols[b0 + a];
      int32_t* rowacc = acc + ca * n;
      for (int64_t b = a + 1 + lane; b < k; b += 64) atomicAdd(&rowacc[cols[b0 + b]], 1);
    }
  }
}

// 5. Epilogue over the 64 x 64 output tiles (I <= J): one 256-thread block
//    per tile, 16 rows per thread group pass.
struct SpEpi {
  const int32_t* acc;
  const int32_t* colsum;
  int32_t m, n;
  float* out;
  int32_t* n11_out;
  int32_t* colsum_out;
  int32_t epi;
  float tau;
  int32_t* pairs;
  int64_t pairs_cap;
  unsigned long long* pairs_count;
  float thr;
  int32_t ntb;  // tile blocks per side
};

template <int EPI>
__device__ void sp_tile(const SpEpi& E, int I, int J) {
  __shared__ float sv[64][65];
  __shared__ int32_t sn[64][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;  // 4 waves, each 16 rows
  const int n = E.n, m = E.m;
  const float fm = (float)m, rfm = 1.0f / fm;
  const int j = J * 64 + lane;
  const int cj = j < n ? E.colsum[j] : 0;
  // Column-variable factors 1 / c_j and 1 / (m - c_j), 0 for a zero count.
  const float r1j = cj > 0 ? 1.0f / (float)cj : 0.0f;
  const float r0j = (m - cj) > 0 ? 1.0f / (float)(m - cj) : 0.0f;
  for (int rr = w; rr < 64; rr += 4) {
    const int i = I * 64 + rr;
    float v = 0.0f;
    int v11 = 0;
    const bool upper = i < n && j < n && j >= i;
    if (upper) {
      const int ci = E.colsum[i];
      v11 = (i == j) ? ci : E.acc[(int64_t)i * n + j];
      if (EPI == 2) {
        v = mi_value64(m, ci, cj, v11);
      } else {
        // Row-variable factors m / c_i and m / (m - c_i), as in the fused kernel.
        const float a1i = ci > 0 ? fm / (float)ci : 0.0f;
        const float a0i = (m - ci) > 0 ? fm / (float)(m - ci) : 0.0f;
        v = mi_value32(m, ci, cj, v11, a1i, a0i, r1j, r0j, rfm);
        if (EPI == 1 && v < E.tau) v = mi_value64(m, ci, cj, v11);
      }
      if (E.out) E.out[(int64_t)i * n + j] = v;
      if (E.n11_out) E.n11_out[(int64_t)i * n + j] = v11;
    }
    sv[rr][lane] = v;
    sn[rr][lane] = v11;
    if (E.pairs) {
      const bool q = upper && j > i && v >= E.thr;
      const unsigned long long mask = __ballot(q);
      if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(E.pairs_count, (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
        if (q) {
          const unsigned long long idx = base + __popcll(mask & ((1ull << lane) - 1ull));
          if (idx < (unsigned long long)E.pairs_cap) {
            int32_t* e3 = E.pairs + 3 * idx;
            e3[0] = i;
            e3[1] = j;
            e3[2] = __float_as_int(v);
          }
        }
      }
    }
  }
  __syncthreads();
  // Mirror: row j of the output gets column i, for j > i.
  if (E.out || E.n11_out) {
    for (int cc = w; cc < 64; cc += 4) {
      const int jm = J * 64 + cc, i = I * 64 + lane;
      if (jm < n && i < n && jm > i) {
        if (E.out) E.out[(int64_t)jm * n + i] = sv[lane][cc];
        if (E.n11_out) E.n11_out[(int64_t)jm * n + i] = sn[lane][cc];
      }
    }
  }
  if (E.colsum_out && I == J && w == 0) {
    const int c = I * 64 + lane;
    if (c < n) E.colsum_out[c] = E.colsum[c];
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void k_sp_epi(SpEpi E) {
  // Tile t of the upper triangle in row-major order of (I, J), I <= J.
  const int64_t t = blockIdx.x;
  int I = 0;
  int64_t first = 0;  // tiles before block row I
  while (first + (E.ntb - I) <= t) {
    first += E.ntb - I;
    ++I;
  }
  const int J = I + (int)(t - first);
  sp_tile<EPI>(E, I, J);
}

// 2. Exclusive scan of `count` int64 values, in chunks of kScanChunk per
//    256-thread block (16 consecutive values per thread).
constexpr int kScanChunk = 4096;

// Exclusive prefix of v over the block's NT threads; *total receives the sum.
template <int NT>
__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    before += k < w ? wsum[k] : 0;
    all += wsum[k];
  }
  __syncthreads();  // wsum is reused by the next call
  *total = all;
  return before + incl - v;
}

// Sum of each chunk.
__global__ __launch_bounds__(256) void k_scan_sums(const int64_t* __restrict__ in, int64_t count,
                                                   int64_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + 16 * (int64_t)threadIdx.x;
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (base + k < count) v += in[base + k];
  int64_t total = 0;
  (void)block_exclusive<256>(v, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the nb chunk sums in place, by one block, 1024 at a time.
__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ sums, int64_t nb) {
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {  // uniform
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nb ? sums[i] : 0;
    int64_t total = 0;
    const int64_t ex = block_exclusive<1024>(v, &total);
    if (i < nb) sums[i] = carry + ex;
    carry += total;
  }
}

// Each chunk's exclusive scan, offset by the scanned chunk sums.
__global__ __launch_bounds__(256) void k_scan_apply(const int64_t* __restrict__ in, int64_t count,
                                                    const int64_t* __restrict__ offs, int64_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + 16 * (int64_t)threadIdx.x;
  int64_t v[16];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = base + k < count ? in[base + k] : 0;
    local += v[k];
  }
  int64_t total = 0;
  int64_t run = offs[blockIdx.x] + block_exclusive<256>(local, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (base + k < count) out[base + k] = run;
    run += v[k];
  }
}

// Ones and pairs of ones (k (k - 1) / 2) summed over a sample of rows: row
// s = 0 .. S - 1 is r = (hash of s + seed) scaled to [0, m).  Each wave takes
// every (4 gridDim)-th sample, the block adds its waves' sums, and one lane
// per block adds them to out[0] (ones) and out[1] (pairs).
__device__ __forceinline__ uint32_t sample_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(256) void k_sp_sample(const uint8_t* __restrict__ X, int64_t m, int32_t n, int64_t ldx,
                                                   bool vec, int32_t samples, uint32_t seed,
                                                   unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[2];
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) part[0] = part[1] = 0ull;
  __syncthreads();
  unsigned long long ones = 0, pairs = 0;
  for (int s = blockIdx.x * 4 + (threadIdx.x >> 6); s < samples; s += gridDim.x * 4) {  // uniform per wave
    const int64_t r = (int64_t)(((uint64_t)sample_hash((uint32_t)s + seed) * (uint64_t)m) >> 32);
    const uint8_t* row = X + r * ldx;
    int cnt = 0;
    for (int64_t c = 16 * (int64_t)lane; c < n; c += 16 * 64) {
      uint8_t b[16];
      chunk_bytes(row, c, n, vec, b);
#pragma unroll
      for (int k = 0; k < 16; ++k) cnt += b[k] ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    ones += (unsigned long long)cnt;
    pairs += (unsigned long long)cnt * (unsigned long long)(cnt > 0 ? cnt - 1 : 0) / 2ull;
  }
  if (lane == 0) {
    atomicAdd(&part[0], ones);
    atomicAdd(&part[1], pairs);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], part[0]);
    atomicAdd(&out[1], part[1]);
  }
}

__global__ void k_fill_i32_64(int32_t* p, int32_t v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// The sparse path, or (auto_choice) the choice between it and the dense path
// from a row sample, then if needed from the full count.  Synchronises the
// stream once or twice.
mi_status run_sparse(const mi_problem* p, int64_t ldx, hipStream_t st, bool auto_choice, bool* used) {
  *used = false;
  const int64_t m = p->m;
  const int32_t n = (int32_t)p->n;
  const bool vec = ((uintptr_t)p->X % 16 == 0) && (ldx % 16 == 0);
  DeviceInfo di;
  mi_status s = device_info(&di);
  if (s != MI_OK) return s;
  // Scratch: row counts/offsets (m + 1 int64), column sums (n int32), the
  // scan's chunk sums, the sample's two counters, then (after the count is
  // known) the index list and the n x n count accumulator.
  const int64_t scan_blocks = cdiv64(m + 1, kScanChunk);
  const size_t o_nnz = 0;
  const size_t o_ptr = align256(o_nnz + (size_t)(m + 2) * sizeof(int64_t));
  const size_t o_col = align256(o_ptr + (size_t)(m + 1) * sizeof(int64_t));
  const size_t o_scan = align256(o_col + (size_t)n * sizeof(int32_t));
  const size_t o_smp = align256(o_scan + (size_t)scan_blocks * sizeof(int64_t));
  const size_t head_bytes = align256(o_smp + 2 * sizeof(unsigned long long));
  void* head = nullptr;
  s = scratch(st, 2, 0, head_bytes, &head);
  if (s != MI_OK) return s;
  char* h8 = (char*)head;
  int64_t* row_nnz = (int64_t*)(h8 + o_nnz);
  int64_t* row_ptr = (int64_t*)(h8 + o_ptr);
  int32_t* colsum = (int32_t*)(h8 + o_col);
  int64_t* chunk_sums = (int64_t*)(h8 + o_scan);
  const int blocks = (int)std::min<int64_t>(cdiv64(m, 4), (int64_t)di.cus * 16);
  // Modelled times (rates measured on this device at 1,000,000 x 4,096):
  // the dense kernel sustains ~1.4e15 pair-updates/s with the int8 Gram and
  // ~2.56e15 with the FP4 Gram, after a conversion pass that moves 1.5 bytes
  // per entry at ~5.1 TB/s; the sparse path reads X twice at ~2.7 TB/s, adds
  // ~2.8e10 pair counts/s (random int32 atomics) and writes the n^2 output.
  const double pu = (double)m * (double)n * ((double)n + 1.0) / 2.0;
  const double dense_s = converts_to_fp4(p) ? pu / 2.56e15 + 1.5 * (double)m * (double)n / 5.1e12 : pu / 1.4e15;
  auto sparse_s = [&](double pairs) {
    return (double)m * (double)ldx / 2.7e12 + pairs / 2.8e10 + 4.0 * (double)n * (double)n / 4.0e12;
  };
  if (auto_choice && m > 2 * kSampleRows) {
    // A sample of rows first: its pairs of ones, scaled to m, estimate the
    // sparse path's work.  Clearly dense (sparse estimated 1.5x slower):
    // done, without the count pass.
    unsigned long long* smp = (unsigned long long*)(h8 + o_smp);
    hipLaunchKernelGGL(k_fill_i32_64, dim3(1), dim3(64), 0, st, (int32_t*)smp, 0, (int64_t)4);
    hipLaunchKernelGGL(k_sp_sample, dim3((unsigned)std::min<int64_t>(di.cus, cdiv64(kSampleRows, 4))), dim3(256), 0, st, p->X, m, n, ldx, vec,
                       (int32_t)kSampleRows, 0x9E3779B9u, smp);
    HIPCHK(hipGetLastError());
    unsigned long long hs[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hs, smp, sizeof hs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double est_pairs = (double)hs[1] * (double)m / (double)kSampleRows;
    if (sparse_s(est_pairs) > 1.5 * dense_s) return MI_OK;  // dense: *used stays false
  }
  hipLaunchKernelGGL(k_fill_i32_64, dim3(64), dim3(256), 0, st, colsum, 0, (int64_t)n);
  // row_nnz[m] = 0 closes the scan; row_nnz[m + 1] counts the pairs.
  hipLaunchKernelGGL(k_fill_i32_64, dim3(1), dim3(64), 0, st, (int32_t*)(row_nnz + m), 0, (int64_t)4);
  unsigned long long* pair_total = reinterpret_cast<unsigned long long*>(row_nnz + m + 1);
  hipLaunchKernelGGL(k_sp_count, dim3(blocks), dim3(256), 0, st, p->X, m, n, ldx, vec, row_nnz, colsum, pair_total);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)scan_blocks), dim3(256), 0, st, row_nnz, m + 1, chunk_sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, chunk_sums, scan_blocks);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)scan_blocks), dim3(256), 0, st, row_nnz, m + 1, chunk_sums, row_ptr);
  HIPCHK(hipGetLastError());
  int64_t nnz = 0;
  unsigned long long npairs = 0;
  HIPCHK(hipMemcpyAsync(&nnz, row_ptr + m, sizeof nnz, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&npairs, pair_total, sizeof npairs, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // The exact decision once the count pass ran.
  if (auto_choice && sparse_s((double)npairs) >= dense_s) return MI_OK;  // dense: *used stays false
  *used = true;
  const size_t cols_bytes = align256((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));
  const size_t acc_bytes = align256((size_t)n * (size_t)n * sizeof(int32_t));
  void* body = nullptr;
  s = scratch(st, 3, 0, cols_bytes + acc_bytes, &body);
  if (s != MI_OK) return s;
  int32_t* cols = (int32_t*)body;
  int32_t* acc = (int32_t*)((char*)body + cols_bytes);
  hipLaunchKernelGGL(k_sp_fill, dim3(blocks), dim3(256), 0, st, p->X, m, n, ldx, vec, row_ptr, cols);
  hipLaunchKernelGGL(k_fill_i32_64, dim3((unsigned)std::min<int64_t>(cdiv64((int64_t)n * n, 256), 65536)), dim3(256), 0,
                     st, acc, 0, (int64_t)n * n);
  hipLaunchKernelGGL(k_sp_pairs, dim3(blocks), dim3(256), 0, st, row_ptr, m, n, cols, acc);
  HIPCHK(hipGetLastError());
  SpEpi E;
  std::memset(&E, 0, sizeof E);
  E.acc = acc;
  E.colsum = colsum;
  E.m = (int32_t)m;
  E.n = n;
  E.out = p->out;
  E.n11_out = p->n11_out;
  E.colsum_out = p->colsum_out;
  E.epi = p->epilogue;
  E.tau = p->fallback_tau > 0.0f ? p->fallback_tau : 1e-3f;
  E.pairs = reinterpret_cast<int32_t*>(p->pairs);
  E.pairs_cap = p->pairs_capacity;
  E.pairs_count = p->pairs_count;
  E.thr = p->pairs_threshold;
  E.ntb = (int32_t)cdiv64(n, 64);
  const int64_t tiles = (int64_t)E.ntb * (E.ntb + 1) / 2;
  if (E.epi == 2)
    hipLaunchKernelGGL(k_sp_epi<2>, dim3((unsigned)tiles), dim3(256), 0, st, E);
  else if (E.epi == 1)
    hipLaunchKernelGGL(k_sp_epi<1>, dim3((unsigned)tiles), dim3(256), 0, st, E);
  else
    hipLaunchKernelGGL(k_sp_epi<0>, dim3((unsigned)tiles), dim3(256), 0, st, E);
  HIPCHK(hipGetLastError());
  return MI_OK;
}

}  // namespace mi
