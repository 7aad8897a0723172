// mi_layout.hip -- input layouts: validation of 0/1 inputs, the repack of
// layouts the DMA path cannot read, the byte -> FP4 conversion, bit packing,
// and the autotuner's fill pattern.
#include <algorithm>

#include "mi_internal.hpp"

namespace mi {

// flag |= (some byte of X[:, :n] is not 0/1)
__global__ void k_validate(const uint8_t* __restrict__ X, int64_t m, int64_t n, int64_t ldx, int* flag) {
  int bad = 0;
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const uint8_t* r = X + row * ldx;
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) bad |= (r[c] > 1);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// flag |= (some column c < n of X, in the FP4 layout, holds a code other than
// 0 and 0b0010).  Columns 2 b and 2 b + 1 are the low and high nibble of byte
// b; the high nibble of the last byte is ignored when n is odd.
__global__ void k_validate_fp4(const uint8_t* __restrict__ X, int64_t m, int64_t n, int64_t ldx, int* flag) {
  const int64_t nb = (n + 1) / 2;
  int bad = 0;
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const uint8_t* r = X + row * ldx;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
      const uint32_t v = r[b];
      const uint32_t lo = v & 0xFu, hi = (2 * b + 1 < n) ? (v >> 4) : 0u;
      bad |= (lo != 0u && lo != 2u) || (hi != 0u && hi != 2u);
    }
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Byte -> FP4 packing (the layout of the FP4 path): two columns per byte,
// column 2 c in the low nibble of byte c, the E2M1 code of 1.0 (0b0010) for a
// nonzero byte and 0 for a zero.  Four input bytes give 16 output bits: bit 7
// of each nonzero byte (a carry-free nonzero test) moves to bit 1 of
// its nibble.
__device__ __forceinline__ uint32_t fp4_of(uint32_t d) {
  const uint32_t nz = (((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u;
  return ((nz >> 6) & 0x2u) | ((nz >> 10) & 0x20u) | ((nz >> 14) & 0x200u) | ((nz >> 18) & 0x2000u);
}

// Unaligned sources are read as the aligned 16-byte blocks that hold them.
// A block is read only when it holds a byte of X ([xbeg, xend) = first to one
// past the last byte of X): such a block lies in a page that X occupies, so
// no read can fault.  A block wholly outside X, or one not wanted, reads X's
// first block instead: the load has no branch (a wave issues all its loads
// before it waits for any), and the bytes it brings lie past the end of the
// row being read, which every caller zeroes (zero_past) or never stores.
__device__ __forceinline__ uint4 load_block(const uint8_t* blk, const uint8_t* xbeg, const uint8_t* xend,
                                            bool want = true) {
  const bool in = want && blk < xend && blk + 16 > xbeg;
  const uint8_t* first = reinterpret_cast<const uint8_t*>(reinterpret_cast<uintptr_t>(xbeg) & ~(uintptr_t)15);
  return *reinterpret_cast<const uint4*>(in ? blk : first);
}

// Dwords w[0 .. NW - 1] = bytes [src, src + 4 NW) out of b, the NW / 4 + 1
// aligned blocks from src rounded down to 16: dword q = (src mod 16) / 4 of b
// on, shifted by src mod 4 bytes with v_alignbyte.  q is applied by its two
// bits as masked merges of neighbouring dwords; written as selects, the
// compiler turns them into an indexed access, which moves b to scratch.
template <int NW>
__device__ __forceinline__ void align_words(const uint32_t (&b)[NW + 4], uintptr_t src, uint32_t (&w)[NW]) {
  const uint32_t sh = (uint32_t)(src & 3);
  const bool q1 = (src >> 2) & 1, q2 = (src >> 3) & 1;
  uint32_t s1[NW + 3], s2[NW + 1];
  const uint32_t m1 = 0u - (uint32_t)q1, m2 = 0u - (uint32_t)q2;
#pragma unroll
  for (int j = 0; j < NW + 3; ++j) s1[j] = b[j] ^ ((b[j] ^ b[j + 1]) & m1);
#pragma unroll
  for (int j = 0; j < NW + 1; ++j) s2[j] = s1[j] ^ ((s1[j] ^ s1[j + 2]) & m2);  // b[j + q]
#pragma unroll
  for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(s2[k + 1], s2[k], sh);
}

// The NW / 4 + 1 aligned blocks that hold bytes [src, src + 4 NW) (the last
// is not needed, and not read, for a 16-byte-aligned src: align_words then
// takes b[NW] with a zero shift, which drops it; nor are any read where `ok`
// is false).
template <int NW>
__device__ __forceinline__ void fetch_blocks(const uint8_t* src, bool ok, const uint8_t* xbeg, const uint8_t* xend,
                                             uint32_t (&b)[NW + 4]) {
  constexpr int NB = NW / 4 + 1;
  const uint8_t* a = reinterpret_cast<const uint8_t*>(reinterpret_cast<uintptr_t>(src) & ~(uintptr_t)15);
  const bool aligned = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint4 v = load_block(a + 16 * k, xbeg, xend, ok && (k < NB - 1 || !aligned));
    b[4 * k] = v.x;
    b[4 * k + 1] = v.y;
    b[4 * k + 2] = v.z;
    b[4 * k + 3] = v.w;
  }
}

// Dwords w[0 .. NW - 1] = bytes [src, src + 4 NW), read as aligned blocks.
template <int NW>
__device__ __forceinline__ void load_unaligned(const uint8_t* src, const uint8_t* xbeg, const uint8_t* xend,
                                               uint32_t (&w)[NW]) {
  uint32_t b[NW + 4];
  fetch_blocks<NW>(src, true, xbeg, xend, b);
  align_words<NW>(b, reinterpret_cast<uintptr_t>(src), w);
}

// Bytes at or past `avail` (of the 4 NW) set to 0.
template <int NW>
__device__ __forceinline__ void zero_past(int64_t avail, uint32_t (&w)[NW]) {
  if (avail >= 4 * NW) return;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int64_t keep = avail - 4 * k;  // bytes of dword k to keep
    w[k] = keep >= 4 ? w[k] : (keep <= 0 ? 0u : (w[k] & ((1u << (8 * keep)) - 1u)));
  }
}

// FP4 codes of 32 columns from src (avail = columns of the row from src on;
// those past it are 0), as 16 bytes.  A 16-byte-aligned source is two
// 16-byte loads; any other goes through the aligned blocks around it.
__device__ __forceinline__ uint4 fp4_pack32(const uint8_t* src, int64_t avail, const uint8_t* xbeg,
                                            const uint8_t* xend) {
  uint32_t w[8];
  if (avail >= 32 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    const uint4 a = *reinterpret_cast<const uint4*>(src);
    const uint4 b = *reinterpret_cast<const uint4*>(src + 16);
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
  } else {
    load_unaligned<8>(src, xbeg, xend, w);
    zero_past<8>(avail, w);
  }
  return make_uint4(fp4_of(w[0]) | (fp4_of(w[1]) << 16), fp4_of(w[2]) | (fp4_of(w[3]) << 16),
                    fp4_of(w[4]) | (fp4_of(w[5]) << 16), fp4_of(w[6]) | (fp4_of(w[7]) << 16));
}

// Output chunk of a repack or conversion from its source blocks: the 16
// bytes [16 c, 16 c + 16) of X's row (a repack) or the FP4 codes of its
// columns [32 c, 32 c + 32) (a conversion, FP4), avail = source bytes of the
// row from the chunk's start on (zeros past it).
template <bool FP4>
__device__ __forceinline__ uint4 chunk_out(const uint32_t (&b)[FP4 ? 12 : 8], uintptr_t src, int64_t avail) {
  if constexpr (FP4) {
    uint32_t w[8];
    align_words<8>(b, src, w);
    zero_past<8>(avail, w);
    return make_uint4(fp4_of(w[0]) | (fp4_of(w[1]) << 16), fp4_of(w[2]) | (fp4_of(w[3]) << 16),
                      fp4_of(w[4]) | (fp4_of(w[5]) << 16), fp4_of(w[6]) | (fp4_of(w[7]) << 16));
  } else {
    uint32_t w[4];
    align_words<4>(b, src, w);
    zero_past<4>(avail, w);
    return make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Rows per wave of a layout: one wave per row when a row has 64 or more
// 16-byte chunks, else 64 / chunks rows side by side (so narrow rows keep
// the lanes busy).
__host__ __device__ inline int64_t rows_per_wave(int64_t ldy) {
  const int64_t cpr = ldy >> 4;
  return cpr >= 64 ? 1 : 64 / (cpr > 0 ? cpr : 1);
}

// Work items of a layout, one per wave at a time: a group of rows_per_wave
// rows (narrow rows), or one row (wide rows, 64 chunks per step).
__host__ __device__ inline int64_t repack_items(int64_t m, int64_t ldy) {
  const int64_t rpw = rows_per_wave(ldy);
  return (m + rpw - 1) / rpw;
}

constexpr int kRepackUnroll = 4;  // items a wave loads before it converts any

// Wave w0, w0 + wstride, ... of a layout: its items, kRepackUnroll at a time
// (every source block of a step is loaded before the first is used, so a
// wave keeps that many reads in flight), consecutive lanes on consecutive
// chunks.  Wide rows take ceil(chunks / 64) such steps.
template <bool FP4>
__device__ __forceinline__ void stage_items(const RepackDesc& d, int64_t w0, int64_t wstride, int lane) {
  constexpr int U = kRepackUnroll, NW = FP4 ? 8 : 4, CB = FP4 ? 32 : 16;  // CB: source bytes per chunk
  const uint8_t* xend = d.X + (d.m - 1) * d.ldx + d.n;  // one past the last byte of X that is read
  const int64_t cpr = d.ldy >> 4;
  const bool wide = cpr >= 64;
  const int64_t items = repack_items(d.m, d.ldy);
  const int rpw = (int)rows_per_wave(d.ldy);
  const int lr = wide ? 0 : lane / (int)cpr;              // row of the group (narrow rows)
  const int64_t cl = wide ? lane : lane - lr * cpr;       // chunk of the lane
  const int64_t steps = wide ? (cpr + 63) >> 6 : 1;
  for (int64_t i0 = w0; i0 < items; i0 += U * wstride) {
    for (int64_t st = 0; st < steps; ++st) {
      uint32_t b[U][NW + 4];
      int64_t r[U];
      bool ok[U];
      const int64_t c = cl + 64 * st;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + u * wstride;
        r[u] = i * rpw + lr;
        ok[u] = i < items && lr < rpw && r[u] < d.m && c < cpr;
        fetch_blocks<NW>(d.X + r[u] * d.ldx + CB * c, ok[u], d.X, xend, b[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint4 o = chunk_out<FP4>(b[u], reinterpret_cast<uintptr_t>(d.X + r[u] * d.ldx + CB * c), d.n - CB * c);
        // Streaming store: the Gram reads the result after the whole pass.
        if (ok[u]) __builtin_nontemporal_store(v4u{o.x, o.y, o.z, o.w}, reinterpret_cast<v4u*>(d.Y + r[u] * d.ldy + 16 * c));
      }
    }
  }
}

__device__ __forceinline__ void stage_layout(const RepackDesc& d, int64_t w0, int64_t wstride, int lane) {
  if (d.fp4) stage_items<true>(d, w0, wstride, lane);
  else stage_items<false>(d, w0, wstride, lane);
}

// Repack of a layout the DMA path cannot read (base or pitch not a multiple
// of 16 bytes) into a 16-byte pitch: 4 waves per block, the grid strides
// over the items.
__global__ __launch_bounds__(256) void k_repack(RepackDesc d) {
  stage_layout(d, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), (int64_t)gridDim.x * 4, threadIdx.x & 63);
}

// All repacks and conversions of a batch in one launch: block b belongs to
// the dataset whose block range [first_block, first_block + blocks) holds it.
__global__ __launch_bounds__(256) void k_repack_batch(const RepackDesc* __restrict__ descs, int count) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = count - 1;
  while (lo < hi) {  // uniform: every lane searches the same block index
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].first_block <= b) lo = mid;
    else hi = mid - 1;
  }
  const RepackDesc d = descs[lo];
  stage_layout(d, (b - d.first_block) * 4 + (threadIdx.x >> 6), d.blocks * 4, threadIdx.x & 63);
}

// Byte -> bit packing (the layout of a packed problem).  0x01 in each
// nonzero byte of d, then one multiply gathers byte i into bit 24 + i (the
// shifted copies of the four bytes land on distinct bits, so nothing carries).
__device__ __forceinline__ uint32_t nibble_of(uint32_t d) {
  const uint32_t nz = ((((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u) >> 7;
  return ((nz * 0x01020408u) >> 24) & 0xFu;
}

// One thread per (row, 64-column group): 8 packed bytes.  Blocks cover 4 rows
// x 64 groups.  Groups that end past n, and unaligned layouts, go byte by byte.
__global__ __launch_bounds__(256) void k_pack_bits(const uint8_t* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                                   uint8_t* __restrict__ Xp, int64_t ldp, int32_t vec_in,
                                                   int32_t vec_out) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int64_t g = (int64_t)blockIdx.y * 64 + threadIdx.x % 64;
  const int64_t nbytes = (n + 7) / 8;  // packed bytes of a row that hold columns
  if (r >= m || 8 * g >= nbytes) return;
  const uint8_t* xr = X + r * ldx + 64 * g;
  uint8_t* pr = Xp + r * ldp + 8 * g;
  if (vec_in && 64 * g + 64 <= n) {
    uint32_t o[2] = {0u, 0u};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const uint4 v = *reinterpret_cast<const uint4*>(xr + 16 * h);
      const uint32_t b0 = nibble_of(v.x) | (nibble_of(v.y) << 4);  // packed byte 2h
      const uint32_t b1 = nibble_of(v.z) | (nibble_of(v.w) << 4);  // packed byte 2h + 1
      o[h >> 1] |= (b0 | (b1 << 8)) << (16 * (h & 1));
    }
    if (vec_out) {
      *reinterpret_cast<uint2*>(pr) = make_uint2(o[0], o[1]);
    } else {
#pragma unroll
      for (int b = 0; b < 8; ++b) pr[b] = (uint8_t)(o[b >> 2] >> (8 * (b & 3)));
    }
    return;
  }
  const int64_t cols = n - 64 * g < 64 ? n - 64 * g : 64;
  const int64_t bytes = nbytes - 8 * g < 8 ? nbytes - 8 * g : 8;
  for (int64_t b = 0; b < bytes; ++b) {
    uint32_t v = 0;
    for (int k = 0; k < 8; ++k)
      if (8 * b + k < cols && xr[8 * b + k] != 0) v |= 1u << k;
    pr[b] = (uint8_t)v;
  }
}

hipError_t launch_pack_bits(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xp, int64_t ldp,
                            hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t groups = (n + 63) / 64;
  const int32_t vec_in = ((uintptr_t)X % 16 == 0 && ldx % 16 == 0) ? 1 : 0;
  const int32_t vec_out = ((uintptr_t)Xp % 8 == 0 && ldp % 8 == 0) ? 1 : 0;
  const dim3 grid((unsigned)((m + 3) / 4), (unsigned)((groups + 63) / 64));
  hipLaunchKernelGGL(k_pack_bits, grid, dim3(256), 0, st, X, ldx, m, n, Xp, ldp, vec_in, vec_out);
  return hipGetLastError();
}

// One thread per (row, 32-column group): 16 packed bytes (fp4_pack32).
// Blocks cover 4 rows x 64 groups.  Bytes of the destination past
// ceil(n / 2) are not written.
__global__ __launch_bounds__(256) void k_pack_fp4(const uint8_t* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                                  uint8_t* __restrict__ Xq, int64_t ldq, int32_t vec_out) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int64_t g = (int64_t)blockIdx.y * 64 + threadIdx.x % 64;
  const int64_t nbytes = (n + 1) / 2;  // packed bytes of a row that hold columns
  if (r >= m || 16 * g >= nbytes) return;
  const uint4 o = fp4_pack32(X + r * ldx + 32 * g, n - 32 * g, X, X + (m - 1) * ldx + n);
  uint8_t* qr = Xq + r * ldq + 16 * g;
  if (vec_out && 16 * g + 16 <= nbytes) {
    // A streaming store: the converted matrix is read back by the Gram long
    // after this pass (whole rows later), so keeping it out of the caches
    // loses nothing; measured 1.11 against 1.21 ms at 1,000,000 x 4,096.
    __builtin_nontemporal_store(v4u{o.x, o.y, o.z, o.w}, reinterpret_cast<v4u*>(qr));
  } else {
    const uint32_t w[4] = {o.x, o.y, o.z, o.w};
    const int64_t bytes = nbytes - 16 * g < 16 ? nbytes - 16 * g : 16;
    for (int64_t k = 0; k < bytes; ++k) qr[k] = (uint8_t)(w[k >> 2] >> (8 * (k & 3)));
  }
}

hipError_t launch_pack_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xq, int64_t ldq,
                           hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t groups = (n + 31) / 32;
  const int32_t vec_out = ((uintptr_t)Xq % 16 == 0 && ldq % 16 == 0) ? 1 : 0;
  const dim3 grid((unsigned)((m + 3) / 4), (unsigned)((groups + 63) / 64));
  hipLaunchKernelGGL(k_pack_fp4, grid, dim3(256), 0, st, X, ldx, m, n, Xq, ldq, vec_out);
  return hipGetLastError();
}

// Tuner input: a 0/1 pattern of about 1/8 density from a 32-bit integer
// hash of the entry's position (bytes 1, or the FP4 code 0b0010 per nibble);
// bytes of a row past `bytes` are 0.
__global__ __launch_bounds__(256) void k_fill_pattern(uint8_t* __restrict__ X, int64_t m, int64_t ld, int64_t bytes,
                                                      int32_t fp4) {
  const int64_t total = m * ld;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int64_t row = q / ld, c = q - row * ld;
    uint32_t v = 0;
    if (c < bytes) {
      uint32_t h = (uint32_t)(row * 0x9E3779B1u) ^ (uint32_t)(c * 0x85EBCA77u);
      h ^= h >> 15;
      h *= 0x2C1B3C6Du;
      h ^= h >> 12;
      h *= 0x297A2D39u;
      h ^= h >> 15;
      v = fp4 ? ((((h & 7u) == 0u) ? 0x02u : 0u) | ((((h >> 3) & 7u) == 0u) ? 0x20u : 0u)) : ((h & 7u) == 0u ? 1u : 0u);
    }
    X[q] = (uint8_t)v;
  }
}

hipError_t launch_fill_pattern(uint8_t* X, int64_t m, int64_t ld, int64_t bytes, bool fp4, hipStream_t st) {
  const int64_t chunks = (m * ld + 255) / 256;
  const int64_t blocks = chunks < 65536 ? (chunks > 0 ? chunks : 1) : 65536;
  hipLaunchKernelGGL(k_fill_pattern, dim3((unsigned)blocks), dim3(256), 0, st, X, m, ld, bytes, fp4 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_validate(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st) {
  if (hipError_t e = fill_i32(flag, 0, 1, st); e != hipSuccess) return e;
  const int64_t blocks = m < 4096 ? m : 4096;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, flag);
  return hipGetLastError();
}

hipError_t launch_validate_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st) {
  if (hipError_t e = fill_i32(flag, 0, 1, st); e != hipSuccess) return e;
  const int64_t blocks = m < 4096 ? m : 4096;
  hipLaunchKernelGGL(k_validate_fp4, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, flag);
  return hipGetLastError();
}

// Blocks for one layout: four waves per block, kRepackUnroll items per wave
// (repack_items), at most 65536 blocks (more items loop).
int64_t repack_blocks(int64_t m, int64_t ldy) {
  const int64_t b = (repack_items(m, ldy) + 4 * kRepackUnroll - 1) / (4 * kRepackUnroll);
  return b < 65536 ? (b > 0 ? b : 1) : 65536;
}

hipError_t launch_repack(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Y, int64_t ldy,
                         hipStream_t st) {
  const int64_t blocks = repack_blocks(m, ldy);
  RepackDesc d{X, ldx, Y, ldy, m, n, 0, blocks};
  hipLaunchKernelGGL(k_repack, dim3((unsigned)blocks), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_repack_batch(const RepackDesc* descs, int count, int64_t blocks, hipStream_t st) {
  if (count <= 0 || blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_repack_batch, dim3((unsigned)blocks), dim3(256), 0, st, descs, count);
  return hipGetLastError();
}

}  // namespace mi
