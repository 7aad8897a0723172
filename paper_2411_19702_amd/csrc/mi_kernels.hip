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
// no read can fault; its bytes outside X are never used.  Blocks wholly
// outside X give zeros.
__device__ __forceinline__ uint4 load_block(const uint8_t* blk, const uint8_t* xbeg, const uint8_t* xend) {
  if (blk < xend && blk + 16 > xbeg) return *reinterpret_cast<const uint4*>(blk);
  return make_uint4(0u, 0u, 0u, 0u);
}

// Dwords w[0 .. NW - 1] = bytes [src, src + 4 NW) from the NW / 4 + 1 aligned
// blocks that hold them, shifted into place with v_alignbyte.  The dword
// offset q = (src mod 16) / 4 selects registers with constant indices.
template <int NW>
__device__ __forceinline__ void load_unaligned(const uint8_t* src, const uint8_t* xbeg, const uint8_t* xend,
                                               uint32_t (&w)[NW]) {
  constexpr int NB = NW / 4 + 1;
  const uint8_t* a = reinterpret_cast<const uint8_t*>(reinterpret_cast<uintptr_t>(src) & ~(uintptr_t)15);
  uint32_t b[4 * NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint4 v = load_block(a + 16 * k, xbeg, xend);
    b[4 * k] = v.x;
    b[4 * k + 1] = v.y;
    b[4 * k + 2] = v.z;
    b[4 * k + 3] = v.w;
  }
  const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(src) & 3);
  const uint32_t q = (uint32_t)(reinterpret_cast<uintptr_t>(src) >> 2) & 3u;
  if (q == 0) {
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(b[k + 1], b[k], sh);
  } else if (q == 1) {
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(b[k + 2], b[k + 1], sh);
  } else if (q == 2) {
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(b[k + 3], b[k + 2], sh);
  } else {
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = __builtin_amdgcn_alignbyte(b[k + 4], b[k + 3], sh);
  }
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

// Chunk c of row r of a repack or conversion (d.fp4): Y's row r gets at
// 16 c the bytes [16 c, 16 c + 16) of X's row (a repack) or the FP4 codes of
// its columns [32 c, 32 c + 32) (a conversion); zeros past n.
__device__ __forceinline__ void stage_chunk(const RepackDesc& d, int64_t r, int64_t c) {
  const uint8_t* xend = d.X + (d.m - 1) * d.ldx + d.n;  // one past the last byte of X that is read
  const uint8_t* row = d.X + r * d.ldx;
  uint4 o;
  if (d.fp4) {
    o = fp4_pack32(row + 32 * c, d.n - 32 * c, d.X, xend);
  } else {
    uint32_t w[4];
    load_unaligned<4>(row + 16 * c, d.X, xend, w);
    zero_past<4>(d.n - 16 * c, w);
    o = make_uint4(w[0], w[1], w[2], w[3]);
  }
  *reinterpret_cast<uint4*>(d.Y + r * d.ldy + 16 * c) = o;
}

// Rows per wave of a layout: one wave per row when a row has 64 or more
// 16-byte chunks, else 64 / chunks rows side by side (so narrow rows keep
// the lanes busy).
__host__ __device__ inline int64_t rows_per_wave(int64_t ldy) {
  const int64_t cpr = ldy >> 4;
  return cpr >= 64 ? 1 : 64 / (cpr > 0 ? cpr : 1);
}

// Wave w0, w0 + wstride, ... of a layout: its group of rows_per_wave rows,
// consecutive lanes on consecutive chunks.
__device__ __forceinline__ void stage_rows(const RepackDesc& d, int64_t w0, int64_t wstride, int lane) {
  const int64_t cpr = d.ldy >> 4;
  if (cpr >= 64) {
    for (int64_t r = w0; r < d.m; r += wstride)
      for (int64_t c = lane; c < cpr; c += 64) stage_chunk(d, r, c);
    return;
  }
  const int rpw = (int)rows_per_wave(d.ldy);
  const int lr = lane / (int)cpr, c = lane - lr * (int)cpr;
  for (int64_t g = w0; g * rpw < d.m; g += wstride) {
    const int64_t r = g * rpw + lr;
    if (lr < rpw && r < d.m) stage_chunk(d, r, c);
  }
}

// Repack of a layout the DMA path cannot read (base or pitch not a multiple
// of 16 bytes) into a 16-byte pitch: 4 waves per block, the grid strides
// over the row groups.
__global__ __launch_bounds__(256) void k_repack(RepackDesc d) {
  stage_rows(d, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), (int64_t)gridDim.x * 4, threadIdx.x & 63);
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
  stage_rows(d, (b - d.first_block) * 4 + (threadIdx.x >> 6), d.blocks * 4, threadIdx.x & 63);
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
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flag, 0, 1);
  const int64_t blocks = m < 4096 ? m : 4096;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, flag);
  return hipGetLastError();
}

hipError_t launch_validate_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, flag, 0, 1);
  const int64_t blocks = m < 4096 ? m : 4096;
  hipLaunchKernelGGL(k_validate_fp4, dim3((unsigned)blocks), dim3(256), 0, st, X, m, n, ldx, flag);
  return hipGetLastError();
}

// Blocks for one layout: four waves per block, one group of rows per wave
// (rows_per_wave), at most 65536 blocks (more groups loop).
int64_t repack_blocks(int64_t m, int64_t ldy) {
  const int64_t rpw = rows_per_wave(ldy);
  const int64_t b = ((m + rpw - 1) / rpw + 3) / 4;
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
