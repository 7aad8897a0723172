// mi_categorical.hip -- all-pairs MI of categorical variables (codes 0 .. L-1).
//
// The paper computes MI for binary data and names non-binary data as future
// work (Conclusions); Eq. 1 itself is a sum over the joint value set of two
// discrete variables.  This path keeps the paper's matrix form (Section 3.1):
// one Gram product gives the joint counts where both variables are "on", and
// every other count follows from marginals and m.  For categorical data
// "on" means a code >= 1:
//   1. expand: every variable's codes 1 .. L-1 become indicator columns
//      (N = sum (L_j - 1) of them, in variable order), an m x N 0/1 matrix;
//   2. the fused int8 Gram kernel in its counts-only mode: G = Y^T Y (upper
//      triangle) and the indicator column sums;
//   3. reduce: one thread per variable pair (a <= b) rebuilds the L_a x L_b
//      contingency table (cells with a code 0 from the sums and m, as n10,
//      n01, n00 come from n11 in Eq. 6/7), evaluates Eq. 1 over it and
//      writes both triangles of the v x v output.
// With every level count 2 the indicator matrix is X itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "mi.h"
#include "mi_device.hpp"
#include "mi_host.hpp"
#include "mi_internal.hpp"

namespace mi {

namespace {

// A column of the indicator matrix is described by (variable << 9) | code.
constexpr int32_t kCodeBits = 9;
constexpr int32_t kCodeMask = (1 << kCodeBits) - 1;
constexpr int32_t kPadEntry = 256;  // code 256 of variable 0: matches no byte (padding columns)
constexpr int kTile = 32;           // reduce: 32 x 32 variable pairs per block
constexpr int64_t kMaxVars = (int64_t)65535 * kTile;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

__device__ __forceinline__ uint32_t indicator(const uint8_t* __restrict__ xr, int32_t e) {
  return (uint32_t)xr[e >> kCodeBits] == (uint32_t)(e & kCodeMask) ? 1u : 0u;
}

// 0x01 in every byte where a and b agree, 0x00 elsewhere (exact: the adds
// cannot carry across bytes).
__device__ __forceinline__ uint32_t eq_bytes(uint32_t a, uint32_t b) {
  const uint32_t t = a ^ b;
  return ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t | 0x7F7F7F7Fu) >> 7;
}

// 1. Y[r][k] = (X[r][var(k)] == code(k)); padding columns up to the pitch are
//    0.  A thread owns one 16-byte chunk (16 indicator columns) for a run of
//    rows, so its column descriptors are decoded once.  The chunk's
//    variables are consecutive bytes of the row (each variable has at least
//    one indicator column unless it has a single level), at most 16 of them:
//    the thread loads the 32-byte window from its 16-byte-aligned start
//    (two 16-byte loads), picks each output dword's 4 source bytes from two
//    adjacent window dwords with one byte permute, and compares all 4 codes
//    at once.  Chunks whose variables do not fit that window (single-level
//    variables leave gaps) and unaligned layouts load byte by byte.
//    F4: Y holds the FP4 layout of the indicators instead (two columns per
//    byte, a one as the E2M1 code of 1.0), 8 bytes per chunk, for the FP4 Gram.
template <bool F4>
__global__ __launch_bounds__(256) void k_cat_expand(const uint8_t* __restrict__ X, int64_t ldx, int64_t m,
                                                    const int32_t* __restrict__ colmap, int32_t cpr, int32_t cg,
                                                    int64_t rows_per_block, int32_t aligned,
                                                    uint8_t* __restrict__ Y, int64_t ldy) {
  const int tc = threadIdx.x % cg, tr = threadIdx.x / cg, rstep = blockDim.x / cg;
  const int32_t ch = blockIdx.y * cg + tc;
  if (ch >= cpr) return;  // no barriers below
  int32_t ent[16];
  const int4* cm = reinterpret_cast<const int4*>(colmap) + (int64_t)ch * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int4 e = cm[q];
    ent[4 * q] = e.x;
    ent[4 * q + 1] = e.y;
    ent[4 * q + 2] = e.z;
    ent[4 * q + 3] = e.w;
  }
  // Window start (the first column of a chunk is never padding).
  const int32_t base = (ent[0] >> kCodeBits) & ~15;
  int dq[4];
  uint32_t selq[4], codeq[4];
  bool fast = aligned != 0, second = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int32_t f = ent[4 * q];
    dq[q] = (f & kCodeMask) == kPadEntry ? 0 : ((f >> kCodeBits) - base) >> 2;
    if (dq[q] > 6) fast = false;
    uint32_t sel = 0, code = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int32_t e = ent[4 * q + t];
      const bool pad = (e & kCodeMask) == kPadEntry;
      const int32_t off = (e >> kCodeBits) - base;  // byte of the window
      const int32_t b = off - 4 * dq[q];            // byte of the dword pair
      if (!pad && (b < 0 || b > 7)) fast = false;
      if (!pad && off >= 16) second = true;         // then base + 32 <= ldx (aligned layout)
      sel |= (pad ? 0x0Cu : (uint32_t)b) << (8 * t);  // permute selector 0x0C yields 0x00
      code |= (pad ? 0xFFu : (uint32_t)(e & 0xFF)) << (8 * t);
    }
    selq[q] = sel;
    codeq[q] = code;
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < m ? r0 + rows_per_block : m;
  for (int64_t r = r0 + tr; r < r1; r += rstep) {
    uint32_t o[4];
    if (fast) {
      const uint8_t* xw = X + r * ldx + base;
      const uint4 a = *reinterpret_cast<const uint4*>(xw);
      const uint4 b = second ? *reinterpret_cast<const uint4*>(xw + 16) : make_uint4(0, 0, 0, 0);
      const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t lo = w[0], hi = w[1];
#pragma unroll
        for (int k = 1; k < 7; ++k) {
          lo = dq[q] == k ? w[k] : lo;
          hi = dq[q] == k ? w[k + 1] : hi;
        }
        o[q] = eq_bytes(__builtin_amdgcn_perm(hi, lo, selq[q]), codeq[q]);
      }
    } else {
      const uint8_t* xr = X + r * ldx;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        o[q] = indicator(xr, ent[4 * q]) | (indicator(xr, ent[4 * q + 1]) << 8) |
               (indicator(xr, ent[4 * q + 2]) << 16) | (indicator(xr, ent[4 * q + 3]) << 24);
    }
    if constexpr (F4) {
      // Bytes 0/1 of a dword to the 0b0010 codes of four nibbles (16 bits).
      auto nib = [](uint32_t d) {
        return ((d & 1u) << 1) | ((d >> 3) & 0x20u) | ((d >> 7) & 0x200u) | ((d >> 11) & 0x2000u);
      };
      *reinterpret_cast<uint2*>(Y + r * ldy + (int64_t)ch * 8) =
          make_uint2(nib(o[0]) | (nib(o[1]) << 16), nib(o[2]) | (nib(o[3]) << 16));
    } else {
      *reinterpret_cast<uint4*>(Y + r * ldy + (int64_t)ch * 16) = make_uint4(o[0], o[1], o[2], o[3]);
    }
  }
}

// Code check: flag = 1 if some X[r][j] > L_j - 1 = off[j + 1] - off[j].
__global__ __launch_bounds__(256) void k_cat_validate(const uint8_t* __restrict__ X, int64_t ldx, int64_t m,
                                                      int32_t v, const int32_t* __restrict__ off,
                                                      int32_t* __restrict__ flag) {
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x)
    for (int32_t j = threadIdx.x; j < v; j += blockDim.x)
      if ((int32_t)X[r * ldx + j] > off[j + 1] - off[j]) flag[0] = 1;
}

struct CatEpi {
  const int32_t* G;     // N x N indicator counts; entries i <= j are read
  int64_t ldg;          // N
  const int32_t* sums;  // N indicator column sums (marginal counts of codes >= 1)
  const int32_t* off;   // v + 1: variable j's indicator columns are off[j] .. off[j + 1] - 1
  int32_t m, v;
  float* out;           // v x v, or nullptr
  float tau;            // FP64 fallback threshold
  // Sparse output: pairs a < b with MI >= thr, appended at an atomic counter
  // (stored while the count stays below cap).  pairs == nullptr: none.
  int32_t* pairs;       // cap entries of (a, b, MI as FP32 bits)
  int64_t pairs_cap;
  unsigned long long* pairs_count;
  float thr;
};

__device__ __forceinline__ int32_t gram(const CatEpi& E, int p, int q) {
  const int lo = min(p, q), hi = max(p, q);  // within a variable's own block p > q occurs
  return E.G[(int64_t)lo * E.ldg + hi];
}

// FP32 cell term n log2(n m / (r s)) from ra = m / r: one multiply and one
// IEEE division, so a ratio that is exactly 1 in real arithmetic (r = m, or
// a product design) gives exactly 0.  A zero count gives 0 (0 log 0 = 0).
__device__ __forceinline__ float cat_cell32(int n, float ra, int s) {
#pragma clang fp contract(off)
  if (n <= 0) return 0.0f;
  const float fn = (float)n;
  return fn * __log2f((fn * ra) / (float)s);
}

// MI in bits of variables (a, b) from the indicator counts.  The table:
//   x, y >= 1:       n_xy = G[off_a + x - 1][off_b + y - 1]
//   x >= 1, y = 0:   r_x - sum_{y>=1} n_xy
//   x = 0, y >= 1:   s_y - sum_{x>=1} n_xy
//   x = y = 0:       r_0 - (sum_{y>=1} s_y - sum_{x,y>=1} n_xy)
// with r_x, s_y (x, y >= 1) the indicator sums, r_0 = m - sum r_x and
// s_0 = m - sum s_y.  Each table row is summed, then the rows.
template <bool F64>
__device__ float cat_pair(const CatEpi& E, int a, int b) {
#pragma clang fp contract(off)
  const int pa = E.off[a], na = E.off[a + 1] - pa;
  const int pb = E.off[b], nb = E.off[b + 1] - pb;
  const int m = E.m;
  int sr = 0, ss = 0;
  for (int x = 0; x < na; ++x) sr += E.sums[pa + x];
  for (int y = 0; y < nb; ++y) ss += E.sums[pb + y];
  const int r0 = m - sr, s0 = m - ss;
  int tot = 0;
  if constexpr (F64) {
    double acc = 0.0;
    for (int x = 0; x < na; ++x) {
      const int r = E.sums[pa + x];
      int rs = 0;
      double row = 0.0;
      for (int y = 0; y < nb; ++y) {
        const int n = gram(E, pa + x, pb + y);
        rs += n;
        row += cell64(n, r, E.sums[pb + y], m);
      }
      row += cell64(r - rs, r, s0, m);
      acc += row;
      tot += rs;
    }
    double row0 = 0.0;
    for (int y = 0; y < nb; ++y) {
      const int s = E.sums[pb + y];
      int cs = 0;
      for (int x = 0; x < na; ++x) cs += gram(E, pa + x, pb + y);
      row0 += cell64(s - cs, r0, s, m);
    }
    row0 += cell64(r0 - (ss - tot), r0, s0, m);
    return (float)((acc + row0) / (double)m);
  } else {
    const float fm = (float)m;
    float acc = 0.0f;
    for (int x = 0; x < na; ++x) {
      const int r = E.sums[pa + x];
      const float ra = r > 0 ? fm / (float)r : 0.0f;
      int rs = 0;
      float row = 0.0f;
      for (int y = 0; y < nb; ++y) {
        const int n = gram(E, pa + x, pb + y);
        rs += n;
        row += cat_cell32(n, ra, E.sums[pb + y]);
      }
      row += cat_cell32(r - rs, ra, s0);
      acc += row;
      tot += rs;
    }
    const float ra0 = r0 > 0 ? fm / (float)r0 : 0.0f;
    float row0 = 0.0f;
    for (int y = 0; y < nb; ++y) {
      const int s = E.sums[pb + y];
      int cs = 0;
      for (int x = 0; x < na; ++x) cs += gram(E, pa + x, pb + y);
      row0 += cat_cell32(s - cs, ra0, s);
    }
    row0 += cat_cell32(r0 - (ss - tot), ra0, s0);
    return (acc + row0) / fm;
  }
}

// 3. One block per 32 x 32 tile (A, B) of variable pairs with A <= B; thread
//    (ty, tx) evaluates pairs (A*32 + ty + 8q, B*32 + tx), i.e. rows of the
//    tile written with consecutive lanes on consecutive b, then the tile goes
//    through LDS and the mirror rows are written the same way.  Diagonal
//    tiles evaluate a <= b only, so out is bitwise symmetric.
template <int EPI>
__global__ __launch_bounds__(256) void k_cat_reduce(CatEpi E) {
  const int A = blockIdx.y, B = blockIdx.x;
  if (B < A) return;  // uniform: lower-triangle tiles have no work
  __shared__ float tileT[kTile][kTile + 1];
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  const int b = B * kTile + tx;
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int q = 0; q < kTile / 8; ++q) {
    const int al = ty + 8 * q, a = A * kTile + al;
    float val = 0.0f;
    const bool mine = a < E.v && b < E.v && (A != B || a <= b);
    if (mine) {
      if (EPI == 2) {
        val = cat_pair<true>(E, a, b);
      } else {
        val = cat_pair<false>(E, a, b);
        if (EPI == 1 && val < E.tau) val = cat_pair<true>(E, a, b);
      }
      if (E.out) E.out[(int64_t)a * E.v + b] = val;
    }
    tileT[tx][al] = val;
    if (E.pairs) {
      // Sparse output: one atomic per wave, lanes in order.
      const bool keep = mine && a < b && val >= E.thr;
      const unsigned long long mask = __ballot(keep);
      if (mask) {  // uniform
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(E.pairs_count, (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
        if (keep) {
          const unsigned long long idx = base + __popcll(mask & ((1ull << lane) - 1ull));
          if (idx < (unsigned long long)E.pairs_cap) {
            int32_t* e3 = E.pairs + 3 * idx;
            e3[0] = a;
            e3[1] = b;
            e3[2] = __float_as_int(val);
          }
        }
      }
    }
  }
  if (!E.out) return;  // uniform: the whole block leaves, none waits at the barrier below
  __syncthreads();
#pragma unroll 1
  for (int q = 0; q < kTile / 8; ++q) {
    const int bl = ty + 8 * q, bm = B * kTile + bl, am = A * kTile + tx;
    if (am < E.v && bm < E.v && (A != B || am < bm)) E.out[(int64_t)bm * E.v + am] = tileT[bl][tx];
  }
}

// Pinned staging of the host-built tables, one per (device, stream); the
// event marks the end of the last copy out of it.
struct CatStage {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t copied = nullptr;
};
std::mutex g_cat_mu;
std::map<std::pair<int, hipStream_t>, CatStage> g_cat_stage;

mi_status check_cat(const mi_cat_problem* p, int64_t* ldx_out, int64_t* N_out) {
  if (!p) return fail(MI_ERR_INVALID_ARG, "problem is NULL");
  if (p->m <= 0 || p->m > INT32_MAX)
    return fail(MI_ERR_INVALID_ARG, "m must be in 1 .. 2^31-1 (got %lld)", (long long)p->m);
  if (p->v < 0 || p->v > kMaxVars)
    return fail(MI_ERR_INVALID_ARG, "v must be in 0 .. %lld (got %lld)", (long long)kMaxVars, (long long)p->v);
  const int64_t ldx = p->ldx == 0 ? p->v : p->ldx;
  if (ldx < p->v) return fail(MI_ERR_INVALID_ARG, "ldx (%lld) < v (%lld)", (long long)ldx, (long long)p->v);
  if (p->epilogue < 0 || p->epilogue > 2) return fail(MI_ERR_INVALID_ARG, "bad epilogue mode %d", p->epilogue);
  if (p->tile < 0 || p->tile > 2) return fail(MI_ERR_INVALID_ARG, "bad tile id %d", p->tile);
  if (p->splits < 0) return fail(MI_ERR_INVALID_ARG, "splits must be >= 0");
  if (p->gram < MI_GRAM_AUTO || p->gram > MI_GRAM_FP4) return fail(MI_ERR_INVALID_ARG, "bad gram %d", p->gram);
  int64_t N = 0;
  if (p->pairs && (!p->pairs_count || p->pairs_capacity < 0 || !std::isfinite(p->pairs_threshold)))
    return fail(MI_ERR_INVALID_ARG, "pairs needs pairs_count, pairs_capacity >= 0 and a finite threshold");
  if (p->v > 0) {
    if (!p->X || !p->levels) return fail(MI_ERR_INVALID_ARG, "X and levels must be non-NULL when v > 0");
    if (!p->out && !p->pairs) return fail(MI_ERR_INVALID_ARG, "out or the sparse pairs output must be given");
    for (int64_t j = 0; j < p->v; ++j) {
      if (p->levels[j] < 1 || p->levels[j] > 256)
        return fail(MI_ERR_INVALID_ARG, "levels[%lld] = %d is outside 1 .. 256", (long long)j, p->levels[j]);
      N += p->levels[j] - 1;
    }
  }
  if (packed_pitch(N) > ((int64_t)1 << 24))
    return fail(MI_ERR_INVALID_ARG, "%lld indicator columns exceed the supported 2^24", (long long)N);
  *ldx_out = ldx;
  *N_out = N;
  return MI_OK;
}

mi_status run_categorical(const mi_cat_problem* p, hipStream_t st) {
  int64_t ldx = 0, N = 0;
  mi_status s = check_cat(p, &ldx, &N);
  if (s != MI_OK) return s;
  if (p->pairs) HIPCHK(fill_i32(reinterpret_cast<int*>(p->pairs_count), 0, 2, st));  // 64-bit counter
  const int64_t v = p->v, m = p->m;
  if (v == 0) return MI_OK;
  const int64_t ldy = packed_pitch(N);
  // Device tables: off[v + 1] | colmap[ldy] | sums[N] | flag.
  const size_t off_bytes = align256((size_t)(v + 1) * sizeof(int32_t));
  const size_t map_bytes = align256((size_t)std::max<int64_t>(ldy, 1) * sizeof(int32_t));
  const size_t sums_bytes = align256((size_t)std::max<int64_t>(N, 1) * sizeof(int32_t));
  const size_t tab_bytes = off_bytes + map_bytes;
  void* dev = nullptr;
  s = scratch(st, 5, 0, tab_bytes + sums_bytes + 256, &dev);
  if (s != MI_OK) return s;
  char* base = (char*)dev;
  int32_t* d_off = (int32_t*)base;
  int32_t* d_map = (int32_t*)(base + off_bytes);
  int32_t* d_sums = (int32_t*)(base + tab_bytes);
  int32_t* d_flag = (int32_t*)(base + tab_bytes + sums_bytes);
  {
    int devid = 0;
    HIPCHK(hipGetDevice(&devid));
    std::lock_guard<std::mutex> lk(g_cat_mu);
    CatStage& cs = g_cat_stage[std::make_pair(devid, st)];
    if (cs.copied) HIPCHK(hipEventSynchronize(cs.copied));  // the staging is free again
    if (cs.bytes < tab_bytes) {
      if (cs.host) HIPCHK(hipHostFree(cs.host));
      cs.host = nullptr;
      cs.bytes = 0;
      if (hipHostMalloc(&cs.host, tab_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        cs.host = nullptr;
        return fail(MI_ERR_OUT_OF_MEMORY, "pinned staging of %zu bytes failed", tab_bytes);
      }
      cs.bytes = tab_bytes;
    }
    if (!cs.copied) HIPCHK(hipEventCreateWithFlags(&cs.copied, hipEventDisableTiming));
    int32_t* h_off = (int32_t*)cs.host;
    int32_t* h_map = (int32_t*)((char*)cs.host + off_bytes);
    int64_t k = 0;
    for (int64_t j = 0; j < v; ++j) {
      h_off[j] = (int32_t)k;
      for (int32_t c = 1; c < p->levels[j]; ++c) h_map[k++] = (int32_t)((j << kCodeBits) | c);
    }
    h_off[v] = (int32_t)k;
    for (; k < std::max<int64_t>(ldy, 1); ++k) h_map[k] = kPadEntry;
    HIPCHK(hipMemcpyAsync(dev, cs.host, tab_bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(cs.copied, st));
  }
  if (p->validate) {
    HIPCHK(fill_i32(d_flag, 0, 1, st));
    const unsigned vb = (unsigned)std::min<int64_t>(m, 65536);
    hipLaunchKernelGGL(k_cat_validate, dim3(vb), dim3(256), 0, st, p->X, ldx, m, (int32_t)v, d_off, d_flag);
    HIPCHK(hipGetLastError());
    int32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, d_flag, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h) return fail(MI_ERR_BAD_CODE, "X holds a code that is not below its variable's level count");
  }
  int32_t* sums = p->sums_out ? p->sums_out : d_sums;
  const int32_t* G = nullptr;
  if (N > 0) {
    // The indicators go straight to the FP4 layout (half the bytes, no
    // conversion pass) when the FP4 Gram runs.
    const bool f4 = p->gram == MI_GRAM_FP4 || (p->gram == MI_GRAM_AUTO && fp4_preferred(m, N));
    const int64_t ldyg = f4 ? packed_pitch((N + 1) / 2) : ldy;  // pitch of the Gram's input
    void* ybuf = nullptr;
    s = scratch(st, 4, 0, (size_t)m * (size_t)ldyg, &ybuf);
    if (s != MI_OK) return s;
    uint8_t* Y = (uint8_t*)ybuf;
    const int32_t cpr = (int32_t)(ldy / 16);
    int32_t cg = 1;  // chunks per block row: up to 64, the rest of the 256 threads take more rows
    while (cg < 64 && cg < cpr) cg *= 2;
    const int64_t rows_per_block = 256;
    const dim3 eg((unsigned)cdiv(m, rows_per_block), (unsigned)cdiv(cpr, cg));
    const int32_t aligned = ((uintptr_t)p->X % 16 == 0 && ldx % 16 == 0) ? 1 : 0;
    if (f4)
      hipLaunchKernelGGL(k_cat_expand<true>, eg, dim3(256), 0, st, p->X, ldx, m, d_map, cpr, cg, rows_per_block,
                         aligned, Y, ldyg);
    else
      hipLaunchKernelGGL(k_cat_expand<false>, eg, dim3(256), 0, st, p->X, ldx, m, d_map, cpr, cg, rows_per_block,
                         aligned, Y, ldyg);
    HIPCHK(hipGetLastError());
    int32_t* Gw = p->counts_out;
    if (!Gw) {
      void* gb = nullptr;
      s = scratch(st, 6, 0, (size_t)N * (size_t)N * sizeof(int32_t), &gb);
      if (s != MI_OK) return s;
      Gw = (int32_t*)gb;
    }
    mi_problem q;
    mi_problem_init(&q, Y, m, N, nullptr);
    q.ldx = ldyg;
    q.packed = f4 ? MI_INPUT_FP4 : MI_INPUT_BYTES;
    q.n11_out = Gw;
    q.colsum_out = sums;
    q.tile = p->tile;
    q.splits = p->splits;
    s = run_one(&q, st, 0, /*upper_only=*/p->counts_out == nullptr);
    if (s != MI_OK) return s;
    G = Gw;
  }
  CatEpi E;
  std::memset(&E, 0, sizeof E);
  E.G = G;
  E.ldg = N;
  E.sums = sums;
  E.off = d_off;
  E.m = (int32_t)m;
  E.v = (int32_t)v;
  E.out = p->out;
  E.tau = p->fallback_tau > 0.0f ? p->fallback_tau : 1e-3f;
  E.pairs = reinterpret_cast<int32_t*>(p->pairs);
  E.pairs_cap = p->pairs_capacity;
  E.pairs_count = p->pairs_count;
  E.thr = p->pairs_threshold;
  const unsigned T = (unsigned)cdiv(v, kTile);
  const dim3 grid(T, T);
  if (p->epilogue == 2)
    hipLaunchKernelGGL(k_cat_reduce<2>, grid, dim3(256), 0, st, E);
  else if (p->epilogue == 1)
    hipLaunchKernelGGL(k_cat_reduce<1>, grid, dim3(256), 0, st, E);
  else
    hipLaunchKernelGGL(k_cat_reduce<0>, grid, dim3(256), 0, st, E);
  HIPCHK(hipGetLastError());
  return MI_OK;
}

}  // namespace

}  // namespace mi

extern "C" {

void mi_cat_problem_init(mi_cat_problem* p, const uint8_t* X, int64_t m, int64_t v, const int32_t* levels,
                         float* out) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->X = X;
  p->m = m;
  p->v = v;
  p->ldx = v;
  p->levels = levels;
  p->out = out;
  p->epilogue = MI_EPI_FP32;
  p->fallback_tau = 1e-3f;
}

mi_status mi_cat_indicators(const int32_t* levels, int64_t v, int64_t* N) {
  mi::clear_error();
  if (!N || v < 0 || (v > 0 && !levels)) return mi::fail(MI_ERR_INVALID_ARG, "levels and N must be non-NULL, v >= 0");
  int64_t k = 0;
  for (int64_t j = 0; j < v; ++j) {
    if (levels[j] < 1 || levels[j] > 256)
      return mi::fail(MI_ERR_INVALID_ARG, "levels[%lld] = %d is outside 1 .. 256", (long long)j, levels[j]);
    k += levels[j] - 1;
  }
  *N = k;
  return MI_OK;
}

mi_status mi_all_pairs_categorical(const mi_cat_problem* p, void* stream) {
  mi::clear_error();
  return mi::run_categorical(p, (hipStream_t)stream);
}

}  // extern "C"
