// mi_device.hpp -- device side of the fused all-pairs binary MI kernel (gfx950).
//
// One work unit = (dataset, output tile (I, J) with I <= J, K-split s).  A unit
//   1. streams its rows [k0, k1) of the two column panels X[:, I] and X[:, J]
//      from HBM through LDS (double-buffered, one barrier per 64-row stage),
//      transposing 4x4 byte blocks in registers so that each column's samples
//      are contiguous, as the int8 matrix-core operands need;
//   2. accumulates the 1-1 counts n11 = X_I^T X_J (the Gram product of
//      Section 2 step 2 / Section 3, the only matrix product of the method)
//      with v_mfma_i32_16x16x64_i8, exact in int32;
//   3. accumulates the column sums c_I, c_J of its rows with v_dot4_u32_u8 on
//      the already-transposed bytes (Section 2 step 3 / Section 3.1 "Term 2");
//   4. with several K-splits, adds its partial counts into a per-tile int32
//      workspace; the last unit to arrive at a tile reads the totals back,
//      clears the workspace, and alone runs the epilogue;
//   5. epilogue: derives n10, n01, n00 from n11, c and m (Section 3.1,
//      Eq. 6/7), evaluates MI (Eq. 2/3) per element in FP32 (FP64 on demand)
//      and writes the tile and its mirror.
//
// Only upper-triangular tiles exist; the mirror write fills the lower one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mi {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int KT = 64;          // rows (samples) per LDS stage = one MFMA K step
constexpr int NTHREADS = 256;   // 4 waves
constexpr int HALF = NTHREADS / 2;

// Everything a unit needs to know about its dataset.
struct ProbDev {
  const uint8_t* X;
  int64_t ldx;
  int32_t m, n;
  float* out;
  int32_t* n11_out;     // optional
  int32_t* colsum_out;  // optional
  int32_t* ws_n11;      // splits > 1: ntiles * BT * BT int32, all zero between calls
  int32_t* ws_col;      // splits > 1: ntiles * 2 * BT int32
  int32_t* counters;    // splits > 1: ntiles int32
  int32_t ntp;          // panels = ceil(n / BT)
  int32_t ntiles;       // ntp (ntp + 1) / 2
  int32_t splits;
  int32_t kchunk;       // rows per split, a multiple of KT
  int32_t epi;          // mi_epilogue
  float tau;
  int32_t aligned;      // X 16-byte aligned and ldx % 16 == 0
};

// ---------------------------------------------------------------------------
// Epilogue arithmetic: MI of one pair from (m, c_i, c_j, n11).
// Written so that swapping (i, j) gives bitwise the same result: every
// product is a single commutative IEEE multiply and the four cell terms are
// summed as (t11 + t00) + (t10 + t01).  Contraction into FMAs is disabled so
// the compiler cannot break that symmetry.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float cell32(int nxy, int nx, int ny, float fm) {
#pragma clang fp contract(off)
  if (nxy <= 0) return 0.0f;                      // 0 log 0 = 0
  float fn = (float)nxy;
  float num = fn * fm;                            // n_xy * m
  float den = (float)nx * (float)ny;              // n_x * n_y
  return fn * __log2f(__fdividef(num, den));
}

__device__ __forceinline__ double cell64(int nxy, int nx, int ny, int m) {
#pragma clang fp contract(off)
  if (nxy <= 0) return 0.0;
  double num = (double)((int64_t)nxy * (int64_t)m);   // exact below 2^53
  double den = (double)((int64_t)nx * (int64_t)ny);
  return (double)nxy * log2(num / den);
}

__device__ __forceinline__ float mi_value64(int m, int ci, int cj, int n11) {
#pragma clang fp contract(off)
  const int n10 = ci - n11, n01 = cj - n11, ni0 = m - ci, nj0 = m - cj, n00 = ni0 - n01;
  const double d11 = cell64(n11, ci, cj, m);
  const double d00 = cell64(n00, ni0, nj0, m);
  const double d10 = cell64(n10, ci, nj0, m);
  const double d01 = cell64(n01, ni0, cj, m);
  return (float)(((d11 + d00) + (d10 + d01)) / (double)m);
}

__device__ __forceinline__ float mi_value(int m, int ci, int cj, int n11, int epi, float tau) {
#pragma clang fp contract(off)
  if (epi == 2) return mi_value64(m, ci, cj, n11);
  const int n10 = ci - n11;          // X_i = 1, X_j = 0
  const int n01 = cj - n11;          // X_i = 0, X_j = 1
  const int ni0 = m - ci;            // marginal count of X_i = 0
  const int nj0 = m - cj;            // marginal count of X_j = 0
  const int n00 = ni0 - n01;         // = m - c_i - c_j + n11, without overflow
  const float fm = (float)m;
  const float t11 = cell32(n11, ci, cj, fm);
  const float t00 = cell32(n00, ni0, nj0, fm);
  const float t10 = cell32(n10, ci, nj0, fm);
  const float t01 = cell32(n01, ni0, cj, fm);
  const float v = ((t11 + t00) + (t10 + t01)) / fm;
  if (epi == 1 && v < tau) return mi_value64(m, ci, cj, n11);
  return v;
}

// ---------------------------------------------------------------------------
// LDS layout of one staged panel: BT columns x 64 samples, no padding.  Four
// consecutive columns share one 256-byte bank row; inside it the 16 slots of
// 16 bytes (4 columns x 4 sample chunks g) are permuted by
//     slot = 4 * (t ^ g ^ 2b) + (q ^ g),   t = col & 3,
//     q = ((col >> 2) ^ (col >> 4)) & 3,   b = (col >> 6) & 1,
// which makes both access patterns conflict-free on the 64 banks:
//   * operand reads: 16 lanes read 16 consecutive columns at one chunk g;
//   * staging writes: 64 lanes write one dword each for 8 column chunks x
//     8 row quads (the mapping used by stage_store below).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lds_off(int col, int g) {
  const int t = col & 3;
  const int q = ((col >> 2) ^ (col >> 4)) & 3;
  const int b = (col >> 6) & 1;
  const int slot = 4 * (t ^ g ^ (b << 1)) + (q ^ g);
  return ((col >> 2) << 8) + (slot << 4);
}

// Staging work split: a panel of BT columns x 64 rows is 16-column x 4-row
// chunks; chunk q of a panel goes to thread (q mod HALF) of that panel's half
// of the workgroup.  Within a block of 128 chunks: cc = q % 8 selects 16
// columns, rq = (q / 8) % 16 selects 4 rows; block q / 128 adds 128 columns.
template <int BT>
struct Staging {
  static constexpr int CHUNKS = BT / 16 * (KT / 4);
  static constexpr int G = CHUNKS / HALF;       // chunks per thread
  static_assert(G >= 1 && CHUNKS % HALF == 0, "tile / thread mismatch");
  __device__ static __forceinline__ int chunk_col(int q) { return ((q & 7) + 8 * (q >> 7)) * 16; }
  __device__ static __forceinline__ int chunk_row(int q) { return ((q >> 3) & 15) * 4; }
};

__device__ __forceinline__ uint32_t keep_mask(int valid, int w) {
  // bytes of dword w (columns 4w..4w+3 of a 16-byte chunk) with index < valid
  const int k = min(max(valid - 4 * w, 0), 4);
  return (uint32_t)((1ull << (8 * k)) - 1ull);
}

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Per-thread staging context, fixed for a whole unit.
template <int BT>
struct StageCtx {
  int voff[Staging<BT>::G];     // byte offset of the chunk's first row inside a stage
  int col[Staging<BT>::G];      // first matrix column of the chunk
  int row[Staging<BT>::G];      // first row of the chunk inside a stage (0..60)
  uint32_t cm[Staging<BT>::G][4];  // keep-masks for columns >= n
};

template <int BT>
__device__ __forceinline__ void stage_ctx(StageCtx<BT>& c, const ProbDev& P, int colbase, int p) {
#pragma unroll
  for (int gi = 0; gi < Staging<BT>::G; ++gi) {
    const int q = p + gi * HALF;
    c.col[gi] = colbase + Staging<BT>::chunk_col(q);
    c.row[gi] = Staging<BT>::chunk_row(q);
    const int valid = min(P.n - c.col[gi], 16);
    // A chunk entirely right of column n reads at an offset past every stage's
    // buffer range, which the hardware returns as zeros.
    c.voff[gi] = valid > 0 ? c.row[gi] * (int)P.ldx + c.col[gi] : KT * (int)P.ldx;
#pragma unroll
    for (int w = 0; w < 4; ++w) c.cm[gi][w] = keep_mask(valid, w);
  }
}

// Global -> registers for the stage starting at row ks (rows >= kend read as 0).
// Aligned layout: raw buffer loads whose range ends at row min(kend, ks + KT),
// so out-of-range rows come back as zeros without any branch; the loads of a
// stage issue back to back and only the consumer waits for them.
template <int BT, bool ALIGNED>
__device__ __forceinline__ void stage_load(uint4 (&r)[Staging<BT>::G][4], const ProbDev& P, const StageCtx<BT>& c,
                                           int ks, int kend) {
  if (ALIGNED) {
    // ks and kend are uniform across the workgroup; readfirstlane keeps the
    // descriptor in scalar registers (no per-lane waterfall around the loads).
    const int rows = __builtin_amdgcn_readfirstlane(max(0, min(kend - ks, KT)));
    const int ld = __builtin_amdgcn_readfirstlane((int)P.ldx);
    const uint64_t base = (uint64_t)(P.X + (int64_t)min(ks, P.m - 1) * P.ldx);
    const uint32_t blo = __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t bhi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
    __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(((uint64_t)bhi << 32) | blo), 0, rows * ld, 0x00020000);
#pragma unroll
    for (int gi = 0; gi < Staging<BT>::G; ++gi)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        // the whole offset goes in the vector operand, which the range check covers
        const v4u v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, c.voff[gi] + rr * ld, 0, 0);
        r[gi][rr] = make_uint4(v.x, v.y, v.z, v.w);
      }
  } else {
#pragma unroll
    for (int gi = 0; gi < Staging<BT>::G; ++gi) {
      const int valid = min(P.n - c.col[gi], 16);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = ks + c.row[gi] + rr;
        uint32_t w4[4] = {0u, 0u, 0u, 0u};
        if (row < kend && valid > 0) {
          const uint8_t* src = P.X + (int64_t)row * P.ldx + c.col[gi];
#pragma unroll
          for (int b = 0; b < 16; ++b)
            if (b < valid) w4[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
        }
        r[gi][rr] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
      }
    }
  }
}

__device__ __forceinline__ uint32_t u4get(const uint4& v, int w) {
  return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// Registers -> LDS for one stage of one panel: mask columns >= n, 4x4 byte
// transposes so that a dword holds 4 consecutive samples of one column, and
// column-sum updates.
template <int BT>
__device__ __forceinline__ void stage_store(uint8_t* sbuf, const uint4 (&r)[Staging<BT>::G][4], const StageCtx<BT>& c,
                                            uint32_t (&csum)[Staging<BT>::G][16]) {
#pragma unroll
  for (int gi = 0; gi < Staging<BT>::G; ++gi) {
    const int c0 = c.col[gi] & (BT - 1);          // column inside the panel
    const int rq = c.row[gi] >> 2;                // row quad 0..15
    const int g = rq >> 2, d = rq & 3;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t m = c.cm[gi][w];
      const uint32_t a = u4get(r[gi][0], w) & m, b = u4get(r[gi][1], w) & m;
      const uint32_t cc = u4get(r[gi][2], w) & m, e = u4get(r[gi][3], w) & m;
      const uint32_t x0 = __builtin_amdgcn_perm(b, a, 0x05010400u);  // a0 b0 a1 b1
      const uint32_t x1 = __builtin_amdgcn_perm(b, a, 0x07030602u);  // a2 b2 a3 b3
      const uint32_t y0 = __builtin_amdgcn_perm(e, cc, 0x05010400u); // c0 e0 c1 e1
      const uint32_t y1 = __builtin_amdgcn_perm(e, cc, 0x07030602u); // c2 e2 c3 e3
      uint32_t o[4];
      o[0] = __builtin_amdgcn_perm(y0, x0, 0x05040100u);  // column 4w+0, rows 0..3
      o[1] = __builtin_amdgcn_perm(y0, x0, 0x07060302u);  // column 4w+1
      o[2] = __builtin_amdgcn_perm(y1, x1, 0x05040100u);  // column 4w+2
      o[3] = __builtin_amdgcn_perm(y1, x1, 0x07060302u);  // column 4w+3
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = c0 + 4 * w + t;
        *reinterpret_cast<uint32_t*>(sbuf + lds_off(col, g) + 4 * d) = o[t];
        csum[gi][4 * w + t] = __builtin_amdgcn_udot4(o[t], 0x01010101u, csum[gi][4 * w + t], false);
      }
    }
  }
}

// Tile geometry for the 4-wave workgroup: waves in a 2 x 2 grid, each wave
// owns a (BT/2) x (BT/2) block made of 16 x 16 MFMA fragments.
template <int BT>
struct TileGeom {
  static constexpr int WT = BT / 2;
  static constexpr int F = WT / 16;          // fragments per side of a wave block
  static constexpr int PANEL_BYTES = BT * KT;
  static constexpr int STAGE_BYTES = 2 * PANEL_BYTES;  // panel I then panel J
  static constexpr int LDS_BYTES = 2 * STAGE_BYTES + 2 * BT * 4 + 16;
  static_assert(4 * 2 * 16 * WT * 4 <= 2 * STAGE_BYTES, "epilogue strips must fit in the stage buffers");
};

// Decode upper-triangular tile t (row-major over I <= J) into (I, J).
__device__ __forceinline__ void tile_ij(int t, int ntp, int& I, int& J) {
  int i = 0;
  int rem = t;
  while (rem >= ntp - i) { rem -= ntp - i; ++i; }
  I = i;
  J = i + rem;
}

// One work unit.  smem must hold TileGeom<BT>::LDS_BYTES bytes, 16-aligned.
template <int BT, bool ALIGNED>
__device__ __forceinline__ void run_unit(const ProbDev& P, int t, int s, uint8_t* smem) {
  using TG = TileGeom<BT>;
  using ST = Staging<BT>;
  constexpr int F = TG::F;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  int I, J;
  tile_ij(t, P.ntp, I, J);
  const bool diag = (I == J);
  const int k0 = s * P.kchunk;
  const int k1 = min(P.m, k0 + P.kchunk);
  const int nsteps = (k1 > k0) ? (k1 - k0 + KT - 1) / KT : 0;

  int32_t* sColA = reinterpret_cast<int32_t*>(smem + 2 * TG::STAGE_BYTES);
  int32_t* sColB = sColA + BT;
  int32_t* sFlag = sColB + BT;

  // Staging role: threads [0, HALF) stage panel I, [HALF, 2 HALF) panel J (on a
  // diagonal tile both halves stage the same panel, which keeps the pipeline
  // free of divergent branches).
  const int half = tid / HALF;
  const int p = tid % HALF;
  const int colbase = (half == 0 ? I : J) * BT;
  const int soff = half * TG::PANEL_BYTES;
  StageCtx<BT> ctx;
  stage_ctx<BT>(ctx, P, colbase, p);

  for (int c = tid; c < 2 * BT; c += NTHREADS) sColA[c] = 0;

  v4i acc[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  uint32_t csum[ST::G][16];
#pragma unroll
  for (int gi = 0; gi < ST::G; ++gi)
#pragma unroll
    for (int c = 0; c < 16; ++c) csum[gi][c] = 0u;

  const int g = lane >> 4;
  auto mma_stage = [&](const uint8_t* cur) {
    const uint8_t* sA = cur;
    const uint8_t* sB = cur + TG::PANEL_BYTES;
    v4i fa[F], fb[F];
#pragma unroll
    for (int a = 0; a < F; ++a)
      fa[a] = *reinterpret_cast<const v4i*>(sA + lds_off(wm * TG::WT + a * 16 + (lane & 15), g));
#pragma unroll
    for (int b = 0; b < F; ++b)
      fb[b] = *reinterpret_cast<const v4i*>(sB + lds_off(wn * TG::WT + b * 16 + (lane & 15), g));
#pragma unroll
    for (int a = 0; a < F; ++a)
#pragma unroll
      for (int b = 0; b < F; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
  };

  // Two register sets: during step s the loads of step s + 2 are in flight
  // while step s + 1 waits in the other set, so each load has two steps of
  // matrix work to hide behind.  Loads past the unit's rows are zeroed, not
  // skipped, so the loop body has no data-dependent branches.
  uint4 r0[ST::G][4], r1[ST::G][4];
  stage_load<BT, ALIGNED>(r0, P, ctx, k0, k1);
  stage_load<BT, ALIGNED>(r1, P, ctx, k0 + KT, k1);
  stage_store<BT>(smem + soff, r0, ctx, csum);
  __syncthreads();

  // An even number of steps, no exits inside the body: a stage past the
  // unit's last row loads as zeros and adds nothing to the counts.
  for (int step = 0; step < nsteps; step += 2) {
    // even step: compute buffer 0, refill r0 with step + 2, store r1 (step + 1) into buffer 1
    stage_load<BT, ALIGNED>(r0, P, ctx, k0 + (step + 2) * KT, k1);
    mma_stage(smem);
    stage_store<BT>(smem + TG::STAGE_BYTES + soff, r1, ctx, csum);
    __syncthreads();
    // odd step: compute buffer 1, refill r1 with step + 3, store r0 (step + 2) into buffer 0
    stage_load<BT, ALIGNED>(r1, P, ctx, k0 + (step + 3) * KT, k1);
    mma_stage(smem + TG::STAGE_BYTES);
    stage_store<BT>(smem + soff, r0, ctx, csum);
    __syncthreads();
  }

  // Column sums of this unit's rows: reduce the per-thread partials in LDS.
  {
    int32_t* dst = (half == 0) ? sColA : sColB;
#pragma unroll
    for (int gi = 0; gi < Staging<BT>::G; ++gi) {
      const int c0 = ctx.col[gi] & (BT - 1);
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (csum[gi][c]) atomicAdd(&dst[c0 + c], (int32_t)csum[gi][c]);
    }
  }
  __syncthreads();

  // Split-K: publish partials; the last unit of the tile takes over.
  if (P.splits > 1) {
    int32_t* wsn = P.ws_n11 + (int64_t)t * BT * BT;
    int32_t* wsc = P.ws_col + (int64_t)t * 2 * BT;
#pragma unroll
    for (int a = 0; a < F; ++a)
#pragma unroll
      for (int b = 0; b < F; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wm * TG::WT + a * 16 + 4 * (lane >> 4) + r;
          const int col = wn * TG::WT + b * 16 + (lane & 15);
          const int v = acc[a][b][r];
          if (v) __hip_atomic_fetch_add(&wsn[row * BT + col], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    for (int c = tid; c < 2 * BT; c += NTHREADS) {
      const int v = sColA[c];
      if (v) __hip_atomic_fetch_add(&wsc[c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const int prev = __hip_atomic_fetch_add(&P.counters[t], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      sFlag[0] = (prev == P.splits - 1);
    }
    __syncthreads();
    if (!sFlag[0]) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // Last arrival: totals back into registers and LDS, then clear the workspace.
#pragma unroll
    for (int a = 0; a < F; ++a)
#pragma unroll
      for (int b = 0; b < F; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wm * TG::WT + a * 16 + 4 * (lane >> 4) + r;
          const int col = wn * TG::WT + b * 16 + (lane & 15);
          int32_t* w = &wsn[row * BT + col];
          acc[a][b][r] = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(w, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    __syncthreads();
    for (int c = tid; c < 2 * BT; c += NTHREADS) {
      sColA[c] = __hip_atomic_load(&wsc[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&wsc[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) __hip_atomic_store(&P.counters[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }

  // Epilogue: derived cells, MI, tile and mirror write-back.  Each wave moves
  // its accumulators through LDS (the stage buffers are free now) one 16-row
  // strip at a time: pass 1 reads the strip row-wise, evaluates MI once per
  // element and writes the tile rows (consecutive lanes, consecutive j); pass 2
  // reads the strip column-wise and writes the mirror rows (consecutive i).
  const int n = P.n;
  const int64_t ln = n;
  if (diag && P.colsum_out) {
    for (int c = tid; c < BT; c += NTHREADS) {
      const int i = I * BT + c;
      if (i < n) P.colsum_out[i] = sColA[c];
    }
  }
  constexpr int WT = TG::WT;
  constexpr int STRIP = 16 * WT;                       // elements per strip
  int32_t* sN = reinterpret_cast<int32_t*>(smem) + wave * 2 * STRIP;
  float* sM = reinterpret_cast<float*>(sN + STRIP);
  const int ibase = I * BT + wm * WT;
  const int jbase = J * BT + wn * WT;
#pragma unroll
  for (int a = 0; a < F; ++a) {
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) sN[(4 * (lane >> 4) + r) * WT + b * 16 + (lane & 15)] = acc[a][b][r];
    __builtin_amdgcn_wave_barrier();
    const int i0 = ibase + a * 16;
    for (int e = lane; e < STRIP; e += 64) {
      const int rr = e / WT, cc = e % WT;
      const int i = i0 + rr, j = jbase + cc;
      const int v11 = sN[e];
      const float v = mi_value(P.m, sColA[i - I * BT], sColB[j - J * BT], v11, P.epi, P.tau);
      sM[e] = v;
      if (i < n && j < n) {
        P.out[i * ln + j] = v;
        if (P.n11_out) P.n11_out[i * ln + j] = v11;
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (!diag) {
      for (int e = lane; e < STRIP; e += 64) {
        const int cc = e / 16, rr = e % 16;
        const int i = i0 + rr, j = jbase + cc;
        if (i < n && j < n) {
          P.out[j * ln + i] = sM[rr * WT + cc];
          if (P.n11_out) P.n11_out[j * ln + i] = sN[rr * WT + cc];
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace mi
