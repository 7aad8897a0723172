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

__device__ __forceinline__ float mi_value(int m, int ci, int cj, int n11, int epi, float tau) {
#pragma clang fp contract(off)
  const int n10 = ci - n11;          // X_i = 1, X_j = 0
  const int n01 = cj - n11;          // X_i = 0, X_j = 1
  const int ni0 = m - ci;            // marginal count of X_i = 0
  const int nj0 = m - cj;            // marginal count of X_j = 0
  const int n00 = ni0 - n01;         // = m - c_i - c_j + n11, without overflow
  float v = 0.0f;
  if (epi != 2) {
    const float fm = (float)m;
    float t11 = cell32(n11, ci, cj, fm);
    float t00 = cell32(n00, ni0, nj0, fm);
    float t10 = cell32(n10, ci, nj0, fm);
    float t01 = cell32(n01, ni0, cj, fm);
    v = ((t11 + t00) + (t10 + t01)) / fm;
    if (epi == 0 || !(v < tau)) return v;
  }
  double d11 = cell64(n11, ci, cj, m);
  double d00 = cell64(n00, ni0, nj0, m);
  double d10 = cell64(n10, ci, nj0, m);
  double d01 = cell64(n01, ni0, cj, m);
  return (float)(((d11 + d00) + (d10 + d01)) / (double)m);
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
  // bytes of dword w (columns 4w..4w+3 of a 16-byte chunk) that are < valid
  const int lo = 4 * w;
  if (valid >= lo + 4) return 0xFFFFFFFFu;
  if (valid <= lo) return 0u;
  return (1u << (8 * (valid - lo))) - 1u;
}

// Global -> registers for one stage of one panel.
template <int BT, bool ALIGNED>
__device__ __forceinline__ void stage_load(uint4 (&r)[Staging<BT>::G][4], const ProbDev& P, int colbase,
                                           int k0, int kend, int p) {
#pragma unroll
  for (int gi = 0; gi < Staging<BT>::G; ++gi) {
    const int q = p + gi * HALF;
    const int col = colbase + Staging<BT>::chunk_col(q);
    const int row0 = k0 + Staging<BT>::chunk_row(q);
    const int valid = P.n - col;  // columns of this chunk inside the matrix
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int row = row0 + rr;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (row < kend && valid > 0) {
        const uint8_t* src = P.X + (int64_t)row * P.ldx + col;
        if (ALIGNED) {
          v = *reinterpret_cast<const uint4*>(src);
        } else {
          uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int b = 0; b < 16; ++b)
            if (b < valid) w[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
          v = make_uint4(w[0], w[1], w[2], w[3]);
        }
        if (valid < 16) {
          v.x &= keep_mask(valid, 0);
          v.y &= keep_mask(valid, 1);
          v.z &= keep_mask(valid, 2);
          v.w &= keep_mask(valid, 3);
        }
      }
      r[gi][rr] = v;
    }
  }
}

__device__ __forceinline__ uint32_t u4get(const uint4& v, int w) {
  return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// Registers -> LDS for one stage of one panel: 4x4 byte transposes so that a
// dword holds 4 consecutive samples of one column, plus column-sum updates.
template <int BT>
__device__ __forceinline__ void stage_store(uint8_t* sbuf, const uint4 (&r)[Staging<BT>::G][4],
                                            uint32_t (&csum)[Staging<BT>::G][16], int p) {
#pragma unroll
  for (int gi = 0; gi < Staging<BT>::G; ++gi) {
    const int q = p + gi * HALF;
    const int c0 = Staging<BT>::chunk_col(q);
    const int rq = Staging<BT>::chunk_row(q) >> 2;  // row quad 0..15
    const int g = rq >> 2, d = rq & 3;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t a = u4get(r[gi][0], w), b = u4get(r[gi][1], w);
      const uint32_t c = u4get(r[gi][2], w), e = u4get(r[gi][3], w);
      const uint32_t x0 = __builtin_amdgcn_perm(b, a, 0x05010400u);  // a0 b0 a1 b1
      const uint32_t x1 = __builtin_amdgcn_perm(b, a, 0x07030602u);  // a2 b2 a3 b3
      const uint32_t y0 = __builtin_amdgcn_perm(e, c, 0x05010400u);  // c0 e0 c1 e1
      const uint32_t y1 = __builtin_amdgcn_perm(e, c, 0x07030602u);  // c2 e2 c3 e3
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
__device__ void run_unit(const ProbDev& P, int t, int s, uint8_t* smem) {
  using TG = TileGeom<BT>;
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

  // Staging role: threads [0, HALF) stage panel I, [HALF, 2 HALF) panel J.
  // On a diagonal tile both operands come from panel I, the second half idles.
  const int half = tid / HALF;
  const int p = tid % HALF;
  const bool stager = !(diag && half == 1);
  const int colbase = (half == 0 ? I : J) * BT;

  for (int c = tid; c < 2 * BT; c += NTHREADS) sColA[c] = 0;

  v4i acc[F][F];
#pragma unroll
  for (int a = 0; a < F; ++a)
#pragma unroll
    for (int b = 0; b < F; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  uint32_t csum[Staging<BT>::G][16];
#pragma unroll
  for (int gi = 0; gi < Staging<BT>::G; ++gi)
#pragma unroll
    for (int c = 0; c < 16; ++c) csum[gi][c] = 0u;

  uint4 regs[Staging<BT>::G][4];
  if (nsteps > 0 && stager) {
    stage_load<BT, ALIGNED>(regs, P, colbase, k0, k1, p);
    stage_store<BT>(smem + half * TG::PANEL_BYTES, regs, csum, p);
  }
  __syncthreads();

  for (int step = 0; step < nsteps; ++step) {
    uint8_t* cur = smem + (step & 1) * TG::STAGE_BYTES;
    uint8_t* nxt = smem + ((step + 1) & 1) * TG::STAGE_BYTES;
    const bool more = (step + 1 < nsteps);
    if (more && stager) stage_load<BT, ALIGNED>(regs, P, colbase, k0 + (step + 1) * KT, k1, p);

    const uint8_t* sA = cur;
    const uint8_t* sB = diag ? cur : cur + TG::PANEL_BYTES;
    const int g = lane >> 4;
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

    if (more && stager) stage_store<BT>(nxt + half * TG::PANEL_BYTES, regs, csum, p);
    __syncthreads();
  }

  // Column sums of this unit's rows: reduce the per-thread partials in LDS.
  if (stager) {
    int32_t* dst = (half == 0) ? sColA : sColB;
#pragma unroll
    for (int gi = 0; gi < Staging<BT>::G; ++gi) {
      const int c0 = Staging<BT>::chunk_col(p + gi * HALF);
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (csum[gi][c]) atomicAdd(&dst[c0 + c], (int32_t)csum[gi][c]);
    }
  }
  __syncthreads();
  if (diag)
    for (int c = tid; c < BT; c += NTHREADS) sColB[c] = sColA[c];
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

  // Epilogue: derived cells, MI, tile and mirror write-back.
  const int n = P.n;
  const int64_t ln = n;
  if (diag && P.colsum_out) {
    for (int c = tid; c < BT; c += NTHREADS) {
      const int i = I * BT + c;
      if (i < n) P.colsum_out[i] = sColA[c];
    }
  }
#pragma unroll
  for (int a = 0; a < F; ++a) {
#pragma unroll
    for (int b = 0; b < F; ++b) {
      const int col = wn * TG::WT + b * 16 + (lane & 15);
      const int j = J * BT + col;
      const int cj = sColB[col];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * TG::WT + a * 16 + 4 * (lane >> 4) + r;
        const int i = I * BT + row;
        if (i < n && j < n) {
          const int v11 = acc[a][b][r];
          const float v = mi_value(P.m, sColA[row], cj, v11, P.epi, P.tau);
          P.out[i * ln + j] = v;
          if (!diag) P.out[j * ln + i] = v;
          if (P.n11_out) {
            P.n11_out[i * ln + j] = v11;
            if (!diag) P.n11_out[j * ln + i] = v11;
          }
        }
      }
    }
  }
}

}  // namespace mi
