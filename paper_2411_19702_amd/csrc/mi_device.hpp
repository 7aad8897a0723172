// mi_device.hpp -- device side of the fused all-pairs binary MI kernel (gfx950).
//
// One work unit = (dataset, output tile (I, J) with I <= J, rows [k0, k1)).
// A unit
//   1. streams its rows [k0, k1) of the two column panels X[:, I] and X[:, J]
//      from HBM into a 4-stage LDS ring with buffer->LDS DMA loads (no
//      registers, no VALU); rows past k1 come back as zeros from the buffer
//      range check, so the loop has no data-dependent branches;
//   2. reads its int8 matrix-core operands with ds_read_b64_tr_b8, which
//      transposes the sample-major panel (row = sample, as in X) into the
//      operand layout (each lane: 8 consecutive samples of one column);
//   3. accumulates the 1-1 counts n11 = X_I^T X_J (the Gram product of
//      Section 2 step 2 / Section 3, the only matrix product of the method)
//      with v_mfma_i32_32x32x32_i8, exact in int32 (on gfx950 this shape has
//      twice the int8 throughput of v_mfma_i32_16x16x64_i8);
//   4. accumulates the column sums c_I, c_J of its rows from the operand
//      registers with bytewise adds folded by v_dot4_u32_u8 (Section 2 step 3
//      / Section 3.1 "Term 2");
//   5. when it covers only part of the rows, adds its partial counts into a
//      per-tile int32 workspace and its row steps into the tile's arrival
//      counter; the unit that completes the count reads the totals back,
//      clears the workspace, and alone runs the epilogue;
//   6. epilogue: derives n10, n01, n00 from n11, c and m (Section 3.1,
//      Eq. 6/7), evaluates MI (Eq. 2/3) per element in FP32 (FP64 on demand)
//      and writes the tile and its mirror.
// Only upper-triangular tiles exist; the mirror write fills the lower one.
//
// Requirements checked on the host: X 16-byte aligned, ldx % 16 == 0 and
// 64 * ldx < 2^31 (other layouts are repacked first).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mi {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
#define MI_LDS __attribute__((address_space(3)))

constexpr int KT = 64;  // samples per stage = one MFMA K step
// Input layouts of the plain kernel: 0/1 bytes, 8 columns per byte (bits),
// or 2 columns per byte as E2M1 (FP4) codes for the FP4 matrix path.
constexpr int kInBytes = 0, kInBits = 1, kInFp4 = 2;
// Bit-packed input unpacked on chip to FP4 codes for the FP4 Gram.
constexpr int kInBitsFp4 = 3;
constexpr int KT4 = 128;  // samples per stage of the FP4 layout: two K steps of 64
// An FP4 unit accumulates in FP32, exact for counts up to 2^24: at most this
// many rows per unit.
constexpr int64_t kFp4MaxUnitRows = (int64_t)1 << 24;

// Tile configuration: BT x BT output tile, WGM x WGN waves, NS-stage LDS ring.
template <int BT_, int WGM_, int WGN_, int NS_>
struct Cfg {
  static constexpr int BT = BT_, WGM = WGM_, WGN = WGN_, NS = NS_;
  static constexpr int NWAVES = WGM * WGN;
  static constexpr int NT = 64 * NWAVES;
  static constexpr int WTM = BT / WGM, WTN = BT / WGN;  // wave tile
  static constexpr int FM = WTM / 32, FN = WTN / 32;    // 32x32 fragments
  static constexpr int PANEL = BT * KT;                 // bytes of one panel stage
  static constexpr int STAGE = 2 * PANEL;               // panel I then panel J
  static constexpr int REGIONS = STAGE / 1024;          // 1 KB DMA regions
  static constexpr int LOADS = REGIONS / NWAVES;        // DMA instructions per wave per stage
  static constexpr int ROWS_PER_REGION = 1024 / BT;
  static constexpr int SEGS = BT / 16;                  // 16-byte segments per row
  static constexpr int RB4 = BT / 2;                    // FP4 layout: bytes of one panel row
  static constexpr int ROWS_PER_REGION4 = 1024 / RB4;
  static constexpr int SEGS4 = RB4 / 16;
  static_assert(NS == 4, "the K loop is unrolled over four ring slots");
  static_assert(KT4 * RB4 == PANEL, "an FP4 stage holds as many bytes as a byte stage");
  static_assert(REGIONS % NWAVES == 0, "DMA regions must split evenly over waves");
};
using Cfg128 = Cfg<128, 2, 2, 4>;  // 4 waves of 64 x 64; 65 KB LDS, 2 workgroups per CU
using Cfg256 = Cfg<256, 2, 4, 4>;  // 8 waves of 128 x 64; 130 KB LDS, 1 workgroup per CU

// Epilogue mode of a problem that asks for counts alone (no MI output).
constexpr int kEpiCounts = 3;

// Everything a unit needs to know about its dataset.
struct ProbDev {
  const uint8_t* X;
  int64_t ldx;
  int32_t m, n;
  float* out;
  int32_t* n11_out;     // optional
  int32_t* colsum_out;  // optional
  int32_t* ws_n11;      // partial units: ntiles * BT * BT int32 (register order), all zero between calls
  int32_t* ws_col;      // partial units: ntiles * 2 * BT int32
  int32_t* counters;    // partial units: ntiles int32 (row steps arrived)
  const int32_t* tiles; // tile order: ntiles entries of (I << 16) | J; nullptr: decoded from the rank
  int32_t ntp;          // panels = ceil(n / BT)
  int32_t ntiles;       // ntp (ntp + 1) / 2
  int32_t ksteps;       // row steps of a whole tile = ceil(m / KT)
  int32_t splits;       // K splits per tile
  int32_t kchunk;       // rows per split, a multiple of KT
  int32_t tiles_per_xcd;  // plain launch: tiles owned by each of the 8 XCDs
  int32_t epi;          // mi_epilogue, or kEpiCounts: counts only, no MI evaluated
  int32_t upper_only;   // nonzero: store i <= j only (no mirror writes)
  int32_t packed;       // kInBytes; kInBits: bit k of byte b = column 8 b + k; kInFp4: two E2M1
                        // codes per byte (column 2 b in the low nibble); ldx in bytes
  float tau;
  // Sparse output: pairs i < j with MI >= thr, appended at an atomic counter
  // (stored while the count stays below cap).  pairs == nullptr: none.
  int32_t* pairs;       // cap entries of (i, j, MI as FP32 bits)
  int64_t pairs_cap;
  unsigned long long* pairs_count;
  float thr;
};

// ---------------------------------------------------------------------------
// Epilogue arithmetic: MI of one pair from (m, c_i, c_j, n11).
// Written so that swapping (i, j) gives bitwise the same result: every
// product is a single commutative IEEE multiply and the four cell terms are
// summed as (t11 + t00) + (t10 + t01).  Contraction into FMAs is disabled so
// the compiler cannot break that symmetry.
// ---------------------------------------------------------------------------
// FP32 cell term n_xy log2(n_xy m / (n_x n_y)) from the count and the
// product a = (m / n_x) (1 / n_y) of the two marginal factors: two
// multiplies and no division.  A zero count gives 0 (0 log 0 = 0): its ratio
// is 0 and is raised to FLT_MIN before the log, a finite value that the zero
// count then cancels.  Factors of zero marginals are stored as 0 (never
// infinite), and a positive count implies positive marginals.
__device__ __forceinline__ float cell32(int nxy, float a) {
#pragma clang fp contract(off)
  const float fn = (float)nxy;
  return fn * __log2f(fmaxf(fn * a, 1.17549435e-38f));
}

__device__ __forceinline__ double cell64(int nxy, int nx, int ny, int m) {
#pragma clang fp contract(off)
  if (nxy <= 0) return 0.0;
  const double num = (double)((int64_t)nxy * (int64_t)m);  // exact below 2^53
  const double den = (double)((int64_t)nx * (int64_t)ny);
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

// The FP64 evaluation as a call: the unrolled epilogue evaluates 64-128
// elements per wave, and inlining the FP64 logarithms at each would blow up
// the code of the FP32 + fallback and FP64 modes.
static __device__ __noinline__ float mi_value64_call(int m, int ci, int cj, int n11) { return mi_value64(m, ci, cj, n11); }

// FP32 MI of one pair (Eq. 2 / 3).  a1i = m / c_i and a0i = m / (m - c_i)
// for the row variable, r1j = 1 / c_j and r0j = 1 / (m - c_j) for the column
// variable (0 where the marginal count is 0); rfm = 1 / m.
__device__ __forceinline__ float mi_value32(int m, int ci, int cj, int n11, float a1i, float a0i, float r1j,
                                            float r0j, float rfm) {
#pragma clang fp contract(off)
  const int n10 = ci - n11;         // X_i = 1, X_j = 0
  const int n01 = cj - n11;         // X_i = 0, X_j = 1
  const int n00 = (m - ci) - n01;   // = m - c_i - c_j + n11, without overflow
  const float t11 = cell32(n11, a1i * r1j);
  const float t00 = cell32(n00, a0i * r0j);
  const float t10 = cell32(n10, a1i * r0j);
  const float t01 = cell32(n01, a0i * r1j);
  return ((t11 + t00) + (t10 + t01)) * rfm;
}

// ---------------------------------------------------------------------------
// LDS layout of one staged panel: 64 rows (samples) of BT bytes, row-major as
// in X, with the 16-byte segments of row r permuted by  seg' = seg ^ f(r).
//
// Operands of v_mfma_i32_32x32x32_i8: lane l holds 16 consecutive samples
// (k = (l / 32) * 16 ..) of fragment column l % 32.  They are read with
// ds_read_b64_tr_b8, which transposes within each group of 16 lanes: if the
// even lanes of a group address 8 bytes (columns c..c+7) of 8 consecutive
// rows and the odd lanes the next 8 columns of the same rows, output lane i of
// the group receives column c + i of those 8 rows.  Lane group G = l / 16
// therefore reads column segment s + (G & 1) at sample rows (G / 2) * 16 + 0..7
// (and + 8 for the second half of its 16 samples).
//
// A half-wave (two groups) reads 8 rows x 2 adjacent segments {s, s + 1}
// (s even); f makes those 16 segment reads land in 16 distinct 4-bank groups:
//   BT = 256 (a row spans all 64 banks): f = 2 (r & 7);
//   BT = 128 (two rows per 64 banks):    f = 2 ((r >> 1) & 3).
// f(r + 8) = f(r) and f(r + 32) = f(r), so the other reads of a fragment are
// at fixed offsets 8 BT, 32 BT, 40 BT from the first.  The DMA writes are
// contiguous 1 KB runs and conflict-free whatever f is.
// ---------------------------------------------------------------------------
template <int BT>
__device__ __forceinline__ int seg_swz(int row) {
  if (BT == 256) return 2 * (row & 7);
  return 2 * ((row >> 1) & 3);
}

// Byte offset (inside one panel) of this lane's first transposed read for the
// 32-column fragment starting at (even) segment s: samples (G/2)*16 + 0..7.
template <int BT>
__device__ __forceinline__ int frag_off(int s, int lane) {
  const int G = lane >> 4, j = lane & 15;
  const int row = (G >> 1) * 16 + (j >> 1);
  const int seg = s + (G & 1);
  return row * BT + ((seg ^ seg_swz<BT>(row)) << 4) + ((j & 1) << 3);
}

// One operand fragment (32 columns x 16 samples per lane, one 32-sample K
// step): two transposed 8-sample reads, 8 rows apart.  The compiler tracks
// these reads (and, because every ring slot is its own LDS object, which DMA
// writes they depend on), so it can issue them ahead of the MFMAs that use them.
template <int BT>
__device__ __forceinline__ v4i read_frag(const uint8_t* p) {
  const v2i lo = __builtin_amdgcn_ds_read_tr8_b64_v2i32((MI_LDS v2i*)(p));
  const v2i hi = __builtin_amdgcn_ds_read_tr8_b64_v2i32((MI_LDS v2i*)(p + 8 * BT));
  return v4i{lo.x, lo.y, hi.x, hi.y};
}

// ---------------------------------------------------------------------------
// FP4 layout: two columns per byte (column 2 c in the low nibble of byte c), a
// one stored as the E2M1 code of 1.0 and a zero as 0.  The exact 0/1 products
// then sum to the integer counts in the FP32 accumulator (exact below 2^24).
// A stage is 128 sample rows of BT / 2 bytes per panel: the same bytes as 64
// rows of the byte layout, for twice the samples.
//
// Operands of v_mfma_scale_f32_32x32x64_f8f6f4 with E2M1 operands and unit
// scales: lane l holds 32 samples (k = (l / 32) * 32 ..) of fragment column
// l % 32, one per nibble, in four registers (the upper four of the 8-register
// operand are not read for E2M1).  They are read with ds_read_b64_tr_b4, a
// nibble transpose within each group of 16 lanes: source lane q addresses 8
// bytes (16 columns) of one sample row, and output lane i receives column i of
// the 16 rows, in source-lane order.  Lane group G = l / 16 therefore reads the
// column half G & 1 (8 bytes of the fragment's 16-byte segment) at sample rows
// (G / 2) * 32 + 0..15, and + 16 for its other 16 samples.
//
// A half-wave reads 16 consecutive rows at one segment; g spreads them over 16
// distinct 4-bank groups:
//   BT = 256 (a row is 128 bytes, two rows span the 64 banks): g = (r >> 1) & 7;
//   BT = 128 (a row is 64 bytes, four rows span the banks):     g = (r >> 2) & 3.
// g(r + 16) = g(r), so the second read (rows + 16) and the second K step of a
// stage (rows + 64) are at fixed offsets from the first read.
// ---------------------------------------------------------------------------
template <int BT>
__device__ __forceinline__ int seg_swz4(int row) {
  if (BT == 256) return (row >> 1) & 7;
  return (row >> 2) & 3;
}

// Byte offset (inside one panel) of this lane's first transposed read for the
// 32-column fragment in segment s (columns 32 s ..).
template <int BT>
__device__ __forceinline__ int frag_off4(int s, int lane) {
  const int G = lane >> 4, q = lane & 15;
  const int row = (G >> 1) * 32 + q;
  return row * (BT / 2) + ((s ^ seg_swz4<BT>(row)) << 4) + ((G & 1) << 3);
}

// One FP4 operand fragment (32 columns x 32 samples per lane, one 64-sample K
// step): two transposed 16-sample reads, 16 rows apart.
template <int BT>
__device__ __forceinline__ v4i read_frag4(const uint8_t* p) {
  const v2i lo = __builtin_amdgcn_ds_read_tr4_b64_v2i32((MI_LDS v2i*)(p));
  const v2i hi = __builtin_amdgcn_ds_read_tr4_b64_v2i32((MI_LDS v2i*)(p + 16 * (BT / 2)));
  return v4i{lo.x, lo.y, hi.x, hi.y};
}

__device__ __forceinline__ uint32_t sgpr(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Buffer descriptor for one stage: `rem` rows of X are left from `base` on
// (rem <= 0 past the end of the unit); reads at byte offsets past
// min(rem, kt) rows return zeros and touch no memory.  All arguments are
// workgroup-uniform scalars.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stage_rsrc(uint64_t base, int rem, int ldx, int kt = KT) {
  const int rows = rem >= kt ? kt : max(rem, 0);
  const uint32_t lo = sgpr((uint32_t)base), hi = sgpr((uint32_t)(base >> 32));
  const int nrec = (int)sgpr((uint32_t)(rows * ldx));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), 0, nrec, 0x00020000);
}

// Tiles (I, J), 0 <= I <= J < ntp, of the aligned square block with corner
// (x0, y0) and side h: for each J of the block below ntp, the I of the block
// up to J.
__host__ __device__ inline int64_t tiles_in_block(int64_t x0, int64_t y0, int64_t h, int64_t ntp) {
  const int64_t jlo = y0, jhi = (y0 + h < ntp ? y0 + h : ntp) - 1;
  if (jhi < jlo) return 0;
  int64_t c = 0;
  // J in [x0, x0 + h - 2]: J - x0 + 1 tiles each.
  const int64_t a = jlo > x0 ? jlo : x0, b = jhi < x0 + h - 2 ? jhi : x0 + h - 2;
  if (a <= b) c += (b - a + 1) * (a + b - 2 * x0 + 2) / 2;
  // J >= x0 + h - 1: the whole column of h tiles.
  const int64_t d = jlo > x0 + h - 1 ? jlo : x0 + h - 1;
  if (d <= jhi) c += h * (jhi - d + 1);
  return c;
}

// The tile of rank t in the order of the tile table (upper-triangular tiles
// sorted by the Morton code that puts bit b of I at position 2 b + 1 and bit
// b of J at 2 b), without the table: descend the quadrant tree, whose
// quadrants come in the order (I low, J low), (I low, J high), (I high, J
// low), (I high, J high), skipping the tiles of the quadrants before the one
// holding rank t.  At most 15 levels (ntp <= 32,767).
__host__ __device__ inline void morton_tile(int ntp, int t, int& I, int& J) {
  int64_t h = 1;
  while (h < ntp) h <<= 1;
  int64_t x0 = 0, y0 = 0, r = t;
  while (h > 1) {
    h >>= 1;
    const int64_t c0 = tiles_in_block(x0, y0, h, ntp);
    if (r < c0) continue;
    r -= c0;
    const int64_t c1 = tiles_in_block(x0, y0 + h, h, ntp);
    if (r < c1) { y0 += h; continue; }
    r -= c1;
    const int64_t c2 = tiles_in_block(x0 + h, y0, h, ntp);
    if (r < c2) { x0 += h; continue; }
    r -= c2;
    x0 += h;
    y0 += h;
  }
  I = (int)x0;
  J = (int)y0;
}

// Decode an upper-triangular tile from the order table, or from its rank
// when the problem carries no table.
__device__ __forceinline__ void tile_ij(const ProbDev& P, int t, int& I, int& J) {
  if (P.tiles) {
    const int v = P.tiles[t];
    I = v >> 16;
    J = v & 0xFFFF;
  } else {
    morton_tile(P.ntp, t, I, J);
  }
}

// LDS of one workgroup: the four ring slots are separate objects (so the
// compiler can tell which DMA each operand read depends on), plus the column
// sums and a flag, and the epilogue's per-column reciprocals.
template <class C>
struct Smem {
  uint8_t* slot[4];
  int32_t* cols;  // 2 * BT + 4 int32
  float* rcp;     // 4 * BT float
  float* mir;     // epilogue mirror buffers (NWAVES x 16 x 36 float), or nullptr: in the ring
};

// Bit-packed input: 16 columns from 2 packed bytes (the low 16 bits of w,
// bit k of a byte = its k-th column), one 0/1 byte per column.  Each nibble
// is spread to one bit per byte by one multiply: its copies shifted by 0, 7,
// 14 and 21 bits do not overlap, so nothing carries.
__device__ __forceinline__ uint4 unpack16(uint32_t w) {
  const uint32_t k = 0x00204081u;
  return make_uint4(((w & 0xFu) * k) & 0x01010101u, (((w >> 4) & 0xFu) * k) & 0x01010101u,
                    (((w >> 8) & 0xFu) * k) & 0x01010101u, (((w >> 12) & 0xFu) * k) & 0x01010101u);
}

// One work unit.  IN: the input layout (kInBytes, kInBits, kInFp4).  With
// kInFp4 the stages are 128 rows of FP4 codes and the Gram runs on the FP4
// matrix instructions (FP32 accumulators, converted to the int32 counts after
// the K loop).  With kInBits X is bit-packed; each stage is loaded into registers
// (one 8-byte load per thread, four stages ahead), unpacked to bytes and
// written to the ring, instead of the buffer-to-LDS DMA of the byte layout.
template <class C, int IN = kInBytes>
__device__ __forceinline__ void run_unit(const ProbDev& P, int t, int k0, int k1, const Smem<C>& sm) {
#if defined(__HIP_DEVICE_COMPILE__)  // device-only body (gfx950 builtins and asm)
  constexpr int BT = C::BT, FM = C::FM, FN = C::FN;
  // PK: bits unpacked to bytes (int8 Gram); PK4: bits unpacked to FP4 codes;
  // F4: the FP4 Gram (FP4 input by DMA, or PK4).
  constexpr bool PK = IN == kInBits, PK4 = IN == kInBitsFp4, F4 = IN == kInFp4 || PK4;
  constexpr int KS = F4 ? KT4 : KT;  // sample rows per stage
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = (int)sgpr((uint32_t)(tid >> 6));  // wave-uniform: scalar branches on it
  const int wm = wave / C::WGN, wn = wave % C::WGN;

  int I, J;
  tile_ij(P, t, I, J);
  const bool diag = (I == J);
  const int nsteps = (k1 - k0 + KT - 1) / KT;
  const bool whole = (k0 == 0 && k1 == P.m);

  int32_t* sColA = sm.cols;
  int32_t* sColB = sColA + BT;
  int32_t* sFlag = sColB + BT;
  for (int c = tid; c < 2 * BT; c += C::NT) sColA[c] = 0;

  // DMA source offsets of this lane's LOADS regions (fixed for the unit).
  // Region R = i * NWAVES + wave holds ROWS_PER_REGION rows of one panel;
  // lane l of it lands at R * 1024 + 16 l, i.e. row R' * RPR + l / SEGS at
  // physical segment l % SEGS, which holds logical segment (l % SEGS) ^ f(row).
  int voff[C::LOADS];
  uint32_t ldsoff[C::LOADS];
  if constexpr (F4 && !PK4) {
    // The same regions over 128 rows of BT / 2 bytes (ROWS_PER_REGION4 rows each).
#pragma unroll
    for (int i = 0; i < C::LOADS; ++i) {
      const int R = i * C::NWAVES + wave;
      const int panel = R / (C::REGIONS / 2);
      const int row = (R % (C::REGIONS / 2)) * C::ROWS_PER_REGION4 + lane / C::SEGS4;
      const int seg = (lane % C::SEGS4) ^ seg_swz4<BT>(row);
      const int col0 = (panel == 0 ? I : J) * C::RB4;
      voff[i] = row * (int)P.ldx + col0 + 16 * seg;
      ldsoff[i] = (uint32_t)R * 1024u;
    }
  } else if constexpr (!PK && !PK4) {
#pragma unroll
    for (int i = 0; i < C::LOADS; ++i) {
      const int R = i * C::NWAVES + wave;
      const int panel = R / (C::REGIONS / 2);
      const int row = (R % (C::REGIONS / 2)) * C::ROWS_PER_REGION + lane / C::SEGS;
      const int seg = (lane % C::SEGS) ^ seg_swz<BT>(row);
      const int col0 = (panel == 0 ? I : J) * BT;
      voff[i] = row * (int)P.ldx + col0 + 16 * seg;
      ldsoff[i] = (uint32_t)R * 1024u;
    }
  }
  // Packed layout: thread tid owns 64 columns (8 packed bytes, 4 segments)
  // of one row of one panel; its segments land at their swizzled places.
  constexpr int TPR = BT / 64;  // threads per panel row
  static_assert(2 * KT * TPR == C::NT, "one 8-byte packed piece per thread and stage");
  int pvoff = 0;
  uint32_t pwoff[4] = {0u, 0u, 0u, 0u};
  if constexpr (PK) {
    const int panel = tid / (KT * TPR), row = (tid / TPR) % KT, q = tid % TPR;
    pvoff = row * (int)P.ldx + ((panel == 0 ? I : J) * BT) / 8 + 8 * q;
#pragma unroll
    for (int g = 0; g < 4; ++g)
      pwoff[g] = (uint32_t)(panel * C::PANEL + row * BT + (((4 * q + g) ^ seg_swz<BT>(row)) << 4));
  }
  // Bits to FP4 codes: thread tid owns 128 columns (16 packed bytes, four
  // 32-column FP4 segments) of one of the stage's 128 rows of one panel.
  constexpr int TPR4 = BT / 128;
  static_assert(2 * KT4 * TPR4 == C::NT, "one 16-byte packed piece per thread and FP4 stage");
  if constexpr (PK4) {
    const int panel = tid / (KT4 * TPR4), row = (tid / TPR4) % KT4, q = tid % TPR4;
    pvoff = row * (int)P.ldx + ((panel == 0 ? I : J) * BT) / 8 + 16 * q;
#pragma unroll
    for (int g = 0; g < 4; ++g)
      pwoff[g] = (uint32_t)(panel * C::PANEL + row * C::RB4 + (((4 * q + g) ^ seg_swz4<BT>(row)) << 4));
  }
  // Stage j of the unit starts at row k0 + j KS; its base address advances by
  // KS * ldx bytes per stage (scalar adds, no per-stage multiplies).
  const int ldx32 = (int)P.ldx;
  const uint64_t stage_bytes = (uint64_t)KS * (uint64_t)P.ldx;
  const uint64_t xk0 = (uint64_t)(P.X + (int64_t)k0 * P.ldx);
  auto dma_stage = [&](uint64_t base, int rem, uint8_t* slot) {
    const __amdgpu_buffer_rsrc_t rs = stage_rsrc(base, rem, ldx32, KS);
#pragma unroll
    for (int i = 0; i < C::LOADS; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (MI_LDS void*)(slot + ldsoff[i]), 16, voff[i], 0, 0, 0);
  };

  // Column sums: the WGN waves that share an A panel block each sum SA of its
  // FM fragments, and the WGM waves that share a B block each sum SB of its FN
  // fragments, so each column of both panels is summed by exactly one wave
  // and the work is the same for all waves.  Register fragment a of a wave
  // holds column block (a + ra) mod FM of its A block (b: (b + rb) mod FN of
  // its B block); the rotation puts the fragments the wave sums at registers
  // 0 .. SA-1 (0 .. SB-1), so the loop sums fixed registers, without branches.
  constexpr int SA = FM / C::WGN, SB = FN / C::WGM;
  static_assert(SA * C::WGN == FM && SB * C::WGM == FN, "column sums split evenly over the waves");
  static_assert((FM & (FM - 1)) == 0 && (FN & (FN - 1)) == 0, "fragment counts are powers of two");
  const int ra = wn * SA, rb = wm * SB;
  auto blk_a = [&](int a) { return (a + ra) & (FM - 1); };
  auto blk_b = [&](int b) { return (b + rb) & (FN - 1); };

  // Operand read offsets (inside a stage) for this lane's fragments.
  uint32_t aoff[FM], boff[FN];
  if constexpr (F4) {
#pragma unroll
    for (int a = 0; a < FM; ++a) aoff[a] = (uint32_t)frag_off4<BT>((wm * C::WTM) / 32 + blk_a(a), lane);
#pragma unroll
    for (int b = 0; b < FN; ++b) boff[b] = (uint32_t)(C::PANEL + frag_off4<BT>((wn * C::WTN) / 32 + blk_b(b), lane));
  } else {
#pragma unroll
    for (int a = 0; a < FM; ++a) aoff[a] = (uint32_t)frag_off<BT>((wm * C::WTM) / 16 + 2 * blk_a(a), lane);
#pragma unroll
    for (int b = 0; b < FN; ++b) boff[b] = (uint32_t)(C::PANEL + frag_off<BT>((wn * C::WTN) / 16 + 2 * blk_b(b), lane));
  }

  v16i acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;
  // Column-sum registers.  Bytes are 0/1: the four dwords of a fragment half
  // add bytewise without carries (<= 4 per byte), accumulate bytewise for
  // four steps (<= 32 per byte), and are folded into 32-bit totals with v_dot4
  // once per four steps.
  uint32_t pkA[SA], pkB[SB], csA[SA], csB[SB];
#pragma unroll
  for (int x = 0; x < SA; ++x) pkA[x] = csA[x] = 0u;
#pragma unroll
  for (int y = 0; y < SB; ++y) pkB[y] = csB[y] = 0u;

  // Fragments are read one K half ahead of their MFMAs (two register sets):
  // while the MFMAs of one half execute, the wave reads the next half, and
  // the barrier that publishes the next stage sits between the two halves,
  // so matrix work is queued while the wave waits at it.
  v4i fa0[FM], fb0[FN], fa1[FM], fb1[FN];
  // Half kk of a stage starts at byte kk * 32 * BT of each panel in both
  // layouts (32 byte rows, or 64 FP4 rows of BT / 2 bytes).
  auto read_half = [&](const uint8_t* slot, int kk, v4i (&fa)[FM], v4i (&fb)[FN]) {
    const uint8_t* kb = slot + kk * 32 * BT;
    if constexpr (F4) {
#pragma unroll
      for (int b = 0; b < FN; ++b) fb[b] = read_frag4<BT>(kb + boff[b]);
#pragma unroll
      for (int a = 0; a < FM; ++a) fa[a] = read_frag4<BT>(kb + aoff[a]);
    } else {
#pragma unroll
      for (int b = 0; b < FN; ++b) fb[b] = read_frag<BT>(kb + boff[b]);
#pragma unroll
      for (int a = 0; a < FM; ++a) fa[a] = read_frag<BT>(kb + aoff[a]);
    }
  };
  auto mma_half = [&](const v4i (&fa)[FM], const v4i (&fb)[FN]) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
#pragma unroll
    for (int x = 0; x < SA; ++x) pkA[x] += ((uint32_t)fa[x].x + (uint32_t)fa[x].y) + ((uint32_t)fa[x].z + (uint32_t)fa[x].w);
#pragma unroll
    for (int y = 0; y < SB; ++y) pkB[y] += ((uint32_t)fb[y].x + (uint32_t)fb[y].y) + ((uint32_t)fb[y].z + (uint32_t)fb[y].w);
    // Keep each half's sums here: left alone, the compiler may re-associate
    // the chain and defer all adds to the end of the unrolled loop, which
    // keeps every fragment register of four steps alive.
#pragma unroll
    for (int x = 0; x < SA; ++x) asm volatile("" : "+v"(pkA[x]));
#pragma unroll
    for (int y = 0; y < SB; ++y) asm volatile("" : "+v"(pkB[y]));
  };
  // Stage `step + 1` complete for every wave, and every wave done reading the
  // slot that the next DMA refills: this wave waits for its own DMA of that
  // stage (at most two later stages outstanding) and its own LDS reads, then
  // the barrier extends both to the workgroup.
  auto stage_barrier = [&]() {
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"i"(2 * C::LOADS) : "memory");
  };

  const int rows = k1 - k0;
  // FP4 Gram (both FP4 paths): FP32 accumulators and one 64-sample K step.
  // Column sums: a one is the code 0b0010, so a fragment's popcount is its
  // count of ones.
  v16f accf[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) accf[a][b][r] = 0.0f;
  auto mma_half4 = [&](const v4i (&fa)[FM], const v4i (&fb)[FN]) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
        accf[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            v8i{fa[a].x, fa[a].y, fa[a].z, fa[a].w, 0, 0, 0, 0}, v8i{fb[b].x, fb[b].y, fb[b].z, fb[b].w, 0, 0, 0, 0},
            accf[a][b], 4, 4, 0, 127, 0, 127);  // E2M1 x E2M1, scales 2^0
#pragma unroll
    for (int x = 0; x < SA; ++x)
      csA[x] += (__builtin_popcount((uint32_t)fa[x].x) + __builtin_popcount((uint32_t)fa[x].y)) +
                (__builtin_popcount((uint32_t)fa[x].z) + __builtin_popcount((uint32_t)fa[x].w));
#pragma unroll
    for (int y = 0; y < SB; ++y)
      csB[y] += (__builtin_popcount((uint32_t)fb[y].x) + __builtin_popcount((uint32_t)fb[y].y)) +
                (__builtin_popcount((uint32_t)fb[y].z) + __builtin_popcount((uint32_t)fb[y].w));
  };
  // Counts of at most 2^24 rows are exact in FP32.
  auto fp4_counts = [&]() {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][r] = (int)accf[a][b][r];
  };
  if constexpr (PK) {
    // Stage j's 8 packed bytes of this thread (zeros past the unit's rows).
    auto pload = [&](uint64_t base, int rem) -> uint2 {
      const __amdgpu_buffer_rsrc_t rs = stage_rsrc(base, rem, ldx32);
      const v2u v = __builtin_amdgcn_raw_buffer_load_b64(rs, pvoff, 0, 0);
      return make_uint2(v.x, v.y);
    };
    // The two halves of this thread's piece (segments 0-1 and 2-3).
    auto pstore_lo = [&](uint2 v, uint8_t* slot) {
      *(MI_LDS uint4*)(slot + pwoff[0]) = unpack16(v.x);
      *(MI_LDS uint4*)(slot + pwoff[1]) = unpack16(v.x >> 16);
    };
    auto pstore_hi = [&](uint2 v, uint8_t* slot) {
      *(MI_LDS uint4*)(slot + pwoff[2]) = unpack16(v.y);
      *(MI_LDS uint4*)(slot + pwoff[3]) = unpack16(v.y >> 16);
    };
    // Every wave's ring writes (and its own reads) done, workgroup-wide.
    auto write_barrier = [&]() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };
    // Registers pk[j % 4] hold stage j until it is written to the ring.
    // Stages 0 and 1 are written before the loop; step `step` writes stage
    // step + 2 in two halves, one beside each half's MFMAs (its slot was last
    // read two steps before), then loads stage step + 6 into the freed
    // registers.
    uint2 pk0 = pload(xk0, rows), pk1 = pload(xk0 + stage_bytes, rows - KT);
    uint2 pk2 = pload(xk0 + 2 * stage_bytes, rows - 2 * KT), pk3 = pload(xk0 + 3 * stage_bytes, rows - 3 * KT);
    pstore_lo(pk0, sm.slot[0]);
    pstore_hi(pk0, sm.slot[0]);
    pstore_lo(pk1, sm.slot[1]);
    pstore_hi(pk1, sm.slot[1]);
    pk0 = pload(xk0 + 4 * stage_bytes, rows - 4 * KT);
    pk1 = pload(xk0 + 5 * stage_bytes, rows - 5 * KT);
    write_barrier();
    read_half(sm.slot[0], 0, fa0, fb0);
    uint64_t pbase = xk0 + 6 * stage_bytes;  // stage step + 6, loaded during step `step`
    int prem = rows - 6 * KT;
    auto do_step_pk = [&](uint8_t* cur, uint8_t* nxt, uint8_t* ahead, uint2& reg) {
      read_half(cur, 1, fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      mma_half(fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      pstore_lo(reg, ahead);
      write_barrier();
      read_half(nxt, 0, fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      mma_half(fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      pstore_hi(reg, ahead);
      reg = pload(pbase, prem);
      pbase += stage_bytes;
      prem -= KT;
    };
    for (int step = 0; step < nsteps; step += 4) {
      do_step_pk(sm.slot[0], sm.slot[1], sm.slot[2], pk2);
      do_step_pk(sm.slot[1], sm.slot[2], sm.slot[3], pk3);
      do_step_pk(sm.slot[2], sm.slot[3], sm.slot[0], pk0);
      do_step_pk(sm.slot[3], sm.slot[0], sm.slot[1], pk1);
#pragma unroll
      for (int x = 0; x < SA; ++x) {
        csA[x] = __builtin_amdgcn_udot4(pkA[x], 0x01010101u, csA[x], false);
        pkA[x] = 0u;
      }
#pragma unroll
      for (int y = 0; y < SB; ++y) {
        csB[y] = __builtin_amdgcn_udot4(pkB[y], 0x01010101u, csB[y], false);
        pkB[y] = 0u;
      }
    }
  } else if constexpr (PK4) {
    // The bit-packed schedule over 128-row FP4 stages: each stage is one
    // 16-byte load per thread, four stages ahead, unpacked to FP4 codes in
    // two halves beside the half-steps' instructions.  A packed byte spreads
    // to one nibble per bit (three shift-or-mask steps), then to the code
    // 0b0010 per one.
    auto pload4 = [&](uint64_t base, int rem) -> uint4 {
      const __amdgpu_buffer_rsrc_t rs = stage_rsrc(base, rem, ldx32, KT4);
      const v4i v = __builtin_amdgcn_raw_buffer_load_b128(rs, pvoff, 0, 0);
      return make_uint4((uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w);
    };
    auto spread8 = [](uint32_t b) {  // bit k of b -> 0b0010 in nibble k
      uint32_t t = b & 0xFFu;
      t = (t | (t << 12)) & 0x000F000Fu;
      t = (t | (t << 6)) & 0x03030303u;
      t = (t | (t << 3)) & 0x11111111u;
      return t << 1;
    };
    auto seg4 = [&](uint32_t w) {  // 32 columns (4 packed bytes) -> one 16-byte FP4 segment
      return make_uint4(spread8(w), spread8(w >> 8), spread8(w >> 16), spread8(w >> 24));
    };
    auto pstore_lo4 = [&](uint4 v, uint8_t* slot) {
      *(MI_LDS uint4*)(slot + pwoff[0]) = seg4(v.x);
      *(MI_LDS uint4*)(slot + pwoff[1]) = seg4(v.y);
    };
    auto pstore_hi4 = [&](uint4 v, uint8_t* slot) {
      *(MI_LDS uint4*)(slot + pwoff[2]) = seg4(v.z);
      *(MI_LDS uint4*)(slot + pwoff[3]) = seg4(v.w);
    };
    auto write_barrier = [&]() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };
    uint4 pk0 = pload4(xk0, rows), pk1 = pload4(xk0 + stage_bytes, rows - KS);
    uint4 pk2 = pload4(xk0 + 2 * stage_bytes, rows - 2 * KS), pk3 = pload4(xk0 + 3 * stage_bytes, rows - 3 * KS);
    pstore_lo4(pk0, sm.slot[0]);
    pstore_hi4(pk0, sm.slot[0]);
    pstore_lo4(pk1, sm.slot[1]);
    pstore_hi4(pk1, sm.slot[1]);
    pk0 = pload4(xk0 + 4 * stage_bytes, rows - 4 * KS);
    pk1 = pload4(xk0 + 5 * stage_bytes, rows - 5 * KS);
    write_barrier();
    read_half(sm.slot[0], 0, fa0, fb0);
    uint64_t pbase = xk0 + 6 * stage_bytes;  // stage step + 6, loaded during step `step`
    int prem = rows - 6 * KS;
    auto do_step_pk4 = [&](uint8_t* cur, uint8_t* nxt, uint8_t* ahead, uint4& reg) {
      read_half(cur, 1, fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      mma_half4(fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      pstore_lo4(reg, ahead);
      write_barrier();
      read_half(nxt, 0, fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      mma_half4(fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      pstore_hi4(reg, ahead);
      reg = pload4(pbase, prem);
      pbase += stage_bytes;
      prem -= KS;
    };
    const int nstages = (rows + KS - 1) / KS;
    for (int step = 0; step < nstages; step += 4) {
      do_step_pk4(sm.slot[0], sm.slot[1], sm.slot[2], pk2);
      do_step_pk4(sm.slot[1], sm.slot[2], sm.slot[3], pk3);
      do_step_pk4(sm.slot[2], sm.slot[3], sm.slot[0], pk0);
      do_step_pk4(sm.slot[3], sm.slot[0], sm.slot[1], pk1);
    }
    fp4_counts();
  } else if constexpr (F4) {
    // The byte loop's schedule over 128-row FP4 stages (DMA); each half is
    // one 64-sample K step of the FP4 instruction.
    dma_stage(xk0, rows, sm.slot[0]);
    dma_stage(xk0 + stage_bytes, rows - KS, sm.slot[1]);
    dma_stage(xk0 + 2 * stage_bytes, rows - 2 * KS, sm.slot[2]);
    stage_barrier();
    dma_stage(xk0 + 3 * stage_bytes, rows - 3 * KS, sm.slot[3]);
    read_half(sm.slot[0], 0, fa0, fb0);
    uint64_t dbase = xk0 + 4 * stage_bytes;
    int drem = rows - 4 * KS;
    auto do_step4 = [&](uint8_t* cur, uint8_t* nxt) {
      read_half(cur, 1, fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      mma_half4(fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      stage_barrier();
      dma_stage(dbase, drem, cur);
      dbase += stage_bytes;
      drem -= KS;
      read_half(nxt, 0, fa0, fb0);
      __builtin_amdgcn_sched_barrier(0);
      mma_half4(fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
    };
    const int nstages = (rows + KS - 1) / KS;
    for (int step = 0; step < nstages; step += 4) {
      do_step4(sm.slot[0], sm.slot[1]);
      do_step4(sm.slot[1], sm.slot[2]);
      do_step4(sm.slot[2], sm.slot[3]);
      do_step4(sm.slot[3], sm.slot[0]);
    }
    fp4_counts();
  } else {
  // Prologue: stages 0 .. 2 in flight in slots 0 .. 2; once stage 0 is in,
  // stage 3 goes to slot 3 and the first half of stage 0 is read.
  dma_stage(xk0, rows, sm.slot[0]);
  dma_stage(xk0 + stage_bytes, rows - KT, sm.slot[1]);
  dma_stage(xk0 + 2 * stage_bytes, rows - 2 * KT, sm.slot[2]);
  stage_barrier();
  dma_stage(xk0 + 3 * stage_bytes, rows - 3 * KT, sm.slot[3]);
  read_half(sm.slot[0], 0, fa0, fb0);
  uint64_t dbase = xk0 + 4 * stage_bytes;  // stage step + 4, loaded during step `step`
  int drem = rows - 4 * KT;

  // Step `step` (stage in slot cur, the next stage in slot nxt).
  auto do_step = [&](uint8_t* cur, uint8_t* nxt) {
    read_half(cur, 1, fa1, fb1);
    __builtin_amdgcn_sched_barrier(0);
    mma_half(fa0, fb0);
    __builtin_amdgcn_sched_barrier(0);
    stage_barrier();
    dma_stage(dbase, drem, cur);  // stage step + 4 into the slot just consumed
    dbase += stage_bytes;
    drem -= KT;
    read_half(nxt, 0, fa0, fb0);
    __builtin_amdgcn_sched_barrier(0);
    mma_half(fa1, fb1);
    __builtin_amdgcn_sched_barrier(0);
  };

  // Unrolled over the four slots; a unit whose step count is not a multiple
  // of four runs up to three extra steps on zeros (rows past k1 read as zero).
  for (int step = 0; step < nsteps; step += 4) {
    do_step(sm.slot[0], sm.slot[1]);
    do_step(sm.slot[1], sm.slot[2]);
    do_step(sm.slot[2], sm.slot[3]);
    do_step(sm.slot[3], sm.slot[0]);
#pragma unroll
    for (int x = 0; x < SA; ++x) {
      csA[x] = __builtin_amdgcn_udot4(pkA[x], 0x01010101u, csA[x], false);
      pkA[x] = 0u;
    }
#pragma unroll
    for (int y = 0; y < SB; ++y) {
      csB[y] = __builtin_amdgcn_udot4(pkB[y], 0x01010101u, csB[y], false);
      pkB[y] = 0u;
    }
  }
  }
  // Drain the DMA of stages past the end before the ring is reused.
  asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");

  // Column sums of this unit's rows: lanes l and l + 32 hold partial sums of
  // the same fragment column; combine them in LDS.
#pragma unroll
  for (int x = 0; x < SA; ++x) atomicAdd(&sColA[wm * C::WTM + (wn * SA + x) * 32 + (lane & 31)], (int)csA[x]);
#pragma unroll
  for (int y = 0; y < SB; ++y) atomicAdd(&sColB[wn * C::WTN + (wm * SB + y) * 32 + (lane & 31)], (int)csB[y]);
  __syncthreads();

  // Partial unit: publish partials; the unit that completes the tile's row
  // steps takes over.  The tile's workspace holds the counts in register
  // order (wave, block, register pair, lane): every unit's wave w holds the
  // same elements in the same registers, so the order only has to agree
  // between units.  Registers 2 k and 2 k + 1 go out as one 64-bit atomic
  // add of the two int32 counts packed side by side: every partial count is
  // non-negative and their total is at most m < 2^31, so the low half never
  // carries into the high one and both sums are exact.  One instruction
  // covers 512 consecutive bytes.
  static_assert(C::NWAVES * FM * FN * 16 * 64 == BT * BT, "the register order covers the tile's workspace");
  if (!whole) {
    unsigned long long* wsn = reinterpret_cast<unsigned long long*>(P.ws_n11 + (int64_t)t * BT * BT) +
                              (int64_t)wave * (FM * FN * 8 * 64) + lane;
    int32_t* wsc = P.ws_col + (int64_t)t * 2 * BT;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const unsigned long long v = (unsigned long long)(uint32_t)acc[a][b][2 * k] |
                                       ((unsigned long long)(uint32_t)acc[a][b][2 * k + 1] << 32);
          if (v) __hip_atomic_fetch_add(wsn + ((a * FN + b) * 8 + k) * 64, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    for (int c = tid; c < 2 * BT; c += C::NT) {
      const int v = sColA[c];
      if (v) __hip_atomic_fetch_add(&wsc[c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const int prev = __hip_atomic_fetch_add(&P.counters[t], nsteps, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      sFlag[0] = (prev + nsteps == P.ksteps);
    }
    __syncthreads();
    if (!sFlag[0]) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // Last arrival: totals back into registers and LDS, then clear the
    // workspace.  The acquire fence orders these plain (cached, coalesced)
    // loads after every other unit's published adds.
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const unsigned long long v = wsn[((a * FN + b) * 8 + k) * 64];
          acc[a][b][2 * k] = (int)(uint32_t)v;
          acc[a][b][2 * k + 1] = (int)(uint32_t)(v >> 32);
        }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int k = 0; k < 8; ++k) wsn[((a * FN + b) * 8 + k) * 64] = 0ull;
    __syncthreads();
    for (int c = tid; c < 2 * BT; c += C::NT) {
      sColA[c] = wsc[c];
      wsc[c] = 0;
    }
    if (tid == 0) __hip_atomic_store(&P.counters[t], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }

  // Epilogue: derived cells, MI, tile and mirror write-back, straight from
  // the accumulator registers.  In a 32 x 32 accumulator block, register r of
  // lane l holds the count of tile row 8 (r / 4) + 4 (l / 32) + r % 4 and
  // column l % 32: one register is two 32-column half rows (128-byte stores),
  // and a lane's registers 4 g .. 4 g + 3 are four consecutive rows of one
  // column (one 16-byte store into the mirror row of that column).
  const int n = P.n;
  const int64_t ln = n;
  if (diag && P.colsum_out) {
    for (int c = tid; c < BT; c += C::NT) {
      const int i = I * BT + c;
      if (i < n) P.colsum_out[i] = sColA[c];
    }
  }
  // Marginal factors of both panels' columns (IEEE division, once per
  // column): m / c and m / (m - c) for the rows' variables (panel I), 1 / c
  // and 1 / (m - c) for the columns' (panel J); 0 where the count is 0.
  const float fm = (float)P.m, rfm = 1.0f / fm;
  float* rA1 = sm.rcp;    // m / c_i
  float* rA0 = rA1 + BT;  // m / (m - c_i)
  float* rB1 = rA0 + BT;  // 1 / c_j
  float* rB0 = rB1 + BT;  // 1 / (m - c_j)
  for (int c = tid; c < 2 * BT; c += C::NT) {
    const int v = sColA[c];  // sColA, then sColB
    const int w = P.m - v;
    if (c < BT) {
      rA1[c] = v > 0 ? fm / (float)v : 0.0f;
      rA0[c] = w > 0 ? fm / (float)w : 0.0f;
    } else {
      rB1[c - BT] = v > 0 ? 1.0f / (float)v : 0.0f;
      rB0[c - BT] = w > 0 ? 1.0f / (float)w : 0.0f;
    }
  }
  __syncthreads();
  const int ibase = I * BT + wm * C::WTM;  // first row and column of this wave's block
  const int jbase = J * BT + wn * C::WTN;
  if (ibase >= n || jbase >= n) return;  // the wave's block lies in tile padding (uniform)
  // Column factors of this lane's column in each fragment column block.
  int cjb[FN];
  float r1b[FN], r0b[FN];
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int jl = wn * C::WTN + blk_b(b) * 32 + (lane & 31);
    cjb[b] = sColB[jl];
    r1b[b] = rB1[jl];
    r0b[b] = rB0[jl];
  }
  // Addresses: a wave-uniform 64-bit base per group of rows plus this lane's
  // 32-bit byte offset (tile rows: row 4 (lane / 32), column lane % 32).  The
  // offsets stay below 2^32 for n below 2^25.
  const uint32_t lane_tile = (uint32_t)(((lane >> 5) * 4) * n + (lane & 31)) * 4u;
  const uint32_t lane_mir = (uint32_t)((lane & 31) * n + (lane >> 5) * 4) * 4u;
  const uint32_t row_bytes = (uint32_t)n * 4u;
  // 16-byte mirror stores need 16-byte aligned outputs and n % 4 == 0.
  const bool vec = (n & 3) == 0 && ((uintptr_t)P.out & 15) == 0 && ((uintptr_t)P.n11_out & 15) == 0;
  // A block strictly above the diagonal (every j > i) and inside the matrix
  // stores without per-element tests.
  const bool full = ibase + C::WTM <= n && jbase + C::WTN <= n && jbase >= ibase + C::WTM && vec;
  const bool mirror = !P.upper_only && (P.out || P.n11_out);
  // The FP32 mirror goes through LDS: a lane's registers 4 g .. 4 g + 3 are
  // four consecutive mirror columns of one mirror row, but 32 rows per store
  // would write a quarter of each 128-byte line per instruction (measured:
  // a third more bytes written than the output).  Half a 32 x 32 block at a
  // time (16 mirror rows, padded to 36 floats against bank conflicts) is
  // transposed in a per-wave LDS buffer and stored as whole rows, 8 lanes per
  // row.  The buffer is in the ring (128-wide tiles) or its own array.
  constexpr int kMirPitch = 36;
  float* mbuf = sm.mir ? sm.mir + wave * (16 * kMirPitch)
                       : reinterpret_cast<float*>(wave == 0 ? sm.slot[0] : (wave == 1 ? sm.slot[1] : (wave == 2 ? sm.slot[2] : sm.slot[3])));
  // Evaluate and store accumulator block rows [A0, A0 + 2).  The epilogue
  // mode and the block test are template arguments, so the FP32 path carries
  // neither mode tests nor bounds tests (the sparse output's too).  A scheduling barrier after each group of four rows
  // keeps the compiler from hoisting later groups' loads and arithmetic,
  // whose registers on top of the live accumulators would spill.
  auto emit_rows = [&](auto A0, auto EPI, auto FULL, auto PAIRS) {
    constexpr int epi = decltype(EPI)::value;
    constexpr bool fast = decltype(FULL)::value;
    constexpr bool pairs = decltype(PAIRS)::value;  // the sparse output's code is compiled in
#pragma unroll
    for (int a = decltype(A0)::value; a < decltype(A0)::value + 2 && a < FM; ++a) {
      if (ibase + blk_a(a) * 32 >= n) continue;  // block rows past n (uniform)
      const int ia = I * BT + wm * C::WTM + blk_a(a) * 32;  // first row of the block row
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int jb = jbase + blk_b(b) * 32;  // first column of the block
        const int j = jb + (lane & 31);
        if (jb >= n) continue;  // uniform
        v4f vs[4];  // this lane's values of register groups g = 0 .. 3
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          __builtin_amdgcn_sched_barrier(0);
          const int il = wm * C::WTM + blk_a(a) * 32 + g * 8 + (lane >> 5) * 4;  // tile row of register 4 g
          const int row0 = ia + g * 8;
          const int i0 = il + I * BT;
          const v4f a1 = *(const MI_LDS v4f*)(const MI_LDS float*)(rA1 + il);
          const v4f a0 = *(const MI_LDS v4f*)(const MI_LDS float*)(rA0 + il);
          const v4i ci = *(const MI_LDS v4i*)(const MI_LDS int32_t*)(sColA + il);
          v4f v;
          v4i c;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            c[q] = acc[a][b][4 * g + q];
            if (epi == kEpiCounts) {
              v[q] = 0.0f;
            } else if (epi == 2) {
              v[q] = mi_value64_call(P.m, ci[q], cjb[b], c[q]);
            } else {
              v[q] = mi_value32(P.m, ci[q], cjb[b], c[q], a1[q], a0[q], r1b[b], r0b[b], rfm);
              if (epi == 1 && v[q] < P.tau) v[q] = mi_value64_call(P.m, ci[q], cjb[b], c[q]);
            }
          }
          vs[g] = v;
          // Tile rows (i, j): two 128-byte half rows per store.  In a
          // diagonal tile only j >= i is stored; the mirror fills j < i.
          const int64_t tb = (int64_t)row0 * ln + jb;  // element (row0, jb)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = i0 + q;
            if (fast || (i < n && j < n && (!diag || j >= i))) {
              const uint32_t off = lane_tile + (uint32_t)q * row_bytes;
              if (P.out) *(float*)((char*)(P.out + tb) + off) = v[q];
              if (P.n11_out) *(int32_t*)((char*)(P.n11_out + tb) + off) = c[q];
            }
          }
          // The counts' mirror (j, i .. i + 3) directly (a rare output).
          if (mirror && P.n11_out) {
            const int64_t mb = (int64_t)jb * ln + row0;
            if (fast) {
              *(v4i*)((char*)(P.n11_out + mb) + lane_mir) = c;
            } else {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int i = i0 + q;
                if (i < n && j < n && (!diag || j > i)) *(int32_t*)((char*)(P.n11_out + mb) + lane_mir + 4u * q) = c[q];
              }
            }
          }
          if (pairs && P.pairs) {
            // Sparse output: pairs i < j at or above the threshold, one
            // atomic per wave and register.
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int i = i0 + q;
              const bool sel = (fast || (i < n && j < n && j > i)) && v[q] >= P.thr;
              const unsigned long long mask = __ballot(sel);
              if (mask) {  // uniform
                const int leader = __ffsll((long long)mask) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(P.pairs_count, (unsigned long long)__popcll(mask));
                base = __shfl(base, leader);
                if (sel) {
                  const unsigned long long idx = base + __popcll(mask & ((1ull << lane) - 1ull));
                  if (idx < (unsigned long long)P.pairs_cap) {
                    int32_t* e3 = P.pairs + 3 * idx;
                    e3[0] = i;
                    e3[1] = j;
                    e3[2] = __float_as_int(v[q]);
                  }
                }
              }
            }
          }
        }
        // The FP32 mirror of block (a, b): mirror rows jb .. jb + 31, columns
        // ia .. ia + 31, in two halves of 16 rows.  Lanes l and l + 32 hold
        // mirror row jb + l % 32; each writes its four 16-byte groups into
        // the buffer, then 8 lanes per row read whole rows and store them.
        // The lanes exchange data through LDS, so the compiler must not move
        // the reads above the other lanes' writes, nor the next half's writes
        // above this half's reads: a memory-clobbering wait orders both (LDS
        // operations of one wave then complete in order).
        if (mirror && P.out) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            if (((lane & 31) >> 4) == h) {
#pragma unroll
              for (int g = 0; g < 4; ++g)
                *(MI_LDS v4f*)(mbuf + (lane & 15) * kMirPitch + g * 8 + (lane >> 5) * 4) = vs[g];
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const int rr = k * 8 + (lane >> 3);  // buffer row
              const int jm = jb + h * 16 + rr;     // mirror row
              const int ic = ia + (lane & 7) * 4;  // first of its four columns
              const v4f t = *(const MI_LDS v4f*)(mbuf + rr * kMirPitch + (lane & 7) * 4);
              float* dst = P.out + (int64_t)jm * ln + ic;
              if (fast) {
                *(v4f*)dst = t;
              } else if (vec && jm < n && ic + 3 < n && (!diag || jm > ic + 3)) {
                *(v4f*)dst = t;
              } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  if (jm < n && ic + e < n && (!diag || jm > ic + e)) dst[e] = t[e];
              }
            }
          }
        }
      }
    }
  };
  // The FP32 and counts-only modes have both paths; the FP64 modes take the
  // tested one.  The FP32 fast path is compiled twice, with and without the
  // sparse output's code (which costs the dense path 1.5% when compiled in).
  const bool fast = full;
  auto rows_mode = [&](auto A0) {
    switch (P.epi) {
      case 0:
        if (fast && P.pairs) emit_rows(A0, std::integral_constant<int, 0>{}, std::true_type{}, std::true_type{});
        else if (fast) emit_rows(A0, std::integral_constant<int, 0>{}, std::true_type{}, std::false_type{});
        else emit_rows(A0, std::integral_constant<int, 0>{}, std::false_type{}, std::true_type{});
        break;
      case 1: emit_rows(A0, std::integral_constant<int, 1>{}, std::false_type{}, std::true_type{}); break;
      case 2: emit_rows(A0, std::integral_constant<int, 2>{}, std::false_type{}, std::true_type{}); break;
      default:  // counts only: no MI, no sparse output
        if (fast) emit_rows(A0, std::integral_constant<int, kEpiCounts>{}, std::true_type{}, std::false_type{});
        else emit_rows(A0, std::integral_constant<int, kEpiCounts>{}, std::false_type{}, std::false_type{});
        break;
    }
  };
  static_assert(FM == 2 || FM == 4, "block rows are evaluated two at a time");
  if constexpr (FM == 4) {
    // 128 accumulators plus the epilogue's working set exceed the two-wave
    // register budget: block rows 2 and 3 wait in LDS (the ring is free now;
    // 16 KB per wave, consecutive lanes on consecutive 16 bytes) while rows
    // 0 and 1 are evaluated.
    const int sl = wave >> 1;
    uint8_t* stash = (sl == 0 ? sm.slot[0] : (sl == 1 ? sm.slot[1] : (sl == 2 ? sm.slot[2] : sm.slot[3]))) +
                     (wave & 1) * 16384;
    static_assert(C::NWAVES <= 8 && C::STAGE >= 2 * 16384, "two 16 KB stashes per ring slot");
#pragma unroll
    for (int a = 2; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int g = 0; g < 4; ++g)
          *(MI_LDS v4i*)(stash + ((((a - 2) * FN + b) * 4 + g) * 64 + lane) * 16) =
              v4i{acc[a][b][4 * g], acc[a][b][4 * g + 1], acc[a][b][4 * g + 2], acc[a][b][4 * g + 3]};
    rows_mode(std::integral_constant<int, 0>{});
    // The stashed values must come back from LDS (no forwarding of the
    // stored registers, which would keep them live).
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int a = 2; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const v4i t = *(const MI_LDS v4i*)(stash + ((((a - 2) * FN + b) * 4 + g) * 64 + lane) * 16);
          acc[a][b][4 * g] = t.x;
          acc[a][b][4 * g + 1] = t.y;
          acc[a][b][4 * g + 2] = t.z;
          acc[a][b][4 * g + 3] = t.w;
        }
    rows_mode(std::integral_constant<int, 2>{});
  } else {
    rows_mode(std::integral_constant<int, 0>{});
  }
#endif
}

}  // namespace mi
