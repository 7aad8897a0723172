// mi_internal.hpp -- declarations shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mi_device.hpp"

namespace mi {

// One entry of the persistent kernel's work list.
struct UnitRef {
  int32_t prob;
  int32_t tile;
  int32_t split;
  int32_t pad;
};

// One layout to repack into a 16-byte pitch (Y is m x ldy, ldy % 16 == 0).
struct RepackDesc {
  const uint8_t* X;
  int64_t ldx;
  uint8_t* Y;
  int64_t ldy;
  int64_t m, n;
  int64_t first_block;  // batched launch: first block of this layout
  int64_t blocks;       // blocks that work on this layout
  int32_t fp4;          // nonzero: convert bytes (n columns) to the FP4 layout instead of copying
  int32_t pad;
};

// Tile configurations: 0 = 128 x 128 (Cfg128), 1 = 256 x 256 (Cfg256).
constexpr int kNumCfg = 2;
int cfg_tile(int cfg);
int cfg_threads(int cfg);

hipError_t launch_plain(int cfg, const ProbDev& P, hipStream_t st);
hipError_t launch_persistent(int cfg, bool fp4, const ProbDev* probs, const UnitRef* units, int nunits, int* head,
                             int grid, hipStream_t st);
hipError_t launch_validate(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st);
hipError_t launch_validate_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, int* flag, hipStream_t st);
hipError_t launch_repack(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Y, int64_t ldy,
                         hipStream_t st);
hipError_t launch_repack_batch(const RepackDesc* descs, int count, int64_t blocks, hipStream_t st);
int64_t repack_blocks(int64_t m, int64_t ldy);
hipError_t launch_pack_bits(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xp, int64_t ldp,
                            hipStream_t st);
hipError_t launch_pack_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xq, int64_t ldq,
                           hipStream_t st);
hipError_t fill_i32(int* p, int v, int count, hipStream_t st);
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st);  // bytes a multiple of 4
hipError_t launch_fill_pattern(uint8_t* X, int64_t m, int64_t ld, int64_t bytes, bool fp4, hipStream_t st);
int occupancy(int cfg);
int persistent_occupancy(int cfg, bool fp4);

}  // namespace mi
