// mi_host.hpp -- host-runtime helpers shared by the C ABI and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "mi.h"
#include "mi_internal.hpp"

namespace mi {

mi_status fail(mi_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
const char* last_error();

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return ::mi::fail(MI_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct DeviceInfo {
  int device = 0;
  int cus = 0;
  int occ[kNumCfg] = {1, 1};   // plain kernel workgroups per CU, per configuration
  int pocc[kNumCfg][2] = {{1, 1}, {1, 1}};  // persistent kernel workgroups per CU [cfg][int8, FP4]
};

struct Plan {
  int cfg = 0;          // 0: 128 x 128 tiles, 1: 256 x 256 tiles
  int bt = 128;
  int ntp = 0;          // column panels
  int ntiles = 0;       // upper-triangular tiles
  int tpx = 0;          // tiles per XCD in the plain launch
  int64_t ksteps = 0;   // 64-row steps of a whole tile
  int splits = 1;       // equal K splits per tile
  int kchunk = 0;       // rows per split
};

mi_status device_info(DeviceInfo* out);
mi_status workspace(hipStream_t st, int slot, size_t bytes, void** out);  // zeroed split-K scratch
size_t workspace_bytes(const Plan& pl);
Plan make_plan(int64_t m, int64_t n, int cfg, int splits);
const int32_t* tile_table(int ntp, hipError_t* err);
// fp4: the plan of the FP4 Gram (heuristic only, at most 2^24 rows per unit).
mi_status choose_plan(int64_t m, int64_t n, bool aligned, int tile_req, int splits_req, Plan* out,
                      bool fp4 = false);
// The library's choice of the FP4 Gram for an m x n 0/1 problem.
bool fp4_preferred(int64_t m, int64_t n);
// Byte input that the dense path converts to FP4 first (requested, or the library's choice).
bool converts_to_fp4(const mi_problem* p);
// Bit input unpacked on chip to FP4 codes (requested, or the library's choice).
bool bits_to_fp4(const mi_problem* p);
// The problem runs the FP4 Gram (FP4 input, converted bytes or bits to FP4).
bool runs_fp4(const mi_problem* p);
// need_output: n > 0 needs out, n11_out or pairs (not for planning queries).
mi_status check_problem(const mi_problem* p, int64_t* ldx_out, bool need_output = true);
bool is_aligned(const uint8_t* X, int64_t ldx);
int64_t row_bytes(const mi_problem& p);
ProbDev make_probdev(const mi_problem* p, const uint8_t* X, int64_t ldx, const Plan& pl, void* ws,
                     const int32_t* tiles);
mi_status scratch(hipStream_t st, int kind, int slot, size_t bytes, void** out);
int64_t packed_pitch(int64_t n);
// upper_only: the fused kernel stores the i <= j half of n11_out and out only.
mi_status run_one(const mi_problem* p, hipStream_t st, int ws_slot, bool upper_only = false);
// Sparse-input path (mi_sparse.hip).  With auto_choice it first measures the
// density and returns with *used == false when the dense path is cheaper.
mi_status run_sparse(const mi_problem* p, int64_t ldx, hipStream_t st, bool auto_choice, bool* used);
void release_scratch_of(hipStream_t st);
void release_stream_resources(hipStream_t st);  // scratch and batch descriptors of a stream
// A persistent batch's plan (see plan_persistent in mi_api.hip).
struct BatchChoice {
  int tile = 0;        // 0: one tile by the work's majority width; MI_TILE_128 / _256; 3: by dataset width
  int narrow_n = 512;  // tile 3: datasets narrower than this take 128-wide tiles
  int fdiv = 1;        // K-split target: the batch's work over (persistent slots x fdiv)
};
// choice: the persistent mode's plan (nullptr: the tuned one for this batch, else the heuristic).
// plans_out: planning query (checks and plans only, nothing launched or allocated).
mi_status run_batched(const mi_problem* probs, int64_t count, hipStream_t st, int mode,
                      const BatchChoice* choice = nullptr, std::vector<Plan>* plans_out = nullptr);

}  // namespace mi
