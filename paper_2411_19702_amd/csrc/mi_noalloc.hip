// mi_noalloc.hip -- mi_all_pairs_noalloc: the dense path of mi_all_pairs_ex
// with all of its library scratch in one fixed device array, for callers
// that cannot allocate device memory (code under stream capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The scratch of the dense path is
//   - the split-K workspace (per tile BT^2 partial counts, 2 BT partial column
//     sums, one arrival counter; the kernels leave it zeroed),
//   - the 0/1 validation flag,
//   - the tile-order table, which this path does without: the kernel decodes
//     each tile from its rank (morton_tile).
// Layouts that would need a copy (unaligned X, byte input converted to the
// FP4 layout) and the sparse-input algorithm are rejected instead.
#include <cstring>
#include <mutex>

#include "mi.h"
#include "mi_host.hpp"
#include "mi_internal.hpp"

namespace mi {
constexpr size_t kNoAllocFlagBytes = 256;
constexpr size_t kNoAllocWsBytes = (size_t)64 << 20;
constexpr size_t kNoAllocBytes = kNoAllocFlagBytes + kNoAllocWsBytes;
}  // namespace mi

// One copy per GPU that loads the library, held until the process ends.  In
// host code its name is a host-side stand-in: device code gets it only
// through the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[mi::kNoAllocBytes];

namespace mi {

constexpr int kMaxDevices = 64;
static std::mutex g_na_mu;
static void* g_na_ptr[kMaxDevices];  // device address of `scratch`, per device; nullptr: not set up

// The array's address on the current device.  First call on a device: look
// it up, then clear the workspace on `st` (a fill kernel, no memset node),
// ordered before the caller's kernels on that stream.
static mi_status noalloc_scratch(hipStream_t st, uint8_t** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MI_ERR_DEVICE, "device %d beyond the supported %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
    if (e != hipSuccess || !ptr) return fail(MI_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    HIPCHK(fill_i32(reinterpret_cast<int*>(ptr), 0, (int)(kNoAllocBytes / sizeof(int)), st));
    g_na_ptr[dev] = ptr;
  }
  *out = reinterpret_cast<uint8_t*>(g_na_ptr[dev]);
  return MI_OK;
}

static mi_status run_noalloc(const mi_problem* p, hipStream_t st) {
  int64_t ldx = 0;
  mi_status s = check_problem(p, &ldx);
  if (s != MI_OK) return s;
  if (p->algo != MI_ALGO_DENSE) return fail(MI_ERR_INVALID_ARG, "the no-allocation entry point runs the dense algorithm only");
  if (p->packed == MI_INPUT_BYTES && p->gram == MI_GRAM_FP4)
    return fail(MI_ERR_INVALID_ARG,
                "the no-allocation entry point does not convert bytes to the FP4 layout: pass FP4 input "
                "(mi_pack_fp4) or take the int8 Gram");
  if (p->n > 0 && !is_aligned(p->X, ldx))
    return fail(MI_ERR_INVALID_ARG, "the no-allocation entry point needs X 16-byte aligned and ldx %% 16 == 0");
  if (p->pairs) HIPCHK(fill_i32(reinterpret_cast<int*>(p->pairs_count), 0, 2, st));  // 64-bit counter
  if (p->n == 0) return MI_OK;
  uint8_t* base = nullptr;
  s = noalloc_scratch(st, &base);
  if (s != MI_OK) return s;
  if (p->validate && p->packed != MI_INPUT_BITS) {
    int* flag = reinterpret_cast<int*>(base);
    const bool fp4in = p->packed == MI_INPUT_FP4;
    HIPCHK(fp4in ? launch_validate_fp4(p->X, p->m, p->n, ldx, flag, st) : launch_validate(p->X, p->m, p->n, ldx, flag, st));
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h && fp4in) return fail(MI_ERR_NOT_BINARY, "X holds an FP4 code other than 0 and 0b0010 (1.0)");
    if (h) return fail(MI_ERR_NOT_BINARY, "X holds a byte other than 0 or 1");
  }
  // Byte input takes the int8 Gram here (no conversion pass); bits follow
  // the library's choice (unpacked on chip); FP4 input the FP4 Gram.
  mi_problem q = *p;
  if (q.packed == MI_INPUT_BYTES) q.gram = MI_GRAM_INT8;
  const bool bits4 = bits_to_fp4(&q);
  const bool fp4 = runs_fp4(&q);
  Plan pl;
  s = choose_plan(q.m, q.n, true, q.tile, q.splits, &pl, fp4);
  if (s != MI_OK) return s;
  if (workspace_bytes(pl) > kNoAllocWsBytes && q.splits <= 0) {
    // The library's split count needs more workspace than the array holds:
    // the fewest splits that keep FP4 counts exact (none for int8).
    pl = make_plan(q.m, q.n, pl.cfg, 1);
    while (fp4 && pl.kchunk > kFp4MaxUnitRows) pl = make_plan(q.m, q.n, pl.cfg, pl.splits + 1);
  }
  if (workspace_bytes(pl) > kNoAllocWsBytes)
    return fail(MI_ERR_INVALID_ARG,
                "%d splits of %d tiles need %zu bytes of split-K workspace; the no-allocation entry point has %zu",
                pl.splits, pl.ntiles, workspace_bytes(pl), kNoAllocWsBytes);
  ProbDev P = make_probdev(&q, p->X, ldx, pl, base + kNoAllocFlagBytes, /*tiles=*/nullptr);
  if (bits4) P.packed = kInBitsFp4;
  HIPCHK(launch_plain(pl.cfg, P, st));
  return MI_OK;
}

}  // namespace mi

extern "C" mi_status mi_all_pairs_noalloc(const mi_problem* p, void* stream) {
  mi::clear_error();
  return mi::run_noalloc(p, (hipStream_t)stream);
}
