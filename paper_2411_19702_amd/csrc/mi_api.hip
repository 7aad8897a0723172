// mi_api.hip -- the C ABI (include/mi.h): argument checks, planning, the
// split-K workspace, the batched modes and the autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mi.h"
#include "mi_internal.hpp"
#include "mi_host.hpp"

namespace mi {

// ------------------------------------------------------------------ errors --
static thread_local std::string g_err;

mi_status fail(mi_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

// ------------------------------------------------------------- device info --
static std::mutex g_info_mu;
static std::map<int, DeviceInfo> g_info;

mi_status device_info(DeviceInfo* out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_info_mu);
  auto it = g_info.find(dev);
  if (it == g_info.end()) {
    DeviceInfo di;
    di.device = dev;
    HIPCHK(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (int c = 0; c < kNumCfg; ++c) {
      di.occ[c] = occupancy(c);
      di.pocc[c][0] = persistent_occupancy(c, false);
      di.pocc[c][1] = persistent_occupancy(c, true);
    }
    it = g_info.emplace(dev, di).first;
  }
  *out = it->second;
  return MI_OK;
}

// ----------------------------------------------------------------- scratch --
// Device scratch keyed by (device, stream, kind, slot).  Work on one stream is
// ordered, so a buffer can be reused by the next call on the same stream.
//   kind 0: split-K workspace.  Kernels leave it zeroed again, so it is
//           cleared only when it is (re)allocated.
//   kind 1: repacked copies of inputs whose layout the DMA path cannot read.
//   kind 7: byte input converted to the FP4 layout for the FP4 Gram.
struct WsKey {
  int dev;
  hipStream_t st;
  int kind;
  int slot;
  bool operator<(const WsKey& o) const {
    return std::tie(dev, st, kind, slot) < std::tie(o.dev, o.st, o.kind, o.slot);
  }
};
struct WsBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};
static std::mutex g_ws_mu;
static std::map<WsKey, WsBuf> g_ws;

mi_status scratch(hipStream_t st, int kind, int slot, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return MI_OK;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ws_mu);
  WsBuf& w = g_ws[WsKey{dev, st, kind, slot}];
  if (w.bytes < bytes) {
    if (w.ptr) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    const size_t sz = std::max(bytes + bytes / 8, (size_t)1 << 20);
    if (hipMalloc(&w.ptr, sz) != hipSuccess) {
      (void)hipGetLastError();
      w.ptr = nullptr;
      return fail(MI_ERR_OUT_OF_MEMORY, "scratch allocation of %zu bytes failed", sz);
    }
    // Zeroed on the stream that uses it: a memset on the legacy default
    // stream is not ordered before kernels on a non-blocking stream (the
    // server's), which could then add into a workspace not yet cleared.
    if (kind == 0) HIPCHK(fill_zero(w.ptr, sz, st));
    w.bytes = sz;
  }
  *out = w.ptr;
  return MI_OK;
}

mi_status workspace(hipStream_t st, int slot, size_t bytes, void** out) { return scratch(st, 0, slot, bytes, out); }

void release_scratch_of(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto it = g_ws.begin(); it != g_ws.end();) {
    if (it->first.st == st) {
      (void)hipFree(it->second.ptr);
      it = g_ws.erase(it);
    } else {
      ++it;
    }
  }
}

int64_t packed_pitch(int64_t n) { return (n + 15) / 16 * 16; }

// --------------------------------------------------------------- tile order --
// Upper-triangular tiles (I <= J) sorted along a Morton curve of (I, J): a
// contiguous run of the order is a compact block of the triangle, so the
// tiles one XCD owns share few column panels.  One table per panel count.
static std::mutex g_tiles_mu;
static std::map<std::pair<int, int>, int32_t*> g_tiles;

static uint32_t morton2(uint32_t x, uint32_t y) {
  uint32_t r = 0;
  for (int b = 0; b < 16; ++b) r |= ((x >> b) & 1u) << (2 * b + 1) | ((y >> b) & 1u) << (2 * b);
  return r;
}

const int32_t* tile_table(int ntp, hipError_t* err) {
  *err = hipSuccess;
  int dev = 0;
  if ((*err = hipGetDevice(&dev)) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_tiles_mu);
  auto it = g_tiles.find({dev, ntp});
  if (it != g_tiles.end()) return it->second;
  std::vector<std::pair<uint32_t, int32_t>> order;
  order.reserve((size_t)ntp * (ntp + 1) / 2);
  for (int I = 0; I < ntp; ++I)
    for (int J = I; J < ntp; ++J) order.push_back({morton2((uint32_t)I, (uint32_t)J), (int32_t)((I << 16) | J)});
  std::sort(order.begin(), order.end());
  std::vector<int32_t> h(order.size());
  for (size_t k = 0; k < order.size(); ++k) h[k] = order[k].second;
  int32_t* d = nullptr;
  if ((*err = hipMalloc(&d, std::max<size_t>(h.size(), 1) * sizeof(int32_t))) != hipSuccess) return nullptr;
  if ((*err = hipMemcpy(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  g_tiles[{dev, ntp}] = d;
  return d;
}

// ----------------------------------------------------------------- planner --
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workspace of a plan with several K splits: per tile BT^2 int32 partial
// counts, then 2 BT partial column sums, then one arrival counter per tile.
size_t workspace_bytes(const Plan& pl) {
  if (pl.splits <= 1) return 0;
  const int64_t per = (int64_t)pl.bt * pl.bt + 2 * pl.bt + 1;
  return (size_t)(pl.ntiles * per * sizeof(int32_t) + 256);
}

Plan make_plan(int64_t m, int64_t n, int cfg, int splits) {
  Plan pl;
  pl.cfg = cfg;
  pl.bt = cfg_tile(cfg);
  pl.ntp = (int)cdiv(std::max<int64_t>(n, 1), pl.bt);
  pl.ntiles = pl.ntp * (pl.ntp + 1) / 2;
  pl.tpx = (int)cdiv(pl.ntiles, 8);
  pl.ksteps = cdiv(m, KT);
  if (splits < 1) splits = 1;
  if (splits > pl.ksteps) splits = (int)pl.ksteps;
  pl.kchunk = (int)(cdiv(pl.ksteps, splits) * KT);
  pl.splits = (int)cdiv(m, pl.kchunk);
  return pl;
}

// Heuristic when the tuner has no entry.  The plain grid is 8 * tpx * splits
// workgroups (tiles split evenly over the 8 XCDs), and one workgroup per CU
// keeps a CU's matrix cores and LDS busy (a second one per CU measured
// slower), so the launch runs in ceil(grid / CUs) waves of units.  A unit
// costs its rows plus, when the tile is split, about kPublishRows rows' worth
// of time to publish its partial counts (measured: ~20 us against ~0.6 us
// per 64-row step) while the workspace of partial sums stays in the
// last-level cache; a larger workspace sends the atomics to HBM, and the
// cost grows with its size (fitted on 100,000 x 8,192 and 100,000 x 16,384,
// whose workspaces are 138 MB and 545 MB: 3 and 1 splits measured best).
// Pick the split count with the least modelled time, keeping at least
// kMinRows rows per split.
// With the FP4 Gram a row costs about half as much (rows_per_step_time = 2),
// so publishing costs twice as many rows' worth.
static int heuristic_splits(int64_t m, const Plan& p1, int cus, double rows_per_step_time = 1.0) {
  const int64_t kMinRows = 4096;
  const double ws_bytes = (double)p1.ntiles * p1.bt * p1.bt * 4.0;
  const double kPublishRows = rows_per_step_time * 2048.0 * std::max(1.0, ws_bytes / (64.0 * 1048576.0));
  const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(512, m / kMinRows));
  int best = 1;
  double best_t = 1e300;
  for (int64_t s = 1; s <= smax; ++s) {
    const double waves = std::ceil(8.0 * p1.tpx * (double)s / cus);
    const double rows = (double)cdiv(p1.ksteps, s) * KT + (s > 1 ? kPublishRows : 0.0);
    const double t = waves * rows;
    if (t < best_t * 0.99) {  // prefer fewer splits unless clearly faster
      best_t = t;
      best = (int)s;
    }
  }
  // 128-wide tiles fit two workgroups on a CU, and split units that share a
  // CU measured slower than fewer, longer units each on a CU of its own:
  // at most one unit per CU, and for short units (under 32,768 rows) at most
  // 7/8 of the CUs.  Measured (ms, heuristic before -> with these caps):
  // 1,000,000 x 1,024 1.213 -> 0.930 (19 -> 6 splits; 5: 1.000),
  // 100,000 x 1,024 0.123 -> 0.105 (6 -> 5), 100,000 x 1,400 on the FP4
  // Gram 0.240 -> 0.197 (7 -> 3), 100,000 x 512 0.085 -> 0.082 (16 -> 14),
  // 200,000 x 768 0.138 against 0.140 (10 -> 9); 300,000 x 1,024 keeps 6
  // (0.300; 5: 0.320).
  if (p1.bt == 128) {
    while (best > 1 && 8 * (int64_t)p1.tpx * best > cus) --best;
    if (cdiv(p1.ksteps, best) * KT < 32768)
      while (best > 1 && 64 * (int64_t)p1.tpx * best > 7 * (int64_t)cus) --best;
  }
  return best;
}

// 256-wide tiles halve the panel traffic per MAC, but need enough tiles to
// occupy the chip, and with few rows the per-tile epilogue (MI of BT^2 pairs
// and their mirror) dominates the tile's time: 128-wide tiles, two
// workgroups per CU, then overlap one tile's epilogue with another's Gram
// steps (measured 1.24x faster at 2,000 x 8,192).
static int heuristic_cfg(int64_t m, int64_t n) { return (n >= 1536 && m >= 16384) ? 1 : 0; }

// Tuned entries, keyed by a shape class: m in quarter octaves, n in 64-column
// steps, whether the fast aligned load path applies, and the Gram (FP4
// entries time the converted, always aligned, layout).
struct ShapeKey {
  int mb, nb, aligned, fp4;
  bool operator<(const ShapeKey& o) const {
    return std::tie(mb, nb, aligned, fp4) < std::tie(o.mb, o.nb, o.aligned, o.fp4);
  }
};
struct Tuned {
  int cfg, splits;
  double ms;
};
static std::mutex g_tune_mu;
static std::map<ShapeKey, Tuned> g_tuned;

static ShapeKey shape_key(int64_t m, int64_t n, bool aligned, bool fp4) {
  ShapeKey k;
  k.mb = (int)std::lround(4.0 * std::log2((double)std::max<int64_t>(m, 1)));
  k.nb = (int)cdiv(n, 64);
  k.aligned = (aligned || fp4) ? 1 : 0;
  k.fp4 = fp4 ? 1 : 0;
  return k;
}

mi_status choose_plan(int64_t m, int64_t n, bool aligned, int tile_req, int splits_req, Plan* out, bool fp4) {
  DeviceInfo di;
  mi_status s = device_info(&di);
  if (s != MI_OK) return s;
  int cfg = tile_req == MI_TILE_256 ? 1 : (tile_req == MI_TILE_128 ? 0 : -1);
  int splits = splits_req;
  if (splits <= 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(shape_key(m, n, aligned, fp4));
    if (it != g_tuned.end() && (cfg < 0 || cfg == it->second.cfg)) {
      cfg = it->second.cfg;
      splits = it->second.splits;
    }
  }
  if (cfg < 0) cfg = heuristic_cfg(m, n);
  if (splits <= 0) splits = heuristic_splits(m, make_plan(m, n, cfg, 1), di.cus, fp4 ? 2.0 : 1.0);
  *out = make_plan(m, n, cfg, splits);
  // FP4 units accumulate in FP32: at most 2^24 rows each (more splits if needed).
  while (fp4 && out->kchunk > kFp4MaxUnitRows) *out = make_plan(m, n, cfg, out->splits + 1);
  return MI_OK;
}

// The FP4 Gram for byte input when the library chooses.  The conversion pass
// (read the input, write half of it) costs one launch plus m n 1.5 B at HBM
// speed; the FP4 Gram halves the row steps and runs its instruction ~1.7x
// faster.  Measured (conversion included, against the int8 Gram): 0.95-0.98x
// up to m n^2 ~ 3.4e10 (2,000 x 4,096; 5,000 x 2,048), 1.00x at 1.7e11
// (10,000 x 4,096), 1.06-1.07x from 6.7e10 (1,000 x 8,192; 20,000 x 2,048),
// 1.33x at 50,000 x 4,096 and 1,000,000 x 4,096 (1.25x); at 1,024 columns
// the two tie (100,000 x 1,024).
bool fp4_preferred(int64_t m, int64_t n) { return n >= 1536 && (double)m * (double)n * (double)n >= 6.0e10; }

// Byte input converted to the FP4 layout first (requested, or the library's
// choice).  A layout that the DMA path cannot read (X not 16-byte aligned or
// ldx % 16 != 0) needs a copy anyway: the conversion writes half the bytes of
// a repack and the FP4 Gram that follows is the faster one, so the library
// converts such layouts at every shape.
bool converts_to_fp4(const mi_problem* p) {
  if (p->packed != MI_INPUT_BYTES) return false;
  if (p->gram == MI_GRAM_FP4) return true;
  if (p->gram != MI_GRAM_AUTO) return false;
  const int64_t ldx = p->ldx == 0 ? p->n : p->ldx;
  return fp4_preferred(p->m, p->n) || !is_aligned(p->X, ldx);
}

// Bit-packed input unpacked on chip to FP4 codes: requested, or the
// library's choice from 512 columns on.  No conversion pass is needed, and
// each stage carries twice the rows: measured against unpacking to bytes for
// the int8 Gram, 3.89 against 6.72 ms at 1,000,000 x 4,096, 0.113 against
// 0.148 ms at 100,000 x 1,024, 0.176 against 0.205 ms at 2,000 x 8,192.
bool bits_to_fp4(const mi_problem* p) {
  return p->packed == MI_INPUT_BITS && (p->gram == MI_GRAM_FP4 || (p->gram == MI_GRAM_AUTO && p->n >= 512));
}

// The problem runs the FP4 Gram.
bool runs_fp4(const mi_problem* p) {
  return converts_to_fp4(p) || p->packed == MI_INPUT_FP4 || bits_to_fp4(p);
}

// -------------------------------------------------------------- arguments --
// Rows of one 64-row stage are addressed with 32-bit offsets.
static constexpr int64_t kMaxPitch = (int64_t)1 << 24;
static constexpr int64_t kMaxCols = (int64_t)32767 * 128;
mi_status check_problem(const mi_problem* p, int64_t* ldx_out, bool need_output) {
  if (!p) return fail(MI_ERR_INVALID_ARG, "problem is NULL");
  if (p->m <= 0) return fail(MI_ERR_INVALID_ARG, "m must be >= 1 (got %lld)", (long long)p->m);
  if (p->m > INT32_MAX) return fail(MI_ERR_INVALID_ARG, "m must be <= 2^31-1 (int32 counts), got %lld", (long long)p->m);
  if (p->n < 0) return fail(MI_ERR_INVALID_ARG, "n must be >= 0 (got %lld)", (long long)p->n);
  // Tiles are encoded as (I << 16) | J in int32, so at most 32,767 column
  // panels of the narrowest (128-wide) tile.
  if (p->n > kMaxCols)
    return fail(MI_ERR_INVALID_ARG, "n must be <= %lld (got %lld)", (long long)kMaxCols, (long long)p->n);
  const int64_t rb = row_bytes(*p);
  const int64_t ldx = p->ldx == 0 ? rb : p->ldx;
  if (ldx < rb) return fail(MI_ERR_INVALID_ARG, "ldx (%lld) < %lld bytes of a row", (long long)ldx, (long long)rb);
  if (p->packed < MI_INPUT_BYTES || p->packed > MI_INPUT_FP4)
    return fail(MI_ERR_INVALID_ARG, "bad input layout (packed = %d)", p->packed);
  if (p->gram < MI_GRAM_AUTO || p->gram > MI_GRAM_FP4) return fail(MI_ERR_INVALID_ARG, "bad gram %d", p->gram);
  if (p->packed == MI_INPUT_FP4 && p->gram == MI_GRAM_INT8)
    return fail(MI_ERR_INVALID_ARG, "FP4 input takes the FP4 Gram");
  if (p->packed && p->algo != MI_ALGO_DENSE)
    return fail(MI_ERR_INVALID_ARG, "packed input takes only the dense algorithm");
  if (p->gram == MI_GRAM_FP4 && p->algo == MI_ALGO_SPARSE)
    return fail(MI_ERR_INVALID_ARG, "the FP4 Gram is a dense-algorithm choice");
  if (ldx > kMaxPitch) return fail(MI_ERR_INVALID_ARG, "ldx (%lld) above the supported 2^24", (long long)ldx);
  // 128-row FP4 stages are addressed with 32-bit offsets.
  if (p->packed == MI_INPUT_FP4 && ldx > kMaxPitch / 2)
    return fail(MI_ERR_INVALID_ARG, "ldx (%lld) above the supported 2^23 for FP4 input", (long long)ldx);
  if (p->n > 0 && !p->X) return fail(MI_ERR_INVALID_ARG, "X must be non-NULL when n > 0");
  if (need_output && p->n > 0 && !p->out && !p->pairs && !p->n11_out)
    return fail(MI_ERR_INVALID_ARG, "out, n11_out or the sparse pairs output must be given when n > 0");
  if (p->algo < MI_ALGO_DENSE || p->algo > MI_ALGO_AUTO) return fail(MI_ERR_INVALID_ARG, "bad algo %d", p->algo);
  if (p->pairs && (!p->pairs_count || p->pairs_capacity < 0 || !std::isfinite(p->pairs_threshold)))
    return fail(MI_ERR_INVALID_ARG, "pairs needs pairs_count, pairs_capacity >= 0 and a finite threshold");

  if (p->epilogue < 0 || p->epilogue > 2) return fail(MI_ERR_INVALID_ARG, "bad epilogue mode %d", p->epilogue);
  if (p->tile < 0 || p->tile > 2) return fail(MI_ERR_INVALID_ARG, "bad tile id %d", p->tile);
  if (p->splits < 0) return fail(MI_ERR_INVALID_ARG, "splits must be >= 0");
  *ldx_out = ldx;
  return MI_OK;
}

bool is_aligned(const uint8_t* X, int64_t ldx) { return ((uintptr_t)X % 16 == 0) && (ldx % 16 == 0); }

// Bytes of a row that hold columns: n, ceil(n / 8) for bit-packed input,
// ceil(n / 2) for FP4 input.
int64_t row_bytes(const mi_problem& p) {
  return p.packed == MI_INPUT_BITS ? (p.n + 7) / 8 : (p.packed == MI_INPUT_FP4 ? (p.n + 1) / 2 : p.n);
}

ProbDev make_probdev(const mi_problem* p, const uint8_t* X, int64_t ldx, const Plan& pl, void* ws,
                     const int32_t* tiles) {
  ProbDev P;
  std::memset(&P, 0, sizeof P);
  P.X = X;
  P.ldx = ldx;
  P.m = (int32_t)p->m;
  P.n = (int32_t)p->n;
  P.out = p->out;
  P.pairs = reinterpret_cast<int32_t*>(p->pairs);
  P.pairs_cap = p->pairs_capacity;
  P.pairs_count = p->pairs_count;
  P.thr = p->pairs_threshold;
  P.n11_out = p->n11_out;
  P.colsum_out = p->colsum_out;
  P.tiles = tiles;
  P.ntp = pl.ntp;
  P.ntiles = pl.ntiles;
  P.ksteps = (int32_t)pl.ksteps;
  P.kchunk = pl.kchunk;
  P.epi = (!p->out && !p->pairs) ? kEpiCounts : p->epilogue;  // counts alone: no MI evaluated
  P.packed = p->packed;
  P.tau = p->fallback_tau > 0.0f ? p->fallback_tau : 1e-3f;
  P.splits = pl.splits;
  P.tiles_per_xcd = pl.tpx;
  if (pl.splits > 1 && ws) {
    int32_t* base = reinterpret_cast<int32_t*>(ws);
    P.ws_n11 = base;
    P.ws_col = base + (int64_t)pl.ntiles * pl.bt * pl.bt;
    P.counters = P.ws_col + (int64_t)pl.ntiles * 2 * pl.bt;
  }
  return P;
}

static std::mutex g_flag_mu;
static std::map<int, int*> g_flag;

mi_status validate_binary(const mi_problem* p, int64_t ldx, hipStream_t st) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int* flag = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_flag_mu);
    int*& f = g_flag[dev];
    if (!f) HIPCHK(hipMalloc(&f, 256));
    flag = f;
  }
  const bool fp4 = p->packed == MI_INPUT_FP4;
  HIPCHK(fp4 ? launch_validate_fp4(p->X, p->m, p->n, ldx, flag, st) : launch_validate(p->X, p->m, p->n, ldx, flag, st));
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h && fp4) return fail(MI_ERR_NOT_BINARY, "X holds an FP4 code other than 0 and 0b0010 (1.0)");
  if (h) return fail(MI_ERR_NOT_BINARY, "X holds a byte other than 0 or 1");
  return MI_OK;
}

mi_status run_one(const mi_problem* p, hipStream_t st, int ws_slot, bool upper_only) {
  int64_t ldx = 0;
  mi_status s = check_problem(p, &ldx);
  if (s != MI_OK) return s;
  if (p->pairs) HIPCHK(fill_i32(reinterpret_cast<int*>(p->pairs_count), 0, 2, st));  // 64-bit counter
  if (p->n == 0) return MI_OK;
  if (p->validate && p->packed != MI_INPUT_BITS) {  // packed bits are 0 or 1 by construction
    s = validate_binary(p, ldx, st);
    if (s != MI_OK) return s;
  }
  if (p->algo != MI_ALGO_DENSE) {
    bool used = false;
    s = run_sparse(p, ldx, st, p->algo == MI_ALGO_AUTO, &used);
    if (s != MI_OK || used) return s;
  }
  const bool aligned = is_aligned(p->X, ldx);
  const bool convert = converts_to_fp4(p);
  const bool fp4 = runs_fp4(p);
  Plan pl;
  s = choose_plan(p->m, p->n, aligned || convert, p->tile, p->splits, &pl, fp4);
  if (s != MI_OK) return s;
  const uint8_t* X = p->X;
  int64_t ld = ldx;
  mi_problem q = *p;  // the problem as the kernel sees it
  if (convert) {
    q.packed = MI_INPUT_FP4;
    ld = packed_pitch(row_bytes(q));
    void* buf = nullptr;
    s = scratch(st, 7, ws_slot, (size_t)p->m * (size_t)ld, &buf);
    if (s != MI_OK) return s;
    HIPCHK(launch_pack_fp4(p->X, p->m, p->n, ldx, (uint8_t*)buf, ld, st));
    X = (const uint8_t*)buf;
  } else if (!aligned) {
    ld = packed_pitch(row_bytes(*p));
    void* buf = nullptr;
    s = scratch(st, 1, ws_slot, (size_t)p->m * (size_t)ld, &buf);
    if (s != MI_OK) return s;
    HIPCHK(launch_repack(p->X, p->m, row_bytes(*p), ldx, (uint8_t*)buf, ld, st));
    X = (const uint8_t*)buf;
  }
  void* ws = nullptr;
  s = workspace(st, ws_slot, workspace_bytes(pl), &ws);
  if (s != MI_OK) return s;
  hipError_t e;
  const int32_t* tiles = tile_table(pl.ntp, &e);
  if (!tiles) return fail(MI_ERR_DEVICE, "tile table: %s", hipGetErrorString(e));
  ProbDev P = make_probdev(&q, X, ld, pl, ws, tiles);
  if (bits_to_fp4(p)) P.packed = kInBitsFp4;
  P.upper_only = upper_only ? 1 : 0;
  HIPCHK(launch_plain(pl.cfg, P, st));
  return MI_OK;
}

// ----------------------------------------------------------------- batched --
struct BatchBufs {
  void* dev = nullptr;  // ProbDev[count] + UnitRef[units] + heads
  size_t dev_bytes = 0;
  void* host = nullptr;  // pinned staging
  size_t host_bytes = 0;
  hipEvent_t copied = nullptr;
};
static std::mutex g_batch_mu;
static std::map<std::pair<int, hipStream_t>, BatchBufs> g_batch;

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
};
static std::mutex g_graph_mu;
static std::map<std::string, GraphEntry> g_graphs;
static std::map<int, hipStream_t> g_capture_stream;
static std::mutex g_capture_mu;

static std::string batch_key(const mi_problem* probs, int64_t count, const std::vector<Plan>& plans, hipStream_t st) {
  std::string k;
  char buf[256];
  snprintf(buf, sizeof buf, "%p|%lld|", (void*)st, (long long)count);
  k += buf;
  for (int64_t d = 0; d < count; ++d) {
    const mi_problem& p = probs[d];
    snprintf(buf, sizeof buf, "%p,%lld,%lld,%lld,%p,%p,%p,%d,%g,%d,%d,%p,%lld,%p,%a;", (const void*)p.X,
             (long long)p.m, (long long)p.n, (long long)p.ldx, (void*)p.out, (void*)p.n11_out, (void*)p.colsum_out,
             p.epilogue, (double)p.fallback_tau, plans[d].cfg, plans[d].splits, (void*)p.pairs,
             (long long)p.pairs_capacity, (void*)p.pairs_count, (double)p.pairs_threshold);
    k += buf;
    snprintf(buf, sizeof buf, "%d,%d,%d,%d;", p.packed, p.gram, converts_to_fp4(&p) ? 1 : 0, runs_fp4(&p) ? 1 : 0);
    k += buf;
  }
  return k;
}


// ------------------------------------------------------- persistent batches --
// How a persistent batch is planned: the tile of the datasets whose tile is
// left to the library, and the K-split target.
//   tile kBatchTileAuto: one tile for all of them, 256-wide unless most of
//        the work (m n^2) is in datasets narrower than 512 columns;
//   MI_TILE_128 / MI_TILE_256: that tile for all of them;
//   kBatchTileByWidth: 128-wide below narrow_n columns, 256-wide from there
//        (two launches, one per tile).
//   fdiv: each dataset is split so that no unit is much larger than the
//        batch's MAC work over (persistent slots x fdiv); units of very
//        different datasets then balance in the dynamic queue.
// The heuristic is {kBatchTileAuto, 512, 1} (units at most one slot's share:
// with splits published by atomics and units sorted by decreasing rows, fewer
// and larger units measured faster); the batch tuner (mi_tune_batched)
// times candidates on the caller's batch and stores the fastest under the
// batch's signature.
constexpr int kBatchTileAuto = 0, kBatchTileByWidth = 3;

static BatchChoice heuristic_batch_choice() { return BatchChoice{kBatchTileAuto, 512, 1}; }

// Batch signature: the multiset of the datasets' shape classes (the single
// tuner's m and n classes), layouts, Gram choices and explicit tile / split
// requests, hashed (FNV-1a, 64 bits) in sorted order.
static uint64_t batch_signature(const mi_problem* probs, int64_t count, const std::vector<char>& aligned,
                                const std::vector<char>& f4) {
  std::vector<std::tuple<int, int, int, int, int, int, int>> keys;
  keys.reserve(count);
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0) continue;
    const ShapeKey k = shape_key(probs[d].m, probs[d].n, aligned[d] != 0, f4[d] != 0);
    keys.emplace_back(k.mb, k.nb, k.aligned, k.fp4, probs[d].packed, probs[d].tile, probs[d].splits);
  }
  std::sort(keys.begin(), keys.end());
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (uint64_t)((uint32_t)v >> (8 * b)) & 0xFFu;
      h *= 1099511628211ull;
    }
  };
  mix((int)keys.size());
  for (const auto& k : keys) {
    mix(std::get<0>(k)); mix(std::get<1>(k)); mix(std::get<2>(k)); mix(std::get<3>(k));
    mix(std::get<4>(k)); mix(std::get<5>(k)); mix(std::get<6>(k));
  }
  return h;
}

static std::map<uint64_t, std::pair<BatchChoice, double>> g_batch_tuned;  // under g_tune_mu

static BatchChoice batch_choice(const mi_problem* probs, int64_t count, const std::vector<char>& aligned,
                                const std::vector<char>& f4) {
  const uint64_t sig = batch_signature(probs, count, aligned, f4);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_batch_tuned.find(sig);
  return it != g_batch_tuned.end() ? it->second.first : heuristic_batch_choice();
}

static mi_status plan_persistent(const mi_problem* probs, int64_t count, const std::vector<char>& aligned,
                                 const std::vector<char>& conv, const std::vector<char>& f4, const BatchChoice& ch,
                                 const DeviceInfo& di, std::vector<Plan>& plans) {
  int batch_tile = ch.tile;
  if (batch_tile == kBatchTileAuto) {
    // In a shared work queue the 256-wide tiles measured faster even for
    // small datasets (5.6 ms against 8.3 ms for the 256-dataset mix), so they
    // are used unless most of the work is in datasets narrower than 512
    // columns, which would mostly compute padding.
    double wide = 0.0, narrow = 0.0;
    for (int64_t d = 0; d < count; ++d) {
      if (probs[d].n == 0 || probs[d].tile != MI_TILE_AUTO) continue;
      const double w = (double)probs[d].m * (double)probs[d].n * (double)probs[d].n;
      (probs[d].n >= 512 ? wide : narrow) += w;
    }
    batch_tile = wide >= narrow ? MI_TILE_256 : MI_TILE_128;
  }
  double total = 0.0;
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0) continue;
    int tile = probs[d].tile;
    if (tile == MI_TILE_AUTO)
      tile = batch_tile == kBatchTileByWidth ? (probs[d].n < ch.narrow_n ? MI_TILE_128 : MI_TILE_256) : batch_tile;
    Plan p0;
    mi_status s = choose_plan(probs[d].m, probs[d].n, aligned[d] || conv[d], tile, 1, &p0, f4[d]);
    if (s != MI_OK) return s;
    total += (double)p0.ntiles * p0.bt * p0.bt * (double)probs[d].m;
    plans[d] = p0;
  }
  const double slots = (double)di.cus * di.pocc[0][0];
  const double target = std::max(total / (slots * std::max(ch.fdiv, 1)), 1.0);
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0) continue;
    int sp = probs[d].splits;
    if (sp <= 0) {
      const double unit = (double)plans[d].bt * plans[d].bt * (double)probs[d].m;
      sp = (int)std::min<double>(std::ceil(unit / target), std::max<int64_t>(1, probs[d].m / 1024));
      sp = std::max(sp, 1);
    }
    plans[d] = make_plan(probs[d].m, probs[d].n, plans[d].cfg, sp);
    while (f4[d] && plans[d].kchunk > kFp4MaxUnitRows)  // exact FP32 counts
      plans[d] = make_plan(probs[d].m, probs[d].n, plans[d].cfg, plans[d].splits + 1);
  }
  return MI_OK;
}

// The Gram of each dataset of a batch (conv: converted from bytes first; f4:
// runs the FP4 Gram), by each problem's own choice.  In the persistent mode
// each Gram is one more launch whose tail the batch waits for, so when the
// datasets on the FP4 Gram hold at least half of the batch's pair-updates,
// the byte datasets left to the library run it too (their conversion joins
// the batch's one conversion launch; the outputs are the same either way).
// On the 256-dataset recipe that moves the 11 aligned datasets (1.5% of the
// pair-updates) off a second launch of 0.2 ms: 3.16 -> 3.04 ms.
static void batch_grams(const mi_problem* probs, int64_t count, bool persistent, std::vector<char>& conv,
                        std::vector<char>& f4) {
  conv.assign(count, 0);
  f4.assign(count, 0);
  double pu_all = 0.0, pu_f4 = 0.0;
  for (int64_t d = 0; d < count; ++d) {
    conv[d] = converts_to_fp4(&probs[d]) ? 1 : 0;
    f4[d] = runs_fp4(&probs[d]) ? 1 : 0;
    const double n = (double)std::max<int64_t>(probs[d].n, 0);
    const double pu = (double)probs[d].m * n * (n + 1.0) / 2.0;
    pu_all += pu;
    if (f4[d]) pu_f4 += pu;
  }
  if (!persistent || pu_f4 < 0.5 * pu_all) return;
  for (int64_t d = 0; d < count; ++d)
    if (!f4[d] && probs[d].n > 0 && probs[d].packed == MI_INPUT_BYTES && probs[d].gram == MI_GRAM_AUTO)
      conv[d] = f4[d] = 1;
}

mi_status run_batched(const mi_problem* probs, int64_t count, hipStream_t st, int mode, const BatchChoice* choice,
                      std::vector<Plan>* plans_out) {
  if (count < 0) return fail(MI_ERR_INVALID_ARG, "count < 0");
  if (count == 0) return MI_OK;
  if (!probs) return fail(MI_ERR_INVALID_ARG, "probs is NULL");
  if (mode < 0 || mode > 2) return fail(MI_ERR_INVALID_ARG, "bad batch mode %d", mode);
  if (count > INT32_MAX / 4) return fail(MI_ERR_INVALID_ARG, "count too large");
  std::vector<int64_t> ldx(count);
  std::vector<Plan> plans(count);
  mi_status s = MI_OK;
  for (int64_t d = 0; d < count; ++d) {
    s = check_problem(&probs[d], &ldx[d]);
    if (s != MI_OK) {
      const std::string why = last_error();
      return fail(s, "problem %lld: %s", (long long)d, why.c_str());
    }
    if (probs[d].validate) return fail(MI_ERR_INVALID_ARG, "problem %lld: validate is not supported in batches", (long long)d);
    if (probs[d].algo != MI_ALGO_DENSE)
      return fail(MI_ERR_INVALID_ARG, "problem %lld: batches take only the dense algorithm", (long long)d);
    if (probs[d].packed == MI_INPUT_BITS && mode == MI_BATCH_PERSISTENT)
      return fail(MI_ERR_INVALID_ARG, "problem %lld: the persistent mode takes bytes or FP4 input, not bits",
                  (long long)d);
  }
  // Per dataset: converted from bytes to the FP4 layout first, and run on the FP4 Gram.
  std::vector<char> conv, f4;
  batch_grams(probs, count, mode == MI_BATCH_PERSISTENT, conv, f4);
  DeviceInfo di;
  s = device_info(&di);
  if (s != MI_OK) return s;
  std::vector<char> aligned(count);
  for (int64_t d = 0; d < count; ++d) aligned[d] = is_aligned(probs[d].X, ldx[d]) ? 1 : 0;

  if (mode == MI_BATCH_PERSISTENT) {
    BatchChoice ch = choice ? *choice : batch_choice(probs, count, aligned, f4);
    s = plan_persistent(probs, count, aligned, conv, f4, ch, di, plans);
    if (s != MI_OK) return s;
  } else {
    for (int64_t d = 0; d < count; ++d) {
      if (probs[d].n == 0) continue;
      s = choose_plan(probs[d].m, probs[d].n, aligned[d] || conv[d], probs[d].tile, probs[d].splits, &plans[d],
                      f4[d]);
      if (s != MI_OK) return s;
    }
  }
  if (plans_out) {  // planning query: nothing launched
    *plans_out = plans;
    return MI_OK;
  }

  // One split-K workspace and one buffer for the repacked and converted
  // inputs hold every dataset's region.  ld_in[d]: the pitch the kernel reads.
  std::vector<size_t> ws_off(count, 0), rp_off(count, 0);
  std::vector<int64_t> ld_in(count, 0);
  size_t ws_total = 0, rp_total = 0;
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0) continue;
    ws_off[d] = ws_total;
    ws_total += (workspace_bytes(plans[d]) + 255) & ~(size_t)255;
    ld_in[d] = conv[d] ? packed_pitch((probs[d].n + 1) / 2) : (aligned[d] ? ldx[d] : packed_pitch(row_bytes(probs[d])));
    if (conv[d] || !aligned[d]) {
      rp_off[d] = rp_total;
      rp_total += ((size_t)probs[d].m * (size_t)ld_in[d] + 255) & ~(size_t)255;
    }
  }
  void* ws = nullptr;
  void* rp = nullptr;
  s = workspace(st, 1, ws_total, &ws);
  if (s != MI_OK) return s;
  s = scratch(st, 1, 1, rp_total, &rp);
  if (s != MI_OK) return s;
  std::vector<ProbDev> P(count);
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0) continue;
    hipError_t e;
    const int32_t* tiles = tile_table(plans[d].ntp, &e);
    if (!tiles) return fail(MI_ERR_DEVICE, "tile table: %s", hipGetErrorString(e));
    const uint8_t* X = (aligned[d] && !conv[d]) ? probs[d].X : (const uint8_t*)rp + rp_off[d];
    mi_problem q = probs[d];  // the problem as the kernel sees it
    if (conv[d]) q.packed = MI_INPUT_FP4;
    P[d] = make_probdev(&q, X, ld_in[d], plans[d], ws ? (char*)ws + ws_off[d] : nullptr, tiles);
    if (bits_to_fp4(&probs[d])) P[d].packed = kInBitsFp4;
  }
  // The input staging of dataset d (conversion or repack), if it has one.
  auto stage_input = [&](int64_t d, hipStream_t s_) -> hipError_t {
    if (conv[d]) return launch_pack_fp4(probs[d].X, probs[d].m, probs[d].n, ldx[d], (uint8_t*)P[d].X, P[d].ldx, s_);
    if (!aligned[d])
      return launch_repack(probs[d].X, probs[d].m, row_bytes(probs[d]), ldx[d], (uint8_t*)P[d].X, P[d].ldx, s_);
    return hipSuccess;
  };
  auto repack_all = [&]() -> hipError_t {
    for (int64_t d = 0; d < count; ++d) {
      if (probs[d].n == 0) continue;
      hipError_t e = stage_input(d, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };

  if (mode == MI_BATCH_SEQUENTIAL) {
    HIPCHK(repack_all());
    for (int64_t d = 0; d < count; ++d) {
      if (probs[d].pairs) HIPCHK(fill_i32(reinterpret_cast<int*>(probs[d].pairs_count), 0, 2, st));
      if (probs[d].n > 0) HIPCHK(launch_plain(plans[d].cfg, P[d], st));
    }
    return MI_OK;
  }

  if (mode == MI_BATCH_GRAPH) {
    // The captured launches bake in the workspace and repack addresses, so
    // they are part of the cache key: a reallocated buffer means a new graph.
    char extra[96];
    snprintf(extra, sizeof extra, "|ws=%p|rp=%p", ws, rp);
    const std::string key = batch_key(probs, count, plans, st) + extra;
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_graph_mu);
      auto it = g_graphs.find(key);
      if (it != g_graphs.end()) exec = it->second.exec;
    }
    if (!exec) {
      // Capture on a private stream (the caller's may be the legacy default
      // stream, which cannot be captured); the graph is launched on st.
      hipStream_t cap = nullptr;
      {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        hipStream_t& c = g_capture_stream[di.device];
        if (!c) HIPCHK(hipStreamCreateWithFlags(&c, hipStreamNonBlocking));
        cap = c;
      }
      std::lock_guard<std::mutex> cap_lk(g_capture_mu);  // one capture at a time on that stream
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int64_t d = 0; d < count && e == hipSuccess; ++d) {
        if (probs[d].pairs) e = fill_i32(reinterpret_cast<int*>(probs[d].pairs_count), 0, 2, cap);
        if (e != hipSuccess || probs[d].n == 0) continue;
        e = stage_input(d, cap);
        if (e == hipSuccess) e = launch_plain(plans[d].cfg, P[d], cap);
      }
      if (e != hipSuccess) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(cap, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        return fail(MI_ERR_DEVICE, "launch during capture: %s", hipGetErrorString(e));
      }
      HIPCHK(hipStreamEndCapture(cap, &graph));
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(MI_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      std::lock_guard<std::mutex> lk(g_graph_mu);
      if (g_graphs.size() > 64) {
        for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second.exec);
        g_graphs.clear();
      }
      g_graphs[key].exec = exec;
    }
    HIPCHK(hipGraphLaunch(exec, st));
    return MI_OK;
  }

  // Persistent: work lists sorted by decreasing unit rows, one launch per tile
  // size and Gram (list g * kNumCfg + c; the FP4 lists, which hold the
  // largest datasets, launch first).
  constexpr int kLists = 2 * kNumCfg;
  const int order[kLists] = {kNumCfg + 1, kNumCfg + 0, 1, 0};
  static_assert(kNumCfg == 2, "launch order lists every (Gram, tile) pair");
  // The units of one (dataset, split) share their row count, so the groups
  // are sorted (stably, in dataset and split order) and then expanded tile
  // by tile: the order of sorting every unit, at the cost of sorting the
  // groups.
  struct Group {
    int64_t rows;
    int32_t prob, split;
  };
  std::vector<Group> groups[kLists];
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0) continue;
    const int li = (f4[d] ? kNumCfg : 0) + plans[d].cfg;
    for (int sp = 0; sp < plans[d].splits; ++sp)
      groups[li].push_back(Group{std::min<int64_t>(P[d].kchunk, P[d].m - (int64_t)sp * P[d].kchunk), (int32_t)d, sp});
  }
  std::vector<UnitRef> units[kLists];
  for (int c = 0; c < kLists; ++c) {
    std::stable_sort(groups[c].begin(), groups[c].end(), [](const Group& x, const Group& y) { return x.rows > y.rows; });
    size_t nu = 0;
    for (const Group& g : groups[c]) nu += (size_t)plans[g.prob].ntiles;
    units[c].reserve(nu);
    for (const Group& g : groups[c])
      for (int t = 0; t < plans[g.prob].ntiles; ++t) units[c].push_back(UnitRef{g.prob, t, g.split, 0});
  }
  const size_t probs_bytes = ((sizeof(ProbDev) * count) + 255) & ~(size_t)255;
  size_t nunits = 0;
  for (int c = 0; c < kLists; ++c) nunits += units[c].size();
  const size_t units_bytes = ((sizeof(UnitRef) * nunits) + 255) & ~(size_t)255;
  // Every repack of the batch runs as one launch from a descriptor list.
  std::vector<RepackDesc> rdesc;
  int64_t rblocks = 0;
  for (int64_t d = 0; d < count; ++d) {
    if (probs[d].n == 0 || (aligned[d] && !conv[d])) continue;
    // At most 2^22 blocks in all (the grid stays far below 2^32 work-items);
    // layouts with fewer blocks than their chunks loop.  A conversion reads
    // the n byte columns; a repack copies the row's bytes.
    const int64_t cap = std::max<int64_t>(1, ((int64_t)1 << 22) / count);
    RepackDesc r{probs[d].X, ldx[d], (uint8_t*)P[d].X, P[d].ldx, probs[d].m,
                 conv[d] ? probs[d].n : row_bytes(probs[d]), rblocks,
                 std::min<int64_t>(repack_blocks(probs[d].m, P[d].ldx), cap), conv[d] ? 1 : 0, 0};
    rblocks += r.blocks;
    rdesc.push_back(r);
  }
  const size_t rdesc_bytes = ((sizeof(RepackDesc) * rdesc.size()) + 255) & ~(size_t)255;
  const size_t total = probs_bytes + units_bytes + rdesc_bytes + 256;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchBufs& bb = g_batch[{dev, st}];
  if (bb.copied) HIPCHK(hipEventSynchronize(bb.copied));  // staging buffer free again
  if (bb.host_bytes < total) {
    if (bb.host) HIPCHK(hipHostFree(bb.host));
    bb.host = nullptr;
    HIPCHK(hipHostMalloc(&bb.host, total, hipHostMallocDefault));
    bb.host_bytes = total;
  }
  if (bb.dev_bytes < total) {
    if (bb.dev) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipFree(bb.dev));
    }
    bb.dev = nullptr;
    if (hipMalloc(&bb.dev, total) != hipSuccess) {
      (void)hipGetLastError();
      bb.dev_bytes = 0;
      return fail(MI_ERR_OUT_OF_MEMORY, "batch descriptor allocation failed");
    }
    bb.dev_bytes = total;
  }
  if (!bb.copied) HIPCHK(hipEventCreateWithFlags(&bb.copied, hipEventDisableTiming));
  char* h = (char*)bb.host;
  std::memcpy(h, P.data(), sizeof(ProbDev) * count);
  size_t uoff = probs_bytes;
  for (int li : order) {
    std::memcpy(h + uoff, units[li].data(), sizeof(UnitRef) * units[li].size());
    uoff += sizeof(UnitRef) * units[li].size();
  }
  if (!rdesc.empty()) std::memcpy(h + probs_bytes + units_bytes, rdesc.data(), sizeof(RepackDesc) * rdesc.size());
  HIPCHK(hipMemcpyAsync(bb.dev, bb.host, probs_bytes + units_bytes + rdesc_bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(bb.copied, st));
  for (int64_t d = 0; d < count; ++d)
    if (probs[d].pairs) HIPCHK(fill_i32(reinterpret_cast<int*>(probs[d].pairs_count), 0, 2, st));
  char* dv = (char*)bb.dev;
  HIPCHK(launch_repack_batch((const RepackDesc*)(dv + probs_bytes + units_bytes), (int)rdesc.size(), rblocks, st));
  const ProbDev* dP = (const ProbDev*)dv;
  const UnitRef* dU = (const UnitRef*)(dv + probs_bytes);
  int* head = (int*)(dv + probs_bytes + units_bytes + rdesc_bytes);
  for (int li : order) {
    const int c = li % kNumCfg, g = li / kNumCfg;
    const int64_t grid = std::min<int64_t>((int64_t)di.cus * di.pocc[c][g], (int64_t)units[li].size());
    HIPCHK(launch_persistent(c, g == 1, dP, dU, (int)units[li].size(), head + li, (int)grid, st));
    dU += units[li].size();
  }
  return MI_OK;
}

void release_stream_resources(hipStream_t st) {
  release_scratch_of(st);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (auto it = g_batch.begin(); it != g_batch.end();) {
    if (it->first.second == st) {
      if (it->second.copied) {
        (void)hipEventSynchronize(it->second.copied);
        (void)hipEventDestroy(it->second.copied);
      }
      if (it->second.host) (void)hipHostFree(it->second.host);
      if (it->second.dev) (void)hipFree(it->second.dev);
      it = g_batch.erase(it);
    } else {
      ++it;
    }
  }
}

// ------------------------------------------------------------------- tuner --
mi_status tune(int64_t m, int64_t n, int64_t ldx, int32_t* tile, int32_t* splits, double* best_ms) {
  if (m <= 0 || m > INT32_MAX || n <= 0 || n > kMaxCols) return fail(MI_ERR_INVALID_ARG, "bad shape for tuning");
  if (ldx == 0) ldx = n;
  if (ldx < n || ldx > kMaxPitch) return fail(MI_ERR_INVALID_ARG, "bad ldx for tuning");
  DeviceInfo di;
  mi_status s = device_info(&di);
  if (s != MI_OK) return s;
  // The Gram the library would run for byte input of this shape and pitch
  // (FP4 for large shapes and for pitches that are not a multiple of 16,
  // whose input is converted first), timed on a matrix in the layout that
  // Gram reads.  It holds a hashed 0/1 pattern of
  // density 1/8 (the kernels' time depends on the data only through the
  // split-K partials they skip when zero, which are then rare).
  const bool aligned = ldx % 16 == 0;
  const bool fp4 = fp4_preferred(m, n) || !aligned;  // unaligned byte layouts are converted to FP4
  const int64_t ld = fp4 ? packed_pitch((n + 1) / 2) : (aligned ? ldx : packed_pitch(n));
  uint8_t* X = nullptr;
  float* out = nullptr;
  const size_t xbytes = (size_t)m * (size_t)ld;
  if (hipMalloc(&X, xbytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MI_ERR_OUT_OF_MEMORY, "tuner: X allocation failed");
  }
  if (hipMalloc(&out, (size_t)n * n * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(X);
    return fail(MI_ERR_OUT_OF_MEMORY, "tuner: out allocation failed");
  }
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Tuned best{-1, 0, 1e30};
  auto body = [&]() -> mi_status {
    HIPCHK(hipStreamCreate(&st));
    HIPCHK(launch_fill_pattern(X, m, ld, fp4 ? (n + 1) / 2 : n, fp4, st));
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipError_t te;
    // Median of five launches after a warm-up.
    auto time_plan = [&](const Plan& pl, double* ms_out) -> mi_status {
      const int32_t* tiles = tile_table(pl.ntp, &te);
      if (!tiles) return fail(MI_ERR_DEVICE, "tile table: %s", hipGetErrorString(te));
      void* ws = nullptr;
      mi_status ss = workspace(st, 0, workspace_bytes(pl), &ws);
      if (ss != MI_OK) return ss;
      mi_problem pr;
      mi_problem_init(&pr, X, m, n, out);
      pr.ldx = ld;
      pr.packed = fp4 ? MI_INPUT_FP4 : MI_INPUT_BYTES;
      const ProbDev P = make_probdev(&pr, X, ld, pl, ws, tiles);
      HIPCHK(launch_plain(pl.cfg, P, st));  // warm-up
      std::vector<float> ts;
      for (int rep = 0; rep < 5; ++rep) {
        HIPCHK(hipEventRecord(e0, st));
        HIPCHK(launch_plain(pl.cfg, P, st));
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        ts.push_back(ms);
      }
      std::sort(ts.begin(), ts.end());
      *ms_out = ts[ts.size() / 2];
      return MI_OK;
    };
    // The heuristic plan first: another candidate replaces it only when at
    // least 3% faster, so timing noise cannot make a tuned plan slower.
    const int hcfg = heuristic_cfg(m, n);
    Plan hp = make_plan(m, n, hcfg, heuristic_splits(m, make_plan(m, n, hcfg, 1), di.cus, fp4 ? 2.0 : 1.0));
    while (fp4 && hp.kchunk > kFp4MaxUnitRows) hp = make_plan(m, n, hcfg, hp.splits + 1);
    double heur = 0.0;
    mi_status hs = time_plan(hp, &heur);
    if (hs != MI_OK) return hs;
    best = Tuned{hp.cfg, hp.splits, heur};
    for (int cfg = 0; cfg < kNumCfg; ++cfg) {
      const Plan p1 = make_plan(m, n, cfg, 1);
      std::vector<int> cands;
      for (int sp = 1; sp <= 16; ++sp) cands.push_back(sp);
      for (int sp : {20, 24, 32, 48, 64, 96, 128, 192, 256}) cands.push_back(sp);
      for (int sp : cands) {
        if (sp > p1.ksteps) continue;
        const Plan pl = make_plan(m, n, cfg, sp);
        if (pl.splits != sp || (double)pl.ntiles * pl.splits > 4.0e6) continue;
        if (fp4 && pl.kchunk > kFp4MaxUnitRows) continue;  // FP32 counts exact per unit
        if (cfg == hp.cfg && sp == hp.splits) continue;    // the heuristic, timed above
        double ms = 0.0;
        mi_status ss = time_plan(pl, &ms);
        if (ss != MI_OK) return ss;
        if (ms < 0.97 * heur && ms < best.ms) best = Tuned{cfg, pl.splits, ms};
      }
    }
    return MI_OK;
  };
  s = body();
  if (st) (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) {
    release_scratch_of(st);
    (void)hipStreamDestroy(st);
  }
  (void)hipFree(X);
  (void)hipFree(out);
  if (s != MI_OK) return s;
  if (best.cfg < 0) return fail(MI_ERR_DEVICE, "tuner found no runnable configuration");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[shape_key(m, n, aligned, fp4)] = best;
  }
  if (tile) *tile = best.cfg == 1 ? MI_TILE_256 : MI_TILE_128;
  if (splits) *splits = best.splits;
  if (best_ms) *best_ms = best.ms;
  return MI_OK;
}

// Batch tuner: time the persistent mode of the caller's own batch (its data,
// its outputs, which every candidate overwrites with the same results) under
// candidate plans, and keep the fastest under the batch's signature.  The
// heuristic is kept unless a candidate is at least 3% faster (medians of five
// runs after one warm-up).
mi_status tune_batched(const mi_problem* probs, int64_t count, hipStream_t st, double* best_ms, double* heur_ms,
                       BatchChoice* chosen) {
  std::vector<Plan> plans;
  mi_status s = run_batched(probs, count, st, MI_BATCH_PERSISTENT, nullptr, &plans);  // checks the batch
  if (s != MI_OK) return s;
  std::vector<char> aligned(count), f4(count);
  for (int64_t d = 0; d < count; ++d) {
    int64_t ldx = 0;
    s = check_problem(&probs[d], &ldx);
    if (s != MI_OK) return s;
    aligned[d] = is_aligned(probs[d].X, ldx) ? 1 : 0;
  }
  std::vector<char> conv;
  batch_grams(probs, count, true, conv, f4);
  std::vector<BatchChoice> cands;
  cands.push_back(heuristic_batch_choice());
  const std::pair<int, int> tiles[] = {{kBatchTileAuto, 512},    {(int)MI_TILE_128, 512}, {(int)MI_TILE_256, 512},
                                       {kBatchTileByWidth, 512}, {kBatchTileByWidth, 1024}};
  for (const auto& tn : tiles)
    for (int fdiv : {1, 2, 4, 8, 16}) {
      const BatchChoice c{tn.first, tn.second, fdiv};
      if (c.tile == kBatchTileAuto && c.fdiv == 1) continue;  // the heuristic, already first
      cands.push_back(c);
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 1e30, heur = 1e30;
  BatchChoice best_c = heuristic_batch_choice();
  auto body = [&]() -> mi_status {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      mi_status r = run_batched(probs, count, st, MI_BATCH_PERSISTENT, &cands[ci]);  // warm-up
      if (r != MI_OK) return r;
      std::vector<float> ts;
      for (int rep = 0; rep < 5; ++rep) {
        HIPCHK(hipEventRecord(e0, st));
        r = run_batched(probs, count, st, MI_BATCH_PERSISTENT, &cands[ci]);
        if (r != MI_OK) return r;
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        ts.push_back(ms);
      }
      std::sort(ts.begin(), ts.end());
      const double med = ts[ts.size() / 2];
      if (ci == 0) {
        heur = best = med;
      } else if (med < 0.97 * heur && med < best) {
        best = med;
        best_c = cands[ci];
      }
    }
    return MI_OK;
  };
  s = body();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s != MI_OK) return s;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_batch_tuned[batch_signature(probs, count, aligned, f4)] = {best_c, best};
  }
  if (best_ms) *best_ms = best;
  if (heur_ms) *heur_ms = heur;
  if (chosen) *chosen = best_c;
  return MI_OK;
}

mi_status tuner_save(const char* path) {
  if (!path) return fail(MI_ERR_INVALID_ARG, "path is NULL");
  FILE* f = fopen(path, "w");
  if (!f) return fail(MI_ERR_INVALID_ARG, "cannot open %s for writing", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tuned)
    fprintf(f, "{\"mb\": %d, \"nb\": %d, \"aligned\": %d, \"tile\": %d, \"splits\": %d, \"ms\": %.6f, \"fp4\": %d}\n",
            kv.first.mb, kv.first.nb, kv.first.aligned, cfg_tile(kv.second.cfg), kv.second.splits, kv.second.ms,
            kv.first.fp4);
  for (auto& kv : g_batch_tuned)
    fprintf(f, "{\"batch\": \"%016llx\", \"tile\": %d, \"narrow\": %d, \"fdiv\": %d, \"ms\": %.6f}\n",
            (unsigned long long)kv.first, kv.second.first.tile, kv.second.first.narrow_n, kv.second.first.fdiv,
            kv.second.second);
  fclose(f);
  return MI_OK;
}

mi_status tuner_load(const char* path) {
  if (!path) return fail(MI_ERR_INVALID_ARG, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return fail(MI_ERR_INVALID_ARG, "cannot open %s", path);
  char line[512];
  int nread = 0;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  while (fgets(line, sizeof line, f)) {
    unsigned long long sig = 0;
    BatchChoice bc;
    double bms = 0.0;
    if (sscanf(line, " {\"batch\": \"%16llx\", \"tile\": %d, \"narrow\": %d, \"fdiv\": %d, \"ms\": %lf}", &sig, &bc.tile,
               &bc.narrow_n, &bc.fdiv, &bms) == 5) {
      if (bc.tile >= 0 && bc.tile <= kBatchTileByWidth && bc.narrow_n >= 1 && bc.fdiv >= 1 && bc.fdiv <= 1024) {
        g_batch_tuned[(uint64_t)sig] = {bc, bms};
        ++nread;
      }
      continue;
    }
    ShapeKey k;
    Tuned t;
    int tile = 0;
    k.fp4 = 0;  // entries without the field time the int8 Gram
    const int got = sscanf(line, " {\"mb\": %d, \"nb\": %d, \"aligned\": %d, \"tile\": %d, \"splits\": %d, \"ms\": %lf, \"fp4\": %d}",
                           &k.mb, &k.nb, &k.aligned, &tile, &t.splits, &t.ms, &k.fp4);
    if (got >= 6 && (tile == 128 || tile == 256) && t.splits >= 1 && (k.fp4 == 0 || k.fp4 == 1)) {
      t.cfg = tile == 256 ? 1 : 0;
      g_tuned[k] = t;
      ++nread;
    }
  }
  fclose(f);
  (void)nread;
  return MI_OK;
}

void tuner_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  g_batch_tuned.clear();
}

}  // namespace mi

// ===================================================================== C ABI
using namespace mi;

extern "C" {

void mi_problem_init(mi_problem* p, const uint8_t* X, int64_t m, int64_t n, float* out) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->X = X;
  p->m = m;
  p->n = n;
  p->ldx = n;
  p->out = out;
  p->epilogue = MI_EPI_FP32;
  p->fallback_tau = 1e-3f;
}

mi_status mi_all_pairs_ex(const mi_problem* p, void* stream) {
  clear_error();
  return run_one(p, (hipStream_t)stream, 0);
}

mi_status mi_all_pairs_async(const uint8_t* X, int64_t m, int64_t n, float* out, void* stream) {
  mi_problem p;
  mi_problem_init(&p, X, m, n, out);
  return mi_all_pairs_ex(&p, stream);
}

mi_status mi_all_pairs(const uint8_t* X, int64_t m, int64_t n, float* out) {
  mi_status s = mi_all_pairs_async(X, m, n, out, nullptr);
  if (s != MI_OK) return s;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return fail(MI_ERR_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  return MI_OK;
}

mi_status mi_all_pairs_batched(const mi_problem* probs, int64_t count, void* stream, int32_t mode) {
  clear_error();
  return run_batched(probs, count, (hipStream_t)stream, mode);
}

mi_status mi_pack_bits(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xp, int64_t ldp, void* stream) {
  clear_error();
  if (m < 0 || n < 0) return fail(MI_ERR_INVALID_ARG, "m and n must be >= 0");
  if (m == 0 || n == 0) return MI_OK;
  if (!X || !Xp) return fail(MI_ERR_INVALID_ARG, "X and Xp must be non-NULL");
  if (ldx < n) return fail(MI_ERR_INVALID_ARG, "ldx (%lld) < n (%lld)", (long long)ldx, (long long)n);
  if (ldp < (n + 7) / 8) return fail(MI_ERR_INVALID_ARG, "ldp (%lld) < ceil(n / 8)", (long long)ldp);
  if ((n + 63) / 64 > (int64_t)64 * 65535) return fail(MI_ERR_INVALID_ARG, "n too large");
  HIPCHK(launch_pack_bits(X, m, n, ldx, Xp, ldp, (hipStream_t)stream));
  return MI_OK;
}

mi_status mi_pack_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xq, int64_t ldq, void* stream) {
  clear_error();
  if (m < 0 || n < 0) return fail(MI_ERR_INVALID_ARG, "m and n must be >= 0");
  if (m == 0 || n == 0) return MI_OK;
  if (!X || !Xq) return fail(MI_ERR_INVALID_ARG, "X and Xq must be non-NULL");
  if (ldx < n) return fail(MI_ERR_INVALID_ARG, "ldx (%lld) < n (%lld)", (long long)ldx, (long long)n);
  if (ldq < (n + 1) / 2) return fail(MI_ERR_INVALID_ARG, "ldq (%lld) < ceil(n / 2)", (long long)ldq);
  if ((n + 31) / 32 > (int64_t)64 * 65535) return fail(MI_ERR_INVALID_ARG, "n too large");
  if ((m + 3) / 4 > (int64_t)UINT32_MAX) return fail(MI_ERR_INVALID_ARG, "m too large");
  HIPCHK(launch_pack_fp4(X, m, n, ldx, Xq, ldq, (hipStream_t)stream));
  return MI_OK;
}

mi_status mi_plan_ex(const mi_problem* p, int32_t* tile, int32_t* splits, int32_t* gram) {
  clear_error();
  int64_t ldx = 0;
  mi_status s = check_problem(p, &ldx, /*need_output=*/false);
  if (s != MI_OK) return s;
  const bool convert = converts_to_fp4(p);
  const bool fp4 = runs_fp4(p);
  Plan pl;
  s = choose_plan(p->m, std::max<int64_t>(p->n, 1), is_aligned(p->X, ldx) || convert, p->tile, p->splits, &pl, fp4);
  if (s != MI_OK) return s;
  if (tile) *tile = pl.cfg == 1 ? MI_TILE_256 : MI_TILE_128;
  if (splits) *splits = pl.splits;
  if (gram) *gram = fp4 ? MI_GRAM_FP4 : MI_GRAM_INT8;
  return MI_OK;
}

mi_status mi_plan(int64_t m, int64_t n, int64_t ldx, int32_t* tile, int32_t* splits) {
  clear_error();
  if (m <= 0 || m > INT32_MAX || n < 0 || n > kMaxCols) return fail(MI_ERR_INVALID_ARG, "bad shape");
  if (ldx == 0) ldx = n;
  if (ldx < n) return fail(MI_ERR_INVALID_ARG, "ldx < n");
  Plan pl;
  mi_status s = choose_plan(m, std::max<int64_t>(n, 1), ldx % 16 == 0, 0, 0, &pl);
  if (s != MI_OK) return s;
  if (tile) *tile = pl.cfg == 1 ? MI_TILE_256 : MI_TILE_128;
  if (splits) *splits = pl.splits;
  return MI_OK;
}

mi_status mi_tune(int64_t m, int64_t n, int64_t ldx, int32_t* tile, int32_t* splits, double* best_ms) {
  clear_error();
  return tune(m, n, ldx, tile, splits, best_ms);
}

mi_status mi_tune_batched(const mi_problem* probs, int64_t count, void* stream, double* best_ms,
                          double* heuristic_ms) {
  clear_error();
  return tune_batched(probs, count, (hipStream_t)stream, best_ms, heuristic_ms, nullptr);
}

mi_status mi_plan_batched(const mi_problem* probs, int64_t count, int32_t* tiles, int32_t* splits) {
  clear_error();
  std::vector<Plan> plans;
  mi_status s = run_batched(probs, count, nullptr, MI_BATCH_PERSISTENT, nullptr, &plans);
  if (s != MI_OK) return s;
  for (int64_t d = 0; d < count; ++d) {
    const bool empty = probs[d].n == 0;
    if (tiles) tiles[d] = empty ? MI_TILE_AUTO : (plans[d].cfg == 1 ? MI_TILE_256 : MI_TILE_128);
    if (splits) splits[d] = empty ? 0 : plans[d].splits;
  }
  return MI_OK;
}

mi_status mi_tuner_save(const char* path) {
  clear_error();
  return tuner_save(path);
}

mi_status mi_tuner_load(const char* path) {
  clear_error();
  return tuner_load(path);
}

void mi_tuner_clear(void) { tuner_clear(); }

const char* mi_last_error(void) { return last_error(); }

const char* mi_version(void) { return "mi355x-binary-mi 0.2 (gfx950, int8 and FP4 MFMA)"; }

}  // extern "C"
