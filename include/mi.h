/*
 * mi.h -- all-pairs mutual information of a binary dataset on an MI355X GPU.
 *
 * The operation (paper Section 1, Eq. 1, unrolled in Eq. 2/3): for an m x n
 * binary matrix X (rows are samples, columns are variables, Section 2 step 1)
 * compute for every column pair (i, j)
 *
 *     MI_ij = sum_{x,y in {0,1}} p(x,y) log2( p(x,y) / (p(x) p(y)) )   [bits]
 *
 * the matrix way: one Gram product n11 = X^T X (Section 2 step 2, Section 3),
 * column sums c = diag(n11) (Section 2 step 3, Section 3.1 "Term 2"), and the
 * other joint counts derived without further products (Section 3.1, Eq. 6
 * and Eq. 7, orientation taken from first principles):
 *
 *     n10 = c_i - n11,   n01 = c_j - n11,   n00 = m - c_i - c_j + n11.
 *
 * A cell with n_xy = 0 contributes exactly 0 (0 log 0 = 0); the paper's
 * unspecified epsilon (Section 2 step 5) is not used.  The diagonal holds
 * H(X_i).  Counts are exact (int8 x int8 -> int32 matrix cores); MI is
 * evaluated in FP32, optionally recomputed in FP64 (see mi_epilogue).
 *
 * Conventions for every entry point:
 *   - Data pointers are DEVICE pointers on the current HIP device.  The
 *     caller owns them; the library never frees them.  They must stay valid
 *     until the work completes (stream order, or ticket completion for the
 *     server).
 *   - X is row-major, m rows of ldx >= n bytes; entries must be 0 or 1
 *     (other values give undefined results unless `validate` is set).  Bytes
 *     in columns [n, ldx) are ignored.  The fast load path is taken when X is
 *     16-byte aligned and ldx is a multiple of 16; other layouts are correct
 *     but slower.
 *   - out is n x n FP32, row-major, the full symmetric matrix (both
 *     triangles are written; out[i][j] and out[j][i] are bitwise equal).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Nothing is thrown across the ABI: every call returns an mi_status and
 *     mi_last_error() gives a thread-local message for the last failure.
 *   - Limits: 1 <= m <= 2^31 - 1 (int32 counts), 0 <= n <= 4,194,176 (32,767
 *     column panels of 128); n == 0 is a successful no-op.  Counts convert exactly to FP32 below 2^24 rows;
 *     above that the FP32 epilogue rounds them (the FP64 modes stay exact).
 */
#ifndef MI_H_
#define MI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mi_status {
  MI_OK = 0,
  MI_ERR_INVALID_ARG = 1,   /* bad size, NULL pointer, bad enum value        */
  MI_ERR_NOT_BINARY = 2,    /* validate != 0 and X holds a byte other than 0/1 */
  MI_ERR_OUT_OF_MEMORY = 3, /* workspace allocation failed                    */
  MI_ERR_BUDGET = 4,        /* server: request alone exceeds the HBM budget   */
  MI_ERR_QUEUE_FULL = 5,    /* server: bounded queue is full                  */
  MI_ERR_NOT_READY = 6,     /* server: ticket not finished yet (poll)         */
  MI_ERR_DEVICE = 7,        /* a HIP call failed                              */
  MI_ERR_TIMEOUT = 8,       /* server: wait timed out                         */
  MI_ERR_UNKNOWN_TICKET = 9, /* server: ticket was never issued or already collected */
  MI_ERR_BAD_CODE = 10       /* categorical, validate != 0: a code is not below its level count */
} mi_status;

/* How MI is evaluated from the exact counts (the counts are always exact). */
typedef enum mi_epilogue {
  MI_EPI_FP32 = 0,               /* FP32 log2 per cell                                    */
  MI_EPI_FP32_FP64_FALLBACK = 1, /* FP32, recomputed in FP64 where the FP32 MI < tau       */
  MI_EPI_FP64 = 2                /* FP64 for every pair (rounded to FP32 on output)        */
} mi_epilogue;

/* Tile configurations of the fused kernel (0 = let the library choose). */
typedef enum mi_tile {
  MI_TILE_AUTO = 0,
  MI_TILE_128 = 1,  /* 128 x 128 output tile, 4 waves of 64 x 64 */
  MI_TILE_256 = 2   /* 256 x 256 output tile, 8 waves of 128 x 64 */
} mi_tile;

/* How the 1-1 counts are computed. */
typedef enum mi_algo {
  MI_ALGO_DENSE = 0,   /* int8 matrix-core Gram over upper-triangular tiles (default)        */
  MI_ALGO_SPARSE = 1,  /* sum over rows of the pairs of ones (work ~ m (n d)^2 at density d);  */
                       /* synchronises the stream once                                        */
  MI_ALGO_AUTO = 2     /* estimate the pairs of ones from a 4,096-row sample (synchronises */
                       /* once); dense when a cost model from measured rates says so       */
                       /* clearly, else count every row (synchronises again) and take the  */
                       /* faster path (at 1M x 4096 the sparse one below ~0.3% density)     */
} mi_algo;

/* Input layouts (mi_problem.packed). */
typedef enum mi_input {
  MI_INPUT_BYTES = 0,  /* one 0/1 byte per entry                                          */
  MI_INPUT_BITS = 1,   /* 8 columns per byte (mi_pack_bits)                                */
  MI_INPUT_FP4 = 2     /* 2 columns per byte as E2M1 codes: 0b0010 (1.0) or 0 (mi_pack_fp4) */
} mi_input;

/* Matrix instructions of the dense Gram (mi_problem.gram).  Both give the same
 * exact counts, hence bitwise the same outputs; they differ in speed.  The
 * n11 = X^T X contraction over 0/1 entries is exact with FP4 (E2M1) operands,
 * whose 1.0 products sum to integers in the FP32 accumulator; each work unit
 * then covers at most 2^24 rows, so every partial count is exact. */
typedef enum mi_gram {
  MI_GRAM_AUTO = 0,  /* the library's choice: FP4 for byte input with n >= 1536 and       */
                     /* m n^2 >= 6e10, and for byte input whose layout needs a copy      */
                     /* (X not 16-byte aligned or ldx % 16 != 0: the conversion replaces */
                     /* the repack), converted to the FP4 layout first in scratch memory */
                     /* of half the input's size; for bit input with n >= 512 (unpacked  */
                     /* on chip to FP4 codes); for FP4 input; int8 otherwise             */
  MI_GRAM_INT8 = 1,  /* v_mfma_i32_32x32x32_i8 on bytes (or bits unpacked to bytes)       */
  MI_GRAM_FP4 = 2    /* v_mfma_scale_f32_32x32x64_f8f6f4 on E2M1 codes: twice the samples */
                     /* per byte staged and ~1.7x the int8 instruction rate               */
} mi_gram;

/* One entry of the sparse (threshold) output: MI(X_i; X_j) in bits, i < j. */
typedef struct mi_pair {
  int32_t i, j;
  float mi;
} mi_pair;

typedef struct mi_problem {
  const uint8_t* X;      /* device, m x ldx bytes, row-major, 0/1                   */
  int64_t m;             /* rows (samples), >= 1                                    */
  int64_t n;             /* columns (variables), >= 0                               */
  int64_t ldx;           /* row pitch in bytes, >= n; 0 means n                     */
  float* out;            /* device, n x n FP32 row-major; may be NULL when `pairs`  */
                         /* or n11_out is given (then no dense MI matrix is written; */
                         /* with neither out nor pairs no MI is evaluated at all)   */
  int32_t* n11_out;      /* optional device n x n int32: the 1-1 counts X^T X        */
  int32_t* colsum_out;   /* optional device int32[n]: column sums c                 */
  int32_t epilogue;      /* mi_epilogue                                             */
  float fallback_tau;    /* MI_EPI_FP32_FP64_FALLBACK threshold in bits; <= 0: 1e-3  */
  int32_t validate;      /* nonzero: check X is 0/1 first (one extra pass, blocking); */
                         /* FP4 input: every code 0 or 0b0010                       */
  int32_t tile;          /* mi_tile; 0 = autotuned / heuristic                      */
  int32_t splits;        /* K-splits over the rows; 0 = autotuned / heuristic       */
  /* Sparse output (blockwise use when the n x n matrix is not wanted or does
   * not fit): every pair i < j with MI >= pairs_threshold is appended to
   * `pairs`, in no particular order.  *pairs_count (device, zeroed by the
   * call) receives the number of such pairs; if it exceeds pairs_capacity,
   * only pairs_capacity of them (an unspecified subset) are stored.  The same
   * evaluation as the dense output (same epilogue mode, same values). */
  mi_pair* pairs;                   /* optional device array of pairs_capacity entries */
  int64_t pairs_capacity;           /* >= 0                                           */
  unsigned long long* pairs_count;  /* device; required when pairs is given           */
  float pairs_threshold;            /* bits                                           */
  int32_t algo;                     /* mi_algo; batches and the server take only DENSE */
  /* Input layout (mi_input).  MI_INPUT_BITS: X holds 8 columns per byte, bit
   * k (least significant first) of byte b of a row being column 8 b + k; ldx
   * is then the row pitch in bytes, >= ceil(n / 8) (0 means ceil(n / 8)).  The
   * kernel reads an eighth of the bytes and unpacks them on chip (to bytes
   * for the int8 Gram, to FP4 codes for the FP4 Gram); validate is a no-op
   * (every bit is 0 or 1).  MI_INPUT_FP4: X holds 2 columns per byte,
   * column 2 c in the low nibble of byte c, each nibble 0b0010 (a one) or 0
   * (as mi_pack_fp4 writes them; other codes give undefined counts unless
   * validate is set, which then checks every code of columns < n and returns
   * MI_ERR_NOT_BINARY); ldx >= ceil(n / 2), at most 2^23.  Results are the same as
   * for the byte layout.  Packed layouts take the dense algorithm only; bits
   * in single calls and the graph / sequential batch modes, FP4 in single
   * calls and every batch mode; the server takes the byte layout only. */
  int32_t packed;
  /* mi_gram.  MI_GRAM_INT8 needs byte or bit input; MI_GRAM_FP4 takes any
   * input.  Batches and the server follow each problem's choice (byte input
   * converted in library scratch; the server charges that buffer to the
   * request's HBM budget). */
  int32_t gram;
} mi_problem;

/* Fill *p with defaults for X (m x n, ldx = n) and out: FP32 epilogue, auto config. */
void mi_problem_init(mi_problem* p, const uint8_t* X, int64_t m, int64_t n, float* out);

/* Blocking: computes out on the default stream and synchronises it. */
mi_status mi_all_pairs(const uint8_t* X, int64_t m, int64_t n, float* out);

/* Asynchronous on `stream`; returns once the work is enqueued. */
mi_status mi_all_pairs_async(const uint8_t* X, int64_t m, int64_t n, float* out, void* stream);

/* Full control (pitch, counts export, epilogue mode, config).  Asynchronous on
 * `stream` unless p->validate is set (then it synchronises to read the check). */
mi_status mi_all_pairs_ex(const mi_problem* p, void* stream);

/* Many independent datasets in one call, asynchronous on `stream`.
 *   mode MI_BATCH_PERSISTENT: one persistent launch per (tile configuration,
 *        Gram) pulls (dataset, tile, split) work units from a device queue,
 *        after one launch that converts (or repacks) every input that needs
 *        it.  When the datasets on the FP4 Gram hold at least half of the
 *        batch's pair-updates, byte datasets left to MI_GRAM_AUTO run the
 *        FP4 Gram too (one Gram, one launch; the outputs do not change);
 *   mode MI_BATCH_GRAPH: `count` plain launches captured once into a hipGraph
 *        and replayed (the graph is cached for identical batches);
 *   mode MI_BATCH_SEQUENTIAL: `count` plain launches, one after another.
 * All three give bitwise identical outputs.  validate is not allowed here. */
typedef enum mi_batch_mode {
  MI_BATCH_PERSISTENT = 0,
  MI_BATCH_GRAPH = 1,
  MI_BATCH_SEQUENTIAL = 2
} mi_batch_mode;
mi_status mi_all_pairs_batched(const mi_problem* probs, int64_t count, void* stream, int32_t mode);

/* mi_all_pairs_ex for callers that cannot allocate device memory: code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or other allocating routine.  Its scratch (the
 * split-K workspace and the validation flag) is one fixed device array of
 * 64 MiB + 256 bytes inside the library; each GPU the library runs on holds
 * its own copy until the process ends, and the first call on a device clears
 * it on `stream`.  The caller passes inputs and outputs as for
 * mi_all_pairs_ex; the results are bitwise those of mi_all_pairs_ex with the
 * same Gram, tile and splits.
 * Differences from mi_all_pairs_ex:
 *   - byte input runs the int8 Gram (MI_GRAM_AUTO included): there is no
 *     scratch for the FP4 conversion, so MI_GRAM_FP4 with byte input is
 *     MI_ERR_INVALID_ARG (pass MI_INPUT_FP4 input from mi_pack_fp4 instead);
 *     bit and FP4 input follow mi_all_pairs_ex;
 *   - X must be 16-byte aligned with ldx % 16 == 0 (no repack copy), else
 *     MI_ERR_INVALID_ARG;
 *   - algo must be MI_ALGO_DENSE, else MI_ERR_INVALID_ARG;
 *   - a plan whose split-K workspace (tiles x (BT^2 + 2 BT + 1) x 4 bytes)
 *     exceeds 64 MiB runs with the fewest splits instead (one, or what keeps
 *     FP4 units at <= 2^24 rows); an explicit `splits` that does not fit, or
 *     an FP4 problem whose minimum does not, is MI_ERR_INVALID_ARG.
 * Every call on a device shares that device's array and leaves its workspace
 * zeroed: calls that overlap on one GPU (other streams, other threads, graph
 * replays running concurrently) race and give undefined results.  Calls
 * ordered on one stream, or separated by synchronisation, do not.
 * Asynchronous on `stream` unless validate is set. */
mi_status mi_all_pairs_noalloc(const mi_problem* p, void* stream);

/* Categorical variables: the extension to non-binary data that the paper's
 * Conclusions name as future work.  Column j of X holds codes
 * 0 .. levels[j] - 1, and MI runs over the whole joint value set (Eq. 1):
 *
 *     MI_ab = (1/m) sum_{x,y} n_xy log2( n_xy m / (r_x s_y) )      [bits]
 *
 * with n_xy the L_a x L_b contingency table of the pair and r_x, s_y its
 * marginal counts.  The matrix way, generalising Section 3.1: the codes
 * 1 .. L_j - 1 of every variable become indicator columns (N = sum (L_j - 1)
 * of them, in variable order); ONE int8 Gram product of the indicator matrix
 * gives every cell with both codes >= 1, its column sums give the marginals
 * of codes >= 1, and every cell with a code 0 follows from those and m, as
 * n10, n01 and n00 follow from n11 (Eq. 6/7).  With every level count 2 the
 * indicators are X itself and this is the binary computation.
 *
 * Steps, all on `stream`: expand X into the m x N indicator matrix (device
 * scratch, about m * N bytes), the fused Gram kernel in a counts-only mode
 * (upper triangle, N x N int32 scratch unless counts_out is given), then one
 * thread per variable pair evaluates the table's MI (FP32 log2 per cell, or
 * FP64 per `epilogue`) and writes both triangles of out.  Asynchronous unless
 * validate is set; `levels` is read during the call only. */
typedef struct mi_cat_problem {
  const uint8_t* X;        /* device, m x ldx bytes, row-major codes                  */
  int64_t m;               /* rows (samples), 1 .. 2^31 - 1                           */
  int64_t v;               /* variables (columns), >= 0; v == 0 is a no-op            */
  int64_t ldx;             /* row pitch in bytes, >= v; 0 means v                     */
  const int32_t* levels;   /* HOST int32[v]: level count of each variable, 1 .. 256   */
  float* out;              /* device v x v FP32 row-major, both triangles (bitwise    */
                           /* symmetric); the diagonal holds H(X_j); may be NULL when */
                           /* `pairs` is given                                        */
  int32_t epilogue;        /* mi_epilogue                                            */
  float fallback_tau;      /* MI_EPI_FP32_FP64_FALLBACK threshold in bits; <= 0: 1e-3 */
  int32_t validate;        /* nonzero: check every code is below its level count      */
                           /* first (one extra pass, synchronises; MI_ERR_BAD_CODE).  */
                           /* Without it an out-of-range code counts as code 0.       */
  int32_t tile;            /* mi_tile of the Gram kernel; 0 = library's choice        */
  int32_t splits;          /* K-splits of the Gram kernel; 0 = library's choice       */
  int32_t* counts_out;     /* optional device N x N int32, both triangles: the        */
                           /* indicator Gram (cells with both codes >= 1)             */
  int32_t* sums_out;       /* optional device int32[N]: indicator column sums         */
  /* Sparse output, as in mi_problem: every pair a < b with MI >= pairs_threshold
   * is appended to `pairs` (order unspecified), *pairs_count (device, zeroed
   * by the call) receives their number, and out may then be NULL. */
  mi_pair* pairs;
  int64_t pairs_capacity;
  unsigned long long* pairs_count;
  float pairs_threshold;
  /* mi_gram of the indicator Gram: with FP4 the indicators are expanded
   * straight into the FP4 layout (no conversion pass).  MI_GRAM_AUTO: the
   * library's choice from m and N, as for mi_problem. */
  int32_t gram;
} mi_cat_problem;

/* Fill *p with defaults (ldx = v, FP32 epilogue, library's configuration). */
void mi_cat_problem_init(mi_cat_problem* p, const uint8_t* X, int64_t m, int64_t v, const int32_t* levels,
                         float* out);

/* Number of indicator columns N = sum (levels[j] - 1) (the side of counts_out). */
mi_status mi_cat_indicators(const int32_t* levels, int64_t v, int64_t* N);

mi_status mi_all_pairs_categorical(const mi_cat_problem* p, void* stream);

/* Pack a 0/1 byte matrix into the bit layout of mi_problem.packed:
 * Xp[r][b] bit k = (X[r][8 b + k] != 0) for 8 b + k < n, other bits 0.  X is
 * m x ldx bytes (ldx >= n), Xp is m x ldp bytes (ldp >= ceil(n / 8)); both
 * device pointers.  Asynchronous on `stream`. */
mi_status mi_pack_bits(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xp, int64_t ldp, void* stream);

/* Pack a 0/1 byte matrix into the FP4 layout of MI_INPUT_FP4: the low nibble
 * of Xq[r][c] is 0b0010 if X[r][2 c] != 0, else 0, and the high nibble the same
 * for X[r][2 c + 1] (0 past column n - 1).  X is m x ldx bytes (ldx >= n), Xq
 * is m x ldq bytes (ldq >= ceil(n / 2)); bytes of Xq past ceil(n / 2) in a
 * row are not written.  Both device pointers.  Asynchronous on `stream`. */
mi_status mi_pack_fp4(const uint8_t* X, int64_t m, int64_t n, int64_t ldx, uint8_t* Xq, int64_t ldq, void* stream);

/* What the library would run for *p (its dense path): the tile (mi_tile), the
 * K-split count and the Gram (MI_GRAM_INT8 or MI_GRAM_FP4; FP4 for byte input
 * means a conversion pass first).  Checks *p like mi_all_pairs_ex, except that
 * no output is required; launches nothing.  Any of the outputs may be NULL. */
mi_status mi_plan_ex(const mi_problem* p, int32_t* tile, int32_t* splits, int32_t* gram);

/* Configuration the library would use for an (m, n, ldx) byte problem with the
 * int8 Gram. */
mi_status mi_plan(int64_t m, int64_t n, int64_t ldx, int32_t* tile, int32_t* splits);

/* Autotuner: time the candidate (tile, splits) configurations for this shape
 * on the current device, with the Gram the library would run for byte input
 * of this shape and pitch (FP4 from n >= 1536 and m n^2 >= 6e10 or when ldx %
 * 16 != 0, else int8), on a
 * scratch matrix in that layout holding a hashed 0/1 pattern of density 1/8,
 * and remember the fastest for every later call with the same shape class
 * and Gram.  Each candidate's time is the median of five launches after a
 * warm-up; the library's heuristic plan is kept unless a candidate is at
 * least 3% faster.  *best_ms receives the chosen plan's time (may be NULL).
 * The tuner file holds one JSON line per entry; lines without the "fp4" field
 * are int8 entries. */
mi_status mi_tune(int64_t m, int64_t n, int64_t ldx, int32_t* tile, int32_t* splits, double* best_ms);

/* Batch autotuner for the persistent mode of mi_all_pairs_batched: runs the
 * caller's batch itself (its data and outputs; every run writes the same
 * results) under candidate plans -- the tile of the datasets whose tile is
 * left to the library (one 256- or 128-wide tile for all, or 128-wide below
 * 512 / 1,024 columns and 256-wide above) and the K-split target (the batch's
 * work over the persistent slots times 1, 2, 4, 8 or 16) -- and remembers
 * the fastest for every later persistent call on a batch with the same
 * signature (the multiset of the datasets' shape classes, as mi_tune's,
 * layouts, Gram choices and explicit tile / split requests).  The
 * library's heuristic plan is kept unless a candidate is at least 3% faster.
 * Times are medians of five runs after a warm-up, on `stream`, which it
 * synchronises.  *best_ms and *heuristic_ms (either may be NULL) receive the
 * chosen and the heuristic plan's times.  Entries are saved and loaded with
 * the tuner file ("batch" lines) and cleared by mi_tuner_clear. */
mi_status mi_tune_batched(const mi_problem* probs, int64_t count, void* stream, double* best_ms,
                          double* heuristic_ms);

/* The plan the persistent mode would run for this batch (tuned or heuristic):
 * per dataset, its tile (mi_tile; MI_TILE_AUTO for n == 0) and K-split count
 * (0 for n == 0), into HOST arrays of `count` entries (either may be NULL).
 * Checks the batch like mi_all_pairs_batched; launches nothing. */
mi_status mi_plan_batched(const mi_problem* probs, int64_t count, int32_t* tiles, int32_t* splits);

mi_status mi_tuner_save(const char* path);   /* JSON lines */
mi_status mi_tuner_load(const char* path);
void mi_tuner_clear(void);

/* Thread-local message describing the last failure on the calling thread. */
const char* mi_last_error(void);

/* Library version string. */
const char* mi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI_H_ */
