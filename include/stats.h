/* stats.h -- C ABI of libstats.so: single-pass sufficient statistics on one
 * MI355X (gfx950) GPU.
 *
 * What is computed (arxiv 2604.23826, section "Data Representation and
 * Sufficient Statistics"): one streaming pass over an N x p table produces
 * the row count N, the column sums s = X^T 1 and the cross products
 * C = X^T X; means, covariance, correlation and principal components are
 * then derived from (N, s, C) alone, without revisiting the rows (same
 * section; section "Principal Component Analysis Results").  Each device
 * call reduces a disjoint subset of rows and partial results are combined
 * (section "Validation and Infrastructure Testing"), which is what
 * stats_accumulate (one chunk) and stats_merge (two handles) do.
 *
 * Numerics (section "Numerical Considerations": X^T X and N mu mu^T must not
 * be formed separately and subtracted in floating point):
 *  - rows are reduced in blocks shifted by the block's first row; integer
 *    columns are reduced exactly and kept as 128-bit integers, so their sums,
 *    cross products and covariances are exact (covariance correctly rounded);
 *  - pairs involving a floating-point column are combined by the pairwise
 *    update of Chan, Golub and LeVeque on (n, mean, centred co-moment).
 *  - identifier columns (flag STATS_COL_IDENTIFIER) are left out of
 *    covariance, correlation and PCA by default (same section).
 *
 * Conventions for every entry point:
 *  - returns STATS_OK (0) or a negative STATS_E_* code; nothing throws or
 *    aborts across the ABI; stats_last_error() gives a thread-local message;
 *  - a handle is not thread-safe; distinct handles are independent;
 *  - after STATS_E_HIP a handle is poisoned: later calls return STATS_E_STATE;
 *  - all work of a handle is ordered on its stream (stats_config.stream or a
 *    stream the library creates); accumulate calls return after enqueueing.
 *    Device and pinned inputs must stay valid and unchanged until the next
 *    stats_sync / stats_finalize / stats_raw on the handle returns.
 *  - the caller owns every input and output buffer; the library owns all
 *    device state of a handle and frees it in stats_close.
 *  - outputs are host arrays, row-major; p x p matrices are full symmetric.
 */
#ifndef STATS_H
#define STATS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STATS_MAX_P 1024
#define STATS_MAX_PLANES 32
#define STATS_MASK_WORDS (STATS_MAX_P / 64)

typedef struct stats_ctx stats_ctx; /* opaque, owned by the library */

/* Two's-complement 128-bit integer, value = hi * 2^64 + lo. */
typedef struct {
  uint64_t lo;
  int64_t hi;
} stats_i128;

enum {
  STATS_OK = 0,
  STATS_E_ARG = -1,      /* invalid argument or configuration */
  STATS_E_STATE = -2,    /* poisoned or wrong-kind handle, or nothing to do */
  STATS_E_HIP = -3,      /* a HIP runtime call failed (handle poisoned) */
  STATS_E_NOMEM = -4,    /* device or pinned allocation failed */
  STATS_E_INEXACT = -5,  /* an integer column left the exact range */
  STATS_E_PARSE = -6,    /* malformed text input */
  STATS_E_MISMATCH = -7, /* stats_merge of incompatible handles */
  STATS_E_IO = -8        /* a file could not be opened or read */
};

/* Column storage types. */
enum { STATS_I32 = 1, STATS_I64 = 2, STATS_F32 = 3, STATS_F64 = 4 };

/* Column flags.  I32 / I64 columns are always integer-valued.  An F32 / F64
 * column flagged INTEGER must hold integers; it is then reduced exactly and
 * every value is checked (a fraction gives STATS_E_INEXACT). */
enum { STATS_COL_INTEGER = 1u, STATS_COL_IDENTIFIER = 2u };

/* Where an input buffer lives. */
enum { STATS_MEM_DEVICE = 0, STATS_MEM_HOST_PINNED = 1, STATS_MEM_HOST = 2 };

/* Arithmetic of the cross-product pass for wide tables (p > 16). */
enum {
  STATS_PREC_FP64 = 0,  /* FP64 throughout */
  STATS_PREC_SPLIT = 1, /* fixed-point digits of the block-shifted values on
                           the matrix cores, exact integer (FP32 row-major
                           layout: int8 digits, blocks outside the sampled
                           grid redone in FP64) or exact FP32 (other layouts:
                           BF16 digits, 2^-27 of the block range) sums,
                           FP64 merge */
  STATS_PREC_AUTO = 2   /* p <= 16: FP64; wider: split when the FP32
                           row-major int8 kernel applies, else FP64 */
};
/* Former name of STATS_PREC_SPLIT. */
enum { STATS_PREC_SPLIT_BF16 = STATS_PREC_SPLIT };

/* Configuration flags. */
enum {
  STATS_CFG_TIMING = 1u,   /* record per-kernel HIP event timings */
  STATS_CFG_PAIRWISE = 2u  /* missing values: NaN entries are absent, statistics per
                              pair of columns over the rows where both are present
                              (stats_finalize_pairwise); p <= 16, FP32/FP64 columns */
};

/* Column c of a row: element of type dtype at byte offset byte_offset inside
 * row r of plane `plane`, i.e. at planes[plane] + r * row_stride[plane] +
 * byte_offset. */
typedef struct {
  int32_t dtype;
  int32_t plane;
  int32_t byte_offset;
  uint32_t flags;
} stats_column;

typedef struct {
  int32_t p;                  /* columns, 1..STATS_MAX_P */
  const stats_column* cols;   /* p descriptors (copied by stats_open) */
  int32_t n_planes;           /* 1..STATS_MAX_PLANES */
  int64_t row_stride[STATS_MAX_PLANES]; /* bytes between rows of each plane */
  int32_t precision;          /* STATS_PREC_* */
  int32_t device;             /* HIP device ordinal */
  void* stream;               /* hipStream_t to order work on, or NULL */
  int64_t staging_rows;       /* rows per pinned staging slot; 0 = 2^28 */
  int64_t block_rows;         /* rows per shifted block; 0 = automatic */
  uint32_t flags;             /* STATS_CFG_* */
} stats_config;

typedef struct {
  uint64_t column_mask[STATS_MASK_WORDS]; /* bit c set = keep column c; all 0 =
                                             every column not flagged IDENTIFIER */
  int32_t ddof;         /* divisor N - ddof; 1 = sample covariance */
  int32_t pca_on;       /* 0 = correlation matrix (default), 1 = covariance */
  int32_t want_vectors; /* 0 = eigenvalues only: eigvec is not written */
} stats_finalize_opts;

/* Opens a handle on cfg->device for one table whose rows are described by
 * cfg's columns (section "Data Representation and Sufficient Statistics":
 * fixed-width records, row-major, with contiguous access from host and
 * device; several planes allow column-major data as well).  Checks:
 * 1 <= p <= STATS_MAX_P; planes in range; each column's element inside its
 * row stride; INTEGER only on integer-capable columns; block_rows 0 or a
 * multiple of 1024.  On error *out is NULL. */
int stats_open(const stats_config* cfg, stats_ctx** out);

/* Adds nrows rows: the single streaming pass of section "Data
 * Representation and Sufficient Statistics" (column sums and X^T X of a
 * chunk, shifted by each block's first row as section "Numerical
 * Considerations" requires), merged into the handle.  Chunks streamed from
 * host memory follow section "System Overview" (storage -> host memory ->
 * GPU).  planes[k] is the base of plane k (device address for
 * STATS_MEM_DEVICE; host address otherwise).  Device planes must be 16-byte
 * aligned.  Host input is streamed in chunks of staging_rows rows through two
 * device staging slots, the copy of one chunk (on a second stream)
 * overlapping the reduction of the previous one: HOST_PINNED input is copied
 * by DMA straight from the caller's page-locked buffer; pageable HOST input is
 * first copied by the CPU into two page-locked slots and may be reused once
 * the call returns.  nrows == 0 is a no-op. */
int stats_accumulate(stats_ctx* h, const void* const* planes, int64_t nrows, int32_t mem_kind);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reduction as stats_accumulate with STATS_MEM_DEVICE input, for handles of
 * p <= 16 columns (else STATS_E_ARG), performing no allocation.  The block
 * records of each launch go to one fixed device array of
 * STATS_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends) instead
 * of handle-owned memory; rows are cut into launches whose records fit it.
 * Every call on one GPU shares that array: calls that overlap in time on the
 * same GPU (different streams, or host threads) race and must be ordered by
 * the caller.  The first call on a device looks the array's address up
 * (hipGetSymbolAddress); later calls only launch kernels.  Results equal
 * stats_accumulate's (integer columns bit for bit; the 128-byte FP64 record
 * layout with 11 <= p <= 16 takes the per-lane kernels here, so floating
 * entries may differ in summation order). */
#define STATS_NOALLOC_SCRATCH_BYTES (8u << 20)
int stats_accumulate_noalloc(stats_ctx* h, const void* const* planes, int64_t nrows);

/* Adds nrows fixed-width records read from a file: the storage -> host
 * memory -> GPU path of section "System Overview", on the binary form that
 * section "Data Representation and Sufficient Statistics" makes canonical.
 * The handle must have one plane; record r starts at byte
 * offset + r * row_stride[0] of the file at path.  Chunks of staging_rows
 * records are read by positioned reads on up to eight host threads into two
 * page-locked slots; each chunk's read overlaps the copy and reduction of
 * the previous chunk (same two-slot ring as STATS_MEM_HOST input).  The call
 * returns once every row has been read (the reduction of the last chunk may
 * still run).  STATS_E_IO: the file cannot be opened, is shorter than
 * offset + nrows * row_stride[0] bytes, or a read fails. */
int stats_accumulate_file(stats_ctx* h, const char* path, int64_t offset, int64_t nrows);

/* Adds the complete lines of a CSV text chunk, parsed on the GPU and fed
 * straight into the same accumulation (the paper's first pipeline streamed
 * CSV in fixed-size chunks: section "Validation and Infrastructure Testing";
 * its parsing cost: section "Data Representation and Sufficient
 * Statistics").  Lines must end in '\n'; one row per line, p fields
 * separated by ',', integer columns in decimal, floating columns as decimal
 * floating-point text (parsed with correct rounding; magnitudes below 1e73
 * with the last written digit's decimal exponent >= -57 always convert,
 * fields beyond about 2.3e74 or with a later last digit are malformed).
 * Only complete lines
 * are consumed unless is_last != 0, when a final unterminated line counts
 * too; *bytes_consumed receives the bytes used (the caller passes the rest
 * again at the front of the next chunk).  A malformed field gives
 * STATS_E_PARSE with the byte offset of its line in stats_last_error(),
 * counted from the start of the handle's text: the bytes that earlier
 * calls since stats_open / stats_reset consumed included. */
int stats_accumulate_text(stats_ctx* h, const char* buf, int64_t nbytes, int32_t mem_kind,
                          int32_t is_last, int64_t* bytes_consumed);

/* Converts the complete lines of a CSV text chunk into fixed-width binary
 * rows on the GPU: the one-time conversion of section "Data Representation
 * and Sufficient Statistics" (the binary form replaces repeated CSV parsing),
 * whose output is then checked as in section "Validation and Infrastructure
 * Testing" (file size, row count, layout, sample records).  The handle only
 * describes the layout: line k of the chunk becomes row k of the output,
 * field c written at out_planes[cols[c].plane] + k * row_stride[plane] +
 * cols[c].byte_offset (device memory) as cols[c].dtype; its statistics are
 * not touched.  Text rules and chunking as stats_accumulate_text (the same
 * parser: integer columns exactly, decimal columns correctly rounded to
 * FP64; *bytes_consumed = bytes of the complete lines).  Column types: I32,
 * I64 or F64 for integer columns, F64 for decimal columns (else STATS_E_ARG;
 * FP32 output would round twice).  *rows_out = lines converted; the chunk
 * may hold at most max_rows lines (else STATS_E_ARG, nothing written).
 * STATS_E_PARSE: a malformed field, an integer outside int32 for an I32
 * column or beyond 2^53 for an F64 one; the byte offset of its line (from
 * the start of the handle's text, as above) is in stats_last_error() and
 * the output rows are then unspecified.  Returns
 * after the conversion has finished.  p <= 16. */
int stats_text_to_binary(stats_ctx* h, const char* buf, int64_t nbytes, int32_t mem_kind,
                         int32_t is_last, void* const* out_planes, int64_t max_rows,
                         int64_t* rows_out, int64_t* bytes_consumed);

/* Statistics with missing values (handle opened with STATS_CFG_PAIRWISE):
 * the extension to incomplete data that section "Limitations and Future
 * Work" names.  A NaN entry is absent; for every pair of columns (i, j) the
 * rows where both are present form the pair's sample (pairwise deletion).
 * stats_accumulate (any memory kind) and stats_merge (two pairwise handles)
 * work as for complete data; stats_raw, stats_finalize, stats_serialize and
 * text input return STATS_E_STATE on such a handle.  Outputs, host arrays
 * (any may be NULL): n_out p x p counts n_ij (n_ii = present entries of
 * column i); mean_out p means of each column over its own present entries;
 * cov_out p x p, cov_ij = sum over the pair's rows of (x_i - m_i)(x_j - m_j)
 * / (n_ij - ddof) with m_i, m_j the means over those same rows (NaN when
 * n_ij <= ddof); corr_out p x p, corr_ij = that co-moment over the square
 * root of the two centred sums of squares over the same rows (diagonal 1,
 * NaN when a column is constant or absent on them).  Such a matrix need not
 * be positive semi-definite, so no components are formed from it.  FP64
 * throughout, no exact integer path. */
int stats_finalize_pairwise(stats_ctx* h, int32_t ddof, int64_t* n_out, double* mean_out,
                            double* cov_out, double* corr_out);

/* Batched groups: a handle holding ngroups independent sets of the
 * statistics of section "Data Representation and Sufficient Statistics"
 * (one per group of rows), for many tables of uneven size in one launch. */
int stats_open_groups(const stats_config* cfg, int32_t ngroups, stats_ctx** out);

/* Adds rows to every group in one launch: group g receives the rows
 * [row_offsets[g], row_offsets[g+1]) of the planes (ngroups + 1 offsets,
 * non-decreasing, host memory).  Repeated calls keep adding. */
int stats_accumulate_segmented(stats_ctx* h, const void* const* planes,
                               const int64_t* row_offsets, int32_t mem_kind);

/* dst := statistics of rows(dst) and rows(src); src unchanged: the
 * combination of the partial results of disjoint row subsets (section
 * "Validation and Infrastructure Testing"; the partials are combined without
 * forming X^T X - N mu mu^T, section "Numerical Considerations").  Both must
 * have the same columns (else STATS_E_MISMATCH) and be single-group.  A
 * deferred error of src (STATS_E_INEXACT, STATS_E_PARSE) carries over to dst
 * and is reported by dst's next sync, raw or finalize. */
int stats_merge(stats_ctx* dst, const stats_ctx* src);

/* Clears the statistics of the handle (all groups) so it can take a new
 * dataset; buffers and configuration are kept.  Stream-ordered. */
int stats_reset(stats_ctx* h);

/* Waits for all work of the handle; reports a deferred STATS_E_INEXACT or
 * STATS_E_PARSE. */
int stats_sync(stats_ctx* h);

/* The sufficient statistics (N, s, C) themselves (section "Data
 * Representation and Sufficient Statistics").  s_int / C_int hold exact
 * values where the column (pair) is integer, zero elsewhere; s_f64 / C_f64
 * hold every entry in FP64 (integer entries correctly rounded);
 * exact_mask[i*p+j] = 1 where the entry is exact.  C arrays are p x p.  Any
 * output pointer may be NULL. */
int stats_raw(stats_ctx* h, int64_t* n, stats_i128* s_int, double* s_f64, stats_i128* C_int,
              double* C_f64, uint8_t* exact_mask);

/* Means, covariance, correlation and PCA of the kept columns (p' of them,
 * written to *p_out), from the statistics alone (section "Data
 * Representation and Sufficient Statistics"; the identifier is left out by
 * default, section "Numerical Considerations"; eigenpairs, variance % and
 * cumulative % as in section "Principal Component Analysis Results",
 * Table 3).  cov = centred co-moment / (N - ddof), correctly
 * rounded for integer pairs; corr = cov_ij / sqrt(cov_ii cov_jj) with a unit
 * diagonal (NaN where a variance is zero); eigenpairs of corr (or cov) by
 * FP64 Jacobi on the GPU, eigenvalues descending, eigvec row k = component k
 * with unit norm and its largest-magnitude entry positive (lowest index on
 * ties); var_pct = 100 lambda / sum(lambda); cum_pct its running sum.
 * Arrays: mean p', cov / corr / eigvec p' x p', eigval / var_pct / cum_pct p'.
 * Any output pointer may be NULL.  N <= ddof gives STATS_E_STATE. */
int stats_finalize(stats_ctx* h, const stats_finalize_opts* opts, int32_t* p_out, double* mean,
                   double* cov, double* corr, double* eigval, double* eigvec, double* var_pct,
                   double* cum_pct);

/* Per-group results of a groups handle: n_out[ngroups], mean_out[ngroups *
 * p'], cov_out[ngroups * p' * p'] (any may be NULL).  Groups with N <= ddof
 * get NaN covariances. */
int stats_finalize_groups(stats_ctx* h, const stats_finalize_opts* opts, int32_t* p_out,
                          int64_t* n_out, double* mean_out, double* cov_out);

/* stats_raw for group g of a groups handle. */
int stats_group_raw(stats_ctx* h, int32_t g, int64_t* n, stats_i128* s_int, double* s_f64,
                    stats_i128* C_int, double* C_f64, uint8_t* exact_mask);

/* Checkpoint: the statistics of a single-group handle as bytes (partial
 * results moved to the host for combination, section "Validation and
 * Infrastructure Testing").  With buf
 * NULL, *len receives the size needed; otherwise *len is the capacity and
 * receives the size written. */
int stats_serialize(stats_ctx* h, void* buf, size_t* len);

/* New handle with cfg's columns holding the checkpoint in buf (same column
 * layout required, else STATS_E_MISMATCH). */
int stats_deserialize(const void* buf, size_t len, const stats_config* cfg, stats_ctx** out);

/* Kernel timing of a handle opened with STATS_CFG_TIMING: number of launches
 * and total milliseconds of kernel `which` (STATS_K_*) measured with HIP
 * events on the handle's stream, up to the last stats_sync. */
enum { STATS_K_ACCUM = 0, STATS_K_MERGE = 1, STATS_K_FINALIZE = 2, STATS_K_SYRK = 3,
       STATS_K_SEGMENTED = 4, STATS_K_TEXT = 5, STATS_K_COPY = 6, STATS_K_COUNT = 7 };
int stats_kernel_time(stats_ctx* h, int32_t which, int64_t* launches, double* total_ms);

/* Measured read bandwidth (a measurement aid, not part of the statistics):
 * the second denominator, beside the 8 TB/s HBM specification, for the
 * achieved bandwidth of the reduction kernels.  For each of the n device
 * buffers one kernel reads its nbytes[k] / 16 whole 16-byte vectors once
 * (non-temporal loads; a tail below 16 bytes is not read) and discards them.
 * bufs[k]: device address, 16-byte aligned unless nbytes[k] < 16.  Work is
 * ordered on `stream` (hipStream_t, NULL = default stream); the call waits
 * for it and stores the summed kernel time in ms into *ms_out (HIP events).
 * Errors: STATS_E_ARG (NULL, negative or unaligned arguments), STATS_E_HIP. */
int stats_read_probe(const void* const* bufs, const int64_t* nbytes, int32_t n, void* stream,
                     double* ms_out);

/* Releases the handle (NULL-safe; waits for its work first). */
void stats_close(stats_ctx* h);

/* Thread-local message describing the last error on this thread. */
const char* stats_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STATS_H */
