// Wide-table (p > 16) kernels: shared definitions.
#pragma once
#include "common.hpp"

namespace st {
namespace wide {

constexpr int kThreads = 256;
constexpr int KR = 32;  // rows staged per step

enum { MODE_FP64 = 0, MODE_SPLIT = 1 };

// One column slot: element r at base + r * stride, of type kind (STATS_*).
struct SlotInfo {
  const char* base;
  int64_t stride;
  int32_t kind;
  uint8_t chk;    // FP column flagged INTEGER: check values
  uint8_t isint;  // integer column: shift stored as int64
  uint8_t pad[2];
};

struct Args {
  const SlotInfo* slots;  // p entries (device)
  int p;
  const int2* tiles;      // (A, B) super-group pairs with A <= B (device)
  int ntiles;
  int64_t nblocks;
  int64_t nrows;
  int64_t R;              // rows per block (multiple of KR)
  uint64_t* rec;          // block records
  DevStatus* status;
};

// Batched groups: row tile [r0, r1) of group `group` (rows relative to the
// planes' base).
struct SegTile {
  int64_t r0, r1;
  int32_t group;
  int32_t pad;
};

struct SegArgs {
  const SegTile* rowtiles;            // row tiles, sorted by group (device)
  const int64_t* nrowtiles;           // number of row tiles (device word)
  unsigned long long* counter;        // work queue head (device word)
  int64_t tile_rows = 0;              // > 0: no table; item k is rows [k tile_rows,
  int64_t total_rows = 0;             //   min((k + 1) tile_rows, total_rows))
};

// FP32 matrix on the int8 matrix cores (wide_syrk.hip): F vector columns at
// consecutive 4-byte offsets of one plane, up to kSyrkMaxExtra other columns.
constexpr int kSyrkGroup = 128;
constexpr int kSyrkMaxExtra = 2;
constexpr int kSyrkMaxPairs = 72;  // F <= 1024: at most 8 groups; every pair in two halves

struct SyrkExtra {
  const char* base;  // element of row 0 of the launch
  int64_t stride;
  int32_t kind;      // STATS_*
  uint8_t chk;       // FP column flagged INTEGER: check values
  uint8_t isint;     // integer column: shift stored as an integer
  uint8_t pad[2];
};

struct SyrkArgs {
  const char* xbase;        // vector column 0 in row 0 of the launch (16-byte aligned)
  int64_t xstride;          // row stride in bytes (multiple of 16)
  int F;                    // vector columns (multiple of 4), slots 0..F-1
  int ne;                   // extra columns, slots F..F+ne-1
  SyrkExtra ex[kSyrkMaxExtra];
  int npairs;
  int2 pairs[kSyrkMaxPairs];  // (A + 16 half, B): group pairs A <= B, each in two halves
  int p;                    // F + ne
  const int32_t* col_of;    // user column of each slot (device)
  int64_t nblocks, nrows, R;  // R: rows per block (multiple of 64)
  uint64_t* rec;
  DevStatus* status;
  int* ovf;                 // per block: nonzero = recompute in FP64 (device)
  int* sexp;                // grid exponents, nblocks x F (device; written by the matrix-core kernel)
};

}  // namespace wide

void launch_syrk_split(const wide::SyrkArgs& a, hipStream_t s);
// FP64 records again for the blocks whose ovf flag is set (a.rec, a.R, a.nrows,
// a.nblocks as for the launch that set them).
void launch_wide_fixup(const wide::Args& a, int st, const int* ovf, hipStream_t s);

// Persistent segmented launch (zeroes the queue first): nwg workgroups.
void launch_seg(const wide::Args& a, const wide::SegArgs& g, int st, int nwg, hipStream_t s);
// The same for FP64 records of 256 bytes, column c at byte 8c, p <= 32.
void launch_seg_aos64(const wide::Args& a, const wide::SegArgs& g, int nwg, hipStream_t s, int row_bytes = 256);

// st = super-group width (32 or 64); mode = MODE_FP64 or MODE_SPLIT.
void launch_wide(const wide::Args& a, int st, int mode, hipStream_t s);
void launch_wide_split(const wide::Args& a, int st, hipStream_t s);

}  // namespace st
