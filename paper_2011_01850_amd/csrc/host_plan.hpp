// Host-side planning of libgmres: the tables that the engine builds from a
// system's CSR structure before any kernel runs (the Arnoldi product's row
// blocks, the split of the persistent basis passes, the ILU(0) dependency
// levels, the sliced ELL layout, the size checks).
//
// Plain C++17 with no HIP dependency, so the same code is also compiled on
// the host alone, with the address and undefined-behaviour sanitizers, and
// checked there against brute-force recomputation of every table.
#pragma once

#include <stdint.h>

#include <vector>

namespace gm {

// Rows are grouped in tiles of kTile rows: one row per thread of a kBlock
// workgroup.  Every system is padded to a whole number of tiles (padding rows
// of the basis, w, x and b are zero and stay zero), so no kernel needs tail
// handling inside a tile.
constexpr int kBlock = 256;
constexpr int kTile = 256;

// SpMV row sums follow one canonical order that depends only on the row's
// length len: T = row_lanes(len) partial sums, partial l adding products
// l, l + T, l + 2T, ... in turn, then the T partials combined by a fixed
// butterfly.  T doubles from 1 while it stays <= 16 and every partial still
// gets at least kRowLanePer products.  (constexpr: usable in device code.)
constexpr int kRowLaneMax = 16;
constexpr int kRowLanePer = 4;
constexpr int row_lanes(int len) {
  int T = 1;
  while (T < kRowLaneMax && 2 * T * kRowLanePer <= len) T *= 2;
  return T;
}

namespace plan {

// Sizes that the kernels can address: per system n and nnz below 2^31, the
// tile-padded row count and the total non-zeros (plus the SpMV pad) below
// 2^31, and the basis, max(m + 1, 4) columns of the padded rows at
// elem_bytes each, below 2^32 bytes (32-bit buffer offsets).
bool sizes_fit(int32_t nsys, const int64_t* n, const int64_t* nnz, int m, int64_t elem_bytes);

// Entries [i0, i1) of one system's row pointer v (n rows, nnz entries) do not
// decrease; the successor of the last row's entry is nnz.  (The caller checks
// v[0] = 0 and v[n] = nnz.)
bool row_ptr_piece_ok(const int32_t* v, int64_t n, int32_t nnz, int64_t i0, int64_t i1);

// Adaptive-CSR row blocks over global rows [r_begin, r_end) of the row
// pointer rp: up to kBlock rows (2 kBlock with budgets of 4096 and more)
// whose non-zeros fit `budget`, or a single longer row.  Appends each block's
// first row to rb and, if lanes is given, row_lanes of its longest row.
void build_row_blocks(const int32_t* rp, int64_t r_begin, int64_t r_end, int budget, std::vector<int32_t>& rb,
                      std::vector<int32_t>* lanes);

// Work split of a persistent basis pass over the tiles of nsys systems
// (system k owns tiles [t0[k], t0[k] + nt[k]), consecutive, from 0) for G
// workgroups: workgroup b owns tiles [b T / G, (b + 1) T / G), cut at system
// boundaries into segments.
struct TileSplit {
  std::vector<int32_t> bseg0;    // [G + 1] first segment of each workgroup
  std::vector<int32_t> seg_t0;   // first tile of each segment
  std::vector<int32_t> seg_nt;   // tiles of each segment
  std::vector<int32_t> seg_sys;  // system of each segment
  std::vector<int32_t> sys_sg0;  // first segment of each system (-1 if it has none)
  std::vector<int32_t> sys_nsg;  // segments of each system
};
TileSplit split_tiles(const int32_t* t0, const int32_t* nt, int32_t nsys, int G);

// ILU(0) plan of a padded global CSR with ld rows: the diagonal's position in
// every row, and the rows ordered by dependency level of the lower triangle
// (a row's level is one more than the highest level among the rows its
// strictly lower entries name; rows with none are level 0).  Padding rows
// (empty) are level 0 with diag = their (empty) start.  Needs every stored
// row to hold its diagonal and its columns in strictly increasing order (the
// factorisation merges sorted column lists).
struct IluPlan {
  std::vector<int32_t> diag;   // [ld] position of a_rr
  std::vector<int32_t> order;  // [ld] rows by level, ascending row order within a level
  std::vector<int32_t> count;  // [depth_l + 1] order[count[l] .. count[l + 1]) is level l
  int32_t depth_l = 0;         // levels of the lower triangle
  int32_t depth_u = 0;         // levels of the upper triangle (the U sweeps' exact count)
};
enum IluStatus { ILU_OK = 0, ILU_NO_DIAGONAL = 1, ILU_UNSORTED = 2 };
int ilu_plan(const int32_t* rp, const int32_t* ci, int64_t ld, IluPlan& out);

// Sliced ELL layout of a padded CSR with ld rows (a multiple of 64): slice s
// holds rows [64 s, 64 s + 64) column-major with the width of its longest
// row, from off[s]; len[r] is row r's length.  Returns false (off and len
// unspecified) when a row has 2 kRowLanePer entries or more (its canonical
// sum would not be its plain sum) or the padded copy reaches 2^31 entries.
bool sell_layout(const int32_t* rp, int64_t ld, std::vector<int32_t>& off, std::vector<uint8_t>& len);
// The same in two steps, for callers that split the rows: the widths of
// slices [s0, s1) into w[s0 .. s1), then the offsets from all nslice widths
// (false when a width reaches 2 kRowLanePer or the total 2^31).
void sell_widths(const int32_t* rp, int64_t s0, int64_t s1, int32_t* w);
bool sell_offsets(const int32_t* w, int64_t nslice, std::vector<int32_t>& off);

// Rows per thread of a system of n rows in the persistent batch kernel
// (1024 threads): the smallest power of two that covers n, at most kMaxPR.
int persistent_rows_per_thread(int64_t n, int max_rows);

}  // namespace plan
}  // namespace gm
