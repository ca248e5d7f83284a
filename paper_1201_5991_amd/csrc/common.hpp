// Shared definitions of the MI355X multilevel BDDC library: tile layout,
// status plumbing and small host helpers.
//
// Every dense matrix in the library (subdomain matrices, augmented local
// problems, coarse matrices) is stored "tile-packed lower": the matrix is cut
// into 64x64 tiles, only tiles (r, s) with r >= s are stored, tiles are laid
// out column after column (tile column s holds tiles s..nt-1), and each tile
// is a contiguous 64x64 column-major block.  Diagonal tiles hold both
// triangles.  A tile is one 32 KiB (FP64) or 16 KiB (FP32) coalesced burst.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>

#include <hip/hip_runtime.h>

#include "../../include/mlbddc.h"

namespace mlbddc {

constexpr int TS = 64;             // tile edge
constexpr int TE = TS * TS;        // elements per tile

// Offset (in tiles) of tile (r, s), r >= s, in a tile-packed lower matrix of nt x nt tiles.
__host__ __device__ inline int64_t tile_col_start(int64_t s, int64_t nt) { return s * nt - s * (s - 1) / 2; }
__host__ __device__ inline int64_t tile_index(int64_t r, int64_t s, int64_t nt) { return tile_col_start(s, nt) + (r - s); }
__host__ __device__ inline int64_t packed_tiles(int64_t nt) { return nt * (nt + 1) / 2; }
// Storage slot of tile (r, s) of matrix `item`: matrices with a tile map
// (tmap_off[item] >= 0) store only the tiles some kernel touches, the map
// gives each packed-lower tile index its slot (-1: not stored); the others
// are dense packed-lower (slot = tile index).
__host__ __device__ inline int64_t tile_slot(const int32_t* tmap, const int64_t* tmap_off, int item, int64_t r, int64_t s,
                                             int64_t nt) {
  const int64_t ti = tile_index(r, s, nt);
  if (!tmap) return ti;
  const int64_t o = tmap_off[item];
  return o < 0 ? ti : (int64_t)tmap[o + ti];
}

// Element offset of entry (p, q) (p/64 >= q/64 required) in a tile-packed matrix.
__host__ __device__ inline int64_t packed_offset(int64_t p, int64_t q, int64_t nt) {
  return tile_index(p / TS, q / TS, nt) * TE + (q % TS) * TS + (p % TS);
}

inline int64_t round_up(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

// Factorization task packing: item (16 bits), r (13), s (13), kf (13) and
// nk (8): an update task sums the products of tile columns kf .. kf + nk.
constexpr int64_t MAX_TASK_ITEMS = 1 << 16;
constexpr int MAX_TASK_NK = 255;
__host__ __device__ inline uint64_t pack_task(uint64_t item, uint64_t r, uint64_t s, uint64_t kf, uint64_t nk = 0) {
  return item | (r << 16) | (s << 29) | (kf << 42) | (nk << 55);
}
__host__ __device__ inline int task_item(uint64_t t) { return (int)(t & 0xFFFFull); }
__host__ __device__ inline int task_r(uint64_t t) { return (int)((t >> 16) & 0x1FFF); }
__host__ __device__ inline int task_s(uint64_t t) { return (int)((t >> 29) & 0x1FFF); }
__host__ __device__ inline int task_kf(uint64_t t) { return (int)((t >> 42) & 0x1FFF); }
__host__ __device__ inline int task_nk(uint64_t t) { return (int)((t >> 55) & 0xFF); }
// Bit 63: a task of the second elimination phase of a two-phase item, whose
// trailing block the first phase leaves as the negative of the matrix the
// second phase factors.  Such tasks read that block with the opposite sign:
// the diagonal factor negates its tile on load, a panel product stores
// -(T W^T), an update adds its product instead of subtracting it.  Tiles the
// second phase does not factor keep the opposite sign to the end.
constexpr uint64_t TASK_NEG = 1ull << 63;
__host__ __device__ inline bool task_neg(uint64_t t) { return (t >> 63) != 0; }

// Kinds of factorization steps (one launch each; L_NEGATE is no longer scheduled).
enum LaunchKind { L_NEGATE = 0, L_INPANEL = 1, L_DIAG = 2, L_PANEL = 3, L_TRAIL = 4 };

struct Error {
  mlbddc_status status = MLBDDC_OK;
  int level = 0, subdomain = -1, column = -1;
  std::string message;
};

}  // namespace mlbddc
