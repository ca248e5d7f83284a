// Device kernels of the MI355X multilevel BDDC library (declarations of the
// host-side launchers).  All launchers are asynchronous on `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace mlbddc {

// ---------------------------------------------------------------- assembly
// Add element matrices into tile-packed subdomain matrices.  Elements listed
// in `elems` (one colour: no two share a subdomain DOF) are processed; element
// e of subdomain el_sub[e] adds entry (a, c) of its matrix at local position
// (el_local[ptr+a], el_local[ptr+c]).  The element matrix is
// scale[e] * Kref (Kref != null) or ekc[ekc_off[e] ...] (row-major, nloc^2).
// Subdomain b's matrix is tile-mapped when tmap is set and tmap_off[b] >= 0;
// an entry in a tile the map does not store is skipped and sets *err to 1.
template <typename T>
void launch_assemble(hipStream_t st, const int64_t* elems, int64_t n, const int32_t* el_local_ptr,
                     const int32_t* el_local, int nd, const int32_t* el_sub, const int64_t* sub_off, const int32_t* sub_nt,
                     const double* Kref, const double* scale, const int64_t* ekc_off, const double* ekc, T* A,
                     const int32_t* tmap, const int64_t* tmap_off, int32_t* err);
// Zero `bytes` bytes at p (16-byte aligned, bytes a multiple of 16) with at
// most max_blocks workgroups (fewer leave HBM bandwidth to concurrent work).
void launch_zero(hipStream_t st, void* p, size_t bytes, int max_blocks = 16384);

// Set entries A[row0+i][col0+i] = val for every segment (tile-packed
// matrices; `item` indexes the tile map, -1 = dense packed-lower).
struct DiagSeg { int64_t off; int32_t nt; int32_t row0, col0, count; double val; int32_t item = -1; };
template <typename T>
void launch_set_diag(hipStream_t st, const DiagSeg* segs, int64_t nseg, int32_t max_count, T* A,
                     const int32_t* tmap = nullptr, const int64_t* tmap_off = nullptr);

// ---------------------------------------------------------- factorization
struct FactorArgs {
  const uint64_t* tasks;
  const int64_t* off;      // element offset of each item's matrix
  const int32_t* nt;       // tiles per side of each item
  const int64_t* inv_off;  // element offset of each item's inverse diagonal tiles
  int32_t* err;            // [0] = failing item + 1, [1] = column
  const int32_t* tmap;     // tile maps (tile_slot), or null: every matrix dense packed-lower
  const int64_t* tmap_off;
  int stage = 32;          // columns staged per step of the tile products: 16, 32 or 64
  int pstage = 0;          // the same for the panel products (one tile times W); 0: stage
  int shape = 16;          // FP32 MFMA shape of the tile products: 16 (16x16x4) or 32 (32x32x2)
};
template <typename T>
void launch_factor_step(hipStream_t st, int kind, int k, const FactorArgs& a, int64_t first, int64_t count, T* A, T* Inv);

// ----------------------------------------------------- preconditioner set-up
// Copy the interface block (tile rows/cols t0.. of the FP64 K matrices) into
// the top-left block of the preconditioner matrices, converting to TP.
struct CopyDesc { int64_t src_off; int32_t src_nt, src_t0; int64_t dst_off; int32_t dst_nt, nblk; };
template <typename TK, typename TP>
void launch_copy_block(hipStream_t st, const CopyDesc* d, int32_t nitems, int32_t max_blk, const TK* K, TP* P);

// Add the constraint penalty rho_c c_c^T c_c to the S block and write the C
// rows; rho_c (the sum of the glob's diagonal entries of S) goes to rho[row].
struct ConsDesc { int64_t kdiag_off; int32_t k_nt, k_g0; int64_t p_off; int32_t p_nt, c_row0; int32_t ptr0, ptr1; };
template <typename TK, typename TP>
void launch_constraints(hipStream_t st, const ConsDesc* d, int64_t nrows, const int32_t* cols, const TK* K, TP* P,
                        double* rho);

// Coarse matrices K_Ci = Psi_i^T S_i Psi_i = A_i^{-1} - W_i, read from the
// eliminated constrained problem (its coarse block holds -A_i^{-1}) and the
// penalties W_i = diag(rho); written row-major nc x nc (FP64) at out_off.
struct KcDesc {
  int64_t p_off; int32_t p_nt, p_c0;    // preconditioner matrix; first tile of its coarse block
  int32_t nc;                           // coarse DOFs of the subdomain
  int64_t out_off;                      // output offset (nc x nc)
  int64_t rho_off;                      // first constraint row of the subdomain
};
template <typename TP>
void launch_coarse_matrix(hipStream_t st, const KcDesc* d, int32_t nitems, int32_t max_nc, const TP* P, const double* rho,
                          double* out);

// ------------------------------------------------------------------ apply
// Batched tile-block matrix-vector products  y = alpha * op(A_blk) x (+ y).
enum MvMode { MV_SYM = 0, MV_N = 1, MV_T = 2 };
struct MvDesc {
  int64_t a_off; int32_t a_nt;   // tile-packed matrix
  int32_t r0, nr, c0, nc;        // block: tile rows r0..r0+nr-1, tile cols c0..c0+nc-1
  int64_t x_off, y_off;          // vector offsets (x has nc*64 (N, SYM) or nr*64 (T) entries)
  int64_t p_off;                 // partial-sum scratch offset (nr*nc*64 entries)
  const int32_t* env;            // optional first nonzero tile column per row of A (global tile index) or null
  // Valid rows / columns of the block (the rest of its last tile row / column
  // is padding).  k_mv_tiles reads no padding entry of A or x and no
  // upper-triangle entry of a diagonal tile of a symmetric block (it uses the
  // lower triangle for both products); its outputs at padded positions are
  // unspecified.  (k_mv_rows reads whole tiles: there padded entries of x
  // must be finite.)
  int32_t vr = 1 << 30, vc = 1 << 30;
};
// Products with at most SMALL_MV_TILES tiles in all run as one launch with a
// workgroup per output tile; larger ones as a workgroup per tile plus a
// reduction of the partial tiles.
constexpr int64_t SMALL_MV_TILES = 64;
// y = alpha (A1 x + A2 x2) (+ y) for two small product sets whose items
// write the same output tiles (item i of both: equal output count and y_off),
// in one launch.
template <typename TA, typename TX, typename TY>
void launch_tile_mv_sum(hipStream_t st, int mode, const MvDesc* d, int mode2, const MvDesc* d2, int32_t nitems,
                        int32_t max_out_tiles, const TA* A, const TX* x, const TX* x2, TY* y, double alpha, bool accumulate);
// ev0 / ev1 (optional): recorded on `st` right before and after the product
// kernel itself (k_mv_tiles or k_mv_rows), for kernel timing.  tpw = 2: two
// tiles per workgroup, groups2 workgroups with per-item prefix group_prefix2
// (ceil(tiles / 2) per item); else one tile per workgroup (tile_prefix).
template <typename TA, typename TX, typename TY>
void launch_tile_mv(hipStream_t st, int mode, const MvDesc* d, int32_t nitems, int64_t total_tiles,
                    const int64_t* tile_prefix, const TA* A, const TX* x, TY* y, double alpha, bool accumulate,
                    TA* partials, int32_t max_out_tiles, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int tpw = 1,
                    int64_t groups2 = 0, const int64_t* group_prefix2 = nullptr);

// out[i] = (w ? w[i] : 1) * in[idx[i]] (0 where idx < 0), converting types.
template <typename TI, typename TO>
void launch_gather(hipStream_t st, int64_t n, const int32_t* idx, const double* w, const TI* in, TO* out);
// out[g] = beta*out[g] + sum_{j in ptr[g]..ptr[g+1]} (w ? w[list[j]] : 1) * (in[list[j]] (+ in2[list[j]]))
// (FP64 accumulation; in2 optional)
template <typename TI>
void launch_seg_reduce(hipStream_t st, int64_t n, const int64_t* ptr, const int64_t* list, const double* w, const TI* in,
                       double* out, double beta, const TI* in2 = nullptr);
// out[g] = base[bidx[g]] + sum_{j in ptr[g]..ptr[g+1]} in[list[j]]  (FP64): a gather and a
// segmented sum in one launch.
void launch_gather_seg(hipStream_t st, int64_t n, const int32_t* bidx, const double* base, const int64_t* ptr,
                       const int64_t* list, const double* in, double* out);
// out[i1[i]] = in1[i] (i1 >= 0), i < n1, and out[i2[i]] = in2[i], i < n2: two scatters to
// disjoint targets in one launch.
template <typename TI>
void launch_scatter2(hipStream_t st, int64_t n1, const int32_t* i1, const TI* in1, int64_t n2, const int32_t* i2,
                     const double* in2, double* out);
// out[idx[i]] = in[i] for idx >= 0 (a permutation scatter)
template <typename TI, typename TO>
void launch_scatter(hipStream_t st, int64_t n, const int32_t* idx, const TI* in, TO* out);

// Tile-list products with FP64 tiles: entry e multiplies the 64x64 tile at
// element offset tiles[e].a (transposed if trans) by the 64-block of x at
// tiles[e].x into the scratch vector P[64 e ..]; then output o sums its entries
// outs[o].p0 .. outs[o].p1 - 1 in order:  y[y .. y + 63] = alpha * sum (+ y if acc).
// Used where a block's nonzero tiles are a sparse subset (the L_GI products
// and the off-group parts of the triangular solves).
struct TileRef { int64_t a, x; };
struct OutRef { int64_t y; int32_t p0, p1; };
void launch_tile_list_mv(hipStream_t st, bool trans, const TileRef* tiles, int64_t ntiles, const OutRef* outs, int64_t nouts,
                         const double* A, const double* x, double* P, double* y, double alpha, bool acc);

// Blocked triangular solves with the interior factor of tile-packed FP64 K
// matrices and the stored inverse diagonal tiles.  One workgroup per item: a
// group of tile rows k0..k1-1 of one matrix; the items of one launch must not
// depend on one another (groups of one height of a dissection tree).  Nonzero
// interior tiles: row k holds columns rcol[rptr[p_row + k] .. rptr[p_row + k + 1])
// (all < k), column k holds rows crow[cptr[p_col + k] .. cptr[p_col + k + 1])
// (all > k and inside the interior).
// rslot / cslot: storage slot (relative to a_off) of the tile of every rcol / crow entry.
struct TrsvDesc { int64_t a_off; int32_t a_nt, k0, k1, p_row, p_col, pad; int64_t inv_off, v_off; };
void launch_trsv(hipStream_t st, bool transposed, const TrsvDesc* d, int32_t nitems, const double* A, const double* Inv,
                 const int32_t* rptr, const int32_t* rcol, const int32_t* rslot, const int32_t* cptr, const int32_t* crow,
                 const int32_t* cslot, double* v);

// ------------------------------------------------------------------- PCG
// Deterministic dot product: partial sums per block then a single-block finish.
void launch_dot(hipStream_t st, int64_t n, const double* a, const double* b, double* partial, int32_t nblocks, double* out);
constexpr int DOT_BLOCKS = 4096;  // at most one partial per 256 entries, as many blocks as the other vector kernels

// Scalars used by the PCG kernels (device array).
// S_DONE: set (sticky) once the iteration converged or broke down; the
// PCG update kernels then leave x, r, p and the history untouched.
enum PcgScalar { S_RZ = 0, S_PQ = 1, S_ALPHA = 2, S_RR = 3, S_RZNEW = 4, S_BETA = 5, S_GG = 6, S_DONE = 7, S_NSCAL = 8 };
void launch_set_int(hipStream_t st, int* p, int v);
// p = z + beta p (unless done); when copies is given, also copies[list[j]] = p[g]
// for j in ptr[g]..ptr[g+1] (the gather that starts the interface product).
void launch_pcg_update_p(hipStream_t st, int64_t n, double* p, const double* z, const double* s, const int64_t* ptr = nullptr,
                         const int64_t* list = nullptr, double* copies = nullptr);
// Steps that the single-block finish of a PCG dot product does after it:
// DOT_ALPHA alpha = rz / pq (slot S_PQ), or s[S_DONE] = 1 without a step when
// p.q <= 0 or not finite (breakdown); DOT_CHECK the stopping
// test, s[S_DONE] = 1 (sticky) when p.q <= 0 or not finite or r.r < rtol2 g.g
// (slot S_RR); DOT_BETA beta = rznew / rz, rz = rznew, ++it (slot S_RZNEW).
enum DotStep { DOT_ALPHA = 1, DOT_CHECK = 2, DOT_BETA = 3 };
// A segmented sum (as launch_seg_reduce with beta 0) whose blocks also form
// the partial sums of out.dotv, then the dot product's finish and step.
template <typename TI>
void launch_seg_reduce_dot(hipStream_t st, int64_t n, const int64_t* ptr, const int64_t* list, const double* w, const TI* in,
                           double* out, const double* dotv, double* partial, double* s, int slot, int step, double* hist,
                           int* it, double rtol2, const TI* in2 = nullptr);
// x += alpha p, r -= alpha q (unless done) and the partial sums of r.r in one
// launch, then the finish of r.r with the stopping test; when copies is given
// the launch also writes copies[list[j]] = w[list[j]] r[g] for j in
// ptr[g]..ptr[g+1] (the weighted restriction that starts the preconditioner).
template <typename TC>
void launch_pcg_update_xr_check(hipStream_t st, int64_t n, double* x, double* r, const double* p, const double* q,
                                double* partial, double* s, double rtol2, const int64_t* ptr, const int64_t* list,
                                const double* w, TC* copies);
void launch_axpby(hipStream_t st, int64_t n, double a, const double* x, double b, double* y);

// Element energies out_e = E_e a_e^T K0 b_e (level-1 mesh).
void launch_element_energy(hipStream_t st, int64_t ne, int nloc, const int32_t* edof, const double* K0,
                           const double* scale, const double* a, const double* b, double* out);
void launch_fill(hipStream_t st, int64_t n, double v, double* y);
// out[i] = A[pos[i]] with 64-bit element positions.
template <typename T>
void launch_gather64(hipStream_t st, int64_t n, const int64_t* pos, const T* A, double* out);
// w[i] = d[i] / s[i] where idx[i] >= 0, else 0.
void launch_ratio(hipStream_t st, int64_t n, const double* d, const double* s, const int32_t* idx, double* w);
// out[idx[i]] = in[i] (every idx valid).
void launch_scatter_idx(hipStream_t st, int64_t n, const int32_t* idx, const double* in, double* out);

}  // namespace mlbddc
