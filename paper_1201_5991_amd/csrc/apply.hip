// Per-iteration kernels of the multilevel BDDC-PCG for gfx950: batched
// tile-block matrix-vector products (the interface operator S^, the explicit
// local BDDC operators and coarse bases), weighted gathers and atomic-free
// segmented reductions for restriction / averaging (E_i^T and E_i), blocked
// triangular solves for condensation and interior recovery, and the PCG
// vector operations with device-resident scalars.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mlbddc {

namespace {

// ---------------------------------------------------------------- tile mv
// A workgroup per TPW consecutive stored tiles of a block (TPW = 1 or 2, a
// tuning parameter; tiles in column-major order for symmetric blocks): it
// loads all its tiles, then forms for each tile both A x_s (for the tile's
// row) and, for symmetric blocks, A^T x_r (for its column); results go to a
// partial-sum array reduced by k_mv_reduce.  The arithmetic of a tile does
// not depend on TPW, so neither do the results.
// Lane l of the workgroup's 256 keeps rows a0..a0+3 (a0 = 4 (l & 15)) of the
// columns g, g + 16, g + 32, g + 48 (g = l >> 4), loaded as 32-byte runs of a
// column.  Runs that hold only padding (rows or columns beyond the block's
// valid extent) or only upper-triangle entries of a diagonal tile of a
// symmetric block are not loaded: the diagonal tile contributes L x (its
// lower triangle with the diagonal) plus L_strict^T x to its own output, so
// the whole product streams the stored lower triangle and nothing else.
// `prefix` counts workgroups per block (ceil(tiles / TPW)).
template <typename TA, typename TX, int TPW>
__global__ void __launch_bounds__(256) k_mv_tiles(int mode, const MvDesc* __restrict__ d, int nitems,
                                                  const int64_t* __restrict__ prefix, const TA* __restrict__ A,
                                                  const TX* __restrict__ x, TA* __restrict__ P) {
  const int64_t bid = blockIdx.x;
  int lo = 0, hi = nitems;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= bid) lo = mid; else hi = mid;
  }
  const MvDesc D = d[lo];
  const int64_t ntiles = mode == MV_SYM ? (int64_t)D.nr * (D.nr + 1) / 2 : (int64_t)D.nr * D.nc;
  const int64_t local0 = (bid - prefix[lo]) * TPW;
  const int nt = (int)(ntiles - local0 < TPW ? ntiles - local0 : TPW);
  int rr[TPW], ss[TPW];
  if (mode == MV_SYM) {
    // column-major unranking of the lower tiles of an nr x nr block
    int s0 = 0;
    int64_t rem = local0;
    while (rem >= D.nr - s0) { rem -= D.nr - s0; ++s0; }
    rr[0] = s0 + (int)rem;
    ss[0] = s0;
#pragma unroll
    for (int j = 1; j < TPW; ++j) {
      rr[j] = rr[j - 1] + 1;
      ss[j] = ss[j - 1];
      if (rr[j] >= D.nr) ss[j] = rr[j] = ss[j - 1] + 1;
    }
  } else {
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      rr[j] = (int)((local0 + j) % D.nr);
      ss[j] = (int)((local0 + j) / D.nr);
    }
  }
  const int t = threadIdx.x;
  __shared__ TA red[TPW][16][TS];
  __shared__ TA vcol[TPW][TS];
  const int a0 = 4 * (t & 15), g = t >> 4;
  const bool need_v = mode == MV_T || mode == MV_SYM;  // transposed product (strictly lower part on a diagonal tile)
  const bool need_u = mode != MV_T;
  // all tiles of the workgroup in flight before any is multiplied
  TA av[TPW][4][4];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int r = rr[j], s = ss[j];
    const int R = D.r0 + r, S = D.c0 + s;
    const bool live = j < nt && !(D.env && S < D.env[R]);
    const bool diag = mode == MV_SYM && r == s;
    const int rv = D.vr - r * TS, cv = D.vc - s * TS;  // valid rows / columns of this tile (may exceed 64)
    const TA* tile = A + D.a_off + tile_index(R, S, D.a_nt) * TE;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int b = g + 16 * m;
#pragma unroll
      for (int i = 0; i < 4; ++i) av[j][m][i] = 0;
      if (live && b < cv && a0 < rv && (!diag || a0 + 3 >= b)) {
        const TA* col = tile + b * TS + a0;
#pragma unroll
        for (int i = 0; i < 4; ++i) av[j][m][i] = col[i];
      }
    }
  }
  TA v_part[TPW][4];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int r = rr[j], s = ss[j];
    const bool live = j < nt && !(D.env && D.c0 + s < D.env[D.r0 + r]);
    const bool diag = mode == MV_SYM && r == s;
    const int rv = D.vr - r * TS, cv = D.vc - s * TS;
#pragma unroll
    for (int m = 0; m < 4; ++m) v_part[j][m] = 0;
    if (live) {
      const TX* xs = x + D.x_off + (int64_t)s * TS;
      const TX* xr = x + D.x_off + (int64_t)r * TS;
      TA up[4] = {0, 0, 0, 0};
      TA xra[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xra[i] = (need_v && a0 + i < rv) ? (TA)xr[a0 + i] : (TA)0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int b = g + 16 * m;
        const bool col_ok = b < cv;
        const TA xb = (need_u && col_ok) ? (TA)xs[b] : (TA)0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = a0 + i;
          const TA al = (a < rv && (!diag || a >= b)) ? av[j][m][i] : (TA)0;  // lower triangle with the diagonal
          up[i] += al * xb;
          v_part[j][m] += (diag && a == b) ? (TA)0 : al * xra[i];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) red[j][g][a0 + i] = up[i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) red[j][g][a0 + i] = 0;
    }
    // reduce v over the 16 lanes sharing g
#pragma unroll
    for (int m = 0; m < 4; ++m)
      for (int off = 8; off > 0; off >>= 1) v_part[j][m] += __shfl_xor(v_part[j][m], off, 16);
    if (diag && (t & 15) == 0)
#pragma unroll
      for (int m = 0; m < 4; ++m) vcol[j][g + 16 * m] = v_part[j][m];
  }
  __syncthreads();
  TA* pbase = P + D.p_off;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    if (j >= nt) break;
    const int r = rr[j], s = ss[j];
    const bool diag = mode == MV_SYM && r == s;
    TA u_out = 0;
    if (t < TS) {
      TA acc = 0;
#pragma unroll
      for (int q = 0; q < 16; ++q) acc += red[j][q][t];
      u_out = diag ? acc + vcol[j][t] : acc;
    }
    if (mode == MV_SYM) {
      if (t < TS) pbase[((int64_t)r * D.nr + s) * TS + t] = u_out;
      if (r != s && (t & 15) == 0)
        for (int m = 0; m < 4; ++m) pbase[((int64_t)s * D.nr + r) * TS + g + 16 * m] = v_part[j][m];
    } else if (mode == MV_N) {
      if (t < TS) pbase[((int64_t)r * D.nc + s) * TS + t] = u_out;
    } else {
      if ((t & 15) == 0)
        for (int m = 0; m < 4; ++m) pbase[((int64_t)s * D.nr + r) * TS + g + 16 * m] = v_part[j][m];
    }
  }
}

// Sum of the partial tiles of one output tile: the four wavefronts take every
// fourth partial (two accumulators each, loads unrolled), then wavefront 0
// adds the four sums in a fixed order.
template <typename TA, typename TY>
__global__ void __launch_bounds__(256) k_mv_reduce(int mode, const MvDesc* __restrict__ d, const TA* __restrict__ P, TY* y,
                                                   double alpha, int accumulate) {
  const MvDesc D = d[blockIdx.y];
  const int i = blockIdx.x;
  const int nout = mode == MV_T ? D.nc : D.nr;
  const int nsum = mode == MV_N ? D.nc : D.nr;
  if (i >= nout) return;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  __shared__ double red[4][TS];
  const TA* p = P + D.p_off + (int64_t)i * nsum * TS + lane;
  double a0 = 0.0, a1 = 0.0;
  int j = q;
#pragma unroll 4
  for (; j + 4 < nsum; j += 8) {
    a0 += (double)p[(int64_t)j * TS];
    a1 += (double)p[(int64_t)(j + 4) * TS];
  }
  if (j < nsum) a0 += (double)p[(int64_t)j * TS];
  red[q][lane] = a0 + a1;
  __syncthreads();
  if (q == 0) {
    const double acc = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    TY* yy = y + D.y_off + (int64_t)i * TS + lane;
    double v = alpha * acc;
    if (accumulate) v += (double)*yy;
    *yy = (TY)v;
  }
}

// Small products (the coarse levels): one workgroup per output tile walks
// the tiles that feed it, plain ones in its tile row and, for symmetric
// blocks, transposed ones in its tile column below the diagonal, and writes
// the result directly (FP64 sums; no partial tiles, one launch instead of two).
template <typename TA, typename TX, typename TY>
__global__ void __launch_bounds__(256) k_mv_rows(int mode, const MvDesc* __restrict__ d, const TA* __restrict__ A,
                                                 const TX* __restrict__ x, TY* y, double alpha, int accumulate, int mode2,
                                                 const MvDesc* __restrict__ d2, const TX* __restrict__ x2) {
  const MvDesc D = d[blockIdx.y];
  const int o = blockIdx.x;
  const int nout = mode == MV_T ? D.nc : D.nr;
  if (o >= nout) return;
  const int t = threadIdx.x, a0 = 4 * (t & 15), g = t >> 4;
  __shared__ double red[16][TS];
  __shared__ double vcol[TS];
  double up[4] = {0.0, 0.0, 0.0, 0.0}, vp[4] = {0.0, 0.0, 0.0, 0.0};
  // plain tile: up(rows a0..a0+3) += A(:, b) x[b]; transposed: vp(col b) += A(a0.., b) . x[a0..]
  auto tile = [&](const MvDesc& DD, int R, int S, const TX* xv, bool transposed) {
    if (DD.env && S < DD.env[R]) return;
    const TA* a = A + DD.a_off + tile_index(R, S, DD.a_nt) * TE;
    double xa[4];
    if (transposed)
#pragma unroll
      for (int i = 0; i < 4; ++i) xa[i] = (double)xv[a0 + i];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int b = g + 16 * m;
      const TA* col = a + b * TS + a0;
      if (transposed) {
#pragma unroll
        for (int i = 0; i < 4; ++i) vp[m] += (double)col[i] * xa[i];
      } else {
        const double xb = (double)xv[b];
#pragma unroll
        for (int i = 0; i < 4; ++i) up[i] += (double)col[i] * xb;
      }
    }
  };
  auto walk = [&](const MvDesc& DD, int md, const TX* xx) {
    const TX* xb = xx + DD.x_off;
    if (md == MV_N) {
      for (int j = 0; j < DD.nc; ++j) tile(DD, DD.r0 + o, DD.c0 + j, xb + (int64_t)j * TS, false);
    } else if (md == MV_T) {
      for (int j = 0; j < DD.nr; ++j) tile(DD, DD.r0 + j, DD.c0 + o, xb + (int64_t)j * TS, true);
    } else {
      for (int j = 0; j <= o; ++j) tile(DD, DD.r0 + o, DD.r0 + j, xb + (int64_t)j * TS, false);
      for (int j = o + 1; j < DD.nr; ++j) tile(DD, DD.r0 + j, DD.r0 + o, xb + (int64_t)j * TS, true);
    }
  };
  walk(D, mode, x);
  if (d2) walk(d2[blockIdx.y], mode2, x2);  // a second product into the same output tiles
#pragma unroll
  for (int i = 0; i < 4; ++i) red[g][a0 + i] = up[i];
#pragma unroll
  for (int m = 0; m < 4; ++m)
    for (int off = 8; off > 0; off >>= 1) vp[m] += __shfl_xor(vp[m], off, 16);
  if ((t & 15) == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) vcol[g + 16 * m] = vp[m];
  __syncthreads();
  if (t < TS) {
    double acc = vcol[t];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += red[q][t];
    TY* yy = y + D.y_off + (int64_t)o * TS + t;
    double v = alpha * acc;
    if (accumulate) v += (double)*yy;
    *yy = (TY)v;
  }
}

// --------------------------------------------------------- gather / scatter
template <typename TI, typename TO>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ idx, const double* __restrict__ w, const TI* __restrict__ in,
                         TO* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t j = idx[i];
    double v = j >= 0 ? (double)in[j] : 0.0;
    if (w) v *= w[i];
    out[i] = (TO)v;
  }
}

template <typename TI>
__global__ void k_seg_reduce(int64_t n, const int64_t* __restrict__ ptr, const int64_t* __restrict__ list,
                             const double* __restrict__ w, const TI* __restrict__ in, const TI* __restrict__ in2,
                             double* __restrict__ out, double beta) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double acc = beta != 0.0 ? beta * out[g] : 0.0;
    for (int64_t j = ptr[g]; j < ptr[g + 1]; ++j) {
      int64_t q = list[j];
      const double v = in2 ? (double)in[q] + (double)in2[q] : (double)in[q];
      acc += (w ? w[q] : 1.0) * v;
    }
    out[g] = acc;
  }
}

// out[g] = base[bidx[g]] + sum_{j in ptr[g]..ptr[g+1]} in[list[j]]  (FP64)
__global__ void k_gather_seg(int64_t n, const int32_t* __restrict__ bidx, const double* __restrict__ base,
                             const int64_t* __restrict__ ptr, const int64_t* __restrict__ list, const double* __restrict__ in,
                             double* __restrict__ out) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double acc = base[bidx[g]];
    for (int64_t j = ptr[g]; j < ptr[g + 1]; ++j) acc += in[list[j]];
    out[g] = acc;
  }
}

// out[i1[i]] = in1[i] (i1 >= 0) for i < n1, then out[i2[i]] = in2[i] for i < n2 (disjoint targets)
template <typename TI>
__global__ void k_scatter2(int64_t n1, const int32_t* __restrict__ i1, const TI* __restrict__ in1, int64_t n2,
                           const int32_t* __restrict__ i2, const double* __restrict__ in2, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1 + n2; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n1) {
      const int32_t j = i1[i];
      if (j >= 0) out[j] = (double)in1[i];
    } else {
      out[i2[i - n1]] = in2[i - n1];
    }
  }
}

template <typename TI, typename TO>
__global__ void k_scatter(int64_t n, const int32_t* __restrict__ idx, const TI* __restrict__ in, TO* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t j = idx[i];
    if (j >= 0) out[j] = (TO)in[i];
  }
}

// ------------------------------------------------------------ tile lists
// One wavefront per listed tile.  Lane l = 16 cq + sub loads rows
// 4 sub .. 4 sub + 3 of the columns 4 m + cq (m = 0..15) as 16-byte vectors,
// so one instruction reads four whole columns; the sums are finished across
// lanes by butterflies (a lane keeps half of its partial sums, adds the
// partner's matching half and passes on the other), which leaves the entry
// 4 sub + cq of T x (trans 0) or of T^T x (trans 1) in lane l.
__device__ inline double tile_quad_dot(const double* __restrict__ T, int trans, const double* x, int lane) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int sub = lane & 15, cq = lane >> 4;
  double v[16][4];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const d2* q = reinterpret_cast<const d2*>(T + (4 * m + cq) * TS + 4 * sub);
    const d2 a = q[0], b = q[1];
    v[m][0] = a[0];
    v[m][1] = a[1];
    v[m][2] = b[0];
    v[m][3] = b[1];
  }
  if (!trans) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const double xb = x[4 * m + cq];
#pragma unroll
      for (int i = 0; i < 4; ++i) r[i] += v[m][i] * xb;
    }
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double send = b5 ? r[k] : r[k + 2], keep = b5 ? r[k + 2] : r[k];
      r[k] = keep + __shfl_xor(send, 32);
    }
    const double send = b4 ? r[0] : r[1], keep = b4 ? r[1] : r[0];
    return keep + __shfl_xor(send, 16);
  }
  double xr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) xr[i] = x[4 * sub + i];
  double c[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) c[m] = (v[m][0] * xr[0] + v[m][1] * xr[1]) + (v[m][2] * xr[2] + v[m][3] * xr[3]);
#pragma unroll
  for (int h = 8; h >= 1; h >>= 1) {
    const bool bit = (sub & h) != 0;
#pragma unroll
    for (int k = 0; k < h; ++k) {
      const double send = bit ? c[k] : c[k + h], keep = bit ? c[k + h] : c[k];
      c[k] = keep + __shfl_xor(send, h);
    }
  }
  return c[0];
}

constexpr int TL_WAVES = 4;

__global__ void __launch_bounds__(TL_WAVES * 64) k_tl_products(int trans, const TileRef* __restrict__ tiles, int64_t n,
                                                              const double* __restrict__ A, const double* __restrict__ x,
                                                              double* __restrict__ P) {
  __shared__ double sx[TL_WAVES][TS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * TL_WAVES + w;
  if (e >= n) return;
  const TileRef R = tiles[e];
  sx[w][lane] = x[R.x + lane];
  __builtin_amdgcn_wave_barrier();
  const double val = tile_quad_dot(A + R.a, trans, sx[w], lane);
  P[e * TS + 4 * (lane & 15) + (lane >> 4)] = val;
}

__global__ void __launch_bounds__(256) k_tl_reduce(const OutRef* __restrict__ outs, int64_t n, const double* __restrict__ P,
                                                   double* y, double alpha, int acc) {
  const int lane = threadIdx.x & 63;
  const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= n) return;
  const OutRef O = outs[o];
  double s0 = 0.0, s1 = 0.0;
  int p = O.p0;
  for (; p + 1 < O.p1; p += 2) {
    s0 += P[(int64_t)p * TS + lane];
    s1 += P[(int64_t)(p + 1) * TS + lane];
  }
  if (p < O.p1) s0 += P[(int64_t)p * TS + lane];
  double v = alpha * (s0 + s1);
  if (acc) v += y[O.y + lane];
  y[O.y + lane] = v;
}

// ------------------------------------------------------------------ trsv
// Blocked triangular solve with the interior factor over one group of tile
// rows per workgroup of eight wavefronts (the nonzero tiles of a row or a
// column come from host-built lists).  Block row k:
//   v_k <- W_k (v_k - sum_{s<k} L_ks v_s)          (forward, W_k = L_kk^{-1})
//   v_k <- W_k^T (v_k - sum_{r>k} L_rk^T v_r)      (backward)
// Wavefronts 1..7 take the nonzero tiles of the block row in turn; each
// loads a whole tile (64 values per lane in flight) and the matching block of
// v (broadcast through LDS).  Wavefront 0 meanwhile stages W_k in LDS, so the
// product with the diagonal inverse at the end of the step waits on no global
// load.
// Forward: lane a holds row a of a tile (coalesced columns); backward: lane b
// holds column b (16-byte loads along the column).
constexpr int TRSV_WAVES = 8;

__device__ inline void load_tile_rows(const double* __restrict__ g, int lane, double (&a)[TS]) {
#pragma unroll
  for (int b = 0; b < TS; ++b) a[b] = g[b * TS + lane];
}
__device__ inline void load_tile_cols(const double* __restrict__ g, int lane, double (&a)[TS]) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2* c = reinterpret_cast<const d2*>(g + lane * TS);
#pragma unroll
  for (int q = 0; q < TS / 2; ++q) {
    const d2 v = c[q];
    a[2 * q] = v[0];
    a[2 * q + 1] = v[1];
  }
}
__device__ inline double dot64(const double (&a)[TS], const double* __restrict__ x) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2* x2 = reinterpret_cast<const d2*>(x);
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
  for (int b = 0; b < TS; b += 4) {
    const d2 u = x2[b / 2], v = x2[b / 2 + 1];
    s0 += a[b] * u[0];
    s1 += a[b + 1] * u[1];
    s2 += a[b + 2] * v[0];
    s3 += a[b + 3] * v[1];
  }
  return (s0 + s1) + (s2 + s3);
}

__global__ void __launch_bounds__(TRSV_WAVES * 64) k_trsv(int trans, const TrsvDesc* __restrict__ d,
                                                         const double* __restrict__ A, const double* __restrict__ Inv,
                                                         const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol,
                                                         const int32_t* __restrict__ rslot,
                                                         const int32_t* __restrict__ cptr, const int32_t* __restrict__ crow,
                                                         const int32_t* __restrict__ cslot, double* v) {
  const TrsvDesc D = d[blockIdx.x];
  constexpr int LDW = TS + 1;
  __shared__ double sw[TS * LDW];
  __shared__ double sv[TRSV_WAVES][TS];
  __shared__ double red[TRSV_WAVES][TS];
  __shared__ double acc[TS];
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const double* base = A + D.a_off;
  double* vv = v + D.v_off;
  for (int step = 0; step < D.k1 - D.k0; ++step) {
    const int k = trans ? D.k1 - 1 - step : D.k0 + step;
    double part = 0.0;
    double a[TS];
    if (w == 0) {
      // stage W_k (column-major, padded) while the other wavefronts work
      load_tile_rows(Inv + D.inv_off + (int64_t)k * TE, lane, a);
#pragma unroll
      for (int b = 0; b < TS; ++b) sw[b * LDW + lane] = a[b];
    } else if (!trans) {
      const int q0 = rptr[D.p_row + k], q1 = rptr[D.p_row + k + 1];
      for (int q = q0 + w - 1; q < q1; q += TRSV_WAVES - 1) {
        const int s = rcol[q];
        sv[w][lane] = vv[(int64_t)s * TS + lane];
        load_tile_rows(base + (int64_t)rslot[q] * TE, lane, a);
        __builtin_amdgcn_wave_barrier();
        part += dot64(a, sv[w]);
        __builtin_amdgcn_wave_barrier();
      }
    } else {
      const int q0 = cptr[D.p_col + k], q1 = cptr[D.p_col + k + 1];
      for (int q = q0 + w - 1; q < q1; q += TRSV_WAVES - 1) {
        const int r = crow[q];
        sv[w][lane] = vv[(int64_t)r * TS + lane];
        load_tile_cols(base + (int64_t)cslot[q] * TE, lane, a);
        __builtin_amdgcn_wave_barrier();
        part += dot64(a, sv[w]);
        __builtin_amdgcn_wave_barrier();
      }
    }
    red[w][lane] = part;
    __syncthreads();
    if (w == 0) {
      double sum = 0.0;
#pragma unroll
      for (int q = 1; q < TRSV_WAVES; ++q) sum += red[q][lane];
      acc[lane] = vv[(int64_t)k * TS + lane] - sum;
      __builtin_amdgcn_wave_barrier();
      double s0 = 0, s1 = 0;
      if (!trans) {
#pragma unroll
        for (int b = 0; b < TS; b += 2) {
          s0 += sw[b * LDW + lane] * acc[b];
          s1 += sw[(b + 1) * LDW + lane] * acc[b + 1];
        }
      } else {
#pragma unroll
        for (int q = 0; q < TS; q += 2) {
          s0 += sw[lane * LDW + q] * acc[q];
          s1 += sw[lane * LDW + q + 1] * acc[q + 1];
        }
      }
      vv[(int64_t)k * TS + lane] = s0 + s1;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- PCG
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_dot_final(int nb, const double* __restrict__ partial, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// Sum of the block partials (fixed order) and the scalar step after it.  The
// iteration counter lives on the device (so that an iteration can be
// replayed from a captured graph): alpha_j goes to hist[2j], beta_j to
// hist[2j+1], after which the counter moves on.
__global__ void __launch_bounds__(256) k_dot_step(int nb, const double* __restrict__ partial, double* s, int slot, int step,
                                                  double* hist, int* it, double rtol2) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += partial[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double tot = red[0];
  s[slot] = tot;
  if (step == DOT_CHECK) {
    const double pq = s[S_PQ];
    const bool stop = !(pq > 0.0) || !(pq < INFINITY) || tot < rtol2 * s[S_GG];
    if (s[S_DONE] != 0.0 || stop) s[S_DONE] = 1.0;
    return;
  }
  if (s[S_DONE] != 0.0) return;
  if (step == DOT_ALPHA) {
    if (!(tot > 0.0) || !(tot < INFINITY)) {  // breakdown: no step is taken, x keeps the last iterate
      s[S_DONE] = 1.0;
      return;
    }
    s[S_ALPHA] = s[S_RZ] / tot;
    if (hist) hist[2 * (*it)] = s[S_ALPHA];
  } else if (step == DOT_BETA) {
    s[S_BETA] = tot / s[S_RZ];
    s[S_RZ] = tot;
    if (hist) hist[2 * (*it) + 1] = s[S_BETA];
    *it += 1;
  }
}

// out[g] = sum_{j in ptr[g]..ptr[g+1]} (w ? w[list[j]] : 1) in[list[j]], and
// per-block partial sums of out[g] dotv[g].
template <typename TI>
__global__ void __launch_bounds__(256) k_seg_reduce_dot(int64_t n, const int64_t* __restrict__ ptr,
                                                        const int64_t* __restrict__ list, const double* __restrict__ w,
                                                        const TI* __restrict__ in, const TI* __restrict__ in2,
                                                        double* __restrict__ out,
                                                        const double* __restrict__ dotv, double* __restrict__ partial) {
  __shared__ double red[256];
  double v = 0.0;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int64_t j = ptr[g]; j < ptr[g + 1]; ++j) {
      const int64_t q = list[j];
      const double v = in2 ? (double)in[q] + (double)in2[q] : (double)in[q];
      acc += (w ? w[q] : 1.0) * v;
    }
    out[g] = acc;
    v += acc * dotv[g];
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// x += alpha p, r -= alpha q (unless done), and per-block partial sums of r.r.
template <typename TC>
__global__ void __launch_bounds__(256) k_pcg_update_xr_partial(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                               const double* __restrict__ p, const double* __restrict__ q,
                                                               const double* __restrict__ s, double* __restrict__ partial,
                                                               const int64_t* __restrict__ ptr, const int64_t* __restrict__ list,
                                                               const double* __restrict__ w, TC* __restrict__ copies) {
  __shared__ double red[256];
  const bool done = s[S_DONE] != 0.0;
  const double a = s[S_ALPHA];
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double ri = r[i];
    if (!done) {
      x[i] += a * p[i];
      ri -= a * q[i];
      r[i] = ri;
    }
    v += ri * ri;
    if (copies)  // weighted subdomain copies of the new residual
      for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) {
        const int64_t c = list[j];
        copies[c] = (TC)(w[c] * ri);
      }
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// p = z + beta p (unless done); with copies, also copies[list[j]] = p[g] for
// j in ptr[g]..ptr[g+1] (the subdomain copies of every interface entry).
__global__ void k_pcg_update_p(int64_t n, double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ s,
                               const int64_t* __restrict__ ptr, const int64_t* __restrict__ list, double* __restrict__ copies) {
  const bool done = s[S_DONE] != 0.0;
  if (done && !copies) return;
  const double b = s[S_BETA];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = p[i];
    if (!done) {
      v = z[i] + b * v;
      p[i] = v;
    }
    if (copies)
      for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) copies[list[j]] = v;
  }
}
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = v;
}

__global__ void k_element_energy(int64_t ne, int nloc, const int32_t* __restrict__ edof, const double* __restrict__ K0,
                                 const double* __restrict__ scale, const double* __restrict__ a, const double* __restrict__ b,
                                 double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    double av[24], bv[24];
    for (int i = 0; i < nloc; ++i) {
      int32_t j = edof[e * nloc + i];
      av[i] = j >= 0 ? a[j] : 0.0;
      bv[i] = j >= 0 ? b[j] : 0.0;
    }
    double s = 0.0;
    for (int i = 0; i < nloc; ++i) {
      double t = 0.0;
      for (int j = 0; j < nloc; ++j) t += K0[i * nloc + j] * bv[j];
      s += av[i] * t;
    }
    out[e] = scale[e] * s;
  }
}

template <typename T>
__global__ void k_gather64(int64_t n, const int64_t* __restrict__ pos, const T* __restrict__ A, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)A[pos[i]];
}
__global__ void k_ratio(int64_t n, const double* __restrict__ d, const double* __restrict__ s, const int32_t* __restrict__ idx,
                        double* __restrict__ w) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = idx[i] >= 0 ? d[i] / s[i] : 0.0;
}
__global__ void k_scatter_idx(int64_t n, const int32_t* __restrict__ idx, const double* __restrict__ in,
                              double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[idx[i]] = in[i];
}

inline unsigned grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

}  // namespace

template <typename TA, typename TX, typename TY>
void launch_tile_mv(hipStream_t st, int mode, const MvDesc* d, int32_t nitems, int64_t total_tiles, const int64_t* tile_prefix,
                    const TA* A, const TX* x, TY* y, double alpha, bool accumulate, TA* partials, int32_t max_out_tiles,
                    hipEvent_t ev0, hipEvent_t ev1, int tpw, int64_t groups2, const int64_t* group_prefix2) {
  if (nitems <= 0 || total_tiles <= 0) return;
  if (ev0) (void)hipEventRecord(ev0, st);
  if (total_tiles <= SMALL_MV_TILES) {  // coarse levels: one launch, no partial tiles
    hipLaunchKernelGGL((k_mv_rows<TA, TX, TY>), dim3((unsigned)max_out_tiles, (unsigned)nitems), dim3(256), 0, st, mode, d, A,
                       x, y, alpha, accumulate ? 1 : 0, 0, (const MvDesc*)nullptr, (const TX*)nullptr);
    if (ev1) (void)hipEventRecord(ev1, st);
    return;
  }
  if (tpw == 2)
    hipLaunchKernelGGL((k_mv_tiles<TA, TX, 2>), dim3((unsigned)groups2), dim3(256), 0, st, mode, d, nitems, group_prefix2, A, x,
                       partials);
  else
    hipLaunchKernelGGL((k_mv_tiles<TA, TX, 1>), dim3((unsigned)total_tiles), dim3(256), 0, st, mode, d, nitems, tile_prefix, A,
                       x, partials);
  if (ev1) (void)hipEventRecord(ev1, st);
  hipLaunchKernelGGL((k_mv_reduce<TA, TY>), dim3((unsigned)max_out_tiles, (unsigned)nitems), dim3(256), 0, st, mode, d,
                     partials, y, alpha, accumulate ? 1 : 0);
}

template <typename TA, typename TX, typename TY>
void launch_tile_mv_sum(hipStream_t st, int mode, const MvDesc* d, int mode2, const MvDesc* d2, int32_t nitems,
                        int32_t max_out_tiles, const TA* A, const TX* x, const TX* x2, TY* y, double alpha, bool accumulate) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL((k_mv_rows<TA, TX, TY>), dim3((unsigned)max_out_tiles, (unsigned)nitems), dim3(256), 0, st, mode, d, A, x,
                     y, alpha, accumulate ? 1 : 0, mode2, d2, x2);
}

template <typename TI, typename TO>
void launch_gather(hipStream_t st, int64_t n, const int32_t* idx, const double* w, const TI* in, TO* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_gather<TI, TO>), dim3(grid_for(n)), dim3(256), 0, st, n, idx, w, in, out);
}

template <typename TI>
void launch_seg_reduce(hipStream_t st, int64_t n, const int64_t* ptr, const int64_t* list, const double* w, const TI* in,
                       double* out, double beta, const TI* in2) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_seg_reduce<TI>), dim3(grid_for(n)), dim3(256), 0, st, n, ptr, list, w, in, in2, out, beta);
}

template <typename TI, typename TO>
void launch_scatter(hipStream_t st, int64_t n, const int32_t* idx, const TI* in, TO* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_scatter<TI, TO>), dim3(grid_for(n)), dim3(256), 0, st, n, idx, in, out);
}

void launch_tile_list_mv(hipStream_t st, bool trans, const TileRef* tiles, int64_t ntiles, const OutRef* outs, int64_t nouts,
                         const double* A, const double* x, double* P, double* y, double alpha, bool acc) {
  if (nouts <= 0) return;
  if (ntiles > 0)
    hipLaunchKernelGGL(k_tl_products, dim3((unsigned)((ntiles + TL_WAVES - 1) / TL_WAVES)), dim3(TL_WAVES * 64), 0, st,
                       trans ? 1 : 0, tiles, ntiles, A, x, P);
  hipLaunchKernelGGL(k_tl_reduce, dim3((unsigned)((nouts + 3) / 4)), dim3(256), 0, st, outs, nouts, P, y, alpha, acc ? 1 : 0);
}

void launch_trsv(hipStream_t st, bool transposed, const TrsvDesc* d, int32_t nitems, const double* A, const double* Inv,
                 const int32_t* rptr, const int32_t* rcol, const int32_t* rslot, const int32_t* cptr, const int32_t* crow,
                 const int32_t* cslot, double* v) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_trsv, dim3(nitems), dim3(TRSV_WAVES * 64), 0, st, transposed ? 1 : 0, d, A, Inv, rptr, rcol, rslot,
                     cptr, crow, cslot, v);
}

static unsigned dot_blocks(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(DOT_BLOCKS, (n + 255) / 256));
}

void launch_dot(hipStream_t st, int64_t n, const double* a, const double* b, double* partial, int32_t nblocks, double* out) {
  const unsigned nb = std::min<unsigned>((unsigned)std::max(nblocks, 1), dot_blocks(n));
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, st, n, a, b, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, (int)nb, partial, out);
}

template <typename TI>
void launch_seg_reduce_dot(hipStream_t st, int64_t n, const int64_t* ptr, const int64_t* list, const double* w, const TI* in,
                           double* out, const double* dotv, double* partial, double* s, int slot, int step, double* hist,
                           int* it, double rtol2, const TI* in2) {
  const unsigned nb = dot_blocks(n);
  hipLaunchKernelGGL(k_seg_reduce_dot<TI>, dim3(nb), dim3(256), 0, st, n, ptr, list, w, in, in2, out, dotv, partial);
  hipLaunchKernelGGL(k_dot_step, dim3(1), dim3(256), 0, st, (int)nb, partial, s, slot, step, hist, it, rtol2);
}
template void launch_seg_reduce_dot<double>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*, const double*,
                                            double*, const double*, double*, double*, int, int, double*, int*, double,
                                            const double*);
template void launch_seg_reduce_dot<float>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*, const float*,
                                           double*, const double*, double*, double*, int, int, double*, int*, double,
                                           const float*);

template <typename TC>
void launch_pcg_update_xr_check(hipStream_t st, int64_t n, double* x, double* r, const double* p, const double* q,
                                double* partial, double* s, double rtol2, const int64_t* ptr, const int64_t* list,
                                const double* w, TC* copies) {
  const unsigned nb = dot_blocks(n);
  hipLaunchKernelGGL(k_pcg_update_xr_partial<TC>, dim3(nb), dim3(256), 0, st, n, x, r, p, q, s, partial, ptr, list, w, copies);
  hipLaunchKernelGGL(k_dot_step, dim3(1), dim3(256), 0, st, (int)nb, partial, s, (int)S_RR, (int)DOT_CHECK, nullptr, nullptr,
                     rtol2);
}
template void launch_pcg_update_xr_check<double>(hipStream_t, int64_t, double*, double*, const double*, const double*,
                                                 double*, double*, double, const int64_t*, const int64_t*, const double*,
                                                 double*);
template void launch_pcg_update_xr_check<float>(hipStream_t, int64_t, double*, double*, const double*, const double*, double*,
                                                double*, double, const int64_t*, const int64_t*, const double*, float*);

void launch_set_int(hipStream_t st, int* p, int v) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v); }
void launch_pcg_update_p(hipStream_t st, int64_t n, double* p, const double* z, const double* s, const int64_t* ptr,
                         const int64_t* list, double* copies) {
  hipLaunchKernelGGL(k_pcg_update_p, dim3(grid_for(n)), dim3(256), 0, st, n, p, z, s, ptr, list, copies);
}
void launch_axpby(hipStream_t st, int64_t n, double a, const double* x, double b, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, n, a, x, b, y);
}
void launch_fill(hipStream_t st, int64_t n, double v, double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, st, n, v, y);
}
void launch_element_energy(hipStream_t st, int64_t ne, int nloc, const int32_t* edof, const double* K0, const double* scale,
                           const double* a, const double* b, double* out) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(k_element_energy, dim3(grid_for(ne)), dim3(256), 0, st, ne, nloc, edof, K0, scale, a, b, out);
}

template <typename T>
void launch_gather64(hipStream_t st, int64_t n, const int64_t* pos, const T* A, double* out) {
  if (n > 0) hipLaunchKernelGGL(k_gather64<T>, dim3(grid_for(n)), dim3(256), 0, st, n, pos, A, out);
}
template void launch_gather64<float>(hipStream_t, int64_t, const int64_t*, const float*, double*);
template void launch_gather64<double>(hipStream_t, int64_t, const int64_t*, const double*, double*);
void launch_ratio(hipStream_t st, int64_t n, const double* d, const double* s, const int32_t* idx, double* w) {
  if (n > 0) hipLaunchKernelGGL(k_ratio, dim3(grid_for(n)), dim3(256), 0, st, n, d, s, idx, w);
}
void launch_scatter_idx(hipStream_t st, int64_t n, const int32_t* idx, const double* in, double* out) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_idx, dim3(grid_for(n)), dim3(256), 0, st, n, idx, in, out);
}

#define INST_MV(TA, TX, TY)                                                                                             \
  template void launch_tile_mv_sum<TA, TX, TY>(hipStream_t, int, const MvDesc*, int, const MvDesc*, int32_t, int32_t, \
                                               const TA*, const TX*, const TX*, TY*, double, bool);                   \
  template void launch_tile_mv<TA, TX, TY>(hipStream_t, int, const MvDesc*, int32_t, int64_t, const int64_t*, const TA*, \
                                           const TX*, TY*, double, bool, TA*, int32_t, hipEvent_t, hipEvent_t, int, int64_t, \
                                           const int64_t*);
INST_MV(double, double, double)
INST_MV(float, float, float)
INST_MV(float, float, double)
INST_MV(double, double, float)
#undef INST_MV
template void launch_gather<double, double>(hipStream_t, int64_t, const int32_t*, const double*, const double*, double*);
template void launch_gather<double, float>(hipStream_t, int64_t, const int32_t*, const double*, const double*, float*);
template void launch_gather<float, float>(hipStream_t, int64_t, const int32_t*, const double*, const float*, float*);
template void launch_gather<float, double>(hipStream_t, int64_t, const int32_t*, const double*, const float*, double*);
template void launch_seg_reduce<double>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*, const double*,
                                        double*, double, const double*);
template void launch_seg_reduce<float>(hipStream_t, int64_t, const int64_t*, const int64_t*, const double*, const float*,
                                       double*, double, const float*);
void launch_gather_seg(hipStream_t st, int64_t n, const int32_t* bidx, const double* base, const int64_t* ptr,
                       const int64_t* list, const double* in, double* out) {
  if (n > 0) hipLaunchKernelGGL(k_gather_seg, dim3(grid_for(n)), dim3(256), 0, st, n, bidx, base, ptr, list, in, out);
}
template <typename TI>
void launch_scatter2(hipStream_t st, int64_t n1, const int32_t* i1, const TI* in1, int64_t n2, const int32_t* i2,
                     const double* in2, double* out) {
  if (n1 + n2 > 0) hipLaunchKernelGGL(k_scatter2<TI>, dim3(grid_for(n1 + n2)), dim3(256), 0, st, n1, i1, in1, n2, i2, in2, out);
}
template void launch_scatter2<double>(hipStream_t, int64_t, const int32_t*, const double*, int64_t, const int32_t*,
                                      const double*, double*);
template void launch_scatter2<float>(hipStream_t, int64_t, const int32_t*, const float*, int64_t, const int32_t*,
                                     const double*, double*);
template void launch_scatter<double, double>(hipStream_t, int64_t, const int32_t*, const double*, double*);
template void launch_scatter<float, float>(hipStream_t, int64_t, const int32_t*, const float*, float*);
template void launch_scatter<double, float>(hipStream_t, int64_t, const int32_t*, const double*, float*);
template void launch_scatter<float, double>(hipStream_t, int64_t, const int32_t*, const float*, double*);

}  // namespace mlbddc
