// Batched tile factorization engine and set-up kernels for gfx950.
//
// The engine performs a right-looking blocked Cholesky on tile-packed lower
// matrices, eliminating a given number of leading tile columns of every
// matrix in a batch (a partial factorization leaves the Schur complement of
// the eliminated block in the trailing tiles).  Work is organised as task
// lists built on the host from each matrix's tile envelope, so tiles that
// stay zero are never touched, and all matrices of a level advance in one
// launch per step:
//   DIAG    factor the diagonal tile in LDS and store its inverse;
//   PANEL   A_rk <- A_rk inv(L_kk)^T                      (MFMA)
//   UPDATE  A_rs <- A_rs - sum_k A_rk A_sk^T              (MFMA)
//   NEGATE  flip the sign of a trailing block between two phases.
// MFMA tiles use v_mfma_f64_16x16x4f64 (FP64) and v_mfma_f32_16x16x4f32 (FP32)
// with 64-wide wavefronts; a 64x64 output tile is split over 4 wavefronts.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace mlbddc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int LDT = TS + 1;  // LDS leading dimension of a staged tile (odd: conflict-free columns)

template <typename T> struct Mfma;
// Output layout of the 16x16x4 products: register v of lane l holds row
// row(l/16, v) and column l%16 of the 16x16 block; the FP64 instruction
// interleaves the rows (g + 4v), the FP32 one keeps them contiguous (4g + v).
template <> struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static int row(int g, int v) { return g + 4 * v; }
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t mac(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static int row(int g, int v) { return 4 * g + v; }
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t mac(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// Stage a 64x64 column-major tile from global memory into LDS (ld LDT),
// optionally transposed, converting from TS_ to T.
template <typename T, typename TSRC>
__device__ inline void stage_tile(T* __restrict__ s, const TSRC* __restrict__ g, bool trans) {
  // 256 threads: every load is issued before the first LDS store
  constexpr int PER = TE / 256;
  TSRC v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) v[q] = g[threadIdx.x + 256 * q];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = threadIdx.x + 256 * q, i = idx & (TS - 1), j = idx >> 6;
    if (trans) s[i * LDT + j] = (T)v[q]; else s[j * LDT + i] = (T)v[q];
  }
}

// acc(i, j) += sum_k R(i, k) S(j, k) over one staged k-tile.  Wave w owns
// rows (w&1)*32.. and columns (w>>1)*32.. of the output; lane l of block
// (bi, bj) ends with rows i0 + l%16, columns j0 + Mfma<T>::row(l/16, v).
template <typename T>
__device__ inline void tile_nt(typename Mfma<T>::acc_t (&acc)[2][2], const T* __restrict__ sR, const T* __restrict__ sS) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < TS; k0 += 4) {
    const int kk = k0 + kq;
    T a[2], b[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) a[bj] = sS[kk * LDT + jw + bj * 16 + l16];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) b[bi] = sR[kk * LDT + iw + bi * 16 + l16];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mfma<T>::mac(a[bj], b[bi], acc[bi][bj]);
  }
}

// Global address helpers for the accumulator layout.
template <typename T, typename F>
__device__ inline void for_acc(typename Mfma<T>::acc_t (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = iw + bi * 16 + (lane & 15);
        int j = jw + bj * 16 + Mfma<T>::row(lane >> 4, v);
        f(i, j, acc[bi][bj][v]);
      }
}

// ------------------------------------------------------------------ assembly
// One wavefront per element (four per workgroup): A += scale * Ke on the
// lower tiles of the owning subdomain's matrix.  el_local holds, per element
// node, the local index of the node's first DOF (its nd DOFs are consecutive)
// or -1.  Consecutive lanes take consecutive rows of one element column, so a
// node's nd rows are one contiguous run of a tile column.  An entry that falls
// in a tile the map does not store is skipped and raises *err.
template <typename T>
__global__ void __launch_bounds__(256) k_assemble(const int64_t* __restrict__ elems, int64_t n,
                                                  const int32_t* __restrict__ el_local_ptr,
                                                  const int32_t* __restrict__ el_local, int nd, const int32_t* __restrict__ el_sub,
                                                  const int64_t* __restrict__ sub_off, const int32_t* __restrict__ sub_nt,
                                                  const double* __restrict__ Kref, const double* __restrict__ scale,
                                                  const int64_t* __restrict__ ekc_off, const double* __restrict__ ekc, T* A,
                                                  const int32_t* __restrict__ tmap, const int64_t* __restrict__ tmap_off,
                                                  int32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t e = elems[i];
  const int b = el_sub[e];
  const int32_t base = el_local_ptr[e];
  const int nloc = (el_local_ptr[e + 1] - base) * nd;
  const int64_t off = sub_off[b];
  const int nt = sub_nt[b];
  const double sc = Kref ? scale[e] : 1.0;
  const double* M = Kref ? Kref : ekc + ekc_off[e];
  for (int idx = lane; idx < nloc * nloc; idx += 64) {
    const int c = idx / nloc, a = idx - c * nloc;
    const int na = a / nd, nc = c / nd;
    const int ka = el_local[base + na], kc = el_local[base + nc];
    if (ka < 0 || kc < 0) continue;
    const int p = ka + (a - na * nd), q = kc + (c - nc * nd);
    if (p / TS < q / TS) continue;
    const int64_t slot = tile_slot(tmap, tmap_off, b, p / TS, q / TS, nt);
    if (slot < 0) {
      atomicOr(err, 1);
      continue;
    }
    A[off + slot * TE + (q % TS) * TS + (p % TS)] += (T)(sc * M[a * nloc + c]);
  }
}

// Zero n16 16-byte words.
__global__ void __launch_bounds__(256) k_zero16(uint4* __restrict__ p, int64_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256) p[i] = z;
}

template <typename T>
__global__ void k_set_diag(const DiagSeg* __restrict__ segs, T* A, const int32_t* __restrict__ tmap,
                           const int64_t* __restrict__ tmap_off) {
  const DiagSeg s = segs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.count; i += gridDim.x * blockDim.x) {
    const int64_t p = s.row0 + i, q = s.col0 + i;
    const int64_t slot = s.item >= 0 ? tile_slot(tmap, tmap_off, s.item, p / TS, q / TS, s.nt) : tile_index(p / TS, q / TS, s.nt);
    A[s.off + slot * TE + (q % TS) * TS + (p % TS)] = (T)s.val;
  }
}

// ------------------------------------------------------------ factorization
// Value of v in lane n of the caller's row of 16 lanes (DPP row_newbcast).
template <int N>
__device__ inline double row_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x150 + N, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + N, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int N>
__device__ inline float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + N, 0xf, 0xf, false));
}

// 1/sqrt(x) for a positive finite pivot: the hardware estimate refined by one
// Newton step y <- y + y (1/2 - x y^2 / 2) (relative error ~3e-14 in FP64).
__device__ inline double rsqrt_pivot(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double r = fma(-0.5 * x * y, y, 0.5);
  return fma(y, r, y);
}
__device__ inline float rsqrt_pivot(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float r = fmaf(-0.5f * x * y, y, 0.5f);
  return fmaf(y, r, y);
}

// Compile-time loop: f(integral_constant<J>) for J = B..E-1.
template <int B, int E, typename F>
__device__ inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// 16x16 block products on MFMA between blocks held in LDS with leading
// dimension LDT: acc += sx * X * Y.  Lane l supplies X(m, k) and Y(k, n) for
// m = n = l%16 and k = 4s + l/16, and holds the result entries
// (Mfma<T>::row(l/16, v), l%16).  Operand storage forms:
//   X: XC  X(m, k) = X[k*LDT + m] (column-major)
//      XR  X(m, k) = X[m*LDT + k], zero above the diagonal (m < k)
//   Y: YR  Y(k, n) = Y[k*LDT + n], optionally zero where k < n
//      YC  Y(k, n) = Y[n*LDT + k], zero where n < k
enum { XC = 0, XR = 1, YR = 0, YRL = 1, YC = 2 };
template <typename T, int XF, int YF>
__device__ inline void mm16(typename Mfma<T>::acc_t& acc, const T* X, const T* Y, T sx) {
  const int l16 = threadIdx.x & 15, g = (threadIdx.x >> 4) & 3;
  T a[4], b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + g;
    a[s] = XF == XC ? X[k * LDT + l16] : (l16 >= k ? X[l16 * LDT + k] : (T)0);
    a[s] *= sx;
    b[s] = YF == YR ? Y[k * LDT + l16] : YF == YRL ? (k >= l16 ? Y[k * LDT + l16] : (T)0)
                                                    : (l16 >= k ? Y[l16 * LDT + k] : (T)0);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = Mfma<T>::mac(a[s], b[s], acc);
}
// Result block stored column-major (O[n*LDT + m]) or transposed (O[m*LDT + n]).
template <typename T>
__device__ inline void load16(typename Mfma<T>::acc_t& acc, const T* O) {
  const int l16 = threadIdx.x & 15, g = (threadIdx.x >> 4) & 3;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = O[l16 * LDT + Mfma<T>::row(g, v)];
}
template <typename T>
__device__ inline void store16(const typename Mfma<T>::acc_t& acc, T* O) {
  const int l16 = threadIdx.x & 15, g = (threadIdx.x >> 4) & 3;
#pragma unroll
  for (int v = 0; v < 4; ++v) O[l16 * LDT + Mfma<T>::row(g, v)] = acc[v];
}
template <typename T>
__device__ inline void store16t(const typename Mfma<T>::acc_t& acc, T* O) {
  const int l16 = threadIdx.x & 15, g = (threadIdx.x >> 4) & 3;
#pragma unroll
  for (int v = 0; v < 4; ++v) O[Mfma<T>::row(g, v) * LDT + l16] = acc[v];
}

// Diagonal tile: Cholesky factor L and W = L^{-1}, blocked by 16, in one
// LDS tile (small enough to share a CU with the update kernel).
// For each block column jb: wavefront 0 factors the 16x16 diagonal block in
// registers (lane i keeps row i; pivots and the column of L are read from
// the owning lanes), writes that block of L to global memory, and forms the
// block's inverse by forward substitution; the blocks below are multiplied
// by that inverse and the trailing blocks updated with MFMA products, one
// block per wavefront.  The off-diagonal blocks of W follow from
// W_ij = -inv(L_ii) sum_{j<=m<i} L_im W_mj, one block column per wavefront.
// W is kept transposed in the upper triangle of the tile (entry (r, c) of W
// at LDS position (c, r)), the strict lower triangle holds L.  A
// non-positive pivot is reported in err (first failing item, then its
// column) and turns the rest of the tile into NaN.
template <typename T>
__global__ void __launch_bounds__(256) k_diag(const uint64_t* __restrict__ tasks, const int64_t* __restrict__ off,
                                              const int32_t* __restrict__ ntv, const int64_t* __restrict__ inv_off,
                                              int32_t* err, T* A, T* Inv, const int32_t* __restrict__ tmap,
                                              const int64_t* __restrict__ tmap_off) {
  __shared__ T sA[TS * LDT];
  __shared__ T colbuf[16];
  typedef typename Mfma<T>::acc_t acc_t;
  const uint64_t t = tasks[blockIdx.x];
  const int item = task_item(t), k = task_r(t);
  const int nt = ntv[item];
  T* gA = A + off[item] + tile_slot(tmap, tmap_off, item, k, k, nt) * TE;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  stage_tile<T, T>(sA, gA, false);
  if (task_neg(t))  // second phase: the stored block is the negative of the matrix factored (own entries only)
    for (int idx = tid; idx < TE; idx += 256) sA[(idx >> 6) * LDT + (idx & (TS - 1))] = -sA[(idx >> 6) * LDT + (idx & (TS - 1))];
  __syncthreads();
  int badcol = -1;
#pragma unroll 1
  for (int jb = 0; jb < 4; ++jb) {
    const int j0 = 16 * jb;
    T* D = &sA[j0 * LDT + j0];
    if (w == 0) {
      // Lane l = 16 q + i keeps row i of the block in the columns m = 4 t + q
      // (d[t]) and row i of V, the inverse of the block's factor, in the same
      // columns (v[t]).  Step j: the lanes owning column j put it in LDS; every
      // lane reads the pivot, its own row's entry and the entries of its
      // columns, finishes column j of L and eliminates it from its trailing
      // columns; then row j of V is scaled and eliminated from the rows of V
      // below (row j of V lives in lane j of each row of 16 lanes, broadcast
      // with DPP).
      const int i = lane & 15, q = lane >> 4;
      T d[4], v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        d[t] = D[(4 * t + q) * LDT + i];
        v[t] = 4 * t + q == i ? (T)1 : (T)0;
      }
      static_for<0, 16>([&](auto J) {
        constexpr int j = decltype(J)::value, qj = j & 3, tj = j >> 2;
        if (q == qj) colbuf[i] = d[tj];
        __builtin_amdgcn_wave_barrier();
        T piv = colbuf[j];
        const T ai = colbuf[i];
        T am[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) am[t] = 4 * t + 3 > j ? colbuf[(4 * t + q) & 15] : (T)0;
        __builtin_amdgcn_wave_barrier();
        const bool ok = piv > (T)0;
        badcol = (!ok && badcol < 0) ? j0 + j : badcol;
        piv = ok ? piv : (T)NAN;
        const T inv = rsqrt_pivot(piv), sq = piv * inv;
        const T lij = i > j ? ai * inv : (i == j ? sq : (T)0);
        if (q == qj) d[tj] = lij;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (4 * t + 3 > j) {
            const int m = 4 * t + q;
            if (m > j) d[t] -= lij * (am[t] * inv);
          }
        const T lv = i > j ? lij : (T)0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (4 * t <= j) {
            const int c = 4 * t + q;
            if (i == j) v[t] *= inv;
            const T vj = row_bcast<j>(v[t]);
            if (c <= j) v[t] -= lv * vj;
          }
      });
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = 4 * t + q;
        gA[(j0 + m) * TS + j0 + i] = m <= i ? d[t] : (T)0;
        if (m < i) D[m * LDT + i] = d[t];
        if (m <= i) D[i * LDT + m] = v[t];  // V(i, m) at block position (m, i)
      }
    }
    __syncthreads();
    if (w < 3 - jb) {  // L(ib, jb) = A(ib, jb) V^T
      const int ib = jb + 1 + w;
      acc_t acc = Mfma<T>::zero();
      mm16<T, XC, YC>(acc, &sA[j0 * LDT + 16 * ib], D, (T)1);
      store16<T>(acc, &sA[j0 * LDT + 16 * ib]);
    }
    __syncthreads();
    const int nb = (3 - jb) * (4 - jb) / 2;  // trailing blocks (ib, kb), jb < kb <= ib
    for (int b = w; b < nb; b += 4) {
      int kb = jb + 1, rem = b;
      while (rem >= 4 - kb) {
        rem -= 4 - kb;
        ++kb;
      }
      const int ib = kb + rem;
      acc_t acc;
      load16<T>(acc, &sA[16 * kb * LDT + 16 * ib]);
      mm16<T, XC, YR>(acc, &sA[j0 * LDT + 16 * ib], &sA[j0 * LDT + 16 * kb], (T)-1);
      store16<T>(acc, &sA[16 * kb * LDT + 16 * ib]);
    }
    __syncthreads();
  }
  // off-diagonal blocks of W: wavefront w computes block column w
#pragma unroll 1
  for (int step = 1; step <= 3; ++step) {
    const int jb = w, ib = w + step;
    const bool act = ib <= 3;
    T* Wij = &sA[16 * ib * LDT + 16 * jb];  // W(ib, jb), transposed storage
    acc_t acc = Mfma<T>::zero();
    if (act) {
      mm16<T, XC, YRL>(acc, &sA[16 * jb * LDT + 16 * ib], &sA[16 * jb * LDT + 16 * jb], (T)1);
      for (int mb = jb + 1; mb < ib; ++mb) mm16<T, XC, YR>(acc, &sA[16 * mb * LDT + 16 * ib], &sA[16 * mb * LDT + 16 * jb], (T)1);
      store16t<T>(acc, Wij);
    }
    __syncthreads();
    if (act) {
      acc = Mfma<T>::zero();
      mm16<T, XR, YR>(acc, &sA[16 * ib * LDT + 16 * ib], Wij, (T)-1);
      store16t<T>(acc, Wij);
    }
    __syncthreads();
  }
  if (tid == 0 && badcol >= 0 && atomicCAS(&err[0], 0, item + 1) == 0) err[1] = k * TS + badcol;
  T* gI = Inv + inv_off[item] + (int64_t)k * TE;
#pragma unroll
  for (int q = 0; q < TE / 256; ++q) {
    const int idx = tid + 256 * q, r = idx & (TS - 1), c = idx >> 6;
    if ((r >> 4) != (c >> 4)) gA[idx] = r > c ? sA[c * LDT + r] : (T)0;
    gI[idx] = r >= c ? sA[r * LDT + c] : (T)0;
  }
}

// Register staging of NE consecutive elements of a column-major 64x64 tile
// (the whole tile, or the 32 columns of one half): each of the 256 threads
// holds NE/256 elements as 16-byte vectors (coalesced loads), then stores
// them to LDS with leading dimension LD.
template <typename T, int NE>
struct ChunkRegs {
  static constexpr int V = 16 / sizeof(T);          // elements per 16-byte vector
  static constexpr int N = NE / (256 * V);          // vectors per thread
  typedef T vec __attribute__((ext_vector_type(V)));
  vec v[N];
  __device__ void load(const T* __restrict__ g) {
    const vec* gv = reinterpret_cast<const vec*>(g);
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = gv[threadIdx.x + 256 * m];
  }
  template <int LD>
  __device__ void store(T* __restrict__ s) const {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int e = (threadIdx.x + 256 * m) * V;     // first element: row e%64, column e/64
      const int i = e & (TS - 1), j = e >> 6;
#pragma unroll
      for (int q = 0; q < V; ++q) s[j * LD + i + q] = v[m][q];
    }
  }
};

// acc(i, j) += sum_k R(i, k) S(j, k) over KN staged columns k (LDS leading dimension LD).
template <typename T, int LD, int KN>
__device__ inline void tile_nt_ld(typename Mfma<T>::acc_t (&acc)[2][2], const T* __restrict__ sR, const T* __restrict__ sS) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < KN; k0 += 4) {
    const int kk = k0 + kq;
    T a[2], b[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) a[bj] = sS[kk * LD + jw + bj * 16 + l16];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) b[bi] = sR[kk * LD + iw + bi * 16 + l16];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mfma<T>::mac(a[bj], b[bi], acc[bi][bj]);
  }
}

constexpr int LDU = TS + 16;  // keeps the four k-groups of a fragment read on distinct LDS banks

// Output accumulators of a workgroup's 64x64 tile product, per MFMA shape:
// SH = 16 takes 2x2 blocks of 16x16x4 per wavefront (FP64 and FP32), SH = 32
// one 32x32x2 block (FP32; lane l holds rows i0 + l % 32 of the columns
// j0 + (v % 4) + 8 (v / 4) + 4 (l / 32), v = 0..15).  Wave w owns rows
// (w & 1) * 32.. and columns (w >> 1) * 32.. of the output either way; each()
// visits a lane's outputs in a fixed order.
typedef float f16v __attribute__((ext_vector_type(16)));
template <typename T, int SH> struct TileAcc;
template <typename T> struct TileAcc<T, 16> {
  typename Mfma<T>::acc_t a[2][2];
  __device__ void zero() {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) a[i][j] = Mfma<T>::zero();
  }
  template <int LD, int KN>
  __device__ void mul(const T* __restrict__ sR, const T* __restrict__ sS) { tile_nt_ld<T, LD, KN>(a, sR, sS); }
  template <typename F>
  __device__ void each(F f) { for_acc<T>(a, f); }
};
template <> struct TileAcc<float, 32> {
  f16v a;
  __device__ void zero() {
#pragma unroll
    for (int v = 0; v < 16; ++v) a[v] = 0.f;
  }
  // acc(i, j) += sum_k R(i, k) S(j, k) over KN staged columns k, two per instruction
  template <int LD, int KN>
  __device__ void mul(const float* __restrict__ sR, const float* __restrict__ sS) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
    const int l32 = lane & 31, kq = lane >> 5;
#pragma unroll
    for (int k0 = 0; k0 < KN; k0 += 2) {
      const int kk = k0 + kq;
      a = __builtin_amdgcn_mfma_f32_32x32x2f32(sS[kk * LD + jw + l32], sR[kk * LD + iw + l32], a, 0, 0, 0);
    }
  }
  template <typename F>
  __device__ void each(F f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
#pragma unroll
    for (int v = 0; v < 16; ++v) f(iw + (lane & 31), jw + (v & 3) + 8 * (v >> 2) + 4 * (lane >> 5), a[v]);
  }
};

// SH = SH_BF3: FP32 tile products from bfloat16 pieces on the bf16 MFMA
// (16x16x32, sixteen times the FP32 MFMA rate).  A staged FP32 value x is
// split by round-to-nearest in turn, h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m); both subtractions are exact in FP32, and the last
// remainder has at most 8 significant bits, so h + m + l = x exactly for
// |x| above 2^-100.  A product keeps the six terms down to weight 2^-16
// (hh, hm, mh, hl, lh, mm; the dropped ones are below 2^-23 |a||b|), each
// exact in FP32, summed by the MFMA into the running accumulator, smallest
// weight first.  The k dimension advances 32 columns per instruction, so
// the products take KS >= 32.  Measured on the 96^3 elasticity workload:
// the FP32 updates of the constrained problems 13 % faster than with the
// FP32 MFMA, the preconditioner's error against FP64 two to four times as
// large (2.5e-3 against 5.6e-4 at four levels; keeping all nine terms, or
// adding the chunk sums by FP32 adds, did not reduce it); an option, not the
// default.
//
// LDS holds three planes per operand in the order the MFMA operands are
// read: for each 32-column chunk and each block of 16 rows, 512 values with
// row r, column k at ((k % 32) / 8 * 16 + r % 16) * 8 + k % 8, so lane l of
// a fragment read takes the 16 bytes at l * 16 and a wavefront's read is 1
// KiB contiguous; a staging write by 16 lanes of consecutive rows is 256
// contiguous bytes.  Every 16-byte access of lane l lands on the banks of
// l % 16, whichever lanes the hardware serves together.
constexpr int SH_BF3 = 3;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
template <int KS> struct SplitLds {
  static constexpr int PL = TS * KS;         // values per plane
  static constexpr int floats = 3 * PL / 2;  // LDS per operand, in floats
  // first value of the 8 at row i, columns k..k+7 (k a multiple of 8)
  __device__ static int at(int i, int k) { return ((k >> 5) * 4 + (i >> 4)) * 512 + (((k & 31) >> 3) * 16 + (i & 15)) * 8; }
};

// Two FP32 values rounded to nearest bf16, packed (a low, b high), and back.
__device__ inline uint32_t pack_bf16(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  typedef float fl2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2){a, b}, bf2));
}
__device__ inline float lo_bf16(uint32_t p) { return __uint_as_float(p << 16); }
__device__ inline float hi_bf16(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// Register staging of KS columns of a column-major 64x64 FP32 tile for the
// split products: thread t holds row t % 64, columns (t / 64) * KS/4 + m
// (each load instruction reads 256 contiguous bytes across the wavefront),
// and stores the three pieces as 16-byte LDS writes.
template <int KS>
struct SplitRegs {
  static constexpr int N = KS / 4;
  float v[N];
  __device__ void load(const float* __restrict__ g) {
    const int i = threadIdx.x & 63, k0 = (threadIdx.x >> 6) * N;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = g[(k0 + m) * TS + i];
  }
  template <int LD>
  __device__ void store(float* __restrict__ s) const {
    constexpr int PL = SplitLds<KS>::PL;
    __bf16* p = reinterpret_cast<__bf16*>(s);
    const int i = threadIdx.x & 63, k0 = (threadIdx.x >> 6) * N;
#pragma unroll
    for (int c = 0; c < N / 8; ++c) {
      uint32_t h[4], m[4], l[4];  // bf16 pairs: element 2q in the low half, 2q + 1 in the high half
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float x0 = v[8 * c + 2 * q], x1 = v[8 * c + 2 * q + 1];
        h[q] = pack_bf16(x0, x1);
        const float r0 = x0 - lo_bf16(h[q]), r1 = x1 - hi_bf16(h[q]);
        m[q] = pack_bf16(r0, r1);
        l[q] = pack_bf16(r0 - lo_bf16(m[q]), r1 - hi_bf16(m[q]));
      }
      const int e = SplitLds<KS>::at(i, k0 + 8 * c);
      *reinterpret_cast<uint4*>(p + e) = make_uint4(h[0], h[1], h[2], h[3]);
      *reinterpret_cast<uint4*>(p + PL + e) = make_uint4(m[0], m[1], m[2], m[3]);
      *reinterpret_cast<uint4*>(p + 2 * PL + e) = make_uint4(l[0], l[1], l[2], l[3]);
    }
  }
};

// acc(i, j) += sum_k R(i, k) S(j, k) over KN staged columns from the split
// planes; the 16x16 output blocks and their lane layout are those of the
// FP32 16x16x4 products.
template <> struct TileAcc<float, SH_BF3> {
  f4 a[2][2];
  __device__ void zero() {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) a[i][j] = Mfma<float>::zero();
  }
  template <int LD, int KN>
  __device__ void mul(const float* __restrict__ sR, const float* __restrict__ sS) {
    constexpr int PL = SplitLds<KN>::PL;
    const __bf16* pR = reinterpret_cast<const __bf16*>(sR);
    const __bf16* pS = reinterpret_cast<const __bf16*>(sS);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
    // (piece of S, piece of R) per term, smallest weight first
    constexpr int PS[6] = {1, 2, 0, 1, 0, 0}, PR[6] = {1, 0, 2, 0, 1, 0};
#pragma unroll
    for (int k0 = 0; k0 < KN; k0 += 32) {
      bf8 sa[3][2], rb[3][2];
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          sa[p][b] = *reinterpret_cast<const bf8*>(pS + p * PL + ((k0 >> 5) * 4 + (jw >> 4) + b) * 512 + lane * 8);
          rb[p][b] = *reinterpret_cast<const bf8*>(pR + p * PL + ((k0 >> 5) * 4 + (iw >> 4) + b) * 512 + lane * 8);
        }
#pragma unroll
      for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            a[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sa[PS[q]][bj], rb[PR[q]][bi], a[bi][bj], 0, 0, 0);
    }
  }
  template <typename F>
  __device__ void each(F f) { for_acc<float>(a, f); }
};

// Workgroups are dealt to the 8 XCDs of the chip round-robin by launch
// index; this maps launch index b to a task index so that each XCD receives
// one contiguous slice of the task list (tasks of the same matrix, which
// share panel tiles, then meet in the same L2).
__device__ inline int64_t xcd_slice(int64_t b, int64_t n) {
  constexpr int64_t NX = 8;
  const int64_t x = b % NX, j = b / NX, q = n / NX, rem = n % NX;
  return x * q + (x < rem ? x : rem) + j;
}

// Tile products on MFMA, one 64x64 output tile per workgroup:
//   UPDATE  A_rs <- A_rs - sum_{kk=kf..kf+nk} A_{r,kk} A_{s,kk}^T   (kf, nk from the task)
//   PANEL   A_rk <- A_rk inv(L_kk)^T
// The k dimension advances KS columns at a time (KS = 16, 32 or 64, a tuning
// parameter; 2 x KS x LDU values of LDS).  The next pair of column blocks is
// loaded into registers while the current pair is multiplied from LDS;
// during the last pair the registers freed by that prefetch receive the
// output tile of an UPDATE.  The products accumulate over k in the same order
// for every KS, so the results do not depend on it.
template <int KS> struct StageOcc { static constexpr int blocks = 4; };
template <> struct StageOcc<64> { static constexpr int blocks = 2; };  // twice the LDS and staging registers

template <typename T, bool PANEL, int KS, int SH = 16>
__global__ void __launch_bounds__(256, StageOcc<KS>::blocks) k_tile_mm(
    const uint64_t* __restrict__ tasks, const int64_t* __restrict__ off, const int32_t* __restrict__ ntv,
    const int64_t* __restrict__ inv_off, T* A, const T* __restrict__ Inv, const int32_t* __restrict__ tmap,
    const int64_t* __restrict__ tmap_off) {
  static_assert(KS == 16 || KS == 32 || KS == 64, "staged columns");
  static_assert(SH != SH_BF3 || (std::is_same<T, float>::value && KS >= 32), "split products: FP32, KS >= 32");
  constexpr int SPT = TS / KS;  // steps per tile
  constexpr int NS = SH == SH_BF3 ? SplitLds<KS>::floats : KS * LDU;
  __shared__ __attribute__((aligned(16))) T sR[NS];
  __shared__ __attribute__((aligned(16))) T sS[NS];
  using Regs = typename std::conditional<SH == SH_BF3, SplitRegs<KS>, ChunkRegs<T, KS * TS>>::type;
  const uint64_t t = tasks[xcd_slice(blockIdx.x, gridDim.x)];
  const int item = task_item(t), r = task_r(t), s = task_s(t);
  const int kf = PANEL ? s : task_kf(t);
  const int nsteps = PANEL ? SPT : SPT * (task_nk(t) + 1);
  const int nt = ntv[item];
  T* base = A + off[item];
  T* g = base + tile_slot(tmap, tmap_off, item, r, s, nt) * TE;
  const bool same = !PANEL && r == s;
  // a tile-mapped matrix: lane j holds the slots of tiles (r, kf + j) and
  // (s, kf + j), loaded together up front (the schedule keeps at most 64
  // columns per task on such matrices)
  const int64_t mo = tmap ? tmap_off[item] : -1;
  int32_t rslot = 0, sslot = 0;
  if (mo >= 0) {
    const int j = threadIdx.x & 63;
    if (j < (PANEL ? 1 : task_nk(t) + 1)) {
      rslot = tmap[mo + tile_index(r, kf + j, nt)];
      if (!PANEL) sslot = tmap[mo + tile_index(s, kf + j, nt)];
    }
  }
  auto rtile = [&](int j) -> int64_t { return mo >= 0 ? __builtin_amdgcn_readlane(rslot, j) : tile_index(r, kf + j, nt); };
  auto stile = [&](int j) -> int64_t { return mo >= 0 ? __builtin_amdgcn_readlane(sslot, j) : tile_index(s, kf + j, nt); };
  auto rsrc = [&](int q) { return base + rtile(q / SPT) * TE + (q % SPT) * (TE / SPT); };
  auto ssrc = [&](int q) -> const T* {
    return PANEL ? Inv + inv_off[item] + (int64_t)s * TE + (q % SPT) * (TE / SPT)
                 : base + stile(q / SPT) * TE + (q % SPT) * (TE / SPT);
  };
  TileAcc<T, SH> acc;
  acc.zero();
  Regs pr, ps;
  pr.load(rsrc(0));
  if (!same) ps.load(ssrc(0));
  for (int q = 0; q + 1 < nsteps; ++q) {
    pr.template store<LDU>(sR);
    if (!same) ps.template store<LDU>(sS);
    __syncthreads();
    pr.load(rsrc(q + 1));
    if (!same) ps.load(ssrc(q + 1));
    acc.template mul<LDU, KS>(sR, same ? sR : sS);
    __syncthreads();
  }
  pr.template store<LDU>(sR);
  if (!same) ps.template store<LDU>(sS);
  __syncthreads();
  T creg[16];
  if (!PANEL) {
    int n = 0;
    acc.each([&](int i, int j, T) { creg[n++] = g[j * TS + i]; });
  }
  acc.template mul<LDU, KS>(sR, same ? sR : sS);
  int n = 0;
  const T sg = task_neg(t) ? (T)-1 : (T)1;  // second-phase task: the block is stored negated
  if (PANEL) acc.each([&](int i, int j, T v) { g[j * TS + i] = sg * v; });
  else acc.each([&](int i, int j, T v) { g[j * TS + i] = creg[n++] - sg * v; });
}

// ----------------------------------------------------- preconditioner set-up
template <typename TK, typename TP>
__global__ void __launch_bounds__(256) k_copy_block(const CopyDesc* __restrict__ d, const TK* __restrict__ K, TP* P) {
  const CopyDesc c = d[blockIdx.z];
  const int r = blockIdx.x, s = blockIdx.y;
  if (r >= c.nblk || s > r) return;
  const TK* src = K + c.src_off + tile_index(c.src_t0 + r, c.src_t0 + s, c.src_nt) * TE;
  TP* dst = P + c.dst_off + tile_index(r, s, c.dst_nt) * TE;
  for (int idx = threadIdx.x; idx < TE; idx += blockDim.x) dst[idx] = (TP)src[idx];
}

// One workgroup per constraint row: rho = m * mean(S_kk) over the row's DOFs;
// S~ += (rho / m^2) 1 1^T on those DOFs; C row entries 1/m.
template <typename TK, typename TP>
__global__ void __launch_bounds__(256) k_constraints(const ConsDesc* __restrict__ d, const int32_t* __restrict__ cols,
                                                     const TK* __restrict__ K, TP* P, double* rho_out) {
  const ConsDesc c = d[blockIdx.x];
  const int m = c.ptr1 - c.ptr0;
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    int64_t p = c.k_g0 + cols[c.ptr0 + i];
    s += (double)K[c.kdiag_off + packed_offset(p, p, c.k_nt)];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double rho = red[0];  // m * mean = sum of the diagonal entries
  if (threadIdx.x == 0) rho_out[blockIdx.x] = rho;
  const double add = rho / ((double)m * (double)m);
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    int a = idx / m, b = idx - a * m;
    int64_t p = cols[c.ptr0 + a], q = cols[c.ptr0 + b];
    if (p / TS < q / TS) continue;
    P[c.p_off + packed_offset(p, q, c.p_nt)] += (TP)add;
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x)
    P[c.p_off + packed_offset(c.c_row0, cols[c.ptr0 + i], c.p_nt)] = (TP)(1.0 / m);
}

// K_Ci = A_i^{-1} - W_i: after both elimination phases the coarse block of
// the constrained-problem matrix holds A_i^{-1} (A_i = C S~^{-1} C^T; the
// second phase leaves the blocks it does not factor with the opposite sign
// of the eliminated matrix's -A_i^{-1}); since C Psi = I,
// Psi^T S Psi = Psi^T S~ Psi - W = A^{-1} - W.  Lower triangle read, full
// row-major block written.
template <typename TP>
__global__ void k_coarse_from_M(const KcDesc* __restrict__ d, const TP* __restrict__ P, const double* __restrict__ rho,
                                double* __restrict__ out) {
  const KcDesc c = d[blockIdx.y];
  const int nc = c.nc;
  const int64_t c0 = (int64_t)c.p_c0 * TS;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nc * nc; idx += gridDim.x * blockDim.x) {
    const int a = idx / nc, b = idx - a * nc;
    const int hi = a > b ? a : b, lo = a > b ? b : a;
    double v = (double)P[c.p_off + packed_offset(c0 + hi, c0 + lo, c.p_nt)];
    if (a == b) v -= rho[c.rho_off + a];
    out[c.out_off + idx] = v;
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_assemble(hipStream_t st, const int64_t* elems, int64_t n, const int32_t* el_local_ptr, const int32_t* el_local,
                     int nd, const int32_t* el_sub, const int64_t* sub_off, const int32_t* sub_nt, const double* Kref,
                     const double* scale, const int64_t* ekc_off, const double* ekc, T* A, const int32_t* tmap,
                     const int64_t* tmap_off, int32_t* err) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_assemble<T>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, elems, n, el_local_ptr, el_local, nd,
                     el_sub, sub_off, sub_nt, Kref, scale, ekc_off, ekc, A, tmap, tmap_off, err);
}

void launch_zero(hipStream_t st, void* p, size_t bytes, int max_blocks) {
  if (bytes == 0) return;
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, std::max(1, max_blocks));
  hipLaunchKernelGGL(k_zero16, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, (uint4*)p, n16);
}

template <typename T>
void launch_set_diag(hipStream_t st, const DiagSeg* segs, int64_t nseg, int32_t max_count, T* A, const int32_t* tmap,
                     const int64_t* tmap_off) {
  if (nseg <= 0 || max_count <= 0) return;
  unsigned gx = (unsigned)std::min<int64_t>((max_count + 255) / 256, 1024);
  hipLaunchKernelGGL(k_set_diag<T>, dim3(gx, (unsigned)nseg), dim3(256), 0, st, segs, A, tmap, tmap_off);
}

template <typename T>
void launch_factor_step(hipStream_t st, int kind, int k, const FactorArgs& a, int64_t first, int64_t count, T* A, T* Inv) {
  (void)k;  // the tasks carry their tile columns
  if (count <= 0) return;
  const uint64_t* tk = a.tasks + first;
  dim3 grid((unsigned)count), blk(256);
  auto mm = [&](bool panel) {
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, blk, 0, st, tk, a.off, a.nt, a.inv_off, A, Inv, a.tmap, a.tmap_off); };
    auto shape = [&](auto pnl, auto ks) {
      constexpr bool P = decltype(pnl)::value;
      constexpr int K = decltype(ks)::value;
      if constexpr (std::is_same<T, float>::value) {
        if (a.shape == 32) { go(k_tile_mm<T, P, K, 32>); return; }
        if (a.shape == SH_BF3) { go(k_tile_mm<T, P, (K < 32 ? 32 : K), SH_BF3>); return; }
      }
      go(k_tile_mm<T, P, K, 16>);
    };
    using PT = std::true_type;
    using PF = std::false_type;
    if (panel) {
      const int ps = a.pstage > 0 ? a.pstage : a.stage;
      if (ps == 16) shape(PT{}, std::integral_constant<int, 16>{});
      else if (ps == 64) shape(PT{}, std::integral_constant<int, 64>{});
      else shape(PT{}, std::integral_constant<int, 32>{});
    } else {
      if (a.stage == 16) shape(PF{}, std::integral_constant<int, 16>{});
      else if (a.stage == 64) shape(PF{}, std::integral_constant<int, 64>{});
      else shape(PF{}, std::integral_constant<int, 32>{});
    }
  };
  switch (kind) {
    case L_INPANEL: mm(false); break;
    case L_DIAG:
      hipLaunchKernelGGL(k_diag<T>, grid, blk, 0, st, tk, a.off, a.nt, a.inv_off, a.err, A, Inv, a.tmap, a.tmap_off);
      break;
    case L_PANEL: mm(true); break;
    case L_TRAIL: mm(false); break;
  }
}

template <typename TK, typename TP>
void launch_copy_block(hipStream_t st, const CopyDesc* d, int32_t nitems, int32_t max_blk, const TK* K, TP* P) {
  if (nitems <= 0 || max_blk <= 0) return;
  hipLaunchKernelGGL((k_copy_block<TK, TP>), dim3(max_blk, max_blk, nitems), dim3(256), 0, st, d, K, P);
}

template <typename TK, typename TP>
void launch_constraints(hipStream_t st, const ConsDesc* d, int64_t nrows, const int32_t* cols, const TK* K, TP* P,
                        double* rho) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL((k_constraints<TK, TP>), dim3((unsigned)nrows), dim3(256), 0, st, d, cols, K, P, rho);
}

template <typename TP>
void launch_coarse_matrix(hipStream_t st, const KcDesc* d, int32_t nitems, int32_t max_nc, const TP* P, const double* rho,
                          double* out) {
  if (nitems <= 0 || max_nc <= 0) return;
  unsigned gx = (unsigned)std::max(1, std::min(64, (max_nc * max_nc + 255) / 256));
  hipLaunchKernelGGL((k_coarse_from_M<TP>), dim3(gx, (unsigned)nitems), dim3(256), 0, st, d, P, rho, out);
}

#define INST_T(T)                                                                                                         \
  template void launch_assemble<T>(hipStream_t, const int64_t*, int64_t, const int32_t*, const int32_t*, int, const int32_t*, \
                                   const int64_t*, const int32_t*, const double*, const double*, const int64_t*,        \
                                   const double*, T*, const int32_t*, const int64_t*, int32_t*);                        \
  template void launch_set_diag<T>(hipStream_t, const DiagSeg*, int64_t, int32_t, T*, const int32_t*, const int64_t*); \
  template void launch_factor_step<T>(hipStream_t, int, int, const FactorArgs&, int64_t, int64_t, T*, T*);             \

INST_T(double)
INST_T(float)
#undef INST_T
#define INST_KP(TK, TP)                                                                                              \
  template void launch_copy_block<TK, TP>(hipStream_t, const CopyDesc*, int32_t, int32_t, const TK*, TP*);          \
  template void launch_constraints<TK, TP>(hipStream_t, const ConsDesc*, int64_t, const int32_t*, const TK*, TP*,   \
                                           double*);
INST_KP(double, double)
INST_KP(double, float)
INST_KP(float, float)
#undef INST_KP
template void launch_coarse_matrix<double>(hipStream_t, const KcDesc*, int32_t, int32_t, const double*, const double*,
                                           double*);
template void launch_coarse_matrix<float>(hipStream_t, const KcDesc*, int32_t, int32_t, const float*, const double*, double*);

}  // namespace mlbddc
