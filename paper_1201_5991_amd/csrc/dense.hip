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
  for (int idx = threadIdx.x; idx < TE; idx += blockDim.x) {
    int i = idx & (TS - 1), j = idx >> 6;
    T v = (T)g[idx];
    if (trans) s[i * LDT + j] = v; else s[j * LDT + i] = v;
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
template <typename T>
__global__ void __launch_bounds__(256) k_assemble(const int64_t* __restrict__ elems, const int32_t* __restrict__ el_local_ptr,
                                                  const int32_t* __restrict__ el_local, const int32_t* __restrict__ el_sub,
                                                  const int64_t* __restrict__ sub_off, const int32_t* __restrict__ sub_nt,
                                                  const double* __restrict__ Kref, const double* __restrict__ scale,
                                                  const int64_t* __restrict__ ekc_off, const double* __restrict__ ekc, T* A) {
  const int64_t e = elems[blockIdx.x];
  const int b = el_sub[e];
  const int32_t base = el_local_ptr[e];
  const int nloc = el_local_ptr[e + 1] - base;
  const int64_t off = sub_off[b];
  const int nt = sub_nt[b];
  const double sc = Kref ? scale[e] : 1.0;
  const double* M = Kref ? Kref : ekc + ekc_off[e];
  for (int idx = threadIdx.x; idx < nloc * nloc; idx += blockDim.x) {
    int a = idx / nloc, c = idx - a * nloc;
    int p = el_local[base + a], q = el_local[base + c];
    if (p < 0 || q < 0 || p / TS < q / TS) continue;
    A[off + packed_offset(p, q, nt)] += (T)(sc * M[idx]);
  }
}

template <typename T>
__global__ void k_set_diag(const DiagSeg* __restrict__ segs, T* A) {
  const DiagSeg s = segs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.count; i += gridDim.x * blockDim.x)
    A[s.off + packed_offset(s.row0 + i, s.col0 + i, s.nt)] = (T)s.val;
}

// ------------------------------------------------------------ factorization
// Exchange within groups of four lanes through DPP (quad permutations).
template <int CTRL>
__device__ inline double quad_perm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ inline float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int DPP_XOR1 = 0xB1;  // quad_perm(1, 0, 3, 2)
constexpr int DPP_XOR2 = 0x4E;  // quad_perm(2, 3, 0, 1)

// Diagonal tile: Cholesky factor and inverse of the lower factor.
// Factor: wavefront 0, lane i keeps row i in registers; per column j the pivot
// and then the new column of L are broadcast through LDS (reads issued
// unconditionally, so they pipeline), and the right-looking update touches
// registers only.  Entries right of a lane's diagonal are left as they are
// and ignored.  Inverse W = L^{-1}: four neighbouring lanes own column c of W
// (lane p keeps W(p+4m, c)); W(r, c) = (delta_rc - sum_{q<r} L(r, q) W(q, c)) /
// L(r, r).  Entries of W not yet computed are zero, so the sum runs over all
// of the lane's entries without predicates; the four partial sums are combined
// with DPP quad permutations.
template <typename T>
__global__ void __launch_bounds__(256) k_diag(const uint64_t* __restrict__ tasks, const int64_t* __restrict__ off,
                                              const int32_t* __restrict__ ntv, const int64_t* __restrict__ inv_off,
                                              int32_t* err, T* A, T* Inv) {
  __shared__ T sA[TS * LDT];
  __shared__ T dinv[TS];
  const uint64_t t = tasks[blockIdx.x];
  const int item = task_item(t), k = task_r(t);
  const int nt = ntv[item];
  T* g = A + off[item] + tile_index(k, k, nt) * TE;
  const int tid = threadIdx.x;
  // factor in LDS: per column one pivot/scale pass (wavefront 0) and one
  // branch-free rank-1 update (each thread owns 16 entries of the tile)
  stage_tile<T, T>(sA, g, false);
  __syncthreads();
  bool bad = false;
  int badcol = 0;
  {
    const int i = tid & (TS - 1), l0 = tid >> 6;
    for (int j = 0; j < TS; ++j) {
      if (tid < TS) {
        T d = sA[j * LDT + j];
        if (!(d > (T)0)) {
          if (!bad) badcol = j;
          bad = true;
          d = (T)NAN;
        }
        const T sq = sqrt(d);
        const T v = sA[j * LDT + tid];
        __builtin_amdgcn_wave_barrier();
        sA[j * LDT + tid] = tid > j ? v / sq : (tid == j ? sq : v);
      }
      __syncthreads();
      const T lij = sA[j * LDT + i];
      T lj[16], cur[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        lj[m] = sA[j * LDT + l0 + 4 * m];
        cur[m] = sA[(l0 + 4 * m) * LDT + i];
      }
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int l = l0 + 4 * m;
        sA[l * LDT + i] = (l > j && i >= l) ? cur[m] - lij * lj[m] : cur[m];
      }
      __syncthreads();
    }
  }
  if (bad && tid == 0 && atomicCAS(&err[0], 0, item + 1) == 0) err[1] = k * TS + badcol;
  for (int idx = tid; idx < TE; idx += blockDim.x) {
    const int r = idx & (TS - 1), cc = idx >> 6;
    if (r < cc) sA[cc * LDT + r] = (T)0;
  }
  __syncthreads();
  for (int idx = tid; idx < TE; idx += blockDim.x) g[idx] = sA[(idx >> 6) * LDT + (idx & (TS - 1))];
  if (tid < TS) dinv[tid] = (T)1 / sA[tid * LDT + tid];
  __syncthreads();
  // inverse
  const int c = tid >> 2, p = tid & 3;
  T w[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) w[m] = (T)0;
  for (int r = 0; r < TS; ++r) {
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int m = 0; m < 16; m += 2) {
      s0 += sA[(p + 4 * m) * LDT + r] * w[m];
      s1 += sA[(p + 4 * m + 4) * LDT + r] * w[m + 1];
    }
    T s = s0 + s1;
    s += quad_perm<DPP_XOR1>(s);
    s += quad_perm<DPP_XOR2>(s);
    const T v = ((r == c ? (T)1 : (T)0) - s) * dinv[r];
#pragma unroll
    for (int m = 0; m < 16; ++m)
      if (p + 4 * m == r) w[m] = v;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 16; ++m) sA[c * LDT + p + 4 * m] = w[m];
  __syncthreads();
  T* gi = Inv + inv_off[item] + (int64_t)k * TE;
  for (int idx = tid; idx < TE; idx += blockDim.x) gi[idx] = sA[(idx >> 6) * LDT + (idx & (TS - 1))];
}

template <typename T>
__global__ void __launch_bounds__(256) k_panel(const uint64_t* __restrict__ tasks, const int64_t* __restrict__ off,
                                               const int32_t* __restrict__ ntv, const int64_t* __restrict__ inv_off, T* A,
                                               const T* __restrict__ Inv) {
  __shared__ T sR[TS * LDT];
  __shared__ T sS[TS * LDT];
  const uint64_t t = tasks[blockIdx.x];
  const int item = task_item(t), r = task_r(t), k = task_s(t);
  const int nt = ntv[item];
  T* g = A + off[item] + tile_index(r, k, nt) * TE;
  stage_tile<T, T>(sR, g, false);
  stage_tile<T, T>(sS, Inv + inv_off[item] + (int64_t)k * TE, false);
  __syncthreads();
  typename Mfma<T>::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::zero();
  tile_nt<T>(acc, sR, sS);
  for_acc<T>(acc, [&](int i, int j, T v) { g[j * TS + i] = v; });
}

// Register staging of one 64x64 tile: each of the 256 threads holds 16
// elements as 16-byte vectors (coalesced loads), then stores them to LDS.
template <typename T>
struct TileRegs {
  static constexpr int V = 16 / sizeof(T);          // elements per 16-byte vector
  static constexpr int N = TE / (256 * V);          // vectors per thread
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

// acc(i, j) += sum_k R(i, k) S(j, k) from LDS tiles with leading dimension LD.
template <typename T, int LD>
__device__ inline void tile_nt_ld(typename Mfma<T>::acc_t (&acc)[2][2], const T* __restrict__ sR, const T* __restrict__ sS) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < TS; k0 += 4) {
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

// A_rs <- A_rs - sum_{kk=kf..klast} A_{r,kk} A_{s,kk}^T.  The output tile is
// prefetched into registers at the start; the next pair of k-tiles is loaded
// into registers while the current pair is multiplied from LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_update(const uint64_t* __restrict__ tasks, const int64_t* __restrict__ off,
                                                const int32_t* __restrict__ ntv, int klast, T* A) {
  __shared__ T sR[TS * LDU];
  __shared__ T sS[TS * LDU];
  const uint64_t t = tasks[blockIdx.x];
  const int item = task_item(t), r = task_r(t), s = task_s(t), kf = task_kf(t);
  const int nt = ntv[item];
  T* base = A + off[item];
  T* g = base + tile_index(r, s, nt) * TE;
  T creg[16];
  {
    int n = 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int iw = (w & 1) * 32, jw = (w >> 1) * 32;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = iw + bi * 16 + (lane & 15), j = jw + bj * 16 + Mfma<T>::row(lane >> 4, v);
          creg[n++] = g[j * TS + i];
        }
  }
  typename Mfma<T>::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::zero();
  TileRegs<T> pr, ps;
  const bool diag = r == s;
  pr.load(base + tile_index(r, kf, nt) * TE);
  if (!diag) ps.load(base + tile_index(s, kf, nt) * TE);
  for (int kk = kf; kk <= klast; ++kk) {
    pr.template store<LDU>(sR);
    if (!diag) ps.template store<LDU>(sS);
    __syncthreads();
    if (kk < klast) {
      pr.load(base + tile_index(r, kk + 1, nt) * TE);
      if (!diag) ps.load(base + tile_index(s, kk + 1, nt) * TE);
    }
    tile_nt_ld<T, LDU>(acc, sR, diag ? sR : sS);
    __syncthreads();
  }
  int n = 0;
  for_acc<T>(acc, [&](int i, int j, T v) { g[j * TS + i] = creg[n++] - v; });
}

template <typename T>
__global__ void __launch_bounds__(256) k_negate(const uint64_t* __restrict__ tasks, const int64_t* __restrict__ off,
                                                const int32_t* __restrict__ ntv, T* A) {
  const uint64_t t = tasks[blockIdx.x];
  const int item = task_item(t), r = task_r(t), s = task_s(t);
  T* g = A + off[item] + tile_index(r, s, ntv[item]) * TE;
  for (int idx = threadIdx.x; idx < TE; idx += blockDim.x) g[idx] = -g[idx];
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
                                                     const TK* __restrict__ K, TP* P) {
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

// T_{i,c} = sum_s S_{i,s} Psi_{s,c}: S from the FP64 K matrix (symmetric,
// lower tiles), Psi^T tile (c, s) from the preconditioner matrix.
template <typename TK, typename TP>
__global__ void __launch_bounds__(256) k_kc_stage1(const KcDesc* __restrict__ d, const TK* __restrict__ K,
                                                   const TP* __restrict__ P, double* Tscr) {
  __shared__ double sR[TS * LDT];
  __shared__ double sS[TS * LDT];
  const KcDesc c = d[blockIdx.z];
  const int i = blockIdx.x, cc = blockIdx.y;
  if (i >= c.ntg || cc >= c.ntc) return;
  typename Mfma<double>::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<double>::zero();
  for (int s = 0; s < c.ntg; ++s) {
    if (i >= s) stage_tile<double, TK>(sR, K + c.k_off + tile_index(c.k_g0 + i, c.k_g0 + s, c.k_nt) * TE, false);
    else stage_tile<double, TK>(sR, K + c.k_off + tile_index(c.k_g0 + s, c.k_g0 + i, c.k_nt) * TE, true);
    stage_tile<double, TP>(sS, P + c.p_off + tile_index(c.p_c0 + cc, c.p_d0 + s, c.p_nt) * TE, false);
    __syncthreads();
    tile_nt<double>(acc, sR, sS);
    __syncthreads();
  }
  double* g = Tscr + c.t_off + ((int64_t)cc * c.ntg + i) * TE;
  for_acc<double>(acc, [&](int a, int b, double v) { g[b * TS + a] = v; });
}

// KC_{c1,c2} = sum_s Psi^T_{c1,s} T_{s,c2}
template <typename TP>
__global__ void __launch_bounds__(256) k_kc_stage2(const KcDesc* __restrict__ d, const TP* __restrict__ P,
                                                   const double* __restrict__ Tscr, double* KC) {
  __shared__ double sR[TS * LDT];
  __shared__ double sS[TS * LDT];
  const KcDesc c = d[blockIdx.z];
  const int c1 = blockIdx.x, c2 = blockIdx.y;
  if (c1 >= c.ntc || c2 >= c.ntc) return;
  typename Mfma<double>::acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<double>::zero();
  for (int s = 0; s < c.ntg; ++s) {
    stage_tile<double, TP>(sR, P + c.p_off + tile_index(c.p_c0 + c1, c.p_d0 + s, c.p_nt) * TE, false);
    stage_tile<double, double>(sS, Tscr + c.t_off + ((int64_t)c2 * c.ntg + s) * TE, true);
    __syncthreads();
    tile_nt<double>(acc, sR, sS);
    __syncthreads();
  }
  double* g = KC + c.kc_off + ((int64_t)c2 * c.ntc + c1) * TE;
  for_acc<double>(acc, [&](int a, int b, double v) { g[b * TS + a] = v; });
}

__global__ void k_compact_kc(const int64_t* __restrict__ kc_off, const int32_t* __restrict__ ntc, const int32_t* __restrict__ ncv,
                             const int64_t* __restrict__ out_off, const double* __restrict__ KC, double* out) {
  const int item = blockIdx.y;
  const int nc = ncv[item], nt = ntc[item];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nc * nc; idx += gridDim.x * blockDim.x) {
    int a = idx / nc, b = idx - a * nc;  // row-major output (a, b)
    int64_t tile = (int64_t)(b / TS) * nt + a / TS;
    double v1 = KC[kc_off[item] + tile * TE + (b % TS) * TS + (a % TS)];
    int64_t tile2 = (int64_t)(a / TS) * nt + b / TS;
    double v2 = KC[kc_off[item] + tile2 * TE + (a % TS) * TS + (b % TS)];
    out[out_off[item] + idx] = 0.5 * (v1 + v2);  // symmetrize rounding
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_assemble(hipStream_t st, const int64_t* elems, int64_t n, const int32_t* el_local_ptr, const int32_t* el_local,
                     const int32_t* el_sub, const int64_t* sub_off, const int32_t* sub_nt, const double* Kref,
                     const double* scale, const int64_t* ekc_off, const double* ekc, T* A) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_assemble<T>, dim3((unsigned)n), dim3(256), 0, st, elems, el_local_ptr, el_local, el_sub, sub_off,
                     sub_nt, Kref, scale, ekc_off, ekc, A);
}

template <typename T>
void launch_set_diag(hipStream_t st, const DiagSeg* segs, int64_t nseg, int32_t max_count, T* A) {
  if (nseg <= 0 || max_count <= 0) return;
  unsigned gx = (unsigned)std::min<int64_t>((max_count + 255) / 256, 1024);
  hipLaunchKernelGGL(k_set_diag<T>, dim3(gx, (unsigned)nseg), dim3(256), 0, st, segs, A);
}

template <typename T>
void launch_factor_step(hipStream_t st, int kind, int k, const FactorArgs& a, int64_t first, int64_t count, T* A, T* Inv) {
  if (count <= 0) return;
  const uint64_t* tk = a.tasks + first;
  dim3 grid((unsigned)count), blk(256);
  switch (kind) {
    case L_NEGATE: hipLaunchKernelGGL(k_negate<T>, grid, blk, 0, st, tk, a.off, a.nt, A); break;
    case L_INPANEL: hipLaunchKernelGGL(k_update<T>, grid, blk, 0, st, tk, a.off, a.nt, k - 1, A); break;
    case L_DIAG: hipLaunchKernelGGL(k_diag<T>, grid, blk, 0, st, tk, a.off, a.nt, a.inv_off, a.err, A, Inv); break;
    case L_PANEL: hipLaunchKernelGGL(k_panel<T>, grid, blk, 0, st, tk, a.off, a.nt, a.inv_off, A, Inv); break;
    case L_TRAIL: hipLaunchKernelGGL(k_update<T>, grid, blk, 0, st, tk, a.off, a.nt, k, A); break;
  }
}

template <typename TK, typename TP>
void launch_copy_block(hipStream_t st, const CopyDesc* d, int32_t nitems, int32_t max_blk, const TK* K, TP* P) {
  if (nitems <= 0 || max_blk <= 0) return;
  hipLaunchKernelGGL((k_copy_block<TK, TP>), dim3(max_blk, max_blk, nitems), dim3(256), 0, st, d, K, P);
}

template <typename TK, typename TP>
void launch_constraints(hipStream_t st, const ConsDesc* d, int64_t nrows, const int32_t* cols, const TK* K, TP* P) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL((k_constraints<TK, TP>), dim3((unsigned)nrows), dim3(256), 0, st, d, cols, K, P);
}

template <typename TK, typename TP>
void launch_coarse_matrix(hipStream_t st, const KcDesc* d, int32_t nitems, int32_t max_ntg, int32_t max_ntc, const TK* K,
                          const TP* P, double* Tscr, double* KC) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL((k_kc_stage1<TK, TP>), dim3(max_ntg, max_ntc, nitems), dim3(256), 0, st, d, K, P, Tscr);
  hipLaunchKernelGGL(k_kc_stage2<TP>, dim3(max_ntc, max_ntc, nitems), dim3(256), 0, st, d, P, Tscr, KC);
}

void launch_compact_kc(hipStream_t st, const int64_t* kc_off, const int32_t* ntc, const int32_t* nc, const int64_t* out_off,
                       int32_t nitems, int32_t max_nc, const double* KC, double* out) {
  if (nitems <= 0) return;
  unsigned gx = (unsigned)std::max(1, std::min(64, (max_nc * max_nc + 255) / 256));
  hipLaunchKernelGGL(k_compact_kc, dim3(gx, nitems), dim3(256), 0, st, kc_off, ntc, nc, out_off, KC, out);
}

#define INST_T(T)                                                                                                         \
  template void launch_assemble<T>(hipStream_t, const int64_t*, int64_t, const int32_t*, const int32_t*, const int32_t*, \
                                   const int64_t*, const int32_t*, const double*, const double*, const int64_t*,        \
                                   const double*, T*);                                                                  \
  template void launch_set_diag<T>(hipStream_t, const DiagSeg*, int64_t, int32_t, T*);                                 \
  template void launch_factor_step<T>(hipStream_t, int, int, const FactorArgs&, int64_t, int64_t, T*, T*);             \

INST_T(double)
INST_T(float)
#undef INST_T
#define INST_KP(TK, TP)                                                                                              \
  template void launch_copy_block<TK, TP>(hipStream_t, const CopyDesc*, int32_t, int32_t, const TK*, TP*);          \
  template void launch_constraints<TK, TP>(hipStream_t, const ConsDesc*, int64_t, const int32_t*, const TK*, TP*);  \
  template void launch_coarse_matrix<TK, TP>(hipStream_t, const KcDesc*, int32_t, int32_t, int32_t, const TK*,      \
                                             const TP*, double*, double*);
INST_KP(double, double)
INST_KP(double, float)
INST_KP(float, float)
#undef INST_KP

}  // namespace mlbddc
