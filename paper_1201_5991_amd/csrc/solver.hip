// Orchestration of the multilevel BDDC-PCG on one gfx950 device and the C ABI.
//
// Set-up (Algorithm 1), per level l = 1..L-1 and the top coarse level:
//   K job  : assemble the subdomain matrices K_i (tile-packed), partially
//            factorize them (interior block eliminated).  Level 1 keeps the
//            interface Schur complement S_i = K_GG - K_GI K_II^{-1} K_IG in the
//            trailing tiles.  Levels >= 2 and the top level carry an identity
//            block, so the trailing tiles also hold -K_II^{-1} K_IG and
//            -K_II^{-1} (the interior pre-/post-correction operators; at the
//            top level simply -K_C^{-1}).
//   M job  : for every subdomain the augmented matrix
//              [ S+C^T W C   C^T   I    0  ]
//              [ C           0     0    I  ]
//              [ I           0     0    0  ]
//              [ 0           I     0    0  ]
//            is eliminated in two phases (the second factors the negative of
//            the first phase's trailing block, reading it with the opposite
//            sign, so the blocks it leaves hold -G_i, -Psi_i and A^{-1}).  The result holds G_i = S~^{-1} - S~^{-1}C^T A^{-1} C S~^{-1}
//            (A = C S~^{-1} C^T), the operator of the constrained local problem
//            of Eq. (2) restricted to the interface, and Psi_i^T, the coarse basis
//            of Eq. (1); the penalty W (rho = sum of the glob's diagonal entries
//            of S) makes S~ definite on floating subdomains and does not change
//            the solution.
//   K_Ci = Psi_i^T S_i Psi_i (= -Lambda_i), assembled as the elements of the next level.
// Apply (Algorithm 2), level l interface vector r^:
//   r_i = D_i R_i r^;  r_C = sum R_Ci^T Psi_i^T r_i;  z_C from the next level
//   (interior pre-correction, BDDC, post-correction) or the top solve;
//   z^ = sum R_i^T D_i (G_i r_i + Psi_i R_Ci z_C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <array>
#include <atomic>
#include <fstream>
#include <future>
#include <map>
#include <sstream>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace mlbddc {

// Device scratch of the entry point that allocates nothing
// (mlbddc_apply_schur_noalloc): the gathered input and the product output of
// the interface operator, 2 * 8 bytes per flat interface entry.  Every device
// the library runs on holds it until the process ends.  In host code the
// array's name is not a device address: the address comes from
// hipGetSymbolAddress, once per device (scratch_address).
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Address of `scratch` on `device` (that device current), looked up once.
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define HIPCHK(x)                                                                                  \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess) return herr(#x, e_);                                                     \
  } while (0)

// A batch of tile-packed matrices factorized together.
struct Job {
  bool fp32 = false;
  void* buf = nullptr;
  void* inv = nullptr;
  int64_t elems = 0, inv_elems = 0;
  std::vector<int64_t> off, inv_off;
  std::vector<int32_t> nt;
  std::vector<FactorItemDesc> items;
  std::vector<std::vector<int32_t>> env;
  FactorSchedule sched;
  int64_t* d_off = nullptr;
  int64_t* d_inv_off = nullptr;
  int32_t* d_nt = nullptr;
  uint64_t* d_tasks = nullptr;
  int32_t* d_err = nullptr;
  int panel = 4;
  int stage = 32;  // staged columns of the tile products
  int pstage = 0;  // staged columns of the panel products (0: stage)
  // Tile maps (tile_slot): a matrix with a tile structure stores only the
  // tiles some kernel reads; tmap_off[i] = -1 for a dense packed-lower one.
  // A mapped matrix keeps its eliminated columns at off[i] (nlead[i] tiles)
  // and its trailing (interface) block, packed like a matrix of its own, in
  // one region after every matrix's leading part, from slot tslot0[i] on:
  // the trailing blocks of the job lie back to back.
  std::vector<int32_t> tmap;
  std::vector<int64_t> tmap_off;
  std::vector<int64_t> nlead;   // tiles stored at off[i] (every tile of a dense matrix)
  std::vector<int64_t> tslot0;  // first slot of the trailing block (mapped matrices), else -1
  int32_t* d_tmap = nullptr;
  int64_t* d_tmap_off = nullptr;
  int64_t slot(size_t i, int r, int s) const {
    return tile_slot(tmap.empty() ? nullptr : tmap.data(), tmap_off.data(), (int)i, r, s, nt[i]);
  }
  // The trailing block of matrix i from tile t0 on (its interface block;
  // t0 = e1 for a mapped matrix) as a tile-packed matrix: element offset,
  // tiles per side, first tile.
  void trailing(size_t i, int t0, int64_t& o, int32_t& n, int32_t& f) const {
    if (tmap_off[i] >= 0) {
      o = off[i] + tslot0[i] * TE;
      n = nt[i] - t0;
      f = 0;
    } else {
      o = off[i];
      n = nt[i];
      f = t0;
    }
  }
};

// A batched tile-block matrix-vector product.
struct MvSet {
  int mode = MV_SYM;
  std::vector<MvDesc> h;
  MvDesc* d = nullptr;
  int64_t* d_prefix = nullptr;
  int64_t* d_prefix2 = nullptr;  // workgroups per item with two tiles per workgroup
  int64_t tiles = 0, groups2 = 0;
  int32_t max_out = 0;
  int64_t partial_elems = 0;
};

struct LevelDev {
  LevelPlan* P = nullptr;
  bool kfp32 = false, mfp32 = false;
  Job K, M;
  // flat local layouts
  int64_t nG_flat = 0, nI_flat = 0, nC_flat = 0;
  std::vector<int64_t> gofs, iofs, cofs;
  int32_t* d_gidx = nullptr;      // flat interface position -> level interface index (-1 pad)
  int32_t* d_iidx = nullptr;      // flat interior position -> level DOF (-1 pad)
  int32_t* d_cidx = nullptr;      // flat coarse position -> level coarse DOF (-1 pad)
  int32_t* d_iface_dofs = nullptr;// level interface index -> level DOF
  int64_t* d_gptr = nullptr;  int64_t* d_glist = nullptr;   // interface DOF -> flat positions
  int64_t* d_cptr = nullptr;  int64_t* d_clist = nullptr;   // coarse DOF -> flat positions
  double* d_w = nullptr;          // weights D_i (flat interface)
  int64_t* d_gdiag_pos = nullptr; // element offsets of the interface diagonal of K (for weights)
  // work vectors
  void* rl = nullptr;   // flat interface, M precision
  void* yl = nullptr;   // flat interface, M precision
  void* yl2 = nullptr;  // flat interface, M precision: Psi_i z_Ci when the G product runs beside the coarse levels
  void* zcl = nullptr;  // flat coarse, M precision
  double* rcl = nullptr;// flat coarse, FP64
  double* rC = nullptr; // level coarse vector (next level's DOFs)
  double* zC = nullptr;
  double* rhat = nullptr; // level interface vector (levels >= 2)
  double* zhat = nullptr;
  void* rI = nullptr;   // flat interior, K precision
  void* uI = nullptr;
  void* zG = nullptr;   // flat interface, K precision (post-correction input)
  double* tG = nullptr; // flat interface FP64
  double* gd = nullptr; // flat interface FP64 work (weights, S^ product)
  double* gd2 = nullptr;
  double* wI = nullptr; // flat interior FP64 (level 1 condensation)
  void* partial = nullptr;
  void* partial_g = nullptr;  // partial sums of the G product when it runs beside the coarse correction
  // tile mat-vec sets
  MvSet mvS, mvG, mvPsiN, mvPsiT, mvPre, mvPreT, mvPostN;
  bool g_psi_sum = false;  // y = G r + Psi z_C as one launch (both products small, items aligned)
  // triangular solves: items sorted by dissection height (trsv_lvl[h] = first
  // item of height h, last entry = item count) and the tile lists
  std::vector<TrsvDesc> trsv_h;
  std::vector<int32_t> trsv_lvl;
  std::vector<int32_t> tr_rptr, tr_rcol, tr_cptr, tr_crow;
  std::vector<int32_t> tr_rslot, tr_cslot;  // storage slot of each listed tile
  TrsvDesc* d_trsv = nullptr;
  int32_t *d_tr_rptr = nullptr, *d_tr_rcol = nullptr, *d_tr_cptr = nullptr, *d_tr_crow = nullptr;
  int32_t *d_tr_rslot = nullptr, *d_tr_cslot = nullptr;
  // tile-list products over nonzero tiles of the level-1 factor: L_GI and
  // L_GI^T (condensation, recovery) and, per dissection height, the coupling of
  // a height's groups to lower groups (forward) or higher groups (backward)
  struct TileList {
    std::vector<TileRef> t;
    std::vector<OutRef> o;
    TileRef* dt = nullptr;
    OutRef* dout = nullptr;
  };
  TileList lgiN, lgiT;
  std::vector<TileList> trF, trB;
  double* tl_partial = nullptr;
  // coarse matrices of this level (inputs of the next level's assembly)
  double* kc_compact = nullptr;
  std::vector<int64_t> kc_off;
  int64_t* d_kc_off = nullptr;
  std::vector<KcDesc> kcd_h;
  KcDesc* d_kcd = nullptr;
  int32_t max_nc = 0;
  double* d_rho = nullptr;  // constraint penalties rho_c, one per constraint row
  std::vector<CopyDesc> copy_h;
  CopyDesc* d_copy = nullptr;
  int32_t copy_max = 0;
  std::vector<ConsDesc> cons_h;
  ConsDesc* d_cons = nullptr;
  int32_t* d_ccols = nullptr;
  std::vector<int32_t> ccols_h;
  std::vector<DiagSeg> ksegs_h, msegs_h;
  DiagSeg* d_ksegs = nullptr;
  DiagSeg* d_msegs = nullptr;
  int32_t kseg_max = 0, mseg_max = 0;
  // assembly
  int64_t* d_sub_off = nullptr;
  int32_t* d_sub_nt = nullptr;
  int64_t* d_elems_by_color = nullptr;
  std::vector<int64_t> color_ptr;
  int32_t* d_el_local_ptr = nullptr;
  int32_t* d_el_local = nullptr;
  int32_t* d_el_sub = nullptr;
  int64_t* d_ekc_off = nullptr;   // element -> offset of its matrix in the previous level's kc_compact
};

}  // namespace

struct Handle {
  mlbddc_options opt{};
  hipStream_t stream = nullptr;
  Error err;
  Plan plan;
  bool planned = false, ready = false;
  std::vector<std::pair<void*, size_t>> allocs;
  std::multimap<size_t, void*> pool;
  std::vector<LevelDev> lev;
  // mesh data kept for updates and element energies
  int32_t nloc1 = 0;
  int64_t n_elems = 0;
  double* d_Kref = nullptr;
  double* d_scale = nullptr;
  int32_t* d_edof = nullptr;       // element DOF -> free DOF (-1 fixed)
  hipEvent_t ev_edof = nullptr;     // its upload (on the upload stream) done
  // PCG state
  double *d_x = nullptr, *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr, *d_g = nullptr;
  double* d_s = nullptr;           // scalars
  double* d_hist = nullptr;        // alpha/beta history
  double* d_dotp = nullptr;
  double* h_s = nullptr;           // pinned mirror of the scalars, then two per-iteration snapshots
  int32_t* h_err = nullptr;        // pinned error words of the factorization jobs
  size_t h_err_cap = 0;
  hipEvent_t ev_snap[2] = {nullptr, nullptr};
  int32_t* d_it = nullptr;         // device iteration counter
  // HIP graph of one PCG iteration (captured on an internal stream)
  hipStream_t cap = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  // second stream for the look-ahead factorization schedule
  hipStream_t fstream = nullptr;
  // stream of the level-0 G product, which runs beside the coarse correction
  hipStream_t gstream = nullptr;
  hipEvent_t ev_gfork = nullptr, ev_gjoin = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  int32_t max_hist = 0;
  double t_plan = 0, t_setup = 0;
  double flops_K = 0, flops_M = 0;
  // profiling
  bool prof = false;
  bool verbose = false;  // MLBDDC_VERBOSE set: set-up phase times on stderr
  mlbddc_profile pdata{};
  int panel_nt[2] = {0, 0};  // largest matrix (tiles per side) of each job kind in this set-up
  std::vector<hipEvent_t> events;

  std::mutex err_mu;  // set-up threads (checks, queueing) may fail together
  mlbddc_status herr(const char* what, hipError_t e) {
    std::lock_guard<std::mutex> g(err_mu);
    err.status = MLBDDC_E_HIP;
    err.message = std::string(what) + ": " + hipGetErrorString(e);
    return err.status;
  }
  mlbddc_status fail(mlbddc_status st, const std::string& m, int level = 0, int sub = -1, int col = -1) {
    std::lock_guard<std::mutex> g(err_mu);
    err.status = st;
    err.message = m;
    err.level = level;
    err.subdomain = sub;
    err.column = col;
    return st;
  }
  // Device memory comes from the caller's allocator when one was given to
  // mlbddc_create (e.g. a framework's caching allocator), else from hipMalloc.
  mlbddc_allocator ext_alloc{};
  bool has_ext_alloc = false;
  void* raw_alloc(size_t bytes) {
    if (has_ext_alloc) {
      void* q = ext_alloc.alloc(bytes, ext_alloc.ctx);
      if ((uintptr_t)q & 255) {  // the kernels assume 256-byte alignment
        ext_alloc.free(q, ext_alloc.ctx);
        return nullptr;
      }
      return q;
    }
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return q;
  }
  void raw_free(void* q) {
    if (!q) return;
    if (has_ext_alloc) ext_alloc.free(q, ext_alloc.ctx);
    else (void)hipFree(q);
  }
  template <typename T>
  mlbddc_status dalloc(T** p, int64_t n) {
    *p = nullptr;
    if (n <= 0) return MLBDDC_OK;
    const size_t bytes = (size_t)round_up((int64_t)(sizeof(T) * (size_t)n), 256);
    void* q = nullptr;
    auto it = pool.find(bytes);
    if (it != pool.end()) {  // reuse a block of the previous set-up
      q = it->second;
      pool.erase(it);
    } else {
      q = raw_alloc(bytes);
      if (!q) {
        trim_pool();  // retry once without the previous set-up's blocks
        q = raw_alloc(bytes);
        if (!q) return fail(MLBDDC_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
      }
    }
    allocs.push_back({q, bytes});
    *p = (T*)q;
    return MLBDDC_OK;
  }
  // Pool blocks are never in use by queued work: set-up moves the previous
  // set-up's blocks to the pool only after synchronizing the library stream,
  // and every other library stream joins that stream before its work ends.
  void trim_pool() {
    for (auto& kv : pool) raw_free(kv.second);
    pool.clear();
  }
  // Host-to-device copies of set-up data: staged in pinned host memory kept
  // by the handle (chunks reused by every set-up) and copied asynchronously on
  // their own stream, so that the host goes on preparing while the device
  // factorizes the parts already prepared.  upload_fence() orders the
  // library stream after every copy issued so far.
  hipStream_t ustream = nullptr;
  hipEvent_t ev_upl = nullptr;
  std::vector<std::pair<char*, size_t>> staging;  // pinned chunks
  size_t stage_chunk = 0, stage_used = 0;
  mlbddc_status stage_reset() {
    if (ustream) HIPCHK(hipStreamSynchronize(ustream));
    stage_chunk = 0;
    stage_used = 0;
    return MLBDDC_OK;
  }
  mlbddc_status stage(size_t bytes, char** out) {
    bytes = (bytes + 255) / 256 * 256;
    while (stage_chunk < staging.size() && stage_used + bytes > staging[stage_chunk].second) {
      ++stage_chunk;
      stage_used = 0;
    }
    if (stage_chunk == staging.size()) {
      const size_t cap = std::max<size_t>(bytes, (size_t)16 << 20);
      char* q = nullptr;
      HIPCHK(hipHostMalloc((void**)&q, cap, hipHostMallocDefault));
      staging.push_back({q, cap});
      stage_used = 0;
    }
    *out = staging[stage_chunk].first + stage_used;
    stage_used += bytes;
    return MLBDDC_OK;
  }
  mlbddc_status ensure_ustream() {
    if (!ustream) {
      HIPCHK(hipStreamCreateWithFlags(&ustream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&ev_upl, hipEventDisableTiming));
    }
    return MLBDDC_OK;
  }
  template <typename T, typename A>
  mlbddc_status upload(T** p, const std::vector<T, A>& v) {
    mlbddc_status st = dalloc(p, (int64_t)v.size());
    if (st) return st;
    if (!v.empty()) {
      if ((st = ensure_ustream())) return st;
      char* h = nullptr;
      const size_t bytes = sizeof(T) * v.size();
      if ((st = stage(bytes, &h))) return st;
      // large arrays (task lists of several MB) are staged by several threads
      const int nth = (int)std::min<size_t>(8, bytes >> 20);
      const char* src = reinterpret_cast<const char*>(v.data());
      if (nth > 1)
        parallel_run(nth, [&](int t) {
          const size_t b0 = bytes * t / nth, b1 = bytes * (t + 1) / nth;
          std::memcpy(h + b0, src + b0, b1 - b0);
        });
      else
        std::memcpy(h, src, bytes);
      HIPCHK(hipMemcpyAsync(*p, h, bytes, hipMemcpyHostToDevice, ustream));
    }
    return MLBDDC_OK;
  }
  // Like upload, for an array that fill(dst) writes straight into the pinned
  // staging memory (no host copy of it is kept)
  template <typename T, typename F>
  mlbddc_status upload_fill(T** p, int64_t n, F&& fill) {
    mlbddc_status st = dalloc(p, n);
    if (st || n <= 0) return st;
    if ((st = ensure_ustream())) return st;
    char* h = nullptr;
    const size_t bytes = sizeof(T) * (size_t)n;
    if ((st = stage(bytes, &h))) return st;
    if ((st = fill(reinterpret_cast<T*>(h)))) return st;
    HIPCHK(hipMemcpyAsync(*p, h, bytes, hipMemcpyHostToDevice, ustream));
    return MLBDDC_OK;
  }
  // Zero device memory with the wide fill kernel (16-byte stores over many
  // workgroups), or hipMemsetAsync for an unaligned block.
  mlbddc_status zero_async(void* p, size_t bytes, hipStream_t s) {
    if (((uintptr_t)p % 16) == 0 && bytes % 16 == 0) launch_zero(s, p, bytes);
    else HIPCHK(hipMemsetAsync(p, 0, bytes, s));
    HIPCHK(hipGetLastError());
    return MLBDDC_OK;
  }
  mlbddc_status upload_fence() {
    if (!ustream) return MLBDDC_OK;
    HIPCHK(hipEventRecord(ev_upl, ustream));
    HIPCHK(hipStreamWaitEvent(stream, ev_upl, 0));
    return MLBDDC_OK;
  }
  // keep = true: device blocks go to a size-keyed pool that the next set-up
  // reuses (a new set-up of the same problem then allocates nothing); blocks
  // the next set-up does not take are released at its end.
  void free_all(bool keep = false) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
    if (keep) {
      for (auto& a : allocs) pool.emplace(a.second, a.first);
    } else {
      for (auto& a : allocs) raw_free(a.first);
      trim_pool();
    }
    allocs.clear();
    lev.clear();
    ready = false;
  }
  mlbddc_status sync() {
    HIPCHK(hipStreamSynchronize(stream));
    return MLBDDC_OK;
  }

  mlbddc_status setup(const mlbddc_mesh* mesh, const mlbddc_partition* part);
  mlbddc_status validate_level(int li, int part);
  mlbddc_status enqueue_K(int li, bool zero);
  mlbddc_status enqueue_K_assembly(int li, bool zero);
  mlbddc_status enqueue_K_factor(int li);
  mlbddc_status enqueue_weights(int li);
  mlbddc_status enqueue_rest(int li, bool zero);
  mlbddc_status finish_numeric();
  mlbddc_status numeric();
  bool lookahead = false;
  std::vector<std::array<int, 5>> tune;   // (job 0=K/1=M, fp32, log2 bucket, panel, staged columns or 0)
  int mv_tpw[2] = {1, 1};                 // tiles per workgroup of the large tile products: [0] FP64, [1] FP32
  int panel_stage[2] = {0, 0};            // staged columns of the panel products per precision (0: the job's)
  int mfma_f32 = 16;                      // FP32 tile products: 16 (16x16x4), 32 (32x32x2) or 3 (split bf16)
  int pick_panel(int job, bool fp32, int ntmax) const;
  int pick_stage(int job, bool fp32, int ntmax) const;
  mlbddc_status reserve_job(Job& J, bool fp32);
  mlbddc_status prepare_job(Job& J, bool fp32, int job = 0);
  mlbddc_status factor(Job& J, int level, bool precond);
  mlbddc_status build_mv(MvSet& s, int mode, std::vector<MvDesc> descs);
  mlbddc_status build_trsv(LevelDev& D);
  void run_trsv(LevelDev& D, bool transposed);
  // cls >= 0: time the product kernel as profile class cls (algorithmic bytes `bytes`)
  template <typename TA, typename TX, typename TY>
  void run_mv(MvSet& s, const Job& J, const TX* x, TY* y, double alpha, bool acc, void* partial,
              hipStream_t on = nullptr, int cls = -1, double bytes = 0.0);
  // Timing of the level-1 tile products while profiling (outside stream capture).
  struct MvTiming {
    int cls;
    hipEvent_t e0, e1;
    double bytes;
  };
  std::vector<MvTiming> mv_pending;
  std::vector<hipEvent_t> mv_spare;
  double alg_bytes_S = 0.0, alg_bytes_G = 0.0;  // lower triangles of the S_i / G_i, bytes
  void mv_timing(int cls, double bytes, hipStream_t on, hipEvent_t* e0, hipEvent_t* e1);
  mlbddc_status collect_mv_timing();
  // A PCG dot product formed by the last kernel of a product: its scalar slot,
  // the step after it (DotStep) and the squared tolerance of the stopping test.
  struct DotFinish {
    int slot, step;
    double rtol2;
  };
  // r_copied: the weighted copies of rhat are already in place (written by the PCG update)
  mlbddc_status apply_interface(int li, const double* rhat, double* zhat, const DotFinish* ds = nullptr, bool r_copied = false);
  mlbddc_status apply_full(int li, const double* r, double* z);
  // x_copied: the subdomain copies of x are already in place (written by the PCG update)
  mlbddc_status schur(const double* x, double* y, const DotFinish* ds = nullptr, bool x_copied = false);
  // y = S^ x with the device scratch array for its work vectors (no device memory of the handle
  // beyond the operator itself; nothing allocated)
  void* scratch_ptr = nullptr;  // address of `scratch` on this handle's device
  mlbddc_status schur_noalloc(const double* x, double* y);
  mlbddc_status condense(const double* f, double* g);
  mlbddc_status recover(const double* uhat, double* u);
  mlbddc_status solve(const double* f, double* u, const double* u0, mlbddc_stats* st);
  mlbddc_status pcg_body(bool first);
  mlbddc_status capture_pcg();
  mlbddc_status solve_on_stream(const double* f, double* u, const double* u0, mlbddc_stats* st);
};

// ----------------------------------------------------------------- helpers
mlbddc_status Handle::build_mv(MvSet& s, int mode, std::vector<MvDesc> descs) {
  s.mode = mode;
  s.h = std::move(descs);
  std::vector<int64_t> prefix(s.h.size() + 1, 0), prefix2(s.h.size() + 1, 0);
  int64_t poff = 0;
  s.max_out = 0;
  for (size_t i = 0; i < s.h.size(); ++i) {
    MvDesc& d = s.h[i];
    int64_t tiles = mode == MV_SYM ? (int64_t)d.nr * (d.nr + 1) / 2 : (int64_t)d.nr * d.nc;
    prefix[i + 1] = prefix[i] + tiles;
    prefix2[i + 1] = prefix2[i] + (tiles + 1) / 2;
    d.p_off = poff;
    poff += (int64_t)d.nr * d.nc * TS;
    s.max_out = std::max(s.max_out, mode == MV_T ? d.nc : d.nr);
  }
  s.tiles = prefix.back();
  s.groups2 = prefix2.back();
  s.partial_elems = poff;
  mlbddc_status st = upload(&s.d, s.h);
  if (st) return st;
  if ((st = upload(&s.d_prefix2, prefix2))) return st;
  return upload(&s.d_prefix, prefix);
}

template <typename TA, typename TX, typename TY>
void Handle::run_mv(MvSet& s, const Job& J, const TX* x, TY* y, double alpha, bool acc, void* partial, hipStream_t on,
                    int cls, double bytes) {
  hipStream_t st = on ? on : stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (cls >= 0 && prof) mv_timing(cls, bytes, st, &e0, &e1);
  launch_tile_mv<TA, TX, TY>(st, s.mode, s.d, (int32_t)s.h.size(), s.tiles, s.d_prefix, (const TA*)J.buf, x, y, alpha, acc,
                             (TA*)partial, s.max_out, e0, e1, sizeof(TA) == 4 ? mv_tpw[1] : mv_tpw[0], s.groups2,
                             s.d_prefix2);
}

void Handle::mv_timing(int cls, double bytes, hipStream_t on, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(on, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return;
  }
  if (mv_pending.size() >= 4096) (void)collect_mv_timing();
  hipEvent_t ev[2];
  for (hipEvent_t& e : ev) {
    if (!mv_spare.empty()) {
      e = mv_spare.back();
      mv_spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
  }
  mv_pending.push_back({cls, ev[0], ev[1], bytes});
  *e0 = ev[0];
  *e1 = ev[1];
}

mlbddc_status Handle::collect_mv_timing() {
  mlbddc_status st = MLBDDC_OK;
  for (const MvTiming& t : mv_pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(t.e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.e0, t.e1);
    if (e != hipSuccess) {
      if (!st) st = herr("product timing", e);
    } else {
      pdata.time_s[t.cls] += 1e-3 * ms;
      pdata.launches[t.cls] += 1;
      pdata.bytes[t.cls] += t.bytes;
    }
    mv_spare.push_back(t.e0);
    mv_spare.push_back(t.e1);
  }
  mv_pending.clear();
  return st;
}

// Lists of the nonzero tiles of every level-1 factor (from the tile
// structure, else every tile of the envelope): one triangular-solve item per
// interior group with the group's own tiles, ordered by the group's height in
// the dissection tree (the groups of one height depend only on lower groups
// in the forward solve and on higher groups in the backward one); the tiles
// coupling a group to other groups and the L_GI tiles go to tile lists.
mlbddc_status Handle::build_trsv(LevelDev& D) {
  const LevelPlan& P = *D.P;
  D.trsv_h.clear();
  D.tr_rptr.clear();
  D.tr_rcol.clear();
  D.tr_cptr.clear();
  D.tr_crow.clear();
  D.tr_rslot.clear();
  D.tr_cslot.clear();
  D.lgiN = LevelDev::TileList{};
  D.lgiT = LevelDev::TileList{};
  D.trF.clear();
  D.trB.clear();
  std::vector<std::vector<TrsvDesc>> by_h;
  std::vector<std::vector<int32_t>> cols;  // per tile column k: rows r > k of L (interior and interface)
  std::vector<std::vector<std::pair<int32_t, int32_t>>> grow;  // per interface row: (column, -) pairs
  std::vector<int32_t> grp, g0v, g1v, hgt, rcnt;
  for (int b = 0; b < P.n_sub; ++b) {
    const SubPlan& S = P.subs[b];
    const int tI = (int)(S.nIp / TS), tG = (int)(S.nGp / TS), nt = D.K.nt[b];
    const int64_t aoff = D.K.off[b], io = D.iofs[b], go = D.gofs[b];
    bool unstored = false;
    auto tile = [&](int r, int c) {
      const int64_t q = D.K.slot(b, r, c);
      unstored = unstored || q < 0;
      return aoff + q * TE;
    };
    cols.assign(tI, {});
    for (int k = 0; k < tI; ++k) {
      if (!S.sptr.empty()) {
        for (int32_t q = S.sptr[k]; q < S.sptr[k + 1]; ++q) cols[k].push_back(S.srow[q]);
      } else {
        for (int r = k + 1; r < tI + tG; ++r)
          if (S.envK[r] <= k) cols[k].push_back(r);
      }
    }
    // groups
    grp.assign(tI, 0);
    g0v.clear();
    g1v.clear();
    hgt.clear();
    if (!S.gtile.empty()) {
      for (size_t g = 0; g + 1 < S.gtile.size(); ++g) {
        g0v.push_back(S.gtile[g]);
        g1v.push_back(S.gtile[g + 1]);
        hgt.push_back(S.gheight[g]);
        for (int k = S.gtile[g]; k < S.gtile[g + 1]; ++k) grp[k] = (int32_t)g;
      }
    } else {
      g0v.push_back(0);
      g1v.push_back(tI);
      hgt.push_back(0);
    }
    const int H = *std::max_element(hgt.begin(), hgt.end()) + 1;
    if ((int)D.trF.size() < H) {
      D.trF.resize(H);
      D.trB.resize(H);
    }
    // order check: a tile below the diagonal couples a column to its own group or a higher one
    for (int k = 0; k < tI; ++k)
      for (int32_t r : cols[k])
        if (r < tI && grp[r] != grp[k] && hgt[grp[r]] <= hgt[grp[k]])
          return fail(MLBDDC_E_ARG, "internal layout check failed: dissection groups couple out of order");
    // in-group lists for the triangular solves (columns, then their transpose)
    const int32_t p_col = (int32_t)D.tr_cptr.size(), p_row = (int32_t)D.tr_rptr.size();
    const size_t c0 = D.tr_crow.size();
    for (int k = 0; k < tI; ++k) {
      D.tr_cptr.push_back((int32_t)D.tr_crow.size());
      for (int32_t r : cols[k])
        if (r < tI && grp[r] == grp[k]) {
          D.tr_crow.push_back(r);
          const int64_t q = D.K.slot(b, r, k);
          unstored = unstored || q < 0;
          D.tr_cslot.push_back((int32_t)q);
        }
    }
    D.tr_cptr.push_back((int32_t)D.tr_crow.size());
    rcnt.assign(tI + 1, 0);
    for (size_t q = c0; q < D.tr_crow.size(); ++q) rcnt[D.tr_crow[q] + 1]++;
    for (int r = 0; r < tI; ++r) rcnt[r + 1] += rcnt[r];
    const int32_t r0 = (int32_t)D.tr_rcol.size();
    D.tr_rcol.resize(D.tr_rcol.size() + (D.tr_crow.size() - c0));
    D.tr_rslot.resize(D.tr_rcol.size());
    for (int r = 0; r <= tI; ++r) D.tr_rptr.push_back(r0 + rcnt[r]);
    for (int k = 0; k < tI; ++k)
      for (int32_t q = D.tr_cptr[p_col + k]; q < D.tr_cptr[p_col + k + 1]; ++q) {
        const int32_t pos = r0 + rcnt[D.tr_crow[q]]++;
        D.tr_rcol[pos] = k;
        D.tr_rslot[pos] = D.tr_cslot[q];
      }
    for (size_t g = 0; g < g0v.size(); ++g) {
      if (g1v[g] <= g0v[g]) continue;
      if ((int)by_h.size() <= hgt[g]) by_h.resize(hgt[g] + 1);
      by_h[hgt[g]].push_back(TrsvDesc{aoff, nt, g0v[g], g1v[g], p_row, p_col, 0, D.K.inv_off[b], io});
    }
    // coupling lists: forward, row k of a group takes the tiles (k, s) of lower
    // groups; backward, column k takes the tiles (r, k) of higher groups
    {
      std::vector<std::vector<int32_t>> rowlow(tI);
      for (int s = 0; s < tI; ++s)
        for (int32_t r : cols[s])
          if (r < tI && grp[r] != grp[s]) rowlow[r].push_back(s);
      for (int k = 0; k < tI; ++k) {
        LevelDev::TileList& F = D.trF[hgt[grp[k]]];
        if (!rowlow[k].empty()) {
          const int32_t p0 = (int32_t)F.t.size();
          for (int32_t sc : rowlow[k]) F.t.push_back(TileRef{tile(k, sc), io + (int64_t)sc * TS});
          F.o.push_back(OutRef{io + (int64_t)k * TS, p0, (int32_t)F.t.size()});
        }
        LevelDev::TileList& Bk = D.trB[hgt[grp[k]]];
        const int32_t q0 = (int32_t)Bk.t.size();
        for (int32_t r : cols[k])
          if (r < tI && grp[r] != grp[k]) Bk.t.push_back(TileRef{tile(r, k), io + (int64_t)r * TS});
        if ((int32_t)Bk.t.size() > q0) Bk.o.push_back(OutRef{io + (int64_t)k * TS, q0, (int32_t)Bk.t.size()});
      }
    }
    // L_GI: column k takes its interface rows (transposed product into w_I);
    // interface row r takes its columns (product into the interface block)
    {
      std::vector<std::vector<int32_t>> gcols(tG);
      for (int k = 0; k < tI; ++k) {
        const int32_t q0 = (int32_t)D.lgiT.t.size();
        for (int32_t r : cols[k])
          if (r >= tI) {
            D.lgiT.t.push_back(TileRef{tile(r, k), go + (int64_t)(r - tI) * TS});
            gcols[r - tI].push_back(k);
          }
        if ((int32_t)D.lgiT.t.size() > q0) D.lgiT.o.push_back(OutRef{io + (int64_t)k * TS, q0, (int32_t)D.lgiT.t.size()});
      }
      for (int r = 0; r < tG; ++r) {  // every interface block is written (sum of nothing = 0)
        const int32_t q0 = (int32_t)D.lgiN.t.size();
        for (int32_t k : gcols[r]) D.lgiN.t.push_back(TileRef{tile(tI + r, k), io + (int64_t)k * TS});
        D.lgiN.o.push_back(OutRef{go + (int64_t)r * TS, q0, (int32_t)D.lgiN.t.size()});
      }
    }
    if (unstored) return fail(MLBDDC_E_ARG, "internal layout check failed: a factor tile of the solves is not stored");
  }
  D.trsv_lvl.assign(1, 0);
  for (auto& v : by_h) {
    D.trsv_h.insert(D.trsv_h.end(), v.begin(), v.end());
    D.trsv_lvl.push_back((int32_t)D.trsv_h.size());
  }
  if (D.trF.size() < by_h.size()) {
    D.trF.resize(by_h.size());
    D.trB.resize(by_h.size());
  }
  mlbddc_status st;
  if ((st = upload(&D.d_trsv, D.trsv_h))) return st;
  if ((st = upload(&D.d_tr_rptr, D.tr_rptr))) return st;
  if ((st = upload(&D.d_tr_rcol, D.tr_rcol))) return st;
  if ((st = upload(&D.d_tr_cptr, D.tr_cptr))) return st;
  if ((st = upload(&D.d_tr_crow, D.tr_crow))) return st;
  if ((st = upload(&D.d_tr_rslot, D.tr_rslot))) return st;
  if ((st = upload(&D.d_tr_cslot, D.tr_cslot))) return st;
  int64_t pmax = 1;
  auto up = [&](LevelDev::TileList& T) -> mlbddc_status {
    pmax = std::max<int64_t>(pmax, (int64_t)T.t.size());
    mlbddc_status s2;
    if ((s2 = upload(&T.dt, T.t))) return s2;
    return upload(&T.dout, T.o);
  };
  if ((st = up(D.lgiN)) || (st = up(D.lgiT))) return st;
  for (auto& T : D.trF)
    if ((st = up(T))) return st;
  for (auto& T : D.trB)
    if ((st = up(T))) return st;
  return dalloc(&D.tl_partial, pmax * TS);
}

void Handle::run_trsv(LevelDev& D, bool transposed) {
  const int nh = (int)D.trsv_lvl.size() - 1;
  for (int i = 0; i < nh; ++i) {
    const int h = transposed ? nh - 1 - i : i;
    LevelDev::TileList& C = transposed ? D.trB[h] : D.trF[h];
    launch_tile_list_mv(stream, transposed, C.dt, (int64_t)C.t.size(), C.dout, (int64_t)C.o.size(), (const double*)D.K.buf,
                        D.wI, D.tl_partial, D.wI, -1.0, true);
    launch_trsv(stream, transposed, D.d_trsv + D.trsv_lvl[h], D.trsv_lvl[h + 1] - D.trsv_lvl[h], (const double*)D.K.buf,
                (const double*)D.K.inv, D.d_tr_rptr, D.d_tr_rcol, D.d_tr_rslot, D.d_tr_cptr, D.d_tr_crow, D.d_tr_cslot,
                D.wI);
  }
}

// Panel width of a factorization job: explicit option, else the tune table's
// entry for (job kind, precision, ceil(log2(max tiles per side))), else the
// nearest bucket of the same kind, else 4.
int Handle::pick_panel(int job, bool fp32, int ntmax) const {
  const int explicit_p = job == 0 ? opt.panel_tiles : opt.panel_tiles_precond;
  if (explicit_p > 0) return explicit_p;
  int bucket = 0;
  while ((1 << bucket) < ntmax) ++bucket;
  int best = -1, bestd = 1 << 30;
  for (const auto& t : tune) {
    if (t[0] != job || t[1] != (fp32 ? 1 : 0)) continue;
    int d = std::abs(t[2] - bucket);
    if (d < bestd) { bestd = d; best = t[3]; }
  }
  return best > 0 ? best : 4;
}

// Staged columns of the tile products of a job: explicit option, else the
// tune table's entry chosen as for the panel width, else 32.
int Handle::pick_stage(int job, bool fp32, int ntmax) const {
  if (opt.stage_cols > 0) return opt.stage_cols;
  int bucket = 0;
  while ((1 << bucket) < ntmax) ++bucket;
  int best = 0, bestd = 1 << 30;
  for (const auto& t : tune) {
    if (t[0] != job || t[1] != (fp32 ? 1 : 0)) continue;
    int d = std::abs(t[2] - bucket);
    if (d < bestd) { bestd = d; best = t[4]; }
  }
  return best > 0 ? best : 32;
}

// Matrix layout and storage of a job (J.nt and the items' e1, e2 and tile
// structure set): the matrices are zeroed on the upload stream right away,
// while the host keeps preparing (the upload fence orders this before the
// assembly).  A matrix with a tile structure stores only the tiles that the
// factorization, the assembly and the solves read (read_before_write_tiles):
// the tiles of its eliminated columns in the order listed there, then, in a
// region shared by the job's mapped matrices, its trailing block packed like
// a matrix of its own.
mlbddc_status Handle::reserve_job(Job& J, bool fp32) {
  J.fp32 = fp32;
  const size_t esz = fp32 ? 4 : 8;
  const int ni = (int)J.nt.size();
  J.off.resize(ni);
  J.inv_off.resize(ni);
  J.tmap_off.assign(ni, -1);
  J.nlead.resize(ni);
  J.tslot0.assign(ni, -1);
  int64_t msz = 0;
  for (int i = 0; i < ni; ++i)
    if (J.items[i].sptr) {
      J.tmap_off[i] = msz;
      msz += packed_tiles(J.nt[i]);
    }
  J.tmap.assign(msz, -1);
  const int T = std::min(16, std::max(1, ni / 4));
  parallel_run(T, [&](int t) {  // the leading tiles of every matrix
    for (int i = ni * t / T; i < ni * (t + 1) / T; ++i) {
      if (J.tmap_off[i] < 0) {
        J.nlead[i] = packed_tiles(J.nt[i]);
        continue;
      }
      int32_t* m = J.tmap.data() + J.tmap_off[i];
      const int nt = J.nt[i], e1 = J.items[i].e1;
      int32_t next = 0;
      read_before_write_tiles(J.items[i], [&](int r0, int k, int count) {
        if (k < e1)
          for (int c = 0; c < count; ++c) m[tile_index(r0 + c, k, nt)] = next++;
      });
      J.nlead[i] = next;
    }
  });
  int64_t tot = 0, itot = 0;
  for (int i = 0; i < ni; ++i) {
    J.off[i] = tot;
    tot += J.nlead[i] * TE;
    J.inv_off[i] = itot;
    itot += (int64_t)(J.items[i].e1 + J.items[i].e2) * TE;
  }
  for (int i = 0; i < ni; ++i)  // the trailing blocks, back to back
    if (J.tmap_off[i] >= 0) {
      J.tslot0[i] = (tot - J.off[i]) / TE;
      tot += packed_tiles(J.nt[i] - J.items[i].e1) * TE;
    }
  if (tot / TE >= INT32_MAX) return fail(MLBDDC_E_ARG, "matrix job too large for 32-bit tile slots");
  parallel_run(T, [&](int t) {
    for (int i = ni * t / T; i < ni * (t + 1) / T; ++i) {
      if (J.tmap_off[i] < 0) continue;
      int32_t* m = J.tmap.data() + J.tmap_off[i];
      const int nt = J.nt[i], e1 = J.items[i].e1;
      for (int c = e1; c < nt; ++c)
        for (int r = c; r < nt; ++r) m[tile_index(r, c, nt)] = (int32_t)(J.tslot0[i] + tile_index(r - e1, c - e1, nt - e1));
    }
  });
  J.elems = tot;
  J.inv_elems = itot;
  if (verbose && msz > 0) {
    int64_t dense = 0;
    for (int i = 0; i < ni; ++i) dense += packed_tiles(J.nt[i]);
    std::fprintf(stderr, "[mlbddc setup]     tile-mapped storage: %lld of %lld tiles (%.1f%%)\n", (long long)(tot / TE),
                 (long long)dense, 100.0 * (double)(tot / TE) / (double)std::max<int64_t>(dense, 1));
  }
  void* b = nullptr;
  void* iv = nullptr;
  mlbddc_status st = fp32 ? dalloc((float**)&b, std::max<int64_t>(tot, 1)) : dalloc((double**)&b, std::max<int64_t>(tot, 1));
  if (st) return st;
  st = fp32 ? dalloc((float**)&iv, std::max<int64_t>(itot, 1)) : dalloc((double**)&iv, std::max<int64_t>(itot, 1));
  if (st) return st;
  J.buf = b;
  J.inv = iv;
  if ((st = ensure_ustream())) return st;
  if (tot > 0 && (st = zero_async(J.buf, (size_t)tot * esz, ustream))) return st;
  if (msz > 0) {
    if ((st = upload(&J.d_tmap, J.tmap))) return st;
    if ((st = upload(&J.d_tmap_off, J.tmap_off))) return st;
  }
  return MLBDDC_OK;
}

mlbddc_status Handle::prepare_job(Job& J, bool fp32, int job) {
  mlbddc_status st;
  double tm = now();
  auto mark = [&](const char* what) {
    if (verbose) std::fprintf(stderr, "[mlbddc setup]     %-24s %8.2f ms\n", what, (now() - tm) * 1e3);
    tm = now();
  };
  if (!J.buf && (st = reserve_job(J, fp32))) return st;
  mark("storage");
  for (size_t i = 0; i < J.nt.size(); ++i) J.items[i].env = J.env[i].data();
  int ntmax = 1;
  for (int32_t x : J.nt) ntmax = std::max(ntmax, x);
  J.panel = pick_panel(job, fp32, ntmax);
  J.stage = pick_stage(job, fp32, ntmax);
  J.pstage = opt.stage_cols > 0 ? opt.stage_cols : panel_stage[fp32 ? 1 : 0];
  if (!J.tmap.empty()) J.panel = std::min(J.panel, 64);  // k_tile_mm holds a task's tile slots in one wavefront
  if (ntmax >= panel_nt[job]) {  // report the panel width of the largest job of the set-up
    panel_nt[job] = ntmax;
    pdata.panel[job] = J.panel;
    pdata.stage[job] = J.stage;
  }
  build_factor_schedule(J.items, J.panel, J.sched, lookahead);
  mark("schedule");
  if ((st = upload(&J.d_off, J.off))) return st;
  if ((st = upload(&J.d_inv_off, J.inv_off))) return st;
  if ((st = upload(&J.d_nt, J.nt))) return st;
  if ((st = upload(&J.d_tasks, J.sched.tasks))) return st;
  // [0] item + 1 and [1] column of the first non-positive pivot; [2] set by
  // an assembly entry that falls in an unstored tile
  if ((st = dalloc(&J.d_err, 3))) return st;
  mark("uploads");
  return MLBDDC_OK;
}

mlbddc_status Handle::factor(Job& J, int level, bool precond) {
  HIPCHK(hipMemsetAsync(J.d_err, 0, 2 * sizeof(int32_t), stream));
  if (prof) HIPCHK(hipStreamSynchronize(stream));  // job time excludes earlier queued work
  const double tj0 = prof ? now() : 0.0;
  FactorArgs a{J.d_tasks, J.d_off, J.d_nt, J.d_inv_off, J.d_err, J.d_tmap, J.d_tmap_off, J.stage, J.pstage,
               J.fp32 ? mfma_f32 : 16};
  const size_t nl = J.sched.launches.size();
  if (prof)
    while (events.size() < 2 * nl) {
      hipEvent_t ev;
      HIPCHK(hipEventCreate(&ev));
      events.push_back(ev);
    }
  bool two = false;
  for (const FactorLaunch& L : J.sched.launches) two = two || L.stream == 1;
  if (two && !fstream) {
    HIPCHK(hipStreamCreateWithFlags(&fstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ev_a, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_b, hipEventDisableTiming));
  }
  if (two) {  // the second stream starts after everything queued so far
    HIPCHK(hipEventRecord(ev_a, stream));
    HIPCHK(hipStreamWaitEvent(fstream, ev_a, 0));
  }
  for (size_t i = 0; i < nl; ++i) {
    const FactorLaunch& L = J.sched.launches[i];
    hipStream_t s0 = L.stream == 1 ? fstream : stream;
    if (L.wait && two) {
      hipStream_t other = L.stream == 1 ? stream : fstream;
      hipEvent_t ev = L.stream == 1 ? ev_a : ev_b;
      HIPCHK(hipEventRecord(ev, other));
      HIPCHK(hipStreamWaitEvent(s0, ev, 0));
    }
    if (prof) HIPCHK(hipEventRecord(events[2 * i], s0));
    if (J.fp32)
      launch_factor_step<float>(s0, L.kind, L.k, a, L.first, L.count, (float*)J.buf, (float*)J.inv);
    else
      launch_factor_step<double>(s0, L.kind, L.k, a, L.first, L.count, (double*)J.buf, (double*)J.inv);
    if (prof) HIPCHK(hipEventRecord(events[2 * i + 1], s0));
  }
  if (two) {  // everything on the second stream before the caller's stream continues
    HIPCHK(hipEventRecord(ev_b, fstream));
    HIPCHK(hipStreamWaitEvent(stream, ev_b, 0));
  }
  HIPCHK(hipGetLastError());
  if (prof) {
    HIPCHK(hipStreamSynchronize(stream));
    pdata.job_time_s[precond ? 1 : 0] += now() - tj0;
    for (size_t i = 0; i < nl; ++i) {
      const FactorLaunch& L = J.sched.launches[i];
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, events[2 * i], events[2 * i + 1]));
      int c = MLBDDC_PROF_NEGATE;
      if (L.kind == L_TRAIL || L.kind == L_INPANEL) c = J.fp32 ? MLBDDC_PROF_UPDATE_FP32 : MLBDDC_PROF_UPDATE_FP64;
      else if (L.kind == L_PANEL) c = MLBDDC_PROF_PANEL;
      else if (L.kind == L_DIAG) c = MLBDDC_PROF_DIAG;
      pdata.time_s[c] += 1e-3 * ms;
      pdata.flops[c] += L.flops;
      pdata.launches[c] += 1;
      pdata.tiles[c] += L.count;
    }
  }
  (void)level;
  return MLBDDC_OK;
}

// --------------------------------------------------------------------- setup
mlbddc_status Handle::setup(const mlbddc_mesh* mesh, const mlbddc_partition* part) {
  if (!mesh || !part) return fail(MLBDDC_E_ARG, "null mesh or partition");
  if (!mesh->elem_matrix_ref || !mesh->elem_scale) return fail(MLBDDC_E_ARG, "missing element matrix or scales");
  double t0 = now();
  HIPCHK(hipStreamSynchronize(stream));
  if (mlbddc_status sr = stage_reset()) return sr;
  free_all(true);
  panel_nt[0] = panel_nt[1] = 0;
  verbose = std::getenv("MLBDDC_VERBOSE") != nullptr;
  double tm = t0;
  auto mark = [&](const char* what) {
    if (verbose) std::fprintf(stderr, "[mlbddc setup] %-28s %8.2f ms\n", what, (now() - tm) * 1e3);
    tm = now();
  };
  mark("wait, release previous");
  // Queuing a factorization can block the host once the launch queue is
  // full, so each level's numeric work is queued by a worker thread while
  // this thread prepares the next part.  At most one part is being queued at
  // a time (join() before the next upload fence and enqueue), so the library
  // stream sees the same order as a sequential set-up.
  std::future<mlbddc_status> pending;
  auto join = [&]() -> mlbddc_status { return pending.valid() ? pending.get() : MLBDDC_OK; };
  // part 0: K assembly (and the interface diagonal for the weights); 1: K
  // factorization; 3: interface weights (needs the flat layouts); 2: the rest
  auto enqueue_async = [&](int li, int part) {
    const int dev = opt.device;
    pending = std::async(std::launch::async, [this, li, part, dev]() -> mlbddc_status {
      if (hipSetDevice(dev) != hipSuccess) return herr("hipSetDevice", hipGetLastError());
      return part == 0 ? enqueue_K_assembly(li, false) : part == 1 ? enqueue_K_factor(li)
                       : part == 3 ? enqueue_weights(li) : enqueue_rest(li, false);
    });
  };
  PlanInput in;
  in.dim = mesh->dim;
  in.ndof = mesh->ndof_per_node;
  in.n_nodes = mesh->n_nodes;
  in.n_elems = mesh->n_elems;
  in.nodes_per_elem = mesh->nodes_per_elem;
  in.elem_nodes = mesh->elem_nodes;
  in.dirichlet = mesh->dirichlet_nodes;
  in.n_levels = part->n_levels;
  in.elem_to_sub = part->elem_to_sub;
  in.sub_to_parent = part->sub_to_parent;
  in.constraints = part->constraints;
  if (in.nodes_per_elem != (1 << in.dim)) return fail(MLBDDC_E_ARG, "nodes_per_elem must be 2^dim");
  Error e;
  mlbddc_status st = build_plan(in, plan, e);
  if (st) {
    err = e;
    return st;
  }
  planned = true;
  mark("build_plan");
  const int nd = in.ndof;
  nloc1 = in.nodes_per_elem * nd;
  n_elems = in.n_elems;
  const int nlev = (int)plan.levels.size();
  lev.assign(nlev, LevelDev());
  const bool mixed = opt.precision == MLBDDC_MIXED;

  // ---- mesh data on the device
  {
    std::vector<double> kref(mesh->elem_matrix_ref, mesh->elem_matrix_ref + (size_t)nloc1 * nloc1);
    if ((st = upload(&d_Kref, kref))) return st;
    std::vector<double> sc(mesh->elem_scale, mesh->elem_scale + n_elems);
    if ((st = upload(&d_scale, sc))) return st;
  }

  // element DOF map (only the element energies use it): filled by a thread
  // of its own into pinned staging memory while the device factorizes
  const size_t edof_n = (size_t)n_elems * nloc1;
  int32_t* h_edof = nullptr;
  std::future<void> edof_job;
  if (edof_n && (st = stage(sizeof(int32_t) * edof_n, (char**)&h_edof))) return st;
  auto start_edof = [&]() {
    const int npe = in.nodes_per_elem;
    const int32_t* en = mesh->elem_nodes;
    edof_job = std::async(std::launch::async, [this, h_edof, en, npe, nd]() {
      for (int64_t el = 0; el < n_elems; ++el)
        for (int a = 0; a < npe; ++a) {
          const int64_t fnode = plan.node_to_free[en[el * npe + a]];
          for (int c = 0; c < nd; ++c) h_edof[el * nloc1 + a * nd + c] = fnode < 0 ? -1 : (int32_t)(fnode * nd + c);
        }
    });
  };
  for (int li = 0; li < nlev; ++li) {
    LevelDev& D = lev[li];
    LevelPlan& P = plan.levels[li];
    D.P = &P;
    D.kfp32 = mixed && li > 0 && !P.top;
    D.mfp32 = mixed;
    const int ns = P.n_sub;
    // ---- storage of the constrained problems first: zeroing it on the upload
    // stream (at full bandwidth) starts while the host lays out the K job, and
    // no zeroing runs beside a factorization
    if (!P.top) {
      D.M.nt.resize(ns);
      D.M.items.resize(ns);
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        const int tG = (int)(S.nGp / TS), tC = S.ncp / TS;
        D.M.nt[b] = 2 * (tG + tC);
        D.M.items[b].nt = D.M.nt[b];
        D.M.items[b].e1 = tG;
        D.M.items[b].e2 = tC;
      }
      if ((st = reserve_job(D.M, D.mfp32))) return st;
      mark("  M job storage");
    }
    // ---- K job
    D.K.nt.resize(ns);
    D.K.items.resize(ns);
    D.K.env.resize(ns);
    for (int b = 0; b < ns; ++b) {
      const SubPlan& S = P.subs[b];
      int64_t nK = S.nIp + S.nGp + (P.augmentK ? S.nIp : 0);
      D.K.nt[b] = (int32_t)(nK / TS);
      D.K.items[b].nt = D.K.nt[b];
      D.K.items[b].e1 = (int32_t)(S.nIp / TS);
      D.K.items[b].e2 = 0;
      D.K.env[b] = S.envK;
      if (!S.sptr.empty() && !P.augmentK) {  // nested-dissection interior: tile structure
        D.K.items[b].sptr = S.sptr.data();
        D.K.items[b].srow = S.srow.data();
        D.K.items[b].gtile = S.gtile.data();
        D.K.items[b].gheight = S.gheight.data();
        D.K.items[b].ngroups = (int32_t)S.gtile.size() - 1;
      }
    }
    if ((st = prepare_job(D.K, D.kfp32))) return st;
    flops_K += D.K.sched.flops;
    mark("  K job layout + schedule");

    // diagonal segments of the K matrices: padding and identity block
    for (int b = 0; b < ns; ++b) {
      const SubPlan& S = P.subs[b];
      int32_t nt = D.K.nt[b];
      auto add = [&](int64_t r0, int64_t c0, int64_t cnt, double v) {
        if (cnt > 0) D.ksegs_h.push_back(DiagSeg{D.K.off[b], nt, (int32_t)r0, (int32_t)c0, (int32_t)cnt, v, b});
      };
      for (size_t q = 0; q + 1 < S.padI.size(); q += 2) add(S.padI[q], S.padI[q], S.padI[q + 1], 1.0);
      add(S.nIp + S.nG, S.nIp + S.nG, S.nGp - S.nG, 1.0);
      if (P.augmentK) add(S.nIp + S.nGp, 0, S.nIp, 1.0);
    }
    for (auto& s : D.ksegs_h) D.kseg_max = std::max(D.kseg_max, s.count);
    if ((st = upload(&D.d_ksegs, D.ksegs_h))) return st;
    // the layout checks of what assembly, weights and the K job use run on
    // another thread while this one builds the assembly and flat layouts
    // (they read only the plan, the K job and the segments above)
    std::future<mlbddc_status> checked = std::async(std::launch::async, [this, li] { return validate_level(li, 0); });
    std::future<mlbddc_status> checked_job = std::async(std::launch::async, [this, li] { return validate_level(li, 2); });

    // assembly data
    {
      // elements grouped by colour, within a colour by subdomain (each matrix
      // entry gets at most one contribution per colour, so the order inside a
      // colour does not change the sums); counts per (colour, subdomain) on
      // threads, then every subdomain places its elements
      const int nc = P.n_colors;
      std::vector<int64_t> cnt((size_t)nc * ns + 1, 0);  // [colour][subdomain]
      const int T = std::min(16, std::max(1, ns / 16));
      parallel_run(T, [&](int t) {
        for (int b = ns * t / T; b < ns * (t + 1) / T; ++b)
          for (int64_t e : P.subs[b].elems) cnt[(size_t)P.el_color[e] * ns + b + 1]++;
      });
      for (size_t q = 1; q < cnt.size(); ++q) cnt[q] += cnt[q - 1];
      D.color_ptr.assign(nc + 1, 0);
      for (int c = 0; c <= nc; ++c) D.color_ptr[c] = cnt[(size_t)c * ns];
      if ((st = upload_fill(&D.d_elems_by_color, (int64_t)P.el_color.size(), [&](int64_t* byc) {
             parallel_run(T, [&](int t) {
               std::vector<int64_t> pos(nc);
               for (int b = ns * t / T; b < ns * (t + 1) / T; ++b) {
                 for (int c = 0; c < nc; ++c) pos[c] = cnt[(size_t)c * ns + b];
                 for (int64_t e : P.subs[b].elems) byc[pos[P.el_color[e]]++] = e;
               }
             });
             return MLBDDC_OK;
           })))
        return st;
      mark("    colour order");
      if ((st = upload(&D.d_el_local_ptr, P.el_local_ptr))) return st;
      if ((st = upload(&D.d_el_local, P.el_local))) return st;
      if ((st = upload(&D.d_el_sub, P.el_sub))) return st;
      if ((st = upload(&D.d_sub_off, D.K.off))) return st;
      if ((st = upload(&D.d_sub_nt, D.K.nt))) return st;
      if (li > 0) {
        if ((st = upload(&D.d_ekc_off, lev[li - 1].kc_off))) return st;
      }
      mark("    element uploads");
    }

    // flat offsets and the positions of the interface diagonal in the K
    // matrices (the assembly saves that diagonal for the weights)
    D.gofs.assign(ns + 1, 0);
    D.iofs.assign(ns + 1, 0);
    D.cofs.assign(ns + 1, 0);
    for (int b = 0; b < ns; ++b) {
      D.gofs[b + 1] = D.gofs[b] + P.subs[b].nGp;
      D.iofs[b + 1] = D.iofs[b] + P.subs[b].nIp;
      D.cofs[b + 1] = D.cofs[b] + P.subs[b].ncp;
    }
    D.nG_flat = D.gofs[ns];
    D.nI_flat = D.iofs[ns];
    D.nC_flat = D.cofs[ns];
    if (!P.top) {
      std::atomic<bool> gbad{false};
      if ((st = upload_fill(&D.d_gdiag_pos, D.nG_flat, [&](int64_t* gdiag) {
             parallel_run(std::min(16, ns), [&](int t) {
               for (int b = t; b < ns; b += std::min(16, ns)) {
                 const SubPlan& S = P.subs[b];
                 int64_t o;
                 int32_t n, f;
                 D.K.trailing(b, (int)(S.nIp / TS), o, n, f);
                 for (int64_t k = 0; k < S.nGp; ++k) {
                   const int64_t v = o + packed_offset(f * TS + k, f * TS + k, n);
                   gdiag[D.gofs[b] + k] = v;
                   if (v < 0 || v >= D.K.elems) gbad = true;
                 }
               }
             });
             return gbad ? fail(MLBDDC_E_ARG, "internal layout check failed: interface diagonal position") : MLBDDC_OK;
           })))
        return st;
    }
    if ((st = dalloc(&D.gd, std::max<int64_t>(D.nG_flat, 1)))) return st;

    mark("  assembly maps");
    // the device assembles and factorizes K while the host builds the flat
    // layouts; the factorization is queued once its own checks are done
    if ((st = checked.get())) return st;
    mark("  validate (assembly)");
    if ((st = join())) return st;
    if ((st = upload_fence())) return st;
    enqueue_async(li, 0);
    if ((st = join())) return st;
    if ((st = checked_job.get())) return st;
    mark("  validate (K job)");
    enqueue_async(li, 1);
    // flat layouts
    {
      std::vector<int32_t> gidx(D.nG_flat, -1), iidx(D.nI_flat, -1), cidx(D.nC_flat, -1);
      const int64_t nif = (int64_t)P.iface_dofs.size();
      std::vector<int64_t> gcnt(nif + 1, 0), ccnt(P.n_coarse + 1, 0);
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        for (int64_t k = 0; k < S.nG; ++k) {
          gidx[D.gofs[b] + k] = S.iface[k];
          gcnt[S.iface[k] + 1]++;
        }
        for (int64_t k = 0; k < S.nIp; ++k) iidx[D.iofs[b] + k] = (int32_t)S.dofI[k];
        for (int k = 0; k < S.nc; ++k) {
          cidx[D.cofs[b] + k] = S.coarse[k];
          ccnt[S.coarse[k] + 1]++;
        }
      }
      for (int64_t g = 0; g < nif; ++g) gcnt[g + 1] += gcnt[g];
      for (int64_t g = 0; g < P.n_coarse; ++g) ccnt[g + 1] += ccnt[g];
      std::vector<int64_t> glist(gcnt[nif]), clist(ccnt[P.n_coarse]);
      {
        std::vector<int64_t> pos(gcnt.begin(), gcnt.end() - 1), cpos(ccnt.begin(), ccnt.end() - 1);
        for (int b = 0; b < ns; ++b) {
          const SubPlan& S = P.subs[b];
          for (int64_t k = 0; k < S.nG; ++k) glist[pos[S.iface[k]]++] = D.gofs[b] + k;
          for (int k = 0; k < S.nc; ++k) clist[cpos[S.coarse[k]]++] = D.cofs[b] + k;
        }
      }
      std::vector<int32_t> ifd(nif);
      for (int64_t g = 0; g < nif; ++g) ifd[g] = (int32_t)P.iface_dofs[g];
      if ((st = upload(&D.d_gidx, gidx))) return st;
      if ((st = upload(&D.d_iidx, iidx))) return st;
      if ((st = upload(&D.d_cidx, cidx))) return st;
      if ((st = upload(&D.d_iface_dofs, ifd))) return st;
      if ((st = upload(&D.d_gptr, gcnt))) return st;
      if ((st = upload(&D.d_glist, glist))) return st;
      if ((st = upload(&D.d_cptr, ccnt))) return st;
      if ((st = upload(&D.d_clist, clist))) return st;
    }
    const size_t mesz = D.mfp32 ? 4 : 8, kesz = D.kfp32 ? 4 : 8;
    auto valloc = [&](void** p, int64_t n, size_t esz) -> mlbddc_status {
      return esz == 4 ? dalloc((float**)p, std::max<int64_t>(n, 1)) : dalloc((double**)p, std::max<int64_t>(n, 1));
    };
    if ((st = dalloc(&D.d_w, std::max<int64_t>(D.nG_flat, 1)))) return st;
    if ((st = valloc(&D.rl, D.nG_flat, mesz))) return st;
    if ((st = valloc(&D.yl, D.nG_flat, mesz))) return st;
    if ((st = valloc(&D.zcl, D.nC_flat, mesz))) return st;
    if ((st = dalloc(&D.rcl, std::max<int64_t>(D.nC_flat, 1)))) return st;
    if ((st = dalloc(&D.rC, std::max<int64_t>(P.n_coarse, 1)))) return st;
    if ((st = dalloc(&D.zC, std::max<int64_t>(P.n_coarse, 1)))) return st;
    if ((st = dalloc(&D.rhat, std::max<int64_t>((int64_t)P.iface_dofs.size(), 1)))) return st;
    if ((st = dalloc(&D.zhat, std::max<int64_t>((int64_t)P.iface_dofs.size(), 1)))) return st;
    if ((st = valloc(&D.rI, D.nI_flat, kesz))) return st;
    if ((st = valloc(&D.uI, D.nI_flat, kesz))) return st;
    if ((st = valloc(&D.zG, D.nG_flat, kesz))) return st;
    if ((st = dalloc(&D.tG, std::max<int64_t>(D.nG_flat, 1)))) return st;
    if ((st = dalloc(&D.gd2, std::max<int64_t>(D.nG_flat, 1)))) return st;
    if ((st = dalloc(&D.wI, std::max<int64_t>(D.nI_flat, 1)))) return st;

    mark("  flat layouts + vectors");
    // the weights, queued behind the K factorization
    if ((st = join())) return st;
    if ((st = upload_fence())) return st;
    enqueue_async(li, 3);
    // K-job tile mat-vecs
    {
      std::vector<MvDesc> s, pre;
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        int tI = (int)(S.nIp / TS), tG = (int)(S.nGp / TS);
        if (li == 0) {
          int64_t o;
          int32_t n, f;
          D.K.trailing(b, tI, o, n, f);
          s.push_back(MvDesc{o, n, f, tG, f, tG, D.gofs[b], D.gofs[b], 0, nullptr, (int32_t)S.nG, (int32_t)S.nG});
        } else if (tI > 0) {
          int tId = tI + tG;
          pre.push_back(MvDesc{D.K.off[b], D.K.nt[b], tId, tI, tId, tI, D.iofs[b], D.iofs[b], 0, nullptr, (int32_t)S.nI,
                               (int32_t)S.nI});
        }
      }
      if (li == 0) {
        if ((st = build_mv(D.mvS, MV_SYM, s))) return st;
        // triangular solves and the L_GI products of condensation and recovery
        if ((st = build_trsv(D))) return st;
      } else {
        if ((st = build_mv(D.mvPre, MV_SYM, pre))) return st;
        if (!P.top) {
          std::vector<MvDesc> pt, pn;
          for (int b = 0; b < ns; ++b) {
            const SubPlan& S = P.subs[b];
            int tI = (int)(S.nIp / TS), tG = (int)(S.nGp / TS);
            if (tI == 0 || tG == 0) continue;
            int tId = tI + tG;
            pt.push_back(MvDesc{D.K.off[b], D.K.nt[b], tId, tI, tI, tG, D.iofs[b], D.gofs[b], 0, nullptr, (int32_t)S.nI,
                                (int32_t)S.nG});
            pn.push_back(MvDesc{D.K.off[b], D.K.nt[b], tId, tI, tI, tG, D.gofs[b], D.iofs[b], 0, nullptr, (int32_t)S.nI,
                                (int32_t)S.nG});
          }
          if ((st = build_mv(D.mvPreT, MV_T, pt))) return st;
          if ((st = build_mv(D.mvPostN, MV_N, pn))) return st;
        }
      }
    }

    mark("  K mat-vec sets");
    // ---- preconditioner job and coarse matrices
    if (!P.top) {
      D.M.nt.resize(ns);
      D.M.items.resize(ns);
      D.M.env.resize(ns);
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        int tG = (int)(S.nGp / TS), tC = S.ncp / TS;
        int nt = 2 * (tG + tC);
        D.M.nt[b] = nt;
        D.M.items[b].nt = nt;
        D.M.items[b].e1 = tG;
        D.M.items[b].e2 = tC;
        std::vector<int32_t> env(nt, 0);
        // C rows: first interface tile touched by the row's glob
        std::vector<int32_t> cfirst(tC, tG);
        for (int c = 0; c < S.nc; ++c) {
          int m = INT32_MAX;
          for (int j = S.crow_ptr[c]; j < S.crow_ptr[c + 1]; ++j) m = std::min(m, S.crow_col[j]);
          cfirst[c / TS] = std::min(cfirst[c / TS], m / TS);
        }
        for (int r = 0; r < tC; ++r) env[tG + r] = std::min(cfirst[r], tG + r);
        for (int r = 0; r < tG; ++r) env[tG + tC + r] = r;
        for (int r = 0; r < tC; ++r) env[2 * tG + tC + r] = tG;
        D.M.env[b] = env;
      }
      if ((st = prepare_job(D.M, D.mfp32, 1))) return st;
      flops_M += D.M.sched.flops;
      mark("  M job layout + schedule");
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        int tG = (int)(S.nGp / TS);
        int64_t ko;
        int32_t kn, kf;
        D.K.trailing(b, (int)(S.nIp / TS), ko, kn, kf);
        D.copy_h.push_back(CopyDesc{ko, kn, kf, D.M.off[b], D.M.nt[b], tG});
        D.copy_max = std::max(D.copy_max, tG);
        auto add = [&](int64_t r0, int64_t c0, int64_t cnt, double v) {
          if (cnt > 0) D.msegs_h.push_back(DiagSeg{D.M.off[b], D.M.nt[b], (int32_t)r0, (int32_t)c0, (int32_t)cnt, v});
        };
        add(S.nGp + S.nc, S.nGp + S.nc, S.ncp - S.nc, -1.0);
        add(S.nGp + S.ncp, 0, S.nGp, 1.0);
        add(2 * S.nGp + S.ncp, S.nGp, S.ncp, 1.0);
      }
      for (auto& s : D.msegs_h) D.mseg_max = std::max(D.mseg_max, s.count);
      if ((st = upload(&D.d_msegs, D.msegs_h))) return st;
      if ((st = upload(&D.d_copy, D.copy_h))) return st;
      std::vector<int32_t>& ccols = D.ccols_h;
      ccols.clear();
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        for (int c = 0; c < S.nc; ++c) {
          ConsDesc cd;
          int32_t kf;
          D.K.trailing(b, (int)(S.nIp / TS), cd.kdiag_off, cd.k_nt, kf);
          cd.k_g0 = kf * TS;
          cd.p_off = D.M.off[b];
          cd.p_nt = D.M.nt[b];
          cd.c_row0 = (int32_t)S.nGp + c;
          cd.ptr0 = (int32_t)ccols.size();
          for (int j = S.crow_ptr[c]; j < S.crow_ptr[c + 1]; ++j) ccols.push_back(S.crow_col[j]);
          cd.ptr1 = (int32_t)ccols.size();
          D.cons_h.push_back(cd);
        }
      }
      if ((st = upload(&D.d_cons, D.cons_h))) return st;
      if ((st = upload(&D.d_ccols, ccols))) return st;
      // coarse matrices (read from the eliminated constrained problems)
      int64_t cmp = 0, roff = 0;
      D.kc_off.resize(ns);
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        int tG = (int)(S.nGp / TS), tC = S.ncp / TS;
        KcDesc kd;
        kd.p_off = D.M.off[b];
        kd.p_nt = D.M.nt[b];
        kd.p_c0 = 2 * tG + tC;
        kd.nc = S.nc;
        kd.out_off = cmp;
        kd.rho_off = roff;
        D.kcd_h.push_back(kd);
        D.max_nc = std::max(D.max_nc, S.nc);
        D.kc_off[b] = cmp;
        cmp += (int64_t)S.nc * S.nc;
        roff += S.nc;
      }
      if ((st = upload(&D.d_kcd, D.kcd_h))) return st;
      if ((st = dalloc(&D.d_rho, std::max<int64_t>(roff, 1)))) return st;
      if ((st = dalloc(&D.kc_compact, std::max<int64_t>(cmp, 1)))) return st;
      // M-job tile mat-vecs
      std::vector<MvDesc> g, pn, pt;
      for (int b = 0; b < ns; ++b) {
        const SubPlan& S = P.subs[b];
        int tG = (int)(S.nGp / TS), tC = S.ncp / TS;
        int id0 = tG + tC, ic0 = 2 * tG + tC;
        g.push_back(MvDesc{D.M.off[b], D.M.nt[b], id0, tG, id0, tG, D.gofs[b], D.gofs[b], 0, nullptr, (int32_t)S.nG,
                           (int32_t)S.nG});
        pn.push_back(MvDesc{D.M.off[b], D.M.nt[b], ic0, tC, id0, tG, D.gofs[b], D.cofs[b], 0, nullptr, (int32_t)S.nc,
                            (int32_t)S.nG});
        pt.push_back(MvDesc{D.M.off[b], D.M.nt[b], ic0, tC, id0, tG, D.cofs[b], D.gofs[b], 0, nullptr, (int32_t)S.nc,
                            (int32_t)S.nG});
      }
      if ((st = build_mv(D.mvG, MV_SYM, g))) return st;
      if ((st = build_mv(D.mvPsiN, MV_N, pn))) return st;
      if ((st = build_mv(D.mvPsiT, MV_T, pt))) return st;
      D.g_psi_sum = D.mvG.tiles <= SMALL_MV_TILES && D.mvPsiT.tiles <= SMALL_MV_TILES && D.mvG.h.size() == D.mvPsiT.h.size() &&
                    D.mvG.max_out == D.mvPsiT.max_out;
      for (size_t q = 0; D.g_psi_sum && q < D.mvG.h.size(); ++q)
        D.g_psi_sum = D.mvG.h[q].nr == D.mvPsiT.h[q].nc && D.mvG.h[q].y_off == D.mvPsiT.h[q].y_off;
    }
    // partial-sum scratch: the largest of this level's products
    int64_t pmax = 1;
    for (MvSet* s : {&D.mvS, &D.mvG, &D.mvPsiN, &D.mvPsiT, &D.mvPre, &D.mvPreT, &D.mvPostN})
      pmax = std::max(pmax, s->partial_elems);
    if ((st = dalloc((double**)&D.partial, pmax))) return st;
    // The level-0 G product runs beside the coarse levels when it is FP32: at
    // 48^3 elasticity this took 18 us (9%) off a preconditioner apply, while
    // with an FP64 G product (twice the bytes) the overlap cost 2 us.
    // Level 0 in mixed precision sums G_i r_i and Psi_i z_Ci in the averaging
    // (two buffers), so that the G product may run on a stream of its own.
    if (li == 0 && !D.g_psi_sum && D.mfp32 && (st = dalloc((float**)&D.yl2, std::max<int64_t>(1, D.nG_flat)))) return st;
    if (li == 0 && !D.g_psi_sum && D.mfp32 && opt.side_stream &&
        (st = dalloc((double**)&D.partial_g, std::max<int64_t>(1, D.mvG.partial_elems))))
      return st;
    mark("  constraints, coarse, M mat-vecs");
    if ((st = validate_level(li, 1))) return st;
    mark("  validate (rest)");
    if ((st = join())) return st;
    if ((st = upload_fence())) return st;
    enqueue_async(li, 2);
    if (li == 0 && h_edof) start_edof();  // the next levels wait for the device
  }
  if (h_edof && !edof_job.valid()) start_edof();


  // algorithmic bytes of the level-1 products (stored lower triangles), for profiling
  alg_bytes_S = alg_bytes_G = 0.0;
  for (const SubPlan& S : plan.levels[0].subs) alg_bytes_S += 0.5 * (double)S.nG * (double)(S.nG + 1);
  alg_bytes_G = alg_bytes_S * (!lev.empty() && lev[0].mfp32 ? 4.0 : 8.0);
  alg_bytes_S *= 8.0;
  // PCG vectors
  const int64_t nif = (int64_t)plan.levels[0].iface_dofs.size();
  const int64_t ndofs = plan.levels[0].n_dofs;
  for (double** p : {&d_x, &d_r, &d_z, &d_p, &d_q, &d_g})
    if ((st = dalloc(p, std::max<int64_t>(nif, 1)))) return st;
  max_hist = std::max(opt.max_iter, 1) + 2;
  if ((st = dalloc(&d_s, S_NSCAL))) return st;
  if ((st = dalloc(&d_hist, 2 * (int64_t)max_hist))) return st;
  if ((st = dalloc(&d_dotp, DOT_BLOCKS))) return st;
  if ((st = dalloc(&d_it, 1))) return st;
  if (!h_s) HIPCHK(hipHostMalloc((void**)&h_s, sizeof(double) * 3 * S_NSCAL, hipHostMallocDefault));
  (void)ndofs;
  mark("PCG vectors");
  if ((st = join())) return st;
  if ((st = upload_fence())) return st;
  // host preparation done; the device may still be factorizing the last parts
  t_plan = now() - t0;
  if (opt.use_graph && !lev.empty() && !lev[0].P->top && (st = capture_pcg())) return st;
  st = finish_numeric();
  if (h_edof) {  // copied beside the solve; element energies wait for it
    edof_job.get();
    if (!st && !(st = dalloc(&d_edof, (int64_t)edof_n))) {
      if ((st = ensure_ustream())) return st;
      if (!ev_edof) HIPCHK(hipEventCreateWithFlags(&ev_edof, hipEventDisableTiming));
      HIPCHK(hipMemcpyAsync(d_edof, h_edof, sizeof(int32_t) * edof_n, hipMemcpyHostToDevice, ustream));
      HIPCHK(hipEventRecord(ev_edof, ustream));
    }
  }
  t_setup = now() - t0 - t_plan;
  mark("device work after the host preparation");
  trim_pool();
  if (st) return st;
  ready = true;
  return MLBDDC_OK;
}

// Host check of every index the kernels will use against the buffers they
// address, run once per set-up before any kernel touches the data: part 0
// what the assembly and the weights use, part 2 the K job, part 1 the rest
// (whether every element entry falls in a stored tile the assembly kernel
// checks itself: it skips such an entry and raises the K job's error word).
mlbddc_status Handle::validate_level(int li, int part) {
  auto bad = [&](const std::string& what) { return fail(MLBDDC_E_ARG, "internal layout check failed: " + what); };
  LevelDev& D = lev[li];
  LevelPlan& P = *D.P;
  const std::string L = "level " + std::to_string(li + 1) + ": ";
  double t_v = now();
  auto vmark = [&](const char* what) {
    if (verbose) std::fprintf(stderr, "[mlbddc check L%d] %-24s %8.2f ms\n", li + 1, what, (now() - t_v) * 1e3);
    t_v = now();
  };
  auto job_ok = [&](const Job& J) -> mlbddc_status {
    if (J.nt.empty()) return MLBDDC_OK;
    const size_t ni = J.nt.size();
    if (J.tmap_off.size() != ni || J.nlead.size() != ni || J.tslot0.size() != ni) return bad(L + "tile maps");
    int64_t lead_end = 0, trail_end = -1;  // the leading parts, then the trailing blocks, in item order without overlap
    for (size_t i = 0; i < ni; ++i) {
      if (J.off[i] < lead_end || J.nlead[i] < 0) return bad(L + "job matrix extent");
      lead_end = J.off[i] + J.nlead[i] * TE;
      if (lead_end > J.elems) return bad(L + "job matrix extent");
      if (J.tmap_off[i] >= 0) {
        const int nt = J.nt[i], e1 = J.items[i].e1;
        if (!J.items[i].sptr || J.tmap_off[i] + packed_tiles(nt) > (int64_t)J.tmap.size() || e1 > nt)
          return bad(L + "tile map extent");
        const int64_t t0 = J.off[i] + J.tslot0[i] * TE, t1 = t0 + packed_tiles(nt - e1) * TE;
        if (J.tslot0[i] < 0 || t0 < std::max(trail_end, (int64_t)0) || t1 > J.elems) return bad(L + "tile map trailing block");
        trail_end = t1;
      } else if (J.nlead[i] != packed_tiles(J.nt[i]) || J.tslot0[i] != -1) {
        return bad(L + "job matrix extent");
      }
      if (J.inv_off[i] + (int64_t)(J.items[i].e1 + J.items[i].e2) * TE > std::max<int64_t>(J.inv_elems, 1))
        return bad(L + "inverse tile extent");
      if (J.items[i].e1 + J.items[i].e2 > J.nt[i]) return bad(L + "elimination beyond the matrix");
      if ((int)J.env[i].size() != J.nt[i]) return bad(L + "envelope size");
      if (J.nt[i] >= 8192) return bad(L + "matrix too large for the task encoding");
    }
    for (size_t i = 0; i < ni; ++i)  // the first trailing block lies after every leading part
      if (J.tmap_off[i] >= 0) {
        if (J.off[i] + J.tslot0[i] * TE < lead_end) return bad(L + "tile map trailing block");
        break;
      }
    vmark("job extents");
    // per matrix (on several threads): map entries in range, the trailing block
    // packed on its own, every tile of the structure stored, and a column's rows
    // below the diagonal in its own dissection group or in higher groups
    auto item_ok = [&](size_t i) -> const char* {
      const FactorItemDesc& it = J.items[i];
      const int nt = J.nt[i];
      if (J.tmap_off[i] >= 0) {
        const int e1 = it.e1;
        const int32_t* m = J.tmap.data() + J.tmap_off[i];
        for (int c = 0; c < e1; ++c)
          for (int r = c; r < nt; ++r) {
            const int32_t q = m[tile_index(r, c, nt)];
            if (q < -1 || q >= J.nlead[i]) return "tile map entry";
          }
        for (int c = e1; c < nt; ++c)
          for (int r = c; r < nt; ++r)
            if (m[tile_index(r, c, nt)] != J.tslot0[i] + tile_index(r - e1, c - e1, nt - e1)) return "tile map trailing block";
        for (int k = 0; k < e1; ++k)  // the structure's tiles and the diagonal
          if (m[tile_index(k, k, nt)] < 0) return "tile map misses a tile";
        for (int k = 0; k < e1; ++k)
          for (int32_t q = it.sptr[k]; q < it.sptr[k + 1]; ++q)
            if (it.srow[q] > k && it.srow[q] < nt && m[tile_index(it.srow[q], k, nt)] < 0) return "tile map misses a tile";
      }
      if (it.sptr) {
        if (it.e2 != 0 || !it.gtile || !it.gheight || it.ngroups < 1 || it.gtile[0] != 0 || it.gtile[it.ngroups] != it.e1)
          return "tile structure groups";
        std::vector<int32_t> grp(it.e1, 0);
        for (int g = 0; g < it.ngroups; ++g) {
          if (it.gtile[g + 1] < it.gtile[g]) return "tile structure groups";
          for (int k = it.gtile[g]; k < it.gtile[g + 1]; ++k) grp[k] = g;
        }
        for (int k = 0; k < it.e1; ++k)
          for (int32_t q = it.sptr[k]; q < it.sptr[k + 1]; ++q) {
            const int r = it.srow[q];
            if (r <= k || r >= nt) return "tile structure rows";
            if (r < it.e1 && grp[r] != grp[k] && it.gheight[grp[r]] <= it.gheight[grp[k]])
              return "dissection groups couple out of order";
          }
      }
      return nullptr;
    };
    {
      const int T = (int)std::min<size_t>(16, std::max<size_t>(1, ni / 8));
      std::vector<const char*> whys(T, nullptr);
      parallel_run(T, [&](int t) {
        for (size_t i = ni * t / T; i < ni * (t + 1) / T && !whys[t]; ++i) whys[t] = item_ok(i);
      });
      for (const char* w : whys)
        if (w) return bad(L + w);
    }
    vmark("job matrices");
    if ((int64_t)ni >= MAX_TASK_ITEMS) return bad(L + "too many matrices for the task encoding");
    // every task against its launch kind and its matrix (launches split over threads)
    auto check = [&](size_t l0, size_t l1) -> const char* {
      for (size_t l = l0; l < l1; ++l) {
        const FactorLaunch& F = J.sched.launches[l];
        if (F.first < 0 || F.count < 0 || F.first + F.count > (int64_t)J.sched.tasks.size()) return "task range";
        for (int64_t q = F.first; q < F.first + F.count; ++q) {
          uint64_t t = J.sched.tasks[q];
          size_t it = (size_t)task_item(t);
          int r = task_r(t), c = task_s(t), kf = task_kf(t), kl = kf + task_nk(t);
          if (it >= ni) return "task item";
          int nt = J.nt[it], ee = J.items[it].e1 + J.items[it].e2;
          if (r >= nt || c > r) return "task tile";
          if (J.tmap_off[it] >= 0) {  // every tile the task reads or writes is stored
            const int32_t* m = J.tmap.data() + J.tmap_off[it];
            if (m[tile_index(r, c, nt)] < 0) return "task tile not stored";
            if (F.kind == L_INPANEL || F.kind == L_TRAIL) {
              if (kl - kf + 1 > 64 || kl >= c) return "task columns";
              for (int kk = kf; kk <= kl; ++kk)
                if (m[tile_index(r, kk, nt)] < 0 || m[tile_index(c, kk, nt)] < 0) return "task tile not stored";
            }
          }
          switch (F.kind) {
            case L_DIAG: if (r != c || c >= ee) return "diag task"; break;
            case L_PANEL: if (r <= c || c >= ee) return "panel task"; break;
            case L_INPANEL: if (kl != c - 1 || kf > kl) return "in-panel task"; break;
            case L_TRAIL: if (c <= kl || kl >= ee) return "trailing task"; break;
            default: return "task kind";
          }
        }
      }
      return nullptr;
    };
    const size_t nl = J.sched.launches.size();
    const int T = (int)std::min<size_t>(16, std::max<size_t>(1, J.sched.tasks.size() / 30000));
    std::vector<const char*> whys(T, nullptr);
    parallel_run(T, [&](int t) { whys[t] = check(nl * t / T, nl * (t + 1) / T); });
    for (const char* w : whys)
      if (w) return bad(L + w);
    vmark("job tasks");
    return MLBDDC_OK;
  };
  auto seg_ok = [&](const std::vector<DiagSeg>& v) {
    for (const DiagSeg& g : v) {
      if (g.row0 < g.col0 || (int64_t)g.row0 + g.count > (int64_t)g.nt * TS || (int64_t)g.col0 + g.count > (int64_t)g.nt * TS)
        return false;
      // a segment of a tile-mapped matrix lies on its diagonal (diagonal tiles are always stored)
      if (g.item >= 0 && (g.item >= (int32_t)D.K.nt.size() || (D.K.tmap_off[g.item] >= 0 && g.row0 != g.col0))) return false;
    }
    return true;
  };
  mlbddc_status st;
  if (part == 2) return job_ok(D.K);  // the K job's matrices and tasks
  if (part == 0) {  // what assembly and weights use
    // element maps and subdomain maps, split over threads (that every entry
    // falls in a stored tile is checked by the assembly kernel itself)
    const int64_t ne = (int64_t)P.el_local_ptr.size() - 1, ns = (int64_t)P.subs.size();
    const int T = (int)std::min<int64_t>(16, std::max<int64_t>(1, ne / 4096));
    std::vector<const char*> whys(T, nullptr);
    parallel_run(T, [&](int t) {
      for (int64_t e = ne * t / T; e < ne * (t + 1) / T; ++e) {
        int b = P.el_sub[e];
        if (b < 0 || b >= (int64_t)P.subs.size()) { whys[t] = "element subdomain"; return; }
        int64_t nK = (int64_t)D.K.nt[b] * TS;
        for (int32_t j = P.el_local_ptr[e]; j < P.el_local_ptr[e + 1]; ++j)
          if (P.el_local[j] < -1 || (int64_t)P.el_local[j] + P.ndof > nK) { whys[t] = "element map"; return; }
        if (li > 0) {
          const LevelPlan& PP = *lev[li - 1].P;
          int64_t nloc = (int64_t)(P.el_local_ptr[e + 1] - P.el_local_ptr[e]) * P.ndof;
          const SubPlan& S = PP.subs[e];
          if (nloc != S.nc || lev[li - 1].kc_off[e] + nloc * nloc > (int64_t)lev[li - 1].kc_off.back() + (int64_t)PP.subs.back().nc * PP.subs.back().nc) {
            whys[t] = "coarse element matrix";
            return;
          }
        }
      }
      for (int64_t b = ns * t / T; b < ns * (t + 1) / T; ++b) {
        if ((int64_t)P.subs[b].dofI.size() != P.subs[b].nIp) { whys[t] = "interior map size"; return; }
        for (int64_t d : P.subs[b].dofI)
          if (d < -1 || d >= P.n_dofs) { whys[t] = "interior map"; return; }
        for (int32_t g : P.subs[b].iface)
          if (g < 0 || g >= (int64_t)P.iface_dofs.size()) { whys[t] = "interface map"; return; }
      }
    });
    for (const char* w : whys)
      if (w) return bad(L + w);
    if (!seg_ok(D.ksegs_h)) return bad(L + "diagonal segment");
    for (int64_t d : P.iface_dofs)
      if (d < 0 || d >= P.n_dofs) return bad(L + "interface DOF");
    vmark("elements, subdomain maps");
    return MLBDDC_OK;
  }
  // M job, products of the apply, coarse matrices
  if ((st = job_ok(D.M))) return st;
  if (!seg_ok(D.msegs_h)) return bad(L + "diagonal segment");
  auto mv_ok = [&](const MvSet& s, const Job& J, int64_t xlen, int64_t ylen) {
    for (const MvDesc& d : s.h) {
      if (d.r0 + d.nr > d.a_nt || d.c0 + d.nc > d.a_nt) return false;
      if (s.mode == MV_SYM && (d.r0 != d.c0 || d.nr != d.nc)) return false;
      if (s.mode != MV_SYM && d.r0 < d.c0 + d.nc) return false;
      if (d.a_off + packed_tiles(d.a_nt) * TE > J.elems) return false;
      int64_t nx = (s.mode == MV_T ? d.nr : d.nc) * (int64_t)TS, ny = (s.mode == MV_T ? d.nc : d.nr) * (int64_t)TS;
      if (d.x_off + nx > xlen || d.y_off + ny > ylen) return false;
      if (d.p_off + (int64_t)d.nr * d.nc * TS > s.partial_elems) return false;
    }
    return true;
  };
  if (li == 0) {
    if (!mv_ok(D.mvS, D.K, D.nG_flat, D.nG_flat)) return bad(L + "S mat-vec");
    // tile lists: tiles inside the K job, x and y blocks inside their vectors, entries in range
    auto tl_ok = [&](const LevelDev::TileList& T, int64_t xlen, int64_t ylen) {
      for (const TileRef& t : T.t)
        if (t.a < 0 || t.a + TE > D.K.elems || t.x < 0 || t.x + TS > xlen) return false;
      for (const OutRef& o : T.o)
        if (o.y < 0 || o.y + TS > ylen || o.p0 < 0 || o.p1 < o.p0 || o.p1 > (int64_t)T.t.size()) return false;
      return true;
    };
    if (!tl_ok(D.lgiN, D.nI_flat, D.nG_flat) || !tl_ok(D.lgiT, D.nG_flat, D.nI_flat)) return bad(L + "L_GI tile list");
    for (size_t h = 0; h < D.trF.size(); ++h)
      if (!tl_ok(D.trF[h], D.nI_flat, D.nI_flat) || !tl_ok(D.trB[h], D.nI_flat, D.nI_flat)) return bad(L + "coupling tile list");
    if (D.trF.size() + 1 < D.trsv_lvl.size()) return bad(L + "coupling tile list heights");
    for (const TrsvDesc& t : D.trsv_h) {
      if (t.k0 < 0 || t.k1 <= t.k0 || t.k1 > t.a_nt || t.v_off + (int64_t)t.k1 * TS > D.nI_flat ||
          t.inv_off + (int64_t)t.k1 * TE > D.K.inv_elems || t.p_row < 0 || t.p_col < 0 ||
          t.p_row + t.k1 >= (int64_t)D.tr_rptr.size() || t.p_col + t.k1 >= (int64_t)D.tr_cptr.size())
        return bad(L + "triangular solve");
      for (int k = t.k0; k < t.k1; ++k) {
        const int32_t a0 = D.tr_rptr[t.p_row + k], a1 = D.tr_rptr[t.p_row + k + 1];
        const int32_t b0 = D.tr_cptr[t.p_col + k], b1 = D.tr_cptr[t.p_col + k + 1];
        if (a0 < 0 || a1 < a0 || a1 > (int64_t)D.tr_rcol.size() || b0 < 0 || b1 < b0 || b1 > (int64_t)D.tr_crow.size())
          return bad(L + "triangular solve lists");
        if (D.tr_rslot.size() != D.tr_rcol.size() || D.tr_cslot.size() != D.tr_crow.size())
          return bad(L + "triangular solve lists");
        for (int32_t q = a0; q < a1; ++q)
          if (D.tr_rcol[q] < 0 || D.tr_rcol[q] >= k || D.tr_rslot[q] < 0 || t.a_off + (int64_t)(D.tr_rslot[q] + 1) * TE > D.K.elems)
            return bad(L + "triangular solve row list");
        for (int32_t q = b0; q < b1; ++q)
          if (D.tr_crow[q] <= k || D.tr_crow[q] >= t.a_nt || t.v_off + (int64_t)(D.tr_crow[q] + 1) * TS > D.nI_flat ||
              D.tr_cslot[q] < 0 || t.a_off + (int64_t)(D.tr_cslot[q] + 1) * TE > D.K.elems)
            return bad(L + "triangular solve column list");
      }
    }
    if (D.trsv_lvl.empty() || D.trsv_lvl.back() != (int32_t)D.trsv_h.size()) return bad(L + "triangular solve heights");
  } else {
    if (!mv_ok(D.mvPre, D.K, D.nI_flat, D.nI_flat)) return bad(L + "interior mat-vec");
    if (!P.top && (!mv_ok(D.mvPreT, D.K, D.nI_flat, D.nG_flat) || !mv_ok(D.mvPostN, D.K, D.nG_flat, D.nI_flat)))
      return bad(L + "correction mat-vec");
  }
  if (!P.top) {
    if (!mv_ok(D.mvG, D.M, D.nG_flat, D.nG_flat)) return bad(L + "G mat-vec");
    if (!mv_ok(D.mvPsiN, D.M, D.nG_flat, D.nC_flat)) return bad(L + "Psi^T mat-vec");
    if (!mv_ok(D.mvPsiT, D.M, D.nC_flat, D.nG_flat)) return bad(L + "Psi mat-vec");
    {
      int64_t rows = 0, cmp = 0;
      for (size_t b = 0; b < D.kcd_h.size(); ++b) {
        const KcDesc& k = D.kcd_h[b];
        if ((int64_t)k.p_c0 * TS + k.nc > (int64_t)k.p_nt * TS || k.nc > D.max_nc || k.rho_off != rows || k.out_off != cmp ||
            k.p_off + packed_tiles(k.p_nt) * TE > D.M.elems || k.p_nt != D.M.nt[b])
          return bad(L + "coarse matrix descriptor");
        rows += k.nc;
        cmp += (int64_t)k.nc * k.nc;
      }
      if (rows != (int64_t)D.cons_h.size()) return bad(L + "constraint rows vs coarse DOFs");
    }
    for (const CopyDesc& c : D.copy_h)
      if (c.src_t0 + c.nblk > c.src_nt || c.nblk > c.dst_nt || c.src_off + packed_tiles(c.src_nt) * TE > D.K.elems ||
          c.dst_off + packed_tiles(c.dst_nt) * TE > D.M.elems)
        return bad(L + "copy descriptor");
    for (const ConsDesc& c : D.cons_h) {
      int32_t mx = -1;
      if (c.ptr0 < 0 || c.ptr1 < c.ptr0 || c.ptr1 > (int32_t)D.ccols_h.size()) return bad(L + "constraint descriptor");
      for (int32_t q = c.ptr0; q < c.ptr1; ++q) mx = std::max(mx, D.ccols_h[q]);
      if (c.kdiag_off + packed_tiles(c.k_nt) * TE > D.K.elems || (int64_t)c.k_g0 + mx >= (int64_t)c.k_nt * TS ||
          c.p_off + packed_tiles(c.p_nt) * TE > D.M.elems)
        return bad(L + "constraint descriptor");
    }
    for (size_t b = 0; b < P.subs.size(); ++b) {
      const SubPlan& S = P.subs[b];
      for (int32_t col : S.crow_col)
        if (col >= S.nG) return bad(L + "constraint column");
      for (int32_t c : S.coarse)
        if (c < 0 || c >= P.n_coarse) return bad(L + "coarse map");
      if (S.nGp + S.nc > (int64_t)D.M.nt[b] * TS) return bad(L + "constraint rows");
    }
  }
  return MLBDDC_OK;
}

// Numeric set-up of level li, first part: assemble K (FP64 or FP32), take
// the interface weights from its diagonal, factor the K job.  Queued on the
// library stream only; errors are collected by finish_numeric().
mlbddc_status Handle::enqueue_K(int li, bool zero) {
  mlbddc_status st;
  if ((st = enqueue_K_assembly(li, zero))) return st;
  if ((st = enqueue_K_factor(li))) return st;
  return enqueue_weights(li);
}

mlbddc_status Handle::enqueue_K_assembly(int li, bool zero) {
  mlbddc_status st;
  LevelDev& D = lev[li];
  LevelPlan& P = *D.P;
  // assemble K
  if (zero && (st = zero_async(D.K.buf, (size_t)D.K.elems * (D.kfp32 ? 4 : 8), stream))) return st;
  HIPCHK(hipMemsetAsync(D.K.d_err + 2, 0, sizeof(int32_t), stream));
  for (int c = 0; c < P.n_colors; ++c) {
    int64_t n = D.color_ptr[c + 1] - D.color_ptr[c];
    const int64_t* el = D.d_elems_by_color + D.color_ptr[c];
    const double* kref = li == 0 ? d_Kref : nullptr;
    const double* ekc = li == 0 ? nullptr : lev[li - 1].kc_compact;
    if (D.kfp32)
      launch_assemble<float>(stream, el, n, D.d_el_local_ptr, D.d_el_local, P.ndof, D.d_el_sub, D.d_sub_off, D.d_sub_nt, kref,
                             d_scale, D.d_ekc_off, ekc, (float*)D.K.buf, D.K.d_tmap, D.K.d_tmap_off, D.K.d_err + 2);
    else
      launch_assemble<double>(stream, el, n, D.d_el_local_ptr, D.d_el_local, P.ndof, D.d_el_sub, D.d_sub_off, D.d_sub_nt, kref,
                              d_scale, D.d_ekc_off, ekc, (double*)D.K.buf, D.K.d_tmap, D.K.d_tmap_off,
                              D.K.d_err + 2);
  }
  if (D.kfp32)
    launch_set_diag<float>(stream, D.d_ksegs, (int64_t)D.ksegs_h.size(), D.kseg_max, (float*)D.K.buf, D.K.d_tmap,
                           D.K.d_tmap_off);
  else
    launch_set_diag<double>(stream, D.d_ksegs, (int64_t)D.ksegs_h.size(), D.kseg_max, (double*)D.K.buf, D.K.d_tmap,
                            D.K.d_tmap_off);
  // the assembled (sub-assembled) interface diagonal, kept for the weights:
  // the factorization overwrites it with that of the Schur complement
  if (!P.top) {
    if (opt.weights == MLBDDC_W_MULTIPLICITY) launch_fill(stream, D.nG_flat, 1.0, D.gd);
    else if (D.kfp32) launch_gather64<float>(stream, D.nG_flat, D.d_gdiag_pos, (const float*)D.K.buf, D.gd);
    else launch_gather64<double>(stream, D.nG_flat, D.d_gdiag_pos, (const double*)D.K.buf, D.gd);
  }
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

mlbddc_status Handle::enqueue_K_factor(int li) {
  LevelDev& D = lev[li];
  return factor(D.K, D.P->level, false);
}

// Weights D_i = d_i / sum_j d_j per interface DOF from the diagonal saved by
// the assembly (needs the flat layouts, so it is queued after them).
mlbddc_status Handle::enqueue_weights(int li) {
  LevelDev& D = lev[li];
  LevelPlan& P = *D.P;
  if (P.top) return MLBDDC_OK;
  const int64_t nif = (int64_t)P.iface_dofs.size();
  launch_seg_reduce<double>(stream, nif, D.d_gptr, D.d_glist, nullptr, D.gd, D.rhat, 0.0);
  launch_gather<double, double>(stream, D.nG_flat, D.d_gidx, nullptr, D.rhat, D.gd2);
  launch_ratio(stream, D.nG_flat, D.gd, D.gd2, D.d_gidx, D.d_w);
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

// Second part: the constrained local problems (M job) and the coarse
// matrices Psi^T S Psi that the next level assembles.
mlbddc_status Handle::enqueue_rest(int li, bool zero) {
  mlbddc_status st;
  LevelDev& D = lev[li];
  LevelPlan& P = *D.P;
  if (P.top) return MLBDDC_OK;
  // preconditioner matrices
  if (zero && (st = zero_async(D.M.buf, (size_t)D.M.elems * (D.mfp32 ? 4 : 8), stream))) return st;
  if (D.kfp32) {  // K is FP32 only when M is FP32
    launch_copy_block<float, float>(stream, D.d_copy, P.n_sub, D.copy_max, (const float*)D.K.buf, (float*)D.M.buf);
    launch_constraints<float, float>(stream, D.d_cons, (int64_t)D.cons_h.size(), D.d_ccols, (const float*)D.K.buf,
                                     (float*)D.M.buf, D.d_rho);
    launch_set_diag<float>(stream, D.d_msegs, (int64_t)D.msegs_h.size(), D.mseg_max, (float*)D.M.buf);
  } else if (D.mfp32) {
    launch_copy_block<double, float>(stream, D.d_copy, P.n_sub, D.copy_max, (const double*)D.K.buf, (float*)D.M.buf);
    launch_constraints<double, float>(stream, D.d_cons, (int64_t)D.cons_h.size(), D.d_ccols, (const double*)D.K.buf,
                                      (float*)D.M.buf, D.d_rho);
    launch_set_diag<float>(stream, D.d_msegs, (int64_t)D.msegs_h.size(), D.mseg_max, (float*)D.M.buf);
  } else {
    launch_copy_block<double, double>(stream, D.d_copy, P.n_sub, D.copy_max, (const double*)D.K.buf, (double*)D.M.buf);
    launch_constraints<double, double>(stream, D.d_cons, (int64_t)D.cons_h.size(), D.d_ccols, (const double*)D.K.buf,
                                       (double*)D.M.buf, D.d_rho);
    launch_set_diag<double>(stream, D.d_msegs, (int64_t)D.msegs_h.size(), D.mseg_max, (double*)D.M.buf);
  }
  HIPCHK(hipGetLastError());
  if ((st = factor(D.M, P.level, true))) return st;
  // K_Ci = Psi^T S Psi = A^{-1} - W
  if (D.mfp32) launch_coarse_matrix<float>(stream, D.d_kcd, P.n_sub, D.max_nc, (const float*)D.M.buf, D.d_rho, D.kc_compact);
  else launch_coarse_matrix<double>(stream, D.d_kcd, P.n_sub, D.max_nc, (const double*)D.M.buf, D.d_rho, D.kc_compact);
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

// Wait for the queued numeric set-up and report the first factorization
// that met a non-positive pivot (levels in order, K job before M job).
mlbddc_status Handle::finish_numeric() {
  // every job's error words copied behind the last job, then one wait
  const size_t nw = 6 * lev.size();
  if (h_err_cap < nw) {
    if (h_err) (void)hipHostFree(h_err);
    h_err = nullptr;
    HIPCHK(hipHostMalloc((void**)&h_err, sizeof(int32_t) * nw, hipHostMallocDefault));
    h_err_cap = nw;
  }
  for (size_t li = 0; li < lev.size(); ++li)
    for (int j = 0; j < 2; ++j) {
      const Job& J = j == 0 ? lev[li].K : lev[li].M;
      int32_t* e = h_err + 6 * li + 3 * j;
      e[0] = e[1] = e[2] = 0;
      if (J.d_err) HIPCHK(hipMemcpyAsync(e, J.d_err, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    }
  HIPCHK(hipStreamSynchronize(stream));
  for (size_t li = 0; li < lev.size(); ++li)
    for (int j = 0; j < 2; ++j) {
      const int32_t* e = h_err + 6 * li + 3 * j;
      if (j == 0 && e[2] != 0)
        return fail(MLBDDC_E_ARG, "internal layout check failed: level " + std::to_string(lev[li].P->level) +
                                      ": element entry in an unstored tile");
      if (e[0] != 0) {
        const int level = lev[li].P->level, sub = e[0] - 1;
        if (j == 1) return fail(MLBDDC_E_SINGULAR_CONSTRAINTS, "constrained local problem is singular", level, sub, e[1]);
        return fail(MLBDDC_E_NOT_SPD, "non-positive pivot in a subdomain factorization", level, sub, e[1]);
      }
    }
  return MLBDDC_OK;
}

// Whole numeric set-up on an existing plan (coefficient updates).
mlbddc_status Handle::numeric() {
  double t0 = now();
  mlbddc_status st;
  for (int li = 0; li < (int)lev.size(); ++li) {
    if ((st = enqueue_K(li, true))) return st;
    if ((st = enqueue_rest(li, true))) return st;
  }
  st = finish_numeric();
  t_setup = now() - t0;
  if (st) return st;
  ready = true;
  return MLBDDC_OK;
}

// --------------------------------------------------------------------- apply
// The elimination of the constrained problems leaves -G_i and -Psi_i in the
// M job (its second phase reads the first phase's trailing block with the
// opposite sign instead of negating it): every product with those blocks
// takes alpha = MSIGN.
constexpr double MSIGN = -1.0;

mlbddc_status Handle::apply_interface(int li, const double* rhat, double* zhat, const DotFinish* ds, bool r_copied) {
  LevelDev& D = lev[li];
  LevelPlan& P = *D.P;
  mlbddc_status st;
  // r_i = D_i R_i r^
  if (!r_copied) {
    if (D.mfp32) launch_gather<double, float>(stream, D.nG_flat, D.d_gidx, D.d_w, rhat, (float*)D.rl);
    else launch_gather<double, double>(stream, D.nG_flat, D.d_gidx, D.d_w, rhat, (double*)D.rl);
  }
  // y_i = G_i r_i needs no coarse correction: on level 0 it runs on a stream
  // of its own beside the coarse correction (Psi^T r, the coarse levels,
  // Psi z_C), which takes less time than this product
  const bool g_side = D.partial_g != nullptr;
  if (g_side) {
    if (!gstream) {
      HIPCHK(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&ev_gfork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev_gjoin, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(ev_gfork, stream));
    HIPCHK(hipStreamWaitEvent(gstream, ev_gfork, 0));
    const int gcls = li == 0 ? MLBDDC_PROF_PRECOND_MV : -1;
    if (D.mfp32)
      run_mv<float, float, float>(D.mvG, D.M, (const float*)D.rl, (float*)D.yl, MSIGN, false, D.partial_g, gstream, gcls, alg_bytes_G);
    else
      run_mv<double, double, double>(D.mvG, D.M, (const double*)D.rl, (double*)D.yl, MSIGN, false, D.partial_g, gstream, gcls,
                                     alg_bytes_G);
    HIPCHK(hipEventRecord(ev_gjoin, gstream));
  }
  // r_C = sum R_Ci^T Psi_i^T r_i
  if (D.mfp32) run_mv<float, float, double>(D.mvPsiN, D.M, (const float*)D.rl, D.rcl, MSIGN, false, D.partial);
  else run_mv<double, double, double>(D.mvPsiN, D.M, (const double*)D.rl, D.rcl, MSIGN, false, D.partial);
  launch_seg_reduce<double>(stream, P.n_coarse, D.d_cptr, D.d_clist, nullptr, D.rcl, D.rC, 0.0);
  // coarse correction: the next level
  if ((st = apply_full(li + 1, D.rC, D.zC))) return st;
  // y_i = G_i r_i + Psi_i R_Ci z_C
  if (D.mfp32) {
    launch_gather<double, float>(stream, D.nC_flat, D.d_cidx, nullptr, D.zC, (float*)D.zcl);
    if (D.g_psi_sum) {
      launch_tile_mv_sum<float, float, float>(stream, MV_SYM, D.mvG.d, MV_T, D.mvPsiT.d, (int32_t)D.mvG.h.size(), D.mvG.max_out,
                                              (const float*)D.M.buf, (const float*)D.rl, (const float*)D.zcl, (float*)D.yl, MSIGN,
                                              false);
    } else if (D.yl2) {
      // Psi_i z_Ci into a buffer of its own (while the G product may still
      // run beside); the averaging below sums both
      run_mv<float, float, float>(D.mvPsiT, D.M, (const float*)D.zcl, (float*)D.yl2, MSIGN, false, D.partial);
      if (g_side) HIPCHK(hipStreamWaitEvent(stream, ev_gjoin, 0));
      else
        run_mv<float, float, float>(D.mvG, D.M, (const float*)D.rl, (float*)D.yl, MSIGN, false, D.partial, nullptr,
                                    li == 0 ? MLBDDC_PROF_PRECOND_MV : -1, alg_bytes_G);
    } else {
      run_mv<float, float, float>(D.mvG, D.M, (const float*)D.rl, (float*)D.yl, MSIGN, false, D.partial, nullptr,
                                  li == 0 ? MLBDDC_PROF_PRECOND_MV : -1, alg_bytes_G);
      run_mv<float, float, float>(D.mvPsiT, D.M, (const float*)D.zcl, (float*)D.yl, MSIGN, true, D.partial);
    }
    const float* y2 = D.yl2 ? (const float*)D.yl2 : nullptr;
    if (ds)  // with rhat.zhat and its scalar step
      launch_seg_reduce_dot<float>(stream, (int64_t)P.iface_dofs.size(), D.d_gptr, D.d_glist, D.d_w, (const float*)D.yl, zhat,
                                   rhat, d_dotp, d_s, ds->slot, ds->step, d_hist, d_it, ds->rtol2, y2);
    else
      launch_seg_reduce<float>(stream, (int64_t)P.iface_dofs.size(), D.d_gptr, D.d_glist, D.d_w, (const float*)D.yl, zhat, 0.0,
                               y2);
  } else {
    launch_gather<double, double>(stream, D.nC_flat, D.d_cidx, nullptr, D.zC, (double*)D.zcl);
    if (D.g_psi_sum) {
      launch_tile_mv_sum<double, double, double>(stream, MV_SYM, D.mvG.d, MV_T, D.mvPsiT.d, (int32_t)D.mvG.h.size(),
                                                 D.mvG.max_out, (const double*)D.M.buf, (const double*)D.rl,
                                                 (const double*)D.zcl, (double*)D.yl, MSIGN, false);
    } else {
      if (g_side) HIPCHK(hipStreamWaitEvent(stream, ev_gjoin, 0));
      else
        run_mv<double, double, double>(D.mvG, D.M, (const double*)D.rl, (double*)D.yl, MSIGN, false, D.partial, nullptr,
                                       li == 0 ? MLBDDC_PROF_PRECOND_MV : -1, alg_bytes_G);
      run_mv<double, double, double>(D.mvPsiT, D.M, (const double*)D.zcl, (double*)D.yl, MSIGN, true, D.partial);
    }
    if (ds)
      launch_seg_reduce_dot<double>(stream, (int64_t)P.iface_dofs.size(), D.d_gptr, D.d_glist, D.d_w, (const double*)D.yl,
                                    zhat, rhat, d_dotp, d_s, ds->slot, ds->step, d_hist, d_it, ds->rtol2);
    else
      launch_seg_reduce<double>(stream, (int64_t)P.iface_dofs.size(), D.d_gptr, D.d_glist, D.d_w, (const double*)D.yl, zhat,
                                0.0);
  }
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

// One step of the level-li preconditioner on a whole level vector (interior
// pre-correction, interface BDDC, post-correction), or the top solve.
mlbddc_status Handle::apply_full(int li, const double* r, double* z) {
  LevelDev& D = lev[li];
  LevelPlan& P = *D.P;
  mlbddc_status st;
  const bool f32 = D.kfp32;
  // u_I = K_II^{-1} r_I  (the stored block is -K_II^{-1})
  if (f32) {
    launch_gather<double, float>(stream, D.nI_flat, D.d_iidx, nullptr, r, (float*)D.rI);
    run_mv<float, float, float>(D.mvPre, D.K, (const float*)D.rI, (float*)D.uI, -1.0, false, D.partial);
  } else {
    launch_gather<double, double>(stream, D.nI_flat, D.d_iidx, nullptr, r, (double*)D.rI);
    run_mv<double, double, double>(D.mvPre, D.K, (const double*)D.rI, (double*)D.uI, -1.0, false, D.partial);
  }
  if (P.top) {
    if (f32) launch_scatter<float, double>(stream, D.nI_flat, D.d_iidx, (const float*)D.uI, z);
    else launch_scatter<double, double>(stream, D.nI_flat, D.d_iidx, (const double*)D.uI, z);
    HIPCHK(hipGetLastError());
    return MLBDDC_OK;
  }
  // r^ = r_G - sum R^T K_GI u_I   (the stored block is -K_II^{-1} K_IG)
  const int64_t nif = (int64_t)P.iface_dofs.size();
  if (f32) run_mv<float, float, double>(D.mvPreT, D.K, (const float*)D.rI, D.tG, 1.0, false, D.partial);
  else run_mv<double, double, double>(D.mvPreT, D.K, (const double*)D.rI, D.tG, 1.0, false, D.partial);
  launch_gather_seg(stream, nif, D.d_iface_dofs, r, D.d_gptr, D.d_glist, D.tG, D.rhat);
  if ((st = apply_interface(li, D.rhat, D.zhat))) return st;
  // z_I = u_I - K_II^{-1} K_IG z_G
  if (f32) {
    launch_gather<double, float>(stream, D.nG_flat, D.d_gidx, nullptr, D.zhat, (float*)D.zG);
    run_mv<float, float, float>(D.mvPostN, D.K, (const float*)D.zG, (float*)D.uI, 1.0, true, D.partial);
    launch_scatter2<float>(stream, D.nI_flat, D.d_iidx, (const float*)D.uI, nif, D.d_iface_dofs, D.zhat, z);
  } else {
    launch_gather<double, double>(stream, D.nG_flat, D.d_gidx, nullptr, D.zhat, (double*)D.zG);
    run_mv<double, double, double>(D.mvPostN, D.K, (const double*)D.zG, (double*)D.uI, 1.0, true, D.partial);
    launch_scatter2<double>(stream, D.nI_flat, D.d_iidx, (const double*)D.uI, nif, D.d_iface_dofs, D.zhat, z);
  }
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

mlbddc_status Handle::schur(const double* x, double* y, const DotFinish* ds, bool x_copied) {
  LevelDev& D = lev[0];
  if (!x_copied) launch_gather<double, double>(stream, D.nG_flat, D.d_gidx, nullptr, x, D.gd);
  run_mv<double, double, double>(D.mvS, D.K, D.gd, D.gd2, 1.0, false, D.partial, nullptr, MLBDDC_PROF_SCHUR_MV, alg_bytes_S);
  const int64_t nif = (int64_t)D.P->iface_dofs.size();
  if (ds)  // with x.y and its scalar step
    launch_seg_reduce_dot<double>(stream, nif, D.d_gptr, D.d_glist, nullptr, D.gd2, y, x, d_dotp, d_s, ds->slot, ds->step,
                                  d_hist, d_it, ds->rtol2);
  else
    launch_seg_reduce<double>(stream, nif, D.d_gptr, D.d_glist, nullptr, D.gd2, y, 0.0);
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

mlbddc_status Handle::schur_noalloc(const double* x, double* y) {
  LevelDev& D = lev[0];
  if (!scratch_ptr) return fail(MLBDDC_E_STATE, "apply_schur_noalloc: no scratch address on this device");
  const int64_t n = D.nG_flat, n_al = round_up(n, 32);
  const size_t need = sizeof(double) * (size_t)(2 * n_al);
  if (need > SCRATCH_BYTES)
    return fail(MLBDDC_E_ARG, "apply_schur_noalloc: the interface work vectors need " + std::to_string(need) +
                                  " bytes, more than the " + std::to_string(SCRATCH_BYTES) + "-byte device scratch");
  double* xs = (double*)scratch_ptr;
  double* ys = xs + n_al;
  // every flat position of xs is written (0 at padding); the product writes
  // every entry of ys that the segmented sum reads
  launch_gather<double, double>(stream, n, D.d_gidx, nullptr, x, xs);
  launch_tile_mv_sum<double, double, double>(stream, MV_SYM, D.mvS.d, MV_SYM, nullptr, (int32_t)D.mvS.h.size(), D.mvS.max_out,
                                             (const double*)D.K.buf, xs, nullptr, ys, 1.0, false);
  launch_seg_reduce<double>(stream, (int64_t)D.P->iface_dofs.size(), D.d_gptr, D.d_glist, nullptr, ys, y, 0.0);
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

mlbddc_status Handle::condense(const double* f, double* g) {
  LevelDev& D = lev[0];
  const int64_t nif = (int64_t)D.P->iface_dofs.size();
  launch_gather<double, double>(stream, D.nI_flat, D.d_iidx, nullptr, f, D.wI);
  run_trsv(D, false);
  launch_tile_list_mv(stream, false, D.lgiN.dt, (int64_t)D.lgiN.t.size(), D.lgiN.dout, (int64_t)D.lgiN.o.size(),
                      (const double*)D.K.buf, D.wI, D.tl_partial, D.tG, -1.0, false);
  launch_gather<double, double>(stream, nif, D.d_iface_dofs, nullptr, f, g);
  launch_seg_reduce<double>(stream, nif, D.d_gptr, D.d_glist, nullptr, D.tG, g, 1.0);
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

mlbddc_status Handle::recover(const double* uhat, double* u) {
  LevelDev& D = lev[0];
  const int64_t nif = (int64_t)D.P->iface_dofs.size();
  launch_gather<double, double>(stream, D.nG_flat, D.d_gidx, nullptr, uhat, D.gd);
  launch_tile_list_mv(stream, true, D.lgiT.dt, (int64_t)D.lgiT.t.size(), D.lgiT.dout, (int64_t)D.lgiT.o.size(),
                      (const double*)D.K.buf, D.gd, D.tl_partial, D.wI, -1.0, true);
  run_trsv(D, true);
  launch_scatter<double, double>(stream, D.nI_flat, D.d_iidx, D.wI, u);
  launch_scatter_idx(stream, nif, D.d_iface_dofs, uhat, u);
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

// Lanczos estimates from the CG coefficients (tridiagonal eigenvalues by bisection).
static void lanczos(const std::vector<double>& al, const std::vector<double>& be, double& lo, double& hi) {
  const int k = (int)al.size();
  lo = hi = 0.0;
  if (k == 0) return;
  std::vector<double> d(k), e(k, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < k) e[j] = std::sqrt(std::max(be[j], 0.0)) / al[j];
  }
  double gl = 1e300, gh = -1e300;
  for (int j = 0; j < k; ++j) {
    double rad = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < k ? std::fabs(e[j]) : 0.0);
    gl = std::min(gl, d[j] - rad);
    gh = std::max(gh, d[j] + rad);
  }
  auto count_below = [&](double x) {  // Sturm count of eigenvalues < x
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int j = 1; j < k; ++j) {
      double qq = q == 0.0 ? 1e-300 : q;
      q = d[j] - x - e[j - 1] * e[j - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  auto kth = [&](int idx) {
    double a = gl, b = gh;
    for (int it = 0; it < 200; ++it) {
      double m = 0.5 * (a + b);
      if (count_below(m) > idx) b = m; else a = m;
    }
    return 0.5 * (a + b);
  };
  lo = kth(0);
  hi = kth(k - 1);
}

// One PCG iteration after the first (first == false) or the first one:
//   [p = z + beta p]   (not in the first iteration)
//   q = S^ p;  p.q and alpha = rz / p.q
//   x += alpha p;  r -= alpha q with r.r, then the stopping test
//   z = M r;  rz_new = r.z, then beta = rz_new / rz for the next iteration
// Each dot product ends in one single-block launch that also does the scalar
// step after it; p.q and r.z take their partial sums in the segmented sums
// that finish q and z.  The host reads rr (and p.q) after the iteration.
mlbddc_status Handle::pcg_body(bool first) {
  mlbddc_status st;
  const int64_t n = (int64_t)lev[0].P->iface_dofs.size();
  LevelDev& D = lev[0];
  // p and r are written to their subdomain copies by the updates themselves
  // (the padding entries of the copies keep the zeros of the first gathers)
  if (!first) launch_pcg_update_p(stream, n, d_p, d_z, d_s, D.d_gptr, D.d_glist, D.gd);
  const DotFinish pq{S_PQ, DOT_ALPHA, 0.0}, rz{S_RZNEW, DOT_BETA, 0.0};
  if ((st = schur(d_p, d_q, &pq, !first))) return st;
  if (D.mfp32)
    launch_pcg_update_xr_check<float>(stream, n, d_x, d_r, d_p, d_q, d_dotp, d_s, opt.rtol * opt.rtol, D.d_gptr, D.d_glist,
                                      D.d_w, (float*)D.rl);
  else
    launch_pcg_update_xr_check<double>(stream, n, d_x, d_r, d_p, d_q, d_dotp, d_s, opt.rtol * opt.rtol, D.d_gptr, D.d_glist,
                                       D.d_w, (double*)D.rl);
  if ((st = apply_interface(0, d_r, d_z, &rz, true))) return st;
  HIPCHK(hipGetLastError());
  return MLBDDC_OK;
}

// With graphs the whole solve runs on an internal stream ordered after the
// caller's stream (the caller's stream may be the null stream, which cannot
// be captured); the caller's stream waits for it at the end.
// Capture one PCG iteration (a non-first pcg_body) as a HIP graph on the
// internal stream; the set-up does it while the device factorizes, so that a
// solve does not wait for it.
mlbddc_status Handle::capture_pcg() {
  if (!cap) {
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  }
  if (gexec) return MLBDDC_OK;
  hipStream_t user = stream;
  stream = cap;
  hipGraph_t graph = nullptr;
  hipError_t be = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  mlbddc_status cst = be == hipSuccess ? pcg_body(false) : MLBDDC_OK;
  hipError_t ce = be == hipSuccess ? hipStreamEndCapture(stream, &graph) : hipSuccess;
  stream = user;
  if (be != hipSuccess) return herr("hipStreamBeginCapture", be);
  if (cst) {
    if (graph) (void)hipGraphDestroy(graph);
    return cst;
  }
  if (ce != hipSuccess) return herr("hipStreamEndCapture", ce);
  hipError_t ie = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    gexec = nullptr;
    return herr("hipGraphInstantiate", ie);
  }
  return MLBDDC_OK;
}

mlbddc_status Handle::solve(const double* f, double* u, const double* u0, mlbddc_stats* stt) {
  if (!opt.use_graph) return solve_on_stream(f, u, u0, stt);
  if (!cap) {
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  }
  hipStream_t user = stream;
  HIPCHK(hipEventRecord(ev_in, user));
  HIPCHK(hipStreamWaitEvent(cap, ev_in, 0));
  stream = cap;
  mlbddc_status st = solve_on_stream(f, u, u0, stt);
  stream = user;
  HIPCHK(hipEventRecord(ev_out, cap));
  HIPCHK(hipStreamWaitEvent(user, ev_out, 0));
  return st;
}

mlbddc_status Handle::solve_on_stream(const double* f, double* u, const double* u0, mlbddc_stats* stt) {
  double t0 = now();
  mlbddc_status st;
  LevelDev& D = lev[0];
  const int64_t n = (int64_t)D.P->iface_dofs.size();
  if ((st = condense(f, d_g))) return st;
  // x0
  if (u0) launch_gather<double, double>(stream, n, D.d_iface_dofs, nullptr, u0, d_x);
  else launch_fill(stream, n, 0.0, d_x);
  // r = g - S x0
  if (u0) {
    if ((st = schur(d_x, d_r))) return st;
    launch_axpby(stream, n, 1.0, d_g, -1.0, d_r);
  } else {
    HIPCHK(hipMemcpyAsync(d_r, d_g, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
  }
  launch_dot(stream, n, d_g, d_g, d_dotp, DOT_BLOCKS, d_s + S_GG);
  launch_dot(stream, n, d_r, d_r, d_dotp, DOT_BLOCKS, d_s + S_RR);
  HIPCHK(hipMemcpyAsync(h_s, d_s, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, stream));
  for (hipEvent_t& e : ev_snap)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev_snap[0], stream));
  // z0 = M^-1 r0, <r0,z0> and p0 = z0 are queued before the host reads the
  // initial norms, so the device works while the host waits; they write only
  // z, p and the RZ scalar, which nothing reads if r0 already meets the
  // tolerance (a zero r0 gives a zero z0).
  if ((st = apply_interface(0, d_r, d_z))) return st;
  launch_dot(stream, n, d_r, d_z, d_dotp, DOT_BLOCKS, d_s + S_RZ);
  HIPCHK(hipMemcpyAsync(d_p, d_z, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
  launch_set_int(stream, d_it, 0);
  launch_fill(stream, 1, 0.0, d_s + S_DONE);
  HIPCHK(hipEventSynchronize(ev_snap[0]));
  const double gnorm = std::sqrt(h_s[S_GG]);
  // a non-finite condensed right-hand side (or initial residual) is a breakdown before the first step
  bool breakdown = !std::isfinite(gnorm) || !std::isfinite(h_s[S_RR]);
  double rel = breakdown ? NAN : gnorm > 0 ? std::sqrt(h_s[S_RR]) / gnorm : 0.0;
  int it = 0;
  bool conv = !breakdown && rel < opt.rtol;
  if (!conv && !breakdown) {
    // Iteration k+1 is normally queued before the host reads iteration k's
    // scalars (snapshot k&1), so the device does not wait for the host; once
    // the device flags convergence or breakdown a queued iteration changes
    // nothing (its products recompute the same scalars).
    auto issue = [&](int k) -> mlbddc_status {
      mlbddc_status sb;
      if (k == 0 || !opt.use_graph) {
        if ((sb = pcg_body(k == 0))) return sb;
      } else {
        if (!gexec && (sb = capture_pcg())) return sb;
        HIPCHK(hipGraphLaunch(gexec, stream));
      }
      HIPCHK(hipMemcpyAsync(h_s + S_NSCAL * (1 + (k & 1)), d_s, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, stream));
      HIPCHK(hipEventRecord(ev_snap[k & 1], stream));
      return MLBDDC_OK;
    };
    if ((st = issue(0))) return st;
    int issued = 1;
    std::vector<double> rels;  // relative residuals read so far
    while (true) {
      // Queue the next iteration before reading the one in flight, unless the
      // residual trend (geometric, over the last three iterations) says that
      // the one in flight probably meets the tolerance: a queued iteration
      // would then be wasted work, and waiting for the host costs less.
      bool ahead = issued == it + 1 && issued < opt.max_iter;
      const size_t m = rels.size();
      if (ahead && m >= 2) {
        const double ratio = m >= 4 ? std::cbrt(rels[m - 1] / rels[m - 4]) : rels[m - 1] / rels[m - 2];
        if (rels[m - 1] * ratio < opt.rtol) ahead = false;
      }
      if (ahead) {
        if ((st = issue(issued))) return st;
        ++issued;
      }
      HIPCHK(hipEventSynchronize(ev_snap[it & 1]));
      const double* hs = h_s + S_NSCAL * (1 + (it & 1));
      ++it;
      rel = std::sqrt(hs[S_RR]) / gnorm;
      rels.push_back(rel);
      if (hs[S_DONE] != 0.0) {
        if (!(hs[S_PQ] > 0.0) || !std::isfinite(hs[S_PQ])) breakdown = true;
        else conv = true;
        break;
      }
      if (it >= opt.max_iter) break;
      if (issued == it) {  // held back and not converged: queue the next one now
        if ((st = issue(issued))) return st;
        ++issued;
      }
    }
  }
  if ((st = recover(d_x, u))) return st;
  // history for the Lanczos estimate
  std::vector<double> hist(2 * (size_t)std::max(it, 1));
  if (it > 0) HIPCHK(hipMemcpyAsync(hist.data(), d_hist, sizeof(double) * 2 * it, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (stt) {
    // a breakdown iteration records no step: its alpha is not part of the history
    const int nal = breakdown ? it - 1 : it;
    std::vector<double> al, be;
    for (int j = 0; j < nal; ++j) al.push_back(hist[2 * j]);
    for (int j = 0; j + 1 < nal; ++j) be.push_back(hist[2 * j + 1]);
    double lo, hi;
    lanczos(al, be, lo, hi);
    stt->iterations = it;
    stt->converged = conv ? 1 : 0;
    stt->rel_res = rel;
    stt->lambda_min = lo;
    stt->lambda_max = hi;
    stt->t_plan = t_plan;
    stt->t_setup_num = t_setup;
    stt->t_solve = now() - t0;
  }
  if (breakdown) return fail(MLBDDC_E_BREAKDOWN, "PCG breakdown: p^T S p <= 0 or not finite");
  if (!conv) return fail(MLBDDC_E_NOT_CONVERGED, "PCG did not reach the tolerance");
  return MLBDDC_OK;
}

}  // namespace mlbddc

// ======================================================================= ABI
using mlbddc::Handle;

struct mlbddc_handle_s {
  Handle h;
};

static mlbddc::Error g_create_error;

extern "C" {

const char* mlbddc_status_string(mlbddc_status code) {
  switch (code) {
    case MLBDDC_OK: return "ok";
    case MLBDDC_E_ARG: return "invalid argument";
    case MLBDDC_E_HIP: return "HIP runtime error";
    case MLBDDC_E_NOMEM: return "out of memory";
    case MLBDDC_E_STATE: return "call out of order";
    case MLBDDC_E_NOT_SPD: return "subdomain matrix not positive definite";
    case MLBDDC_E_SINGULAR_CONSTRAINTS: return "constrained local problem singular";
    case MLBDDC_E_NOT_CONVERGED: return "PCG did not converge";
    case MLBDDC_E_BREAKDOWN: return "PCG breakdown";
    case MLBDDC_E_NO_DEVICE: return "no HIP device";
  }
  return "unknown status";
}

void mlbddc_default_options(mlbddc_options* o) {
  if (!o) return;
  o->precision = MLBDDC_FP64;
  o->rtol = 1e-8;
  o->max_iter = 1000;
  o->weights = MLBDDC_W_STIFFNESS;
  o->use_graph = 0;
  o->panel_tiles = 0;
  o->device = 0;
  o->panel_tiles_precond = 0;
  o->tune_table = nullptr;
  o->lookahead = 0;
  o->side_stream = 1;
  o->stage_cols = 0;
  o->mv_group_tiles = 0;
  o->mfma_f32 = 0;
}

mlbddc_status mlbddc_create(mlbddc_t* out, const mlbddc_options* opt, const mlbddc_allocator* alloc, void* stream) {
  if (!out) return MLBDDC_E_ARG;
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) {
    g_create_error.status = MLBDDC_E_ARG;
    g_create_error.message = "allocator without alloc or free function";
    return MLBDDC_E_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    g_create_error.status = MLBDDC_E_NO_DEVICE;
    g_create_error.message = "no HIP device available";
    return MLBDDC_E_NO_DEVICE;
  }
  mlbddc_options o;
  mlbddc_default_options(&o);
  if (opt) o = *opt;
  if (o.device < 0 || o.device >= ndev || !(o.rtol > 0) || o.max_iter < 1 ||
      (o.precision != MLBDDC_FP64 && o.precision != MLBDDC_MIXED) ||
      (o.stage_cols != 0 && o.stage_cols != 16 && o.stage_cols != 32 && o.stage_cols != 64) ||
      (o.mfma_f32 != 0 && o.mfma_f32 != 16 && o.mfma_f32 != 32 && o.mfma_f32 != 3) ||
      (o.mv_group_tiles != 0 && o.mv_group_tiles != 1 && o.mv_group_tiles != 2)) {
    g_create_error.status = MLBDDC_E_ARG;
    g_create_error.message = "invalid options";
    return MLBDDC_E_ARG;
  }
  if (hipSetDevice(o.device) != hipSuccess) {
    g_create_error.status = MLBDDC_E_HIP;
    g_create_error.message = "hipSetDevice failed";
    return MLBDDC_E_HIP;
  }
  void* sp = nullptr;
  if (hipError_t e = mlbddc::scratch_address(o.device, &sp); e != hipSuccess) {
    (void)hipGetLastError();
    g_create_error.status = MLBDDC_E_HIP;
    g_create_error.message = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return MLBDDC_E_HIP;
  }
  auto* h = new mlbddc_handle_s();
  h->h.opt = o;
  h->h.scratch_ptr = sp;
  h->h.lookahead = o.lookahead != 0;
  if (o.tune_table) {
    std::ifstream in(o.tune_table);
    std::string line;
    while (std::getline(in, line)) {
      if (line.empty() || line[0] == '#') continue;
      std::istringstream ls(line);
      std::string job, prec;
      int bucket = 0, panel = 0, stage = 0;
      if (!(ls >> job >> prec >> bucket >> panel)) continue;
      if (job == "MV") {  // tiles per workgroup of the tile products
        if (panel == 1 || panel == 2) h->h.mv_tpw[prec == "f32" ? 1 : 0] = panel;
        continue;
      }
      if (job == "PANEL") {  // staged columns of the panel products
        if (panel == 16 || panel == 32 || panel == 64) h->h.panel_stage[prec == "f32" ? 1 : 0] = panel;
        continue;
      }
      if (job == "SHAPE") {  // FP32 MFMA shape of the tile products
        if (prec == "f32" && (panel == 16 || panel == 32 || panel == 3)) h->h.mfma_f32 = panel;
        continue;
      }
      if (panel < 1 || panel > 16) continue;
      if (!(ls >> stage) || (stage != 16 && stage != 32 && stage != 64)) stage = 0;
      h->h.tune.push_back({job == "M" ? 1 : 0, prec == "f32" ? 1 : 0, bucket, panel, stage});
    }
    h->h.opt.tune_table = nullptr;  // the path is not kept
  }
  if (o.mv_group_tiles > 0) h->h.mv_tpw[0] = h->h.mv_tpw[1] = o.mv_group_tiles;
  if (o.mfma_f32 > 0) h->h.mfma_f32 = o.mfma_f32;
  h->h.stream = (hipStream_t)stream;
  if (alloc) {
    h->h.ext_alloc = *alloc;
    h->h.has_ext_alloc = true;
  }
  *out = h;
  return MLBDDC_OK;
}

mlbddc_status mlbddc_setup(mlbddc_t h, const mlbddc_mesh* mesh, const mlbddc_partition* part) {
  if (!h) return MLBDDC_E_ARG;
  h->h.err = mlbddc::Error();
  return h->h.setup(mesh, part);
}

mlbddc_status mlbddc_update_coefficients(mlbddc_t h, const double* scale_dev) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.planned) return h->h.fail(MLBDDC_E_STATE, "update_coefficients before setup");
  if (!scale_dev) return h->h.fail(MLBDDC_E_ARG, "null scale pointer");
  hipError_t e = hipMemcpyAsync(h->h.d_scale, scale_dev, sizeof(double) * h->h.n_elems, hipMemcpyDeviceToDevice, h->h.stream);
  if (e != hipSuccess) return h->h.herr("hipMemcpyAsync", e);
  h->h.ready = false;
  return h->h.numeric();
}

int64_t mlbddc_num_dofs(mlbddc_t h) { return h && h->h.planned ? h->h.plan.levels[0].n_dofs : -1; }
int64_t mlbddc_interface_size(mlbddc_t h) {
  return h && h->h.planned ? (int64_t)h->h.plan.levels[0].iface_dofs.size() : -1;
}
int64_t mlbddc_coarse_size(mlbddc_t h, int32_t level) {
  if (!h || !h->h.planned || level < 1 || level >= (int32_t)h->h.plan.levels.size() + 0) return -1;
  return h->h.plan.levels[level - 1].n_coarse;
}
int64_t mlbddc_num_subdomains(mlbddc_t h, int32_t level) {
  if (!h || !h->h.planned || level < 1 || level > (int32_t)h->h.plan.levels.size()) return -1;
  return h->h.plan.levels[level - 1].n_sub;
}

mlbddc_status mlbddc_interface_dofs(mlbddc_t h, int64_t* out) {
  if (!h || !out) return MLBDDC_E_ARG;
  if (!h->h.planned) return h->h.fail(MLBDDC_E_STATE, "interface_dofs before setup");
  const auto& v = h->h.plan.levels[0].iface_dofs;
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i];
  return MLBDDC_OK;
}

mlbddc_status mlbddc_subdomain_sizes(mlbddc_t h, int32_t level, int64_t* out) {
  if (!h || !out) return MLBDDC_E_ARG;
  if (!h->h.planned) return h->h.fail(MLBDDC_E_STATE, "subdomain_sizes before setup");
  if (level < 1 || level > (int32_t)h->h.plan.levels.size()) return h->h.fail(MLBDDC_E_ARG, "bad level");
  const auto& L = h->h.plan.levels[level - 1];
  for (int b = 0; b < L.n_sub; ++b) {
    out[3 * b] = L.subs[b].nI;
    out[3 * b + 1] = L.subs[b].nG;
    out[3 * b + 2] = L.subs[b].nc;
  }
  return MLBDDC_OK;
}

mlbddc_status mlbddc_apply(mlbddc_t h, const double* r, double* z) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.ready) return h->h.fail(MLBDDC_E_STATE, "apply before setup");
  if (!r || !z || r == z) return h->h.fail(MLBDDC_E_ARG, "bad vector pointers");
  return h->h.apply_interface(0, r, z);
}

mlbddc_status mlbddc_apply_schur(mlbddc_t h, const double* x, double* y) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.ready) return h->h.fail(MLBDDC_E_STATE, "apply_schur before setup");
  if (!x || !y || x == y) return h->h.fail(MLBDDC_E_ARG, "bad vector pointers");
  return h->h.schur(x, y);
}

mlbddc_status mlbddc_apply_schur_noalloc(mlbddc_t h, const double* x, double* y) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.ready) return h->h.fail(MLBDDC_E_STATE, "apply_schur_noalloc before setup");
  if (!x || !y || x == y) return h->h.fail(MLBDDC_E_ARG, "bad vector pointers");
  return h->h.schur_noalloc(x, y);
}

mlbddc_status mlbddc_condense(mlbddc_t h, const double* f, double* g) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.ready) return h->h.fail(MLBDDC_E_STATE, "condense before setup");
  if (!f || !g) return h->h.fail(MLBDDC_E_ARG, "bad vector pointers");
  return h->h.condense(f, g);
}

mlbddc_status mlbddc_solve(mlbddc_t h, const double* f, double* u, const double* u0, mlbddc_stats* st) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.ready) return h->h.fail(MLBDDC_E_STATE, "solve before setup");
  if (!f || !u || f == u) return h->h.fail(MLBDDC_E_ARG, "bad vector pointers");
  return h->h.solve(f, u, u0, st);
}

mlbddc_status mlbddc_element_energy(mlbddc_t h, const double* a, const double* b, double* out) {
  if (!h) return MLBDDC_E_ARG;
  if (!h->h.ready) return h->h.fail(MLBDDC_E_STATE, "element_energy before setup");
  if (!a || !b || !out) return h->h.fail(MLBDDC_E_ARG, "bad vector pointers");
  if (h->h.ev_edof) {
    hipError_t we = hipStreamWaitEvent(h->h.stream, h->h.ev_edof, 0);
    if (we != hipSuccess) return h->h.herr("hipStreamWaitEvent", we);
  }
  mlbddc::launch_element_energy(h->h.stream, h->h.n_elems, h->h.nloc1, h->h.d_edof, h->h.d_Kref, h->h.d_scale, a, b, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return h->h.herr("element_energy", e);
  return MLBDDC_OK;
}

mlbddc_status mlbddc_get_coarse_matrix(mlbddc_t h, int32_t level, double* out) {
  if (!h || !out) return MLBDDC_E_ARG;
  Handle& H = h->h;
  if (!H.ready) return H.fail(MLBDDC_E_STATE, "get_coarse_matrix before setup");
  if (level < 1 || level >= (int32_t)H.lev.size()) return H.fail(MLBDDC_E_ARG, "bad level");
  auto& D = H.lev[level - 1];
  auto& P = *D.P;
  const int64_t n = P.n_coarse;
  std::vector<double> kc(D.kc_off.empty() ? 0 : (size_t)(D.kc_off.back() + (int64_t)P.subs.back().nc * P.subs.back().nc));
  if (!kc.empty()) {
    hipError_t e = hipMemcpyAsync(kc.data(), D.kc_compact, sizeof(double) * kc.size(), hipMemcpyDeviceToHost, H.stream);
    if (e != hipSuccess) return H.herr("hipMemcpyAsync", e);
    e = hipStreamSynchronize(H.stream);
    if (e != hipSuccess) return H.herr("hipStreamSynchronize", e);
  }
  std::fill(out, out + n * n, 0.0);
  for (int b = 0; b < P.n_sub; ++b) {
    const auto& S = P.subs[b];
    for (int a = 0; a < S.nc; ++a)
      for (int c = 0; c < S.nc; ++c) out[(int64_t)S.coarse[a] * n + S.coarse[c]] += kc[D.kc_off[b] + (int64_t)a * S.nc + c];
  }
  return MLBDDC_OK;
}

mlbddc_status mlbddc_set_profiling(mlbddc_t h, int32_t enable) {
  if (!h) return MLBDDC_E_ARG;
  if (mlbddc_status st = h->h.collect_mv_timing()) return st;
  h->h.prof = enable != 0;
  int p0 = h->h.pdata.panel[0], p1 = h->h.pdata.panel[1], s0 = h->h.pdata.stage[0], s1 = h->h.pdata.stage[1];
  h->h.pdata = mlbddc_profile{};
  h->h.pdata.panel[0] = p0;
  h->h.pdata.panel[1] = p1;
  h->h.pdata.stage[0] = s0;
  h->h.pdata.stage[1] = s1;
  return MLBDDC_OK;
}

mlbddc_status mlbddc_get_profile(mlbddc_t h, mlbddc_profile* out) {
  if (!h || !out) return MLBDDC_E_ARG;
  if (mlbddc_status st = h->h.collect_mv_timing()) return st;
  *out = h->h.pdata;
  return MLBDDC_OK;
}

mlbddc_status mlbddc_destroy(mlbddc_t h) {
  if (!h) return MLBDDC_OK;
  // every library stream drains before its blocks go back to the allocator
  (void)hipStreamSynchronize(h->h.stream);
  for (hipStream_t s : {h->h.cap, h->h.fstream, h->h.gstream, h->h.ustream})
    if (s) (void)hipStreamSynchronize(s);
  h->h.free_all(false);
  if (h->h.cap) {
    (void)hipStreamSynchronize(h->h.cap);
    (void)hipStreamDestroy(h->h.cap);
  }
  if (h->h.fstream) {
    (void)hipStreamSynchronize(h->h.fstream);
    (void)hipStreamDestroy(h->h.fstream);
  }
  if (h->h.gstream) {
    (void)hipStreamSynchronize(h->h.gstream);
    (void)hipStreamDestroy(h->h.gstream);
  }
  if (h->h.ev_gfork) (void)hipEventDestroy(h->h.ev_gfork);
  if (h->h.ev_gjoin) (void)hipEventDestroy(h->h.ev_gjoin);
  if (h->h.ustream) {
    (void)hipStreamSynchronize(h->h.ustream);
    (void)hipStreamDestroy(h->h.ustream);
  }
  if (h->h.h_s) (void)hipHostFree(h->h.h_s);
  if (h->h.h_err) (void)hipHostFree(h->h.h_err);
  for (hipEvent_t e : h->h.ev_snap)
    if (e) (void)hipEventDestroy(e);
  for (auto& c : h->h.staging) (void)hipHostFree(c.first);
  if (h->h.ev_upl) (void)hipEventDestroy(h->h.ev_upl);
  if (h->h.ev_edof) (void)hipEventDestroy(h->h.ev_edof);
  if (h->h.ev_a) (void)hipEventDestroy(h->h.ev_a);
  if (h->h.ev_b) (void)hipEventDestroy(h->h.ev_b);
  if (h->h.ev_in) (void)hipEventDestroy(h->h.ev_in);
  if (h->h.ev_out) (void)hipEventDestroy(h->h.ev_out);
  (void)h->h.collect_mv_timing();
  for (hipEvent_t e : h->h.mv_spare) (void)hipEventDestroy(e);
  delete h;
  return MLBDDC_OK;
}

mlbddc_status mlbddc_last_error(mlbddc_t h, mlbddc_error* info) {
  if (!info) return MLBDDC_E_ARG;
  const mlbddc::Error& e = h ? h->h.err : g_create_error;
  info->status = e.status;
  info->level = e.level;
  info->subdomain = e.subdomain;
  info->column = e.column;
  std::snprintf(info->message, sizeof(info->message), "%s", e.message.c_str());
  return MLBDDC_OK;
}

mlbddc_status mlbddc_plan_counts(const mlbddc_mesh* mesh, const mlbddc_partition* part, int64_t* counts) {
  if (!mesh || !part || !counts) return MLBDDC_E_ARG;
  mlbddc::PlanInput in;
  in.dim = mesh->dim;
  in.ndof = mesh->ndof_per_node;
  in.n_nodes = mesh->n_nodes;
  in.n_elems = mesh->n_elems;
  in.nodes_per_elem = mesh->nodes_per_elem;
  in.elem_nodes = mesh->elem_nodes;
  in.dirichlet = mesh->dirichlet_nodes;
  in.n_levels = part->n_levels;
  in.elem_to_sub = part->elem_to_sub;
  in.sub_to_parent = part->sub_to_parent;
  in.constraints = part->constraints;
  mlbddc::Plan plan;
  mlbddc::Error err;
  mlbddc_status st = mlbddc::build_plan(in, plan, err);
  if (st) return st;
  for (int l = 0; l + 1 < (int)plan.levels.size(); ++l) {
    const auto& L = plan.levels[l];
    int64_t* c = counts + 6 * l;
    c[0] = L.n_sub;
    c[1] = (int64_t)L.iface_dofs.size();
    c[2] = L.n_coarse;
    c[3] = L.counts[0];
    c[4] = L.counts[1];
    c[5] = L.counts[2];
  }
  return MLBDDC_OK;
}

mlbddc_status mlbddc_plan_interface(const mlbddc_mesh* mesh, const mlbddc_partition* part, int64_t* iface_dofs, int32_t sub,
                                    int64_t* n_gamma, int64_t* sub_iface) {
  if (!mesh || !part) return MLBDDC_E_ARG;
  mlbddc::PlanInput in;
  in.dim = mesh->dim;
  in.ndof = mesh->ndof_per_node;
  in.n_nodes = mesh->n_nodes;
  in.n_elems = mesh->n_elems;
  in.nodes_per_elem = mesh->nodes_per_elem;
  in.elem_nodes = mesh->elem_nodes;
  in.dirichlet = mesh->dirichlet_nodes;
  in.n_levels = 2;
  in.elem_to_sub = part->elem_to_sub;
  in.sub_to_parent = nullptr;
  in.constraints = part->constraints;
  mlbddc::Plan plan;
  mlbddc::Error err;
  mlbddc_status st = mlbddc::build_plan(in, plan, err);
  if (st) return st;
  const auto& L = plan.levels[0];
  if (iface_dofs) std::copy(L.iface_dofs.begin(), L.iface_dofs.end(), iface_dofs);
  if (sub >= 0 && sub < L.n_sub) {
    const auto& S = L.subs[sub];
    if (n_gamma) *n_gamma = S.nG;
    if (sub_iface) std::copy(S.iface.begin(), S.iface.end(), sub_iface);
  } else if (n_gamma) {
    *n_gamma = -1;
  }
  return MLBDDC_OK;
}

}  // extern "C"
