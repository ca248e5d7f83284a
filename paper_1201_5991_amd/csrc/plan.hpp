// Host planning of the multilevel decomposition (set-up, Algorithm 1: the
// integer part).  Builds, level by level, the subdomain node sets, the
// interface, its classification into faces / edges / vertices ("globs"),
// the corners, the constraint rows of C_i, the local DOF orderings and tile
// layouts, the element colouring used by assembly, and the pseudo-mesh of
// the next level (subdomains become elements, constrained globs become nodes).
//
// Readings of the paper's unspecified steps (shared with the written
// description of the method, not with any other code):
//  * a glob is a class of interface nodes with the same set of subdomains;
//    a glob of three or more subdomains made of one node is a corner; in 3D
//    a glob of two subdomains is a face, one of three or more with several
//    nodes an edge; in 2D a glob of two subdomains is an edge;
//  * Dirichlet nodes are removed before the interface is formed;
//  * constraints: one row per glob and component, the value at a corner or
//    the arithmetic mean (weights 1/m) over an edge or face;
//  * globs are ordered by their smallest node; coarse DOFs glob by glob,
//    component innermost.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <utility>
#include <vector>

#include "common.hpp"

namespace mlbddc {

enum GlobKind { G_CORNER = 0, G_EDGE = 1, G_FACE = 2 };

struct Glob {
  std::vector<int64_t> nodes;  // level nodes, sorted
  std::vector<int32_t> subs;   // sorted subdomains sharing it
  int kind = G_EDGE;
  bool constrained = false;
  int64_t coarse_node = -1;
};

// One subdomain of one level.
struct SubPlan {
  int64_t nI = 0, nG = 0;      // interior / interface DOFs
  int64_t nIp = 0, nGp = 0;    // padded to the tile edge (nIp: every interior group padded)
  std::vector<int64_t> dofI;   // level DOF of each interior position 0..nIp-1 (-1: padding)
  std::vector<int32_t> padI;   // (start, count) runs of interior padding positions
  // Level 1: interior numbered by nested dissection in groups (parts and
  // separators) that each start on a tile; gtile holds the first tile column
  // of every group, then nIp / 64.  sptr / srow: tile rows r > k with
  // L(r, k) != 0 for every interior tile column k (symbolic factorization).
  // All empty when the interior is one group in node order.
  std::vector<int32_t> gtile, sptr, srow;
  // height of every group in the dissection tree (parts 0, a separator one
  // more than the higher of its two halves); one group of height 0 otherwise
  std::vector<int32_t> gheight;
  std::vector<int64_t> dofG;   // level DOFs of the interface, local order
  std::vector<int32_t> iface;  // R_i: local interface position -> level interface index
  std::vector<int32_t> coarse; // R_Ci: local coarse DOF -> level coarse DOF
  int32_t nc = 0, ncp = 0;     // constraints and padded count
  // constraint rows: row c averages local interface positions crow_col[crow_ptr[c]..crow_ptr[c+1])
  std::vector<int32_t> crow_ptr, crow_col;
  // elements of the subdomain (ids in the level's element numbering)
  std::vector<int64_t> elems;
  // tile envelope (first nonzero tile column per tile row) of the local K matrix
  std::vector<int32_t> envK;
  // empty every field, keeping the vectors' storage for the next plan
  void reset() {
    nI = nG = nIp = nGp = 0;
    nc = ncp = 0;
    for (auto* v : {&dofI, &dofG, &elems}) v->clear();
    for (auto* v : {&padI, &gtile, &sptr, &srow, &gheight, &iface, &coarse, &crow_ptr, &crow_col, &envK}) v->clear();
  }
};

struct LevelPlan {
  int level = 1;               // 1-based
  int dim = 3, ndof = 3;
  int64_t n_nodes = 0, n_dofs = 0;
  int32_t n_sub = 0;
  bool augmentK = false;       // K matrix carries an identity block (levels >= 2)
  bool top = false;            // single subdomain without interface: the coarse problem
  // elements of this level: node lists (-1 = eliminated node) in CSR form
  std::vector<int64_t> el_ptr, el_nodes;
  std::vector<int32_t> el_sub;
  // per element and element DOF: position in the padded local K ordering (-1 = none)
  std::vector<int32_t> el_local_ptr;    // start of an element's node entries in el_local (= el_ptr)
  std::vector<int32_t> el_local;        // per element node: local matrix index of the node's first DOF
                                        // (its ndof DOFs are consecutive), -1 for an eliminated node
  std::vector<int32_t> el_color;
  int32_t n_colors = 0;
  std::vector<SubPlan> subs;
  std::vector<int64_t> iface_dofs;      // level interface DOFs, increasing
  std::vector<Glob> globs;
  int64_t n_coarse_nodes = 0, n_coarse = 0;
  int32_t counts[3] = {0, 0, 0};        // corners, edges, faces
};

struct PlanInput {
  int dim = 3, ndof = 3;
  int64_t n_nodes = 0, n_elems = 0;
  int nodes_per_elem = 8;
  const int32_t* elem_nodes = nullptr;
  const uint8_t* dirichlet = nullptr;
  int n_levels = 2;
  const int32_t* elem_to_sub = nullptr;
  const int32_t* const* sub_to_parent = nullptr;
  int constraints = MLBDDC_CORNERS | MLBDDC_EDGES | MLBDDC_FACES;
  bool reuse_layouts = true;  // structurally equal subdomains share one dissection (same result)
};

// Per-thread host scratch of the planner, kept by the plan between set-ups.
// The node-indexed arrays are left clean after use (every touched entry is
// reset), so a repeated set-up of the same mesh touches no new pages.
struct PlanScratch {
  std::vector<int32_t> node_local;      // node -> local slot in the current subdomain, -1
  std::vector<uint64_t> node_mask;      // node -> colours of the subdomain's elements at the node, 0
  std::vector<int32_t> stamp;           // node -> last subdomain that listed the node, -1
  void ensure(int64_t n) {
    if ((int64_t)node_local.size() < n) {
      node_local.resize(n, -1);
      node_mask.resize(n, 0);
      stamp.resize(n, -1);
    }
  }
};

struct Plan {
  std::vector<LevelPlan> levels;        // BDDC levels 1..L-1, then the top (coarse) level
  std::vector<int64_t> node_to_free;    // mesh node -> free node (-1 for Dirichlet)
  int64_t n_free_nodes = 0;
  // planner work space reused by the next build_plan on the same plan
  std::vector<PlanScratch> scratch;
  std::vector<int32_t> w_cnt;
  std::vector<int64_t> w_nptr, w_pos, w_node_iface;
  std::vector<int32_t> w_nsub;
  std::vector<char> w_is_g;
  std::vector<std::vector<int32_t>> w_keys;  // structure keys of the subdomains (layout reuse)
};

// Build the whole plan.  Returns MLBDDC_OK or an error with a message.
mlbddc_status build_plan(const PlanInput& in, Plan& plan, Error& err);

// Factorization schedule of a batch of tile-packed matrices, each eliminated
// in one or two phases (the second factors the negative of the first phase's
// trailing block: its tasks carry TASK_NEG).
struct FactorItemDesc {
  int32_t nt = 0;                       // tiles per side
  int32_t e1 = 0, e2 = 0;               // tile columns eliminated per phase
  const int32_t* env = nullptr;         // first nonzero tile column per tile row (size nt)
  // optional tile structure of the phase-1 columns (e2 == 0): rows of L per
  // column (CSR over columns 0..e1-1) and group boundaries (ngroups + 1
  // entries, last = e1) that panels do not cross; null: the envelope is used
  const int32_t* sptr = nullptr;
  const int32_t* srow = nullptr;
  const int32_t* gtile = nullptr;
  const int32_t* gheight = nullptr;     // height of every group in the dissection tree
  int32_t ngroups = 0;
};

// Allocator whose value construction leaves scalars uninitialized: a vector
// that is filled completely right after resize() skips the zeroing pass.
template <typename T>
struct NoInitAllocator : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAllocator<U>;
  };
  NoInitAllocator() = default;
  template <typename U>
  NoInitAllocator(const NoInitAllocator<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};

struct FactorLaunch {
  int kind;
  int k;                                // global tile column of this step
  int64_t first, count;                 // task range
  double flops;                         // algorithmic flops of the launch's tasks
  int stream;                           // 0: critical path, 1: bulk trailing updates (look-ahead)
  bool wait;                            // wait for the other stream's work issued so far
};

struct FactorSchedule {
  std::vector<uint64_t, NoInitAllocator<uint64_t>> tasks;  // every element is written by the builder
  std::vector<FactorLaunch> launches;
  double flops = 0.0;                   // dense flops of the tasks (for rooflines)
  int64_t update_tasks = 0;
};

// panel: tile columns per panel.  lookahead: split each trailing update into
// the next panel's columns (stream 0) and the rest (stream 1), so that the
// next panel's factorization overlaps the bulk of the update (items with a
// tile structure keep one stream).  Launch k is a step index: the tile column
// for items scheduled by envelope; for items with a tile structure the groups
// of one dissection height advance together (step = first step of the height
// + column within the group).
void build_factor_schedule(const std::vector<FactorItemDesc>& items, int panel, FactorSchedule& out,
                           bool lookahead = false);

// Tiles of a tile-structured matrix (it.sptr set) that the factorization,
// the assembly and the solves read before writing, as runs of consecutive
// rows r0 .. r0 + count - 1 of column k; no kernel reads any other tile.  The
// update tasks of a panel read tile (r, kk) for every column kk of the panel
// and every row r in the structure of one of them; panels lie within one
// dissection group, so the tiles (r, k) with k in a group and r in the union
// of the group's column structures and its own rows cover them; the trailing
// (interface) block is dense.
void read_before_write_tiles(const FactorItemDesc& it, const std::function<void(int r0, int k, int count)>& emit);

// Runs body(t) for t = 0..T-1 concurrently and returns when every call has
// returned; the caller runs t = 0, persistent worker threads the others (a
// call made while another thread is inside parallel_run, or from inside a
// body, gets threads of its own).  T is clamped to 1..16.
void parallel_run(int T, const std::function<void(int)>& body);

}  // namespace mlbddc
