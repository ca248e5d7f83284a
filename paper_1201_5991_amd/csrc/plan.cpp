// Host planning of the multilevel decomposition; see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <iterator>
#include <cstring>
#include <map>
#include <memory>
#include <unordered_map>
#include <numeric>
#include <thread>
#include <mutex>
#include <atomic>
#include <condition_variable>
#include <unistd.h>
#include <chrono>
#include <cstdio>
#include <cstdlib>

namespace mlbddc {

// ------------------------------------------------------------ worker pool
// Spawning and joining 16 threads costs about half a millisecond, as much as
// several of the planner's parallel loops themselves, so the loops run on
// threads that are started once and then wait for work.  One loop at a time
// uses the pool; a loop started meanwhile (another handle's set-up on another
// thread, or a loop nested in a body) spawns threads of its own.  After a
// fork the child starts a new pool (the parent's workers do not exist there).
namespace {

thread_local bool in_parallel_body = false;  // set while a thread runs a body

class WorkerPool {
 public:
  static constexpr int MAXT = 16;
  explicit WorkerPool(pid_t pid) : pid_(pid) {}
  pid_t pid() const { return pid_; }

  // false when the pool is busy (the caller then spawns its own threads)
  bool run(int T, const std::function<void(int)>& body) {
    if (in_parallel_body) return false;
    std::unique_lock<std::mutex> own(run_mx_, std::try_to_lock);
    if (!own.owns_lock()) return false;
    {
      std::lock_guard<std::mutex> g(mx_);
      while ((int)workers_.size() < T - 1) {
        const int w = (int)workers_.size() + 1;
        workers_.emplace_back([this, w] { loop(w); });
        workers_.back().detach();
      }
      body_ = &body;
      active_ = T;
      pending_ = T - 1;
      ++gen_;
    }
    cv_.notify_all();
    in_parallel_body = true;
    body(0);
    in_parallel_body = false;
    std::unique_lock<std::mutex> g(mx_);
    done_cv_.wait(g, [this] { return pending_ == 0; });
    body_ = nullptr;
    return true;
  }

 private:
  void loop(int w) {
    uint64_t seen = 0;
    {
      std::lock_guard<std::mutex> g(mx_);
      seen = gen_ - 1;  // a worker created for the current loop joins it
    }
    for (;;) {
      const std::function<void(int)>* body;
      {
        std::unique_lock<std::mutex> g(mx_);
        cv_.wait(g, [&] { return gen_ != seen; });
        seen = gen_;
        if (w >= active_) continue;
        body = body_;
      }
      in_parallel_body = true;
      (*body)(w);
      in_parallel_body = false;
      std::lock_guard<std::mutex> g(mx_);
      if (--pending_ == 0) done_cv_.notify_one();
    }
  }

  pid_t pid_;
  std::mutex run_mx_, mx_;
  std::condition_variable cv_, done_cv_;
  std::vector<std::thread> workers_;
  const std::function<void(int)>* body_ = nullptr;
  int active_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
};

WorkerPool* pool_for_this_process() {
  static std::mutex mx;
  static WorkerPool* pool = nullptr;  // never destroyed: its workers wait until the process ends
  std::lock_guard<std::mutex> g(mx);
  const pid_t pid = getpid();
  if (!pool || pool->pid() != pid) pool = new WorkerPool(pid);
  return pool;
}

}  // namespace

void read_before_write_tiles(const FactorItemDesc& it, const std::function<void(int, int, int)>& emit) {
  const int nt = it.nt;
  std::vector<char> rows;
  for (int g = 0; g < it.ngroups; ++g) {
    rows.assign(nt, 0);
    for (int k = it.gtile[g]; k < it.gtile[g + 1]; ++k) {
      rows[k] = 1;
      for (int32_t q = it.sptr[k]; q < it.sptr[k + 1]; ++q) rows[it.srow[q]] = 1;
    }
    for (int k = it.gtile[g]; k < it.gtile[g + 1]; ++k)
      for (int r = k; r < nt;) {
        if (!rows[r]) { ++r; continue; }
        int r1 = r;
        while (r1 < nt && rows[r1]) ++r1;
        emit(r, k, r1 - r);
        r = r1;
      }
  }
  for (int k = it.e1; k < nt; ++k) emit(k, k, nt - k);
}

void parallel_run(int T, const std::function<void(int)>& body) {
  T = std::max(1, std::min(T, (int)WorkerPool::MAXT));
  if (T == 1) { body(0); return; }
  if (pool_for_this_process()->run(T, body)) return;
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back([&body, t] { body(t); });
  body(0);
  for (auto& x : th) x.join();
}

namespace {

mlbddc_status fail(Error& err, mlbddc_status st, const std::string& msg) {
  err.status = st;
  err.message = msg;
  return st;
}

// Classification of a glob from its subdomain count and node count.
int classify(size_t n_subs, size_t n_nodes, int dim) {
  if (n_subs >= 3 && n_nodes == 1) return G_CORNER;
  if (n_subs == 2) return dim == 3 ? G_FACE : G_EDGE;
  return G_EDGE;
}

// Threads used for n work items (at most 16, at least 4 items per thread).
int plan_threads(int64_t n) {
  unsigned hw = std::thread::hardware_concurrency();
  int T = (int)std::max(1u, std::min(16u, hw ? hw : 1u));
  return (int)std::max<int64_t>(1, std::min<int64_t>(T, n / 4));
}

// Run work(t, begin, end) over [0, n) split into plan_threads(n) contiguous ranges.
template <typename F>
void parallel_ranges(int64_t n, F&& work) {
  const int T = plan_threads(n);
  if (T <= 1) { work(0, (int64_t)0, n); return; }
  parallel_run(T, [&](int t) { work(t, n * t / T, n * (t + 1) / T); });
}

// ------------------------------------------------------ nested dissection
// Interior DOFs below which a subdomain keeps one group in node order, and
// the largest part left undivided (in DOFs).
constexpr int64_t ND_MIN_DOFS = 16 * TS;
constexpr int64_t ND_LEAF_DOFS = 12 * TS;

// Nested-dissection order of a subdomain's interior nodes 0..n-1 (adjacency
// CSR ptr / adj).  The separators are level sets of breadth-first distances
// grown from the interior nodes next to one side of the subdomain (dist[s],
// one array per side, INT32_MAX where unreached): adjacent nodes differ by at
// most one level, so every level set separates the nodes below it from the
// nodes above it, and on box subdomains the level sets are planes parallel to
// the side.  A part of more than `leaf` nodes is cut at the level set that
// leaves both halves at most 70% of the part with the smallest separator (else
// the best balance); the order is [half A][half B][separator], and every
// undivided part and every separator is one group (sizes in gsize).
struct NdOrder {
  const std::vector<std::vector<int32_t>>& dist;
  int64_t leaf;
  std::vector<int32_t>& order;
  std::vector<int32_t>& gsize;
  std::vector<int32_t>& gheight;
  std::vector<int32_t> hist;
  int leaf_group(std::vector<int32_t>& X, int height) {
    if (X.empty()) return -1;
    std::sort(X.begin(), X.end());
    order.insert(order.end(), X.begin(), X.end());
    gsize.push_back((int32_t)X.size());
    gheight.push_back(height);
    return height;
  }
  // returns the height of the part's last group (-1 for an empty part)
  int run(std::vector<int32_t> X) {
    if ((int64_t)X.size() <= leaf) return leaf_group(X, 0);
    const int64_t nx = (int64_t)X.size();
    int best_s = -1, best_L = 0;
    int64_t best_sep = 0, best_big = 0;
    bool best_bal = false;
    for (size_t s = 0; s < dist.size(); ++s) {
      const std::vector<int32_t>& d = dist[s];
      int32_t lo = INT32_MAX, hi = -1;
      bool all = true;
      for (int32_t x : X) {
        if (d[x] == INT32_MAX) { all = false; break; }
        lo = std::min(lo, d[x]);
        hi = std::max(hi, d[x]);
      }
      if (!all || hi - lo < 2) continue;
      hist.assign((size_t)(hi - lo + 1), 0);
      for (int32_t x : X) hist[d[x] - lo]++;
      int64_t below = hist[0];
      for (int32_t L = lo + 1; L < hi; ++L) {
        const int64_t sep = hist[L - lo], above = nx - below - sep;
        const int64_t big = std::max(below, above);
        const bool bal = 10 * big <= 7 * nx;
        bool better;
        if (best_s < 0) better = true;
        else if (bal != best_bal) better = bal;
        else if (bal) better = sep < best_sep || (sep == best_sep && big < best_big);
        else better = big < best_big || (big == best_big && sep < best_sep);
        if (better) { best_s = (int)s; best_L = L; best_sep = sep; best_big = big; best_bal = bal; }
        below += sep;
      }
    }
    if (best_s < 0) return leaf_group(X, 0);
    const std::vector<int32_t>& d = dist[best_s];
    std::vector<int32_t> A, B, S;
    for (int32_t x : X) (d[x] < best_L ? A : d[x] > best_L ? B : S).push_back(x);
    X.clear();
    X.shrink_to_fit();
    const int ha = run(std::move(A));
    const int hb = run(std::move(B));
    const int hs = leaf_group(S, std::max(ha, hb) + 1);
    return hs >= 0 ? hs : std::max(ha, hb);
  }
};

// Interior order of subdomain b by nested dissection.  node_local maps the
// subdomain's interior nodes to 0..n-1 and its interface nodes to 0..ng-1;
// sides are the neighbouring subdomains (interface nodes shared with them).
// Distances grow from at most three sides whose interior layers touch one
// another, each layer at least a quarter of the largest.
void nd_interior(const LevelPlan& L, const SubPlan& S, int32_t b, const std::vector<int64_t>& inodes,
                 const std::vector<int64_t>& gnodes, const std::vector<int32_t>& node_local,
                 const std::vector<char>& node_is_g, const int64_t* nptr, const int32_t* nsub, int nd,
                 std::vector<int32_t>& order, std::vector<int32_t>& gsize, std::vector<int32_t>& gheight) {
  const int32_t n = (int32_t)inodes.size(), ng = (int32_t)gnodes.size();
  const int64_t ne = (int64_t)S.elems.size();
  // element-local slots: interior nodes 0..n-1, interface nodes n..n+ng-1
  // work arrays kept by the planning thread between subdomains
  static thread_local std::vector<int32_t> eptr, eslot, ecnt, elist, ptr, adj, stamp, queue, pos;
  eptr.assign(ne + 1, 0);
  eslot.clear();
  for (int64_t i = 0; i < ne; ++i) {
    const int64_t e = S.elems[i];
    for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
      const int64_t v = L.el_nodes[j];
      if (v >= 0) eslot.push_back(node_is_g[v] ? n + node_local[v] : node_local[v]);
    }
    eptr[i + 1] = (int32_t)eslot.size();
  }
  // slot -> elements (CSR)
  ecnt.assign(n + ng + 1, 0);
  for (int32_t x : eslot) ecnt[x + 1]++;
  for (int32_t i = 0; i < n + ng; ++i) ecnt[i + 1] += ecnt[i];
  elist.resize(ecnt[n + ng]);
  {
    pos.assign(ecnt.begin(), ecnt.end() - 1);
    for (int64_t i = 0; i < ne; ++i)
      for (int32_t q = eptr[i]; q < eptr[i + 1]; ++q) elist[pos[eslot[q]]++] = (int32_t)i;
  }
  // interior adjacency (CSR, no duplicates; branch-free inner loop)
  ptr.assign(n + 1, 0);
  if (adj.size() < (size_t)n * 32 + 64) adj.resize((size_t)n * 32 + 64);
  stamp.assign(n + ng, -1);
  int64_t na = 0;
  for (int32_t u = 0; u < n; ++u) {
    stamp[u] = u;
    for (int32_t q = ecnt[u]; q < ecnt[u + 1]; ++q) {
      const int32_t i = elist[q];
      if (na + (eptr[i + 1] - eptr[i]) > (int64_t)adj.size()) adj.resize(adj.size() * 2);
      for (int32_t r = eptr[i]; r < eptr[i + 1]; ++r) {
        const int32_t w = eslot[r];
        const int32_t old = stamp[w];
        stamp[w] = u;
        adj[na] = w;
        na += (w < n) & (old != u);
      }
    }
    ptr[u + 1] = (int32_t)na;
  }
  // sides: (neighbour, interface slot) pairs grouped by neighbour
  std::vector<std::pair<int32_t, int32_t>> ns_pairs;
  for (int32_t gi = 0; gi < ng; ++gi) {
    const int64_t v = gnodes[gi];
    for (int64_t q = nptr[v]; q < nptr[v + 1]; ++q)
      if (nsub[q] != b) ns_pairs.push_back({nsub[q], gi});
  }
  std::sort(ns_pairs.begin(), ns_pairs.end());
  std::vector<std::vector<int32_t>> layer;
  std::fill(stamp.begin(), stamp.end(), -1);
  for (size_t q = 0; q < ns_pairs.size();) {
    size_t q1 = q;
    while (q1 < ns_pairs.size() && ns_pairs[q1].first == ns_pairs[q].first) ++q1;
    const int32_t sid = (int32_t)layer.size();
    layer.emplace_back();
    std::vector<int32_t>& l = layer.back();
    for (size_t t = q; t < q1; ++t) {
      const int32_t gs = n + ns_pairs[t].second;
      for (int32_t r = ecnt[gs]; r < ecnt[gs + 1]; ++r) {
        const int32_t i = elist[r];
        for (int32_t z = eptr[i]; z < eptr[i + 1]; ++z) {
          const int32_t w = eslot[z];
          if (w < n && stamp[w] != sid) { stamp[w] = sid; l.push_back(w); }
        }
      }
    }
    q = q1;
  }
  // up to three sides that touch one another (on a box: three perpendicular
  // faces), largest layers first
  std::vector<int32_t> by_size(layer.size());
  std::iota(by_size.begin(), by_size.end(), 0);
  std::sort(by_size.begin(), by_size.end(), [&](int32_t x, int32_t y) {
    return layer[x].size() != layer[y].size() ? layer[x].size() > layer[y].size() : x < y;
  });
  std::vector<int32_t> chosen;
  std::vector<uint8_t> in_chosen(n, 0);
  for (int32_t c : by_size) {
    if (chosen.size() == 3 || layer[c].empty()) break;
    if (4 * layer[c].size() < layer[by_size[0]].size()) break;
    uint8_t touch = 0;
    for (int32_t x : layer[c]) touch |= in_chosen[x];
    if (touch != (uint8_t)((1u << chosen.size()) - 1)) continue;  // must touch every side chosen so far
    for (int32_t x : layer[c]) in_chosen[x] |= (uint8_t)(1u << chosen.size());
    chosen.push_back(c);
  }
  std::vector<std::vector<int32_t>> dist;
  queue.resize(n + 1);
  for (int32_t c : chosen) {
    dist.emplace_back(n, INT32_MAX);
    std::vector<int32_t>& d = dist.back();
    int32_t qh = 0, qt = 0;
    for (int32_t x : layer[c]) { d[x] = 0; queue[qt++] = x; }
    while (qh < qt) {
      const int32_t u = queue[qh++];
      const int32_t du = d[u] + 1;
      for (int32_t q = ptr[u]; q < ptr[u + 1]; ++q) {
        const int32_t w = adj[q];
        const bool fresh = d[w] == INT32_MAX;
        d[w] = fresh ? du : d[w];
        queue[qt] = w;
        qt += fresh;
      }
    }
  }
  order.clear();
  gsize.clear();
  gheight.clear();
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  NdOrder nd_rec{dist, std::max<int64_t>(1, ND_LEAF_DOFS / nd), order, gsize, gheight, {}};
  nd_rec.run(std::move(all));
}

// Symbolic factorization at tile level: structure of L over the interior
// tile columns 0..tI-1 of a matrix of nt tile rows, from the tiles every
// element couples.  Column k's rows are passed on to its parent (its first
// row below k) when k is eliminated.
void tile_structure(const LevelPlan& L, const SubPlan& S, int nd, int tI, int nt, std::vector<int32_t>& sptr,
                    std::vector<int32_t>& srow) {
  const int W = (nt + 63) / 64;
  std::vector<uint64_t> bits((size_t)tI * W, 0);
  int32_t tl[64];
  for (int64_t e : S.elems) {
    int m = 0;
    for (int64_t j = L.el_local_ptr[e]; j < L.el_local_ptr[e + 1]; ++j) {
      const int32_t p = L.el_local[j];
      if (p < 0) continue;
      for (int t = p / TS; t <= (p + nd - 1) / TS; ++t) {  // tiles of the node's DOFs
        int x = 0;
        while (x < m && tl[x] != t) ++x;
        if (x == m && m < 64) tl[m++] = t;
      }
    }
    for (int x = 0; x < m; ++x) {
      const int a = tl[x];
      if (a >= tI) continue;
      uint64_t* col = bits.data() + (size_t)a * W;
      for (int y = 0; y < m; ++y)
        if (tl[y] > a) col[tl[y] / 64] |= 1ull << (tl[y] % 64);
    }
  }
  for (int k = 0; k < tI; ++k) {
    uint64_t* col = bits.data() + (size_t)k * W;
    int par = -1;
    for (int w = 0; w < W && par < 0; ++w)
      if (col[w]) par = w * 64 + __builtin_ctzll(col[w]);
    if (par < 0 || par >= tI) continue;
    uint64_t* pc = bits.data() + (size_t)par * W;
    for (int w = 0; w < W; ++w) pc[w] |= col[w];
    pc[par / 64] &= ~(1ull << (par % 64));
  }
  sptr.assign(tI + 1, 0);
  srow.clear();
  for (int k = 0; k < tI; ++k) {
    const uint64_t* col = bits.data() + (size_t)k * W;
    for (int w = 0; w < W; ++w)
      for (uint64_t m = col[w]; m; m &= m - 1) srow.push_back(w * 64 + __builtin_ctzll(m));
    sptr[k + 1] = (int32_t)srow.size();
  }
}

// Globs of a level: the classes of interface nodes with one subdomain set,
// each split into its connected parts (two nodes of a class are connected
// when one element holds both).  Every class has an owner, the first
// subdomain of its set, which holds all its nodes; the owners form their
// classes and split them along their own elements, on several threads.  A
// class left in several parts by its owner's elements is joined again over
// the elements of all its subdomains (the only elements holding its nodes).
// Globs come out in no particular order; nodes increase within each.
void build_globs(LevelPlan& L, const std::vector<int64_t>& node_iface, const std::vector<int64_t>& nptr,
                 const std::vector<int32_t>& nsub, const std::vector<std::vector<int64_t>>& sub_nodes, Plan& plan) {
  const int32_t ns = L.n_sub;
  auto set_less = [&](int64_t a, int64_t b) {  // lexicographic order of the subdomain sets of nodes a, b
    return std::lexicographical_compare(nsub.begin() + nptr[a], nsub.begin() + nptr[a + 1], nsub.begin() + nptr[b],
                                        nsub.begin() + nptr[b + 1]);
  };
  auto set_equal = [&](int64_t a, int64_t b) {
    return nptr[a + 1] - nptr[a] == nptr[b + 1] - nptr[b] &&
           std::equal(nsub.begin() + nptr[a], nsub.begin() + nptr[a + 1], nsub.begin() + nptr[b]);
  };
  auto find = [](std::vector<int32_t>& par, int32_t x) {
    while (par[x] != x) x = par[x] = par[par[x]];
    return x;
  };
  std::vector<std::vector<Glob>> cand(ns);
  std::vector<std::vector<char>> whole(ns);  // per candidate: its class is in one part at its owner
  if ((int)plan.scratch.size() < plan_threads(ns)) plan.scratch.resize(plan_threads(ns));
  parallel_ranges(ns, [&](int t, int64_t b0, int64_t b1) {
    PlanScratch& W = plan.scratch[t];
    W.ensure(L.n_nodes);
    std::vector<int32_t>& loc = W.node_local;  // node -> index among the owned nodes, -1
    std::vector<int64_t> own;
    std::vector<int32_t> ord, cls, par, ii;
    std::vector<std::array<int32_t, 3>> key;  // (class, part root, owned index)
    for (int64_t b = b0; b < b1; ++b) {
      own.clear();
      for (int64_t n : sub_nodes[b])
        if (node_iface[n] >= 0 && nsub[nptr[n]] == b) own.push_back(n);
      const int32_t m = (int32_t)own.size();
      if (m == 0) continue;
      ord.resize(m);
      std::iota(ord.begin(), ord.end(), 0);
      std::sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
        return set_less(own[x], own[y]) || (!set_less(own[y], own[x]) && x < y);
      });
      cls.assign(m, 0);
      for (int32_t q = 1; q < m; ++q) cls[ord[q]] = cls[ord[q - 1]] + (set_equal(own[ord[q]], own[ord[q - 1]]) ? 0 : 1);
      par.resize(m);
      for (int32_t k = 0; k < m; ++k) {
        loc[own[k]] = k;
        par[k] = k;
      }
      for (int64_t e : L.subs[b].elems) {
        ii.clear();
        for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
          const int64_t v = L.el_nodes[j];
          if (v >= 0 && loc[v] >= 0) ii.push_back(loc[v]);
        }
        for (size_t q = 1; q < ii.size(); ++q)
          for (size_t p = 0; p < q; ++p)
            if (cls[ii[p]] == cls[ii[q]]) {
              const int32_t x = find(par, ii[p]), y = find(par, ii[q]);
              if (x != y) par[std::max(x, y)] = std::min(x, y);
              break;
            }
      }
      key.resize(m);
      for (int32_t k = 0; k < m; ++k) key[k] = {cls[k], find(par, k), k};
      std::sort(key.begin(), key.end());
      for (int32_t q = 0; q < m;) {
        int32_t q1 = q;
        while (q1 < m && key[q1][0] == key[q][0]) ++q1;  // one class
        const bool one = key[q][1] == key[q1 - 1][1];
        for (int32_t r = q; r < q1;) {
          int32_t r1 = r;
          while (r1 < q1 && key[r1][1] == key[r][1]) ++r1;  // one part
          Glob g;
          const int64_t n0 = own[key[r][2]];
          g.subs.assign(nsub.begin() + nptr[n0], nsub.begin() + nptr[n0 + 1]);
          for (int32_t z = r; z < r1; ++z) g.nodes.push_back(own[key[z][2]]);
          cand[b].push_back(std::move(g));
          whole[b].push_back(one ? 1 : 0);
          r = r1;
        }
        q = q1;
      }
      for (int64_t n : own) loc[n] = -1;
    }
  });
  L.globs.clear();
  std::vector<std::vector<int64_t>> rejoin;  // classes in several parts at their owner: all nodes
  for (int32_t b = 0; b < ns; ++b) {
    std::vector<int64_t>* cur = nullptr;
    const std::vector<int32_t>* cur_subs = nullptr;
    for (size_t c = 0; c < cand[b].size(); ++c) {
      if (whole[b][c]) {
        L.globs.push_back(std::move(cand[b][c]));
        continue;
      }
      if (!cur || *cur_subs != cand[b][c].subs) {  // parts of one class are adjacent in cand[b]
        rejoin.emplace_back();
        cur = &rejoin.back();
        cur_subs = &cand[b][c].subs;
      }
      cur->insert(cur->end(), cand[b][c].nodes.begin(), cand[b][c].nodes.end());
    }
  }
  if (rejoin.empty()) return;
  // classes split at their owner: union-find over the elements of all their subdomains
  const int64_t ni = (int64_t)L.iface_dofs.size() / L.ndof;
  std::vector<int32_t> rc(ni, -1), par(ni);
  std::iota(par.begin(), par.end(), 0);
  std::vector<char> sub_in(ns, 0);
  for (size_t c = 0; c < rejoin.size(); ++c) {
    std::sort(rejoin[c].begin(), rejoin[c].end());
    for (int64_t n : rejoin[c]) rc[node_iface[n]] = (int32_t)c;
    const int64_t n0 = rejoin[c][0];
    for (int64_t q = nptr[n0]; q < nptr[n0 + 1]; ++q) sub_in[nsub[q]] = 1;
  }
  std::vector<int32_t> ii;
  for (int32_t b = 0; b < ns; ++b) {
    if (!sub_in[b]) continue;
    for (int64_t e : L.subs[b].elems) {
      ii.clear();
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
        const int64_t v = L.el_nodes[j];
        if (v >= 0 && node_iface[v] >= 0 && rc[node_iface[v]] >= 0) ii.push_back((int32_t)node_iface[v]);
      }
      for (size_t q = 1; q < ii.size(); ++q)
        for (size_t p = 0; p < q; ++p)
          if (rc[ii[p]] == rc[ii[q]]) {
            const int32_t x = find(par, ii[p]), y = find(par, ii[q]);
            if (x != y) par[std::max(x, y)] = std::min(x, y);
            break;
          }
    }
  }
  std::vector<int32_t> roots;
  for (auto& nodes : rejoin) {
    roots.clear();
    for (int64_t n : nodes) {
      const int32_t r = find(par, (int32_t)node_iface[n]);
      if (std::find(roots.begin(), roots.end(), r) == roots.end()) roots.push_back(r);
    }
    const size_t base = L.globs.size();
    for (size_t k = 0; k < roots.size(); ++k) {
      L.globs.emplace_back();
      L.globs.back().subs.assign(nsub.begin() + nptr[nodes[0]], nsub.begin() + nptr[nodes[0] + 1]);
    }
    for (int64_t n : nodes) {  // increasing within every part
      const int32_t r = find(par, (int32_t)node_iface[n]);
      L.globs[base + (std::find(roots.begin(), roots.end(), r) - roots.begin())].nodes.push_back(n);
    }
  }
}

// Subdomains with the same local structure get the same interior order and
// tile structure: the key lists the local slot of every node of every element
// (interior nodes in node order, then interface nodes) and, per interface
// node, the ranks of its other subdomains among the subdomain's neighbours,
// which is everything the nested dissection and the tile structure read.
// The keys of all subdomains are built first (on threads); the first
// subdomain of every key hash computes its layout (the leaders, on threads),
// then every other subdomain takes its leader's layout after comparing the
// keys in full (a hash collision falls back to its own dissection), so no
// thread waits for another.  A box division repeats few structures.
struct LayoutEntry {
  std::vector<int32_t> key;
  std::vector<int32_t> order, gsize, gheight, sptr, srow;  // dissection and tile structure
  std::vector<int32_t> gperm;                              // interface order (positions in node order)
  std::vector<int32_t> elocal, envK, ecolor;               // element maps, envelope, element colours
  int32_t ncolor = 0;
};

uint64_t key_hash(const std::vector<int32_t>& k) {
  uint64_t h = 1469598103934665603ull;
  for (int32_t v : k) h = (h ^ (uint64_t)(uint32_t)v) * 1099511628211ull;
  return h;
}

// Build one level from its elements (node lists, -1 = eliminated node) and
// the subdomain of every element.
mlbddc_status build_level(LevelPlan& L, int constraints, Error& err, Plan& plan, bool reuse_layouts) {
  const bool verbose = std::getenv("MLBDDC_VERBOSE") != nullptr;
  auto t_last = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) {
    auto t = std::chrono::steady_clock::now();
    if (verbose)
      std::fprintf(stderr, "[mlbddc plan L%d] %-24s %8.2f ms\n", L.level, what,
                   std::chrono::duration<double, std::milli>(t - t_last).count());
    t_last = t;
  };
  const int nd = L.ndof;
  const int64_t ne = (int64_t)L.el_sub.size();
  const int32_t ns = L.n_sub;

  // --- subdomain node sets and elements
  std::vector<std::vector<int64_t>> sub_nodes(ns);
  L.subs.resize(ns);  // a previous plan's subdomains keep their storage
  for (SubPlan& S : L.subs) S.reset();
  {
    std::vector<int64_t> cnt(ns, 0);
    for (int64_t e = 0; e < ne; ++e) {
      int32_t b = L.el_sub[e];
      if (b < 0 || b >= ns) return fail(err, MLBDDC_E_ARG, "element assigned to a non-existent subdomain");
      cnt[b]++;
    }
    for (int32_t b = 0; b < ns; ++b) L.subs[b].elems.reserve(cnt[b]);
    for (int64_t e = 0; e < ne; ++e) L.subs[L.el_sub[e]].elems.push_back(e);
  }
  if ((int)plan.scratch.size() < plan_threads(ns)) plan.scratch.resize(plan_threads(ns));
  parallel_ranges(ns, [&](int t, int64_t b0, int64_t b1) {
    PlanScratch& W = plan.scratch[t];
    W.ensure(L.n_nodes);
    std::vector<int32_t>& stamp = W.stamp;  // last subdomain that listed the node
    for (int32_t b = (int32_t)b0; b < (int32_t)b1; ++b) {
      auto& v = sub_nodes[b];
      for (int64_t e : L.subs[b].elems)
        for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
          int64_t n = L.el_nodes[j];
          if (n >= 0 && stamp[n] != b) {
            stamp[n] = b;
            v.push_back(n);
          }
        }
      for (int64_t n : v) stamp[n] = -1;
      std::sort(v.begin(), v.end());
    }
  });
  for (int32_t b = 0; b < ns; ++b)
    if (L.subs[b].elems.empty() || sub_nodes[b].empty())
      return fail(err, MLBDDC_E_ARG, "level " + std::to_string(L.level) + ": subdomain " + std::to_string(b) + " is empty");

  mark("subdomain node sets");
  // --- node -> subdomains (CSR, sorted by subdomain)
  // (threads own node ranges; each visits every subdomain's sorted node list
  // from the first node of its range, so subdomains stay in increasing order)
  std::vector<int32_t>& cnt = plan.w_cnt;
  cnt.assign(L.n_nodes + 1, 0);
  const int TN = std::min(plan_threads(L.n_nodes), std::max(1, (int)std::min<int64_t>(16, L.n_nodes / 65536)));
  auto node_range = [&](int t, auto&& visit) {
    const int64_t n0 = L.n_nodes * t / TN, n1 = L.n_nodes * (t + 1) / TN;
    for (int32_t b = 0; b < ns; ++b) {
      const auto& v = sub_nodes[b];
      for (auto it = std::lower_bound(v.begin(), v.end(), n0); it != v.end() && *it < n1; ++it) visit(*it, b);
    }
  };
  parallel_run(TN, [&](int t) { node_range(t, [&](int64_t n, int32_t) { cnt[n + 1]++; }); });
  std::vector<int64_t>& nptr = plan.w_nptr;
  nptr.assign(L.n_nodes + 1, 0);
  for (int64_t n = 0; n < L.n_nodes; ++n) nptr[n + 1] = nptr[n] + cnt[n + 1];
  std::vector<int32_t>& nsub = plan.w_nsub;
  nsub.resize(nptr[L.n_nodes]);
  {
    std::vector<int64_t>& pos = plan.w_pos;
    pos.assign(nptr.begin(), nptr.end() - 1);
    parallel_run(TN, [&](int t) { node_range(t, [&](int64_t n, int32_t b) { nsub[pos[n]++] = b; }); });
  }
  auto mult = [&](int64_t n) { return nptr[n + 1] - nptr[n]; };

  mark("node subdomain lists");
  // --- interface nodes and globs
  std::vector<int64_t> iface_nodes;
  if (!L.top)
    for (int64_t n = 0; n < L.n_nodes; ++n)
      if (mult(n) >= 2) iface_nodes.push_back(n);
  std::vector<int64_t>& node_iface = plan.w_node_iface;
  node_iface.assign(L.n_nodes, -1);
  for (size_t i = 0; i < iface_nodes.size(); ++i) node_iface[iface_nodes[i]] = (int64_t)i;
  L.iface_dofs.resize(iface_nodes.size() * nd);
  for (size_t i = 0; i < iface_nodes.size(); ++i)
    for (int c = 0; c < nd; ++c) L.iface_dofs[i * nd + c] = iface_nodes[i] * nd + c;

  L.globs.clear();
  if (constraints & MLBDDC_ALL_PRIMAL) {
    for (int64_t n : iface_nodes) {
      Glob g;
      g.nodes = {n};
      g.subs.assign(nsub.begin() + nptr[n], nsub.begin() + nptr[n + 1]);
      g.kind = G_CORNER;
      L.globs.push_back(std::move(g));
    }
  } else {
    build_globs(L, node_iface, nptr, nsub, sub_nodes, plan);
    for (auto& g : L.globs) g.kind = classify(g.subs.size(), g.nodes.size(), L.dim);
  }
  std::sort(L.globs.begin(), L.globs.end(), [](const Glob& a, const Glob& b) { return a.nodes[0] < b.nodes[0]; });
  L.counts[0] = L.counts[1] = L.counts[2] = 0;
  L.n_coarse_nodes = 0;
  for (auto& g : L.globs) {
    L.counts[g.kind]++;
    bool on = (constraints & MLBDDC_ALL_PRIMAL) || (g.kind == G_CORNER && (constraints & MLBDDC_CORNERS)) ||
              (g.kind == G_EDGE && (constraints & MLBDDC_EDGES)) || (g.kind == G_FACE && (constraints & MLBDDC_FACES));
    g.constrained = on;
    g.coarse_node = on ? L.n_coarse_nodes++ : -1;
  }
  L.n_coarse = L.n_coarse_nodes * nd;
  if (!L.top) {
    if (iface_nodes.empty()) return fail(err, MLBDDC_E_ARG, "level " + std::to_string(L.level) + " has no interface");
    if (L.n_coarse == 0) return fail(err, MLBDDC_E_ARG, "level " + std::to_string(L.level) + " has no coarse DOFs");
  }

  mark("globs");
  // subdomain -> constrained globs (in glob order)
  std::vector<std::vector<int32_t>> sub_globs(ns);
  for (size_t gi = 0; gi < L.globs.size(); ++gi)
    if (L.globs[gi].constrained)
      for (int32_t b : L.globs[gi].subs) sub_globs[b].push_back((int32_t)gi);

  // --- local orderings, element maps, envelopes, constraints
  if (L.el_ptr[ne] >= INT32_MAX) return fail(err, MLBDDC_E_ARG, "too many element nodes on one level");
  L.el_local_ptr.resize(ne + 1);
  for (int64_t e = 0; e <= ne; ++e) L.el_local_ptr[e] = (int32_t)L.el_ptr[e];
  L.el_local.resize(L.el_ptr[ne]);  // every entry is written by the subdomain owning the element
  L.el_color.resize(ne);
  std::vector<int32_t> sub_colors(ns, 0);
  std::vector<int32_t> sub_fail(ns, 0);

  // interface flag of every node (a property of the level)
  std::vector<char>& node_is_g = plan.w_is_g;
  node_is_g.assign(L.n_nodes, 0);
  if (!L.top)
    for (int64_t n = 0; n < L.n_nodes; ++n) node_is_g[n] = mult(n) >= 2;

  // Per-subdomain work is independent: split the subdomains over threads, each
  // with its own node-indexed scratch (reset only where it was touched).
  if ((int)plan.scratch.size() < plan_threads(ns)) plan.scratch.resize(plan_threads(ns));
  std::atomic<int32_t> reused{0};
  // structure keys (level 1 with nested dissection), the leader of every key
  // hash, and the entries the leaders fill
  const bool keyed_level = L.level == 1 && !L.top && reuse_layouts;
  std::vector<std::vector<int32_t>>& keys = plan.w_keys;
  std::vector<std::shared_ptr<LayoutEntry>> entry_of(ns);
  std::vector<char> is_leader(ns, 0);
  if (keyed_level) {
    if ((int32_t)keys.size() < ns) keys.resize(ns);
    parallel_ranges(ns, [&](int t, int64_t b0, int64_t b1) {
      PlanScratch& W = plan.scratch[t];
      W.ensure(L.n_nodes);
      std::vector<int32_t>& node_local = W.node_local;
      std::vector<int64_t> gnodes;
      std::vector<int32_t> nb;
      for (int32_t b = (int32_t)b0; b < (int32_t)b1; ++b) {
        std::vector<int32_t>& skey = keys[b];
        skey.clear();
        const SubPlan& S = L.subs[b];
        int32_t ni = 0;
        gnodes.clear();
        for (int64_t n : sub_nodes[b]) {
          if (mult(n) >= 2) { node_local[n] = (int32_t)gnodes.size(); gnodes.push_back(n); }
          else node_local[n] = ni++;
        }
        if ((int64_t)ni * nd >= ND_MIN_DOFS) {
          size_t nel = 0, nnb = 0;  // element node entries; other subdomains of the interface nodes and separators
          for (int64_t e : S.elems) nel += (size_t)(L.el_ptr[e + 1] - L.el_ptr[e]);
          for (int64_t v : gnodes) nnb += (size_t)(nptr[v + 1] - nptr[v]);
          skey.reserve(4 + nel + nnb);
          skey.resize(4 + nel);
          skey[0] = ni;
          skey[1] = (int32_t)gnodes.size();
          skey[2] = nd;
          skey[3] = (int32_t)S.elems.size();
          int32_t* kp = skey.data() + 4;
          for (int64_t e : S.elems)
            for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
              const int64_t v = L.el_nodes[j];
              *kp++ = v < 0 ? -1 : node_local[v] + (node_is_g[v] ? ni : 0);
            }
          nb.clear();
          for (int64_t v : gnodes)
            for (int64_t q = nptr[v]; q < nptr[v + 1]; ++q)
              if (nsub[q] != b) nb.push_back(nsub[q]);
          std::sort(nb.begin(), nb.end());
          nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
          for (int64_t v : gnodes) {
            for (int64_t q = nptr[v]; q < nptr[v + 1]; ++q)
              if (nsub[q] != b) skey.push_back((int32_t)(std::lower_bound(nb.begin(), nb.end(), nsub[q]) - nb.begin()));
            skey.push_back(-2);
          }
        }
        for (int64_t n : sub_nodes[b]) node_local[n] = -1;
      }
    });
    std::unordered_map<uint64_t, int32_t> first;
    std::vector<uint64_t> hsh(ns, 0);
    parallel_ranges(ns, [&](int, int64_t b0, int64_t b1) {
      for (int64_t b = b0; b < b1; ++b)
        if (!keys[b].empty()) hsh[b] = key_hash(keys[b]);
    });
    for (int32_t b = 0; b < ns; ++b) {
      if (keys[b].empty()) continue;
      auto it = first.find(hsh[b]);
      if (it == first.end()) {
        first.emplace(hsh[b], b);
        is_leader[b] = 1;
        entry_of[b] = std::make_shared<LayoutEntry>();
      } else {
        entry_of[b] = entry_of[it->second];
      }
    }
  }
  auto work = [&](int t, int64_t b_begin, int64_t b_end) {
  PlanScratch& W = plan.scratch[t];
  W.ensure(L.n_nodes);
  std::vector<int32_t>& node_local = W.node_local;  // node -> local node slot (interior or interface)
  std::vector<uint64_t>& node_mask = W.node_mask;
  for (int32_t b = (int32_t)b_begin; b < (int32_t)b_end; ++b) {
    SubPlan& S = L.subs[b];
    std::vector<int64_t> inodes, gnodes;
    for (int64_t n : sub_nodes[b]) (mult(n) >= 2 && !L.top ? gnodes : inodes).push_back(n);
    S.nI = (int64_t)inodes.size() * nd;
    S.nG = (int64_t)gnodes.size() * nd;
    S.nGp = round_up(S.nG, TS);
    for (size_t i = 0; i < inodes.size(); ++i) node_local[inodes[i]] = (int32_t)i;
    for (size_t i = 0; i < gnodes.size(); ++i) node_local[gnodes[i]] = (int32_t)i;

    // interior numbering: nested dissection on level 1 (groups padded to whole
    // tiles), else node order; node_local of an interior node becomes the
    // local position of its first DOF
    std::vector<int32_t> iorder, gsize;
    const bool use_nd = L.level == 1 && !L.top && S.nI >= ND_MIN_DOFS;
    std::shared_ptr<LayoutEntry> mine, hit;  // the entry this subdomain computes, or reuses
    if (use_nd && entry_of[b]) {
      if (is_leader[b]) {
        mine = entry_of[b];
        mine->key.swap(keys[b]);
      } else if (entry_of[b]->key == keys[b]) {
        hit = entry_of[b];
      }
    }
    if (hit) {
      iorder = hit->order;
      gsize = hit->gsize;
      S.gheight = hit->gheight;
      reused++;
    } else if (use_nd) {
      nd_interior(L, S, b, inodes, gnodes, node_local, node_is_g, nptr.data(), nsub.data(), nd, iorder, gsize,
                  S.gheight);
    } else {
      iorder.resize(inodes.size());
      std::iota(iorder.begin(), iorder.end(), 0);
      gsize.assign(1, (int32_t)inodes.size());
      S.gheight.assign(1, 0);
    }
    S.padI.clear();
    S.gtile.clear();
    S.sptr.clear();
    S.srow.clear();
    {
      std::vector<int32_t> ipos(inodes.size());
      int64_t pos = 0;
      size_t q = 0;
      for (int32_t gs : gsize) {
        if (use_nd) S.gtile.push_back((int32_t)(pos / TS));
        for (int32_t i = 0; i < gs; ++i, ++q) ipos[iorder[q]] = (int32_t)(pos + (int64_t)i * nd);
        const int64_t end = pos + (int64_t)gs * nd, pend = round_up(end, TS);
        if (pend > end) {
          S.padI.push_back((int32_t)end);
          S.padI.push_back((int32_t)(pend - end));
        }
        pos = pend;
      }
      S.nIp = pos;
      if (use_nd) S.gtile.push_back((int32_t)(pos / TS));
      S.dofI.assign(S.nIp, -1);
      for (size_t i = 0; i < inodes.size(); ++i) {
        node_local[inodes[i]] = ipos[i];
        for (int c = 0; c < nd; ++c) S.dofI[ipos[i] + c] = inodes[i] * nd + c;
      }
    }

    // interface nodes sorted by the first interior position they couple to, so
    // that the tile envelope of the interface rows is tight
    std::vector<int64_t> key(hit ? 0 : gnodes.size(), INT64_MAX);
    for (int64_t e : S.elems) {
      if (hit) break;
      int64_t mn = INT64_MAX;
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
        int64_t n = L.el_nodes[j];
        if (n >= 0 && !node_is_g[n]) mn = std::min(mn, (int64_t)node_local[n]);
      }
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
        int64_t n = L.el_nodes[j];
        if (n >= 0 && node_is_g[n]) key[node_local[n]] = std::min(key[node_local[n]], mn);
      }
    }
    std::vector<int32_t> order(gnodes.size());
    if (hit) {
      order = hit->gperm;
    } else {
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        return key[a] != key[c] ? key[a] < key[c] : gnodes[a] < gnodes[c];
      });
    }
    std::vector<int64_t> gsorted(gnodes.size());
    for (size_t i = 0; i < order.size(); ++i) gsorted[i] = gnodes[order[i]];
    gnodes.swap(gsorted);
    for (size_t i = 0; i < gnodes.size(); ++i) node_local[gnodes[i]] = (int32_t)i;

    S.dofG.resize(S.nG);
    S.iface.resize(S.nG);
    for (size_t i = 0; i < gnodes.size(); ++i)
      for (int c = 0; c < nd; ++c) {
        S.dofG[i * nd + c] = gnodes[i] * nd + c;
        S.iface[i * nd + c] = (int32_t)(node_iface[gnodes[i]] * nd + c);
      }

    // local K index of a level DOF of this subdomain
    auto kidx = [&](int64_t n, int c) -> int64_t {
      return node_is_g[n] ? S.nIp + (int64_t)node_local[n] * nd + c : (int64_t)node_local[n] + c;
    };
    const int64_t nK = S.nIp + S.nGp + (L.augmentK ? S.nIp : 0);
    const int64_t ntK = nK / TS;
    if (hit) {  // the element maps and the envelope of the equal structure
      size_t q = 0;
      for (int64_t e : S.elems)
        for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) L.el_local[j] = hit->elocal[q++];
      S.envK = hit->envK;
    } else {
    std::vector<int64_t> first(nK);
    for (int64_t p = 0; p < nK; ++p) first[p] = p;
    if (L.augmentK)
      for (int64_t p = S.nIp + S.nGp; p < nK; ++p) first[p] = p - (S.nIp + S.nGp);
    for (int64_t e : S.elems) {
      int64_t mn = INT64_MAX;
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
        int64_t n = L.el_nodes[j];
        int64_t p = n < 0 ? -1 : kidx(n, 0);
        L.el_local[j] = (int32_t)p;
        if (p >= 0) mn = std::min(mn, p);
      }
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) {
        int32_t p = L.el_local[j];
        if (p >= 0)
          for (int c = 0; c < nd; ++c) first[p + c] = std::min(first[p + c], mn);
      }
    }
    S.envK.assign(ntK, 0);
    for (int64_t r = 0; r < ntK; ++r) {
      int64_t m = INT64_MAX;
      for (int64_t p = r * TS; p < (r + 1) * TS; ++p) m = std::min(m, first[p]);
      S.envK[r] = (int32_t)(m / TS);
    }
    }
    if (hit) {
      S.sptr = hit->sptr;
      S.srow = hit->srow;
    } else if (use_nd) {
      tile_structure(L, S, nd, (int)(S.nIp / TS), (int)ntK, S.sptr, S.srow);
    }
    if (mine) {
      mine->order = iorder;
      mine->gsize = gsize;
      mine->gheight = S.gheight;
      mine->sptr = S.sptr;
      mine->srow = S.srow;
      mine->gperm = order;
      mine->envK = S.envK;
      for (int64_t e : S.elems)
        for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j) mine->elocal.push_back(L.el_local[j]);
    }

    // constraint rows and R_Ci
    S.crow_ptr.assign(1, 0);
    S.crow_col.clear();
    S.coarse.clear();
    for (int32_t gi : sub_globs[b]) {
      const Glob& g = L.globs[gi];
      for (int c = 0; c < nd; ++c) {
        for (int64_t n : g.nodes) S.crow_col.push_back((int32_t)((int64_t)node_local[n] * nd + c));
        S.crow_ptr.push_back((int32_t)S.crow_col.size());
        S.coarse.push_back((int32_t)(g.coarse_node * nd + c));
      }
    }
    S.nc = (int32_t)S.coarse.size();
    S.ncp = (int32_t)round_up(S.nc, TS);
    if (!L.top && S.nc == 0) sub_fail[b] = 1;

    // greedy colouring of the subdomain's elements: elements sharing a node get
    // different colours (only elements of one subdomain write the same matrix)
    int ncol = 0;
    if (hit) {
      if (hit->ecolor.size() != S.elems.size()) sub_fail[b] = 2;  // the colouring of the structure failed
      else
        for (size_t q = 0; q < S.elems.size(); ++q) L.el_color[S.elems[q]] = hit->ecolor[q];
      ncol = hit->ncolor;
    }
    for (int64_t e : S.elems) {
      if (hit) break;
      uint64_t used = 0;
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j)
        if (L.el_nodes[j] >= 0) used |= node_mask[L.el_nodes[j]];
      if (used == ~0ull) { sub_fail[b] = 2; break; }
      int c = __builtin_ctzll(~used);
      L.el_color[e] = c;
      ncol = std::max(ncol, c + 1);
      for (int64_t j = L.el_ptr[e]; j < L.el_ptr[e + 1]; ++j)
        if (L.el_nodes[j] >= 0) node_mask[L.el_nodes[j]] |= (1ull << c);
    }
    sub_colors[b] = ncol;
    if (mine) {
      for (int64_t e : S.elems) mine->ecolor.push_back(L.el_color[e]);
      mine->ncolor = ncol;
    }

    for (int64_t n : sub_nodes[b]) { node_local[n] = -1; node_mask[n] = 0; }
  }
  };
  // subdomains handed out one at a time, largest first (the cost grows with
  // the node count; interior subdomains are cut by the dissection)
  {
    std::vector<int32_t> order(ns);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t c) { return sub_nodes[a].size() > sub_nodes[c].size(); });
    // the leaders first, in a pass of their own: the others then find their
    // entries complete
    std::vector<int32_t> lead, rest;
    for (int32_t b : order) (is_leader[b] ? lead : rest).push_back(b);
    for (const std::vector<int32_t>* part : {&lead, &rest}) {
      const int32_t np = (int32_t)part->size();
      std::atomic<int32_t> next{0};
      parallel_run(plan_threads(np), [&](int t) {
        for (int32_t i = next++; i < np; i = next++) work(t, (*part)[i], (*part)[i] + 1);
      });
    }
  }
  if (verbose && reused > 0)
    std::fprintf(stderr, "[mlbddc plan L%d] %d of %d subdomain layouts reuse the dissection of an equal structure\n", L.level,
                 (int)reused, (int)ns);
  mark("local layouts (parallel)");
  for (int32_t b = 0; b < ns; ++b) {
    if (sub_fail[b] == 1)
      return fail(err, MLBDDC_E_ARG, "level " + std::to_string(L.level) + ": subdomain " + std::to_string(b) + " has no constraints");
    if (sub_fail[b] == 2) return fail(err, MLBDDC_E_ARG, "element colouring needs more than 64 colours");
  }
  L.n_colors = 0;
  for (int32_t b = 0; b < ns; ++b) L.n_colors = std::max(L.n_colors, sub_colors[b]);
  return MLBDDC_OK;
}

}  // namespace

mlbddc_status build_plan(const PlanInput& in, Plan& plan, Error& err) {
  if (in.dim != 2 && in.dim != 3) return fail(err, MLBDDC_E_ARG, "dim must be 2 or 3");
  if (in.ndof < 1 || in.ndof > 3) return fail(err, MLBDDC_E_ARG, "ndof_per_node must be 1..3");
  if (in.n_levels < 2) return fail(err, MLBDDC_E_ARG, "n_levels must be >= 2");
  if (in.n_elems <= 0 || in.n_nodes <= 0 || !in.elem_nodes || !in.elem_to_sub)
    return fail(err, MLBDDC_E_ARG, "empty mesh or missing arrays");
  if (in.n_levels > 2 && !in.sub_to_parent) return fail(err, MLBDDC_E_ARG, "sub_to_parent missing");

  const bool verbose = std::getenv("MLBDDC_VERBOSE") != nullptr;
  auto t_last = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) {
    auto t = std::chrono::steady_clock::now();
    if (verbose)
      std::fprintf(stderr, "[mlbddc plan] %-30s %8.2f ms\n", what, std::chrono::duration<double, std::milli>(t - t_last).count());
    t_last = t;
  };
  // level storage of the previous plan is reused (capacity kept)
  std::vector<LevelPlan> old = std::move(plan.levels);
  plan.levels.clear();
  auto take_level = [&](size_t i) {
    LevelPlan L;
    if (i < old.size()) {
      L.el_ptr.swap(old[i].el_ptr);
      L.el_nodes.swap(old[i].el_nodes);
      L.el_sub.swap(old[i].el_sub);
      L.el_local_ptr.swap(old[i].el_local_ptr);
      L.el_local.swap(old[i].el_local);
      L.el_color.swap(old[i].el_color);
      L.subs.swap(old[i].subs);
      L.el_nodes.clear();
    }
    return L;
  };
  plan.node_to_free.assign(in.n_nodes, -1);
  int64_t nf = 0;
  for (int64_t n = 0; n < in.n_nodes; ++n)
    if (!in.dirichlet || !in.dirichlet[n]) plan.node_to_free[n] = nf++;
  plan.n_free_nodes = nf;

  // ---- level 1 from the mesh (element ranges on threads)
  LevelPlan L1 = take_level(0);
  L1.level = 1;
  L1.dim = in.dim;
  L1.ndof = in.ndof;
  L1.n_nodes = nf;
  L1.n_dofs = nf * in.ndof;
  const int npe = in.nodes_per_elem;
  L1.el_ptr.resize(in.n_elems + 1);
  L1.el_nodes.resize(in.n_elems * npe);
  L1.el_sub.resize(in.n_elems);
  std::vector<int32_t> t_nsub(plan_threads(in.n_elems), 0);
  std::vector<char> t_bad(t_nsub.size(), 0);
  parallel_ranges(in.n_elems, [&](int t, int64_t e0, int64_t e1) {
    int32_t nsub_t = 0;
    for (int64_t e = e0; e < e1; ++e) {
      L1.el_ptr[e] = e * npe;
      for (int a = 0; a < npe; ++a) {
        int32_t n = in.elem_nodes[e * npe + a];
        if (n < 0 || n >= in.n_nodes) { t_bad[t] = 1; n = 0; }
        L1.el_nodes[e * npe + a] = plan.node_to_free[n];
      }
      int32_t s = in.elem_to_sub[e];
      if (s < 0) { t_bad[t] = 2; s = 0; }
      L1.el_sub[e] = s;
      nsub_t = std::max(nsub_t, s + 1);
    }
    t_nsub[t] = nsub_t;
  });
  for (char b : t_bad) {
    if (b == 1) return fail(err, MLBDDC_E_ARG, "element node out of range");
    if (b == 2) return fail(err, MLBDDC_E_ARG, "element without a subdomain");
  }
  int32_t nsub = 0;
  for (int32_t x : t_nsub) nsub = std::max(nsub, x);
  L1.el_ptr[in.n_elems] = in.n_elems * npe;
  L1.n_sub = nsub;
  mark("level-1 element arrays");
  mlbddc_status st = build_level(L1, in.constraints, err, plan, in.reuse_layouts);
  if (st != MLBDDC_OK) return st;
  plan.levels.push_back(std::move(L1));
  mark("level 1 done");

  // ---- levels 2..L-1 and the top level from the pseudo-mesh
  for (int l = 2; l <= in.n_levels; ++l) {
    const LevelPlan& P = plan.levels.back();
    LevelPlan L = take_level(l - 1);
    L.level = l;
    L.dim = in.dim;
    L.ndof = in.ndof;
    L.n_nodes = P.n_coarse_nodes;
    L.n_dofs = P.n_coarse;
    L.augmentK = true;
    L.top = (l == in.n_levels);
    L.el_ptr.assign(P.n_sub + 1, 0);
    L.el_sub.resize(P.n_sub);
    // pseudo-elements: the previous level's subdomains, nodes = their constrained globs
    std::vector<std::vector<int64_t>> gl(P.n_sub);
    for (const Glob& g : P.globs)
      if (g.constrained)
        for (int32_t b : g.subs) gl[b].push_back(g.coarse_node);
    int32_t ns = 1;
    for (int32_t b = 0; b < P.n_sub; ++b) {
      L.el_ptr[b + 1] = L.el_ptr[b] + (int64_t)gl[b].size();
      L.el_nodes.insert(L.el_nodes.end(), gl[b].begin(), gl[b].end());
      if (L.top) {
        L.el_sub[b] = 0;
      } else {
        int32_t p = in.sub_to_parent[l - 2] ? in.sub_to_parent[l - 2][b] : -1;
        if (p < 0) return fail(err, MLBDDC_E_ARG, "level " + std::to_string(l) + ": subdomain without a parent");
        L.el_sub[b] = p;
        ns = std::max(ns, p + 1);
      }
    }
    L.n_sub = ns;
    st = build_level(L, L.top ? 0 : (in.constraints & ~MLBDDC_ALL_PRIMAL), err, plan, in.reuse_layouts);
    if (st != MLBDDC_OK) return st;
    plan.levels.push_back(std::move(L));
  }
  mark("levels 2..L");
  old.clear();
  mark("release previous plan");
  return MLBDDC_OK;
}

namespace {

// Step kinds, in launch order within a step.  The trailing updates of the
// sibling groups of one step (tile-structured items) each get their own kind,
// SK_NXT for the first sibling and SK_SIB + j for sibling j: siblings update
// shared separator and interface tiles, so they must not share a launch.
constexpr int MAX_SIBLINGS = 32;
enum { SK_INP = 0, SK_DIA = 1, SK_PAN = 2, SK_NXT = 3, SK_RST = 4, SK_SIB = 4, SK_N = 4 + MAX_SIBLINGS };

// Step layout of a tile-structured item: first step of every group and the
// sibling index of the group among the groups of its height; false when the
// groups cannot advance together (more siblings than launch kinds).
bool tree_steps(const FactorItemDesc& it, std::vector<int32_t>& gstep, std::vector<int32_t>& gsib, int& nsteps) {
  const int ng = it.ngroups;
  int H = 0;
  for (int g = 0; g < ng; ++g) H = std::max(H, (int)it.gheight[g] + 1);
  std::vector<int32_t> width(H, 0), count(H, 0);
  gsib.assign(ng, 0);
  for (int g = 0; g < ng; ++g) {
    const int h = it.gheight[g];
    width[h] = std::max(width[h], it.gtile[g + 1] - it.gtile[g]);
    gsib[g] = count[h]++;
    if (count[h] > MAX_SIBLINGS) return false;
  }
  std::vector<int32_t> base(H + 1, 0);
  for (int h = 0; h < H; ++h) base[h + 1] = base[h] + width[h];
  gstep.assign(ng, 0);
  for (int g = 0; g < ng; ++g) gstep[g] = base[it.gheight[g]];
  nsteps = base[H];
  return true;
}

// Steps of an item (the launch steps its tasks use).
int item_steps(const FactorItemDesc& it) {
  if (it.sptr && it.e2 == 0 && it.gheight) {
    std::vector<int32_t> gstep, gsib;
    int n = 0;
    if (tree_steps(it, gstep, gsib, n)) return n;
  }
  return it.e1 + it.e2;
}

// Tasks of an item with a tile structure (phase 1 only).  Panels start at
// every group boundary.  Column k of a panel starting at k0 takes the
// in-panel update from the panel's earlier columns j whose structure holds k
// (rows: those columns' rows from k on), then its diagonal factor and the
// panel solves of its rows; after the panel, every pair of rows r >= s beyond
// it in the union of the panel's structures is updated.  Rows outside a
// structure hold zero tiles, so the products they add are zero.  Groups of
// one height of the dissection tree advance together: they couple only to
// groups above them, and their trailing updates go to separate launches.
template <typename F>
void enumerate_item_tiles(const FactorItemDesc& it, uint64_t b, int panel, F&& emit) {
  const double t3 = (double)TS * TS * TS;
  const int32_t *sp = it.sptr, *sr = it.srow, *gt = it.gtile;
  std::vector<int32_t> gstep, gsib;
  int nsteps = 0;
  const bool tree = it.gheight && tree_steps(it, gstep, gsib, nsteps);
  std::vector<int32_t> U, V, rows;
  for (int g = 0; g < it.ngroups; ++g) {
    const int g0 = gt[g], g1 = gt[g + 1];
    auto step = [&](int k) { return tree ? gstep[g] + (k - g0) : k; };
    const int trail_kind = !tree || gsib[g] == 0 ? SK_NXT : SK_SIB + gsib[g];
    for (int k0 = g0; k0 < g1; k0 += panel) {
      const int kend = std::min(k0 + panel, g1);
      U.clear();
      for (int k = k0; k < kend; ++k) {
        if (k > k0) {
          rows.clear();
          for (int j = k0; j < k; ++j) {
            const int32_t *c0 = sr + sp[j], *c1 = sr + sp[j + 1];
            const int32_t* q = std::lower_bound(c0, c1, k);
            if (q == c1 || *q != k) continue;
            rows.insert(rows.end(), q, c1);
          }
          std::sort(rows.begin(), rows.end());
          rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
          for (int32_t r : rows) emit(step(k), SK_INP, pack_task(b, r, k, k0, k - 1 - k0), 2.0 * t3 * (k - k0));
        }
        emit(step(k), SK_DIA, pack_task(b, k, k, 0), 2.0 * t3 / 3.0);
        for (int32_t q = sp[k]; q < sp[k + 1]; ++q) emit(step(k), SK_PAN, pack_task(b, sr[q], k, 0), 2.0 * t3);
        V.clear();
        std::set_union(U.begin(), U.end(), sr + sp[k], sr + sp[k + 1], std::back_inserter(V));
        U.swap(V);
      }
      const int k = kend - 1;
      const auto first = std::upper_bound(U.begin(), U.end(), k);
      for (auto qs = first; qs != U.end(); ++qs)
        for (auto qr = qs; qr != U.end(); ++qr)
          emit(step(k), trail_kind, pack_task(b, *qr, *qs, k0, k - k0), 2.0 * t3 * (k - k0 + 1));
    }
  }
}

// All tasks of one item, in (tile column, step kind) order: emit(k, kind, task, flops).
// Rows enter a sorted active list when the elimination reaches their
// envelope, so the loops visit only rows whose tiles are in use.
template <typename F>
void enumerate_item(const FactorItemDesc& it, uint64_t b, int panel, bool lookahead, F&& emit) {
  if (it.sptr && it.e2 == 0) {
    enumerate_item_tiles(it, b, panel, emit);
    return;
  }
  const double t3 = (double)TS * TS * TS;
  const int e1 = it.e1, e2 = it.e2, nt = it.nt;
  const int32_t* env = it.env;
  // rows bucketed by envelope (counting sort, rows increasing within a bucket)
  std::vector<int32_t> start(nt + 1, 0), rows(nt);
  for (int r = 0; r < nt; ++r) start[std::min(std::max(env[r], 0), nt - 1) + 1]++;
  for (int e = 0; e < nt; ++e) start[e + 1] += start[e];
  {
    std::vector<int32_t> pos(start.begin(), start.end() - 1);
    for (int r = 0; r < nt; ++r) rows[pos[std::min(std::max(env[r], 0), nt - 1)]++] = r;
  }
  std::vector<int32_t> act;  // rows with env <= current column, increasing
  act.reserve(nt);
  auto admit = [&](int e) {
    if (e >= nt) return;
    for (int q = start[e]; q < start[e + 1]; ++q) act.insert(std::upper_bound(act.begin(), act.end(), rows[q]), rows[q]);
  };
  admit(0);
  for (int k = 0; k < e1 + e2; ++k) {
    int ph0 = k < e1 ? 0 : e1, ph1 = k < e1 ? e1 : e1 + e2;
    int k0 = ph0 + ((k - ph0) / panel) * panel;
    int kend = std::min(k0 + panel, ph1);
    // second phase: the trailing block after the first is the negative of the
    // matrix it factors; its tasks carry TASK_NEG instead of a negation pass
    const uint64_t neg = k >= e1 ? TASK_NEG : 0;
    // act holds the rows with env <= k - 1 here
    if (k > k0 && env[k] <= k - 1)
      for (auto q = std::lower_bound(act.begin(), act.end(), k); q != act.end(); ++q)
        emit(k, SK_INP, pack_task(b, *q, k, k0, k - 1 - k0) | neg, 2.0 * t3 * (k - k0));
    if (k > 0) admit(k);  // now env <= k
    emit(k, SK_DIA, pack_task(b, k, k, 0) | neg, 2.0 * t3 / 3.0);
    const auto first_after_k = std::upper_bound(act.begin(), act.end(), k);
    for (auto q = first_after_k; q != act.end(); ++q) emit(k, SK_PAN, pack_task(b, *q, k, 0) | neg, 2.0 * t3);
    if (k == kend - 1) {
      // columns of the item's next panel (same phase): with look-ahead they are
      // updated first, on the critical stream
      int nxt_end = k + 1;
      if (lookahead && k + 1 < ph1) nxt_end = std::min(k + 1 + panel, ph1);
      else if (lookahead && k + 1 == e1 && e2 > 0) nxt_end = nt;  // the second phase starts on this block next
      for (auto qs = first_after_k; qs != act.end(); ++qs) {
        const int s = *qs;
        const int dst = (!lookahead || s < nxt_end) ? SK_NXT : SK_RST;
        for (auto qr = qs; qr != act.end(); ++qr)
          emit(k, dst, pack_task(b, *qr, s, k0, k - k0) | neg, 2.0 * t3 * (k - k0 + 1));
      }
    }
  }
}

}  // namespace

// Tasks are ordered by tile column, step kind and item; built in two parallel
// passes over contiguous item ranges (count, then place at prefix offsets).
void build_factor_schedule(const std::vector<FactorItemDesc>& items, int panel, FactorSchedule& out, bool lookahead) {
  out.tasks.clear();
  out.launches.clear();
  out.flops = 0.0;
  out.update_tasks = 0;
  if (panel < 1) panel = 1;
  if (panel > MAX_TASK_NK + 1) panel = MAX_TASK_NK + 1;
  int maxk = 0;
  for (auto& it : items) maxk = std::max(maxk, item_steps(it));
  const int32_t ni = (int32_t)items.size();
  unsigned hw = std::thread::hardware_concurrency();
  int T = (int)std::max(1u, std::min(16u, hw ? hw : 1u));
  T = std::max(1, std::min<int>(T, ni / 4));
  const size_t slots = (size_t)maxk * SK_N;
  std::vector<std::vector<int64_t>> cnt(T, std::vector<int64_t>(slots, 0));
  std::vector<std::vector<double>> fl(T, std::vector<double>(slots, 0.0));
  auto range = [&](int t, int32_t& b0, int32_t& b1) {
    b0 = (int32_t)((int64_t)ni * t / T);
    b1 = (int32_t)((int64_t)ni * (t + 1) / T);
  };
  auto run = [&](auto&& body) { parallel_run(T, body); };
  run([&](int t) {
    int32_t b0, b1;
    range(t, b0, b1);
    for (int32_t b = b0; b < b1; ++b)
      enumerate_item(items[b], (uint64_t)b, panel, lookahead, [&](int k, int kind, uint64_t, double f) {
        cnt[t][(size_t)k * SK_N + kind]++;
        fl[t][(size_t)k * SK_N + kind] += f;
      });
  });
  // offsets: slot-major, thread-minor (= item order within a slot)
  std::vector<std::vector<int64_t>> off(T, std::vector<int64_t>(slots, 0));
  int64_t total = 0;
  auto kind_of = [](int l) { return l == SK_INP ? L_INPANEL : l == SK_DIA ? L_DIAG : l == SK_PAN ? L_PANEL : L_TRAIL; };
  for (size_t sl = 0; sl < slots; ++sl) {
    int64_t n = 0;
    double f = 0.0;
    for (int t = 0; t < T; ++t) {
      off[t][sl] = total + n;
      n += cnt[t][sl];
      f += fl[t][sl];
    }
    if (n > 0) {
      const int k = (int)(sl / SK_N), l = (int)(sl % SK_N);
      FactorLaunch L{kind_of(l), k, total, n, f, 0, false};
      if (lookahead) {
        if (l == SK_RST) { L.stream = 1; L.wait = true; }   // after the panel and the next-panel update
        if (l == SK_NXT) L.wait = true;                    // after the previous bulk update
      }
      if (L.kind == L_TRAIL || L.kind == L_INPANEL) out.update_tasks += n;
      out.flops += f;
      out.launches.push_back(L);
    }
    total += n;
  }
  out.tasks.resize(total);
  run([&](int t) {
    int32_t b0, b1;
    range(t, b0, b1);
    std::vector<int64_t>& o = off[t];
    for (int32_t b = b0; b < b1; ++b)
      enumerate_item(items[b], (uint64_t)b, panel, lookahead, [&](int k, int kind, uint64_t task, double) {
        out.tasks[o[(size_t)k * SK_N + kind]++] = task;
      });
  });
}

}  // namespace mlbddc
