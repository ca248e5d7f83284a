// Test program (CPU only): plans a mesh with the library's host planner,
// builds the factorization schedule of one level-1 subdomain and runs its
// tasks on the host in launch order on a random symmetric positive definite
// matrix with the subdomain's element pattern; compares the eliminated
// columns and the updated trailing block with a dense right-looking Cholesky
// of the interior columns, and checks that no two tasks of one launch write
// the same tile.  Tiles outside the set the library zeroes before the
// assembly (read_before_write_tiles) start as NaN: a task that read one would
// spread NaN into the compared tiles.  Before that, the level-1 layouts of
// the plan must equal those of a plan built without reusing the dissection of
// structurally equal subdomains.
//
// usage: schedule_check <dir with meta.txt and *.bin> <subdomain> <panel>
// prints one line; exit status 0 when the comparison passes.
#include "../paper_1201_5991_amd/csrc/plan.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <random>
#include <set>
#include <string>
#include <vector>

using namespace mlbddc;

template <typename T>
static std::vector<T> read_bin(const std::string& f) {
  std::ifstream in(f, std::ios::binary | std::ios::ate);
  const size_t n = (size_t)in.tellg();
  in.seekg(0);
  std::vector<T> v(n / sizeof(T));
  in.read(reinterpret_cast<char*>(v.data()), (std::streamsize)n);
  return v;
}

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  const std::string dir = argv[1];
  const int want = std::atoi(argv[2]), panel = std::atoi(argv[3]);
  std::ifstream meta(dir + "/meta.txt");
  PlanInput in;
  int nparents = 0;
  int64_t nn = 0, ne = 0;
  meta >> in.dim >> in.ndof >> nn >> ne >> in.nodes_per_elem >> in.n_levels >> nparents >> in.constraints;
  in.n_nodes = nn;
  in.n_elems = ne;
  auto en = read_bin<int32_t>(dir + "/elem_nodes.bin");
  auto di = read_bin<uint8_t>(dir + "/dirichlet.bin");
  auto es = read_bin<int32_t>(dir + "/elem_to_sub.bin");
  std::vector<std::vector<int32_t>> par(nparents);
  std::vector<const int32_t*> pp;
  for (int i = 0; i < nparents; ++i) par[i] = read_bin<int32_t>(dir + "/parent" + std::to_string(i) + ".bin");
  for (auto& v : par) pp.push_back(v.data());
  in.elem_nodes = en.data();
  in.dirichlet = di.data();
  in.elem_to_sub = es.data();
  in.sub_to_parent = pp.empty() ? nullptr : pp.data();
  Plan plan;
  Error err;
  if (build_plan(in, plan, err) != MLBDDC_OK) {
    std::printf("plan failed: %s\n", err.message.c_str());
    return 1;
  }
  // the same plan without reusing the dissection of structurally equal
  // subdomains: every level-1 layout must come out the same
  {
    PlanInput in2 = in;
    in2.reuse_layouts = false;
    Plan plan2;
    Error err2;
    if (build_plan(in2, plan2, err2) != MLBDDC_OK) {
      std::printf("plan without reuse failed: %s\n", err2.message.c_str());
      return 1;
    }
    const LevelPlan& A = plan.levels[0];
    const LevelPlan& B = plan2.levels[0];
    for (int b = 0; b < A.n_sub; ++b) {
      const SubPlan& x = A.subs[b];
      const SubPlan& y = B.subs[b];
      if (x.dofI != y.dofI || x.dofG != y.dofG || x.iface != y.iface || x.padI != y.padI || x.gtile != y.gtile ||
          x.gheight != y.gheight || x.sptr != y.sptr || x.srow != y.srow || x.envK != y.envK || x.nIp != y.nIp ||
          x.nGp != y.nGp || x.crow_col != y.crow_col) {
        std::printf("layout of subdomain %d differs with reuse\n", b);
        return 1;
      }
    }
    if (A.el_local != B.el_local || A.el_color != B.el_color) {
      std::printf("element maps differ with reuse\n");
      return 1;
    }
  }
  const LevelPlan& P = plan.levels[0];
  if (want < 0 || want >= P.n_sub) return 2;
  const SubPlan& S = P.subs[want];
  const int tI = (int)(S.nIp / TS), nt = (int)((S.nIp + S.nGp) / TS), N = nt * TS, nI = tI * TS;
  std::vector<FactorItemDesc> items(1);
  items[0].nt = nt;
  items[0].e1 = tI;
  items[0].env = S.envK.data();
  if (!S.sptr.empty()) {
    items[0].sptr = S.sptr.data();
    items[0].srow = S.srow.data();
    items[0].gtile = S.gtile.data();
    items[0].gheight = S.gheight.data();
    items[0].ngroups = (int32_t)S.gtile.size() - 1;
  }
  FactorSchedule fs;
  build_factor_schedule(items, panel, fs, false);

  // A = sum over elements of B_e B_e^T on the element's local positions; a
  // unit diagonal on padding positions, half a unit elsewhere (column-major)
  std::vector<double> A((size_t)N * N, 0.0);
  std::mt19937_64 rng(12345 + want);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<int> dofs;
  std::vector<double> B;
  for (int64_t e : S.elems) {
    dofs.clear();
    for (int32_t j = P.el_local_ptr[e]; j < P.el_local_ptr[e + 1]; ++j)
      if (P.el_local[j] >= 0)
        for (int c = 0; c < P.ndof; ++c) dofs.push_back(P.el_local[j] + c);
    const int d = (int)dofs.size();
    B.resize((size_t)d * d);
    for (auto& x : B) x = nd(rng);
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) {
        double s = 0.0;
        for (int q = 0; q < d; ++q) s += B[a * d + q] * B[c * d + q];
        A[(size_t)dofs[c] * N + dofs[a]] += s;
      }
  }
  for (int i = 0; i < N; ++i) A[(size_t)i * N + i] += A[(size_t)i * N + i] == 0.0 ? 1.0 : 0.5;

  // reference: dense partial Cholesky of the interior columns (column-major,
  // lower triangle), the trailing block updated
  std::vector<double> R = A;
  for (int k = 0; k < nI; ++k) {
    double* ck = R.data() + (size_t)k * N;
    const double p = std::sqrt(ck[k]);
    ck[k] = p;
    for (int i = k + 1; i < N; ++i) ck[i] /= p;
    for (int j = k + 1; j < N; ++j) {
      const double l = ck[j];
      if (l == 0.0) continue;
      double* cj = R.data() + (size_t)j * N;
      for (int i = j; i < N; ++i) cj[i] -= ck[i] * l;
    }
  }

  // tiles the library zeroes before assembling (all of them without a tile structure)
  std::vector<char> zset((size_t)nt * nt, 0);
  if (!S.sptr.empty())
    read_before_write_tiles(items[0], [&](int r0, int k, int count) {
      for (int r = r0; r < r0 + count; ++r) zset[(size_t)k * nt + r] = 1;
    });
  else
    for (int k = 0; k < nt; ++k)
      for (int r = k; r < nt; ++r) zset[(size_t)k * nt + r] = 1;
  auto tile_nonzero = [&](const std::vector<double>& M, int r, int k) {
    for (int j = 0; j < TS; ++j)
      for (int i = 0; i < TS; ++i)
        if (M[(size_t)(k * TS + j) * N + r * TS + i] != 0.0) return true;
    return false;
  };
  bool cover = true;  // every assembled or factor tile lies in the zeroed set
  for (int k = 0; k < nt; ++k)
    for (int r = k; r < nt; ++r)
      if (!zset[(size_t)k * nt + r] && (tile_nonzero(A, r, k) || tile_nonzero(R, r, k))) cover = false;

  // the schedule's tasks on tiles of X (column-major N x N; tile (r, s) at
  // rows 64 r.., columns 64 s..), inverse diagonal tiles in W
  std::vector<double> X = A, W((size_t)tI * TE, 0.0), tmp(TE);
  auto el = [&](int r, int s, int i, int j) -> double& { return X[(size_t)(s * TS + j) * N + r * TS + i]; };
  for (int k = 0; k < nt; ++k)
    for (int r = k; r < nt; ++r)
      if (!zset[(size_t)k * nt + r])
        for (int j = 0; j < TS; ++j)
          for (int i = 0; i < TS; ++i) el(r, k, i, j) = std::nan("");
  bool conflict = false;
  for (const FactorLaunch& F : fs.launches) {
    std::set<std::pair<int, int>> written;
    for (int64_t q = F.first; q < F.first + F.count; ++q) {
      const uint64_t t = fs.tasks[q];
      const int r = task_r(t), s = task_s(t), kf = task_kf(t), kl = kf + task_nk(t);
      if (!written.insert({r, s}).second) conflict = true;
      if (F.kind == L_DIAG) {
        for (int c = 0; c < TS; ++c) {
          const double pv = std::sqrt(el(r, r, c, c));
          el(r, r, c, c) = pv;
          for (int i = c + 1; i < TS; ++i) el(r, r, i, c) /= pv;
          for (int j = c + 1; j < TS; ++j)
            for (int i = j; i < TS; ++i) el(r, r, i, j) -= el(r, r, i, c) * el(r, r, j, c);
        }
        double* w = W.data() + (size_t)r * TE;  // w = L^{-1}, row-major
        for (int c = 0; c < TS; ++c)
          for (int i = 0; i < TS; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) v -= el(r, r, i, j) * w[j * TS + c];
            w[i * TS + c] = v / el(r, r, i, i);
          }
      } else if (F.kind == L_PANEL) {  // A_rs <- A_rs L_ss^{-T}
        const double* w = W.data() + (size_t)s * TE;
        for (int i = 0; i < TS; ++i)
          for (int j = 0; j < TS; ++j) {
            double v = 0.0;
            for (int k = 0; k < TS; ++k) v += el(r, s, i, k) * w[j * TS + k];
            tmp[i * TS + j] = v;
          }
        for (int i = 0; i < TS; ++i)
          for (int j = 0; j < TS; ++j) el(r, s, i, j) = tmp[i * TS + j];
      } else if (F.kind == L_TRAIL || F.kind == L_INPANEL) {  // A_rs -= sum_kk A_r,kk A_s,kk^T
        for (int kk = kf; kk <= kl; ++kk)
          for (int j = 0; j < TS; ++j)
            for (int k = 0; k < TS; ++k) {
              const double b = el(s, kk, j, k);
              if (b == 0.0) continue;
              for (int i = 0; i < TS; ++i) el(r, s, i, j) -= el(r, kk, i, k) * b;
            }
      } else {
        std::printf("unexpected launch kind %d\n", F.kind);
        return 1;
      }
    }
  }
  double md = 0.0, mr = 0.0;
  bool finite = true;
  for (int j = 0; j < N; ++j)
    for (int i = j; i < N; ++i) {
      if (!zset[(size_t)(j / TS) * nt + i / TS]) continue;
      const double a = X[(size_t)j * N + i], c = R[(size_t)j * N + i];
      if (!std::isfinite(a)) finite = false;
      md = std::max(md, std::fabs(a - c));
      mr = std::max(mr, std::fabs(c));
    }
  const bool ok = !conflict && cover && finite && md <= 1e-10 * mr;
  long nz = 0;
  for (char z : zset) nz += z;
  std::printf("subdomain %d tiles %d interior %d groups %d launches %zu tasks %zu zeroed tiles %ld of %d conflict %d "
              "cover %d finite %d max|diff| %.3e max|ref| %.3e %s\n",
              want, nt, tI, S.gtile.empty() ? 1 : (int)S.gtile.size() - 1, fs.launches.size(), fs.tasks.size(), nz,
              nt * (nt + 1) / 2, (int)conflict, (int)cover, (int)finite, md, mr, ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}
