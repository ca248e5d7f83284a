// Element matrices and loads of the model problems (host, FP64).
//
// The library's set-up takes the unit-modulus element matrix K_e^0 and the
// per-element moduli E_e as input (K_e = E_e K_e^0); these helpers produce
// K_e^0 for the structured meshes used by the benchmarks:
//  * Q1 -Laplace on a square: integral of grad N_a . grad N_b, 2x2 Gauss;
//  * trilinear hexahedron, isotropic linear elasticity in index form
//      K_(a,i)(b,j) = int lam dN_a/dx_i dN_b/dx_j
//                     + mu (dN_a/dx_j dN_b/dx_i + delta_ij grad N_a . grad N_b),
//    with lam = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu)), 2x2x2 Gauss.
// Node order: counter-clockwise in 2D; bottom face then top face in 3D.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace {

const int kQuadCorner[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
const int kHexCorner[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

// Gradient of the d-linear shape function of corner `c` at the unit-cube point x (side h).
template <int D>
void shape_grad(const int (*corner)[D], int a, const double* x, double h, double* g) {
  for (int i = 0; i < D; ++i) {
    double v = 1.0 / h;
    for (int j = 0; j < D; ++j) {
      if (j == i) {
        v *= corner[a][j] ? 1.0 : -1.0;
      } else {
        v *= corner[a][j] ? x[j] : 1.0 - x[j];
      }
    }
    g[i] = v;
  }
}

}  // namespace

extern "C" mlbddc_status mlbddc_element_matrix(int32_t kind, double h, double nu, double* out) {
  if (!out || !(h > 0)) return MLBDDC_E_ARG;
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  if (kind == MLBDDC_POISSON_Q1) {
    std::memset(out, 0, sizeof(double) * 16);
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q) {
        double x[2] = {gp[p], gp[q]};
        double g[4][2];
        for (int a = 0; a < 4; ++a) shape_grad<2>(kQuadCorner, a, x, h, g[a]);
        const double w = 0.25 * h * h;  // weight of each Gauss point on the square
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) out[a * 4 + b] += w * (g[a][0] * g[b][0] + g[a][1] * g[b][1]);
      }
    return MLBDDC_OK;
  }
  if (kind == MLBDDC_ELASTICITY_HEX8) {
    if (!(nu > -1.0 && nu < 0.5)) return MLBDDC_E_ARG;
    const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double mu = 1.0 / (2.0 * (1.0 + nu));
    std::memset(out, 0, sizeof(double) * 576);
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 2; ++q)
        for (int r = 0; r < 2; ++r) {
          double x[3] = {gp[p], gp[q], gp[r]};
          double g[8][3];
          for (int a = 0; a < 8; ++a) shape_grad<3>(kHexCorner, a, x, h, g[a]);
          const double w = 0.125 * h * h * h;
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) {
              double dot = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
              for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                  double v = lam * g[a][i] * g[b][j] + mu * (g[a][j] * g[b][i] + (i == j ? dot : 0.0));
                  out[(3 * a + i) * 24 + (3 * b + j)] += w * v;
                }
            }
        }
    return MLBDDC_OK;
  }
  return MLBDDC_E_ARG;
}

extern "C" mlbddc_status mlbddc_element_load(int32_t kind, double h, const double* force, double* out) {
  if (!out || !force || !(h > 0)) return MLBDDC_E_ARG;
  if (kind == MLBDDC_POISSON_Q1) {
    for (int a = 0; a < 4; ++a) out[a] = force[0] * h * h / 4.0;
    return MLBDDC_OK;
  }
  if (kind == MLBDDC_ELASTICITY_HEX8) {
    for (int a = 0; a < 8; ++a)
      for (int c = 0; c < 3; ++c) out[a * 3 + c] = force[c] * h * h * h / 8.0;
    return MLBDDC_OK;
  }
  return MLBDDC_E_ARG;
}

// f = sum over elements of the element load vector, scattered to the free
// DOFs (free nodes in increasing order, components innermost); DOFs of
// Dirichlet nodes are dropped.
extern "C" mlbddc_status mlbddc_assemble_load(const mlbddc_mesh* mesh, const double* elem_load, double* f,
                                              int64_t n_free_dofs) {
  if (!mesh || !elem_load || !f || !mesh->elem_nodes || !mesh->dirichlet_nodes || mesh->n_nodes <= 0 ||
      mesh->n_elems < 0 || mesh->nodes_per_elem <= 0 || mesh->ndof_per_node <= 0)
    return MLBDDC_E_ARG;
  const int64_t nn = mesh->n_nodes;
  const int nd = mesh->ndof_per_node, npe = mesh->nodes_per_elem;
  std::vector<int64_t> free_of(nn);
  int64_t nf = 0;
  for (int64_t v = 0; v < nn; ++v) free_of[v] = mesh->dirichlet_nodes[v] ? -1 : nf++;
  if (nf * nd != n_free_dofs) return MLBDDC_E_ARG;
  std::fill(f, f + n_free_dofs, 0.0);
  for (int64_t e = 0; e < mesh->n_elems; ++e)
    for (int a = 0; a < npe; ++a) {
      const int64_t v = mesh->elem_nodes[e * npe + a];
      if (v < 0 || v >= nn) return MLBDDC_E_ARG;
      if (free_of[v] < 0) continue;
      for (int c = 0; c < nd; ++c) f[free_of[v] * nd + c] += elem_load[a * nd + c];
    }
  return MLBDDC_OK;
}
