// Host helpers that build the coarse grids the solver takes as input.
//
// Matrix (Sec. 3, Fig. 2): primal blocks of c cells per axis (the last one
// possibly shorter); the coarse node of a block is its centre cell per axis;
// a cell's wirebasket class is the number of its coordinates on a node plane
// (3 = vertex, 2 = edge, 1 = face, 0 = interior).
//
// Fractures: the distance-based coarsening of Table 2 on the x-y projection
// of each network, extruded along z (Sec. 4.3).  The choices the paper
// leaves open are fixed as documented in fams.h.
#include <algorithm>
#include <cstdint>
#include <deque>
#include <limits>
#include <vector>

#include "../../include/fams.h"

namespace {

std::vector<int64_t> axis_nodes(int n, int c) {
  std::vector<int64_t> v;
  for (int s = 0; s < n; s += c) {
    int e = std::min(s + c, n);
    v.push_back(s + (e - s) / 2);
  }
  return v;
}

// Table 2 on a graph given in CSR: returns the vertex flag of every node.
std::vector<char> distance_coarsening(int64_t n, const int64_t* ptr, const int32_t* adj,
                                      int32_t d_min) {
  const int64_t INF = std::numeric_limits<int64_t>::max();
  const int64_t dmax = d_min <= 0 ? INF : d_min;
  std::vector<int64_t> level(n, INF);
  std::vector<char> is_vertex(n, 0), seen(n, 0), queued(n, 0);
  std::vector<int64_t> stack;
  for (int64_t start = 0; start < n; ++start) {
    if (seen[start]) continue;
    stack.assign(1, start);
    seen[start] = 1;
    while (!stack.empty()) {
      int64_t c = stack.back();
      stack.pop_back();
      for (int64_t q = ptr[c]; q < ptr[c + 1]; ++q)
        if (!seen[adj[q]]) {
          seen[adj[q]] = 1;
          stack.push_back(adj[q]);
        }
    }
    std::deque<int64_t> qv{start};
    queued[start] = 1;
    while (!qv.empty()) {
      int64_t v = qv.front();
      qv.pop_front();
      queued[v] = 0;
      is_vertex[v] = 1;
      level[v] = 0;
      std::vector<int64_t> q1{v}, q2;
      int64_t dist = 1;
      while (dist <= dmax && !q1.empty()) {
        q2.clear();
        for (int64_t c : q1)
          for (int64_t q = ptr[c]; q < ptr[c + 1]; ++q) {
            int64_t nb = adj[q];
            if (level[nb] > dist) {
              if (queued[nb]) {
                qv.erase(std::find(qv.begin(), qv.end(), nb));
                queued[nb] = 0;
              }
              level[nb] = dist;
              q2.push_back(nb);
            }
          }
        q1.swap(q2);
        ++dist;
      }
      if (dist > dmax)
        for (int64_t c : q1) {
          qv.push_back(c);
          queued[c] = 1;
        }
    }
  }
  return is_vertex;
}

}  // namespace

extern "C" fams_status_t fams_grid_structured(int32_t nx, int32_t ny, int32_t nz, int32_t cx,
                                              int32_t cy, int32_t cz, int8_t* wb_type,
                                              int32_t* primal, int64_t* vertex,
                                              int64_t* n_coarse) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || cx <= 0 || cy <= 0 || cz <= 0 || !n_coarse)
    return FAMS_ERR_INVALID_ARG;
  auto X = axis_nodes(nx, cx), Y = axis_nodes(ny, cy), Z = axis_nodes(nz, cz);
  const int64_t bx = X.size(), by = Y.size(), bz = Z.size();
  *n_coarse = bx * by * bz;
  if (!wb_type && !primal && !vertex) return FAMS_OK;
  std::vector<char> ox(nx, 0), oy(ny, 0), oz(nz, 0);
  for (auto v : X) ox[v] = 1;
  for (auto v : Y) oy[v] = 1;
  for (auto v : Z) oz[v] = 1;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t i = x + static_cast<int64_t>(nx) * (y + static_cast<int64_t>(ny) * z);
        if (wb_type) wb_type[i] = static_cast<int8_t>(ox[x] + oy[y] + oz[z]);
        if (primal) primal[i] = static_cast<int32_t>(x / cx + bx * (y / cy + by * (z / cz)));
      }
  if (vertex)
    for (int64_t k = 0; k < bz; ++k)
      for (int64_t j = 0; j < by; ++j)
        for (int64_t i = 0; i < bx; ++i)
          vertex[i + bx * (j + by * k)] = X[i] + nx * (Y[j] + static_cast<int64_t>(ny) * Z[k]);
  return FAMS_OK;
}

extern "C" fams_status_t fams_grid_fracture(
    int64_t n_matrix, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
    const int32_t* cell_col, const int32_t* cell_z, int64_t n_cols, const int32_t* col_plate,
    const int64_t* col_ptr, const int32_t* col_adj, int64_t n_plates, const int32_t* plate_zlo,
    const int32_t* plate_zhi, int32_t d_min, int32_t r_z, int64_t n_coarse_matrix,
    int8_t* wb_type, int32_t* primal, int64_t* vertex, int64_t* n_coarse_frac) {
  if (!n_coarse_frac || n < n_matrix || r_z < 1) return FAMS_ERR_INVALID_ARG;
  const int64_t nf = n - n_matrix;
  *n_coarse_frac = 0;
  if (nf == 0) return FAMS_OK;
  if (!row_ptr || !col_idx || !cell_col || !cell_z || !col_plate || !col_ptr || !plate_zlo ||
      !plate_zhi || !wb_type || !primal || !vertex)
    return FAMS_ERR_INVALID_ARG;
  std::vector<char> vcol = distance_coarsening(n_cols, col_ptr, col_adj, d_min);
  // coarse layers of every plate
  std::vector<std::vector<int32_t>> layers(n_plates);
  for (int64_t p = 0; p < n_plates; ++p) {
    for (int32_t k = plate_zlo[p]; k < plate_zhi[p]; ++k)
      if (k % r_z == r_z / 2) layers[p].push_back(k);
    if (layers[p].empty()) layers[p].push_back(plate_zlo[p] + (plate_zhi[p] - plate_zlo[p] - 1) / 2);
  }
  for (int64_t c = 0; c < nf; ++c) {
    bool a = vcol[cell_col[c]] != 0;
    const auto& L = layers[col_plate[cell_col[c]]];
    bool b = std::find(L.begin(), L.end(), cell_z[c]) != L.end();
    wb_type[c] = static_cast<int8_t>(a && b ? 3 : (a || b ? 2 : 1));
  }
  // fracture-fracture adjacency (local indices)
  std::vector<int64_t> fptr(nf + 1, 0);
  std::vector<int64_t> fadj;
  for (int64_t c = 0; c < nf; ++c) {
    int64_t i = n_matrix + c;
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      int64_t j = col_idx[q];
      if (j >= n_matrix && j < n && j != i) fadj.push_back(j - n_matrix);  // fracture cells only
    }
    fptr[c + 1] = static_cast<int64_t>(fadj.size());
  }
  // blocks of one class without a higher-class neighbour: promote lowest cell
  auto repair = [&](int cls, int min_higher) {
    std::vector<char> done(nf, 0);
    std::vector<int64_t> members, st;
    for (int64_t s = 0; s < nf; ++s) {
      if (wb_type[s] != cls || done[s]) continue;
      members.assign(1, s);
      st.assign(1, s);
      done[s] = 1;
      while (!st.empty()) {
        int64_t c = st.back();
        st.pop_back();
        for (int64_t q = fptr[c]; q < fptr[c + 1]; ++q) {
          int64_t nb = fadj[q];
          if (wb_type[nb] == cls && !done[nb]) {
            done[nb] = 1;
            members.push_back(nb);
            st.push_back(nb);
          }
        }
      }
      bool ok = false;
      for (int64_t c : members)
        for (int64_t q = fptr[c]; q < fptr[c + 1] && !ok; ++q)
          if (wb_type[fadj[q]] >= min_higher) ok = true;
      if (!ok) wb_type[*std::min_element(members.begin(), members.end())] = 3;
    }
  };
  repair(2, 3);
  repair(1, 2);
  // coarse ids of fracture vertices: ascending fine index
  std::vector<int64_t> coarse(nf, -1);
  int64_t nv = 0;
  for (int64_t c = 0; c < nf; ++c)
    if (wb_type[c] == 3) {
      coarse[c] = n_coarse_matrix + nv;
      vertex[nv++] = n_matrix + c;
    }
  *n_coarse_frac = nv;
  // nearest-vertex primal blocks (breadth-first from all vertices at once)
  std::vector<int64_t> dist(nf, -1), owner(nf, -1), frontier, next;
  for (int64_t c = 0; c < nf; ++c)
    if (wb_type[c] == 3) {
      dist[c] = 0;
      owner[c] = coarse[c];
      frontier.push_back(c);
    }
  for (int64_t d = 0; !frontier.empty(); ++d) {
    next.clear();
    for (int64_t c : frontier)
      for (int64_t q = fptr[c]; q < fptr[c + 1]; ++q) {
        int64_t nb = fadj[q];
        if (dist[nb] < 0) {
          dist[nb] = d + 1;
          owner[nb] = owner[c];
          next.push_back(nb);
        } else if (dist[nb] == d + 1 && owner[c] < owner[nb]) {
          owner[nb] = owner[c];
        }
      }
    frontier.swap(next);
  }
  for (int64_t c = 0; c < nf; ++c) {
    if (owner[c] < 0) return FAMS_ERR_BAD_GRID;
    primal[c] = static_cast<int32_t>(owner[c]);
  }
  return FAMS_OK;
}
