// Cell grid over a design's leading coordinates, for nearest-row queries
// over the whole design (the ray search's snap when it is not restricted to
// the N' nearest candidates, Sec. 5).
//
// The first q = min(p, 3) coordinates are cut into G_k equal cells between
// the design's per-dimension minimum and maximum (G_k = 1 where they are
// equal).  Rows are grouped by cell: entry e of the grouping holds design
// row rows[e] and its p coordinates Xs[e p .. e p + p - 1]; cell c holds
// entries start[c] .. start[c + 1] - 1.  The grid only decides which rows
// are examined; distances and the order of results are those of the rows
// themselves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lagp {

constexpr int GRID_Q = 3;  // grid dimensions at most

struct GridDev {
  const double* Xs;      // N x p coordinates, grouped by cell
  const int32_t* rows;   // N: the design row of each grouped entry
  const int32_t* start;  // cells + 1: first entry of each cell
  int32_t q;             // coordinates the grid cuts (the first q), 1 .. 3
  int32_t G[GRID_Q];     // cells per grid coordinate (1 past q)
  double lo[GRID_Q];     // origin per grid coordinate
  double inv_w[GRID_Q];  // cells per unit length (0 where G_k = 1)
  double wmin;           // narrowest cell width over coordinates with G_k > 1 (+inf if none)
};

// Cell coordinate of value v along grid coordinate k (clamped to the grid;
// NaN lands in cell 0).  Index and build use this same function.
__host__ __device__ inline int grid_coord(const GridDev& g, int k, double v) {
  const double t = (v - g.lo[k]) * g.inv_w[k];
  if (!(t >= 0.0)) return 0;
  return t < (double)g.G[k] ? (int)t : g.G[k] - 1;
}

__host__ __device__ inline int64_t grid_cell(const GridDev& g, const int (&c)[GRID_Q]) {
  return ((int64_t)c[2] * g.G[1] + c[1]) * g.G[0] + c[0];
}

}  // namespace lagp
