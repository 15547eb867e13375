// Building a design's cell grid (grid.h): cell of every row, counts, an
// exclusive scan into cell starts, then each row and its coordinates
// scattered to its cell's range.  Rows of one cell land in any order (the
// queries order results by (distance, row) themselves).
#include <cmath>

#include "grid.h"
#include "lagp_internal.h"

namespace lagp {

namespace {

__global__ __launch_bounds__(256) void k_grid_count(const double* X, int64_t N, int p, GridDev g, int32_t* cid,
                                                    int32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int c[GRID_Q] = {0, 0, 0};
  for (int k = 0; k < g.q; ++k) c[k] = grid_coord(g, k, X[i * p + k]);
  const int64_t cell = grid_cell(g, c);
  cid[i] = (int32_t)cell;
  atomicAdd(&cnt[cell], 1);
}

// One workgroup: exclusive scan of cnt[0 .. cells) into start[0 .. cells]
// (start may alias cnt only past the counts it has read: it does not here).
constexpr int SCAN_T = 1024;
__global__ __launch_bounds__(SCAN_T) void k_grid_scan(const int32_t* cnt, int64_t cells, int32_t* start) {
  __shared__ int64_t part[SCAN_T];
  const int t = threadIdx.x;
  const int64_t per = (cells + SCAN_T - 1) / SCAN_T;
  const int64_t b = t * per, e = b + per < cells ? b + per : cells;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int k = 0; k < SCAN_T; ++k) {
      const int64_t v = part[k];
      part[k] = run;
      run += v;
    }
    start[cells] = (int32_t)run;
  }
  __syncthreads();
  int64_t run = part[t];
  for (int64_t i = b; i < e; ++i) {
    start[i] = (int32_t)run;
    run += cnt[i];
  }
}

__global__ __launch_bounds__(256) void k_grid_fill(const double* X, int64_t N, int p, const int32_t* cid,
                                                   const int32_t* start, int32_t* cursor, double* Xs, int32_t* rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t cell = cid[i];
  const int64_t e = start[cell] + atomicAdd(&cursor[cell], 1);
  rows[e] = (int32_t)i;
  for (int k = 0; k < p; ++k) Xs[e * p + k] = X[i * p + k];
}

}  // namespace

GridDev grid_plan(int64_t N, int p, const double* lo, const double* hi) {
  GridDev g{};
  g.q = p < GRID_Q ? p : GRID_Q;
  // about two rows per cell, at most 2^22 cells
  int G = (int)std::floor(std::pow((double)N / 2.0, 1.0 / g.q));
  const int gmax = (int)std::floor(std::pow(4194304.0, 1.0 / g.q));
  G = G < 1 ? 1 : (G > gmax ? gmax : G);
  g.wmin = __builtin_huge_val();
  for (int k = 0; k < GRID_Q; ++k) {
    g.G[k] = 1;
    g.lo[k] = 0.0;
    g.inv_w[k] = 0.0;
    if (k >= g.q) continue;
    g.lo[k] = lo[k];
    const double ext = hi[k] - lo[k];
    if (ext > 0.0 && G > 1) {
      g.G[k] = G;
      g.inv_w[k] = (double)G / ext;
      const double w = ext / (double)G;
      g.wmin = w < g.wmin ? w : g.wmin;
    }
  }
  return g;
}

int64_t grid_cells(const GridDev& g) { return (int64_t)g.G[0] * g.G[1] * g.G[2]; }

hipError_t launch_grid_build(const double* X, int64_t N, int p, GridDev& g, int32_t* cid, int32_t* cnt,
                             int32_t* start, double* Xs, int32_t* rows, hipStream_t s) {
  const int64_t cells = grid_cells(g);
  const unsigned nb = (unsigned)((N + 255) / 256);
  hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * cells, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grid_count, dim3(nb), dim3(256), 0, s, X, N, p, g, cid, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(SCAN_T), 0, s, cnt, cells, start);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * cells, s)) != hipSuccess) return e;  // now the cursors
  hipLaunchKernelGGL(k_grid_fill, dim3(nb), dim3(256), 0, s, X, N, p, cid, start, cnt, Xs, rows);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  g.Xs = Xs;
  g.rows = rows;
  g.start = start;
  return hipSuccess;
}

}  // namespace lagp
