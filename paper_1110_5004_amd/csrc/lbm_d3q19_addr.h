// lbm_d3q19_addr.h -- node and pull-source addressing of the D3Q19 kernels
// (periodic wrap, halfway bounce-back and mirror ghosts at walls), shared by
// the fused and the three-kernel step.
#pragma once

#include "lbm_dev.h"
#include "lbm_lattice.h"

namespace lbm {
namespace d3q19 {

__device__ __forceinline__ void coords(const CaseDev& c, unsigned idx, int& x, int& y, int& z) {
  x = idx % c.nx;
  const unsigned r = idx / c.nx;
  y = r % c.ny;
  z = r / c.ny;
}

// Node of the stencil neighbour x + e_i (periodic wrap or mirror ghost).
__device__ __forceinline__ unsigned nbr(const CaseDev& c, int x, int y, int z, int i,
                                        bool interior, unsigned idx) {
  if (interior) return idx + EX(i) + c.nx * (EY(i) + c.ny * EZ(i));
  const int mx = map_axis(x + EX(i), c.nx, c.wall_x);
  const int my = map_axis(y + EY(i), c.ny, c.wall_y);
  const int mz = map_axis(z + EZ(i), c.nz, c.wall_z);
  return mx + c.nx * (my + c.ny * mz);
}

// A node of the node-parallel kernels and its place at the grid's faces.
// The kernels run one grid row (y, z) per blockIdx.x and x across
// blockIdx.y * blockDim.x + threadIdx.x, so y, z and their face flags are
// uniform and only x is per lane; neighbour and pull offsets are then formed
// from compile-time e_i without branches or per-lane division.
struct Node3 {
  int x;
  unsigned idx;
  bool x0, x1, y0, y1, z0, z1;  // x == 0, x == nx - 1, ...
  __device__ __forceinline__ Node3(const CaseDev& c, int xx, int row)
      : Node3(c, xx, row % c.ny, row / c.ny) {}
  __device__ __forceinline__ Node3(const CaseDev& c, int xx, int y, int z) : x(xx) {
    idx = (unsigned)x + (unsigned)c.nx * ((unsigned)y + (unsigned)c.ny * (unsigned)z);
    x0 = x == 0;
    x1 = x == c.nx - 1;
    y0 = y == 0;
    y1 = y == c.ny - 1;
    z0 = z == 0;
    z1 = z == c.nz - 1;
  }
};

// Offset, along one axis of pitch `pitch` and n nodes, of the stencil
// neighbour one step s in {-1, 0, 1} away: the next node; across a periodic
// seam its image; across a wall the mirror ghost, which is the node itself.
__device__ __forceinline__ int face_step(int s, bool lo, bool hi, int wall, int n, int pitch) {
  if (s == 0) return 0;
  const bool out = s > 0 ? hi : lo;
  return out ? (wall ? 0 : -s * (n - 1) * pitch) : s * pitch;
}

// Node of the stencil neighbour x + e_i.
__device__ __forceinline__ unsigned nbr3(const CaseDev& c, const Node3& nd, int i) {
  return nd.idx + face_step(EX(i), nd.x0, nd.x1, c.wall_x, c.nx, 1) +
         face_step(EY(i), nd.y0, nd.y1, c.wall_y, c.ny, c.nx) +
         face_step(EZ(i), nd.z0, nd.z1, c.wall_z, c.nz, c.nx * c.ny);
}

// Offset of the pull source x - s along one axis: the previous node, across a
// periodic seam its image; across a wall the node itself, and bb is set (the
// population is then read in the opposite direction: halfway bounce-back).
__device__ __forceinline__ int pull_step(int s, bool lo, bool hi, int wall, int n, int pitch,
                                         bool& bb) {
  if (s == 0) return 0;
  const bool out = s > 0 ? lo : hi;
  bb = bb || (out && wall);
  return out ? (wall ? 0 : s * (n - 1) * pitch) : -s * pitch;
}

// Byte offset of the population of direction i pulled by the node.
template <int S, bool G, class N>
__device__ __forceinline__ unsigned pull3(const CaseDev& c, const N& nd, int i) {
  using P = Pops<S, Q>;
  if (i == 0) return G ? P::gofs(c, 0, nd.idx) : P::fofs(c, 0, nd.idx);
  bool bb = false;
  const int d = pull_step(EX(i), nd.x0, nd.x1, c.wall_x, c.nx, 1, bb) +
                pull_step(EY(i), nd.y0, nd.y1, c.wall_y, c.ny, c.nx, bb) +
                pull_step(EZ(i), nd.z0, nd.z1, c.wall_z, c.nz, c.nx * c.ny, bb);
  const unsigned j = nd.idx + d;
  if (G) return bb ? P::gofs(c, OPP(i), nd.idx) : P::gofs(c, i, j);
  return bb ? P::fofs(c, OPP(i), nd.idx) : P::fofs(c, i, j);
}

// A staging coordinate g of a tile plus its halo mapped into the grid: the
// periodic image or the wall mirror, then clamped.  Positions a real node
// reads lie at most 2 <= n outside the grid, where one fold is exact; farther
// ones occur only in the unused part of a ragged tile.
__device__ __forceinline__ int fold3(int g, int n, int wall) {
  if (g < 0) g = wall ? -g - 1 : g + n;
  else if (g >= n) g = wall ? 2 * n - 1 - g : g - n;
  return min(max(g, 0), n - 1);
}

}  // namespace d3q19
}  // namespace lbm
