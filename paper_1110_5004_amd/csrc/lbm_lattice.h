// lbm_lattice.h -- velocity sets of the gfx950 kernels.
//
// D2Q9 (the paper's lattice, weights 4/9, 1/9, 1/36):
//   0 rest; 1..4 = +x, +y, -x, -y; 5..8 = (+,+), (-,+), (-,-), (+,-).
// D3Q19 (weights 1/3, 1/18, 1/36):
//   0 rest; 1..6 = +x, -x, +y, -y, +z, -z; 7..18 = the 12 edge diagonals in
//   opposite pairs (+x+y, -x-y), (+x-y, -x+y), (+x+z, -x-z), (+x-z, -x+z),
//   (+y+z, -y-z), (+y-z, -y+z).
// Plane i of the stored populations holds direction i.
#pragma once

namespace lbm {
namespace d2q9 {
constexpr int Q = 9;
__host__ __device__ constexpr int EX(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int EY(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int OPP(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
__host__ __device__ constexpr float WT(int i) {
  return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
}
}  // namespace d2q9

namespace d3q19 {
constexpr int Q = 19;
__host__ __device__ constexpr int EX(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13)
             ? 1
             : ((i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0);
}
__host__ __device__ constexpr int EY(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17)
             ? 1
             : ((i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0);
}
__host__ __device__ constexpr int EZ(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18)
             ? 1
             : ((i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0);
}
__host__ __device__ constexpr int OPP(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr float WT(int i) {
  return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
}  // namespace d3q19
}  // namespace lbm
