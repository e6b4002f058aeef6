// lbm_d3q19_march.hip -- the fused D3Q19 step for 16-bit population storage.
//
// k3_march<S, TX, TY, RF>: one workgroup owns a TX x TY tile of the x-y plane
// and the planes [za, zb) of one z chunk, and marches up the chunk with rings
// of planes in LDS (one float per position):
//   RF = 1 (a lap mu term in the step: the corrected model of Eq. 5):
//     phi over the tile + 3 (4 planes), mu over the tile + 2 (3 planes), p over
//     the tile + 1 (3 planes); iteration z stages phi(z + 3) from the pulled f,
//     forms mu(z + 2), pulls the gbar moments and forms grad phi, lap mu, u and
//     p at z + 1, then collides plane z;
//   RF = 0 (no lap mu term: the original model): phi over the tile + 2 (3
//     planes), p over the tile + 1; iteration z stages phi(z + 2), forms mu,
//     grad phi, u and p at z + 1 from the phi stencil at the position, then
//     collides plane z.
// Each population is fetched from HBM about once: a thread keeps its own
// node's pulled f as packed 16-bit words from the phi stage to the collision,
// and its gbar from the u, p stage to the collision one plane later (both in
// a private part of LDS); the halo positions mostly hit L2.  The per-node
// arithmetic is the lean form of lbm_d3q19_lean.h, shared with the
// three-kernel step, so both give the same bits.
//
// Memory instructions, not bytes, bound a 16-bit step: one 2-byte access per
// lane and population keeps the texture addresser busy.  So lanes 2m and
// 2m + 1, which hold x-adjacent nodes x (even) and x + 1, share their
// accesses: for a pair of populations (i, i') the even lane loads population
// i and the odd lane population i' as one 32-bit word covering both nodes (a
// pull shifted along x is a 2-byte-aligned word), then a DPP swap between the
// two lanes and one v_perm give each lane its own node's (i, i') pair -- the
// packed layout the collision takes.  Stores run the same exchange backwards.
// This halves the memory instructions of interior tiles.
//
// Addressing of the pulls, chosen per tile (uniform):
//   inner  every pull source of the staged region lies inside the grid in x
//          and y: lane-pair words, the direction's shift and plane in the
//          uniform offset (z: wrap, or bounce-back at a z wall, a uniform
//          choice per plane);
//   seam   no wall in x or y but a periodic seam within reach: one 16-bit
//          word per lane and population, nine wrapped per-lane offsets;
//   wall   a wall in x or y: the general pull with halfway bounce-back.
// Staged regions are pair-aligned along x (the phi region spans the tile + 4
// for radius 3, the u, p region the tile + 2); positions beyond what a stencil
// needs are loaded for the pair and not computed.  Positions beyond a wall:
// phi is staged from the mirror node; mu, u and p at a position beyond an x
// or y wall are formed around the mirror position; along z, planes beyond a
// wall are not formed and their reads go to the mirror plane.  The grid must
// be even along x (odd widths run the three-kernel step).
#include "lbm_d3q19_addr.h"
#include "lbm_d3q19_lean.h"
#include "lbm_dev.h"
#include "lbm_kernels.h"
#include "lbm_lattice.h"

namespace lbm {
namespace d3q19 {

template <int TX, int TY, int RF>
struct MarchLds {
  static constexpr int NT = TX * TY;
  static constexpr int R = RF ? 3 : 2;        // radius of the phi stencil chain
  static constexpr int RX = (R + 1) & ~1;     // x margin of the phi region (pair-aligned)
  static constexpr int PX = TX + 2 * RX, PY = TY + 2 * R, NP = PX * PY;
  static constexpr int NPH = RF ? 4 : 3;      // phi planes
  static constexpr int MX = TX + 4, MY = TY + 4, NM = RF ? MX * MY : 1;
  static constexpr int UX = TX + 4, UY = TY + 2, NU = UX * UY;  // u, p region (x margin 2)
  static constexpr int NFC = RF ? 3 : 2;      // planes of the own node's carried f words
  float ph[NPH][NP];
  float mu[RF ? 3 : 1][NM];
  float p[3][NU];
  // per thread (private, no barrier): the own node's packed f words of the
  // planes between its phi stage and its collision, and its packed gbar words
  // from the u, p stage to the collision one plane later; word j of thread t
  // at [slot][j][t], so a wave's accesses fall in consecutive banks
  uint32_t fw[NFC][9][NT];
  uint32_t gw[2][10][NT];
};

enum { AD_INNER = 0, AD_SEAM = 1, AD_WALL = 2 };

// The plane whose mu / p a read of plane k takes: k itself, or across a wall
// along z the mirror plane (a halfway wall mirrors the plane next to it).
__device__ __forceinline__ int zread_m(const CaseDev& c, int k) {
  return c.wall_z ? min(max(k, 0), c.nz - 1) : k;
}

__device__ __forceinline__ int ring3(int k) { return (k + 6) % 3; }
__device__ __forceinline__ int ring4(int k) { return (k + 8) & 3; }
template <int RF>
__device__ __forceinline__ int phslot(int k) {
  if constexpr (RF) return ring4(k);
  else return ring3(k);
}

// Buffer access to one state copy: a 128-bit resource in scalar registers,
// a 32-bit uniform offset in one scalar register and a 32-bit per-lane offset
// (buffer_load / buffer_store ... offen).  The uniform part of an address
// (plane, z plane, the inner pull shift) costs one scalar add, and no pair of
// scalar registers per plane stays live.  A copy is below 4 GiB, so 32-bit
// offsets cover it; the resource spans the whole 32-bit range.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc copy_rsrc(const char* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), 0, -1, 0x00020000);
}
__device__ __forceinline__ uint16_t bload16(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ uint32_t bload32(Rsrc r, unsigned voff, unsigned soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ float bload32f(Rsrc r, unsigned voff, unsigned soff) {
  return __uint_as_float(bload32(r, voff, soff));
}
// Stores carry the non-temporal cache policy (bit 1 of the buffer
// instruction's cache-policy operand): a stored population is not read again
// until the next step, and streaming it past the caches leaves them to the
// halo lines the march re-reads.
constexpr int kStoreNT = 2;
__device__ __forceinline__ void bstore16(Rsrc r, unsigned voff, unsigned soff, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)voff, (int)soff, kStoreNT);
}
__device__ __forceinline__ void bstore32(Rsrc r, unsigned voff, unsigned soff, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, kStoreNT);
}
__device__ __forceinline__ void bstore32f(Rsrc r, unsigned voff, unsigned soff, float v) {
  bstore32(r, voff, soff, __float_as_uint(v));
}

// Lane pairs.  The even lane of a pair holds word A, the odd lane word B,
// each covering the pair's two nodes (low half: even node, high half: odd
// node).  Returns the calling lane's own node's halves of A and B, as (A, B)
// in (low, high): a swap of the pair's registers (DPP quad_perm [1,0,3,2])
// and a byte permutation whose selector depends on the lane's parity
// (psel: 0x01000504 on even lanes, 0x07060302 on odd lanes; v_perm numbers
// the bytes of its second operand 0..3 and of its first 4..7).
__device__ __forceinline__ uint32_t pair_xchg(uint32_t own, uint32_t psel) {
  const uint32_t other = (uint32_t)__builtin_amdgcn_mov_dpp((int)own, 0xB1, 0xF, 0xF, false);
  return __builtin_amdgcn_perm(own, other, psel);
}

// Load of a lane pair: the even lane's word at uniform offset a, the odd
// lane's at b, both from the pair's even node (lane offset base).  Buffer
// addressing adds a 32-bit lane offset zero-extended, so the smaller of a and
// b goes in the uniform offset and only the (non-negative) difference is added
// on the lanes that need it.
__device__ __forceinline__ uint32_t pair_load(Rsrc src, unsigned base, unsigned a, unsigned b,
                                              uint32_t oddmask) {
  if (b >= a) return bload32(src, base + ((b - a) & oddmask), a);
  return bload32(src, base + ((a - b) & ~oddmask), b);
}

// Offsets of one plane of the copy: st2 = 2 x the plane stride (bytes of a
// 16-bit plane), z2 = 2 nx ny (bytes of one z plane in a 16-bit plane).
// Both are passed through an empty asm once per z iteration of the kernel,
// which keeps the compiler from hoisting every plane's offset out of the
// loop into its own scalar register.
struct PlaneOfs {
  unsigned st2, z2;
  // byte offset of plane i of f (i > 0) or gbar in the 16-bit layout (f_0 is
  // the float plane at offset 0)
  template <bool G>
  __device__ __forceinline__ unsigned plane(int i) const {
    return st2 * (unsigned)(G ? Q + 1 + i : i + 1);
  }
};

// Uniform offset of the pull of direction i into plane k (0 <= k < nz) of an
// inner site whose lane offset is the node's own: the source plane k - e_z
// (wrapped), the xy shift -e_i, or across a z wall the opposite direction at
// the node itself (halfway bounce-back).
template <bool G>
__device__ __forceinline__ unsigned inner_soff(const CaseDev& c, const PlaneOfs& po, int k,
                                               int i) {
  int zs = k - EZ(i);
  if (EZ(i) != 0 && (zs < 0 || zs >= c.nz)) {
    if (c.wall_z) return po.plane<G>(OPP(i)) + po.z2 * (unsigned)k;
    zs = zs < 0 ? zs + c.nz : zs - c.nz;
  }
  // every f or gbar plane lies past the f_0 plane, so the shift keeps the
  // offset non-negative
  return po.plane<G>(i) + po.z2 * (unsigned)zs - 2u * (unsigned)(EX(i) + c.nx * EY(i));
}

// Per-lane pull offsets of one staged position (qx, qy) in the x-y plane.
struct Site {
  unsigned self;    // 2 (qx + nx qy): byte offset of the node in a 16-bit plane
  unsigned cmb[9];  // seam: 2 (x_src + nx y_src) for e_x, e_y in {-1, 0, 1}
};
template <int MODE>
__device__ __forceinline__ Site make_site(const CaseDev& c, int qx, int qy) {
  Site s{};  // every member defined: the aggregate is returned as a noundef value
  s.self = 2u * (unsigned)(qx + c.nx * qy);
  if constexpr (MODE == AD_SEAM) {
    // source x - e_x for e_x = -1, 0, 1 (periodic wrap)
    const int xs[3] = {qx + 1 == c.nx ? 0 : qx + 1, qx, qx == 0 ? c.nx - 1 : qx - 1};
    const int ys[3] = {qy + 1 == c.ny ? 0 : qy + 1, qy, qy == 0 ? c.ny - 1 : qy - 1};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) s.cmb[a + 3 * b] = 2u * (unsigned)(xs[a] + c.nx * ys[b]);
  }
  return s;
}
// Combination index of direction i in Site::cmb.
__device__ __forceinline__ constexpr int cmb_of(int i) { return (EX(i) + 1) + 3 * (EY(i) + 1); }

// One 16-bit word of direction i (G: gbar, else f) for the site at plane k,
// seam or wall addressing (one word per lane).
template <int S, bool G, int MODE>
__device__ __forceinline__ uint16_t pull_word(const CaseDev& c, Rsrc src, const PlaneOfs& po,
                                              const Site& s, int qx, int qy, int k, int i) {
  if constexpr (MODE == AD_WALL) {
    const Node3 nd(c, qx, qy, k);
    return bload16(src, pull3<S, G>(c, nd, i), 0u);
  } else {
    int zs = k - EZ(i);
    if (EZ(i) != 0 && (zs < 0 || zs >= c.nz)) {
      if (c.wall_z) return bload16(src, s.self, po.plane<G>(OPP(i)) + po.z2 * (unsigned)k);
      zs = zs < 0 ? zs + c.nz : zs - c.nz;
    }
    return bload16(src, s.cmb[cmb_of(i)], po.plane<G>(i) + po.z2 * (unsigned)zs);
  }
}

// Position (px, py) in a region of PXr x PYr of the r-th ring position
// around its inner part: WY rows at the top, WY at the bottom, then WX
// columns on each side of the middle rows.  With PXr and WX even, ring
// positions 2m and 2m + 1 are x-adjacent with the even one at even px.
template <int PXr, int PYr, int WX, int WY>
__device__ __forceinline__ void ring_pos(int r, int& px, int& py) {
  if (r < WY * PXr) {
    px = r % PXr;
    py = r / PXr;
  } else if (r < 2 * WY * PXr) {
    const int q = r - WY * PXr;
    px = q % PXr;
    py = PYr - WY + q / PXr;
  } else {
    const int q = r - 2 * WY * PXr, col = q % (2 * WX);
    px = col < WX ? col : PXr - 2 * WX + col;
    py = WY + q / (2 * WX);
  }
}

// Everything a workgroup needs about its tile.
struct MarchTile {
  int x0, y0, za, zb;
  bool wall_xy;  // positions beyond an x or y wall within reach
};

// The raw loads of one site, packed per node as the collision takes them:
// f[j] = (f_{2j-1}, f_{2j}) (j = 1..9), g[k] = (gbar_{2k}, gbar_{2k+1})
// (gbar_18 in the low half of g[9]).  Inner sites hold the pair words until
// pair_xchg turns them into the lane's own node's words.
struct FLoads {
  float f0;
  uint32_t w[10];
};
struct GLoads {
  uint32_t w[10];
};

// Issue the loads of one site.  Inner: the lane-pair words (even lane: the
// first population of each packed pair, odd lane: the second; the odd lane's
// offset adds the uniform difference between the two pulls).  Seam / wall:
// one word per population, packed.
// Inner sites load a pair of planes as lane-pair words only where both pulls
// keep the 4-byte alignment of the pair's even node (no x shift: e_x = 0);
// pulls shifted along x would make those words straddle 4-byte boundaries,
// and the unaligned dword costs more than the two 2-byte loads it saves.
__device__ __forceinline__ constexpr bool f_paired(int j) { return EX(PI(j)) == 0; }
__device__ __forceinline__ constexpr bool g_paired(int q) {
  return EX(2 * q) == 0 && (2 * q + 1 >= Q || EX(2 * q + 1) == 0);
}

template <int S, int MODE>
__device__ __forceinline__ void issue_f(const CaseDev& c, Rsrc src, const PlaneOfs& po, int qx,
                                        int qy, int k, uint32_t odd, FLoads& L) {
  const Site s = make_site<MODE>(c, qx, qy);
  if constexpr (MODE == AD_INNER) {
    const unsigned base = s.self - 2u * odd;  // the pair's even node
#pragma unroll
    for (int j = 1; j <= 9; ++j) {
      const unsigned a = inner_soff<false>(c, po, k, PI(j));
      const unsigned b = inner_soff<false>(c, po, k, PI(j) + 1);
      if (f_paired(j)) L.w[j] = pair_load(src, base, a, b, 0u - odd);
      else L.w[j] = pack16(bload16(src, s.self, a), bload16(src, s.self, b));
    }
    L.f0 = bload32f(src, 2u * s.self, 2u * po.z2 * (unsigned)k);
  } else {
    uint16_t h[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) h[i] = pull_word<S, false, MODE>(c, src, po, s, qx, qy, k, i);
#pragma unroll
    for (int j = 1; j <= 9; ++j) L.w[j] = pack16(h[PI(j)], h[PI(j) + 1]);
    L.f0 = MODE == AD_WALL ? bload32f(src, 4u * (unsigned)(qx + c.nx * (qy + c.ny * k)), 0u)
                           : bload32f(src, 2u * s.self, 2u * po.z2 * (unsigned)k);
  }
}
template <int S, int MODE>
__device__ __forceinline__ void issue_g(const CaseDev& c, Rsrc src, const PlaneOfs& po, int qx,
                                        int qy, int k, uint32_t odd, GLoads& L) {
  const Site s = make_site<MODE>(c, qx, qy);
  if constexpr (MODE == AD_INNER) {
    const unsigned base = s.self - 2u * odd;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const int i = 2 * q, i2 = 2 * q + 1 < Q ? 2 * q + 1 : 2 * q;
      const unsigned a = inner_soff<true>(c, po, k, i), b = inner_soff<true>(c, po, k, i2);
      if (g_paired(q)) L.w[q] = pair_load(src, base, a, b, 0u - odd);
      else L.w[q] = pack16(bload16(src, s.self, a), i2 != i ? bload16(src, s.self, b) : (uint16_t)0);
    }
  } else {
    uint16_t h[Q + 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = pull_word<S, true, MODE>(c, src, po, s, qx, qy, k, i);
    h[Q] = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q) L.w[q] = pack16(h[2 * q], h[2 * q + 1]);
  }
}

// The z march of one tile with the pulls in addressing mode MODE.  The
// global loads of an iteration (f of the phi stage, gbar of the u, p stage,
// for the own node and the ring positions) are issued one iteration ahead,
// after the u, p stage and before the collision, so they are in flight while
// the collision computes and cost one memory round trip per plane.
template <int S, int TX, int TY, int RF, int MODE>
__device__ __forceinline__ void march_loop(const CaseDev& c, MarchLds<TX, TY, RF>& L,
                                           const MarchTile& tl, Rsrc src, Rsrc dst,
                                           uint32_t skey) {
  using T = MarchLds<TX, TY, RF>;
  constexpr int NT = TX * TY, R = T::R, RX = T::RX, PX = T::PX, PY = T::PY, MX = T::MX,
                MY = T::MY, UX = T::UX, UY = T::UY;
  constexpr int NPRING = T::NP - NT;  // positions of the phi region outside the tile
  constexpr int NRING = T::NU - NT;   // positions of the u, p region outside the tile
  constexpr int KP = (NPRING + NT - 1) / NT;  // phi ring positions per thread (at most)
  constexpr int KU = (NRING + NT - 1) / NT;   // u, p ring positions per thread (at most)
  static_assert(NT % 2 == 0 && NPRING % 2 == 0 && NRING % 2 == 0 && TX % 2 == 0,
                "lane pairs hold x-adjacent positions");
  const int x0 = tl.x0, y0 = tl.y0, za = tl.za, zb = tl.zb;
  const int tid = threadIdx.x;
  const uint32_t odd = tid & 1;
  const uint32_t psel = odd ? 0x07060302u : 0x01000504u;
  const int lx = tid % TX, ly = tid / TX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool own = gx < c.nx && gy < c.ny;
  float* const php = &L.ph[0][0];
  float* const mup = &L.mu[0][0];
  float* const pp = &L.p[0][0];

  // the sites of this thread: own node, ring positions of the phi stage
  // (rounds q: position tid - NT + q NT of the ring) and of the u, p stage
  auto phi_pos = [&](int r, int& px, int& py) {
    if (r < 0) {
      px = lx + RX;
      py = ly + R;
    } else {
      ring_pos<PX, PY, RX, R>(r, px, py);
    }
  };
  auto up_pos = [&](int r, int& ux, int& uy) {
    if (r < 0) {
      ux = lx + 2;
      uy = ly + 1;
    } else {
      ring_pos<UX, UY, 2, 1>(r, ux, uy);
    }
  };
  auto fold_x = [&](int q) { return MODE == AD_INNER ? q : fold3(q, c.nx, c.wall_x); };
  auto fold_y = [&](int q) { return MODE == AD_INNER ? q : fold3(q, c.ny, c.wall_y); };
  auto up_needed = [&](int k) { return k >= za - 1 && !(c.wall_z && (k < 0 || k >= c.nz)); };

  FLoads lf[1 + KP];  // [0]: own node
  GLoads lg[1 + KU];
  // issue the loads of iteration z: f at plane z + R, gbar at plane z + 1
  auto issue = [&](int z, const PlaneOfs& po) {
    const int kf = fold3(z + R, c.nz, c.wall_z);
#pragma unroll
    for (int q = 0; q <= KP; ++q) {
      const int r = tid - NT + q * NT;
      if (r < NPRING) {
        int px, py;
        phi_pos(r, px, py);
        issue_f<S, MODE>(c, src, po, fold_x(x0 - RX + px), fold_y(y0 - R + py), kf, odd, lf[q]);
      }
    }
    if (up_needed(z + 1)) {
      const int kg = fold3(z + 1, c.nz, c.wall_z);
#pragma unroll
      for (int q = 0; q <= KU; ++q) {
        const int r = tid - NT + q * NT;
        if (r < NRING) {
          int ux, uy;
          up_pos(r, ux, uy);
          issue_g<S, MODE>(c, src, po, fold_x(x0 - 2 + ux), fold_y(y0 - 1 + uy), kg, odd, lg[q]);
        }
      }
    }
  };

  LeanNode cur{}, nxt{};  // own node at plane z (collided now) and z + 1
  uint32_t fn[10] = {};   // own node's f words of the plane being staged
  {
    PlaneOfs po{2u * c.stride, 2u * (unsigned)(c.nx * c.ny)};
    issue(za - 2 * R, po);
  }
  for (int z = za - 2 * R; z < zb; ++z) {
    PlaneOfs po{2u * c.stride, 2u * (unsigned)(c.nx * c.ny)};
    asm volatile("" : "+s"(po.st2), "+s"(po.z2));
    // ---- phi at plane k = z + R over the phi region from the loaded f
    {
      const int b = phslot<RF>(z + R) * T::NP;
#pragma unroll
      for (int q = 0; q <= KP; ++q) {
        const int r = tid - NT + q * NT;
        if (r < NPRING) {
          uint32_t w[10];
#pragma unroll
          for (int j = 1; j <= 9; ++j)
            w[j] = MODE == AD_INNER && f_paired(j) ? pair_xchg(lf[q].w[j], psel) : lf[q].w[j];
          int px, py;
          phi_pos(r, px, py);
          php[b + px + PX * py] = lean_phi_packed<S>(c, lf[q].f0, w);
          if (q == 0) {
#pragma unroll
            for (int j = 1; j <= 9; ++j) fn[j] = w[j];
          }
        }
      }
    }
    __syncthreads();

    // ---- mu at plane z + 2 over the tile + 2 (RF = 1)
    if constexpr (RF) {
      const int k = z + 2;
      if (k >= za - 2 && !(c.wall_z && (k < 0 || k >= c.nz))) {
        const int bm = ring4(k - 1) * T::NP, b0 = ring4(k) * T::NP, bp = ring4(k + 1) * T::NP;
        const int b = ring3(k) * T::NM;
        for (int pos = tid; pos < T::NM; pos += NT) {
          int mx = pos % MX, my = pos / MX;
          if constexpr (MODE == AD_WALL) {
            if (tl.wall_xy) {
              mx = mirror_local(mx, x0 - 2, c.nx, c.wall_x, MX);
              my = mirror_local(my, y0 - 2, c.ny, c.wall_y, MY);
            }
          }
          const int pc = (mx - 2 + RX) + PX * (my - 2 + R);
          float v[Q];
#pragma unroll
          for (int i = 1; i < Q; ++i)
            v[i] = php[(EZ(i) < 0 ? bm : (EZ(i) > 0 ? bp : b0)) + pc + EX(i) + PX * EY(i)];
          const float h0 = php[b0 + pc];
          mup[b + pos] = lean_mu(c, h0, lean_lap(v, h0));
        }
      }
      __syncthreads();
    }

    // ---- gbar moments, grad phi, (lap mu,) u and p at plane z + 1 over the
    // tile + 1 from the loaded gbar (own node's words kept for the collision)
    {
      const int k = z + 1;
      if (up_needed(k)) {
        const int bm = phslot<RF>(k - 1) * T::NP, b0 = phslot<RF>(k) * T::NP,
                  bp = phslot<RF>(k + 1) * T::NP;
        const int pb = ring3(k) * T::NU;
#pragma unroll
        for (int q = 0; q <= KU; ++q) {
          const int r = tid - NT + q * NT;
          if (r < NRING) {
            uint32_t gwd[10];
#pragma unroll
            for (int kq = 0; kq < 10; ++kq)
              gwd[kq] = MODE == AD_INNER && g_paired(kq) ? pair_xchg(lg[q].w[kq], psel)
                                                         : lg[q].w[kq];
            if (q == 0) {
              const int gs = (k + 2) & 1;
#pragma unroll
              for (int kq = 0; kq < 10; ++kq) L.gw[gs][kq][tid] = gwd[kq];
            }
            int ux, uy;
            up_pos(r, ux, uy);
            // the pair-alignment columns at x0 - 2 and x0 + TX + 1 are not
            // needed by the collision
            if (ux != 0 && ux != UX - 1) {
              int mx = ux, my = uy;
              if constexpr (MODE == AD_WALL) {
                if (tl.wall_xy) {
                  mx = mirror_local(ux, x0 - 2, c.nx, c.wall_x, UX);
                  my = mirror_local(uy, y0 - 1, c.ny, c.wall_y, UY);
                }
              }
              float m0, m1x, m1y, m1z;
              lean_moments_packed<S>(c, gwd, m0, m1x, m1y, m1z);
              const int pc = (mx - 2 + RX) + PX * (my - 1 + R);
              float v[Q];
#pragma unroll
              for (int i = 1; i < Q; ++i)
                v[i] = php[(EZ(i) < 0 ? bm : (EZ(i) > 0 ? bp : b0)) + pc + EX(i) + PX * EY(i)];
              const float ph = php[b0 + pc];
              float g0, g1, g2;
              lean_grad(v, g0, g1, g2);
              float mu, cc = 0.0f;
              if constexpr (RF) {
                const int mc = mx + MX * (my + 1);
                const int um = ring3(zread_m(c, k - 1)) * T::NM, u0 = ring3(k) * T::NM,
                          up = ring3(zread_m(c, k + 1)) * T::NM;
                mu = mup[u0 + mc];
                float w[Q];
#pragma unroll
                for (int i = 1; i < Q; ++i)
                  w[i] = mup[(EZ(i) < 0 ? um : (EZ(i) > 0 ? up : u0)) + mc + EX(i) + MX * EY(i)];
                cc = c.corr * lean_lap(w, mu);
              } else {
                mu = lean_mu(c, ph, lean_lap(v, ph));
              }
              const LeanUP rp = lean_recover(c, ph, mu, g0, g1, g2, cc, m0, m1x, m1y, m1z);
              pp[pb + ux + UX * uy] = rp.p;
              if (q == 0) {
                nxt.ph = ph;
                nxt.mu = mu;
                nxt.cc = cc;
                nxt.p = rp.p;
                nxt.ux = rp.ux;
                nxt.uy = rp.uy;
                nxt.uz = rp.uz;
                nxt.gx = g0;
                nxt.gy = g1;
                nxt.gz = g2;
              }
            }
          }
        }
      }
    }
    __syncthreads();

    // the loads of the next iteration, in flight during the collision
    if (z + 1 < zb) issue(z + 1, po);

    // ---- grad p and the collision of the tile's nodes at plane z (a lane
    // pair is own or not as a whole: nx and TX are even)
    if (z >= za && own) {
      const int uc = (lx + 2) + UX * (ly + 1);
      const int pm = ring3(zread_m(c, z - 1)) * T::NU, p0 = ring3(z) * T::NU,
                pq = ring3(zread_m(c, z + 1)) * T::NU;
      float v[Q];
#pragma unroll
      for (int i = 1; i < Q; ++i)
        v[i] = pp[(EZ(i) < 0 ? pm : (EZ(i) > 0 ? pq : p0)) + uc + EX(i) + UX * EY(i)];
      float gp0, gp1, gp2;
      lean_grad(v, gp0, gp1, gp2);
      uint32_t og[10], of[10], fa[10], gc[10];
      const int fs = z % T::NFC, gs = z & 1;  // z >= 0 here
#pragma unroll
      for (int j = 1; j <= 9; ++j) fa[j] = L.fw[fs][j - 1][tid];
#pragma unroll
      for (int kq = 0; kq < 10; ++kq) gc[kq] = L.gw[gs][kq][tid];
      const uint32_t nkey = sr_node_key(skey, (unsigned)(gx + c.nx * (gy + c.ny * z)));
      const float f0 = lean_collide<S>(c, cur, gp0, gp1, gp2, gc, fa, og, of, nkey);
      // stores: lane-pair words (even lane: the first population of each
      // packed pair, odd lane: the second, one plane further), the plane and
      // z plane in the uniform offset
      const unsigned self = 2u * (unsigned)(gx + c.nx * gy);
      const unsigned zo = po.z2 * (unsigned)z;
      const unsigned vpair = self - 2u * odd + (po.st2 & (0u - odd));
      bstore32f(dst, 2u * self, 2u * zo, f0);
#pragma unroll
      for (int j = 1; j <= 9; ++j)
        bstore32(dst, vpair, zo + po.plane<false>(PI(j)), pair_xchg(of[j], psel));
#pragma unroll
      for (int q = 0; q < 9; ++q)
        bstore32(dst, vpair, zo + po.plane<true>(2 * q), pair_xchg(og[q], psel));
      {
        const uint32_t w = pair_xchg(og[9], psel);  // even lane: gbar_18 of both nodes
        if (!odd) bstore32(dst, vpair, zo + po.plane<true>(18), w);
      }
    }
    cur = nxt;
    // the staged plane's f words take the slot the collision just read
    {
      const int fs = (z + R + 3 * T::NFC) % T::NFC;
#pragma unroll
      for (int j = 1; j <= 9; ++j) L.fw[fs][j - 1][tid] = fn[j];
    }
  }
}

template <int S, int TX, int TY, int RF>
__global__ void __launch_bounds__(TX * TY) k3_march(CaseDev c, int parity, int zs) {
  using T = MarchLds<TX, TY, RF>;
  constexpr int R = T::R, RX = T::RX;
  __shared__ T L;
  // XCD-aware tile order: x fastest, then y, then the z chunk; workgroup b
  // runs on XCD b % 8 and takes the b / 8-th tile of that XCD's contiguous
  // chunk, so an XCD's consecutive tiles share their x-y halos in its L2
  const int ntx = (c.nx + TX - 1) / TX, nty = (c.ny + TY - 1) / TY;
  const int ntiles = ntx * nty * ((c.nz + zs - 1) / zs);
  const int chunk = (ntiles + 7) >> 3;
  const int t = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  const uint32_t skey = sr_step_key(sr_clock(c, parity));  // stochastic rounding of g
  if (blockIdx.x >= (unsigned)(8 * chunk) || t >= ntiles) return;
  MarchTile tl;
  tl.x0 = (t % ntx) * TX;
  tl.y0 = ((t / ntx) % nty) * TY;
  tl.za = (t / (ntx * nty)) * zs;
  tl.zb = min(tl.za + zs, c.nz);
  // every pull source of the staged region inside the grid (a pull reaches
  // one position beyond it)
  const bool inner = tl.x0 >= RX + 1 && tl.x0 + TX + RX + 1 <= c.nx && tl.y0 >= R + 1 &&
                     tl.y0 + TY + R + 1 <= c.ny;
  tl.wall_xy = (c.wall_x && (tl.x0 < RX || tl.x0 + TX + RX > c.nx)) ||
               (c.wall_y && (tl.y0 < R || tl.y0 + TY + R > c.ny));
  const Rsrc src = copy_rsrc(parity ? c.state[1] : c.state[0]);
  const Rsrc dst = copy_rsrc(parity ? c.state[0] : c.state[1]);
  if (inner) march_loop<S, TX, TY, RF, AD_INNER>(c, L, tl, src, dst, skey);
  else if (c.wall_x || c.wall_y) march_loop<S, TX, TY, RF, AD_WALL>(c, L, tl, src, dst, skey);
  else march_loop<S, TX, TY, RF, AD_SEAM>(c, L, tl, src, dst, skey);
}

}  // namespace d3q19

// Launch one fused 16-bit step of case c: TX x TY tiles, chunks of zs planes.
template <int S, int TX, int TY>
static void march_case(const CaseDev& c, int parity, int zs, int rf, hipStream_t s) {
  const int ft = ((c.nx + TX - 1) / TX) * ((c.ny + TY - 1) / TY) * ((c.nz + zs - 1) / zs);
  if (rf)
    hipLaunchKernelGGL((d3q19::k3_march<S, TX, TY, 1>), dim3(8 * ((ft + 7) / 8)), dim3(TX * TY),
                       0, s, c, parity, zs);
  else
    hipLaunchKernelGGL((d3q19::k3_march<S, TX, TY, 0>), dim3(8 * ((ft + 7) / 8)), dim3(TX * TY),
                       0, s, c, parity, zs);
}

hipError_t d3q19_march(const CaseDev& c, int storage, int tx, int ty, int zs, int parity,
                       hipStream_t s) {
  const int rf = c.corr != 0.0f;
  if (storage == ST_FP16) {
    if (tx == 32 && ty == 8) march_case<ST_FP16, 32, 8>(c, parity, zs, rf, s);
    else if (tx == 64) march_case<ST_FP16, 64, 8>(c, parity, zs, rf, s);
    else march_case<ST_FP16, 32, 16>(c, parity, zs, rf, s);
  } else {
    if (tx == 32 && ty == 8) march_case<ST_BF16, 32, 8>(c, parity, zs, rf, s);
    else if (tx == 64) march_case<ST_BF16, 64, 8>(c, parity, zs, rf, s);
    else march_case<ST_BF16, 32, 16>(c, parity, zs, rf, s);
  }
  return hipGetLastError();
}

}  // namespace lbm
