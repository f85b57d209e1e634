// Internal declarations shared by the host setup (rt_host.cpp), the ABI layer
// (rt_abi.hip) and the device kernels (rt_kernels.hip).  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rt_lbm.h"

namespace rtl {

constexpr int kMaxDirs = 256;
constexpr int kTileRows = 32;  // rows of one MFMA output tile (32x32 family)

// Host-side description of the direction grid and the operators, float64.
struct HostPlan {
  int nx = 0, ny = 0, n = 0;   // ny: rows of cells (ny_lattice * nz on a 3-D lattice)
  int nz = 1, ny_lattice = 0;  // 3-D lattice: layers and rows per layer
  int R = 0;      // 4n: rows of the contraction
  int Rpad = 0;   // R rounded up to kTileRows
  std::vector<double> theta, phi, domega;   // [n]
  std::vector<double> kvec, eth, eph;       // [n][3]
  std::vector<double> lx, ly, lz;           // [n] displacement per step (lz: 3-D only)
  std::vector<int> outmask;                 // [n] bit e: leaves through edge (3-D: face) e
  // Collision matrix in ABI order: row 4*d_out + s_out, column 4*d_in + s_in.
  std::vector<double> M;                    // [R][R]
};

// Builds directions, displacements and the collision matrix; returns RT_OK or
// an error with msg set.  Pure host code (no HIP calls).
rt_status build_plan(const rt_problem *p, HostPlan *out, std::string *msg);

// Per-direction streaming taps in float32 for the device.
struct DirTaps {
  int32_t ox0, oy0;   // base offsets floor(l_x), floor(l_y)
  float wx0, wx1;     // weights of offsets ox0 and ox0 + 1
  float wy0, wy1;
  float w00, w10, w01, w11;   // products wx_b * wy_b' (tap (bx, by) -> w_{bx by})
};

// Per-direction trilinear taps of a 3-D lattice: base offsets floor(l) and
// the weights w[4 bz + 2 by + bx] = wx_bx wy_by wz_bz of offsets (base + b).
struct DirTaps3 {
  int32_t ox0, oy0, oz0, pad;
  float w[8];
};

// Contraction tables in the row order used by the kernels: GEMM row
// r = 4 d + s (the state's own plane order), padded to Rpad.  For every
// 32-row tile t, columns [klo[t], khi[t]) cover all its non-zero entries
// (rounded to the fragment K step).  Every fragment table ends with one
// K step of zeros (64 lane records) at zero_off, which kernels read for
// steps past a tile's range.
struct TileRange {
  int32_t klo, khi;   // K range
  int32_t frag_off;   // offset (in 16-byte lane records) of the tile's fragments
  int32_t zero_off;   // offset of the table's zero block
};

enum FragKind { FRAG_F32 = 0, FRAG_BF16 = 1, FRAG_F16 = 2 };

// Packs A = (transpose ? G^T : G) of the GEMM-ordered matrix G into MFMA lane
// fragments: for each tile, each K step, 64 lanes x 16 bytes, then one zero
// K step.  For FRAG_F32
// one record feeds four 32x32x2 steps (K step 8); for bf16/f16 one record is
// one 32x32x16 step (K step 16).  `scale` multiplies every entry; `lo` selects
// the low part of a bf16 hi/lo split.
void pack_fragments(const HostPlan &hp, bool transpose, FragKind kind, double scale, bool lo,
                    std::vector<TileRange> *tiles, std::vector<uint8_t> *bytes);

// GEMM-order matrix G[r_out][r_in] (Rpad x Rpad, zero padded).
std::vector<double> gemm_order(const HostPlan &hp);

int gemm_row(int n, int d, int s);

}  // namespace rtl
